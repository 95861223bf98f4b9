// Host FP64 symmetric eigensolver for the PCA of Algorithm 1 (training P_p and the residual
// variances lambda_i): Householder reduction to tridiagonal form followed by the implicit-shift QL
// iteration (the classical EISPACK tred2 / tql2 scheme; Golub & Van Loan, Section 8.3).  The
// covariance is at most a few thousand square, so an O(n^3) host pass is a small part of the build.
// Matrices are held column-major so the inner loops walk contiguous memory.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "mrq_internal.h"

namespace mrq {

namespace {

struct ColMajor {
    int n;
    std::vector<double> a;
    double& operator()(int r, int c) { return a[(size_t)c * n + r]; }
};

// Householder tridiagonalisation: on return V holds the accumulated orthogonal transform, d the
// diagonal and e the sub-diagonal (e[0] = 0).
void tridiagonalize(ColMajor& V, std::vector<double>& d, std::vector<double>& e) {
    const int n = V.n;
    for (int j = 0; j < n; j++) d[j] = V(n - 1, j);
    for (int i = n - 1; i > 0; i--) {
        double scale = 0.0, h = 0.0;
        for (int k = 0; k < i; k++) scale += std::fabs(d[k]);
        if (scale == 0.0) {
            e[i] = d[i - 1];
            for (int j = 0; j < i; j++) {
                d[j] = V(i - 1, j);
                V(i, j) = 0.0;
                V(j, i) = 0.0;
            }
        } else {
            for (int k = 0; k < i; k++) {
                d[k] /= scale;
                h += d[k] * d[k];
            }
            double f = d[i - 1];
            double g = std::sqrt(h);
            if (f > 0) g = -g;
            e[i] = scale * g;
            h -= f * g;
            d[i - 1] = f - g;
            for (int j = 0; j < i; j++) e[j] = 0.0;
            for (int j = 0; j < i; j++) {
                f = d[j];
                V(j, i) = f;
                g = e[j] + V(j, j) * f;
                double* col = &V(0, j);
                for (int k = j + 1; k <= i - 1; k++) {
                    g += col[k] * d[k];
                    e[k] += col[k] * f;
                }
                e[j] = g;
            }
            f = 0.0;
            for (int j = 0; j < i; j++) {
                e[j] /= h;
                f += e[j] * d[j];
            }
            const double hh = f / (h + h);
            for (int j = 0; j < i; j++) e[j] -= hh * d[j];
            for (int j = 0; j < i; j++) {
                f = d[j];
                g = e[j];
                double* col = &V(0, j);
                for (int k = j; k <= i - 1; k++) col[k] -= (f * e[k] + g * d[k]);
                d[j] = V(i - 1, j);
                V(i, j) = 0.0;
            }
        }
        d[i] = h;
    }
    for (int i = 0; i < n - 1; i++) {
        V(n - 1, i) = V(i, i);
        V(i, i) = 1.0;
        const double h = d[i + 1];
        if (h != 0.0) {
            double* ci1 = &V(0, i + 1);
            for (int k = 0; k <= i; k++) d[k] = ci1[k] / h;
            for (int j = 0; j <= i; j++) {
                double* cj = &V(0, j);
                double g = 0.0;
                for (int k = 0; k <= i; k++) g += ci1[k] * cj[k];
                for (int k = 0; k <= i; k++) cj[k] -= g * d[k];
            }
        }
        for (int k = 0; k <= i; k++) V(k, i + 1) = 0.0;
    }
    for (int j = 0; j < n; j++) {
        d[j] = V(n - 1, j);
        V(n - 1, j) = 0.0;
    }
    V(n - 1, n - 1) = 1.0;
    e[0] = 0.0;
}

// Implicit-shift QL on the tridiagonal (d, e), accumulating rotations into V's columns.
void ql_implicit(ColMajor& V, std::vector<double>& d, std::vector<double>& e) {
    const int n = V.n;
    for (int i = 1; i < n; i++) e[i - 1] = e[i];
    e[n - 1] = 0.0;
    double f = 0.0, tst1 = 0.0;
    const double eps = std::ldexp(1.0, -52);
    for (int l = 0; l < n; l++) {
        tst1 = std::max(tst1, std::fabs(d[l]) + std::fabs(e[l]));
        int m = l;
        while (m < n) {
            if (std::fabs(e[m]) <= eps * tst1) break;
            m++;
        }
        if (m > l) {
            int guard = 0;
            do {
                double g = d[l];
                double p = (d[l + 1] - g) / (2.0 * e[l]);
                double r = std::hypot(p, 1.0);
                if (p < 0) r = -r;
                d[l] = e[l] / (p + r);
                d[l + 1] = e[l] * (p + r);
                const double dl1 = d[l + 1];
                double h = g - d[l];
                for (int i = l + 2; i < n; i++) d[i] -= h;
                f += h;
                p = d[m];
                double c = 1.0, c2 = c, c3 = c, s = 0.0, s2 = 0.0;
                const double el1 = e[l + 1];
                for (int i = m - 1; i >= l; i--) {
                    c3 = c2;
                    c2 = c;
                    s2 = s;
                    g = c * e[i];
                    h = c * p;
                    r = std::hypot(p, e[i]);
                    e[i + 1] = s * r;
                    s = e[i] / r;
                    c = p / r;
                    p = c * d[i] - s * g;
                    d[i + 1] = h + s * (c * g + s * d[i]);
                    double* ci = &V(0, i);
                    double* ci1 = &V(0, i + 1);
                    for (int k = 0; k < n; k++) {
                        const double t = ci1[k];
                        ci1[k] = s * ci[k] + c * t;
                        ci[k] = c * ci[k] - s * t;
                    }
                }
                p = -s * s2 * c3 * el1 * e[l] / dl1;
                e[l] = s * p;
                d[l] = c * p;
            } while (std::fabs(e[l]) > eps * tst1 && ++guard < 200);
        }
        d[l] += f;
        e[l] = 0.0;
    }
}

}  // namespace

void eigh_host(const double* A, int n, double* evals, double* evecs_rows) {
    ColMajor V{n, std::vector<double>((size_t)n * n)};
    for (int c = 0; c < n; c++)
        for (int r = 0; r < n; r++) V(r, c) = A[(size_t)r * n + c];
    std::vector<double> d(n), e(n);
    tridiagonalize(V, d, e);
    ql_implicit(V, d, e);
    std::vector<int> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return d[a] > d[b]; });
    for (int i = 0; i < n; i++) {
        const int c = order[i];
        evals[i] = d[c];
        const double* col = &V(0, c);
        int arg = 0;
        double best = -1.0;
        for (int r = 0; r < n; r++)
            if (std::fabs(col[r]) > best) { best = std::fabs(col[r]); arg = r; }
        const double sg = col[arg] < 0 ? -1.0 : 1.0;
        for (int r = 0; r < n; r++) evecs_rows[(size_t)i * n + r] = sg * col[r];
    }
}

}  // namespace mrq
