/*
 * MRQ CPU oracle — TEST INFRASTRUCTURE ONLY (see mrq_oracle.h).
 *
 * Plain single-threaded C99, FP64 throughout except where a floating-point value decides an integer
 * code: the query quantizer takes its decisions in FP32, the precision the device kernels use
 * (the paper fixes no precision for it).  Build with -O2 -ffp-contract=off and no fast-math so every
 * FP32 step is one IEEE-rounded operation.
 *
 * Readings of points the paper leaves open (each one is restated where it is used):
 *   R1  data and queries are centred before PCA: x_p = P_p (x - mu)               (Algorithm 1)
 *   R2  covariance normalised by 1/N; eigenvalues descending; each eigenvector's largest-magnitude
 *       entry is made positive (ties -> lower index)
 *   R3  c in Eq 2 is the vector's own IVF centroid in the d-dim projected space
 *   R4  query normalisation / rotation / quantisation is done per (query, list) pair
 *   R5  codebook dimension is d (the quantised subspace), x' = P_r^T (x_d - c)/||x_d - c||
 *   R6  a coordinate equal to 0 gets sign bit 1
 *   R7  query quantisation: B_q bits, v_l = min q', Delta = (max q' - v_l)/(2^B_q - 1),
 *       u_i = floor((q'_i - v_l) * (1/Delta) + 1/2) clamped; Delta = 1, u = 0 when max == min
 *   R8  eps_b = 2 n_x n_q sqrt(1 - xi^2)/xi * eps0/sqrt(d - 1)   (Eq 5 scaled by C2's factor)
 *   R9  eps_r = 2 m sigma with sigma^2 = sum_{i>d} lambda_i q_{p,i}^2   (Eq 6; C3 = -2<x_r,q_r>)
 *   R10 ||x||^2, ||q||^2 of Eq 7 are ||x_p||^2, ||q_p||^2
 *   R11 tau = +inf until k results are held; strict "<" in both tests; results ordered by (dis, id)
 *   R12 lists probed nearest-first (ties -> smaller list id), vectors in ascending id within a list
 *   R13 B-bit codes: y_i = s_i (m_i + 1/2), s_i = sign(x'_i), m_i = min(2^(B-1)-1, floor(t |x'_i|)),
 *       at the scale t maximising <y, x'>/||y|| (ties -> smaller t); level index u_i = y_i + h with
 *       h = (2^B - 1)/2, so the top bit of u_i is the sign bit; xi_B = <y, x'>/||y||
 *   R14 degenerate n_x = 0: the quantised term and eps_b are 0 (xi := 1, all sign bits 1)
 *   R15 k-means: seeded distinct-point init, Lloyd until no change or iters, empty cluster takes
 *       the farthest point of the largest cluster, ties -> lower index; final lists are the nearest
 *       centroid of each x_d under the stored centroids
 *   R16 P_r: Haar orthogonal matrix from modified Gram-Schmidt (twice) of a seeded Gaussian matrix
 *   R17 ||x_r||^2 of an imported index is ||x - mu||^2 - ||x_d||^2 (P_p orthogonal; Eq 1)
 *   R18 the variances lambda_i of Eq 6 are non-negative: an eigenvalue that round-off puts below zero
 *       (rank-deficient data) counts as 0
 *
 * MR-SQ (Appendix A.2, Exp-5: the projection and split of MRQ applied to 8-bit scalar quantisation):
 *   S1  the codes quantise the leading d PCA coordinates, one uniform 8-bit grid per coordinate over
 *       that coordinate's range in the data set, [lo_i, hi_i] = min / max of the FP32 coordinates
 *   S2  delta_i = (hi_i - lo_i)/255, u_i = min(255, floor((x_i - lo_i) * (1/delta_i) + 1/2)), each step
 *       one FP32 rounding (an integer decided from floating point: FP32, the device precision);
 *       delta_i = 1 and u_i = 0 when hi_i == lo_i; the reconstruction is lo_i + delta_i u_i
 *   S3  estimate = ||xhat_d - q_d||^2 + ||x_r||^2 + ||q_r||^2, i.e. Eq 7's projected distance with x_d
 *       replaced by its reconstruction (the tail enters through its norms only, as in MRQ)
 *   S4  with no error bound, the R candidates of the probed lists with the smallest (estimate, id) are
 *       re-ranked by exact distance and the result is their k nearest by (dis, id); R = 500 by default
 *
 * Parity unpinned: the absolute constant c0 of Eq 5 (the paper gives none), hence the exact failure
 * probability of eps_b; recall figures on synthetic data (no paper value applies).
 */
#include "mrq_oracle.h"

#include <float.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------------------------------ */
/* Seeded randomness: SplitMix64 (Steele, Lea, Flood 2014) and Box-Muller.                          */

uint64_t orc_splitmix64(uint64_t *state) {
    uint64_t z = (*state += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static double uniform01(uint64_t *s) { /* in [0, 1) with 53 random bits */
    return (double)(orc_splitmix64(s) >> 11) * (1.0 / 9007199254740992.0);
}

void orc_gaussian(uint64_t seed, int64_t n, double *out) {
    uint64_t s = seed;
    const double two_pi = 6.283185307179586476925286766559;
    for (int64_t i = 0; i < n; i += 2) {
        double u1 = 1.0 - uniform01(&s); /* (0, 1] so the log is finite */
        double u2 = uniform01(&s);
        double r = sqrt(-2.0 * log(u1));
        out[i] = r * cos(two_pi * u2);
        if (i + 1 < n) out[i + 1] = r * sin(two_pi * u2);
    }
}

/* ------------------------------------------------------------------------------------------------ */
/* Symmetric eigendecomposition by the cyclic Jacobi method (textbook; FP64).                       */
/* evecs is row-major with eigenvector i in row i; eigenvalues descending; sign rule R2.             */

int orc_eigh(const double *A, int n, double *evals, double *evecs) {
    double *a = malloc(sizeof(double) * n * n);
    double *v = malloc(sizeof(double) * n * n);
    int *order = malloc(sizeof(int) * n);
    if (!a || !v || !order) { free(a); free(v); free(order); return -1; }
    memcpy(a, A, sizeof(double) * n * n);
    for (int i = 0; i < n * n; i++) v[i] = 0.0;
    for (int i = 0; i < n; i++) v[i * n + i] = 1.0;
    double scale = 0.0;
    for (int i = 0; i < n * n; i++) scale += a[i] * a[i];
    for (int sweep = 0; sweep < 100; sweep++) {
        double off = 0.0;
        for (int p = 0; p < n; p++)
            for (int q = p + 1; q < n; q++) off += a[p * n + q] * a[p * n + q];
        if (off <= 1e-30 * scale || off == 0.0) break;
        for (int p = 0; p < n - 1; p++) {
            for (int q = p + 1; q < n; q++) {
                double apq = a[p * n + q];
                if (fabs(apq) < 1e-300) continue;
                double theta = (a[q * n + q] - a[p * n + p]) / (2.0 * apq);
                double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                for (int r = 0; r < n; r++) { /* A <- A J */
                    double arp = a[r * n + p], arq = a[r * n + q];
                    a[r * n + p] = c * arp - s * arq;
                    a[r * n + q] = s * arp + c * arq;
                }
                for (int r = 0; r < n; r++) { /* A <- J^T A */
                    double apr = a[p * n + r], aqr = a[q * n + r];
                    a[p * n + r] = c * apr - s * aqr;
                    a[q * n + r] = s * apr + c * aqr;
                }
                for (int r = 0; r < n; r++) { /* V <- V J */
                    double vrp = v[r * n + p], vrq = v[r * n + q];
                    v[r * n + p] = c * vrp - s * vrq;
                    v[r * n + q] = s * vrp + c * vrq;
                }
            }
        }
    }
    for (int i = 0; i < n; i++) order[i] = i;
    for (int i = 1; i < n; i++) { /* insertion sort, descending eigenvalue, stable */
        int key = order[i], j = i - 1;
        while (j >= 0 && a[order[j] * n + order[j]] < a[key * n + key]) { order[j + 1] = order[j]; j--; }
        order[j + 1] = key;
    }
    for (int i = 0; i < n; i++) {
        int col = order[i];
        evals[i] = a[col * n + col];
        int arg = 0;
        double best = -1.0;
        for (int r = 0; r < n; r++) {
            double m = fabs(v[r * n + col]);
            if (m > best) { best = m; arg = r; }
        }
        double sgn = v[arg * n + col] < 0.0 ? -1.0 : 1.0;
        for (int r = 0; r < n; r++) evecs[i * n + r] = sgn * v[r * n + col];
    }
    free(a); free(v); free(order);
    return 0;
}

/* ------------------------------------------------------------------------------------------------ */
/* Haar random orthogonal d x d matrix (R16). Columns are orthonormal; row-major storage.           */

int orc_haar(int d, uint64_t seed, double *P) {
    double *g = malloc(sizeof(double) * d * d);
    if (!g) return -1;
    orc_gaussian(seed, (int64_t)d * d, g);
    for (int j = 0; j < d; j++) {
        for (int pass = 0; pass < 2; pass++) {
            for (int i = 0; i < j; i++) {
                double dot = 0.0;
                for (int r = 0; r < d; r++) dot += g[r * d + i] * g[r * d + j];
                for (int r = 0; r < d; r++) g[r * d + j] -= dot * g[r * d + i];
            }
        }
        double nrm = 0.0;
        for (int r = 0; r < d; r++) nrm += g[r * d + j] * g[r * d + j];
        nrm = sqrt(nrm);
        for (int r = 0; r < d; r++) g[r * d + j] /= nrm;
    }
    memcpy(P, g, sizeof(double) * d * d);
    free(g);
    return 0;
}

/* ------------------------------------------------------------------------------------------------ */
/* Codes (Section 4.2 and R13).                                                                     */

/* 1-bit code: b_i = [x'_i >= 0] (R6) and xi = <xbar, x_b> = sum_i |x'_i| / sqrt(d). */
void orc_encode_sign(const double *xprime, int d, uint8_t *bits, double *xi) {
    double s = 0.0;
    for (int i = 0; i < d; i++) {
        bits[i] = xprime[i] >= 0.0 ? 1 : 0;
        s += (bits[i] ? 1.0 : -1.0) * xprime[i];
    }
    *xi = s / sqrt((double)d);
}

static double ext_cosine(const double *a, const int *m, int d) {
    double num = 0.0, den = 0.0;
    for (int k = 0; k < d; k++) {
        double y = m[k] + 0.5;
        num += y * a[k];
        den += y * y;
    }
    return num / sqrt(den);
}

/* B-bit code (R13): enumerate every scale t at which some floor(t |x'_k|) steps, evaluate the code
 * there and keep the best cosine (ties -> smaller t, then smaller dimension). */
double orc_encode_ext(const double *xprime, int d, int B, uint8_t *u) {
    const int M = (1 << (B - 1)) - 1;
    double *a = malloc(sizeof(double) * d);
    int *m = malloc(sizeof(int) * d), *best_m = malloc(sizeof(int) * d);
    for (int k = 0; k < d; k++) { a[k] = fabs(xprime[k]); m[k] = 0; best_m[k] = 0; }
    double best = ext_cosine(a, m, d), best_t = 0.0;
    int best_i = -1;
    for (int i = 0; i < d; i++) {
        if (a[i] <= 0.0) continue;
        for (int j = 1; j <= M; j++) {
            double t = (double)j / a[i];
            for (int k = 0; k < d; k++) {
                double f = floor(t * a[k]);
                m[k] = f > M ? M : (int)f;
            }
            m[i] = j;
            double c = ext_cosine(a, m, d);
            if (c > best || (c == best && (t < best_t || (t == best_t && i < best_i)))) {
                best = c; best_t = t; best_i = i;
                memcpy(best_m, m, sizeof(int) * d);
            }
        }
    }
    const int half = 1 << (B - 1);
    for (int k = 0; k < d; k++)
        u[k] = (uint8_t)(xprime[k] >= 0.0 ? half + best_m[k] : half - 1 - best_m[k]);
    /* xi_B = <y, x'>/||y|| with the signed levels */
    double num = 0.0, den = 0.0, h = (double)((1 << B) - 1) / 2.0;
    for (int k = 0; k < d; k++) {
        double y = (double)u[k] - h;
        num += y * xprime[k];
        den += y * y;
    }
    free(a); free(m); free(best_m);
    return num / sqrt(den);
}

/* Brute force over all (2^B)^d level vectors (tiny d, B only): max of <y, x'>/||y||. */
double orc_ext_exhaustive(const double *xprime, int d, int B, uint8_t *u) {
    const int L = 1 << B;
    double h = (double)(L - 1) / 2.0, best = -2.0;
    int64_t total = 1;
    for (int k = 0; k < d; k++) total *= L;
    for (int64_t c = 0; c < total; c++) {
        int64_t r = c;
        double num = 0.0, den = 0.0;
        for (int k = 0; k < d; k++) {
            double y = (double)(r % L) - h;
            r /= L;
            num += y * xprime[k];
            den += y * y;
        }
        double cs = num / sqrt(den);
        if (cs > best) {
            best = cs;
            r = c;
            for (int k = 0; k < d; k++) { u[k] = (uint8_t)(r % L); r /= L; }
        }
    }
    return best;
}

/* Query quantisation (Algorithm 2, query quantisation; R7), decisions in FP32. */
void orc_quantize_query_f32(const float *qprime, int d, int bq, uint8_t *u, float *vl, float *delta,
                            int32_t *su) {
    const int levels = (1 << bq) - 1;
    float lo = qprime[0], hi = qprime[0];
    for (int i = 1; i < d; i++) {
        if (qprime[i] < lo) lo = qprime[i];
        if (qprime[i] > hi) hi = qprime[i];
    }
    int32_t s = 0;
    if (!(hi > lo)) {
        *vl = lo;
        *delta = 1.0f;
        for (int i = 0; i < d; i++) u[i] = 0;
        *su = 0;
        return;
    }
    volatile float dl = (hi - lo) / (float)levels;
    volatile float inv = 1.0f / dl;
    for (int i = 0; i < d; i++) {
        volatile float t = qprime[i] - lo;
        volatile float t2 = t * inv;
        volatile float t3 = t2 + 0.5f;
        int v = (int)floorf(t3);
        if (v < 0) v = 0;
        if (v > levels) v = levels;
        u[i] = (uint8_t)v;
        s += v;
    }
    *vl = lo;
    *delta = dl;
    *su = s;
}

/* ------------------------------------------------------------------------------------------------ */
/* k-means (R15), FP64.                                                                             */

static double sqdist(const double *a, const double *b, int n) {
    double s = 0.0;
    for (int i = 0; i < n; i++) { double t = a[i] - b[i]; s += t * t; }
    return s;
}

static int nearest(const double *x, const double *C, int k, int dim, double *best_d) {
    int arg = 0;
    double best = DBL_MAX;
    for (int j = 0; j < k; j++) {
        double dd = sqdist(x, C + (int64_t)j * dim, dim);
        if (dd < best) { best = dd; arg = j; }
    }
    if (best_d) *best_d = best;
    return arg;
}

int orc_kmeans(const double *P, int64_t n, int dim, int k, uint64_t seed, int iters, double *C,
               int32_t *assign) {
    if (k > n || k < 1) return -1;
    int64_t *perm = malloc(sizeof(int64_t) * n);
    int64_t *cnt = malloc(sizeof(int64_t) * k);
    if (!perm || !cnt) { free(perm); free(cnt); return -1; }
    for (int64_t i = 0; i < n; i++) perm[i] = i;
    uint64_t s = seed;
    for (int j = 0; j < k; j++) { /* partial Fisher-Yates: k distinct points */
        int64_t r = j + (int64_t)(orc_splitmix64(&s) % (uint64_t)(n - j));
        int64_t t = perm[j]; perm[j] = perm[r]; perm[r] = t;
        memcpy(C + (int64_t)j * dim, P + perm[j] * dim, sizeof(double) * dim);
    }
    for (int64_t i = 0; i < n; i++) assign[i] = -1;
    for (int it = 0; it < iters; it++) {
        int64_t changed = 0;
        for (int64_t i = 0; i < n; i++) {
            int a = nearest(P + i * dim, C, k, dim, NULL);
            if (a != assign[i]) { changed++; assign[i] = a; }
        }
        if (changed == 0) break;
        for (int j = 0; j < k; j++) cnt[j] = 0;
        for (int64_t j = 0; j < (int64_t)k * dim; j++) C[j] = 0.0;
        for (int64_t i = 0; i < n; i++) {
            cnt[assign[i]]++;
            for (int t = 0; t < dim; t++) C[(int64_t)assign[i] * dim + t] += P[i * dim + t];
        }
        for (int j = 0; j < k; j++)
            if (cnt[j] > 0)
                for (int t = 0; t < dim; t++) C[(int64_t)j * dim + t] /= (double)cnt[j];
        for (int j = 0; j < k; j++) {
            if (cnt[j] > 0) continue;
            int big = 0;
            for (int t = 1; t < k; t++) if (cnt[t] > cnt[big]) big = t;
            int64_t far = -1;
            double fd = -1.0;
            for (int64_t i = 0; i < n; i++) {
                if (assign[i] != big) continue;
                double dd = sqdist(P + i * dim, C + (int64_t)big * dim, dim);
                if (dd > fd) { fd = dd; far = i; }
            }
            memcpy(C + (int64_t)j * dim, P + far * dim, sizeof(double) * dim);
            assign[far] = j;
            cnt[big]--;
            cnt[j] = 1;
        }
    }
    for (int64_t i = 0; i < n; i++) assign[i] = nearest(P + i * dim, C, k, dim, NULL);
    free(perm); free(cnt);
    return 0;
}

/* ------------------------------------------------------------------------------------------------ */
/* Index.                                                                                           */

struct orc_index {
    int64_t N;
    int32_t D, d, B, nlist;
    double *mu, *Pp, *lam, *Pr, *C;  /* D, D*D (row i = axis i), D, d*d, nlist*d */
    int64_t *off, *lid;               /* list boundaries; ids in list order */
    int64_t *pos;                     /* per id: its list position (inverse of lid), or -1 */
    uint8_t *code;                    /* per list position: d level indices */
    float *sq_lo, *sq_delta;          /* MR-SQ grid (S1, S2): d each, or NULL */
    uint8_t *sq_code;                 /* MR-SQ codes per list position: d bytes each */
    double *xd;                       /* per list position: leading d coordinates of x_p */
    double *nx, *tx, *ax, *xi1, *xiB, *yn;
    const float *X;                   /* caller-owned original vectors, id order */
};

void orc_free(orc_index *ix) {
    if (!ix) return;
    free(ix->mu); free(ix->Pp); free(ix->lam); free(ix->Pr); free(ix->C);
    free(ix->off); free(ix->lid); free(ix->pos); free(ix->code); free(ix->xd);
    free(ix->nx); free(ix->tx); free(ix->ax); free(ix->xi1); free(ix->xiB); free(ix->yn);
    free(ix->sq_lo); free(ix->sq_delta); free(ix->sq_code);
    free(ix);
}

static orc_index *alloc_index(int64_t N, int32_t D, int32_t d, int32_t B, int32_t nlist) {
    orc_index *ix = calloc(1, sizeof(orc_index));
    if (!ix) return NULL;
    ix->N = N; ix->D = D; ix->d = d; ix->B = B; ix->nlist = nlist;
    ix->mu = calloc(D, sizeof(double));
    ix->Pp = calloc((size_t)D * D, sizeof(double));
    ix->lam = calloc(D, sizeof(double));
    ix->Pr = calloc((size_t)d * d, sizeof(double));
    ix->C = calloc((size_t)nlist * d, sizeof(double));
    ix->off = calloc(nlist + 1, sizeof(int64_t));
    ix->lid = calloc(N, sizeof(int64_t));
    ix->pos = calloc(N, sizeof(int64_t));
    ix->code = calloc((size_t)N * d, 1);
    ix->xd = calloc((size_t)N * d, sizeof(double));
    ix->nx = calloc(N, sizeof(double)); ix->tx = calloc(N, sizeof(double));
    ix->ax = calloc(N, sizeof(double)); ix->xi1 = calloc(N, sizeof(double));
    ix->xiB = calloc(N, sizeof(double)); ix->yn = calloc(N, sizeof(double));
    if (!ix->mu || !ix->Pp || !ix->lam || !ix->Pr || !ix->C || !ix->off || !ix->lid || !ix->pos || !ix->code ||
        !ix->xd || !ix->nx || !ix->tx || !ix->ax || !ix->xi1 || !ix->xiB || !ix->yn) {
        orc_free(ix);
        return NULL;
    }
    return ix;
}

/* pos[id] = list position of id (ids outside [0, N) are ignored; an id listed twice keeps its last). */
static void index_positions(orc_index *ix) {
    for (int64_t n = 0; n < ix->N; n++) ix->pos[n] = -1;
    for (int64_t p = 0; p < ix->N; p++)
        if (ix->lid[p] >= 0 && ix->lid[p] < ix->N) ix->pos[ix->lid[p]] = p;
}

/* Encode list position p from its x_d and centroid (Algorithm 1, normalise-and-quantise step). */
static void encode_position(orc_index *ix, int64_t p, const double *c) {
    const int d = ix->d, B = ix->B;
    double *o = malloc(sizeof(double) * d), *xp = malloc(sizeof(double) * d);
    uint8_t *bits = malloc(d);
    double n2 = 0.0;
    for (int i = 0; i < d; i++) { o[i] = ix->xd[p * d + i] - c[i]; n2 += o[i] * o[i]; }
    double nx = sqrt(n2);
    ix->nx[p] = nx;
    if (nx == 0.0) { /* R14 */
        for (int j = 0; j < d; j++) ix->code[p * d + j] = (uint8_t)(1 << (B - 1));
        ix->xi1[p] = 1.0; ix->xiB[p] = 1.0;
    } else {
        for (int j = 0; j < d; j++) { /* x' = P_r^T o / n_x */
            double s = 0.0;
            for (int i = 0; i < d; i++) s += ix->Pr[i * d + j] * o[i];
            xp[j] = s / nx;
        }
        double xi;
        orc_encode_sign(xp, d, bits, &xi);
        ix->xi1[p] = xi;
        if (B == 1) {
            for (int j = 0; j < d; j++) ix->code[p * d + j] = bits[j];
            ix->xiB[p] = xi;
        } else {
            ix->xiB[p] = orc_encode_ext(xp, d, B, ix->code + p * d);
        }
    }
    double h = (double)((1 << B) - 1) / 2.0, y2 = 0.0;
    for (int j = 0; j < d; j++) { double y = ix->code[p * d + j] - h; y2 += y * y; }
    ix->yn[p] = sqrt(y2);
    free(o); free(xp); free(bits);
}

orc_index *orc_build(const float *X, int64_t N, int32_t D, int32_t d, int32_t B, int32_t nlist,
                     uint64_t seed, int32_t kmeans_iters) {
    if (N < 1 || D < 2 || d < 2 || d > D || B < 1 || B > 8 || nlist < 1 || nlist > N) return NULL;
    orc_index *ix = alloc_index(N, D, d, B, nlist);
    if (!ix) return NULL;
    ix->X = X;
    /* PCA (Algorithm 1, first two steps; R1, R2) */
    for (int64_t n = 0; n < N; n++)
        for (int i = 0; i < D; i++) ix->mu[i] += X[n * D + i];
    for (int i = 0; i < D; i++) ix->mu[i] /= (double)N;
    double *S = calloc((size_t)D * D, sizeof(double)), *xc = malloc(sizeof(double) * D);
    double *xp = malloc(sizeof(double) * D);
    for (int64_t n = 0; n < N; n++) {
        for (int i = 0; i < D; i++) xc[i] = X[n * D + i] - ix->mu[i];
        for (int i = 0; i < D; i++)
            for (int j = 0; j < D; j++) S[(size_t)i * D + j] += xc[i] * xc[j];
    }
    for (size_t i = 0; i < (size_t)D * D; i++) S[i] /= (double)N;
    orc_eigh(S, D, ix->lam, ix->Pp);
    free(S);
    /* rotate, residual norms, leading d coordinates (Algorithm 1, rotation steps) */
    double *xd_id = malloc(sizeof(double) * N * d), *tx_id = malloc(sizeof(double) * N);
    double *ax_id = malloc(sizeof(double) * N);
    for (int64_t n = 0; n < N; n++) {
        for (int i = 0; i < D; i++) xc[i] = X[n * D + i] - ix->mu[i];
        double a = 0.0, t = 0.0;
        for (int r = 0; r < D; r++) {
            double s = 0.0;
            for (int i = 0; i < D; i++) s += ix->Pp[(size_t)r * D + i] * xc[i];
            xp[r] = s;
            a += s * s;
            if (r >= d) t += s * s;
        }
        memcpy(xd_id + n * d, xp, sizeof(double) * d);
        tx_id[n] = t;
        ax_id[n] = a;
    }
    free(xc); free(xp);
    /* IVF on x_d (Algorithm 1, IVF step; R15) */
    int32_t *assign = malloc(sizeof(int32_t) * N);
    orc_kmeans(xd_id, N, d, nlist, seed ^ 0x4B4D45414E53ULL, kmeans_iters, ix->C, assign);
    for (int64_t n = 0; n < N; n++) ix->off[assign[n] + 1]++;
    for (int j = 0; j < nlist; j++) ix->off[j + 1] += ix->off[j];
    int64_t *fill = malloc(sizeof(int64_t) * nlist);
    for (int j = 0; j < nlist; j++) fill[j] = ix->off[j];
    for (int64_t n = 0; n < N; n++) ix->lid[fill[assign[n]]++] = n; /* ascending id per list */
    free(fill);
    index_positions(ix);
    /* random rotation and codes (Algorithm 1, last two steps) */
    orc_haar(d, seed ^ 0x524F54415445ULL, ix->Pr);
    for (int j = 0; j < nlist; j++) {
        for (int64_t p = ix->off[j]; p < ix->off[j + 1]; p++) {
            int64_t id = ix->lid[p];
            memcpy(ix->xd + p * d, xd_id + id * d, sizeof(double) * d);
            ix->tx[p] = tx_id[id];
            ix->ax[p] = ax_id[id];
            encode_position(ix, p, ix->C + (int64_t)j * d);
        }
    }
    free(assign); free(xd_id); free(tx_id); free(ax_id);
    return ix;
}

/* Import an index written by the device library (format in include/mrq.h), searching it with this
 * oracle's own arithmetic.  When X is given, every per-vector quantity is re-derived here in FP64
 * from X and the imported P_p, mu, centroids, P_r and codes (R17); without X the stored per-vector
 * summaries (the paper's Algorithm 2 precomputed inputs) are used as they are. */
orc_index *orc_import(const char *path, const float *X, int64_t Nx, int32_t Dx) {
    FILE *f = fopen(path, "rb");
    if (!f) return NULL;
    char magic[8];
    int64_t N;
    int32_t hdr[4];
    if (fread(magic, 1, 8, f) != 8 || memcmp(magic, "MRQX0001", 8) != 0 ||
        fread(&N, 8, 1, f) != 1 || fread(hdr, 4, 4, f) != 4) { fclose(f); return NULL; }
    int32_t D = hdr[0], d = hdr[1], B = hdr[2], nlist = hdr[3];
    if (X && (Nx != N || Dx != D)) { fclose(f); return NULL; }
    orc_index *ix = alloc_index(N, D, d, B, nlist);
    if (!ix) { fclose(f); return NULL; }
    ix->X = X;
    int ok = 1;
#define RD_F32(dst, cnt)                                                              \
    do {                                                                              \
        size_t n_ = (size_t)(cnt);                                                    \
        float *t_ = malloc(sizeof(float) * (n_ ? n_ : 1));                            \
        if (!t_ || fread(t_, 4, n_, f) != n_) ok = 0;                                 \
        else for (size_t i_ = 0; i_ < n_; i_++) (dst)[i_] = t_[i_];                   \
        free(t_);                                                                     \
    } while (0)
    RD_F32(ix->mu, D);
    RD_F32(ix->Pp, (size_t)D * D);
    if (ok && fread(ix->lam, 8, D, f) != (size_t)D) ok = 0;
    RD_F32(ix->Pr, (size_t)d * d);
    RD_F32(ix->C, (size_t)nlist * d);
    if (ok && fread(ix->off, 8, nlist + 1, f) != (size_t)nlist + 1) ok = 0;
    if (ok && fread(ix->lid, 8, N, f) != (size_t)N) ok = 0;
    if (ok && fread(ix->code, 1, (size_t)N * d, f) != (size_t)N * d) ok = 0;
    RD_F32(ix->xd, (size_t)N * d);
    RD_F32(ix->nx, N);
    RD_F32(ix->tx, N);
    RD_F32(ix->ax, N);
    RD_F32(ix->xi1, N);
    RD_F32(ix->xiB, N);
    RD_F32(ix->yn, N);
#undef RD_F32
    if (ok) { /* optional MR-SQ section: "SQ8G", lo and delta (d FP32 each), codes (N x d bytes) */
        char tag[4];
        if (fread(tag, 1, 4, f) == 4) {
            if (memcmp(tag, "SQ8G", 4) != 0) ok = 0;
            else {
                ix->sq_lo = malloc(sizeof(float) * d);
                ix->sq_delta = malloc(sizeof(float) * d);
                ix->sq_code = malloc((size_t)N * d);
                if (!ix->sq_lo || !ix->sq_delta || !ix->sq_code ||
                    fread(ix->sq_lo, 4, d, f) != (size_t)d || fread(ix->sq_delta, 4, d, f) != (size_t)d ||
                    fread(ix->sq_code, 1, (size_t)N * d, f) != (size_t)N * d)
                    ok = 0;
            }
        }
    }
    fclose(f);
    if (!ok) { orc_free(ix); return NULL; }
    index_positions(ix);
    if (X) {
        double *xc = malloc(sizeof(double) * D), *o = malloc(sizeof(double) * d);
        double *xp = malloc(sizeof(double) * d);
        const double h = (double)((1 << B) - 1) / 2.0;
        for (int j = 0; j < nlist; j++) {
            const double *c = ix->C + (int64_t)j * d;
            for (int64_t p = ix->off[j]; p < ix->off[j + 1]; p++) {
                const float *x = X + ix->lid[p] * D;
                double a = 0.0, q2 = 0.0, n2 = 0.0;
                for (int i = 0; i < D; i++) { xc[i] = x[i] - ix->mu[i]; a += xc[i] * xc[i]; }
                for (int r = 0; r < d; r++) {
                    double s = 0.0;
                    for (int i = 0; i < D; i++) s += ix->Pp[(size_t)r * D + i] * xc[i];
                    ix->xd[p * d + r] = s;
                    q2 += s * s;
                    o[r] = s - c[r];
                    n2 += o[r] * o[r];
                }
                ix->ax[p] = a;
                ix->tx[p] = d == D ? 0.0 : a - q2;
                double nx = sqrt(n2);
                ix->nx[p] = nx;
                const uint8_t *u = ix->code + p * d;
                double y2 = 0.0;
                for (int r = 0; r < d; r++) y2 += (u[r] - h) * (u[r] - h);
                ix->yn[p] = sqrt(y2);
                if (nx == 0.0) { ix->xi1[p] = 1.0; ix->xiB[p] = 1.0; continue; }
                for (int r = 0; r < d; r++) {
                    double s = 0.0;
                    for (int i = 0; i < d; i++) s += ix->Pr[i * d + r] * o[i];
                    xp[r] = s / nx;
                }
                double s1 = 0.0, sb = 0.0;
                for (int r = 0; r < d; r++) {
                    int sign = (u[r] >> (B - 1)) & 1;
                    s1 += (sign ? 1.0 : -1.0) * xp[r];
                    sb += (u[r] - h) * xp[r];
                }
                ix->xi1[p] = s1 / sqrt((double)d);
                ix->xiB[p] = sb / ix->yn[p];
            }
        }
        free(xc); free(o); free(xp);
    }
    return ix;
}

/* Give an index imported without X the caller-owned original vectors (exact distances only). */
int orc_attach(orc_index *ix, const float *X, int64_t N, int32_t D) {
    if (!ix || N != ix->N || D != ix->D) return -1;
    ix->X = X;
    return 0;
}

int orc_info(const orc_index *ix, int64_t *N, int32_t *D, int32_t *d, int32_t *B, int32_t *nlist) {
    if (!ix) return -1;
    *N = ix->N; *D = ix->D; *d = ix->d; *B = ix->B; *nlist = ix->nlist;
    return 0;
}

int orc_get(const orc_index *ix, const char *name, void *out) {
    const int64_t N = ix->N, D = ix->D, d = ix->d, L = ix->nlist;
    struct { const char *n; const void *p; size_t bytes; } t[] = {
        {"mu", ix->mu, sizeof(double) * D},      {"Pp", ix->Pp, sizeof(double) * D * D},
        {"lam", ix->lam, sizeof(double) * D},    {"Pr", ix->Pr, sizeof(double) * d * d},
        {"C", ix->C, sizeof(double) * L * d},    {"off", ix->off, sizeof(int64_t) * (L + 1)},
        {"lid", ix->lid, sizeof(int64_t) * N},   {"code", ix->code, (size_t)(N * d)},
        {"xd", ix->xd, sizeof(double) * N * d},  {"nx", ix->nx, sizeof(double) * N},
        {"tx", ix->tx, sizeof(double) * N},      {"ax", ix->ax, sizeof(double) * N},
        {"xi1", ix->xi1, sizeof(double) * N},    {"xiB", ix->xiB, sizeof(double) * N},
        {"yn", ix->yn, sizeof(double) * N},
        {"sq_lo", ix->sq_lo, sizeof(float) * d},  {"sq_delta", ix->sq_delta, sizeof(float) * d},
        {"sq_code", ix->sq_code, (size_t)(N * d)},
    };
    for (size_t i = 0; i < sizeof(t) / sizeof(t[0]); i++)
        if (strcmp(t[i].n, name) == 0) {
            if (!t[i].p) return -1;
            memcpy(out, t[i].p, t[i].bytes);
            return 0;
        }
    return -1;
}

/* ------------------------------------------------------------------------------------------------ */
/* Query side.                                                                                      */

typedef struct {
    double *qp;     /* D: q_p = P_p (q - mu) */
    double qn2;     /* ||q_p||^2 */
    double Tq;      /* ||q_r||^2 */
    double sq;      /* sigma of Eq 6 */
    double er;      /* eps_r = 2 m sigma (R9) */
} qstate;

static void query_state(const orc_index *ix, const float *q, double m, qstate *s) {
    const int D = ix->D, d = ix->d;
    double *qc = malloc(sizeof(double) * D);
    for (int i = 0; i < D; i++) qc[i] = (double)q[i] - ix->mu[i];
    s->qn2 = 0.0; s->Tq = 0.0;
    double var = 0.0;
    for (int r = 0; r < D; r++) {
        double v = 0.0;
        for (int i = 0; i < D; i++) v += ix->Pp[(size_t)r * D + i] * qc[i];
        s->qp[r] = v;
        s->qn2 += v * v;
        /* Eq 6: sigma_i^2 = lambda_i is a variance; round-off below zero counts as 0 (R18) */
        if (r >= d) { s->Tq += v * v; var += (ix->lam[r] > 0.0 ? ix->lam[r] : 0.0) * v * v; }
    }
    s->sq = sqrt(var);
    s->er = 2.0 * m * s->sq;
    free(qc);
}

typedef struct { double g; int32_t j; } gent;
static int cmp_gent(const void *a, const void *b) {
    const gent *x = a, *y = b;
    if (x->g < y->g) return -1;
    if (x->g > y->g) return 1;
    return x->j < y->j ? -1 : (x->j > y->j);
}

/* Algorithm 2, centroid ranking: the nprobe lists nearest to q_d (ties -> smaller id, R12). */
static void rank_lists(const orc_index *ix, const double *qd, int32_t nprobe, int32_t *lists, double *g) {
    gent *e = malloc(sizeof(gent) * ix->nlist);
    for (int j = 0; j < ix->nlist; j++) {
        e[j].g = sqdist(qd, ix->C + (int64_t)j * ix->d, ix->d);
        e[j].j = j;
    }
    qsort(e, ix->nlist, sizeof(gent), cmp_gent);
    for (int r = 0; r < nprobe; r++) { lists[r] = e[r].j; if (g) g[r] = e[r].g; }
    free(e);
}

int orc_probe(const orc_index *ix, const float *q, int32_t nprobe, int32_t *lists, double *g) {
    if (nprobe < 1 || nprobe > ix->nlist) return -1;
    qstate s;
    s.qp = malloc(sizeof(double) * ix->D);
    query_state(ix, q, 0.0, &s);
    rank_lists(ix, s.qp, nprobe, lists, g);
    free(s.qp);
    return 0;
}

/* Per-pair query code: n_q, q' and its quantisation (R4, R5, R7). */
typedef struct {
    double nq;
    double *qprime;  /* d */
    uint8_t *u;      /* d */
    float vl, delta;
    int32_t su;
    double *qbar;    /* d: v_l + Delta u_i */
} pstate;

static void pair_state(const orc_index *ix, const double *qd, int32_t j, int bq, pstate *ps) {
    const int d = ix->d;
    const double *c = ix->C + (int64_t)j * d;
    double *w = malloc(sizeof(double) * d);
    float *qf = calloc(d, sizeof(float));
    double n2 = 0.0;
    for (int i = 0; i < d; i++) { w[i] = qd[i] - c[i]; n2 += w[i] * w[i]; }
    ps->nq = sqrt(n2);
    for (int r = 0; r < d; r++) {
        double s = 0.0;
        for (int i = 0; i < d; i++) s += ix->Pr[i * d + r] * w[i];
        ps->qprime[r] = ps->nq > 0.0 ? s / ps->nq : 0.0;
        qf[r] = (float)ps->qprime[r];
    }
    orc_quantize_query_f32(qf, d, bq, ps->u, &ps->vl, &ps->delta, &ps->su);
    for (int i = 0; i < d; i++) ps->qbar[i] = (double)ps->vl + (double)ps->delta * (double)ps->u[i];
    free(w); free(qf);
}

/* Stage values of one candidate (Eq 4, Eq 5 with R8, Eq 7). */
typedef struct {
    double dis1, eb1, lb1;   /* 1-bit estimate, its error radius, lower bound */
    double disB, ebB, lbB;   /* B-bit estimate (== 1-bit values when B == 1) */
    double diso;             /* Eq 7 projected distance */
    double ip, pc;           /* sum_i b_i u_i and sum_i b_i (sign plane) */
} cstate;

static void cand_state(const orc_index *ix, int64_t p, const qstate *qs, const pstate *ps,
                       double eps0, cstate *cs) {
    const int d = ix->d, B = ix->B;
    const uint8_t *u = ix->code + p * d;
    const double h = (double)((1 << B) - 1) / 2.0;
    double s1 = 0.0, sB = 0.0, ip = 0.0, pc = 0.0;
    for (int i = 0; i < d; i++) {
        int b = (u[i] >> (B - 1)) & 1;
        s1 += (b ? 1.0 : -1.0) * ps->qbar[i];     /* sqrt(d) <xbar_b, qbar> */
        sB += ((double)u[i] - h) * ps->qbar[i];   /* <y, qbar> */
        ip += b * (double)ps->u[i];
        pc += b;
    }
    const double nx = ix->nx[p], nq = ps->nq, sd = sqrt((double)d), rt = eps0 / sqrt((double)(d - 1));
    const double C1 = nx * nx + ix->tx[p] + nq * nq + qs->Tq;
    double est1 = s1 / (sd * ix->xi1[p]);
    double estB = sB / (ix->yn[p] * ix->xiB[p]);
    cs->dis1 = C1 - 2.0 * nx * nq * est1;
    cs->eb1 = 2.0 * nx * nq * sqrt(fmax(0.0, 1.0 - ix->xi1[p] * ix->xi1[p])) / ix->xi1[p] * rt;
    cs->lb1 = cs->dis1 - cs->eb1 - qs->er;
    cs->disB = C1 - 2.0 * nx * nq * estB;
    cs->ebB = 2.0 * nx * nq * sqrt(fmax(0.0, 1.0 - ix->xiB[p] * ix->xiB[p])) / ix->xiB[p] * rt;
    cs->lbB = cs->disB - cs->ebB - qs->er;
    double dot = 0.0;
    for (int i = 0; i < d; i++) dot += ix->xd[p * d + i] * qs->qp[i];
    cs->diso = ix->ax[p] + qs->qn2 - 2.0 * dot;
    cs->ip = ip;
    cs->pc = pc;
}

static double exact_dist(const orc_index *ix, int64_t id, const float *q) {
    const float *x = ix->X + id * ix->D;
    double s = 0.0;
    for (int i = 0; i < ix->D; i++) { double t = (double)x[i] - (double)q[i]; s += t * t; }
    return s;
}

/* Sorted result queue of at most k (dis, id) pairs (Algorithm 2's result queue; R11). */
typedef struct { double *dis; int64_t *id; int n, k; } topk;

static int key_less(double da, int64_t ia, double db, int64_t ib) {
    return da < db || (da == db && ia < ib);
}

static void topk_push(topk *t, double dis, int64_t id) {
    if (t->n == t->k && !key_less(dis, id, t->dis[t->n - 1], t->id[t->n - 1])) return;
    int pos = t->n < t->k ? t->n : t->k - 1;
    while (pos > 0 && key_less(dis, id, t->dis[pos - 1], t->id[pos - 1])) {
        t->dis[pos] = t->dis[pos - 1];
        t->id[pos] = t->id[pos - 1];
        pos--;
    }
    t->dis[pos] = dis;
    t->id[pos] = id;
    if (t->n < t->k) t->n++;
}

static double topk_tau(const topk *t) { return t->n < t->k ? INFINITY : t->dis[t->k - 1]; }

int orc_search(const orc_index *ix, const float *q, int32_t k, int32_t nprobe, const orc_params *p,
               int32_t mode, int64_t *ids, double *dists, orc_counters *cnt) {
    if (!ix || !ix->X || k < 1 || nprobe < 1 || nprobe > ix->nlist) return -1;
    const int d = ix->d, D = ix->D;
    qstate qs;
    qs.qp = malloc(sizeof(double) * D);
    query_state(ix, q, p->m, &qs);
    int32_t *lists = malloc(sizeof(int32_t) * nprobe);
    rank_lists(ix, qs.qp, nprobe, lists, NULL);
    pstate ps;
    ps.qprime = malloc(sizeof(double) * d);
    ps.u = malloc(d);
    ps.qbar = malloc(sizeof(double) * d);
    topk t = {malloc(sizeof(double) * k), malloc(sizeof(int64_t) * k), 0, k};
    orc_counters c = {0, 0, 0, 0, 0, 0, 0};
    const int verify = p->verify && cnt != NULL;
    for (int r = 0; r < nprobe; r++) {
        const int32_t j = lists[r];
        if (mode == ORC_ALG2) pair_state(ix, qs.qp, j, p->bq, &ps);
        for (int64_t pos = ix->off[j]; pos < ix->off[j + 1]; pos++) {
            const int64_t id = ix->lid[pos];
            c.scanned++;
            if (mode == ORC_EXACT_IVF) { topk_push(&t, exact_dist(ix, id, q), id); continue; }
            cstate cs;
            cand_state(ix, pos, &qs, &ps, p->eps0, &cs);
            if (verify) {
                double dx = exact_dist(ix, id, q);
                if (cs.lb1 > dx) c.viol1++;
                if (ix->B > 1 && p->use_ext && cs.lbB > dx) c.viol_ext++;
                if (cs.diso - qs.er > dx) c.viol2++;
            }
            const double tau = topk_tau(&t);
            if (!(cs.lb1 < tau)) continue;
            c.pass1++;
            if (ix->B > 1 && p->use_ext && !(cs.lbB < tau)) continue;
            c.pass_ext++;
            if (p->stage2 && !(cs.diso - qs.er < tau)) continue;
            c.pass2++;
            topk_push(&t, exact_dist(ix, id, q), id);
        }
    }
    for (int i = 0; i < k; i++) {
        ids[i] = i < t.n ? t.id[i] : -1;
        dists[i] = i < t.n ? t.dis[i] : INFINITY;
    }
    if (cnt) *cnt = c;
    free(qs.qp); free(lists); free(ps.qprime); free(ps.u); free(ps.qbar); free(t.dis); free(t.id);
    return t.n;
}

/* Everything the search computes for one (query, list) pair, for element-wise comparison.
 * qscal: [n_q, T_q, eps_r, ||q_p||^2, v_l, Delta, S_u, sigma]; cand rows of 10:
 * [dis1, eb1, lb1, disB, ebB, lbB, diso, exact dis, ip, pc]. Returns the list length. */
int orc_pair_trace(const orc_index *ix, const float *q, int32_t list, const orc_params *p,
                   double *qscal, double *qprime, uint8_t *u, int64_t *ids, double *cand) {
    if (!ix || list < 0 || list >= ix->nlist) return -1;
    const int d = ix->d;
    qstate qs;
    qs.qp = malloc(sizeof(double) * ix->D);
    query_state(ix, q, p->m, &qs);
    pstate ps;
    ps.qprime = qprime;
    ps.u = u;
    ps.qbar = malloc(sizeof(double) * d);
    pair_state(ix, qs.qp, list, p->bq, &ps);
    qscal[0] = ps.nq; qscal[1] = qs.Tq; qscal[2] = qs.er; qscal[3] = qs.qn2;
    qscal[4] = ps.vl; qscal[5] = ps.delta; qscal[6] = ps.su; qscal[7] = qs.sq;
    int n = 0;
    for (int64_t pos = ix->off[list]; pos < ix->off[list + 1]; pos++, n++) {
        cstate cs;
        cand_state(ix, pos, &qs, &ps, p->eps0, &cs);
        ids[n] = ix->lid[pos];
        double *row = cand + (int64_t)n * 10;
        row[0] = cs.dis1; row[1] = cs.eb1; row[2] = cs.lb1;
        row[3] = cs.disB; row[4] = cs.ebB; row[5] = cs.lbB;
        row[6] = cs.diso;
        row[7] = ix->X ? exact_dist(ix, ids[n], q) : NAN;
        row[8] = cs.ip; row[9] = cs.pc;
    }
    free(qs.qp); free(ps.qbar);
    return n;
}

/* EXACT-IVF top-k plus, for each member, whether a pruning test could drop it: bit 1 = stage-1
 * bound within `margin` of (or above) its exact distance, bit 2 = B-bit bound, bit 4 = stage 2.
 * Such members may be missed by any correct multi-stage search when its bounds fail. */
int orc_topk_risk(const orc_index *ix, const float *q, int32_t k, int32_t nprobe, const orc_params *p,
                  double margin, int64_t *ids, double *dists, uint8_t *risk) {
    int n = orc_search(ix, q, k, nprobe, p, ORC_EXACT_IVF, ids, dists, NULL);
    if (n < 0) return n;
    const int d = ix->d;
    qstate qs;
    qs.qp = malloc(sizeof(double) * ix->D);
    query_state(ix, q, p->m, &qs);
    pstate ps;
    ps.qprime = malloc(sizeof(double) * d);
    ps.u = malloc(d);
    ps.qbar = malloc(sizeof(double) * d);
    for (int i = 0; i < k; i++) {
        risk[i] = 0;
        if (ids[i] < 0) continue;
        const int64_t pos = ix->pos[ids[i]];
        /* the list holding position pos: the largest j with off[j] <= pos (every earlier list, empty or
         * not, also has off[j] <= pos, at a smaller index; a later list starts beyond pos) */
        int32_t list = 0;
        for (int32_t lo = 0, hi = ix->nlist - 1; lo <= hi;) {
            const int32_t mid = lo + (hi - lo) / 2;
            if (ix->off[mid] <= pos) { list = mid; lo = mid + 1; } else hi = mid - 1;
        }
        pair_state(ix, qs.qp, list, p->bq, &ps);
        cstate cs;
        cand_state(ix, pos, &qs, &ps, p->eps0, &cs);
        double thr = dists[i] - margin;
        if (cs.lb1 >= thr) risk[i] |= 1;
        if (ix->B > 1 && p->use_ext && cs.lbB >= thr) risk[i] |= 2;
        if (p->stage2 && cs.diso - qs.er >= thr) risk[i] |= 4;
    }
    free(qs.qp); free(ps.qprime); free(ps.u); free(ps.qbar);
    return n;
}

/* ------------------------------------------------------------------------------------------------ */
/* MR-SQ (S1-S4).                                                                                   */

/* S1, S2: the grid of each of the d coordinates from N rows (row stride ld) of FP32 values. */
void orc_sq8_range(const float *xd, int64_t N, int d, int ld, float *lo, float *delta) {
    for (int i = 0; i < d; i++) {
        float a = xd[i], b = xd[i];
        for (int64_t n = 1; n < N; n++) {
            float v = xd[n * ld + i];
            if (v < a) a = v;
            if (v > b) b = v;
        }
        lo[i] = a;
        delta[i] = b > a ? (b - a) / 255.0f : 1.0f;
    }
}

/* S2: the 8-bit code of one row (FP32 steps; -ffp-contract=off keeps them separate roundings). */
void orc_sq8_encode(const float *x, int d, const float *lo, const float *delta, uint8_t *u) {
    for (int i = 0; i < d; i++) {
        const float inv = 1.0f / delta[i];
        const float t = (x[i] - lo[i]) * inv + 0.5f;
        float fl = floorf(t);
        int v = (int)fl;
        u[i] = (uint8_t)(v < 0 ? 0 : (v > 255 ? 255 : v));
    }
}

/* MR-SQ codes of an index from its own leading coordinates x_d (rounded to FP32). */
int orc_sq8_build(orc_index *ix) {
    const int64_t N = ix->N;
    const int d = ix->d;
    float *xf = malloc(sizeof(float) * (size_t)N * d);
    free(ix->sq_lo); free(ix->sq_delta); free(ix->sq_code);
    ix->sq_lo = malloc(sizeof(float) * d);
    ix->sq_delta = malloc(sizeof(float) * d);
    ix->sq_code = malloc((size_t)N * d);
    if (!xf || !ix->sq_lo || !ix->sq_delta || !ix->sq_code) { free(xf); return -1; }
    for (int64_t i = 0; i < N * d; i++) xf[i] = (float)ix->xd[i];
    orc_sq8_range(xf, N, d, d, ix->sq_lo, ix->sq_delta);
    for (int64_t p = 0; p < N; p++) orc_sq8_encode(xf + p * d, d, ix->sq_lo, ix->sq_delta, ix->sq_code + p * d);
    free(xf);
    return 0;
}

/* S3 for every candidate of the nprobe probed lists (lists nearest first, R12), FP64: ids, estimates
 * and (with X attached) exact distances.  Returns the number of candidates, or -1. */
int orc_mrsq_estimates(const orc_index *ix, const float *q, int32_t nprobe, int64_t *ids, double *est,
                       double *exact) {
    if (!ix || !ix->sq_code || nprobe < 1 || nprobe > ix->nlist) return -1;
    const int d = ix->d;
    qstate qs;
    qs.qp = malloc(sizeof(double) * ix->D);
    query_state(ix, q, 0.0, &qs);
    int32_t *lists = malloc(sizeof(int32_t) * nprobe);
    rank_lists(ix, qs.qp, nprobe, lists, NULL);
    int n = 0;
    for (int r = 0; r < nprobe; r++) {
        const int32_t j = lists[r];
        for (int64_t pos = ix->off[j]; pos < ix->off[j + 1]; pos++, n++) {
            const uint8_t *u = ix->sq_code + pos * d;
            double s = 0.0;
            for (int i = 0; i < d; i++) {
                const double xh = (double)ix->sq_lo[i] + (double)ix->sq_delta[i] * (double)u[i];
                const double t = xh - qs.qp[i];
                s += t * t;
            }
            ids[n] = ix->lid[pos];
            est[n] = s + ix->tx[pos] + qs.Tq;
            if (exact) exact[n] = ix->X ? exact_dist(ix, ids[n], q) : NAN;
        }
    }
    free(qs.qp); free(lists);
    return n;
}

typedef struct { double e; int64_t id; } eent;
static int cmp_eent(const void *a, const void *b) {
    const eent *x = a, *y = b;
    if (x->e < y->e) return -1;
    if (x->e > y->e) return 1;
    return x->id < y->id ? -1 : (x->id > y->id);
}

/* S4: MR-SQ search of one query; returns the number of results (<= k), or -1. */
int orc_mrsq_search(const orc_index *ix, const float *q, int32_t k, int32_t nprobe, int32_t R, int64_t *ids,
                    double *dists) {
    if (!ix || !ix->X || !ix->sq_code || k < 1 || R < k || nprobe < 1 || nprobe > ix->nlist) return -1;
    int64_t cap = 0;
    {
        int32_t *lists = malloc(sizeof(int32_t) * nprobe);
        if (orc_probe(ix, q, nprobe, lists, NULL) != 0) { free(lists); return -1; }
        for (int r = 0; r < nprobe; r++) cap += ix->off[lists[r] + 1] - ix->off[lists[r]];
        free(lists);
    }
    int64_t *cid = malloc(sizeof(int64_t) * (cap ? cap : 1));
    double *ce = malloc(sizeof(double) * (cap ? cap : 1));
    const int n = orc_mrsq_estimates(ix, q, nprobe, cid, ce, NULL);
    eent *e = malloc(sizeof(eent) * (n ? n : 1));
    for (int i = 0; i < n; i++) { e[i].e = ce[i]; e[i].id = cid[i]; }
    qsort(e, n, sizeof(eent), cmp_eent);
    topk t = {malloc(sizeof(double) * k), malloc(sizeof(int64_t) * k), 0, k};
    const int take = n < R ? n : R;
    for (int i = 0; i < take; i++) topk_push(&t, exact_dist(ix, e[i].id, q), e[i].id);
    for (int i = 0; i < k; i++) {
        ids[i] = i < t.n ? t.id[i] : -1;
        dists[i] = i < t.n ? t.dis[i] : INFINITY;
    }
    const int got = t.n;
    free(cid); free(ce); free(e); free(t.dis); free(t.id);
    return got;
}

/* Exact k-NN over the whole set (Section 2.1 problem statement), FP64, ties -> smaller id. */
void orc_bruteforce(const float *X, int64_t N, int32_t D, const float *Q, int64_t nq, int32_t k,
                    int64_t *ids, double *dists) {
    topk t = {malloc(sizeof(double) * k), malloc(sizeof(int64_t) * k), 0, k};
    for (int64_t qi = 0; qi < nq; qi++) {
        t.n = 0;
        const float *q = Q + qi * D;
        for (int64_t n = 0; n < N; n++) {
            double s = 0.0;
            const float *x = X + n * D;
            for (int i = 0; i < D; i++) { double v = (double)x[i] - (double)q[i]; s += v * v; }
            topk_push(&t, s, n);
        }
        for (int i = 0; i < k; i++) {
            ids[qi * k + i] = i < t.n ? t.id[i] : -1;
            dists[qi * k + i] = i < t.n ? t.dis[i] : INFINITY;
        }
    }
    free(t.dis); free(t.id);
}
