// Build-side kernels of the MRQ index (Algorithm 1 of arXiv 2411.06158) for gfx950: FP64 mean and
// covariance for the PCA, FP64 per-vector norms, k-means on the leading coordinates, the list-major
// layout, and the per-vector codes and normalisation factors (FP64) of Section 4.2.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>

#include "mrq_internal.h"

namespace mrq {

namespace {
__device__ __forceinline__ double wave_sum_d(double v) {
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ __forceinline__ int wave_sum_int(int v) {
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
}  // namespace

// ------------------------------------------------------------------------------------------------
// Mean (Algorithm 1, PCA training): per-chunk column sums, then a fixed-order sum of the chunks.

__global__ void k_colsum(const float* __restrict__ X, int64_t N, int D, int64_t rpc, double* __restrict__ part) {
    const int col = blockIdx.x * 256 + threadIdx.x;
    const int64_t ch = blockIdx.y;
    if (col >= D) return;
    const int64_t r0 = ch * rpc, r1 = r0 + rpc < N ? r0 + rpc : N;
    double s = 0.0;
    for (int64_t r = r0; r < r1; r++) s += (double)X[r * D + col];
    part[ch * D + col] = s;
}

__global__ void k_colmean(const double* __restrict__ part, int nchunk, int D, int64_t N, double* __restrict__ mu) {
    const int col = blockIdx.x * 256 + threadIdx.x;
    if (col >= D) return;
    double s = 0.0;
    for (int c = 0; c < nchunk; c++) s += part[(int64_t)c * D + col];
    mu[col] = s / (double)N;
}

hipError_t launch_colmean(const float* X, int64_t N, int D, double* part, int nchunk, double* mu64,
                          hipStream_t s) {
    const int64_t rpc = (N + nchunk - 1) / nchunk;
    hipLaunchKernelGGL(k_colsum, dim3((D + 255) / 256, nchunk), dim3(256), 0, s, X, N, D, rpc, part);
    hipLaunchKernelGGL(k_colmean, dim3((D + 255) / 256), dim3(256), 0, s, part, nchunk, D, N, mu64);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------------
// Covariance Sigma = (1/N) sum (x - mu)(x - mu)^T in FP64: 64 x 64 tiles of the upper triangle, the
// rows split into `nsplit` ranges whose partial sums are added in a fixed order afterwards.

__global__ __launch_bounds__(256) void k_cov_tile(const float* __restrict__ X, int64_t N, int D,
                                                  const double* __restrict__ mu, int64_t rps, int ntd,
                                                  double* __restrict__ part) {
    __shared__ double As[16][64];
    __shared__ double Bs[16][64];
    int tix = blockIdx.x, ti = 0;
    while (tix >= ntd - ti) { tix -= ntd - ti; ti++; }
    const int tj = ti + tix;
    const int64_t split = blockIdx.y;
    const int64_t r0 = split * rps, r1 = r0 + rps < N ? r0 + rps : N;
    const int t = threadIdx.x, tx = t & 15, ty = t >> 4;
    double acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int j = 0; j < 4; j++) acc[i][j] = 0.0;
    for (int64_t rb = r0; rb < r1; rb += 16) {
        // 16 rows x 64 columns for each operand: 1024 values, 4 per thread
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int e = t + 256 * u;
            const int rr = e >> 6, cc = e & 63;
            const int64_t r = rb + rr;
            const int ca = ti * 64 + cc, cb = tj * 64 + cc;
            double va = 0.0, vb = 0.0;
            if (r < r1) {
                if (ca < D) va = (double)X[r * D + ca] - mu[ca];
                if (cb < D) vb = (double)X[r * D + cb] - mu[cb];
            }
            As[rr][cc] = va;
            Bs[rr][cc] = vb;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; kk++) {
            double a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; i++) { a[i] = As[kk][ty * 4 + i]; b[i] = Bs[kk][tx * 4 + i]; }
#pragma unroll
            for (int i = 0; i < 4; i++)
#pragma unroll
                for (int j = 0; j < 4; j++) acc[i][j] = fma(a[i], b[j], acc[i][j]);
        }
        __syncthreads();
    }
    double* P = part + split * (int64_t)D * D;
#pragma unroll
    for (int i = 0; i < 4; i++) {
        const int gi = ti * 64 + ty * 4 + i;
        if (gi >= D) continue;
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int gj = tj * 64 + tx * 4 + j;
            if (gj < D) P[(int64_t)gi * D + gj] = acc[i][j];
        }
    }
}

__global__ void k_cov_final(const double* __restrict__ part, int nsplit, int D, int64_t N, double* __restrict__ S) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= (int64_t)D * D) return;
    int i = (int)(e / D), j = (int)(e % D);
    if (i / 64 > j / 64) { int t = i; i = j; j = t; }  // lower-triangle tiles mirror the upper ones
    double s = 0.0;
    for (int sp = 0; sp < nsplit; sp++) s += part[(int64_t)sp * D * D + (int64_t)i * D + j];
    S[e] = s / (double)N;
}

int cov_splits(int64_t N, int D) {
    const int ntd = (D + 63) / 64;
    const int ntiles = ntd * (ntd + 1) / 2;
    int ns = 2048 / ntiles;
    if (ns < 1) ns = 1;
    if (ns > 256) ns = 256;
    if (ns > (N + 63) / 64) ns = (int)((N + 63) / 64);
    return ns < 1 ? 1 : ns;
}

hipError_t launch_cov(const float* X, int64_t N, int D, const double* mu64, double* part, int nsplit,
                      double* S, hipStream_t s) {
    const int ntd = (D + 63) / 64;
    const int ntiles = ntd * (ntd + 1) / 2;
    const int64_t rps = (N + nsplit - 1) / nsplit;
    hipLaunchKernelGGL(k_cov_tile, dim3(ntiles, nsplit), dim3(256), 0, s, X, N, D, mu64, rps, ntd, part);
    const int64_t tot = (int64_t)D * D;
    hipLaunchKernelGGL(k_cov_final, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, part, nsplit, D, N, S);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------------
// Per-vector ||x - mu||^2 and ||x_r||^2 = ||x - mu||^2 - ||x_d||^2 in FP64 (Algorithm 1, residual
// norms; the rotation is orthogonal so the tail norm needs no tail coordinates).

__global__ __launch_bounds__(256) void k_rownorms(const float* __restrict__ X, int64_t N, int D,
                                                  const double* __restrict__ mu, const float* __restrict__ xd,
                                                  int d4, int d, double* __restrict__ ax, double* __restrict__ tx) {
    const int64_t r = blockIdx.x * 4ll + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (r >= N) return;
    double a = 0.0, b = 0.0;
    for (int i = lane; i < D; i += 64) { double v = (double)X[r * D + i] - mu[i]; a += v * v; }
    for (int i = lane; i < d; i += 64) { double v = (double)xd[r * d4 + i]; b += v * v; }
    a = wave_sum_d(a);
    b = wave_sum_d(b);
    if (lane == 0) {
        ax[r] = a;
        tx[r] = d == D ? 0.0 : (a - b > 0.0 ? a - b : 0.0);
    }
}

hipError_t launch_rownorms(const float* X, int64_t N, int D, const double* mu64, const float* xd, int d4,
                           int d, double* ax64, double* tx64, hipStream_t s) {
    hipLaunchKernelGGL(k_rownorms, dim3((unsigned)((N + 3) / 4)), dim3(256), 0, s, X, N, D, mu64, xd, d4, d,
                       ax64, tx64);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_sqnorms(const float* __restrict__ A, int64_t n, int lda, int dim,
                                                 float* __restrict__ out) {
    const int64_t r = blockIdx.x * 4ll + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (r >= n) return;
    float s = 0.f;
    for (int i = lane; i < dim; i += 64) { float v = A[r * lda + i]; s = fmaf(v, v, s); }
    for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) out[r] = s;
}

hipError_t launch_sqnorms(const float* A, int64_t n, int lda, int dim, float* out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sqnorms, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, A, n, lda, dim, out);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------------
// k-means on x_d (Algorithm 1, IVF training).  Assignment: argmin_j ||c_j||^2 - 2 <x, c_j> with ties
// to the smaller j, as a tiled FP32 product with the argmin folded in.

__global__ __launch_bounds__(256) void k_kmeans_assign(const float* __restrict__ P, int64_t n, int ldp, int dim,
                                                       const float* __restrict__ C, int ldc,
                                                       const float* __restrict__ cn2, int k,
                                                       const float* __restrict__ pn2,
                                                       int32_t* __restrict__ assign, float* __restrict__ mind) {
    __shared__ float As[16][68];
    __shared__ float Bs[16][68];
    const int t = threadIdx.x, tx = t & 15, ty = t >> 4;
    const int64_t m0 = (int64_t)blockIdx.x * 64;
    float best[4];
    int bidx[4];
#pragma unroll
    for (int i = 0; i < 4; i++) { best[i] = FLT_MAX; bidx[i] = 0x7fffffff; }
    const int lr = t >> 2, lk = (t & 3) * 4;
    for (int c0 = 0; c0 < k; c0 += 64) {
        float acc[4][4];
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
            for (int j = 0; j < 4; j++) acc[i][j] = 0.f;
        for (int k0 = 0; k0 < dim; k0 += 16) {
#pragma unroll
            for (int u = 0; u < 4; u++) {
                const int kk = k0 + lk + u;
                const int64_t mr = m0 + lr;
                As[lk + u][lr] = (mr < n && kk < dim) ? P[mr * ldp + kk] : 0.f;
                const int cr = c0 + lr;
                Bs[lk + u][lr] = (cr < k && kk < dim) ? C[(int64_t)cr * ldc + kk] : 0.f;
            }
            __syncthreads();
#pragma unroll
            for (int kk = 0; kk < 16; kk++) {
                float4 a = *reinterpret_cast<const float4*>(&As[kk][ty * 4]);
                float4 b = *reinterpret_cast<const float4*>(&Bs[kk][tx * 4]);
                float av[4] = {a.x, a.y, a.z, a.w}, bv[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
                for (int i = 0; i < 4; i++)
#pragma unroll
                    for (int j = 0; j < 4; j++) acc[i][j] = fmaf(av[i], bv[j], acc[i][j]);
            }
            __syncthreads();
        }
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int cj = c0 + tx * 4 + j;
            if (cj >= k) continue;
            const float cn = cn2[cj];
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const float v = fmaf(-2.f, acc[i][j], cn);
                if (v < best[i] || (v == best[i] && cj < bidx[i])) { best[i] = v; bidx[i] = cj; }
            }
        }
    }
#pragma unroll
    for (int i = 0; i < 4; i++) {
        for (int o = 8; o >= 1; o >>= 1) {
            const float ov = __shfl_xor(best[i], o);
            const int oi = __shfl_xor(bidx[i], o);
            if (ov < best[i] || (ov == best[i] && oi < bidx[i])) { best[i] = ov; bidx[i] = oi; }
        }
        const int64_t m = m0 + ty * 4 + i;
        if (tx == 0 && m < n) {
            assign[m] = bidx[i];
            if (mind) mind[m] = best[i] + pn2[m];
        }
    }
}

hipError_t launch_kmeans_assign(const float* P, int64_t n, int ldp, int dim, const float* C, int ldc,
                                const float* cn2, int k, const float* pn2, int32_t* assign, float* mind,
                                hipStream_t s) {
    hipLaunchKernelGGL(k_kmeans_assign, dim3((unsigned)((n + 63) / 64)), dim3(256), 0, s, P, n, ldp, dim, C,
                       ldc, cn2, k, pn2, assign, mind);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_kmeans_accum(const float* __restrict__ P, int64_t n, int ldp, int dim,
                                                      const int32_t* __restrict__ assign,
                                                      const int32_t* __restrict__ prev, double* __restrict__ sums,
                                                      int32_t* __restrict__ cnt, int32_t* __restrict__ changed) {
    const int64_t r = blockIdx.x * 4ll + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (r >= n) return;
    const int a = assign[r];
    for (int i = lane; i < dim; i += 64) atomicAdd(&sums[(int64_t)a * dim + i], (double)P[r * ldp + i]);
    if (lane == 0) {
        atomicAdd(&cnt[a], 1);
        if (prev && prev[r] != a) atomicAdd(changed, 1);
    }
}

hipError_t launch_kmeans_accum(const float* P, int64_t n, int ldp, int dim, const int32_t* assign,
                               const int32_t* prev, double* sums, int32_t* cnt, int32_t* changed,
                               hipStream_t s) {
    hipLaunchKernelGGL(k_kmeans_accum, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, P, n, ldp, dim, assign,
                       prev, sums, cnt, changed);
    return hipGetLastError();
}

__global__ void k_kmeans_centroids(const double* __restrict__ sums, const int32_t* __restrict__ cnt, int k,
                                   int dim, float* __restrict__ C, int ldc, float* __restrict__ cn2) {
    const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (j >= k) return;
    const int c = cnt[j];
    float s = 0.f;
    for (int i = lane; i < dim; i += 64) {
        float v = C[(int64_t)j * ldc + i];
        if (c > 0) {
            v = (float)(sums[(int64_t)j * dim + i] / (double)c);
            C[(int64_t)j * ldc + i] = v;
        }
        s = fmaf(v, v, s);
    }
    for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) cn2[j] = s;
}

hipError_t launch_kmeans_centroids(const double* sums, const int32_t* cnt, int k, int dim, float* C, int ldc,
                                   float* cn2, hipStream_t s) {
    hipLaunchKernelGGL(k_kmeans_centroids, dim3((k + 3) / 4), dim3(256), 0, s, sums, cnt, k, dim, C, ldc, cn2);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------------
// List-major layout: row r of the index holds vector perm[r] (or padding when perm[r] < 0).

__global__ __launch_bounds__(256) void k_gather_layout(
    const float* __restrict__ Xraw, int D, int D4, const int32_t* __restrict__ perm, int64_t Npad,
    const float* __restrict__ xd_id, int d, int d4, const double* __restrict__ ax64,
    const double* __restrict__ tx64, const int64_t* __restrict__ list_off, int nlist,
    const float* __restrict__ C, float* __restrict__ Xl, float* __restrict__ xdl, float* __restrict__ axl,
    double* __restrict__ txr, int32_t* __restrict__ ids, int32_t* __restrict__ row_list, float* __restrict__ O,
    const float* __restrict__ xt_id, int Dr, int Dr4, float* __restrict__ xrl) {
    const int64_t r = blockIdx.x * 4ll + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (r >= Npad) return;
    const int id = perm[r];
    int lo = 0, hi = nlist - 1;  // list of row r: last j with list_off[j] <= r
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (list_off[mid] <= r) lo = mid; else hi = mid - 1;
    }
    const int j = lo;
    // the original vector, zero padded to D4 (the exact stage computes ||x - q||^2 = ||x_p - q_p||^2 from
    // it, so no projection rounding enters the exact distances)
    for (int i = lane; i < D4; i += 64) Xl[r * D4 + i] = (id >= 0 && i < D) ? Xraw[(int64_t)id * D + i] : 0.f;
    // the tail coordinates of x_p (split exact stage), zero padded to Dr4
    if (xrl)
        for (int i = lane; i < Dr4; i += 64) xrl[r * Dr4 + i] = (id >= 0 && i < Dr) ? xt_id[(int64_t)id * Dr + i] : 0.f;
    for (int i = lane; i < d4; i += 64) {
        float v = (id >= 0 && i < d) ? xd_id[(int64_t)id * d4 + i] : 0.f;
        xdl[r * d4 + i] = v;
        O[r * d4 + i] = (id >= 0 && i < d) ? v - C[(int64_t)j * d4 + i] : 0.f;
    }
    if (lane == 0) {
        ids[r] = id;
        axl[r] = id >= 0 ? (float)ax64[id] : 0.f;
        txr[r] = id >= 0 ? tx64[id] : 0.0;
        row_list[r] = j;
    }
}

hipError_t launch_gather_layout(const Index& ix, const float* Xraw, const int32_t* perm, const float* xd_id,
                                const double* ax64, const double* tx64, double* txr, int32_t* row_list, float* O,
                                const float* xt_id, hipStream_t s) {
    hipLaunchKernelGGL(k_gather_layout, dim3((unsigned)((ix.Npad + 3) / 4)), dim3(256), 0, s, Xraw, ix.D, ix.D4,
                       perm, ix.Npad, xd_id, ix.d, ix.d4, ax64, tx64, ix.list_off, ix.nlist, ix.C, ix.X, ix.xd,
                       ix.ax, txr, ix.ids, row_list, O, xt_id, ix.Dr, ix.Dr4, ix.xr);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------------
// Codes and factors (Section 4.2; Algorithm 1, last two steps), one wave per row:
//   o = x_d - c, n_x = ||o|| (FP64), x'' = P_r^T o (FP32 product), x' = x'' / n_x,
//   sign bits b_i = [x'_i >= 0], xi1 = sum |x'_i| / sqrt(d),
//   B > 1: the level vector y_i = s_i (m_i + 1/2) with m_i = min(2^(B-1) - 1, floor(t |x'_i|)) at the
//   scale t of largest <y, x'>/||y|| among every scale where some m_i steps (ties -> smaller t, then
//   smaller dimension), u_i = y_i + (2^B - 1)/2, xiB = <y, x'>/||y||.
// Factors are formed in FP64 and stored as FP32.

constexpr int kEncMaxD = 1536;

__global__ __launch_bounds__(64) void k_encode(const float* __restrict__ O, const float* __restrict__ Xpp,
                                               const double* __restrict__ txr, int64_t Npad, int d, int d4, int B,
                                               int WP, const int32_t* __restrict__ ids, uint32_t* __restrict__ code,
                                               uint32_t* __restrict__ ext, float* __restrict__ fA,
                                               float* __restrict__ fF, float* __restrict__ fE,
                                               float* __restrict__ fFB, float* __restrict__ fEB,
                                               float* __restrict__ fSX, float* __restrict__ nxo,
                                               float* __restrict__ txo, float* __restrict__ xi1o,
                                               float* __restrict__ xiBo, float* __restrict__ yno) {
    __shared__ double a_s[kEncMaxD];
    const int64_t r = blockIdx.x;
    const int lane = threadIdx.x;
    const int nh = (d + 63) / 64;
    uint32_t* cw = code + r * WP;
    const int id = ids[r];
    if (id < 0) {  // padding row: never passes (A = +inf), zero code
        for (int w = lane; w < WP; w += 64) cw[w] = 0u;
        if (B > 1)
            for (int w = lane; w < (B - 1) * WP; w += 64) ext[r * (B - 1) * WP + w] = 0u;
        if (lane == 0) {
            fA[r] = INFINITY; fF[r] = 0.f; fE[r] = 0.f; fFB[r] = 0.f; fEB[r] = 0.f; fSX[r] = 0.f;
            nxo[r] = 0.f; txo[r] = 0.f; xi1o[r] = 1.f; xiBo[r] = 1.f; yno[r] = 0.f;
        }
        return;
    }
    double so = 0.0;
    for (int h = 0; h < nh; h++) {
        const int i = lane + 64 * h;
        if (i < d) { double v = (double)O[r * d4 + i]; so += v * v; }
    }
    so = wave_sum_d(so);
    const double nx = sqrt(so);
    const double sd = sqrt((double)d);
    const double tx = txr[r];
    double sabs = 0.0;
    for (int h = 0; h < nh; h++) {
        const int i = lane + 64 * h;
        if (i < d) sabs += fabs((double)Xpp[r * d4 + i]);
    }
    sabs = wave_sum_d(sabs);
    const double xi1 = nx > 0.0 ? sabs / (sd * nx) : 1.0;
    // sign plane
    for (int h = 0; h < (WP + 1) / 2; h++) {
        const int i = lane + 64 * h;
        const bool bit = i < d && (nx == 0.0 || Xpp[r * d4 + (i < d ? i : 0)] >= 0.f);
        const unsigned long long bm = __ballot(bit);
        if (lane == 0) {
            if (2 * h < WP) cw[2 * h] = (uint32_t)bm;
            if (2 * h + 1 < WP) cw[2 * h + 1] = (uint32_t)(bm >> 32);
        }
    }
    const int half = 1 << (B - 1);
    const int M = half - 1;
    double xiB = xi1, yn = 0.5 * sd;
    int sumu = half * d;  // sum of levels when every m_i = 0 and every sign bit is 1
    if (nx > 0.0) {
        int sgn_pos = 0;
        for (int h = 0; h < nh; h++) {
            const int i = lane + 64 * h;
            if (i < d && Xpp[r * d4 + i] >= 0.f) sgn_pos++;
        }
        sgn_pos = wave_sum_int(sgn_pos);
        sumu = half * sgn_pos + (half - 1) * (d - sgn_pos);
    }
    int best_c = 0;  // candidate 0: every m_i = 0
    if (B > 1 && nx > 0.0) {
        for (int h = 0; h < nh; h++) {
            const int i = lane + 64 * h;
            if (i < d) a_s[i] = fabs((double)Xpp[r * d4 + i]) / nx;
        }
        __syncthreads();
        double bc = -2.0, bt = 0.0;
        int bi = -1;
        const int ncand = 1 + d * M;
        for (int cix = lane; cix < ncand; cix += 64) {
            int ci = -1, cj = 0;
            double tt = 0.0;
            if (cix > 0) {
                ci = (cix - 1) / M;
                cj = (cix - 1) % M + 1;
                if (!(a_s[ci] > 0.0)) continue;
                tt = (double)cj / a_s[ci];
            }
            double num = 0.0, den = 0.0;
            for (int kk = 0; kk < d; kk++) {
                const double ak = a_s[kk];
                int mk;
                if (kk == ci) mk = cj;
                else if (cix == 0) mk = 0;
                else {
                    const double f = floor(tt * ak);
                    mk = f > (double)M ? M : (int)f;
                }
                const double y = mk + 0.5;
                num += y * ak;
                den += y * y;
            }
            const double cs = num / sqrt(den);
            if (cs > bc || (cs == bc && (tt < bt || (tt == bt && ci < bi)))) { bc = cs; bt = tt; bi = ci; best_c = cix; }
        }
        for (int o = 32; o >= 1; o >>= 1) {
            const double oc = __shfl_xor(bc, o), ot = __shfl_xor(bt, o);
            const int oi = __shfl_xor(bi, o), ocx = __shfl_xor(best_c, o);
            if (oc > bc || (oc == bc && (ot < bt || (ot == bt && oi < bi)))) { bc = oc; bt = ot; bi = oi; best_c = ocx; }
        }
        const int ci = best_c > 0 ? (best_c - 1) / M : -1;
        const int cj = best_c > 0 ? (best_c - 1) % M + 1 : 0;
        const double tt = best_c > 0 ? (double)cj / a_s[ci] : 0.0;
        double num = 0.0, den = 0.0;
        int su = 0;
        uint32_t uvals[24];
        for (int h = 0; h < nh; h++) {
            const int i = lane + 64 * h;
            uint32_t u = 0;
            if (i < d) {
                int mk;
                if (i == ci) mk = cj;
                else if (best_c == 0) mk = 0;
                else {
                    const double f = floor(tt * a_s[i]);
                    mk = f > (double)M ? M : (int)f;
                }
                const double xp = (double)Xpp[r * d4 + i] / nx;
                u = xp >= 0.0 ? (uint32_t)(half + mk) : (uint32_t)(half - 1 - mk);
                const double y = (double)u - (double)((1 << B) - 1) * 0.5;
                num += y * xp;
                den += y * y;
                su += (int)u;
            }
            uvals[h] = u;
        }
        num = wave_sum_d(num);
        den = wave_sum_d(den);
        su = wave_sum_int(su);
        yn = sqrt(den);
        xiB = num / yn;
        sumu = su;
        uint32_t* ew = ext + r * (B - 1) * WP;
        for (int a = 0; a < B - 1; a++) {
            for (int h = 0; h < (WP + 1) / 2; h++) {
                const bool bit = h < nh && ((uvals[h < nh ? h : 0] >> a) & 1u);
                const unsigned long long bm = __ballot(bit);
                if (lane == 0) {
                    if (2 * h < WP) ew[a * WP + 2 * h] = (uint32_t)bm;
                    if (2 * h + 1 < WP) ew[a * WP + 2 * h + 1] = (uint32_t)(bm >> 32);
                }
            }
        }
    } else if (B > 1) {  // n_x = 0 or no refinement possible: levels = half (m = 0, sign bit 1) or sign code
        uint32_t* ew = ext + r * (B - 1) * WP;
        for (int a = 0; a < B - 1; a++) {
            for (int h = 0; h < (WP + 1) / 2; h++) {
                // level half + 0 or half - 1: lower bits all 0 for sign 1, all 1 for sign 0
                const int i = lane + 64 * h;
                const bool neg = i < d && nx > 0.0 && Xpp[r * d4 + (i < d ? i : 0)] < 0.f;
                const unsigned long long bm = __ballot(neg);
                if (lane == 0) {
                    if (2 * h < WP) ew[a * WP + 2 * h] = (uint32_t)bm;
                    if (2 * h + 1 < WP) ew[a * WP + 2 * h + 1] = (uint32_t)(bm >> 32);
                }
            }
        }
        xiB = 1.0;
        yn = 0.5 * sd;  // |y_i| = 1/2 for every i
    }
    if (lane == 0) {
        const double xi1s = nx > 0.0 ? xi1 : 1.0;
        const double xiBs = nx > 0.0 ? xiB : 1.0;
        fA[r] = (float)(nx * nx + tx);
        fF[r] = (float)(nx > 0.0 ? nx / (sd * xi1s) : 0.0);
        fE[r] = (float)(nx > 0.0 ? nx * sqrt(fmax(0.0, 1.0 - xi1s * xi1s)) / xi1s : 0.0);
        fFB[r] = (float)(nx > 0.0 ? nx / (2.0 * yn * xiBs) : 0.0);
        fEB[r] = (float)(nx > 0.0 ? nx * sqrt(fmax(0.0, 1.0 - xiBs * xiBs)) / xiBs : 0.0);
        fSX[r] = (float)(2 * sumu - ((1 << B) - 1) * d);
        nxo[r] = (float)nx;
        txo[r] = (float)tx;
        xi1o[r] = (float)xi1s;
        xiBo[r] = (float)xiBs;
        yno[r] = (float)yn;
    }
}

hipError_t launch_encode(const Index& ix, const float* O, const float* Xpp, const double* tx64_rows,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_encode, dim3((unsigned)ix.Npad), dim3(64), 0, s, O, Xpp, tx64_rows, ix.Npad, ix.d, ix.d4,
                       ix.B, ix.WP, ix.ids, ix.code, ix.ext, ix.fA, ix.fF, ix.fE, ix.fFB, ix.fEB, ix.fSX, ix.nx,
                       ix.tx, ix.xi1, ix.xiB, ix.yn);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------------
// MR-SQ codes (Appendix A.2, Exp-5): 8-bit scalar quantisation of the leading d coordinates of x_p.
//   grid of coordinate i: [lo_i, hi_i] = min / max of x_{p,i} over the data set, delta_i = (hi_i - lo_i)/255
//   (1 when hi_i == lo_i); code u_i = min(255, floor((x_i - lo_i) * (1/delta_i) + 1/2)), every step one
//   IEEE-rounded FP32 operation.  A row's dq = 16 ceil(d / 16) bytes are stored in scan order: dimension
//   16 t + 4 g + e at byte g (dq / 4) + 4 t + e, so lane group g of the scan reads its bytes contiguously.

// Partial min / max of 64 coordinates over a chunk of rows (real rows only), four row streams per block.
__global__ __launch_bounds__(256) void k_sq_minmax_part(const float* __restrict__ xd, const int32_t* __restrict__ ids,
                                                        int64_t Npad, int d, int d4, int64_t rpc,
                                                        float* __restrict__ plo, float* __restrict__ phi) {
    __shared__ float slo[4][64], shi[4][64];
    const int lane = threadIdx.x & 63, sub = threadIdx.x >> 6;
    const int c = blockIdx.x * 64 + lane;
    const int64_t r0 = (int64_t)blockIdx.y * rpc, r1 = r0 + rpc < Npad ? r0 + rpc : Npad;
    float lo = INFINITY, hi = -INFINITY;
    if (c < d)
        for (int64_t r = r0 + sub; r < r1; r += 4)
            if (ids[r] >= 0) {
                const float v = xd[r * d4 + c];
                lo = fminf(lo, v);
                hi = fmaxf(hi, v);
            }
    slo[sub][lane] = lo;
    shi[sub][lane] = hi;
    __syncthreads();
    if (sub == 0 && c < d) {
        for (int t = 1; t < 4; t++) {
            lo = fminf(lo, slo[t][lane]);
            hi = fmaxf(hi, shi[t][lane]);
        }
        plo[(int64_t)blockIdx.y * d + c] = lo;
        phi[(int64_t)blockIdx.y * d + c] = hi;
    }
}

// The grid of every coordinate from the partials; coordinates d .. dq - 1 get lo 0 and delta 1.
__global__ void k_sq_grid(const float* __restrict__ plo, const float* __restrict__ phi, int nchunk, int d, int dq,
                          float* __restrict__ lo, float* __restrict__ delta) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= dq) return;
    if (c >= d) {
        lo[c] = 0.f;
        delta[c] = 1.f;
        return;
    }
    float a = INFINITY, b = -INFINITY;
    for (int ch = 0; ch < nchunk; ch++) {
        a = fminf(a, plo[(int64_t)ch * d + c]);
        b = fmaxf(b, phi[(int64_t)ch * d + c]);
    }
    lo[c] = a;
    delta[c] = b > a ? __fdiv_rn(__fsub_rn(b, a), 255.f) : 1.f;
}

// One wave per row: the codes, and A = ||xhat_d||^2 + ||x_r||^2 in FP64 (+inf on padding rows, so their
// estimate is +inf and they are never re-ranked).
__global__ __launch_bounds__(64) void k_sq_encode(const float* __restrict__ xd, const int32_t* __restrict__ ids,
                                                  const double* __restrict__ tx64, int d, int d4, int dq,
                                                  const float* __restrict__ lo, const float* __restrict__ delta,
                                                  uint8_t* __restrict__ code, float* __restrict__ A) {
    const int64_t r = blockIdx.x;
    const int lane = threadIdx.x;
    const bool real = ids[r] >= 0;
    double s = 0.0;
    for (int i = lane; i < dq; i += 64) {
        int u = 0;
        if (real && i < d) {
            const float inv = __fdiv_rn(1.f, delta[i]);
            const float t = __fadd_rn(__fmul_rn(__fsub_rn(xd[r * d4 + i], lo[i]), inv), 0.5f);
            u = (int)floorf(t);
            u = u < 0 ? 0 : (u > 255 ? 255 : u);
            const double xh = (double)lo[i] + (double)delta[i] * (double)u;
            s += xh * xh;
        }
        code[r * dq + ((i >> 2) & 3) * (dq >> 2) + 4 * (i >> 4) + (i & 3)] = (uint8_t)u;
    }
    s = wave_sum_d(s);
    if (lane == 0) A[r] = real ? (float)(s + tx64[r]) : INFINITY;
}

hipError_t launch_sq8_build(Index& ix, const double* tx64_rows, float* scratch, int nchunk, hipStream_t s) {
    const int d = ix.d, dq = ix.dq;
    const int64_t rpc = (ix.Npad + nchunk - 1) / nchunk;
    float* plo = scratch;
    float* phi = scratch + (int64_t)nchunk * d;
    hipLaunchKernelGGL(k_sq_minmax_part, dim3((unsigned)((d + 63) / 64), (unsigned)nchunk), dim3(256), 0, s, ix.xd,
                       ix.ids, ix.Npad, d, ix.d4, rpc, plo, phi);
    hipLaunchKernelGGL(k_sq_grid, dim3((unsigned)((dq + 255) / 256)), dim3(256), 0, s, plo, phi, nchunk, d, dq,
                       ix.sq_lo, ix.sq_delta);
    hipLaunchKernelGGL(k_sq_encode, dim3((unsigned)ix.Npad), dim3(64), 0, s, ix.xd, ix.ids, tx64_rows, d, ix.d4, dq,
                       ix.sq_lo, ix.sq_delta, ix.sq_code, ix.sq_A);
    return hipGetLastError();
}

__global__ void k_check_finite(const float* __restrict__ X, int64_t n, int32_t* __restrict__ bad) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        if (!isfinite(X[i])) { atomicOr(bad, 1); return; }
}

hipError_t launch_check_finite(const float* X, int64_t n, int32_t* bad, hipStream_t s) {
    int64_t b = (n + 255) / 256;
    hipLaunchKernelGGL(k_check_finite, dim3((unsigned)(b > 8192 ? 8192 : (b < 1 ? 1 : b))), dim3(256), 0, s, X, n, bad);
    return hipGetLastError();
}

}  // namespace mrq
