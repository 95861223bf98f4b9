// Query-time kernels of the MRQ search path (Algorithm 2 with Eq 4-7 of arXiv 2411.06158), written
// for gfx950: the projection and probe distances on the FP32 matrix cores; the probe ranking one wave
// per query; per-(query, list) query codes; a persistent scan in which a wave takes a 64-vector list
// block against a group of queries as 16 x 16 tiles (stage 1 and the B-bit refinement as int8
// matrix-core products of sign bits and query levels, stage 2 as an FP32 matrix-core chain), with its
// operands staged in LDS by direct global-to-LDS loads; survivors binned per query and their exact
// distances computed one block per query, whose result queue (a sorted array of 64-bit (distance, id)
// keys) is updated in LDS; and a seed pass over each query's nearest list, one wave per query, that
// gives the first batched phase its threshold.
//
// Batch independence: every value a query's result depends on (projection, probe ranking, query
// codes, stage values, exact distances, the pruning thresholds) is computed by a fixed sequence of
// operations that depends only on that query, so a query returns bit-identical results alone, in any
// batch, and on the per-query path.  The pruning threshold of a phase is the k-th best exact distance
// after the previous phase (phases split the probe ranks at fixed boundaries), not a value that
// depends on the timing of other work.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cmath>

#include "mrq_internal.h"

namespace mrq {

typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------------------------------------
// small helpers

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }

__device__ __forceinline__ float wave_sum(float v) {
    // xor butterfly: every lane ends with the same value (each step adds the same two operands)
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ __forceinline__ float wave_min(float v) {
    for (int o = 32; o >= 1; o >>= 1) v = fminf(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ float wave_max(float v) {
    for (int o = 32; o >= 1; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ int wave_sum_i(int v) {
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
// Ordering of LDS accesses between the lanes of one wave (they execute in program order; this only
// keeps the compiler from moving them).
__device__ __forceinline__ void wave_lds_fence() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront"); }

// Read data that no kernel of the current launch writes through the constant address space, so a
// wave-uniform address becomes a scalar load.
__device__ __forceinline__ uint32_t const_load(const uint32_t* p) {
    return *(const __attribute__((address_space(4))) uint32_t*)(p);
}
__device__ __forceinline__ PairRec const_load(const PairRec* p) {
    const __attribute__((address_space(4))) uint32_t* w = (const __attribute__((address_space(4))) uint32_t*)(p);
    uint32_t v[12];
#pragma unroll
    for (int i = 0; i < 12; i++) v[i] = w[i];
    PairRec r;
    __builtin_memcpy(&r, v, sizeof(r));
    return r;
}

// Order-preserving map of a float onto uint32 (for keys that may be negative).
__device__ __forceinline__ uint32_t ord_bits(float f) {
    uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// Exact squared distance (Algorithm 2, exact stage) ||x - q||^2 (= ||x_p - q_p||^2, Eq 1) of two
// zero-padded rows of D4 floats (the original vectors), computed by a group of 16 lanes: lane l of the group
// accumulates the float4 chunks l, l + 16, l + 32, ... in ascending order, then a butterfly over the
// group.  A wave evaluates four pairs at once; the value of a pair depends only on its two rows.
__device__ __forceinline__ void acc_sqdiff(float& s, const float4& a, const float4& b) {
    float t;
    t = a.x - b.x; s = fmaf(t, t, s);
    t = a.y - b.y; s = fmaf(t, t, s);
    t = a.z - b.z; s = fmaf(t, t, s);
    t = a.w - b.w; s = fmaf(t, t, s);
}
// Split exact stage: <x_r, q_r> of zero-padded tail rows (Dr4 floats), the same group layout and chunk order;
// the exact distance is then fmaf(-2, <x_r, q_r>, dis_o').
__device__ __forceinline__ void acc_dot4(float& s, const float4& a, const float4& b) {
    s = fmaf(a.x, b.x, s);
    s = fmaf(a.y, b.y, s);
    s = fmaf(a.z, b.z, s);
    s = fmaf(a.w, b.w, s);
}
// One routine for both terms (dot = false: squared differences, true: products), so a kernel that may compute
// either holds one set of row registers.
__device__ __forceinline__ float row_group(const float* __restrict__ x, const float* __restrict__ q, int n4x4,
                                           int l16, bool dot) {
    const int nc = n4x4 >> 2;  // float4 chunks per row
    const float4* __restrict__ xa = reinterpret_cast<const float4*>(x);
    const float4* __restrict__ qa = reinterpret_cast<const float4*>(q);
    float s = 0.f;
    for (int base = 0; base < nc; base += 128) {  // 8 chunks per lane in flight per round
        float4 a[8], b[8];
#pragma unroll
        for (int u = 0; u < 8; u++) {
            const int ci = base + 16 * u + l16;
            a[u] = ci < nc ? xa[ci] : make_float4(0.f, 0.f, 0.f, 0.f);
            b[u] = ci < nc ? qa[ci] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int u = 0; u < 8; u++) {
            if (base + 16 * u + l16 >= nc) break;
            if (dot) acc_dot4(s, a[u], b[u]);
            else acc_sqdiff(s, a[u], b[u]);
        }
    }
    for (int o = 8; o >= 1; o >>= 1) s += __shfl_xor(s, o);
    return s;
}
// The same with the query row in LDS and up to 16 chunks per lane in flight (one round for D <= 1024);
// same operation order, hence the same results.
__device__ __forceinline__ float row_group_lds(const float* __restrict__ x, const float4* qs, int n4x4, int l16,
                                               bool dot) {
    const int nc = n4x4 >> 2;
    const float4* __restrict__ xa = reinterpret_cast<const float4*>(x);
    float s = 0.f;
    for (int base = 0; base < nc; base += 256) {
        float4 a[16];
#pragma unroll
        for (int u = 0; u < 16; u++) {
            const int ci = base + 16 * u + l16;
            a[u] = ci < nc ? xa[ci] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int u = 0; u < 16; u++) {
            const int ci = base + 16 * u + l16;
            if (ci >= nc) break;
            if (dot) acc_dot4(s, a[u], qs[ci]);
            else acc_sqdiff(s, a[u], qs[ci]);
        }
    }
    for (int o = 8; o >= 1; o >>= 1) s += __shfl_xor(s, o);
    return s;
}
// Low-register form with the same operation order (hence the same results), for the rarely taken
// in-place path of the scan kernel.
__device__ __forceinline__ float row_group_small(const float* __restrict__ x, const float* __restrict__ q, int n4x4,
                                                 int l16, bool dot) {
    float s = 0.f;
    for (int ci = l16; ci < (n4x4 >> 2); ci += 16) {
        const float4 a = reinterpret_cast<const float4*>(x)[ci], b = reinterpret_cast<const float4*>(q)[ci];
        if (dot) acc_dot4(s, a, b);
        else acc_sqdiff(s, a, b);
    }
    for (int o = 8; o >= 1; o >>= 1) s += __shfl_xor(s, o);
    return s;
}
__device__ __forceinline__ float exact_dist_group(const float* __restrict__ x, const float* __restrict__ q, int D4,
                                                  int l16) {
    return row_group(x, q, D4, l16, false);
}
__device__ __forceinline__ float exact_dist_group_lds(const float* __restrict__ x, const float4* qs, int D4, int l16) {
    return row_group_lds(x, qs, D4, l16, false);
}
__device__ __forceinline__ float exact_dist_group_small(const float* __restrict__ x, const float* __restrict__ q,
                                                        int D4, int l16) {
    return row_group_small(x, q, D4, l16, false);
}

// <x_d, q_d> of Eq 7 (rows zero padded to d4) as one chain of fused multiply-adds, in the order in which
// the scan's FP32 matrix-core tiles accumulate it: for each 16-dimension slice t, element e of each lane
// group's float4, then lane group g = 0..3, i.e. dimension 16t + 4g + e.  A v_mfma_f32_16x16x4_f32 chain
// rounds every element of its tile in exactly this sequence, so the seed pass (which calls this) and the
// scan give every (query, vector) pair the same stage-2 value.
__device__ __forceinline__ float dot_lane(const float* __restrict__ a, const float* __restrict__ b, int d4) {
    float s = 0.f;
    for (int t = 0; t < d4; t += 16) {
        float4 x[4], y[4];
#pragma unroll
        for (int g = 0; g < 4; g++) {
            const bool in = t + 4 * g < d4;
            x[g] = in ? *reinterpret_cast<const float4*>(a + t + 4 * g) : make_float4(0.f, 0.f, 0.f, 0.f);
            y[g] = in ? *reinterpret_cast<const float4*>(b + t + 4 * g) : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int g = 0; g < 4; g++) if (t + 4 * g < d4) s = fmaf(x[g].x, y[g].x, s);
#pragma unroll
        for (int g = 0; g < 4; g++) if (t + 4 * g < d4) s = fmaf(x[g].y, y[g].y, s);
#pragma unroll
        for (int g = 0; g < 4; g++) if (t + 4 * g < d4) s = fmaf(x[g].z, y[g].z, s);
#pragma unroll
        for (int g = 0; g < 4; g++) if (t + 4 * g < d4) s = fmaf(x[g].w, y[g].w, s);
    }
    return s;
}

// The same chain with q_d in LDS and two 16-dimension slices of the row in flight per round (the seed
// pass); float4s beyond d4 are read at a valid index and zeroed, which adds nothing to the chain.
__device__ __forceinline__ float dot_lane_lds(const float* __restrict__ a, const float4* yq, int d4) {
    const float4* __restrict__ xa = reinterpret_cast<const float4*>(a);
    const int n4 = d4 >> 2;
    const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
    float s = 0.f;
    for (int t4 = 0; t4 < n4; t4 += 8) {
        float4 x[8];
#pragma unroll
        for (int i = 0; i < 8; i++) {
            const int f = t4 + i;
            x[i] = xa[f < n4 ? f : n4 - 1];
            if (f >= n4) x[i] = z;
        }
#pragma unroll
        for (int sl = 0; sl < 2; sl++) {
            float4 y[4];
#pragma unroll
            for (int g = 0; g < 4; g++) {
                const int f = t4 + 4 * sl + g;
                y[g] = yq[f < n4 ? f : n4 - 1];
                if (f >= n4) y[g] = z;
            }
#pragma unroll
            for (int g = 0; g < 4; g++) s = fmaf(x[4 * sl + g].x, y[g].x, s);
#pragma unroll
            for (int g = 0; g < 4; g++) s = fmaf(x[4 * sl + g].y, y[g].y, s);
#pragma unroll
            for (int g = 0; g < 4; g++) s = fmaf(x[4 * sl + g].z, y[g].z, s);
#pragma unroll
            for (int g = 0; g < 4; g++) s = fmaf(x[4 * sl + g].w, y[g].w, s);
        }
    }
    return s;
}

// Take up to four set lanes of *mask (lowest first) and give each 16-lane group one of them: returns
// the source lane of this lane's group, or -1.
__device__ __forceinline__ int take4(unsigned long long* mask, int lane) {
    int src = -1;
#pragma unroll
    for (int g = 0; g < 4; g++) {
        const int s = *mask ? __ffsll((long long)*mask) - 1 : -1;
        if (s >= 0) *mask &= *mask - 1;
        if ((lane >> 4) == g) src = s;
    }
    return src;
}

// Insert a (distance, id) key into a query's sorted k-slot array.  Each slot only ever decreases
// (atomicMin), so the array stays sorted and the final content is the k smallest keys inserted,
// whatever the order of the inserts.
__device__ void topk_insert(unsigned long long* slots, int k, unsigned long long key) {
    volatile unsigned long long* vs = slots;
    if (key >= vs[k - 1]) return;
    int lo = 0, hi = k - 1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (vs[mid] > key) hi = mid; else lo = mid + 1;
    }
    for (int i = lo; i < k; i++) {
        const unsigned long long old = atomicMin(slots + i, key);
        if (old > key) key = old;
        if (key == kEmptyKey) return;
    }
}

// ||x - q||^2 of the split exact stage, dis_o' - 2 <x_r, q_r>, clamped at zero (a near-duplicate of the
// query can round below it, and a negative value's bit pattern would not order as a distance).
__device__ __forceinline__ float split_dist(float dso, float r) {
    const float v = fmaf(-2.f, r, dso);
    return v > 0.f ? v : 0.f;
}

// The bit pattern of the distance in a sorted k-slot array's last key (the array's admission bound: a key
// with a larger distance cannot enter, so its id need not be read).
__device__ __forceinline__ uint32_t last_dist_bits(const unsigned long long* slots, int k) {
    return (uint32_t)(((const volatile unsigned long long*)slots)[k - 1] >> 32);
}

// Probe-rank phases for a growth g = 2^sh: rank 0 (the seed pass), then [1, g), [g, g^2), ... up to
// rank 1023 (at most 10 more phases).
__device__ __forceinline__ int phase_of(int r, int sh) { return r == 0 ? 0 : (32 - __clz(r) + sh - 1) / sh; }
__host__ __device__ __forceinline__ int phase_lo(int p, int sh) { return p == 0 ? 0 : (1 << (sh * (p - 1))); }

// ------------------------------------------------------------------------------------------------
// fill helpers (kernels rather than memset nodes so the sequence can be captured in a graph)

__global__ void k_fill_u64(unsigned long long* p, unsigned long long v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void k_fill_i32(int32_t* p, int32_t v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void k_fill_f32(float* p, float v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}
static int fill_grid(int64_t n) {
    int64_t b = (n + 255) / 256;
    return (int)(b < 1 ? 1 : (b > 4096 ? 4096 : b));
}
hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3(fill_grid(n)), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}
hipError_t launch_fill_f32(float* p, float v, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_f32, dim3(fill_grid(n)), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}
static hipError_t fill_u64(unsigned long long* p, unsigned long long v, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u64, dim3(fill_grid(n)), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

// Per-query metadata for a uniform (k, nprobe) batch.
__global__ void k_uniform_meta(int64_t nq, int k, int np, int32_t* __restrict__ kq, int32_t* __restrict__ npq,
                               int64_t* __restrict__ slot_off, int64_t* __restrict__ pair_off,
                               int64_t* __restrict__ out_off) {
    int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q > nq) return;
    slot_off[q] = q * k;
    pair_off[q] = q * np;
    if (q < nq) {
        kq[q] = k;
        npq[q] = np;
        out_off[q] = q * k;
    }
}
// Per-query metadata of a batch whose k[i] / nprobe[i] (and optionally out_off[i]) are device arrays, with
// upper bounds kb, npb given by the caller: a query whose k is outside [1, kb], nprobe outside [1, npb] or
// out_off negative is rejected (k = nprobe = 0: no pairs, no output) and counted into *rejected; slot_off
// and pair_off are the exclusive prefix sums of the accepted k and nprobe (n + 1 entries), out_off the
// caller's offsets or, when none are given, slot_off.  One block of 1024 threads; thread t takes a
// contiguous chunk of queries.
__global__ __launch_bounds__(1024) void k_mixed_meta(int64_t nq, const int32_t* __restrict__ k_in,
                                                    const int32_t* __restrict__ np_in,
                                                    const int64_t* __restrict__ oo_in, int kb, int npb,
                                                    int32_t* __restrict__ kq, int32_t* __restrict__ npq,
                                                    int64_t* __restrict__ slot_off, int64_t* __restrict__ pair_off,
                                                    int64_t* __restrict__ out_off, int32_t* __restrict__ rejected) {
    __shared__ long long ws[16], wp[16];
    __shared__ int wr[16];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int64_t per = (nq + 1023) / 1024;
    const int64_t b = (int64_t)t * per, e = b + per < nq ? b + per : nq;
    long long sk = 0, sp = 0;
    int bad = 0;
    for (int64_t i = b; i < e; i++) {
        const int k = k_in[i], np = np_in[i];
        const bool ok = k >= 1 && k <= kb && np >= 1 && np <= npb && (!oo_in || oo_in[i] >= 0);
        kq[i] = ok ? k : 0;
        npq[i] = ok ? np : 0;
        sk += ok ? k : 0;
        sp += ok ? np : 0;
        bad += ok ? 0 : 1;
    }
    // exclusive scan of the per-thread sums over the block
    long long ik = sk, ip = sp;
    for (int o = 1; o < 64; o <<= 1) {
        const long long yk = __shfl_up(ik, o), yp = __shfl_up(ip, o);
        if (lane >= o) { ik += yk; ip += yp; }
    }
    int rb = bad;
    for (int o = 32; o >= 1; o >>= 1) rb += __shfl_xor(rb, o);
    if (lane == 63) { ws[w] = ik; wp[w] = ip; }
    if (lane == 0) wr[w] = rb;
    __syncthreads();
    long long bk = 0, bp = 0;
    for (int i = 0; i < w; i++) { bk += ws[i]; bp += wp[i]; }
    bk += ik - sk;
    bp += ip - sp;
    for (int64_t i = b; i < e; i++) {
        slot_off[i] = bk;
        pair_off[i] = bp;
        out_off[i] = oo_in ? oo_in[i] : bk;
        bk += kq[i];
        bp += npq[i];
    }
    if (t == 1023) {
        slot_off[nq] = bk;
        pair_off[nq] = bp;
        int tot = 0;
        for (int i = 0; i < 16; i++) tot += wr[i];
        if (rejected) *rejected = tot;
    }
}
hipError_t launch_mixed_meta(int64_t nq, const int32_t* k, const int32_t* np, const int64_t* out_off_in, int kb,
                             int npb, int32_t* kq, int32_t* npq, int64_t* slot_off, int64_t* pair_off,
                             int64_t* out_off, int32_t* rejected, hipStream_t s) {
    hipLaunchKernelGGL(k_mixed_meta, dim3(1), dim3(1024), 0, s, nq, k, np, out_off_in, kb, npb, kq, npq, slot_off,
                       pair_off, out_off, rejected);
    return hipGetLastError();
}

hipError_t launch_uniform_meta(int64_t nq, int k, int np, int32_t* kq, int32_t* npq, int64_t* slot_off,
                               int64_t* pair_off, int64_t* out_off, hipStream_t s) {
    hipLaunchKernelGGL(k_uniform_meta, dim3((unsigned)((nq + 256) / 256)), dim3(256), 0, s, nq, k, np, kq, npq,
                       slot_off, pair_off, out_off);
    return hipGetLastError();
}

// dst[i, :dim] = src[idx[i], :dim]
__global__ void k_gather_rows(const float* __restrict__ src, int64_t lds, const int32_t* __restrict__ idx,
                              int64_t n, int dim, float* __restrict__ dst, int64_t ldd) {
    const int64_t r = blockIdx.x * 4ll + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (r >= n) return;
    const int64_t sr = idx[r];
    for (int i = lane; i < dim; i += 64) dst[r * ldd + i] = src[sr * lds + i];
}
hipError_t launch_gather_rows(const float* src, int64_t lds, const int32_t* idx, int64_t n, int dim, float* dst,
                              int64_t ldd, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, src, lds, idx, n, dim, dst, ldd);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------------
// FP32 "NT" GEMM: C[m, n] = sum_k (A[m, k] - asub[k]) * B[n, k]; 64 x 64 tile per 256 threads, 4 x 4
// outputs per thread, k in steps of 16 through LDS.  Each output is a sequential FMA chain over k in
// ascending order, so its value depends only on its own row and column.
// EPI 0: store;  EPI 1: C = max(0, rowv[m] + colv[n] - 2 acc)  (squared distances via norms)

template <int EPI>
__global__ __launch_bounds__(256) void k_gemm_nt(const float* __restrict__ A, int64_t lda,
                                                 const float* __restrict__ asub,
                                                 const float* __restrict__ Bm, int64_t ldb,
                                                 float* __restrict__ Cm, int64_t ldc, int64_t M, int N,
                                                 int K, const float* __restrict__ rowv,
                                                 const float* __restrict__ colv) {
    __shared__ float As[16][68];
    __shared__ float Bs[16][68];
    const int t = threadIdx.x;
    const int tx = t & 15, ty = t >> 4;
    const int64_t m0 = (int64_t)blockIdx.x * 64;
    const int n0 = blockIdx.y * 64;
    float acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int j = 0; j < 4; j++) acc[i][j] = 0.f;
    const int lr = t >> 2, lk = (t & 3) * 4;
    for (int k0 = 0; k0 < K; k0 += 16) {
#pragma unroll
        for (int u = 0; u < 4; u++) {
            int kk = k0 + lk + u;
            int64_t mr = m0 + lr;
            float av = 0.f;
            if (mr < M && kk < K) {
                av = A[mr * lda + kk];
                if (asub) av -= asub[kk];
            }
            As[lk + u][lr] = av;
            int nr = n0 + lr;
            Bs[lk + u][lr] = (nr < N && kk < K) ? Bm[(int64_t)nr * ldb + kk] : 0.f;
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
    for (int i = 0; i < 4; i++) {
        int64_t m = m0 + ty * 4 + i;
        if (m >= M) continue;
#pragma unroll
        for (int j = 0; j < 4; j++) {
            int n = n0 + tx * 4 + j;
            if (n >= N) continue;
            float v = acc[i][j];
            if (EPI == 1) v = fmaxf(0.f, fmaf(-2.f, v, rowv[m] + colv[n]));
            Cm[m * ldc + n] = v;
        }
    }
}

hipError_t launch_gemm_nt(const float* A, int64_t lda, const float* asub, const float* Bm, int64_t ldb,
                          float* Cm, int64_t ldc, int64_t M, int N, int K, hipStream_t s) {
    if (M <= 0 || N <= 0) return hipSuccess;
    dim3 grid((unsigned)((M + 63) / 64), (N + 63) / 64);
    hipLaunchKernelGGL(k_gemm_nt<0>, grid, dim3(256), 0, s, A, lda, asub, Bm, ldb, Cm, ldc, M, N, K,
                       nullptr, nullptr);
    return hipGetLastError();
}
static hipError_t launch_gemm_dist(const float* A, int64_t lda, const float* Bm, int64_t ldb, float* Cm,
                                   int64_t ldc, int64_t M, int N, int K, const float* rowv,
                                   const float* colv, hipStream_t s) {
    dim3 grid((unsigned)((M + 63) / 64), (N + 63) / 64);
    hipLaunchKernelGGL(k_gemm_nt<1>, grid, dim3(256), 0, s, A, lda, nullptr, Bm, ldb, Cm, ldc, M, N, K,
                       rowv, colv);
    return hipGetLastError();
}

// FP32 matrix-core form of the same product, C = (A - asub) B^T, for the large query-side products.
// One wave computes a 64 x 64 tile of C as 4 x 4 v_mfma_f32_16x16x4_f32 sub-tiles; its A and B
// fragments are read straight from memory (rows are K-contiguous), VEC = 4: one dwordx4 per lane per
// fragment and 16-wide K step (lane group g feeds k = 16s + 4g + e in multiply step e), VEC = 1: one
// float per lane per 4-wide K step.  Every element is one chain of fused multiply-adds over k in a fixed
// order that depends only on K and VEC, so a row's result does not depend on the other rows.
// EPI 0: C[m][n];  EPI 1: max(0, rowv[m] + colv[n] - 2 C) (squared distances), and with tmin the smallest
// distance of each row within each 64-column tile, tmin[m * gridDim.y + tile];  EPI 2: columns below
// nsplit go to C (ldc), the others to C2 (ldc2) at column n - nsplit.
template <int VEC, int EPI, int MI>
__global__ __launch_bounds__(256) void k_gemm_mfma(const float* __restrict__ A, int64_t lda,
                                                   const float* __restrict__ asub,
                                                   const float* __restrict__ Bm, int64_t ldb,
                                                   float* __restrict__ Cm, int64_t ldc, int64_t M, int N, int K,
                                                   const float* __restrict__ rowv, const float* __restrict__ colv,
                                                   float* __restrict__ C2, int64_t ldc2, int nsplit,
                                                   float* __restrict__ tmin) {
    const int lane = threadIdx.x & 63;
    const int li = lane & 15, kg = lane >> 4;
    const int64_t m0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * (16 * MI);
    const int n0 = blockIdx.y * 64;
    if (m0 >= M) return;
    const float* ar[MI];
    const float* br[4];
#pragma unroll
    for (int i = 0; i < MI; i++) {
        const int64_t m = m0 + 16 * i + li;
        ar[i] = A + (m < M ? m : M - 1) * lda;
    }
#pragma unroll
    for (int i = 0; i < 4; i++) {
        const int n = n0 + 16 * i + li;
        br[i] = Bm + (int64_t)(n < N ? n : N - 1) * ldb;
    }
    f32x4 acc[MI][4];
#pragma unroll
    for (int i = 0; i < MI; i++)
#pragma unroll
        for (int j = 0; j < 4; j++) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    if (VEC == 4) {
        for (int k0 = 0; k0 < K; k0 += 16) {
            const int k = k0 + 4 * kg;
            const int kc = k < K ? k : 0;  // in-row offset actually read (always valid)
            const bool e0 = k < K, e1 = k + 1 < K, e2 = k + 2 < K, e3 = k + 3 < K;
            // every load of the step is issued before any is used (the subtraction used to wait on each)
            float4 av[MI], bv[4];
            const float4 sub = *reinterpret_cast<const float4*>((asub ? asub : ar[0]) + kc);
#pragma unroll
            for (int i = 0; i < MI; i++) av[i] = *reinterpret_cast<const float4*>(ar[i] + kc);
#pragma unroll
            for (int j = 0; j < 4; j++) bv[j] = *reinterpret_cast<const float4*>(br[j] + kc);
#pragma unroll
            for (int i = 0; i < MI; i++) {
                float4 a = av[i];
                if (asub) { a.x -= sub.x; a.y -= sub.y; a.z -= sub.z; a.w -= sub.w; }
                av[i] = make_float4(e0 ? a.x : 0.f, e1 ? a.y : 0.f, e2 ? a.z : 0.f, e3 ? a.w : 0.f);
            }
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const float4 b = bv[j];
                bv[j] = make_float4(e0 ? b.x : 0.f, e1 ? b.y : 0.f, e2 ? b.z : 0.f, e3 ? b.w : 0.f);
            }
#pragma unroll
            for (int i = 0; i < MI; i++)
#pragma unroll
                for (int j = 0; j < 4; j++) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i].x, bv[j].x, acc[i][j], 0, 0, 0);
#pragma unroll
            for (int i = 0; i < MI; i++)
#pragma unroll
                for (int j = 0; j < 4; j++) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i].y, bv[j].y, acc[i][j], 0, 0, 0);
#pragma unroll
            for (int i = 0; i < MI; i++)
#pragma unroll
                for (int j = 0; j < 4; j++) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i].z, bv[j].z, acc[i][j], 0, 0, 0);
#pragma unroll
            for (int i = 0; i < MI; i++)
#pragma unroll
                for (int j = 0; j < 4; j++) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i].w, bv[j].w, acc[i][j], 0, 0, 0);
        }
    } else {
        for (int k0 = 0; k0 < K; k0 += 4) {
            const int k = k0 + kg;
            const bool in = k < K;
            const int kc = in ? k : 0;
            const float sub = asub ? asub[kc] : 0.f;
            float av[MI], bv[4];
#pragma unroll
            for (int i = 0; i < MI; i++) {
                const float a = ar[i][kc] - sub;
                av[i] = in ? a : 0.f;
            }
#pragma unroll
            for (int j = 0; j < 4; j++) bv[j] = in ? br[j][kc] : 0.f;
#pragma unroll
            for (int i = 0; i < MI; i++)
#pragma unroll
                for (int j = 0; j < 4; j++) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i], bv[j], acc[i][j], 0, 0, 0);
        }
    }
    // lane holds C[m0 + 16 i + 4 kg + v][n0 + 16 j + li]; the four column sub-tiles of an output row are
    // stored by consecutive instructions (64 B of the row per lane group each), so its 256 B reach the
    // cache together
    float cv[4];
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const int n = n0 + 16 * j + li;
        cv[j] = EPI == 1 && n < N ? colv[n] : 0.f;
    }
#pragma unroll
    for (int i = 0; i < MI; i++) {
#pragma unroll
        for (int v = 0; v < 4; v++) {
            const int64_t m = m0 + 16 * i + 4 * kg + v;
            const bool mok = m < M;
            const float rv = EPI == 1 && mok ? rowv[m] : 0.f;
            float mn = __int_as_float(0x7f800000);  // the row's smallest stored value in this tile
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const int n = n0 + 16 * j + li;
                float r = acc[i][j][v];
                if (EPI == 1) r = fmaxf(0.f, fmaf(-2.f, r, rv + cv[j]));
                if (mok && n < N) {
                    if (EPI == 2 && n >= nsplit) C2[m * ldc2 + (n - nsplit)] = r;
                    else Cm[m * ldc + n] = r;
                }
                if (EPI == 1 && n < N) mn = fminf(mn, r);
            }
            if (EPI == 1 && tmin) {  // (kernel-uniform) the 16 lanes of the row's lane group
                mn = fminf(mn, __shfl_xor(mn, 1));
                mn = fminf(mn, __shfl_xor(mn, 2));
                mn = fminf(mn, __shfl_xor(mn, 4));
                mn = fminf(mn, __shfl_xor(mn, 8));
                if (li == 0 && mok) tmin[m * gridDim.y + blockIdx.y] = mn;
            }
        }
    }
}

static bool vec4_ok(const void* p, int64_t ld) { return ((uintptr_t)p & 15) == 0 && (ld & 3) == 0; }

template <int EPI>
static hipError_t launch_gemm_mfma(const float* A, int64_t lda, const float* asub, const float* Bm, int64_t ldb,
                                   float* Cm, int64_t ldc, int64_t M, int N, int K, const float* rowv,
                                   const float* colv, float* C2, int64_t ldc2, int nsplit, hipStream_t s,
                                   float* tmin = nullptr);

hipError_t launch_project(const float* X, int64_t M, int D, const float* mu, const float* Pp, int d, float* lead,
                          int64_t ld_lead, float* tail, int64_t ld_tail, hipStream_t s) {
    return launch_gemm_mfma<2>(X, D, mu, Pp, D, lead, ld_lead, M, D, D, nullptr, nullptr, tail, ld_tail, d, s);
}

template <int EPI>
static hipError_t launch_gemm_mfma(const float* A, int64_t lda, const float* asub, const float* Bm, int64_t ldb,
                                   float* Cm, int64_t ldc, int64_t M, int N, int K, const float* rowv,
                                   const float* colv, float* C2, int64_t ldc2, int nsplit, hipStream_t s,
                                   float* tmin) {
    if (M <= 0 || N <= 0) return hipSuccess;
    // 64 x 64 output tiles per wave, or 32 x 64 when that gives fewer than about 4 waves per SIMD (the
    // projection): the products of an output element are the same chain either way
    const bool v4 = vec4_ok(A, lda) && vec4_ok(Bm, ldb) && (!asub || vec4_ok(asub, 0));
    const bool half = ((M + 63) / 64) * ((N + 63) / 64) < 4096;
    const dim3 grid((unsigned)((M + (half ? 127 : 255)) / (half ? 128 : 256)), (unsigned)((N + 63) / 64));
#define GEMM_LAUNCH(V, MIV) \
    hipLaunchKernelGGL((k_gemm_mfma<V, EPI, MIV>), grid, dim3(256), 0, s, A, lda, asub, Bm, ldb, Cm, ldc, M, N, K, \
                       rowv, colv, C2, ldc2, nsplit, tmin)
    if (v4 && half) GEMM_LAUNCH(4, 2);
    else if (v4) GEMM_LAUNCH(4, 4);
    else if (half) GEMM_LAUNCH(1, 2);
    else GEMM_LAUNCH(1, 4);
#undef GEMM_LAUNCH
    return hipGetLastError();
}

// The query's tail coordinates (axes d .. D-1 of q_p = P_p (q - mu)) on the BF16 matrix cores, when they only
// feed sigma and eps_r (Eq 6): the exact stage then reads the original vectors and q_d comes from the FP32
// product.  (The split exact stage needs them in FP32 and takes the FP32 product of all D axes instead.)  The
// operands are first converted once per search into BF16 rows of Kp = 32 ceil(K / 32) elements, zero beyond
// K: bf16(q - mu) per query and bf16(P_p row) per tail axis.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// out[r][k] = bf16(src[r][k] - sub[k]) for k < K (sub may be null), 0 for K <= k < Kp; one thread per element
__global__ void k_to_bf16(const float* __restrict__ src, int64_t lds, const float* __restrict__ sub, int K, int Kp,
                          int64_t rows, __bf16* __restrict__ out) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= rows * Kp) return;
    const int64_t r = t / Kp;
    const int k = (int)(t - r * Kp);
    out[t] = (__bf16)(k < K ? src[r * lds + k] - (sub ? sub[k] : 0.f) : 0.f);
}

// C[m][n] = sum_{k < Kp} A[m][k] B[n][k] for BF16 rows of Kp elements (Kp a multiple of 32), FP32 accumulation
// (v_mfma_f32_16x16x32_bf16: lane l feeds row l % 16 of both operands with k = 8 (l / 16) .. + 7 of the step and
// holds C[16 i + 4 (l / 16) + v][16 j + l % 16]), one wave per 64 x 64 tile.
__global__ __launch_bounds__(256) void k_gemm_bf16(const __bf16* __restrict__ A, const __bf16* __restrict__ Bm, int Kp,
                                                   float* __restrict__ Cm, int64_t ldc, int64_t M, int N) {
    const int lane = threadIdx.x & 63;
    const int li = lane & 15, kg = lane >> 4;
    const int64_t m0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 64;
    const int n0 = blockIdx.y * 64;
    if (m0 >= M) return;
    const bf16x8* ar[4];
    const bf16x8* br[4];
#pragma unroll
    for (int i = 0; i < 4; i++) {
        const int64_t m = m0 + 16 * i + li;
        ar[i] = reinterpret_cast<const bf16x8*>(A + (m < M ? m : M - 1) * Kp) + kg;
        const int n = n0 + 16 * i + li;
        br[i] = reinterpret_cast<const bf16x8*>(Bm + (int64_t)(n < N ? n : N - 1) * Kp) + kg;
    }
    f32x4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int j = 0; j < 4; j++) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int s4 = 0; s4 < Kp / 8; s4 += 4) {  // K step of 32: bf16x8 index s4 + kg
        bf16x8 av[4], bv[4];
#pragma unroll
        for (int i = 0; i < 4; i++) {
            av[i] = ar[i][s4];
            bv[i] = br[i][s4];
        }
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
            for (int j = 0; j < 4; j++) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const int n = n0 + 16 * j + li;
        if (n >= N) continue;
#pragma unroll
        for (int i = 0; i < 4; i++) {
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const int64_t m = m0 + 16 * i + 4 * kg + v;
                if (m < M) Cm[m * ldc + n] = acc[i][j][v];
            }
        }
    }
}

// BF16 staging for the tail product of nq queries: nq + D - d rows of 32 ceil(D / 32) elements
static int64_t bf16_stage_elems(const Index& ix, int64_t nq) {
    return (nq + (ix.D - ix.d)) * (int64_t)((ix.D + 31) / 32 * 32);
}

// Algorithm 2, projection of a query batch: q_d = P_p[:d] (q - mu) (FP32 matrix cores; zero padded to d4)
// and the tail coordinates for Eq 6 (BF16 matrix cores when a staging buffer of bf16_stage_elems is given,
// else FP32 with q_d in the same product).
static hipError_t launch_query_projection(const Index& ix, const float* Q, int64_t nq, float* qd, float* qtail,
                                          int64_t ldt, __bf16* stage, hipStream_t s) {
    const int D = ix.D, d = ix.d, d4 = ix.d4;
    hipError_t e = launch_fill_f32(qd, 0.f, nq * d4, s);
    if (e != hipSuccess) return e;
    if (ldt > D - d) {  // padded tail rows: zero beyond D - d
        e = launch_fill_f32(qtail, 0.f, nq * ldt, s);
        if (e != hipSuccess) return e;
    }
    if (stage && D > d) {
        e = launch_gemm_mfma<0>(Q, D, ix.mu, ix.Pp, D, qd, d4, nq, d, D, nullptr, nullptr, nullptr, 0, 0, s);
        if (e != hipSuccess) return e;
        const int Kp = (D + 31) / 32 * 32;
        __bf16* qb = stage;
        __bf16* pb = stage + nq * (int64_t)Kp;
        const int64_t nqe = nq * (int64_t)Kp, npe = (int64_t)(D - d) * Kp;
        hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)((nqe + 255) / 256)), dim3(256), 0, s, Q, (int64_t)D, ix.mu, D,
                           Kp, nq, qb);
        hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)((npe + 255) / 256)), dim3(256), 0, s, ix.Pp + (size_t)d * D,
                           (int64_t)D, (const float*)nullptr, D, Kp, (int64_t)(D - d), pb);
        const dim3 grid((unsigned)((nq + 255) / 256), (unsigned)((D - d + 63) / 64));
        hipLaunchKernelGGL(k_gemm_bf16, grid, dim3(256), 0, s, qb, pb, Kp, qtail, ldt, nq, D - d);
        return hipGetLastError();
    }
    // all D axes in one FP32 product: columns < d are q_d, the rest the tail coordinates
    return launch_gemm_mfma<2>(Q, D, ix.mu, ix.Pp, D, qd, d4, nq, D, D, nullptr, nullptr, qtail, ldt, d, s);
}

// ------------------------------------------------------------------------------------------------
// Exclusive prefix sum of an int32 array in one workgroup (256 threads x 64 items per pass, so the
// (phase, list) buckets of the phases a search uses take one pass).  One wave per SIMD, so it finds room
// on a CU beside the long-lived waves of a concurrent kernel.

constexpr int kScanThreads = 256;
constexpr int kScanItems = 64;

__global__ __launch_bounds__(kScanThreads) void k_scan_excl(const int32_t* __restrict__ in, int32_t* __restrict__ out,
                                                           int64_t n) {
    __shared__ int32_t wsum[kScanThreads / 64];
    __shared__ int32_t carry_s;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const bool vec = ((reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(out)) & 15) == 0;
    if (t == 0) carry_s = 0;
    __syncthreads();
    for (int64_t base = 0; base < n; base += kScanThreads * kScanItems) {
        int32_t v[kScanItems];
        int32_t tot = 0;
        const int64_t b0 = base + (int64_t)t * kScanItems;
        const bool full = vec && b0 + kScanItems <= n;
        if (full) {
#pragma unroll
            for (int i = 0; i < kScanItems / 4; i++) {
                const int4 x = reinterpret_cast<const int4*>(in + b0)[i];
                v[4 * i] = x.x; v[4 * i + 1] = x.y; v[4 * i + 2] = x.z; v[4 * i + 3] = x.w;
            }
        } else {
#pragma unroll
            for (int i = 0; i < kScanItems; i++) v[i] = b0 + i < n ? in[b0 + i] : 0;
        }
#pragma unroll
        for (int i = 0; i < kScanItems; i++) tot += v[i];
        int32_t incl = tot;
        for (int o = 1; o < 64; o <<= 1) {
            int32_t y = __shfl_up(incl, o);
            if (lane >= o) incl += y;
        }
        if (lane == 63) wsum[w] = incl;
        __syncthreads();
        int32_t woff = 0;
        for (int i = 0; i < w; i++) woff += wsum[i];
        int32_t run = carry_s + woff + incl - tot;
#pragma unroll
        for (int i = 0; i < kScanItems; i++) {
            const int32_t x = v[i];
            v[i] = run;
            run += x;
        }
        if (full) {
#pragma unroll
            for (int i = 0; i < kScanItems / 4; i++)
                reinterpret_cast<int4*>(out + b0)[i] = make_int4(v[4 * i], v[4 * i + 1], v[4 * i + 2], v[4 * i + 3]);
        } else {
#pragma unroll
            for (int i = 0; i < kScanItems; i++)
                if (b0 + i < n) out[b0 + i] = v[i];
        }
        __syncthreads();
        if (t == kScanThreads - 1) carry_s = run;
        __syncthreads();
    }
    if (t == 0) out[n] = carry_s;
}

// The same exclusive prefix sum over many workgroups (segments of kSeg entries): the segment sums, then
// each segment's scan from the sum of the segments before it.  Beside a kernel that fills the GPU, a
// single workgroup gets one CU's share of issue slots; these spread over as many CUs as segments.
constexpr int kSegItems = 4;
constexpr int kSeg = kScanThreads * kSegItems;

__device__ __forceinline__ int block_sum_256(int v, int* red) {
    v = wave_sum_i(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    return red[0] + red[1] + red[2] + red[3];
}

__global__ __launch_bounds__(kScanThreads) void k_seg_sums(const int32_t* __restrict__ in, int64_t n,
                                                          int32_t* __restrict__ sums) {
    __shared__ int red[kScanThreads / 64];
    const int64_t b0 = (int64_t)blockIdx.x * kSeg + threadIdx.x * kSegItems;
    int t = 0;
#pragma unroll
    for (int i = 0; i < kSegItems; i++) t += b0 + i < n ? in[b0 + i] : 0;
    t = block_sum_256(t, red);
    if (threadIdx.x == 0) sums[blockIdx.x] = t;
}

__global__ __launch_bounds__(kScanThreads) void k_seg_scan(const int32_t* __restrict__ in, int32_t* __restrict__ out,
                                                          int64_t n, const int32_t* __restrict__ sums) {
    __shared__ int red[kScanThreads / 64], wsum[kScanThreads / 64];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    int o = 0;  // the entries before this segment
    for (int i = t; i < (int)blockIdx.x; i += kScanThreads) o += sums[i];
    o = block_sum_256(o, red);
    const int64_t b0 = (int64_t)blockIdx.x * kSeg + t * kSegItems;
    int32_t v[kSegItems];
    int32_t tot = 0;
#pragma unroll
    for (int i = 0; i < kSegItems; i++) {
        v[i] = b0 + i < n ? in[b0 + i] : 0;
        tot += v[i];
    }
    int32_t incl = tot;
    for (int d = 1; d < 64; d <<= 1) {
        const int32_t y = __shfl_up(incl, d);
        if (lane >= d) incl += y;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    int32_t run = o + incl - tot;
    for (int i = 0; i < w; i++) run += wsum[i];
#pragma unroll
    for (int i = 0; i < kSegItems; i++) {
        if (b0 + i < n) out[b0 + i] = run;
        run += v[i];
    }
    if (blockIdx.x == gridDim.x - 1 && t == kScanThreads - 1) out[n] = run;  // the total
}

// out[0..n]: the exclusive prefix sums of in[0..n-1] and the total; sums: ceil(n / kSeg) entries of scratch
static void launch_scan_excl_seg(const int32_t* in, int32_t* out, int64_t n, int32_t* sums, hipStream_t s) {
    const unsigned nseg = (unsigned)std::max<int64_t>(1, (n + kSeg - 1) / kSeg);
    hipLaunchKernelGGL(k_seg_sums, dim3(nseg), dim3(kScanThreads), 0, s, in, n, sums);
    hipLaunchKernelGGL(k_seg_scan, dim3(nseg), dim3(kScanThreads), 0, s, in, out, n, sums);
}

// ------------------------------------------------------------------------------------------------
// Per-query statistics (Algorithm 2, first three steps; Eq 6):
//   qpad = q (zero padded to D4), ||q_p||^2 = ||q - mu||^2, ||q_d||^2, ||q_r||^2 = ||q_p||^2 - ||q_d||^2,
//   sigma^2 = sum_{i > d} lambda_i q_{p,i}^2,  eps_r = 2 m sigma.

__global__ __launch_bounds__(64) void k_query_stats(const float* __restrict__ Q, int D, int D4,
                                                    const float* __restrict__ mu,
                                                    const float* __restrict__ qd, int d, int d4,
                                                    const float* __restrict__ qtail, int64_t ldt,
                                                    const float* __restrict__ lam_tail, float m,
                                                    float* __restrict__ qpad, float* __restrict__ qn2,
                                                    float* __restrict__ qd2, float* __restrict__ Tq,
                                                    float* __restrict__ er) {
    const int64_t q = blockIdx.x;
    const int lane = threadIdx.x;
    const float* qr = Q + q * D;
    const int r = D - d;
    float s = 0.f;
    for (int i = lane; i < D4; i += 64) {
        // the query as given, padded to D4, for the exact stage (||x - q||^2 from the original vectors)
        qpad[q * D4 + i] = i < D ? qr[i] : 0.f;
        if (i < D) {
            float c = qr[i] - mu[i];
            s = fmaf(c, c, s);
        }
    }
    s = wave_sum(s);
    float sd = 0.f;
    for (int i = lane; i < d; i += 64) {
        float v = qd[q * d4 + i];
        sd = fmaf(v, v, sd);
    }
    sd = wave_sum(sd);
    float var = 0.f;
    for (int i = lane; i < r; i += 64) {
        float v = qtail[q * ldt + i];
        var = fmaf(lam_tail[i], v * v, var);
    }
    var = wave_sum(var);
    if (lane == 0) {
        qn2[q] = s;
        qd2[q] = sd;
        Tq[q] = r == 0 ? 0.f : fmaxf(0.f, s - sd);
        er[q] = r == 0 ? 0.f : 2.f * m * sqrtf(var);
    }
}

// ------------------------------------------------------------------------------------------------
// Probe selection (Algorithm 2, centroid ranking): the np nearest lists by g_j = ||q_d - c_j||^2,
// ties -> smaller list id, nearest first.  One block per query (4 or 8 waves), each thread holding up to 32
// of the query's nlist distances in registers (non-negative, so their bit patterns order like the values),
// the row read once.  Up to np = one per thread the keys at or below the np-th smallest per-thread minimum
// are gathered and ranked; otherwise (or when too many keys fall there) a bitwise search for the np-th smallest
// pattern T (32 block-wide counting rounds), then every j with g_j <= T is gathered in LDS and the
// gathered (g, j) keys are sorted; the first np are the probe lists.

// sort 64 keys held one per lane, ascending (bitonic network over shuffles)
__device__ __forceinline__ unsigned long long wave_sort64(unsigned long long v, int lane) {
    for (int size = 2; size <= 64; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            unsigned long long o = __shfl_xor(v, stride);
            bool up = (lane & size) == 0;
            bool lower = (lane & stride) == 0;
            unsigned long long mn = v < o ? v : o, mx = v < o ? o : v;
            v = (lower == up) ? mn : mx;
        }
    }
    return v;
}

constexpr int kSelCap = kMaxProbe + 1024;   // gathered keys (np plus ties at T)

template <int NW>
__device__ __forceinline__ int block_sum_w(int v, int* red) {
    v = wave_sum_i(v);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    int r = 0;
#pragma unroll
    for (int i = 0; i < NW; i++) r += red[i];
    return r;
}

// NW waves per block, V values per thread (nlist <= 64 NW V); query q (block-uniform); every thread of the
// block returns at the same point
template <int V, int NW>
__device__ __forceinline__ void select_block(const int q, const float* __restrict__ G, int nlist,
                                             const int32_t* __restrict__ npq, const int64_t* __restrict__ pair_off,
                                             int32_t* __restrict__ pair_list, int32_t* __restrict__ pair_q) {
    __shared__ unsigned long long sel[kSelCap];
    __shared__ unsigned long long mins[NW][64];
    __shared__ unsigned long long s_thr;
    __shared__ int red[NW];
    __shared__ int s_cnt, s_wt[NW];
    constexpr int NT = 64 * NW;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const float* g = G + (int64_t)q * nlist;
    const int np = npq[q];
    if (np == 0) return;  // block-uniform
    uint32_t v[V];
#pragma unroll
    for (int u = 0; u < V; u++) {
        const int j = t + NT * u;
        v[u] = j < nlist ? __float_as_uint(g[j]) : 0xFFFFFFFFu;
    }
    if (np <= NT) {
        // Keys (g_j, j) are unique.  The np-th smallest of the NT per-thread minimum keys, thr, has at least
        // np keys at or below it (those np minima), so the np smallest keys are among the keys <= thr, which
        // are usually few: they are gathered and ranked by counting.  (Keys of j >= nlist exceed every real
        // key and are never gathered.)
        unsigned long long mk = kEmptyKey;
#pragma unroll
        for (int u = 0; u < V; u++) {
            const unsigned long long key = ((unsigned long long)v[u] << 32) | (uint32_t)(t + NT * u);
            mk = key < mk ? key : mk;
        }
        const unsigned long long sk = wave_sort64(mk, lane);
        mins[w][lane] = sk;
        __syncthreads();
        int r = lane;  // rank of sk among the NT minima
        for (int w2 = 0; w2 < NW; w2++) {
            if (w2 == w) continue;
            int lo = 0, hi = 64;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (mins[w2][mid] < sk) lo = mid + 1; else hi = mid;
            }
            r += lo;
        }
        if (r == np - 1) s_thr = sk;
        __syncthreads();
        const unsigned long long thr = s_thr;
        int cnt = 0;
#pragma unroll
        for (int u = 0; u < V; u++)
            cnt += t + NT * u < nlist && (((unsigned long long)v[u] << 32) | (uint32_t)(t + NT * u)) <= thr;
        int inc = cnt;  // inclusive prefix over the wave
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(inc, o);
            if (lane >= o) inc += y;
        }
        if (lane == 63) s_wt[w] = inc;
        __syncthreads();
        int m = 0;
#pragma unroll
        for (int i = 0; i < NW; i++) m += s_wt[i];
        if (m <= kSelCap) {  // block-uniform
            int at = inc - cnt;
            for (int i = 0; i < w; i++) at += s_wt[i];
#pragma unroll
            for (int u = 0; u < V; u++) {
                const unsigned long long key = ((unsigned long long)v[u] << 32) | (uint32_t)(t + NT * u);
                if (t + NT * u < nlist && key <= thr) sel[at++] = key;
            }
            __syncthreads();
            const int64_t o = pair_off[q];
            for (int i = t; i < m; i += NT) {
                const unsigned long long key = sel[i];
                int rk = 0;
                for (int x = 0; x < m; x++) rk += sel[x] < key;
                if (rk < np) {
                    pair_list[o + rk] = (int32_t)(key & 0xFFFFFFFFull);
                    pair_q[o + rk] = q;
                }
            }
            return;
        }
        __syncthreads();  // more than kSelCap keys at or below thr: the bitwise search below
    }
    uint32_t T = 0;  // the np-th smallest pattern: the largest value with fewer than np patterns below it
    for (int b = 31; b >= 0; b--) {
        const uint32_t cand = T | (1u << b);
        int c = 0;
#pragma unroll
        for (int u = 0; u < V; u++) c += v[u] < cand;
        if (block_sum_w<NW>(c, red) < np) T = cand;
    }
    int cl = 0, ce = 0;
#pragma unroll
    for (int u = 0; u < V; u++) { cl += v[u] < T; ce += v[u] == T; }
    const int nless = block_sum_w<NW>(cl, red);  // < np
    const int neq = block_sum_w<NW>(ce, red);    // >= np - nless
    if (t == 0) s_cnt = 0;
    __syncthreads();
    const bool all_ties = nless + neq <= kSelCap;
#pragma unroll
    for (int u = 0; u < V; u++) {
        const int j = t + NT * u;
        if (j < nlist && (v[u] < T || (all_ties && v[u] == T))) {
            const int at = atomicAdd(&s_cnt, 1);
            sel[at] = ((unsigned long long)v[u] << 32) | (uint32_t)j;
        }
    }
    __syncthreads();
    int m = s_cnt;
    if (!all_ties) {  // more ties at T than fit: take the first np - nless of them in list order
        int taken = 0;
        for (int u = 0; u < V && taken < np - nless; u++) {
            const int j = t + NT * u;
            // re-read rather than index v (a runtime index would move v out of registers)
            const bool eq = j < nlist && __float_as_uint(g[j]) == T;
            const unsigned long long bm = __ballot(eq);
            if (lane == 0) s_wt[w] = __popcll(bm);
            __syncthreads();
            int r = taken + __popcll(bm & ((1ull << lane) - 1ull));
            for (int i = 0; i < w; i++) r += s_wt[i];
            if (eq && r < np - nless) sel[nless + r] = ((unsigned long long)T << 32) | (uint32_t)j;
#pragma unroll
            for (int i = 0; i < NW; i++) taken += s_wt[i];
            __syncthreads();
        }
        m = np;
    }
    int P = 64;
    while (P < m) P <<= 1;
    for (int i = m + t; i < P; i += NT) sel[i] = kEmptyKey;
    __syncthreads();
    for (int size = 2; size <= P; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = t; i < P; i += NT) {
                const int ixj = i ^ stride;
                if (ixj > i) {
                    const bool asc = (i & size) == 0;
                    const unsigned long long a = sel[i], bb = sel[ixj];
                    if ((a > bb) == asc) { sel[i] = bb; sel[ixj] = a; }
                }
            }
            __syncthreads();
        }
    }
    const int64_t o = pair_off[q];
    for (int r = t; r < np; r += NT) {
        pair_list[o + r] = (int32_t)(sel[r] & 0xFFFFFFFFull);
        pair_q[o + r] = q;
    }
}

template <int V, int NW>
__global__ __launch_bounds__(64 * NW) void k_select(const float* __restrict__ G, int nlist,
                                               const int32_t* __restrict__ npq,
                                               const int64_t* __restrict__ pair_off,
                                               int32_t* __restrict__ pair_list,
                                               int32_t* __restrict__ pair_q) {
    select_block<V, NW>(blockIdx.x, G, nlist, npq, pair_off, pair_list, pair_q);
}

// The block selection of the queries listed in redo[1 .. redo[0]] (those the tile selection below hands
// back), blocks striding over the list.
template <int V, int NW>
__global__ __launch_bounds__(64 * NW) void k_select_redo(const float* __restrict__ G, int nlist,
                                                    const int32_t* __restrict__ npq,
                                                    const int64_t* __restrict__ pair_off,
                                                    int32_t* __restrict__ pair_list, int32_t* __restrict__ pair_q,
                                                    const int32_t* __restrict__ redo) {
    const int n = redo[0];
    for (int i = blockIdx.x; i < n; i += gridDim.x) {
        select_block<V, NW>(redo[1 + i], G, nlist, npq, pair_off, pair_list, pair_q);
        __syncthreads();  // the shared arrays are reused by the next query
    }
}


// The same selection for np <= 64 and nlist <= 64 V, one wave per query (four per block, no barriers):
// lane l holds the patterns of lists j = l + 64 u.  The np-th smallest of the 64 lane minima is a
// threshold t with at least np patterns <= t, so the lists with g_j <= t hold the np smallest keys
// (g_j, j); when there are at most 64 of them they are gathered one per lane and sorted, and the first np
// are taken.  Otherwise the np-th smallest key is found bitwise: 32 wave-wide counting rounds give its
// pattern T, then, among the ties at T, rounds over the list id give the last one taken (unless every tie
// is taken), and the np lists are gathered and sorted.  Either way the lists and their order are those
// of k_select.
template <int V>
__global__ __launch_bounds__(256) void k_select_w(const float* __restrict__ G, int nlist,
                                                 const int32_t* __restrict__ npq,
                                                 const int64_t* __restrict__ pair_off,
                                                 int32_t* __restrict__ pair_list, int32_t* __restrict__ pair_q,
                                                 int64_t nq) {
    __shared__ unsigned long long sel_s[4][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t q = blockIdx.x * 4ll + w;
    if (q >= nq) return;
    const float* g = G + q * nlist;
    const int np = npq[q];
    if (np == 0) return;  // wave-uniform
    uint32_t v[V];
#pragma unroll
    for (int u = 0; u < V; u++) {
        const int j = lane + 64 * u;
        v[u] = j < nlist ? __float_as_uint(g[j]) : 0xFFFFFFFFu;
    }
    const unsigned long long lt = (1ull << lane) - 1ull;
    uint32_t mn = 0xFFFFFFFFu;
#pragma unroll
    for (int u = 0; u < V; u++) mn = min(mn, v[u]);
    const uint32_t t = (uint32_t)__shfl(wave_sort64(mn, lane), np - 1);
    int cc = 0;
#pragma unroll
    for (int u = 0; u < V; u++) cc += v[u] <= t;
    if (wave_sum_i(cc) <= 64) {
        int at = 0;
#pragma unroll
        for (int u = 0; u < V; u++) {
            const bool sel = v[u] <= t;
            const unsigned long long m = __ballot(sel);
            if (sel) sel_s[w][at + __popcll(m & lt)] = ((unsigned long long)v[u] << 32) | (uint32_t)(lane + 64 * u);
            at += __popcll(m);
        }
        wave_lds_fence();
        const unsigned long long key = wave_sort64(lane < at ? sel_s[w][lane] : kEmptyKey, lane);
        if (lane < np) {
            const int64_t o = pair_off[q];
            pair_list[o + lane] = (int32_t)(key & 0xFFFFFFFFull);
            pair_q[o + lane] = (int32_t)q;
        }
        return;
    }
    uint32_t T = 0;  // the np-th smallest pattern
    for (int b = 31; b >= 0; b--) {
        const uint32_t cand = T | (1u << b);
        int c = 0;
#pragma unroll
        for (int u = 0; u < V; u++) c += v[u] < cand;
        if (wave_sum_i(c) < np) T = cand;
    }
    int cl = 0, ce = 0;
#pragma unroll
    for (int u = 0; u < V; u++) { cl += v[u] < T; ce += v[u] == T; }
    const int need = np - wave_sum_i(cl);  // ties at T to take, smallest list ids first (>= 1)
    int J = 64 * V;                        // lists j < J among the ties are taken
    if (wave_sum_i(ce) > need) {
        uint32_t Jb = 0;  // the need-th smallest tied list id
        for (int b = 31 - __clz(64 * V - 1); b >= 0; b--) {
            const uint32_t cand = Jb | (1u << b);
            int c = 0;
#pragma unroll
            for (int u = 0; u < V; u++) c += v[u] == T && (uint32_t)(lane + 64 * u) < cand;
            if (wave_sum_i(c) < need) Jb = cand;
        }
        J = (int)Jb + 1;
    }
    int at = 0;
#pragma unroll
    for (int u = 0; u < V; u++) {
        const int j = lane + 64 * u;
        const bool sel = v[u] < T || (v[u] == T && j < J);
        const unsigned long long m = __ballot(sel);
        if (sel) sel_s[w][at + __popcll(m & lt)] = ((unsigned long long)v[u] << 32) | (uint32_t)j;
        at += __popcll(m);
    }
    wave_lds_fence();
    const unsigned long long key = wave_sort64(lane < np ? sel_s[w][lane] : kEmptyKey, lane);
    if (lane < np) {
        const int64_t o = pair_off[q];
        pair_list[o + lane] = (int32_t)(key & 0xFFFFFFFFull);
        pair_q[o + lane] = (int32_t)q;
    }
}

// Selection from the tile minima of the distance product (np <= 64, nlist in (4096, 16384]), one wave per
// query.  Tile t holds lists 64 t .. 64 t + 63 and m_t is their smallest distance.  Let T be the np-th
// smallest tile minimum: the np tiles whose minima are at most T hold np distinct lists at most T, so the
// np-th smallest distance is at most T, and every list among the np smallest keys (g_j, j) lies in a tile
// with m_t <= T.  Those tiles (np of them, more only with ties at T) are the candidates: with at most 64,
// slot u of lane l holds list 64 tile_u + l and the wave ranks the candidates as k_select_w ranks a row
// (the np-th smallest lane minimum bounds the selection; the keys at or below it, when at most 64, are
// sorted; otherwise a bitwise search of the np-th pattern, then of the last list id taken among its
// ties).  A query with more candidate tiles is listed in redo for the block selection.  Same lists, same
// order as k_select.
constexpr int kTileSlots = 64;
template <int VT>
__global__ __launch_bounds__(256) void k_select_t(const float* __restrict__ G, const float* __restrict__ TM,
                                                 int nlist, int ntiles, const int32_t* __restrict__ npq,
                                                 const int64_t* __restrict__ pair_off,
                                                 int32_t* __restrict__ pair_list, int32_t* __restrict__ pair_q,
                                                 int64_t nq, int32_t* __restrict__ redo) {
    __shared__ unsigned long long sel_s[4][64];
    __shared__ int tile_s[4][kTileSlots];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t q = blockIdx.x * 4ll + w;
    if (q >= nq) return;
    const int np = npq[q];
    if (np == 0) return;  // wave-uniform
    const unsigned long long lt = (1ull << lane) - 1ull;
    // T: the np-th smallest tile-minimum pattern (the largest pattern with fewer than np below it)
    uint32_t tv[VT];
#pragma unroll
    for (int u = 0; u < VT; u++) {
        const int t = lane + 64 * u;
        tv[u] = t < ntiles ? __float_as_uint(TM[q * ntiles + t]) : 0xFFFFFFFFu;
    }
    uint32_t T = 0;
    for (int b = 31; b >= 0; b--) {
        const uint32_t cand = T | (1u << b);
        int c = 0;
#pragma unroll
        for (int u = 0; u < VT; u++) c += tv[u] < cand;
        if (wave_sum_i(c) < np) T = cand;
    }
    int mt = 0;  // candidate tiles, in increasing tile order
#pragma unroll
    for (int u = 0; u < VT; u++) {
        const bool sel = lane + 64 * u < ntiles && tv[u] <= T;
        const unsigned long long m = __ballot(sel);
        const int at = mt + __popcll(m & lt);
        if (sel && at < kTileSlots) tile_s[w][at] = lane + 64 * u;
        mt += __popcll(m);
    }
    if (mt > kTileSlots) {  // wave-uniform
        if (lane == 0) redo[1 + atomicAdd(redo, 1)] = (int32_t)q;
        return;
    }
    wave_lds_fence();
    // slot u: list 64 tile_u + lane (no list beyond the candidates or nlist: the empty pattern)
    const float* g = G + q * nlist;
    uint32_t v[kTileSlots];
#pragma unroll
    for (int u = 0; u < kTileSlots; u++) {
        const int j = (u < mt ? tile_s[w][u] : 0) * 64 + lane;
        v[u] = u < mt && j < nlist ? __float_as_uint(g[j]) : 0xFFFFFFFFu;
    }
    auto list_of = [&](int u) { return tile_s[w][u < mt ? u : 0] * 64 + lane; };
    uint32_t mn = 0xFFFFFFFFu;
#pragma unroll
    for (int u = 0; u < kTileSlots; u++) mn = min(mn, v[u]);
    const uint32_t t = (uint32_t)__shfl(wave_sort64(mn, lane), np - 1);
    int cc = 0;
#pragma unroll
    for (int u = 0; u < kTileSlots; u++) cc += v[u] <= t;
    int at = 0;
    if (wave_sum_i(cc) <= 64) {
#pragma unroll
        for (int u = 0; u < kTileSlots; u++) {
            const bool sel = v[u] <= t;
            const unsigned long long m = __ballot(sel);
            if (sel) sel_s[w][at + __popcll(m & lt)] = ((unsigned long long)v[u] << 32) | (uint32_t)list_of(u);
            at += __popcll(m);
        }
    } else {
        uint32_t P = 0;  // the np-th smallest pattern
        for (int b = 31; b >= 0; b--) {
            const uint32_t cand = P | (1u << b);
            int c = 0;
#pragma unroll
            for (int u = 0; u < kTileSlots; u++) c += v[u] < cand;
            if (wave_sum_i(c) < np) P = cand;
        }
        int cl = 0, ce = 0;
#pragma unroll
        for (int u = 0; u < kTileSlots; u++) { cl += v[u] < P; ce += v[u] == P; }
        const int need = np - wave_sum_i(cl);  // ties at P to take, smallest list ids first (>= 1)
        int J = nlist;                         // lists j < J among the ties are taken
        if (wave_sum_i(ce) > need) {
            uint32_t Jb = 0;  // the need-th smallest tied list id
            for (int b = 31 - __clz(nlist - 1); b >= 0; b--) {
                const uint32_t cand = Jb | (1u << b);
                int c = 0;
#pragma unroll
                for (int u = 0; u < kTileSlots; u++) c += v[u] == P && (uint32_t)list_of(u) < cand;
                if (wave_sum_i(c) < need) Jb = cand;
            }
            J = (int)Jb + 1;
        }
#pragma unroll
        for (int u = 0; u < kTileSlots; u++) {
            const int j = list_of(u);
            const bool sel = v[u] < P || (v[u] == P && j < J);
            const unsigned long long m = __ballot(sel);
            if (sel) sel_s[w][at + __popcll(m & lt)] = ((unsigned long long)v[u] << 32) | (uint32_t)j;
            at += __popcll(m);
        }
    }
    wave_lds_fence();
    const unsigned long long key = wave_sort64(lane < at ? sel_s[w][lane] : kEmptyKey, lane);
    if (lane < np) {
        const int64_t o = pair_off[q];
        pair_list[o + lane] = (int32_t)(key & 0xFFFFFFFFull);
        pair_q[o + lane] = (int32_t)q;
    }
}

// The tile selection serves np <= 64 with nlist in (4096, 16384] (at most 256 tiles, four per lane).
static bool tile_select(int nlist, int np_max) { return np_max <= 64 && nlist > 64 * 64 && nlist <= 64 * 256; }

// TM: the tile minima of the product (tile_select), with redo (nq + 1 entries) for the queries it hands back;
// otherwise null.
static void launch_select(const float* G, int nlist, const int32_t* npq, const int64_t* pair_off, int32_t* pair_list,
                          int32_t* pair_q, int64_t nq, int np_max, hipStream_t s, const float* TM = nullptr,
                          int32_t* redo = nullptr) {
    if (TM) {
        const int ntiles = (nlist + 63) / 64;
        (void)launch_fill_i32(redo, 0, 1, s);  // (a launch error surfaces at the caller's hipGetLastError)
        hipLaunchKernelGGL(k_select_t<4>, dim3((unsigned)((nq + 3) / 4)), dim3(256), 0, s, G, TM, nlist, ntiles, npq,
                           pair_off, pair_list, pair_q, nq, redo);
        const unsigned rb = (unsigned)std::min<int64_t>(nq, 256);
        if (nlist <= 256 * 32) hipLaunchKernelGGL((k_select_redo<32, 4>), dim3(rb), dim3(256), 0, s, G, nlist, npq, pair_off, pair_list, pair_q, redo);
        else hipLaunchKernelGGL((k_select_redo<32, 8>), dim3(rb), dim3(512), 0, s, G, nlist, npq, pair_off, pair_list, pair_q, redo);
        return;
    }
    if (np_max <= 64 && nlist <= 64 * 64) {
        const dim3 gw((unsigned)((nq + 3) / 4)), bw(256);
        if (nlist <= 64 * 16) hipLaunchKernelGGL(k_select_w<16>, gw, bw, 0, s, G, nlist, npq, pair_off, pair_list, pair_q, nq);
        else if (nlist <= 64 * 32) hipLaunchKernelGGL(k_select_w<32>, gw, bw, 0, s, G, nlist, npq, pair_off, pair_list, pair_q, nq);
        else hipLaunchKernelGGL(k_select_w<64>, gw, bw, 0, s, G, nlist, npq, pair_off, pair_list, pair_q, nq);
        return;
    }
    // one block per query, at most 32 values per thread (blocks of up to 8 waves)
    const dim3 grid((unsigned)nq);
    if (nlist <= 256 * 16) hipLaunchKernelGGL((k_select<16, 4>), grid, dim3(256), 0, s, G, nlist, npq, pair_off, pair_list, pair_q);
    else if (nlist <= 256 * 32) hipLaunchKernelGGL((k_select<32, 4>), grid, dim3(256), 0, s, G, nlist, npq, pair_off, pair_list, pair_q);
    else hipLaunchKernelGGL((k_select<32, 8>), grid, dim3(512), 0, s, G, nlist, npq, pair_off, pair_list, pair_q);
}

// ------------------------------------------------------------------------------------------------
// Pair bucketing by (phase, list) and per-pair query codes.

// The pair total is read from the device offsets (pair_total = pair_off + nq): a batch whose per-query
// k / nprobe live on the device is launched for an upper bound of the pairs.
__global__ void k_pair_count(const int32_t* __restrict__ pair_list, const int32_t* __restrict__ pair_q,
                             const int64_t* __restrict__ pair_off, const int64_t* __restrict__ pair_total, int nlist,
                             int sh, int32_t* __restrict__ cnt) {
    int64_t pi = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (pi >= *pair_total) return;
    const int q = pair_q[pi];
    const int r = (int)(pi - pair_off[q]);
    atomicAdd(&cnt[phase_of(r, sh) * nlist + pair_list[pi]], 1);
}

// ---- tracing (mrq_search_trace): records written by the tracing instantiations only ----
__device__ __forceinline__ bool trace_on(const TraceSink* tr, int q) { return tr->qflag[q] != 0; }

__device__ __noinline__ void trace_cand(const TraceSink* tr, int kind, int phase, int q, int list, int64_t id, int ip,
                                        int pc, float v0, float v1, float v2, float v3) {
    const unsigned long long t = atomicAdd(tr->n + 1, 1ull);
    if (t >= (unsigned long long)tr->max_cands) return;
    mrq_trace_cand e;
    e.kind = kind;
    e.phase = phase;
    e.q = q;
    e.list = list;
    e.id = id;
    e.ip = ip;
    e.pc = pc;
    e.v0 = v0;
    e.v1 = v1;
    e.v2 = v2;
    e.v3 = v3;
    tr->cands[t] = e;
}
// A record slot for a traced pair (-1 when the buffer is full).
__device__ __forceinline__ long long trace_pair_slot(const TraceSink* tr) {
    const unsigned long long t = atomicAdd(tr->n, 1ull);
    return t < (unsigned long long)tr->max_pairs ? (long long)t : -1ll;
}
__device__ __forceinline__ void trace_pair(const TraceSink* tr, long long t, int phase, const PairRec& R) {
    mrq_trace_pair e;
    e.phase = phase;
    e.q = R.q;
    e.list = R.list;
    e.su = (int)R.su;
    e.nq = 0.5f * R.two_nq;
    e.vl = R.vl;
    e.delta = R.delta;
    e.kr = R.Kr;
    e.ebc = R.ebc;
    e.er = R.er;
    e.qn2 = R.qn2;
    e.pad = 0.f;
    tr->pairs[t] = e;
}

// Query code of one (query, list) pair by a group of L lanes (Algorithm 2: normalise, rotate and quantise
// q_d for list j):
//   w = P_r^T q_d - P_r^T c_j,  n_q = ||w||,  q' = w / n_q,
//   v_l = min q', Delta = (max q' - v_l) / (2^bq - 1), u_i = floor((q'_i - v_l) * (1/Delta) + 1/2)
// (each step one IEEE-rounded FP32 operation, no contraction); bit plane b of u is written as d-bit
// masks (pl: bq x WP words, or null; L = 64 only), the levels as signed bytes (qbyte: KP bytes, or null),
// and the pair's scalars (the group's first lane writes *rec).
// The dims follow a 64-lane layout (virtual lane v holds v, v + 64, ..., NH of them; any NH >= ceil(d / 64)
// gives the same values); lane g of the group holds virtual lanes g, g + L, ....  ||w||^2 is summed per
// virtual lane, then by the xor butterfly of wave_sum (steps 32, 16, ..., 1), its steps o >= L inside the
// lane, so every L gives the same bits.
// TR (tracing): qp_out / u_out, when not null, receive q' and u of the d dimensions.
template <int NH, int L, bool TR = false>
__device__ __forceinline__ void pair_code(int lane, int q, int j, const float* __restrict__ rq,
                                          const float* __restrict__ RC, int d, int d4, int WP, int bq, float eps0,
                                          const float* __restrict__ Tq, const float* __restrict__ er,
                                          const float* __restrict__ qn2, int KP, PairRec* rec, uint32_t* pl,
                                          int8_t* qbyte, float* qp_out = nullptr, uint8_t* u_out = nullptr) {
    static_assert(L == 16 || L == 32 || L == 64, "lanes per pair");
    constexpr int V = 64 / L;
    const int g = lane & (L - 1);
    float wv[V][NH];
    float pv[V];
#pragma unroll
    for (int t = 0; t < V; t++) {
        pv[t] = 0.f;
#pragma unroll
        for (int h = 0; h < NH; h++) {
            const int i = g + L * t + 64 * h;
            float v = 0.f;
            if (i < d) v = __fsub_rn(rq[(int64_t)q * d4 + i], RC[(int64_t)j * d4 + i]);
            wv[t][h] = v;
            pv[t] = fmaf(v, v, pv[t]);
        }
    }
#pragma unroll
    for (int o = 32; o >= L; o >>= 1) {  // butterfly steps between virtual lanes of one lane
        float nv[V];
#pragma unroll
        for (int t = 0; t < V; t++) nv[t] = pv[t] + pv[t ^ (o / L)];
#pragma unroll
        for (int t = 0; t < V; t++) pv[t] = nv[t];
    }
    float n2 = pv[0];
#pragma unroll
    for (int o = L / 2; o >= 1; o >>= 1) n2 += __shfl_xor(n2, o);
    const float nq = sqrtf(n2);
    float lo = FLT_MAX, hi = -FLT_MAX;
#pragma unroll
    for (int t = 0; t < V; t++) {
#pragma unroll
        for (int h = 0; h < NH; h++) {
            const int i = g + L * t + 64 * h;
            const float v = nq > 0.f ? __fdiv_rn(wv[t][h], nq) : 0.f;
            wv[t][h] = v;
            if (i < d) { lo = fminf(lo, v); hi = fmaxf(hi, v); }
        }
    }
#pragma unroll
    for (int o = L / 2; o >= 1; o >>= 1) {
        lo = fminf(lo, __shfl_xor(lo, o));
        hi = fmaxf(hi, __shfl_xor(hi, o));
    }
    const int levels = (1 << bq) - 1;
    float delta = 1.f;
    int su = 0;
    int uv[V][NH];
    if (hi > lo) {
        delta = __fdiv_rn(__fsub_rn(hi, lo), (float)levels);
        const float inv = __fdiv_rn(1.f, delta);
#pragma unroll
        for (int t = 0; t < V; t++) {
#pragma unroll
            for (int h = 0; h < NH; h++) {
                const int i = g + L * t + 64 * h;
                int u = 0;
                if (i < d) {
                    float tt = __fadd_rn(__fmul_rn(__fsub_rn(wv[t][h], lo), inv), 0.5f);
                    u = (int)floorf(tt);
                    u = u < 0 ? 0 : (u > levels ? levels : u);
                }
                uv[t][h] = u;
                su += u;
            }
        }
    } else {
#pragma unroll
        for (int t = 0; t < V; t++)
#pragma unroll
            for (int h = 0; h < NH; h++) uv[t][h] = 0;
    }
#pragma unroll
    for (int o = L / 2; o >= 1; o >>= 1) su += __shfl_xor(su, o);
    if constexpr (TR) {
        if (qp_out) {
#pragma unroll
            for (int t = 0; t < V; t++) {
#pragma unroll
                for (int h = 0; h < NH; h++) {
                    const int i = g + L * t + 64 * h;
                    if (i < d) {
                        qp_out[i] = wv[t][h];
                        u_out[i] = (uint8_t)uv[t][h];
                    }
                }
            }
        }
    }
    if (qbyte) {  // levels as signed bytes for the i8 matrix-core scan (u - 128 when bq = 8), zero beyond d
        const int ob = bq == 8 ? 128 : 0;
#pragma unroll
        for (int t = 0; t < V; t++) {
#pragma unroll
            for (int h = 0; h < NH; h++) {
                const int i = g + L * t + 64 * h;
                if (i < KP) qbyte[i] = (int8_t)(i < d ? uv[t][h] - ob : 0);
            }
        }
    }
    if constexpr (L == 64) {
        for (int b = 0; pl && b < bq; b++) {
#pragma unroll
            for (int h = 0; h < (NH > 0 ? NH : 1); h++) {
                unsigned long long bm = __ballot(((uv[0][h] >> b) & 1) != 0);
                if (lane == 0) {
                    if (2 * h < WP) pl[b * WP + 2 * h] = (uint32_t)bm;
                    if (2 * h + 1 < WP) pl[b * WP + 2 * h + 1] = (uint32_t)(bm >> 32);
                }
            }
            for (int w = 2 * NH + lane; w < WP; w += 64) pl[b * WP + w] = 0u;  // words beyond the last lane dim
        }
    }
    if (g == 0) {
        PairRec R;
        R.q = q;
        R.list = j;
        R.Kr = (n2 + Tq[q]) - er[q];
        R.two_nq = 2.f * nq;
        R.vl = lo;
        R.delta = delta;
        R.su = (float)su;
        R.ebc = 2.f * nq * eps0 / sqrtf((float)(d - 1));
        R.tau = INFINITY;
        R.er = er[q];
        R.qn2 = qn2[q];
        R.pad = 0.f;
        if (!(hi > lo)) { R.vl = nq > 0.f ? lo : 0.f; }
        *rec = R;
    }
}

// One group of L lanes per (query, list) pair (256 / L pairs per block): its slot in the (phase, list)
// bucket and its query code (the level bytes the scan multiplies; the seed pass builds the bit planes of
// its own pairs).
template <int NH, int L, bool TR>
__global__ __launch_bounds__(256) void k_pair_prep(
    const int32_t* __restrict__ pair_list, const int32_t* __restrict__ pair_q,
    const int64_t* __restrict__ pair_off, const int64_t* __restrict__ pair_total, int nlist, int sh,
    const float* __restrict__ rq,
    const float* __restrict__ RC, int d, int d4, int WP, int bq, float eps0,
    const float* __restrict__ Tq, const float* __restrict__ er, const float* __restrict__ qn2,
    const int32_t* __restrict__ boff, int32_t* __restrict__ fill, int KP,
    PairRec* __restrict__ recs, int8_t* __restrict__ qu8, int32_t* __restrict__ pair_pos, const TraceSink* tr) {
    const int64_t pi = blockIdx.x * (int64_t)(256 / L) + threadIdx.x / L;
    if (pi >= *pair_total) return;  // whole groups: the group's shuffles stay among active lanes
    const int lane = threadIdx.x & 63;
    const int q = pair_q[pi];
    const int j = pair_list[pi];
    const int r = (int)(pi - pair_off[q]);
    const int p = phase_of(r, sh);
    const int first = lane & ~(L - 1);
    int pos = 0;
    if (lane == first) pos = boff[p * nlist + j] + atomicAdd(&fill[p * nlist + j], 1);
    pos = __shfl(pos, first);
    if (lane == first) pair_pos[pi] = pos;
    if constexpr (TR) {
        long long ts = -1;
        if (lane == first && trace_on(tr, q)) ts = trace_pair_slot(tr);
        ts = __shfl(ts, first);
        pair_code<NH, L, true>(lane, q, j, rq, RC, d, d4, WP, bq, eps0, Tq, er, qn2, KP, recs + pos, nullptr,
                               qu8 + (int64_t)pos * KP, ts >= 0 ? tr->qp + ts * d : nullptr,
                               ts >= 0 ? tr->u + ts * d : nullptr);
        if (lane == first && ts >= 0) trace_pair(tr, ts, p, recs[pos]);  // the record this lane just wrote
    } else {
        pair_code<NH, L>(lane, q, j, rq, RC, d, d4, WP, bq, eps0, Tq, er, qn2, KP, recs + pos, nullptr,
                         qu8 + (int64_t)pos * KP);
    }
}

__global__ void k_items(const int32_t* __restrict__ cnt, const int32_t* __restrict__ list_nb, int nlist,
                        int G, int n, int32_t* __restrict__ items) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    int c = cnt[t];
    int j = t % nlist;
    items[t] = c == 0 ? 0 : list_nb[j] * ((c + G - 1) / G);
}

// Work-item descriptors of every phase: item ioff[t] + local of (phase, list) t = p nlist + j is block
// local % nb of list j against the pair chunk local / nb (up to G pairs):
//   {first row of the block, first pair record, number of pairs, list}.
// One wave per (phase, list); items are written in ascending order, neighbouring blocks of a list next
// to each other.
__global__ __launch_bounds__(256) void k_item_desc(const int32_t* __restrict__ ioff, const int32_t* __restrict__ boff,
                                                   const int32_t* __restrict__ list_nb,
                                                   const int64_t* __restrict__ list_off, int nlist, int G,
                                                   int64_t n, int4* __restrict__ desc) {
    const int64_t t = blockIdx.x * 4ll + (threadIdx.x >> 6);
    if (t >= n) return;
    const int lane = threadIdx.x & 63;
    const int i0 = ioff[t], ni = ioff[t + 1] - i0;
    if (ni == 0) return;
    const int j = (int)(t % nlist);
    const int nb = list_nb[j];
    const int b0 = boff[t], b1 = boff[t + 1];
    const int64_t r0 = list_off[j];
    for (int local = lane; local < ni; local += 64) {
        const int blk = local % nb, ch = local / nb;
        const int pbeg = b0 + ch * G;
        desc[i0 + local] = make_int4((int)(r0 + 64ll * blk), pbeg, min(G, b1 - pbeg), j);
    }
}

// ------------------------------------------------------------------------------------------------
// Stage 1 (Eq 4 with the Eq 5 and Eq 6 bounds) of one candidate against one pair, from the integer
// inner product of the candidate's sign code b with the query levels u:
//   ip = sum_i b_i u_i,   I = Delta (2 ip - S_u) + v_l (2 popcount(b) - d) = sqrt(d) <xbar_b, qbar_b>,
//   dis' = (A_x + K) - 2 n_q F_x I,   LB = dis' - ebc E_x - eps_r  (evaluated as (A_x + Kr) - ...).
// stage1_inner = dis' - eps_r; the bound subtracts eps_b = ebc E_x from it with one fused step.
__device__ __forceinline__ float stage1_inner(int ip, int pc, float A, float F, const PairRec& R, int d) {
    const float J1 = (float)(2 * ip - (int)R.su);
    const float J2 = (float)(2 * pc - d);
    const float I = fmaf(R.delta, J1, R.vl * J2);
    return fmaf(-(R.two_nq * F), I, A + R.Kr);
}
__device__ __forceinline__ float stage1_from_ip(int ip, int pc, float A, float F, float E, const PairRec& R,
                                                int d) {
    return fmaf(-R.ebc, E, stage1_inner(ip, pc, A, F, R, d));
}

// The same with ip from the bit planes U_b of the query levels: ip = sum_b 2^b popcount(b & U_b)
// (the seed pass, one candidate per lane).
template <int WP, int BQT>
__device__ __forceinline__ int plane_ip(const uint32_t (&c)[WP], const uint32_t* __restrict__ U, int bq) {
    const int nb = BQT > 0 ? BQT : bq;
    int ip = 0;
#pragma unroll
    for (int b = 0; b < (BQT > 0 ? BQT : 8); b++) {
        if (BQT == 0 && b >= nb) break;
        int acc = 0;
#pragma unroll
        for (int w = 0; w < WP; w++) acc += __builtin_popcount(c[w] & U[b * WP + w]);
        ip += acc << b;
    }
    return ip;
}

// B-bit refinement of a stage-1 survivor (extended code whose top plane is the sign plane), from
// ipB = sum_i ux_i u_i with ux the candidate's level indices:
//   I_B = Delta (2 ipB - (2^B - 1) S_u) + v_l SX_x = 2 <y, qbar'>,
//   dis_B = (A_x + K) - 2 n_q FB_x I_B,   LB_B = dis_B - ebc EB_x - eps_r.
__device__ __forceinline__ float ext_inner(long long ip, int B, float A, float FB, float SX, const PairRec& R) {
    const float J1 = (float)(2 * ip - (long long)((1 << B) - 1) * (long long)R.su);
    const float I = fmaf(R.delta, J1, R.vl * SX);
    return fmaf(-(R.two_nq * FB), I, A + R.Kr);
}
__device__ __forceinline__ float ext_from_ip(long long ip, int B, float A, float FB, float EB, float SX,
                                             const PairRec& R) {
    return fmaf(-R.ebc, EB, ext_inner(ip, B, A, FB, SX, R));
}

// ipB = sum_{a, b} 2^(a + b) popcount(X_a & U_b) from the planes (the seed pass).
__device__ __forceinline__ long long ext_plane_ip(const uint32_t* __restrict__ sign, const uint32_t* __restrict__ extp,
                                                  int B, int WP, const uint32_t* __restrict__ U, int bq) {
    long long ip = 0;
    for (int a = 0; a < B; a++) {
        const uint32_t* X = a == B - 1 ? sign : extp + a * WP;
        for (int b = 0; b < bq; b++) {
            int acc = 0;
            for (int w = 0; w < WP; w++) acc += __builtin_popcount(X[w] & U[b * WP + w]);
            ip += (long long)acc << (a + b);
        }
    }
    return ip;
}

struct ScanCtx {
    const PairRec* recs;
    const int8_t* qu8;   // per pair: KP signed bytes u_i - ob (0 beyond d), i8 matrix-core operand
    const int32_t* boff;
    const int32_t* ioff;
    const int4* desc;    // work-item descriptors of all phases (k_item_desc)
    const int64_t* list_off;
    const int32_t* list_nb;
    const int32_t* list_len;
    const uint32_t* code;
    const uint32_t* ext;
    const float *fA, *fF, *fE, *fFB, *fEB, *fSX;
    const float* xd;
    const float* ax;
    const float* X;
    const int32_t* ids;
    const float* qd;
    const float* qpad;
    const float* qn2;
    const float* er;
    const int32_t* kq;
    const int32_t* npq;
    const int64_t* slot_off;
    const int64_t* pair_off;
    const int32_t* pair_pos;
    unsigned long long* slots;
    int32_t* surv;       // exact-stage candidates of the current phase: rows, in a bin of cq entries per query
    int32_t* qcnt;       // candidates offered to each query's bin (the first cq are in it); zero between phases
    int64_t* counters;
    // inputs of the seed pass's own pair code (it runs beside the pair preparation)
    const int32_t* pair_list;
    const float* rq;
    const float* RC;
    const float* Tq;
    const TraceSink* tr;  // tracing instantiations only
    int cnt_ext;          // counters has 16 entries: the scan also counts its work units into [8..11]
    int split;            // split exact stage: exact = fmaf(-2, <x_r, q_r>, dis_o') from the tail rows
    int Dr4;              // tail row length (split)
    int RX4;              // length of the row the exact stage reads: Dr4 (split) or D4
    const float* xr;      // Npad x Dr4 tail rows (split)
    const float* qr;      // nq x Dr4 query tails, FP32 (split)
    float* survd;         // split: dis_o' of each exact-stage candidate, beside surv
    float eps0;
    int nlist, d, d4, D4, B, bq, WP, KI, KP, G, stage2, use_ext, phase, k_max, cq;
};

// The launch context of a kernel that takes a ScanCtx as its only argument, read again from the kernel-argument
// segment through a pointer the compiler cannot see through: the fields that only rarely taken paths use are
// then loaded where they are used, instead of being held in scalar registers across the whole kernel (which
// spilled them into vector registers).
__device__ __forceinline__ const ScanCtx& ctx_here() {
    const __attribute__((address_space(4))) char* k =
        (const __attribute__((address_space(4))) char*)__builtin_amdgcn_kernarg_segment_ptr();
    asm volatile("" : "+s"(k));
    return *reinterpret_cast<const ScanCtx*>((const char*)k);
}

__device__ __forceinline__ float ord_to_float(uint32_t o) {
    return __uint_as_float((o & 0x80000000u) ? (o & 0x7FFFFFFFu) : ~o);
}

// ------------------------------------------------------------------------------------------------
// Batched scan of one phase (list-major, persistent), stages 1 to 2 on the matrix cores.
//
// A work item is (list j, 64-row block, chunk of up to GT pair records of list j in this phase).  The
// wave treats it as a 64-row x GT-query tile, in 16 x 16 sub-tiles (rows = candidates, columns =
// queries):
//   stage 1   ip = <b_x, u_q> for all pairs of the sub-tile with v_mfma_i32_16x16x64_i8 (sign bits
//             expanded to bytes in registers, query levels stored as bytes per pair), then the Eq 4-6
//             test per entry;
//   B bits    where any entry survived: ipB = <ux_x, u_q> the same way from the extended levels;
//   stage 2   where any entry survived: <x_d, q_d> for the sub-tile with a v_mfma_f32_16x16x4_f32 chain
//             and the Eq 7 test.
// Integer products are exact; the FP32 chain rounds every element in the fixed order of dot_lane, so an
// entry's values do not depend on its position in the tile, i.e. on the other queries of the batch.
// Survivors go to their query's bin of the phase's exact-stage buffer (one atomic per sub-tile and query
// with survivors); entries beyond a bin's capacity get their exact distance inside this kernel, with the
// same arithmetic as k_exact.  Every decision of a
// phase uses the phase threshold stored in the pair record, so the set of candidates reaching each
// stage does not depend on the order in which items run.

// 4 bits -> 4 bytes holding 0 or 1 (byte e <- bit e); the shifted copies never overlap, so no carries.
__device__ __forceinline__ int nib_bytes(uint32_t n) { return (int)(((n & 0xFu) * 0x00204081u) & 0x01010101u); }

// Bits of dimensions 64m + 16g .. 64m + 16g + 15 of a plane of WP words (bits beyond d are 0), as the
// byte operand of lane group g in K-slice m: byte 4t + e of the operand is dimension 64m + 16g + 4t + e.
__device__ __forceinline__ uint32_t plane_piece(const uint32_t* __restrict__ plane, int WP, int m, int g) {
    const int w = 2 * m + (g >> 1);
    const uint32_t word = plane[w < WP ? w : 0];  // unconditional load; words beyond WP read as 0
    return w < WP ? (word >> ((g & 1) << 4)) & 0xFFFFu : 0u;
}
// Query operand of K-slice m (qb points at a valid pair; an invalid column is zeroed after the load).
__device__ __forceinline__ i32x4 qop(const int8_t* __restrict__ qb, int m, bool qv) {
    const i32x4 v = *reinterpret_cast<const i32x4*>(qb + 64 * m);
    return qv ? v : i32x4{0, 0, 0, 0};
}
__device__ __forceinline__ i32x4 piece_bytes(uint32_t p) {
    i32x4 r;
    r.x = nib_bytes(p);
    r.y = nib_bytes(p >> 4);
    r.z = nib_bytes(p >> 8);
    r.w = nib_bytes(p >> 12);
    return r;
}

// Exact distances of the sub-tile entries in mask m (bit l: row rbase + (l & 15), query of pair slot
// cbase + 4 (l >> 4) + v) that did not fit the buffer, four at a time, into the result queues.
template <bool SPL>
__device__ void finish_inline(const ScanCtx& c, const PairRec* rec, unsigned long long m, int64_t rbase,
                              int cbase, int v, int lane, const float* dso) {
    const int first = __ffsll((long long)m) - 1;  // a valid entry, evaluated by groups without one
    while (m) {
        const int src = take4(&m, lane);
        const int s0 = src < 0 ? first : src;
        const int64_t row = rbase + (s0 & 15);
        const int q = rec[cbase + 4 * (s0 >> 4) + v].q;
        // split: dis_o' of the entry from the wave's stash (lane s0 of the sub-tile's slot)
        const float dist = SPL ? split_dist(dso[s0], row_group_small(c.xr + row * c.Dr4, c.qr + (int64_t)q * c.Dr4,
                                                                      c.Dr4, lane & 15, true))
                               : exact_dist_group_small(c.X + row * c.D4, c.qpad + (int64_t)q * c.D4, c.D4, lane & 15);
        if (src >= 0 && (lane & 15) == 0) {
            unsigned long long* slots = c.slots + c.slot_off[q];
            const int k = c.kq[q];
            const uint32_t db = __float_as_uint(dist);
            if (db <= last_dist_bits(slots, k)) topk_insert(slots, k, ((unsigned long long)db << 32) | (uint32_t)c.ids[row]);
        }
    }
}

__device__ __forceinline__ int4 const_load4(const int4* p) {
    const uint32_t* w = reinterpret_cast<const uint32_t*>(p);
    return make_int4((int)const_load(w), (int)const_load(w + 1), (int)const_load(w + 2), (int)const_load(w + 3));
}

// <q_d, x_d> for the 16 x 16 sub-tile (A operand: the query of pair slot li, B operand: row li), lane
// group kg feeding dimensions 16t + 4kg .. 16t + 4kg + 3 of slice t.  Both row pointers are valid rows
// (already offset by 4kg); slices beyond d4 and an invalid query column read offset 0 and are zeroed, so
// every load is an unconditional dwordx4.  SU > 0: at most SU slices, two loaded ahead of their
// multiply-adds; SU = 0: any d4.
__device__ __forceinline__ void mfma4(f32x4& acc, const float4& q, const float4& x) {
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(q.x, x.x, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(q.y, x.y, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(q.z, x.z, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(q.w, x.w, acc, 0, 0, 0);
}
__device__ __forceinline__ float4 zero_unless(float4 v, bool keep) {
    return make_float4(keep ? v.x : 0.f, keep ? v.y : 0.f, keep ? v.z : 0.f, keep ? v.w : 0.f);
}
template <int SU>
__device__ __forceinline__ f32x4 dot_tile(const float* __restrict__ qp, const float* __restrict__ xp, bool qv,
                                          int d4, int kg) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    const float4* __restrict__ q4 = reinterpret_cast<const float4*>(qp);
    const float4* __restrict__ x4 = reinterpret_cast<const float4*>(xp);
    if (SU > 0) {
        constexpr int CH = 2;
#pragma unroll
        for (int t0 = 0; t0 < (SU > 0 ? SU : 1); t0 += CH) {
            float4 xa[CH], qa[CH];
#pragma unroll
            for (int u = 0; u < CH; u++) {
                const bool in = 16 * (t0 + u) + 4 * kg < d4;
                const int o = in ? 4 * (t0 + u) : 0;
                xa[u] = zero_unless(x4[o], in);
                qa[u] = zero_unless(q4[o], in && qv);
            }
#pragma unroll
            for (int u = 0; u < CH; u++) mfma4(acc, qa[u], xa[u]);
        }
    } else {
        for (int t = 0; 16 * t < d4; t++) {
            const bool in = 16 * t + 4 * kg < d4;
            const int o = in ? 4 * t : 0;
            mfma4(acc, zero_unless(q4[o], in && qv), zero_unless(x4[o], in));
        }
    }
    return acc;
}

// The same product with the row tile's x_d slices already in registers (SU slices covering d4 = 16 SU
// exactly, the LDS-staged form's shape: no slice needs zeroing, so nothing touches the loaded registers
// before their products and the loads stay in flight until then).
template <int SU>
__device__ __forceinline__ void load_x_slices(float4 (&xa)[SU], const float* __restrict__ xp) {
    const float4* __restrict__ x4 = reinterpret_cast<const float4*>(xp);
#pragma unroll
    for (int t = 0; t < SU; t++) xa[t] = x4[4 * t];
}
template <int SU>
__device__ __forceinline__ f32x4 dot_tile_x(const float4 (&xa)[SU], const float* __restrict__ qp, bool qv, int d4,
                                            int kg) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    const float4* __restrict__ q4 = reinterpret_cast<const float4*>(qp);
    float4 qa[SU];
#pragma unroll
    for (int t = 0; t < SU; t++) {
        const bool in = 16 * t + 4 * kg < d4;
        qa[t] = zero_unless(q4[in ? 4 * t : 0], in && qv);
    }
#pragma unroll
    for (int t = 0; t < SU; t++) mfma4(acc, qa[t], xa[t]);
    return acc;
}

// LDS staging of an item's q_d rows for stage 2 (QL): rows of d4 floats, d4 a multiple of 64, float4
// column f of pair slot s stored at f ^ (s & 15), so the 16 lanes of a lane group read 16 different banks.
__device__ __forceinline__ int qsh_index(int slot, int f4, int nf4) { return slot * nf4 + (f4 ^ (slot & 15)); }

// One phase of the batched scan.  KIT > 0: d <= 64 KIT (stage-1 operands of an item loaded up front);
// KIT = 0: any d.  QL (d4 = 64 KIT, KIT <= 2): operands reach LDS by direct global-to-LDS loads ahead of
// their use (the next item's stage-1 operands during the current item, the current item's q_d rows at its
// start) and the x_d slices of a row tile are loaded while the previous tile is multiplied.
// The LDS-staged form at 16 queries per item sits at the edge of two waves per SIMD (VGPRs + AGPRs <= 256).
// Declaring that occupancy (a minimum of two waves) made the compiler keep the accumulators out of AGPRs and
// the scan 25 % slower (measured), so the budget is left to the compiler's own heuristic.
// EXT = false: an index without extended codes (B = 1) or a search without the B-bit refinement; the
// refinement's code (and the registers it holds) is then not in the kernel at all.
template <int GT, int KIT, bool QL, bool TR, bool SPL, bool EXT = true>
__global__ __launch_bounds__(256) void k_scan(ScanCtx c) {
    constexpr int NCT = GT / 16;
    constexpr int KA = KIT > 0 ? KIT : 1;
    constexpr int XS = QL && KIT > 0 ? 4 * KIT : 1;  // x_d slices of a row tile held in registers
    static_assert(!QL || (KIT == 1 || KIT == 2), "QL: one direct load per lane covers an item's code block");
    // QL staging area of the next item's stage-1 operands, per wave: the 64-row code block (64 x WP <= 2 KA
    // words), the A, F, E factors of the block, the query levels of up to GT pairs (KP = 64 KA bytes each)
    constexpr int PF_CODE = QL ? 512 * KA : 16;
    constexpr int PF_FAC = QL ? 768 : 16;
    constexpr int PF_LEV = QL ? GT * 64 * KA : 16;
    __shared__ PairRec sh_rec[4][GT];
    __shared__ unsigned long long sh_m[4][NCT * 16];  // surviving entries per (column tile, row tile, v)
    __shared__ uint4 sh_pf[4][(PF_CODE + PF_FAC + PF_LEV) / 16];
    extern __shared__ float4 qsh_dyn[];               // QL: 4 x GT rows of d4 / 4 float4
    typedef __attribute__((address_space(3))) void* lds_ptr;
    const int lane = lane_id();
    const int wv = threadIdx.x >> 6;
    const int li = lane & 15, kg = lane >> 4;
    const int p = c.phase;
    const int base_item = (int)const_load((const uint32_t*)(c.ioff + p * c.nlist));
    const int total = (int)const_load((const uint32_t*)(c.ioff + (p + 1) * c.nlist)) - base_item;
    const int KI = KIT > 0 ? KIT : c.KI;
    const int nf4 = c.d4 >> 2;
    const int ob = c.bq == 8 ? 128 : 0;  // query levels are stored as the signed bytes u - ob
    const int oa = c.B == 8 ? 128 : 0;   // extended levels enter the product as the signed bytes ux - oa
    const bool do_ext = EXT && c.B > 1 && c.use_ext;
    const int WP = c.WP;
    PairRec* rec = sh_rec[wv];
    unsigned long long* msk = sh_m[wv];
    uint4* pf = sh_pf[wv];
    float4* qsh = qsh_dyn + (QL ? wv * GT * nf4 : 0);
    // split: the stage-2 value of each entry, indexed like the masks (slot (ct * 4 + rt) * 4 + v, lane), after
    // the q_d rows in dynamic LDS
    float* dstash = reinterpret_cast<float*>(qsh_dyn + (QL ? 4 * GT * nf4 : 0)) + wv * (NCT * 16 * 64);
    const int wid = uniform(blockIdx.x * 4 + wv);
    int nreg = 0;  // candidates this wave passed to the exact stage (bins or in place)
    long long nscan = 0, n1 = 0, next = 0;
    // extended counters: row tiles whose x_d entered stage 2, accumulated in the wave's LDS slot (nothing
    // held in registers across items); the wave's item count follows from the loop bounds
    __shared__ int sh_tiles[4];
    if (lane == 0) sh_tiles[wv] = 0;
    // Items are dealt to the waves round-robin (neighbouring waves take neighbouring blocks of a list).
    // Descriptors are read two items ahead; the pair records of the next item travel in registers (three
    // float4 per lane) until they are stored.
    const int nwaves = gridDim.x * 4;
    auto fetch_recs = [&](const int4 d, float4& r0, float4& r1, float4& r2) {
        const float4* rp = reinterpret_cast<const float4*>(c.recs + d.y + (lane < d.z ? lane : 0));
        r0 = rp[0];
        r1 = rp[1];
        r2 = rp[2];
    };
    // QL: the stage-1 operands of item d into this wave's staging area (rows d.x .. d.x + 63, pairs d.y ..
    // d.y + d.z - 1; every source is 16-byte aligned)
    auto stage_operands = [&](const int4 d) {
        if (lane < 16 * WP)
            __builtin_amdgcn_global_load_lds((const void*)(reinterpret_cast<const uint4*>(c.code + (int64_t)d.x * WP) + lane),
                                             (lds_ptr)pf, 16, 0, 0);
        if (lane < 48) {
            const float* fb = lane < 16 ? c.fA : (lane < 32 ? c.fF : c.fE);
            __builtin_amdgcn_global_load_lds((const void*)(reinterpret_cast<const uint4*>(fb + d.x) + (lane & 15)),
                                             (lds_ptr)(pf + PF_CODE / 16), 16, 0, 0);
        }
        const int nlev = d.z * (c.KP >> 4);
        const uint4* ls = reinterpret_cast<const uint4*>(c.qu8 + (int64_t)d.y * c.KP);
        for (int e0 = 0; e0 < nlev; e0 += 64)
            if (e0 + lane < nlev)
                __builtin_amdgcn_global_load_lds((const void*)(ls + e0 + lane),
                                                 (lds_ptr)(pf + (PF_CODE + PF_FAC) / 16 + e0), 16, 0, 0);
    };
    int4 dcur = make_int4(0, 0, 1, 0), dnext = dcur;
    float4 r0 = make_float4(0.f, 0.f, 0.f, 0.f), r1 = r0, r2 = r0;
    if (wid < total) {
        dcur = const_load4(c.desc + base_item + wid);
        fetch_recs(dcur, r0, r1, r2);
        if (QL) {
            stage_operands(dcur);
            __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): the first item's staged operands have landed
        }
        if (wid + nwaves < total) dnext = const_load4(c.desc + base_item + wid + nwaves);
    }
    for (int it = wid; it < total; it += nwaves) {
        const int64_t row0 = dcur.x;
        const int pbeg = dcur.y, ng = dcur.z;
        const int nct = (ng + 15) >> 4;
        if (lane < ng) {
            float4* rw = reinterpret_cast<float4*>(rec + lane);
            rw[0] = r0;
            rw[1] = r1;
            rw[2] = r2;
        }
        // stage-1 operands of this item into registers: QL from the staging area (which is then refilled
        // for the next item), otherwise from global memory
        uint32_t cw[4][KA];
        float fa[4], ff[4], fe[4];
        i32x4 qa[NCT][KA];
        if (KIT > 0) {
            if (QL) {
                // this item's staged operands have landed: the previous item waited for them before its stage
                // 2 (the first item, in the prologue), so the stores still in flight from the previous item's
                // bins are not waited for here
                wave_lds_fence();
                const uint32_t* pcode = reinterpret_cast<const uint32_t*>(pf);
                const float* pfac = reinterpret_cast<const float*>(pf + PF_CODE / 16);
                const int8_t* plev = reinterpret_cast<const int8_t*>(pf + (PF_CODE + PF_FAC) / 16);
#pragma unroll
                for (int rt = 0; rt < 4; rt++) {
                    const int r = 16 * rt + li;
#pragma unroll
                    for (int m = 0; m < KA; m++) {
                        const int w = 2 * m + (kg >> 1);
                        const uint32_t word = pcode[r * WP + (w < WP ? w : 0)];
                        cw[rt][m] = w < WP ? (word >> ((kg & 1) << 4)) & 0xFFFFu : 0u;
                    }
                    fa[rt] = pfac[r];
                    ff[rt] = pfac[64 + r];
                    fe[rt] = pfac[128 + r];
                }
                // columns beyond ng read stale levels: they only reach their own (never tested) outputs
#pragma unroll
                for (int ct = 0; ct < NCT; ct++)
#pragma unroll
                    for (int m = 0; m < KA; m++)
                        qa[ct][m] = *reinterpret_cast<const i32x4*>(plev + (ct * 16 + li) * c.KP + 16 * kg + 64 * m);
                __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0): read out before the area is refilled
                wave_lds_fence();
            } else {
#pragma unroll
                for (int rt = 0; rt < 4; rt++) {
                    const int64_t row = row0 + 16 * rt + li;
#pragma unroll
                    for (int m = 0; m < KA; m++) {
                        const int w = 2 * m + (kg >> 1);
                        const uint32_t word = c.code[row * WP + (w < WP ? w : 0)];
                        cw[rt][m] = w < WP ? (word >> ((kg & 1) << 4)) & 0xFFFFu : 0u;
                    }
                    fa[rt] = c.fA[row];
                    ff[rt] = c.fF[row];
                    fe[rt] = c.fE[row];
                }
#pragma unroll
                for (int ct = 0; ct < NCT; ct++) {
                    const int qs = ct * 16 + li;
                    const bool qv = qs < ng;
                    const int8_t* qb = c.qu8 + (int64_t)(pbeg + (qv ? qs : 0)) * c.KP + 16 * kg;
#pragma unroll
                    for (int m = 0; m < KA; m++) qa[ct][m] = qop(qb, m, qv);
                }
            }
        }
        if (QL && c.stage2) {
            // the item's q_d rows into LDS, requested once its stage-1 operands are read out (so that they
            // land during stage 1) and waited for before stage 2; LDS float4 f of slot s holds column
            // f ^ (s & 15) of the slot's query (the swizzle of qsh_index, applied on the source side)
            constexpr int NF4 = 16 * KA;
            const int myq = __float_as_int(r2.x);  // query of the pair held by this lane
            const float4* q4 = reinterpret_cast<const float4*>(c.qd);
            const int tot = ng * NF4;
            for (int e0 = 0; e0 < tot; e0 += 64) {
                const int e = e0 + lane;
                const int slot = e / NF4, f = e - slot * NF4;
                const int qr = __shfl(myq, slot < ng ? slot : 0);
                if (e < tot)
                    __builtin_amdgcn_global_load_lds((const void*)(q4 + (int64_t)qr * NF4 + (f ^ (slot & 15))),
                                                     (lds_ptr)(qsh + e0), 16, 0, 0);
            }
        }
        // requests for the next item, then the x_d slices and norms of the row tiles (nearly every tile
        // reaches stage 2): tile 0, or at d4 = 64 all four, whose loads are then in flight together
        // (the records are fetched unconditionally, from a valid descriptor either way: a conditional
        // fetch makes the compiler merge the registers right after it, waiting for the loads there)
        int4 dnn = dnext;
        fetch_recs(dnext, r0, r1, r2);
        if (it + nwaves < total) {
            if (QL) stage_operands(dnext);
            if (it + 2 * nwaves < total) dnn = const_load4(c.desc + base_item + it + 2 * nwaves);
        }
        constexpr bool XALL = QL && KIT == 1;
        float4 xs0[XS];
        float ax0 = 0.f;
        float4 xall[XALL ? 3 : 1][XS];
        float axall[XALL ? 3 : 1];
        if (QL && c.stage2) {
            load_x_slices<XS>(xs0, c.xd + (row0 + li) * c.d4 + 4 * kg);
            ax0 = c.ax[row0 + li];
            if constexpr (XALL) {
#pragma unroll
                for (int rt = 1; rt < 4; rt++) {
                    load_x_slices<XS>(xall[rt - 1], c.xd + (row0 + 16 * rt + li) * c.d4 + 4 * kg);
                    axall[rt - 1] = c.ax[row0 + 16 * rt + li];
                }
            }
        }

        // ---- stage 1 for every 16 x 16 sub-tile: pass masks into msk ----
        int cnt = 0;
        uint32_t rt1 = 0;  // row tiles holding a stage-1 survivor (wave-uniform, from the ballots)
        // HR (the staged form with one column tile at d_r 64): the pair records of the lane's four query
        // columns are read from LDS once per item and kept in registers for stages 1 and 2, so no row tile
        // waits on them
        constexpr bool HR = QL && NCT == 1 && KIT == 1;
        PairRec Rh[HR ? 4 : 1];
        if (KIT > 0) {
            wave_lds_fence();
            if constexpr (HR) {
#pragma unroll
                for (int v = 0; v < 4; v++) Rh[v] = rec[4 * kg + v < ng ? 4 * kg + v : 0];
            }
#pragma unroll
            for (int rt = 0; rt < 4; rt++) {
                int sp = 0;
#pragma unroll
                for (int m = 0; m < KA; m++) sp += __builtin_popcount(cw[rt][m]);
                const int s2 = sp + __shfl_xor(sp, 16);
                const int pc = s2 + __shfl_xor(s2, 32);  // popcount of the whole sign code of the row
#pragma unroll
                for (int ct = 0; ct < NCT; ct++) {
                    if (ct < nct) {
                        i32x4 acc = {0, 0, 0, 0};
#pragma unroll
                        for (int m = 0; m < KA; m++)
                            acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(qa[ct][m], piece_bytes(cw[rt][m]), acc, 0, 0, 0);
#pragma unroll
                        for (int v = 0; v < 4; v++) {
                            const int g = ct * 16 + 4 * kg + v;
                            const PairRec& R = HR ? Rh[HR ? v : 0] : rec[g < ng ? g : 0];
                            const bool ps = g < ng &&
                                            stage1_from_ip(acc[v] + ob * pc, pc, fa[rt], ff[rt], fe[rt], R, c.d) < R.tau;
                            if constexpr (TR) {
                                if (g < ng && trace_on(c.tr, R.q)) {
                                    const int ip = acc[v] + ob * pc;
                                    const float in1 = stage1_inner(ip, pc, fa[rt], ff[rt], R, c.d);
                                    trace_cand(c.tr, MRQ_TRACE_STAGE1, p, R.q, R.list, c.ids[row0 + 16 * rt + li], ip, pc,
                                               in1, R.ebc * fe[rt], fmaf(-R.ebc, fe[rt], in1), R.tau);
                                }
                            }
                            const unsigned long long mv = __ballot(ps);
                            if (lane == 0) msk[(ct * 4 + rt) * 4 + v] = mv;
                            cnt += __popcll(mv);
                            rt1 |= (mv != 0ull ? 1u : 0u) << rt;
                        }
                    }
                }
            }
        } else {
            wave_lds_fence();
            for (int rt = 0; rt < 4; rt++) {
                const int64_t row = row0 + 16 * rt + li;
                const uint32_t* cp = c.code + row * WP;
                int sp = 0;
                for (int m = 0; m < KI; m++) sp += __builtin_popcount(plane_piece(cp, WP, m, kg));
                const int s2 = sp + __shfl_xor(sp, 16);
                const int pc = s2 + __shfl_xor(s2, 32);
                const float A = c.fA[row], F = c.fF[row], E = c.fE[row];
                for (int ct = 0; ct < nct; ct++) {
                    const int qs = ct * 16 + li;
                    const bool qv = qs < ng;
                    const int8_t* qb = c.qu8 + (int64_t)(pbeg + (qv ? qs : 0)) * c.KP + 16 * kg;
                    i32x4 acc = {0, 0, 0, 0};
                    for (int m = 0; m < KI; m++)
                        acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(qop(qb, m, qv), piece_bytes(plane_piece(cp, WP, m, kg)),
                                                                     acc, 0, 0, 0);
#pragma unroll
                    for (int v = 0; v < 4; v++) {
                        const int g = ct * 16 + 4 * kg + v;
                        const PairRec& R = rec[g < ng ? g : 0];
                        const bool ps = g < ng && stage1_from_ip(acc[v] + ob * pc, pc, A, F, E, R, c.d) < R.tau;
                        if constexpr (TR) {
                            if (g < ng && trace_on(c.tr, R.q)) {
                                const int ip = acc[v] + ob * pc;
                                const float in1 = stage1_inner(ip, pc, A, F, R, c.d);
                                trace_cand(c.tr, MRQ_TRACE_STAGE1, p, R.q, R.list, c.ids[row], ip, pc, in1, R.ebc * E,
                                           fmaf(-R.ebc, E, in1), R.tau);
                            }
                        }
                        const unsigned long long mv = __ballot(ps);
                        if (lane == 0) msk[(ct * 4 + rt) * 4 + v] = mv;
                        cnt += __popcll(mv);
                    }
                }
            }
        }
        nscan += 64ll * ng;
        n1 += cnt;

        wave_lds_fence();
        // ---- B-bit refinement of the stage-1 survivors ----
        if (cnt > 0 && do_ext) {
            const ScanCtx& ce = ctx_here();  // (a rarely taken path: its fields loaded here)
            cnt = 0;
            for (int rt = 0; rt < 4; rt++) {
                const int64_t row = row0 + 16 * rt + li;
                const uint32_t* cp = ce.code + row * WP;
                const uint32_t* ew = ce.ext + row * (int64_t)(ce.B - 1) * WP;
                for (int ct = 0; ct < nct; ct++) {
                    unsigned long long mv[4];
                    bool any = false;
#pragma unroll
                    for (int v = 0; v < 4; v++) { mv[v] = msk[(ct * 4 + rt) * 4 + v]; any |= mv[v] != 0; }
                    if (!any) continue;
                    const int qs = ct * 16 + li;
                    const bool qv = qs < ng;
                    const int8_t* qb = ce.qu8 + (int64_t)(pbeg + (qv ? qs : 0)) * ce.KP + 16 * kg;
                    i32x4 acc2 = {0, 0, 0, 0};
                    for (int m = 0; m < KI; m++) {
                        i32x4 ub = piece_bytes(plane_piece(cp, WP, m, kg)) << (ce.B - 1);
                        for (int a = 0; a < ce.B - 1; a++) ub |= piece_bytes(plane_piece(ew + a * WP, WP, m, kg)) << a;
                        if (oa) ub ^= (int)0x80808080u;
                        acc2 = __builtin_amdgcn_mfma_i32_16x16x64_i8(qop(qb, m, qv), ub, acc2, 0, 0, 0);
                    }
                    const float A = ce.fA[row], FB = ce.fFB[row], EB = ce.fEB[row], SX = ce.fSX[row];
                    const long long sumux = ((long long)SX + (long long)((1 << ce.B) - 1) * ce.d) / 2;
#pragma unroll
                    for (int v = 0; v < 4; v++) {
                        bool ps = (mv[v] >> lane) & 1ull;
                        if (ps) {
                            const PairRec& R = rec[ct * 16 + 4 * kg + v];
                            // sum_i ux_i u_i from sum_i (ux_i - oa)(u_i - ob) over the d real dimensions
                            const long long ipB = (long long)acc2[v] + ob * sumux + oa * (long long)R.su -
                                                  (long long)oa * ob * ce.d;
                            ps = ext_from_ip(ipB, ce.B, A, FB, EB, SX, R) < R.tau;
                            if constexpr (TR) {
                                if (trace_on(ce.tr, R.q)) {
                                    const float inB = ext_inner(ipB, ce.B, A, FB, SX, R);
                                    trace_cand(ce.tr, MRQ_TRACE_EXT, p, R.q, R.list, ce.ids[row], (int)ipB, 0, inB,
                                               R.ebc * EB, fmaf(-R.ebc, EB, inB), R.tau);
                                }
                            }
                        }
                        const unsigned long long nm = __ballot(ps);
                        if (lane == 0) msk[(ct * 4 + rt) * 4 + v] = nm;
                        cnt += __popcll(nm);
                    }
                }
            }
            wave_lds_fence();
        }
        next += cnt;
        if constexpr (QL) {  // (the staged form always runs stage 2; a compile-time branch keeps the
                             // compiler's own wait tracking aware of this wait)
            __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): the item's q_d rows have landed in LDS
            wave_lds_fence();
        }

        // ---- stage 2 (Eq 7) of the remaining survivors ----
        if (cnt > 0 && c.stage2) {
            cnt = 0;
            if constexpr (QL) {
                // row tiles holding a surviving entry (wave-uniform): stage 1's, unless the B-bit refinement
                // has since cleared entries
                uint32_t rtany = rt1;
                if (do_ext) {
                    rtany = 0;
#pragma unroll
                    for (int rt = 0; rt < 4; rt++)
                        for (int ct = 0; ct < nct; ct++)
#pragma unroll
                            for (int v = 0; v < 4; v++) rtany |= (msk[(ct * 4 + rt) * 4 + v] != 0ull ? 1u : 0u) << rt;
                }
                if (c.cnt_ext && lane == 0) sh_tiles[wv] += __popc(rtany);
                float4 xb[2][XS];
                float axb[2] = {0.f, 0.f};
                // HR: the q_d slices of the lane's query row (the same for every row tile), read once
                float4 qh[HR ? XS : 1];
                if constexpr (HR) {
#pragma unroll
                    for (int t = 0; t < XS; t++) qh[t] = qsh[qsh_index(li, 4 * t + kg, nf4)];
                }
#pragma unroll
                for (int rt = 0; rt < 4; rt++) {
                    // the next tile's slices and norms are requested before this tile's products
                    if (!XALL && rt < 3 && ((rtany >> (rt + 1)) & 1u)) {
                        const int64_t rn = row0 + 16 * (rt + 1) + li;
                        load_x_slices<XS>(xb[(rt + 1) & 1], c.xd + rn * c.d4 + 4 * kg);
                        axb[(rt + 1) & 1] = c.ax[rn];
                    }
                    if (!((rtany >> rt) & 1u)) continue;
                    const float4(&xa)[XS] = rt == 0 ? xs0 : (XALL ? xall[rt - 1] : xb[rt & 1]);
                    const float axr = rt == 0 ? ax0 : (XALL ? axall[rt - 1] : axb[rt & 1]);
                    for (int ct = 0; ct < nct; ct++) {
                        unsigned long long mv[4];
                        bool any = false;
#pragma unroll
                        for (int v = 0; v < 4; v++) { mv[v] = msk[(ct * 4 + rt) * 4 + v]; any |= mv[v] != 0; }
                        // (one column tile: the row tile's flag already says that a mask is set, so the
                        // products need not wait for the masks)
                        if (NCT > 1 && !any) continue;
                        // slots beyond ng hold stale rows: they only reach their own (never tested) outputs
                        f32x4 dot = {0.f, 0.f, 0.f, 0.f};
                        if constexpr (HR) {
#pragma unroll
                            for (int t = 0; t < XS; t++) mfma4(dot, qh[t], xa[t]);
                        } else {
                            float4 qv4[XS];
#pragma unroll
                            for (int t = 0; t < XS; t++) qv4[t] = qsh[qsh_index(ct * 16 + li, 4 * t + kg, nf4)];
#pragma unroll
                            for (int t = 0; t < XS; t++) mfma4(dot, qv4[t], xa[t]);
                        }
#pragma unroll
                        for (int v = 0; v < 4; v++) {
                            bool ps = (mv[v] >> lane) & 1ull;
                            if (ps) {
                                const PairRec& R = HR ? Rh[HR ? v : 0] : rec[ct * 16 + 4 * kg + v];
                                const float dso = fmaf(-2.f, dot[v], axr + R.qn2);
                                ps = dso - R.er < R.tau;
                                if constexpr (SPL) dstash[((ct * 4 + rt) * 4 + v) * 64 + lane] = dso;
                                if constexpr (TR) {
                                    if (trace_on(c.tr, R.q))
                                        trace_cand(c.tr, MRQ_TRACE_STAGE2, p, R.q, R.list, c.ids[row0 + 16 * rt + li], 0, 0,
                                                   dso, R.er, dso - R.er, R.tau);
                                }
                            }
                            const unsigned long long nm = __ballot(ps);
                            if (lane == 0) msk[(ct * 4 + rt) * 4 + v] = nm;
                            cnt += __popcll(nm);
                        }
                    }
                }
            } else {
                for (int rt = 0; rt < 4; rt++) {
                    const int64_t row = row0 + 16 * rt + li;
                    bool tile_used = false;
                    for (int ct = 0; ct < nct; ct++) {
                        unsigned long long mv[4];
                        bool any = false;
#pragma unroll
                        for (int v = 0; v < 4; v++) { mv[v] = msk[(ct * 4 + rt) * 4 + v]; any |= mv[v] != 0; }
                        if (!any) continue;
                        tile_used = true;
                        const int qs = ct * 16 + li;
                        const bool qv = qs < ng;
                        const int qrow = rec[qv ? qs : 0].q;
                        const f32x4 dot = dot_tile<4 * KIT>(c.qd + (int64_t)qrow * c.d4 + 4 * kg,
                                                            c.xd + row * c.d4 + 4 * kg, qv, c.d4, kg);
                        const float axr = c.ax[row];
#pragma unroll
                        for (int v = 0; v < 4; v++) {
                            bool ps = (mv[v] >> lane) & 1ull;
                            if (ps) {
                                const PairRec& R = rec[ct * 16 + 4 * kg + v];
                                const float dso = fmaf(-2.f, dot[v], axr + R.qn2);
                                ps = dso - R.er < R.tau;
                                if constexpr (SPL) dstash[((ct * 4 + rt) * 4 + v) * 64 + lane] = dso;
                                if constexpr (TR) {
                                    if (trace_on(c.tr, R.q))
                                        trace_cand(c.tr, MRQ_TRACE_STAGE2, p, R.q, R.list, c.ids[row], 0, 0, dso, R.er,
                                                   dso - R.er, R.tau);
                                }
                            }
                            const unsigned long long nm = __ballot(ps);
                            if (lane == 0) msk[(ct * 4 + rt) * 4 + v] = nm;
                            cnt += __popcll(nm);
                        }
                    }
                    if (c.cnt_ext && lane == 0 && tile_used) sh_tiles[wv] += 1;
                }
            }
            wave_lds_fence();
        }

        // ---- exact-stage candidates into their queries' bins: lane t < ng gathers the rows of query column t
        // (column tile t / 16, lane group t / 4 % 4, v = t % 4) that survived, in (row tile, row) order, reserves
        // room for them with one atomic (one instruction for the whole item) and writes them itself, four at a
        // time with their stage-2 values read together; no step of the writes needs another lane ----
        if (cnt > 0) {
            const int tc = lane >> 4, tg = (lane >> 2) & 3, tv = lane & 3;
            unsigned long long cm = 0ull;  // bit r: row r of the block survived for this lane's column
            int base = 0, n = 0, qcol = 0;
            if (lane < ng) {
#pragma unroll
                for (int rt = 0; rt < 4; rt++)
                    cm |= ((msk[(tc * 4 + rt) * 4 + tv] >> (16 * tg)) & 0xFFFFull) << (16 * rt);
                n = __popcll(cm);
                qcol = rec[lane].q;
                if (n) base = atomicAdd(&c.qcnt[qcol], n);
            }
            // entry (row 16 rt + l, column t) of the stage-2 values sits at slot (tc * 4 + rt) * 4 + tv, lane
            // l + 16 tg (lanes without a column read a slot of column 0, within the wave's stash)
            const float* cst = dstash + (lane < ng ? tc * 1024 + tv * 64 + 16 * tg : 0);
            int r[4];
            float sv[4];
            auto take4 = [&]() {  // the column's next four rows (-1 past its last) and their stage-2 values
#pragma unroll
                for (int u = 0; u < 4; u++) {
                    r[u] = cm ? (int)__builtin_ctzll(cm) : -1;
                    cm &= cm - 1ull;
                }
                if constexpr (SPL) {
#pragma unroll
                    for (int u = 0; u < 4; u++) {
                        const int ru = r[u] < 0 ? 0 : r[u];
                        sv[u] = cst[(ru >> 4) * 256 + (ru & 15)];
                    }
                }
            };
            take4();  // requested before the reservation's result is needed
            for (int i = 0;; i += 4) {
#pragma unroll
                for (int u = 0; u < 4; u++) {
                    const int pos = base + i + u;
                    if (r[u] >= 0 && pos < c.cq) {
                        const int64_t at = (int64_t)qcol * c.cq + pos;
                        c.surv[at] = (int)(row0 + r[u]);
                        if constexpr (SPL) c.survd[at] = sv[u];
                    }
                }
                if (!__ballot(cm != 0ull)) break;
                take4();
            }
            // the reservation is consumed here on every path (an unconsumed result register would make the
            // next item wait for all memory operations in flight before its first write to that register);
            // the writes above wait for it only where they use it, after the stage-2 values are requested
            asm volatile("" ::"v"(base));
            nreg += cnt;
            // a bin that overflowed: its entries beyond the capacity are finished in place, found by the
            // sub-tile walk (which writes the fitting entries again, with the same values)
            if (__ballot(lane < ng && base + n > c.cq)) {
                const ScanCtx& cf = ctx_here();  // (a rarely taken path: its fields loaded here)
                for (int ct = 0; ct < nct; ct++) {
                    int bb[4], off[4];
#pragma unroll
                    for (int v = 0; v < 4; v++) {
                        bb[v] = __shfl(base, ct * 16 + 4 * kg + v);
                        off[v] = 0;
                    }
                    for (int rt = 0; rt < 4; rt++) {
#pragma unroll
                        for (int v = 0; v < 4; v++) {
                            const unsigned long long mv = msk[(ct * 4 + rt) * 4 + v];
                            if (!mv) continue;
                            const bool mine = (mv >> lane) & 1ull;
                            const uint32_t gm = (uint32_t)(mv >> (lane & 48)) & 0xFFFFu;
                            const int pos = bb[v] + off[v] + __popc(gm & ((1u << li) - 1u));
                            off[v] += __popc(gm);
                            const bool fits = mine && pos < c.cq;
                            const int slot = ((ct * 4 + rt) * 4 + v) * 64;
                            if (fits) {
                                const int64_t at = (int64_t)rec[ct * 16 + 4 * kg + v].q * c.cq + pos;
                                c.surv[at] = (int)(row0 + 16 * rt + li);
                                if constexpr (SPL) c.survd[at] = dstash[slot + lane];
                            }
                            const unsigned long long rest = __ballot(mine && !fits);
                            if (rest) finish_inline<SPL>(cf, rec, rest, row0 + 16 * rt, ct * 16, v, lane, dstash + slot);
                        }
                    }
                }
            }
        }
        wave_lds_fence();
        dcur = dnext;
        dnext = dnn;
    }
    if (c.counters && lane == 0) {  // the counts are wave-uniform
        atomicAdd((unsigned long long*)&c.counters[0], (unsigned long long)nscan);
        atomicAdd((unsigned long long*)&c.counters[1], (unsigned long long)n1);
        atomicAdd((unsigned long long*)&c.counters[2], (unsigned long long)next);
        atomicAdd((unsigned long long*)&c.counters[3], (unsigned long long)nreg);
        if (c.cnt_ext) {
            const int items = wid < total ? (total - wid - 1) / nwaves + 1 : 0;
            atomicAdd((unsigned long long*)&c.counters[8], (unsigned long long)items);
            atomicAdd((unsigned long long*)&c.counters[9], (unsigned long long)sh_tiles[wv]);
        }
    }
}

// Exact stage of a phase: block q takes the candidates in query q's bin, 16 lanes per candidate (16 at a
// time).  The block is the only writer of the query's result queue during the launch, so the queue is
// copied to LDS, updated there with the same insertion as in global memory, and written back.  QL: the
// query row is staged in LDS too and read from memory once per block.  Dynamic shared memory: D4 floats
// (QL, D4 <= kExactLdsFloats), then k_max keys.  The bin's count is cleared for the next phase.
constexpr int kExactLdsFloats = 8192;
constexpr int kExactRows = 4;  // candidates per 16-lane group at a time when rows are at most 64 floats

template <bool QL, bool TR, bool SPL>
__global__ __launch_bounds__(256) void k_exact(ScanCtx c) {
    extern __shared__ float4 dyn_x[];
    __shared__ int n_s;
    float4* qs = dyn_x;
    unsigned long long* queue = reinterpret_cast<unsigned long long*>(dyn_x + (QL ? (c.RX4 >> 2) : 0));
    const int q = blockIdx.x;
    const int lane = lane_id();
    if (threadIdx.x == 0) n_s = c.qcnt[q];
    __syncthreads();
    const int n = min(n_s, c.cq);
    if (n == 0) return;
    if (threadIdx.x == 0) c.qcnt[q] = 0;
    // the row the exact stage reads: the query (original coordinates), or its tail (split exact stage)
    const int RX4 = c.RX4;
    const float* qrow = SPL ? c.qr + (int64_t)q * c.Dr4 : c.qpad + (int64_t)q * c.D4;
    if (QL)
        for (int i = threadIdx.x; i < (RX4 >> 2); i += 256) qs[i] = reinterpret_cast<const float4*>(qrow)[i];
    unsigned long long* slots = c.slots + c.slot_off[q];
    const int k = c.kq[q];
    for (int i = threadIdx.x; i < k; i += 256) queue[i] = slots[i];
    __syncthreads();
    const int32_t* bin = c.surv + (int64_t)q * c.cq;
    if (RX4 <= 64) {
        // rows of at most 16 float4 (the split form's short tails): one chunk per lane, so a group takes
        // kExactRows candidates at a time with their loads in flight together; each candidate's sum is the
        // same as the one-candidate form's (its lane's single chunk, then the same 16-lane reduction)
        const int l16 = lane & 15, nc = RX4 >> 2;
        const float4 zero4 = make_float4(0.f, 0.f, 0.f, 0.f);
        const float4 qv = l16 < nc ? (QL ? qs[l16] : reinterpret_cast<const float4*>(qrow)[l16]) : zero4;
        const float* xbase = SPL ? c.xr : c.X;
        const int ld = SPL ? c.Dr4 : c.D4;
        for (int i = threadIdx.x >> 4; i - (lane >> 4) < n; i += 16 * kExactRows) {
            int64_t row[kExactRows];
            float4 xa[kExactRows];
            float dso[kExactRows];
#pragma unroll
            for (int u = 0; u < kExactRows; u++) {
                const int iu = i + 16 * u < n ? i + 16 * u : 0;
                row[u] = bin[iu];
                dso[u] = SPL ? c.survd[(int64_t)q * c.cq + iu] : 0.f;
            }
#pragma unroll
            for (int u = 0; u < kExactRows; u++)
                xa[u] = l16 < nc ? reinterpret_cast<const float4*>(xbase + row[u] * ld)[l16] : zero4;
#pragma unroll
            for (int u = 0; u < kExactRows; u++) {
                const int iu = i + 16 * u;
                const bool valid = iu < n;
                float r = 0.f;
                if (l16 < nc) {
                    if (SPL) acc_dot4(r, xa[u], qv);
                    else acc_sqdiff(r, xa[u], qv);
                }
                for (int o = 8; o >= 1; o >>= 1) r += __shfl_xor(r, o);
                const float dist = SPL ? split_dist(dso[u], r) : r;
                if (valid && l16 == 0) {
                    const uint32_t db = __float_as_uint(dist);
                    if (db <= last_dist_bits(queue, k))
                        topk_insert(queue, k, ((unsigned long long)db << 32) | (uint32_t)c.ids[row[u]]);
                    if constexpr (TR) {
                        if (trace_on(c.tr, q))
                            trace_cand(c.tr, MRQ_TRACE_EXACT, c.phase, q, -1, c.ids[row[u]], 0, 0, dist, 0.f, 0.f, 0.f);
                    }
                }
            }
        }
        __syncthreads();
        for (int i = threadIdx.x; i < k; i += 256) slots[i] = queue[i];
        return;
    }
    for (int i = threadIdx.x >> 4; i - (lane >> 4) < n; i += 16) {
        const bool valid = i < n;
        const int64_t row = bin[valid ? i : 0];
        // the exact distance, or (split) the tail product with dis_o' - 2 <x_r, q_r>
        const float* xrow = SPL ? c.xr + row * c.Dr4 : c.X + row * c.D4;
        const float r = QL ? row_group_lds(xrow, qs, RX4, lane & 15, SPL) : row_group(xrow, qrow, RX4, lane & 15, SPL);
        const float dist = SPL ? split_dist(c.survd[(int64_t)q * c.cq + (valid ? i : 0)], r) : r;
        if (valid && (lane & 15) == 0) {
            const uint32_t db = __float_as_uint(dist);
            if (db <= last_dist_bits(queue, k)) topk_insert(queue, k, ((unsigned long long)db << 32) | (uint32_t)c.ids[row]);
            if constexpr (TR) {
                if (trace_on(c.tr, q))
                    trace_cand(c.tr, MRQ_TRACE_EXACT, c.phase, q, -1, c.ids[row], 0, 0, dist, 0.f, 0.f, 0.f);
            }
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < k; i += 256) slots[i] = queue[i];
}

// Seed pass: each query's nearest list (probe rank 0), one wave per query, before the batched phases,
// so that the first batched phase starts from a finite threshold.  The wave holds the query's result
// queue in LDS and treats the list in two deterministic rounds:
//   1. the s = min(max(k, 32), n') candidates with the smallest (stage-1 lower bound, row) among the first
//      n' = min(n, kSeedMax) rows of the list (found by a bitwise search for the s-th smallest key);
//   2. every other candidate of the list whose bound is below tau, in row order,
// gathered into dense batches of 64; each candidate of a batch goes through the Algorithm 2 steps
// (stage-1 bound, B-bit refinement, Eq 7 re-check, exact distance) against the queue's threshold tau,
// which is updated after every batch.
// Round 1 fills the queue with candidates the estimator ranks best, so round 2 prunes with a tight tau.

constexpr int kSeedMax = 512;  // candidate keys held in LDS for the round-1 selection
constexpr int kSeedFirst = 32;  // round 1 takes at least this many best-bound candidates
constexpr int kSeedLdsFloats = 2048;  // query rows up to this length are staged in LDS
constexpr int kSeedRows = 4;  // short exact rows per lane group at a time

struct QueryState {
    unsigned long long* tk[2];
    int cur, have, k;
    float tau;
    // the current / other queue, selected without indexing the pointer pair (which would put it in scratch)
    __device__ __forceinline__ unsigned long long* now() const { return cur ? tk[1] : tk[0]; }
    __device__ __forceinline__ unsigned long long* other() const { return cur ? tk[0] : tk[1]; }
};

// One batch of at most 64 candidates (one per lane; `pass` = passed stage 1 against st.tau): B-bit
// refinement, Eq 7 re-check, exact distances four at a time, then a merge of the new keys into the
// sorted queue and the new tau.
template <int WP, bool TR, bool SR>
__device__ __forceinline__ void seed_batch(const ScanCtx& c, int q, float er, const PairRec& R, const uint32_t* U, bool pass, int64_t row,
                           QueryState& st, unsigned long long* nk, const float4* qs, bool qlds, int lane,
                           long long* n1, long long* next, long long* n2) {
    *n1 += __popcll(__ballot(pass));
    const bool open = st.tau == INFINITY;  // every test passes until the queue holds k results
    if (pass && !open && c.B > 1 && c.use_ext) {
        const long long ipB = ext_plane_ip(c.code + row * WP, c.ext + row * (c.B - 1) * WP, c.B, WP, U, c.bq);
        const float inB = ext_inner(ipB, c.B, c.fA[row], c.fFB[row], c.fSX[row], R);
        const float lb = fmaf(-R.ebc, c.fEB[row], inB);
        if constexpr (TR) {
            if (trace_on(c.tr, q))
                trace_cand(c.tr, MRQ_TRACE_EXT, 0, q, R.list, c.ids[row], (int)ipB, 0, inB, R.ebc * c.fEB[row], lb,
                           st.tau);
        }
        pass = lb < st.tau;
    }
    *next += __popcll(__ballot(pass));
    // dis_o' (Eq 7): tested once the queue is full; the split exact stage also needs it for every candidate
    // that reaches the exact distance
    float dso = 0.f;
    if (pass && ((!open && c.stage2) || c.split)) {
        const float dot = qlds ? dot_lane_lds(c.xd + row * c.d4, qs + (c.RX4 >> 2), c.d4)
                               : dot_lane(c.xd + row * c.d4, c.qd + (int64_t)q * c.d4, c.d4);
        dso = fmaf(-2.f, dot, c.ax[row] + R.qn2);
        if (!open && c.stage2) {
            pass = dso - er < st.tau;
            if constexpr (TR) {
                if (trace_on(c.tr, q))
                    trace_cand(c.tr, MRQ_TRACE_STAGE2, 0, q, R.list, c.ids[row], 0, 0, dso, er, dso - er, st.tau);
            }
        }
    }
    const unsigned long long m2 = __ballot(pass);
    *n2 += __popcll(m2);
    if (!m2) return;
    // exact distances, four candidates at a time (16 lanes each); rows of at most 64 floats (one chunk per
    // lane) 4 kSeedRows at a time, kSeedRows per lane group, with the same arithmetic per candidate
    unsigned long long mine = kEmptyKey;
    unsigned long long mm = m2;
    const int first = __ffsll((long long)m2) - 1;
    if constexpr (SR) {
        const int l16 = lane & 15, nc = c.RX4 >> 2;
        const float4 zero4 = make_float4(0.f, 0.f, 0.f, 0.f);
        const float* qx = c.split ? c.qr + (int64_t)q * c.Dr4 : c.qpad + (int64_t)q * c.D4;
        const float4 qv = l16 < nc ? (qlds ? qs[l16] : reinterpret_cast<const float4*>(qx)[l16]) : zero4;
        const float* xbase = c.split ? c.xr : c.X;
        const int ld = c.split ? c.Dr4 : c.D4;
        while (mm) {
            int sr[kSeedRows];
            int64_t rs[kSeedRows];
            float4 xa[kSeedRows];
#pragma unroll
            for (int u = 0; u < kSeedRows; u++) {
                sr[u] = take4(&mm, lane);
                rs[u] = __shfl(row, sr[u] < 0 ? first : sr[u]);
            }
#pragma unroll
            for (int u = 0; u < kSeedRows; u++) xa[u] = l16 < nc ? reinterpret_cast<const float4*>(xbase + rs[u] * ld)[l16] : zero4;
            int idv[kSeedRows];  // requested with the rows, so no round trip follows the distances
#pragma unroll
            for (int u = 0; u < kSeedRows; u++) idv[u] = c.ids[rs[u]];
#pragma unroll
            for (int u = 0; u < kSeedRows; u++) {
                float r = 0.f;
                if (l16 < nc) {
                    if (c.split) acc_dot4(r, xa[u], qv);
                    else acc_sqdiff(r, xa[u], qv);
                }
                for (int o = 8; o >= 1; o >>= 1) r += __shfl_xor(r, o);
                const float dist = c.split ? split_dist(__shfl(dso, sr[u] < 0 ? first : sr[u]), r) : r;
                const unsigned long long key = (sr[u] >= 0 && (st.tau == INFINITY || dist <= st.tau))
                                                   ? ((unsigned long long)__float_as_uint(dist) << 32) | (uint32_t)idv[u]
                                                   : kEmptyKey;
                if constexpr (TR) {
                    if (sr[u] >= 0 && l16 == 0 && trace_on(c.tr, q))
                        trace_cand(c.tr, MRQ_TRACE_EXACT, 0, q, R.list, c.ids[rs[u]], 0, 0, dist, 0.f, 0.f, st.tau);
                }
                for (int g = 0; g < 4; g++) {
                    const int sg = __shfl(sr[u], g * 16);
                    const unsigned long long kgv = __shfl(key, g * 16);
                    if (sg >= 0 && lane == sg) mine = kgv;
                }
            }
        }
    } else while (mm) {
        const int src = take4(&mm, lane);
        const int64_t rs = __shfl(row, src < 0 ? first : src);
        const int idv = c.ids[rs];  // requested before the row, so no round trip follows the distance
        // the exact distance, or (split) the tail product with dis_o' - 2 <x_r, q_r>
        const float* xrow = c.split ? c.xr + rs * c.Dr4 : c.X + rs * c.D4;
        const float* qrow = c.split ? c.qr + (int64_t)q * c.Dr4 : c.qpad + (int64_t)q * c.D4;
        const float r = qlds ? row_group_lds(xrow, qs, c.RX4, lane & 15, c.split)
                             : row_group(xrow, qrow, c.RX4, lane & 15, c.split);
        const float dist = c.split ? split_dist(__shfl(dso, src < 0 ? first : src), r) : r;
        // a key whose distance is above a full queue's last cannot survive the merge: it stays empty
        const unsigned long long key = (src >= 0 && (st.tau == INFINITY || dist <= st.tau))
                                           ? ((unsigned long long)__float_as_uint(dist) << 32) | (uint32_t)idv
                                           : kEmptyKey;
        if constexpr (TR) {
            if (src >= 0 && (lane & 15) == 0 && trace_on(c.tr, q))
                trace_cand(c.tr, MRQ_TRACE_EXACT, 0, q, R.list, c.ids[rs], 0, 0, dist, 0.f, 0.f, st.tau);
        }
        for (int g = 0; g < 4; g++) {
            const int sg = __shfl(src, g * 16);
            const unsigned long long kgv = __shfl(key, g * 16);
            if (sg >= 0 && lane == sg) mine = kgv;
        }
    }
    // merge the new keys into the sorted queue
    const unsigned long long sv = wave_sort64(mine, lane);
    const int mnew = __popcll(__ballot(sv != kEmptyKey));
    nk[lane] = sv;
    __syncthreads();
    const unsigned long long* src = st.now();
    unsigned long long* dst = st.other();
    for (int i = lane; i < st.have; i += 64) {  // existing key: rank among the new keys
        const unsigned long long e = src[i];
        int lo = 0, hi = mnew;
        while (lo < hi) { int mid = (lo + hi) >> 1; if (nk[mid] < e) lo = mid + 1; else hi = mid; }
        if (i + lo < st.k) dst[i + lo] = e;
    }
    if (lane < mnew) {
        int lo = 0, hi = st.have;
        while (lo < hi) { int mid = (lo + hi) >> 1; if (src[mid] < sv) lo = mid + 1; else hi = mid; }
        if (lane + lo < st.k) dst[lane + lo] = sv;
    }
    __syncthreads();
    st.cur ^= 1;
    st.have = st.have + mnew < st.k ? st.have + mnew : st.k;
    if (st.have == st.k) st.tau = __uint_as_float((uint32_t)(st.now()[st.k - 1] >> 32));
}

template <int WP, int BQT, bool TR>
__device__ __forceinline__ float seed_lb(const ScanCtx& c, int64_t row, const PairRec& R, const uint32_t* U) {
    uint32_t cw[WP];
    int pc = 0;
#pragma unroll
    for (int w = 0; w < WP; w++) { cw[w] = c.code[row * WP + w]; pc += __builtin_popcount(cw[w]); }
    const int ip = plane_ip<WP, BQT>(cw, U, c.bq);
    const float E = c.fE[row];
    const float in1 = stage1_inner(ip, pc, c.fA[row], c.fF[row], R, c.d);
    const float lb = fmaf(-R.ebc, E, in1);
    if constexpr (TR) {
        if (trace_on(c.tr, R.q))
            trace_cand(c.tr, MRQ_TRACE_STAGE1, 0, R.q, R.list, c.ids[row], ip, pc, in1, R.ebc * E, lb, NAN);
    }
    return lb;
}

// SR: rows of the exact stage of at most 64 floats (RX4 <= 64), taken several per lane group at a time
template <int WP, int BQT, bool TR, bool SR>
__global__ __launch_bounds__(64) void k_seed(ScanCtx c) {
    __shared__ unsigned long long nk[64];
    __shared__ int32_t pend_row[128];
    __shared__ float pend_lb[128];
    extern __shared__ unsigned long long dyn[];  // queue: 2 x k_max keys, kSeedMax candidate keys, query rows
    const int q = blockIdx.x;
    const int lane = threadIdx.x;
    if (c.npq[q] == 0 || c.kq[q] == 0) return;  // a query without pairs (rejected by the mixed-batch check)
    QueryState st;
    st.tk[0] = dyn;
    st.tk[1] = dyn + c.k_max;
    unsigned long long* keys = dyn + 2 * c.k_max;
    // the query row (exact distances) and q_d (stage 2) in LDS, D4 + d4 floats (D4 <= kSeedLdsFloats)
    const bool qlds = c.RX4 <= kSeedLdsFloats;
    float4* qs = reinterpret_cast<float4*>(keys + kSeedMax);
    if (qlds) {
        const float* qx = c.split ? c.qr + (int64_t)q * c.Dr4 : c.qpad + (int64_t)q * c.D4;
        for (int i = lane; i < (c.RX4 >> 2); i += 64) qs[i] = reinterpret_cast<const float4*>(qx)[i];
        for (int i = lane; i < (c.d4 >> 2); i += 64)
            qs[(c.RX4 >> 2) + i] = reinterpret_cast<const float4*>(c.qd + (int64_t)q * c.d4)[i];
    }
    st.cur = 0;
    st.k = c.kq[q];
    st.have = 0;
    st.tau = INFINITY;
    const float er = c.er[q];
    // the query code of the pair (q, nearest list), computed here into LDS
    __shared__ PairRec sh_R;
    __shared__ uint32_t sh_U[8 * WP];
    const int j = c.pair_list[c.pair_off[q]];
    long long ts = -1;  // trace record of the pair (tracing instantiation)
    if constexpr (TR) {
        if (lane == 0 && trace_on(c.tr, q)) ts = trace_pair_slot(c.tr);
        ts = __shfl(ts, 0);
    }
    pair_code<(WP <= 2 ? 1 : WP / 2), 64, TR>(lane, q, j, c.rq, c.RC, c.d, c.d4, WP, c.bq, c.eps0, c.Tq, c.er, c.qn2, 0,
                                              &sh_R, sh_U, nullptr, TR && ts >= 0 ? c.tr->qp + ts * c.d : nullptr,
                                              TR && ts >= 0 ? c.tr->u + ts * c.d : nullptr);
    __syncthreads();
    if constexpr (TR) {
        if (lane == 0 && ts >= 0) trace_pair(c.tr, ts, 0, sh_R);
    }
    const PairRec R = sh_R;
    const uint32_t* U = sh_U;
    const int n = c.list_len[j];
    const int64_t base = c.list_off[j];
    const int nsel = n < kSeedMax ? n : kSeedMax;
    long long n1 = 0, next = 0, n2 = 0;
    // round 1: keys (ord(lb), row) of the first nsel rows, and the s-th smallest of them (two chunks of 64
    // rows with their loads in flight together)
#pragma unroll 2
    for (int i = lane; i < nsel; i += 64) {
        const float lb = seed_lb<WP, BQT, TR>(c, base + i, R, U);
        keys[i] = ((unsigned long long)ord_bits(lb) << 32) | (uint32_t)i;
    }
    __syncthreads();
    const int s0 = st.k > kSeedFirst ? st.k : kSeedFirst;
    const int s = s0 < nsel ? s0 : nsel;
    // the s-th smallest key: the largest value with fewer than s keys below it, by a bitwise search over
    // the keys held in registers (slot u of lane l: key l + 64 u; beyond nsel ~0, never counted); each
    // step counts with one ballot per slot.  Bits 31..9 are zero in every key (row index < kSeedMax), so
    // they are zero in the s-th smallest and are not searched.
    static_assert(kSeedMax <= 512, "row index of a seed key fits in 9 bits");
    unsigned long long kr[kSeedMax / 64];
#pragma unroll
    for (int u = 0; u < kSeedMax / 64; u++) kr[u] = lane + 64 * u < nsel ? keys[lane + 64 * u] : ~0ull;
    unsigned long long T = 0;
    for (int b = 63; b >= 0; b = b == 32 ? 8 : b - 1) {
        const unsigned long long t = T | (1ull << b);
        int cnt = 0;
#pragma unroll
        for (int u = 0; u < kSeedMax / 64; u++) cnt += __popcll(__ballot(kr[u] < t));
        if (cnt < s) T = t;
    }
    // candidates of a round are gathered, in row order, into dense batches of 64 (LDS list `pend`);
    // a batch re-checks each bound against the queue's current tau
    const unsigned long long lt = (1ull << lane) - 1ull;
    int np = 0;
    auto flush = [&](int cnt) __attribute__((always_inline)) {
        const bool in = lane < cnt;
        const int i = in ? pend_row[lane] : 0;
        const float lb = in ? pend_lb[lane] : INFINITY;
        seed_batch<WP, TR, SR>(c, q, er, R, U, in && lb < st.tau, base + i, st, nk, qs, qlds, lane, &n1, &next, &n2);
        const int rest = np - cnt;  // move the remaining entries to the front
        int r_row = 0;
        float r_lb = 0.f;
        if (lane < rest) { r_row = pend_row[cnt + lane]; r_lb = pend_lb[cnt + lane]; }
        __syncthreads();
        if (lane < rest) { pend_row[lane] = r_row; pend_lb[lane] = r_lb; }
        __syncthreads();
        np = rest;
    };
    auto append = [&](bool take, int i, float lb) __attribute__((always_inline)) {
        const unsigned long long m = __ballot(take);
        if (take) {
            const int at = np + __popcll(m & lt);
            pend_row[at] = i;
            pend_lb[at] = lb;
        }
        np += __popcll(m);
        __syncthreads();
        if (np >= 64) flush(64);
    };
    // round 1: the selected candidates
    for (int i0 = 0; i0 < nsel; i0 += 64) {
        const int i = i0 + lane;
        const unsigned long long key = i < nsel ? keys[i] : ~0ull;
        append(i < nsel && key <= T, i, ord_to_float((uint32_t)(key >> 32)));
    }
    if (np > 0) flush(np);
    // round 2: every other candidate in row order
    for (int i0 = 0; i0 < n; i0 += 64) {
        const int i = i0 + lane;
        bool take = false;
        float lb = INFINITY;
        if (i < n) {
            if (i < nsel) {
                const unsigned long long key = keys[i];
                lb = ord_to_float((uint32_t)(key >> 32));
                take = key > T && lb < st.tau;
            } else {
                lb = seed_lb<WP, BQT, TR>(c, base + i, R, U);
                take = lb < st.tau;
            }
        }
        append(take, i, lb);
    }
    if (np > 0) flush(np);
    unsigned long long* slots = c.slots + c.slot_off[q];
    for (int i = lane; i < st.k; i += 64) slots[i] = i < st.have ? st.now()[i] : kEmptyKey;
    if (c.counters && lane == 0) {
        atomicAdd((unsigned long long*)&c.counters[4], (unsigned long long)n);
        atomicAdd((unsigned long long*)&c.counters[5], (unsigned long long)n1);
        atomicAdd((unsigned long long*)&c.counters[6], (unsigned long long)next);
        atomicAdd((unsigned long long*)&c.counters[7], (unsigned long long)n2);
    }
}

// Threshold of a phase: the k-th best exact distance held after the previous phases, written into
// every pair record of the phase.
__global__ void k_tau_snap(const unsigned long long* __restrict__ slots, const int64_t* __restrict__ slot_off,
                           const int32_t* __restrict__ kq, const int32_t* __restrict__ boff, int nlist, int phase,
                           const int64_t* __restrict__ pair_total, PairRec* __restrict__ recs) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t pos = boff[phase * nlist] + i;
    if (i >= *pair_total || pos >= boff[(phase + 1) * nlist]) return;
    const int q = recs[pos].q;
    const unsigned long long v = slots[slot_off[q] + kq[q] - 1];
    recs[pos].tau = v == kEmptyKey ? INFINITY : __uint_as_float((uint32_t)(v >> 32));
}

__global__ void k_finalize(const unsigned long long* __restrict__ slots, const int64_t* __restrict__ slot_off,
                           const int32_t* __restrict__ kq, const int64_t* __restrict__ out_off,
                           int64_t* __restrict__ ids, float* __restrict__ dists) {
    const int64_t q = blockIdx.x;
    const int k = kq[q];
    const unsigned long long* s = slots + slot_off[q];
    for (int i = threadIdx.x; i < k; i += blockDim.x) {
        unsigned long long v = s[i];
        int64_t o = out_off[q] + i;
        if (v == kEmptyKey) {
            ids[o] = -1;
            dists[o] = INFINITY;
        } else {
            ids[o] = (int64_t)(uint32_t)(v & 0xFFFFFFFFull);
            dists[o] = __uint_as_float((uint32_t)(v >> 32));
        }
    }
}

// ------------------------------------------------------------------------------------------------
// host side: workspace layout and the launch sequence

// ------------------------------------------------------------------------------------------------
// MR-SQ search (Appendix A.2, Exp-5).  Every candidate of the probed lists gets the estimate
//   ||xhat_d - q_d||^2 + ||x_r||^2 + ||q_r||^2 = A_x + K_q - 2 <u_x, w_q>,
//   A_x = ||xhat_d||^2 + ||x_r||^2 (per row, from the build),  K_q = ||q_p||^2 - 2 <lo, q_d>,
//   w_q = delta (.) q_d  (xhat = lo + delta u, u the 8-bit codes),
// in FP32; then per query the R candidates with the smallest (estimate, id) get their exact distance.
// Queries are processed in chunks; a chunk's estimates are written to one buffer, each query's
// candidates contiguous (its probed lists in probe order, whole 64-row blocks, padding rows +inf).

// One wave per query of the chunk: offsets of its lists in its estimate range, w_q and K_q.
__global__ __launch_bounds__(64) void k_sq_query(int q0, const int32_t* __restrict__ npq,
                                                 const int64_t* __restrict__ pair_off,
                                                 const int32_t* __restrict__ pair_list,
                                                 const int32_t* __restrict__ list_nb,
                                                 const int32_t* __restrict__ list_len, const float* __restrict__ qd,
                                                 int d, int d4, int dq, const float* __restrict__ qn2,
                                                 const float* __restrict__ lo, const float* __restrict__ delta,
                                                 float* __restrict__ wq, float* __restrict__ Kq,
                                                 int32_t* __restrict__ pair_loc, int32_t* __restrict__ qcount,
                                                 int64_t* __restrict__ counters) {
    const int qi = blockIdx.x, q = q0 + qi, lane = threadIdx.x;
    if (lane == 0) {
        const int64_t pb = pair_off[q];
        int run = 0;
        long long real = 0;
        for (int r = 0; r < npq[q]; r++) {
            const int j = pair_list[pb + r];
            pair_loc[pb + r] = run;
            run += 64 * list_nb[j];
            real += list_len[j];
        }
        qcount[qi] = run;
        if (counters) atomicAdd((unsigned long long*)&counters[0], (unsigned long long)real);
    }
    float s = 0.f;
    for (int i = lane; i < dq; i += 64) {
        const float v = i < d ? qd[(int64_t)q * d4 + i] : 0.f;
        wq[(int64_t)q * dq + i] = i < d ? delta[i] * v : 0.f;
        s = fmaf(lo[i], v, s);
    }
    s = wave_sum(s);
    if (lane == 0) Kq[q] = fmaf(-2.f, s, qn2[q]);
}

// Pairs of the chunk bucketed by list (one bucket per list), then placed: sorted pair -> (query, offset of
// its list in the estimate buffer).
__global__ void k_sq_pair_count(int q0, const int32_t* __restrict__ npq, const int64_t* __restrict__ pair_off,
                                const int32_t* __restrict__ pair_list, int32_t* __restrict__ cnt) {
    const int q = q0 + blockIdx.x;
    const int64_t pb = pair_off[q];
    for (int r = threadIdx.x; r < npq[q]; r += blockDim.x) atomicAdd(&cnt[pair_list[pb + r]], 1);
}
__global__ void k_sq_pair_place(int q0, const int32_t* __restrict__ npq, const int64_t* __restrict__ pair_off,
                                const int32_t* __restrict__ pair_list, const int32_t* __restrict__ pair_loc,
                                const int32_t* __restrict__ qbase, const int32_t* __restrict__ boff,
                                int32_t* __restrict__ fill, int32_t* __restrict__ sp_q, int32_t* __restrict__ sp_off) {
    const int qi = blockIdx.x, q = q0 + qi;
    const int64_t pb = pair_off[q];
    for (int r = threadIdx.x; r < npq[q]; r += blockDim.x) {
        const int j = pair_list[pb + r];
        const int pos = boff[j] + atomicAdd(&fill[j], 1);
        sp_q[pos] = q;
        sp_off[pos] = qbase[qi] + pair_loc[pb + r];
    }
}

// The estimates of one work item (64-row block of a list x up to GT of the list's pairs) on the matrix
// cores: for each 16 x 16 sub-tile a v_mfma_f32_16x16x4_f32 chain over the dq coordinates, A operand the
// queries' w_q (lane group g feeding coordinates 16 t + 4 g .. + 3 of slice t), B operand the rows' codes
// converted to FP32 (the bytes of lane group g of a row are contiguous in the scan-order layout).
// Persistent grid, items dealt round-robin.  TS: 16-coordinate slices per row (0 = any).
template <int GT, int TS>
__global__ __launch_bounds__(256) void k_sq_scan(const int32_t* __restrict__ ioff, int nlist, const int4* __restrict__ desc,
                                                 const int32_t* __restrict__ sp_q, const int32_t* __restrict__ sp_off,
                                                 const uint8_t* __restrict__ code, const float* __restrict__ A,
                                                 const int64_t* __restrict__ list_off, const float* __restrict__ wq,
                                                 const float* __restrict__ Kq, int dq, float* __restrict__ est) {
    constexpr int NCT = GT / 16;
    __shared__ int32_t sh_q[4][GT];
    __shared__ int32_t sh_o[4][GT];
    __shared__ float sh_k[4][GT];
    const int lane = lane_id();
    const int wv = threadIdx.x >> 6;
    const int li = lane & 15, kg = lane >> 4;
    const int ts = TS > 0 ? TS : dq >> 4;
    const int total = (int)const_load((const uint32_t*)(ioff + nlist));
    const int nwaves = gridDim.x * 4;
    for (int it = uniform(blockIdx.x * 4 + wv); it < total; it += nwaves) {
        const int4 dsc = const_load4(desc + it);
        const int64_t row0 = dsc.x;
        const int pbeg = dsc.y, ng = dsc.z, j = dsc.w;
        const int rbase = (int)(row0 - list_off[j]);  // the block's first row within its list
        if (lane < ng) {
            const int q = sp_q[pbeg + lane];
            sh_q[wv][lane] = q;
            sh_o[wv][lane] = sp_off[pbeg + lane] + rbase;
            sh_k[wv][lane] = Kq[q];
        }
        wave_lds_fence();
#pragma unroll
        for (int ct = 0; ct < NCT; ct++) {
            if (16 * ct >= ng) break;
            // w_q of this lane's query column (slots beyond ng read slot 0; their outputs are not written)
            const int qs = ct * 16 + li;
            const float4* wp = reinterpret_cast<const float4*>(wq + (int64_t)sh_q[wv][qs < ng ? qs : 0] * dq + 4 * kg);
            for (int rt = 0; rt < 4; rt++) {
                const int64_t row = row0 + 16 * rt + li;
                const float a = A[row];
                f32x4 acc = {0.f, 0.f, 0.f, 0.f};
                if constexpr (TS > 0 && TS % 4 == 0) {
                    const uint4* cp = reinterpret_cast<const uint4*>(code + row * dq + kg * (dq >> 2));
#pragma unroll
                    for (int t4 = 0; t4 < TS / 4; t4++) {
                        const uint4 cw = cp[t4];
                        const uint32_t w4[4] = {cw.x, cw.y, cw.z, cw.w};
#pragma unroll
                        for (int u = 0; u < 4; u++) {
                            const uint32_t c = w4[u];
                            const float4 x = make_float4((float)(c & 0xFFu), (float)((c >> 8) & 0xFFu),
                                                         (float)((c >> 16) & 0xFFu), (float)(c >> 24));
                            mfma4(acc, wp[4 * (4 * t4 + u)], x);
                        }
                    }
                } else {
                    const uint32_t* cp = reinterpret_cast<const uint32_t*>(code + row * dq + kg * (dq >> 2));
                    for (int t = 0; t < ts; t++) {
                        const uint32_t c = cp[t];
                        const float4 x = make_float4((float)(c & 0xFFu), (float)((c >> 8) & 0xFFu),
                                                     (float)((c >> 16) & 0xFFu), (float)(c >> 24));
                        mfma4(acc, wp[4 * t], x);
                    }
                }
#pragma unroll
                for (int v = 0; v < 4; v++) {
                    const int slot = ct * 16 + 4 * kg + v;
                    if (slot < ng) est[sh_o[wv][slot] + 16 * rt + li] = fmaf(-2.f, acc[v], a + sh_k[wv][slot]);
                }
            }
        }
        wave_lds_fence();
    }
}

// Row of position i of a query's estimate range (its lists' offsets loc[0..np) ascending).
__device__ __forceinline__ int64_t sq_row_of(int i, const int32_t* loc, const int32_t* lst, int np,
                                             const int64_t* __restrict__ list_off) {
    int lo = 0, hi = np - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (loc[mid] <= i) lo = mid; else hi = mid - 1;
    }
    return list_off[lst[lo]] + (i - loc[lo]);
}

// One block per query of the chunk: the R candidates with the smallest (estimate, id) among the finite
// estimates, found by a radix selection over the order-preserving key bits (8 bits per pass) and, when
// the boundary estimate is shared, over the ids of those equal to it; their rows are written in any order.
// Every pass reads the query's estimates from global memory (L2), eight loads in flight per thread.

// Radix-selection step (run by the first wave of the block): the bin of hist[256] holding rank `want`
// (1-based) of the counted keys, by a prefix sum over the lanes (four bins each); the one lane whose
// range holds the rank writes the rank left within that bin, the extended prefix and the bin's count.
__device__ __forceinline__ void sq_pick_bin(const int32_t* hist, int want, uint32_t pre, int shift, int lane,
                                            int32_t* s_want, uint32_t* s_pre, int32_t* s_eq) {
    const int h0 = hist[4 * lane], h1 = hist[4 * lane + 1], h2 = hist[4 * lane + 2], h3 = hist[4 * lane + 3];
    const int loc = h0 + h1 + h2 + h3;
    int inc = loc;
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(inc, o);
        if (lane >= o) inc += y;
    }
    const int exc = inc - loc;
    if (exc < want && want <= inc) {
        int c = exc, b = 4 * lane;
        if (c + h0 < want) {
            c += h0;
            b++;
            if (c + h1 < want) {
                c += h1;
                b++;
                if (c + h2 < want) {
                    c += h2;
                    b++;
                }
            }
        }
        *s_want = want - c;
        *s_pre = pre | ((uint32_t)b << shift);
        *s_eq = hist[b];
    }
}

__global__ __launch_bounds__(256) void k_sq_select(int q0, const float* __restrict__ est, const int32_t* __restrict__ qbase,
                                                   const int32_t* __restrict__ npq, const int64_t* __restrict__ pair_off,
                                                   const int32_t* __restrict__ pair_list,
                                                   const int32_t* __restrict__ pair_loc,
                                                   const int64_t* __restrict__ list_off, const int32_t* __restrict__ ids,
                                                   int R, int32_t* __restrict__ sel, int32_t* __restrict__ selcnt) {
    __shared__ int32_t hist[256];
    __shared__ int32_t s_loc[kMaxProbe], s_lst[kMaxProbe];
    __shared__ uint32_t s_pre;
    __shared__ int32_t s_want, s_num, s_eq;
    const int qi = blockIdx.x, q = q0 + qi, t = threadIdx.x;
    const int base = qbase[qi], n = qbase[qi + 1] - base;
    const float* e = est + base;
    const uint32_t kinf = ord_bits(INFINITY);  // keys below it are finite estimates
    const int np = npq[q];
    const int64_t pb = pair_off[q];
    for (int r = t; r < np; r += 256) {
        s_loc[r] = pair_loc[pb + r];
        s_lst[r] = pair_list[pb + r];
    }
    if (t == 0) s_num = 0;
    __syncthreads();
    // visit every key, eight loads in flight per thread
    auto each_key = [&](auto&& f) {
        for (int i0 = t; i0 < n; i0 += 256 * 8) {
            float v[8];
#pragma unroll
            for (int u = 0; u < 8; u++) v[u] = i0 + 256 * u < n ? e[i0 + 256 * u] : INFINITY;
#pragma unroll
            for (int u = 0; u < 8; u++)
                if (i0 + 256 * u < n) f(i0 + 256 * u, ord_bits(v[u]));
        }
    };
    int fin = 0;
    each_key([&](int, uint32_t k) { fin += k < kinf ? 1 : 0; });
    atomicAdd(&s_num, fin);
    __syncthreads();
    const int take = min(R, s_num);
    __syncthreads();
    if (take == 0) {
        if (t == 0) selcnt[qi] = 0;
        return;
    }
    // the take-th smallest key T, and how many of the keys equal to T are taken
    uint32_t pre = 0, msk = 0;
    int want = take;
    for (int shift = 24; shift >= 0; shift -= 8) {
        hist[t] = 0;
        __syncthreads();
        each_key([&](int, uint32_t k) {
            if (k < kinf && (k & msk) == pre) atomicAdd(&hist[(k >> shift) & 255u], 1);
        });
        __syncthreads();
        if (t < 64) sq_pick_bin(hist, want, pre, shift, t, &s_want, &s_pre, &s_eq);
        __syncthreads();
        want = s_want;
        pre = s_pre;
        msk |= 255u << shift;
        __syncthreads();
    }
    const uint32_t T = pre;
    const bool tie = want < s_eq;  // only some of the keys equal to T are taken: the smallest ids
    uint32_t idT = 0xFFFFFFFFu;
    if (tie) {
        uint32_t ip = 0, im = 0;
        for (int shift = 24; shift >= 0; shift -= 8) {
            hist[t] = 0;
            __syncthreads();
            each_key([&](int i, uint32_t k) {
                if (k != T) return;
                const uint32_t id = (uint32_t)ids[sq_row_of(i, s_loc, s_lst, np, list_off)];
                if ((id & im) == ip) atomicAdd(&hist[(id >> shift) & 255u], 1);
            });
            __syncthreads();
            if (t < 64) sq_pick_bin(hist, want, ip, shift, t, &s_want, &s_pre, &s_eq);
            __syncthreads();
            want = s_want;
            ip = s_pre;
            im |= 255u << shift;
            __syncthreads();
        }
        idT = ip;
    }
    if (t == 0) s_num = 0;
    __syncthreads();
    int32_t* out = sel + (int64_t)qi * R;
    each_key([&](int i, uint32_t k) {
        if (k > T) return;  // T < kinf, so the infinite keys are skipped here
        const int64_t row = sq_row_of(i, s_loc, s_lst, np, list_off);
        if (k == T && tie && (uint32_t)ids[row] > idT) return;
        const int p = atomicAdd(&s_num, 1);  // exactly `take` positions are taken
        if (p < R) out[p] = (int32_t)row;
    });
    __syncthreads();
    if (t == 0) selcnt[qi] = min(s_num, R);
}

// One block per query of the chunk: exact distances ||x - q||^2 of its re-rank candidates (16 lanes
// per candidate, as in the exact stage of the MRQ path) into its result slots.
__global__ __launch_bounds__(256) void k_sq_exact(int q0, const int32_t* __restrict__ sel, const int32_t* __restrict__ selcnt,
                                                  int R, const float* __restrict__ X, const float* __restrict__ qpad,
                                                  int D4, const int32_t* __restrict__ ids,
                                                  const int64_t* __restrict__ slot_off, const int32_t* __restrict__ kq,
                                                  unsigned long long* __restrict__ slots, int64_t* __restrict__ counters) {
    const int qi = blockIdx.x, q = q0 + qi, lane = lane_id();
    const int n = selcnt[qi];
    const int32_t* rows = sel + (int64_t)qi * R;
    for (int i = threadIdx.x >> 4; i - (lane >> 4) < n; i += 16) {
        const bool valid = i < n;
        const int64_t row = rows[valid ? i : 0];
        const float dist = exact_dist_group(X + row * D4, qpad + (int64_t)q * D4, D4, lane & 15);
        if (valid && (lane & 15) == 0) {
            const unsigned long long key = ((unsigned long long)__float_as_uint(dist) << 32) | (uint32_t)ids[row];
            topk_insert(slots + slot_off[q], kq[q], key);
        }
    }
    if (counters && threadIdx.x == 0) atomicAdd((unsigned long long*)&counters[3], (unsigned long long)n);
}

// Query-level bytes stored per pair: the K slices the scan multiplies, 64 dimensions each (zero beyond d).
// d in (128, 192] takes the 4-slice scan, so its rows are padded to 256 bytes and the fourth slice's
// loads stay inside the pair's own row.
static int level_bytes(int d) {
    const int ki = (d + 63) / 64;
    return 64 * (ki == 3 ? 4 : ki);
}

namespace {
struct Carve {
    char* p;
    size_t used = 0;
    template <class T>
    T* take(int64_t n) {
        size_t b = ((size_t)(n > 0 ? n : 1) * sizeof(T) + 255) & ~(size_t)255;
        T* r = reinterpret_cast<T*>(p ? p + used : nullptr);
        used += b;
        return r;
    }
};

struct WsPtrs {
    float *qd, *qtail, *qpad, *rq, *qn2, *qd2, *Tq, *er, *G;
    float* TM;      // tile minima of the probe distances (tile selection)
    int32_t* redo;  // queries the tile selection hands back: count, then the list
    int32_t* segsum;  // segment sums of the (phase, list) prefix sums
    int32_t *pair_list, *pair_q, *pair_pos, *cnt, *boff, *fill, *items, *ioff, *qcnt;
    __bf16* qbf;  // BF16 staging of the tail product
    int4* desc;
    PairRec* recs;
    int8_t* qu8;
    unsigned long long* slots;
    int32_t* surv;
    float* survd;  // split exact stage: dis_o' of each bin entry
};

// Exact-stage buffer capacity of a phase (entries): 1/16 of the candidates the search can scan, within
// [2^16, 2^27]; candidates beyond it get their exact distance inside the scan kernel (same arithmetic).
int64_t surv_capacity(const Index& ix, int64_t total_pairs) {
    const int64_t avg = (ix.N + ix.nlist - 1) / ix.nlist;
    int64_t want = total_pairs * avg / 16;
    if (want < ((int64_t)1 << 16)) want = (int64_t)1 << 16;
    if (want > ((int64_t)1 << 27)) want = (int64_t)1 << 27;
    return want;
}

// Upper bound of the work items of all phases: sum over (phase, list) of blocks(list) * ceil(pairs / G)
// <= max_blocks * pairs / 16 + phases * (sum of blocks), for any G >= 16.
constexpr int kMaxScanBlocks = 2048;

int64_t max_items(const Index& ix, int64_t total_pairs) {
    const int64_t max_nb = (ix.max_list_len + 63) / 64;
    const int64_t sum_nb = ix.Npad / 64;
    return max_nb * ((total_pairs + 15) / 16) + std::min<int64_t>((int64_t)kPhases * sum_nb, total_pairs * max_nb) + 1;
}

WsPtrs carve(void* base, const Index& ix, int64_t nq, int64_t total_slots, int64_t total_pairs, int bq,
             int np_max, size_t* used) {
    Carve c{reinterpret_cast<char*>(base)};
    WsPtrs w;
    const int64_t P = (int64_t)kPhases * ix.nlist;
    w.qd = c.take<float>(nq * ix.d4);
    w.qtail = c.take<float>(nq * (int64_t)std::max(ix.D - ix.d, ix.Dr4));
    w.qpad = c.take<float>(nq * ix.D4);
    w.rq = c.take<float>(nq * ix.d4);
    w.qn2 = c.take<float>(nq);
    w.qd2 = c.take<float>(nq);
    w.Tq = c.take<float>(nq);
    w.er = c.take<float>(nq);
    w.G = c.take<float>(nq * (int64_t)ix.nlist);
    const bool ts = tile_select(ix.nlist, np_max);
    w.TM = ts ? c.take<float>(nq * (int64_t)((ix.nlist + 63) / 64)) : nullptr;
    w.redo = ts ? c.take<int32_t>(nq + 1) : nullptr;
    w.pair_list = c.take<int32_t>(total_pairs);
    w.pair_q = c.take<int32_t>(total_pairs);
    w.pair_pos = c.take<int32_t>(total_pairs);
    w.segsum = c.take<int32_t>(P / kSeg + 1);
    w.cnt = c.take<int32_t>(P);
    w.boff = c.take<int32_t>(P + 1);
    w.fill = c.take<int32_t>(P);
    w.items = c.take<int32_t>(P);
    w.ioff = c.take<int32_t>(P + 1);
    w.desc = c.take<int4>(max_items(ix, total_pairs));
    w.recs = c.take<PairRec>(total_pairs);
    w.qu8 = c.take<int8_t>(total_pairs * (int64_t)level_bytes(ix.d));
    w.slots = c.take<unsigned long long>(total_slots);
    w.qcnt = c.take<int32_t>(nq);
    w.qbf = c.take<__bf16>(bf16_stage_elems(ix, nq));
    const int64_t cap = surv_capacity(ix, total_pairs);
    w.surv = c.take<int32_t>(cap);
    w.survd = ix.split ? c.take<float>(cap) : nullptr;
    *used = c.used;
    return w;
}

struct Timed {
    KernelTimer* t;
    hipStream_t s;
    KernelTimer::Pending p;
    Timed(KernelTimer* tm, hipStream_t st, const char* name) : t(tm), s(st) {
        p.slot = -1;
        if (t && t->on) t->begin(s, name, &p);
    }
    ~Timed() {
        if (t && t->on && p.slot >= 0) t->end(s, &p);
    }
};
}  // namespace

size_t search_workspace_bytes(const Index& ix, int64_t nq, int64_t total_slots, int64_t total_pairs, int bq,
                              int np_max, int method, int rerank);

template <int WP, int BQT, bool TR>
static void launch_seed_t(const ScanCtx& c, int64_t nq, hipStream_t s) {
    const size_t lds = sizeof(unsigned long long) * (2 * c.k_max + kSeedMax) +
                       (c.RX4 <= kSeedLdsFloats ? sizeof(float) * (c.RX4 + c.d4) : 0);
    if (c.RX4 <= 64) hipLaunchKernelGGL((k_seed<WP, BQT, TR, true>), dim3((unsigned)nq), dim3(64), lds, s, c);
    else hipLaunchKernelGGL((k_seed<WP, BQT, TR, false>), dim3((unsigned)nq), dim3(64), lds, s, c);
}

// Blocks of a persistent kernel that are resident at once on the current device (cached per device).
template <class K>
static int resident_blocks(K kernel, int threads, int slot, size_t lds) {
    static int cache[16][64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 16) dev = 0;
    int& v = cache[dev][slot];
    if (v == 0) {
        int per_cu = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, lds) != hipSuccess || per_cu < 1)
            per_cu = 1;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
            cus = 256;
        v = per_cu * cus;
    }
    return v;
}

template <int GT, int KIT>
static bool scan_ql(const ScanCtx& c) {
    return (KIT == 1 || KIT == 2) && c.d4 == 64 * KIT && c.stage2;
}
static size_t scan_lds(const ScanCtx& c, int GT) { return (size_t)4 * GT * c.d4 * sizeof(float); }
// split: the stage-2 stash of the four waves (GT / 16 column tiles x 16 slots x 64 lanes each)
static size_t scan_stash(const ScanCtx& c, int GT) { return c.split ? (size_t)4 * (GT / 16) * 16 * 64 * sizeof(float) : 0; }

// TR: the tracing instantiations (c.tr set; query group 16 only).
static bool scan_ext(const ScanCtx& c) { return c.B > 1 && c.use_ext; }

template <int GT, int KIT, bool TR, bool SPL>
static void launch_scan_k(const ScanCtx& c, hipStream_t s, int blocks) {
    if constexpr (KIT == 1 || KIT == 2) {
        if (scan_ql<GT, KIT>(c) && scan_lds(c, GT) <= 65536) {
            if (scan_ext(c))
                hipLaunchKernelGGL((k_scan<GT, KIT, true, TR, SPL, true>), dim3(blocks), dim3(256),
                                   scan_lds(c, GT) + scan_stash(c, GT), s, c);
            else
                hipLaunchKernelGGL((k_scan<GT, KIT, true, TR, SPL, false>), dim3(blocks), dim3(256),
                                   scan_lds(c, GT) + scan_stash(c, GT), s, c);
            return;
        }
    }
    hipLaunchKernelGGL((k_scan<GT, KIT, false, TR, SPL>), dim3(blocks), dim3(256), scan_stash(c, GT), s, c);
}

template <int GT, bool TR, bool SPL>
static void launch_scan_g(const ScanCtx& c, hipStream_t s, int blocks) {
    switch (c.KI) {
        case 1: launch_scan_k<GT, 1, TR, SPL>(c, s, blocks); break;
        case 2: launch_scan_k<GT, 2, TR, SPL>(c, s, blocks); break;
        case 3: case 4: launch_scan_k<GT, 4, TR, SPL>(c, s, blocks); break;
        default: launch_scan_k<GT, 0, TR, SPL>(c, s, blocks); break;
    }
}

// Query groups: 16 (the tracing instantiations), 16 / 32 with the split exact stage, 16 / 32 / 64 otherwise.
static void launch_scan(const ScanCtx& c, hipStream_t s, int blocks) {
    if (c.tr && c.split) launch_scan_g<16, true, true>(c, s, blocks);
    else if (c.tr) launch_scan_g<16, true, false>(c, s, blocks);
    else if (c.split && c.G <= 16) launch_scan_g<16, false, true>(c, s, blocks);
    else if (c.split) launch_scan_g<32, false, true>(c, s, blocks);
    else if (c.G <= 16) launch_scan_g<16, false, false>(c, s, blocks);
    else if (c.G <= 32) launch_scan_g<32, false, false>(c, s, blocks);
    else launch_scan_g<64, false, false>(c, s, blocks);
}

// Blocks of the persistent scan grid: what is resident at once on the device, at most kMaxScanBlocks.
// slot: the resident-block cache entry of the staged form with the B-bit refinement; xslot: without it
template <int GT, int KIT, bool TR, bool SPL>
static int scan_grid_k(const ScanCtx& c, int slot, int xslot = -1) {
    if constexpr (KIT == 1 || KIT == 2) {
        if (scan_ql<GT, KIT>(c) && scan_lds(c, GT) <= 65536) {
            const size_t lds = scan_lds(c, GT) + scan_stash(c, GT);
            return std::min(scan_ext(c) ? resident_blocks(k_scan<GT, KIT, true, TR, SPL, true>, 256, slot, lds)
                                        : resident_blocks(k_scan<GT, KIT, true, TR, SPL, false>, 256, xslot, lds),
                            kMaxScanBlocks);
        }
    }
    return std::min(resident_blocks(k_scan<GT, KIT, false, TR, SPL>, 256, slot + 1, scan_stash(c, GT)), kMaxScanBlocks);
}
template <int GT, bool TR, bool SPL>
static int scan_grid_g(const ScanCtx& c, int slot) {
    switch (c.KI) {
        // (slots 4 and 6, which the forms below leave free, hold the staged forms without the refinement)
        case 1: return scan_grid_k<GT, 1, TR, SPL>(c, slot + 0, slot + 4);
        case 2: return scan_grid_k<GT, 2, TR, SPL>(c, slot + 2, slot + 6);
        case 3: case 4: return scan_grid_k<GT, 4, TR, SPL>(c, slot + 4);
        default: return scan_grid_k<GT, 0, TR, SPL>(c, slot + 6);
    }
}
static int scan_grid(const ScanCtx& c) {
    if (c.tr && c.split) return scan_grid_g<16, true, true>(c, 40);
    if (c.tr) return scan_grid_g<16, true, false>(c, 32);
    if (c.split && c.G <= 16) return scan_grid_g<16, false, true>(c, 48);
    if (c.split) return scan_grid_g<32, false, true>(c, 56);
    if (c.G <= 16) return scan_grid_g<16, false, false>(c, 0);
    if (c.G <= 32) return scan_grid_g<32, false, false>(c, 8);
    return scan_grid_g<64, false, false>(c, 16);
}

template <int WP, bool TR>
static void launch_seed_w(const ScanCtx& c, int64_t nq, hipStream_t s) {
    if (c.bq == 4) launch_seed_t<WP, 4, TR>(c, nq, s);
    else launch_seed_t<WP, 0, TR>(c, nq, s);
}

template <bool TR>
static void launch_seed_tr(const ScanCtx& c, int64_t nq, hipStream_t s) {
    switch (c.WP) {
        case 1: launch_seed_w<1, TR>(c, nq, s); break;
        case 2: launch_seed_w<2, TR>(c, nq, s); break;
        case 4: launch_seed_w<4, TR>(c, nq, s); break;
        case 8: launch_seed_w<8, TR>(c, nq, s); break;
        case 16: launch_seed_w<16, TR>(c, nq, s); break;
        case 32: launch_seed_w<32, TR>(c, nq, s); break;
        default: launch_seed_w<48, TR>(c, nq, s); break;
    }
}
static void launch_seed(const ScanCtx& c, int64_t nq, hipStream_t s) {
    if (c.tr) launch_seed_tr<true>(c, nq, s);
    else launch_seed_tr<false>(c, nq, s);
}

int padded_words(int d) {
    const int W = (d + 31) / 32;
    const int opts[] = {1, 2, 4, 8, 16, 32, 48};
    for (int o : opts)
        if (o >= W) return o;
    return -1;
}

#define HIP_TRY(x)                              \
    do {                                        \
        hipError_t e_ = (x);                    \
        if (e_ != hipSuccess) return e_;        \
    } while (0)

// ---- MR-SQ search (host side) -------------------------------------------------------------------

namespace {
// A chunk's estimate buffer holds at most this many entries (1 GiB), or one query's worth.
constexpr int64_t kSqEstCap = (int64_t)1 << 28;

// Estimate entries of one query at most: its probed lists are distinct, each whole 64-row blocks.
int64_t sq_query_bound(const Index& ix, int np_max) {
    const int64_t max_nb = (ix.max_list_len + 63) / 64;
    return std::max<int64_t>(1, std::min<int64_t>(ix.Npad, (int64_t)np_max * 64 * max_nb));
}
int64_t sq_chunk(const Index& ix, int64_t nq, int np_max) {
    return std::max<int64_t>(1, std::min<int64_t>(nq, kSqEstCap / sq_query_bound(ix, np_max)));
}

struct WsSq {
    float *qd, *qtail, *qpad, *qn2, *qd2, *Tq, *er, *G, *wq, *Kq, *est;
    int32_t *pair_list, *pair_q, *pair_loc, *qcount, *qbase, *cnt, *boff, *fill, *items, *ioff, *sp_q, *sp_off;
    int32_t *sel, *selcnt;
    int4* desc;
    unsigned long long* slots;
};

WsSq carve_sq(void* base, const Index& ix, int64_t nq, int64_t total_slots, int64_t total_pairs, int np_max, int R,
              size_t* used) {
    Carve c{reinterpret_cast<char*>(base)};
    WsSq w;
    const int64_t ch = sq_chunk(ix, nq, np_max);
    const int64_t chp = std::min<int64_t>(total_pairs, ch * np_max);  // pairs of one chunk at most
    const int64_t max_nb = (ix.max_list_len + 63) / 64;
    const int64_t L = ix.nlist;
    w.qd = c.take<float>(nq * ix.d4);
    w.qtail = c.take<float>(nq * (int64_t)(ix.D - ix.d));
    w.qpad = c.take<float>(nq * ix.D4);
    w.qn2 = c.take<float>(nq);
    w.qd2 = c.take<float>(nq);
    w.Tq = c.take<float>(nq);
    w.er = c.take<float>(nq);
    w.G = c.take<float>(nq * L);
    w.pair_list = c.take<int32_t>(total_pairs);
    w.pair_q = c.take<int32_t>(total_pairs);
    w.pair_loc = c.take<int32_t>(total_pairs);
    w.wq = c.take<float>(nq * ix.dq);
    w.Kq = c.take<float>(nq);
    w.qcount = c.take<int32_t>(ch);
    w.qbase = c.take<int32_t>(ch + 1);
    w.cnt = c.take<int32_t>(L);
    w.boff = c.take<int32_t>(L + 1);
    w.fill = c.take<int32_t>(L);
    w.items = c.take<int32_t>(L);
    w.ioff = c.take<int32_t>(L + 1);
    // work items: sum over lists of blocks * ceil(pairs / G) <= max_nb * pairs / 16 + all blocks (G >= 16)
    w.desc = c.take<int4>(max_nb * ((chp + 15) / 16) + ix.Npad / 64 + 1);
    w.sp_q = c.take<int32_t>(chp);
    w.sp_off = c.take<int32_t>(chp);
    w.est = c.take<float>(ch * sq_query_bound(ix, np_max));
    w.sel = c.take<int32_t>(ch * R);
    w.selcnt = c.take<int32_t>(ch);
    w.slots = c.take<unsigned long long>(total_slots);
    *used = c.used;
    return w;
}
}  // namespace

template <int GT, int TS>
static void launch_sq_scan_t(const WsSq& w, const Index& ix, hipStream_t s, int slot) {
    const int blocks = std::min(resident_blocks(k_sq_scan<GT, TS>, 256, slot, 0), kMaxScanBlocks);
    hipLaunchKernelGGL((k_sq_scan<GT, TS>), dim3((unsigned)blocks), dim3(256), 0, s, w.ioff, ix.nlist, w.desc, w.sp_q,
                       w.sp_off, ix.sq_code, ix.sq_A, ix.list_off, w.wq, w.Kq, ix.dq, w.est);
}
template <int GT>
static void launch_sq_scan_g(const WsSq& w, const Index& ix, hipStream_t s, int slot) {
    switch (ix.dq) {
        case 64: launch_sq_scan_t<GT, 4>(w, ix, s, slot); break;
        case 128: launch_sq_scan_t<GT, 8>(w, ix, s, slot + 1); break;
        case 256: launch_sq_scan_t<GT, 16>(w, ix, s, slot + 2); break;
        default: launch_sq_scan_t<GT, 0>(w, ix, s, slot + 3); break;
    }
}

size_t search_workspace_bytes(const Index& ix, int64_t nq, int64_t total_slots, int64_t total_pairs, int bq,
                              int np_max, int method, int rerank) {
    size_t used = 0;
    if (method == MRQ_METHOD_MRSQ) carve_sq(nullptr, ix, nq, total_slots, total_pairs, np_max, rerank, &used);
    else carve(nullptr, ix, nq, total_slots, total_pairs, bq, np_max, &used);
    return used;
}

static hipError_t launch_search_mrsq(const SearchArgs& a, void* ws, size_t ws_bytes, hipStream_t s) {
    const Index& ix = *a.ix;
    size_t used = 0;
    WsSq w = carve_sq(ws, ix, a.nq, a.total_slots, a.total_pairs, a.np_max, a.rerank, &used);
    if (used > ws_bytes) return hipErrorOutOfMemory;
    KernelTimer* tm = a.timed ? &ix.timer : nullptr;
    const int64_t nq = a.nq;
    const int d = ix.d, d4 = ix.d4, D = ix.D, D4 = ix.D4, nlist = ix.nlist, dq = ix.dq;
    const int G = a.group > 16 ? 32 : 16;
    {   // the projection and the centroid ranking of the MRQ path
        Timed t(tm, s, "project");
        HIP_TRY(launch_query_projection(ix, a.Q, nq, w.qd, w.qtail, (int64_t)(D - d), nullptr, s));
        hipLaunchKernelGGL(k_query_stats, dim3((unsigned)nq), dim3(64), 0, s, a.Q, D, D4, ix.mu, w.qd, d, d4, w.qtail,
                           (int64_t)(D - d), ix.lamTail, a.m, w.qpad, w.qn2, w.qd2, w.Tq, w.er);
        HIP_TRY(hipGetLastError());
    }
    {
        Timed t(tm, s, "probe");
        HIP_TRY(launch_gemm_mfma<1>(w.qd, d4, nullptr, ix.C, d4, w.G, nlist, nq, nlist, d, w.qd2, ix.Cn2, nullptr, 0, 0, s));
        launch_select(w.G, nlist, a.npq, a.pair_off, w.pair_list, w.pair_q, nq, a.np_max, s);
        HIP_TRY(fill_u64(w.slots, kEmptyKey, a.total_slots, s));
        HIP_TRY(hipGetLastError());
    }
    const int64_t ch = sq_chunk(ix, nq, a.np_max);
    for (int64_t q0 = 0; q0 < nq; q0 += ch) {
        const int cn = (int)std::min<int64_t>(ch, nq - q0);
        {   // estimate ranges, w_q, K_q; pairs bucketed by list into work items
            Timed t(tm, s, "sq_prep");
            hipLaunchKernelGGL(k_sq_query, dim3((unsigned)cn), dim3(64), 0, s, (int)q0, a.npq, a.pair_off, w.pair_list,
                               ix.list_nb, ix.list_len, w.qd, d, d4, dq, w.qn2, ix.sq_lo, ix.sq_delta, w.wq, w.Kq,
                               w.pair_loc, w.qcount, a.counters);
            hipLaunchKernelGGL(k_scan_excl, dim3(1), dim3(kScanThreads), 0, s, w.qcount, w.qbase, (int64_t)cn);
            HIP_TRY(launch_fill_i32(w.cnt, 0, nlist, s));
            HIP_TRY(launch_fill_i32(w.fill, 0, nlist, s));
            hipLaunchKernelGGL(k_sq_pair_count, dim3((unsigned)cn), dim3(64), 0, s, (int)q0, a.npq, a.pair_off,
                               w.pair_list, w.cnt);
            hipLaunchKernelGGL(k_scan_excl, dim3(1), dim3(kScanThreads), 0, s, w.cnt, w.boff, (int64_t)nlist);
            hipLaunchKernelGGL(k_sq_pair_place, dim3((unsigned)cn), dim3(64), 0, s, (int)q0, a.npq, a.pair_off,
                               w.pair_list, w.pair_loc, w.qbase, w.boff, w.fill, w.sp_q, w.sp_off);
            hipLaunchKernelGGL(k_items, dim3((unsigned)((nlist + 255) / 256)), dim3(256), 0, s, w.cnt, ix.list_nb, nlist,
                               G, nlist, w.items);
            hipLaunchKernelGGL(k_scan_excl, dim3(1), dim3(kScanThreads), 0, s, w.items, w.ioff, (int64_t)nlist);
            hipLaunchKernelGGL(k_item_desc, dim3((unsigned)((nlist + 3) / 4)), dim3(256), 0, s, w.ioff, w.boff,
                               ix.list_nb, ix.list_off, nlist, G, (int64_t)nlist, w.desc);
            HIP_TRY(hipGetLastError());
        }
        {
            Timed t(tm, s, "sq_scan");
            if (G == 16) launch_sq_scan_g<16>(w, ix, s, 24);
            else launch_sq_scan_g<32>(w, ix, s, 28);
            HIP_TRY(hipGetLastError());
        }
        {
            Timed t(tm, s, "sq_select");
            hipLaunchKernelGGL(k_sq_select, dim3((unsigned)cn), dim3(256), 0, s, (int)q0, w.est, w.qbase, a.npq,
                               a.pair_off, w.pair_list, w.pair_loc, ix.list_off, ix.ids, a.rerank, w.sel, w.selcnt);
            HIP_TRY(hipGetLastError());
        }
        {
            Timed t(tm, s, "sq_exact");
            hipLaunchKernelGGL(k_sq_exact, dim3((unsigned)cn), dim3(256), 0, s, (int)q0, w.sel, w.selcnt, a.rerank,
                               ix.X, w.qpad, D4, ix.ids, a.slot_off, a.kq, w.slots, a.counters);
            HIP_TRY(hipGetLastError());
        }
    }
    {
        Timed t(tm, s, "finalize");
        hipLaunchKernelGGL(k_finalize, dim3((unsigned)nq), dim3(64), 0, s, w.slots, a.slot_off, a.kq, a.out_off, a.ids,
                           a.dists);
        HIP_TRY(hipGetLastError());
    }
    return hipSuccess;
}

// ---- streaming copy: the achievable HBM bandwidth the scan is measured against -----------------------
// Each thread moves four 16-byte words per step (all four loads issued before the stores), grid-stride,
// with non-temporal hints: every byte is read once and written once.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_stream_copy(const u32x4* __restrict__ src, u32x4* __restrict__ dst,
                                                     int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * 1024;
    for (int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x; i < n; i += stride) {
        u32x4 v[4];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int64_t j = i + 256 * u;
            if (j < n) v[u] = __builtin_nontemporal_load(src + j);
        }
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int64_t j = i + 256 * u;
            if (j < n) __builtin_nontemporal_store(v[u], dst + j);
        }
    }
}

hipError_t launch_stream_copy(void* dst, const void* src, size_t bytes, hipStream_t s) {
    const int64_t n = (int64_t)(bytes / 16);
    if (n == 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((n + 1023) / 1024, 8192);
    hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)blocks), dim3(256), 0, s, reinterpret_cast<const u32x4*>(src),
                       reinterpret_cast<u32x4*>(dst), n);
    return hipGetLastError();
}

// ---- fixed device buffer of the allocation-free search ---------------------------------------------
// One array per device, held for the life of the process.  Host code must not pass `scratch` itself to a
// kernel (in host code the name stands for a host-side shadow, not a device address): its device address
// is looked up once per device with hipGetSymbolAddress and only that address is used.

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

hipError_t noalloc_scratch(void** p, size_t* bytes) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void* addr[kMaxDevices] = {};
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void* a = nullptr;
        HIP_TRY(hipGetSymbolAddress(&a, HIP_SYMBOL(scratch)));  // with `dev` current
        if (!a) return hipErrorInvalidSymbol;
        addr[dev] = a;
    }
    *p = addr[dev];
    *bytes = kNoAllocBytes;
    return hipSuccess;
}

hipError_t launch_search(const SearchArgs& a, void* ws, size_t ws_bytes, hipStream_t s) {
    if (a.method == MRQ_METHOD_MRSQ) return launch_search_mrsq(a, ws, ws_bytes, s);
    const Index& ix = *a.ix;
    size_t used = 0;
    WsPtrs w = carve(ws, ix, a.nq, a.total_slots, a.total_pairs, a.bq, a.np_max, &used);
    if (used > ws_bytes) return hipErrorOutOfMemory;
    KernelTimer* tm = a.timed ? &ix.timer : nullptr;
    const int64_t nq = a.nq;
    const int d = ix.d, d4 = ix.d4, D = ix.D, D4 = ix.D4, nlist = ix.nlist;
    // the (phase, list) buckets of the phases this search reaches (phase p starts at probe rank phase_lo(p))
    int nph = 1;
    while (nph < kPhases && phase_lo(nph, a.phase_shift) < a.np_max) nph++;
    const int64_t P = (int64_t)nph * nlist;
    // queries per scan work item (the tracing instantiations exist for 16 only, the split ones for 16 and 32)
    const bool split_g = ix.split && a.stage2;
    const int G = a.trace || a.group <= 16 ? 16 : (a.group <= 32 || split_g ? 32 : 64);

    // the split exact stage (an index whose tail is no wider than its leading block, with the Eq 7 stage on)
    // needs the query's tail coordinates in FP32 (rows padded to Dr4); otherwise they only feed Eq 6 and come
    // from the BF16 product
    const bool split = ix.split && a.stage2;
    const int64_t ldt = split ? (int64_t)ix.Dr4 : (int64_t)(D - d);
    {   // Algorithm 2, projection: q_d = P_p[:d] (q - mu) and the tail coordinates for Eq 6
        Timed t(tm, s, "project");
        HIP_TRY(launch_query_projection(ix, a.Q, nq, w.qd, w.qtail, ldt, split ? nullptr : w.qbf, s));
        hipLaunchKernelGGL(k_query_stats, dim3((unsigned)nq), dim3(64), 0, s, a.Q, D, D4, ix.mu, w.qd, d, d4,
                           w.qtail, ldt, ix.lamTail, a.m, w.qpad, w.qn2, w.qd2, w.Tq, w.er);
        HIP_TRY(hipGetLastError());
        HIP_TRY(launch_gemm_mfma<0>(w.qd, d4, nullptr, ix.PrT, d4, w.rq, d4, nq, d, d, nullptr, nullptr, nullptr, 0,
                                    0, s));
    }
    {   // centroid ranking
        Timed t(tm, s, "probe");
        HIP_TRY(launch_gemm_mfma<1>(w.qd, d4, nullptr, ix.C, d4, w.G, nlist, nq, nlist, d, w.qd2, ix.Cn2, nullptr,
                                    0, 0, s, w.TM));
        launch_select(w.G, nlist, a.npq, a.pair_off, w.pair_list, w.pair_q, nq, a.np_max, s, w.TM, w.redo);
        HIP_TRY(hipGetLastError());
    }
    ScanCtx c;
    c.recs = w.recs; c.qu8 = w.qu8; c.boff = w.boff; c.ioff = w.ioff; c.desc = w.desc;
    c.list_off = ix.list_off; c.list_nb = ix.list_nb; c.list_len = ix.list_len; c.code = ix.code; c.ext = ix.ext;
    c.fA = ix.fA; c.fF = ix.fF; c.fE = ix.fE; c.fFB = ix.fFB; c.fEB = ix.fEB; c.fSX = ix.fSX;
    c.xd = ix.xd; c.ax = ix.ax; c.X = ix.X; c.ids = ix.ids; c.qd = w.qd; c.qpad = w.qpad; c.qn2 = w.qn2; c.er = w.er;
    c.kq = a.kq; c.npq = a.npq; c.slot_off = a.slot_off; c.pair_off = a.pair_off; c.pair_pos = w.pair_pos;
    c.slots = w.slots; c.surv = w.surv; c.qcnt = w.qcnt; c.counters = a.counters;
    c.pair_list = w.pair_list; c.rq = w.rq; c.RC = ix.RC; c.Tq = w.Tq; c.eps0 = a.eps0; c.tr = a.trace;
    c.cnt_ext = a.counters && a.ncounters >= 16;
    c.split = split;
    c.Dr4 = ix.Dr4;
    c.RX4 = split ? ix.Dr4 : ix.D4;
    c.xr = ix.xr;
    c.qr = w.qtail;
    c.survd = w.survd;
    c.nlist = nlist; c.d = d; c.d4 = d4; c.D4 = D4; c.B = ix.B; c.bq = a.bq; c.G = G;
    c.WP = ix.WP; c.KI = (d + 63) / 64; c.KP = level_bytes(d);
    c.stage2 = a.stage2; c.use_ext = a.use_ext; c.phase = 0; c.k_max = a.k_max;
    // persistent scan grid (resident blocks) and each query's bin of the exact-stage buffer
    const int scan_blocks = scan_grid(c);
    int64_t cap = surv_capacity(ix, a.total_pairs);
    if (a.exact_cap > 0 && a.exact_cap < cap) cap = a.exact_cap;
    c.cq = (int)(cap / nq);
    // The seed pass (each query's nearest list; it computes that pair's query code itself) runs on the
    // index's auxiliary stream beside the pair preparation; the phases wait for both.
    // Without a fork (the allocation-free search) the seed pass runs first on the search stream.
    HIP_TRY(fill_u64(w.slots, kEmptyKey, a.total_slots, s));
    HIP_TRY(launch_fill_i32(w.qcnt, 0, nq, s));
    // The fork's stream and events are the caller's (a server slot's) or the index's own.
    hipStream_t aux = a.aux;
    hipEvent_t ev_fork = a.ev_fork, ev_join = a.ev_join;
    if (a.fork_seed) {
        if (!aux) {
            if (!ix.aux) {
                HIP_TRY(hipStreamCreateWithFlags(&ix.aux, hipStreamNonBlocking));
                HIP_TRY(hipEventCreateWithFlags(&ix.ev_fork, hipEventDisableTiming));
                HIP_TRY(hipEventCreateWithFlags(&ix.ev_join, hipEventDisableTiming));
            }
            aux = ix.aux;
            ev_fork = ix.ev_fork;
            ev_join = ix.ev_join;
        }
        HIP_TRY(hipEventRecord(ev_fork, s));
        HIP_TRY(hipStreamWaitEvent(aux, ev_fork, 0));
    }
    const hipStream_t seed_s = a.fork_seed ? aux : s;
    {
        Timed t(tm, seed_s, "seed");
        launch_seed(c, nq, seed_s);
        HIP_TRY(hipGetLastError());
    }
    if (a.fork_seed) HIP_TRY(hipEventRecord(ev_join, aux));
    {   // per-pair query codes, grouped by (phase, list)
        Timed t(tm, s, "pair_prep");
        HIP_TRY(launch_fill_i32(w.cnt, 0, P, s));
        HIP_TRY(launch_fill_i32(w.fill, 0, P, s));
        hipLaunchKernelGGL(k_pair_count, dim3((unsigned)((a.total_pairs + 255) / 256)), dim3(256), 0, s,
                           w.pair_list, w.pair_q, a.pair_off, a.pair_off + nq, nlist, a.phase_shift, w.cnt);
        launch_scan_excl_seg(w.cnt, w.boff, P, w.segsum, s);
        const int nh = (d + 63) / 64;
        const int KP = level_bytes(d);
        // 16 lanes per pair up to d = 256 (4 pairs per wave: the kernel is bound by the latency of its loads
        // and atomic), a whole wave beyond
#define PREP_T(NHV, LV, TRV)                                                                                \
    hipLaunchKernelGGL((k_pair_prep<NHV, LV, TRV>), dim3((unsigned)((a.total_pairs + 256 / LV - 1) / (256 / LV))), \
                       dim3(256), 0, s, w.pair_list, w.pair_q, a.pair_off, a.pair_off + nq, nlist, a.phase_shift, \
                       w.rq, ix.RC, d, d4, ix.WP, a.bq, a.eps0, w.Tq, w.er, w.qn2, w.boff, w.fill, KP, w.recs,  \
                       w.qu8, w.pair_pos, a.trace)
#define PREP(NHV, LV)                     \
    do {                                  \
        if (a.trace) PREP_T(NHV, LV, true);  \
        else PREP_T(NHV, LV, false);      \
    } while (0)
        if (nh <= 1) PREP(1, 16);
        else if (nh <= 2) PREP(2, 16);
        else if (nh <= 4) PREP(4, 16);
        else if (nh <= 8) PREP(8, 64);
        else if (nh <= 16) PREP(16, 64);
        else PREP(24, 64);
#undef PREP
#undef PREP_T
        hipLaunchKernelGGL(k_items, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, w.cnt, ix.list_nb,
                           nlist, G, (int)P, w.items);
        launch_scan_excl_seg(w.items, w.ioff, P, w.segsum, s);
        hipLaunchKernelGGL(k_item_desc, dim3((unsigned)((P + 3) / 4)), dim3(256), 0, s, w.ioff, w.boff, ix.list_nb,
                           ix.list_off, nlist, G, P, w.desc);
        HIP_TRY(hipGetLastError());
    }
    if (a.fork_seed) HIP_TRY(hipStreamWaitEvent(s, ev_join, 0));
    for (int p = 1; p < kPhases; p++) {
        if (a.np_max <= phase_lo(p, a.phase_shift)) break;
        c.phase = p;
        {
            Timed t(tm, s, "tau");
            hipLaunchKernelGGL(k_tau_snap, dim3((unsigned)((a.total_pairs + 255) / 256)), dim3(256), 0, s,
                               w.slots, a.slot_off, a.kq, w.boff, nlist, p, a.pair_off + nq, w.recs);
        }
        {
            Timed t(tm, s, "scan");
            launch_scan(c, s, scan_blocks);
            HIP_TRY(hipGetLastError());
        }
        {
            Timed t(tm, s, "exact");
            const size_t qk = (size_t)a.k_max * sizeof(unsigned long long);
            const size_t ql = (size_t)c.RX4 * sizeof(float) + qk;
#define EXACT(QLV, TRV, SPV, LDS) hipLaunchKernelGGL((k_exact<QLV, TRV, SPV>), dim3((unsigned)nq), dim3(256), LDS, s, c)
            const bool ql_ex = c.RX4 <= kExactLdsFloats;
            if (ql_ex && split) { if (a.trace) EXACT(true, true, true, ql); else EXACT(true, false, true, ql); }
            else if (ql_ex) { if (a.trace) EXACT(true, true, false, ql); else EXACT(true, false, false, ql); }
            else if (split) { if (a.trace) EXACT(false, true, true, qk); else EXACT(false, false, true, qk); }
            else { if (a.trace) EXACT(false, true, false, qk); else EXACT(false, false, false, qk); }
#undef EXACT
            HIP_TRY(hipGetLastError());
        }
    }
    {
        Timed t(tm, s, "finalize");
        hipLaunchKernelGGL(k_finalize, dim3((unsigned)nq), dim3(64), 0, s, w.slots, a.slot_off, a.kq,
                           a.out_off, a.ids, a.dists);
        HIP_TRY(hipGetLastError());
    }
    return hipSuccess;
}

}  // namespace mrq
