// Internal definitions shared by the host runtime and the HIP kernels of the MRQ library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "mrq.h"

namespace mrq {

constexpr int kWave = 64;        // gfx950 wavefront width
constexpr int kBlockVecs = 64;   // vectors per code block = one vector per lane
constexpr int kPhases = 11;      // probe-rank phases: {0}, [1,2), [2,4), [4,8), ..., [512,1024)
// log2 of a phase growth g (a power of two in [2, 1024]); 0 -> `dflt`; -1 for any other value
inline int phase_shift_of(int g, int dflt) {
    if (g == 0) return dflt;
    for (int sh = 1; sh <= 10; sh++)
        if (g == (1 << sh)) return sh;
    return -1;
}
constexpr int kMaxK = 1024;
constexpr int kMaxProbe = 1024;
constexpr uint64_t kEmptyKey = ~0ull;

// Per (query, list) pair: everything the stage-1, B-bit and Eq 7 tests need besides the query codes
// (12 dwords; the first eight are the test scalars).
struct PairRec {
    float Kr;        // ||q_d - c||^2 + ||q_r||^2 - eps_r  (query part of C1 minus the residual radius)
    float two_nq;    // 2 ||q_d - c||
    float vl;        // quantised query: lowest level
    float delta;     // quantised query: level step
    float su;        // sum of the query levels (exact integer)
    float ebc;       // 2 ||q_d - c|| eps0 / sqrt(d - 1)
    float tau;       // pruning threshold of the query for the current phase
    float er;        // eps_r = 2 m sigma of the query (Eq 6)
    int32_t q;       // query index in the batch
    int32_t list;    // IVF list id
    float qn2;       // ||q - mu||^2 = ||q_p||^2 (Eq 7)
    float pad;
};
static_assert(sizeof(PairRec) == 48, "PairRec layout");

// Code words per row: the smallest instantiated width >= ceil(d / 32).
int padded_words(int d);

struct KernelTimer {
    bool on = false;
    std::vector<std::string> names;
    std::vector<double> ms;
    std::vector<int64_t> launches;
    struct Pending { int slot; hipEvent_t a, b; };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> pool;
    int slot_of(const char* name);
    void begin(hipStream_t s, const char* name, Pending* p);
    void end(hipStream_t s, Pending* p);
    void collect();   // synchronises on the recorded events and accumulates
    ~KernelTimer();
};

struct Workspace {
    // grow-only device scratch for one search call
    void* base = nullptr;
    size_t bytes = 0;
    bool captured = false;       // a captured graph refers to `base`: growth must not free it
    std::vector<void*> retired;  // earlier buffers kept for captured graphs, freed with the index
};

struct Index {
    int64_t N = 0;
    int32_t D = 0, d = 0, B = 1, nlist = 0;
    int32_t W = 0, WP = 0;       // code words per row: needed / stored (padded)
    int32_t d4 = 0, D4 = 0;      // d and D rounded up to a multiple of 4 (padded row strides)
    int64_t Npad = 0;            // rows after padding every list to a multiple of 64
    int device = 0;

    // device arrays
    float* mu = nullptr;         // D
    float* Pp = nullptr;         // D x D, row i = axis i
    float* PpLead = nullptr;     // d x D (rows 0..d-1 of Pp), contiguous
    float* PpTail = nullptr;     // (D - d) x D
    float* lamTail = nullptr;    // D - d
    float* PrT = nullptr;        // d4 x d4: row j = column j of P_r (zero padded)
    float* C = nullptr;          // nlist x d4 centroids (zero padded)
    float* Cn2 = nullptr;        // nlist: ||c_j||^2
    float* RC = nullptr;         // nlist x d4: P_r^T c_j
    int64_t* list_off = nullptr; // nlist + 1 padded row offsets
    int32_t* list_len = nullptr; // nlist real lengths
    int32_t* list_nb = nullptr;  // nlist: 64-row blocks per list
    int32_t* ids = nullptr;      // Npad, -1 on padding rows
    uint32_t* code = nullptr;    // Npad x WP sign plane
    uint32_t* ext = nullptr;     // Npad x (B - 1) x WP lower planes of the B-bit code
    float* fA = nullptr;         // Npad: ||x_d - c||^2 + ||x_r||^2 (+inf on padding rows)
    float* fF = nullptr;         // Npad: ||x_d - c|| / (sqrt(d) xi1)
    float* fE = nullptr;         // Npad: ||x_d - c|| sqrt(1 - xi1^2) / xi1
    float* fFB = nullptr;        // Npad: ||x_d - c|| / (2 ||y|| xiB)
    float* fEB = nullptr;        // Npad: ||x_d - c|| sqrt(1 - xiB^2) / xiB
    float* fSX = nullptr;        // Npad: 2 sum_i u_i - (2^B - 1) d
    float* xd = nullptr;         // Npad x d4 leading coordinates of x_p
    float* ax = nullptr;         // Npad: ||x - mu||^2
    float* X = nullptr;          // Npad x D4 original vectors (zero padded), list order: the exact stage
    // split exact stage (when the tail is no wider than the leading block, D - d <= d): the exact distance
    // is the stage-2 value minus twice the tail product, ||x - q||^2 = dis_o' - 2 <x_r, q_r>, so stage 3
    // reads only the tail coordinates (d = D: nothing)
    bool split = false;
    int32_t Dr = 0, Dr4 = 0;     // tail width D - d and its padding to a multiple of 4
    float* xr = nullptr;         // Npad x Dr4 tail coordinates of x_p (zero padded), list order
    // export-only per-row summaries (list order)
    float *nx = nullptr, *tx = nullptr, *xi1 = nullptr, *xiB = nullptr, *yn = nullptr;
    // MR-SQ codes (built on request): dq = 16 ceil(d / 16) (0 = none); per coordinate the grid lo / delta
    // (dq entries, lo 0 and delta 1 beyond d); per row dq code bytes in scan order; per row
    // A = ||xhat_d||^2 + ||x_r||^2 (+inf on padding rows)
    int32_t dq = 0;
    float* sq_lo = nullptr;
    float* sq_delta = nullptr;
    uint8_t* sq_code = nullptr;
    float* sq_A = nullptr;

    // host copies
    std::vector<double> lam64;
    std::vector<int64_t> h_off_real;   // nlist + 1 unpadded offsets (export)
    std::vector<int64_t> h_list_off;   // nlist + 1 padded offsets
    int32_t max_list_len = 0;

    std::vector<void*> allocations;
    int64_t device_bytes = 0;

    // search workspace (grow-only) and instrumentation
    mutable Workspace ws;
    mutable KernelTimer timer;
    mutable std::mutex mu_ws;
    int group_default = 32;
    int phase_shift_default = 2;  // log2 of the default phase growth
    // auxiliary stream (default priority) on which the seed pass runs beside the pair preparation, and
    // the events that fork it from and join it to the search stream; created by the first search
    mutable hipStream_t aux = nullptr;
    mutable hipEvent_t ev_fork = nullptr, ev_join = nullptr;

    ~Index();
};

// Where the tracing instantiation of the search kernels records per-stage values (mrq_search_trace);
// device memory, null in ordinary searches.
struct TraceSink {
    const uint8_t* qflag;          // nq: 1 = the query is traced
    mrq_trace_pair* pairs;         // max_pairs
    float* qp;                     // max_pairs x d: q' of the pair
    uint8_t* u;                    // max_pairs x d: levels of the pair
    mrq_trace_cand* cands;         // max_cands
    unsigned long long* n;         // [0] pair records, [1] candidate records (counted beyond the maxima)
    int64_t max_pairs, max_cands;
};

// ---- kernels (defined in mrq_search.hip and mrq_build.hip) --------------------------------------------------------
struct SearchArgs {
    const Index* ix;
    const float* Q;        // device nq x D
    int64_t nq;
    const int32_t* kq;     // device nq
    const int32_t* npq;    // device nq
    const int64_t* slot_off;   // device nq + 1
    const int64_t* pair_off;   // device nq + 1
    const int64_t* out_off;    // device nq
    int64_t total_slots, total_pairs;
    int32_t np_max, k_max;
    int32_t bq;
    float eps0, m;
    int32_t stage2, use_ext, group;
    int64_t exact_cap = 0;  // exact-stage buffer entries per phase (0 = automatic)
    int32_t method = 0;     // MRQ_METHOD_MRQ or MRQ_METHOD_MRSQ
    int32_t phase_shift = 2;  // phases [1, 2^s), [2^s, 2^2s), ... of the probe ranks
    int32_t rerank = 500;   // MR-SQ: candidates re-ranked by exact distance per query
    int64_t* ids;          // device output
    float* dists;          // device output
    int64_t* counters;     // device int64[ncounters] or null
    int32_t ncounters = 8; // 8 or 16
    bool timed = true;     // record per-kernel events when the index timer is on
    bool fork_seed = true; // run the seed pass on the index's auxiliary stream beside the pair preparation
    const TraceSink* trace = nullptr;  // device; non-null: run the tracing instantiations (query group 16)
    // stream and events of the seed pass's fork (null: the index's own, created by its first search)
    hipStream_t aux = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
};

size_t search_workspace_bytes(const Index& ix, int64_t nq, int64_t total_slots, int64_t total_pairs,
                              int bq, int np_max, int method, int rerank);
hipError_t launch_search(const SearchArgs& a, void* ws, size_t ws_bytes, hipStream_t s);

// The allocation-free search's fixed device buffer on the current device (a file-scope device array of
// kNoAllocBytes, its address looked up once per device).
constexpr size_t kNoAllocBytes = MRQ_NOALLOC_BYTES;
hipError_t noalloc_scratch(void** p, size_t* bytes);
// Streaming copy of bytes / 16 words (16-byte aligned device pointers).
hipError_t launch_stream_copy(void* dst, const void* src, size_t bytes, hipStream_t s);

// build-side launchers
// MR-SQ codes of an index whose x_d and ids are in place (tx64_rows: FP64 ||x_r||^2 per row; scratch:
// 2 nchunk d floats)
hipError_t launch_sq8_build(Index& ix, const double* tx64_rows, float* scratch, int nchunk, hipStream_t s);
hipError_t launch_colmean(const float* X, int64_t N, int D, double* part, int nchunk, double* mu64,
                          hipStream_t s);
hipError_t launch_cov(const float* X, int64_t N, int D, const double* mu64, double* part, int nsplit,
                      double* S, hipStream_t s);
int cov_splits(int64_t N, int D);
// x_p = P_p (x - mu) for M rows of X (row stride D) on the matrix cores: coordinates < d into lead
// (row stride ld_lead), the others into tail (row stride ld_tail).
hipError_t launch_project(const float* X, int64_t M, int D, const float* mu, const float* Pp, int d, float* lead,
                          int64_t ld_lead, float* tail, int64_t ld_tail, hipStream_t s);
hipError_t launch_gemm_nt(const float* A, int64_t lda, const float* asub, const float* Bm, int64_t ldb,
                          float* Cm, int64_t ldc, int64_t M, int N, int K, hipStream_t s);
hipError_t launch_rownorms(const float* X, int64_t N, int D, const double* mu64, const float* xd,
                           int d4, int d, double* ax64, double* tx64, hipStream_t s);
hipError_t launch_kmeans_assign(const float* P, int64_t n, int ldp, int dim, const float* C, int ldc,
                                const float* cn2, int k, const float* pn2, int32_t* assign, float* mind,
                                hipStream_t s);
hipError_t launch_kmeans_accum(const float* P, int64_t n, int ldp, int dim, const int32_t* assign,
                               const int32_t* prev, double* sums, int32_t* cnt, int32_t* changed,
                               hipStream_t s);
hipError_t launch_kmeans_centroids(const double* sums, const int32_t* cnt, int k, int dim, float* C,
                                   int ldc, float* cn2, hipStream_t s);
hipError_t launch_sqnorms(const float* A, int64_t n, int lda, int dim, float* out, hipStream_t s);
hipError_t launch_gather_layout(const Index& ix, const float* Xraw, const int32_t* perm,
                                const float* xd_id, const double* ax64, const double* tx64, double* txr,
                                int32_t* row_list, float* O, const float* xt_id, hipStream_t s);
hipError_t launch_encode(const Index& ix, const float* O, const float* Xpp, const double* tx64_rows,
                         hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s);
hipError_t launch_uniform_meta(int64_t nq, int k, int np, int32_t* kq, int32_t* npq, int64_t* slot_off,
                               int64_t* pair_off, int64_t* out_off, hipStream_t s);
hipError_t launch_mixed_meta(int64_t nq, const int32_t* k, const int32_t* np, const int64_t* out_off_in, int kb,
                             int npb, int32_t* kq, int32_t* npq, int64_t* slot_off, int64_t* pair_off,
                             int64_t* out_off, int32_t* rejected, hipStream_t s);
hipError_t launch_gather_rows(const float* src, int64_t lds, const int32_t* idx, int64_t n, int dim,
                              float* dst, int64_t ldd, hipStream_t s);
hipError_t launch_fill_f32(float* p, float v, int64_t n, hipStream_t s);
hipError_t launch_check_finite(const float* X, int64_t n, int32_t* bad, hipStream_t s);

// host eigensolver (eigen_host.cpp): symmetric n x n (row-major) -> eigenvalues descending and
// eigenvectors as rows, sign rule: largest-magnitude entry positive.
void eigh_host(const double* A, int n, double* evals, double* evecs_rows);

}  // namespace mrq

// The opaque handle of the C ABI.
struct mrq_index : mrq::Index {
    hipEvent_t ws_event = nullptr;  // last use of the default search workspace
    bool ws_event_recorded = false;
};
