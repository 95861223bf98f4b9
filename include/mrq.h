/*
 * mrq.h — C ABI of the MI355X (gfx950) MRQ search library.
 *
 * MRQ ("Quantization Meets Projection", arXiv 2411.06158) answers approximate k-NN queries under
 * squared Euclidean distance (Section 2.1) with an IVF index over PCA-projected vectors whose leading
 * d_r dimensions carry RaBitQ-style codes (Section 4, Algorithm 1) and a three-stage query
 * (Algorithm 2 with Eq 4-7): a bit-code estimate with error bounds, the projected distance, then the
 * exact distance for the survivors.
 *
 * Conventions for every entry point:
 *   - Vectors are row-major FP32 (row stride = D floats).  X, Q and the output buffers may be device
 *     pointers (e.g. torch's data_ptr() of a CUDA tensor) or ordinary host pointers; the kind is
 *     detected per call.  The caller owns them.  The library owns the index and all its device
 *     memory.
 *   - A `stream` of NULL means the legacy default stream.  Calls are asynchronous on `stream` unless
 *     documented otherwise; device outputs are valid once the stream has been synchronised.  Host
 *     outputs are complete when the call returns.
 *   - Distances are squared L2 (Eq 1), ascending; ties are broken by the smaller id.  When fewer
 *     than k candidates exist the tail of a result row is padded with id = -1, dist = +inf.
 *   - Every call returns an mrq_status; the message of the last failure on the calling thread is
 *     available from mrq_last_error().  No exception crosses the ABI.
 *   - Calls that use the same index from several host threads must not overlap (the index holds the
 *     search workspace); different indexes are independent.
 *
 * On-disk formats (little-endian) written by mrq_save / mrq_export:
 *   "MRQX0001" export layout, field by field:
 *     char magic[8]; int64 N; int32 D, d, B, nlist;
 *     f32 mu[D]; f32 Pp[D*D] (row i = i-th principal axis, eigenvalues descending);
 *     f64 lambda[D]; f32 Pr[d*d] (row-major, x' = Pr^T (x_d - c)/||x_d - c||);
 *     f32 C[nlist*d]; i64 off[nlist+1]; i64 ids[N] (list order, ascending id inside a list);
 *     u8 code[N*d] (per leading dim the level index u in [0, 2^B), top bit = sign bit);
 *     f32 xd[N*d]; f32 nx[N], tx[N], ax[N], xi1[N], xiB[N], yn[N]   (all in list order)
 *   where nx = ||x_d - c||, tx = ||x_r||^2, ax = ||x - mu||^2, xi1 = <xbar_1bit, x_b>,
 *   xiB = <xbar_Bbit, x_b>, yn = ||u - (2^B - 1)/2||.
 *   An index built with MR-SQ codes appends: char tag[4] = "SQ8G"; f32 lo[d], delta[d];
 *   u8 sq[N*d] (list order, leading dim i of vector n at n*d + i).
 */
#ifndef MRQ_H
#define MRQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mrq_index mrq_index;   /* opaque, library-owned */
typedef struct mrq_server mrq_server; /* opaque, library-owned */
typedef void *mrq_stream;             /* a hipStream_t */

typedef enum {
    MRQ_OK = 0,
    MRQ_EINVAL = 1,  /* an argument is out of range, a pointer is NULL or an input is not finite */
    MRQ_ENOMEM = 2,  /* device or host allocation failed */
    MRQ_EDEVICE = 3, /* a HIP runtime call failed */
    MRQ_ESTATE = 4,  /* the object is not in a state that allows the call */
    MRQ_EIO = 5      /* file could not be read / written or has the wrong format */
} mrq_status;

enum { MRQ_BATCHED = 0, MRQ_PER_QUERY = 1 };

/* Search methods over one index (mrq_search_opts.method). */
enum {
    MRQ_METHOD_MRQ = 0,  /* Algorithm 2 with the Eq 7 stage (Section 5.2) */
    MRQ_METHOD_MRSQ = 1  /* MR-SQ (Appendix A.2, Exp-5): 8-bit scalar codes of the leading d_r PCA
                            coordinates, estimate = Eq 7's projected distance with x_d replaced by its
                            reconstruction, then exact re-ranking of a fixed number of candidates */
};

typedef struct {
    uint64_t seed;        /* k-means initialisation and the random rotation P_r; default 4001 */
    int32_t kmeans_iters; /* Lloyd iterations (stops early when no assignment changes); default 25 */
    int32_t sq8;          /* 1 = also build the MR-SQ codes (needed by MRQ_METHOD_MRSQ); default 0 */
    int32_t reserved[6];
} mrq_build_opts;

typedef struct {
    int32_t mode;           /* MRQ_BATCHED (default) or MRQ_PER_QUERY (one query per pipeline pass) */
    int32_t bq;             /* query code bits B_q in [1, 8]; default 4 (Algorithm 2, quantise q) */
    float eps0;             /* Eq 5 confidence parameter; default 1.9; <= 0 selects the default */
    float m;                /* Eq 6 / Chebyshev multiplier; eps_r = 2 m sigma; default 3 */
    int32_t stage2;         /* 1 = use the Eq 7 projected-distance stage (MRQ+), 0 = plain MRQ; default 1 */
    int32_t use_ext;        /* 1 = refine stage-1 survivors with the B-bit code when B > 1; default 1 */
    int64_t *counters;      /* optional device or host int64[ncounters], accumulated (not cleared):
                               [0..3] batched scan: candidates scanned, stage-1 survivors, B-bit
                               survivors, exact distances; [4..7] the same for the seed pass over
                               each query's nearest list */
    int32_t group;          /* queries per scan work item: 16, 32 or 64 (0 = the index default) */
    int32_t exact_cap;      /* exact-stage buffer entries per phase (0 = automatic), split evenly into
                               one bin per query; candidates beyond a bin are finished inside the
                               scan; results do not depend on it */
    int32_t method;         /* MRQ_METHOD_MRQ (default) or MRQ_METHOD_MRSQ (index built with sq8) */
    int32_t rerank;         /* MRQ_METHOD_MRSQ: candidates re-ranked by exact distance per query, R in
                               [k, 16384]; 0 = 500.  The MRQ fields bq, eps0, m, stage2, use_ext, group
                               and exact_cap do not apply to MR-SQ; counters [0] and [3] count its
                               scanned candidates and exact distances */
    int32_t phase_growth;   /* MRQ: probe ranks are scanned in phases [1, g), [g, g^2), ... (after the nearest
                               list), each against the threshold tau reached before it; g a power of two
                               in [2, 1024] (1024: one phase after the nearest list), 0 = the index default
                               (4, or what mrq_tune chose).  A result may differ between values only where
                               an error bound fails */
    int32_t ncounters;      /* entries of `counters`: 8 (0 = 8) or 16.  With 16, [8] and [9] also count the
                               batched scan's work: work items (a 64-vector list block against up to `group`
                               pairs) and 16-row tiles whose x_d rows entered stage 2; [10..15] are left
                               untouched */
} mrq_search_opts;

/* Defaults for the option structs (pass NULL to any call to use them). */
void mrq_build_opts_default(mrq_build_opts *o);
void mrq_search_opts_default(mrq_search_opts *o);

/*
 * mrq_build — Algorithm 1 (Section 5.1): PCA of X (mean-centred, FP64 covariance), residual
 * variances lambda_i, rotation x_p = P_p (x - mu), residual norms ||x_r||, IVF with nlist lists
 * trained on the leading d_r coordinates x_d, and the per-vector code of (x_d - c)/||x_d - c|| under
 * a random orthogonal P_r (Section 4.2) with B bits per leading dimension (B = 1: sign code; B > 1:
 * extended code whose top bit is the sign bit), plus the normalisation factors ||x_d - c||,
 * ||x_r||, <xbar, x_b>.  Every original vector is also kept (FP32, list order) for the exact stage,
 * which computes ||x - q||^2 (= ||x_p - q_p||^2, Eq 1).
 *   X      N x D FP32, host or device, finite values only (checked: MRQ_EINVAL otherwise)
 *   d_r    in [2, min(D, 1536)], or 0 for the Eq 8 choice (mrq_choose_dr on the data's eigenvalues);
 *          bits B in [1, 8];  nlist in [1, min(N, 16384)]
 *   opts   with sq8 = 1 the index also holds MR-SQ codes (Appendix A.2, Exp-5): per leading coordinate i
 *          the range [lo_i, hi_i] over the data set, step delta_i = (hi_i - lo_i)/255 (1 when
 *          hi_i == lo_i) and code u_i = min(255, floor((x_i - lo_i) * (1/delta_i) + 1/2)), each step
 *          one FP32 rounding; d_r bytes per vector
 *   stream where the device work runs; the call synchronises it before returning
 *   out    receives a new index on MRQ_OK (free with mrq_free); untouched on failure
 */
mrq_status mrq_build(const float *X, int64_t N, int32_t D, int32_t d_r, int32_t bits, int32_t nlist,
                     const mrq_build_opts *opts, mrq_stream stream, mrq_index **out);

/*
 * mrq_search — Algorithm 2 with the Eq 7 stage for nq queries at once: project each query with
 * P_p (Algorithm 2, first steps), compute sigma of Eq 6, rank the centroids by distance to q_d and
 * take the nprobe nearest lists, quantise the normalised and rotated q_d per (query, list) pair,
 * then for every candidate: estimate (Eq 4), prune with the bound of Eq 5 plus the residual bound
 * (Eq 6), re-check with Eq 7, and compute the exact distance for the survivors.
 *   Q      nq x D FP32 (host or device);  nq >= 1;  1 <= k <= 1024;  1 <= nprobe <= min(nlist, 1024)
 *   ids    nq x k int64 output (host or device);  dists  nq x k FP32 output (host or device)
 * The result of a query does not depend on the other queries of the batch nor on `mode`.
 * The call may be recorded into a HIP graph (stream capture on `stream`) when Q, ids, dists and counters
 * are device buffers, kernel timing is off and the same search (same nq, k, nprobe, options) ran once
 * before on this index, which sizes its workspace; otherwise MRQ_ESTATE.  Replays use the index's
 * workspace and must not overlap other searches on the index; a later search that needs a larger
 * workspace keeps the captured one allocated until mrq_free.
 * With opts->method = MRQ_METHOD_MRSQ (index built with sq8, else MRQ_ESTATE): for every candidate of
 * the probed lists the estimate ||xhat_d - q_d||^2 + ||x_r||^2 + ||q_r||^2 (xhat_i = lo_i + delta_i u_i,
 * FP32), then per query the R candidates with the smallest (estimate, id) get their exact distance and
 * the k nearest of them are returned (R = opts->rerank, k <= R).
 */
mrq_status mrq_search(const mrq_index *index, const float *Q, int64_t nq, int32_t k, int32_t nprobe,
                      int64_t *ids, float *dists, const mrq_search_opts *opts, mrq_stream stream);

/*
 * mrq_search_noalloc — mrq_search for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same kernels and results as
 * mrq_search, with the search's workspace taken from a fixed device buffer of MRQ_NOALLOC_BYTES that the
 * library holds on each device it runs on until the process ends.  The call makes no device or host
 * allocation: no hipMalloc / hipFree, no stream or event creation (the seed pass runs on `stream` itself,
 * before the pair preparation), no kernel-timing events (timing is ignored).
 *   Q, ids, dists (and opts->counters, if set) must be device pointers; otherwise MRQ_EINVAL.
 *   A search whose workspace (metadata, projected queries, probe distances nq x nlist, pair records and
 *   query levels, the exact-stage buffer) exceeds MRQ_NOALLOC_BYTES fails with MRQ_EINVAL before any
 *   device work; split the batch.  Other arguments and errors as for mrq_search.
 * Every call on a device shares that device's buffer and leaves its contents behind (the search clears
 * what it needs with its own fill kernels), so calls that overlap on one device — on different streams or
 * host threads, on any index — race and must be serialised by the caller.
 */
#define MRQ_NOALLOC_BYTES ((size_t)128 << 20)
mrq_status mrq_search_noalloc(const mrq_index *index, const float *Q, int64_t nq, int32_t k, int32_t nprobe,
                              int64_t *ids, float *dists, const mrq_search_opts *opts, mrq_stream stream);

/*
 * mrq_stream_copy — measurement aid: copies `bytes` from src to dst (device pointers, 16-byte aligned, bytes a
 * multiple of 16) with a plain streaming kernel (each byte read once and written once, 16-byte accesses),
 * asynchronously on `stream`.  Timed over a buffer far larger than the caches, 2 x bytes / time is the HBM
 * bandwidth a streaming kernel achieves on the device, the reference the scan's bandwidth is compared with.
 */
mrq_status mrq_stream_copy(void *dst, const void *src, size_t bytes, mrq_stream stream);

/*
 * mrq_search_trace — mrq_search with the per-stage values of chosen queries recorded by the search
 * kernels themselves (a tracing instantiation of the same device code, same arithmetic), for checking
 * each stage element by element against a reference:
 *   per (query, list) pair (Algorithm 2, normalise / rotate / quantise the query for the list): the pair's
 *   scalars, its FP32 rotated unit vector q' (d floats) and its B_q-bit levels u (d bytes);
 *   per candidate and stage: stage 1 (Eq 4 estimate with the Eq 5 and Eq 6 bounds, from the integer inner
 *   product ip = sum_i b_i u_i and pc = popcount(b)), the B-bit refinement (ip = sum_i ux_i u_i), stage 2
 *   (Eq 7) and the exact distance, each with the threshold tau it was tested against.
 * Q is nq x D (host), ids / dists nq x k (host); traced[] holds ntraced distinct query indices of the batch.
 * pairs / qprime (max_pairs x d) / levels (max_pairs x d) and cands (max_cands) are host arrays; *npairs and
 * *ncands receive the number of records produced (records beyond max_* are counted, not written).  The
 * search runs with query group 16 (results never depend on it); opts->mode must be MRQ_BATCHED and
 * opts->method MRQ_METHOD_MRQ; synchronous.  Debugging and testing only: slower than mrq_search.
 */
enum { MRQ_TRACE_STAGE1 = 1, MRQ_TRACE_EXT = 2, MRQ_TRACE_STAGE2 = 3, MRQ_TRACE_EXACT = 4 };

typedef struct {
    int32_t phase;    /* 0 = the seed pass (nearest list), p >= 1 = batched phase p */
    int32_t q;        /* query index in the batch */
    int32_t list;     /* IVF list */
    int32_t su;       /* sum_i u_i */
    float nq;         /* ||q_d - c|| */
    float vl, delta;  /* lowest level and level step of the quantised q' */
    float kr;         /* ||q_d - c||^2 + ||q_r||^2 - eps_r */
    float ebc;        /* 2 ||q_d - c|| eps0 / sqrt(d - 1) */
    float er;         /* eps_r = 2 m sigma (Eq 6) */
    float qn2;        /* ||q - mu||^2 */
    float pad;
} mrq_trace_pair;

typedef struct {
    int32_t kind;     /* MRQ_TRACE_* */
    int32_t phase;    /* as in mrq_trace_pair */
    int32_t q, list;
    int64_t id;       /* vector id */
    int32_t ip;       /* STAGE1: sum_i b_i u_i; EXT: sum_i ux_i u_i (ux: the B-bit level index); else 0 */
    int32_t pc;       /* STAGE1: popcount of the sign code; else 0 */
    float v0;         /* STAGE1 / EXT: estimate minus eps_r, dis' - eps_r;  STAGE2: dis_o';  EXACT: ||x - q||^2 */
    float v1;         /* STAGE1 / EXT: eps_b (Eq 5 in distance units);  STAGE2: eps_r */
    float v2;         /* STAGE1 / EXT: the lower bound tested, dis' - eps_b - eps_r;  STAGE2: dis_o' - eps_r */
    float v3;         /* the threshold tau of the test (+inf while the result queue is not full); NaN in the seed
                         pass's stage 1, whose candidates are tested later against the tau of their batch */
} mrq_trace_cand;

mrq_status mrq_search_trace(const mrq_index *index, const float *Q, int64_t nq, int32_t k, int32_t nprobe,
                            const mrq_search_opts *opts, const int32_t *traced, int32_t ntraced, int64_t *ids,
                            float *dists, mrq_trace_pair *pairs, float *qprime, uint8_t *levels, int64_t max_pairs,
                            int64_t *npairs, mrq_trace_cand *cands, int64_t max_cands, int64_t *ncands);

/*
 * mrq_tune — autotuner of the scan schedule: runs mrq_search on Q (nq queries, host or device) with each
 * query-group size of the scan work items (16, 32, 64 queries per 64-vector block) and each phase growth
 * (2, 4, 8), times each on `stream` with HIP events, and makes the fastest pair the index's default (used
 * when mrq_search_opts.group / phase_growth are 0).  The group size never changes a result; the phase
 * growth can only where an error bound fails.  Synchronous; `group` and `phase_growth` (either may be
 * NULL) receive the choice.  The index must not be in use by another call meanwhile.
 */
mrq_status mrq_tune(mrq_index *index, const float *Q, int64_t nq, int32_t k, int32_t nprobe, mrq_stream stream,
                    int32_t *group, int32_t *phase_growth);

/*
 * mrq_search_mixed — as mrq_search, with a per-query k[i] and nprobe[i] (host or device int32
 * arrays of nq entries) in one launch.  Results of query i are written at ids + out_off[i] and
 * dists + out_off[i] (k[i] entries); out_off is an int64 array of nq entries (host or device).
 */
mrq_status mrq_search_mixed(const mrq_index *index, const float *Q, int64_t nq, const int32_t *k,
                            const int32_t *nprobe, const int64_t *out_off, int64_t *ids, float *dists,
                            const mrq_search_opts *opts, mrq_stream stream);

/*
 * mrq_search_mixed_dev — mrq_search_mixed for a batch whose per-query k[i] and nprobe[i] (Algorithm 2's
 * inputs, per query) are device arrays, with host upper bounds k_max >= every k[i] and nprobe_max >= every
 * nprobe[i].  The per-query offsets are formed and the entries checked on the device, so the call neither
 * synchronises with the host nor copies anything to it, and it may be recorded into a HIP graph (stream
 * capture) once a search of the same nq, bounds and options has run, like mrq_search.
 *   k, nprobe   nq int32 each (device); a query with k outside [1, k_max], nprobe outside [1, nprobe_max] or
 *               a negative out_off is rejected: nothing is searched or written for it, and the number of
 *               rejected queries is written to *rejected (device int32, may be NULL)
 *   out_off     nq int64 (device) offsets of the result rows, or NULL: rows packed in query order, query i
 *               at sum_{j < i} k[j] over the accepted queries
 *   k_max       in [1, 1024]; nprobe_max in [1, min(nlist, 1024)]; the workspace is sized for nq x k_max
 *               result slots and nq x nprobe_max pairs
 *   Q, ids, dists and opts->counters are device pointers; opts->mode must be MRQ_BATCHED and opts->method
 *   MRQ_METHOD_MRQ (MRQ_EINVAL otherwise).  Results equal mrq_search_mixed's.
 */
mrq_status mrq_search_mixed_dev(const mrq_index *index, const float *Q, int64_t nq, const int32_t *k,
                                const int32_t *nprobe, const int64_t *out_off, int32_t k_max, int32_t nprobe_max,
                                int64_t *ids, float *dists, int32_t *rejected, const mrq_search_opts *opts,
                                mrq_stream stream);

/*
 * mrq_choose_dr — the rule of Eq 8 (Section 5.3): the smallest power of two d = 2^i with d >= 128 whose
 * leading eigenvalues hold at least 80 % of the total variance, sum_{j<d} lambda_j >= 0.8 sum_j lambda_j
 * (lambda: the D eigenvalues in descending order, host FP64).  A choice reaching D returns D; above
 * 1536 dimensions (the largest supported d_r) it returns 1536 when D <= 1536, else 1024.  Host only;
 * returns -1 for a NULL pointer or D < 2.
 */
int32_t mrq_choose_dr(const double *lambda, int32_t D);

/* Index shape: any pointer may be NULL. */
mrq_status mrq_index_info(const mrq_index *index, int64_t *N, int32_t *D, int32_t *d_r, int32_t *bits,
                          int32_t *nlist, int64_t *device_bytes);

/* Write the index in the "MRQX0001" layout above (lossless for everything the search reads except
 * the original vectors, which the caller keeps).  Synchronous. */
mrq_status mrq_export(const mrq_index *index, const char *path);

/* Persist / restore a complete index: "MRQS0005", the shape (N, padded rows, D, d_r, bits, nlist, code
 * words per row, longest list, MR-SQ flag), the FP64 eigenvalues, the list offsets, then every device
 * array of the index (projection, rotation, centroids, codes, factors, x_d, the vectors in PCA
 * coordinates, the tail rows x_r of the split exact stage and the MR-SQ codes when present) in a fixed
 * order.  The format is private to this library version.  mrq_load allocates on the current device.
 * Synchronous. */
mrq_status mrq_save(const mrq_index *index, const char *path);
mrq_status mrq_load(const char *path, mrq_index **out);

/* Release an index and all its device memory.  NULL is ignored. */
void mrq_free(mrq_index *index);

/* Message of the last failed call on this thread ("" if none). */
const char *mrq_last_error(void);

/*
 * Per-kernel device time of the last search calls on this index, measured with HIP events recorded
 * on the search stream around each kernel.  names: a '\n'-separated list written into `names`
 * (capacity `cap` bytes); ms[i] / launches[i] accumulate per kernel; returns the kernel count, or
 * -1 on error.  mrq_timing_enable(index, 1) turns the events on (off by default), 0 off; reset
 * clears the accumulators.
 */
int mrq_timing(const mrq_index *index, char *names, size_t cap, double *ms, int64_t *launches, int max);
mrq_status mrq_timing_enable(mrq_index *index, int on, int reset);

/*
 * Serving (continuous batching) of mrq_search for requests that arrive one at a time.  A server owns a
 * host thread and two batch slots (each with its own stream, its own auxiliary stream and events for the
 * search's seed pass, pinned staging buffers and a device buffer).  Submitted requests wait in arrival
 * order; whenever a slot is free the thread admits the waiting requests (up to max_slots per batch) whose
 * batch still fits the slot's device buffer, copies them to the device, runs one mixed-k / nprobe batched
 * search and copies the results back on the slot's stream, so a new batch is packed and launched while
 * the previous one is still on the device.  A request's result is the same as mrq_search's for that query
 * alone (search results do not depend on the batch).  The server shares only the index's read-only
 * arrays, so the index may also be searched directly while the server runs (not tuned or freed).
 *   mrq_server_create:  mem_budget = device bytes of the server (0 = no limit): each slot's buffer is half
 *                       of it, allocated here, so nothing is allocated or freed while batches run;
 *                       max_slots in [1, 65536] queries per batch; opts as for mrq_search (mode and
 *                       counters are ignored); the index must outlive the server
 *   mrq_server_submit:  q_host = D floats (copied before return); MRQ_EINVAL for a bad k or nprobe,
 *                       MRQ_ENOMEM when one such request alone would exceed a slot's half of the budget;
 *                       otherwise the request is queued until it can be admitted
 *   mrq_server_poll:    moves up to max_done finished requests out: req_ids[i], ks[i] (may be NULL),
 *                       ids / dists rows of stride `row` (>= the request's k), latency_ms[i] = arrival
 *                       to completion (may be NULL; -1 if the batch failed, its row is -1 / +inf);
 *                       returns the number written, or -1 on bad arguments
 *   mrq_server_drain:   waits until every submitted request has finished; MRQ_ESTATE on timeout
 *   mrq_server_destroy: stops the thread after the batches in flight and frees the server
 * The submit / poll / drain calls are thread-safe.
 */
mrq_status mrq_server_create(const mrq_index *index, size_t mem_budget, int32_t max_slots,
                             const mrq_search_opts *opts, mrq_server **out);
mrq_status mrq_server_submit(mrq_server *server, uint64_t req_id, const float *q_host, int32_t k,
                             int32_t nprobe);
int mrq_server_poll(mrq_server *server, uint64_t *req_ids, int32_t *ks, int64_t *ids, float *dists,
                    int32_t row, int32_t max_done, double *latency_ms);
mrq_status mrq_server_drain(mrq_server *server, int64_t timeout_ms);
void mrq_server_destroy(mrq_server *server);
/* Server statistics (any pointer may be NULL): device bytes held now and at most, batches launched, and the
 * largest number of batches on the device at once (2 when a batch was launched while the other slot's was
 * still running). */
mrq_status mrq_server_stats(const mrq_server *server, int64_t *device_bytes, int64_t *peak_device_bytes,
                            int64_t *batches, int32_t *max_in_flight);

#ifdef __cplusplus
}
#endif
#endif /* MRQ_H */
