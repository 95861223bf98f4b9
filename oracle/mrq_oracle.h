/*
 * MRQ CPU oracle — TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded FP64 implementation of what the MRQ search path computes
 * ("Quantization Meets Projection", arXiv 2411.06158).  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it; the product library never does.  It shares no code
 * with the GPU library.
 *
 * Paper map:
 *   Eq 1-3 (Section 4.1)       projection split and the three-term distance decomposition
 *   Section 4.2, Eq 4-6        sign codes, unbiased estimator, error bounds
 *   Algorithm 1 (Section 5.1)  index build: PCA, residual variances, IVF on x_d, encoding
 *   Algorithm 2 + Eq 7 (5.2)   the multi-stage query
 *   Appendix A.2, Exp-5        MR-SQ: 8-bit scalar codes of the leading dimensions, fixed re-ranking
 *
 * Parity pins live in tests/test_oracle_*.py; "parity unpinned" items are named in the .c header.
 */
#ifndef MRQ_ORACLE_H
#define MRQ_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc_index orc_index;

typedef struct {
    double eps0;     /* Eq 5 confidence parameter */
    double m;        /* Chebyshev multiplier of Eq 6 */
    int32_t bq;      /* query code bits (Algorithm 2, query quantization) */
    int32_t stage2;  /* 1 = MRQ+ (Eq 7 stage on), 0 = plain MRQ */
    int32_t use_ext; /* 1 = refine stage-1 survivors with the B-bit code when B > 1 */
    int32_t verify;  /* 1 = also compute every exact distance and count bound violations */
} orc_params;

typedef struct {
    int64_t scanned;    /* candidates visited */
    int64_t pass1;      /* survived the 1-bit stage-1 test */
    int64_t pass_ext;   /* survived the B-bit refinement (== pass1 when B == 1) */
    int64_t pass2;      /* survived the stage-2 (Eq 7) test = exact distances computed */
    int64_t viol1;      /* candidates whose stage-1 lower bound exceeded the exact distance */
    int64_t viol_ext;   /* same for the B-bit lower bound */
    int64_t viol2;      /* candidates with dis_o' - eps_r > exact distance */
} orc_counters;

enum { ORC_EXACT_IVF = 0, ORC_ALG2 = 1 };

/* ---- building blocks (exposed for the pins) ---- */
uint64_t orc_splitmix64(uint64_t *state);
void orc_gaussian(uint64_t seed, int64_t n, double *out);
int orc_eigh(const double *A, int n, double *evals, double *evecs);
int orc_haar(int d, uint64_t seed, double *P);
void orc_encode_sign(const double *xprime, int d, uint8_t *bits, double *xi);
double orc_encode_ext(const double *xprime, int d, int B, uint8_t *u);
double orc_ext_exhaustive(const double *xprime, int d, int B, uint8_t *u);
void orc_quantize_query_f32(const float *qprime, int d, int bq, uint8_t *u, float *vl, float *delta,
                            int32_t *su);
int orc_kmeans(const double *P, int64_t n, int dim, int k, uint64_t seed, int iters, double *C,
               int32_t *assign);

/* ---- index ---- */
orc_index *orc_build(const float *X, int64_t N, int32_t D, int32_t d, int32_t B, int32_t nlist,
                     uint64_t seed, int32_t kmeans_iters);
orc_index *orc_import(const char *path, const float *X, int64_t N, int32_t D);
int orc_attach(orc_index *ix, const float *X, int64_t N, int32_t D);
void orc_free(orc_index *ix);
int orc_info(const orc_index *ix, int64_t *N, int32_t *D, int32_t *d, int32_t *B, int32_t *nlist);
int orc_get(const orc_index *ix, const char *name, void *out);

/* ---- search ---- */
int orc_probe(const orc_index *ix, const float *q, int32_t nprobe, int32_t *lists, double *g);
int orc_search(const orc_index *ix, const float *q, int32_t k, int32_t nprobe, const orc_params *p,
               int32_t mode, int64_t *ids, double *dists, orc_counters *cnt);
int orc_pair_trace(const orc_index *ix, const float *q, int32_t list, const orc_params *p,
                   double *qscal, double *qprime, uint8_t *u, int64_t *ids, double *cand);
int orc_topk_risk(const orc_index *ix, const float *q, int32_t k, int32_t nprobe, const orc_params *p,
                  double margin, int64_t *ids, double *dists, uint8_t *risk);
void orc_bruteforce(const float *X, int64_t N, int32_t D, const float *Q, int64_t nq, int32_t k,
                    int64_t *ids, double *dists);
/* ---- MR-SQ (Appendix A.2, Exp-5; readings S1-S4 in the .c header) ---- */
void orc_sq8_range(const float *xd, int64_t N, int d, int ld, float *lo, float *delta);
void orc_sq8_encode(const float *x, int d, const float *lo, const float *delta, uint8_t *u);
int orc_sq8_build(orc_index *ix);
int orc_mrsq_estimates(const orc_index *ix, const float *q, int32_t nprobe, int64_t *ids, double *est,
                       double *exact);
int orc_mrsq_search(const orc_index *ix, const float *q, int32_t k, int32_t nprobe, int32_t R, int64_t *ids,
                    double *dists);

#ifdef __cplusplus
}
#endif
#endif
