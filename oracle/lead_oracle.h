/*
 * LEAD oracle: a plain, single-threaded FP64 CPU implementation of the
 * quantum Tanner code construction (Section II) and of the LEAD decoder
 * (Algorithm 1, Section III-B) with belief propagation as both the local and
 * the global decoder.
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU decoder;
 * only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load it.  It shares no source with the GPU library.
 *
 * What pins each part (tests/test_oracle_*.py):
 *   construction   square/view incidence from the face definition (Sec. II-A),
 *                  the Appendix-A local check rows, tensor/RREF structure,
 *                  CSS, brute-force rank and logicals on 10- and 12-qubit codes
 *   oracle_bp      brute-force exact marginals / min-cost differences on
 *                  depth-1..3 computation trees and on forest views; scaled
 *                  single-check min-cost after one iteration; stopping rule
 *   oracle_aggregate  Appendix-A aggregation example (0.21, 0.25 -> 0.23)
 *   oracle_decode  zero-syndrome closed form, converged => H e = s, invalid
 *                  syndromes never converge, boost is a no-op for BP, local
 *                  slices against computation trees, equivariance under the
 *                  centre of D_6
 *   oracle_global_bp  the same BP routine as oracle_bp; its first iteration
 *                  against the scaled single-check min-cost closed form on
 *                  the global graph, its zero-syndrome closed form
 *   oracle_osd     OSD-0 is the information-set solution (brute force on
 *                  small matrices), unreachable syndromes reported; the
 *                  combination sweep returns the cheapest of its candidates
 *                  (enumerated independently), the cost unit against its
 *                  closed form; local and global OSD inside LEAD rebuilt
 *                  step by step from the oracle's own intermediate outputs
 *   stored outcomes  tests/golden/outcomes_*.json: 10^4-shot outcomes,
 *                  re-decoded on a sample by the current oracle
 *   margin output  diagnostic only: parity unpinned
 */
#ifndef LEAD_ORACLE_H
#define LEAD_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct oracle_code oracle_code;

/* Check type: OR_Z = Z-type checks on V0 (decode X errors),
 *             OR_X = X-type checks on V1 (decode Z errors). */
enum { OR_Z = 0, OR_X = 1 };
enum { OR_MINSUM = 0, OR_SUMPRODUCT = 1 };
enum { OR_STAGE_FULL = 0, OR_STAGE_LOCAL = 1 };

typedef struct {
    double alpha;        /* regularisation scale in (0,1]               */
    int    bp;           /* OR_MINSUM or OR_SUMPRODUCT                  */
    double ms_scale;     /* min-sum scale beta                          */
    int    max_iter_local;
    int    max_iter_global;
    double llr_clamp;    /* |mu|, |L| and |lambda'| clamped to this     */
    int    early_exit;   /* stop a BP run as soon as H e = s            */
    int    stage;        /* OR_STAGE_FULL or OR_STAGE_LOCAL             */
    int    boost;        /* apply Phase-1 confidence boost (1) or not (0) */
    /* Rounding-sensitivity probe (Monte Carlo arithmetic): when perturb > 0,
     * every computed mu, message, posterior sum and lambda' is multiplied by
     * (1 + perturb * xi), xi uniform in [-1, 1) from a SplitMix64 stream
     * keyed by perturb_seed.  perturb = 0 is the plain oracle.  Used by the
     * tests to tell well-conditioned shots from ones whose result is not
     * determined to the tolerance by FP32-sized rounding. */
    double perturb;
    uint64_t perturb_seed;
    /* 1: a local BP run that ends with H_v e_v != s_v is followed by OSD-0
     * on the view (ordered statistics decoding of order 0 with the BP
     * posteriors as reliabilities); its estimate satisfies the local
     * syndrome, so the view counts as converged for the confidence boost. */
    int    local_osd;
    /* 1: where global BP ends with H e != s, OSD on H with the global
     * posteriors as reliabilities replaces e (stats converged = 2). */
    int    global_osd;
    /* order of both OSDs: 0 = OSD-0, lambda >= 1 = combination sweep of
     * order lambda, candidate costs from the decoder's prior (the view's
     * channel priors locally; lambda' in LEAD's global stage, the channel
     * prior in global BP alone); see oracle_osd. */
    int    osd_order;
    /* 1: both OSDs rank by the exact FP64 posterior (ties in position
     * order) and price candidates with exact FP64 weights ln(1 + e^lambda),
     * instead of round(64 L) keys and round(64 ln(1 + e^lambda)) integer
     * weights.  0 (the reading shared with the GPU) is the default; 1
     * exists to measure what the rounding to 1/64 changes. */
    int    osd_exact;
} oracle_params;

/* info[] layout for oracle_info */
enum { OI_ORDER, OI_DELTA, OI_N, OI_RZ, OI_RX, OI_MZ, OI_MX, OI_RANKZ, OI_RANKX,
       OI_K, OI_ELOCZ, OI_ELOCX, OI_COUNT };

/* Build the code; returns 0 on success or a negative code with a message in
 * err: -1 argument, -2 group table, -3 symmetry/identity, -4 TNC,
 * -5 local code. */
int  oracle_build(int order, const uint16_t *mul, int delta, const int *A, const int *B,
                  int kA, const uint64_t *GA, int kB, const uint64_t *GB,
                  oracle_code **out, char *err, int errlen);
void oracle_free(oracle_code *c);
void oracle_info(const oracle_code *c, int *info);
void oracle_views(const oracle_code *c, int type, int32_t *out);      /* order x delta^2 */
void oracle_hloc(const oracle_code *c, int type, uint8_t *out);       /* r x delta^2     */
void oracle_H(const oracle_code *c, int type, uint8_t *out);          /* m x n dense     */
void oracle_logicals(const oracle_code *c, int type, uint8_t *out);   /* k x n           */

/* s = H e for `shots` packed error rows. */
void oracle_syndrome(const oracle_code *c, int type, int shots, const uint64_t *err,
                     int err_words, uint64_t *synd, int synd_words);

/* Full LEAD decode of `shots` syndromes.  prior: shots x n channel LLRs.
 * Outputs (any may be NULL): ehat packed, post (L_post), lam (lambda'),
 * stats shots x 6 {converged (1: by global BP, 2: by OSD-0), global_iters, local_iters_sum, local_iters_max,
 * local_converged_views (by BP), views resolved by OSD-0}, margin (min |mu|,
 * |L| seen), local_llr
 * (shots x order x delta^2 local posteriors). */
int  oracle_decode(const oracle_code *c, int type, const oracle_params *p, int shots,
                   const uint64_t *synd, int synd_words, const double *prior,
                   uint64_t *ehat, int ehat_words, double *post, double *lam,
                   int32_t *stats, double *margin, double *local_llr);

/* OSD-0 of H e = s with reliabilities L (see lead_oracle.c); 0 or -1. */
int  oracle_osd0(int rows, int cols, const uint8_t *H, const uint8_t *s, const double *L, uint8_t *e);
/* OSD of order `order` (0: OSD-0; >= 1: combination sweep) with candidate
 * costs from the prior LLRs `prior` (unused at order 0; see lead_oracle.c). */
int  oracle_osd(int rows, int cols, const uint8_t *H, const uint8_t *s, const double *L,
                const double *prior, int order, uint8_t *e);
/* The same with exact FP64 ranking and costs when exact = 1 (see
 * oracle_params.osd_exact). */
int  oracle_osd_ex(int rows, int cols, const uint8_t *H, const uint8_t *s, const double *L,
                   const double *prior, int order, int exact, uint8_t *e);
/* Cost of setting a bit whose prior LLR is lambda: round(64 ln(1 + e^lambda)). */
long oracle_osd_weight(double lambda);

/* Phase 2 (soft-information regularisation) alone: phat_i = alpha * mean of
 * pv over the views holding qubit i; lam_i = clamp(ln(1-phat_i) - ln phat_i).
 * view, pv: nviews x vsize.  phat, lam may be NULL. */
void oracle_aggregate(int n, int nviews, int vsize, const int32_t *view, const double *pv,
                      double alpha, double llr_clamp, double *phat, double *lam);

/* Plain BP on a dense 0/1 matrix (rows x cols): the building block of both
 * stages, exported for the pins.  Returns iterations run; *conv set. */
int  oracle_bp(int rows, int cols, const uint8_t *H, const uint8_t *s, const double *lam,
               const oracle_params *p, int max_iter, double *L, uint8_t *e, int *conv);

/* Standalone global BP with channel priors (no local phase), followed by
 * OSD-0 on H_t where BP misses the syndrome when p->global_osd is set
 * (converged = 2 then; a syndrome outside the column space keeps BP's
 * estimate). */
int  oracle_global_bp(const oracle_code *c, int type, const oracle_params *p, int shots,
                      const uint64_t *synd, int synd_words, const double *prior,
                      uint64_t *ehat, int ehat_words, double *post, int32_t *stats);

/* 1 if the residual (packed, H r = 0 assumed) is a non-trivial logical.
 * route 0: pairing with the logical basis; route 1: rowspace rank test. */
int  oracle_logical_failure(const oracle_code *c, int type, const uint64_t *residual, int route);

#ifdef __cplusplus
}
#endif
#endif
