/*
 * liblead -- LEAD decoding of quantum Tanner codes on AMD Instinct MI355X
 * (gfx950).  C ABI: plain pointers and sizes only.
 *
 * The method is LEAD (arXiv 2605.17796): project the syndrome onto the local
 * views of the vertices of the left-right Cayley complex, decode every local
 * view in parallel, aggregate the local soft outputs with the
 * alpha-regularisation, and run the global decoder with that prior
 * (Algorithm 1).  Both the local and the global decoder here are flooding
 * min-sum belief propagation.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  * Bit packing: bit i of a packed row is bit (i % 64) of 64-bit word i / 64.
 *  * Check types: LEAD_CHECK_Z are the Z-type generators C_A (x) C_B on the
 *    vertex set V0 and detect X errors; LEAD_CHECK_X are the X-type
 *    generators C_A^perp (x) C_B^perp on V1 and detect Z errors (Sec. II-B).
 *  * Numbering: check (g, rho) of type t is global check g * r_t + rho, where
 *    rho = rho_A * k_B + rho_B enumerates the reduced-echelon bases of the
 *    two local codes (their duals for X checks); local variable (i, j) of a
 *    view is i * Delta + j, i indexing A and j indexing B (Appendix A,
 *    eq. (product) is this layout).  Qubit ids rank the squares by their
 *    lexicographically smallest V0 description (g, i, j).
 *  * Status codes: every call returns lead_status; on failure
 *    lead_last_error() returns a message (thread-local, valid until the next
 *    call on the same thread).
 *  * Device pointers are HIP device addresses (for example the data_ptr of a
 *    torch tensor on the GPU); `stream` is a hipStream_t (NULL = the default
 *    stream).  Device work is enqueued asynchronously on that stream and the
 *    call returns without waiting; device faults surface on a later call.
 *  * Ownership: callers own every buffer they pass.  Code objects own host
 *    tables; decoders own their device tables and workspace.  A code may be
 *    shared between threads; a decoder must be used by one host thread at a
 *    time and must outlive the device work it enqueued.
 */
#ifndef LEAD_H
#define LEAD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LEAD_OK = 0,
    LEAD_E_ARG = -1,          /* NULL pointer, size out of range, bad enum      */
    LEAD_E_GROUP = -2,        /* table is not a group                           */
    LEAD_E_SYMMETRY = -3,     /* A or B not inverse-closed, repeated, identity  */
    LEAD_E_TNC = -4,          /* Total No-Conjugacy condition fails             */
    LEAD_E_LOCALCODE = -5,    /* local code rank/distance, or CSS fails         */
    LEAD_E_NOMEM = -6,        /* host or device allocation failed               */
    LEAD_E_DEVICE = -7,       /* HIP runtime error (message has the HIP string) */
    LEAD_E_CAPACITY = -8,     /* batch larger than the decoder was sized for    */
    LEAD_E_UNSUPPORTED = -9,  /* shape the compiled kernels do not cover        */
    LEAD_E_CLOSED = -10       /* the server no longer accepts requests          */
} lead_status;

typedef enum { LEAD_CHECK_Z = 0, LEAD_CHECK_X = 1 } lead_check_type;
typedef enum { LEAD_PRIOR_PER_SHOT = 0, LEAD_PRIOR_SHARED = 1, LEAD_PRIOR_FULL = 2 } lead_prior_mode;
/* FULL: Algorithm 1 (Phases 1-3).  LOCAL: Phases 1-2 only (lambda' out).
 * GLOBAL: global BP alone with the channel priors as its prior, no local
 * phase: the standard single-stage decoder LEAD is compared against. */
typedef enum { LEAD_STAGE_FULL = 0, LEAD_STAGE_LOCAL = 1, LEAD_STAGE_GLOBAL = 2 } lead_stage;
/* BP flavour of both stages: flooding min-sum with scale ms_scale, or
 * flooding sum-product (no scale). */
typedef enum { LEAD_BP_MINSUM = 0, LEAD_BP_SUMPRODUCT = 1 } lead_bp;

typedef struct lead_code lead_code;
typedef struct lead_decoder lead_decoder;

const char *lead_last_error(void);

/* ------------------------------------------------------------------------ */
/* Code construction (host only; no device work).  Sec. II-A, II-B.          */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t order;            /* |G|, 1..65535                                   */
    const uint16_t *mul;      /* order*order, mul[g*order + h] = index of g*h    */
    int32_t delta;            /* |A| = |B|, 2..8                                 */
    const int32_t *A;         /* delta element indices; order = local coords     */
    const int32_t *B;
    int32_t kA, kB;           /* local code dimensions, 1..delta-1               */
    const uint64_t *GA;       /* kA generator rows of C_A, bit c = coordinate c  */
    const uint64_t *GB;       /* kB generator rows of C_B                        */
} lead_code_desc;

typedef struct {
    int32_t order, delta, n;  /* n = order * delta^2 / 2 qubits                  */
    int32_t r[2];             /* checks per vertex, indexed by lead_check_type   */
    int32_t m[2];             /* global checks = order * r[t]                    */
    int32_t rank[2];          /* GF(2) rank of H_Z, H_X                          */
    int32_t k;                /* logical qubits n - rank[0] - rank[1]            */
    int32_t eloc[2];          /* edges of one local Tanner graph                 */
} lead_code_info;

/* Validates (group axioms, A = A^-1, B = B^-1, identity excluded, TNC,
 * full-rank local codes with distance >= 2 and dual distance >= 2, CSS) and
 * builds the code.  The descriptor's arrays are copied. */
lead_status lead_code_create(const lead_code_desc *desc, lead_code **out);
lead_status lead_code_query(const lead_code *code, lead_code_info *out);
/* Host CSR of H_t: indptr has m[t]+1 entries, indices one per edge (row
 * order, columns ascending).  Pass indices = NULL to get only indptr. */
lead_status lead_code_get_H(const lead_code *code, lead_check_type t, int32_t *indptr, int32_t *indices);
/* Host view table of type t: order x delta^2 qubit ids (V0 for Z, V1 for X). */
lead_status lead_code_get_views(const lead_code *code, lead_check_type t, int32_t *view);
/* Compiles, for gfx950 and without touching a GPU, the decoding kernels
 * specialised to the local check structure of type t (its check masks and
 * the local position map of the two occurrences of a qubit, Sec. II-B), and
 * caches the code objects for the rest of the process and on disk (the
 * directory $LEAD_JIT_CACHE, "off" to disable, else _build/jit beside the
 * library; a later process with the same compiler, library headers and code
 * loads them instead of compiling) (the min-sum forms,
 * and the sum-product form where views have at most 192 local edges);
 * lead_decoder_create does the same on first use and then loads them.  LEAD_E_UNSUPPORTED (with the
 * reason in lead_last_error) when the code has no position map or the
 * run-time compiler is unavailable; decoders then use the precompiled
 * kernels, with identical results. */
lead_status lead_code_specialize(const lead_code *code, lead_check_type t);
void lead_code_destroy(lead_code *code);

/* ------------------------------------------------------------------------ */
/* Decoding (Algorithm 1).                                                    */
/* ------------------------------------------------------------------------ */

typedef struct {
    float alpha;              /* regularisation scale, (0, 1]  (Alg. 1 Phase 2)   */
    float ms_scale;           /* min-sum scale beta, (0, 1]                       */
    int32_t max_iter_local;   /* local BP iteration cap, 1..1000                  */
    int32_t max_iter_global;  /* global BP iteration cap, 1..1000                 */
    float llr_clamp;          /* |mu|, |L|, |lambda'| clamped to this, > 0        */
    int32_t early_exit;       /* 1: stop a BP run at the first H e = s            */
    int32_t stage;            /* lead_stage: FULL, LOCAL or GLOBAL                */
    int32_t boost;            /* 1: Phase-1 confidence boost (Alg. 1)             */
    int32_t fixed_point_stop; /* 1: end a BP run whose messages reproduce
                                 themselves bit for bit (every later iteration
                                 would repeat it; local runs are tested at
                                 even iterations, global runs at every one);
                                 results and reported
                                 iteration counts are identical to running to
                                 the cap.  2: local BP runs only (global BP
                                 then runs kernels without the per-message
                                 comparison, and reports global_fixed_iter =
                                 0).  0: off.  Other values: LEAD_E_ARG     */
    int32_t local_post;       /* 1: a local BP run that ends with H_v e_v != s_v
                                 is followed by OSD on its view (ordered
                                 statistics decoding: variables ranked by
                                 posterior LLR, most likely in error first,
                                 ties in position order; the solution
                                 supported on the first independent columns,
                                 or with osd_order > 0 the sweep's cheapest
                                 candidate).  The view then counts as converged
                                 and the confidence boost applies to its
                                 estimate.  Kernels compiled for the code
                                 only (not plain, not stage GLOBAL).  0: none */
    int32_t bp;               /* lead_bp.  Sum-product runs on the kernels
                                 compiled for the code with one register per
                                 message (views of at most 192 local edges),
                                 in lead_decode, batches and the server,
                                 stage GLOBAL included; lead_decode_plain is
                                 min-sum only (LEAD_E_UNSUPPORTED)            */
    int32_t global_post;      /* 1: a shot whose global BP ends with H e != s
                                 is followed by OSD-0 on H_t with the global
                                 posteriors as reliabilities (ranked as for
                                 local_post, round(64 L) ascending, ties in
                                 qubit order); it then reports converged = 2
                                 and its estimate is the OSD-0 solution.  A
                                 syndrome outside the column space of H_t
                                 keeps BP's estimate and report.  Stages FULL
                                 and GLOBAL, kernels compiled for the code
                                 (lead_schedule.global_osd_form picks the
                                 kernel; LEAD_E_UNSUPPORTED from
                                 lead_decode_plain).  0: none                  */
    int32_t osd_order;        /* order lambda of the OSDs of local_post and
                                 global_post, 0..8 (needs one of them).
                                 0: OSD-0.  lambda >= 1: combination sweep
                                 (the paper runs its global BP-OSD in this
                                 mode at order 3): candidates are the OSD-0
                                 solution, the solution with one bit set on
                                 each column outside the information set, and
                                 the one with two bits set on each pair among
                                 the first lambda of those columns (rank
                                 order); the estimate is the first candidate
                                 of least cost sum over set bits of
                                 round(64 ln(1 + e^{lambda_j})), lambda the
                                 decoder's prior: the view's channel LLRs
                                 locally; lambda' globally (the channel prior
                                 in stage GLOBAL).                            */
} lead_params;

/* Per-shot statistics (32 bytes). */
typedef struct {
    int32_t converged;              /* 1: global BP reached H e = s; 2: reached by
                                       OSD-0 after it (global_post); 0 otherwise,
                                       and in the LOCAL stage                    */
    int32_t global_iters;           /* global BP iterations run                    */
    int32_t local_iters_sum;        /* sum over vertices of local iterations       */
    int32_t local_iters_max;
    int32_t local_converged_views;  /* vertices whose local BP reached H_v e_v = s_v */
    int32_t local_fixed_views;      /* local runs ended at a message fixed point   */
    int32_t global_fixed_iter;      /* iteration at which global BP reached a fixed
                                       point (0: it did not)                       */
    int32_t local_osd_views;        /* vertices resolved by OSD-0 (local_post = 1) */
} lead_shot_stats;

/* Creates a decoder for the checks of type `t` and uploads the device tables
 * of the code to the current HIP device.  `max_shots` bounds the batch size
 * of every later call.  The decoder allocates a workspace for min(max_shots,
 * W) shots, W = max(32768, the shots whose local posteriors (order * delta^2
 * floats per shot) and flags fit in 1 GiB); larger batches are decoded chunk
 * by chunk on the same stream.  lead_decode_plain
 * allocates its per-round state (for max_shots shots) on first use. */
lead_status lead_decoder_create(const lead_code *code, lead_check_type t, const lead_params *params,
                                int64_t max_shots, lead_decoder **out);
lead_status lead_decoder_set_params(lead_decoder *dec, const lead_params *params);
void lead_decoder_destroy(lead_decoder *dec);

/* LEAD decode of `shots` syndromes: Phase 1 (local BP on each vertex view),
 * Phase 2 (aggregation) and, in the FULL stage, Phase 3 (global BP).  The
 * schedule (lead_decoder_set_schedule) picks the kernels: by default a
 * work-queue kernel for Phase 1 and a per-shot kernel for Phases 2-3, both
 * compiled for the decoder's code; or one fused per-shot kernel.  Every
 * schedule gives bit-identical outputs.  In the GLOBAL stage only the global
 * BP runs (on the per-shot kernel compiled for the code, or the fused
 * precompiled kernel), with prior lambda' = the channel LLR of each qubit.
 *   d_synd      shots x synd_words packed syndromes, synd_words >= ceil(m/64)
 *   d_prior     channel LLRs ln((1-p)/p): PER_SHOT: shots floats; SHARED: n
 *               floats; FULL: shots x n floats
 *   d_ehat      shots x ehat_words packed estimates (FULL stage; may be NULL
 *               in the LOCAL stage), ehat_words >= ceil(n/64)
 *   d_post      shots x n posterior LLRs of global BP, or NULL
 *   d_prior_llr shots x n regularised priors lambda' (Phase 2 output; the
 *               channel LLRs in the GLOBAL stage), or NULL; required in the
 *               LOCAL stage
 *   d_stats     shots lead_shot_stats, or NULL
 * A shot that does not converge is not an error: its estimate and
 * posteriors are still written and stats.converged is 0. */
lead_status lead_decode(lead_decoder *dec, int64_t shots, const uint64_t *d_synd, int64_t synd_words,
                        const float *d_prior, lead_prior_mode mode, uint64_t *d_ehat, int64_t ehat_words,
                        float *d_post, float *d_prior_llr, lead_shot_stats *d_stats, void *stream);

/* The same decode for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): outputs
 * are bit-identical to lead_decode's, from the same kernels and launches,
 * but every buffer the kernels need beyond the caller's inputs and outputs
 * (local posteriors, view flags, queue counters, the local OSD list and,
 * with global_post, the global OSD's buffers for outputs passed as NULL) is
 * taken from a static device array of LEAD_NOALLOC_SCRATCH_BYTES bytes that
 * each GPU holds until the process ends.  The call allocates nothing (no
 * hipMalloc, hipFree, event or stream creation) and records no phase
 * timing; the device's array address is looked up once, on its first call
 * on that device, which must be the decoder's device (LEAD_E_ARG
 * otherwise).  Shots are decoded in one pass through the scratch, so a call
 * takes at most (LEAD_NOALLOC_SCRATCH_BYTES - 2048) / b shots, b = 4 *
 * order * delta^2 + 8 * order bytes per shot (plus 4n, 32 and 4n with
 * global_post for the post, stats and, with osd_order > 0, lambda' outputs
 * passed as NULL; the global OSD with the matrix in device memory also
 * takes its matrix slots from the scratch, as many as fit beside the batch,
 * at least one): about 7 300 A5 shots or 1 500 PSL(2,7) shots.  Larger
 * batches return LEAD_E_CAPACITY with the limit in lead_last_error and
 * enqueue nothing.  Every call on one GPU uses that GPU's one array, which
 * keeps the last call's contents (the queue counters are cleared by a fill
 * kernel at the start of each call): calls whose device work overlaps on one
 * GPU (other host threads, or other streams not ordered with this one) race
 * and give undefined results.  Arguments and the other errors are as for
 * lead_decode. */
#define LEAD_NOALLOC_SCRATCH_BYTES ((int64_t)64 << 20)
lead_status lead_decode_noalloc(lead_decoder *dec, int64_t shots, const uint64_t *d_synd, int64_t synd_words,
                                const float *d_prior, lead_prior_mode mode, uint64_t *d_ehat, int64_t ehat_words,
                                float *d_post, float *d_prior_llr, lead_shot_stats *d_stats, void *stream);

/* The same decode as a plain sequence of launches: the Phase 1 launch, then
 * one launch per global BP round (Phases 2-3 of that round, the per-view sums
 * and check state kept in device memory between launches; the first round
 * also forms lambda'), a host-visible count of shots still running after
 * every round (the call synchronises `stream` once per round), and a last
 * launch ending the shots that ran to the cap.  On the kernels compiled for
 * the code (the default schedule) every parameter is supported, sum-product
 * and OSD included; with the precompiled kernels (specialized = 0) min-sum
 * without OSD only (LEAD_E_UNSUPPORTED otherwise).  The per-round state is
 * allocated on first use (about 31 KB per A5 shot, for min(max_shots,
 * workspace) shots).  Outputs are identical to lead_decode's. */
lead_status lead_decode_plain(lead_decoder *dec, int64_t shots, const uint64_t *d_synd, int64_t synd_words,
                              const float *d_prior, lead_prior_mode mode, uint64_t *d_ehat,
                              int64_t ehat_words, float *d_post, float *d_prior_llr,
                              lead_shot_stats *d_stats, void *stream);

/* s = H_t e for `shots` packed error rows (device pointers). */
lead_status lead_syndrome(const lead_decoder *dec, int64_t shots, const uint64_t *d_err, int64_t err_words,
                          uint64_t *d_synd, int64_t synd_words, void *stream);

/* Launch geometry of lead_decode.  Results never depend on it (every shot's
 * arithmetic is the same under every schedule); zeros select the library's
 * defaults. */
typedef struct {
    int32_t shots_per_workgroup;  /* shots per workgroup of the per-shot kernel     */
    int32_t fused;                /* 1: Phase 1 runs inside the per-shot kernel (a
                                     wave waits for its slowest view); 0: Phase 1
                                     runs in a work-queue kernel first           */
    int32_t local_chunk;          /* queue items a wave takes at a time            */
    int32_t local_waves;          /* waves of the work-queue kernel                 */
    int32_t specialized;          /* (3 with sum-product, whatever is asked)
                                     the work-queue form (fused = 0) runs the
                                     kernels compiled for this code (see
                                     lead_code_specialize; they pick their own
                                     workgroup shape): 1 with the compressed
                                     min-sum check state, 2 with one register
                                     per message (views of at most 192 edges;
                                     above 128 edges the Phases 2-3 kernel
                                     keeps the compressed state on the
                                     highest-degree checks, same outputs);
                                     0: the precompiled kernels.  Reads back as
                                     the form in use (a form that was not
                                     compiled is replaced by the other). The
                                     default is 2 where compiled, else 1.       */
    int32_t chunk_shots;          /* shots per launch of the work-queue form
                                     (at most the workspace); 0: the workspace.
                                     Larger launches leave fewer kernel tails. */
    int32_t global_osd_form;      /* kernel of the global OSD (global_post):
                                     1: the rows of [H_t | s] in registers
                                     (codes with ceil(m/256) * ceil(n/64) <= 64);
                                     2: the matrix in device memory, one slot
                                     of (ceil(n/64) + 1) * m words per
                                     workgroup (any code up to 32768 checks and
                                     65535 qubits; the decoder allocates a slot
                                     per compute unit); 0: 1 where it fits, else
                                     2.  Same outputs.  Reads back as the form
                                     in use (2 where 1 does not fit). */
    int32_t global_tiles;         /* Phases 2-3 kernel of the compiled min-sum
                                     forms for codes of more than 64 views
                                     (views spanning several waves):
                                     1: persistent workgroups of 512 lanes
                                     (eight waves, two per SIMD), each holding
                                     floor(512 / views) shots and taking the
                                     next shot from a device counter when one
                                     ends (compiled where that many shots fit
                                     in LDS, at least two); 2: one workgroup
                                     of whole waves per shot.  0: 1 where
                                     compiled.  Same outputs bit for bit.
                                     Reads back as the kernel in use (0 for
                                     codes of at most 64 views, which run
                                     whole shots in one wave). */
} lead_schedule;
lead_status lead_decoder_set_schedule(lead_decoder *dec, const lead_schedule *schedule);
lead_status lead_decoder_get_schedule(const lead_decoder *dec, lead_schedule *schedule);

/* Device time per phase of the work-queue form (fused = 0).  While timing
 * is on, lead_decode brackets each Phase 1 launch and each Phases 2-3 launch
 * with HIP events on its stream (except while that stream is being captured
 * into a graph).  lead_decoder_phase_times waits for the last recorded event
 * and returns the milliseconds and launch counts summed since timing was
 * last switched on; switching it on clears the sums. */
typedef struct {
    double local_ms;              /* Phase 1 (work-queue local BP kernel)        */
    double global_ms;             /* Phases 2-3 (aggregation and global BP)      */
    int64_t local_launches, global_launches;
} lead_phase_times;
lead_status lead_decoder_time_phases(lead_decoder *dec, int32_t enable);
lead_status lead_decoder_phase_times(lead_decoder *dec, lead_phase_times *out);

/* Times candidate schedules (fused / work-queue Phase 1, shots per
 * workgroup, queue chunk) on the caller's batch (at most 16384 of its shots)
 * and keeps the fastest; `best` (may be NULL) receives it.  Synchronises
 * `stream`; allocates temporary output buffers for the trials. */
lead_status lead_decoder_autotune(lead_decoder *dec, int64_t shots, const uint64_t *d_synd, int64_t synd_words,
                                  const float *d_prior, lead_prior_mode mode, void *stream, lead_schedule *best);

/* ------------------------------------------------------------------------ */
/* Batched decoding: several decode requests, possibly of different codes,   */
/* check types, shot counts and priors, in one call.                         */
/* ------------------------------------------------------------------------ */

typedef struct {
    lead_decoder *decoder;        /* decoder of this item's code and check type  */
    int64_t shots;
    const uint64_t *d_synd;       /* as for lead_decode                          */
    int64_t synd_words;
    const float *d_prior;
    lead_prior_mode mode;
    uint64_t *d_ehat;
    int64_t ehat_words;
    float *d_post;                /* nullable                                    */
    float *d_prior_llr;           /* nullable (required in the LOCAL stage)      */
    lead_shot_stats *d_stats;     /* nullable                                    */
} lead_batch_item;

/* Decodes every item with lead_decode semantics.  Items of different
 * decoders run concurrently on library streams forked from `stream` and
 * joined back to it; items sharing a decoder run in order (they share its
 * workspace).  Returns after enqueueing; completion is ordered on `stream`. */
lead_status lead_batch_decode(const lead_batch_item *items, int32_t n_items, void *stream);

/* The same work captured once into a HIP graph and replayed by
 * lead_batch_graph_launch (one launch for the whole batch).  The graph
 * reads and writes the buffers named in `items` at capture time; callers
 * refill those buffers between launches.  A graph must not be launched
 * concurrently with other work that uses the same decoders. */
typedef struct lead_batch_graph lead_batch_graph;
lead_status lead_batch_graph_create(const lead_batch_item *items, int32_t n_items, void *stream,
                                    lead_batch_graph **out);
lead_status lead_batch_graph_launch(lead_batch_graph *graph, void *stream);
void lead_batch_graph_destroy(lead_batch_graph *graph);

/* Fused batch: the requests of up to 8 items (codes of different sizes,
 * check types, shot counts, priors) decoded by one persistent Phase 1
 * launch and one Phases 2-3 launch shared by all of them, captured as a
 * hipGraph and replayed by lead_batch_fused_launch.
 *   Phase 1: 64-lane waves, as many as the device holds; every wave drains
 *   the local-BP work queue of item 0 (its lanes refilled one (shot, vertex)
 *   view at a time as their runs end, Alg. 1 Phase 1), then moves on to
 *   item 1's queue, and so on, so no lane waits at the end of one item's
 *   work while another's remains.
 *   Phases 2-3: one grid holding every item's per-shot blocks (a workgroup
 *   of the largest per-shot block size runs one block of a large code, or
 *   several of a small one, each wave-aligned with its own LDS); the branch
 *   on the item is uniform per workgroup.  Items whose decoders run the
 *   persistent Phases 2-3 kernel (lead_schedule.global_tiles, codes of more
 *   than 64 views) get persistent 512-lane workgroups of their own in the
 *   grid, and the other items' blocks then run eight waves to a workgroup
 *   (where a per-shot block of another item does not divide 512 lanes, or
 *   needs the whole register file, no item uses the persistent kernel).
 * The phases are ordered by the stream (no workgroup waits on another).
 * Outputs are those of lead_decode on each item bit for bit.  Every item's
 * decoder must run the kernels compiled for its code (schedule specialized
 * > 0, not fused) without OSD post-processing (LEAD_E_UNSUPPORTED
 * otherwise); the kernels of a batch's composition (codes, check types,
 * forms, prior modes) are compiled on first use, or ahead of time with
 * lead_batch_fused_specialize.  The batch owns its own workspace (local
 * posteriors and flags for every item's shots; several items may share a
 * decoder) and reads and writes the buffers named in `items` at creation:
 * callers refill those between launches.  Work on other streams that uses
 * the same output buffers must be ordered by the caller. */
typedef struct lead_batch_fused lead_batch_fused;
lead_status lead_batch_fused_create(const lead_batch_item *items, int32_t n_items, lead_batch_fused **out);
lead_status lead_batch_fused_launch(lead_batch_fused *fused, void *stream);
void lead_batch_fused_destroy(lead_batch_fused *fused);
/* Compiles (no GPU) the fused kernels of a batch composition: item i of
 * code codes[i], check type types[i], kernel form forms[i] (as
 * lead_schedule.specialized: 1 compressed, 2 one register per message, 3
 * sum-product) and prior mode modes[i]; cached in the process and on disk
 * like lead_code_specialize. */
lead_status lead_batch_fused_specialize(const lead_code *const *codes, const lead_check_type *types,
                                        const int32_t *forms, const lead_prior_mode *modes, int32_t n);

/* ------------------------------------------------------------------------ */
/* Serving: a request loop with continuous batching.                          */
/* ------------------------------------------------------------------------ */

/* A server decodes requests (host syndrome batches with per-shot channel
 * LLRs) for a fixed set of decoders.  A worker thread packs waiting requests
 * of one decoder, in arrival order, into launch slots of up to
 * `max_batch_shots` shots (splitting larger requests); each slot has its own
 * decoder copy (device-resident code tables and workspace), device buffers,
 * pinned staging and stream, and runs copy-in, decode and copy-out.  Requests
 * that arrive while slots are busy are admitted into the next slot that
 * frees, so their work overlaps the work already on the device.
 *
 * Admission by device memory: a slot's device memory is counted as its
 * decoder copy's actual allocation plus its input/output buffers, and the
 * slots together stay within `mem_budget_bytes`.  One slot per decoder is
 * created with the server (LEAD_E_CAPACITY if the budget cannot hold them);
 * further slots are created while a decoder has waiting shots and no idle
 * slot, up to `max_slots_per_decoder` and within the budget; when the budget
 * is full, an idle extra slot of a decoder with nothing waiting is freed to
 * make room.  Waiting requests hold no device memory.
 *
 * Back-pressure: at most `max_pending_shots` shots may be pending (submitted
 * and not yet released by lead_server_result); a submit beyond that returns
 * LEAD_E_CAPACITY and queues nothing (the caller retries once results have
 * been collected), and a request larger than the limit on its own is
 * refused with LEAD_E_CAPACITY as oversize. */
typedef struct lead_server lead_server;

typedef struct {
    int64_t mem_budget_bytes;       /* device memory for slots (0 = 1 GiB)          */
    int32_t max_batch_shots;        /* shots per launch slot (0 = 4096)             */
    int32_t max_slots_per_decoder;  /* (0 = 4)                                      */
    int32_t return_posteriors;      /* 1: keep L_post of every shot for the result */
    int32_t reserved;
    int64_t max_pending_shots;      /* submitted, unreleased shots (0 = 2^24)       */
} lead_server_config;

typedef struct {
    int64_t submitted, completed, shots_completed, launches;
    int32_t slots;                  /* launch slots in existence                    */
    int32_t slots_created;          /* slots created since the server started       */
    int64_t slot_bytes;             /* device bytes of the slots in existence       */
    int64_t evictions;              /* idle slots freed to make room for another    */
    int64_t refused;                /* submits refused (pending limit, oversize)    */
    int64_t pending_shots;          /* submitted shots not yet released             */
} lead_server_stats;

/* Decoders are used as templates: the server clones them (parameters and
 * schedule included); the caller keeps ownership of the originals. */
lead_status lead_server_create(lead_decoder *const *decoders, int32_t n_decoders, const lead_server_config *config,
                               lead_server **out);
/* Copies the request's inputs (h_synd: shots x synd_words, h_prior: shots
 * LLRs, one per shot) and queues it; *ticket identifies it.  Thread-safe.
 * LEAD_E_CAPACITY (nothing queued) when the pending-shot limit would be
 * exceeded or the request alone exceeds it; LEAD_E_CLOSED after
 * lead_server_close. */
lead_status lead_server_submit(lead_server *server, int32_t decoder_index, int64_t shots, const uint64_t *h_synd,
                               int64_t synd_words, const float *h_prior, int64_t *ticket);
/* *done = 1 once every shot of the request is decoded (0 otherwise). */
lead_status lead_server_poll(lead_server *server, int64_t ticket, int32_t *done);
/* Blocks until the request is decoded. */
lead_status lead_server_wait(lead_server *server, int64_t ticket);
/* Copies the results of a finished request (h_ehat: shots x ceil(n/64);
 * h_post: shots x n, only with return_posteriors; h_stats: shots; any may be
 * NULL), reports its submit and completion times (nanoseconds of the
 * library's steady clock; may be NULL), and releases it. */
lead_status lead_server_result(lead_server *server, int64_t ticket, uint64_t *h_ehat, float *h_post,
                               lead_shot_stats *h_stats, int64_t *submit_ns, int64_t *done_ns);
lead_status lead_server_get_stats(lead_server *server, lead_server_stats *out);
/* Stops accepting requests (later submits return LEAD_E_CLOSED) and blocks
 * until every request already submitted is decoded; their results stay
 * available to lead_server_result.  LEAD_E_DEVICE if a launch failed. */
lead_status lead_server_close(lead_server *server);
/* Current value of the clock used for request timestamps. */
int64_t lead_server_clock_ns(void);
/* Finishes the work on the device, stops the worker, frees everything;
 * unreleased requests are dropped. */
void lead_server_destroy(lead_server *server);

#ifdef __cplusplus
}
#endif
#endif
