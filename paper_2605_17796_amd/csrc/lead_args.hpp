// Argument blocks passed by value to the decoding kernels.  The run-time
// compiler sees this header too; it has no <cstdint>, and its own fixed-width
// types live in __hip_internal.
#pragma once
#ifdef __HIPCC_RTC__
using __hip_internal::int32_t;
using __hip_internal::int64_t;
using __hip_internal::uint32_t;
using __hip_internal::uint64_t;
#else
#include <cstdint>
#endif

namespace lead {

constexpr int kMaxChecks = 16;       // checks per vertex covered by the kernels
constexpr int kMaxOsdOrder = 8;      // largest order of the OSD combination sweep
constexpr int kMaxOsdOrderLocal = kMaxOsdOrder;
// Lanes of a workgroup of the persistent Phases 2-3 kernel for views that
// span several waves (eight waves: two per SIMD).
constexpr int kTileWG = 512;

// Per-shot statistics as the kernels write them (the layout of the public
// lead_shot_stats).
struct ShotStats {
    int32_t converged, global_iters, local_iters_sum, local_iters_max, local_converged_views, local_fixed_views,
        global_fixed_iter, local_osd_views;
};

// Everything a decode launch needs, passed by value in the kernel argument
// segment (so the check masks live in scalar registers).
struct DecodeArgs {
    const uint64_t *synd;
    const float *prior;
    uint64_t *ehat;
    float *post;
    float *lam_out;
    void *stats;               // ShotStats[shots]
    const int32_t *view;       // [N][D2] qubit ids
    const uint32_t *own;       // [N][own_max] packed j | j' << 8 | v' << 16
    int64_t shots;
    int64_t synd_words, ehat_words;
    int32_t prior_mode, spw, N, n, r, own_max;
    float alpha, beta, clampv;
    int32_t Tl, Tg, early_exit, stage, boost;
    int32_t fixed_stop;        // fixed-point exit of local BP runs (Phase 1)
    int32_t fixed_stop_g;      // ... of global BP runs (Phase 3, global BP alone)
    int32_t global_only;       // no Phase 1; lambda' = the channel prior
    int32_t local_osd;         // OSD-0 after local BP runs that miss the local syndrome
    int32_t osd_order;         // order of the OSDs' combination sweep (0: OSD-0)
    uint64_t mask[kMaxChecks];
};

// Workspace of the split path (Phase 1 in its own work-queue kernel).
struct LocalArgs {
    float *Lv;                 // [shots][N][D2] clamped local posteriors
    uint32_t *vflag;           // [shots][N] iterations | converged << 16 | fixed point << 17
                               //            | resolved by OSD-0 << 18
    int64_t *counter;          // [0] work-queue head, [1] entries of osd_list,
                               // [3] next shot of the persistent Phases 2-3 kernel
    uint32_t *osd_list;        // items whose local BP missed the local syndrome (local OSD-0 pending)
    int64_t items;             // shots * N
    int32_t chunk;             // items a wave takes at a time
    int32_t waves;             // waves launched
};

// Extra tables of the Phase 2-3 kernel compiled for one code: for view v and
// local position j, the view holding the other occurrence of the qubit
// (pv[v * ceil(D2/2) + j/2], 16 bits per position, even j in the low half),
// and for views whose qubits at fixed points of the position map are owned
// by the view, the owned positions as a bit mask (fown[v]).
struct SpecArgs {
    const uint32_t *pv;
    const uint64_t *fown;
};

// Tables of the global OSD-0 kernel: H_t as row lists (CSR, rows g*r + rho,
// columns ascending).
struct OsdArgs {
    const int32_t *rptr;
    const int32_t *ridx;
};

// State of the plain per-round form of the Phases 2-3 kernel compiled for a
// code: one launch per global round, the per-view sums and check state kept
// in device memory between launches ([shot][word][view] floats, so a wave's
// accesses coalesce), a per-shot flag set when the shot's run has ended, and
// a count of the shots still running after the round (read by the host).
// round = 1 .. Tg runs that round; round = Tg + 1 ends the shots that ran to
// the cap.
struct PlainArgs {
    float *S;                  // [shot][D2][N] variable sums
    float *st;                 // [shot][words][N] check state
    int32_t *ended;            // [shot] 1 once the shot's outputs are written
    int32_t *active;           // shots still running after this round
    int32_t round;
};

// Arguments of the kernels fusing the decode requests of several codes into
// one launch per phase (lead_batch_fused_*): per request its decode
// arguments, workspace and partner tables, and for the Phases 2-3 kernel the
// first workgroup of each request's range of the grid (first[k] .. first[k+1]).
constexpr int kFusedMax = 8;
struct FusedItem {
    DecodeArgs a;
    LocalArgs w;
    SpecArgs x;
};
struct FusedArgs {
    FusedItem it[kFusedMax];
    int64_t first[kFusedMax + 1];
};

// Workspace of the global OSD kernel that keeps [H_t | s] in device memory
// (codes whose rows do not fit in registers): one matrix slot per
// workgroup, (ceil(n/64) + 1) x m words, word-major (word k of row r at
// k * m + r; the last word column holds s in bit 0), and the queue of
// shots the workgroups take one at a time.
struct OsdBigArgs {
    uint64_t *mat;
    int64_t *queue;            // [0] next shot (cleared before each launch)
};

}  // namespace lead
