// C ABI of liblead: code construction, decoder objects, decode entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "../../include/lead.h"
#include "code_build.hpp"
#include "lead_internal.hpp"
#include "lead_jit.hpp"
#include "lead_kernels.hpp"
#include "lead_scratch.hpp"

static_assert(sizeof(lead::ShotStats) == sizeof(lead_shot_stats), "ShotStats layout");
static_assert(offsetof(lead::ShotStats, global_fixed_iter) == offsetof(lead_shot_stats, global_fixed_iter),
              "ShotStats layout");

struct lead_code {
    lead::Code c;
};

struct lead_batch_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

struct lead_batch_fused {
    std::shared_ptr<const lead::jit::FusedKernels> k;
    lead::FusedArgs args{};
    int n = 0;
    int64_t local_waves = 0, global_wgs = 0;
    std::vector<void *> bufs;               // per request: local posteriors, view flags
    int64_t *counters = nullptr;            // 4 per request: queue head, local OSD list, -, next shot of
                                            // the persistent Phases 2-3 kernel
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

struct lead_decoder {
    lead::Code const *code = nullptr;
    std::shared_ptr<lead::Code> keep;       // decoders keep their own copy of the tables
    int type = 0;
    lead_params params{};
    int64_t max_shots = 0;
    int device = 0;
    int D = 0, N = 0, n = 0, r = 0, m = 0, own_max = 0, spw = 1;
    uint64_t mask[lead::kMaxChecks] = {};
    int32_t *d_view = nullptr;
    uint32_t *d_own = nullptr;
    // kernels compiled for this code's check structure, with their tables
    std::shared_ptr<const lead::jit::Kernels> spec;
    uint32_t *d_pv = nullptr;
    uint64_t *d_fown = nullptr;
    // global OSD-0: H_t as row lists, and posterior / statistics buffers for
    // calls that do not ask for them (ws_shots shots)
    int32_t *d_rptr = nullptr, *d_ridx = nullptr;
    float *d_gpost = nullptr, *d_glam = nullptr;
    lead_shot_stats *d_gstats = nullptr;
    // schedule and split-path workspace (for ws_shots shots)
    lead_schedule sched{};
    int64_t ws_shots = 0;
    int cus = 0;
    int waves_per_cu[2] = {4, 4};
    float *d_Lv = nullptr;
    uint32_t *d_vflag = nullptr;
    int64_t *d_counter = nullptr;          // [0] queue head, [1] local OSD list length,
                                           // [2] global OSD shot queue (matrix in HBM)
    uint64_t *d_osd_mat = nullptr;         // global OSD matrix slots (matrix in HBM)
    int osd_slots = 0;
    uint32_t *d_osd_list = nullptr;        // views pending local OSD-0 (ws_shots * N)
    // phase timing: event triples (before Phase 1, between, after Phases 2-3)
    bool timing = false;
    std::vector<std::array<hipEvent_t, 3>> tev;
    lead_phase_times tsum{};
    // per-round state of lead_decode_plain (allocated on first use): the
    // precompiled round kernel's, and the compiled round kernels' (sums,
    // check state, ended flags for plain_shots shots, running-shot count)
    float *d_S = nullptr, *d_cst = nullptr, *d_lamp = nullptr;
    int32_t *d_status = nullptr, *d_active = nullptr, *h_active = nullptr;
    float *d_pS = nullptr, *d_pst = nullptr;
    int32_t *d_pended = nullptr;
    int64_t *d_pactive = nullptr;
    int64_t plain_shots = 0;
};

namespace {

thread_local std::string g_err;

lead_status fail(lead_status s, const std::string &msg) {
    g_err = msg;
    return s;
}

lead_status hip_fail(hipError_t e, const char *what) {
    return fail(LEAD_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// Device buffers a decode launch works in beyond its inputs and outputs:
// the work-queue form's local posteriors, flags, queue counters and local
// OSD list, and the global OSD's posterior / statistics / prior buffers for
// calls that pass none; `shots` is how many shots they hold.
struct Workspace {
    float *Lv = nullptr;
    uint32_t *vflag = nullptr;
    int64_t *counter = nullptr;
    uint32_t *osd_list = nullptr;
    float *gpost = nullptr, *glam = nullptr;
    lead_shot_stats *gstats = nullptr;
    uint64_t *osd_mat = nullptr;   // global OSD matrix slots (matrix in HBM)
    int osd_slots = 0;
    int64_t shots = 0;
};

lead_status check_params(const lead_params *p) {
    if (!p) return fail(LEAD_E_ARG, "params is NULL");
    if (!(p->alpha > 0.f && p->alpha <= 1.f)) return fail(LEAD_E_ARG, "alpha must be in (0, 1]");
    if (!(p->ms_scale > 0.f && p->ms_scale <= 1.f)) return fail(LEAD_E_ARG, "ms_scale must be in (0, 1]");
    if (p->max_iter_local < 1 || p->max_iter_local > 1000 || p->max_iter_global < 1 || p->max_iter_global > 1000)
        return fail(LEAD_E_ARG, "iteration caps must be in 1..1000");
    if (!(p->llr_clamp > 0.f) || !std::isfinite(p->llr_clamp)) return fail(LEAD_E_ARG, "llr_clamp must be > 0");
    if (p->stage != LEAD_STAGE_FULL && p->stage != LEAD_STAGE_LOCAL && p->stage != LEAD_STAGE_GLOBAL)
        return fail(LEAD_E_ARG, "bad stage");
    if (p->bp != LEAD_BP_MINSUM && p->bp != LEAD_BP_SUMPRODUCT) return fail(LEAD_E_ARG, "bad bp");
    if (p->fixed_point_stop < 0 || p->fixed_point_stop > 2) return fail(LEAD_E_ARG, "fixed_point_stop must be 0, 1 or 2");
    if (p->local_post != 0 && p->local_post != 1) return fail(LEAD_E_ARG, "bad local_post");
    if (p->local_post && p->stage == LEAD_STAGE_GLOBAL)
        return fail(LEAD_E_UNSUPPORTED, "stage GLOBAL has no local phase to post-process");
    if (p->global_post != 0 && p->global_post != 1) return fail(LEAD_E_ARG, "bad global_post");
    if (p->global_post && p->stage == LEAD_STAGE_LOCAL)
        return fail(LEAD_E_UNSUPPORTED, "stage LOCAL has no global BP to post-process");
    if (p->osd_order < 0 || p->osd_order > lead::kMaxOsdOrder)
        return fail(LEAD_E_ARG, "osd_order must be in 0.." + std::to_string(lead::kMaxOsdOrder));
    if (p->osd_order > 0 && !p->global_post && !p->local_post)
        return fail(LEAD_E_ARG, "osd_order needs local_post or global_post");
    return LEAD_OK;
}

// Shots per launch of the work-queue form: at least kChunkShots, more while
// the Phase 1 workspace (local posteriors and flags) stays within
// kChunkBytes (fewer launches, so fewer kernel tails).
constexpr int64_t kChunkShots = 32768;
constexpr int64_t kChunkBytes = int64_t(1) << 30;

int default_spw(int N) { return std::max(1, 64 / N); }

bool use_spec(const lead_decoder *d) { return d->spec && d->sched.specialized && !d->sched.fused; }

bool sum_product(const lead_decoder *d) { return d->params.bp == LEAD_BP_SUMPRODUCT; }

// Sum-product and OSD-0 run only on the kernels compiled for the code.
bool needs_spec(const lead_decoder *d) { return sum_product(d) || d->params.local_post != 0; }

bool osd_kernels(const lead::jit::Kernels *k) {
    return k && ((k->osd && k->osd_cs) || (k->osd_big && k->osd_big_cs));
}

bool osd_ready(const lead_decoder *d) { return osd_kernels(d->spec.get()) && d->d_rptr; }

// The global OSD kernel in use keeps [H_t | s] in device memory (asked for,
// or the rows do not fit in registers).
bool osd_big(const lead_decoder *d) {
    const lead::jit::Kernels *k = d->spec.get();
    if (!k || !k->osd_big) return false;
    return d->sched.global_osd_form == 2 || !(k->osd && k->osd_cs);
}

// Posterior and statistics buffers of the global OSD-0 for calls that pass
// none, and the matrix slots of the kernel with the matrix in device memory
// (one per compute unit: the kernel's LDS admits one workgroup per CU);
// allocated when global_post is first set or that kernel is first chosen.
hipError_t ensure_osd_workspace(lead_decoder *d) {
    hipError_t e = hipSuccess;
    if (!d->d_gpost) e = hipMalloc(&d->d_gpost, sizeof(float) * (size_t)d->ws_shots * d->n);
    if (e == hipSuccess && !d->d_gstats) e = hipMalloc(&d->d_gstats, sizeof(lead_shot_stats) * (size_t)d->ws_shots);
    if (e == hipSuccess && !d->d_glam) e = hipMalloc(&d->d_glam, sizeof(float) * (size_t)d->ws_shots * d->n);
    if (e == hipSuccess && osd_big(d) && !d->d_osd_mat) {
        const int slots = std::max(1, d->cus);
        e = hipMalloc(&d->d_osd_mat, lead::jit::osd_big_slot_bytes(*d->code, d->type) * (size_t)slots);
        if (e == hipSuccess) d->osd_slots = slots;
    }
    return e;
}

// OSD on H_t for the shots of `a` that global BP left unresolved: with the
// rows in registers, one workgroup per shot (the others exit at once); with
// the matrix in device memory, one persistent workgroup per matrix slot
// taking unresolved shots from a queue.
hipError_t launch_osd(const lead_decoder *d, lead::DecodeArgs a, const Workspace &ws, hipStream_t s) {
    lead::OsdArgs o{d->d_rptr, d->d_ridx};
    if (osd_big(d)) {
        lead::OsdBigArgs b{ws.osd_mat, ws.counter + 2};
        hipError_t e = lead::launch_clear_i64(b.queue, 1, s);
        if (e != hipSuccess) return e;
        const int64_t grid = std::min<int64_t>(ws.osd_slots, a.shots);
        void *args[] = {&a, &o, &b};
        return hipModuleLaunchKernel(a.osd_order > 0 ? d->spec->osd_big_cs : d->spec->osd_big, (unsigned)grid, 1, 1,
                                     (unsigned)d->spec->osd_big_wg, 1, 1, 0, s, args, nullptr);
    }
    void *args[] = {&a, &o};
    return hipModuleLaunchKernel(a.osd_order > 0 ? d->spec->osd_cs : d->spec->osd, (unsigned)a.shots, 1, 1,
                                 (unsigned)d->spec->osd_wg, 1, 1, 0, s, args, nullptr);
}

// The specialised form a schedule asks for, or the one compiled when it
// asks for the other (0: precompiled kernels).  Sum-product has one form.
int spec_form(const lead_decoder *d, int want) {
    if (sum_product(d)) return d->spec && d->spec->has[2] ? lead::jit::kSumProduct : 0;
    if (!d->spec || want <= 0) return 0;
    if (want == lead::jit::kExplicit && d->spec->has[1]) return lead::jit::kExplicit;
    if (want == lead::jit::kCompressed && d->spec->has[0]) return lead::jit::kCompressed;
    return d->spec->best_form();
}

// Whether the Phases 2-3 kernel of form f + 1 is the persistent one
// (compiled for codes whose views span several waves, unless the schedule
// asks for one workgroup per shot).
bool use_tiles(const lead_decoder *d, int f) {
    return d->spec && f >= 0 && f < lead::jit::kForms && d->spec->tile[f] && d->sched.global_tiles != 2;
}

// LDS bytes of the Phases 2-3 kernel compiled for the code (form f + 1).
size_t spec_global_lds(const lead_decoder *d, int f) {
    const lead::jit::Kernels &k = *d->spec;
    const int D2 = d->D * d->D, ew32 = (d->n + 31) / 32;
    const bool lam_in_lds = f + 1 == lead::jit::kCompressed || (f + 1 == lead::jit::kExplicit && k.hybrid);
    const size_t lam_lds = lam_in_lds ? sizeof(float) * (size_t)k.lam_slots * k.wg : 0;
    return (k.bperm ? 0 : sizeof(float) * (size_t)D2 * k.wg) + lam_lds + sizeof(int) * (size_t)k.spw * 9 +
           sizeof(uint32_t) * (size_t)k.spw * ew32;   // 9: the kernel's per-shot flag stride
}

// Split-path launches with the kernels compiled for the decoder's code.
hipError_t launch_spec(const lead_decoder *d, lead::DecodeArgs a, lead::LocalArgs w, hipStream_t s,
                       std::array<hipEvent_t, 3> *ev) {
    const lead::jit::Kernels &k = *d->spec;
    const int f = d->sched.specialized - 1;
    hipError_t e = hipSuccess;
    if (a.global_only) {
        // global BP alone: no Phase 1
        if (ev) e = hipEventRecord((*ev)[0], s);
        if (e == hipSuccess && ev) e = hipEventRecord((*ev)[1], s);
    } else {
        e = lead::launch_reset_counter(w.counter, s);
        if (e == hipSuccess && ev) e = hipEventRecord((*ev)[0], s);
        if (e != hipSuccess) return e;
        void *largs[] = {&a, &w};
        e = hipModuleLaunchKernel(k.local[f][a.prior_mode == LEAD_PRIOR_PER_SHOT ? 0 : 1], (unsigned)w.waves, 1, 1,
                                  64, 1, 1, (unsigned)k.local_lds[f][a.prior_mode == LEAD_PRIOR_PER_SHOT ? 0 : 1], s,
                                  largs, nullptr);
        // local OSD-0 of the views the queue kernel listed (lanes stride over the list)
        if (e == hipSuccess && a.local_osd)
            e = hipModuleLaunchKernel(k.local_osd, (unsigned)(8 * d->cus), 1, 1, 64, 1, 1, 0, s, largs, nullptr);
        if (e == hipSuccess && ev) e = hipEventRecord((*ev)[1], s);
    }
    if (e != hipSuccess) return e;
    a.spw = k.spw;
    lead::SpecArgs x{d->d_pv, d->d_fown};
    void *gargs[] = {&a, &w, &x};
    if (use_tiles(d, f) && a.stage != LEAD_STAGE_LOCAL) {
        // persistent workgroups taking shots from w.counter[3] (cleared with
        // the queue counters before Phase 1, here when there is none)
        if (a.global_only) e = lead::launch_reset_counter(w.counter, s);
        const int64_t need = (a.shots + k.tile_shots - 1) / k.tile_shots;
        const int64_t grid = std::max<int64_t>(1, std::min<int64_t>(need, d->cus));
        // (the kernel without the fixed-point test when global BP runs without it)
        hipFunction_t fn = !a.fixed_stop_g && k.tile_nf[f] ? k.tile_nf[f] : k.tile[f];
        if (e == hipSuccess)
            e = hipModuleLaunchKernel(fn, (unsigned)grid, 1, 1, (unsigned)lead::kTileWG, 1, 1, (unsigned)k.tile_lds, s,
                                      gargs, nullptr);
    } else {
        const size_t lds = spec_global_lds(d, f);
        const int64_t grid = (a.shots + k.spw - 1) / k.spw;
        hipFunction_t fn = !a.fixed_stop_g && k.global_nf[f] ? k.global_nf[f] : k.global[f];
        e = hipModuleLaunchKernel(fn, (unsigned)grid, 1, 1, (unsigned)k.wg, 1, 1, (unsigned)lds, s, gargs, nullptr);
    }
    if (e == hipSuccess && ev) e = hipEventRecord((*ev)[2], s);
    return e;
}

Workspace decoder_workspace(const lead_decoder *d) {
    Workspace ws;
    ws.Lv = d->d_Lv;
    ws.vflag = d->d_vflag;
    ws.counter = d->d_counter;
    ws.osd_list = d->d_osd_list;
    ws.gpost = d->d_gpost;
    ws.glam = d->d_glam;
    ws.gstats = d->d_gstats;
    ws.osd_mat = d->d_osd_mat;
    ws.osd_slots = d->osd_slots;
    ws.shots = d->ws_shots;
    return ws;
}

lead::LocalArgs local_args(const lead_decoder *d, const Workspace &ws, int64_t shots, lead_prior_mode mode) {
    lead::LocalArgs w{};
    w.Lv = ws.Lv;
    w.vflag = ws.vflag;
    w.counter = ws.counter;
    w.osd_list = ws.osd_list;
    w.items = shots * d->N;
    w.chunk = d->sched.local_chunk;
    const int pm = mode == LEAD_PRIOR_PER_SHOT ? 0 : 1;
    const int64_t per_cu =
        use_spec(d) ? d->spec->local_waves_per_cu[d->sched.specialized - 1][pm] : d->waves_per_cu[pm];
    int64_t waves = d->sched.local_waves > 0 ? d->sched.local_waves : per_cu * d->cus;
    const int64_t need = (w.items + w.chunk - 1) / w.chunk;
    w.waves = (int32_t)std::max<int64_t>(1, std::min(waves, need));
    return w;
}

void free_plain(lead_decoder *d) {
    (void)hipFree(d->d_S);
    (void)hipFree(d->d_cst);
    (void)hipFree(d->d_lamp);
    (void)hipFree(d->d_status);
    (void)hipFree(d->d_active);
    (void)hipFree(d->d_pS);
    (void)hipFree(d->d_pst);
    (void)hipFree(d->d_pended);
    (void)hipFree(d->d_pactive);
    if (d->h_active) (void)hipHostFree(d->h_active);
    d->d_S = d->d_cst = d->d_lamp = d->d_pS = d->d_pst = nullptr;
    d->d_status = d->d_active = d->h_active = d->d_pended = nullptr;
    d->d_pactive = nullptr;
    d->plain_shots = 0;
}


lead::DecodeArgs base_args(const lead_decoder *d) {
    lead::DecodeArgs a{};
    a.view = d->d_view;
    a.own = d->d_own;
    a.N = d->N;
    a.n = d->n;
    a.r = d->r;
    a.own_max = d->own_max;
    a.spw = d->spw;
    a.alpha = d->params.alpha;
    a.beta = d->params.ms_scale;
    a.clampv = d->params.llr_clamp;
    a.Tl = d->params.max_iter_local;
    a.Tg = d->params.max_iter_global;
    a.early_exit = d->params.early_exit ? 1 : 0;
    a.stage = d->params.stage;
    a.boost = d->params.boost ? 1 : 0;
    a.fixed_stop = d->params.fixed_point_stop != 0 ? 1 : 0;   // 1 or 2: local BP runs
    a.fixed_stop_g = d->params.fixed_point_stop == 1 ? 1 : 0;  // 1: global BP runs too
    a.local_osd = d->params.local_post ? 1 : 0;
    a.osd_order = d->params.osd_order;
    for (int c = 0; c < lead::kMaxChecks; ++c) a.mask[c] = c < d->r ? d->mask[c] : 0;
    return a;
}

lead_status check_decode_args(const lead_decoder *d, int64_t shots, const uint64_t *synd, int64_t synd_words,
                              const float *prior, lead_prior_mode mode, const uint64_t *ehat,
                              int64_t ehat_words, const float *lam) {
    if (!d) return fail(LEAD_E_ARG, "decoder is NULL");
    if (shots < 0) return fail(LEAD_E_ARG, "shots < 0");
    if (shots > d->max_shots) return fail(LEAD_E_CAPACITY, "shots exceeds the decoder's max_shots");
    if (shots == 0) return LEAD_OK;
    if (!synd || !prior) return fail(LEAD_E_ARG, "syndrome or prior pointer is NULL");
    if (synd_words < (d->m + 63) / 64) return fail(LEAD_E_ARG, "synd_words < ceil(m/64)");
    if (mode != LEAD_PRIOR_PER_SHOT && mode != LEAD_PRIOR_SHARED && mode != LEAD_PRIOR_FULL)
        return fail(LEAD_E_ARG, "bad prior mode");
    if (ehat && ehat_words < (d->n + 63) / 64) return fail(LEAD_E_ARG, "ehat_words < ceil(n/64)");
    if (d->params.stage == LEAD_STAGE_LOCAL && !lam) return fail(LEAD_E_ARG, "LOCAL stage needs d_prior_llr");
    return LEAD_OK;
}

// Events of one timed split launch, or nullptr when not timing (or while s
// is being captured).
std::array<hipEvent_t, 3> *timing_events(lead_decoder *d, hipStream_t s) {
    if (!d->timing) return nullptr;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return nullptr;
    std::array<hipEvent_t, 3> ev{};
    for (auto &x : ev)
        if (hipEventCreate(&x) != hipSuccess) {
            for (auto &y : ev)
                if (y) (void)hipEventDestroy(y);
            return nullptr;
        }
    d->tev.push_back(ev);
    return &d->tev.back();
}

// Adds the recorded event triples to the sums and releases them.
hipError_t drain_timing(lead_decoder *d) {
    hipError_t e = hipSuccess;
    for (auto &ev : d->tev) {
        if (e == hipSuccess) e = hipEventSynchronize(ev[2]);
        float a = 0.f, b = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&a, ev[0], ev[1]);
        if (e == hipSuccess) e = hipEventElapsedTime(&b, ev[1], ev[2]);
        if (e == hipSuccess) {
            d->tsum.local_ms += a;
            d->tsum.global_ms += b;
            d->tsum.local_launches++;
            d->tsum.global_launches++;
        }
        for (auto &x : ev) (void)hipEventDestroy(x);
    }
    d->tev.clear();
    return e;
}

// Launches the decode of `shots` shots (in workspace-sized chunks for the
// split path) on stream s.
hipError_t decode_chunks(lead_decoder *d, int64_t shots, const uint64_t *synd, int64_t synd_words,
                         const float *prior, lead_prior_mode mode, uint64_t *ehat, int64_t ehat_words, float *post,
                         float *lam, lead_shot_stats *stats, int stage, hipStream_t s, const Workspace &ws,
                         bool allow_timing = true) {
    // global BP alone: the per-shot kernel alone (there is no Phase 1); the
    // precompiled form runs it fused
    const bool gonly = d->params.stage == LEAD_STAGE_GLOBAL;
    const bool split = !d->sched.fused && (!gonly || use_spec(d));
    // global OSD-0 after global BP (its buffers hold ws_shots shots)
    const bool gpost = d->params.global_post && stage != LEAD_STAGE_LOCAL;
    // equal chunks of at most the schedule's chunk (no small tail launch)
    const int64_t chunk = d->sched.chunk_shots > 0 ? std::min<int64_t>(d->sched.chunk_shots, ws.shots) : ws.shots;
    const int64_t nchunks = split || gpost ? (shots + chunk - 1) / chunk : 1;
    const int64_t step = (shots + nchunks - 1) / nchunks;
    for (int64_t off = 0; off < shots; off += step) {
        const int64_t cnt = std::min(step, shots - off);
        lead::DecodeArgs a = base_args(d);
        a.synd = synd + off * synd_words;
        a.synd_words = synd_words;
        a.prior = prior + (mode == LEAD_PRIOR_PER_SHOT ? off : mode == LEAD_PRIOR_FULL ? off * d->n : 0);
        a.prior_mode = mode;
        a.ehat = ehat ? ehat + off * ehat_words : nullptr;
        a.ehat_words = ehat_words;
        a.post = post ? post + off * d->n : nullptr;
        a.lam_out = lam ? lam + off * d->n : nullptr;
        a.stats = stats ? stats + off : nullptr;
        a.shots = cnt;
        a.stage = stage == LEAD_STAGE_LOCAL ? LEAD_STAGE_LOCAL : LEAD_STAGE_FULL;
        a.global_only = gonly ? 1 : 0;
        const lead::LocalArgs w = local_args(d, ws, cnt, mode);
        std::array<hipEvent_t, 3> *ev = split && allow_timing ? timing_events(d, s) : nullptr;
        if (gpost) {
            if (!a.post) a.post = ws.gpost;
            if (!a.stats) a.stats = ws.gstats;
            if (!a.lam_out && d->params.osd_order > 0) a.lam_out = ws.glam;   // the sweep's costs
        }
        hipError_t e = split && use_spec(d) ? launch_spec(d, a, w, s, ev)
                                   : lead::launch_decode(d->D, d->r, a, w, split, s, ev ? ev->data() : nullptr);
        if (e == hipSuccess && gpost) e = launch_osd(d, a, ws, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Library streams (default priority) used to run batch items concurrently.
struct StreamPool {
    int device = -1;
    std::vector<hipStream_t> streams;
};
thread_local StreamPool g_pool;

hipError_t pool_streams(int count, std::vector<hipStream_t> &out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (g_pool.device != dev) {
        g_pool.streams.clear();   // streams of another device are left to the runtime
        g_pool.device = dev;
    }
    while ((int)g_pool.streams.size() < count) {
        hipStream_t st = nullptr;
        if ((e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking)) != hipSuccess) return e;
        g_pool.streams.push_back(st);
    }
    out.assign(g_pool.streams.begin(), g_pool.streams.begin() + count);
    return hipSuccess;
}

lead_status check_item(const lead_batch_item &it) {
    return check_decode_args(it.decoder, it.shots, it.d_synd, it.synd_words, it.d_prior, it.mode, it.d_ehat,
                             it.ehat_words, it.d_prior_llr);
}

// Groups items by decoder (items sharing a decoder share its workspace and
// must run in order).
int group_items(const lead_batch_item *items, int32_t n, std::vector<int> &group) {
    std::vector<lead_decoder *> decs;
    group.resize(n);
    for (int i = 0; i < n; ++i) {
        auto it = std::find(decs.begin(), decs.end(), items[i].decoder);
        group[i] = (int)(it - decs.begin());
        if (it == decs.end()) decs.push_back(items[i].decoder);
    }
    return (int)decs.size();
}

// Fork from `stream`, run each decoder's items in order on its own library
// stream, join back into `stream`.  The events used are appended to `events`
// (the caller destroys them, after the end of a capture when capturing).
lead_status enqueue_batch(const lead_batch_item *items, int32_t n, hipStream_t stream,
                          const std::vector<hipStream_t> &streams, const std::vector<int> &group, int ngroups,
                          std::vector<hipEvent_t> &events) {
    hipError_t e;
    hipEvent_t start = nullptr;
    if ((e = hipEventCreateWithFlags(&start, hipEventDisableTiming)) != hipSuccess) return hip_fail(e, "event");
    events.push_back(start);
    if ((e = hipEventRecord(start, stream)) != hipSuccess) return hip_fail(e, "event record");
    for (int g = 0; g < ngroups; ++g)
        if ((e = hipStreamWaitEvent(streams[g], start, 0)) != hipSuccess) return hip_fail(e, "stream wait");
    for (int i = 0; i < n; ++i) {
        const lead_batch_item &it = items[i];
        if (it.shots == 0) continue;
        e = decode_chunks(it.decoder, it.shots, it.d_synd, it.synd_words, it.d_prior, it.mode, it.d_ehat,
                          it.ehat_words, it.d_post, it.d_prior_llr, it.d_stats, it.decoder->params.stage,
                          streams[group[i]], decoder_workspace(it.decoder));
        if (e != hipSuccess) return hip_fail(e, "batch launch");
    }
    for (int g = 0; g < ngroups; ++g) {
        hipEvent_t done = nullptr;
        if ((e = hipEventCreateWithFlags(&done, hipEventDisableTiming)) != hipSuccess) return hip_fail(e, "event");
        events.push_back(done);
        if ((e = hipEventRecord(done, streams[g])) != hipSuccess) return hip_fail(e, "event record");
        if ((e = hipStreamWaitEvent(stream, done, 0)) != hipSuccess) return hip_fail(e, "stream wait");
    }
    return LEAD_OK;
}

void destroy_events(std::vector<hipEvent_t> &events) {
    for (auto ev : events) (void)hipEventDestroy(ev);
    events.clear();
}

}  // namespace

extern "C" {

const char *lead_last_error(void) { return g_err.c_str(); }

lead_status lead_code_create(const lead_code_desc *desc, lead_code **out) {
    if (!desc || !out) return fail(LEAD_E_ARG, "NULL argument");
    *out = nullptr;
    lead_code *c = new (std::nothrow) lead_code();
    if (!c) return fail(LEAD_E_NOMEM, "out of host memory");
    std::string err;
    int rc;
    try {
        rc = lead::build_code(desc->order, desc->mul, desc->delta, desc->A, desc->B, desc->kA, desc->GA,
                              desc->kB, desc->GB, c->c, err);
    } catch (const std::bad_alloc &) {
        delete c;
        return fail(LEAD_E_NOMEM, "out of host memory");
    }
    if (rc != 0) {
        delete c;
        return fail((lead_status)rc, err);
    }
    *out = c;
    return LEAD_OK;
}

lead_status lead_code_query(const lead_code *code, lead_code_info *o) {
    if (!code || !o) return fail(LEAD_E_ARG, "NULL argument");
    const lead::Code &c = code->c;
    o->order = c.order;
    o->delta = c.delta;
    o->n = c.n;
    for (int t = 0; t < 2; ++t) {
        o->r[t] = c.t[t].r;
        o->m[t] = c.order * c.t[t].r;
        o->rank[t] = c.t[t].rank;
        o->eloc[t] = c.t[t].eloc;
    }
    o->k = c.k;
    return LEAD_OK;
}

lead_status lead_code_get_H(const lead_code *code, lead_check_type t, int32_t *indptr, int32_t *indices) {
    if (!code || !indptr || (t != LEAD_CHECK_Z && t != LEAD_CHECK_X)) return fail(LEAD_E_ARG, "bad argument");
    const lead::TypeTables &tt = code->c.t[t];
    std::copy(tt.csr_ptr.begin(), tt.csr_ptr.end(), indptr);
    if (indices) std::copy(tt.csr_idx.begin(), tt.csr_idx.end(), indices);
    return LEAD_OK;
}

lead_status lead_code_get_views(const lead_code *code, lead_check_type t, int32_t *view) {
    if (!code || !view || (t != LEAD_CHECK_Z && t != LEAD_CHECK_X)) return fail(LEAD_E_ARG, "bad argument");
    std::copy(code->c.t[t].view.begin(), code->c.t[t].view.end(), view);
    return LEAD_OK;
}

lead_status lead_code_specialize(const lead_code *code, lead_check_type t) {
    if (!code || (t != LEAD_CHECK_Z && t != LEAD_CHECK_X)) return fail(LEAD_E_ARG, "bad argument");
    const std::string src = lead::jit::source(code->c, t);
    if (src.empty()) return fail(LEAD_E_UNSUPPORTED, "the code has no local position map");
    std::vector<char> obj;
    std::string err;
    if (!lead::jit::compile(src, obj, err)) return fail(LEAD_E_UNSUPPORTED, err);
    // the sum-product form, where a view is small enough for it
    const std::string sp = lead::jit::source(code->c, t, true);
    if (!sp.empty() && !lead::jit::compile(sp, obj, err)) return fail(LEAD_E_UNSUPPORTED, err);
    return LEAD_OK;
}

lead_status lead_batch_fused_specialize(const lead_code *const *codes, const lead_check_type *types,
                                        const int32_t *forms, const lead_prior_mode *modes, int32_t n) {
    if (!codes || !types || !forms || !modes || n <= 0) return fail(LEAD_E_ARG, "bad argument");
    std::vector<lead::jit::FusedPart> parts;
    for (int i = 0; i < n; ++i) {
        if (!codes[i] || (types[i] != LEAD_CHECK_Z && types[i] != LEAD_CHECK_X)) return fail(LEAD_E_ARG, "bad request");
        // the persistent Phases 2-3 kernel wherever the code has it (the
        // default schedule of a decoder)
        parts.push_back(lead::jit::FusedPart{&codes[i]->c, (int)types[i], (int)forms[i],
                                             modes[i] == LEAD_PRIOR_PER_SHOT ? 0 : 1, true});
    }
    lead::jit::settle_fused_tiles(parts);
    lead::jit::FusedKernels k;
    std::string err;
    const std::string src = lead::jit::fused_source(parts, k, err);
    if (src.empty()) return fail(LEAD_E_UNSUPPORTED, err);
    std::vector<char> obj;
    if (!lead::jit::compile(src, obj, err)) return fail(LEAD_E_UNSUPPORTED, err);
    return LEAD_OK;
}

void lead_code_destroy(lead_code *code) { delete code; }

}  // extern "C"

namespace {

lead_status create_decoder(std::shared_ptr<lead::Code> code, int t, const lead_params *params, int64_t max_shots,
                           lead_decoder **out) {
    *out = nullptr;
    if (max_shots < 0) return fail(LEAD_E_ARG, "max_shots < 0");
    lead_status st = check_params(params);
    if (st != LEAD_OK) return st;
    const lead::Code &c = *code;
    const lead::TypeTables &tt = c.t[t];
    const int D = c.delta, D2 = D * D;
    if (!lead::kernel_supported(D, tt.r))
        return fail(LEAD_E_UNSUPPORTED, "no kernel for delta=" + std::to_string(D) + " with " +
                                            std::to_string(tt.r) + " checks per vertex");
    for (uint64_t mk : tt.mask)
        if (__builtin_popcountll(mk) > 32 || __builtin_popcountll(mk) < 2)
            return fail(LEAD_E_UNSUPPORTED, "local check weight outside 2..32");
    if (c.order > lead::kMaxWorkgroup)
        return fail(LEAD_E_UNSUPPORTED, "group order above " + std::to_string(lead::kMaxWorkgroup));
    std::unique_ptr<lead_decoder> d(new (std::nothrow) lead_decoder());
    if (!d) return fail(LEAD_E_NOMEM, "out of host memory");
    d->keep = std::move(code);
    d->code = d->keep.get();
    d->type = t;
    d->params = *params;
    d->max_shots = max_shots;
    d->D = D;
    d->N = c.order;
    d->n = c.n;
    d->r = tt.r;
    d->m = c.order * tt.r;
    d->own_max = tt.own_max;
    for (int i = 0; i < tt.r; ++i) d->mask[i] = tt.mask[i];
    d->spw = default_spw(d->N);
    d->sched.shots_per_workgroup = d->spw;
    d->sched.fused = 0;
    d->sched.local_chunk = 256;
    d->sched.local_waves = 0;
    hipError_t e = hipGetDevice(&d->device);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    e = hipDeviceGetAttribute(&d->cus, hipDeviceAttributeMultiprocessorCount, d->device);
    if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute");
    const int64_t per_shot = (int64_t)d->N * ((int64_t)D2 * (int64_t)sizeof(float) + (int64_t)sizeof(uint32_t));
    d->ws_shots = std::min<int64_t>(std::max<int64_t>(max_shots, 1), std::max<int64_t>(kChunkShots, kChunkBytes / per_shot));
    d->waves_per_cu[0] = lead::local_waves_per_cu(D, 0);
    d->waves_per_cu[1] = lead::local_waves_per_cu(D, 1);
    // owner lists: per view, owned local positions in increasing order
    std::vector<uint32_t> own((size_t)d->N * d->own_max, lead::kNoOwn);
    for (int v = 0; v < d->N; ++v) {
        int k = 0;
        for (int j = 0; j < D2; ++j) {
            const int sl = v * D2 + j;
            if (!tt.owned[sl]) continue;
            const int p = tt.partner[sl];
            own[(size_t)v * d->own_max + k++] =
                (uint32_t)j | ((uint32_t)(p % D2) << 8) | ((uint32_t)(p / D2) << 16);
        }
    }
    e = hipMalloc(&d->d_view, sizeof(int32_t) * tt.view.size());
    if (e == hipSuccess) e = hipMalloc(&d->d_own, sizeof(uint32_t) * own.size());
    if (e == hipSuccess) e = hipMemcpy(d->d_view, tt.view.data(), sizeof(int32_t) * tt.view.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d->d_own, own.data(), sizeof(uint32_t) * own.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc(&d->d_Lv, sizeof(float) * (size_t)d->ws_shots * d->N * D2);
    if (e == hipSuccess) e = hipMalloc(&d->d_vflag, sizeof(uint32_t) * (size_t)d->ws_shots * d->N);
    if (e == hipSuccess) e = hipMalloc(&d->d_counter, 4 * sizeof(int64_t));
    if (e == hipSuccess) e = hipMalloc(&d->d_osd_list, sizeof(uint32_t) * (size_t)d->ws_shots * d->N);
    // kernels for this code's check structure (the precompiled ones serve
    // when they cannot be built)
    if (e == hipSuccess) {
        std::string jerr;
        d->spec = lead::jit::load(c, t, d->device, sum_product(d.get()), jerr);
        if (!d->spec && needs_spec(d.get())) e = hipErrorNotSupported;
        if (d->spec) {
            std::vector<uint32_t> pv;
            std::vector<uint64_t> fown;
            lead::jit::partner_tables(c, t, pv, fown);
            e = hipMalloc(&d->d_pv, sizeof(uint32_t) * pv.size());
            if (e == hipSuccess) e = hipMalloc(&d->d_fown, sizeof(uint64_t) * fown.size());
            if (e == hipSuccess) e = hipMemcpy(d->d_pv, pv.data(), sizeof(uint32_t) * pv.size(), hipMemcpyHostToDevice);
            if (e == hipSuccess)
                e = hipMemcpy(d->d_fown, fown.data(), sizeof(uint64_t) * fown.size(), hipMemcpyHostToDevice);
            if (e == hipSuccess && (d->spec->osd || d->spec->osd_big)) {
                e = hipMalloc(&d->d_rptr, sizeof(int32_t) * tt.csr_ptr.size());
                if (e == hipSuccess) e = hipMalloc(&d->d_ridx, sizeof(int32_t) * std::max<size_t>(tt.csr_idx.size(), 1));
                if (e == hipSuccess)
                    e = hipMemcpy(d->d_rptr, tt.csr_ptr.data(), sizeof(int32_t) * tt.csr_ptr.size(), hipMemcpyHostToDevice);
                if (e == hipSuccess && !tt.csr_idx.empty())
                    e = hipMemcpy(d->d_ridx, tt.csr_idx.data(), sizeof(int32_t) * tt.csr_idx.size(),
                                  hipMemcpyHostToDevice);
            }
        }
        if (e == hipSuccess && d->params.global_post) {
            if (!osd_ready(d.get())) {
                jerr = d->spec ? "the code is too large for the global OSD kernels" : jerr;
                e = hipErrorNotSupported;
            } else {
                e = ensure_osd_workspace(d.get());
            }
        }
        d->sched.specialized = spec_form(d.get(), lead::jit::kExplicit);
        if (e == hipErrorNotSupported) {
            (void)hipFree(d->d_view);
            (void)hipFree(d->d_own);
            (void)hipFree(d->d_Lv);
            (void)hipFree(d->d_vflag);
            (void)hipFree(d->d_counter);
            (void)hipFree(d->d_osd_list);
            (void)hipFree(d->d_pv);
            (void)hipFree(d->d_fown);
            (void)hipFree(d->d_rptr);
            (void)hipFree(d->d_ridx);
            return fail(LEAD_E_UNSUPPORTED, "sum-product or OSD-0 needs the kernels compiled for the code: " + jerr);
        }
    }
    if (e != hipSuccess) {
        (void)hipFree(d->d_view);
        (void)hipFree(d->d_own);
        (void)hipFree(d->d_Lv);
        (void)hipFree(d->d_vflag);
        (void)hipFree(d->d_counter);
        (void)hipFree(d->d_osd_list);
        (void)hipFree(d->d_pv);
        (void)hipFree(d->d_fown);
        (void)hipFree(d->d_rptr);
        (void)hipFree(d->d_ridx);
        (void)hipFree(d->d_gpost);
        (void)hipFree(d->d_glam);
        (void)hipFree(d->d_gstats);
        (void)hipFree(d->d_osd_mat);
        return hip_fail(e, "device allocation");
    }
    *out = d.release();
    return LEAD_OK;
}

}  // namespace

namespace lead {

lead_status clone_decoder(const lead_decoder *src, int64_t max_shots, lead_decoder **out) {
    if (!src || !out) return fail(LEAD_E_ARG, "bad argument");
    lead_status st = create_decoder(src->keep, src->type, &src->params, max_shots, out);
    if (st != LEAD_OK) return st;
    (*out)->sched = src->sched;
    (*out)->spw = src->spw;
    return LEAD_OK;
}

void decoder_shape(const lead_decoder *d, int *n, int *m) {
    *n = d->n;
    *m = d->m;
}

int64_t decoder_device_bytes(const lead_decoder *d) {
    const lead::TypeTables &tt = d->code->t[d->type];
    const int64_t D2 = (int64_t)d->D * d->D, N = d->N, ws = d->ws_shots;
    int64_t b = 4 * (int64_t)tt.view.size() + 4 * N * d->own_max;            // view table, owner lists
    b += ws * (N * D2 * 4 + N * 4 + N * 4) + 4 * 8;                          // workspace, counters
    if (d->d_pv) b += 4 * N * ((D2 + 1) / 2) + 8 * N;                        // partner tables
    if (d->d_rptr) b += 4 * (int64_t)(tt.csr_ptr.size() + tt.csr_idx.size());
    if (d->d_gpost) b += ws * (4 * (int64_t)d->n * 2 + (int64_t)sizeof(lead_shot_stats));
    if (d->d_osd_mat) b += (int64_t)lead::jit::osd_big_slot_bytes(*d->code, d->type) * d->osd_slots;
    if (d->d_pS)
        b += d->plain_shots * (N * D2 * 4 + N * 4 * lead::jit::plain_state_words(*d->code, d->type) + 4) + 8;
    return b;
}

lead_status set_error(lead_status s, const char *msg) { return fail(s, msg); }

}  // namespace lead

extern "C" {

lead_status lead_decoder_create(const lead_code *code, lead_check_type t, const lead_params *params,
                                int64_t max_shots, lead_decoder **out) {
    if (!code || !out || (t != LEAD_CHECK_Z && t != LEAD_CHECK_X)) return fail(LEAD_E_ARG, "bad argument");
    std::shared_ptr<lead::Code> copy;
    try {
        copy = std::make_shared<lead::Code>(code->c);
    } catch (const std::bad_alloc &) {
        return fail(LEAD_E_NOMEM, "out of host memory");
    }
    return create_decoder(std::move(copy), t, params, max_shots, out);
}

lead_status lead_decoder_set_params(lead_decoder *d, const lead_params *params) {
    if (!d) return fail(LEAD_E_ARG, "decoder is NULL");
    lead_status st = check_params(params);
    if (st != LEAD_OK) return st;
    if (params->global_post) {
        if (!osd_ready(d)) return fail(LEAD_E_UNSUPPORTED, "no global OSD-0 kernel for this code");
        hipError_t e = ensure_osd_workspace(d);
        if (e != hipSuccess) return hip_fail(e, "OSD-0 workspace allocation");
    }
    if (params->bp != d->params.bp) {
        // the other BP flavour needs the other set of compiled kernels
        std::string jerr;
        auto k = lead::jit::load(*d->code, d->type, d->device, params->bp == LEAD_BP_SUMPRODUCT, jerr);
        if (!k && params->bp == LEAD_BP_SUMPRODUCT) return fail(LEAD_E_UNSUPPORTED, "sum-product: " + jerr);
        if (k && !d->d_pv) return fail(LEAD_E_UNSUPPORTED, "no partner tables");
        if (params->global_post && !osd_kernels(k.get())) return fail(LEAD_E_UNSUPPORTED, "no global OSD kernel");
        d->spec = k;
        d->params = *params;
        if (params->global_post) {
            hipError_t e = ensure_osd_workspace(d);
            if (e != hipSuccess) return hip_fail(e, "OSD workspace allocation");
        }
        d->sched.specialized = spec_form(d, lead::jit::kExplicit);
        if (needs_spec(d)) d->sched.fused = 0;
        return LEAD_OK;
    }
    if (params->local_post && !d->spec) return fail(LEAD_E_UNSUPPORTED, "OSD-0 needs the kernels compiled for the code");
    d->params = *params;
    if (needs_spec(d)) {
        d->sched.fused = 0;
        if (!d->sched.specialized) d->sched.specialized = spec_form(d, lead::jit::kExplicit);
    }
    return LEAD_OK;
}

lead_status lead_decoder_set_schedule(lead_decoder *d, const lead_schedule *sc) {
    if (!d || !sc) return fail(LEAD_E_ARG, "bad argument");
    if (sc->shots_per_workgroup < 0 || sc->local_chunk < 0 || sc->local_waves < 0 || sc->chunk_shots < 0)
        return fail(LEAD_E_ARG, "negative schedule field");
    if (sc->global_osd_form < 0 || sc->global_osd_form > 2) return fail(LEAD_E_ARG, "bad global_osd_form");
    if (sc->global_tiles < 0 || sc->global_tiles > 2) return fail(LEAD_E_ARG, "bad global_tiles");
    const int spw = sc->shots_per_workgroup ? sc->shots_per_workgroup : default_spw(d->N);
    if (lead::workgroup_size(d->N, spw) > lead::kMaxWorkgroup)
        return fail(LEAD_E_UNSUPPORTED, "shots_per_workgroup too large for the workgroup limit");
    if (lead::decode_lds_bytes(d->D, lead::workgroup_size(d->N, spw), spw, d->n) > 65536)
        return fail(LEAD_E_UNSUPPORTED, "shots_per_workgroup needs more than 64 KiB of LDS");
    d->spw = spw;
    d->sched.shots_per_workgroup = spw;
    d->sched.fused = sc->fused ? 1 : 0;
    d->sched.local_chunk = sc->local_chunk ? sc->local_chunk : 256;
    d->sched.local_waves = sc->local_waves;
    d->sched.chunk_shots = sc->chunk_shots;
    d->sched.global_osd_form = sc->global_osd_form;
    d->sched.global_tiles = sc->global_tiles;
    d->sched.specialized = spec_form(d, sc->specialized);
    if (needs_spec(d)) {   // sum-product and OSD-0 run the kernels compiled for the code only
        d->sched.fused = 0;
        if (!d->sched.specialized) d->sched.specialized = spec_form(d, lead::jit::kExplicit);
    }
    if (d->params.global_post && osd_ready(d)) {
        hipError_t e = ensure_osd_workspace(d);
        if (e != hipSuccess) return hip_fail(e, "OSD workspace allocation");
    }
    return LEAD_OK;
}

lead_status lead_decoder_get_schedule(const lead_decoder *d, lead_schedule *sc) {
    if (!d || !sc) return fail(LEAD_E_ARG, "bad argument");
    *sc = d->sched;
    if (d->spec) sc->global_osd_form = osd_big(d) ? 2 : (d->spec->osd ? 1 : 0);
    sc->global_tiles = d->spec && !d->spec->bperm && d->sched.specialized > 0
                           ? (use_tiles(d, d->sched.specialized - 1) ? 1 : 2)
                           : 0;
    return LEAD_OK;
}

lead_status lead_decoder_time_phases(lead_decoder *d, int32_t enable) {
    if (!d) return fail(LEAD_E_ARG, "decoder is NULL");
    hipError_t e = drain_timing(d);
    d->tsum = lead_phase_times{};
    d->timing = enable != 0;
    if (e != hipSuccess) return hip_fail(e, "phase timing");
    return LEAD_OK;
}

lead_status lead_decoder_phase_times(lead_decoder *d, lead_phase_times *out) {
    if (!d || !out) return fail(LEAD_E_ARG, "bad argument");
    hipError_t e = drain_timing(d);
    if (e != hipSuccess) return hip_fail(e, "phase timing");
    *out = d->tsum;
    return LEAD_OK;
}

void lead_decoder_destroy(lead_decoder *d) {
    if (!d) return;
    (void)hipFree(d->d_view);
    (void)hipFree(d->d_own);
    (void)hipFree(d->d_Lv);
    (void)hipFree(d->d_vflag);
    (void)hipFree(d->d_counter);
    (void)hipFree(d->d_osd_list);
    (void)hipFree(d->d_pv);
    (void)hipFree(d->d_fown);
    (void)hipFree(d->d_rptr);
    (void)hipFree(d->d_ridx);
    (void)hipFree(d->d_gpost);
    (void)hipFree(d->d_glam);
    (void)hipFree(d->d_gstats);
    (void)hipFree(d->d_osd_mat);
    (void)drain_timing(d);
    free_plain(d);
    delete d;
}

lead_status lead_decode(lead_decoder *d, int64_t shots, const uint64_t *synd, int64_t synd_words,
                        const float *prior, lead_prior_mode mode, uint64_t *ehat, int64_t ehat_words, float *post,
                        float *lam, lead_shot_stats *stats, void *stream) {
    lead_status st = check_decode_args(d, shots, synd, synd_words, prior, mode, ehat, ehat_words, lam);
    if (st != LEAD_OK || shots == 0) return st;
    if (lead::decode_lds_bytes(d->D, lead::workgroup_size(d->N, d->spw), d->spw, d->n) > 65536)
        return fail(LEAD_E_UNSUPPORTED, "workgroup needs more than 64 KiB of LDS");
    hipError_t e = decode_chunks(d, shots, synd, synd_words, prior, mode, ehat, ehat_words, post, lam, stats,
                                 d->params.stage, (hipStream_t)stream, decoder_workspace(d));
    if (e != hipSuccess) return hip_fail(e, "decode launch");
    return LEAD_OK;
}

lead_status lead_decode_noalloc(lead_decoder *d, int64_t shots, const uint64_t *synd, int64_t synd_words,
                                const float *prior, lead_prior_mode mode, uint64_t *ehat, int64_t ehat_words,
                                float *post, float *lam, lead_shot_stats *stats, void *stream) {
    lead_status st = check_decode_args(d, shots, synd, synd_words, prior, mode, ehat, ehat_words, lam);
    if (st != LEAD_OK || shots == 0) return st;
    if (lead::decode_lds_bytes(d->D, lead::workgroup_size(d->N, d->spw), d->spw, d->n) > 65536)
        return fail(LEAD_E_UNSUPPORTED, "workgroup needs more than 64 KiB of LDS");
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev != d->device)
        return fail(LEAD_E_ARG, "lead_decode_noalloc: the current device is not the decoder's device");
    // scratch layout: queue counters (256 B), then per shot the local
    // posteriors, view flags and local OSD list, then (global_post) the
    // global OSD's buffers for outputs the caller does not pass
    const bool gpost = d->params.global_post && d->params.stage != LEAD_STAGE_LOCAL;
    const size_t lv = sizeof(float) * (size_t)d->N * d->D * d->D, vf = sizeof(uint32_t) * (size_t)d->N;
    const size_t gp = gpost && !post ? sizeof(float) * (size_t)d->n : 0;
    const size_t gs = gpost && !stats ? sizeof(lead_shot_stats) : 0;
    const size_t gl = gpost && !lam && d->params.osd_order > 0 ? sizeof(float) * (size_t)d->n : 0;
    const size_t per_shot = lv + 2 * vf + gp + gs + gl;
    const size_t head = 256, slack = 8 * 256;   // counters, alignment of the eight arrays
    // the global OSD with the matrix in device memory works in matrix slots
    // (one per workgroup): as many as fit beside the batch, at most one per CU
    const size_t slot = gpost && osd_big(d) ? lead::jit::osd_big_slot_bytes(*d->code, d->type) : 0;
    const size_t slot_room = slot ? slot * (size_t)std::min<int64_t>(std::max(1, d->cus), shots) : 0;
    if (slot && lead::kScratchBytes < head + slack + slot)
        return fail(LEAD_E_CAPACITY, "lead_decode_noalloc: one global OSD matrix slot (" + std::to_string(slot) +
                                         " bytes) does not fit the static scratch");
    const int64_t capacity = (int64_t)((lead::kScratchBytes - head - slack - slot) / per_shot);
    if (shots > capacity)
        return fail(LEAD_E_CAPACITY, "lead_decode_noalloc: " + std::to_string(shots) + " shots need " +
                                         std::to_string(per_shot * (size_t)shots + head) +
                                         " bytes of scratch; the static scratch holds " +
                                         std::to_string(lead::kScratchBytes) + " bytes (at most " +
                                         std::to_string(capacity) + " shots of this decoder per call)");
    void *base = nullptr;
    if ((e = lead::scratch_address(d->device, &base)) != hipSuccess) return hip_fail(e, "scratch address");
    char *p = static_cast<char *>(base);
    size_t off = 0;
    auto carve = [&](size_t bytes) {
        char *q = bytes ? p + off : nullptr;
        off = (off + bytes + 255) & ~size_t(255);
        return q;
    };
    Workspace ws;
    ws.counter = reinterpret_cast<int64_t *>(carve(head));
    ws.Lv = reinterpret_cast<float *>(carve(lv * (size_t)shots));
    ws.vflag = reinterpret_cast<uint32_t *>(carve(vf * (size_t)shots));
    ws.osd_list = reinterpret_cast<uint32_t *>(carve(vf * (size_t)shots));
    ws.gpost = reinterpret_cast<float *>(carve(gp * (size_t)shots));
    ws.gstats = reinterpret_cast<lead_shot_stats *>(carve(gs * (size_t)shots));
    ws.glam = reinterpret_cast<float *>(carve(gl * (size_t)shots));
    if (slot) {
        const size_t room = lead::kScratchBytes - std::min(lead::kScratchBytes, off);
        ws.osd_slots = (int)std::min<size_t>(room / slot, std::min(slot_room / slot, (size_t)std::max(1, d->cus)));
        ws.osd_mat = reinterpret_cast<uint64_t *>(carve(slot * (size_t)ws.osd_slots));
    }
    ws.shots = shots;
    if (off > lead::kScratchBytes) return fail(LEAD_E_CAPACITY, "lead_decode_noalloc: scratch layout overflow");
    // every launch is enqueued without timing events (no event objects are
    // created); the queue counters are cleared by a fill kernel
    e = decode_chunks(d, shots, synd, synd_words, prior, mode, ehat, ehat_words, post, lam, stats, d->params.stage,
                      (hipStream_t)stream, ws, false);
    if (e != hipSuccess) return hip_fail(e, "decode launch");
    return LEAD_OK;
}

}  // extern "C"

namespace {

// The plain form on the kernels compiled for the code: per chunk of the
// workspace, Phase 1 exactly as in lead_decode, then one launch of the
// compiled round kernel per global round (Phases 2-3 of that round, the
// sums and check state restored from and saved to device memory), the count
// of shots still running copied to pinned host memory and the stream
// synchronised after every round, and a last launch ending the shots that
// ran to the cap; then the global OSD if asked for.  Outputs are those of
// lead_decode bit for bit (same arithmetic in the same order).
hipError_t plain_spec(lead_decoder *d, int64_t shots, const uint64_t *synd, int64_t synd_words, const float *prior,
                      lead_prior_mode mode, uint64_t *ehat, int64_t ehat_words, float *post, float *lam,
                      lead_shot_stats *stats, hipStream_t s) {
    const lead::jit::Kernels &k = *d->spec;
    const int f = d->sched.specialized - 1;
    const int D2 = d->D * d->D;
    hipError_t e = hipSuccess;
    if (!d->d_pS) {
        const int64_t ps = std::max<int64_t>(1, std::min<int64_t>(d->max_shots, d->ws_shots));
        const size_t words = (size_t)lead::jit::plain_state_words(*d->code, d->type);
        e = hipMalloc(&d->d_pS, sizeof(float) * (size_t)ps * D2 * d->N);
        if (e == hipSuccess) e = hipMalloc(&d->d_pst, sizeof(float) * (size_t)ps * words * d->N);
        if (e == hipSuccess) e = hipMalloc(&d->d_pended, sizeof(int32_t) * (size_t)ps);
        if (e == hipSuccess) e = hipMalloc(&d->d_pactive, sizeof(int64_t));
        if (e == hipSuccess && !d->h_active) e = hipHostMalloc(&d->h_active, sizeof(int32_t), hipHostMallocDefault);
        if (e != hipSuccess) return e;
        d->plain_shots = ps;
    }
    const bool gonly = d->params.stage == LEAD_STAGE_GLOBAL;
    const bool gpost = d->params.global_post != 0;
    const Workspace ws = decoder_workspace(d);
    const int64_t cap = std::min<int64_t>(ws.shots, d->plain_shots);
    const int64_t chunk = d->sched.chunk_shots > 0 ? std::min<int64_t>(d->sched.chunk_shots, cap) : cap;
    const int64_t nchunks = (shots + chunk - 1) / chunk;
    const int64_t step = (shots + nchunks - 1) / nchunks;
    const size_t lds = spec_global_lds(d, f);
    for (int64_t off = 0; off < shots; off += step) {
        const int64_t cnt = std::min(step, shots - off);
        lead::DecodeArgs a = base_args(d);
        a.synd = synd + off * synd_words;
        a.synd_words = synd_words;
        a.prior = prior + (mode == LEAD_PRIOR_PER_SHOT ? off : mode == LEAD_PRIOR_FULL ? off * d->n : 0);
        a.prior_mode = mode;
        a.ehat = ehat ? ehat + off * ehat_words : nullptr;
        a.ehat_words = ehat_words;
        a.post = post ? post + off * d->n : nullptr;
        a.lam_out = lam ? lam + off * d->n : nullptr;
        a.stats = stats ? stats + off : nullptr;
        a.shots = cnt;
        a.stage = LEAD_STAGE_FULL;
        a.global_only = gonly ? 1 : 0;
        if (gpost) {
            if (!a.post) a.post = ws.gpost;
            if (!a.stats) a.stats = ws.gstats;
            if (!a.lam_out && d->params.osd_order > 0) a.lam_out = ws.glam;   // the sweep's costs
        }
        lead::LocalArgs w = local_args(d, ws, cnt, mode);
        if (!gonly) {
            if ((e = lead::launch_reset_counter(w.counter, s)) != hipSuccess) return e;
            void *largs[] = {&a, &w};
            e = hipModuleLaunchKernel(k.local[f][mode == LEAD_PRIOR_PER_SHOT ? 0 : 1], (unsigned)w.waves, 1, 1, 64, 1,
                                      1, (unsigned)k.local_lds[f][mode == LEAD_PRIOR_PER_SHOT ? 0 : 1], s, largs,
                                      nullptr);
            if (e == hipSuccess && a.local_osd)
                e = hipModuleLaunchKernel(k.local_osd, (unsigned)(8 * d->cus), 1, 1, 64, 1, 1, 0, s, largs, nullptr);
            if (e != hipSuccess) return e;
        }
        a.spw = k.spw;
        lead::SpecArgs x{d->d_pv, d->d_fown};
        lead::PlainArgs pl{d->d_pS, d->d_pst, d->d_pended, reinterpret_cast<int32_t *>(d->d_pactive), 0};
        const int64_t grid = (cnt + k.spw - 1) / k.spw;
        bool running = true;
        for (int t = 1; t <= d->params.max_iter_global + 1 && running; ++t) {
            if ((e = lead::launch_clear_i64(d->d_pactive, 1, s)) != hipSuccess) return e;
            pl.round = t;
            void *rargs[] = {&a, &w, &x, &pl};
            e = hipModuleLaunchKernel(k.round[f], (unsigned)grid, 1, 1, (unsigned)k.wg, 1, 1, (unsigned)lds, s, rargs,
                                      nullptr);
            if (e != hipSuccess) return e;
            if (t <= d->params.max_iter_global) {
                // the host-visible count of shots still running
                e = hipMemcpyAsync(d->h_active, d->d_pactive, sizeof(int32_t), hipMemcpyDeviceToHost, s);
                if (e == hipSuccess) e = hipStreamSynchronize(s);
                if (e != hipSuccess) return e;
                running = *d->h_active != 0;
            }
        }
        if (gpost && (e = launch_osd(d, a, ws, s)) != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

extern "C" {

lead_status lead_decode_plain(lead_decoder *d, int64_t shots, const uint64_t *synd, int64_t synd_words,
                              const float *prior, lead_prior_mode mode, uint64_t *ehat, int64_t ehat_words,
                              float *post, float *lam, lead_shot_stats *stats, void *stream) {
    lead_status st = check_decode_args(d, shots, synd, synd_words, prior, mode, ehat, ehat_words, lam);
    if (st != LEAD_OK || shots == 0) return st;
    if (d->params.stage == LEAD_STAGE_LOCAL)
        return lead_decode(d, shots, synd, synd_words, prior, mode, ehat, ehat_words, post, lam, stats, stream);
    if (use_spec(d) && d->spec->round[d->sched.specialized - 1]) {
        hipError_t e = plain_spec(d, shots, synd, synd_words, prior, mode, ehat, ehat_words, post, lam, stats,
                                  (hipStream_t)stream);
        if (e != hipSuccess) return hip_fail(e, "plain-form launch");
        return LEAD_OK;
    }
    // precompiled kernels (the schedule asks for them, or the code has none
    // compiled): min-sum without OSD
    if (needs_spec(d) || d->params.global_post)
        return fail(LEAD_E_UNSUPPORTED, "the plain form on the precompiled kernels runs min-sum without OSD only");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    const int D2 = d->D * d->D;
    if (!d->d_S) {
        const size_t ms = (size_t)std::max<int64_t>(d->max_shots, 1);
        e = hipMalloc(&d->d_S, sizeof(float) * ms * D2 * d->N);
        if (e == hipSuccess) e = hipMalloc(&d->d_cst, sizeof(float) * ms * d->r * 4 * d->N);
        if (e == hipSuccess) e = hipMalloc(&d->d_lamp, sizeof(float) * ms * d->n);
        if (e == hipSuccess) e = hipMalloc(&d->d_status, sizeof(int32_t) * ms * 4);
        if (e == hipSuccess) e = hipMalloc(&d->d_active, sizeof(int32_t));
        if (e == hipSuccess) e = hipHostMalloc(&d->h_active, sizeof(int32_t), hipHostMallocDefault);
        if (e != hipSuccess) {
            free_plain(d);
            return hip_fail(e, "plain-form workspace allocation");
        }
    }
    // Phases 1-2: lambda' to HBM (and to the caller's buffer if given)
    float *lam_hbm = lam ? lam : d->d_lamp;
    e = decode_chunks(d, shots, synd, synd_words, prior, mode, ehat, ehat_words, post, lam_hbm, stats,
                      LEAD_STAGE_LOCAL, s, decoder_workspace(d));
    if (e != hipSuccess) return hip_fail(e, "local-stage launch");
    lead::DecodeArgs a = base_args(d);
    a.synd = synd;
    a.synd_words = synd_words;
    a.prior = prior;
    a.prior_mode = mode;
    a.ehat = ehat;
    a.ehat_words = ehat_words;
    a.post = post;
    a.lam_out = lam_hbm;
    a.stats = stats;
    a.shots = shots;
    a.stage = LEAD_STAGE_FULL;
    lead::RoundArgs ra{};
    ra.d = a;
    ra.S = d->d_S;
    ra.cst = d->d_cst;
    ra.lamp = a.lam_out;
    ra.status = d->d_status;
    ra.active = d->d_active;
    ra.phase = 0;
    e = lead::launch_round(d->D, d->r, ra, s);
    if (e != hipSuccess) return hip_fail(e, "round launch");
    ra.phase = 1;
    for (int t = 1; t <= d->params.max_iter_global; ++t) {
        if ((e = hipMemsetAsync(d->d_active, 0, sizeof(int32_t), s)) != hipSuccess) return hip_fail(e, "memset");
        ra.round = t;
        if ((e = lead::launch_round(d->D, d->r, ra, s)) != hipSuccess) return hip_fail(e, "round launch");
        if ((e = hipMemcpyAsync(d->h_active, d->d_active, sizeof(int32_t), hipMemcpyDeviceToHost, s)) != hipSuccess)
            return hip_fail(e, "memcpy");
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "synchronize");
        if (*d->h_active == 0) break;
    }
    ra.phase = 2;
    if ((e = lead::launch_round(d->D, d->r, ra, s)) != hipSuccess) return hip_fail(e, "finalize launch");
    return LEAD_OK;
}

lead_status lead_batch_decode(const lead_batch_item *items, int32_t n, void *stream) {
    if (n < 0 || (n > 0 && !items)) return fail(LEAD_E_ARG, "bad item list");
    for (int i = 0; i < n; ++i) {
        lead_status st = check_item(items[i]);
        if (st != LEAD_OK) return fail(st, "item " + std::to_string(i) + ": " + g_err);
    }
    if (n == 0) return LEAD_OK;
    std::vector<int> group;
    const int ng = group_items(items, n, group);
    std::vector<hipStream_t> streams;
    hipError_t e = pool_streams(ng, streams);
    if (e != hipSuccess) return hip_fail(e, "stream creation");
    std::vector<hipEvent_t> events;
    lead_status st = enqueue_batch(items, n, (hipStream_t)stream, streams, group, ng, events);
    destroy_events(events);
    return st;
}

lead_status lead_batch_graph_create(const lead_batch_item *items, int32_t n, void *stream, lead_batch_graph **out) {
    if (!out || n < 0 || (n > 0 && !items)) return fail(LEAD_E_ARG, "bad argument");
    *out = nullptr;
    for (int i = 0; i < n; ++i) {
        lead_status st = check_item(items[i]);
        if (st != LEAD_OK) return fail(st, "item " + std::to_string(i) + ": " + g_err);
    }
    hipStream_t cap = nullptr;
    hipError_t e;
    std::vector<int> group;
    const int ng = group_items(items, n, group);
    std::vector<hipStream_t> streams;
    if ((e = pool_streams(ng, streams)) != hipSuccess) return hip_fail(e, "stream creation");
    // Capture on a private stream so the caller's stream never enters
    // capture mode.  Wait for the caller's prior work first (the graph's
    // launches are ordered on the launch stream).
    if ((e = hipStreamSynchronize((hipStream_t)stream)) != hipSuccess) return hip_fail(e, "synchronize");
    if ((e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking)) != hipSuccess) return hip_fail(e, "stream");
    std::unique_ptr<lead_batch_graph> g(new (std::nothrow) lead_batch_graph());
    if (!g) {
        (void)hipStreamDestroy(cap);
        return fail(LEAD_E_NOMEM, "out of host memory");
    }
    if ((e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal)) != hipSuccess) {
        (void)hipStreamDestroy(cap);
        return hip_fail(e, "begin capture");
    }
    std::vector<hipEvent_t> events;
    lead_status st = n > 0 ? enqueue_batch(items, n, cap, streams, group, ng, events) : LEAD_OK;
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(cap, &graph);
    destroy_events(events);
    (void)hipStreamDestroy(cap);
    if (st != LEAD_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    if (e != hipSuccess) return hip_fail(e, "end capture");
    g->graph = graph;
    if ((e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0)) != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return hip_fail(e, "graph instantiate");
    }
    *out = g.release();
    return LEAD_OK;
}

lead_status lead_batch_fused_create(const lead_batch_item *items, int32_t n, lead_batch_fused **out) {
    if (!out || n <= 0 || !items) return fail(LEAD_E_ARG, "bad argument");
    *out = nullptr;
    if (n > lead::kFusedMax)
        return fail(LEAD_E_UNSUPPORTED, "a fused batch holds at most " + std::to_string(lead::kFusedMax) + " requests");
    std::vector<lead::jit::FusedPart> parts;
    int device = -1;
    for (int i = 0; i < n; ++i) {
        const lead_batch_item &it = items[i];
        lead_status st = check_item(it);
        if (st != LEAD_OK) return fail(st, "item " + std::to_string(i) + ": " + g_err);
        if (it.shots <= 0) return fail(LEAD_E_ARG, "item " + std::to_string(i) + ": a fused request needs shots > 0");
        const lead_decoder *d = it.decoder;
        if (!use_spec(d))
            return fail(LEAD_E_UNSUPPORTED, "item " + std::to_string(i) + ": the fused batch runs the kernels compiled "
                                            "for the code (schedule specialized > 0, not fused)");
        if (d->params.local_post || d->params.global_post)
            return fail(LEAD_E_UNSUPPORTED, "item " + std::to_string(i) + ": OSD post-processing needs launches of its "
                                            "own; decode this request with lead_decode or lead_batch_decode");
        if (device < 0) device = d->device;
        if (d->device != device) return fail(LEAD_E_ARG, "the fused batch's decoders must share one device");
        parts.push_back(lead::jit::FusedPart{d->code, d->type, d->sched.specialized,
                                             it.mode == LEAD_PRIOR_PER_SHOT ? 0 : 1,
                                             use_tiles(d, d->sched.specialized - 1) &&
                                                 d->params.stage != LEAD_STAGE_LOCAL});
    }
    lead::jit::settle_fused_tiles(parts);
    std::string jerr;
    auto k = lead::jit::load_fused(parts, device, jerr);
    if (!k) return fail(LEAD_E_UNSUPPORTED, jerr);
    std::unique_ptr<lead_batch_fused> f(new (std::nothrow) lead_batch_fused());
    if (!f) return fail(LEAD_E_NOMEM, "out of host memory");
    f->k = k;
    f->n = n;
    auto cleanup = [&](lead_batch_fused *x) {
        for (void *b : x->bufs) (void)hipFree(b);
        (void)hipFree(x->counters);
    };
    hipError_t e = hipMalloc(&f->counters, sizeof(int64_t) * 4 * n);
    int64_t first = 0, items_total = 0;
    for (int i = 0; i < n && e == hipSuccess; ++i) {
        const lead_batch_item &it = items[i];
        lead_decoder *d = it.decoder;
        const int D2 = d->D * d->D;
        float *Lv = nullptr;
        uint32_t *vflag = nullptr;
        e = hipMalloc(&Lv, sizeof(float) * (size_t)it.shots * d->N * D2);
        if (e == hipSuccess) f->bufs.push_back(Lv);
        if (e == hipSuccess) e = hipMalloc(&vflag, sizeof(uint32_t) * (size_t)it.shots * d->N);
        if (e == hipSuccess) f->bufs.push_back(vflag);
        if (e != hipSuccess) break;
        lead::DecodeArgs a = base_args(d);
        a.synd = it.d_synd;
        a.synd_words = it.synd_words;
        a.prior = it.d_prior;
        a.prior_mode = it.mode;
        a.ehat = it.d_ehat;
        a.ehat_words = it.ehat_words;
        a.post = it.d_post;
        a.lam_out = it.d_prior_llr;
        a.stats = it.d_stats;
        a.shots = it.shots;
        a.stage = d->params.stage == LEAD_STAGE_LOCAL ? LEAD_STAGE_LOCAL : LEAD_STAGE_FULL;
        a.global_only = d->params.stage == LEAD_STAGE_GLOBAL ? 1 : 0;
        a.spw = k->spw[i];
        lead::LocalArgs w{};
        w.Lv = Lv;
        w.vflag = vflag;
        w.counter = f->counters + 4 * i;
        w.osd_list = nullptr;
        w.items = it.shots * d->N;
        w.chunk = d->sched.local_chunk;
        w.waves = 0;
        if (!a.global_only) items_total += w.items;
        f->args.it[i] = lead::FusedItem{a, w, lead::SpecArgs{d->d_pv, d->d_fown}};
        f->args.first[i] = first;
        if (k->tile_shots[i] > 0) {
            // persistent workgroups taking the request's shots from its
            // counter [3]: as many as hold them, at most one per compute unit
            const int64_t need = (it.shots + k->tile_shots[i] - 1) / k->tile_shots[i];
            first += std::max<int64_t>(1, std::min<int64_t>(need, d->cus));
        } else {
            const int64_t blocks = (it.shots + k->spw[i] - 1) / k->spw[i];
            first += (blocks + k->sub[i] - 1) / k->sub[i];
        }
    }
    if (e != hipSuccess) {
        cleanup(f.get());
        return hip_fail(e, "fused batch allocation");
    }
    for (int i = n; i <= lead::kFusedMax; ++i) f->args.first[i] = first;
    f->global_wgs = first;
    // Phase 1: as many waves as fit the device, at most one per 64 queue items
    const int cus = items[0].decoder->cus;
    f->local_waves = std::max<int64_t>(1, std::min<int64_t>((int64_t)k->local_waves_per_cu * cus, (items_total + 63) / 64));
    // the launch sequence, captured once: clear the queue counters (a fill
    // kernel), Phase 1 of every request, Phases 2-3 of every request
    hipStream_t cap = nullptr;
    e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t le = lead::launch_clear_i64(f->counters, 4 * n, cap);
        void *args[] = {&f->args};
        if (le == hipSuccess && items_total > 0)
            le = hipModuleLaunchKernel(k->local, (unsigned)f->local_waves, 1, 1, 64, 1, 1, (unsigned)k->local_lds, cap,
                                       args, nullptr);
        if (le == hipSuccess)
            le = hipModuleLaunchKernel(k->global, (unsigned)f->global_wgs, 1, 1, (unsigned)k->wg, 1, 1,
                                       (unsigned)k->lds_bytes, cap, args, nullptr);
        hipGraph_t graph = nullptr;
        e = hipStreamEndCapture(cap, &graph);
        if (e == hipSuccess && le != hipSuccess) e = le;
        f->graph = graph;
        if (e == hipSuccess) e = hipGraphInstantiate(&f->exec, graph, nullptr, nullptr, 0);
    }
    if (cap) (void)hipStreamDestroy(cap);
    if (e != hipSuccess) {
        if (f->exec) (void)hipGraphExecDestroy(f->exec);
        if (f->graph) (void)hipGraphDestroy(f->graph);
        cleanup(f.get());
        return hip_fail(e, "fused batch capture");
    }
    *out = f.release();
    return LEAD_OK;
}

lead_status lead_batch_fused_launch(lead_batch_fused *f, void *stream) {
    if (!f || !f->exec) return fail(LEAD_E_ARG, "fused batch is NULL");
    hipError_t e = hipGraphLaunch(f->exec, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "graph launch");
    return LEAD_OK;
}

void lead_batch_fused_destroy(lead_batch_fused *f) {
    if (!f) return;
    if (f->exec) (void)hipGraphExecDestroy(f->exec);
    if (f->graph) (void)hipGraphDestroy(f->graph);
    for (void *b : f->bufs) (void)hipFree(b);
    (void)hipFree(f->counters);
    delete f;
}

lead_status lead_batch_graph_launch(lead_batch_graph *g, void *stream) {
    if (!g || !g->exec) return fail(LEAD_E_ARG, "graph is NULL");
    hipError_t e = hipGraphLaunch(g->exec, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "graph launch");
    return LEAD_OK;
}

void lead_batch_graph_destroy(lead_batch_graph *g) {
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
}

lead_status lead_decoder_autotune(lead_decoder *d, int64_t shots, const uint64_t *synd, int64_t synd_words,
                                  const float *prior, lead_prior_mode mode, void *stream, lead_schedule *best) {
    lead_status st = check_decode_args(d, shots, synd, synd_words, prior, mode, nullptr, 0, nullptr);
    if (st != LEAD_OK) return st;
    if (shots == 0) return fail(LEAD_E_ARG, "autotune needs shots > 0");
    const int64_t n = std::min<int64_t>(shots, 16384);
    hipStream_t s = (hipStream_t)stream;
    const int ew = (d->n + 63) / 64;
    uint64_t *ehat = nullptr;
    float *post = nullptr, *lam = nullptr;
    lead_shot_stats *stats = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMalloc(&ehat, sizeof(uint64_t) * n * ew);
    if (e == hipSuccess) e = hipMalloc(&post, sizeof(float) * n * d->n);
    if (e == hipSuccess) e = hipMalloc(&lam, sizeof(float) * n * d->n);
    if (e == hipSuccess) e = hipMalloc(&stats, sizeof(lead_shot_stats) * n);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    const lead_schedule saved = d->sched;
    lead_schedule win = saved;
    float best_ms = 1e30f;
    if (e == hipSuccess) {
        std::vector<lead_schedule> cand;
        for (int fused = 0; fused < 2 && !needs_spec(d); ++fused)
            for (int spw : {1, 2, 4, 8, 16, 21})
                for (int chunk : {64, 256, 1024}) {
                    if (fused && chunk != 256) continue;
                    if (lead::workgroup_size(d->N, spw) > lead::kMaxWorkgroup) continue;
                    if (lead::decode_lds_bytes(d->D, lead::workgroup_size(d->N, spw), spw, d->n) > 65536) continue;
                    cand.push_back(lead_schedule{spw, fused, chunk, 0, 0, 0, saved.global_osd_form, saved.global_tiles});
                }
        // the specialised split kernels fix their own workgroup shape
        for (int form : {lead::jit::kCompressed, lead::jit::kExplicit, lead::jit::kSumProduct})
            if (d->spec && d->spec->has[form - 1])
                for (int chunk : {64, 256, 1024})
                    cand.push_back(lead_schedule{saved.shots_per_workgroup, 0, chunk, 0, form, 0, saved.global_osd_form,
                                                 saved.global_tiles});
        for (const lead_schedule &c : cand) {
            if (lead_decoder_set_schedule(d, &c) != LEAD_OK) continue;
            float ms_best = 1e30f;
            for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {
                e = hipEventRecord(e0, s);
                if (e == hipSuccess)
                    e = decode_chunks(d, n, synd, synd_words, prior, mode, ehat, ew, post,
                                      d->params.stage == LEAD_STAGE_LOCAL ? lam : nullptr, stats, d->params.stage, s,
                                      decoder_workspace(d));
                if (e == hipSuccess) e = hipEventRecord(e1, s);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                float ms = 0.f;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                if (e == hipSuccess && rep > 0) ms_best = std::min(ms_best, ms);
            }
            if (e != hipSuccess) break;
            if (ms_best < best_ms) {
                best_ms = ms_best;
                win = d->sched;
            }
        }
    }
    (void)hipFree(ehat);
    (void)hipFree(post);
    (void)hipFree(lam);
    (void)hipFree(stats);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e != hipSuccess) {
        d->sched = saved;
        d->spw = saved.shots_per_workgroup;
        return hip_fail(e, "autotune");
    }
    d->sched = win;
    d->spw = win.shots_per_workgroup;
    if (best) (void)lead_decoder_get_schedule(d, best);   // as get_schedule reports it
    return LEAD_OK;
}

lead_status lead_syndrome(const lead_decoder *d, int64_t shots, const uint64_t *err, int64_t err_words,
                          uint64_t *synd, int64_t synd_words, void *stream) {
    if (!d || shots < 0) return fail(LEAD_E_ARG, "bad argument");
    if (shots == 0) return LEAD_OK;
    if (!err || !synd) return fail(LEAD_E_ARG, "NULL buffer");
    if (err_words < (d->n + 63) / 64 || synd_words < (d->m + 63) / 64) return fail(LEAD_E_ARG, "row too short");
    lead::SyndArgs a{};
    a.err = err;
    a.synd = synd;
    a.view = d->d_view;
    a.shots = shots;
    a.err_words = err_words;
    a.synd_words = synd_words;
    a.N = d->N;
    a.D2 = d->D * d->D;
    a.r = d->r;
    a.m = d->m;
    for (int c = 0; c < lead::kMaxChecks; ++c) a.mask[c] = c < d->r ? d->mask[c] : 0;
    hipError_t e = lead::launch_syndrome(a, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "syndrome launch");
    return LEAD_OK;
}

}  // extern "C"
