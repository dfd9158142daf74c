// Kernels compiled at run time for the local check structure of one code.
//
// The check masks and the local position map of a code become compile-time
// constants of lead_spec.hpp's kernels (hipRTC, gfx950).  Code objects are
// cached per process by source text and on disk (keyed by compiler, headers
// and source; $LEAD_JIT_CACHE, else _build/jit beside the library), modules
// per device; neither is ever unloaded.
#pragma once
#include <hip/hip_runtime.h>

#include <memory>
#include <string>
#include <vector>

#include "code_build.hpp"

namespace lead {
namespace jit {

// Check-state forms of the specialised kernels (lead_schedule.specialized):
// min-sum with the compressed state or one register per message, and
// sum-product (one register per message).
enum Form { kCompressed = 1, kExplicit = 2, kSumProduct = 3 };
constexpr int kForms = 3;

// Views with at most this many local edges also get the explicit-message
// min-sum form (one VGPR per message), and at most kSumProductMaxEdges the
// sum-product form.
constexpr int kExplicitMaxEdges = 192;
constexpr int kSumProductMaxEdges = 192;
// Up to this many edges the explicit forms' per-shot kernel keeps one
// register per message; above it, the min-sum per-shot kernel keeps the
// compressed state on the checks of highest degree, leaving at most
// kHybridExplicitEdges messages in registers.  Either way it is held to two
// waves per SIMD (256 VGPRs).
constexpr int kTwoWaveMaxEdges = 128;
// The Phase 1 queue kernel runs three waves per SIMD where a view's check
// state and sums take at most this many registers.
constexpr int kThreeWaveMaxState = 96;
// Views above kTwoWaveMaxEdges edges: the Phase 1 queue kernel of form 2
// keeps the messages of its lowest-degree checks in LDS, so that at most
// this many stay in registers and it runs two waves per SIMD.
constexpr int kLocalRegEdges = 96;
// ... at most kLocalAltRegEdges where the LDS that then takes (64 lanes per
// wave) lets eight waves share a CU's 160 KB: the kernel then runs its
// iterations in pairs, the first without the fixed-point comparison (more
// live registers than one iteration per pass).
constexpr int kLocalAltRegEdges = 80;
constexpr int kLocalAltLdsBytes = 20 * 1024;
// The checks (bit c) whose messages that kernel keeps in LDS, and their
// edges; whether it runs its iterations in pairs (LOCAL_ALT of the code
// struct).
uint32_t local_lds_mask(const TypeTables &tt);
int local_lds_edges(const TypeTables &tt);
bool local_alt(const TypeTables &tt);
constexpr int kHybridExplicitEdges = 72;

// The persistent Phases 2-3 kernel (lead_spec::global_tile_body) for codes
// whose views span several waves: compiled, for the min-sum forms, where a
// workgroup of lead::kTileWG lanes holds at least two shots and its LDS
// (exchange rows, lambda' rows, partner tables, per-slot words and e_hat
// bitmaps) fits the compute unit's 160 KB.
bool tile_fits(const Code &c, int t);
size_t tile_lds_bytes(const Code &c, int t);

// The global OSD-0 kernel keeps ceil(m/256) rows of ceil(n/64) words per lane
// in registers; it is compiled when that product is at most this.
constexpr int kOsdMaxWords = 64;
bool osd_fits(const Code &c, int t);
// Workgroup size of that kernel: the fewest whole waves that hold the m rows
// at ceil(m/256) rows per lane.
int osd_workgroup(const Code &c, int t);

// The global OSD kernel with [H_t | s] in device memory (any code with at
// most kOsdBigMaxRows rows and 65535 qubits): its workgroup size (the fewest
// whole waves, at most 512 lanes so that 256 VGPRs are available, holding
// the rows at ceil(m/512) rows per lane; its LDS admits one workgroup per CU
// for PSL(2,7) anyway) and the bytes of one matrix slot ((ceil(n/64) + 1) * m
// words).
constexpr int kOsdBigMaxRows = 32 * 512;
bool osd_big_fits(const Code &c, int t);
int osd_big_workgroup(const Code &c, int t);
size_t osd_big_slot_bytes(const Code &c, int t);

struct Kernels {
    hipModule_t module = nullptr;
    // [form - 1][prior mode]: Phase 1 queue kernel for per-shot / per-qubit priors
    hipFunction_t local[kForms][2] = {};
    hipFunction_t global[kForms] = {};   // [form - 1]: Phases 2-3
    hipFunction_t round[kForms] = {};    // [form - 1]: one global round (plain form)
    hipFunction_t tile[kForms] = {};     // [form - 1]: persistent Phases 2-3 (views over several waves)
    // [form - 1]: `global` / `tile` without the fixed-point test of global
    // BP (no per-message comparison; compiled for the explicit form, the
    // per-shot one only where `tile` is not, and for sum-product)
    hipFunction_t global_nf[kForms] = {};
    hipFunction_t tile_nf[kForms] = {};
    int tile_shots = 0;                  // shots per workgroup of `tile`
    size_t tile_lds = 0;                 // its LDS bytes
    hipFunction_t local_osd = nullptr;   // OSD-0 on the views listed by the queue kernel
    hipFunction_t osd = nullptr;         // OSD-0 on H_t after global BP (when it fits)
    hipFunction_t osd_cs = nullptr;      // the same with the combination sweep
    int osd_wg = 0;                      // its workgroup size
    hipFunction_t osd_big = nullptr;     // global OSD-0 with [H_t | s] in device memory
    hipFunction_t osd_big_cs = nullptr;  // the same with the combination sweep
    int osd_big_wg = 0;                  // their workgroup size
    bool has[kForms] = {};               // [form - 1]: compiled
    int wg = 0;                          // workgroup size of `global`
    int spw = 0;                         // shots per workgroup of `global`
    bool bperm = false;                  // partner values exchanged within the wave
    int lam_slots = 0;                   // across waves: lambda' slots per lane in LDS
                                         // (form 1, and form 2 with the mixed state)
    bool hybrid = false;                 // form 2 keeps the mixed check state
    int local_waves_per_cu[kForms][2] = {{4, 4}, {4, 4}, {4, 4}};
    size_t local_lds[kForms][2] = {};    // [form - 1][prior mode]: LDS bytes of `local` (messages kept in LDS)
    int best_form() const { return has[2] ? kSumProduct : has[1] ? kExplicit : kCompressed; }
};

// Source text of the kernels for check type t of code c: the min-sum forms,
// or (sp) the sum-product form; empty when the code has no local position map
// (the precompiled kernels serve min-sum) or, for sum-product, when a view
// has more than kSumProductMaxEdges edges.
std::string source(const Code &c, int t, bool sp = false);

// Code object of `src` for gfx950 (compiled once per process, or read from
// the disk cache).  Needs no GPU.
bool compile(const std::string &src, std::vector<char> &obj, std::string &err);

// Kernels of check type t of code c on the current device (device index
// `device`), compiled and loaded on first use.
std::shared_ptr<const Kernels> load(const Code &c, int t, int device, bool sp, std::string &err);

// One request of a fused multi-code module: its code, check type, kernel
// form, prior mode (0 per shot, 1 per qubit) and whether it runs Phase 1.
struct FusedPart {
    const Code *code;
    int t, form, pm;
    bool tiles;   // Phases 2-3 as the persistent kernel (lead_spec::global_tile_body)
};
// Kernels of a fused module: the Phase 1 kernel (64-lane workgroups; each
// wave drains the queues of the requests in order) and the Phases 2-3
// kernel (workgroups of `wg` lanes, each running sub[k] per-shot blocks of
// request k, with lds_words[k] floats of LDS per block, or, where
// tile_shots[k] > 0, persistent workgroups of request k holding that many
// shots each; those make wg = lead::kTileWG).
struct FusedKernels {
    hipModule_t module = nullptr;
    hipFunction_t local = nullptr, global = nullptr;
    int wg = 64;
    std::vector<int> sub, lds_words, spw, tile_shots;
    size_t local_lds = 0;   // LDS bytes of `local` (the largest of the parts')
    int local_waves_per_cu = 1;
    size_t lds_bytes = 0;
};
// The persistent kernel for the parts that ask for it (tiles), if the module
// can run it: every other part's per-shot workgroup divides lead::kTileWG
// and none needs the whole register file; otherwise no part uses it.
void settle_fused_tiles(std::vector<FusedPart> &parts);
// Source and kernels of the fused module of `parts` (at most
// lead::kFusedMax), compiled and loaded on first use; nullptr with the
// reason in err when a part has no compiled kernels of its form.
std::shared_ptr<const FusedKernels> load_fused(const std::vector<FusedPart> &parts, int device, std::string &err);
// The fused module's source, with its launch shape filled into `k` (no
// compilation, no device).  Empty with the reason in err when unsupported.
std::string fused_source(const std::vector<FusedPart> &parts, FusedKernels &k, std::string &err);

// Words of check state per view the plain per-round kernels save between
// launches, at most (an upper bound over the forms): E + 4 r.
int plain_state_words(const Code &c, int t);

// Partner tables of lead::SpecArgs for check type t: pv (order * ceil(D2/2)
// words) and fown (order words).
void partner_tables(const Code &c, int t, std::vector<uint32_t> &pv, std::vector<uint64_t> &fown);

}  // namespace jit
}  // namespace lead
