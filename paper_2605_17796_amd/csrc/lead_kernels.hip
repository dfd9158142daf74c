// LEAD decoding kernels for gfx950 (CDNA4).
//
// Mapping.  One workgroup decodes `spw` shots; lane v of a shot holds the
// local view of vertex v (the Delta^2 qubits of Q(v), Sec. II-B).  Phase 1 of
// Algorithm 1 (local BP on the view) runs entirely inside the lane: the check
// states live in VGPRs (a compressed min-sum state per check: smallest and
// second-smallest |mu|, position of the smallest, and the sign of every
// outgoing message), and the variable sums S_j of the view live in LDS at
// buf[j * WG + lane] (WG the compile-time workgroup size), so every access of the uniform edge loop is
// conflict-free.  The check masks are kernel arguments (scalar registers), so
// the edge loops are uniform scalar loops.
//
// Phase 2 (alpha-regularised aggregation) and Phase 3 (global BP with the
// aggregated prior) couple the two views of each qubit through LDS.  Every
// qubit is owned by one of its two occurrences (decided on the host, at most
// ceil(Delta^2/2) per view); the owner computes
// the shared quantities and writes them to both occurrences, so no two lanes
// ever touch the same LDS word between barriers.
//
// A global check is a local check of one vertex (the global check matrix is
// the union of the placed local matrices), so the global check update is the
// same per-lane routine as the local one; only the variable update differs:
// S_i = lambda'_i + (messages of the owner's checks) + (messages of the
// partner's checks).
#include "lead_kernels.hpp"

namespace lead {
namespace {

using namespace lead_dev;

// Compressed min-sum state of the checks of one vertex: beta * smallest and
// beta * second-smallest |mu|, edge position of the smallest, and the sign
// bit of every outgoing message.
template <int RMAX>
struct CheckState {
    float m1[RMAX], m2[RMAX];
    uint32_t am[RMAX], q[RMAX];
    __device__ __forceinline__ void clear() {
#pragma unroll
        for (int c = 0; c < RMAX; ++c) { m1[c] = 0.f; m2[c] = 0.f; am[c] = 0u; q[c] = 0u; }
    }
};

// Check update of every check of the lane's vertex.  Reads S_j (the variable
// sums of the previous iteration), forms mu_{j->c} = clamp(S_j - m_{c->j}),
// and replaces each check state by the min-sum state of the new messages
//   m_{c->j} = beta (-1)^{s_c} prod_{j' != j} sgn(mu_{j'}) min_{j' != j} |mu_{j'}|.
// Returns whether the hard decisions [S_j < 0] satisfy every check, and sets
// `same` when every new message equals the previous one bit for bit (the
// messages are then a fixed point of the iteration: the next variable sums
// equal the current ones, and so on).
template <int WG, int RMAX>
__device__ __forceinline__ bool check_pass(const DecodeArgs &a, const float *bl, uint64_t sv,
                                           CheckState<RMAX> &st, bool &same) {
    bool sat = true;
    same = true;
#pragma unroll
    for (int c = 0; c < RMAX; ++c) {
        if (c < a.r) {
            uint64_t mk = a.mask[c];
            float n1 = kBig, n2 = kBig;
            uint32_t nam = 0u, sg = 0u, par = 0u, k = 0u;
            while (mk) {
                const int j = __builtin_ctzll(mk);
                mk &= mk - 1;
                const float S = bl[j * WG];
                par ^= __float_as_uint(S);
                const float mu = clampf(S - msg_of(st.m1[c], st.m2[c], st.am[c], st.q[c], k), a.clampv);
                const float ab = fabsf(mu);
                sg |= signbit_of(mu) << k;
                n2 = __builtin_amdgcn_fmed3f(n1, n2, ab);
                const bool lt = ab < n1;
                nam = lt ? k : nam;
                n1 = lt ? ab : n1;
                ++k;
            }
            const uint32_t sc = (uint32_t)(sv >> c) & 1u;
            sat = sat && ((par >> 31) == sc);
            const uint32_t flip = ((uint32_t)__popc(sg) & 1u) ^ sc;
            const uint32_t all = (uint32_t)((1ull << k) - 1ull);
            const uint32_t nq = flip ? (sg ^ all) : sg;
            const float b1 = a.beta * n1, b2 = a.beta * n2;
            // every outgoing message unchanged (the position of the smallest
            // matters only when the two magnitudes differ)
            same = same && nq == st.q[c] && __float_as_uint(b1) == __float_as_uint(st.m1[c]) &&
                   __float_as_uint(b2) == __float_as_uint(st.m2[c]) &&
                   (nam == st.am[c] || __float_as_uint(b1) == __float_as_uint(b2));
            st.q[c] = nq;
            st.m1[c] = b1;
            st.m2[c] = b2;
            st.am[c] = nam;
        }
    }
    return sat;
}

template <int WG, int RMAX>
__device__ __forceinline__ bool parity_pass(const DecodeArgs &a, const float *bl, uint64_t sv) {
    bool sat = true;
#pragma unroll
    for (int c = 0; c < RMAX; ++c) {
        if (c < a.r) {
            uint64_t mk = a.mask[c];
            uint32_t par = 0u;
            while (mk) {
                const int j = __builtin_ctzll(mk);
                mk &= mk - 1;
                par ^= __float_as_uint(bl[j * WG]);
            }
            sat = sat && ((par >> 31) == ((uint32_t)(sv >> c) & 1u));
        }
    }
    return sat;
}

// S_j += m_{c->j} over the lane's checks, in check order.
template <int WG, int RMAX>
__device__ __forceinline__ void accumulate(const DecodeArgs &a, float *bl, const CheckState<RMAX> &st) {
#pragma unroll
    for (int c = 0; c < RMAX; ++c) {
        if (c < a.r) {
            uint64_t mk = a.mask[c];
            uint32_t k = 0u;
            while (mk) {
                const int j = __builtin_ctzll(mk);
                mk &= mk - 1;
                bl[j * WG] += msg_of(st.m1[c], st.m2[c], st.am[c], st.q[c], k);
                ++k;
            }
        }
    }
}

struct Lane {
    int tid, sl, v;
    bool lane_ok, live;
    int64_t shot;
};

__device__ __forceinline__ Lane lane_of(const DecodeArgs &a, int64_t shot_base) {
    Lane L;
    L.tid = threadIdx.x;
    L.sl = L.tid / a.N;
    L.v = L.tid - L.sl * a.N;
    L.lane_ok = L.sl < a.spw;
    L.shot = shot_base + L.sl;
    L.live = L.lane_ok && L.shot < a.shots;
    return L;
}

// r syndrome bits of vertex v: bits v*r .. v*r + r - 1 of the shot's row.
__device__ __forceinline__ uint64_t local_syndrome(const DecodeArgs &a, int64_t shot, int v) {
    const uint64_t *row = a.synd + shot * a.synd_words;
    const int b0 = v * a.r;
    const int w0 = b0 >> 6, off = b0 & 63;
    uint64_t x = row[w0] >> off;
    if (off + a.r > 64) x |= row[w0 + 1] << (64 - off);
    return (a.r >= 64) ? x : (x & ((1ull << a.r) - 1ull));
}

// Owned-qubit entry k of a lane: LDS word offsets of its two occurrences.
template <int WG>
__device__ __forceinline__ void occurrences(uint32_t e, const Lane &L, int N, int &own, int &other) {
    own = (int)(e & 0xffu) * WG + L.tid;
    other = (int)((e >> 8) & 0xffu) * WG + L.sl * N + (int)(e >> 16);
}

// LDS layout of the fused kernel:
//   buf   float [D2][WG]    variable sums / exchanged values
//   convf int   [WG]        local convergence of each lane's view
//   shf   int   [spw][8]    per shot: unsat flags (2), final flag, it_sum, it_max, n_conv,
//                           changed flag, local fixed-point count
//   ebits u32   [spw][ew32] packed hard decisions
enum { SF_FLAG0 = 0, SF_FLAG1 = 1, SF_FINAL = 2, SF_ITSUM = 3, SF_ITMAX = 4, SF_NCONV = 5, SF_CHG = 6, SF_NFIX = 7 };

// Priors of the lane's view: one per shot (PM = 0) or one per qubit (PM = 1,
// SHARED or FULL).  "+ 0.f" maps a -0 prior to +0.
template <int D, int PM>
__device__ __forceinline__ void load_priors(const DecodeArgs &a, int64_t shot, int v, float (&lamv)[PM == 0 ? 1 : D * D]) {
    constexpr int D2 = D * D;
    if (PM == 0) {
        lamv[0] = a.prior[shot] + 0.f;
    } else {
        const int64_t base = a.prior_mode == LEAD_PRIOR_FULL ? shot * a.n : 0;
#pragma unroll
        for (int j = 0; j < (PM == 0 ? 1 : D2); ++j) lamv[j] = a.prior[base + a.view[v * D2 + j]] + 0.f;
    }
}

// One step of the local BP run of a view (Phase 1): the check update of
// iteration t (which also tests S^{t-1}) and, unless the run ends, the
// variable update S^t.  A run ends at the first t > 1 whose S^{t-1} satisfies
// the local syndrome (early exit), when the messages stop changing (a fixed
// point: every later iteration repeats S^{t-1}; tested at even t), or at
// t = Tl + 1 (the cap,
// where the test is the final syndrome test).  On return `fin` tells whether
// the run ended; conv, it, fixed describe it.
template <int D, int RMAX, int WG, int PM>
__device__ __forceinline__ bool local_step(const DecodeArgs &a, float *bl, uint64_t sv, const float (&lamv)[PM == 0 ? 1 : D * D],
                                           CheckState<RMAX> &st, int t, int &conv, int &it, int &fixed) {
    constexpr int D2 = D * D;
    bool same;
    const bool sat = check_pass<WG, RMAX>(a, bl, sv, st, same);
    if (t > a.Tl) {
        conv = sat ? 1 : 0;
        it = a.Tl;
        return true;
    }
    if (t > 1 && sat && a.early_exit) {
        conv = 1;
        it = t - 1;
        return true;
    }
    if ((t & 1) == 0 && same && a.fixed_stop) {   // tested at even t, as in the compiled kernels
        conv = sat ? 1 : 0;
        it = a.Tl;
        fixed = 1;
        return true;
    }
#pragma unroll
    for (int j = 0; j < D2; ++j) bl[j * WG] = lamv[PM == 0 ? 0 : j];
    accumulate<WG, RMAX>(a, bl, st);
    return false;
}

// Phase 1 as its own kernel: every lane of a 64-lane wave runs the local BP
// of one (shot, vertex) item at a time and takes the next item from the
// queue as soon as its run ends, so a wave is never held by its slowest
// view.  Items are numbered shot * N + v; waves take chunks of them from a
// global counter.  Outputs per item: the clamped local posteriors
// (w.Lv[item][j]) and w.vflag[item] = iterations | converged << 16 |
// fixed point << 17.
template <int D, int RMAX, int PM>
__global__ void __launch_bounds__(64) local_kernel(DecodeArgs a, LocalArgs w) {
    constexpr int D2 = D * D;
    constexpr int WG = 64;
    extern __shared__ float lds[];
    const int lane = threadIdx.x;
    float *bl = lds + lane;
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int64_t cur = 0, end = 0;
    bool queue_open = true, valid = false;
    int64_t item = 0;
    int t = 0;
    uint64_t sv = 0;
    float lamv[PM == 0 ? 1 : D2];
#pragma unroll
    for (int j = 0; j < (PM == 0 ? 1 : D2); ++j) lamv[j] = 0.f;
    CheckState<RMAX> st;
    st.clear();
    for (;;) {
        // hand the next items to lanes without a view, in lane order
        uint64_t need = __ballot(!valid);
        while (need && queue_open) {
            if (cur >= end) {
                unsigned long long c0 = 0;
                if (lane == 0) c0 = atomicAdd(reinterpret_cast<unsigned long long *>(w.counter),
                                              (unsigned long long)w.chunk);
                c0 = __shfl(c0, 0);
                if ((int64_t)c0 >= w.items) {
                    queue_open = false;
                    break;
                }
                cur = (int64_t)c0;
                end = cur + w.chunk < w.items ? cur + w.chunk : w.items;
            }
            const int rank = __popcll(need & below);
            const int64_t avail = end - cur;
            if (!valid && rank < avail) {
                item = cur + rank;
                valid = true;
                const int64_t shot = item / a.N;
                const int v = (int)(item - shot * a.N);
                sv = local_syndrome(a, shot, v);
                load_priors<D, PM>(a, shot, v, lamv);
                st.clear();
#pragma unroll
                for (int j = 0; j < D2; ++j) bl[j * WG] = lamv[PM == 0 ? 0 : j];
                t = 1;
            }
            const int64_t taken = __popcll(need) < avail ? __popcll(need) : avail;
            cur += taken;
            need = __ballot(!valid);
        }
        if (__ballot(valid) == 0ull) break;
        if (valid) {
            int conv = 0, it = 0, fixed = 0;
            if (local_step<D, RMAX, WG, PM>(a, bl, sv, lamv, st, t, conv, it, fixed)) {
                float *out = w.Lv + item * D2;
#pragma unroll
                for (int j = 0; j < D2; ++j) out[j] = clampf(bl[j * WG], a.clampv);
                w.vflag[item] = (uint32_t)it | ((uint32_t)conv << 16) | ((uint32_t)fixed << 17);
                valid = false;
            } else {
                ++t;
            }
        }
    }
}

// Work queue reset before a local_kernel launch (a kernel rather than a
// memset, so that the launch sequence can be captured in a graph).
__global__ void clear_i64_kernel(int64_t *p, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

__global__ void reset_counter_kernel(int64_t *counter) {
    counter[0] = 0;   // work-queue head
    counter[1] = 0;   // local OSD-0 list
    counter[3] = 0;   // next shot of the persistent Phases 2-3 kernel
}

// Phases 2-3 of a shot group (and, for SPLIT = false, Phase 1 as well: every
// lane runs its view's local BP in place, and the wave waits for its slowest
// view).  One workgroup decodes spw shots; lane v holds vertex v.
template <int D, int RMAX, int WG, int PM, bool SPLIT>
__global__ void __launch_bounds__(WG) decode_kernel(DecodeArgs a, LocalArgs w) {
    constexpr int D2 = D * D;
    constexpr int OWN = (D2 + 1) / 2;
    extern __shared__ float lds[];
    const Lane L = lane_of(a, (int64_t)blockIdx.x * a.spw);
    const int tid = L.tid;
    float *buf = lds;
    int *convf = reinterpret_cast<int *>(buf + D2 * WG);
    int *shf = convf + WG;
    const int ew32 = (a.n + 31) >> 5;
    uint32_t *ebits = reinterpret_cast<uint32_t *>(shf + a.spw * 8);
    for (int i = tid; i < a.spw * 8; i += WG) shf[i] = 0;
    for (int i = tid; i < a.spw * ew32; i += WG) ebits[i] = 0u;
    float *bl = buf + tid;

    // ---- Phase 1: local BP on the view of vertex v --------------------------
    uint64_t sv = 0;
    int it_v = 0, conv_v = 0, fixed_v = 0;
    if (L.live) sv = local_syndrome(a, L.shot, L.v);
    if (SPLIT) {
        // outputs of local_kernel
        if (L.live) {
            const int64_t item = L.shot * a.N + L.v;
            const float *in = w.Lv + item * D2;
#pragma unroll
            for (int j = 0; j < D2; ++j) bl[j * WG] = in[j];
            const uint32_t f = w.vflag[item];
            it_v = (int)(f & 0xffffu);
            conv_v = (int)((f >> 16) & 1u);
            fixed_v = (int)((f >> 17) & 1u);
        }
    } else if (!a.global_only) {
        float lamv[PM == 0 ? 1 : D2];
#pragma unroll
        for (int j = 0; j < (PM == 0 ? 1 : D2); ++j) lamv[j] = 0.f;
        if (L.live) load_priors<D, PM>(a, L.shot, L.v, lamv);
        CheckState<RMAX> st;
        st.clear();
#pragma unroll
        for (int j = 0; j < D2; ++j) bl[j * WG] = lamv[PM == 0 ? 0 : j];
        if (L.live)
            for (int t = 1;; ++t)
                if (local_step<D, RMAX, WG, PM>(a, bl, sv, lamv, st, t, conv_v, it_v, fixed_v)) break;
    } else {
#pragma unroll
        for (int j = 0; j < D2; ++j) bl[j * WG] = 0.f;   // no local posteriors
    }
    convf[tid] = conv_v;
    __syncthreads();
    if (L.live) {
        atomicAdd(&shf[L.sl * 8 + SF_ITSUM], it_v);
        atomicMax(&shf[L.sl * 8 + SF_ITMAX], it_v);
        atomicAdd(&shf[L.sl * 8 + SF_NCONV], conv_v);
        if (fixed_v) atomicAdd(&shf[L.sl * 8 + SF_NFIX], 1);
    }
    CheckState<RMAX> st;

    // ---- Phase 2: regularised aggregation of the owned qubits, after the
    // confidence boost (aggregate_llr) ----------------------------------------
    uint32_t ent[OWN];
    float lamp[OWN];
#pragma unroll
    for (int k = 0; k < OWN; ++k) {
        ent[k] = (L.live && k < a.own_max) ? a.own[L.v * a.own_max + k] : kNoOwn;
        lamp[k] = 0.f;
        if (ent[k] != kNoOwn) {
            int oa, ob;
            occurrences<WG>(ent[k], L, a.N, oa, ob);
            float La = clampf(buf[oa], a.clampv);
            float Lb = clampf(buf[ob], a.clampv);
            if (a.boost) {
                // p <- max(p, 0.5) on bits a locally consistent view decided
                // as errors; in LLR form L <- min(L, 0) where L < 0.
                if (conv_v && La < 0.f) La = fminf(La, 0.f);
                if (convf[ob % WG] && Lb < 0.f) Lb = fminf(Lb, 0.f);
            }
            lamp[k] = aggregate_llr(La, Lb, a.alpha, a.clampv);
            if (!SPLIT && a.global_only) {
                // global BP alone: the channel prior of the qubit
                const int64_t base = a.prior_mode == LEAD_PRIOR_FULL ? L.shot * a.n : 0;
                lamp[k] = (PM == 0 ? a.prior[L.shot] : a.prior[base + a.view[L.v * D2 + (ent[k] & 0xff)]]) + 0.f;
            }
        }
    }
    if (a.lam_out) {
#pragma unroll
        for (int k = 0; k < OWN; ++k)
            if (ent[k] != kNoOwn) a.lam_out[L.shot * a.n + a.view[L.v * D2 + (ent[k] & 0xff)]] = lamp[k];
    }
    if (a.stage == LEAD_STAGE_LOCAL) {
        __syncthreads();
        if (L.live && L.v == 0 && a.stats) {
            ShotStats s = {};
            s.local_iters_sum = shf[L.sl * 8 + SF_ITSUM];
            s.local_iters_max = shf[L.sl * 8 + SF_ITMAX];
            s.local_converged_views = shf[L.sl * 8 + SF_NCONV];
            s.local_fixed_views = shf[L.sl * 8 + SF_NFIX];
            reinterpret_cast<ShotStats *>(a.stats)[L.shot] = s;
        }
        return;
    }

    // ---- Phase 3: global BP with prior lambda' ------------------------------
    // S_i <- lambda'_i on both occurrences (no messages yet).  Each owned pair
    // is read above and written here by its owner only.
#pragma unroll
    for (int k = 0; k < OWN; ++k)
        if (ent[k] != kNoOwn) {
            int oa, ob;
            occurrences<WG>(ent[k], L, a.N, oa, ob);
            buf[oa] = lamp[k];
            buf[ob] = lamp[k];
        }
    st.clear();
    __syncthreads();
    bool done = !L.live;
    int itg = 0, gconv = 0, gfix = 0;
    for (int t = 1; t <= a.Tg; ++t) {
        // The owner entries are re-materialised every iteration, so the
        // compiler recomputes their LDS offsets (a few VALU ops) instead of
        // keeping 2 * OWN precomputed offsets live across the loop.
#pragma unroll
        for (int k = 0; k < OWN; ++k) asm volatile("" : "+v"(ent[k]));
        bool sat = true, same = true;
        if (!done) sat = check_pass<WG, RMAX>(a, bl, sv, st, same);
        if (!done && !sat) shf[L.sl * 8 + (t & 1)] = 1;
        if (!done && !same) shf[L.sl * 8 + SF_CHG] = t;
        __syncthreads();
        if (!done && t > 1) {
            const bool shot_sat = shf[L.sl * 8 + (t & 1)] == 0;
            if (shot_sat && a.early_exit) {
                done = true;
                gconv = 1;
                itg = t - 1;
            } else if (a.fixed_stop_g && shf[L.sl * 8 + SF_CHG] != t) {
                // no check state of the shot changed: S stays S^{t-1} for
                // every remaining iteration
                done = true;
                gconv = shot_sat ? 1 : 0;
                itg = a.Tg;
                gfix = t;
            }
        }
        if (!__syncthreads_or(done ? 0 : 1)) break;
        if (L.lane_ok && L.v == 0) shf[L.sl * 8 + ((t + 1) & 1)] = 0;
        if (!done) {
            // partial sums of this view: lambda' on owned occurrences, then
            // the messages of this vertex's checks
#pragma unroll
            for (int j = 0; j < D2; ++j) bl[j * WG] = 0.f;
#pragma unroll
            for (int k = 0; k < OWN; ++k)
                if (ent[k] != kNoOwn) bl[(ent[k] & 0xff) * WG] = lamp[k];
            accumulate<WG, RMAX>(a, bl, st);
        }
        __syncthreads();
        if (!done) {
#pragma unroll
            for (int k = 0; k < OWN; ++k)
                if (ent[k] != kNoOwn) {
                    int oa, ob;
                    occurrences<WG>(ent[k], L, a.N, oa, ob);
                    const float s = buf[oa] + buf[ob];
                    buf[oa] = s;
                    buf[ob] = s;
                }
        }
        __syncthreads();
    }
    const bool ran_out = !done;
    if (ran_out && !parity_pass<WG, RMAX>(a, bl, sv)) shf[L.sl * 8 + SF_FINAL] = 1;
    __syncthreads();
    if (ran_out) {
        gconv = shf[L.sl * 8 + SF_FINAL] == 0 ? 1 : 0;
        itg = a.Tg;
    }

    // ---- outputs ------------------------------------------------------------
    if (L.live) {
#pragma unroll
        for (int k = 0; k < OWN; ++k)
            if (ent[k] != kNoOwn) {
                const int j = ent[k] & 0xff;
                const float S = buf[j * WG + tid];
                const int qd = a.view[L.v * D2 + j];
                if (a.post) a.post[L.shot * a.n + qd] = clampf(S, a.clampv);
                if (signbit_of(S)) atomicOr(&ebits[L.sl * ew32 + (qd >> 5)], 1u << (qd & 31));
            }
    }
    __syncthreads();
    if (L.live) {
        if (a.ehat)
            for (int w = L.v; w < a.ehat_words; w += a.N) {
                const uint64_t lo = (2 * w < ew32) ? ebits[L.sl * ew32 + 2 * w] : 0u;
                const uint64_t hi = (2 * w + 1 < ew32) ? ebits[L.sl * ew32 + 2 * w + 1] : 0u;
                a.ehat[L.shot * a.ehat_words + w] = lo | (hi << 32);
            }
        if (L.v == 0 && a.stats) {
            ShotStats s = {};
            s.converged = gconv;
            s.global_iters = itg;
            s.local_iters_sum = shf[L.sl * 8 + SF_ITSUM];
            s.local_iters_max = shf[L.sl * 8 + SF_ITMAX];
            s.local_converged_views = shf[L.sl * 8 + SF_NCONV];
            s.local_fixed_views = shf[L.sl * 8 + SF_NFIX];
            s.global_fixed_iter = gfix;
            reinterpret_cast<ShotStats *>(a.stats)[L.shot] = s;
        }
    }
}

// s = H e: one thread per (shot, 64-bit syndrome word).
__global__ void __launch_bounds__(256) syndrome_kernel(SyndArgs a) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= a.shots * a.synd_words) return;
    const int64_t shot = gid / a.synd_words;
    const int w = (int)(gid - shot * a.synd_words);
    const uint64_t *e = a.err + shot * a.err_words;
    uint64_t out = 0;
    for (int b = 0; b < 64; ++b) {
        const int c = w * 64 + b;
        if (c >= a.m) break;
        const int v = c / a.r, rho = c - v * a.r;
        uint64_t mk = a.mask[rho];
        uint64_t par = 0;
        while (mk) {
            const int j = __builtin_ctzll(mk);
            mk &= mk - 1;
            const int q = a.view[v * a.D2 + j];
            par ^= (e[q >> 6] >> (q & 63)) & 1ull;
        }
        out |= par << b;
    }
    a.synd[gid] = out;
}


// ---------------------------------------------------------------------------
// Plain form: Phase 3 one round per launch, state in HBM.
//   S      [shots][D2][N]     variable sums
//   cst    [shots][r][4][N]   check states (m1, m2, am, q)
//   status [shots][4]         done, converged, global iterations
// phase 0 initialises S = lambda' and zero messages, phase 1 runs round
// `round` of every shot still active (counting them in *active), phase 2
// finalises (syndrome test of shots that ran out of rounds, outputs).  The
// arithmetic is the fused kernel's, in the same order, so outputs are
// bit-identical to lead_decode.
// ---------------------------------------------------------------------------
template <int D, int RMAX, int WG>
__global__ void __launch_bounds__(WG) round_kernel(RoundArgs ra) {
    constexpr int D2 = D * D;
    constexpr int OWN = (D2 + 1) / 2;
    const DecodeArgs &a = ra.d;
    extern __shared__ float lds[];
    const Lane L = lane_of(a, (int64_t)blockIdx.x * a.spw);
    const int tid = L.tid;
    float *buf = lds;
    int *shf = reinterpret_cast<int *>(buf + D2 * WG);
    const int ew32 = (a.n + 31) >> 5;
    uint32_t *ebits = reinterpret_cast<uint32_t *>(shf + a.spw * 8);
    float *bl = buf + tid;
    for (int i = tid; i < a.spw * 8; i += WG) shf[i] = 0;
    for (int i = tid; i < a.spw * ew32; i += WG) ebits[i] = 0u;
    __syncthreads();
    const int N = a.N;
    float *Sg = L.live ? ra.S + (L.shot * D2) * N + L.v : nullptr;
    float *Cg = L.live ? ra.cst + (L.shot * a.r) * 4 * N + L.v : nullptr;
    int32_t *stat = L.live ? ra.status + L.shot * 4 : nullptr;
    const float *lamp_row = L.live ? ra.lamp + L.shot * a.n : nullptr;

    if (ra.phase == 0) {
        if (L.live) {
#pragma unroll
            for (int j = 0; j < D2; ++j) Sg[j * N] = lamp_row[a.view[L.v * D2 + j]];
            for (int c = 0; c < a.r; ++c)
#pragma unroll
                for (int f = 0; f < 4; ++f) Cg[(c * 4 + f) * N] = 0.f;
            if (L.v == 0) { stat[0] = 0; stat[1] = 0; stat[2] = 0; stat[3] = 0; }
        }
        return;
    }

    uint32_t ent[OWN];
#pragma unroll
    for (int k = 0; k < OWN; ++k) ent[k] = (L.live && k < a.own_max) ? a.own[L.v * a.own_max + k] : kNoOwn;
    bool done = !L.live || stat[0] != 0;
    uint64_t sv = 0;
    if (L.live) {
        sv = local_syndrome(a, L.shot, L.v);
#pragma unroll
        for (int j = 0; j < D2; ++j) bl[j * WG] = Sg[j * N];
    }

    if (ra.phase == 1) {
        const int t = ra.round;
        CheckState<RMAX> st;
        st.clear();
        if (!done) {
#pragma unroll
            for (int c = 0; c < RMAX; ++c)
                if (c < a.r) {
                    st.m1[c] = Cg[(c * 4 + 0) * N];
                    st.m2[c] = Cg[(c * 4 + 1) * N];
                    st.am[c] = __float_as_uint(Cg[(c * 4 + 2) * N]);
                    st.q[c] = __float_as_uint(Cg[(c * 4 + 3) * N]);
                }
        }
        bool sat = true, same = true;
        if (!done) sat = check_pass<WG, RMAX>(a, bl, sv, st, same);
        if (!done && !sat) shf[L.sl * 8 + SF_FLAG0] = 1;
        if (!done && !same) shf[L.sl * 8 + SF_CHG] = 1;
        __syncthreads();
        if (!done && t > 1) {
            const bool shot_sat = shf[L.sl * 8 + SF_FLAG0] == 0;
            if (shot_sat && a.early_exit) {
                done = true;
                if (L.v == 0) { stat[0] = 1; stat[1] = 1; stat[2] = t - 1; }
            } else if (a.fixed_stop_g && shf[L.sl * 8 + SF_CHG] == 0) {
                done = true;
                if (L.v == 0) { stat[0] = 1; stat[1] = shot_sat ? 1 : 0; stat[2] = a.Tg; stat[3] = t; }
            }
        }
        if (!done) {
#pragma unroll
            for (int j = 0; j < D2; ++j) bl[j * WG] = 0.f;
#pragma unroll
            for (int k = 0; k < OWN; ++k)
                if (ent[k] != kNoOwn) bl[(ent[k] & 0xff) * WG] = lamp_row[a.view[L.v * D2 + (ent[k] & 0xff)]];
            accumulate<WG, RMAX>(a, bl, st);
        }
        __syncthreads();
        if (!done) {
#pragma unroll
            for (int k = 0; k < OWN; ++k)
                if (ent[k] != kNoOwn) {
                    int oa, ob;
                    occurrences<WG>(ent[k], L, a.N, oa, ob);
                    const float s = buf[oa] + buf[ob];
                    buf[oa] = s;
                    buf[ob] = s;
                }
        }
        __syncthreads();
        if (!done) {
#pragma unroll
            for (int j = 0; j < D2; ++j) Sg[j * N] = bl[j * WG];
#pragma unroll
            for (int c = 0; c < RMAX; ++c)
                if (c < a.r) {
                    Cg[(c * 4 + 0) * N] = st.m1[c];
                    Cg[(c * 4 + 1) * N] = st.m2[c];
                    Cg[(c * 4 + 2) * N] = __uint_as_float(st.am[c]);
                    Cg[(c * 4 + 3) * N] = __uint_as_float(st.q[c]);
                }
            if (L.v == 0) atomicAdd(ra.active, 1);
        }
        return;
    }

    // phase 2: shots that ran out of rounds take the syndrome test of S^{Tg}
    const bool ran_out = !done;
    if (ran_out && !parity_pass<WG, RMAX>(a, bl, sv)) shf[L.sl * 8 + SF_FINAL] = 1;
    __syncthreads();
    int gconv = 0, itg = 0;
    if (L.live) {
        if (ran_out) {
            gconv = shf[L.sl * 8 + SF_FINAL] == 0 ? 1 : 0;
            itg = a.Tg;
        } else {
            gconv = stat[1];
            itg = stat[2];
        }
#pragma unroll
        for (int k = 0; k < OWN; ++k)
            if (ent[k] != kNoOwn) {
                const int j = ent[k] & 0xff;
                const float S = buf[j * WG + tid];
                const int qd = a.view[L.v * D2 + j];
                if (a.post) a.post[L.shot * a.n + qd] = clampf(S, a.clampv);
                if (signbit_of(S)) atomicOr(&ebits[L.sl * ew32 + (qd >> 5)], 1u << (qd & 31));
            }
    }
    __syncthreads();
    if (L.live) {
        if (a.ehat)
            for (int w = L.v; w < a.ehat_words; w += a.N) {
                const uint64_t lo = (2 * w < ew32) ? ebits[L.sl * ew32 + 2 * w] : 0u;
                const uint64_t hi = (2 * w + 1 < ew32) ? ebits[L.sl * ew32 + 2 * w + 1] : 0u;
                a.ehat[L.shot * a.ehat_words + w] = lo | (hi << 32);
            }
        if (L.v == 0 && a.stats) {
            ShotStats *so = reinterpret_cast<ShotStats *>(a.stats) + L.shot;
            so->converged = gconv;
            so->global_iters = itg;
            so->global_fixed_iter = ran_out ? 0 : stat[3];
        }
    }
}

template <int D, int RMAX, int WG>
hipError_t launch_round_t(const RoundArgs &ra, hipStream_t s) {
    const DecodeArgs &a = ra.d;
    const size_t lds = decode_lds_bytes(D, WG, a.spw, a.n);
    const int64_t grid = (a.shots + a.spw - 1) / a.spw;
    hipLaunchKernelGGL((round_kernel<D, RMAX, WG>), dim3((unsigned)grid), dim3(WG), lds, s, ra);
    return hipGetLastError();
}

template <int D, int RMAX>
hipError_t launch_round_d(int wg, const RoundArgs &ra, hipStream_t s) {
    switch (wg) {
        case 64: return launch_round_t<D, RMAX, 64>(ra, s);
        case 128: return launch_round_t<D, RMAX, 128>(ra, s);
        case 192: return launch_round_t<D, RMAX, 192>(ra, s);
        case 256: return launch_round_t<D, RMAX, 256>(ra, s);
        default: return hipErrorInvalidValue;
    }
}

template <int D, int RMAX, int WG>
hipError_t launch_decode_t(const DecodeArgs &a, const LocalArgs &w, bool split, hipStream_t s, hipEvent_t *ev) {
    const size_t lds = decode_lds_bytes(D, WG, a.spw, a.n);
    const int64_t grid = (a.shots + a.spw - 1) / a.spw;
    const bool pm0 = a.prior_mode == LEAD_PRIOR_PER_SHOT;
    if (split) {
        hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, s, w.counter);
        const int waves = w.waves;
        const size_t llds = sizeof(float) * D * D * 64;
        if (ev) (void)hipEventRecord(ev[0], s);
        if (pm0)
            hipLaunchKernelGGL((local_kernel<D, RMAX, 0>), dim3(waves), dim3(64), llds, s, a, w);
        else
            hipLaunchKernelGGL((local_kernel<D, RMAX, 1>), dim3(waves), dim3(64), llds, s, a, w);
        if (ev) (void)hipEventRecord(ev[1], s);
        hipLaunchKernelGGL((decode_kernel<D, RMAX, WG, 0, true>), dim3((unsigned)grid), dim3(WG), lds, s, a, w);
        if (ev) (void)hipEventRecord(ev[2], s);
    } else if (pm0) {
        hipLaunchKernelGGL((decode_kernel<D, RMAX, WG, 0, false>), dim3((unsigned)grid), dim3(WG), lds, s, a, w);
    } else {
        hipLaunchKernelGGL((decode_kernel<D, RMAX, WG, 1, false>), dim3((unsigned)grid), dim3(WG), lds, s, a, w);
    }
    return hipGetLastError();
}

template <int D, int RMAX>
hipError_t launch_decode_d(int wg, const DecodeArgs &a, const LocalArgs &w, bool split, hipStream_t s,
                           hipEvent_t *ev) {
    switch (wg) {
        case 64: return launch_decode_t<D, RMAX, 64>(a, w, split, s, ev);
        case 128: return launch_decode_t<D, RMAX, 128>(a, w, split, s, ev);
        case 192: return launch_decode_t<D, RMAX, 192>(a, w, split, s, ev);
        case 256: return launch_decode_t<D, RMAX, 256>(a, w, split, s, ev);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

int workgroup_size(int N, int spw) { return ((N * spw + 63) / 64) * 64; }

size_t decode_lds_bytes(int D, int wg, int spw, int n) {
    const int ew32 = (n + 31) / 32;
    return sizeof(float) * (size_t)D * D * wg + sizeof(int) * (size_t)wg + sizeof(int) * (size_t)spw * 8 +
           sizeof(uint32_t) * (size_t)spw * ew32;
}

// Resident 64-lane waves of local_kernel per CU (occupancy of the
// instantiation used for this shape and prior mode).
int local_waves_per_cu(int D, int pm) {
    int nb = 0;
    const size_t lds = sizeof(float) * D * D * 64;
    hipError_t e = hipErrorInvalidValue;
    switch (D) {
        case 3: e = pm ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, local_kernel<3, 4, 1>, 64, lds)
                       : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, local_kernel<3, 4, 0>, 64, lds); break;
        case 4: e = pm ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, local_kernel<4, 9, 1>, 64, lds)
                       : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, local_kernel<4, 9, 0>, 64, lds); break;
        case 6: e = pm ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, local_kernel<6, 9, 1>, 64, lds)
                       : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, local_kernel<6, 9, 0>, 64, lds); break;
        case 8: e = pm ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, local_kernel<8, 16, 1>, 64, lds)
                       : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, local_kernel<8, 16, 0>, 64, lds); break;
        default: break;
    }
    return (e == hipSuccess && nb > 0) ? nb : 4;
}

// Compiled shapes: (Delta, maximum checks per vertex).
bool kernel_supported(int D, int r) {
    switch (D) {
        case 3: return r <= 4;
        case 4: return r <= 9;
        case 6: return r <= 9;
        case 8: return r <= 16;
        default: return false;
    }
}

hipError_t launch_decode(int D, int, const DecodeArgs &a, const LocalArgs &w, bool split, hipStream_t s,
                         hipEvent_t *ev) {
    if (a.shots <= 0) return hipSuccess;
    const int wg = workgroup_size(a.N, a.spw);
    switch (D) {
        case 3: return launch_decode_d<3, 4>(wg, a, w, split, s, ev);
        case 4: return launch_decode_d<4, 9>(wg, a, w, split, s, ev);
        case 6: return launch_decode_d<6, 9>(wg, a, w, split, s, ev);
        case 8: return launch_decode_d<8, 16>(wg, a, w, split, s, ev);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_round(int D, int, const RoundArgs &ra, hipStream_t s) {
    if (ra.d.shots <= 0) return hipSuccess;
    const int wg = workgroup_size(ra.d.N, ra.d.spw);
    switch (D) {
        case 3: return launch_round_d<3, 4>(wg, ra, s);
        case 4: return launch_round_d<4, 9>(wg, ra, s);
        case 6: return launch_round_d<6, 9>(wg, ra, s);
        case 8: return launch_round_d<8, 16>(wg, ra, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_clear_i64(int64_t *p, int n, hipStream_t s) {
    hipLaunchKernelGGL(clear_i64_kernel, dim3(1), dim3(64), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_reset_counter(int64_t *counter, hipStream_t s) {
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, s, counter);
    return hipGetLastError();
}

hipError_t launch_syndrome(const SyndArgs &a, hipStream_t s) {
    const int64_t total = a.shots * a.synd_words;
    if (total <= 0) return hipSuccess;
    const int64_t grid = (total + 255) / 256;
    hipLaunchKernelGGL(syndrome_kernel, dim3((unsigned)grid), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace lead
