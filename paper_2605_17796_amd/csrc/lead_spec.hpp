// Decoding kernels specialised for the local check structure of one code.
//
// The library compiles this header at run time for the code of a decoder,
// with a structure `C` that fixes, as compile-time constants,
//   C::D            Delta (a view has D*D local positions),
//   C::R            checks per vertex,
//   C::mask[R]      the local check masks over the D*D positions,
//   C::sigma[D*D]   the local position of the other occurrence of the qubit
//                   at position j (the same map for every view of a Cayley
//                   complex),
//   C::NFIX         the number of fixed points of sigma.
// Every edge loop then unrolls completely: edge positions, register indices
// and sign-bit positions are immediates, and the variable sums S_j of a view
// stay in VGPRs in both phases of BP (the precompiled kernels keep them in
// LDS and walk the masks with scalar bit scans).  The arithmetic is the
// precompiled kernels', operation for operation and in the same order, so the
// outputs are bit-identical to theirs.
//
// Ownership of a qubit (who adds lambda' into its partial sum and writes its
// outputs): position j owns it when j < sigma[j]; at fixed points of sigma
// the owned positions come from the table fown[v].
#pragma once
#include "lead_device.hpp"

namespace lead_spec {

using namespace lead_dev;
using lead::DecodeArgs;
using lead::LocalArgs;
using lead::SpecArgs;

template <int R>
struct State {
    float m1[R], m2[R];
    uint32_t am[R], q[R];
    __device__ __forceinline__ void clear() {
#pragma unroll
        for (int c = 0; c < R; ++c) { m1[c] = 0.f; m2[c] = 0.f; am[c] = 0u; q[c] = 0u; }
    }
};

// Check update of every check of the view from the sums S of the previous
// iteration: mu_{j->c} = clamp(S_j - m_{c->j}) and the new min-sum state
// (beta * smallest |mu|, beta * second smallest, position of the smallest,
// outgoing signs).  Returns whether [S_j < 0] satisfies every check; `same`
// tells whether every state is unchanged bit for bit.
template <class C>
__device__ __forceinline__ bool check_pass(const float (&S)[C::D * C::D], uint64_t sv, float beta, float clampv,
                                           State<C::R> &st, bool &same) {
    constexpr int D2 = C::D * C::D;
    bool sat = true;
    same = true;
#pragma unroll
    for (int c = 0; c < C::R; ++c) {
        float n1 = kBig, n2 = kBig;
        uint32_t nam = 0u, sg = 0u, par = 0u, k = 0u;
#pragma unroll
        for (int j = 0; j < D2; ++j) {
            if ((C::mask[c] >> j) & 1ull) {
                par ^= __float_as_uint(S[j]);
                const float mu = clampf(S[j] - msg_of(st.m1[c], st.m2[c], st.am[c], st.q[c], k), clampv);
                const float ab = fabsf(mu);
                sg |= signbit_of(mu) << k;
                n2 = __builtin_amdgcn_fmed3f(n1, n2, ab);
                const bool lt = ab < n1;
                nam = lt ? k : nam;
                n1 = lt ? ab : n1;
                ++k;
            }
        }
        const uint32_t sc = (uint32_t)(sv >> c) & 1u;
        sat = sat && ((par >> 31) == sc);
        const uint32_t flip = ((uint32_t)__popc(sg) & 1u) ^ sc;
        const uint32_t all = (uint32_t)((1ull << k) - 1ull);
        const uint32_t nq = flip ? (sg ^ all) : sg;
        const float b1 = beta * n1, b2 = beta * n2;
        same = same && nq == st.q[c] && nam == st.am[c] && __float_as_uint(b1) == __float_as_uint(st.m1[c]) &&
               __float_as_uint(b2) == __float_as_uint(st.m2[c]);
        st.q[c] = nq;
        st.m1[c] = b1;
        st.m2[c] = b2;
        st.am[c] = nam;
        // one check at a time: the scheduler would otherwise hoist the mu of
        // every edge of the view ahead of the serial min chains, keeping them
        // all live (VALU results feed the next instruction without stalls,
        // so that buys nothing)
        __builtin_amdgcn_sched_barrier(0);
    }
    return sat;
}

// Whether [S_j < 0] satisfies every check of the view.
template <class C>
__device__ __forceinline__ bool parity(const float (&S)[C::D * C::D], uint64_t sv) {
    constexpr int D2 = C::D * C::D;
    bool sat = true;
#pragma unroll
    for (int c = 0; c < C::R; ++c) {
        uint32_t par = 0u;
#pragma unroll
        for (int j = 0; j < D2; ++j)
            if ((C::mask[c] >> j) & 1ull) par ^= __float_as_uint(S[j]);
        sat = sat && ((par >> 31) == ((uint32_t)(sv >> c) & 1u));
    }
    return sat;
}

// S_j += m_{c->j} for every edge, checks in order.
template <class C>
__device__ __forceinline__ void accumulate(float (&S)[C::D * C::D], const State<C::R> &st) {
    constexpr int D2 = C::D * C::D;
#pragma unroll
    for (int c = 0; c < C::R; ++c) {
        uint32_t k = 0u;
#pragma unroll
        for (int j = 0; j < D2; ++j) {
            if ((C::mask[c] >> j) & 1ull) {
                S[j] += msg_of(st.m1[c], st.m2[c], st.am[c], st.q[c], k);
                ++k;
            }
        }
    }
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

// Phase 1 as a work queue over (shot, vertex) items: a lane runs the local BP
// of one item with S in VGPRs and takes the next item as soon as its run
// ends.  Stopping rules and outputs are those of the precompiled local
// kernel: Lv[item][j] = clamp(S_j), vflag[item] = iterations | converged << 16
// | fixed point << 17.
template <class C, int PM>
__device__ __forceinline__ void local_body(const DecodeArgs &a, const LocalArgs &w) {
    constexpr int D2 = C::D * C::D;
    constexpr int NL = PM == 0 ? 1 : D2;
    const int lane = threadIdx.x;
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int64_t cur = 0, end = 0;
    bool queue_open = true, valid = false;
    int64_t item = 0;
    int t = 0;
    uint64_t sv = 0;
    float lam[NL];
    float S[D2];
#pragma unroll
    for (int j = 0; j < NL; ++j) lam[j] = 0.f;
#pragma unroll
    for (int j = 0; j < D2; ++j) S[j] = 0.f;
    State<C::R> st;
    st.clear();
    for (;;) {
        uint64_t need = __ballot(!valid);
        while (need && queue_open) {
            if (cur >= end) {
                unsigned long long c0 = 0;
                if (lane == 0)
                    c0 = atomicAdd(reinterpret_cast<unsigned long long *>(w.counter), (unsigned long long)w.chunk);
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
                if (PM == 0) {
                    lam[0] = a.prior[shot] + 0.f;
                } else {
                    const int64_t base = a.prior_mode == 2 ? shot * a.n : 0;
#pragma unroll
                    for (int j = 0; j < NL; ++j) lam[j] = a.prior[base + a.view[v * D2 + j]] + 0.f;
                }
                st.clear();
#pragma unroll
                for (int j = 0; j < D2; ++j) S[j] = lam[PM == 0 ? 0 : j];
                t = 1;
            }
            const int64_t taken = __popcll(need) < avail ? __popcll(need) : avail;
            cur += taken;
            need = __ballot(!valid);
        }
        if (__ballot(valid) == 0ull) break;
        if (valid) {
            bool same;
            const bool sat = check_pass<C>(S, sv, a.beta, a.clampv, st, same);
            int conv = 0, it = 0, fixed = 0;
            bool fin = false;
            if (t > a.Tl) {
                conv = sat ? 1 : 0;
                it = a.Tl;
                fin = true;
            } else if (t > 1 && sat && a.early_exit) {
                conv = 1;
                it = t - 1;
                fin = true;
            } else if (t > 1 && same && a.fixed_stop) {
                conv = sat ? 1 : 0;
                it = a.Tl;
                fixed = 1;
                fin = true;
            }
            if (fin) {
                float *out = w.Lv + item * D2;
#pragma unroll
                for (int j = 0; j < D2; ++j) out[j] = clampf(S[j], a.clampv);
                w.vflag[item] = (uint32_t)it | ((uint32_t)conv << 16) | ((uint32_t)fixed << 17);
                valid = false;
            } else {
#pragma unroll
                for (int j = 0; j < D2; ++j) S[j] = lam[PM == 0 ? 0 : j];
                accumulate<C>(S, st);
                ++t;
            }
        }
    }
}

// Per-shot LDS flags (the precompiled kernel's layout).
enum { SF_FLAG0 = 0, SF_FLAG1 = 1, SF_FINAL = 2, SF_ITSUM = 3, SF_ITMAX = 4, SF_NCONV = 5, SF_CHG = 6, SF_NFIX = 7 };

// Value of X at the other occurrence of local position J: lane `addr` (a
// byte address) holds it at position sigma[J].  BPERM: the partner lane is
// in the same wave and is read with ds_bpermute; otherwise X has been stored
// to LDS as buf[j][lane].
template <class C, int WG, bool BPERM, int J>
__device__ __forceinline__ float partner(const float (&X)[C::D * C::D], const float *buf, uint32_t addr) {
    if (BPERM)
        return __int_as_float(__builtin_amdgcn_ds_bpermute((int)addr, __float_as_int(X[C::sigma[J]])));
    return *reinterpret_cast<const float *>(reinterpret_cast<const char *>(buf) + C::sigma[J] * WG * 4 + addr);
}

template <class C, int WG, bool BPERM, int J = 0>
__device__ __forceinline__ void partner_all(const float (&X)[C::D * C::D], float (&Y)[C::D * C::D],
                                            const float *buf, const uint32_t (&pa)[(C::D * C::D + 1) / 2]) {
    if constexpr (J < C::D * C::D) {
        Y[J] = partner<C, WG, BPERM, J>(X, buf, (pa[J >> 1] >> ((J & 1) * 16)) & 0xffffu);
        partner_all<C, WG, BPERM, J + 1>(X, Y, buf, pa);
    }
}

template <class C, int WG, bool BPERM>
__device__ __forceinline__ void store_all(const float (&X)[C::D * C::D], float *buf) {
    if (!BPERM) {
#pragma unroll
        for (int j = 0; j < C::D * C::D; ++j) buf[j * WG + threadIdx.x] = X[j];
        __syncthreads();
    }
}

// Phases 2-3 of `spw` shots per workgroup after the Phase 1 queue kernel;
// lane (slot, v) holds vertex v of shot blockIdx.x * spw + slot.  The same
// computation as the precompiled split kernel: lambda' of every qubit from
// its two clamped local posteriors, then global min-sum rounds in which each
// view forms its partial sum P_j (lambda' on owned positions, then its
// checks' messages in check order) and S_j = P_j + P_j' of the other
// occurrence.
template <class C, int WG, bool BPERM>
__device__ __forceinline__ void global_body(const DecodeArgs &a, const LocalArgs &w, const SpecArgs &x) {
    constexpr int D2 = C::D * C::D;
    constexpr int NP = (D2 + 1) / 2;
    extern __shared__ float lds[];
    float *buf = lds;
    int *shf = reinterpret_cast<int *>(lds + (BPERM ? 0 : D2 * WG));
    const int ew32 = (a.n + 31) >> 5;
    uint32_t *ebits = reinterpret_cast<uint32_t *>(shf + a.spw * 8);
    const int tid = threadIdx.x;
    const int sl = tid / a.N, v = tid - sl * a.N;
    const bool lane_ok = sl < a.spw;
    const int64_t shot = (int64_t)blockIdx.x * a.spw + sl;
    const bool live = lane_ok && shot < a.shots;
    for (int i = tid; i < a.spw * 8; i += WG) shf[i] = 0;
    for (int i = tid; i < a.spw * ew32; i += WG) ebits[i] = 0u;

    float S[D2];
    uint32_t pa[NP];
    uint64_t sv = 0, fown = 0;
    int it_v = 0, conv_v = 0, fixed_v = 0;
    if (live) {
        sv = local_syndrome(a, shot, v);
        const int64_t item = shot * a.N + v;
        const float *in = w.Lv + item * D2;
#pragma unroll
        for (int j = 0; j < D2; ++j) S[j] = in[j];
        const uint32_t f = w.vflag[item];
        it_v = (int)(f & 0xffffu);
        conv_v = (int)((f >> 16) & 1u);
        fixed_v = (int)((f >> 17) & 1u);
        const uint32_t base = (uint32_t)(sl * a.N);
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            const uint32_t p = x.pv[v * NP + k];
            pa[k] = ((base + (p & 0xffffu)) * 4u) | (((base + (p >> 16)) * 4u) << 16);
        }
        if (C::NFIX) fown = x.fown[v];
    } else {
#pragma unroll
        for (int j = 0; j < D2; ++j) S[j] = 0.f;
#pragma unroll
        for (int k = 0; k < NP; ++k) pa[k] = (uint32_t)tid * 4u * 0x10001u;
    }
    __syncthreads();
    if (live) {
        atomicAdd(&shf[sl * 8 + SF_ITSUM], it_v);
        atomicMax(&shf[sl * 8 + SF_ITMAX], it_v);
        atomicAdd(&shf[sl * 8 + SF_NCONV], conv_v);
        if (fixed_v) atomicAdd(&shf[sl * 8 + SF_NFIX], 1);
    }
    auto owned = [&](int j) { return C::sigma[j] > j || (C::sigma[j] == j && ((fown >> j) & 1ull)); };

    // ---- Phase 2: lambda' of every position (symmetric in the two views, so
    // both occurrences of a qubit compute the same value); the confidence
    // boost L <- min(L, 0) on L < 0 leaves L unchanged.
    float lam[D2];
    {
        float Lp[D2];
        store_all<C, WG, BPERM>(S, buf);
        partner_all<C, WG, BPERM>(S, Lp, buf, pa);
#pragma unroll
        for (int j = 0; j < D2; ++j) lam[j] = aggregate_llr(clampf(S[j], a.clampv), clampf(Lp[j], a.clampv), a.alpha, a.clampv);
    }
    if (a.lam_out && live) {
#pragma unroll
        for (int j = 0; j < D2; ++j)
            if (owned(j)) a.lam_out[shot * a.n + a.view[v * D2 + j]] = lam[j];
    }
    if (a.stage == 1) {
        __syncthreads();
        if (live && v == 0 && a.stats) {
            lead::ShotStats s = {};
            s.local_iters_sum = shf[sl * 8 + SF_ITSUM];
            s.local_iters_max = shf[sl * 8 + SF_ITMAX];
            s.local_converged_views = shf[sl * 8 + SF_NCONV];
            s.local_fixed_views = shf[sl * 8 + SF_NFIX];
            reinterpret_cast<lead::ShotStats *>(a.stats)[shot] = s;
        }
        return;
    }

    // ---- Phase 3: global BP with prior lambda' ------------------------------
    // The outputs of a shot are written when its run ends (its S is final).
    auto emit = [&]() {
#pragma unroll
        for (int j = 0; j < D2; ++j)
            if (owned(j)) {
                const int qd = a.view[v * D2 + j];
                if (a.post) a.post[shot * a.n + qd] = clampf(S[j], a.clampv);
                if (signbit_of(S[j])) atomicOr(&ebits[sl * ew32 + (qd >> 5)], 1u << (qd & 31));
            }
    };
#pragma unroll
    for (int j = 0; j < D2; ++j) S[j] = lam[j];
    State<C::R> st;
    st.clear();
    if (!BPERM) __syncthreads();
    bool done = !live;
    int itg = 0, gconv = 0, gfix = 0;
    for (int t = 1; t <= a.Tg; ++t) {
        bool sat = true, same = true;
        if (!done) sat = check_pass<C>(S, sv, a.beta, a.clampv, st, same);
        if (!done && !sat) shf[sl * 8 + (t & 1)] = 1;
        if (!done && !same) shf[sl * 8 + SF_CHG] = t;
        __syncthreads();
        if (!done && t > 1) {
            const bool shot_sat = shf[sl * 8 + (t & 1)] == 0;
            if (shot_sat && a.early_exit) {
                done = true;
                gconv = 1;
                itg = t - 1;
                emit();
            } else if (a.fixed_stop && shf[sl * 8 + SF_CHG] != t) {
                done = true;
                gconv = shot_sat ? 1 : 0;
                itg = a.Tg;
                gfix = t;
                emit();
            }
        }
        if (!__syncthreads_or(done ? 0 : 1)) break;
        if (lane_ok && v == 0) shf[sl * 8 + ((t + 1) & 1)] = 0;
        // partial sums of this view, then S_j = P_j + P of the other occurrence
#pragma unroll
        for (int j = 0; j < D2; ++j) S[j] = owned(j) ? lam[j] : 0.f;
        accumulate<C>(S, st);
        float Q[D2];
        store_all<C, WG, BPERM>(S, buf);
        partner_all<C, WG, BPERM>(S, Q, buf, pa);
#pragma unroll
        for (int j = 0; j < D2; ++j) S[j] += Q[j];
    }
    const bool ran_out = !done;
    if (ran_out && !parity<C>(S, sv)) shf[sl * 8 + SF_FINAL] = 1;
    __syncthreads();
    if (ran_out) {
        gconv = shf[sl * 8 + SF_FINAL] == 0 ? 1 : 0;
        itg = a.Tg;
        emit();
    }
    __syncthreads();
    if (live) {
        if (a.ehat)
            for (int wd = v; wd < a.ehat_words; wd += a.N) {
                const uint64_t lo = (2 * wd < ew32) ? ebits[sl * ew32 + 2 * wd] : 0u;
                const uint64_t hi = (2 * wd + 1 < ew32) ? ebits[sl * ew32 + 2 * wd + 1] : 0u;
                a.ehat[shot * a.ehat_words + wd] = lo | (hi << 32);
            }
        if (v == 0 && a.stats) {
            lead::ShotStats s = {};
            s.converged = gconv;
            s.global_iters = itg;
            s.local_iters_sum = shf[sl * 8 + SF_ITSUM];
            s.local_iters_max = shf[sl * 8 + SF_ITMAX];
            s.local_converged_views = shf[sl * 8 + SF_NCONV];
            s.local_fixed_views = shf[sl * 8 + SF_NFIX];
            s.global_fixed_iter = gfix;
            reinterpret_cast<lead::ShotStats *>(a.stats)[shot] = s;
        }
    }
}

}  // namespace lead_spec
