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
//   C::NFIX         the number of fixed points of sigma,
//   C::E, C::deg[R], C::base[R]
//                   the local edges (numbered check by check, positions
//                   ascending within a check): their count, and per check
//                   the degree and the number of its first edge,
//   C::SPLIT        track the two smallest |mu| in two chains per check,
//   C::LDSMASK      the checks whose messages the Phase 1 queue kernel of
//                   form 2 keeps in LDS (views whose messages do not all fit
//                   beside the sums in 256 VGPRs; 0: none),
//   C::HYB          degree from which the per-shot kernel keeps a check's
//                   compressed state in form 2 (0: none),
//   C::LAM_LDS      the per-shot kernel's LDS has room for lambda' when a
//                   shot spans several waves.
// Every loop below runs over compile-time bounds and indexes arrays with
// loop-constant subscripts only (through tables, not constexpr functions
// with loops of their own), so that each index folds to an immediate once
// the loops are unrolled and no array is left in scratch memory.
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

// Compile-time loops.  Checks and edge positions are template constants, so
// every mask test, edge number and array subscript below is a constant
// expression (no reliance on the optimiser unrolling a loop first; an array
// indexed by a value it could not fold would be left in scratch memory).
template <int V>
struct Int {
    static constexpr int value = V;
};

template <int I, int N, class F>
__device__ __forceinline__ void static_for(const F &f) {
    if constexpr (I < N) {
        f(Int<I>{});
        static_for<I + 1, N>(f);
    }
}

constexpr int rank_below(uint64_t m, int j) {
    int n = 0;
    for (int i = 0; i < j; ++i) n += (int)((m >> i) & 1ull);
    return n;
}

// f(j, k) for the edges of check c in position order: the k-th edge sits at
// local position j.
template <class C, int c, class F>
__device__ __forceinline__ void for_edges(const F &f) {
    static_for<0, C::D * C::D>([&](auto jj) {
        constexpr int j = decltype(jj)::value;
        if constexpr (((C::mask[c] >> j) & 1ull) != 0) f(Int<j>{}, Int<rank_below(C::mask[c], j)>{});
    });
}

// Compressed check state (the precompiled kernels' form): per check
// beta * n1, beta * n2, the position of the smallest and the sign bit of
// every outgoing message; messages are rebuilt from it when needed.
// Check update of check c in the compressed state (m1, m2, am, q of that
// check) from the sums S of the previous iteration: mu_{j->c} = S_j - m_{c->j}
// (not clamped per edge: the clamp goes to the two minima; clamping is
// monotone, and where the unclamped and the clamped position of the smallest
// differ, both minima clamp to the same value and the position does not
// matter) and the new min-sum state.  sat &= [S_j < 0] satisfies the check;
// diff gains the bits that differ between the old and the new state.
template <class C, int c, bool FP = true>
__device__ __forceinline__ void compressed_update(const float (&S)[C::D * C::D], uint64_t sv, float beta, float clampv,
                                                  float keep, float &m1, float &m2, uint32_t &am, uint32_t &q,
                                                  bool &sat, uint32_t &diff) {
    float n1 = kBig, n2 = kBig;
    uint32_t nam = 0u, sg = 0u, par = 0u, pend = 0u;
    for_edges<C, c>([&](auto jj, auto kk) {
        constexpr int j = decltype(jj)::value;
        constexpr uint32_t k = decltype(kk)::value;
        // sign parity of S, two edges per three-input XOR
        if constexpr ((k & 1) == 0) {
            pend = __float_as_uint(S[j]);
            if constexpr (k + 1 == (uint32_t)C::deg[c]) par ^= pend;
        } else {
            par = __builtin_amdgcn_bitop3_b32(par, pend, __float_as_uint(S[j]), 0x96);
        }
        const float mu = __builtin_fmaf(-msg_of(m1, m2, am, q, k), keep, S[j]);
        const float ab = fabsf(mu);
        sg |= signbit_of(mu) << k;
        n2 = __builtin_amdgcn_fmed3f(n1, n2, ab);
        const bool lt = ab < n1;
        nam = lt ? k : nam;
        n1 = lt ? ab : n1;
    });
    const uint32_t sc = (uint32_t)(sv >> c) & 1u;
    sat = sat && ((par >> 31) == sc);
    const uint32_t flip = ((uint32_t)__popc(sg) & 1u) ^ sc;
    constexpr uint32_t all = (uint32_t)((1ull << C::deg[c]) - 1ull);
    uint32_t nq = flip ? (sg ^ all) : sg;
    uint32_t b1u = __float_as_uint(beta * fminf(n1, clampv)), b2u = __float_as_uint(beta * fminf(n2, clampv));
    if constexpr (FP) {
        // every outgoing message unchanged (the position of the smallest
        // matters only when the two magnitudes differ)
        const uint32_t dterm = (nq ^ q) | (b1u ^ __float_as_uint(m1)) | (b2u ^ __float_as_uint(m2)) |
                               (b1u == b2u ? 0u : nam ^ am);
        diff |= dterm;
        // the new state is written from operands that depend on the
        // comparison: the old values are then dead when the new ones are
        // written and can share their registers (no copies at the loop
        // back-edge)
        asm("" : "+v"(nq), "+v"(b1u), "+v"(b2u), "+v"(nam) : "v"(dterm));
    } else {
        // formed here all the same (see explicit_update)
        asm volatile("" : "+v"(nq), "+v"(b1u), "+v"(b2u), "+v"(nam));
    }
    q = nq;
    m1 = __uint_as_float(b1u);
    m2 = __uint_as_float(b2u);
    am = nam;
    asm volatile("" : "+v"(diff));
    __builtin_amdgcn_sched_barrier(0);
}

// Compressed check state (the precompiled kernels' form): per check
// beta * n1, beta * n2, the position of the smallest and the sign bit of
// every outgoing message; messages are rebuilt from it when needed.
template <class C>
struct Compressed {
    static constexpr int R = C::R;
    float m1[R], m2[R];
    uint32_t am[R], q[R];
    __device__ __forceinline__ void clear() {
#pragma unroll
        for (int c = 0; c < R; ++c) { m1[c] = 0.f; m2[c] = 0.f; am[c] = 0u; q[c] = 0u; }
    }
    // clear() where z holds, by selects (no branch around the state)
    __device__ __forceinline__ void reset_where(bool z) {
#pragma unroll
        for (int c = 0; c < R; ++c) {
            m1[c] = z ? 0.f : m1[c];
            m2[c] = z ? 0.f : m2[c];
            am[c] = z ? 0u : am[c];
            q[c] = z ? 0u : q[c];
        }
    }
    // Check update of every check of the view from the sums S of the
    // previous iteration.  Returns whether [S_j < 0] satisfies every check;
    // `same` tells whether every outgoing message is unchanged bit for bit
    // (FP = false: no comparison, same = false).
    template <bool FP = true>
    __device__ __forceinline__ bool check(const float (&S)[C::D * C::D], uint64_t sv, float beta, float clampv,
                                          bool &same, float keep = 1.f) {
        bool sat = true;
        // bits that differ between the old and the new state, accumulated
        // as an integer so that each comparison is done as soon as its
        // operands exist (a chain of boolean ands lets the compiler keep
        // every old value live until the end)
        uint32_t diff = 0u;
        static_for<0, R>([&](auto cc) {
            constexpr int c = decltype(cc)::value;
            compressed_update<C, c, FP>(S, sv, beta, clampv, keep, m1[c], m2[c], am[c], q[c], sat, diff);
        });
        same = FP && diff == 0u;
        return sat;
    }
    // The state as WORDS 32-bit words at p[i * stride] (plain per-round form).
    static constexpr int WORDS = 4 * R;
    __device__ __forceinline__ void save(float *p, int stride) const {
#pragma unroll
        for (int c = 0; c < R; ++c) {
            p[(4 * c) * stride] = m1[c];
            p[(4 * c + 1) * stride] = m2[c];
            p[(4 * c + 2) * stride] = __uint_as_float(am[c]);
            p[(4 * c + 3) * stride] = __uint_as_float(q[c]);
        }
    }
    __device__ __forceinline__ void load(const float *p, int stride) {
#pragma unroll
        for (int c = 0; c < R; ++c) {
            m1[c] = p[(4 * c) * stride];
            m2[c] = p[(4 * c + 1) * stride];
            am[c] = __float_as_uint(p[(4 * c + 2) * stride]);
            q[c] = __float_as_uint(p[(4 * c + 3) * stride]);
        }
    }
    // The message of check c to its k-th edge.
    template <int c, int k>
    __device__ __forceinline__ float msg() const { return msg_of(m1[c], m2[c], am[c], q[c], (uint32_t)k); }
    // S_j += m_{c->j} for every edge, checks in order.
    __device__ __forceinline__ void accumulate(float (&S)[C::D * C::D], float keep = 1.f) const {
        static_for<0, R>([&](auto cc) {
            constexpr int c = decltype(cc)::value;
            for_edges<C, c>([&](auto jj, auto kk) {
                S[decltype(jj)::value] =
                    __builtin_fmaf(msg_of(m1[c], m2[c], am[c], q[c], (uint32_t)decltype(kk)::value), keep, S[decltype(jj)::value]);
            });
        });
    }
};

// Check update of check c with one register per message: the messages of
// its edges are m[b], m[b + 1], ... (b fixed by the caller's layout).  With
// FP the bits that differ between each old and new message go to diff; the
// old message is then still read after the new one is formed, so the two
// take different registers (a copy per message at the loop back-edge).
// Without FP the new message overwrites the old one in place.
template <class C, int c, int b, int E, bool FP = true>
__device__ __forceinline__ void explicit_update(const float (&S)[C::D * C::D], uint64_t sv, float beta, float clampv,
                                                float keep, float (&m)[E], bool &sat, uint32_t &diff) {
    constexpr int D2 = C::D * C::D;
    for_edges<C, c>([&m](auto, auto kk) { asm volatile("" : "+v"(m[b + decltype(kk)::value])); });
    // The clamp of mu is applied to the two minima instead of to
    // every edge: clamping is monotone, so the minimum and second
    // minimum of the clamped magnitudes are the clamped minima, and
    // where |mu_k| == n1 and the clamped comparison differ, both
    // minima clamp to the same value.  Messages are bit for bit those
    // of clamping each mu.
    // With C::SPLIT the two smallest are tracked over the first and
    // the second half of the edges separately and then merged
    // (shorter dependency chains for kernels that run one wave per
    // SIMD); min and max are exact, so n1 and n2 are the same values.
    constexpr int h = C::SPLIT ? C::deg[c] / 2 : C::deg[c];
    float n1 = kBig, n2 = kBig, n1b = kBig, n2b = kBig, mu[D2];
    uint32_t par = 0u, ps = 0u, pend = 0u;
    for_edges<C, c>([&](auto jj, auto kk) {
        constexpr int j = decltype(jj)::value, k = decltype(kk)::value;
        mu[j] = __builtin_fmaf(-m[b + k], keep, S[j]);
        // sign parities of S and mu, two edges per three-input XOR
        if constexpr ((k & 1) == 0) {
            pend = __float_as_uint(S[j]);
            if constexpr (k + 1 == C::deg[c]) par ^= pend;
        } else {
            par = __builtin_amdgcn_bitop3_b32(par, pend, __float_as_uint(S[j]), 0x96);
        }
        if constexpr (k < h) {
            n2 = __builtin_amdgcn_fmed3f(n1, n2, fabsf(mu[j]));
            n1 = fminf(n1, fabsf(mu[j]));
        } else {
            n2b = __builtin_amdgcn_fmed3f(n1b, n2b, fabsf(mu[j]));
            n1b = fminf(n1b, fabsf(mu[j]));
        }
    });
    if constexpr (h < C::deg[c]) {
        n2 = fminf(fmaxf(n1, n1b), fminf(n2, n2b));
        n1 = fminf(n1, n1b);
    }
    for_edges<C, c>([&](auto jj, auto kk) {
        constexpr int j = decltype(jj)::value, k = decltype(kk)::value;
        if constexpr ((k & 1) == 0) {
            pend = __float_as_uint(mu[j]);
            if constexpr (k + 1 == C::deg[c]) ps ^= pend;
        } else {
            ps = __builtin_amdgcn_bitop3_b32(ps, pend, __float_as_uint(mu[j]), 0x96);
        }
    });
    const uint32_t sc = (uint32_t)(sv >> c) & 1u;
    sat = sat && ((par >> 31) == sc);
    // the two candidate messages with the sign of the whole product
    // (check syndrome included); each edge then flips the sign by its
    // own mu's, which takes its mu out of the product
    const uint32_t px = (ps ^ (sc << 31)) & kSign;
    uint32_t b1 = __float_as_uint(beta * fminf(n1, clampv)) ^ px,
             b2 = __float_as_uint(beta * fminf(n2, clampv)) ^ px;
    asm("" : "+v"(b1), "+v"(b2));   // keep the two products (not a product per edge)
    for_edges<C, c>([&](auto jj, auto kk) {
        constexpr int j = decltype(jj)::value, k = decltype(kk)::value;
        const uint32_t sel = fabsf(mu[j]) == n1 ? b2 : b1;
        const uint32_t nm = __builtin_amdgcn_bitop3_b32(sel, __float_as_uint(mu[j]), kSign, 0x78);   // sel ^ (mu & sign)
        if constexpr (FP) diff = __builtin_amdgcn_bitop3_b32(diff, nm, __float_as_uint(m[b + k]), 0xf6);   // diff | (nm ^ old)
        m[b + k] = __uint_as_float(nm);
    });
    // without the comparison the new messages are formed here all the same
    // (not next to their use in the partial sums, which would keep every
    // check's mu live until then)
    if constexpr (!FP) for_edges<C, c>([&m](auto, auto kk) { asm volatile("" : "+v"(m[b + decltype(kk)::value])); });
    asm volatile("" : "+v"(diff));
    __builtin_amdgcn_sched_barrier(0);
}

// Explicit messages: every m_{c->j} of the view in a register (edges
// numbered check by check, positions ascending within a check).  The
// messages are the compressed form's, bit for bit: magnitude beta * n2 on the
// edge of the smallest |mu| and beta * n1 elsewhere, sign = sign(mu_k) xor
// parity of all signs xor syndrome bit.  The edge of the smallest needs no
// tracking: it is an edge with |mu_k| == n1, and where several edges tie at
// n1, n2 == n1 and every choice gives the same message.
template <class C>
struct Explicit {
    static constexpr int R = C::R, E = C::E;
    float m[E];
    __device__ __forceinline__ void clear() {
#pragma unroll
        for (int e = 0; e < E; ++e) m[e] = 0.f;
    }
    __device__ __forceinline__ void reset_where(bool z) {
#pragma unroll
        for (int e = 0; e < E; ++e) m[e] = z ? 0.f : m[e];
    }
    template <bool FP = true>
    __device__ __forceinline__ bool check(const float (&S)[C::D * C::D], uint64_t sv, float beta, float clampv,
                                          bool &same, float keep = 1.f) {
        bool sat = true;
        uint32_t diff = 0u;   // see Compressed::check
        static_for<0, R>([&](auto cc) {
            constexpr int c = decltype(cc)::value;
            explicit_update<C, c, C::base[c], E, FP>(S, sv, beta, clampv, keep, m, sat, diff);
        });
        same = FP && diff == 0u;
        return sat;
    }
    template <int c, int k>
    __device__ __forceinline__ float msg() const { return m[C::base[c] + k]; }
    static constexpr int WORDS = E;
    __device__ __forceinline__ void save(float *p, int stride) const {
#pragma unroll
        for (int e = 0; e < E; ++e) p[e * stride] = m[e];
    }
    __device__ __forceinline__ void load(const float *p, int stride) {
#pragma unroll
        for (int e = 0; e < E; ++e) m[e] = p[e * stride];
    }
    __device__ __forceinline__ void accumulate(float (&S)[C::D * C::D], float keep = 1.f) const {
        static_for<0, R>([&](auto cc) {
            constexpr int c = decltype(cc)::value;
            for_edges<C, c>([&](auto jj, auto kk) {
                S[decltype(jj)::value] = __builtin_fmaf(m[C::base[c] + decltype(kk)::value], keep, S[decltype(jj)::value]);
            });
        });
    }
};

// Mixed storage for views with many edges: the checks of degree at least
// C::HYB keep the compressed state, the others one register per message
// (C::HYB = 0: none compressed).  Each check is updated exactly as in its own
// form, so the messages are bit for bit those of either; the mix keeps a
// view's state small enough for two waves per SIMD.
template <class C>
constexpr bool hyb_compressed(int c) { return C::HYB > 0 && C::deg[c] >= C::HYB; }
template <class C>
constexpr int hyb_index(int c) {   // compressed checks before check c
    int n = 0;
    for (int i = 0; i < c; ++i) n += hyb_compressed<C>(i) ? 1 : 0;
    return n;
}
template <class C>
constexpr int hyb_base(int c) {    // explicit edges before check c
    int n = 0;
    for (int i = 0; i < c; ++i) n += hyb_compressed<C>(i) ? 0 : C::deg[i];
    return n;
}

template <class C>
struct Hybrid {
    static constexpr int R = C::R;
    static constexpr int NC = hyb_index<C>(R) > 0 ? hyb_index<C>(R) : 1, EX = hyb_base<C>(R) > 0 ? hyb_base<C>(R) : 1;
    float m[EX];
    float m1[NC], m2[NC];
    uint32_t am[NC], q[NC];
    __device__ __forceinline__ void clear() {
#pragma unroll
        for (int e = 0; e < EX; ++e) m[e] = 0.f;
#pragma unroll
        for (int c = 0; c < NC; ++c) { m1[c] = 0.f; m2[c] = 0.f; am[c] = 0u; q[c] = 0u; }
    }
    __device__ __forceinline__ void reset_where(bool z) {
#pragma unroll
        for (int e = 0; e < EX; ++e) m[e] = z ? 0.f : m[e];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            m1[c] = z ? 0.f : m1[c];
            m2[c] = z ? 0.f : m2[c];
            am[c] = z ? 0u : am[c];
            q[c] = z ? 0u : q[c];
        }
    }
    template <bool FP = true>
    __device__ __forceinline__ bool check(const float (&S)[C::D * C::D], uint64_t sv, float beta, float clampv,
                                          bool &same, float keep = 1.f) {
        bool sat = true;
        uint32_t diff = 0u;   // see Compressed::check
        static_for<0, R>([&](auto cc) {
            constexpr int c = decltype(cc)::value;
            if constexpr (hyb_compressed<C>(c)) {
                constexpr int i = hyb_index<C>(c);
                compressed_update<C, c, FP>(S, sv, beta, clampv, keep, m1[i], m2[i], am[i], q[i], sat, diff);
            } else {
                explicit_update<C, c, hyb_base<C>(c), EX, FP>(S, sv, beta, clampv, keep, m, sat, diff);
            }
        });
        same = FP && diff == 0u;
        return sat;
    }
    static constexpr int WORDS = EX + 4 * NC;
    __device__ __forceinline__ void save(float *p, int stride) const {
#pragma unroll
        for (int e = 0; e < EX; ++e) p[e * stride] = m[e];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            p[(EX + 4 * c) * stride] = m1[c];
            p[(EX + 4 * c + 1) * stride] = m2[c];
            p[(EX + 4 * c + 2) * stride] = __uint_as_float(am[c]);
            p[(EX + 4 * c + 3) * stride] = __uint_as_float(q[c]);
        }
    }
    __device__ __forceinline__ void load(const float *p, int stride) {
#pragma unroll
        for (int e = 0; e < EX; ++e) m[e] = p[e * stride];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            m1[c] = p[(EX + 4 * c) * stride];
            m2[c] = p[(EX + 4 * c + 1) * stride];
            am[c] = __float_as_uint(p[(EX + 4 * c + 2) * stride]);
            q[c] = __float_as_uint(p[(EX + 4 * c + 3) * stride]);
        }
    }
    template <int c, int k>
    __device__ __forceinline__ float msg() const {
        if constexpr (hyb_compressed<C>(c)) {
            constexpr int i = hyb_index<C>(c);
            return msg_of(m1[i], m2[i], am[i], q[i], (uint32_t)k);
        } else {
            return m[hyb_base<C>(c) + k];
        }
    }
    __device__ __forceinline__ void accumulate(float (&S)[C::D * C::D], float keep = 1.f) const {
        static_for<0, R>([&](auto cc) {
            constexpr int c = decltype(cc)::value;
            for_edges<C, c>([&](auto jj, auto kk) {
                S[decltype(jj)::value] =
                    __builtin_fmaf(this->template msg<c, decltype(kk)::value>(), keep, S[decltype(jj)::value]);
            });
        });
    }
};

// Phase 1 state for views whose messages do not all fit beside the sums in
// the 256 VGPRs of two waves per SIMD: the checks in C::LDSMASK keep their
// messages in the wave's LDS (column lane of rows lm[e * 64], e numbering
// those checks' edges), the others one register per message.  Each check is
// updated exactly as in Explicit (its old messages read from LDS into
// registers, the new ones written back), so the bits do not change; the LDS
// messages start as zeros (the caller clears its column) and stay finite.
template <class C>
constexpr bool in_lds(int c) { return ((C::LDSMASK >> c) & 1u) != 0; }
template <class C>
constexpr int split_base(int c, bool lds) {   // edges before check c in its group
    int n = 0;
    for (int i = 0; i < c; ++i) n += in_lds<C>(i) == lds ? C::deg[i] : 0;
    return n;
}

template <class C>
struct ExplicitSplit {
    static constexpr int R = C::R;
    static constexpr int ER = split_base<C>(C::R, false), EL = split_base<C>(C::R, true);
    float m[ER > 0 ? ER : 1];
    float *lm;   // this lane's LDS column
    __device__ __forceinline__ void clear() {
#pragma unroll
        for (int e = 0; e < ER; ++e) m[e] = 0.f;
    }
    template <bool FP = true>
    __device__ __forceinline__ bool check(const float (&S)[C::D * C::D], uint64_t sv, float beta, float clampv,
                                          bool &same, float keep = 1.f) {
        bool sat = true;
        uint32_t diff = 0u;   // see Compressed::check
        static_for<0, R>([&](auto cc) {
            constexpr int c = decltype(cc)::value;
            if constexpr (in_lds<C>(c)) {
                constexpr int lb = split_base<C>(c, true), DEG = C::deg[c];
                float ml[DEG];
                static_for<0, DEG>([&](auto kk) { ml[decltype(kk)::value] = lm[(lb + decltype(kk)::value) * 64]; });
                explicit_update<C, c, 0, DEG, FP>(S, sv, beta, clampv, keep, ml, sat, diff);
                static_for<0, DEG>([&](auto kk) { lm[(lb + decltype(kk)::value) * 64] = ml[decltype(kk)::value]; });
            } else {
                explicit_update<C, c, split_base<C>(c, false), (ER > 0 ? ER : 1), FP>(S, sv, beta, clampv, keep, m,
                                                                                      sat, diff);
            }
        });
        same = FP && diff == 0u;
        return sat;
    }
    __device__ __forceinline__ void accumulate(float (&S)[C::D * C::D], float keep = 1.f) const {
        static_for<0, R>([&](auto cc) {
            constexpr int c = decltype(cc)::value;
            for_edges<C, c>([&](auto jj, auto kk) {
                constexpr int j = decltype(jj)::value, k = decltype(kk)::value;
                float mk;
                if constexpr (in_lds<C>(c)) mk = lm[(split_base<C>(c, true) + k) * 64];
                else mk = m[split_base<C>(c, false) + k];
                S[j] = __builtin_fmaf(mk, keep, S[j]);
            });
        });
    }
};

// Sum-product check update with one register per message (same storage and
// fixed-point test as Explicit).  Per check: mu_k = clamp(S_j - m_k), f_k =
// phi(|mu_k|); the message to edge k has magnitude phi(sum_{k' != k} f_k')
// and the min-sum sign rule.  The exclusive sums are formed without
// cancellation: with fmax the largest f (first edge a attaining it) and
// rest = the sum of all the others, edge a gets rest and every other edge
// fmax + (rest - f_k) (rest - f_k is small only next to fmax).
template <class C>
struct ExplicitSP {
    static constexpr int R = C::R, E = C::E;
    float m[E];
    __device__ __forceinline__ void clear() {
#pragma unroll
        for (int e = 0; e < E; ++e) m[e] = 0.f;
    }
    template <bool FP = true>
    __device__ __forceinline__ bool check(const float (&S)[C::D * C::D], uint64_t sv, float, float clampv,
                                          bool &same, float keep = 1.f) {
        constexpr int D2 = C::D * C::D;
        bool sat = true;
        uint32_t diff = 0u;
        static_for<0, R>([&](auto cc) {
            constexpr int c = decltype(cc)::value;
            constexpr int b = C::base[c];
            for_edges<C, c>([&](auto, auto kk) { asm volatile("" : "+v"(m[b + decltype(kk)::value])); });
            float mu[D2], f[D2], fmax = 0.f, rest = 0.f;
            uint32_t par = 0u, ps = 0u, amax = 0u;
            for_edges<C, c>([&](auto jj, auto kk) {
                constexpr int j = decltype(jj)::value, k = decltype(kk)::value;
                par ^= __float_as_uint(S[j]);
                mu[j] = clampf(__builtin_fmaf(-m[b + k], keep, S[j]), clampv);
                ps ^= __float_as_uint(mu[j]);
                f[j] = phi(fabsf(mu[j]));
                if constexpr (k == 0) {
                    fmax = f[j];
                    amax = (uint32_t)j;
                } else {
                    const bool gt = f[j] > fmax;
                    rest += gt ? fmax : f[j];
                    amax = gt ? (uint32_t)j : amax;
                    fmax = gt ? f[j] : fmax;
                }
            });
            const uint32_t sc = (uint32_t)(sv >> c) & 1u;
            sat = sat && ((par >> 31) == sc);
            const uint32_t px = (ps ^ (sc << 31)) & kSign;
            for_edges<C, c>([&](auto jj, auto kk) {
                constexpr int j = decltype(jj)::value, k = decltype(kk)::value;
                // fmax = +inf when some |mu| is 0: every other edge's
                // exclusive sum is then +inf (message 0)
                const float ex = (uint32_t)j == amax ? rest : fmax == __builtin_inff() ? fmax : fmax + (rest - f[j]);
                uint32_t mag = __float_as_uint(phi(ex));
                const uint32_t sgn = (__float_as_uint(mu[j]) & kSign) ^ px;
                if constexpr (FP) {
                    const uint32_t dterm = mag ^ sgn ^ __float_as_uint(m[b + k]);
                    diff |= dterm;
                    asm("" : "+v"(mag) : "v"(dterm));
                }
                m[b + k] = __uint_as_float(mag | sgn);
            });
            // without the comparison the new messages are formed here all
            // the same (see explicit_update)
            if constexpr (!FP) for_edges<C, c>([&](auto, auto kk) { asm volatile("" : "+v"(m[b + decltype(kk)::value])); });
            asm volatile("" : "+v"(diff));
            __builtin_amdgcn_sched_barrier(0);
        });
        same = FP && diff == 0u;
        return sat;
    }
    template <int c, int k>
    __device__ __forceinline__ float msg() const { return m[C::base[c] + k]; }
    static constexpr int WORDS = E;
    __device__ __forceinline__ void save(float *p, int stride) const {
#pragma unroll
        for (int e = 0; e < E; ++e) p[e * stride] = m[e];
    }
    __device__ __forceinline__ void load(const float *p, int stride) {
#pragma unroll
        for (int e = 0; e < E; ++e) m[e] = p[e * stride];
    }
    __device__ __forceinline__ void accumulate(float (&S)[C::D * C::D], float keep = 1.f) const {
        static_for<0, R>([&](auto cc) {
            constexpr int c = decltype(cc)::value;
            for_edges<C, c>([&](auto jj, auto kk) {
                S[decltype(jj)::value] = __builtin_fmaf(m[C::base[c] + decltype(kk)::value], keep, S[decltype(jj)::value]);
            });
        });
    }
};

// Check-state forms (lead_schedule.specialized; 3 = sum-product).  check()
// and accumulate() scale the stored messages by `keep`: mu = S - keep * m and
// S += keep * m, each a single fused multiply-add with one rounding, so
// keep = 1 is the plain subtraction / addition bit for bit and keep = 0 reads
// the state as all-zero messages without clearing it (the stored messages
// are always finite).
template <class C, int FORM>
struct Pick {
    using type = Compressed<C>;
};
template <class C>
struct Pick<C, 2> {
    using type = Explicit<C>;
};
template <class C>
struct Pick<C, 3> {
    using type = ExplicitSP<C>;
};
template <class C, int FORM>
using CheckState = typename Pick<C, FORM>::type;
// The Phase 1 queue kernel's state: form 2 with one prior per shot keeps the
// messages of the checks in C::LDSMASK in LDS (ExplicitSplit) where that
// mask is set (with a prior per qubit the kernel runs one wave per SIMD
// anyway).
template <class C, int FORM, int PM, bool SPLITLDS = (FORM == 2 && PM == 0 && C::LDSMASK != 0u)>
struct LocalPick {
    using type = CheckState<C, FORM>;
};
template <class C, int FORM, int PM>
struct LocalPick<C, FORM, PM, true> {
    using type = ExplicitSplit<C>;
};

// The Phases 2-3 kernel keeps the mixed storage where C::HYB is set (views
// whose one-register-per-message state would take more than half the
// register file); the Phase 1 queue kernel keeps the explicit form.
template <class C, int FORM, bool H = (FORM == 2 && C::HYB > 0)>
struct PickGlobal {
    using type = CheckState<C, FORM>;
};
template <class C, int FORM>
struct PickGlobal<C, FORM, true> {
    using type = Hybrid<C>;
};
template <class C, int FORM>
using GlobalState = typename PickGlobal<C, FORM>::type;

// Whether [S_j < 0] satisfies every check of the view.
template <class C>
__device__ __forceinline__ bool parity(const float (&S)[C::D * C::D], uint64_t sv) {
    bool sat = true;
    static_for<0, C::R>([&](auto cc) {
        constexpr int c = decltype(cc)::value;
        uint32_t par = 0u;
        for_edges<C, c>([&](auto jj, auto) { par ^= __float_as_uint(S[decltype(jj)::value]); });
        sat = sat && ((par >> 31) == ((uint32_t)(sv >> c) & 1u));
    });
    return sat;
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

// Cost of setting a bit whose prior LLR is x in the combination sweep:
// round(64 ln(1 + e^x)) = round(64 ln(1/p)), p = 1/(1 + e^x), an exact
// integer so that candidate costs compare the same in any summation order.
__device__ __forceinline__ int32_t osd_weight(float x) {
    const float w = fmaxf(x, 0.f) + log1p_nonneg(exp_hw(-fabsf(x)));
    return (int32_t)__builtin_rintf(64.f * w);
}

// The r-bit column of local position j (runtime j): the view's checks on it.
template <class C>
__device__ __forceinline__ uint32_t local_column(int j) {
    uint32_t col = 0u;
    static_for<0, C::R>([&](auto cc) {
        constexpr int c = decltype(cc)::value;
        col |= (uint32_t)((C::mask[c] >> j) & 1ull) << c;
    });
    return col;
}

// Position of the smallest key among `left` (equal keys: the lowest
// position).
template <int D2>
__device__ __forceinline__ int take_smallest(const float (&key)[D2], uint64_t left) {
    float best = __builtin_inff();
    int bj = -1;
    static_for<0, D2>([&](auto jj) {
        constexpr int j = decltype(jj)::value;
        const bool lt = ((left >> j) & 1ull) && (bj < 0 || key[j] < best);
        best = lt ? key[j] : best;
        bj = lt ? j : bj;
    });
    return bj;
}

// OSD of the view (local post-processing): positions are taken by
// round(64 L) of the clamped posterior LLR ascending (most likely in error
// first; equal keys in position order, so reliabilities that agree to 1/64
// count as equal), each column (the r-bit set of the view's checks on that
// position) is reduced against a GF(2) basis kept by lowest set bit and
// joins it when independent, until the basis has rank r; the OSD-0 estimate
// is the combination of basis columns that gives the local syndrome (a bit
// mask over positions).  With order > 0 (combination sweep) the candidates
// that follow are, in this order, the solutions with one non-basis position
// t set (positions in rank order) and with two set among the first `order`
// non-basis positions; the first candidate of least cost sum_{e_j = 1} q_j
// wins.  ok = false when the syndrome is not reached (H_v not of full row
// rank).
template <class C>
__device__ __forceinline__ uint64_t osd_local(const float (&L)[C::D * C::D], const int32_t (&q)[C::D * C::D],
                                              uint64_t sv, int order, bool &ok) {
    constexpr int D2 = C::D * C::D, R = C::R;
    uint32_t bvec[R];
    uint64_t bcomb[R];
#pragma unroll
    for (int b = 0; b < R; ++b) { bvec[b] = 0u; bcomb[b] = 0ull; }
    uint32_t have = 0u;
    constexpr uint64_t all = D2 == 64 ? ~0ull : ((1ull << D2) - 1ull);
    uint64_t left = all, piv = 0ull;
    float key[D2];
#pragma unroll
    for (int j = 0; j < D2; ++j) key[j] = __builtin_rintf(L[j] * 64.f);   // exact scaling, round half to even
    int nb = 0;
    for (int step = 0; step < D2 && nb < R; ++step) {
        const int bj = take_smallest<D2>(key, left);
        left &= ~(1ull << bj);
        uint32_t col = local_column<C>(bj);
        uint64_t comb = 1ull << bj;
        bool placed = false;
        static_for<0, R>([&](auto bb) {
            constexpr int b = decltype(bb)::value;
            if (!placed && ((col >> b) & 1u)) {
                if ((have >> b) & 1u) {
                    col ^= bvec[b];
                    comb ^= bcomb[b];
                } else {
                    bvec[b] = col;
                    bcomb[b] = comb;
                    have |= 1u << b;
                    placed = true;
                }
            }
        });
        if (placed) piv |= 1ull << bj;
        nb += placed ? 1 : 0;
    }
    // the combination of basis columns that gives x
    auto solve = [&](uint32_t x, uint32_t &rest) {
        uint64_t e = 0ull;
        static_for<0, R>([&](auto bb) {
            constexpr int b = decltype(bb)::value;
            if (((x >> b) & 1u) && ((have >> b) & 1u)) {
                x ^= bvec[b];
                e ^= bcomb[b];
            }
        });
        rest = x;
        return e;
    };
    uint32_t rest;
    uint64_t e = solve((uint32_t)sv, rest);
    ok = rest == 0u;
    if (!ok) return 0ull;
    if (order <= 0) return e;
    auto cost = [&](uint64_t ee) {
        int32_t c = 0;
        static_for<0, D2>([&](auto jj) {
            constexpr int j = decltype(jj)::value;
            c += ((ee >> j) & 1ull) ? q[j] : 0;
        });
        return c;
    };
    int32_t best = cost(e);
    int tl[lead::kMaxOsdOrderLocal];
#pragma unroll
    for (int k = 0; k < lead::kMaxOsdOrderLocal; ++k) tl[k] = 0;
    int nt = 0;
    left = all;
    for (int step = 0; step < D2; ++step) {
        const int bj = take_smallest<D2>(key, left);
        left &= ~(1ull << bj);
        if ((piv >> bj) & 1ull) continue;
        uint32_t r1;
        const uint64_t ee = solve((uint32_t)sv ^ local_column<C>(bj), r1) ^ (1ull << bj);
        const int32_t c = cost(ee);
        if (c < best) {
            best = c;
            e = ee;
        }
#pragma unroll
        for (int k = 0; k < lead::kMaxOsdOrderLocal; ++k) tl[k] = (nt == k) ? bj : tl[k];
        ++nt;
    }
    const int lam = order < nt ? order : nt;
    for (int x = 0; x < lam; ++x)
        for (int y = x + 1; y < lam; ++y) {
            int ta = 0, tb = 0;
#pragma unroll
            for (int k = 0; k < lead::kMaxOsdOrderLocal; ++k) {
                int v = tl[k];
                asm("" : "+v"(v));   // a value, not a load the select could turn into one
                ta = (k == x) ? v : ta;
                tb = (k == y) ? v : tb;
            }
            uint32_t r2;
            const uint64_t ee =
                solve((uint32_t)sv ^ local_column<C>(ta) ^ local_column<C>(tb), r2) ^ (1ull << ta) ^ (1ull << tb);
            const int32_t c = cost(ee);
            if (c < best) {
                best = c;
                e = ee;
            }
        }
    return e;
}

// Phase 1 as a work queue over (shot, vertex) items: a lane runs the local BP
// of one item with S in VGPRs and takes the next item as soon as its run
// ends.  Stopping rules and outputs are those of the precompiled local
// kernel: Lv[item][j] = clamp(S_j), vflag[item] = iterations | converged << 16
// | fixed point << 17.
//
// Every step of the loop is executed by all lanes, with or without an item
// (the variable update S^{t-1} = lambda + sum of messages, then the check
// update of iteration t; a fresh item has all-zero messages, so its first
// variable update gives S^0 = lambda exactly).  Only the output stores are
// divergent.  Updating S or the check states under a divergent branch would
// make the compiler keep the old and the new copies of them live at once.
// Items are tested for a fixed point at even t (the rule of the precompiled
// kernels too).  In form 2 with one prior per shot, where the code allows it
// (C::LOCAL_ALT: the views' messages in registers, or enough of them in LDS
// that two iterations fit the registers of two waves per SIMD), the loop
// runs two iterations per pass, the first without the test (new messages
// overwrite the old ones in place), the second with it, and hands out items
// only before the first, so that every item starts at an odd pass step: the
// comparison, its copies at the back-edge and the hand-out cost once per two
// iterations; a lane whose run ends in the first iteration idles in the
// second.  Elsewhere (a prior per qubit, the other forms, views whose LDS
// share would not leave room for eight waves per CU) one iteration per pass,
// each compiled with the comparison.
template <class C, int PM, int FORM>
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
    typename LocalPick<C, FORM, PM>::type st;
    if constexpr (FORM == 2 && PM == 0 && C::LDSMASK != 0u) {
        extern __shared__ float lds_local[];
        st.lm = lds_local + lane;
#pragma unroll
        for (int e = 0; e < ExplicitSplit<C>::EL; ++e) st.lm[e * 64] = 0.f;
    }
    st.clear();
    float keep = 0.f;
    constexpr bool ALT = FORM == 2 && PM == 0 && C::LOCAL_ALT;
    // One iteration of the item in each lane: the variable update, then the
    // check update with or without the fixed-point test.
    auto step = [&](auto fp_tag) {
        constexpr bool FPT = decltype(fp_tag)::value == 1;
#pragma unroll
        for (int j = 0; j < D2; ++j) S[j] = lam[PM == 0 ? 0 : j];
        st.accumulate(S, keep);
        bool same;
        const bool sat = st.template check<FPT>(S, sv, a.beta, a.clampv, same, keep);
        keep = 1.f;
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
        } else if (FPT && (t & 1) == 0 && same && a.fixed_stop) {
            conv = sat ? 1 : 0;
            it = a.Tl;
            fixed = 1;
            fin = true;
        }
        if (valid && fin) {
            float *out = w.Lv + item * D2;
            float Lc[D2];
#pragma unroll
            for (int j = 0; j < D2; ++j) Lc[j] = clampf(S[j], a.clampv);
#pragma unroll
            for (int j = 0; j < D2; ++j) out[j] = Lc[j];
            w.vflag[item] = (uint32_t)it | ((uint32_t)conv << 16) | ((uint32_t)fixed << 17);
            // a view that missed its local syndrome is post-processed by
            // local_osd_body with every lane busy, not here with one
            if (a.local_osd && !conv)
                w.osd_list[atomicAdd(reinterpret_cast<unsigned long long *>(w.counter + 1), 1ull)] = (uint32_t)item;
            valid = false;
        }
        ++t;
    };
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
                keep = 0.f;   // the previous item's messages read as zero
                if (PM == 0) {
                    lam[0] = a.prior[shot] + 0.f;
                } else {
                    const int64_t base = a.prior_mode == 2 ? shot * a.n : 0;
#pragma unroll
                    for (int j = 0; j < NL; ++j) lam[j] = a.prior[base + a.view[v * D2 + j]] + 0.f;
                }
                t = 1;
            }
            const int64_t taken = __popcll(need) < avail ? __popcll(need) : avail;
            cur += taken;
            need = __ballot(!valid);
        }
        if (__ballot(valid) == 0ull) break;
        if constexpr (ALT) {
            step(Int<0>{});   // odd t: no fixed-point test
            if (__ballot(valid) == 0ull) continue;
        }
        step(Int<1>{});
    }
}

// The first check (in check order) with an edge at local position j, or -1.
template <class C>
constexpr int first_check(int j) {
    for (int c = 0; c < C::R; ++c)
        if ((C::mask[c] >> j) & 1ull) return c;
    return -1;
}

// Partial sums of a view for one global round: P_j = (lambda'_j where the
// view owns position j, else 0) + its checks' messages to j in check order.
// Where the view does not own j the zero start is dropped: 0 + m equals m
// except that -0 becomes +0, and such a P_j is only ever added to the owner's
// P, which is never -0 (it starts from lambda', itself never -0), so every
// sum S_j comes out the same.
template <class C, class ST>
__device__ __forceinline__ void partial_sums(const ST &st, const float (&lam)[C::D * C::D], uint64_t fown,
                                             float (&P)[C::D * C::D]) {
    static_for<0, C::D * C::D>([&](auto jj) {
        constexpr int j = decltype(jj)::value;
        if constexpr (first_check<C>(j) < 0) {
            if constexpr (C::sigma[j] > j) P[j] = lam[j];
            else if constexpr (C::sigma[j] < j) P[j] = 0.f;
            else P[j] = ((fown >> j) & 1ull) ? lam[j] : 0.f;
        }
    });
    static_for<0, C::R>([&](auto cc) {
        constexpr int c = decltype(cc)::value;
        for_edges<C, c>([&](auto jj, auto kk) {
            constexpr int j = decltype(jj)::value, k = decltype(kk)::value;
            const float m = st.template msg<c, k>();
            if constexpr (first_check<C>(j) == c) {
                if constexpr (C::sigma[j] > j) P[j] = lam[j] + m;
                else if constexpr (C::sigma[j] < j) P[j] = m;
                else P[j] = ((fown >> j) & 1ull) ? lam[j] + m : m;
            } else {
                P[j] += m;
            }
        });
    });
}

// Local post-processing of the views listed by the queue kernel: OSD of
// order a.osd_order on the view (osd_local above, costs from the view's
// channel priors); where it reaches the local syndrome the view counts
// as converged, is flagged as resolved by OSD-0, and the confidence boost
// (p <- max(p, 1/2) on its errors, i.e. L <- min(L, 0)) is applied to its
// stored posteriors.  Lanes stride over the list.
template <class C>
__device__ __forceinline__ void local_osd_body(const DecodeArgs &a, const LocalArgs &w) {
    constexpr int D2 = C::D * C::D;
    const int64_t count = w.counter[1];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
        const int64_t item = w.osd_list[i];
        const int64_t shot = item / a.N;
        const int v = (int)(item - shot * a.N);
        const uint64_t sv = local_syndrome(a, shot, v);
        float *io = w.Lv + item * D2;
        float Lc[D2];
#pragma unroll
        for (int j = 0; j < D2; ++j) Lc[j] = io[j];
        int32_t q[D2];
#pragma unroll
        for (int j = 0; j < D2; ++j) q[j] = 0;
        if (a.osd_order > 0) {
            // the sweep's costs: the view's channel priors
            const int64_t base = a.prior_mode == 2 ? shot * a.n : 0;   // LEAD_PRIOR_FULL
#pragma unroll
            for (int j = 0; j < D2; ++j)
                q[j] = osd_weight(a.prior_mode == 0 ? a.prior[shot] : a.prior[base + a.view[v * D2 + j]]);
        }
        bool ok;
        const uint64_t e = osd_local<C>(Lc, q, sv, a.osd_order, ok);
        if (ok) {
            if (a.boost) {
#pragma unroll
                for (int j = 0; j < D2; ++j)
                    if ((e >> j) & 1ull) io[j] = fminf(Lc[j], 0.f);
            }
            w.vflag[item] |= (1u << 16) | (1u << 18);
        }
    }
}

// Per-shot LDS flags (the precompiled kernel's layout).
enum { SF_FLAG0 = 0, SF_FLAG1 = 1, SF_FINAL = 2, SF_ITSUM = 3, SF_ITMAX = 4, SF_NCONV = 5, SF_CHG = 6, SF_NFIX = 7,
       SF_NOSD = 8, SF_STRIDE = 9 };

// Partner addresses: for local position j, the lane that holds the other
// occurrence of the qubit.  Within one wave (BPERM) its byte address
// (lane * 4, 8 bits); across the waves of a workgroup of at most 256 lanes
// the lane itself (8 bits); four per register.  Larger workgroups: the byte
// address in 16 bits, two per register.
template <bool BPERM, int WG>
struct PartnerAddr {
    static constexpr int PER = (BPERM || WG <= 256) ? 4 : 2, BITS = 32 / PER;
    static constexpr uint32_t MASK = PER == 4 ? 0xffu : 0xffffu;
    static constexpr uint32_t SCALE = (BPERM || PER == 2) ? 4u : 1u;   // stored value = lane * SCALE
    template <int D2>
    static constexpr int words() { return (D2 + PER - 1) / PER; }
};

template <bool BPERM, int WG, int J, int NW>
__device__ __forceinline__ uint32_t partner_addr(const uint32_t (&pa)[NW]) {
    using A = PartnerAddr<BPERM, WG>;
    return (pa[J / A::PER] >> ((J % A::PER) * A::BITS)) & A::MASK;
}

// Value of X at the other occurrence of local position J: lane `addr` holds
// it at position sigma[J].  BPERM: the partner lane is in the same wave and
// is read with ds_bpermute; otherwise X has been stored to LDS as
// buf[j][lane].
template <class C, int WG, bool BPERM, int J>
__device__ __forceinline__ float partner(const float (&X)[C::D * C::D], const float *buf, uint32_t addr) {
    if (BPERM)
        return __int_as_float(__builtin_amdgcn_ds_bpermute((int)addr, __float_as_int(X[C::sigma[J]])));
    if (PartnerAddr<BPERM, WG>::SCALE == 1u) return buf[C::sigma[J] * WG + addr];
    return *reinterpret_cast<const float *>(reinterpret_cast<const char *>(buf) + C::sigma[J] * WG * 4 + addr);
}

template <class C, int WG, bool BPERM, int NW, int J = 0>
__device__ __forceinline__ void partner_all(const float (&X)[C::D * C::D], float (&Y)[C::D * C::D],
                                            const float *buf, const uint32_t (&pa)[NW]) {
    if constexpr (J < C::D * C::D) {
        Y[J] = partner<C, WG, BPERM, J>(X, buf, partner_addr<BPERM, WG, J>(pa));
        partner_all<C, WG, BPERM, NW, J + 1>(X, Y, buf, pa);
    }
}

template <class C, int WG, bool BPERM>
__device__ __forceinline__ void store_all(const float (&X)[C::D * C::D], float *buf, int tid) {
    if (!BPERM) {
#pragma unroll
        for (int j = 0; j < C::D * C::D; ++j) buf[j * WG + tid] = X[j];
        __syncthreads();
    }
}

// Positions j with sigma[j] >= j (those a view may own) and the rank of j
// among them.
template <class C>
constexpr int owner_slots() {
    int n = 0;
    for (int j = 0; j < C::D * C::D; ++j) n += C::sigma[j] >= j ? 1 : 0;
    return n;
}
template <class C>
constexpr int owner_slot(int j) {
    int n = 0;
    for (int i = 0; i < j; ++i) n += C::sigma[i] >= i ? 1 : 0;
    return n;
}
template <class C, bool BPERM, int FORM>
constexpr bool lam_in_lds() { return !BPERM && C::LAM_LDS && (FORM == 1 || (FORM == 2 && C::HYB > 0)); }

// Phases 2-3 of `spw` shots per workgroup after the Phase 1 queue kernel;
// lane (slot, v) holds vertex v of shot blk.index * spw + slot.  The same
// computation as the precompiled split kernel: lambda' of every qubit from
// its two clamped local posteriors, then global min-sum rounds in which each
// view forms its partial sum P_j (lambda' on owned positions, then its
// checks' messages in check order) and S_j = P_j + P_j' of the other
// occurrence.
// PLAIN (the plain per-round form): one launch per round pl.round, the sums
// S and the check state restored from and saved to device memory between
// launches, the same arithmetic in the same order (outputs identical bit for
// bit); a shot writes its outputs in the launch where its run ends, and the
// launch of round Tg + 1 ends the shots that ran to the cap.
// The block a call of global_body decodes: its index in the code's grid of
// per-shot blocks, the lane within it, and its LDS.  A kernel launched for
// one code uses the launch's block (of_launch); a kernel fusing several
// codes runs several blocks of a code with a smaller block in one workgroup
// (one per wave or group of waves), each with its own LDS region.
struct Blk {
    int64_t index;
    int tid;
    float *lds;
    __device__ static Blk of_launch() {
        extern __shared__ float lds_launch[];
        return Blk{(int64_t)blockIdx.x, (int)threadIdx.x, lds_launch};
    }
};

template <class C, int WG, bool BPERM, int FORM, bool PLAIN = false, bool FP = true>
__device__ __forceinline__ void global_body(const DecodeArgs &a, const LocalArgs &w, const SpecArgs &x,
                                            const lead::PlainArgs &pl = lead::PlainArgs{},
                                            const Blk blk = Blk::of_launch()) {
    constexpr int D2 = C::D * C::D;
    constexpr int NP = (D2 + 1) / 2;                          // words of the host's 16-bit table
    constexpr int NW = PartnerAddr<BPERM, WG>::template words<D2>();  // words of the packed addresses
    // across waves, with the compressed or the mixed check state, lambda' of
    // the positions a view may own (sigma[j] >= j) waits in LDS between
    // rounds, not in VGPRs (two waves per SIMD)
    constexpr bool LAML = lam_in_lds<C, BPERM, FORM>();
    // within one wave: whether the partner addresses are unpacked each
    // round (the check state, sums and packed addresses plus the round's
    // temporaries would otherwise exceed 256 VGPRs; the 77-edge A5 X-check
    // views of form 2), or kept unpacked across the loop (one instruction
    // per position and round saved)
    constexpr bool REUNPACK = BPERM && (FORM == 1 ? 4 * C::R : C::E) + D2 + NW + 140 > 256;
    constexpr int NO = LAML ? owner_slots<C>() : 0;
    float *lds = blk.lds;
    float *buf = lds;
    float *laml = lds + (BPERM ? 0 : D2 * WG);
    int *shf = reinterpret_cast<int *>(lds + (BPERM ? 0 : D2 * WG) + NO * WG);
    const int ew32 = (a.n + 31) >> 5;
    uint32_t *ebits = reinterpret_cast<uint32_t *>(shf + a.spw * SF_STRIDE);
    const int tid = blk.tid;
    const int sl = tid / a.N, v = tid - sl * a.N;
    const bool lane_ok = sl < a.spw;
    const int64_t shot = blk.index * a.spw + sl;
    bool live = lane_ok && shot < a.shots;
    if constexpr (PLAIN) {
        // a shot whose run ended in an earlier launch is left alone (with
        // one shot per workgroup the whole workgroup leaves)
        if (pl.round > 1) {
            if constexpr (!BPERM) {
                const int64_t ws = blk.index * a.spw;
                if (ws >= a.shots || pl.ended[ws] != 0) return;
            }
            if (live && pl.ended[shot] != 0) live = false;
        }
    }
    for (int i = tid; i < a.spw * SF_STRIDE; i += WG) shf[i] = 0;
    for (int i = tid; i < a.spw * ew32; i += WG) ebits[i] = 0u;

    float S[D2];
    uint32_t pa[NW];
    uint64_t sv = 0, fown = 0;
    int it_v = 0, conv_v = 0, fixed_v = 0, osd_v = 0;
    if (live) {
        sv = local_syndrome(a, shot, v);
        if (a.global_only) {
            // global BP alone: no local phase, lambda' is the channel prior
#pragma unroll
            for (int j = 0; j < D2; ++j) S[j] = 0.f;
        } else {
            const int64_t item = shot * a.N + v;
            const float *in = w.Lv + item * D2;
#pragma unroll
            for (int j = 0; j < D2; ++j) S[j] = in[j];
            const uint32_t f = w.vflag[item];
            it_v = (int)(f & 0xffffu);
            conv_v = (int)((f >> 16) & 1u);
            fixed_v = (int)((f >> 17) & 1u);
            osd_v = (int)((f >> 18) & 1u);
        }
        const uint32_t base = (uint32_t)(sl * a.N);
        using A = PartnerAddr<BPERM, WG>;
#pragma unroll
        for (int k = 0; k < NW; ++k) pa[k] = 0u;
#pragma unroll
        for (int j = 0; j < D2; ++j) {
            const uint32_t vp = (x.pv[v * NP + j / 2] >> (16 * (j & 1))) & 0xffffu;
            pa[j / A::PER] |= ((base + vp) * A::SCALE) << ((j % A::PER) * A::BITS);
        }
        if (C::NFIX) fown = x.fown[v];
    } else {
#pragma unroll
        for (int j = 0; j < D2; ++j) S[j] = 0.f;
        using A = PartnerAddr<BPERM, WG>;
#pragma unroll
        for (int k = 0; k < NW; ++k)
            pa[k] = (uint32_t)tid * A::SCALE * (A::PER == 4 ? 0x01010101u : 0x10001u);
    }
    __syncthreads();
    if (live) {
        atomicAdd(&shf[sl * SF_STRIDE + SF_ITSUM], it_v);
        atomicMax(&shf[sl * SF_STRIDE + SF_ITMAX], it_v);
        atomicAdd(&shf[sl * SF_STRIDE + SF_NCONV], conv_v & (osd_v ^ 1));   // converged by BP
        if (fixed_v) atomicAdd(&shf[sl * SF_STRIDE + SF_NFIX], 1);
        if (osd_v) atomicAdd(&shf[sl * SF_STRIDE + SF_NOSD], 1);
    }
    auto owned = [&](int j) { return C::sigma[j] > j || (C::sigma[j] == j && ((fown >> j) & 1ull)); };

    // ---- Phase 2: lambda' of every position (symmetric in the two views, so
    // both occurrences of a qubit compute the same value); the confidence
    // boost L <- min(L, 0) on L < 0 leaves L unchanged.
    float lam[D2];
    if (a.global_only) {
        const int64_t base = a.prior_mode == 2 ? shot * a.n : 0;   // LEAD_PRIOR_FULL
#pragma unroll
        for (int j = 0; j < D2; ++j)
            lam[j] = live ? (a.prior_mode == 0 ? a.prior[shot] : a.prior[base + a.view[v * D2 + j]]) + 0.f : 0.f;
    } else {
        float Lp[D2];
        store_all<C, WG, BPERM>(S, buf, tid);
        partner_all<C, WG, BPERM, NW>(S, Lp, buf, pa);
#pragma unroll
        for (int j = 0; j < D2; ++j) lam[j] = aggregate_llr(clampf(S[j], a.clampv), clampf(Lp[j], a.clampv), a.alpha, a.clampv);
    }
    if (a.lam_out && live && (!PLAIN || pl.round == 1)) {
#pragma unroll
        for (int j = 0; j < D2; ++j)
            if (owned(j)) a.lam_out[shot * a.n + a.view[v * D2 + j]] = lam[j];
    }
    if constexpr (LAML) {
        static_for<0, D2>([&](auto jj) {
            constexpr int j = decltype(jj)::value;
            if constexpr (C::sigma[j] >= j) laml[owner_slot<C>(j) * WG + tid] = lam[j];
        });
    }
    if (a.stage == 1) {
        __syncthreads();
        if (live && v == 0 && a.stats) {
            lead::ShotStats s = {};
            s.local_iters_sum = shf[sl * SF_STRIDE + SF_ITSUM];
            s.local_iters_max = shf[sl * SF_STRIDE + SF_ITMAX];
            s.local_converged_views = shf[sl * SF_STRIDE + SF_NCONV];
            s.local_fixed_views = shf[sl * SF_STRIDE + SF_NFIX];
            s.local_osd_views = shf[sl * SF_STRIDE + SF_NOSD];
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
    using State = GlobalState<C, FORM>;
    State st;
    bool resumed = false;
    if constexpr (PLAIN) resumed = pl.round > 1 && live;
    if (resumed) {
#pragma unroll
        for (int j = 0; j < D2; ++j) S[j] = pl.S[(shot * D2 + j) * a.N + v];
        st.load(pl.st + shot * State::WORDS * a.N + v, a.N);
    } else {
#pragma unroll
        for (int j = 0; j < D2; ++j) S[j] = lam[j];
        st.clear();
    }
    if (!BPERM) __syncthreads();
    bool done = !live;
    bool wdone = false;   // the workgroup's shot has ended (one shot per workgroup, !BPERM)
    int itg = 0, gconv = 0, gfix = 0;
    // lanes of this lane's shot within the wave (one-wave workgroups)
    const uint64_t smask = lane_ok ? ((a.N >= 64 ? ~0ull : ((1ull << a.N) - 1ull)) << (sl * a.N)) : 0ull;
    int t0 = 1, t1 = a.Tg;
    if constexpr (PLAIN) {
        t0 = pl.round;
        t1 = pl.round <= a.Tg ? pl.round : a.Tg;   // round Tg + 1: no iteration
    }
    for (int t = t0; t <= t1; ++t) {
        // computed by every lane (see local_body); done lanes discard it
        bool same;
        const bool sat = st.template check<FP>(S, sv, a.beta, a.clampv, same);
        bool shot_sat, shot_same = false;
        if constexpr (BPERM) {
            // the shot's flags are ballots over its lanes: no LDS, no barrier
            const uint64_t unsat = __ballot(!done && !sat);
            shot_sat = (unsat & smask) == 0ull;
            if constexpr (FP) shot_same = (__ballot(!done && !same) & smask) == 0ull;
        } else {
            // more than 64 views: one shot per workgroup (its live lanes
            // have sl = 0), whose flags every lane reads, so that the end of
            // its run is known to all lanes without a second barrier
            if (!done && !sat) shf[(t & 1)] = 1;
            if (FP && !done && !same) shf[SF_CHG] = t;
            __syncthreads();
            shot_sat = shf[(t & 1)] == 0;
            if constexpr (FP) shot_same = shf[SF_CHG] != t;
        }
        // (one shot per workgroup, !BPERM: the loop ends right here for
        // every lane, and the outputs are written after it, from the same S)
        if (!done && t > 1) {
            if (shot_sat && a.early_exit) {
                done = true;
                gconv = 1;
                itg = t - 1;
                if constexpr (BPERM) emit();
            } else if (FP && a.fixed_stop_g && shot_same) {
                done = true;
                gconv = shot_sat ? 1 : 0;
                itg = a.Tg;
                gfix = t;
                if constexpr (BPERM) emit();
            }
        }
        if constexpr (BPERM) {
            if (__ballot(!done) == 0ull) break;
        } else {
            // the live lanes' own decision above, taken by every lane
            if (!wdone && t > 1 && ((shot_sat && a.early_exit) || (FP && a.fixed_stop_g && shot_same))) wdone = true;
            if (wdone) break;
            if (tid == 0) shf[((t + 1) & 1)] = 0;
        }
        // partial sums of this view, then S_j = P_j + P of the other occurrence
        if constexpr (LAML) {
            float lr[D2];
            static_for<0, D2>([&](auto jj) {
                constexpr int j = decltype(jj)::value;
                lr[j] = C::sigma[j] >= j ? laml[owner_slot<C>(j) * WG + tid] : 0.f;
            });
            partial_sums<C>(st, lr, fown, S);
        } else {
            partial_sums<C>(st, lam, fown, S);
        }
        if constexpr (BPERM) {
            // the owner of a qubit adds its partner's P (fixed points of
            // sigma: both occurrences, as ownership is known only at run
            // time); the other occurrence then reads the owner's sum, which
            // is the same sum with the operands swapped (IEEE addition is
            // commutative)
            float Q[D2];
            // where the view's state leaves no room for the unpacked
            // partner addresses (one per position) across the loop, they are
            // unpacked here each round
            if constexpr (REUNPACK) {
#pragma unroll
                for (int k = 0; k < NW; ++k) asm volatile("" : "+v"(pa[k]));
            }
            static_for<0, D2>([&](auto jj) {
                constexpr int j = decltype(jj)::value;
                if constexpr (C::sigma[j] >= j) Q[j] = partner<C, WG, BPERM, j>(S, buf, partner_addr<BPERM, WG, j>(pa));
            });
            static_for<0, D2>([&](auto jj) {
                constexpr int j = decltype(jj)::value;
                if constexpr (C::sigma[j] >= j) S[j] += Q[j];
            });
            static_for<0, D2>([&](auto jj) {
                constexpr int j = decltype(jj)::value;
                if constexpr (C::sigma[j] < j) S[j] = partner<C, WG, BPERM, j>(S, buf, partner_addr<BPERM, WG, j>(pa));
            });
        } else {
            // through LDS, sixteen positions at a time (all 64 partner
            // values in flight at once would need 64 more registers); the
            // addresses are unpacked here each round, not kept unpacked
            // across the loop
#pragma unroll
            for (int k = 0; k < NW; ++k) asm volatile("" : "+v"(pa[k]));
            store_all<C, WG, BPERM>(S, buf, tid);
            static_for<0, (D2 + 15) / 16>([&](auto qq) {
                constexpr int j0 = 16 * decltype(qq)::value;
                float Q[16];
                static_for<0, 16>([&](auto ii) {
                    constexpr int j = j0 + decltype(ii)::value;
                    if constexpr (j < D2) Q[j - j0] = partner<C, WG, BPERM, j>(S, buf, partner_addr<BPERM, WG, j>(pa));
                });
                static_for<0, 16>([&](auto ii) {
                    constexpr int j = j0 + decltype(ii)::value;
                    if constexpr (j < D2) S[j] += Q[j - j0];
                });
                __builtin_amdgcn_sched_barrier(0);
            });
        }
        }
    // plain form before the last round: a shot still running keeps its state
    // for the next launch and writes nothing else
    bool hold = false;
    if constexpr (PLAIN) hold = live && !done && pl.round <= a.Tg;
    const bool ran_out = !done && !hold;
    const bool psat = parity<C>(S, sv);
    bool shot_final;
    if constexpr (BPERM) {
        shot_final = (__ballot(ran_out && !psat) & smask) == 0ull;
    } else {
        if (ran_out && !psat) shf[sl * SF_STRIDE + SF_FINAL] = 1;
        __syncthreads();
        shot_final = shf[sl * SF_STRIDE + SF_FINAL] == 0;
    }
    if (ran_out) {
        gconv = shot_final ? 1 : 0;
        itg = a.Tg;
        if constexpr (BPERM) emit();
    }
    if constexpr (!BPERM) {
        if (live && !hold) emit();
    }
    __syncthreads();
    if constexpr (PLAIN) {
        if (hold) {
#pragma unroll
            for (int j = 0; j < D2; ++j) pl.S[(shot * D2 + j) * a.N + v] = S[j];
            st.save(pl.st + shot * State::WORDS * a.N + v, a.N);
            if (v == 0) atomicAdd(pl.active, 1);
        }
        if (live && v == 0) pl.ended[shot] = hold ? 0 : 1;
    }
    if (live && !hold) {
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
            s.local_iters_sum = shf[sl * SF_STRIDE + SF_ITSUM];
            s.local_iters_max = shf[sl * SF_STRIDE + SF_ITMAX];
            s.local_converged_views = shf[sl * SF_STRIDE + SF_NCONV];
            s.local_fixed_views = shf[sl * SF_STRIDE + SF_NFIX];
            s.local_osd_views = shf[sl * SF_STRIDE + SF_NOSD];
            s.global_fixed_iter = gfix;
            reinterpret_cast<lead::ShotStats *>(a.stats)[shot] = s;
        }
    }
}

// ---------------------------------------------------------------------------
// Phases 2-3 for views that span several waves, as a persistent kernel: a
// workgroup of kTileWG lanes (eight waves, two per SIMD) holds K = kTileWG / N
// shots at once (three PSL(2,7) shots on 504 of its 512 lanes), and each of
// its K slots takes the next shot from a device counter (w.counter[3]) as soon
// as its shot ends, so that the SIMDs carry equal numbers of waves and no
// lane waits for another shot's run to end.  Each shot goes through the
// operations of global_body in the same order (outputs identical bit for
// bit); only the partner exchange is staged in two steps:
//   A: a view publishes its value at the positions with sigma[j] <= j, and at
//      the positions with sigma[j] >= j combines its own value with the
//      partner's (a round: S_j = P_j + P'_{sigma j}, global_body's sum);
//   B: it publishes the combined values at the positions with sigma[j] > j,
//      which the partner copies into its positions with sigma[j] < j (for a
//      round the same sum with the operands swapped: IEEE addition is
//      commutative; for Phase 2, lambda' is symmetric in its two operands).
// The exchange buffer then holds half of the positions, which leaves LDS for
// lambda' of the positions with sigma[j] >= j.  Every lane executes every
// step of the loop, with or without a shot, and S and the check state are
// replaced by selects only, never under a branch (which would keep two
// copies of them live).

template <class C>
constexpr int tile_rank_a(int j) {   // rank of j among the positions published in step A
    int n = 0;
    for (int i = 0; i < j; ++i) n += C::sigma[i] <= i ? 1 : 0;
    return n;
}
template <class C>
constexpr int tile_rank_b(int j) {   // ... in step B
    int n = 0;
    for (int i = 0; i < j; ++i) n += C::sigma[i] > i ? 1 : 0;
    return n;
}
template <class C>
constexpr int tile_buf_slots() {
    constexpr int D2 = C::D * C::D;
    return tile_rank_a<C>(D2) > tile_rank_b<C>(D2) ? tile_rank_a<C>(D2) : tile_rank_b<C>(D2);
}

__device__ __forceinline__ float lds_at(const float *buf, uint32_t byte_off) {
    return *reinterpret_cast<const float *>(reinterpret_cast<const char *>(buf) + byte_off);
}

// Partner values for the positions of one exchange step, B at a time:
// f(Int<j>, q) for each position j with STEP's reading rule (A: sigma[j] >=
// j, from row tile_rank_a(sigma[j]); B: sigma[j] < j, from row
// tile_rank_b(sigma[j])).  pr holds the partner views of the lane's view, 8
// bits per position, one 16-byte row per sixteen positions (read from LDS
// by the caller ahead of the barrier before the exchange, so that they hold
// no registers between exchanges and their latency hides behind the wait).
template <class C, int WG, bool STEP_A, int B = 16, int NR, class F>
__device__ __forceinline__ void tile_read(const float *buf, const uint4 (&pr)[NR], uint32_t base4, const F &f) {
    constexpr int D2 = C::D * C::D;
    static_assert(16 % B == 0 && NR * 16 >= D2, "batches within a 16-position row of the partner table");
    static_for<0, (D2 + B - 1) / B>([&](auto qq) {
        constexpr int j0 = B * decltype(qq)::value;
        const uint4 pw = pr[j0 / 16];
        const uint32_t pwk[4] = {pw.x, pw.y, pw.z, pw.w};
        float Q[B];
        static_for<0, B>([&](auto ii) {
            constexpr int i = decltype(ii)::value, j = j0 + i;
            if constexpr (j < D2 && ((STEP_A && C::sigma[j] >= j) || (!STEP_A && C::sigma[j] < j))) {
                constexpr int row = STEP_A ? tile_rank_a<C>(C::sigma[j]) : tile_rank_b<C>(C::sigma[j]);
                const uint32_t col = __builtin_amdgcn_ubfe(pwk[(j % 16) / 4], 8 * (j % 4), 8) * 4u + base4;
                Q[i] = lds_at(buf, (uint32_t)(row * WG * 4) + col);
            }
        });
        static_for<0, B>([&](auto ii) {
            constexpr int j = j0 + decltype(ii)::value;
            if constexpr (j < D2 && ((STEP_A && C::sigma[j] >= j) || (!STEP_A && C::sigma[j] < j)))
                f(Int<j>{}, Q[j - j0]);
        });
        __builtin_amdgcn_sched_barrier(0);
    });
}

// Per-slot words of the persistent kernel, at LDS index sl * N + word (so
// that a lane reaches its slot's words from its slot's lane offset, with no
// address of its own): the unsatisfied-check flags of even and odd rounds,
// the last round that changed a message, the Phase 1 statistics, the slot's
// round, the finished shot's global iterations, converged flag and
// fixed-point round, the shot (low, high) and whether the slot awaits a shot.
enum { TW_F0 = 0, TW_F1, TW_CHG, TW_ITSUM, TW_ITMAX, TW_NCONV, TW_NFIX, TW_NOSD, TW_T, TW_ITG, TW_CONV, TW_FIX,
       TW_SHOT_LO, TW_SHOT_HI, TW_AWAIT, TW_WORDS };

template <class C, int FORM, bool FP = true>
__device__ __forceinline__ void global_tile_body(const DecodeArgs &a, const LocalArgs &w, const SpecArgs &x) {
    constexpr int WG = lead::kTileWG;
    constexpr int D2 = C::D * C::D, NP = (D2 + 1) / 2;
    constexpr int NX = tile_buf_slots<C>(), NO = owner_slots<C>();
    constexpr int NPW = (D2 + 15) / 16 * 4;   // words of a view's partner table (whole 16-byte rows)
    // LDS: the slots' words [WG + 16], four control words ([0] a slot awaits
    // a shot, [1] slots still decoding), the slots' e_hat bitmaps [WG]
    // (slot sl's at sl * N; ceil(n/32) <= N words for Delta <= 8), exchange
    // rows [NX][WG], lambda' rows [NO][WG], the partner views [N][NPW].
    // Every region but the last starts at a compile-time offset, so that
    // its addresses are a lane base plus an instruction's immediate offset
    // (a region at a run-time offset would take a register per row).
    extern __shared__ float lds_tile[];
    constexpr int OFF_CTL = WG + 16, OFF_EB = OFF_CTL + 4, OFF_BUF = OFF_EB + WG, OFF_LAM = OFF_BUF + NX * WG,
                  OFF_PV = OFF_LAM + NO * WG;
    static_assert(TW_WORDS <= 16 && OFF_PV % 4 == 0, "slot words, 16-byte aligned partner tables");
    int *sw = reinterpret_cast<int *>(lds_tile);
    int *ctl = reinterpret_cast<int *>(lds_tile + OFF_CTL);
    uint32_t *ebits = reinterpret_cast<uint32_t *>(lds_tile + OFF_EB);
    float *buf = lds_tile + OFF_BUF;
    float *laml = lds_tile + OFF_LAM;
    uint32_t *pvt = reinterpret_cast<uint32_t *>(lds_tile + OFF_PV);
    const int K = WG / a.N;
    const int ew32 = (a.n + 31) >> 5;
    const int tid = (int)threadIdx.x;
    const int sl = tid / a.N;
    const bool lane_ok = sl < K;
    // the lane's slot offset sl * N (as a byte offset): the lane's view is
    // tid - sl * N, its slot's words sw[sl * N + word], its e_hat words
    // ebits[sl * N + word], its partner columns sl * N + partner view
    const uint32_t base4 = (uint32_t)(sl * a.N) * 4u;
    const int v = tid - sl * a.N;

    // partner views of each view (the same for every slot and shot)
    if (tid < a.N) {
        uint32_t pa[NPW];
#pragma unroll
        for (int k = 0; k < NPW; ++k) pa[k] = 0u;
#pragma unroll
        for (int j = 0; j < D2; ++j) {
            const uint32_t vp = (x.pv[tid * NP + j / 2] >> (16 * (j & 1))) & 0xffffu;
            pa[j / 4] |= vp << (8 * (j % 4));
        }
#pragma unroll
        for (int k = 0; k < NPW; ++k) pvt[tid * NPW + k] = pa[k];
    }
    // the lane's partner table, from its view (no register held for it)
    uint64_t fown = 0;
    if (C::NFIX && lane_ok) fown = x.fown[v];
    for (int i = tid; i < WG + 16; i += WG) sw[i] = -1;   // no shot anywhere
    __syncthreads();
    if (tid == 0) {
        ctl[0] = 1;
        ctl[1] = K;
    }
    if (lane_ok && v == 0) sw[(base4 >> 2) + TW_AWAIT] = 1;
    __syncthreads();
    auto owned = [&](int j) { return C::sigma[j] > j || (C::sigma[j] == j && ((fown >> j) & 1ull)); };

    float S[D2];
#pragma unroll
    for (int j = 0; j < D2; ++j) S[j] = 0.f;
    GlobalState<C, FORM> st;
    st.clear();
    uint64_t sv = 0;
    // the lane's LDS addresses are formed from ti and b4, which the loop
    // re-reads each pass (an asm barrier), so that they are recomputed at
    // each use (a base register plus an immediate) instead of being kept, one
    // register per row, across the loop
    int ti = tid;
    uint32_t b4 = base4;
    auto word = [&](int k) -> int & { return sw[(b4 >> 2) + k]; };
    constexpr int NR = NPW / 4;   // 16-byte rows of a view's partner table
    auto load_pv = [&](uint4 (&pr)[NR]) {
        const uint4 *p = reinterpret_cast<const uint4 *>(reinterpret_cast<const char *>(pvt) + ((uint32_t)ti * 4u - b4) * NPW);
#pragma unroll
        for (int r = 0; r < NR; ++r) pr[r] = p[r];
    };
    auto slot_shot = [&]() {
        return (int64_t)(uint32_t)word(TW_SHOT_LO) | ((int64_t)word(TW_SHOT_HI) << 32);
    };
    for (;;) {
        asm volatile("" : "+v"(ti), "+v"(b4));
        // ---- slots whose shot ended take the next one (uniform: ctl[0] is
        // read after a barrier by every lane)
        if (ctl[0] != 0) {
            const bool fresh = lane_ok && word(TW_AWAIT) == 1;
            const int64_t done_shot = slot_shot();
            if (fresh && done_shot >= 0 && done_shot < a.shots) {   // the outputs of the shot the slot finished
                uint32_t *eb = ebits + (b4 >> 2);
                if (a.ehat)
                    for (int wd = v; wd < a.ehat_words; wd += a.N) {
                        const uint64_t lo = (2 * wd < ew32) ? eb[2 * wd] : 0u;
                        const uint64_t hi = (2 * wd + 1 < ew32) ? eb[2 * wd + 1] : 0u;
                        a.ehat[done_shot * a.ehat_words + wd] = lo | (hi << 32);
                    }
                if (v == 0 && a.stats) {
                    lead::ShotStats s = {};
                    s.converged = word(TW_CONV);
                    s.global_iters = word(TW_ITG);
                    s.local_iters_sum = word(TW_ITSUM);
                    s.local_iters_max = word(TW_ITMAX);
                    s.local_converged_views = word(TW_NCONV);
                    s.local_fixed_views = word(TW_NFIX);
                    s.local_osd_views = word(TW_NOSD);
                    s.global_fixed_iter = word(TW_FIX);
                    reinterpret_cast<lead::ShotStats *>(a.stats)[done_shot] = s;
                }
            }
            __syncthreads();
            if (ti == 0) ctl[0] = 0;
            if (fresh) {
                // the slot's words up to TW_FIX cleared (round 1 next), its
                // e_hat bitmap cleared, its next shot taken
                if (v < TW_SHOT_LO) word(v) = v == TW_T ? 1 : 0;
                for (int i = v; i < ew32; i += a.N) ebits[(b4 >> 2) + i] = 0u;
                if (v == TW_SHOT_LO) {
                    const int64_t nx =
                        (int64_t)atomicAdd(reinterpret_cast<unsigned long long *>(w.counter + 3), 1ull);
                    word(TW_SHOT_LO) = (int)(uint32_t)nx;
                    word(TW_SHOT_HI) = (int)(nx >> 32);
                    word(TW_AWAIT) = 0;
                    if (nx >= a.shots) atomicSub(&ctl[1], 1);
                }
            }
            __syncthreads();
            int64_t shot = 0;
            bool go = false;   // the lane takes up a new shot
            if (fresh) {
                shot = slot_shot();
                go = shot < a.shots;
            }
            const float *in = w.Lv;
            if (go) {
                sv = local_syndrome(a, shot, v);
                if (!a.global_only) {
                    const int64_t item = shot * a.N + v;
                    in = w.Lv + item * D2;
                    const uint32_t f = w.vflag[item];
                    const int it_v = (int)(f & 0xffffu);
                    const int osd_v = (int)((f >> 18) & 1u);
                    atomicAdd(&word(TW_ITSUM), it_v);
                    atomicMax(&word(TW_ITMAX), it_v);
                    atomicAdd(&word(TW_NCONV), (int)((f >> 16) & 1u) & (osd_v ^ 1));   // converged by BP
                    if ((f >> 17) & 1u) atomicAdd(&word(TW_NFIX), 1);
                    if (osd_v) atomicAdd(&word(TW_NOSD), 1);
                }
            }
            // Phase 2: lambda' into S (from the lane's own and its partner's
            // clamped local posteriors), or the channel prior for global BP
            // alone
            if (a.global_only) {
                const int64_t pbase = a.prior_mode == 2 ? shot * a.n : 0;   // LEAD_PRIOR_FULL
                int vb = v * D2;
                asm volatile("" : "+v"(vb));   // the qubit ids are loaded here, not kept across the loop
#pragma unroll
                for (int j = 0; j < D2; ++j) {
                    float lj = 0.f;
                    if (go) lj = (a.prior_mode == 0 ? a.prior[shot] : a.prior[pbase + a.view[vb + j]]) + 0.f;
                    S[j] = go ? lj : S[j];
                }
            } else {
                // (eight positions at a time: the check state of the other
                // slots' lanes is live throughout)
                if (go)
                    static_for<0, D2 / 8>([&](auto qq) {
                        static_for<0, 8>([&](auto ii) {
                            constexpr int j = 8 * decltype(qq)::value + decltype(ii)::value;
                            if constexpr (C::sigma[j] <= j) buf[tile_rank_a<C>(j) * WG + ti] = in[j];
                        });
                        __builtin_amdgcn_sched_barrier(0);
                    });
                uint4 pr[NR];
                load_pv(pr);
                __syncthreads();
                tile_read<C, WG, true, 8>(buf, pr, b4, [&](auto jj, float q) {
                    constexpr int j = decltype(jj)::value;
                    float lj = 0.f;
                    if (go) lj = aggregate_llr(clampf(in[j], a.clampv), clampf(q, a.clampv), a.alpha, a.clampv);
                    S[j] = go ? lj : S[j];
                });
                __syncthreads();
                if (go)
                    static_for<0, D2>([&](auto jj) {
                        constexpr int j = decltype(jj)::value;
                        if constexpr (C::sigma[j] > j) buf[tile_rank_b<C>(j) * WG + ti] = S[j];
                    });
                __syncthreads();
                tile_read<C, WG, false, 8>(buf, pr, b4, [&](auto jj, float q) {
                    constexpr int j = decltype(jj)::value;
                    S[j] = go ? q : S[j];
                });
            }
            if (go) {
                if (a.lam_out) {
                    int vb = v * D2;
                    asm volatile("" : "+v"(vb));
#pragma unroll
                    for (int j = 0; j < D2; ++j)
                        if (owned(j)) a.lam_out[shot * a.n + a.view[vb + j]] = S[j];
                }
                static_for<0, D2>([&](auto jj) {
                    constexpr int j = decltype(jj)::value;
                    if constexpr (C::sigma[j] >= j) laml[owner_slot<C>(j) * WG + ti] = S[j];
                });
            }
            st.reset_where(go);
        }
        if (ctl[1] == 0) break;   // every slot has run out of shots

        // ---- one global round of every slot's shot (Phase 3); the slot's
        // round number and shot are read from its LDS words
        bool same;
        const bool sat = st.template check<FP>(S, sv, a.beta, a.clampv, same);
        const int64_t shot = slot_shot();
        const bool live = lane_ok && shot >= 0 && shot < a.shots;
        const int t = word(TW_T);
        if (live && !sat) word(t & 1) = 1;
        if (FP && live && !same) word(TW_CHG) = t;
        // lambda' of the owned positions for this round's partial sums, read
        // before the barrier so that the wait covers their latency
        float lr[D2];
        static_for<0, D2>([&](auto jj) {
            constexpr int j = decltype(jj)::value;
            lr[j] = C::sigma[j] >= j ? laml[owner_slot<C>(j) * WG + ti] : 0.f;
        });
        __syncthreads();
        if (live) {
            const bool shot_sat = word(t & 1) == 0, shot_same = FP && word(TW_CHG) != t;
            bool end = false;
            int gconv = 0, itg = a.Tg, gfix = 0;
            if (t > 1 && shot_sat && a.early_exit) {
                end = true;
                gconv = 1;
                itg = t - 1;
            } else if (t > a.Tg) {   // ran to the cap: S holds round Tg's sums
                end = true;
                gconv = shot_sat ? 1 : 0;
            } else if (t > 1 && FP && a.fixed_stop_g && shot_same) {
                end = true;
                gconv = shot_sat ? 1 : 0;
                gfix = t;
            }
            if (end) {
                int vb = v * D2;
                asm volatile("" : "+v"(vb));   // the qubit ids are loaded here, not kept across the loop
                uint32_t *eb = ebits + (b4 >> 2);
#pragma unroll
                for (int j = 0; j < D2; ++j)
                    if (owned(j)) {
                        const int qd = a.view[vb + j];
                        if (a.post) a.post[shot * a.n + qd] = clampf(S[j], a.clampv);
                        if (signbit_of(S[j])) atomicOr(&eb[qd >> 5], 1u << (qd & 31));
                    }
            }
            if (v == 0) {
                word((t + 1) & 1) = 0;
                word(TW_T) = t + 1;
                if (end) {
                    word(TW_CONV) = gconv;
                    word(TW_ITG) = itg;
                    word(TW_FIX) = gfix;
                    word(TW_AWAIT) = 1;
                    ctl[0] = 1;
                }
            }
        }
        // partial sums of this view, then the exchange (a slot whose shot
        // ended computes them too, unused)
        partial_sums<C>(st, lr, fown, S);
        static_for<0, D2>([&](auto jj) {
            constexpr int j = decltype(jj)::value;
            if constexpr (C::sigma[j] <= j) buf[tile_rank_a<C>(j) * WG + ti] = S[j];
        });
        uint4 pr[NR];
        load_pv(pr);
        __syncthreads();
        tile_read<C, WG, true>(buf, pr, b4, [&](auto jj, float q) { S[decltype(jj)::value] += q; });
        __syncthreads();
        static_for<0, D2>([&](auto jj) {
            constexpr int j = decltype(jj)::value;
            if constexpr (C::sigma[j] > j) buf[tile_rank_b<C>(j) * WG + ti] = S[j];
        });
        __syncthreads();
        tile_read<C, WG, false>(buf, pr, b4, [&](auto jj, float q) { S[decltype(jj)::value] = q; });
    }
}

// ---------------------------------------------------------------------------
// Global OSD-0 (post-processing of global BP), one workgroup per shot that
// global BP left with H e != s.  G fixes the global sizes:
//   G::M (checks), G::NQ (qubits), G::W = ceil(NQ/64), G::RPL (rows per lane),
//   G::WG (lanes, 64 * ceil(M / (64 RPL))), G::RANK (GF(2) rank of H),
//   G::SORTN (power of two >= NQ).
// Qubits are ranked by round(64 L) of their global posterior, ascending,
// equal keys in index order (bitonic sort of (key, index) pairs in LDS).
// Lane l holds rows l, l + WG, ... of [H | s] with the columns permuted into
// that order, so Gauss-Jordan elimination over columns t = 0, 1, ... selects
// the greedy information set: a column gets a pivot exactly when it is
// independent of the columns before it.  The pivot row is the lowest-numbered
// row that is not yet a pivot row and has bit t (any choice gives the same
// information set, and the solution on it is unique); it is broadcast
// through LDS and XORed into every other row that has bit t.  Only the words
// from the current one on are kept up to date: the earlier ones are never
// read again (the result needs only the s-bits and the pivot columns).
// Once the rank is reached, the estimate is e[order[t_k]] = s-bit of pivot
// row k, provided that every row without a pivot has s-bit 0 (otherwise the
// syndrome is not in the column space of H and BP's estimate and report
// stay).
// CS (combination sweep of order a.osd_order): the elimination runs over
// every word, so that pivot row k ends as [unit k | A_k | s'_k] over the
// ranked columns; the costs of the candidates (OSD-0, one bit set on each
// non-pivot column t, two bits set on each pair among the first osd_order
// non-pivot columns) follow from the s-bits, A and the weights q_t =
// round(64 ln(1 + e^{lambda'})) of the global prior read from a.lam_out:
//   cost(e_T) = C0 + sum_{t in e_T} q_t + sum_k u_k [A_k . e_T odd],
//   C0 = sum_{k: s'_k = 1} q_{piv k},  u_k = (s'_k ? -1 : 1) q_{piv k},
// accumulated in LDS as integers; the least (cost, candidate index) wins,
// i.e. the first candidate of least cost in the order listed.
template <class G, bool CS>
__device__ __forceinline__ void osd_global_body(const DecodeArgs &a, const lead::OsdArgs &o) {
    constexpr int WG = G::WG, NWAVE = WG / 64, W = G::W, RPL = G::RPL, NQ = G::NQ, M = G::M,
                  SORTN = G::SORTN;
    static_assert(RPL <= 32 && NQ <= SORTN && WG % 64 == 0 && WG * RPL >= M, "OSD-0 sizes");
    __shared__ uint64_t keys[SORTN];
    __shared__ uint64_t prow[W];
    __shared__ int32_t inv[NQ];                  // qubit -> rank position
    __shared__ int32_t wmin[2][NWAVE];           // per-wave pivot candidates, by step parity
    __shared__ int32_t flags[2];                 // pivot s-bit, syndrome unreachable
    __shared__ uint32_t ebits[(NQ + 31) / 32];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t shot = blockIdx.x;
    if (shot >= a.shots) return;
    lead::ShotStats *stp = reinterpret_cast<lead::ShotStats *>(a.stats) + shot;
    if (stp->converged != 0) return;             // uniform per workgroup
    const float *Lp = a.post + shot * a.n;

    // ---- ranking.  Key: rint(64 L) (+0 for -0) as an order-preserving
    // unsigned word, then the qubit index.
    for (int i = tid; i < SORTN; i += WG) {
        uint64_t k = ~0ull;
        if (i < NQ) {
            const float q = __builtin_rintf(Lp[i] * 64.f) + 0.f;
            uint32_t u = __float_as_uint(q);
            u = (u >> 31) ? ~u : (u | 0x80000000u);
            k = ((uint64_t)u << 32) | (uint32_t)i;
        }
        keys[i] = k;
    }
    __syncthreads();
    for (int size = 2; size <= SORTN; size <<= 1)
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = tid; i < SORTN / 2; i += WG) {
                const int lo = 2 * i - (i & (stride - 1)), hi = lo + stride;
                const uint64_t x = keys[lo], y = keys[hi];
                if ((x > y) == ((lo & size) == 0)) {
                    keys[lo] = y;
                    keys[hi] = x;
                }
            }
            __syncthreads();
        }
    for (int t = tid; t < NQ; t += WG) inv[(uint32_t)keys[t]] = t;
    for (int i = tid; i < (NQ + 31) / 32; i += WG) ebits[i] = 0u;
    __syncthreads();

    // ---- this lane's rows of [H | s], columns in rank order
    uint64_t row[RPL][W];
    uint32_t sb = 0u, piv = 0u;
    int pcol[RPL];
    const uint64_t *srow = a.synd + shot * a.synd_words;
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
        pcol[i] = 0;
#pragma unroll
        for (int k = 0; k < W; ++k) row[i][k] = 0ull;
        const int r = tid + WG * i;
        if (r < M) {
            sb |= (uint32_t)((srow[r >> 6] >> (r & 63)) & 1ull) << i;
            for (int x = o.rptr[r]; x < o.rptr[r + 1]; ++x) {
                const int t = inv[o.ridx[x]];
                const uint64_t bit = 1ull << (t & 63);
#pragma unroll
                for (int k = 0; k < W; ++k) row[i][k] |= (k == (t >> 6)) ? bit : 0ull;
            }
        }
    }

    // ---- Gauss-Jordan over the ranked columns, one 64-column word at a
    // time (compile-time word index, so each step touches words w.. only)
    __shared__ uint64_t cmw[2][NWAVE];   // per-wave OR of the non-pivot rows' current word
    int rank = 0, par = 0;
    static_for<0, W>([&](auto ww) {
        constexpr int w = decltype(ww)::value;
        if (rank >= G::RANK) return;
        // columns of this word that some non-pivot row has: the others can
        // take no pivot in it (a row added to another is a non-pivot row up
        // to then, so a column no non-pivot row has keeps none)
        uint64_t any = 0ull;
#pragma unroll
        for (int i = 0; i < RPL; ++i) any |= ((piv >> i) & 1u) ? 0ull : row[i][w];
#pragma unroll
        for (int sh = 1; sh < 64; sh <<= 1) {
            const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)any, sh);
            const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(any >> 32), sh);
            any |= ((uint64_t)hi << 32) | lo;
        }
        if (NWAVE > 1) {
            if (lane == 0) cmw[w & 1][wave] = any;
            __syncthreads();
#pragma unroll
            for (int x = 0; x < NWAVE; ++x) any |= cmw[w & 1][x];
        }
        for (uint64_t todo = any; todo && rank < G::RANK; todo &= todo - 1ull, par ^= 1) {
            const int b = __builtin_ctzll(todo);
            // lowest-numbered non-pivot row with bit (w, b): rows are
            // numbered tid + WG i, so the first i with a candidate in any
            // wave wins, then the lowest wave, then the lowest lane
            int cand = 0x7fffffff;
#pragma unroll
            for (int i = RPL - 1; i >= 0; --i) {
                const uint64_t bal = __ballot(!((piv >> i) & 1u) && ((row[i][w] >> b) & 1ull));
                if (bal) cand = WG * i + 64 * wave + __builtin_ctzll(bal);
            }
            if (NWAVE > 1) {
                if (lane == 0) wmin[par][wave] = cand;
                __syncthreads();
            }
            int p = cand;
            if (NWAVE > 1) {
                p = wmin[par][0];
#pragma unroll
                for (int x = 1; x < NWAVE; ++x) p = min(p, wmin[par][x]);
            }
            if (p == 0x7fffffff) continue;       // column t depends on the ones before it
            const int pi = p / WG;
            if (tid == p - WG * pi) {
#pragma unroll
                for (int i = 0; i < RPL; ++i)
                    if (i == pi) {
#pragma unroll
                        for (int k = CS ? 0 : w; k < W; ++k) prow[k] = row[i][k];
                        flags[0] = (int)((sb >> i) & 1u);
                        pcol[i] = 64 * w + b;
                    }
                piv |= 1u << pi;
            }
            __syncthreads();
            const uint32_t ps = (uint32_t)flags[0];
#pragma unroll
            for (int i = 0; i < RPL; ++i)
                if (tid + WG * i != p && ((row[i][w] >> b) & 1ull)) {
#pragma unroll
                    for (int k = CS ? 0 : w; k < W; ++k) row[i][k] ^= prow[k];
                    sb ^= ps << i;
                }
            ++rank;
        }
    });

    // ---- the estimate, or BP's when the syndrome is not reached
    bool bad = false;
#pragma unroll
    for (int i = 0; i < RPL; ++i)
        if (tid + WG * i < M && !((piv >> i) & 1u) && ((sb >> i) & 1u)) bad = true;
    if (tid == 0) flags[1] = 0;
    __syncthreads();
    if (bad) flags[1] = 1;
    int ca = -1, cb = -1;   // non-pivot columns (rank positions) set by the sweep's choice
    if constexpr (CS) {
        __shared__ int32_t qw[NQ];                    // weight of rank position t
        __shared__ int32_t acc[NQ];                   // sum of u_k over pivot rows with bit t
        __shared__ uint32_t pbits[(NQ + 31) / 32];    // pivot columns
        __shared__ int32_t tl[lead::kMaxOsdOrder], pairsum[lead::kMaxOsdOrder * (lead::kMaxOsdOrder - 1) / 2],
            c0s[2];
        __shared__ unsigned long long best;
        const float *lp = a.lam_out + shot * a.n;
        for (int t = tid; t < NQ; t += WG) {
            qw[t] = osd_weight(lp[(uint32_t)keys[t]]);
            acc[t] = 0;
        }
        for (int i = tid; i < (NQ + 31) / 32; i += WG) pbits[i] = 0u;
        if (tid == 0) c0s[0] = 0;
        if (tid < lead::kMaxOsdOrder * (lead::kMaxOsdOrder - 1) / 2) pairsum[tid] = 0;
        __syncthreads();
        int c0p = 0;
#pragma unroll
        for (int i = 0; i < RPL; ++i)
            if ((piv >> i) & 1u) {
                const int pc = pcol[i];
                atomicOr(&pbits[pc >> 5], 1u << (pc & 31));
                const int32_t qv = qw[pc];
                const int32_t u = ((sb >> i) & 1u) ? -qv : qv;
                c0p += ((sb >> i) & 1u) ? qv : 0;
#pragma unroll
                for (int k = 0; k < W; ++k) {
                    uint64_t bits = row[i][k];
                    if (k == (pc >> 6)) bits &= ~(1ull << (pc & 63));
                    while (bits) {
                        atomicAdd(&acc[64 * k + __builtin_ctzll(bits)], u);
                        bits &= bits - 1ull;
                    }
                }
            }
        atomicAdd(&c0s[0], c0p);
        __syncthreads();
        const int32_t C0 = c0s[0];
        if (tid == 0) {
            best = (unsigned long long)(uint32_t)C0 << 32;   // OSD-0 is candidate 0
            int nt = 0;
            for (int t = 0; t < NQ && nt < a.osd_order; ++t)
                if (!((pbits[t >> 5] >> (t & 31)) & 1u)) tl[nt++] = t;
            c0s[1] = nt;
        }
        __syncthreads();
        const int nt = c0s[1];
        // pairs among the first nt non-pivot columns, in lexicographic order
        for (int x = 0, pi = 0; x < nt; ++x)
            for (int y = x + 1; y < nt; ++y, ++pi) {
                const int ta = tl[x], tb = tl[y];
                int part = 0;
#pragma unroll
                for (int i = 0; i < RPL; ++i)
                    if ((piv >> i) & 1u) {
                        uint64_t wa = 0ull, wb = 0ull;
#pragma unroll
                        for (int k = 0; k < W; ++k) {
                            wa = (k == (ta >> 6)) ? row[i][k] : wa;
                            wb = (k == (tb >> 6)) ? row[i][k] : wb;
                        }
                        if (((wa >> (ta & 63)) ^ (wb >> (tb & 63))) & 1ull)
                            part += ((sb >> i) & 1u) ? -qw[pcol[i]] : qw[pcol[i]];
                    }
                if (part) atomicAdd(&pairsum[pi], part);
            }
        __syncthreads();
        unsigned long long mine = ~0ull;
        for (int t = tid; t < NQ; t += WG)
            if (!((pbits[t >> 5] >> (t & 31)) & 1u)) {
                const uint32_t cost = (uint32_t)(C0 + qw[t] + acc[t]);
                const unsigned long long key = ((unsigned long long)cost << 32) | (uint32_t)(t + 1);
                mine = key < mine ? key : mine;
            }
        if (tid < nt * (nt - 1) / 2) {
            int x = 0, r = tid;
            while (r >= nt - 1 - x) { r -= nt - 1 - x; ++x; }
            const int ta = tl[x], tb = tl[x + 1 + r];
            const uint32_t cost = (uint32_t)(C0 + qw[ta] + qw[tb] + pairsum[tid]);
            const unsigned long long key = ((unsigned long long)cost << 32) | (uint32_t)(NQ + 1 + tid);
            mine = key < mine ? key : mine;
        }
        atomicMin(&best, mine);
        __syncthreads();
        const uint32_t idx = (uint32_t)best;
        if (idx >= 1 && idx <= (uint32_t)NQ) {
            ca = (int)idx - 1;
        } else if (idx > (uint32_t)NQ) {
            int x = 0, r = (int)idx - NQ - 1;
            while (r >= nt - 1 - x) { r -= nt - 1 - x; ++x; }
            ca = tl[x];
            cb = tl[x + 1 + r];
        }
        if (tid == 0 && ca >= 0) {
            const int qa = (int)(uint32_t)keys[ca];
            atomicOr(&ebits[qa >> 5], 1u << (qa & 31));
            if (cb >= 0) {
                const int qb = (int)(uint32_t)keys[cb];
                atomicOr(&ebits[qb >> 5], 1u << (qb & 31));
            }
        }
    }
#pragma unroll
    for (int i = 0; i < RPL; ++i)
        if ((piv >> i) & 1u) {
            uint32_t bit = (sb >> i) & 1u;
            if constexpr (CS) {
                if (ca >= 0) {
                    uint64_t wa = 0ull, wb = 0ull;
#pragma unroll
                    for (int k = 0; k < W; ++k) {
                        wa = (k == (ca >> 6)) ? row[i][k] : wa;
                        wb = (cb >= 0 && k == (cb >> 6)) ? row[i][k] : wb;
                    }
                    bit ^= (uint32_t)((wa >> (ca & 63)) & 1ull);
                    if (cb >= 0) bit ^= (uint32_t)((wb >> (cb & 63)) & 1ull);
                }
            }
            if (bit) {
                const int q = (int)(uint32_t)keys[pcol[i]];
                atomicOr(&ebits[q >> 5], 1u << (q & 31));
            }
        }
    __syncthreads();
    if (flags[1] != 0) return;
    if (a.ehat) {
        constexpr int EW32 = (NQ + 31) / 32;
        for (int wd = tid; wd < a.ehat_words; wd += WG) {
            const uint64_t lo = (2 * wd < EW32) ? ebits[2 * wd] : 0u;
            const uint64_t hi = (2 * wd + 1 < EW32) ? ebits[2 * wd + 1] : 0u;
            a.ehat[shot * a.ehat_words + wd] = lo | (hi << 32);
        }
    }
    if (tid == 0) stp->converged = 2;
}

// ---------------------------------------------------------------------------
// Global OSD with [H | s] in device memory, for codes whose rows do not fit
// in registers (PSL(2,7): 2688 x 5376 bits, 1.8 MB per shot).  The method and
// the result are those of osd_global_body (same ranking, same information
// set, same candidates and costs); the organisation differs:
//  * workgroups are persistent: each takes the next shot that global BP left
//    unresolved from a queue and works in its own matrix slot;
//  * the slot is word-major (word k of row r at k*M + r; word column W holds
//    s in bit 0), so a wave's accesses to one word of consecutive rows
//    coalesce;
//  * Gauss-Jordan runs panel by panel, a panel being the 64 ranked columns
//    of one word.  The panel word of every row is held in registers (rows
//    tid + WG i) and reduced pivot by pivot as in osd_global_body, while each
//    row records in a 64-bit mask which of the panel's pivot rows (as they
//    were when the panel started) it has absorbed.  The other words are then
//    updated in one pass, KC words at a time: each row XORs the combination
//    of pivot rows its mask names, read from eight 256-entry tables of the
//    XOR combinations of eight pivot rows each, built in LDS for those words.
//    One pass per panel over the rest of the matrix replaces one pass per
//    pivot;
//  * in the combination sweep, the cost term sum_k u_k A_k[t] of flipping
//    non-pivot column t is accumulated in a register of the lane owning t (a
//    wave per 64-column word), from each row's word read once and spread to
//    the lanes with readlane, instead of LDS atomics per set bit.
// G: M, NQ, W = ceil(NQ/64), WG, RPL = ceil(M/WG) (rows per lane), RANK (of
// H), SORTN (power of two >= NQ), KC (words per update chunk).
template <class G, bool CS>
__device__ __forceinline__ void osd_big_body(const DecodeArgs &a, const lead::OsdArgs &o,
                                             const lead::OsdBigArgs &b) {
    constexpr int WG = G::WG, NWAVE = WG / 64, W = G::W, M = G::M, NQ = G::NQ, RPL = G::RPL,
                  SORTN = G::SORTN, KC = G::KC;
    constexpr int WS = W + 1;                                   // word columns, the last holds s
    constexpr int R0 = SORTN > 2048 * KC ? SORTN : 2048 * KC;   // words of region 0
    constexpr int NPAIR = lead::kMaxOsdOrder * (lead::kMaxOsdOrder - 1) / 2;
    static_assert(RPL <= 32 && NQ <= SORTN && NQ <= 65535 && WG % 64 == 0 && WG * RPL >= M && KC >= 1,
                  "OSD sizes");
    __shared__ uint64_t r0[R0];            // sort keys, then the XOR tables [8][256][KC]
    __shared__ int32_t r1[NQ];             // qubit -> rank position, then weights by rank position
    __shared__ unsigned short order[NQ];   // rank position -> qubit
    __shared__ int32_t uarr[M];            // sweep: u of pivot row r (0 for the other rows)
    __shared__ uint64_t P[64][KC];         // the panel's pivot rows, one word chunk
    __shared__ int32_t prl[64];            // the panel's pivot rows
    __shared__ uint64_t pw[2];             // pivot broadcast: panel word, absorbed mask
    __shared__ uint64_t cmw[2][NWAVE];
    __shared__ int32_t wmin[2][NWAVE];
    __shared__ int32_t misc[4];            // shot, syndrome unreachable, C0, listed non-pivot columns
    __shared__ uint32_t pbits[(NQ + 31) / 32];
    __shared__ uint32_t ebits[(NQ + 31) / 32];
    __shared__ int32_t tl[lead::kMaxOsdOrder], pairsum[NPAIR];
    __shared__ unsigned long long best;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    uint64_t *mat = b.mat + (size_t)blockIdx.x * WS * M;
    lead::ShotStats *stats = reinterpret_cast<lead::ShotStats *>(a.stats);
    for (;;) {
        // ---- the next shot global BP left unresolved (every wave sees the
        // same value and leaves together when the queue is empty)
        if (tid == 0) {
            int64_t sh;
            do {
                sh = (int64_t)atomicAdd(reinterpret_cast<unsigned long long *>(b.queue), 1ull);
            } while (sh < a.shots && stats[sh].converged != 0);
            misc[0] = sh < a.shots ? (int32_t)sh : -1;
            misc[1] = 0;
        }
        __syncthreads();
        if (misc[0] < 0) return;
        const int64_t shot = misc[0];
        const float *Lp = a.post + shot * a.n;

        // ---- ranking: rint(64 L) as an order-preserving word, then the index
        for (int i = tid; i < SORTN; i += WG) {
            uint64_t k = ~0ull;
            if (i < NQ) {
                const float q = __builtin_rintf(Lp[i] * 64.f) + 0.f;
                uint32_t u = __float_as_uint(q);
                u = (u >> 31) ? ~u : (u | 0x80000000u);
                k = ((uint64_t)u << 32) | (uint32_t)i;
            }
            r0[i] = k;
        }
        __syncthreads();
        for (int size = 2; size <= SORTN; size <<= 1)
            for (int stride = size >> 1; stride > 0; stride >>= 1) {
                for (int i = tid; i < SORTN / 2; i += WG) {
                    const int lo = 2 * i - (i & (stride - 1)), hi = lo + stride;
                    const uint64_t x = r0[lo], y = r0[hi];
                    if ((x > y) == ((lo & size) == 0)) {
                        r0[lo] = y;
                        r0[hi] = x;
                    }
                }
                __syncthreads();
            }
        for (int t = tid; t < NQ; t += WG) {
            const int q = (int)(uint32_t)r0[t];
            order[t] = (unsigned short)q;
            r1[q] = t;
        }
        for (int i = tid; i < (NQ + 31) / 32; i += WG) {
            ebits[i] = 0u;
            pbits[i] = 0u;
        }
        __syncthreads();

        // ---- this lane's rows of [H | s], columns in rank order (each row is
        // written only by the lane that owns it)
        const uint64_t *srow = a.synd + shot * a.synd_words;
        uint32_t piv = 0u;
        int pcol[RPL];
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
            pcol[i] = 0;
            const int r = tid + WG * i;
            if (r < M) {
                for (int k = 0; k < W; ++k) mat[(size_t)k * M + r] = 0ull;
                mat[(size_t)W * M + r] = (srow[r >> 6] >> (r & 63)) & 1ull;
                for (int x = o.rptr[r]; x < o.rptr[r + 1]; ++x) {
                    const int t = r1[o.ridx[x]];
                    mat[(size_t)(t >> 6) * M + r] |= 1ull << (t & 63);
                }
            }
        }

        // ---- Gauss-Jordan, panel by panel
        int rank = 0, par = 0;
        for (int w = 0; w < W && rank < G::RANK; ++w) {
            uint64_t cw[RPL], tr[RPL];
#pragma unroll
            for (int i = 0; i < RPL; ++i) {
                const int r = tid + WG * i;
                cw[i] = r < M ? mat[(size_t)w * M + r] : 0ull;
                tr[i] = 0ull;
            }
            // columns of this word that some non-pivot row has (the others
            // can take no pivot in it)
            uint64_t any = 0ull;
#pragma unroll
            for (int i = 0; i < RPL; ++i) any |= ((piv >> i) & 1u) ? 0ull : cw[i];
#pragma unroll
            for (int sh = 1; sh < 64; sh <<= 1) {
                const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)any, sh);
                const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(any >> 32), sh);
                any |= ((uint64_t)hi << 32) | lo;
            }
            if (NWAVE > 1) {
                if (lane == 0) cmw[w & 1][wave] = any;
                __syncthreads();
#pragma unroll
                for (int x = 0; x < NWAVE; ++x) any |= cmw[w & 1][x];
            }
            int np = 0;   // pivots found in this panel
            for (uint64_t todo = any; todo && rank < G::RANK; todo &= todo - 1ull, par ^= 1) {
                const int bb = __builtin_ctzll(todo);
                // lowest-numbered non-pivot row with the bit (row tid + WG i)
                int cand = 0x7fffffff;
#pragma unroll
                for (int i = RPL - 1; i >= 0; --i) {
                    const uint64_t bal = __ballot(!((piv >> i) & 1u) && ((cw[i] >> bb) & 1ull));
                    if (bal) cand = WG * i + 64 * wave + __builtin_ctzll(bal);
                }
                if (NWAVE > 1) {
                    if (lane == 0) wmin[par][wave] = cand;
                    __syncthreads();
                }
                int p = cand;
                if (NWAVE > 1) {
                    p = wmin[par][0];
#pragma unroll
                    for (int x = 1; x < NWAVE; ++x) p = min(p, wmin[par][x]);
                }
                if (p == 0x7fffffff) continue;   // the column depends on the ones before it
                const int pi = p / WG;
                if (tid == p - WG * pi) {
#pragma unroll
                    for (int i = 0; i < RPL; ++i)
                        if (i == pi) {
                            pw[0] = cw[i];
                            pw[1] = tr[i];
                            pcol[i] = 64 * w + bb;
                        }
                    piv |= 1u << pi;
                    prl[np] = p;
                }
                __syncthreads();
                const uint64_t pcw = pw[0], ptr = pw[1] ^ (1ull << np);
#pragma unroll
                for (int i = 0; i < RPL; ++i)
                    if (tid + WG * i != p && ((cw[i] >> bb) & 1ull)) {
                        cw[i] ^= pcw;
                        tr[i] ^= ptr;
                    }
                ++np;
                ++rank;
            }
#pragma unroll
            for (int i = 0; i < RPL; ++i) {
                const int r = tid + WG * i;
                if (r < M) mat[(size_t)w * M + r] = cw[i];
            }
            if (np == 0) continue;
            // the other words (from w + 1 on; every word for the sweep),
            // KC at a time
            const int ng = (np + 7) / 8;
            for (int k0 = CS ? 0 : w + 1; k0 < WS; k0 += KC) {
                __syncthreads();   // the previous chunk's table reads are done
                for (int x = tid; x < 64 * KC; x += WG) {
                    const int j = x / KC, kk = x % KC, k = k0 + kk;
                    P[j][kk] = (j < np && k < WS && k != w) ? mat[(size_t)k * M + prl[j]] : 0ull;
                }
                __syncthreads();
                for (int x = tid; x < ng * 256 * KC; x += WG) {
                    const int g = x / (256 * KC), c = (x / KC) & 255, kk = x % KC;
                    uint64_t v = 0ull;
#pragma unroll
                    for (int bit = 0; bit < 8; ++bit) v ^= ((c >> bit) & 1) ? P[8 * g + bit][kk] : 0ull;
                    r0[(g * 256 + c) * KC + kk] = v;
                }
                __syncthreads();
#pragma unroll
                for (int i = 0; i < RPL; ++i) {
                    const int r = tid + WG * i;
                    const uint64_t t = tr[i];
                    if (r < M && t != 0ull)
#pragma unroll
                        for (int kk = 0; kk < KC; ++kk) {
                            const int k = k0 + kk;
                            if (k < WS && k != w) {
                                uint64_t v = mat[(size_t)k * M + r];
                                for (int g = 0; g < ng; ++g) v ^= r0[(g * 256 + (int)((t >> (8 * g)) & 255u)) * KC + kk];
                                mat[(size_t)k * M + r] = v;
                            }
                        }
                }
            }
        }

        // ---- the estimate, or BP's when the syndrome is not reached
        uint32_t sb = 0u;
        bool bad = false;
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
            const int r = tid + WG * i;
            if (r < M) {
                const uint32_t bit = (uint32_t)(mat[(size_t)W * M + r] & 1ull);
                sb |= bit << i;
                if (!((piv >> i) & 1u) && bit) bad = true;
            }
        }
        if (bad) misc[1] = 1;
        int ca = -1, cb = -1;   // non-pivot columns (rank positions) set by the sweep's choice
        if constexpr (CS) {
            const float *lp = a.lam_out + shot * a.n;
            __syncthreads();   // r1 (qubit -> rank position) is no longer read
            for (int t = tid; t < NQ; t += WG) r1[t] = osd_weight(lp[order[t]]);
            for (int r = tid; r < M; r += WG) uarr[r] = 0;
            if (tid == 0) misc[2] = 0;
            if (tid < NPAIR) pairsum[tid] = 0;
            __syncthreads();
            int c0p = 0;
#pragma unroll
            for (int i = 0; i < RPL; ++i)
                if ((piv >> i) & 1u) {
                    const int pc = pcol[i];
                    atomicOr(&pbits[pc >> 5], 1u << (pc & 31));
                    const int32_t qv = r1[pc];
                    uarr[tid + WG * i] = ((sb >> i) & 1u) ? -qv : qv;
                    c0p += ((sb >> i) & 1u) ? qv : 0;
                }
            atomicAdd(&misc[2], c0p);
            __syncthreads();
            const int32_t C0 = misc[2];
            if (tid == 0) {
                best = (unsigned long long)(uint32_t)C0 << 32;   // OSD-0 is candidate 0
                int nt = 0;
                for (int t = 0; t < NQ && nt < a.osd_order; ++t)
                    if (!((pbits[t >> 5] >> (t & 31)) & 1u)) tl[nt++] = t;
                misc[3] = nt;
            }
            __syncthreads();
            const int nt = misc[3];
            // pairs among the first nt non-pivot columns, in lexicographic order
            for (int x = 0, pi = 0; x < nt; ++x)
                for (int y = x + 1; y < nt; ++y, ++pi) {
                    const int ta = tl[x], tb = tl[y];
                    int part = 0;
#pragma unroll
                    for (int i = 0; i < RPL; ++i)
                        if ((piv >> i) & 1u) {
                            const int r = tid + WG * i;
                            const uint64_t wa = mat[(size_t)(ta >> 6) * M + r], wb = mat[(size_t)(tb >> 6) * M + r];
                            if (((wa >> (ta & 63)) ^ (wb >> (tb & 63))) & 1ull) part += uarr[r];
                        }
                    if (part) atomicAdd(&pairsum[pi], part);
                }
            // single flips: lane l of the wave handling word k owns column
            // 64 k + l; the rows' words are read 64 rows at a time (one row
            // per lane) and handed to every lane with readlane
            unsigned long long mine = ~0ull;
            for (int k = wave; k < W; k += NWAVE) {
                int32_t acc = 0;
                for (int rb = 0; rb < M; rb += 64) {
                    const int r = rb + lane;
                    const int32_t u = r < M ? uarr[r] : 0;
                    if (__ballot(u != 0) == 0ull) continue;
                    const uint64_t wd = u != 0 ? mat[(size_t)k * M + r] : 0ull;
                    const int lo = (int)(uint32_t)wd, hi = (int)(uint32_t)(wd >> 32);
#pragma unroll 8
                    for (int j = 0; j < 64; ++j) {
                        const uint32_t wl = (uint32_t)__builtin_amdgcn_readlane(lo, j);
                        const uint32_t wh = (uint32_t)__builtin_amdgcn_readlane(hi, j);
                        const int32_t uj = __builtin_amdgcn_readlane(u, j);
                        acc += (((lane < 32 ? wl : wh) >> (lane & 31)) & 1u) ? uj : 0;
                    }
                }
                const int t = 64 * k + lane;
                if (t < NQ && !((pbits[t >> 5] >> (t & 31)) & 1u)) {
                    const uint32_t cost = (uint32_t)(C0 + r1[t] + acc);
                    const unsigned long long key = ((unsigned long long)cost << 32) | (uint32_t)(t + 1);
                    mine = key < mine ? key : mine;
                }
            }
            __syncthreads();   // pair sums complete
            if (tid < nt * (nt - 1) / 2) {
                int x = 0, rr = tid;
                while (rr >= nt - 1 - x) {
                    rr -= nt - 1 - x;
                    ++x;
                }
                const int ta = tl[x], tb = tl[x + 1 + rr];
                const uint32_t cost = (uint32_t)(C0 + r1[ta] + r1[tb] + pairsum[tid]);
                const unsigned long long key = ((unsigned long long)cost << 32) | (uint32_t)(NQ + 1 + tid);
                mine = key < mine ? key : mine;
            }
            atomicMin(&best, mine);
            __syncthreads();
            const uint32_t idx = (uint32_t)best;
            if (idx >= 1 && idx <= (uint32_t)NQ) {
                ca = (int)idx - 1;
            } else if (idx > (uint32_t)NQ) {
                int x = 0, rr = (int)idx - NQ - 1;
                while (rr >= nt - 1 - x) {
                    rr -= nt - 1 - x;
                    ++x;
                }
                ca = tl[x];
                cb = tl[x + 1 + rr];
            }
            if (tid == 0 && ca >= 0) {
                const int qa = order[ca];
                atomicOr(&ebits[qa >> 5], 1u << (qa & 31));
                if (cb >= 0) {
                    const int qb = order[cb];
                    atomicOr(&ebits[qb >> 5], 1u << (qb & 31));
                }
            }
        }
#pragma unroll
        for (int i = 0; i < RPL; ++i)
            if ((piv >> i) & 1u) {
                const int r = tid + WG * i;
                uint32_t bit = (sb >> i) & 1u;
                if (CS && ca >= 0) {
                    bit ^= (uint32_t)((mat[(size_t)(ca >> 6) * M + r] >> (ca & 63)) & 1ull);
                    if (cb >= 0) bit ^= (uint32_t)((mat[(size_t)(cb >> 6) * M + r] >> (cb & 63)) & 1ull);
                }
                if (bit) {
                    const int q = order[pcol[i]];
                    atomicOr(&ebits[q >> 5], 1u << (q & 31));
                }
            }
        __syncthreads();
        if (misc[1] == 0) {
            if (a.ehat) {
                constexpr int EW32 = (NQ + 31) / 32;
                for (int wd = tid; wd < a.ehat_words; wd += WG) {
                    const uint64_t lo = (2 * wd < EW32) ? ebits[2 * wd] : 0u;
                    const uint64_t hi = (2 * wd + 1 < EW32) ? ebits[2 * wd + 1] : 0u;
                    a.ehat[shot * a.ehat_words + wd] = lo | (hi << 32);
                }
            }
            if (tid == 0) stats[shot].converged = 2;
        }
        __syncthreads();   // LDS and misc are reused by the next shot
    }
}

}  // namespace lead_spec
