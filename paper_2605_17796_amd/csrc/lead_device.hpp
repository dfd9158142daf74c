// Device arithmetic shared by the precompiled decoding kernels and the
// kernels the library compiles at run time for one code.  Both must produce
// the same bits, so everything here is either a correctly rounded IEEE
// operation or a single hardware instruction (v_exp_f32, v_log_f32,
// v_rcp_f32, v_med3_f32), never a library routine whose rounding could
// differ between compiler versions.  Self-contained for the run-time
// compiler.
#pragma once
#include "lead_args.hpp"

namespace lead_dev {

constexpr float kBig = 1e30f;
constexpr uint32_t kSign = 0x80000000u;

__device__ __forceinline__ float clampf(float x, float c) { return __builtin_amdgcn_fmed3f(x, -c, c); }

// Sign tests use the IEEE sign bit: no variable sum or mu is ever -0 (every
// sum starts from a prior canonicalised to +0 and x + (-x) rounds to +0), so
// signbit(x) == (x < 0) throughout.
__device__ __forceinline__ uint32_t signbit_of(float x) { return __float_as_uint(x) >> 31; }

// Message of min-sum check state (m1, m2, am, q) to its k-th variable:
// (-1)^{q_k} * (k == am ? m2 : m1), with m1, m2 already scaled by beta.  The
// sign bit is moved to bit 31 and merged into the (non-negative) magnitude.
__device__ __forceinline__ float msg_of(float m1, float m2, uint32_t am, uint32_t q, uint32_t k) {
    const float mag = (k == am) ? m2 : m1;
    return __uint_as_float(__float_as_uint(mag) | ((q << (31u - k)) & kSign));
}

// e^x as 2^(x log2 e) on the hardware exponential.
__device__ __forceinline__ float exp_hw(float x) { return __builtin_amdgcn_exp2f(x * 1.44269504088896341f); }

// Phase 2 of Algorithm 1 for one qubit from the clamped posteriors La, Lb of
// its two views (Sec. III, the regularised aggregation):
//   p = sigma(-L) = 1 / (1 + e^L),  q = 1 - p = sigma(L) = 1 / (1 + e^-L),
//   p_hat = alpha * (p_a + p_b) / 2,  1 - p_hat = (1 - alpha) + alpha * (q_a + q_b) / 2,
//   lambda' = ln(1 - p_hat) - ln(p_hat), clamped.
// 1 - p_hat is formed from q rather than by subtraction, so it keeps full
// relative precision when p_hat is close to 1.  Symmetric in (La, Lb) bit for
// bit (only sums of the two views' terms are formed), so either occurrence of
// the qubit computes the same value.
__device__ __forceinline__ float aggregate_llr(float La, float Lb, float alpha, float clampv) {
    const float pa = __builtin_amdgcn_rcpf(1.f + exp_hw(La)), pb = __builtin_amdgcn_rcpf(1.f + exp_hw(Lb));
    const float qa = __builtin_amdgcn_rcpf(1.f + exp_hw(-La)), qb = __builtin_amdgcn_rcpf(1.f + exp_hw(-Lb));
    const float ph = alpha * (0.5f * (pa + pb));
    const float qh = __builtin_fmaf(alpha, 0.5f * (qa + qb), 1.f - alpha);
    const float l2 = __builtin_amdgcn_logf(qh) - __builtin_amdgcn_logf(ph);   // log2 ratio
    return clampf(l2 * 0.693147180559945309f, clampv) + 0.f;
}

// e^x to about two ulps: x log2(e) is formed as hi + lo (log2(e) split into
// a float and its remainder, the product's rounding error recovered with an
// fma), and 2^(hi + lo) = 2^hi (1 + lo ln 2) since |lo| < 2^-18.  exp_hw's
// single rounding of x log2(e) costs up to |x| log2(e) 2^-24 of relative
// error in e^x (about 20 ulps at x = 20).
__device__ __forceinline__ float exp_acc(float x) {
    constexpr float L1 = 1.44269502162933349609375f;      // log2(e) rounded to float
    constexpr float L2 = 1.925963033500011079e-8f;         // log2(e) - L1
    const float hi = x * L1;
    // beyond 128 e^x overflows anyway; there (x = +inf: phi(+inf) = 0 needs
    // e^x = +inf) the correction would be inf - inf
    const float lo = x < 128.f ? __builtin_fmaf(x, L1, -hi) + x * L2 : 0.f;
    return __builtin_amdgcn_exp2f(hi) * __builtin_fmaf(lo, 0.693147180559945309f, 1.f);
}

// Sum-product in the log domain (Gallager's phi):
//   phi(x) = ln((e^x + 1) / (e^x - 1)) = -ln tanh(x / 2) = log1p(2 / expm1(x)),  x >= 0,
// its own inverse, with phi(0) = +inf and phi(+inf) = 0; the check message
// 2 atanh(prod_j' tanh(mu_j' / 2)) has magnitude phi(sum_j' phi(|mu_j'|)).
// expm1 and log1p take a short series where the plain form would cancel, so
// phi keeps full relative precision at both ends (phi(30) ~ 1.9e-13 and
// phi(1e-6) ~ 14.5), and a correction of the rounding of 1 + y elsewhere.
__device__ __forceinline__ float expm1_nonneg(float x) {
    // x (1 + x/2 (1 + x/3 (... (1 + x/8)))) below 1/2: truncation below 1e-8 relative
    float t = __builtin_fmaf(x, 0.125f, 1.f);
    t = __builtin_fmaf(x * (1.f / 7.f), t, 1.f);
    t = __builtin_fmaf(x * (1.f / 6.f), t, 1.f);
    t = __builtin_fmaf(x * 0.2f, t, 1.f);
    t = __builtin_fmaf(x * 0.25f, t, 1.f);
    t = __builtin_fmaf(x * (1.f / 3.f), t, 1.f);
    t = __builtin_fmaf(x * 0.5f, t, 1.f);
    const float series = x * t;
    return x < 0.5f ? series : exp_acc(x) - 1.f;
}

__device__ __forceinline__ float log1p_nonneg(float y) {
    // y - y^2/2 + y^3/3 - y^4/4 + y^5/5 below 1/32: truncation below 1e-9 relative
    float t = __builtin_fmaf(y, 0.2f, -0.25f);
    t = __builtin_fmaf(y, t, 1.f / 3.f);
    t = __builtin_fmaf(y, t, -0.5f);
    t = __builtin_fmaf(y, t, 1.f);
    const float series = y * t;
    // ln(u) for u = fl(1 + y), times y / (u - 1) to undo the rounding of
    // 1 + y (u - 1 is exact below 2); above 1 that rounding is harmless
    const float u = 1.f + y;
    const float lg = __builtin_amdgcn_logf(u) * 0.693147180559945309f;
    const float corr = y < 1.f ? y / (u - 1.f) : 1.f;
    return y < 0.03125f ? series : lg * corr;
}

__device__ __forceinline__ float phi(float x) {
    return log1p_nonneg(2.f * __builtin_amdgcn_rcpf(expm1_nonneg(x)));
}

}  // namespace lead_dev
