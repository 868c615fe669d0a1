// Device arithmetic of one flooding BP iteration, shared by every decode kernel:
// the check-node function phi, the commutation LLR lambda, leave-one-out sums.
//
// Paper: Chen, Yi, Liang, Wang, "Improved Belief Propagation Decoding
// Algorithms for Surface Codes", section II-B1 (eqs. init, h_update, v_update,
// p_update and the lambda function), section III-A2 (eq. boost).
#pragma once

#include "bp4_internal.h"

namespace bp4 {

// Next shot index from a queue head; the head can pass 2^31 near the shot limit,
// so it is compared unsigned and saturated at `shots` (= no shot left).
__device__ __forceinline__ int take_shot(unsigned int *head, int32_t shots)
{
    const unsigned got = atomicAdd(head, 1u);
    return got < (unsigned)shots ? (int)got : shots;
}

__device__ __forceinline__ void wave_sync()
{
    // Lanes of one wavefront exchange data through LDS; LDS operations of a
    // wavefront execute in order, so only compiler reordering must be fenced.
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Clamp to [-c, c] in one instruction (v_med3_f32).
__device__ __forceinline__ float clampf(float x, float c) { return __builtin_amdgcn_fmed3f(x, -c, c); }

constexpr float kLog2e = 1.44269504088896341f;
constexpr float kLn2 = 0.693147180559945309f;

// Hardware base-2 exponential and logarithm (v_exp_f32, v_log_f32).
__device__ __forceinline__ float hw_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float hw_log2(float x) { return __builtin_amdgcn_logf(x); }

// phi(x) = -ln tanh(x/2) = 2 atanh(e^{-x}) for x >= 0, phi(0) = inf, phi(inf) = 0;
// 2 atanh(prod tanh(m_k/2)) = (prod sgn m_k) phi(sum phi(|m_k|)).
//   x >= 5/4: z = e^{-x} < 0.29 and phi = z Q(z^2), Q(w) = 2 atanh(sqrt w)/sqrt w;
//   x <  5/4: phi = -ln x + H(x^2), H(v) = ln 2 - ln(tanh(s)/s) at s = sqrt(v)/2.
// Q is a cubic and H a quartic with H(0) = ln 2, minimax fits on those ranges
// (relative error of phi below 2e-7 from the fits and FP32 rounding, up to
// x = 20; beyond, the rounding of the exponent argument dominates); both forms
// keep full relative accuracy (no 1 - z or log(1 + tiny) cancellation).  Six
// FP32 operations and one transcendental either way.
constexpr float kPhiSplit = 1.25f;
__device__ __forceinline__ float phi(float x)
{
    if (x >= kPhiSplit) {
        const float z = hw_exp2(-x * kLog2e);
        const float w = z * z;
        float q = fmaf(w, 0.32597747557296414f, 0.397865114107555f);
        q = fmaf(w, q, 0.6667023642453243f);
        q = fmaf(w, q, 1.9999999066205403f);
        return z * q;
    }
    const float v = x * x;
    float h = fmaf(v, -1.929226050977351e-05f, 0.0003326163940672604f);
    h = fmaf(v, h, -0.004856116024095805f);
    h = fmaf(v, h, 0.08333242282884455f);
    h = fmaf(v, h, kLn2);
    return fmaf(-hw_log2(x), kLn2, h);
}

// ln(1 + e^{-|y|}): the correction term of a two-term log-sum-exp.
__device__ __forceinline__ float softplus_neg_abs(float y)
{
    return hw_log2(1.0f + hw_exp2(-fabsf(y) * kLog2e)) * kLn2;
}

// lambda_H(Q) = ln(1 + e^{-Q_H}) - ln(e^{-Q_a} + e^{-Q_b}), {a, b} = {X,Y,Z} \ {H}
//             = [max(-Q_H, 0) - max(-Q_a, -Q_b)] + sp(Q_H) - sp(Q_a - Q_b),
// with sp(y) = ln(1 + e^{-|y|}) given precomputed (spH, spAB).
__device__ __forceinline__ float lambda_sp(float qh, float qa, float qb, float spH, float spAB)
{
    return (fmaxf(-qh, 0.0f) - fmaxf(-qa, -qb)) + (spH - spAB);
}

// lambda for the (X, Y, Z) posterior q with a generic label (setup code only).
__device__ __forceinline__ float lambda_lab(uint32_t lab, const float q[3])
{
    const int h = lab == 1u ? 0 : (lab == 3u ? 1 : 2);
    const float qa = q[h == 0 ? 1 : 0], qb = q[h == 2 ? 1 : 2];
    return lambda_sp(q[h], qa, qb, softplus_neg_abs(q[h]), softplus_neg_abs(qa - qb));
}

// Sum of three non-negative values in an order fixed by their values,
// (min + median) + max, so the result depends only on the multiset: a check whose
// inputs are a permutation of another check's gives bitwise equal outputs, and
// exact symmetries of a syndrome survive FP32 rounding.  Non-negative floats order
// like their bit patterns as unsigned integers, so the order comes from integer
// min / max / median (the median written in the form the compiler turns into one
// v_med3_u32) instead of floating-point compares.
__device__ __forceinline__ float sum3_canonical(float a, float b, float c)
{
    const uint32_t ua = __float_as_uint(a), ub = __float_as_uint(b), uc = __float_as_uint(c);
    const uint32_t lo = min(ua, min(ub, uc)), hi = max(ua, max(ub, uc));
    const uint32_t mid = min(max(ua, ub), max(min(ua, ub), uc));   // one v_med3_u32
    return (__uint_as_float(lo) + __uint_as_float(mid)) + __uint_as_float(hi);
}

// Leave-one-out sums of four non-negative values: loo[j] sums the three values other
// than f[j], formed directly (no subtraction) in value order.
__device__ __forceinline__ void loo4(const float f[4], float loo[4])
{
#pragma clang fp contract(off)
    loo[0] = sum3_canonical(f[1], f[2], f[3]);
    loo[1] = sum3_canonical(f[0], f[2], f[3]);
    loo[2] = sum3_canonical(f[0], f[1], f[3]);
    loo[3] = sum3_canonical(f[0], f[1], f[2]);
}

// AdaGrad gradients at or below this fraction of |D| + sum |m| count as 0: FP32
// cannot resolve their sign, and eq. boost's first adaptive step is about
// alpha sign(g').  2^-20 is about eight FP32 roundings of the operands; against
// the FP64 evaluation of eq. boost it kept more entries within 1e-5 than 2^-16,
// and far more than 2^-24 or no threshold (rounding residue of sums that are
// equal in exact arithmetic then takes a full step).
#ifndef BP4_ADAGRAD_DEADBAND
#define BP4_ADAGRAD_DEADBAND 9.5367431640625e-07f   // 2^-20
#endif
constexpr float kAdaGradDeadband = BP4_ADAGRAD_DEADBAND;

// 1 iff single-qubit Paulis a, b (codes) anticommute.
__device__ __forceinline__ uint32_t anticomm(uint32_t a, uint32_t b)
{
    return ((a & (b >> 1)) ^ ((a >> 1) & b)) & 1u;
}


// Per-label sums of a qubit's incoming check messages mc[j] (slot order; label of
// slot j from the packed qubit word; slots >= degree hold 0): S[lab] and the sums
// of magnitudes A[lab], lab = 1 X, 2 Z, 3 Y.  Each label's sum runs over its own
// slots only, so with at most two edges per label the result does not depend on
// the slot order.
// with_y: the code has Y entries (else S[3] = 0); with_abs: also form A.
__device__ __forceinline__ void label_sums(uint32_t info, const float mc[4], bool with_y, bool with_abs,
                                           float S[4], float A[4])
{
    S[0] = A[0] = 0.0f;
    float s1 = 0.0f, s2 = 0.0f, s3 = 0.0f;
#pragma unroll
    for (int j = 0; j < 4; ++j) {   // labels of unused slots are 0
        const uint32_t l = var_lab(info, j);
        s1 += l == 1u ? mc[j] : 0.0f;
        s2 += l == 2u ? mc[j] : 0.0f;
        if (with_y) s3 += l == 3u ? mc[j] : 0.0f;
    }
    S[1] = s1;
    S[2] = s2;
    S[3] = s3;
    float a1 = 0.0f, a2 = 0.0f, a3 = 0.0f;
    if (with_abs) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t l = var_lab(info, j);
            a1 += l == 1u ? fabsf(mc[j]) : 0.0f;
            a2 += l == 2u ? fabsf(mc[j]) : 0.0f;
            a3 += l == 3u ? fabsf(mc[j]) : 0.0f;
        }
    }
    A[1] = a1;
    A[2] = a2;
    A[3] = a3;
}

// Discount of AEWA attempt k: alpha + (alpha_last - alpha) k / (steps - 1).
__device__ __forceinline__ float aewa_alpha(float alpha, float alpha_last, int steps, int k)
{
#pragma clang fp contract(off)
    return steps > 1 ? alpha + (alpha_last - alpha) * ((float)k / (float)(steps - 1)) : alpha;
}

// Hyperparameters a qubit update needs (section III).
struct VariantParams {
    int32_t variant, g_from_t1;
    float alpha, gamma, eps;
};

// Per-qubit state carried between iterations: st = Q^{(t-1)} (EWAInit, Momentum) or
// D^{(t-1)} = Q^{(t-1)} - Pi^{(0)} (AdaGrad); acc = momentum g or AdaGrad's G.
__device__ __forceinline__ void qubit_state_init(int variant, const float pi[3], float st[3], float acc[3])
{
#pragma unroll
    for (int x = 0; x < 3; ++x) {
        st[x] = variant == BP4_ADAGRAD ? 0.0f : pi[x];   // Q^{(0)} = Pi^{(0)}, D^{(0)} = 0
        acc[x] = 0.0f;
    }
}

// Posterior of iteration t from the per-label sums S[lab] of the incoming check
// messages and A[lab] of their magnitudes (lab: 1 X, 2 Z, 3 Y).
//   BP (eq. p_update):     Q = Pi + M
//   EWAInit (eq. EWAInit): Pi^{(t)} = alpha Pi + (1 - alpha) Q^{(t-1)} for t > 1; Q = Pi^{(t)} + M
//   Momentum (eqs. mombp1, mombp2, gradient of mombp3):
//                          g = gamma g + (1 - gamma)(Q^{(t-1)} - Pi - M); Q = Q^{(t-1)} - alpha g
//   AdaGrad (eq. boost):   t = 1: Q = Pi + M; t > 1: g' = D - M, G += g'^2,
//                          D -= alpha g' / (sqrt(G) + eps); Q = Pi + D
// where M_W sums the messages whose label anticommutes with W: the other two labels.
__device__ __forceinline__ void qubit_posterior(const VariantParams &vp, int t, const float pi[3],
                                                const float S[4], const float A[4], float st[3],
                                                float acc[3], float qn[3])
{
    // Every kernel must round these updates identically, so no multiply-add is
    // left to the compiler: the fused ones are written out.
#pragma clang fp contract(off)
    const float M[3] = {S[3] + S[2], S[1] + S[2], S[1] + S[3]};
    if (vp.variant == BP4_BP) {
#pragma unroll
        for (int x = 0; x < 3; ++x) qn[x] = pi[x] + M[x];
    } else if (vp.variant == BP4_EWAINIT || vp.variant == BP4_AEWA) {
#pragma unroll
        for (int x = 0; x < 3; ++x) {
            const float pit = t == 1 ? pi[x] : fmaf(vp.alpha, pi[x], (1.0f - vp.alpha) * st[x]);
            qn[x] = pit + M[x];
            st[x] = qn[x];
        }
    } else if (vp.variant == BP4_MOMENTUM) {
#pragma unroll
        for (int x = 0; x < 3; ++x) {
            const float g = fmaf(vp.gamma, acc[x], (1.0f - vp.gamma) * (st[x] - pi[x] - M[x]));
            acc[x] = g;
            qn[x] = fmaf(-vp.alpha, g, st[x]);
            st[x] = qn[x];
        }
    } else {
        const float Mabs[3] = {A[3] + A[2], A[1] + A[2], A[1] + A[3]};
#pragma unroll
        for (int x = 0; x < 3; ++x) {
            float grad = st[x] - M[x];
            // a gradient below the rounding resolution of its operands is 0
            if (fabsf(grad) <= kAdaGradDeadband * (fabsf(st[x]) + Mabs[x])) grad = 0.0f;
            float d;
            if (t == 1) {
                if (vp.g_from_t1) acc[x] = grad * grad;
                d = M[x];
            } else {
                const float G2 = fmaf(grad, grad, acc[x]);
                acc[x] = G2;
                d = st[x] - (vp.alpha * grad) / (sqrtf(G2) + vp.eps);
            }
            st[x] = d;
            qn[x] = pi[x] + d;
        }
    }
}

// Hard decision (section II-B1): I if every LLR is positive, else the Pauli with the
// smallest LLR, ties to the first of X, Y, Z.  0xFF marks a NaN posterior (the shot
// cannot converge).
__device__ __forceinline__ uint32_t hard_decision(const float q[3])
{
    const float mn = fminf(fminf(q[0], q[1]), q[2]);
    uint32_t e = q[0] == mn ? 1u : (q[1] == mn ? 3u : 2u);
    if (mn > 0.0f) e = 0u;
    if (isnan(q[0]) || isnan(q[1]) || isnan(q[2])) e = 0xFFu;
    return e;
}

// Decision byte of a qubit: bits 0-3 say which stabilizer labels the decision
// anticommutes with (bit L for label L = 1 X, 2 Z, 3 Y; bit 0 marks a NaN
// posterior), bits 4-5 hold the Pauli code itself.  A check then adds
// <H_cv, E^_v> to its parity as bit H_cv of the byte.
//   I: 0x00, X: 0x1C (anticommutes with Z, Y), Z: 0x2A (X, Y), Y: 0x36 (X, Z), NaN: 0x01
__device__ __forceinline__ uint32_t decision_byte(uint32_t e)
{
    if (e == 0xFFu) return 1u;                        // NaN: never satisfies a check
    return ((0x6AC0u >> (4u * e)) & 0xFu) | (e << 4);
}

// The decision byte straight from the posterior (same result as
// decision_byte(hard_decision(q)), without the intermediate code).
__device__ __forceinline__ uint32_t decision_byte_of(const float q[3])
{
    const float mn = fminf(fminf(q[0], q[1]), q[2]);
    uint32_t b = q[0] == mn ? 0x1Cu : (q[1] == mn ? 0x36u : 0x2Au);
    if (mn > 0.0f) b = 0u;
    if (isnan(q[0]) || isnan(q[1]) || isnan(q[2])) b = 1u;
    return b;
}
__device__ __forceinline__ uint32_t decision_pauli(uint32_t byte) { return byte >> 4; }

// lambda_H(Q) for each label present (bit 2 X, 4 Z, 8 Y), indexed by label code.
__device__ __forceinline__ void qubit_lambdas(const float q[3], uint32_t present, float lam[4])
{
    lam[0] = lam[1] = lam[2] = lam[3] = 0.0f;
    if (present & 2u)   // X: anticommuting pair (Y, Z)
        lam[1] = lambda_sp(q[0], q[1], q[2], softplus_neg_abs(q[0]), softplus_neg_abs(q[1] - q[2]));
    if (present & 4u)   // Z: pair (X, Y)
        lam[2] = lambda_sp(q[2], q[0], q[1], softplus_neg_abs(q[2]), softplus_neg_abs(q[0] - q[1]));
    if (present & 8u)   // Y: pair (X, Z)
        lam[3] = lambda_sp(q[1], q[0], q[2], softplus_neg_abs(q[1]), softplus_neg_abs(q[0] - q[2]));
}

// Check-node update (eq. h_update) of one check of degree <= 4 given its incoming
// messages mv[j] (padding: +inf) and syndrome bit s: outputs out[j] for j < 4.
// The sign of each output is the XOR of the syndrome bit and the other inputs'
// sign bits (a -0 input counts as negative: its own phi is +inf, so the only
// outputs it changes are zeros, whose sign it flips).
__device__ __forceinline__ void check_update(const float mv[4], uint32_t s, float C, float out[4])
{
    constexpr uint32_t kSign = 0x80000000u;
    float f[4];
    uint32_t b[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        b[j] = __float_as_uint(mv[j]);
        f[j] = phi(fabsf(mv[j]));
    }
    const uint32_t neg = b[0] ^ b[1] ^ b[2] ^ b[3] ^ (s << 31);   // sign bit: product of all signs
    // leave-one-out sums of phi, formed directly (no subtraction) and in value order,
    // so equal multisets of inputs give bitwise equal outputs
    float loo[4];
    loo4(f, loo);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const float mag = phi(loo[j]);   // >= 0 (or NaN)
        const uint32_t sgn = (neg ^ b[j]) & kSign;
        out[j] = clampf(__uint_as_float(__float_as_uint(mag) ^ sgn), C);
    }
}

}  // namespace bp4
