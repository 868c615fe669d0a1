// Flooding-schedule LLR belief propagation over GF(4) for gfx950: the small and
// medium code kernel.  A group of G lanes decodes one shot at a time (G <= 64:
// groups inside one wavefront; G = 128 or 256: one group per workgroup).  The
// shot's messages, posteriors and accumulators live in LDS; the Tanner graph
// and the priors are staged once per workgroup in LDS and shared by all of its
// groups.  Groups pull shots from a queue and refill as soon as their shot
// stops, so the heavy tail of iteration counts never idles a wavefront.
//
// Paper: Chen, Yi, Liang, Wang, "Improved Belief Propagation Decoding
// Algorithms for Surface Codes".  Section II-B1 (eqs. init, h_update,
// v_update, p_update, lambda, hard decision), section III-A1 (Momentum-BP,
// eqs. mombp1-3), section III-A2 (AdaGrad-BP, eq. boost), section III-B
// (EWAInit-BP, eq. EWAInit, Algorithm 2).
//
// One LDS slot per Tanner edge, in variable-major order, alternately holds
// m_{c->v} (written by the check phase) and m_{v->c} (written by the qubit
// phase): every edge is read and rewritten by exactly one check and one
// qubit, so the two phases never race on a slot.
//
// The qubit phase uses lambda_H(Q - [<W,H>=1] m_{c->v}) = lambda_H(Q) - m_{c->v}
// (both anticommuting LLRs drop by m, which factors out of the denominator),
// so lambda is evaluated once per (qubit, label) instead of once per edge.
#include <cmath>

#include "bp4_internal.h"

namespace bp4 {

namespace {

__device__ __forceinline__ void wave_sync()
{
    // Lanes of one wavefront exchange data through LDS; LDS operations of a
    // wavefront execute in order, so only compiler reordering must be fenced.
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ float clampf(float x, float c) { return fminf(fmaxf(x, -c), c); }

constexpr float kLog2e = 1.44269504088896341f;
constexpr float kLn2 = 0.693147180559945309f;
constexpr float kLn4 = 1.38629436111989061f;

// Hardware base-2 exponential and logarithm (v_exp_f32, v_log_f32).
__device__ __forceinline__ float hw_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float hw_log2(float x) { return __builtin_amdgcn_logf(x); }

// phi(x) = -ln tanh(x/2) = 2 atanh(e^{-x}) for x >= 0, phi(0) = inf, phi(inf) = 0;
// 2 atanh(prod tanh(m_k/2)) = (prod sgn m_k) phi(sum phi(|m_k|)).
//   x >= ln 4: z = e^{-x} <= 1/4 and phi = 2 z P(z^2), P(w) = atanh(sqrt w)/sqrt w;
//   x <  ln 4: phi = ln(2/x) + u G(u), u = x^2/4, u G(u) = -ln(tanh(sqrt u)/sqrt u).
// P and G are least-squares fits on those ranges (relative error < 1e-7 in FP32);
// both forms keep full relative accuracy (no 1 - z or log(1 + tiny) cancellation).
__device__ __forceinline__ float phi(float x)
{
    if (x >= kLn4) {
        const float z = hw_exp2(-x * kLog2e);
        const float w = z * z;
        float p = fmaf(w, 0.12663664294804267f, 0.1419839934660223f);
        p = fmaf(w, p, 0.2000197421889f);
        p = fmaf(w, p, 0.3333331781245287f);
        p = fmaf(w, p, 1.00000000019442f);
        return (2.0f * z) * p;
    }
    const float u = 0.25f * x * x;
    float g = fmaf(u, 0.0014921690150859843f, -0.006451527278442298f);
    g = fmaf(u, g, 0.02182510967622784f);
    g = fmaf(u, g, -0.07777514939719771f);
    g = fmaf(u, g, 0.33333330803159383f);
    return fmaf(-hw_log2(0.5f * x), kLn2, u * g);
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

// Sum of three non-negative values in an order fixed by their values:
// (min + median) + max, so the result depends only on the multiset.
__device__ __forceinline__ float sum3_canonical(float a, float b, float c)
{
    const float lo = fminf(fminf(a, b), c);
    const float hi = fmaxf(fmaxf(a, b), c);
    const float mid = __builtin_amdgcn_fmed3f(a, b, c);
    return (lo + mid) + hi;
}

// AdaGrad gradients at or below this fraction of |D| + sum |m| count as 0.
constexpr float kAdaGradDeadband = 1.52587890625e-05f;   // 2^-16

// 1 iff single-qubit Paulis a, b (codes) anticommute.
__device__ __forceinline__ uint32_t anticomm(uint32_t a, uint32_t b)
{
    return ((a & (b >> 1)) ^ ((a >> 1) & b)) & 1u;
}

template <int G>
struct Group {
    static constexpr int kBlock = G > 64 ? G : 256;
    static constexpr bool kMultiWave = G > 64;
};

template <int G>
__global__ void __launch_bounds__(Group<G>::kBlock)
decode_lds_kernel(DecodeArgs a)
{
    extern __shared__ float lds[];
    constexpr int B = Group<G>::kBlock;
    constexpr bool MW = Group<G>::kMultiWave;
    const int m = a.g.m, n = a.g.n;

    // Workgroup-shared static data: packed check edges, packed qubit words, priors.
    uint32_t *s_ce = reinterpret_cast<uint32_t *>(lds);
    uint32_t *s_vi = s_ce + kMaxCheckDeg * m;
    float *s_pi = reinterpret_cast<float *>(s_vi + n);
    for (int i = threadIdx.x; i < kMaxCheckDeg * m; i += B) s_ce[i] = a.g.cedge[i];
    for (int i = threadIdx.x; i < n; i += B) s_vi[i] = a.g.vinfo[i];
    for (int i = threadIdx.x; i < 3 * n; i += B) s_pi[i] = a.prior[i];

    const int gid = MW ? 0 : (int)threadIdx.x / G;
    const int r = MW ? (int)threadIdx.x : (int)threadIdx.x % G;
    const int lead = MW ? 0 : (((int)threadIdx.x & 63) / G) * G;   // leader lane in the wavefront
    float *msg = lds + a.static_words + gid * a.region_words;
    float *qs = msg + a.q_off;                  // [n][3] posterior of the last iteration (AdaGrad: Q - Pi)
    float *acc = msg + a.acc_off;               // [n][3] momentum / squared-gradient sums
    uint8_t *ehat = reinterpret_cast<uint8_t *>(msg + a.ehat_off);
    __shared__ int bcast;

    __syncthreads();

    auto gsync = [&]() {
        if (MW) __syncthreads();
        else wave_sync();
    };
    const float C = a.clamp;
    const int variant = a.variant;
    const bool keep_q = variant != BP4_BP;
    const bool keep_acc = variant == BP4_MOMENTUM || variant == BP4_ADAGRAD;

    auto fetch = [&]() -> int {
        int s = 0;
        if (r == 0) s = (int)atomicAdd(a.counter, 1u);
        if (MW) {
            if (r == 0) bcast = s;
            __syncthreads();
            s = bcast;
            __syncthreads();
            return s;
        }
        return __shfl(s, lead, 64);
    };

    uint64_t sbits = 0;
    int t = 0;

    // Initialisation (eq. init, Algorithm 2): m^{(0)}_{v->c} = lambda_{H_cv}(Pi^{(0)}_v);
    // Q^{(0)} = Pi^{(0)}; momentum and squared-gradient accumulators start at 0.
    auto init = [&](int s) {
        sbits = 0;
        int k = 0;
        for (int c = r; c < m; c += G, ++k)
            if (a.synd[(size_t)s * m + c]) sbits |= 1ull << k;
        for (int v = r; v < n; v += G) {
            const uint32_t info = s_vi[v];
            const uint32_t base = var_base(info), deg = var_deg(info);
            const float p3[3] = {s_pi[3 * v], s_pi[3 * v + 1], s_pi[3 * v + 2]};
            for (uint32_t j = 0; j < deg; ++j) msg[base + j] = clampf(lambda_lab(var_lab(info, j), p3), C);
            if (keep_q)   // Q^{(0)} = Pi^{(0)}; AdaGrad keeps D^{(0)} = Q^{(0)} - Pi^{(0)} = 0
                for (int w = 0; w < 3; ++w) qs[3 * v + w] = variant == BP4_ADAGRAD ? 0.0f : p3[w];
            if (keep_acc)
                for (int w = 0; w < 3; ++w) acc[3 * v + w] = 0.0f;
        }
        t = 0;
    };

    int shot = fetch();
    if (shot < a.shots) init(shot);
    gsync();

    for (;;) {
        const bool live = shot < a.shots;
        if (MW ? !live : !__any(live)) break;
        if (live) {
            ++t;
            // ---- Horizontal update (eq. h_update) ----------------------------------
            for (int c = r; c < m; c += G) {
                const uint4 w4 = *reinterpret_cast<const uint4 *>(&s_ce[kMaxCheckDeg * c]);
                const uint32_t w[4] = {w4.x, w4.y, w4.z, w4.w};
                float f[4];
                uint32_t sgn[4];
                uint32_t neg = (uint32_t)(sbits >> ((c - r) / G)) & 1u;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const float mv = w[j] != kEdgePad ? msg[edge_slot(w[j])] : INFINITY;
                    sgn[j] = mv < 0.0f ? 1u : 0u;
                    neg ^= sgn[j];
                    f[j] = phi(fabsf(mv));
                }
                // leave-one-out sums of phi, formed directly (no subtraction) and in
                // value order, so equal multisets of inputs give bitwise equal outputs
                const float loo[4] = {sum3_canonical(f[1], f[2], f[3]), sum3_canonical(f[0], f[2], f[3]),
                                      sum3_canonical(f[0], f[1], f[3]), sum3_canonical(f[0], f[1], f[2])};
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    if (w[j] == kEdgePad) continue;
                    const float mag = phi(loo[j]);
                    msg[edge_slot(w[j])] = clampf((neg ^ sgn[j]) ? -mag : mag, C);
                }
            }
        }
        gsync();
        if (live) {
            // ---- Posterior, hard decision and vertical update ------------------------
            for (int v = r; v < n; v += G) {
                const uint32_t info = s_vi[v];
                const uint32_t base = var_base(info), deg = var_deg(info);
                float mc[4];
                // per-label sums of m_{c->v} (index = label code; 1 X, 2 Z, 3 Y)
                float S[4] = {0.0f, 0.0f, 0.0f, 0.0f}, A[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    mc[j] = 0.0f;
                    if ((uint32_t)j < deg) {
                        const uint32_t lab = var_lab(info, j);
                        mc[j] = msg[base + j];
                        S[lab] += mc[j];
                        A[lab] += fabsf(mc[j]);
                    }
                }
                // M_{v,W}: sum of m_{c->v} over edges whose label anticommutes with W,
                // i.e. the two other labels (eqs. p_update, mombp3, boost)
                const float M[3] = {S[3] + S[2], S[1] + S[2], S[1] + S[3]};
                const float p3[3] = {s_pi[3 * v], s_pi[3 * v + 1], s_pi[3 * v + 2]};
                float qn[3];
                if (variant == BP4_BP) {                 // eq. p_update
#pragma unroll
                    for (int x = 0; x < 3; ++x) qn[x] = p3[x] + M[x];
                } else if (variant == BP4_EWAINIT) {     // eq. EWAInit, then eq. p_update
#pragma unroll
                    for (int x = 0; x < 3; ++x) {
                        const float pit = t == 1 ? p3[x] : a.alpha * p3[x] + (1.0f - a.alpha) * qs[3 * v + x];
                        qn[x] = pit + M[x];
                    }
                } else if (variant == BP4_MOMENTUM) {    // eqs. mombp1, mombp2 with the gradient of mombp3
#pragma unroll
                    for (int x = 0; x < 3; ++x) {
                        const float qp = qs[3 * v + x];
                        const float g = a.gamma * acc[3 * v + x] + (1.0f - a.gamma) * (qp - p3[x] - M[x]);
                        acc[3 * v + x] = g;
                        qn[x] = qp - a.alpha * g;
                    }
                } else {                                 // eq. boost, adaptive from t = 2
                    // qs holds D = Q - Pi^{(0)}; the gradient Q^{(t-1)} - Pi - M is D - M.
                    const float Mabs[3] = {A[3] + A[2], A[1] + A[2], A[1] + A[3]};
#pragma unroll
                    for (int x = 0; x < 3; ++x) {
                        const float dp = qs[3 * v + x];
                        float grad = dp - M[x];
                        // a gradient below the rounding resolution of its operands is 0
                        if (fabsf(grad) <= kAdaGradDeadband * (fabsf(dp) + Mabs[x])) grad = 0.0f;
                        float d;
                        if (t == 1) {
                            if (a.g_from_t1) acc[3 * v + x] = grad * grad;
                            d = M[x];
                        } else {
                            const float G2 = acc[3 * v + x] + grad * grad;
                            acc[3 * v + x] = G2;
                            d = dp - a.alpha * grad / (sqrtf(G2) + a.eps);
                        }
                        qs[3 * v + x] = d;
                        qn[x] = p3[x] + d;
                    }
                }
                // Hard decision: I if every LLR > 0, else the smallest (ties: X, Y, Z).
                uint32_t e;
                if (qn[0] > 0.0f && qn[1] > 0.0f && qn[2] > 0.0f) {
                    e = 0u;
                } else {
                    int b = 0;
                    if (qn[1] < qn[b]) b = 1;
                    if (qn[2] < qn[b]) b = 2;
                    e = b == 0 ? 1u : (b == 1 ? 3u : 2u);
                }
                if (isnan(qn[0]) || isnan(qn[1]) || isnan(qn[2])) e = 0xFFu;   // cannot converge
                ehat[v] = (uint8_t)e;
                if (keep_q && variant != BP4_ADAGRAD)
                    for (int x = 0; x < 3; ++x) qs[3 * v + x] = qn[x];
                // Vertical update (eqs. v_update / mombp5): m_{v->c} = lambda_H(Q) - m_{c->v}.
                float lam[4] = {0.0f, 0.0f, 0.0f, 0.0f};   // by label code
                const uint32_t present = var_labels_present(info);
                if (present & 2u)   // X: pair (Y, Z)
                    lam[1] = lambda_sp(qn[0], qn[1], qn[2], softplus_neg_abs(qn[0]), softplus_neg_abs(qn[1] - qn[2]));
                if (present & 4u)   // Z: pair (X, Y)
                    lam[2] = lambda_sp(qn[2], qn[0], qn[1], softplus_neg_abs(qn[2]), softplus_neg_abs(qn[0] - qn[1]));
                if (present & 8u)   // Y: pair (X, Z)
                    lam[3] = lambda_sp(qn[1], qn[0], qn[2], softplus_neg_abs(qn[1]), softplus_neg_abs(qn[0] - qn[2]));
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    if ((uint32_t)j >= deg) continue;
                    const float out = clampf(lam[var_lab(info, j)] - mc[j], C);
                    msg[base + j] = out;
                    if (a.mvc_out) {
                        const size_t o = (size_t)shot * a.g.nnz + a.g.vcanon[base + j];
                        a.mvc_out[o] = out;
                        a.mcv_out[o] = mc[j];
                    }
                }
                if (a.q_out)
                    for (int x = 0; x < 3; ++x) a.q_out[((size_t)shot * n + v) * 3 + x] = qn[x];
            }
        }
        gsync();
        bool fin = false, sat = false;
        if (live) {
            // ---- Syndrome test of the hard decision (Algorithm 2) -------------------
            uint32_t bad = 0;
            for (int c = r; c < m; c += G) {
                const uint4 w4 = *reinterpret_cast<const uint4 *>(&s_ce[kMaxCheckDeg * c]);
                const uint32_t w[4] = {w4.x, w4.y, w4.z, w4.w};
                uint32_t par = (uint32_t)(sbits >> ((c - r) / G)) & 1u;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    if (w[j] == kEdgePad) continue;
                    const uint32_t e = ehat[edge_var(w[j])];
                    if (e == 0xFFu) bad = 1u;
                    else par ^= anticomm(edge_lab(w[j]), e);
                }
                bad |= par;
            }
            if (MW) {
                sat = __syncthreads_or(bad) == 0;
            } else {
                const uint64_t ballot = __ballot(bad != 0);
                const uint64_t gmask = (G == 64) ? ~0ull : (((1ull << G) - 1ull) << lead);
                sat = (ballot & gmask) == 0;
            }
            fin = (a.stop && sat) || t >= a.max_iter;
        }
        if (fin) {
            for (int v = r; v < n; v += G) {
                const uint8_t e = ehat[v];
                a.est[(size_t)shot * n + v] = e == 0xFFu ? 0 : e;
            }
            if (r == 0) {
                a.conv[shot] = sat ? 1 : 0;
                a.iters[shot] = t;
            }
            gsync();
            shot = fetch();
            if (shot < a.shots) init(shot);
        }
        gsync();
    }
}

template <int G>
hipError_t launch_g(const DecodeArgs &a, size_t lds_bytes, hipStream_t s)
{
    constexpr int B = Group<G>::kBlock;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    int cus = 0, per_cu = 0;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, decode_lds_kernel<G>, B, lds_bytes);
    if (e != hipSuccess) return e;
    if (per_cu < 1) return hipErrorInvalidConfiguration;
    const long groups_per_block = B / G;
    const long want = (a.shots + groups_per_block - 1) / groups_per_block;
    long grid = (long)cus * per_cu;
    if (want < grid) grid = want;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(decode_lds_kernel<G>, dim3((unsigned)grid), dim3(B), lds_bytes, s, a);
    return hipGetLastError();
}

}  // namespace

LdsLayout decode_lds_layout(int m, int n, int nnz, int variant, int G)
{
    LdsLayout L;
    L.static_words = kMaxCheckDeg * m + n + 3 * n;
    if (L.static_words & 3) L.static_words += 4 - (L.static_words & 3);
    int w = nnz;
    L.q_off = w;
    if (variant != BP4_BP) w += 3 * n;
    L.acc_off = w;
    if (variant == BP4_MOMENTUM || variant == BP4_ADAGRAD) w += 3 * n;
    L.ehat_off = w;
    w += (n + 3) / 4;
    if ((w & 1) == 0) w += 1;   // odd stride: neighbouring groups start on other banks
    L.region_words = w;
    const int block = G > 64 ? G : 256;
    L.group_lanes = G;
    L.block = block;
    L.bytes = (size_t)4 * (L.static_words + (size_t)(block / G) * L.region_words);
    return L;
}

// Lanes per shot for a code when no tuned choice is given.  Score = lane use
// (padding of m and n up to multiples of G) times an occupancy factor: the
// wavefronts per CU that the LDS allows (up to 16, beyond which latency is
// hidden) over 16.  At most 64 checks per lane; at most `max_lds` bytes of LDS
// per workgroup.
int decode_lds_pick_group(int m, int n, int nnz, int variant, size_t max_lds)
{
    const int cand[7] = {256, 128, 64, 32, 16, 8, 4};
    const double cu_lds = 160.0 * 1024.0;
    int best = -1;
    double best_score = -1.0;
    for (int i = 0; i < 7; ++i) {
        const int G = cand[i];
        if ((m + G - 1) / G > 64) continue;
        const LdsLayout L = decode_lds_layout(m, n, nnz, variant, G);
        if (L.bytes > max_lds) continue;
        const int kc = (m + G - 1) / G, kv = (n + G - 1) / G;
        const double util = 0.5 * ((double)m / (G * kc) + (double)n / (G * kv));
        const double blocks = std::floor(cu_lds / (double)L.bytes);
        double waves = blocks * (L.block / 64);
        if (waves > 16.0) waves = 16.0;
        const double score = util * waves / 16.0;
        if (score > best_score * 1.02) {
            best_score = score;
            best = G;
        }
    }
    return best;
}

hipError_t launch_decode_lds(const DecodeArgs &a, const LdsLayout &L, hipStream_t s)
{
    switch (L.group_lanes) {
    case 256: return launch_g<256>(a, L.bytes, s);
    case 128: return launch_g<128>(a, L.bytes, s);
    case 64: return launch_g<64>(a, L.bytes, s);
    case 32: return launch_g<32>(a, L.bytes, s);
    case 16: return launch_g<16>(a, L.bytes, s);
    case 8: return launch_g<8>(a, L.bytes, s);
    case 4: return launch_g<4>(a, L.bytes, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace bp4
