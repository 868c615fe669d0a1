// Unrolled EWAInit-BP and Momentum-BP over GF(4) with a fixed number T of
// flooding iterations and no early stop, their soft loss, and the hand-written
// adjoint (reverse-mode derivative) with respect to the per-iteration parameters
// and the priors Pi^{(0)}.
//
// Forward (check and qubit rules of section II-B1, the same per-node arithmetic
// as the decode kernels):
//   EWAInit (section III-B, eq. EWAInit and Algorithm 2), a discount alpha_t per
//   iteration: Pi^{(1)} = Pi^{(0)}, Pi^{(t)} = alpha_t Pi^{(0)} + (1 - alpha_t)
//   Q^{(t-1)}, Q^{(t)} = Pi^{(t)} + M^{(t)}.
//   Momentum (section III-A1, eqs. mombp1-3), a step alpha_t and a decay gamma_t
//   per iteration: g^{(t)} = gamma_t g^{(t-1)} + (1 - gamma_t)(Q^{(t-1)} - Pi^{(0)}
//   - M^{(t)}), Q^{(t)} = Q^{(t-1)} - alpha_t g^{(t)}, g^{(0)} = 0.
// Loss: the mean over shots and qubits of ln(1 + sum_W e^{-Q_W}) + Q_{e_v} at
// t = T (Q_I = 0), the negative log GF(4) marginal of the sampled error.
//
// A workgroup of kUnrWaves wavefronts runs a chunk of 64 shots, one shot per
// lane column: wavefront g takes the checks and the qubits whose index is g
// modulo kUnrWaves, with a workgroup barrier between the check and the qubit
// pass.  The state of a shot after iteration t is its messages m_{v->c}^{(t)}
// (E words) and its posterior Q^{(t)} (3N words), for Momentum also g^{(t)} and
// the incoming sums M^{(t)} (3N words each), kept as a column of a per-chunk
// record [chunk][item][64 columns] in HBM.
// The forward keeps the state every `ckpt` iterations; the adjoint walks the
// segments from last to first, recomputes a segment's states from its
// checkpoint, then runs the reverse sweep through it.  Gradient sums over
// shots are wavefront partials in FP64, reduced in a fixed order.
#include "bp4_math.h"

namespace bp4 {
namespace {

constexpr int kUnrWaves = 8;                // wavefronts sharing one chunk of 64 shots
constexpr int kUnrBlock = 64 * kUnrWaves;
constexpr int kUnrRound = 256;               // records are allocated for shots rounded up to this

// Per-variant layout: words per qubit of a state after the messages (Q; Momentum: Q,
// g, M), of the adjoint record after the message adjoints (Q, Pi^{(0)}; Momentum also
// g), and parameters per iteration (alpha_t; Momentum alpha_t, gamma_t).
template <int VAR> struct UnrLayout {
    static_assert(VAR == BP4_EWAINIT || VAR == BP4_MOMENTUM, "unrolled variants: EWAInit, Momentum");
    static constexpr bool kMom = VAR == BP4_MOMENTUM;
    static constexpr int kState = kMom ? 9 : 3;
    static constexpr int kAdj = kMom ? 9 : 6;
    static constexpr int kParams = kMom ? 2 : 1;
};
constexpr int unr_state_words(int variant) { return variant == BP4_MOMENTUM ? 9 : 3; }
constexpr int unr_adj_words(int variant) { return variant == BP4_MOMENTUM ? 9 : 6; }
constexpr int unr_params(int variant) { return variant == BP4_MOMENTUM ? 2 : 1; }

template <typename T> using konst = const __attribute__((address_space(4))) T;
template <typename T> __device__ __forceinline__ konst<T> *as_const(const T *p) { return (konst<T> *)p; }

struct UnrArgs {
    GraphView g;
    const float *param;       // [T][k]: row t-1 at iteration t (EWAInit alpha_t, entry 0 unused;
                              // Momentum alpha_t, gamma_t)
    const float *prior;       // [n][3] Pi^{(0)}
    const uint8_t *synd;      // [shots][m]
    const uint8_t *err;       // [shots][n] Pauli codes of the sampled errors
    float *ckpt;              // [nseg][waves][SI][64] states at t = 0, K, 2K, ... (SI = E + 3N or E + 9N)
    float *seg;               // [K + 1][waves][SI][64] states of one segment
    float *adj;               // [waves][E + 6N or E + 9N][64] adjoints: m (E), Q (3N), Pi^{(0)} (3N),
                              // Momentum g (3N)
    double *partial;          // [waves][nout] per-chunk sums
    float *q_out;             // optional [shots][n][3] Q^{(T)}
    int32_t shots, T, K, nseg, waves, nout;
    float clamp;
};

__device__ __forceinline__ double wave_sum(double x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

// d phi / dx = -1 / sinh(x), x > 0 (series below 1/4, where e^x - e^-x cancels).
__device__ __forceinline__ float dphi(float x)
{
    if (x < 0.25f) {
        const float x2 = x * x;
        return -1.0f / (x * fmaf(x2 * (1.0f / 6.0f), fmaf(x2, 0.05f, 1.0f), 1.0f));
    }
    const float e = hw_exp2(x * kLog2e);
    return -2.0f / (e - 1.0f / e);
}

__device__ __forceinline__ float sigmoid(float x) { return 1.0f / (1.0f + hw_exp2(-x * kLog2e)); }

// Q indices of an edge label H (1 X, 2 Z, 3 Y) and of its anticommuting pair (a, b).
__device__ __forceinline__ void label_indices(uint32_t lab, int &h, int &a, int &b)
{
    h = lab == 1u ? 0 : (lab == 2u ? 2 : 1);
    a = lab == 2u ? 0 : (lab == 1u ? 1 : 0);
    b = lab == 2u ? 1 : 2;
}

// Soft loss of one qubit and its derivative with respect to (Q_X, Q_Y, Q_Z).
__device__ __forceinline__ float qubit_loss(const float q[3], uint32_t e, float dq[3])
{
    float mx = 0.0f;
#pragma unroll
    for (int x = 0; x < 3; ++x) mx = fmaxf(mx, -q[x]);
    float ex[3];
    float s = expf(-mx);
#pragma unroll
    for (int x = 0; x < 3; ++x) {
        ex[x] = expf(-q[x] - mx);
        s += ex[x];
    }
    const int ei = e == 1u ? 0 : (e == 3u ? 1 : (e == 2u ? 2 : -1));
#pragma unroll
    for (int x = 0; x < 3; ++x) dq[x] = (x == ei ? 1.0f : 0.0f) - ex[x] / s;
    return mx + logf(s) + (ei >= 0 ? q[ei] : 0.0f);
}

struct Lane {
    size_t wave;  // chunk of 64 shots (the workgroup)
    int lane;     // column of the shot in the chunk
    int part;     // wavefront of the workgroup: nodes part, part + kUnrWaves, ...
    bool have;    // the column holds a shot
    size_t SI;    // items of one state
    __device__ float *state(float *base, int slot, int waves) const
    {
        return base + ((size_t)slot * waves + wave) * SI * 64 + lane;
    }
};

template <int VAR>
__device__ __forceinline__ Lane lane_of(const UnrArgs &a)
{
    Lane L;
    L.wave = blockIdx.x;
    L.lane = threadIdx.x & 63;
    // read from lane 0: uniform across the wavefront, so the node loops and every graph
    // and prior read indexed by them stay scalar
    L.part = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    L.have = (int64_t)L.wave * 64 + L.lane < a.shots;
    L.SI = (size_t)a.g.nnz + UnrLayout<VAR>::kState * (size_t)a.g.n;
    return L;
}

// Copy of a column's first `items` words, split over the workgroup's wavefronts.
__device__ void copy_column(const Lane &L, float *dst, const float *src, size_t items)
{
    if (L.have)
        for (size_t i = L.part; i < items; i += kUnrWaves) dst[i * 64] = src[i * 64];
}

// Sum over the workgroup of one double per wavefront, in wavefront order; the
// result is valid in thread 0 only.  sh: kUnrWaves doubles of LDS.
__device__ double block_sum(double x, double *sh)
{
    x = wave_sum(x);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = x;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < kUnrWaves; ++w) t += sh[w];
    __syncthreads();
    return t;
}

// m^{(0)}_{v->c} = lambda(Pi^{(0)}) clamped, Q^{(0)} = Pi^{(0)}  (eq. init), Momentum
// g^{(0)} = 0 (and M, unused at t = 0, = 0), written to st and ck.
template <int VAR>
__device__ void init_state(const UnrArgs &a, const Lane &L, float *st, float *ck)
{
    if (!L.have) return;
    konst<uint32_t> *vinfo = as_const(a.g.vinfo);
    konst<float> *prior = as_const(a.prior);
    const int E = a.g.nnz;
    for (int v = L.part; v < a.g.n; v += kUnrWaves) {
        const uint32_t info = vinfo[v];
        const uint32_t base = var_base(info), deg = var_deg(info);
        const float p3[3] = {prior[3 * v], prior[3 * v + 1], prior[3 * v + 2]};
        float lam[4];
        qubit_lambdas(p3, var_labels_present(info), lam);
        for (uint32_t j = 0; j < deg; ++j) {
            const float mj = clampf(lam[var_lab(info, j)], a.clamp);
            st[(size_t)(base + j) * 64] = mj;
            ck[(size_t)(base + j) * 64] = mj;
        }
        for (int x = 0; x < 3; ++x) {
            st[(size_t)(E + 3 * v + x) * 64] = p3[x];
            ck[(size_t)(E + 3 * v + x) * 64] = p3[x];
            if constexpr (UnrLayout<VAR>::kMom) {
                const int n = a.g.n;
                for (int w = 1; w <= 2; ++w) {
                    st[(size_t)(E + 3 * w * n + 3 * v + x) * 64] = 0.0f;
                    ck[(size_t)(E + 3 * w * n + 3 * v + x) * 64] = 0.0f;
                }
            }
        }
    }
}

// One forward iteration t: reads the state of t-1 from `src`, writes that of t to
// `dst` (src == dst: in place).  The check pass writes m_{c->v} into dst's message
// items; the qubit pass turns them into m_{v->c}^{(t)} (skipped at t = T).  Each
// message and posterior item belongs to one check and one qubit, so the passes
// need only the workgroup barrier between them and the one at the end.  Called by
// every thread of the workgroup.
template <int VAR>
__device__ void forward_iteration(const UnrArgs &a, const Lane &L, int t, const float *src, float *dst, int shot)
{
    konst<uint32_t> *cedge = as_const(a.g.cedge);
    konst<uint32_t> *vinfo = as_const(a.g.vinfo);
    konst<float> *prior = as_const(a.prior);
    const int m = a.g.m, n = a.g.n, E = a.g.nnz;
    const float C = a.clamp;
    const uint8_t *s = a.synd + (size_t)shot * m;
    if (L.have) {
        for (int c = L.part; c < m; c += kUnrWaves) {
            uint32_t w[4];
            float mv[4], out[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                w[j] = cedge[kMaxCheckDeg * c + j];
                mv[j] = edge_is_pad(w[j]) ? INFINITY : src[(size_t)edge_slot(w[j]) * 64];
            }
            check_update(mv, s[c] & 1u, C, out);
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (!edge_is_pad(w[j])) dst[(size_t)edge_slot(w[j]) * 64] = out[j];
        }
    }
    __syncthreads();
    constexpr bool kMom = UnrLayout<VAR>::kMom;
    VariantParams vp;
    vp.variant = VAR;
    vp.g_from_t1 = 0;
    vp.alpha = a.param[UnrLayout<VAR>::kParams * (t - 1)];
    vp.gamma = kMom ? a.param[2 * (t - 1) + 1] : 0.0f;
    vp.eps = 0.0f;
    if (L.have) {
        for (int v = L.part; v < n; v += kUnrWaves) {
            const uint32_t info = vinfo[v];
            const uint32_t base = var_base(info), deg = var_deg(info);
            float mc[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) mc[j] = (uint32_t)j < deg ? dst[(size_t)(base + j) * 64] : 0.0f;
            float S[4], A[4];
            label_sums(info, mc, true, false, S, A);
            const float p3[3] = {prior[3 * v], prior[3 * v + 1], prior[3 * v + 2]};
            float st[3], ac[3] = {0.0f, 0.0f, 0.0f}, qn[3];
            for (int x = 0; x < 3; ++x) st[x] = src[(size_t)(E + 3 * v + x) * 64];
            if constexpr (kMom)
                for (int x = 0; x < 3; ++x) ac[x] = src[(size_t)(E + 3 * n + 3 * v + x) * 64];
            qubit_posterior(vp, t, p3, S, A, st, ac, qn);
            for (int x = 0; x < 3; ++x) dst[(size_t)(E + 3 * v + x) * 64] = qn[x];
            if constexpr (kMom) {
                // g^{(t)} and the sums M^{(t)} the posterior rule used (for the adjoint)
                float M[3];
                {
#pragma clang fp contract(off)
                    M[0] = S[3] + S[2];
                    M[1] = S[1] + S[2];
                    M[2] = S[1] + S[3];
                }
                for (int x = 0; x < 3; ++x) {
                    dst[(size_t)(E + 3 * n + 3 * v + x) * 64] = ac[x];
                    dst[(size_t)(E + 6 * n + 3 * v + x) * 64] = M[x];
                }
            }
            if (t < a.T) {
                float lam[4];
                qubit_lambdas(qn, var_labels_present(info), lam);
                for (uint32_t j = 0; j < deg; ++j)
                    dst[(size_t)(base + j) * 64] = clampf(lam[var_lab(info, j)] - mc[j], C);
            }
        }
    }
    __syncthreads();
}

template <int VAR>
__global__ void __launch_bounds__(kUnrBlock) unrolled_forward_kernel(UnrArgs a)
{
    __shared__ double sh[kUnrWaves];
    const Lane L = lane_of<VAR>(a);
    if ((int)L.wave >= a.waves) return;   // the whole workgroup: no such chunk
    const int col = (int)L.wave * 64 + L.lane;
    const int n = a.g.n, E = a.g.nnz;
    float *work = L.state(a.seg, 0, a.waves);
    init_state<VAR>(a, L, work, L.state(a.ckpt, 0, a.waves));
    __syncthreads();
    for (int t = 1; t <= a.T; ++t) {
        forward_iteration<VAR>(a, L, t, work, work, col);
        if (t % a.K == 0 && t < a.T) {
            copy_column(L, L.state(a.ckpt, t / a.K, a.waves), work, L.SI);
            __syncthreads();              // the next check pass rewrites work in place
        }
    }
    double loss = 0.0;
    if (L.have) {
        const uint8_t *e = a.err + (size_t)col * n;
        for (int v = L.part; v < n; v += kUnrWaves) {
            float q[3], dq[3];
            for (int x = 0; x < 3; ++x) q[x] = work[(size_t)(E + 3 * v + x) * 64];
            loss += (double)qubit_loss(q, e[v] & 3u, dq);
            if (a.q_out)
                for (int x = 0; x < 3; ++x) a.q_out[((size_t)col * n + v) * 3 + x] = q[x];
        }
    }
    loss = block_sum(loss, sh);
    if (threadIdx.x == 0) a.partial[L.wave * a.nout] = loss;
}

// Reverse sweep of iteration t.  cur: state t, prev: state t-1.  On entry the
// adjoint holds dL/dm_{v->c}^{(t)} (gm) and dL/dQ^{(t)} (gQ, only the loss term
// at t = T), for Momentum also dL/dg^{(t)} through iteration t+1 (gG); on exit
// those of iteration t-1.  Every message and posterior adjoint belongs to one
// qubit and one check, so the qubit side and the check side need only the
// workgroup barrier between them and the one at the end.  Called by every thread
// of the workgroup; tot gets the workgroup's dL/dalpha_t (and Momentum's
// dL/dgamma_t) in thread 0.
template <int VAR>
__device__ void reverse_iteration(const UnrArgs &a, const Lane &L, int t, const float *cur, const float *prev,
                                  float *adj, int shot, double *sh, double tot[2])
{
    constexpr bool kMom = UnrLayout<VAR>::kMom;
    konst<uint32_t> *cedge = as_const(a.g.cedge);
    konst<uint32_t> *vinfo = as_const(a.g.vinfo);
    konst<float> *prior = as_const(a.prior);
    const int m = a.g.m, n = a.g.n, E = a.g.nnz;
    const float C = a.clamp;
    float *gm = adj;
    float *gQ = adj + (size_t)E * 64;
    float *gP = adj + (size_t)(E + 3 * n) * 64;
    float *gG = adj + (size_t)(E + 6 * n) * 64;   // Momentum
    const float al = a.param[UnrLayout<VAR>::kParams * (t - 1)];
    const float ga = kMom ? a.param[2 * (t - 1) + 1] : 0.0f;
    float galpha = 0.0f, ggamma = 0.0f;
    // ---- qubit side: vertical update (t < T), then posterior and EWA prior ------
    if (L.have) {
        for (int v = L.part; v < n; v += kUnrWaves) {
            const uint32_t info = vinfo[v];
            const uint32_t base = var_base(info), deg = var_deg(info);
            float q[3], g[3];
            for (int x = 0; x < 3; ++x) {
                q[x] = cur[(size_t)(E + 3 * v + x) * 64];
                g[x] = gQ[(size_t)(3 * v + x) * 64];
            }
            float gcv[4] = {0.0f, 0.0f, 0.0f, 0.0f};
            if (t < a.T) {
                // m_{v->c} = clamp(lambda_H(Q) - m_{c->v}): lambda's partials, zero where clamped
                for (uint32_t j = 0; j < deg; ++j) {
                    const size_t sl = (size_t)(base + j) * 64;
                    const float gj = gm[sl];
                    if (!(fabsf(cur[sl]) < C)) continue;
                    int h, ia, ib;
                    label_indices(var_lab(info, j), h, ia, ib);
                    g[h] -= gj * sigmoid(-q[h]);
                    g[ia] += gj * sigmoid(q[ib] - q[ia]);
                    g[ib] += gj * sigmoid(q[ia] - q[ib]);
                    gcv[j] = -gj;
                }
            }
            if constexpr (!kMom) {
                // Q = Pi^{(t)} + M: each m_{c->v} enters the two components that anticommute with H
                for (uint32_t j = 0; j < deg; ++j) {
                    int h, ia, ib;
                    label_indices(var_lab(info, j), h, ia, ib);
                    gm[(size_t)(base + j) * 64] = gcv[j] + g[ia] + g[ib];
                }
                // Pi^{(t)} = alpha_t Pi^{(0)} + (1 - alpha_t) Q^{(t-1)}  (t > 1), Pi^{(1)} = Pi^{(0)}
                for (int x = 0; x < 3; ++x) {
                    const size_t i = (size_t)(3 * v + x) * 64;
                    if (t == 1) {
                        gP[i] += g[x];
                        gQ[i] = 0.0f;
                    } else {
                        const float p0 = prior[3 * v + x];
                        galpha = fmaf(g[x], p0 - prev[(size_t)(E + 3 * v + x) * 64], galpha);
                        gP[i] = fmaf(al, g[x], gP[i]);
                        gQ[i] = (1.0f - al) * g[x];
                    }
                }
            } else {
                // Q^{(t)} = Q^{(t-1)} - alpha_t g^{(t)},
                // g^{(t)} = gamma_t g^{(t-1)} + (1 - gamma_t) d, d = Q^{(t-1)} - Pi^{(0)} - M^{(t)}
                float gM[3];
                for (int x = 0; x < 3; ++x) {
                    const size_t i = (size_t)(3 * v + x) * 64;
                    const float gt = cur[(size_t)(E + 3 * n + 3 * v + x) * 64];
                    const float gprev = prev[(size_t)(E + 3 * n + 3 * v + x) * 64];
                    const float d = (prev[(size_t)(E + 3 * v + x) * 64] - prior[3 * v + x]) -
                                    cur[(size_t)(E + 6 * n + 3 * v + x) * 64];
                    const float ggt = fmaf(-al, g[x], gG[i]);   // dL/dg^{(t)}, all paths
                    galpha = fmaf(-gt, g[x], galpha);
                    ggamma = fmaf(gprev - d, ggt, ggamma);
                    const float gd = (1.0f - ga) * ggt;
                    gM[x] = -gd;
                    gG[i] = ga * ggt;                          // dL/dg^{(t-1)}
                    const float gq = g[x] + gd;                // dL/dQ^{(t-1)}
                    gP[i] -= gd;
                    if (t == 1) {                              // Q^{(0)} = Pi^{(0)}
                        gP[i] += gq;
                        gQ[i] = 0.0f;
                    } else {
                        gQ[i] = gq;
                    }
                }
                // each m_{c->v} enters the two components of M that anticommute with H
                for (uint32_t j = 0; j < deg; ++j) {
                    int h, ia, ib;
                    label_indices(var_lab(info, j), h, ia, ib);
                    gm[(size_t)(base + j) * 64] = gcv[j] + gM[ia] + gM[ib];
                }
            }
        }
    }
    tot[0] = block_sum((double)galpha, sh);   // also the barrier between the sides
    if constexpr (kMom) tot[1] = block_sum((double)ggamma, sh);
    // ---- check side: m_{c->v} = clamp(sign * phi(sum_{v' != v} phi(|m_{v'->c}|))) ----
    const uint8_t *s = a.synd + (size_t)shot * m;
    if (L.have) {
        for (int c = L.part; c < m; c += kUnrWaves) {
            uint32_t w[4];
            float mv[4], f[4], gout[4];
            uint32_t sgn[4];
            uint32_t neg = s[c] & 1u;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                w[j] = cedge[kMaxCheckDeg * c + j];
                const bool pad = edge_is_pad(w[j]);
                const size_t sl = (size_t)edge_slot(w[j]) * 64;
                mv[j] = pad ? INFINITY : prev[sl];
                gout[j] = pad ? 0.0f : gm[sl];
                sgn[j] = mv[j] < 0.0f ? 1u : 0u;
                neg ^= sgn[j];
                f[j] = phi(fabsf(mv[j]));
            }
            float loo[4];
            loo4(f, loo);   // the forward check rule's sums, bit for bit
            float wsum[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float mag = phi(loo[j]);
                const float sj = (neg ^ sgn[j]) ? -1.0f : 1.0f;
                // the clamp passes the derivative only where it did not act
                wsum[j] = (mag < C && gout[j] != 0.0f) ? gout[j] * sj * dphi(loo[j]) : 0.0f;
            }
            // leave-one-out sums formed directly: one term can exceed the others by many
            // orders of magnitude (an output whose other inputs are all saturated), and
            // subtracting it from the total would cancel the rest
            const float others4[4] = {wsum[1] + wsum[2] + wsum[3], wsum[0] + wsum[2] + wsum[3],
                                      wsum[0] + wsum[1] + wsum[3], wsum[0] + wsum[1] + wsum[2]};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (edge_is_pad(w[k])) continue;
                const float others = others4[k];
                // a zero message has phi = inf: its outputs do not depend on it
                const float gk = isinf(f[k]) ? 0.0f : (sgn[k] ? -1.0f : 1.0f) * dphi(fabsf(mv[k])) * others;
                gm[(size_t)edge_slot(w[k]) * 64] = gk;
            }
        }
    }
    __syncthreads();
}

// Adjoint, part 1 for segment sg: recompute the segment's states from its
// checkpoint; for the last segment first clear the adjoint record and seed it
// with dL/dQ^{(T)} of the soft loss (unscaled: the mean's 1/(shots n) comes last).
template <int VAR>
__global__ void __launch_bounds__(kUnrBlock) unrolled_recompute_kernel(UnrArgs a, int sg)
{
    constexpr int kAdj = UnrLayout<VAR>::kAdj;
    const Lane L = lane_of<VAR>(a);
    if ((int)L.wave >= a.waves) return;   // the whole workgroup: no such chunk
    const int col = (int)L.wave * 64 + L.lane;
    const int n = a.g.n, E = a.g.nnz;
    const int t0 = sg * a.K;
    const int t1 = t0 + a.K < a.T ? t0 + a.K : a.T;
    float *adj = a.adj + L.wave * ((size_t)E + kAdj * (size_t)n) * 64 + L.lane;
    copy_column(L, L.state(a.seg, 0, a.waves), L.state(a.ckpt, sg, a.waves), L.SI);
    __syncthreads();
    for (int t = t0 + 1; t <= t1; ++t)
        forward_iteration<VAR>(a, L, t, L.state(a.seg, t - 1 - t0, a.waves), L.state(a.seg, t - t0, a.waves),
                               col);
    if (t1 != a.T) return;
    if (L.have)
        for (size_t i = L.part; i < (size_t)E + kAdj * (size_t)n; i += kUnrWaves) adj[i * 64] = 0.0f;
    __syncthreads();                      // other wavefronts cleared some of the items written below
    if (!L.have) return;
    const float *sT = L.state(a.seg, t1 - t0, a.waves);
    const uint8_t *e = a.err + (size_t)col * n;
    for (int v = L.part; v < n; v += kUnrWaves) {
        float q[3], dq[3];
        for (int x = 0; x < 3; ++x) q[x] = sT[(size_t)(E + 3 * v + x) * 64];
        qubit_loss(q, e[v] & 3u, dq);
        for (int x = 0; x < 3; ++x) adj[(size_t)(E + 3 * v + x) * 64] = dq[x];
    }
}

// Adjoint, part 2 for segment sg: the reverse sweep t = t1 ... t0+1 over the
// recomputed states, then (sg = 0) the initial messages' contribution.  Held to
// 64 VGPRs (8 wavefronts per SIMD): the few values that spill cost less than the
// latency hidden by the extra wavefronts (96 VGPRs without spills: 5 per SIMD,
// 17% slower).
template <int VAR>
__global__ void __launch_bounds__(kUnrBlock) __attribute__((amdgpu_waves_per_eu(8, 8)))
unrolled_reverse_kernel(UnrArgs a, int sg)
{
    constexpr int kAdj = UnrLayout<VAR>::kAdj, kP = UnrLayout<VAR>::kParams;
    __shared__ double sh[kUnrWaves];
    const Lane L = lane_of<VAR>(a);
    if ((int)L.wave >= a.waves) return;   // the whole workgroup: no such chunk
    const int col = (int)L.wave * 64 + L.lane;
    const int n = a.g.n, E = a.g.nnz;
    const int t0 = sg * a.K;
    const int t1 = t0 + a.K < a.T ? t0 + a.K : a.T;
    float *adj = a.adj + L.wave * ((size_t)E + kAdj * (size_t)n) * 64 + L.lane;
    double *part = a.partial + L.wave * a.nout;
    for (int t = t1; t > t0; --t) {
        double tot[2] = {0.0, 0.0};
        reverse_iteration<VAR>(a, L, t, L.state(a.seg, t - t0, a.waves), L.state(a.seg, t - 1 - t0, a.waves), adj,
                               col, sh, tot);
        if (threadIdx.x == 0) {
            if constexpr (kP == 2) {
                part[2 * (t - 1)] = tot[0];
                part[2 * (t - 1) + 1] = tot[1];
            } else {
                part[t - 1] = t == 1 ? 0.0 : tot[0];   // alpha_1 is unused
            }
        }
    }
    if (sg != 0) return;
    // ---- initialisation: m^{(0)}_{v->c} = clamp(lambda_H(Pi^{(0)})) ----------------
    // qubit v is one wavefront's, so its sums run over that wavefront's 64 columns
    konst<uint32_t> *vinfo = as_const(a.g.vinfo);
    konst<float> *prior = as_const(a.prior);
    float *gm = adj;
    float *gP = adj + (size_t)(E + 3 * n) * 64;
    for (int v = L.part; v < n; v += kUnrWaves) {
        float g[3] = {0.0f, 0.0f, 0.0f};
        if (L.have) {
            const uint32_t info = vinfo[v];
            const uint32_t base = var_base(info), deg = var_deg(info);
            const float p3[3] = {prior[3 * v], prior[3 * v + 1], prior[3 * v + 2]};
            float lam[4];
            qubit_lambdas(p3, var_labels_present(info), lam);
            for (int x = 0; x < 3; ++x) g[x] = gP[(size_t)(3 * v + x) * 64];
            for (uint32_t j = 0; j < deg; ++j) {
                const uint32_t lab = var_lab(info, j);
                if (!(fabsf(lam[lab]) < a.clamp)) continue;
                const float gj = gm[(size_t)(base + j) * 64];
                int h, ia, ib;
                label_indices(lab, h, ia, ib);
                g[h] -= gj * sigmoid(-p3[h]);
                g[ia] += gj * sigmoid(p3[ib] - p3[ia]);
                g[ib] += gj * sigmoid(p3[ia] - p3[ib]);
            }
        }
        for (int x = 0; x < 3; ++x) {
            const double tot = wave_sum((double)g[x]);
            if (L.lane == 0) part[kP * a.T + 3 * v + x] = tot;
        }
    }
}

// out[i] = scale * (*dloss) * sum over wavefronts of partial[w][i], in wavefront order.
// The loads of 16 partials are issued before their additions (a few hundred threads
// walk thousands of partials each; one load in flight per thread left the kernel
// waiting on memory); the additions keep the wavefront order.
__global__ void __launch_bounds__(256) unrolled_reduce_kernel(const double *partial, int waves, int nout, double scale,
                                                            const float *dloss, double *out0, int n0, double *out1)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nout) return;
    constexpr int kBatch = 16;
    double s = 0.0;
    int w = 0;
    for (; w + kBatch <= waves; w += kBatch) {
        double v[kBatch];
#pragma unroll
        for (int k = 0; k < kBatch; ++k) v[k] = partial[(size_t)(w + k) * nout + i];
#pragma unroll
        for (int k = 0; k < kBatch; ++k) s += v[k];
    }
    for (; w < waves; ++w) s += partial[(size_t)w * nout + i];
    s *= scale * (dloss ? (double)*dloss : 1.0);
    if (i < n0) out0[i] = s;
    else out1[i - n0] = s;
}

}  // namespace

static size_t up256u(size_t x) { return (x + 255) & ~size_t(255); }

UnrolledSizes unrolled_sizes(int m, int n, int nnz, int variant, int32_t T, int32_t K, int64_t shots)
{
    (void)m;
    UnrolledSizes z;
    const size_t lanes = (size_t)((shots + kUnrRound - 1) / kUnrRound) * kUnrRound;
    const size_t waves = lanes / 64;
    const size_t SI = (size_t)nnz + unr_state_words(variant) * (size_t)n;
    const size_t nseg = (size_t)((T + K - 1) / K);
    z.saved = up256u(nseg * waves * SI * 64 * 4);
    z.ws = up256u((size_t)(K + 1) * waves * SI * 64 * 4) +
           up256u(waves * ((size_t)nnz + unr_adj_words(variant) * (size_t)n) * 64 * 4) +
           up256u(waves * (size_t)(unr_params(variant) * T + 3 * n) * 8);
    return z;
}

static UnrArgs unrolled_args(const GraphView &g, int variant, int32_t T, int32_t K, float clamp, int32_t shots,
                             const float *param, const float *prior, const uint8_t *synd, const uint8_t *err,
                             void *saved, void *ws, int nout)
{
    UnrArgs a;
    a.g = g;
    a.param = param;
    a.prior = prior;
    a.synd = synd;
    a.err = err;
    a.shots = shots;
    a.T = T;
    a.K = K;
    a.nseg = (T + K - 1) / K;
    a.nout = nout;
    a.clamp = clamp;
    a.q_out = nullptr;
    const size_t lanes = (size_t)((shots + kUnrRound - 1) / kUnrRound) * kUnrRound;
    const size_t waves_alloc = lanes / 64;
    const size_t SI = (size_t)g.nnz + unr_state_words(variant) * (size_t)g.n;
    a.ckpt = static_cast<float *>(saved);
    char *w = static_cast<char *>(ws);
    a.seg = reinterpret_cast<float *>(w);
    w += up256u((size_t)(K + 1) * waves_alloc * SI * 64 * 4);
    a.adj = reinterpret_cast<float *>(w);
    w += up256u(waves_alloc * ((size_t)g.nnz + unr_adj_words(variant) * (size_t)g.n) * 64 * 4);
    a.partial = reinterpret_cast<double *>(w);
    // every allocated chunk runs (those past the last shot contribute zeros)
    a.waves = (int)waves_alloc;
    return a;
}

hipError_t launch_unrolled_forward(const GraphView &g, int variant, int32_t T, int32_t K, float clamp, int32_t shots,
                                   const float *param, const float *prior, const uint8_t *synd, const uint8_t *err,
                                   double *loss, float *q_out, void *saved, void *ws, hipStream_t s)
{
    UnrArgs a = unrolled_args(g, variant, T, K, clamp, shots, param, prior, synd, err, saved, ws, 1);
    a.q_out = q_out;
    if (variant == BP4_MOMENTUM)
        hipLaunchKernelGGL(unrolled_forward_kernel<BP4_MOMENTUM>, dim3((unsigned)a.waves), dim3(kUnrBlock), 0, s, a);
    else
        hipLaunchKernelGGL(unrolled_forward_kernel<BP4_EWAINIT>, dim3((unsigned)a.waves), dim3(kUnrBlock), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const double scale = 1.0 / ((double)shots * (double)g.n);
    hipLaunchKernelGGL(unrolled_reduce_kernel, dim3(1), dim3(256), 0, s, a.partial, a.waves, 1, scale,
                       (const float *)nullptr, loss, 1, (double *)nullptr);
    return hipGetLastError();
}

hipError_t launch_unrolled_backward(const GraphView &g, int variant, int32_t T, int32_t K, float clamp, int32_t shots,
                                    const float *param, const float *prior, const uint8_t *synd, const uint8_t *err,
                                    const float *dloss, const void *saved, double *dparam, double *dprior, void *ws,
                                    hipStream_t s)
{
    const int np = unr_params(variant) * T;
    const int nout = np + 3 * g.n;
    UnrArgs a = unrolled_args(g, variant, T, K, clamp, shots, param, prior, synd, err, const_cast<void *>(saved), ws,
                              nout);
    const dim3 grid((unsigned)a.waves), block(kUnrBlock);
    for (int sg = a.nseg - 1; sg >= 0; --sg) {
        if (variant == BP4_MOMENTUM) {
            hipLaunchKernelGGL(unrolled_recompute_kernel<BP4_MOMENTUM>, grid, block, 0, s, a, sg);
            hipLaunchKernelGGL(unrolled_reverse_kernel<BP4_MOMENTUM>, grid, block, 0, s, a, sg);
        } else {
            hipLaunchKernelGGL(unrolled_recompute_kernel<BP4_EWAINIT>, grid, block, 0, s, a, sg);
            hipLaunchKernelGGL(unrolled_reverse_kernel<BP4_EWAINIT>, grid, block, 0, s, a, sg);
        }
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const double scale = 1.0 / ((double)shots * (double)g.n);
    hipLaunchKernelGGL(unrolled_reduce_kernel, dim3((nout + 255) / 256), dim3(256), 0, s, a.partial, a.waves, nout,
                       scale, dloss, dparam, np, dprior);
    return hipGetLastError();
}

}  // namespace bp4
