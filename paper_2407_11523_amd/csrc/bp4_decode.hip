// Flooding-schedule LLR belief propagation over GF(4) for gfx950: the persistent
// LDS-resident kernel for small and medium codes, decoding one or many codes in
// a single launch.  A group of G lanes decodes one shot at a time (G <= 64:
// groups inside one wavefront; G = 128 or 256: groups spanning wavefronts of a
// 256-lane workgroup).  The shot's messages, posteriors and accumulators live in
// LDS; a code's Tanner graph and priors are staged once per workgroup in LDS and
// shared by all of its groups.  Groups pull shots from the code's queue and
// refill as soon as their shot stops, so the heavy tail of iteration counts
// never idles a wavefront; a workgroup moves on to the next code (in the order
// given, largest first) once the current code's queue is empty.
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

#include "bp4_math.h"

namespace bp4 {

namespace {

constexpr int kBlock = 256;

// MW: groups of 128 or 256 lanes spanning wavefronts (workgroup barriers);
// otherwise G in {4, ..., 64} lanes inside one wavefront (wavefront-level sync).
// VAR: the code's variant as a compile-time constant, so the qubit update keeps only
// its own branch.
template <bool MW, int VAR>
__device__ __forceinline__ void run_code(const DecodeArgs &a, float *lds, int *bcast, int *badflag)
{
    const int G = a.group_lanes;
    const int lgG = __builtin_ctz((unsigned)G);
    const int m = a.g.m, n = a.g.n;
    const uint32_t *s_ce = reinterpret_cast<const uint32_t *>(lds);
    const uint32_t *s_vi = s_ce + kMaxCheckDeg * m;
    const float *s_pi = reinterpret_cast<const float *>(s_vi + n);

    const int gid = (int)threadIdx.x >> lgG;                // group within the workgroup
    const int r = (int)threadIdx.x & (G - 1);               // rank within the group
    const int lead = MW ? 0 : (((int)threadIdx.x & 63) >> lgG) << lgG;   // leader lane in the wavefront
    float *msg = lds + a.static_words + gid * a.region_words;
    float *qs = msg + a.q_off;      // [n][3] Q^{(t-1)} (AdaGrad: D = Q - Pi^{(0)})
    float *acc = msg + a.acc_off;   // [n][3] momentum g or AdaGrad G
    uint8_t *ehat = reinterpret_cast<uint8_t *>(msg + a.ehat_off);

    const float C = a.clamp;
    constexpr int variant = VAR;
    const bool keep_q = variant != BP4_BP;
    const bool keep_acc = variant == BP4_MOMENTUM || variant == BP4_ADAGRAD;
    const bool with_y = a.with_y != 0;
    VariantParams vp;
    vp.variant = VAR;
    vp.g_from_t1 = a.g_from_t1;
    vp.alpha = a.alpha;
    vp.gamma = a.gamma;
    vp.eps = a.eps;

    auto gsync = [&]() {
        if (MW) __syncthreads();
        else wave_sync();
    };

    uint64_t sbits = 0;
    int t = 0;
    int par = 0;       // flag slot of this iteration (MW)
    int att = 0;       // AEWA: attempt of the current shot
    int t_before = 0;  // AEWA: iterations of the shot's earlier attempts

    // Initialisation (eq. init, Algorithm 2): m^{(0)}_{v->c} = lambda_{H_cv}(Pi^{(0)}_v);
    // Q^{(0)} = Pi^{(0)}; momentum and squared-gradient accumulators start at 0.
    auto init = [&](int s) {
        if (r == 0) msg[a.g.nnz] = INFINITY;   // padding slot
        sbits = 0;
        int k = 0;
        for (int c = r; c < m; c += G, ++k)
            if (a.synd[(size_t)s * m + c]) sbits |= 1ull << k;
        for (int v = r; v < n; v += G) {
            const uint32_t info = s_vi[v];
            const uint32_t base = var_base(info), deg = var_deg(info);
            const float p3[3] = {s_pi[3 * v], s_pi[3 * v + 1], s_pi[3 * v + 2]};
            float lam[4];
            qubit_lambdas(p3, var_labels_present(info), lam);
            for (uint32_t j = 0; j < deg; ++j) msg[base + j] = clampf(lam[var_lab(info, j)], C);
            float st[3], ac[3];
            qubit_state_init(variant, p3, st, ac);
            if (keep_q)
                for (int w = 0; w < 3; ++w) qs[3 * v + w] = st[w];
            if (keep_acc)
                for (int w = 0; w < 3; ++w) acc[3 * v + w] = ac[w];
        }
        t = 0;
    };

    // Shot queue: the group leader takes the next shot index of this code.
    int shot;
    if (MW) {
        if (r == 0) bcast[gid] = take_shot(a.counter, a.shots);
        __syncthreads();
        shot = bcast[gid];
        __syncthreads();
    } else {
        int s0 = 0;
        if (r == 0) s0 = take_shot(a.counter, a.shots);
        shot = __shfl(s0, lead, 64);
    }
    if (shot < a.shots) init(shot);
    gsync();

    for (;;) {
        const bool live = shot < a.shots;
        if (MW ? !__syncthreads_or(live) : !__any(live)) break;
        if (live) {
            ++t;
            // ---- Horizontal update (eq. h_update) ----------------------------------
            for (int c = r; c < m; c += G) {
                const uint4 w4 = *reinterpret_cast<const uint4 *>(&s_ce[kMaxCheckDeg * c]);
                const uint32_t w[4] = {w4.x, w4.y, w4.z, w4.w};
                float mv[4], out[4];
                // padding edges read and rewrite the padding slot, which holds +inf
                // (phi(+inf) = 0 adds nothing to the sums)
#pragma unroll
                for (int j = 0; j < 4; ++j) mv[j] = msg[edge_slot(w[j])];
                check_update(mv, (uint32_t)(sbits >> ((c - r) >> lgG)), C, out);
#pragma unroll
                for (int j = 0; j < 4; ++j) msg[edge_slot(w[j])] = edge_is_pad(w[j]) ? INFINITY : out[j];
            }
        }
        gsync();
        if (live) {
            // ---- Posterior, hard decision and vertical update ------------------------
            for (int v = r; v < n; v += G) {
                const uint32_t info = s_vi[v];
                const uint32_t base = var_base(info), deg = var_deg(info);
                // the words after a qubit's last slot are in the region (another
                // qubit's slots, the padding slot or the posterior array); their
                // values are read and masked to 0
                float mc[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const float x = msg[base + j];
                    mc[j] = (uint32_t)j < deg ? x : 0.0f;
                }
                float S[4], A[4];
                label_sums(info, mc, with_y, keep_acc && variant == BP4_ADAGRAD, S, A);
                const float p3[3] = {s_pi[3 * v], s_pi[3 * v + 1], s_pi[3 * v + 2]};
                float st[3] = {0.0f, 0.0f, 0.0f}, ac[3] = {0.0f, 0.0f, 0.0f}, qn[3];
                if (keep_q)
                    for (int x = 0; x < 3; ++x) st[x] = qs[3 * v + x];
                if (keep_acc)
                    for (int x = 0; x < 3; ++x) ac[x] = acc[3 * v + x];
                qubit_posterior(vp, t, p3, S, A, st, ac, qn);
                if (keep_q)
                    for (int x = 0; x < 3; ++x) qs[3 * v + x] = st[x];
                if (keep_acc)
                    for (int x = 0; x < 3; ++x) acc[3 * v + x] = ac[x];
                ehat[v] = (uint8_t)decision_byte(hard_decision(qn));
                // Vertical update (eqs. v_update / mombp5): m_{v->c} = lambda_H(Q) - m_{c->v}.
                float lam[4];
                qubit_lambdas(qn, var_labels_present(info), lam);
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
        // ---- Syndrome test of the hard decision (Algorithm 2) -----------------------
        uint32_t bad = 0;
        if (live) {
            for (int c = r; c < m; c += G) {
                const uint4 w4 = *reinterpret_cast<const uint4 *>(&s_ce[kMaxCheckDeg * c]);
                const uint32_t w[4] = {w4.x, w4.y, w4.z, w4.w};
                uint32_t par = (uint32_t)(sbits >> ((c - r) >> lgG)) & 1u, any = 0;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    // <H_cv, E^_v> is bit H_cv of the decision byte (padding edges read
                    // bit 0 of qubit 0's byte, which is set only if that shot already
                    // holds a NaN posterior and cannot converge)
                    const uint32_t b = ehat[edge_var(w[j])];
                    par ^= (b >> edge_lab(w[j])) & 1u;
                    any |= b;
                }
                bad |= par | (any & 1u);   // bit 0: a NaN posterior never converges
            }
        }
        bool sat;
        if (MW) {
            // Two flag slots per group, alternating by iteration: slot `par` is set now
            // and read after the barrier; the other slot, last read one iteration ago
            // (behind the barriers since), is cleared for the next iteration.
            if (bad) badflag[par * (kBlock / 128) + gid] = 1;
            __syncthreads();
            sat = badflag[par * (kBlock / 128) + gid] == 0;
            if (r == 0) badflag[(par ^ 1) * (kBlock / 128) + gid] = 0;
            par ^= 1;
        } else {
            const uint64_t ballot = __ballot(bad != 0);
            const uint64_t gmask = (G == 64) ? ~0ull : (((1ull << G) - 1ull) << lead);
            sat = (ballot & gmask) == 0;
        }
        // AEWA: a failed attempt restarts the shot with the next discount
        const bool restart = VAR == BP4_AEWA && live && !sat && t >= a.max_iter && att + 1 < a.alpha_steps;
        const bool fin = live && !restart && ((a.stop && sat) || t >= a.max_iter);
        if (fin) {
            for (int v = r; v < n; v += G) {
                a.est[(size_t)shot * n + v] = (uint8_t)decision_pauli(ehat[v]);
            }
            if (r == 0) {
                a.conv[shot] = sat ? 1 : 0;
                a.iters[shot] = t_before + t;
            }
        }
        if (VAR == BP4_AEWA && (fin || restart)) {
            t_before = restart ? t_before + t : 0;
            att = restart ? att + 1 : 0;
            vp.alpha = aewa_alpha(a.alpha, a.alpha_last, a.alpha_steps, att);
        }
        if (MW) {
            // No barrier is needed before the refill: nothing reads the messages after
            // the flag barrier, and the outputs read only the decisions, which init
            // leaves alone.  The loop-top barrier publishes init's writes.
            if (fin && r == 0) bcast[gid] = take_shot(a.counter, a.shots);
            __syncthreads();
            if (fin) {
                shot = bcast[gid];
                if (shot < a.shots) init(shot);
            } else if (restart) {
                init(shot);
            }
        } else {
            gsync();
            if (fin) {
                int s0 = 0;
                if (r == 0) s0 = take_shot(a.counter, a.shots);
                shot = __shfl(s0, lead, 64);
                if (shot < a.shots) init(shot);
            } else if (restart) {
                init(shot);
            }
            gsync();
        }
    }
    if (MW && r == 0) {   // leave both flag slots clear for the next code
        badflag[gid] = 0;
        badflag[kBlock / 128 + gid] = 0;
    }
}

template <bool MW>
__device__ __forceinline__ void run_any(const DecodeArgs &a, float *lds, int *bcast, int *badflag)
{
    switch (a.variant) {
    case BP4_BP: run_code<MW, BP4_BP>(a, lds, bcast, badflag); break;
    case BP4_MOMENTUM: run_code<MW, BP4_MOMENTUM>(a, lds, bcast, badflag); break;
    case BP4_ADAGRAD: run_code<MW, BP4_ADAGRAD>(a, lds, bcast, badflag); break;
    case BP4_AEWA: run_code<MW, BP4_AEWA>(a, lds, bcast, badflag); break;
    default: run_code<MW, BP4_EWAINIT>(a, lds, bcast, badflag); break;
    }
}

// VSET: the variant every code of the launch uses, or -1 for a launch that mixes
// variants (a switch per code).  At most 96 VGPRs, so five wavefronts fit per SIMD.
template <int VSET>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(5)))
decode_lds_kernel(MixedArgs args)
{
    extern __shared__ float lds[];
    __shared__ int bcast[kBlock / 128];
    __shared__ int badflag[2 * (kBlock / 128)];
    __shared__ int pending;
    if (threadIdx.x < 2 * (kBlock / 128)) badflag[threadIdx.x] = 0;
    for (int ci = 0; ci < args.ncodes; ++ci) {
        const DecodeArgs &a = args.codes[ci];
        // skip a code whose queue is already empty (a stale read only costs a visit)
        if (threadIdx.x == 0) pending = __hip_atomic_load(a.counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < (unsigned)a.shots;
        __syncthreads();
        if (!pending) continue;
        // stage the code's packed check edges, qubit words and priors
        const int m = a.g.m, n = a.g.n;
        uint32_t *s_ce = reinterpret_cast<uint32_t *>(lds);
        uint32_t *s_vi = s_ce + kMaxCheckDeg * m;
        float *s_pi = reinterpret_cast<float *>(s_vi + n);
        for (int i = threadIdx.x; i < kMaxCheckDeg * m; i += kBlock) s_ce[i] = a.g.cedge[i];
        for (int i = threadIdx.x; i < n; i += kBlock) s_vi[i] = a.g.vinfo[i];
        for (int i = threadIdx.x; i < 3 * n; i += kBlock) s_pi[i] = a.prior[i];
        __syncthreads();
        const bool mw = a.group_lanes > 64;
        if (VSET < 0) {
            if (mw) run_any<true>(a, lds, bcast, badflag);
            else run_any<false>(a, lds, bcast, badflag);
        } else {
            constexpr int V = VSET < 0 ? BP4_EWAINIT : VSET;
            if (mw) run_code<true, V>(a, lds, bcast, badflag);
            else run_code<false, V>(a, lds, bcast, badflag);
        }
        __syncthreads();
    }
}

}  // namespace

LdsLayout decode_lds_layout(int m, int n, int nnz, int variant, int G)
{
    LdsLayout L;
    L.static_words = kMaxCheckDeg * m + n + 3 * n;
    if (L.static_words & 3) L.static_words += 4 - (L.static_words & 3);
    int w = nnz + 1;               // message slots and the padding slot
    L.q_off = w;
    if (variant != BP4_BP) w += 3 * n;
    L.acc_off = w;
    if (variant == BP4_MOMENTUM || variant == BP4_ADAGRAD) w += 3 * n;
    L.ehat_off = w;
    w += (n + 3) / 4;
    // the qubit phase reads four words from each qubit's first slot: keep them inside
    if (w < nnz + 4) w = nnz + 4;
    if ((w & 1) == 0) w += 1;   // odd stride: neighbouring groups start on other banks
    L.region_words = w;
    L.group_lanes = G;
    L.block = kBlock;
    L.bytes = (size_t)4 * (L.static_words + (size_t)(kBlock / G) * L.region_words);
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

template <int VSET>
static hipError_t launch_lds_kernel(const MixedArgs &args, size_t lds_bytes, hipStream_t s, int *grid_out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    int cus = 0, per_cu = 0;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, decode_lds_kernel<VSET>, kBlock, lds_bytes);
    if (e != hipSuccess) return e;
    if (per_cu < 1) return hipErrorInvalidConfiguration;
    long groups = 0;
    for (int i = 0; i < args.ncodes; ++i) {
        const long gpb = kBlock / args.codes[i].group_lanes;
        const long need = (args.codes[i].shots + gpb - 1) / gpb;
        groups = need > groups ? need : groups;
    }
    long grid = (long)cus * per_cu;
    if (groups < grid) grid = groups;
    if (grid < 1) grid = 1;
    if (grid_out) *grid_out = (int)grid;
    hipLaunchKernelGGL(decode_lds_kernel<VSET>, dim3((unsigned)grid), dim3(kBlock), lds_bytes, s, args);
    return hipGetLastError();
}

hipError_t launch_decode_lds(const MixedArgs &args, size_t lds_bytes, hipStream_t s, int *grid_out)
{
    int v = args.codes[0].variant;
    for (int i = 1; i < args.ncodes; ++i)
        if (args.codes[i].variant != v) v = -1;
    switch (v) {
    case BP4_BP: return launch_lds_kernel<BP4_BP>(args, lds_bytes, s, grid_out);
    case BP4_MOMENTUM: return launch_lds_kernel<BP4_MOMENTUM>(args, lds_bytes, s, grid_out);
    case BP4_ADAGRAD: return launch_lds_kernel<BP4_ADAGRAD>(args, lds_bytes, s, grid_out);
    case BP4_EWAINIT: return launch_lds_kernel<BP4_EWAINIT>(args, lds_bytes, s, grid_out);
    case BP4_AEWA: return launch_lds_kernel<BP4_AEWA>(args, lds_bytes, s, grid_out);
    default: return launch_lds_kernel<-1>(args, lds_bytes, s, grid_out);
    }
}

}  // namespace bp4
