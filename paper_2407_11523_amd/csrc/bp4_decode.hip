// Flooding-schedule LLR belief propagation over GF(4) for gfx950: the persistent
// LDS-resident kernel for small and medium codes, decoding one or many codes in
// a single launch.  A group of G lanes decodes one shot at a time (G <= 64:
// groups inside one wavefront), or S shots share a 512-lane workgroup (block
// slots).  The shot's messages, posteriors and accumulators live in
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
#include <type_traits>

#include "bp4_math.h"
#include "bp4_wide.h"

namespace bp4 {

namespace {

// Lanes per workgroup: eight wavefronts, so the code's staged graph is shared by
// twice the shots of a 256-lane workgroup at the same LDS per wavefront (three
// workgroups per CU, 24 wavefronts).  Measured on the mixed batch of surface
// codes: 512 lanes 192 ms, 256 lanes 201 ms, 768 lanes 201 ms.
constexpr int kBlock = kLdsBlock;

// ---- Per-node steps shared by the two lane mappings -------------------------------

// W: the graph is wide (checks of up to 8 edges, 8 edge words per check, qubits of
// up to 7 edges with their slot labels in a separate word); else 4 and 4.
template <bool W> struct Width {
    static constexpr int kCheck = W ? kMaxCheckDegWide : kMaxCheckDeg;   // edge words per check
    static constexpr int kSlots = W ? 8 : 4;                            // message words read per qubit
};

// Message layout of the flooding kernels in LDS: slot j of qubit v at word v + j n
// (slot-major, so the lanes of a qubit pass read and write consecutive words), then
// the padding slot at kSlots n, which holds +inf.  The staged check edges carry
// these positions in their slot field.
template <bool W>
__device__ __forceinline__ uint32_t lds_pad_slot(uint32_t n) { return Width<W>::kSlots * n; }

template <bool W>
__device__ __forceinline__ void load_check(const uint32_t *s_ce, int c, uint32_t w[Width<W>::kCheck])
{
#pragma unroll
    for (int q = 0; q < Width<W>::kCheck / 4; ++q) {
        const uint4 w4 = *reinterpret_cast<const uint4 *>(&s_ce[Width<W>::kCheck * c + 4 * q]);
        w[4 * q] = w4.x;
        w[4 * q + 1] = w4.y;
        w[4 * q + 2] = w4.z;
        w[4 * q + 3] = w4.w;
    }
}

// Horizontal update (eq. h_update) of check c from the messages in `msg`; s: its
// syndrome bit.  Padding edges read and rewrite the padding slot, which holds
// +inf (phi(+inf) = 0 adds nothing to the sums).
template <bool W = false>
__device__ __forceinline__ void check_node(const uint32_t *s_ce, float *msg, int c, uint32_t s, float C)
{
    constexpr int D = Width<W>::kCheck;
    uint32_t w[D];
    load_check<W>(s_ce, c, w);
    float mv[D], out[D];
#pragma unroll
    for (int j = 0; j < D; ++j) mv[j] = msg[edge_slot(w[j])];
    if constexpr (W) check_update_wide(mv, s, C, out);
    else check_update(mv, s, C, out);
#pragma unroll
    for (int j = 0; j < D; ++j) msg[edge_slot(w[j])] = edge_is_pad(w[j]) ? INFINITY : out[j];
}

// Syndrome test of check c against the decision bytes (Algorithm 2): nonzero if
// the decision violates the check or some decision on it is NaN.
template <bool W = false>
__device__ __forceinline__ uint32_t test_node(const uint32_t *s_ce, const uint8_t *ehat, int c, uint32_t s)
{
    constexpr int D = Width<W>::kCheck;
    uint32_t w[D];
    load_check<W>(s_ce, c, w);
    uint32_t par = s & 1u, any = 0;
#pragma unroll
    for (int j = 0; j < D; ++j) {
        // <H_cv, E^_v> is bit H_cv of the decision byte (padding edges read bit 0
        // of qubit 0's byte, which is set only if that shot already holds a NaN
        // posterior and cannot converge)
        const uint32_t b = ehat[edge_var(w[j])];
        par ^= (b >> edge_lab(w[j])) & 1u;
        any |= b;
    }
    return par | (any & 1u);   // bit 0: a NaN posterior never converges
}

// Label word of qubit v: the qubit word shifted right by 20 (narrow), the separate
// label word (wide).
template <bool W>
__device__ __forceinline__ uint32_t label_word(const uint32_t *s_vl, uint32_t info, int v)
{
    if constexpr (W) return s_vl[v];
    else return info >> 20;
}

// Two-plus-two layout (graphs with X and Z labels only, at most two of each per
// qubit): the X-labelled edges of qubit v sit at message positions 0 and 1, the
// Z-labelled ones at 2 and 3, each group in slot order; an unused position holds 0.
// Its label sums are two additions and its outputs need no label routing.
// Position of the qubit's slot j (labels of its slots in the qubit word, bits 20 + 2j).
__device__ __forceinline__ uint32_t c22_pos(uint32_t info, uint32_t j)
{
    const uint32_t l = var_lab(info, (int)j);
    uint32_t r = 0;
    for (uint32_t k = 0; k < j; ++k) r += var_lab(info, (int)k) == l ? 1u : 0u;
    return (l == 2u ? 2u : 0u) + r;
}
// The staged qubit word of the two-plus-two layout: bits 20-23 say which of the four
// positions hold an edge.
__device__ __forceinline__ uint32_t c22_info(uint32_t info)
{
    uint32_t nx = 0, nz = 0;
    for (uint32_t k = 0; k < var_deg(info); ++k) {
        const uint32_t l = var_lab(info, (int)k);
        nx += l == 1u ? 1u : 0u;
        nz += l == 2u ? 1u : 0u;
    }
    const uint32_t mask = (nx >= 1u ? 1u : 0u) | (nx >= 2u ? 2u : 0u) | (nz >= 1u ? 4u : 0u) | (nz >= 2u ? 8u : 0u);
    return (info & ~(0xFFu << 20)) | (mask << 20);
}
// 0 or all ones: position p of a staged two-plus-two qubit word holds an edge
__device__ __forceinline__ uint32_t c22_keep(uint32_t info, int p)
{
    return (uint32_t)__builtin_amdgcn_sbfe((int)info, 20 + p, 1);
}

// Initialisation of qubit v (eq. init, Algorithm 2): m^{(0)}_{v->c} =
// lambda_{H_cv}(Pi^{(0)}_v); Q^{(0)} = Pi^{(0)}; accumulators start at 0.
template <int VAR, bool W = false, bool C22 = false>
__device__ __forceinline__ void init_qubit(const uint32_t *s_vi, const uint32_t *s_vl, const float *s_pi, float *msg,
                                           float *qs, float *acc, int v, int n, float C)
{
    constexpr bool keep_q = VAR != BP4_BP;
    constexpr bool keep_acc = VAR == BP4_MOMENTUM || VAR == BP4_ADAGRAD;
    const uint32_t info = s_vi[v];
    const float p3[3] = {s_pi[3 * v], s_pi[3 * v + 1], s_pi[3 * v + 2]};
    float lam[4];
    qubit_lambdas(p3, var_labels_present(info), lam);
    if constexpr (C22) {
#pragma unroll
        for (int p = 0; p < 4; ++p)
            msg[v + p * n] = __uint_as_float(__float_as_uint(clampf(lam[p < 2 ? 1 : 2], C)) & c22_keep(info, p));
    } else {
        const uint32_t labw = label_word<W>(s_vl, info, v);
        const uint32_t deg = var_deg(info);
        for (uint32_t j = 0; j < deg; ++j) msg[v + j * n] = clampf(lam[slot_label(labw, (int)j)], C);
    }
    float st[3], ac[3];
    qubit_state_init(VAR, p3, st, ac);
    if (keep_q)
        for (int w = 0; w < 3; ++w) qs[3 * v + w] = st[w];
    if (keep_acc)
        for (int w = 0; w < 3; ++w) acc[3 * v + w] = ac[w];
}

// Posterior, hard decision and vertical update of qubit v at iteration t (eqs.
// p_update, v_update and the variant's rule) from its incoming messages mc[j]
// (slot order; slots j >= degree carry label 0 and are never used).  The new
// m_{v->c} of the qubit's slot j goes to store(j, value).  `shot` indexes the
// optional verification outputs (none are written for shot >= shots).  WY: the
// code has Y labels (else every edge label is X or Z).
template <int VAR, bool WY, int DV, typename Store>
__device__ __forceinline__ void qubit_update(const DecodeArgs &a, const float *s_pi, uint32_t info, uint32_t labw,
                                             int v, const float mc[DV], float *qs, float *acc, uint8_t *ehat, int t,
                                             const VariantParams &vp, int shot, Store store)
{
    constexpr bool keep_q = VAR != BP4_BP;
    constexpr bool keep_acc = VAR == BP4_MOMENTUM || VAR == BP4_ADAGRAD;
    const float C = a.clamp;
    const int n = a.g.n;
    const uint32_t base = var_base(info), deg = var_deg(info);
    float S[4], A[4];
    label_sums_w<DV>(labw, mc, WY, keep_acc && VAR == BP4_ADAGRAD, S, A);
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
    ehat[v] = (uint8_t)decision_byte_of(qn);
    // Vertical update (eqs. v_update / mombp5): m_{v->c} = lambda_H(Q) - m_{c->v}.
    float lam[4];
    qubit_lambdas(qn, var_labels_present(info) & (WY ? 0xEu : 0x6u), lam);
    const bool trace = a.mvc_out && shot < a.shots;
#pragma unroll
    for (int j = 0; j < DV; ++j) {
        if ((uint32_t)j >= deg) continue;
        const uint32_t l = slot_label(labw, j);   // 1 X, 2 Z, 3 Y
        float lsel = l == 2u ? lam[2] : lam[1];
        if (WY) lsel = l == 3u ? lam[3] : lsel;
        const float out = clampf(lsel - mc[j], C);
        store((uint32_t)j, out);
        if (trace) {
            const size_t o = (size_t)shot * a.g.nnz + a.g.vcanon[base + j];
            a.mvc_out[o] = out;
            a.mcv_out[o] = mc[j];
        }
    }
    if (a.q_out && shot < a.shots)
        for (int x = 0; x < 3; ++x) a.q_out[((size_t)shot * n + v) * 3 + x] = qn[x];
}

// Flooding qubit step: the incoming messages are the slots' m_{c->v}.
template <int VAR, bool WY, bool W = false>
__device__ __forceinline__ void qubit_node(const DecodeArgs &a, const uint32_t *s_vi, const uint32_t *s_vl,
                                           const float *s_pi, float *msg, float *qs, float *acc, uint8_t *ehat,
                                           int v, int t, const VariantParams &vp, int shot)
{
    constexpr int DV = Width<W>::kSlots;
    const uint32_t info = s_vi[v];
    const uint32_t n = (uint32_t)a.g.n;
    // slots j >= degree are read but never used: they carry label 0, which the
    // label sums skip, and no message is written for them
    float mc[DV];
#pragma unroll
    for (int j = 0; j < DV; ++j) mc[j] = msg[v + j * n];
    qubit_update<VAR, WY, DV>(a, s_pi, info, label_word<W>(s_vl, info, v), v, mc, qs, acc, ehat, t, vp, shot,
                              [&](uint32_t j, float out) { msg[v + j * n] = out; });
}

// Flooding qubit step in the two-plus-two layout (X and Z labels only).  Same
// arithmetic as qubit_update (label sums in slot order, the unused position adding
// +0), without the verification outputs.
template <int VAR>
__device__ __forceinline__ void qubit_node_c22(const DecodeArgs &a, const uint32_t *s_vi, const float *s_pi,
                                               float *msg, float *qs, float *acc, uint8_t *ehat, int v, int t,
                                               const VariantParams &vp)
{
    constexpr bool keep_q = VAR != BP4_BP;
    constexpr bool keep_acc = VAR == BP4_MOMENTUM || VAR == BP4_ADAGRAD;
    const uint32_t info = s_vi[v];
    const int n = a.g.n;
    float mc[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) mc[p] = msg[v + p * n];
    float S[4], A[4];
    {
#pragma clang fp contract(off)
        S[0] = A[0] = 0.0f;
        S[1] = mc[0] + mc[1];
        S[2] = mc[2] + mc[3];
        S[3] = 0.0f;
        A[3] = 0.0f;
        if (VAR == BP4_ADAGRAD) {
            A[1] = fabsf(mc[0]) + fabsf(mc[1]);
            A[2] = fabsf(mc[2]) + fabsf(mc[3]);
        } else {
            A[1] = A[2] = 0.0f;
        }
    }
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
    ehat[v] = (uint8_t)decision_byte_of(qn);
    // Vertical update (eqs. v_update / mombp5): m_{v->c} = lambda_H(Q) - m_{c->v}
    float lam[4];
    qubit_lambdas(qn, var_labels_present(info) & 0x6u, lam);
    const float C = a.clamp;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const float out = clampf(lam[p < 2 ? 1 : 2] - mc[p], C);
        msg[v + p * n] = __uint_as_float(__float_as_uint(out) & c22_keep(info, p));
    }
}

template <int VAR>
__device__ __forceinline__ VariantParams variant_params(const DecodeArgs &a)
{
    VariantParams vp;
    vp.variant = VAR;
    vp.g_from_t1 = a.g_from_t1;
    vp.alpha = a.alpha;
    vp.gamma = a.gamma;
    vp.eps = a.eps;
    return vp;
}

// ---- Wave groups: G in {4, ..., 64} lanes of one wavefront per shot -----------------
// Lane r of a group owns checks and qubits r, r + G, ...; the group's syndrome bits
// sit in a register (bit k: check r + kG); groups synchronise at wavefront level.
template <int VAR, bool W = false, bool C22 = false>
__device__ __forceinline__ void run_wave(const DecodeArgs &a, float *lds)
{
    const int G = a.group_lanes;
    const int lgG = __builtin_ctz((unsigned)G);
    const int m = a.g.m, n = a.g.n;
    const uint32_t *s_ce = reinterpret_cast<const uint32_t *>(lds);
    const uint32_t *s_vi = s_ce + Width<W>::kCheck * m;
    const float *s_pi = reinterpret_cast<const float *>(s_vi + n);
    const uint32_t *s_vl = reinterpret_cast<const uint32_t *>(s_pi + 3 * n);   // wide graphs only

    const int gid = (int)threadIdx.x >> lgG;                // group within the workgroup
    const int r = (int)threadIdx.x & (G - 1);               // rank within the group
    const int lead = (((int)threadIdx.x & 63) >> lgG) << lgG;   // leader lane in the wavefront
    float *msg = lds + a.static_words + gid * a.region_words;
    float *qs = msg + a.q_off;      // [n][3] Q^{(t-1)} (AdaGrad: D = Q - Pi^{(0)})
    float *acc = msg + a.acc_off;   // [n][3] momentum g or AdaGrad G
    uint8_t *ehat = reinterpret_cast<uint8_t *>(msg + a.ehat_off);

    const float C = a.clamp;
    const bool with_y = a.with_y != 0;
    VariantParams vp = variant_params<VAR>(a);

    uint64_t sbits = 0;
    int t = 0;
    int att = 0;       // AEWA: attempt of the current shot
    int t_before = 0;  // AEWA: iterations of the shot's earlier attempts

    auto init = [&](int s) {
        if (r == 0) msg[lds_pad_slot<W>(n)] = INFINITY;
        sbits = 0;
        int k = 0;
        for (int c = r; c < m; c += G, ++k)
            if (a.synd[(size_t)s * m + c]) sbits |= 1ull << k;
        for (int v = r; v < n; v += G) init_qubit<VAR, W, C22>(s_vi, s_vl, s_pi, msg, qs, acc, v, n, C);
        t = 0;
    };

    // Shot queue: the group leader takes the next shot index of this code.
    int s0 = 0;
    if (r == 0) s0 = take_shot(a.counter, a.shots);
    int shot = __shfl(s0, lead, 64);
    if (shot < a.shots) init(shot);
    wave_sync();

    for (;;) {
        const bool live = shot < a.shots;
        if (!__any(live)) break;
        if (live) {
            ++t;
            for (int c = r; c < m; c += G) check_node<W>(s_ce, msg, c, (uint32_t)(sbits >> ((c - r) >> lgG)), C);
        }
        wave_sync();
        if (live) {
            if constexpr (C22) {
                for (int v = r; v < n; v += G) qubit_node_c22<VAR>(a, s_vi, s_pi, msg, qs, acc, ehat, v, t, vp);
            } else if (with_y) {
                for (int v = r; v < n; v += G)
                    qubit_node<VAR, true, W>(a, s_vi, s_vl, s_pi, msg, qs, acc, ehat, v, t, vp, shot);
            } else {
                for (int v = r; v < n; v += G)
                    qubit_node<VAR, false, W>(a, s_vi, s_vl, s_pi, msg, qs, acc, ehat, v, t, vp, shot);
            }
        }
        wave_sync();
        uint32_t bad = 0;
        if (live)
            for (int c = r; c < m; c += G) bad |= test_node<W>(s_ce, ehat, c, (uint32_t)(sbits >> ((c - r) >> lgG)));
        const uint64_t ballot = __ballot(bad != 0);
        const uint64_t gmask = (G == 64) ? ~0ull : (((1ull << G) - 1ull) << lead);
        const bool sat = (ballot & gmask) == 0;
        // AEWA: a failed attempt restarts the shot with the next discount
        const bool restart = VAR == BP4_AEWA && live && !sat && t >= a.max_iter && att + 1 < a.alpha_steps;
        const bool fin = live && !restart && ((a.stop && sat) || t >= a.max_iter);
        if (fin) {
            for (int v = r; v < n; v += G) a.est[(size_t)shot * n + v] = (uint8_t)decision_pauli(ehat[v]);
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
        wave_sync();
        if (fin) {
            s0 = 0;
            if (r == 0) s0 = take_shot(a.counter, a.shots);
            shot = __shfl(s0, lead, 64);
            if (shot < a.shots) init(shot);
        } else if (restart) {
            init(shot);
        }
        wave_sync();
    }
}

// ---- Serial schedule (Algorithm 1) on wave groups -----------------------------------
// One sweep visits the qubits level by level (graph image: sord, slev): the
// qubits of a level share no check, so a group's lanes update them together and
// the result is the qubit-by-qubit sweep's, bit for bit.  A qubit's incoming
// m_{c->v} are formed from the current m_{v'->c} of each check's other qubits,
// as phi((f0 + f1) + (f2 + f3)) over the check's four edge positions (this
// qubit's edge and padding contributing 0).  The slots hold f = phi(|m_{v->c}|)
// with the sign of m_{v->c} (the value phi would be applied to when the message
// is read), so a message is passed through phi once, when it is written.
// Static LDS adds the slot -> check table and the level order; the syndrome is
// kept as bytes in the region.
template <int VAR, bool WY, bool W = false>
__device__ __forceinline__ void run_serial(const DecodeArgs &a, float *lds)
{
    constexpr int D = Width<W>::kCheck, DV = Width<W>::kSlots;
    const int G = a.group_lanes;
    const int lgG = __builtin_ctz((unsigned)G);
    const int m = a.g.m, n = a.g.n, nnz = a.g.nnz;
    const uint32_t *s_ce = reinterpret_cast<const uint32_t *>(lds);
    const uint32_t *s_vi = s_ce + D * m;
    const float *s_pi = reinterpret_cast<const float *>(s_vi + n);
    const uint32_t *s_vchk = reinterpret_cast<const uint32_t *>(s_pi + 3 * n);
    const uint32_t *s_ord = s_vchk + nnz;
    const uint32_t *s_lev = s_ord + n;
    const uint32_t *s_vl = s_lev + a.g.nlev + 1;   // wide graphs: slot labels

    const int gid = (int)threadIdx.x >> lgG;
    const int r = (int)threadIdx.x & (G - 1);
    const int lead = (((int)threadIdx.x & 63) >> lgG) << lgG;
    float *fs = lds + a.static_words + gid * a.region_words;   // [nnz] signed phi(|m_{v->c}|)
    float *qs = fs + a.q_off;
    float *acc = fs + a.acc_off;
    uint8_t *ehat = reinterpret_cast<uint8_t *>(fs + a.ehat_off);
    uint8_t *syn = reinterpret_cast<uint8_t *>(fs + a.syn_off);

    const float C = a.clamp;
    VariantParams vp = variant_params<VAR>(a);
    auto store = [&](uint32_t slot, float out) {
        const float f = phi(fabsf(out));
        fs[slot] = out < 0.0f ? -f : f;
    };

    int t = 0, att = 0, t_before = 0;
    auto init = [&](int s) {
        for (int c = r; c < m; c += G) syn[c] = a.synd[(size_t)s * m + c];
        for (int v = r; v < n; v += G) {
            const uint32_t info = s_vi[v];
            const uint32_t base = var_base(info), deg = var_deg(info);
            const float p3[3] = {s_pi[3 * v], s_pi[3 * v + 1], s_pi[3 * v + 2]};
            float lam[4];
            qubit_lambdas(p3, var_labels_present(info), lam);
            const uint32_t labw = label_word<W>(s_vl, info, v);
            for (uint32_t j = 0; j < deg; ++j) store(base + j, clampf(lam[slot_label(labw, (int)j)], C));
            float st[3], ac[3];
            qubit_state_init(VAR, p3, st, ac);
            if (VAR != BP4_BP)
                for (int w = 0; w < 3; ++w) qs[3 * v + w] = st[w];
            if (VAR == BP4_MOMENTUM || VAR == BP4_ADAGRAD)
                for (int w = 0; w < 3; ++w) acc[3 * v + w] = ac[w];
        }
        t = 0;
    };

    // one qubit of the sweep
    auto serial_qubit = [&](int v, int shot) {
        const uint32_t info = s_vi[v];
        const uint32_t base = var_base(info), deg = var_deg(info);
        float mc[DV];
#pragma unroll
        for (int j = 0; j < DV; ++j) mc[j] = 0.0f;
        for (uint32_t j = 0; j < deg; ++j) {
            const uint32_t slot = base + j;
            const uint32_t c = s_vchk[slot];
            uint32_t w[D];
            load_check<W>(s_ce, (int)c, w);
            uint32_t neg = syn[c] & 1u;
            float f[D];
#pragma unroll
            for (int k = 0; k < D; ++k) {
                // padding and this qubit's own edge take no part
                const bool skip = edge_is_pad(w[k]) || edge_slot(w[k]) == slot;
                const float x = skip ? 0.0f : fs[edge_slot(w[k])];
                neg ^= __float_as_uint(x) >> 31;
                f[k] = fabsf(x);
            }
            // the check's positions summed in order, pairwise
            float sum = (f[0] + f[1]) + (f[2] + f[3]);
            if constexpr (W) sum = sum + ((f[4] + f[5]) + (f[6] + f[7]));
            const float mag = phi(sum);
            mc[j] = clampf(neg ? -mag : mag, C);
        }
        qubit_update<VAR, WY, DV>(a, s_pi, info, label_word<W>(s_vl, info, v), v, mc, qs, acc, ehat, t, vp, shot,
                                  [&](uint32_t j, float out) { store(base + j, out); });
    };

    int s0 = 0;
    if (r == 0) s0 = take_shot(a.counter, a.shots);
    int shot = __shfl(s0, lead, 64);
    if (shot < a.shots) init(shot);
    wave_sync();

    for (;;) {
        const bool live = shot < a.shots;
        if (!__any(live)) break;
        if (live) ++t;
        for (int l = 0; l < a.g.nlev; ++l) {
            if (live)
                for (int i = (int)s_lev[l] + r; i < (int)s_lev[l + 1]; i += G) serial_qubit((int)s_ord[i], shot);
            wave_sync();
        }
        uint32_t bad = 0;
        if (live)
            for (int c = r; c < m; c += G) bad |= test_node<W>(s_ce, ehat, c, syn[c]);
        const uint64_t ballot = __ballot(bad != 0);
        const uint64_t gmask = (G == 64) ? ~0ull : (((1ull << G) - 1ull) << lead);
        const bool sat = (ballot & gmask) == 0;
        const bool restart = VAR == BP4_AEWA && live && !sat && t >= a.max_iter && att + 1 < a.alpha_steps;
        const bool fin = live && !restart && ((a.stop && sat) || t >= a.max_iter);
        if (fin) {
            for (int v = r; v < n; v += G) a.est[(size_t)shot * n + v] = (uint8_t)decision_pauli(ehat[v]);
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
        wave_sync();
        if (fin) {
            s0 = 0;
            if (r == 0) s0 = take_shot(a.counter, a.shots);
            shot = __shfl(s0, lead, 64);
            if (shot < a.shots) init(shot);
        } else if (restart) {
            init(shot);
        }
        wave_sync();
    }
}

// ---- Block slots: S shots share the workgroup's 512 lanes ---------------------------
// The workgroup walks the S*m (slot, check) and S*n (slot, qubit) items of its S
// shot slots in passes of 512 lanes, so a code whose m or n is not a multiple of
// the lanes per shot leaves few lanes idle.  Each slot's region holds its
// messages, posteriors, decisions, syndrome bytes and a header; every slot keeps
// its own iteration count, and a slot whose shot stops takes the next shot from
// the queue while the others run on.  The three phases process every slot, also
// one without a shot (once the queue is empty): its region is only read and
// written by its own items, and nothing from it reaches the outputs, so no phase
// waits on a slot's header before loading its data.
constexpr int kHdrShot = 0;     // current shot (>= shots: the slot is empty)
constexpr int kHdrT = 1;        // iterations of the current attempt completed
constexpr int kHdrAtt = 2;      // AEWA attempt
constexpr int kHdrTBefore = 3;  // AEWA: iterations of the earlier attempts
constexpr int kHdrAlpha = 4;    // AEWA: discount of the current attempt (float bits)
constexpr int kHdrDone = 5;     // shot whose decisions are written out this round, or -1
constexpr int kHdrFresh = 6;    // 1: the slot's state is (re)initialised this round
constexpr int kHdrBad = 7;      // two "syndrome unmet" flags, alternating by iteration

// Walk over the items (slot k, index x < d) of one lane: items tid, tid + B, ...
// (B = kBlock) of the flattened S*d list, advanced without integer multiplies:
// B = q d + rem,
// so a step adds rem to x and q slots to the region offset off = k * region_words,
// plus one carry.  The walk ends at off = S * region_words.
struct ItemWalk {
    uint32_t x, off;
};

__device__ __forceinline__ ItemWalk walk_start(uint32_t tid, uint32_t d, uint32_t magic, uint32_t RW)
{
    ItemWalk w;
    const uint32_t k = __umulhi(tid, magic);   // tid / d: exact for tid < 2^9 and d < 2^14
    w.x = tid - k * d;
    w.off = k * RW;
    return w;
}

__device__ __forceinline__ void walk_next(ItemWalk &w, uint32_t d, uint32_t rem, uint32_t qoff, uint32_t RW)
{
    w.x += rem;
    w.off += qoff;
    if (w.x >= d) {
        w.x -= d;
        w.off += RW;
    }
}

template <int VAR, bool W = false, bool C22 = false>
__device__ __forceinline__ void run_block(const DecodeArgs &a, float *lds, int *events)
{
    const uint32_t S = (uint32_t)a.block_shots;
    const int m = a.g.m, n = a.g.n;
    const int tid = (int)threadIdx.x;
    const uint32_t *s_ce = reinterpret_cast<const uint32_t *>(lds);
    const uint32_t *s_vi = s_ce + Width<W>::kCheck * m;
    const float *s_pi = reinterpret_cast<const float *>(s_vi + n);
    const uint32_t *s_vl = reinterpret_cast<const uint32_t *>(s_pi + 3 * n);   // wide graphs only
    float *reg0 = lds + a.static_words;
    const uint32_t RW = (uint32_t)a.region_words;
    auto hdr = [&](uint32_t k) { return reinterpret_cast<int *>(reg0 + k * RW + a.hdr_off); };
    const float C = a.clamp;
    const bool with_y = a.with_y != 0;
    VariantParams vp = variant_params<VAR>(a);
    // item walks over checks (d = m) and qubits (d = n)
    const uint32_t rm = kBlock % m, rn = kBlock % n;
    const uint32_t qoffm = (kBlock / m) * RW, qoffn = (kBlock / n) * RW;
    uint32_t end = S * RW;   // the walks cover the active slots 0 .. events[1] - 1
    const ItemWalk wm0 = walk_start(tid, m, a.magic_m, RW), wn0 = walk_start(tid, n, a.magic_n, RW);
#define BP4_FOR_CHECKS(w) for (ItemWalk w = wm0; w.off < end; walk_next(w, m, rm, qoffm, RW))
#define BP4_FOR_QUBITS(w) for (ItemWalk w = wn0; w.off < end; walk_next(w, n, rn, qoffn, RW))

    bool more = false;
    if (tid == 0) {
        events[0] = 1;
        events[1] = (int)S;
    }
    if (tid < (int)S) {
        int *h = hdr(tid);
        const int s = take_shot(a.counter, a.shots);
        h[kHdrShot] = s;
        h[kHdrT] = 0;
        h[kHdrAtt] = 0;
        h[kHdrTBefore] = 0;
        h[kHdrAlpha] = __float_as_int(a.alpha);
        h[kHdrDone] = -1;
        h[kHdrFresh] = s < a.shots ? 1 : 0;
        h[kHdrBad] = 0;
        h[kHdrBad + 1] = 0;
        more = s < a.shots;
        if (!more) events[3] = 1;
    }
    bool any_more = __syncthreads_or(more);
    int par = 0;
    for (;;) {
        // outputs of the shots that stopped, initialisation of fresh slots (only in
        // rounds where some slot stopped or restarted)
        if (*events) {
            BP4_FOR_QUBITS(w) {
                float *msg = reg0 + w.off;
                const int *h = reinterpret_cast<const int *>(msg + a.hdr_off);
                if (h[kHdrDone] >= 0) {
                    const uint8_t *ehat = reinterpret_cast<const uint8_t *>(msg + a.ehat_off);
                    a.est[(size_t)h[kHdrDone] * n + w.x] = (uint8_t)decision_pauli(ehat[w.x]);
                }
                if (h[kHdrFresh])
                    init_qubit<VAR, W, C22>(s_vi, s_vl, s_pi, msg, msg + a.q_off, msg + a.acc_off, (int)w.x, n, C);
            }
            BP4_FOR_CHECKS(w) {
                float *msg = reg0 + w.off;
                const int *h = reinterpret_cast<const int *>(msg + a.hdr_off);
                if (h[kHdrFresh]) {
                    uint8_t *syn = reinterpret_cast<uint8_t *>(msg + a.syn_off);
                    syn[w.x] = a.synd[(size_t)h[kHdrShot] * m + w.x];
                }
            }
            if (tid < (int)S && hdr(tid)[kHdrFresh]) reg0[tid * RW + lds_pad_slot<W>(n)] = INFINITY;
        }
        if (events[3]) {   // some slot was left without a shot (the queue is empty)
            // Compaction: once the queue is empty, a slot left without a shot takes
            // the region of the last active slot, so the phases walk only the active
            // slots and the tail of a workgroup (its last long-running shots) costs
            // their items, not S slots' worth
            __syncthreads();
            for (;;) {
                if (tid == 0) {
                    int na = events[1], hole = -1;
                    while (na > 0 && hdr((uint32_t)(na - 1))[kHdrShot] >= a.shots) --na;
                    for (int k = 0; k + 1 < na; ++k)
                        if (hdr((uint32_t)k)[kHdrShot] >= a.shots) {
                            hole = k;
                            break;
                        }
                    events[1] = na;
                    events[2] = hole;
                }
                __syncthreads();
                const int hole = events[2], na = events[1];
                if (hole < 0) break;
                const float *src = reg0 + (uint32_t)(na - 1) * RW;
                float *dst = reg0 + (uint32_t)hole * RW;
                for (uint32_t i = (uint32_t)tid; i < RW; i += kBlock) dst[i] = src[i];
                __syncthreads();
                if (tid == 0) {   // the vacated slot is empty
                    int *h = hdr((uint32_t)(na - 1));
                    h[kHdrShot] = a.shots;
                    h[kHdrDone] = -1;
                    h[kHdrFresh] = 0;
                    events[1] = na - 1;
                }
                __syncthreads();
            }
            end = (uint32_t)events[1] * RW;
        }
        if (!any_more) break;
        __syncthreads();
        if (tid == 0) {   // every lane has read them before the barrier above
            events[0] = 0;
            events[3] = 0;
        }
        // ---- Horizontal update (eq. h_update) ----------------------------------------
        BP4_FOR_CHECKS(w) {
            float *msg = reg0 + w.off;
            const uint8_t *syn = reinterpret_cast<const uint8_t *>(msg + a.syn_off);
            check_node<W>(s_ce, msg, (int)w.x, syn[w.x], C);
        }
        __syncthreads();
        // ---- Posterior, hard decision and vertical update ----------------------------
        auto qubit_phase = [&](auto wy) {
            // the slot's header is read when the walk enters the slot
            uint32_t cur = ~0u;
            int t = 0, shot = 0;
            BP4_FOR_QUBITS(w) {
                float *msg = reg0 + w.off;
                if (w.off != cur) {
                    const int *h = reinterpret_cast<const int *>(msg + a.hdr_off);
                    t = h[kHdrT] + 1;
                    shot = h[kHdrShot];
                    if (VAR == BP4_AEWA) vp.alpha = __int_as_float(h[kHdrAlpha]);
                    cur = w.off;
                }
                if constexpr (C22)
                    qubit_node_c22<VAR>(a, s_vi, s_pi, msg, msg + a.q_off, msg + a.acc_off,
                                        reinterpret_cast<uint8_t *>(msg + a.ehat_off), (int)w.x, t, vp);
                else
                    qubit_node<VAR, decltype(wy)::value, W>(a, s_vi, s_vl, s_pi, msg, msg + a.q_off, msg + a.acc_off,
                                                            reinterpret_cast<uint8_t *>(msg + a.ehat_off), (int)w.x, t,
                                                            vp, shot);
            }
        };
        if (C22 || !with_y) qubit_phase(std::false_type{});
        else qubit_phase(std::true_type{});
        __syncthreads();
        // ---- Syndrome test of the hard decision (Algorithm 2) ---------------------------
        {
            // a lane ORs the results of its consecutive items of one slot and sets that
            // slot's flag once (lanes setting one flag together serialise in LDS)
            uint32_t bad = 0, cur = wm0.off;
            BP4_FOR_CHECKS(w) {
                if (w.off != cur) {
                    if (bad) reinterpret_cast<int *>(reg0 + cur + a.hdr_off)[kHdrBad + par] = 1;
                    bad = 0;
                    cur = w.off;
                }
                const float *msg = reg0 + w.off;
                const uint8_t *syn = reinterpret_cast<const uint8_t *>(msg + a.syn_off);
                bad |= test_node<W>(s_ce, reinterpret_cast<const uint8_t *>(msg + a.ehat_off), (int)w.x, syn[w.x]);
            }
            if (bad) reinterpret_cast<int *>(reg0 + cur + a.hdr_off)[kHdrBad + par] = 1;
        }
        __syncthreads();
        // ---- Per-slot bookkeeping: stop, restart (AEWA) or continue ---------------------
        more = false;
        if (tid < (int)S) {
            int *h = hdr(tid);
            h[kHdrDone] = -1;
            h[kHdrFresh] = 0;
            const int shot = h[kHdrShot];
            if (shot < a.shots) {
                const int t = h[kHdrT] + 1;
                const bool sat = h[kHdrBad + par] == 0;
                const bool restart = VAR == BP4_AEWA && !sat && t >= a.max_iter && h[kHdrAtt] + 1 < a.alpha_steps;
                const bool fin = !restart && ((a.stop && sat) || t >= a.max_iter);
                if (fin || restart) *events = 1;
                if (fin) {
                    a.conv[shot] = sat ? 1 : 0;
                    a.iters[shot] = h[kHdrTBefore] + t;
                    h[kHdrDone] = shot;
                    const int s = take_shot(a.counter, a.shots);
                    h[kHdrShot] = s;
                    h[kHdrT] = 0;
                    h[kHdrAtt] = 0;
                    h[kHdrTBefore] = 0;
                    h[kHdrAlpha] = __float_as_int(a.alpha);
                    h[kHdrFresh] = s < a.shots ? 1 : 0;
                    if (s >= a.shots) events[3] = 1;
                } else if (restart) {
                    h[kHdrTBefore] += t;
                    h[kHdrAtt] += 1;
                    h[kHdrT] = 0;
                    h[kHdrAlpha] = __float_as_int(aewa_alpha(a.alpha, a.alpha_last, a.alpha_steps, h[kHdrAtt]));
                    h[kHdrFresh] = 1;
                } else {
                    h[kHdrT] = t;
                }
            }
            // the other flag was last read one iteration ago: clear it for the next one
            h[kHdrBad + (par ^ 1)] = 0;
            more = h[kHdrShot] < a.shots;
        }
        par ^= 1;
        any_more = __syncthreads_or(more);
    }
#undef BP4_FOR_CHECKS
#undef BP4_FOR_QUBITS
}

// C22OK: the build takes the two-plus-two layout for codes that allow it (the
// single-variant builds; the variant-switching build would hold both paths' registers).
template <int VAR, bool W = false, bool C22OK = false>
__device__ __forceinline__ void run_code(const DecodeArgs &a, float *lds, int *events)
{
    if constexpr (!W && C22OK) {
        if (a.css22) {
            if (a.block_shots > 0) run_block<VAR, false, true>(a, lds, events);
            else run_wave<VAR, false, true>(a, lds);
            return;
        }
    }
    if (a.block_shots > 0) run_block<VAR, W>(a, lds, events);
    else run_wave<VAR, W>(a, lds);
}

// VSET: the variant every code of the launch uses, kMixedVariants for a flooding
// launch that mixes variants (a switch per code), kSerial for the serial schedule
// (one code, a switch on its variant; kSerialWide for a wide graph), kWide for a
// flooding launch of wide graphs (a switch on the variant).  Register budget: 80 VGPRs (six wavefronts per
// SIMD: three 512-lane workgroups per CU) for every build but the wide ones, 128
// (four) for those, whose 8-edge checks hold twice the messages in registers.  The
// AdaGrad and switching builds spill 12-13 registers at 80 and still ran an
// AdaGrad batch 19 % faster than at 96 VGPRs, where only two workgroups fit.
constexpr int kMixedVariants = -1, kSerial = -2, kWide = -3, kSerialWide = -4;
constexpr int lds_kernel_waves(int vset)
{
    return vset == kWide || vset == kSerialWide ? 4 : 6;
}

template <int VSET>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(lds_kernel_waves(VSET))))
decode_lds_kernel(MixedArgs args)
{
    // 16-byte aligned: the packed check edges are read as 16-byte vectors
    extern __shared__ __attribute__((aligned(16))) float lds[];
    __shared__ int pending;
    // block slots: [0] some slot stopped or restarted this round, [1] active slots,
    // [2] a slot to refill by compaction, [3] some slot was left without a shot
    __shared__ int events[4];
    for (int ci = 0; ci < args.ncodes; ++ci) {
        const DecodeArgs &a = args.codes[ci];
        // skip a code whose queue is already empty (a stale read only costs a visit)
        if (threadIdx.x == 0) {
            pending = __hip_atomic_load(a.counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < (unsigned)a.shots;
            events[3] = 0;
        }
        __syncthreads();
        if (!pending) continue;
        // stage the code's packed check edges, qubit words and priors
        const int m = a.g.m, n = a.g.n;
        uint32_t *s_ce = reinterpret_cast<uint32_t *>(lds);
        const int cs = a.g.cstride;
        uint32_t *s_vi = s_ce + cs * m;
        float *s_pi = reinterpret_cast<float *>(s_vi + n);
        constexpr bool SER = VSET == kSerial || VSET == kSerialWide;
        if (SER) {
            for (int i = threadIdx.x; i < cs * m; i += kBlock) s_ce[i] = a.g.cedge[i];
        } else {
            // slot field -> slot-major position v + j n (j: the edge's rank among its
            // qubit's slots); padding -> the padding slot.  kSlots n < 2^16: the
            // layout holds kSlots n message words in LDS.
            // Two-plus-two layout: position = 2 [Z label] + rank among the qubit's slots
            // of the same label.
            constexpr bool W = VSET == kWide;
            const bool c22 = VSET >= 0 && a.css22;
            for (int i = threadIdx.x; i < cs * m; i += kBlock) {
                const uint32_t w = a.g.cedge[i];
                uint32_t slot = lds_pad_slot<W>((uint32_t)n);
                if (!edge_is_pad(w)) {
                    const uint32_t v = edge_var(w);
                    const uint32_t info = a.g.vinfo[v];
                    const uint32_t j = edge_slot(w) - var_base(info);
                    slot = v + (c22 ? c22_pos(info, j) : j) * (uint32_t)n;
                }
                s_ce[i] = (w & ~0xFFFFu) | slot;
            }
        }
        if (VSET >= 0 && a.css22)
            for (int i = threadIdx.x; i < n; i += kBlock) s_vi[i] = c22_info(a.g.vinfo[i]);
        else
            for (int i = threadIdx.x; i < n; i += kBlock) s_vi[i] = a.g.vinfo[i];
        for (int i = threadIdx.x; i < 3 * n; i += kBlock) s_pi[i] = a.prior[i];
        if (VSET == kWide) {   // slot labels of a wide graph
            uint32_t *s_vl = reinterpret_cast<uint32_t *>(s_pi + 3 * n);
            for (int i = threadIdx.x; i < n; i += kBlock) s_vl[i] = a.g.vlab[i];
        }
        if (SER) {   // slot -> check table and the level order (wide graphs: the slot labels)
            uint32_t *s_vchk = reinterpret_cast<uint32_t *>(s_pi + 3 * n);
            uint32_t *s_ord = s_vchk + a.g.nnz;
            uint32_t *s_lev = s_ord + n;
            for (int i = threadIdx.x; i < a.g.nnz; i += kBlock) s_vchk[i] = a.g.vchk[i];
            for (int i = threadIdx.x; i < n; i += kBlock) s_ord[i] = a.g.sord[i];
            for (int i = threadIdx.x; i <= a.g.nlev; i += kBlock) s_lev[i] = a.g.slev[i];
            if (VSET == kSerialWide) {
                uint32_t *s_vl = s_lev + a.g.nlev + 1;
                for (int i = threadIdx.x; i < n; i += kBlock) s_vl[i] = a.g.vlab[i];
            }
        }
        __syncthreads();
        if (SER) {
            constexpr bool SW = VSET == kSerialWide;
            if (a.with_y) {
                switch (a.variant) {
                case BP4_BP: run_serial<BP4_BP, true, SW>(a, lds); break;
                case BP4_MOMENTUM: run_serial<BP4_MOMENTUM, true, SW>(a, lds); break;
                case BP4_ADAGRAD: run_serial<BP4_ADAGRAD, true, SW>(a, lds); break;
                case BP4_AEWA: run_serial<BP4_AEWA, true, SW>(a, lds); break;
                default: run_serial<BP4_EWAINIT, true, SW>(a, lds); break;
                }
            } else {
                switch (a.variant) {
                case BP4_BP: run_serial<BP4_BP, false, SW>(a, lds); break;
                case BP4_MOMENTUM: run_serial<BP4_MOMENTUM, false, SW>(a, lds); break;
                case BP4_ADAGRAD: run_serial<BP4_ADAGRAD, false, SW>(a, lds); break;
                case BP4_AEWA: run_serial<BP4_AEWA, false, SW>(a, lds); break;
                default: run_serial<BP4_EWAINIT, false, SW>(a, lds); break;
                }
            }
        } else if (VSET == kWide) {   // the host launches only wide codes here
            if (a.wide) {
                switch (a.variant) {
                case BP4_BP: run_code<BP4_BP, true>(a, lds, events); break;
                case BP4_MOMENTUM: run_code<BP4_MOMENTUM, true>(a, lds, events); break;
                case BP4_ADAGRAD: run_code<BP4_ADAGRAD, true>(a, lds, events); break;
                case BP4_AEWA: run_code<BP4_AEWA, true>(a, lds, events); break;
                default: run_code<BP4_EWAINIT, true>(a, lds, events); break;
                }
            }
        } else if (VSET == kMixedVariants) {
            switch (a.variant) {
            case BP4_BP: run_code<BP4_BP>(a, lds, events); break;
            case BP4_MOMENTUM: run_code<BP4_MOMENTUM>(a, lds, events); break;
            case BP4_ADAGRAD: run_code<BP4_ADAGRAD>(a, lds, events); break;
            case BP4_AEWA: run_code<BP4_AEWA>(a, lds, events); break;
            default: run_code<BP4_EWAINIT>(a, lds, events); break;
            }
        } else {
            constexpr int V = VSET < 0 ? BP4_EWAINIT : VSET;
            run_code<V, false, true>(a, lds, events);
        }
        __syncthreads();
    }
}

}  // namespace

LdsLayout decode_lds_layout(int m, int n, int nnz, int variant, int G, int S, bool wide)
{
    LdsLayout L;
    // check edges, qubit words, priors (and the slot labels of a wide graph)
    L.static_words = (wide ? kMaxCheckDegWide : kMaxCheckDeg) * m + n + 3 * n + (wide ? n : 0);
    if (L.static_words & 3) L.static_words += 4 - (L.static_words & 3);
    int w = (wide ? 8 : 4) * n + 1;   // slot-major message slots and the padding slot
    L.q_off = w;
    if (variant != BP4_BP) w += 3 * n;
    L.acc_off = w;
    if (variant == BP4_MOMENTUM || variant == BP4_ADAGRAD) w += 3 * n;
    L.ehat_off = w;
    w += (n + 3) / 4;
    if (S > 0) {                   // block slots: syndrome bytes and the slot header
        L.syn_off = w;
        w += (m + 3) / 4;
        L.hdr_off = w;
        w += kHdrBad + 2;
    }
    if ((w & 1) == 0) w += 1;   // odd stride: neighbouring regions start on other banks
    L.region_words = w;
    L.group_lanes = S > 0 ? kBlock : G;
    L.block_shots = S;
    L.block = kBlock;
    const int regions = S > 0 ? S : kBlock / G;
    L.bytes = (size_t)4 * (L.static_words + (size_t)regions * L.region_words);
    return L;
}

LdsLayout decode_lds_serial_layout(int m, int n, int nnz, int nlev, int variant, int G, bool wide)
{
    LdsLayout L;
    // check edges, qubit words, priors, slot -> check, level order and offsets (wide
    // graphs: 8 edge words per check and the slot labels)
    L.static_words = (wide ? kMaxCheckDegWide : kMaxCheckDeg) * m + n + 3 * n + nnz + n + nlev + 1 + (wide ? n : 0);
    if (L.static_words & 3) L.static_words += 4 - (L.static_words & 3);
    int w = nnz;                   // signed phi of each m_{v->c}
    L.q_off = w;
    if (variant != BP4_BP) w += 3 * n;
    L.acc_off = w;
    if (variant == BP4_MOMENTUM || variant == BP4_ADAGRAD) w += 3 * n;
    L.ehat_off = w;
    w += (n + 3) / 4;
    L.syn_off = w;
    w += (m + 3) / 4;
    if ((w & 1) == 0) w += 1;
    L.region_words = w;
    L.group_lanes = G;
    L.block = kBlock;
    L.bytes = (size_t)4 * (L.static_words + (size_t)(kBlock / G) * L.region_words);
    return L;
}

// Lane use of a layout: the share of issued (lane, item) pairs that carry a check
// or a qubit, averaged over the two phases.
static double lane_use(int m, int n, int G, int S)
{
    if (S > 0) {
        const double pc = std::ceil((double)S * m / kBlock), pv = std::ceil((double)S * n / kBlock);
        return 0.5 * ((double)S * m / (kBlock * pc) + (double)S * n / (kBlock * pv));
    }
    const int kc = (m + G - 1) / G, kv = (n + G - 1) / G;
    return 0.5 * ((double)m / (G * kc) + (double)n / (G * kv));
}

bool decode_lds_fits(int m, int n, int G, int S)
{
    if (S > 0) {
        if (S > kBlock) return false;
        if ((uint64_t)S * m * m >= (1ull << 32) || (uint64_t)S * n * n >= (1ull << 32)) return false;
        return ((int64_t)S * m + kBlock - 1) / kBlock <= 64;
    }
    return G >= 4 && G <= 64 && (G & (G - 1)) == 0 && (m + G - 1) / G <= 64;
}

// Lane mapping for a code when no tuned choice is given.  Score = lane use times
// an occupancy factor: the wavefronts per CU that the LDS allows (up to 24, the
// register limit of the single-variant builds) over 24.  Candidates: block slots
// S = 1..64, then wave groups of 64 down to 4 lanes; at most `max_lds` bytes per
// workgroup.  Among block-slot mappings within 2 % of the best score the most
// slots win (each barrier of an iteration then covers more passes of items), up
// to the count that still lets the resident workgroups (three per CU on 256 CUs)
// cycle through `shots` at least 12 times, since a batch of few rounds waits on
// the tail of its last round.
LaneChoice decode_lds_pick(int m, int n, int nnz, int variant, size_t max_lds, bool wide, int64_t shots)
{
    const double cu_lds = 160.0 * 1024.0;
    auto score_of = [&](int G, int S) {
        if (!decode_lds_fits(m, n, G, S)) return -1.0;
        const LdsLayout L = decode_lds_layout(m, n, nnz, variant, G, S, wide);
        if (L.bytes > max_lds) return -1.0;
        // LDS is allocated in granules: a layout occupies its size rounded up to 2 KB
        const double blocks = std::floor(cu_lds / (double)((L.bytes + 2047) / 2048 * 2048));
        double waves = blocks * (L.block / 64);
        if (waves > 24.0) waves = 24.0;
        return lane_use(m, n, G, S) * waves / 24.0;
    };
    int64_t cap = shots > 0 ? shots / (2 * 3 * 256) : 64;
    if (cap < 1) cap = 1;
    if (cap > 64) cap = 64;
    LaneChoice best;
    double best_score = -1.0;
    for (int S = 1; S <= cap; ++S) best_score = std::max(best_score, score_of(kBlock, S));
    for (int G = 64; G >= 4; G /= 2) {
        const double sc = score_of(G, 0);
        if (sc > best_score * 1.02) {
            best_score = sc;
            best.group_lanes = G;
            best.block_shots = 0;
        }
    }
    if (best.group_lanes > 0 && best.block_shots == 0 && best_score > 0.0) return best;   // a wave group won
    for (int S = (int)cap; S >= 1; --S) {
        if (best_score > 0.0 && score_of(kBlock, S) >= best_score * 0.98) {
            best.group_lanes = kBlock;
            best.block_shots = S;
            return best;
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
        const long gpb = args.codes[i].block_shots > 0 ? args.codes[i].block_shots : kBlock / args.codes[i].group_lanes;
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
    bool serial = false;
    for (int i = 0; i < args.ncodes; ++i) serial = serial || args.codes[i].serial;
    if (serial)   // a single code
        return args.codes[0].wide ? launch_lds_kernel<kSerialWide>(args, lds_bytes, s, grid_out)
                                  : launch_lds_kernel<kSerial>(args, lds_bytes, s, grid_out);
    int wide = 0;
    for (int i = 0; i < args.ncodes; ++i) wide += args.codes[i].wide ? 1 : 0;
    if (wide == args.ncodes) return launch_lds_kernel<kWide>(args, lds_bytes, s, grid_out);
    if (wide > 0) {
        // Wide and narrow codes: two persistent launches in stream order, the wide codes
        // on the wide build and the narrow ones on theirs, each with the LDS of its own
        // codes (one build holding both paths needed a 4 KB scratch stack per lane and
        // ran the wide codes three times slower).
        MixedArgs part[2];
        size_t bytes[2] = {0, 0};
        part[0].ncodes = part[1].ncodes = 0;
        for (int i = 0; i < args.ncodes; ++i) {
            const DecodeArgs &c = args.codes[i];
            const int k = c.wide ? 0 : 1;
            part[k].codes[part[k].ncodes++] = c;
            const int regions = c.block_shots > 0 ? c.block_shots : kBlock / c.group_lanes;
            const size_t b = (size_t)4 * ((size_t)c.static_words + (size_t)regions * c.region_words);
            bytes[k] = b > bytes[k] ? b : bytes[k];
        }
        hipError_t e = launch_lds_kernel<kWide>(part[0], bytes[0], s, grid_out);
        if (e != hipSuccess) return e;
        return launch_decode_lds(part[1], bytes[1], s, nullptr);
    }
    switch (v) {
    case BP4_BP: return launch_lds_kernel<BP4_BP>(args, lds_bytes, s, grid_out);
    case BP4_MOMENTUM: return launch_lds_kernel<BP4_MOMENTUM>(args, lds_bytes, s, grid_out);
    case BP4_ADAGRAD: return launch_lds_kernel<BP4_ADAGRAD>(args, lds_bytes, s, grid_out);
    case BP4_EWAINIT: return launch_lds_kernel<BP4_EWAINIT>(args, lds_bytes, s, grid_out);
    case BP4_AEWA: return launch_lds_kernel<BP4_AEWA>(args, lds_bytes, s, grid_out);
    default: return launch_lds_kernel<kMixedVariants>(args, lds_bytes, s, grid_out);
    }
}

}  // namespace bp4
