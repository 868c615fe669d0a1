// Per-code "plain" flooding BP: the textbook GPU mapping, kept as the reference
// point for the persistent kernels.  One kernel per phase per iteration (check
// update, qubit update, syndrome test, bookkeeping of finished shots), one
// thread per (shot, check) or (shot, qubit), messages and per-qubit state in
// HBM as structure-of-arrays [slot][shot] so that consecutive lanes touch
// consecutive shots.  Finished shots are masked, not compacted; the host reads
// the number of unfinished shots after every iteration and stops at zero or at
// iter_max.  The arithmetic per node is the shared device code, so results are
// bitwise equal to the LDS kernel's.  Wide graphs (checks of up to 8 edges, qubits of
// up to 7, their slot labels in a separate word) take the same kernels built at width 8.
#include "bp4_math.h"
#include "bp4_wide.h"

namespace bp4 {
namespace {

constexpr int kTile = 256;   // shots per workgroup (x), one check or qubit per grid row (y)

struct PlainArgs {
    GraphView g;
    const float *prior;
    const uint8_t *synd;
    uint8_t *est, *conv;
    int32_t *iters;
    float *msg;        // [nnz][shots]
    float *st;         // [3n][shots] (EWAInit, Momentum, AdaGrad)
    float *acc;        // [3n][shots] (Momentum, AdaGrad)
    uint8_t *ehat;     // [n][shots]
    uint8_t *active;   // [shots]
    uint8_t *unsat;    // [shots]
    unsigned int *remaining;
    int32_t shots, t, max_iter, stop;
    float clamp;
    VariantParams vp;
};

__global__ void __launch_bounds__(kTile) plain_init_kernel(PlainArgs a)
{
    const int shot = blockIdx.x * kTile + threadIdx.x;
    const int v = blockIdx.y;
    if (shot >= a.shots) return;
    const size_t S = (size_t)a.shots;
    if (v == 0) {
        a.active[shot] = 1;
        a.unsat[shot] = 0;
    }
    const uint32_t info = a.g.vinfo[v];
    const float p3[3] = {a.prior[3 * v], a.prior[3 * v + 1], a.prior[3 * v + 2]};
    float st[3], ac[3];
    qubit_state_init(a.vp.variant, p3, st, ac);
    if (a.vp.variant != BP4_BP)
        for (int x = 0; x < 3; ++x) a.st[(3 * v + x) * S + shot] = st[x];
    if (a.vp.variant == BP4_MOMENTUM || a.vp.variant == BP4_ADAGRAD)
        for (int x = 0; x < 3; ++x) a.acc[(3 * v + x) * S + shot] = ac[x];
    float lam[4];
    qubit_lambdas(p3, var_labels_present(info), lam);
    const uint32_t base = var_base(info), deg = var_deg(info);
    const bool wide = a.g.cstride > kMaxCheckDeg;
    for (uint32_t j = 0; j < deg; ++j) {
        const uint32_t lab = wide ? slot_label(a.g.vlab[v], (int)j) : var_lab(info, j);
        a.msg[(base + j) * S + shot] = clampf(lam[lab], a.clamp);
    }
}

// W: wide graph (8 edge words per check).
template <bool W>
__global__ void __launch_bounds__(kTile) plain_check_kernel(PlainArgs a)
{
    constexpr int D = W ? kMaxCheckDegWide : kMaxCheckDeg;
    const int shot = blockIdx.x * kTile + threadIdx.x;
    const int c = blockIdx.y;
    if (shot >= a.shots || !a.active[shot]) return;
    const size_t S = (size_t)a.shots;
    uint32_t w[D];
    float mv[D], out[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
        w[j] = a.g.cedge[c * D + j];
        mv[j] = edge_is_pad(w[j]) ? INFINITY : a.msg[edge_slot(w[j]) * S + shot];
    }
    const uint32_t sb = a.synd[(size_t)shot * a.g.m + c];
    if constexpr (W) check_update_wide(mv, sb, a.clamp, out);
    else check_update(mv, sb, a.clamp, out);
#pragma unroll
    for (int j = 0; j < D; ++j)
        if (!edge_is_pad(w[j])) a.msg[edge_slot(w[j]) * S + shot] = out[j];
}

template <bool W>
__global__ void __launch_bounds__(kTile) plain_var_kernel(PlainArgs a)
{
    constexpr int DV = W ? 8 : 4;
    const int shot = blockIdx.x * kTile + threadIdx.x;
    const int v = blockIdx.y;
    if (shot >= a.shots || !a.active[shot]) return;
    const size_t S = (size_t)a.shots;
    const uint32_t info = a.g.vinfo[v];
    const uint32_t base = var_base(info), deg = var_deg(info);
    float mc[DV];
#pragma unroll
    for (int j = 0; j < DV; ++j) mc[j] = (uint32_t)j < deg ? a.msg[(base + j) * S + shot] : 0.0f;
    float Sl[4], Al[4];
    const uint32_t labw = W ? a.g.vlab[v] : 0u;
    if constexpr (W) label_sums_w<DV>(labw, mc, true, a.vp.variant == BP4_ADAGRAD, Sl, Al);
    else label_sums(info, mc, true, a.vp.variant == BP4_ADAGRAD, Sl, Al);
    const float p3[3] = {a.prior[3 * v], a.prior[3 * v + 1], a.prior[3 * v + 2]};
    const bool keep_q = a.vp.variant != BP4_BP;
    const bool keep_acc = a.vp.variant == BP4_MOMENTUM || a.vp.variant == BP4_ADAGRAD;
    float st[3] = {0.0f, 0.0f, 0.0f}, ac[3] = {0.0f, 0.0f, 0.0f}, qn[3];
    if (keep_q)
        for (int x = 0; x < 3; ++x) st[x] = a.st[(3 * v + x) * S + shot];
    if (keep_acc)
        for (int x = 0; x < 3; ++x) ac[x] = a.acc[(3 * v + x) * S + shot];
    qubit_posterior(a.vp, a.t, p3, Sl, Al, st, ac, qn);
    if (keep_q)
        for (int x = 0; x < 3; ++x) a.st[(3 * v + x) * S + shot] = st[x];
    if (keep_acc)
        for (int x = 0; x < 3; ++x) a.acc[(3 * v + x) * S + shot] = ac[x];
    a.ehat[(size_t)v * S + shot] = (uint8_t)hard_decision(qn);
    float lam[4];
    qubit_lambdas(qn, var_labels_present(info), lam);
#pragma unroll
    for (int j = 0; j < DV; ++j)
        if ((uint32_t)j < deg) {
            const uint32_t lab = W ? slot_label(labw, j) : var_lab(info, j);
            a.msg[(base + j) * S + shot] = clampf(lam[lab] - mc[j], a.clamp);
        }
}

template <bool W>
__global__ void __launch_bounds__(kTile) plain_test_kernel(PlainArgs a)
{
    constexpr int D = W ? kMaxCheckDegWide : kMaxCheckDeg;
    const int shot = blockIdx.x * kTile + threadIdx.x;
    const int c = blockIdx.y;
    if (shot >= a.shots || !a.active[shot]) return;
    const size_t S = (size_t)a.shots;
    uint32_t par = a.synd[(size_t)shot * a.g.m + c] & 1u, bad = 0;
#pragma unroll
    for (int j = 0; j < D; ++j) {
        const uint32_t w = a.g.cedge[c * D + j];
        if (edge_is_pad(w)) continue;
        const uint32_t e = a.ehat[(size_t)edge_var(w) * S + shot];
        if (e == 0xFFu) bad = 1u;
        else par ^= anticomm(edge_lab(w), e);
    }
    if (par | bad) a.unsat[shot] = 1;   // every writer stores the same value
}

__global__ void __launch_bounds__(kTile) plain_finish_kernel(PlainArgs a)
{
    const int shot = blockIdx.x * kTile + threadIdx.x;
    if (shot >= a.shots || !a.active[shot]) return;
    const size_t S = (size_t)a.shots;
    const bool sat = a.unsat[shot] == 0;
    a.unsat[shot] = 0;
    if ((a.stop && sat) || a.t >= a.max_iter) {
        a.conv[shot] = sat ? 1 : 0;
        a.iters[shot] = a.t;
        a.active[shot] = 0;
        for (int v = 0; v < a.g.n; ++v) {
            const uint8_t e = a.ehat[(size_t)v * S + shot];
            a.est[(size_t)shot * a.g.n + v] = e == 0xFFu ? 0 : e;
        }
    } else {
        atomicAdd(a.remaining, 1u);
    }
}

}  // namespace

size_t plain_workspace_bytes(int n, int nnz, int variant, int64_t shots)
{
    const size_t S = (size_t)shots;
    size_t b = 256;                                   // counter
    b += ((size_t)nnz * S * 4 + 255) & ~size_t(255);  // messages
    if (variant != BP4_BP) b += ((size_t)3 * n * S * 4 + 255) & ~size_t(255);
    if (variant == BP4_MOMENTUM || variant == BP4_ADAGRAD) b += ((size_t)3 * n * S * 4 + 255) & ~size_t(255);
    b += ((size_t)n * S + 255) & ~size_t(255);        // hard decisions
    b += 2 * ((S + 255) & ~size_t(255));              // active, unsat
    return b;
}

hipError_t run_plain(const GraphView &g, const bp4_params &p, int32_t shots, const float *prior,
                     const uint8_t *synd, uint8_t *est, uint8_t *conv, int32_t *iters, void *ws,
                     hipStream_t s, int32_t *iterations_run)
{
    PlainArgs a;
    a.g = g;
    a.prior = prior;
    a.synd = synd;
    a.est = est;
    a.conv = conv;
    a.iters = iters;
    const size_t S = (size_t)shots;
    char *w = static_cast<char *>(ws);
    a.remaining = reinterpret_cast<unsigned int *>(w);
    w += 256;
    a.msg = reinterpret_cast<float *>(w);
    w += ((size_t)g.nnz * S * 4 + 255) & ~size_t(255);
    a.st = nullptr;
    a.acc = nullptr;
    if (p.variant != BP4_BP) {
        a.st = reinterpret_cast<float *>(w);
        w += ((size_t)3 * g.n * S * 4 + 255) & ~size_t(255);
    }
    if (p.variant == BP4_MOMENTUM || p.variant == BP4_ADAGRAD) {
        a.acc = reinterpret_cast<float *>(w);
        w += ((size_t)3 * g.n * S * 4 + 255) & ~size_t(255);
    }
    a.ehat = reinterpret_cast<uint8_t *>(w);
    w += ((size_t)g.n * S + 255) & ~size_t(255);
    a.active = reinterpret_cast<uint8_t *>(w);
    w += (S + 255) & ~size_t(255);
    a.unsat = reinterpret_cast<uint8_t *>(w);
    a.shots = shots;
    a.max_iter = p.max_iter;
    a.stop = p.stop_on_syndrome ? 1 : 0;
    a.clamp = p.llr_clamp;
    a.vp.variant = p.variant;
    a.vp.g_from_t1 = p.adagrad_g_from_t1;
    a.vp.alpha = p.alpha;
    a.vp.gamma = p.gamma;
    a.vp.eps = p.eps;
    a.t = 0;
    const unsigned xb = (unsigned)((shots + kTile - 1) / kTile);
    hipLaunchKernelGGL(plain_init_kernel, dim3(xb, g.n), dim3(kTile), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    *iterations_run = 0;
    for (int t = 1; t <= p.max_iter; ++t) {
        a.t = t;
        e = launch_zero_u32(a.remaining, 1, s);
        if (e != hipSuccess) return e;
        if (g.cstride > kMaxCheckDeg) {
            hipLaunchKernelGGL(plain_check_kernel<true>, dim3(xb, g.m), dim3(kTile), 0, s, a);
            hipLaunchKernelGGL(plain_var_kernel<true>, dim3(xb, g.n), dim3(kTile), 0, s, a);
            hipLaunchKernelGGL(plain_test_kernel<true>, dim3(xb, g.m), dim3(kTile), 0, s, a);
        } else {
            hipLaunchKernelGGL(plain_check_kernel<false>, dim3(xb, g.m), dim3(kTile), 0, s, a);
            hipLaunchKernelGGL(plain_var_kernel<false>, dim3(xb, g.n), dim3(kTile), 0, s, a);
            hipLaunchKernelGGL(plain_test_kernel<false>, dim3(xb, g.m), dim3(kTile), 0, s, a);
        }
        hipLaunchKernelGGL(plain_finish_kernel, dim3(xb), dim3(kTile), 0, s, a);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        unsigned int left = 0;
        e = hipMemcpyAsync(&left, a.remaining, sizeof left, hipMemcpyDeviceToHost, s);
        if (e != hipSuccess) return e;
        e = hipStreamSynchronize(s);
        if (e != hipSuccess) return e;
        *iterations_run = t;
        if (left == 0) break;
    }
    return hipSuccess;
}

}  // namespace bp4
