// Flooding GF(4) BP for large codes: one lane decodes one shot; each lane's
// messages, per-qubit state and syndrome bits live in HBM as a column of a
// structure-of-arrays record [wavefront][item][64 lanes], so the 64 lanes of a
// wavefront touch 64 consecutive words of every item and a wavefront's whole
// state is one contiguous block.  All lanes of a wavefront walk the checks and
// qubits in the same order, so the packed graph words are wavefront-uniform
// (scalar loads).
//
// Iteration blocks: a launch runs the live shots through at most `iter_block`
// iterations.  Shots that stop are written out; the others move their column to
// a second record buffer, densely, so the next launch runs only live shots on
// fully populated wavefronts instead of idling lanes behind the shots that run
// to the iteration limit.  With the flooding schedule the move costs no extra
// traffic: the shots entering a launch's last iteration take their new column
// first, and that iteration reads the old column and writes the new one; a shot
// that stops in it leaves a hole (shot id -1) that the next launch skips.  The
// arithmetic of a shot does not depend on its column, so results do not depend
// on the block length or the compaction order.
//
// Paper: Chen, Yi, Liang, Wang, "Improved Belief Propagation Decoding
// Algorithms for Surface Codes", section II-B1 (eqs. init, h_update,
// v_update, p_update), section III (eqs. mombp1-3, boost, EWAInit, Algorithm 2).
#include "bp4_math.h"

namespace bp4 {
namespace {

constexpr int kSoaBlock = 256;
constexpr int kChunk = 4;   // checks (qubits) whose loads are issued together; divides 32

// The graph and the priors are read-only and read at wavefront-uniform addresses:
// read through the constant address space so they become scalar loads.
template <typename T> using konst = const __attribute__((address_space(4))) T;
template <typename T> __device__ __forceinline__ konst<T> *as_const(const T *p) { return (konst<T> *)p; }

// Items (32-bit words) of one column record: messages, posterior, accumulator,
// syndrome bits.
struct SoaLayout {
    int32_t items, st_off, acc_off, sb_off;
};

SoaLayout soa_layout(int m, int n, int nnz, int variant)
{
    SoaLayout L;
    int o = nnz;
    L.st_off = o;
    if (variant != BP4_BP) o += 3 * n;
    L.acc_off = o;
    if (variant == BP4_MOMENTUM || variant == BP4_ADAGRAD) o += 3 * n;
    L.sb_off = o;
    o += (m + 31) / 32;
    L.items = o;
    return L;
}

struct SoaArgs {
    GraphView g;
    const float *prior;       // [n][3]
    const uint8_t *synd;      // [shots][m]
    uint8_t *est;             // [shots][n]
    uint8_t *conv;            // [shots]
    int32_t *iters;           // [shots]
    float *q_out, *mvc_out, *mcv_out;   // optional verification outputs
    uint32_t *src;            // records of the live shots
    uint32_t *dst;            // records of the shots still live after this block
    const int32_t *src_shot;  // shot of each source column (blocks after the first)
    int32_t *dst_shot;
    const int32_t *src_tb;    // AEWA: iterations of the shot's earlier attempts, per column
    int32_t *dst_tb;
    const unsigned int *src_count;   // live columns (blocks after the first)
    unsigned int *dst_count;  // zeroed before the launch
    uint8_t *ehat;            // [wavefront][n][64] decision bytes
    int32_t first_shot, first_count;   // first block: shots first_shot + column
    int32_t t0, t_end, max_iter, stop, with_y;
    int32_t fresh;            // first block of the first attempt: columns are shots first_shot + column
    int32_t last_attempt;     // a shot that fails this attempt is finished (else it restarts)
    int32_t serial;           // serial schedule (Algorithm 1) instead of flooding
    float clamp;
    VariantParams vp;
    SoaLayout lay;
};

__global__ void __launch_bounds__(kSoaBlock) decode_soa_kernel(SoaArgs a)
{
    const int col = blockIdx.x * kSoaBlock + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const size_t wave = (size_t)(col >> 6);
    const int count = a.fresh ? a.first_count : (int)*a.src_count;
    if ((int)(wave << 6) >= count) return;   // whole wavefront idle
    const int src_shot = col < count && !a.fresh ? a.src_shot[col] : 0;
    const bool have = col < count && src_shot >= 0;   // -1: a hole left by the last block
    const int m = a.g.m, n = a.g.n;
    const int variant = a.vp.variant;
    const bool keep_q = variant != BP4_BP;
    const bool keep_acc = variant == BP4_MOMENTUM || variant == BP4_ADAGRAD;
    const bool with_y = a.with_y != 0;
    const float C = a.clamp;
    const size_t items = (size_t)a.lay.items;
    uint32_t *rec = a.src + wave * items * 64 + lane;    // item i at rec[64 i]
    float *msg = reinterpret_cast<float *>(rec);
    float *st = reinterpret_cast<float *>(rec + (size_t)a.lay.st_off * 64);
    float *acc = reinterpret_cast<float *>(rec + (size_t)a.lay.acc_off * 64);
    uint32_t *sb = rec + (size_t)a.lay.sb_off * 64;
    uint8_t *ehat = a.ehat + wave * (size_t)n * 64 + lane;
    konst<uint32_t> *cedge = as_const(a.g.cedge);
    konst<uint32_t> *vinfo = as_const(a.g.vinfo);
    konst<uint32_t> *vchk = as_const(a.g.vchk);
    konst<float> *prior = as_const(a.prior);

    const int shot = !have ? 0 : a.fresh ? a.first_shot + col : src_shot;
    const int t_before = have && !a.fresh ? a.src_tb[col] : 0;   // earlier AEWA attempts
    bool done = !have;
    int t_end_shot = 0;
    // the iteration's writes: the source record, or in a launch's last iteration the
    // shot's column of the next block's records
    float *wmsg = msg, *wst = st, *wacc = acc;
    int64_t moved = -1;   // column taken in the next block's records

    if (have && a.t0 == 0) {   // first block of an attempt: a fresh decode of the shot
        // ---- Initialisation (eq. init): syndrome bits and m_{v->c} = lambda(Pi) ----
        const uint8_t *srow = a.synd + (size_t)shot * m;
        uint32_t word = 0;
        int c = 0;
        if ((m & 3) == 0 && ((uintptr_t)a.synd & 3u) == 0) {
            // rows start on 4-byte boundaries: four syndrome bytes per load (bit 0 of
            // each byte, at bits 0, 8, 16, 24 of the word)
            for (; c < m; c += 4) {
                const uint32_t x = *reinterpret_cast<const uint32_t *>(srow + c);
                const uint32_t nib = (x & 1u) | ((x >> 7) & 2u) | ((x >> 14) & 4u) | ((x >> 21) & 8u);
                word |= nib << (c & 31);
                if (((c + 4) & 31) == 0) {
                    sb[(size_t)(c >> 5) * 64] = word;
                    word = 0;
                }
            }
        } else {
            for (; c < m; ++c) {
                word |= (uint32_t)(srow[c] & 1u) << (c & 31);
                if ((c & 31) == 31) {
                    sb[(size_t)(c >> 5) * 64] = word;
                    word = 0;
                }
            }
        }
        if (m & 31) sb[(size_t)((m - 1) >> 5) * 64] = word;   // the last, partial word
        for (int v = 0; v < n; ++v) {
            const uint32_t info = vinfo[v];
            const uint32_t base = var_base(info), deg = var_deg(info);
            const float p3[3] = {prior[3 * v], prior[3 * v + 1], prior[3 * v + 2]};
            float lam[4];
            qubit_lambdas(p3, var_labels_present(info), lam);
            for (uint32_t j = 0; j < deg; ++j) msg[(size_t)(base + j) * 64] = clampf(lam[var_lab(info, j)], C);
            float s3[3], a3[3];
            qubit_state_init(variant, p3, s3, a3);
            if (keep_q)
                for (int x = 0; x < 3; ++x) st[(size_t)(3 * v + x) * 64] = s3[x];
            if (keep_acc)
                for (int x = 0; x < 3; ++x) acc[(size_t)(3 * v + x) * 64] = a3[x];
        }
    }

    if (have) {
        for (int t = a.t0 + 1; t <= a.t_end; ++t) {
            uint32_t sw = 0;
            if (!a.serial && t == a.t_end && t < a.max_iter) {
                // last iteration of the block for the shots still here (t is the same
                // for every active lane): take the new columns, one atomic per wavefront
                const uint64_t live = __ballot(1);
                const int leader = __ffsll((long long)live) - 1;
                unsigned b0 = 0;
                if (lane == leader) b0 = atomicAdd(a.dst_count, (unsigned)__popcll(live));
                b0 = (unsigned)__shfl((int)b0, leader, 64);
                const unsigned dcol = b0 + (unsigned)__popcll(live & ((1ull << lane) - 1ull));
                uint32_t *drec = a.dst + (size_t)(dcol >> 6) * items * 64 + (dcol & 63u);
                wmsg = reinterpret_cast<float *>(drec);
                wst = reinterpret_cast<float *>(drec + (size_t)a.lay.st_off * 64);
                wacc = reinterpret_cast<float *>(drec + (size_t)a.lay.acc_off * 64);
                uint32_t *dsb = drec + (size_t)a.lay.sb_off * 64;
                for (int k = 0; k < (m + 31) / 32; ++k) dsb[(size_t)k * 64] = sb[(size_t)k * 64];
                moved = dcol;
            }
            if (!a.serial) {
                // ---- Horizontal update (eq. h_update) ----------------------------------
                // kChunk checks at a time: all their message loads are issued before the
                // first update, so each wavefront keeps several HBM requests in flight.
                // Padding edges (degree-3 checks) read +inf without touching memory.
                for (int c0 = 0; c0 < m; c0 += kChunk) {
                    if ((c0 & 31) == 0) sw = sb[(size_t)(c0 >> 5) * 64];
                    float mv[kChunk][4];
                    uint32_t cw[kChunk][4];
    #pragma unroll
                    for (int k = 0; k < kChunk; ++k)
    #pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            cw[k][j] = c0 + k < m ? cedge[kMaxCheckDeg * (c0 + k) + j] : edge_pad_word(0);
                            mv[k][j] = edge_is_pad(cw[k][j]) ? INFINITY : msg[(size_t)edge_slot(cw[k][j]) * 64];
                        }
    #pragma unroll
                    for (int k = 0; k < kChunk; ++k) {
                        if (c0 + k >= m) break;
                        float out[4];
                        check_update(mv[k], sw >> ((c0 + k) & 31), C, out);
    #pragma unroll
                        for (int j = 0; j < 4; ++j)
                            if (!edge_is_pad(cw[k][j])) wmsg[(size_t)edge_slot(cw[k][j]) * 64] = out[j];
                    }
                }
                // ---- Posterior, hard decision, vertical update --------------------------
                for (int v0 = 0; v0 < n; v0 += kChunk) {
                    uint32_t info[kChunk];
                    float mc[kChunk][4], s3[kChunk][3], a3[kChunk][3];
    #pragma unroll
                    for (int k = 0; k < kChunk; ++k) {
                        const bool in = v0 + k < n;
                        info[k] = in ? vinfo[v0 + k] : 0u;   // degree 0 past the end
                        const uint32_t base = var_base(info[k]), deg = var_deg(info[k]);
    #pragma unroll
                        for (int j = 0; j < 4; ++j) mc[k][j] = (uint32_t)j < deg ? wmsg[(size_t)(base + j) * 64] : 0.0f;
    #pragma unroll
                        for (int x = 0; x < 3; ++x) {
                            s3[k][x] = keep_q && in ? st[(size_t)(3 * (v0 + k) + x) * 64] : 0.0f;
                            a3[k][x] = keep_acc && in ? acc[(size_t)(3 * (v0 + k) + x) * 64] : 0.0f;
                        }
                    }
    #pragma unroll
                    for (int k = 0; k < kChunk; ++k) {
                        const int v = v0 + k;
                        if (v >= n) break;
                        const uint32_t base = var_base(info[k]), deg = var_deg(info[k]);
                        float S[4], A[4];
                        label_sums(info[k], mc[k], with_y, variant == BP4_ADAGRAD, S, A);
                        const float p3[3] = {prior[3 * v], prior[3 * v + 1], prior[3 * v + 2]};
                        float qn[3];
                        qubit_posterior(a.vp, t, p3, S, A, s3[k], a3[k], qn);
                        if (keep_q)
                            for (int x = 0; x < 3; ++x) wst[(size_t)(3 * v + x) * 64] = s3[k][x];
                        if (keep_acc)
                            for (int x = 0; x < 3; ++x) wacc[(size_t)(3 * v + x) * 64] = a3[k][x];
                        ehat[(size_t)v * 64] = (uint8_t)decision_byte_of(qn);
                        float lam[4];
                        qubit_lambdas(qn, var_labels_present(info[k]), lam);
    #pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            if ((uint32_t)j >= deg) break;
                            const float out = clampf(lam[var_lab(info[k], j)] - mc[k][j], C);
                            wmsg[(size_t)(base + j) * 64] = out;
                            if (a.mvc_out) {
                                const size_t o = (size_t)shot * a.g.nnz + a.g.vcanon[base + j];
                                a.mvc_out[o] = out;
                                a.mcv_out[o] = mc[k][j];
                            }
                        }
                        if (a.q_out)
                            for (int x = 0; x < 3; ++x) a.q_out[((size_t)shot * n + v) * 3 + x] = qn[x];
                    }
                }
            } else {
                // ---- Serial schedule (Algorithm 1): qubit by qubit in index order ----
                // Each qubit's incoming m_{c->v} are formed from the current m_{v'->c}
                // of the check's other qubits (already updated this iteration for
                // qubits earlier in the sweep); the slots always hold m_{v->c}.
                for (int v = 0; v < n; ++v) {
                    const uint32_t info = vinfo[v];
                    const uint32_t base = var_base(info), deg = var_deg(info);
                    float mc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
                    for (uint32_t j = 0; j < deg; ++j) {
                        const uint32_t slot = base + j;
                        const uint32_t c = vchk[slot];
                        const uint32_t sbit = (sb[(size_t)(c >> 5) * 64] >> (c & 31)) & 1u;
                        float f[4];
                        uint32_t neg = sbit;
#pragma unroll
                        for (int k = 0; k < 4; ++k) {
                            const uint32_t w = cedge[kMaxCheckDeg * c + k];
                            // padding and this qubit's own edge take no part
                            const float x = (edge_is_pad(w) || edge_slot(w) == slot) ? INFINITY
                                                                                      : msg[(size_t)edge_slot(w) * 64];
                            neg ^= x < 0.0f ? 1u : 0u;
                            f[k] = phi(fabsf(x));
                        }
                        const float mag = phi((f[0] + f[1]) + (f[2] + f[3]));
                        mc[j] = clampf(neg ? -mag : mag, C);
                    }
                    float S[4], A[4];
                    label_sums(info, mc, with_y, variant == BP4_ADAGRAD, S, A);
                    const float p3[3] = {prior[3 * v], prior[3 * v + 1], prior[3 * v + 2]};
                    float s3[3] = {0.0f, 0.0f, 0.0f}, a3[3] = {0.0f, 0.0f, 0.0f}, qn[3];
                    if (keep_q)
                        for (int x = 0; x < 3; ++x) s3[x] = st[(size_t)(3 * v + x) * 64];
                    if (keep_acc)
                        for (int x = 0; x < 3; ++x) a3[x] = acc[(size_t)(3 * v + x) * 64];
                    qubit_posterior(a.vp, t, p3, S, A, s3, a3, qn);
                    if (keep_q)
                        for (int x = 0; x < 3; ++x) st[(size_t)(3 * v + x) * 64] = s3[x];
                    if (keep_acc)
                        for (int x = 0; x < 3; ++x) acc[(size_t)(3 * v + x) * 64] = a3[x];
                    ehat[(size_t)v * 64] = (uint8_t)decision_byte_of(qn);
                    float lam[4];
                    qubit_lambdas(qn, var_labels_present(info), lam);
                    for (uint32_t j = 0; j < deg; ++j) {
                        const float out = clampf(lam[var_lab(info, j)] - mc[j], C);
                        msg[(size_t)(base + j) * 64] = out;
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
            // ---- Syndrome test (Algorithm 2) ---------------------------------------
            uint32_t bad = 0;
            for (int c0 = 0; c0 < m; c0 += 2 * kChunk) {
                if ((c0 & 31) == 0) sw = sb[(size_t)(c0 >> 5) * 64];
                uint32_t b[2 * kChunk][4], cw[2 * kChunk][4];
#pragma unroll
                for (int k = 0; k < 2 * kChunk; ++k)
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        cw[k][j] = c0 + k < m ? cedge[kMaxCheckDeg * (c0 + k) + j] : edge_pad_word(0);
                        b[k][j] = edge_is_pad(cw[k][j]) ? 0u : ehat[(size_t)edge_var(cw[k][j]) * 64];
                    }
#pragma unroll
                for (int k = 0; k < 2 * kChunk; ++k) {
                    if (c0 + k >= m) break;
                    uint32_t par = (sw >> ((c0 + k) & 31)) & 1u, any = 0;
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        par ^= (b[k][j] >> edge_lab(cw[k][j])) & 1u;
                        any |= b[k][j];
                    }
                    bad |= par | (any & 1u);
                }
            }
            const bool sat = bad == 0;
            t_end_shot = t;
            if ((a.stop && sat) || (t >= a.max_iter && a.last_attempt)) {
                for (int v = 0; v < n; ++v) a.est[(size_t)shot * n + v] = (uint8_t)decision_pauli(ehat[(size_t)v * 64]);
                a.conv[shot] = sat ? 1 : 0;
                a.iters[shot] = t_before + t;
                if (moved >= 0) a.dst_shot[moved] = -1;   // its new column stays a hole
                done = true;
                break;
            }
        }
    }

    // ---- Survivors: append their columns to the next block's records ------------
    if (moved >= 0) {   // already written there by the block's last iteration
        if (!done) {
            a.dst_shot[moved] = shot;
            a.dst_tb[moved] = t_before;
        }
        return;
    }
    const uint64_t mask = __ballot(!done);
    if (mask == 0) return;
    const unsigned cnt = (unsigned)__popcll(mask);
    const int leader = __ffsll((long long)mask) - 1;
    unsigned base = 0;
    if (lane == leader) base = atomicAdd(a.dst_count, cnt);
    base = (unsigned)__shfl((int)base, leader, 64);
    if (!done) {
        const unsigned dcol = base + (unsigned)__popcll(mask & ((1ull << lane) - 1ull));
        // a shot at the end of an AEWA attempt restarts from the syndrome and the
        // priors: its record is not needed
        if (t_end_shot < a.max_iter) {
            uint32_t *drec = a.dst + (size_t)(dcol >> 6) * items * 64 + (dcol & 63u);
            for (size_t i = 0; i < items; ++i) drec[i * 64] = rec[i * 64];
        }
        a.dst_shot[dcol] = shot;
        // a shot that ran out of iterations goes on to its next AEWA attempt
        a.dst_tb[dcol] = t_end_shot >= a.max_iter ? t_before + t_end_shot : t_before;
    }
}

}  // namespace

size_t soa_lanes(int64_t shots, int32_t requested)
{
    // default: the resident lanes of a full chip at 16 wavefronts per CU
    const int64_t cap = requested > 0 ? requested : (int64_t)256 * 16 * 64;
    int64_t l = shots < cap ? shots : cap;
    l = (l + kSoaBlock - 1) / kSoaBlock * kSoaBlock;
    return (size_t)(l < kSoaBlock ? kSoaBlock : l);
}

static size_t up256(size_t x) { return (x + 255) & ~size_t(255); }

// The device formula of the AEWA discount, evaluated on the host in the same FP32 steps.
static float aewa_alpha_host(float alpha, float alpha_last, int steps, int k)
{
#pragma clang fp contract(off)
    return steps > 1 ? alpha + (alpha_last - alpha) * ((float)k / (float)(steps - 1)) : alpha;
}

// Workspace: two counters, two record buffers, two shot-id arrays, the decisions.
size_t soa_workspace_bytes(int m, int n, int nnz, int variant, int64_t shots, int32_t lanes)
{
    const size_t L = soa_lanes(shots, lanes);
    const SoaLayout lay = soa_layout(m, n, nnz, variant);
    return 256 + 2 * up256(L * (size_t)lay.items * 4) + 4 * up256(L * 4) + up256(L * (size_t)n);
}

hipError_t launch_decode_soa(const GraphView &g, const bp4_params &p, int32_t shots, const float *prior,
                             const uint8_t *synd, uint8_t *est, uint8_t *conv, int32_t *iters, float *q_out,
                             float *mvc_out, float *mcv_out, void *ws, int32_t lanes, int32_t iter_block,
                             int with_y, hipStream_t s)
{
    const size_t L = soa_lanes(shots, lanes);
    const SoaLayout lay = soa_layout(g.m, g.n, g.nnz, p.variant);
    char *w = static_cast<char *>(ws);
    unsigned int *counters = reinterpret_cast<unsigned int *>(w);
    w += 256;
    uint32_t *recs[2];
    recs[0] = reinterpret_cast<uint32_t *>(w);
    w += up256(L * (size_t)lay.items * 4);
    recs[1] = reinterpret_cast<uint32_t *>(w);
    w += up256(L * (size_t)lay.items * 4);
    int32_t *shot_ids[2];
    shot_ids[0] = reinterpret_cast<int32_t *>(w);
    w += up256(L * 4);
    shot_ids[1] = reinterpret_cast<int32_t *>(w);
    w += up256(L * 4);
    int32_t *tbs[2];
    tbs[0] = reinterpret_cast<int32_t *>(w);
    w += up256(L * 4);
    tbs[1] = reinterpret_cast<int32_t *>(w);
    w += up256(L * 4);
    uint8_t *ehat = reinterpret_cast<uint8_t *>(w);

    SoaArgs a;
    a.g = g;
    a.prior = prior;
    a.synd = synd;
    a.est = est;
    a.conv = conv;
    a.iters = iters;
    a.q_out = q_out;
    a.mvc_out = mvc_out;
    a.mcv_out = mcv_out;
    a.ehat = ehat;
    a.max_iter = p.max_iter;
    a.stop = p.stop_on_syndrome ? 1 : 0;
    a.with_y = with_y;
    a.clamp = p.llr_clamp;
    a.vp.variant = p.variant;
    a.vp.g_from_t1 = p.adagrad_g_from_t1;
    a.vp.alpha = p.alpha;
    a.vp.gamma = p.gamma;
    a.vp.eps = p.eps;
    a.lay = lay;
    a.serial = p.serial;
    const int32_t B = iter_block > 0 ? iter_block : kSoaIterBlock;
    // AEWA runs its attempts one after another over the shots still unsolved
    const int32_t attempts = p.variant == BP4_AEWA ? p.alpha_steps : 1;
    for (int64_t first = 0; first < shots; first += (int64_t)L) {
        const int32_t cnt = (int32_t)((int64_t)shots - first < (int64_t)L ? (int64_t)shots - first : (int64_t)L);
        const unsigned blocks = (unsigned)((cnt + kSoaBlock - 1) / kSoaBlock);
        a.first_shot = (int32_t)first;
        a.first_count = cnt;
        int cur = 0;
        for (int32_t k = 0; k < attempts; ++k) {
            a.last_attempt = k + 1 == attempts ? 1 : 0;
            if (p.variant == BP4_AEWA) a.vp.alpha = aewa_alpha_host(p.alpha, p.alpha_last, p.alpha_steps, k);
            for (int32_t t0 = 0; t0 < p.max_iter; t0 += B) {
                a.fresh = (k == 0 && t0 == 0) ? 1 : 0;
                a.t0 = t0;
                a.t_end = t0 + B < p.max_iter ? t0 + B : p.max_iter;
                a.src = recs[cur];
                a.dst = recs[cur ^ 1];
                a.src_shot = shot_ids[cur];
                a.dst_shot = shot_ids[cur ^ 1];
                a.src_tb = tbs[cur];
                a.dst_tb = tbs[cur ^ 1];
                a.src_count = counters + cur;
                a.dst_count = counters + (cur ^ 1);
                hipError_t e = launch_zero_u32(counters + (cur ^ 1), 1, s);
                if (e != hipSuccess) return e;
                hipLaunchKernelGGL(decode_soa_kernel, dim3(blocks), dim3(kSoaBlock), 0, s, a);
                e = hipGetLastError();
                if (e != hipSuccess) return e;
                cur ^= 1;
            }
        }
    }
    return hipSuccess;
}

}  // namespace bp4
