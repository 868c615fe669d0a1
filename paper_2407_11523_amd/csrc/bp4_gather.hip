// Flooding GF(4) BP for large codes in one pass over HBM per iteration.
//
// One lane decodes one shot; the 64 lanes of a workgroup's wavefronts are its 64
// columns, and every wavefront of the workgroup works on the same 64 shots.  Each
// column keeps, in HBM, two records (iterations alternate between them) laid out
// [item][64 lanes]: the check-major message items 4c + p, each holding the stored
// word of m_{v->c} (phi(|m|) with the sign bit of m), then the posterior state
// (and the momentum or AdaGrad accumulator) by walk position.
//
// An iteration walks the qubits in an order fixed on the host (bands of a few
// breadth-first levels, each band walked breadth first along its length, or strips
// of the layout when qubit positions are given), the workgroup's wavefronts taking
// positions round robin, so the qubits in flight at any time sit close together on
// the lattice.  A qubit reads the other stored words of each of
// its checks from the previous record (eq. h_update in phi form: the sign is the
// syndrome bit times the other signs, the magnitude phi of the sum of the other
// phi values, summed in value order), forms its posterior (eqs. p_update, EWAInit,
// mombp1-3, boost), and writes its new posterior and the stored words of its new
// messages m_{v->c} = lambda(Q - m_{c->v}) (eq. v_update) to the other record.
// Each stored word is written once and read by the check's other qubits within a
// short stretch of the walk, so the re-reads are served by L2: HBM sees each
// message read and written once, and the posterior read and written once, per
// iteration (8E + 24N bytes per shot-iteration for EWAInit).
//
// The syndrome test of Algorithm 2 runs in the same pass: for each edge, a ballot
// over the lanes of whether the qubit's decision anticommutes with the edge label
// is XORed into the check's 64-bit parity word in LDS; after the walk every
// check's parity word is compared with its syndrome word.  A column whose shot
// meets the syndrome (or reaches iter_max) writes its decisions and takes the
// next shot from the queue at once; its next iteration reads the initial messages
// lambda(Pi) from a per-code table instead of its record.  Once the queue is empty
// and the live shots fit in columns 0-31, those of columns 32-63 move there (their
// next pass reads the old column and writes the new one) and columns 32-63 stop
// accessing memory, so the workgroup's last passes touch one L2 line of each record
// row instead of two.  Results do not depend on the column a shot
// runs in, the walk order or the workgroup shape, and equal those of the two-phase
// kernels bit for bit (same arithmetic in the same order).
//
// Paper: Chen, Yi, Liang, Wang, "Improved Belief Propagation Decoding
// Algorithms for Surface Codes", section II-B1 (eqs. init, h_update, v_update,
// p_update), section III (eqs. mombp1-3, boost, EWAInit, Algorithm 2).
#include "bp4_math.h"
#include "bp4_gather.h"

namespace bp4 {
namespace {

constexpr uint32_t kSign = 0x80000000u;
// Steps of the walk between two pacing barriers of the workgroup (even; 0: none).
constexpr int kPaceSteps = 4;
// Resident wavefronts per SIMD the kernel is built for (its register budget), and so
// per CU 4 x this many, in workgroups of 64 x gather_waves lanes.  Each wavefront
// has one qubit's reads in flight at a time; eight per SIMD hide the HBM latency
// (measured: a two-deep software pipeline at four per SIMD was slower).
constexpr int kWavesPerSimd = 8;

template <typename T> using konst = const __attribute__((address_space(4))) T;
template <typename T> __device__ __forceinline__ konst<T> *as_const(const T *p) { return (konst<T> *)p; }

// Stored word of a message m: phi(|m|) carrying the sign bit of m.
__device__ __forceinline__ float stored_word(float m)
{
    return __uint_as_float(__float_as_uint(phi(fabsf(m))) | (__float_as_uint(m) & kSign));
}
// The serial schedule's stored word, as the other serial kernels keep it: phi(|m|),
// negated when m < 0 (a -0 message counts as positive).
__device__ __forceinline__ float serial_word(float m)
{
    const float f = phi(fabsf(m));
    return m < 0.0f ? -f : f;
}

struct GatherArgs {
    const uint32_t *cedge;    // [m][4] packed check edges (padding marked)
    const uint32_t *vinfo;    // [n] packed qubit words
    const uint32_t *gord;     // [n] qubit at each walk position (serial schedule: its level order)
    const uint32_t *gedge;    // [n][4] gather words
    const uint32_t *slev;     // serial schedule: [nlev + 1] level offsets into the walk
    int32_t nlev;
    int32_t serial;           // the records hold serial_word values
    const float *prior;       // [n][3]
    float *finit;             // [4m] stored words of the initial messages
    const uint8_t *synd;      // [shots][m]
    uint8_t *est;             // [shots][n]
    uint8_t *conv;            // [shots]
    int32_t *iters;           // [shots]
    unsigned int *head;       // shot queue (zeroed before the launch)
    char *recs;               // [group][2][items][64] words: the two iteration records
    int32_t m, n, shots, max_iter, stop, with_y;
    int32_t st_off, acc_off;  // first posterior and accumulator items
    uint32_t rec_bytes;       // bytes of one record: items x 256
    float clamp;
    VariantParams vp;
    float alpha_last;         // AEWA: discount of the last attempt (vp.alpha: the first)
    int32_t alpha_steps;      // AEWA: attempts
};

// Initial stored words lambda_{H_cv}(Pi_v) of every edge (eq. init), by walk position;
// padding positions of the checks hold +0 (no stored word is +0: |m| <= clamp keeps
// phi(|m|) above phi(clamp) > 0, so +0 marks padding).
__global__ void gather_init_kernel(GatherArgs a)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < a.m)
        for (int p = 0; p < 4; ++p)
            if (edge_is_pad(a.cedge[4 * i + p])) a.finit[4 * i + p] = 0.0f;
    if (i >= a.n) return;
    const uint32_t v = a.gord[i];
    const uint32_t info = a.vinfo[v];
    const float p3[3] = {a.prior[3 * v], a.prior[3 * v + 1], a.prior[3 * v + 2]};
    float lam[4];
    qubit_lambdas(p3, var_labels_present(info), lam);
    const uint32_t deg = var_deg(info);
    for (uint32_t j = 0; j < deg; ++j) {
        const uint32_t w = a.gedge[4 * i + j];
        const float m0 = clampf(lam[var_lab(info, j)], a.clamp);
        a.finit[gather_item(w)] = a.serial ? serial_word(m0) : stored_word(m0);
    }
}

// What the update of one qubit reads: its walk entry (wavefront-uniform) and, per
// lane, the other stored words of each of its checks and its state.
struct QubitIn {
    uint32_t v, info, ew[4];
    float p3[3];
    float x[4][3];
    float s3[3], a3[3];
};

// The workgroup's records through one buffer resource: item i of record r for lane l
// at byte r * rec_bytes + 256 i + 4 l; the per-lane part (record and lane) is the
// vector offset, the item the scalar one, so no address arithmetic runs per lane,
// and an access past the two records reads 0 and writes nothing.
struct Records {
    __amdgpu_buffer_rsrc_t rs;
    __device__ __forceinline__ float ld(uint32_t item, uint32_t voff) const
    {
        return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, (int)voff, (int)(item * 256u), 0));
    }
    // stores are streamed (nontemporal): the next read is a full pass later
    __device__ __forceinline__ void st(uint32_t item, uint32_t voff, float x) const
    {
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(x), rs, (int)voff, (int)(item * 256u), 2);
    }
};

// SER: the serial schedule (Algorithm 1) instead of flooding.  The walk is then the
// level order of the qubit-by-qubit sweep (a level's qubits share no check); a column
// keeps one record, updated in place, and each level ends with a workgroup barrier, so a
// qubit reads the stored words its check's earlier qubits wrote in this sweep and the
// previous sweep's words of the later ones, exactly as the sweep in index order.  In a
// shot's first sweep the words not yet rewritten come from the initial table.
template <int VAR, bool SER>
__global__ void __launch_bounds__(64 * kGatherMaxWaves, kWavesPerSimd) decode_gather_kernel(GatherArgs a)
{
    extern __shared__ uint64_t lds[];
    const int m = a.m, n = a.n;
    uint64_t *S = lds;               // [m] syndrome bit of each column's shot, per check
    uint64_t *P = lds + m;           // [m] parity of the decisions, per check
    uint64_t *U = lds + 2 * m;       // [2] columns failing the test, alternate iterations
    int32_t *col = reinterpret_cast<int32_t *>(lds + 2 * m + 2);   // [64] shot of each column
    int32_t *mig = col + 64;   // [64] column whose shot moves into this one this pass (-1: none)
    const int lane = threadIdx.x & 63;
    // wavefront index, uniform across the wavefront (read from lane 0 so the compiler
    // keeps the walk positions, and every table read and branch on them, scalar)
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int W = blockDim.x >> 6;
    const float C = a.clamp;
    constexpr bool kAcc = VAR == BP4_MOMENTUM || VAR == BP4_ADAGRAD;
    const bool with_y = a.with_y != 0;
    VariantParams vp = a.vp;
    vp.variant = VAR;
    konst<uint32_t> *vinfo = as_const(a.vinfo);
    konst<uint32_t> *gord = as_const(a.gord);
    konst<uint32_t> *gedge = as_const(a.gedge);
    konst<float> *prior = as_const(a.prior);
    konst<float> *finit = as_const(a.finit);

    // Records 0 and 1 alternate between passes.  A new shot's first pass takes the
    // stored words of lambda(Pi) (eq. init) from the per-code table and the variant's
    // starting state instead of its record's contents.  Padding items are +0 in both
    // records and are never written, so the gathers of a degree-3 check read +0 there
    // (phi's identity) without a test.
    Records R;
    R.rs = __builtin_amdgcn_make_buffer_rsrc(a.recs + (size_t)blockIdx.x * 2 * a.rec_bytes, 0,
                                             (int)(2 * a.rec_bytes), 0x00020000);
    const uint32_t lane_off = (uint32_t)lane * 4u;
    // vector offset of an access that must not happen: past both records, it reads 0
    // and writes nothing (the range check of the buffer resource)
    constexpr uint32_t no_off = 0x80000000u;
    for (int i = wv; i < 4 * m; i += W) {
        if (__float_as_uint(finit[i]) == 0u) {   // padding
            R.st((uint32_t)i, lane_off, 0.0f);
            R.st((uint32_t)i, lane_off + a.rec_bytes, 0.0f);
        }
    }
    for (int c = threadIdx.x; c < m; c += blockDim.x) {
        S[c] = 0;
        P[c] = 0;
    }
    if (threadIdx.x < 64) col[threadIdx.x] = -1;
    if (threadIdx.x == 0) U[0] = U[1] = 0;
    __syncthreads();

    int shot = -1, t = 0, cur = 0;
    // AEWA: the column's attempt, the iterations of its earlier attempts and its discount
    int att = 0, t_before = 0;
    float alpha = a.vp.alpha;
    // Record parity from the workgroup's pass count, the same in every lane (a lane's
    // own iteration count would split a wavefront's accesses over both records):
    // every live column advances one iteration per pass, so the record a pass writes
    // is the one the next pass reads; a new shot reads the initial record instead.
    uint32_t pass = 0;
    bool finish = false;
    bool drained = false;            // wavefront 0: the queue is empty
    for (;;) {
        // ---- columns without a shot take the next ones from the queue ------------------
        if (wv == 0) {
            const bool want = shot < 0 || finish;
            const uint64_t wm = __ballot(want);
            int ns = want ? -1 : shot;
            const bool was_drained = drained;
            if (wm != 0 && !drained) {
                const unsigned cnt = (unsigned)__popcll(wm);
                unsigned base = 0;
                if (lane == 0) base = atomicAdd(a.head, cnt);
                base = (unsigned)__shfl((int)base, 0, 64);
                const unsigned r = base + (unsigned)__popcll(wm & ((1ull << lane) - 1ull));
                if (want && r < (unsigned)a.shots) ns = (int)r;
                drained = base + cnt >= (unsigned)a.shots;
            }
            // Once the queue is empty, the live shots of columns 32-63 move to empty
            // columns 0-31 as soon as they all fit there (the r-th live upper column to
            // the r-th empty lower one): the upper half of every record row, one L2 line,
            // then goes untouched for the rest of the launch.  (Flooding only: the serial
            // sweep's single record is read and rewritten within the pass.)
            int from = -1;
            const uint64_t live = __ballot(ns >= 0);
            if (!SER && was_drained && (live >> 32) != 0 && __popcll(live) <= 32) {
                if (lane < 32 && ns < 0) {
                    const uint64_t holes = ~live & 0xFFFFFFFFull;
                    const int r = __popcll(holes & ((1ull << lane) - 1ull));
                    uint64_t up = live >> 32;
                    if (r < __popcll(up)) {
                        for (int k = 0; k < r; ++k) up &= up - 1ull;
                        from = 32 + __builtin_ctzll(up);
                    }
                }
                const int moved = __shfl(ns, from >= 0 ? from : lane, 64);
                if (from >= 0) ns = moved;
                if (lane >= 32) ns = -1;   // the live upper shots number at most the lower holes
            }
            col[lane] = ns;
            mig[lane] = from;
        }
        __syncthreads();
        const int ns = col[lane];
        const int from = mig[lane];
        const bool refill = ns >= 0 && from < 0 && (shot < 0 || finish);
        {   // a column taking over a moved shot takes its iteration state too
            const int sl = from >= 0 ? from : lane;
            const int t2 = __shfl(t, sl, 64), att2 = __shfl(att, sl, 64), tb2 = __shfl(t_before, sl, 64);
            const float alpha2 = __shfl(alpha, sl, 64);
            if (from >= 0) {
                t = t2;
                att = att2;
                t_before = tb2;
                alpha = alpha2;
            }
        }
        shot = ns;
        finish = false;
        if (__ballot(shot >= 0) == 0) break;   // every column empty (the same in every wavefront)
        if (refill) {
            t = 0;
            att = 0;
            t_before = 0;
            alpha = a.vp.alpha;
        }
        if constexpr (VAR == BP4_AEWA) vp.alpha = alpha;   // per column
        const bool moving = __ballot(from >= 0) != 0;
        // syndrome words of the new and the moved shots
        if (__ballot(refill) != 0 || moving) {
            for (int c = wv; c < m; c += W) {
                uint32_t bit = (uint32_t)(S[c] >> (from >= 0 ? from : lane)) & 1u;
                if (refill) bit = a.synd[(size_t)shot * m + c] & 1u;
                const uint64_t word = __ballot(bit);
                if (lane == 0) S[c] = word;
            }
        }
        __syncthreads();
        ++t;

        // ---- one flooding iteration over the walk ------------------------------------
        const bool fresh = t == 1;
        // A moved shot's pass reads its old column and writes its new one.  Columns
        // 32-63 read and write nothing once all of them are empty; a column without a
        // shot otherwise reads and writes its own column like the others (masking single
        // lanes would leave partly written L2 lines, which measured slower).
        const uint32_t rcol = from >= 0 ? (uint32_t)from * 4u : lane_off;
        const bool skip = lane >= 32 && (__ballot(shot >= 0) >> 32) == 0;
        const uint32_t rd = skip ? no_off : rcol + (SER ? 0u : (pass & 1u) * a.rec_bytes);
        const uint32_t wr = skip ? no_off : lane_off + (SER ? 0u : ((pass + 1u) & 1u) * a.rec_bytes);
        ++pass;
        uint64_t nan_cols = 0;
        // Reads of a qubit: its walk entry (scalar), the other stored words of each of
        // its checks and its state.
        auto load_qubit = [&](int i, QubitIn &q) {
            q.v = gord[i];
            q.info = vinfo[q.v];
#pragma unroll
            for (int j = 0; j < 4; ++j) q.ew[j] = gedge[4 * i + j];
#pragma unroll
            for (int k = 0; k < 3; ++k) q.p3[k] = prior[3 * q.v + k];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const uint32_t item = gather_item(q.ew[j]);
                const uint32_t c4 = item & ~3u, p = item & 3u;
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    // the k-th position of the check other than p (k, or k + 1 past p)
                    const uint32_t pk = (uint32_t)k + (((p - (uint32_t)k - 1u) >> 31) & 1u);
                    q.x[j][k] = R.ld(c4 + pk, rd);
                }
            }
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                q.s3[k] = VAR != BP4_BP ? R.ld(a.st_off + 3 * i + k, rd) : 0.0f;
                q.a3[k] = kAcc ? R.ld(a.acc_off + 3 * i + k, rd) : 0.0f;
            }
        };
        // Update of a qubit from its reads: incoming messages, posterior, parity
        // contributions, outgoing messages; writes to the record the pass writes.
        auto update_qubit = [&](int i, QubitIn &q) {
            const uint32_t deg = var_deg(q.info);
            // check-to-qubit messages (eq. h_update); slots past the degree give 0
            float mc[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const uint32_t item = gather_item(q.ew[j]);
                const uint32_t c4 = item & ~3u, p = item & 3u, c = item >> 2;
                const uint32_t sb = (uint32_t)(S[c] >> lane) & 1u;
                // a new shot's words come from the initial table (a per-lane select after
                // the loads: a per-lane branch would split them)
                float x[3];
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const uint32_t pk = (uint32_t)k + (((p - (uint32_t)k - 1u) >> 31) & 1u);
                    // serial: a word an earlier qubit of this sweep rewrote is read from the record
                    const bool init = fresh && (!SER || ((q.ew[j] >> (kGatherEarlierShift + k)) & 1u) == 0u);
                    x[k] = init ? finit[c4 + pk] : q.x[j][k];
                }
                const uint32_t sgn =
                    ((__float_as_uint(x[0]) ^ __float_as_uint(x[1]) ^ __float_as_uint(x[2])) & kSign) ^ (sb << 31);
                float mag;
                if constexpr (SER) {
                    // the serial kernels' sum over the check's four positions in order, this
                    // qubit's own position (p) contributing 0: the k-th other word sits at
                    // position k below p and k + 1 above it
                    const float f0 = p == 0u ? 0.0f : fabsf(x[0]);
                    const float f1 = p == 1u ? 0.0f : fabsf(x[p < 1u ? 0 : 1]);
                    const float f2 = p == 2u ? 0.0f : fabsf(x[p < 2u ? 1 : 2]);
                    const float f3 = p == 3u ? 0.0f : fabsf(x[2]);
                    mag = phi((f0 + f1) + (f2 + f3));
                } else {
                    mag = phi(sum3_canonical(fabsf(x[0]), fabsf(x[1]), fabsf(x[2])));
                }
                mc[j] = (uint32_t)j < deg ? clampf(__uint_as_float(__float_as_uint(mag) ^ sgn), C) : 0.0f;
            }
            float S4[4], A4[4], qn[3];
            float s3[3], a3[3];
            qubit_state_init(VAR, q.p3, s3, a3);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                s3[k] = fresh ? s3[k] : q.s3[k];
                a3[k] = fresh ? a3[k] : q.a3[k];
            }
            label_sums(q.info, mc, with_y, VAR == BP4_ADAGRAD, S4, A4);
            qubit_posterior(vp, t, q.p3, S4, A4, s3, a3, qn);
            // every variant keeps its posterior state (BP its posterior, for the decisions)
#pragma unroll
            for (int k = 0; k < 3; ++k) R.st(a.st_off + 3 * i + k, wr, VAR == BP4_BP ? qn[k] : s3[k]);
            if (kAcc) {
#pragma unroll
                for (int k = 0; k < 3; ++k) R.st(a.acc_off + 3 * i + k, wr, a3[k]);
            }
            // this qubit's share of every check's parity (Algorithm 2)
            const uint32_t db = decision_byte_of(qn);
            nan_cols |= __ballot(db & 1u);
            float lam[4];
            qubit_lambdas(qn, var_labels_present(q.info), lam);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if ((uint32_t)j >= deg) break;
                const uint32_t lab = var_lab(q.info, j);
                const uint64_t flip = __ballot((db >> lab) & 1u);
                if (flip != 0 && lane == 0)
                    atomicXor(reinterpret_cast<unsigned long long *>(&P[gather_item(q.ew[j]) >> 2]),
                              (unsigned long long)flip);
                // new message (eq. v_update) and its stored word
                const float out = clampf(lam[lab] - mc[j], C);
                R.st(gather_item(q.ew[j]), wr, SER ? serial_word(out) : stored_word(out));
            }
        };
        // The walk.  Step s takes positions s W .. s W + W - 1, one per wavefront; every
        // kPaceSteps steps the wavefronts meet at a barrier, so they stay within a
        // few steps of each other and the re-reads of a check by its other qubits
        // still find it in L2.
        QubitIn qa;
        if constexpr (SER) {
            // level by level, a workgroup barrier (with its memory fences) after each
            konst<uint32_t> *slev = as_const(a.slev);
            for (int l = 0; l < a.nlev; ++l) {
                const int p1 = (int)slev[l + 1];
                for (int i = (int)slev[l] + wv; i < p1; i += W) {
                    load_qubit(i, qa);
                    update_qubit(i, qa);
                }
                __syncthreads();
            }
        } else {
            const int steps = (n + W - 1) / W;
            for (int st = 0; st < steps; ++st) {
                const int i0 = st * W + wv;
                if (i0 < n) {
                    load_qubit(i0, qa);
                    update_qubit(i0, qa);
                }
                if (kPaceSteps > 0 && (st + 1) % kPaceSteps == 0) __builtin_amdgcn_s_barrier();
            }
        }
        __syncthreads();

        // ---- syndrome test -------------------------------------------------------------
        uint64_t bad = nan_cols;
        for (int c = wv; c < m; c += W) {
            bad |= P[c] ^ S[c];
            if (lane == 0) P[c] = 0;
        }
        if (lane == 0 && bad != 0) atomicOr(reinterpret_cast<unsigned long long *>(&U[cur]), (unsigned long long)bad);
        __syncthreads();
        const bool sat = ((U[cur] >> lane) & 1ull) == 0;
        // AEWA: a column whose attempt ends unsolved starts the next attempt of its shot
        // (eq. EWAInit with the next discount, from the initial messages again)
        bool restart = false;
        if constexpr (VAR == BP4_AEWA) restart = shot >= 0 && !sat && t >= a.max_iter && att + 1 < a.alpha_steps;
        finish = shot >= 0 && !restart && ((a.stop && sat) || t >= a.max_iter);
        if (__ballot(finish) != 0) {
            // hard decisions of the finished shots from the posterior just written
            for (int i = wv; i < n; i += W) {
                if (!finish) continue;
                const uint32_t v = gord[i];
                float q[3];
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const float sv = R.ld(a.st_off + 3 * i + k, wr);
                    q[k] = VAR == BP4_ADAGRAD ? prior[3 * v + k] + sv : sv;
                }
                a.est[(size_t)shot * n + v] = (uint8_t)decision_pauli(decision_byte_of(q));
            }
            if (wv == 0 && finish) {
                a.conv[shot] = sat ? 1 : 0;
                a.iters[shot] = t_before + t;
            }
        }
        if (restart) {
            t_before += t;
            ++att;
            alpha = aewa_alpha(a.vp.alpha, a.alpha_last, a.alpha_steps, att);
            t = 0;   // the next pass is the attempt's first: fresh reads, as for a new shot
        }
        if (threadIdx.x == 0) U[cur ^ 1] = 0;
        cur ^= 1;
    }
}

size_t up256(size_t x) { return (x + 255) & ~size_t(255); }

int32_t record_items(int m, int n, int variant, int32_t *st_off, int32_t *acc_off)
{
    int32_t o = 4 * m;
    *st_off = o;
    o += 3 * n;
    *acc_off = o;
    if (variant == BP4_MOMENTUM || variant == BP4_ADAGRAD) o += 3 * n;
    return o;
}

int32_t waves_of(int32_t waves) { return waves > 0 ? waves : kGatherDefaultWaves; }

}  // namespace

size_t gather_lds_bytes(int m) { return (size_t)(2 * m + 2) * 8 + 128 * 4; }

bool gather_supported(int m, int variant, int serial, bool wide, size_t max_lds)
{
    (void)variant;
    (void)serial;
    return !wide && gather_lds_bytes(m) <= max_lds;
}

int32_t gather_groups(int64_t shots, int32_t waves)
{
    const int64_t per_cu = 4 * kWavesPerSimd / waves_of(waves);   // workgroups per CU
    const int64_t cap = (int64_t)kGatherCUs * (per_cu > 0 ? per_cu : 1);
    const int64_t need = (shots + 63) / 64;
    const int64_t g = need < cap ? need : cap;
    return (int32_t)(g > 0 ? g : 1);
}

// Workspace: the queue head, the initial-message table, the column records (two per
// workgroup).
size_t gather_workspace_bytes(int m, int n, int variant, int64_t shots, int32_t waves)
{
    int32_t st_off, acc_off;
    const size_t items = (size_t)record_items(m, n, variant, &st_off, &acc_off);
    return 256 + up256((size_t)4 * m * 4) + (size_t)gather_groups(shots, waves) * 2 * items * 256;
}

hipError_t launch_decode_gather(const GraphView &g, const GatherTables &gt, const bp4_params &p, int32_t shots,
                                const float *prior, const uint8_t *synd, uint8_t *est, uint8_t *conv,
                                int32_t *iters, void *ws, int32_t waves, int with_y, hipStream_t s)
{
    GatherArgs a;
    const bool ser = p.serial != 0;
    a.cedge = g.cedge;
    a.vinfo = g.vinfo;
    a.gord = ser ? gt.sord : gt.gord;
    a.gedge = ser ? gt.sgedge : gt.gedge;
    a.slev = gt.slev;
    a.nlev = gt.nlev;
    a.serial = ser ? 1 : 0;
    a.prior = prior;
    char *w = static_cast<char *>(ws);
    a.head = reinterpret_cast<unsigned int *>(w);
    w += 256;
    a.finit = reinterpret_cast<float *>(w);
    w += up256((size_t)4 * g.m * 4);
    a.recs = w;
    a.synd = synd;
    a.est = est;
    a.conv = conv;
    a.iters = iters;
    a.m = g.m;
    a.n = g.n;
    a.shots = shots;
    a.max_iter = p.max_iter;
    a.stop = p.stop_on_syndrome ? 1 : 0;
    a.with_y = with_y;
    const int32_t items = record_items(g.m, g.n, p.variant, &a.st_off, &a.acc_off);
    a.rec_bytes = (uint32_t)items * 256u;
    a.clamp = p.llr_clamp;
    a.vp.variant = p.variant;
    a.vp.g_from_t1 = p.adagrad_g_from_t1;
    a.vp.alpha = p.alpha;
    a.vp.gamma = p.gamma;
    a.vp.eps = p.eps;
    a.alpha_last = p.alpha_last;
    a.alpha_steps = p.alpha_steps;

    hipError_t e = launch_zero_u32(a.head, 1, s);
    if (e != hipSuccess) return e;
    const int init_threads = g.n > g.m ? g.n : g.m;
    hipLaunchKernelGGL(gather_init_kernel, dim3((unsigned)((init_threads + 255) / 256)), dim3(256), 0, s, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int32_t W = waves_of(waves);
    const dim3 grid((unsigned)gather_groups(shots, waves)), block((unsigned)(64 * W));
    const size_t lds = gather_lds_bytes(g.m);
#define BP4_GATHER_LAUNCH(V)                                                                    \
    do {                                                                                        \
        if (ser) hipLaunchKernelGGL(HIP_KERNEL_NAME(decode_gather_kernel<V, true>), grid, block, lds, s, a);  \
        else hipLaunchKernelGGL(HIP_KERNEL_NAME(decode_gather_kernel<V, false>), grid, block, lds, s, a);     \
    } while (0)
    switch (p.variant) {
    case BP4_BP: BP4_GATHER_LAUNCH(BP4_BP); break;
    case BP4_MOMENTUM: BP4_GATHER_LAUNCH(BP4_MOMENTUM); break;
    case BP4_ADAGRAD: BP4_GATHER_LAUNCH(BP4_ADAGRAD); break;
    case BP4_AEWA: BP4_GATHER_LAUNCH(BP4_AEWA); break;
    default: BP4_GATHER_LAUNCH(BP4_EWAINIT); break;
    }
#undef BP4_GATHER_LAUNCH
    return hipGetLastError();
}

}  // namespace bp4
