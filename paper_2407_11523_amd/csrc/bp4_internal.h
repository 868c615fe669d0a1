// Internal declarations shared by the host ABI layer and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bp4.h"

namespace bp4 {

// Compiled degree limits of the padded (ELL) edge lists: narrow graphs (every check
// and qubit of degree <= 4, all kernels) and wide graphs (checks of degree <= 8,
// qubits of degree <= 7; the LDS flooding kernel, the sampler and bookkeeping).
constexpr int kMaxCheckDeg = 4;
constexpr int kMaxVarDeg = 4;
constexpr int kMaxCheckDegWide = 8;
// Lanes per workgroup of the LDS kernel (block slots share them; group_lanes 128,
// 256 and 512 mean 4, 2 and 1 block slots).
constexpr int kLdsBlock = 512;
constexpr int kMaxVarDegWide = 7;
constexpr int kMaxVars = 16383;      // 14-bit qubit index in a packed check edge
constexpr int kMaxEdges = 65534;     // 16-bit message slot; slot nnz is the padding slot

// Packed check-side edge word: bits 0-15 message slot (variable-major position of
// the edge), bits 16-29 qubit index, bits 30-31 Pauli label (1 X, 2 Z, 3 Y).  A
// check with fewer than kMaxCheckDeg edges is padded with the word nnz: label 0
// (the identity, which commutes with every error), qubit 0, message slot nnz.
__host__ __device__ inline uint32_t edge_pad_word(int nnz) { return (uint32_t)nnz; }
__host__ __device__ inline bool edge_is_pad(uint32_t w) { return (w >> 30) == 0u; }
__host__ __device__ inline uint32_t edge_slot(uint32_t w) { return w & 0xFFFFu; }
__host__ __device__ inline uint32_t edge_var(uint32_t w) { return (w >> 16) & 0x3FFFu; }
__host__ __device__ inline uint32_t edge_lab(uint32_t w) { return w >> 30; }

// Packed qubit word: bits 0-15 first message slot, bits 16-18 degree, bits 20+2j
// the label of the qubit's j-th edge (edges in increasing check order; narrow graphs
// only: a wide graph keeps them in the label word vlab, bits 2j), bits 28-30 the
// labels present (bit 28 + label - 1).
__host__ __device__ inline uint32_t var_base(uint32_t w) { return w & 0xFFFFu; }
__host__ __device__ inline uint32_t var_deg(uint32_t w) { return (w >> 16) & 7u; }
__host__ __device__ inline uint32_t var_lab(uint32_t w, int j) { return (w >> (20 + 2 * j)) & 3u; }
// bit (label) set for each label present: 2 X, 4 Z, 8 Y
__host__ __device__ inline uint32_t var_labels_present(uint32_t w) { return (w >> 27) & 0xEu; }

// Device view of an uploaded graph image.
struct GraphView {
    const uint32_t *cedge;   // [m][kMaxCheckDeg] packed check edges, padded (edge_pad_word)
    const uint32_t *vinfo;   // [n] packed qubit words
    const uint32_t *vcanon;  // [nnz] canonical (row-major) edge id of each message slot
    const uint32_t *vchk;    // [nnz] check of each message slot
    const uint32_t *sord;    // [n] qubits in serial-schedule levels (level, then index)
    const uint32_t *slev;    // [nlev + 1] level offsets into sord
    const uint32_t *vlab;    // [n] wide graphs: labels of each qubit's slots, 2 bits each
    const uint32_t *lptr;    // [nlog + 1] offsets into lent
    const uint32_t *lent;    // logical supports: qubit | (Pauli << 16)
    int32_t m, n, nnz, nlog, nlev;
    int32_t cstride;         // edge words per check: kMaxCheckDeg (narrow) or kMaxCheckDegWide (wide)
};

struct DecodeArgs {
    GraphView g;
    const float *prior;      // [n][3]
    const uint8_t *synd;     // [shots][m]
    uint8_t *est;            // [shots][n]
    uint8_t *conv;           // [shots]
    int32_t *iters;          // [shots]
    float *q_out;            // optional [shots][n][3]
    float *mvc_out;          // optional [shots][nnz] canonical order
    float *mcv_out;          // optional [shots][nnz]
    unsigned int *counter;   // shot queue head (zeroed before launch)
    int32_t shots;
    int32_t variant, max_iter, stop, g_from_t1;
    float alpha, gamma, eps, clamp;
    float alpha_last;        // AEWA: discount of the last attempt
    int32_t alpha_steps;     // AEWA: attempts
    // LDS layout (words): workgroup-static part, then one region per shot group
    // or shot slot
    int32_t static_words, region_words, q_off, acc_off, ehat_off, syn_off, hdr_off;
    int32_t group_lanes;     // wave groups: lanes per shot (4, ..., 64); block slots: 256
    int32_t block_shots;     // block slots: shots per workgroup (0: wave groups)
    uint32_t magic_m, magic_n;   // ceil(2^32 / m), ceil(2^32 / n): item -> slot
    int32_t with_y;          // the code has Y entries
    int32_t serial;          // serial schedule (Algorithm 1) on wave groups
    int32_t wide;            // wide graph (cstride 8, labels in vlab)
    int32_t css22;           // X/Z labels only, at most two of each per qubit: the LDS
                             // kernel keeps a qubit's X messages at positions 0-1 and its Z
                             // messages at 2-3 (unused positions hold 0)
};

// Codes of one persistent launch, decoded in this order (largest first).
constexpr int kMaxMixedCodes = 16;
struct MixedArgs {
    int32_t ncodes;
    DecodeArgs codes[kMaxMixedCodes];
};

// LDS layout of the small-code kernel for one code, variant and lane mapping:
// wave groups of G lanes per shot (S = 0) or S block slots sharing 256 lanes.
struct LdsLayout {
    int32_t static_words = 0, region_words = 0, q_off = 0, acc_off = 0, ehat_off = 0, syn_off = 0, hdr_off = 0;
    int32_t group_lanes = 0, block_shots = 0, block = 0;
    size_t bytes = 0;        // dynamic LDS bytes per workgroup
};
struct LaneChoice {
    int32_t group_lanes = -1, block_shots = 0;
};

LdsLayout decode_lds_layout(int m, int n, int nnz, int variant, int group_lanes, int block_shots,
                            bool wide = false);
// Serial schedule: wave groups of G in {1, ..., 64} lanes; static part adds the
// slot -> check table and the level order, regions hold signed phi values.
LdsLayout decode_lds_serial_layout(int m, int n, int nnz, int nlev, int variant, int group_lanes, bool wide);
// The mapping is valid for the code: G a power of two in [4, 64] with at most 64
// checks per lane, or 1 <= S <= 256 with at most 64 check items per lane.
bool decode_lds_fits(int m, int n, int group_lanes, int block_shots);
LaneChoice decode_lds_pick(int m, int n, int nnz, int variant, size_t max_lds, bool wide = false, int64_t shots = 0);
hipError_t launch_decode_lds(const MixedArgs &args, size_t lds_bytes, hipStream_t s, int *grid_out);

hipError_t launch_sample(const GraphView &g, int32_t shots, int64_t shot0, const uint32_t thr[3],
                         uint64_t seed, uint64_t stream_id, uint8_t *err, uint8_t *synd,
                         hipStream_t s);
hipError_t launch_bookkeep(const GraphView &g, int32_t shots, const uint8_t *err,
                           const uint8_t *est, uint8_t *fail, int64_t *counts, hipStream_t s);
hipError_t launch_zero_u32(unsigned int *p, int count, hipStream_t s);
// bp4_decode_mixed with its shot-queue heads at `counters` (device, >= ncodes words):
// validates, clears the heads with a fill kernel and launches.  Returns a BP4_ code.
int decode_mixed_with(int32_t ncodes, const bp4_code_batch *codes, unsigned int *counters, void *stream);
// Records the calling thread's error message (with the HIP error's text unless e is
// hipSuccess) and returns `code`.
int report_error(int code, const char *what, hipError_t e = hipSuccess);
hipError_t launch_prior_llr(int32_t n, const double *probs, float *prior, hipStream_t s);

size_t plain_workspace_bytes(int n, int nnz, int variant, int64_t shots);

// Lanes (= shots in flight) of the SOA kernel: `requested` (0: default) capped by
// the shot count, rounded up to whole workgroups.
size_t soa_lanes(int64_t shots, int32_t requested);
size_t soa_workspace_bytes(int m, int n, int nnz, int variant, int64_t shots, int32_t lanes);
// Iterations per SOA launch between compactions of the live shots (default).
constexpr int32_t kSoaIterBlock = 24;
hipError_t launch_decode_soa(const GraphView &g, const bp4_params &p, int32_t shots, const float *prior,
                             const uint8_t *synd, uint8_t *est, uint8_t *conv, int32_t *iters, float *q_out,
                             float *mvc_out, float *mcv_out, void *ws, int32_t lanes, int32_t iter_block,
                             int with_y, hipStream_t s);
// Unrolled EWAInit / Momentum forward and adjoint (fixed T, checkpoints every K
// iterations); variant BP4_EWAINIT (param [T]) or BP4_MOMENTUM (param [T][2]).
struct UnrolledSizes {
    size_t saved;   // checkpoints written by the forward, read by the adjoint
    size_t ws;      // segment states, adjoint record, per-wavefront partial sums
};
UnrolledSizes unrolled_sizes(int m, int n, int nnz, int variant, int32_t T, int32_t K, int64_t shots);
hipError_t launch_unrolled_forward(const GraphView &g, int variant, int32_t T, int32_t K, float clamp, int32_t shots,
                                   const float *param, const float *prior, const uint8_t *synd, const uint8_t *err,
                                   double *loss, float *q_out, void *saved, void *ws, hipStream_t s);
hipError_t launch_unrolled_backward(const GraphView &g, int variant, int32_t T, int32_t K, float clamp, int32_t shots,
                                    const float *param, const float *prior, const uint8_t *synd, const uint8_t *err,
                                    const float *dloss, const void *saved, double *dparam, double *dprior, void *ws,
                                    hipStream_t s);

// The large-code kernel is the automatic choice when even 256-lane groups need more
// than this much LDS per workgroup (fewer than two workgroups per CU).
constexpr size_t kLdsAutoLimit = 81920;
hipError_t run_plain(const GraphView &g, const bp4_params &p, int32_t shots, const float *prior,
                     const uint8_t *synd, uint8_t *est, uint8_t *conv, int32_t *iters, void *ws,
                     hipStream_t s, int32_t *iterations_run);

}  // namespace bp4
