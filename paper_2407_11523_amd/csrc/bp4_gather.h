// Internal declarations of the single-pass HBM decode kernel (large codes).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "bp4.h"
#include "bp4_internal.h"

namespace bp4 {

// Gather edge word of the qubit at one position of the walk, one per edge slot j of
// the qubit (slots in increasing check order, as in the packed qubit word):
// bits 0-19 the edge's check-major message item 4c + p (p: the edge's position in
// check c), bits 20-23 the padding positions of check c (bit k: position k holds no
// edge), bit 31 set for slots j >= the qubit's degree (the rest of the word is then
// 0x00F00000: check 0, all positions padding).  Serial walk only: bits 24-26, bit
// 24 + k set when the k-th other position of the check (k, or k + 1 past p) belongs
// to a qubit of a lower level, i.e. one the sweep has already updated.
constexpr uint32_t kGatherAbsent = 0x80F00000u;
constexpr int kGatherEarlierShift = 24;
__host__ __device__ inline uint32_t gather_item(uint32_t w) { return w & 0xFFFFFu; }
__host__ __device__ inline uint32_t gather_pad(uint32_t w) { return (w >> 20) & 0xFu; }

// Device tables of the walks: gord[i] the qubit at position i of the flooding walk,
// gedge[4 i + j] its gather words; the serial schedule's walk sord (qubits by level),
// its gather words sgedge and its level offsets slev[0 .. nlev].
struct GatherTables {
    const uint32_t *gord;
    const uint32_t *gedge;
    const uint32_t *sord;
    const uint32_t *sgedge;
    const uint32_t *slev;
    int32_t nlev;
};

// Host: what the walk builder reads of a narrow graph (packed check edges [m][cstride],
// first message slot of each qubit [n + 1], check of each slot [nnz], position of each
// slot's edge in its check [nnz]).
struct GatherWalkInput {
    int n, m, cstride;
    const uint32_t *cedge;
    const int32_t *vptr;
    const uint32_t *vchk;
    const int32_t *cpos;
};
// Host: the walk order (gord [n]) and its gather words (gedge [4n]); xy: qubit positions
// [n][2] or NULL.
void build_gather_walk(const GatherWalkInput &in, const int32_t *xy, std::vector<uint32_t> &gord,
                       std::vector<uint32_t> &gedge);

// Wavefronts per workgroup: all of them walk the qubits of the same 64 shots.
constexpr int kGatherDefaultWaves = 16;
constexpr int kGatherMaxWaves = 16;
// CUs the persistent grid is sized for.
constexpr int kGatherCUs = 256;

// Whether the kernel takes this code, variant and schedule: flooding (every variant,
// AEWA restarts included), check and qubit degrees <= 4 and the two per-check bit
// masks within the workgroup's LDS (max_lds bytes).
bool gather_supported(int m, int variant, int serial, bool wide, size_t max_lds);
// LDS bytes per workgroup.
size_t gather_lds_bytes(int m);
// Workgroups (64 shots each) in flight for `shots` shots and `waves` wavefronts
// per workgroup (0: default).
int32_t gather_groups(int64_t shots, int32_t waves);
size_t gather_workspace_bytes(int m, int n, int variant, int64_t shots, int32_t waves);
hipError_t launch_decode_gather(const GraphView &g, const GatherTables &gt, const bp4_params &p, int32_t shots,
                                const float *prior, const uint8_t *synd, uint8_t *est, uint8_t *conv,
                                int32_t *iters, void *ws, int32_t waves, int with_y, hipStream_t s);

}  // namespace bp4
