// Error sampling, syndromes and logical-error bookkeeping on the GPU (integer
// work, bit-exact).  Section IV of the paper: i.i.d. Pauli errors per qubit;
// success iff the residual E^ E lies in the stabilizer group.  Also the prior
// LLRs of the noise model (section II-B1).
#include "bp4_internal.h"

namespace bp4 {
namespace {

// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 64-bit
// multiplications with the published multipliers, key bumped by the published
// Weyl constants after each round.
__device__ __forceinline__ void philox4x64_10(uint64_t x[4], uint64_t k0, uint64_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t a = x[0], c = x[2];
        const uint64_t lo0 = a * 0xD2E7470EE14C6C93ull, hi0 = __umul64hi(a, 0xD2E7470EE14C6C93ull);
        const uint64_t lo1 = c * 0xCA5A826395121157ull, hi1 = __umul64hi(c, 0xCA5A826395121157ull);
        const uint64_t y0 = hi1 ^ x[1] ^ k0;
        const uint64_t y2 = hi0 ^ x[3] ^ k1;
        x[0] = y0;
        x[1] = lo1;
        x[2] = y2;
        x[3] = lo0;
        k0 += 0x9E3779B97F4A7C15ull;
        k1 += 0xBB67AE8584CAA73Bull;
    }
}

__device__ __forceinline__ uint32_t anticomm(uint32_t a, uint32_t b)
{
    return ((a & (b >> 1)) ^ ((a >> 1) & b)) & 1u;
}

// One thread per (shot, block of 8 qubits): one Philox call gives 8 32-bit words.
__global__ void __launch_bounds__(256)
sample_errors_kernel(int32_t n, int32_t shots, int64_t shot0, uint32_t t0, uint32_t t1, uint32_t t2,
                     uint64_t seed, uint64_t stream_id, uint8_t *err)
{
    const int blocks = (n + 7) / 8;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)shots * blocks) return;
    const int64_t shot = idx / blocks;
    const int blk = (int)(idx - shot * blocks);
    uint64_t x[4] = {(uint64_t)(shot0 + shot), (uint64_t)blk, 0ull, 0ull};
    philox4x64_10(x, seed, stream_id);
    const uint64_t c0 = t0, c1 = c0 + t1, c2 = c1 + t2;
    uint8_t *row = err + (size_t)shot * n;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int q = blk * 8 + j;
        if (q >= n) break;
        const uint64_t u = (j & 1) ? (x[j >> 1] >> 32) : (x[j >> 1] & 0xFFFFFFFFull);
        row[q] = u < c0 ? 1 : (u < c1 ? 3 : (u < c2 ? 2 : 0));
    }
}

// Tiles of shots: a workgroup stages `rows` consecutive shots' bytes of one or two
// [shots][n] arrays in LDS (XOR of the two when both are given), as 4-byte words
// where the source is aligned and single bytes at the two ends.  dst[i] for
// i < rows * n holds byte first * n + i.
__device__ __forceinline__ void stage_rows(uint8_t *dst, const uint8_t *a, const uint8_t *b, size_t first_byte,
                                           int len)
{
    const uint8_t *pa = a + first_byte;
    const uint8_t *pb = b ? b + first_byte : nullptr;
    // bytes before the first 4-byte boundary of the source, then whole words, then the rest
    int head = (int)((4u - (uint32_t)((uintptr_t)pa & 3u)) & 3u);
    if (head > len) head = len;
    const int words = (len - head) >> 2;
    for (int i = threadIdx.x; i < head; i += blockDim.x) dst[i] = pb ? (uint8_t)(pa[i] ^ pb[i]) : pa[i];
    const uint32_t *wa = reinterpret_cast<const uint32_t *>(pa + head);
    const bool b_aligned = pb && (((uintptr_t)(pb + head) & 3u) == 0);
    for (int i = threadIdx.x; i < words; i += blockDim.x) {
        uint32_t v = wa[i];
        if (pb) {
            if (b_aligned) {
                v ^= reinterpret_cast<const uint32_t *>(pb + head)[i];
            } else {
                const uint8_t *q = pb + head + 4 * i;
                v ^= (uint32_t)q[0] | ((uint32_t)q[1] << 8) | ((uint32_t)q[2] << 16) | ((uint32_t)q[3] << 24);
            }
        }
        uint8_t *d = dst + head + 4 * i;
        d[0] = (uint8_t)v;
        d[1] = (uint8_t)(v >> 8);
        d[2] = (uint8_t)(v >> 16);
        d[3] = (uint8_t)(v >> 24);
    }
    for (int i = head + 4 * words + (int)threadIdx.x; i < len; i += blockDim.x)
        dst[i] = pb ? (uint8_t)(pa[i] ^ pb[i]) : pa[i];
}

// Symplectic product of check c with the Pauli row `row` (bytes per qubit): the
// check's edge words are read as 16-byte vectors; padding words carry label 0.
__device__ __forceinline__ uint32_t check_parity(const GraphView &g, int c, const uint8_t *row)
{
    uint32_t par = 0;
    for (int q = 0; q < g.cstride; q += 4) {
        const uint4 w4 = *reinterpret_cast<const uint4 *>(g.cedge + (size_t)c * g.cstride + q);
        const uint32_t w[4] = {w4.x, w4.y, w4.z, w4.w};
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (!edge_is_pad(w[j])) par ^= anticomm(edge_lab(w[j]), row[edge_var(w[j])]);
    }
    return par;
}

// Walk over the (shot, check) items of a tile: item tid, tid + B, ... of the
// flattened rows * m list, advanced by carries instead of a division per item.
struct RowWalk {
    int sh, c;
};

// Syndromes of a tile of shots: s_c = sum over the check's edges of <H_cv, E_v> mod 2.
__global__ void __launch_bounds__(256)
syndrome_kernel(GraphView g, int32_t shots, int tile, const uint8_t *err, uint8_t *synd)
{
    extern __shared__ uint8_t rows_lds[];   // [tile][n]
    const int64_t first = (int64_t)blockIdx.x * tile;
    const int rows = (int)((shots - first) < tile ? (shots - first) : tile);
    const int n = g.n, m = g.m;
    stage_rows(rows_lds, err, nullptr, (size_t)first * n, rows * n);
    __syncthreads();
    uint8_t *out = synd + (size_t)first * m;
    const int B = (int)blockDim.x, q = B / m, rem = B - q * m;
    RowWalk w{(int)threadIdx.x / m, (int)threadIdx.x % m};
    for (; w.sh < rows;) {
        out[w.sh * m + w.c] = (uint8_t)check_parity(g, w.c, rows_lds + w.sh * n);
        w.sh += q;
        w.c += rem;
        if (w.c >= m) {
            w.c -= m;
            w.sh += 1;
        }
    }
}

// Bookkeeping: a block takes a tile of shots, stages R = E^ xor E in LDS, then
// evaluates every (shot, check) and (shot, logical) symplectic product.
constexpr int kBkBlock = 256;

__global__ void __launch_bounds__(kBkBlock)
bookkeep_kernel(GraphView g, int32_t shots, int tile, const uint8_t *err, const uint8_t *est,
                uint8_t *fail, unsigned long long *counts)
{
    extern __shared__ uint8_t sm[];
    uint8_t *res = sm;                                   // [tile][n]
    unsigned int *flags = reinterpret_cast<unsigned int *>(sm + ((size_t)tile * g.n + 3) / 4 * 4);
    __shared__ unsigned int cnt[3];
    const int64_t first = (int64_t)blockIdx.x * tile;
    const int rows = (int)((shots - first) < tile ? (shots - first) : tile);
    const int n = g.n, m = g.m;
    // bit 0: x part, bit 1: z part of the residual (decision bytes hold only those)
    stage_rows(res, err, est, (size_t)first * n, rows * n);
    for (int i = threadIdx.x; i < rows; i += blockDim.x) flags[i] = 0;
    if (threadIdx.x < 3) cnt[threadIdx.x] = 0;
    __syncthreads();
    // residual syndrome: "detected" when R anticommutes with a stabilizer
    {
        const int B = (int)blockDim.x, q = B / m, rem = B - q * m;
        RowWalk w{(int)threadIdx.x / m, (int)threadIdx.x % m};
        uint32_t bad = 0;
        int cur = w.sh;
        for (; w.sh < rows;) {
            if (w.sh != cur) {
                if (bad) atomicOr(&flags[cur], 1u);
                bad = 0;
                cur = w.sh;
            }
            bad |= check_parity(g, w.c, res + w.sh * n);
            w.sh += q;
            w.c += rem;
            if (w.c >= m) {
                w.c -= m;
                w.sh += 1;
            }
        }
        if (bad && cur < rows) atomicOr(&flags[cur], 1u);
    }
    // logical class: "undetected" when R anticommutes with a logical operator
    for (int i = threadIdx.x; i < rows * g.nlog; i += blockDim.x) {
        const int sh = i / g.nlog, k = i - sh * g.nlog;
        uint32_t par = 0;
        for (uint32_t e = g.lptr[k]; e < g.lptr[k + 1]; ++e) {
            const uint32_t w = g.lent[e];
            par ^= anticomm(w >> 16, res[sh * n + (w & 0xFFFFu)]);
        }
        if (par) atomicOr(&flags[sh], 2u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < rows; i += blockDim.x) {
        const unsigned int f = flags[i];
        const unsigned int kind = (f & 1u) ? 1u : ((f & 2u) ? 2u : 0u);
        fail[first + i] = (uint8_t)kind;
        atomicAdd(&cnt[kind], 1u);
    }
    __syncthreads();
    if (threadIdx.x < 3 && cnt[threadIdx.x]) atomicAdd(&counts[threadIdx.x], (unsigned long long)cnt[threadIdx.x]);
}

__global__ void zero_u32_kernel(unsigned int *p, int count)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0u;
}

// Prior LLRs of section II-B1, one thread per qubit: Pi_W = ln p_I - ln p_W with
// p_I = 1 - (p_X + p_Y + p_Z), in double precision, rounded to float once.  An
// impossible entry (p_W <= 0, p_I <= 0, or a non-finite probability) is NaN.
__global__ void __launch_bounds__(256) prior_llr_kernel(int32_t n, const double *probs, float *prior)
{
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const double px = probs[3 * v], py = probs[3 * v + 1], pz = probs[3 * v + 2];
    const double pi = 1.0 - ((px + py) + pz);
    const bool ok = isfinite(px) && isfinite(py) && isfinite(pz) && px > 0.0 && py > 0.0 && pz > 0.0 && pi > 0.0;
    const double lpi = log(pi);
    prior[3 * v] = ok ? (float)(lpi - log(px)) : __builtin_nanf("");
    prior[3 * v + 1] = ok ? (float)(lpi - log(py)) : __builtin_nanf("");
    prior[3 * v + 2] = ok ? (float)(lpi - log(pz)) : __builtin_nanf("");
}

}  // namespace

hipError_t launch_prior_llr(int32_t n, const double *probs, float *prior, hipStream_t s)
{
    hipLaunchKernelGGL(prior_llr_kernel, dim3((n + 255) / 256), dim3(256), 0, s, n, probs, prior);
    return hipGetLastError();
}

hipError_t launch_sample(const GraphView &g, int32_t shots, int64_t shot0, const uint32_t thr[3],
                         uint64_t seed, uint64_t stream_id, uint8_t *err, uint8_t *synd,
                         hipStream_t s)
{
    if (shots == 0) return hipSuccess;
    const int64_t work = (int64_t)shots * ((g.n + 7) / 8);
    hipLaunchKernelGGL(sample_errors_kernel, dim3((unsigned)((work + 255) / 256)), dim3(256), 0, s,
                       g.n, shots, shot0, thr[0], thr[1], thr[2], seed, stream_id, err);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (g.m == 0) return hipSuccess;
    // shots per workgroup: their error rows fill at most 16 KB of LDS
    int tile = 16384 / (g.n > 0 ? g.n : 1);
    if (tile > 64) tile = 64;
    if (tile < 1) tile = 1;
    const int64_t blocks = ((int64_t)shots + tile - 1) / tile;
    hipLaunchKernelGGL(syndrome_kernel, dim3((unsigned)blocks), dim3(256), (size_t)tile * g.n, s, g, shots, tile,
                       err, synd);
    return hipGetLastError();
}

hipError_t launch_bookkeep(const GraphView &g, int32_t shots, const uint8_t *err, const uint8_t *est,
                           uint8_t *fail, int64_t *counts, hipStream_t s)
{
    if (shots == 0) return hipSuccess;
    int tile = 16384 / g.n;
    if (tile > 64) tile = 64;
    if (tile < 1) tile = 1;
    const size_t lds = ((size_t)tile * g.n + 3) / 4 * 4 + (size_t)tile * 4;
    const int64_t blocks = (shots + tile - 1) / tile;
    hipLaunchKernelGGL(bookkeep_kernel, dim3((unsigned)blocks), dim3(kBkBlock), lds, s, g, shots, tile,
                       err, est, fail, reinterpret_cast<unsigned long long *>(counts));
    return hipGetLastError();
}

hipError_t launch_zero_u32(unsigned int *p, int count, hipStream_t s)
{
    hipLaunchKernelGGL(zero_u32_kernel, dim3((count + 255) / 256), dim3(256), 0, s, p, count);
    return hipGetLastError();
}

}  // namespace bp4
