// Error sampling, syndromes and logical-error bookkeeping on the GPU (integer
// work, bit-exact).  Section IV of the paper: i.i.d. Pauli errors per qubit;
// success iff the residual E^ E lies in the stabilizer group.
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

// One thread per (shot, check): s_c = sum over the check's edges of <H_cv, E_v> mod 2.
__global__ void __launch_bounds__(256)
syndrome_kernel(GraphView g, int32_t shots, const uint8_t *err, uint8_t *synd)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)shots * g.m) return;
    const int64_t shot = idx / g.m;
    const int c = (int)(idx - shot * g.m);
    const uint8_t *row = err + (size_t)shot * g.n;
    uint32_t par = 0;
    for (int j = 0; j < g.cstride; ++j) {   // padding words carry label 0
        const uint32_t w = g.cedge[c * g.cstride + j];
        if (edge_is_pad(w)) continue;
        par ^= anticomm(edge_lab(w), row[edge_var(w)]);
    }
    synd[idx] = (uint8_t)par;
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
    const int n = g.n;
    for (int i = threadIdx.x; i < rows * n; i += blockDim.x) {
        const size_t off = (size_t)first * n + i;
        res[i] = (err[off] ^ est[off]) & 3u;
    }
    for (int i = threadIdx.x; i < rows; i += blockDim.x) flags[i] = 0;
    if (threadIdx.x < 3) cnt[threadIdx.x] = 0;
    __syncthreads();
    // residual syndrome: "detected" when R anticommutes with a stabilizer
    for (int i = threadIdx.x; i < rows * g.m; i += blockDim.x) {
        const int sh = i / g.m, c = i - sh * g.m;
        uint32_t par = 0;
        for (int j = 0; j < g.cstride; ++j) {
            const uint32_t w = g.cedge[c * g.cstride + j];
            if (edge_is_pad(w)) continue;
            par ^= anticomm(edge_lab(w), res[sh * n + edge_var(w)]);
        }
        if (par) atomicOr(&flags[sh], 1u);
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

}  // namespace

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
    const int64_t work2 = (int64_t)shots * g.m;
    if (work2 == 0) return hipSuccess;
    hipLaunchKernelGGL(syndrome_kernel, dim3((unsigned)((work2 + 255) / 256)), dim3(256), 0, s,
                       g, shots, err, synd);
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
