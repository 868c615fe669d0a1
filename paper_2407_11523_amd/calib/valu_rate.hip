// VALU issue-rate calibration for the decode kernels' roofline: the rate at which
// one GPU issues plain (non-packed) FP32 adds and fused multiply-adds, and the
// hardware base-2 exponential and logarithm, in lane-operations per second.
// Each lane runs 8 independent dependency chains, so latency is hidden and the
// rate is the issue throughput.  Prints one JSON line.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

#define CHECK(x)                                                                         \
    do {                                                                                 \
        hipError_t e_ = (x);                                                             \
        if (e_ != hipSuccess) {                                                          \
            std::fprintf(stderr, "HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__); \
            std::exit(1);                                                                \
        }                                                                                \
    } while (0)

namespace {

constexpr int kIters = 2048;
constexpr int kChains = 8;

enum Kind { kAdd = 0, kFma = 1, kExp = 2, kLog = 3 };

template <int K>
__global__ void __launch_bounds__(256) rate_kernel(float *out, float a, float b)
{
    float x[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k) x[k] = 1.0f + threadIdx.x * 1e-6f + k * 1e-3f;
    for (int i = 0; i < kIters; ++i) {
#pragma unroll
        for (int k = 0; k < kChains; ++k) {
            if (K == kAdd) x[k] = x[k] + a;
            if (K == kFma) x[k] = fmaf(x[k], a, b);
            if (K == kExp) x[k] = __builtin_amdgcn_exp2f(-x[k]) * a;     // exp2 + one multiply
            if (K == kLog) x[k] = __builtin_amdgcn_logf(x[k]) + b;       // log2 + one add
        }
    }
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < kChains; ++k) s += x[k];
    out[blockIdx.x * 256 + threadIdx.x] = s;
}

template <int K>
double lane_ops_per_s(float *out, int grid, float a, float b)
{
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    hipLaunchKernelGGL(rate_kernel<K>, dim3(grid), dim3(256), 0, 0, out, a, b);
    CHECK(hipGetLastError());
    CHECK(hipDeviceSynchronize());
    const int reps = 5;
    CHECK(hipEventRecord(e0, 0));
    for (int r = 0; r < reps; ++r) hipLaunchKernelGGL(rate_kernel<K>, dim3(grid), dim3(256), 0, 0, out, a, b);
    CHECK(hipEventRecord(e1, 0));
    CHECK(hipEventSynchronize(e1));
    float ms = 0.0f;
    CHECK(hipEventElapsedTime(&ms, e0, e1));
    CHECK(hipEventDestroy(e0));
    CHECK(hipEventDestroy(e1));
    return (double)reps * grid * 256.0 * kIters * kChains / (ms * 1e-3);
}

}  // namespace

int main()
{
    hipDeviceProp_t p;
    CHECK(hipGetDeviceProperties(&p, 0));
    const int grid = p.multiProcessorCount * 16;
    float *out = nullptr;
    CHECK(hipMalloc(&out, (size_t)grid * 256 * sizeof(float)));
    const double add = lane_ops_per_s<kAdd>(out, grid, 0.999f, 0.001f);
    const double fma = lane_ops_per_s<kFma>(out, grid, 0.999f, 0.001f);
    const double ex = lane_ops_per_s<kExp>(out, grid, 0.999f, 0.001f);
    const double lg = lane_ops_per_s<kLog>(out, grid, 0.999f, 4.0f);
    CHECK(hipFree(out));
    // a transcendental's cost in FP32-op issue slots: the exp/log loop issues one
    // transcendental and one plain op per element
    const double t_exp = fma / ex - 1.0, t_log = fma / lg - 1.0;
    std::printf("{\"device\": \"%s\", \"cus\": %d, \"add_lane_ops_per_s\": %.4e, \"fma_lane_ops_per_s\": %.4e, "
                "\"exp2_plus_mul_per_s\": %.4e, \"log2_plus_add_per_s\": %.4e, \"exp2_slots\": %.3f, "
                "\"log2_slots\": %.3f}\n",
                p.gcnArchName, p.multiProcessorCount, add, fma, ex, lg, t_exp, t_log);
    return 0;
}
