// Per-node steps of wide graphs (checks of up to 8 edges, qubits of up to 7, their
// slot labels in a separate word), shared by the LDS and plain kernels.
#pragma once

#include "bp4_math.h"

namespace bp4 {

// Label of slot j from a qubit's label word (2 bits per slot; 0 for unused slots).
__device__ __forceinline__ uint32_t slot_label(uint32_t labw, int j) { return (labw >> (2 * j)) & 3u; }

// Check rule of a wide check (up to 8 edges, padding +inf): as check_update, with
// the leave-one-out sums of phi formed from prefix and suffix sums in edge order.
__device__ __forceinline__ void check_update_wide(const float mv[8], uint32_t s, float C, float out[8])
{
    float f[8];
    uint32_t b[8];
    uint32_t neg = s << 31;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        b[j] = __float_as_uint(mv[j]);
        neg ^= b[j];
        f[j] = phi(fabsf(mv[j]));
    }
    float pre[8], suf[8];
    pre[0] = 0.0f;
#pragma unroll
    for (int j = 1; j < 8; ++j) pre[j] = pre[j - 1] + f[j - 1];
    suf[7] = 0.0f;
#pragma unroll
    for (int j = 6; j >= 0; --j) suf[j] = suf[j + 1] + f[j + 1];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const float mag = phi(pre[j] + suf[j]);
        out[j] = clampf(__uint_as_float(__float_as_uint(mag) ^ ((neg ^ b[j]) & 0x80000000u)), C);
    }
}

// Per-label sums S[lab] of a qubit's incoming messages and of their magnitudes A[lab]
// over its DV slots (label 0 for unused slots), as label_sums.
template <int DV>
__device__ __forceinline__ void label_sums_w(uint32_t labw, const float mc[DV], bool with_y, bool with_abs, float S[4],
                                             float A[4])
{
    S[0] = A[0] = 0.0f;
    float s1 = 0.0f, s2 = 0.0f, s3 = 0.0f;
#pragma unroll
    for (int j = 0; j < DV; ++j) {
        const uint32_t l = slot_label(labw, j);
        s1 += l == 1u ? mc[j] : 0.0f;
        s2 += l == 2u ? mc[j] : 0.0f;
        if (with_y) s3 += l == 3u ? mc[j] : 0.0f;
    }
    S[1] = s1;
    S[2] = s2;
    S[3] = s3;
    float a1 = 0.0f, a2 = 0.0f, a3 = 0.0f;
    if (with_abs) {
#pragma unroll
        for (int j = 0; j < DV; ++j) {
            const uint32_t l = slot_label(labw, j);
            a1 += l == 1u ? fabsf(mc[j]) : 0.0f;
            a2 += l == 2u ? fabsf(mc[j]) : 0.0f;
            a3 += l == 3u ? fabsf(mc[j]) : 0.0f;
        }
    }
    A[1] = a1;
    A[2] = a2;
    A[3] = a3;
}

}  // namespace bp4
