// mlp_tile.h -- forward pass of the scheduling MLP (16 -> 64 -> 64 -> 1) for 16
// pairs at a time on one wave, with the weights as ready-made MFMA fragments
// in LDS (one 8-byte read per operand).
//
// v_mfma_f32_16x16x16_bf16 lane layout (lane l, r = l % 16, g = 4 (l / 16),
// j = 0..3): A[r][g + j], B[g + j][r], D[g + j][r].  Both layers are computed
// transposed -- H1^T = W1^T X^T and Z2^T = W2^T H1^T -- so that the first
// layer's D fragment (rows g + j of H1^T, column r) is exactly the second
// layer's B fragment, and no activation passes through LDS.  Weights and
// activations are bf16, accumulation float32; biases, the last layer and the
// normalization stay float32.
#pragma once

#include "ccd_internal.h"

namespace ccd {

typedef short mlp_bf16x4 __attribute__((ext_vector_type(4)));
typedef float mlp_f32x4 __attribute__((ext_vector_type(4)));

constexpr int kMlpOffW1 = 0;
constexpr int kMlpOffB1 = kMlpOffW1 + kNumFeatures * kHidden;
constexpr int kMlpOffW2 = kMlpOffB1 + kHidden;
constexpr int kMlpOffB2 = kMlpOffW2 + kHidden * kHidden;
constexpr int kMlpOffW3 = kMlpOffB2 + kHidden;
constexpr int kMlpOffB3 = kMlpOffW3 + kHidden;

// float -> bf16, round to nearest even (v_cvt_pk_bf16_f32)
__device__ __forceinline__ short mlp_bf16(float x) { return __builtin_bit_cast(short, (__bf16)x); }

// max(x, 0) for finite x: the sign bit spread into a mask (fmaxf would also
// quiet NaNs, one more instruction per value)
__device__ __forceinline__ float mlp_relu(float x)
{
    const int i = __float_as_int(x);
    return __int_as_float(i & ~(i >> 31));
}

// Weight fragments, per lane: frag[ob] = block ob of W1^T, frag[4 + 4 ob + kb]
// = block (ob, kb) of W2^T (LDS, 10 KB).
struct MlpWeights {
    mlp_bf16x4 frag[20][64];
};

// Per-workgroup constants (LDS).
struct MlpConsts {
    float b1[kHidden], b2[kHidden], w3[kHidden];
    float mean[kNumFeatures], istd[kNumFeatures];
    float b3;
};

// Fragment idx = 64 fr + lane of the weights (bf16 x 4).
__device__ __forceinline__ mlp_bf16x4 mlp_fragment(const float *__restrict__ prm, int idx)
{
    const int fr = idx >> 6, lane = idx & 63;
    const int r = lane & 15, g = (lane >> 4) * 4;
    mlp_bf16x4 v;
    if (fr < 4) {
#pragma unroll
        for (int j = 0; j < 4; j++) v[j] = mlp_bf16(prm[kMlpOffW1 + (g + j) * kHidden + 16 * fr + r]);
    } else {
        const int ob = (fr - 4) >> 2, kb = (fr - 4) & 3;
#pragma unroll
        for (int j = 0; j < 4; j++) v[j] = mlp_bf16(prm[kMlpOffW2 + (16 * kb + g + j) * kHidden + 16 * ob + r]);
    }
    return v;
}

// Block-wide: fills W, from the float32 parameters, or (packed != nullptr)
// by copying fragments packed once for the call (the caller synchronizes
// before use).
__device__ __forceinline__ void mlp_load_weights(MlpWeights &W, const float *__restrict__ prm,
                                                 const mlp_bf16x4 *__restrict__ packed = nullptr)
{
    for (int idx = threadIdx.x; idx < 20 * 64; idx += blockDim.x)
        W.frag[idx >> 6][idx & 63] = packed ? packed[idx] : mlp_fragment(prm, idx);
}

// Block-wide: fills C (the caller synchronizes before use).
__device__ __forceinline__ void mlp_load_consts(MlpConsts &C, const float *__restrict__ prm,
                                                const float *__restrict__ norm)
{
    for (int i = threadIdx.x; i < kHidden; i += blockDim.x) {
        C.b1[i] = prm[kMlpOffB1 + i];
        C.b2[i] = prm[kMlpOffB2 + i];
        C.w3[i] = prm[kMlpOffW3 + i];
    }
    for (int i = threadIdx.x; i < kNumFeatures; i += blockDim.x) {
        C.mean[i] = norm[i];
        C.istd[i] = norm[kNumFeatures + i];
    }
    if (threadIdx.x == 0) C.b3 = prm[kMlpOffB3];
}

// The layer-1 B fragment: features g .. g + 3 of the tile's row r, normalized
// and rounded to bf16.
__device__ __forceinline__ mlp_bf16x4 mlp_input(const MlpConsts &C, const float f[4], int lane)
{
    const int g = (lane >> 4) * 4;
    mlp_bf16x4 x;
#pragma unroll
    for (int j = 0; j < 4; j++) x[j] = mlp_bf16((f[j] - C.mean[g + j]) * C.istd[g + j]);
    return x;
}

// Prediction for the tile's row r = lane % 16 (every lane of a row holds it).
__device__ __forceinline__ float mlp_forward(const MlpWeights &W, const MlpConsts &C, mlp_bf16x4 x, int lane)
{
    const int g = (lane >> 4) * 4;
    mlp_bf16x4 h1[4];
#pragma unroll
    for (int ob = 0; ob < 4; ob++) {
        mlp_f32x4 acc;
#pragma unroll
        for (int j = 0; j < 4; j++) acc[j] = C.b1[16 * ob + g + j];
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(W.frag[ob][lane], x, acc, 0, 0, 0);
#pragma unroll
        for (int j = 0; j < 4; j++) h1[ob][j] = mlp_bf16(mlp_relu(acc[j]));
    }
    float s = 0.f;
#pragma unroll
    for (int ob = 0; ob < 4; ob++) {
        mlp_f32x4 acc;
#pragma unroll
        for (int j = 0; j < 4; j++) acc[j] = C.b2[16 * ob + g + j];
#pragma unroll
        for (int kb = 0; kb < 4; kb++)
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(W.frag[4 + 4 * ob + kb][lane], h1[kb], acc, 0, 0, 0);
#pragma unroll
        for (int j = 0; j < 4; j++) s += mlp_relu(acc[j]) * C.w3[16 * ob + g + j];
    }
    s += __shfl_xor(s, 16);
    s += __shfl_xor(s, 32);
    return s + C.b3;
}

// Bin of a predicted cost for the schedule's ordering: 256 bins of 1/4 in
// log2 cost, costliest first.  The clamp is done in float before the
// conversion (a float -> int conversion of NaN or of a value out of range is
// undefined); NaN goes to the last bin.
__device__ __forceinline__ int sched_cost_bin(float c)
{
    float x = c * 4.f;
    x = x == x ? fminf(fmaxf(x, 0.f), 255.f) : 0.f;
    return 255 - (int)x;
}

}  // namespace ccd
