// mlp_device.h -- the warm-start network on one wavefront's 64 observations
// with gfx950 BF16 matrix cores (v_mfma_f32_16x16x32_bf16, FP32 accumulate).
//
// Network: 26 -> 128 -> GELU -> 128 -> GELU -> 12 (inputs padded to 32,
// outputs to 16).  Every layer is computed transposed, out^T = W^T in^T, so
// the weight rows are the MFMA A operand (read from LDS, shared by the
// workgroup) and the activations of the wave's 64 observations are the B
// operand (read from the wave's LDS tile [64][kActS], observation-major).
// Lane l = 16 g + i of a 16x16x32 MFMA holds A[i][8g..8g+7], B[8g..8g+7][i]
// and D[4g..4g+3][i]; the epilogue writes D back into the same tile (all B
// operands are loaded first).
#pragma once
#include "dba_internal.h"

namespace dba {
namespace dev {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// LDS row strides (bf16 elements); the +8 keeps 16-byte row reads of
// neighbouring lanes on distinct banks
constexpr int kWs1 = kInPad + 8;     // W1^T rows: 32 inputs
constexpr int kWs2 = kHid + 8;       // W2^T, W3^T, W2, rows of 128
constexpr int kWs3 = kOutPad * 2 + 8;  // W3 rows (backward): 16 outputs padded to 32
constexpr int kActS = kHid + 8;      // activation tile row stride
constexpr int kLdsW1 = kHid * kWs1;
constexpr int kLdsW2 = kHid * kWs2;
constexpr int kLdsW3T = kOutPad * kWs2;
constexpr int kLdsFwd = kLdsW1 + kLdsW2 + kLdsW3T;   // forward weights in LDS (bf16 elements)
constexpr int kLdsAct = 64 * kActS;                  // one wave's activation tile

__device__ __forceinline__ float gelu_f(float z, float *grad)
{
    // tanh form; tanh(u) = 1 - 2 / (1 + e^{2u})
    const float z2 = z * z;
    const float u = 0.7978845608028654f * (z + 0.044715f * z2 * z);
    const float e = __expf(2.0f * u);
    const float t = 1.0f - 2.0f * __builtin_amdgcn_rcpf(1.0f + e);
    if (grad) *grad = 0.5f * (1.0f + t) + 0.5f * z * (1.0f - t * t) * 0.7978845608028654f * (1.0f + 0.134145f * z2);
    return 0.5f * z * (1.0f + t);
}

// Copies a dense [rows][cols] bf16 matrix into LDS with row stride ls
// (cols a multiple of 8), cooperatively by the whole workgroup.
__device__ __forceinline__ void stage_rows(const __bf16 *g, __bf16 *l, int rows, int cols, int ls)
{
    const int per = cols >> 3;
    for (int q = threadIdx.x; q < rows * per; q += blockDim.x) {
        const int r = q / per, c = (q - r * per) << 3;
        *reinterpret_cast<bf16x8 *>(l + r * ls + c) = *reinterpret_cast<const bf16x8 *>(g + (size_t)r * cols + c);
    }
}

// Stages the forward weights (W1^T, W2^T, W3^T) of the packed weight block.
__device__ __forceinline__ void stage_forward_weights(const __bf16 *w, __bf16 *lw)
{
    stage_rows(w + kOffW1T, lw, kHid, kInPad, kWs1);
    stage_rows(w + kOffW2T, lw + kLdsW1, kHid, kHid, kWs2);
    stage_rows(w + kOffW3T, lw + kLdsW1 + kLdsW2, kOutPad, kHid, kWs2);
}

// One dense layer, transposed, for the wave's 64 observations: for unit
// tile u (16 output units) and observation tile t, epi(u, acc) receives
// acc[t][r] = out[obs 16t + i][unit 16u + 4g + r].
template <int MT, int KS, typename Epi>
__device__ __forceinline__ void dense64(const __bf16 *W, int ws, const __bf16 *in, int as, int lane, Epi epi)
{
    const int g = lane >> 4, i = lane & 15;
    bf16x8 b[KS][4];
#pragma unroll
    for (int k = 0; k < KS; ++k)
#pragma unroll
        for (int t = 0; t < 4; ++t)
            b[k][t] = *reinterpret_cast<const bf16x8 *>(in + (16 * t + i) * as + 32 * k + 8 * g);
#pragma unroll 2
    for (int u = 0; u < MT; ++u) {
        f32x4 acc[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int k = 0; k < KS; ++k) {
            const bf16x8 a = *reinterpret_cast<const bf16x8 *>(W + (16 * u + i) * ws + 32 * k + 8 * g);
#pragma unroll
            for (int t = 0; t < 4; ++t) acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[k][t], acc[t], 0, 0, 0);
        }
        epi(u, acc);
    }
}

// Hidden-layer epilogue: + bias, GELU, round to bf16, write back into the
// tile; optionally also store gelu'(z) and the bf16 activation to global
// rows (training forward).
struct HiddenEpi {
    __bf16 *act;
    const float *bias;
    int lane;
    float *gp;            // [64][kHid] global rows or nullptr
    __bf16 *hg;           // [64][kHid] global rows or nullptr
    __device__ __forceinline__ void operator()(int u, const f32x4 *acc) const
    {
        const int g = lane >> 4, i = lane & 15;
        const int unit = 16 * u + 4 * g;
        const float b0 = bias[unit], b1 = bias[unit + 1], b2 = bias[unit + 2], b3 = bias[unit + 3];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int row = 16 * t + i;
            float gr[4];
            bf16x4 h;
            h[0] = (__bf16)gelu_f(acc[t][0] + b0, gp ? &gr[0] : nullptr);
            h[1] = (__bf16)gelu_f(acc[t][1] + b1, gp ? &gr[1] : nullptr);
            h[2] = (__bf16)gelu_f(acc[t][2] + b2, gp ? &gr[2] : nullptr);
            h[3] = (__bf16)gelu_f(acc[t][3] + b3, gp ? &gr[3] : nullptr);
            *reinterpret_cast<bf16x4 *>(act + row * kActS + unit) = h;
            if (gp) *reinterpret_cast<float4 *>(gp + (size_t)row * kHid + unit) = make_float4(gr[0], gr[1], gr[2], gr[3]);
            if (hg) *reinterpret_cast<bf16x4 *>(hg + (size_t)row * kHid + unit) = h;
        }
    }
};

// Output-layer epilogue: + bias, FP32 result into out[64][kOutPad].
struct OutEpi {
    float *out;
    const float *bias;
    int lane;
    __device__ __forceinline__ void operator()(int, const f32x4 *acc) const
    {
        const int g = lane >> 4, i = lane & 15;
#pragma unroll
        for (int t = 0; t < 4; ++t)
            *reinterpret_cast<float4 *>(out + (16 * t + i) * kOutPad + 4 * g) =
                make_float4(acc[t][0] + bias[4 * g], acc[t][1] + bias[4 * g + 1], acc[t][2] + bias[4 * g + 2],
                            acc[t][3] + bias[4 * g + 3]);
    }
};

// Full forward pass of the wave tile.  On entry act[row][0..31] holds the
// bf16 standardized inputs; on exit out[row][0..15] the (standardized)
// outputs.  `out` may alias act (the output layer reads all of act first).
__device__ __forceinline__ void mlp_forward64(const __bf16 *lw, const MlpParams &mp, __bf16 *act, float *out, int lane,
                                              float *gp1 = nullptr, __bf16 *h1 = nullptr, float *gp2 = nullptr,
                                              __bf16 *h2 = nullptr)
{
    dense64<kHid / 16, 1>(lw, kWs1, act, kActS, lane, HiddenEpi{act, mp.b1, lane, gp1, h1});
    dense64<kHid / 16, 4>(lw + kLdsW1, kWs2, act, kActS, lane, HiddenEpi{act, mp.b2, lane, gp2, h2});
    dense64<1, 4>(lw + kLdsW1 + kLdsW2, kWs2, act, kActS, lane, OutEpi{out, mp.b3, lane});
}

}  // namespace dev
}  // namespace dba
