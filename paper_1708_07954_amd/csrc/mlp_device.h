// mlp_device.h -- the warm-start network on one wavefront's 64 observations
// with gfx950 BF16 matrix cores (v_mfma_f32_16x16x32_bf16, FP32 accumulate).
//
// Network: 26 -> 128 -> GELU -> 128 -> GELU -> 12 (inputs padded to 32,
// outputs to 16).  Every layer is computed transposed, out^T = W^T in^T, so
// the weight rows are the MFMA A operand (read from LDS, shared by the
// workgroup) and the activations of the wave's 64 observations are the B
// operand.  Lane l = 16 g + i of a 16x16x32 MFMA holds A[i][8g..8g+7],
// B[8g..8g+7][i] and D[4g..4g+3][i].  The forward pass keeps the activations
// in registers (see chain_unit); the backward pass stages them through a
// per-wave LDS tile [64][kActS].
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

// Activations of the forward pass stay in registers: the 16x16x32 MFMA
// leaves lane (g, i) with units 16u + 4g .. 16u + 4g + 3 of observation
// 16t + i, and a B operand of the next layer needs 8 k-values per lane for
// the same observation.  The two 4-unit pieces a lane holds of unit tiles
// 2kb and 2kb + 1 form k-block kb of the next layer, in the slot order
//   slot 32kb + 8g + j  <->  unit 32kb + 16 (j >> 2) + 4g + (j & 3);
// the packed W2^T and W3^T store their columns in that order, so the
// products are unchanged.
__host__ __device__ constexpr int chain_unit(int slot)
{
    return (slot & ~31) + 16 * ((slot & 7) >> 2) + 4 * ((slot >> 3) & 3) + (slot & 3);
}

// Per-wave I/O tile: bf16 standardized inputs [64][kIoS] on entry, FP32
// outputs [64][kOutS] on exit (same bytes).
constexpr int kIoS = kInPad + 8;
constexpr int kOutS = kOutPad + 4;
constexpr int kLdsIo = 64 * kIoS;   // bf16 elements (= 64 * kOutS floats)
static_assert(64 * kIoS * 2 == 64 * kOutS * 4, "I/O tile views must coincide");

__device__ __forceinline__ float gelu_f(float z, float *grad)
{
    // tanh form: gelu(z) = z sigmoid(2u), u = c (z + 0.044715 z^3); with
    // e = 2^(2u log2 e): z - z / (1 + e)
    const float z2 = z * z;
    const float w = z * (2.3022082f + 0.10294324f * z2);   // 2 u log2(e)
    const float r = __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(w));
    const float s = 1.0f - r;                                // sigmoid(2u)
    if (grad) *grad = s + 2.0f * z * s * r * 0.7978845608028654f * (1.0f + 0.134145f * z2);
    return z - z * r;
}

// bias + GELU + bf16 of one accumulator (4 consecutive units of one
// observation row); optional training stores of gelu'(z) and the activation.
__device__ __forceinline__ bf16x4 hidden_act(const f32x4 &acc, const float *bias, int unit, int row, float *gp,
                                             __bf16 *hg)
{
    float gr[4];
    bf16x4 h;
#pragma unroll
    for (int r = 0; r < 4; ++r) h[r] = (__bf16)gelu_f(acc[r] + bias[unit + r], gp ? &gr[r] : nullptr);
    if (gp) *reinterpret_cast<float4 *>(gp + (size_t)row * kHid + unit) = make_float4(gr[0], gr[1], gr[2], gr[3]);
    if (hg) *reinterpret_cast<bf16x4 *>(hg + (size_t)row * kHid + unit) = h;
    return h;
}

// Forward pass of one wave's 64 observations (training stores optional:
// gelu'(z) and bf16 activations of both hidden layers, [64][kHid] rows).
__device__ __forceinline__ void mlp_forward64(const __bf16 *lw, const MlpParams &mp, __bf16 *io, int lane,
                                              float *gp1 = nullptr, __bf16 *h1 = nullptr, float *gp2 = nullptr,
                                              __bf16 *h2 = nullptr)
{
    const int g = lane >> 4, i = lane & 15;
    const __bf16 *W1 = lw, *W2 = lw + kLdsW1, *W3 = lw + kLdsW1 + kLdsW2;
    const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
    bf16x8 x[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) x[t] = *reinterpret_cast<const bf16x8 *>(io + (16 * t + i) * kIoS + 8 * g);

    // layer 1 -> the B operands of layer 2, b2[k-block][observation tile]
    bf16x8 b2[4][4];
#pragma unroll
    for (int u = 0; u < kHid / 16; ++u) {
        const bf16x8 a = *reinterpret_cast<const bf16x8 *>(W1 + (16 * u + i) * kWs1 + 8 * g);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const f32x4 acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, x[t], zero, 0, 0, 0);
            const bf16x4 h = hidden_act(acc, mp.b1, 16 * u + 4 * g, 16 * t + i, gp1, h1);
#pragma unroll
            for (int r = 0; r < 4; ++r) b2[u >> 1][t][4 * (u & 1) + r] = h[r];
        }
    }
    // layer 2, two unit tiles at a time = one k-block of layer 3
    f32x4 acc3[4] = {zero, zero, zero, zero};
#pragma unroll 1
    for (int kb3 = 0; kb3 < 4; ++kb3) {
        bf16x8 b3[4];
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            const int u = 2 * kb3 + half;
            f32x4 acc[4] = {zero, zero, zero, zero};
#pragma unroll
            for (int kb = 0; kb < 4; ++kb) {
                const bf16x8 a = *reinterpret_cast<const bf16x8 *>(W2 + (16 * u + i) * kWs2 + 32 * kb + 8 * g);
#pragma unroll
                for (int t = 0; t < 4; ++t) acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b2[kb][t], acc[t], 0, 0, 0);
            }
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const bf16x4 h = hidden_act(acc[t], mp.b2, 16 * u + 4 * g, 16 * t + i, gp2, h2);
#pragma unroll
                for (int r = 0; r < 4; ++r) b3[t][4 * half + r] = h[r];
            }
        }
        const bf16x8 a3 = *reinterpret_cast<const bf16x8 *>(W3 + i * kWs2 + 32 * kb3 + 8 * g);
#pragma unroll
        for (int t = 0; t < 4; ++t) acc3[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a3, b3[t], acc3[t], 0, 0, 0);
    }
    // lane (g, i) holds outputs 4g .. 4g + 3 of observation 16t + i
    float *out = reinterpret_cast<float *>(io);
    const float c0 = mp.b3[4 * g], c1 = mp.b3[4 * g + 1], c2 = mp.b3[4 * g + 2], c3 = mp.b3[4 * g + 3];
#pragma unroll
    for (int t = 0; t < 4; ++t)
        *reinterpret_cast<float4 *>(out + (16 * t + i) * kOutS + 4 * g) =
            make_float4(acc3[t][0] + c0, acc3[t][1] + c1, acc3[t][2] + c2, acc3[t][3] + c3);
}

}  // namespace dev
}  // namespace dba
