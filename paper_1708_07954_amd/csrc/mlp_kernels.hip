// mlp_kernels.hip -- training and batch evaluation of the warm-start network,
// and collection of its training pairs, on gfx950.
//
//   pack       FP32 master parameters -> bf16 weight block (W^T for the
//              forward pass, W for the backward pass)
//   prepare    raw features / targets -> standardized bf16 inputs [N][32]
//              and FP32 targets [N][16]
//   forward    64 rows per wave on BF16 MFMA (shared with the fused local
//              solve); optionally keeps gelu'(z) and the bf16 activations
//   backward   activation gradients on BF16 MFMA (dY -> dZ2 -> dZ1)
//   wgrad      weight gradients dW = P^T Q over the batch on BF16 MFMA, four
//              waves per output tile reduced in a fixed order
//   bias, adam column sums of dY, dZ2, dZ1 (fixed order); Adam update
//   collect    (features, converged update) pairs of sampled local problems
// All reductions have a fixed order: training is deterministic.
#include "dba_device.h"
#include "mlp_device.h"

#include <mutex>

namespace dba {

// Scratch of the allocation-free network forward (dba_mlp_forward_noalloc):
// the standardised BF16 inputs [kNoAllocMaxRows][kInPad] followed by the
// padded FP32 outputs [kNoAllocMaxRows][kOutPad].  One copy per GPU for the
// life of the process; every call on a GPU shares it.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

using namespace dev;

// ---------------------------------------------------------------- pack
__global__ void k_mlp_pack(const float *P, __bf16 *w)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= kWTotal) return;
    float x;
    if (q < kOffW2T) {                    // W1^T [128][32]
        const int u = q / kInPad, k = q % kInPad;
        x = P[kPW1 + k * kHid + u];
    } else if (q < kOffW3T) {             // W2^T [128][128], columns in chained slot order
        const int r = q - kOffW2T, u = r / kHid, k = chain_unit(r % kHid);
        x = P[kPW2 + k * kHid + u];
    } else if (q < kOffW2N) {             // W3^T [16][128], columns in chained slot order
        const int r = q - kOffW3T, o = r / kHid, k = chain_unit(r % kHid);
        x = P[kPW3 + k * kOutPad + o];
    } else if (q < kOffW3N) {             // W2 [128][128]
        x = P[kPW2 + (q - kOffW2N)];
    } else {                              // W3 [128][32], outputs padded to 32
        const int r = q - kOffW3N, k = r / (2 * kOutPad), o = r % (2 * kOutPad);
        x = o < kOutPad ? P[kPW3 + k * kOutPad + o] : 0.0f;
    }
    w[q] = (__bf16)x;
}

// ---------------------------------------------------------------- prepare
__global__ void k_mlp_prepare(const float *feat, const float *delta, const float *norm, long long n,
                              __bf16 *xq, float *t)
{
    const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
#pragma unroll
    for (int k = 0; k < kInPad; ++k)
        xq[r * kInPad + k] = k < kIn ? (__bf16)((feat[r * kIn + k] - norm[k]) / norm[kIn + k]) : (__bf16)0.0f;
    if (t) {
#pragma unroll
        for (int o = 0; o < kOutPad; ++o)
            t[r * kOutPad + o] = o < kOut ? (delta[r * kOut + o] - norm[2 * kIn + o]) / norm[2 * kIn + kOut + o] : 0.0f;
    }
}

// ---------------------------------------------------------------- forward
// rows[b] (or b itself when rows == nullptr) for b < n; 4 waves x 64 rows per
// workgroup.  Training mode stores the batch-ordered xb, gelu' and h1/h2.
constexpr int kFwdWaves = 4;

__global__ __launch_bounds__(64 * kFwdWaves) void k_mlp_forward(const __bf16 *xq, const int *rows, int n, MlpParams mp,
                                                               float *y, __bf16 *xb, float *gp1, __bf16 *h1,
                                                               float *gp2, __bf16 *h2)
{
    __shared__ __attribute__((aligned(16))) __bf16 lw[kLdsFwd];
    __shared__ __attribute__((aligned(16))) __bf16 io[kFwdWaves][kLdsIo];
    stage_forward_weights(mp.w, lw);
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int b0 = (blockIdx.x * kFwdWaves + wave) * 64;
    if (b0 >= n) return;  // whole wave; no barrier follows
    const int b = b0 + lane;
    bf16x8 x[4];
    if (b < n) {
        const long long r = rows ? rows[b] : b;
#pragma unroll
        for (int q = 0; q < 4; ++q) x[q] = *reinterpret_cast<const bf16x8 *>(xq + r * kInPad + 8 * q);
    } else {
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int j = 0; j < 8; ++j) x[q][j] = (__bf16)0.0f;
    }
    __bf16 *a = io[wave];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        *reinterpret_cast<bf16x8 *>(a + lane * kIoS + 8 * q) = x[q];
        if (xb && b < n) *reinterpret_cast<bf16x8 *>(xb + (size_t)b * kInPad + 8 * q) = x[q];
    }
    // training stores cover whole 64-row tiles; the caller sizes them so
    mlp_forward64(lw, mp, a, lane, gp1 ? gp1 + (size_t)b0 * kHid : nullptr, h1 ? h1 + (size_t)b0 * kHid : nullptr,
                  gp2 ? gp2 + (size_t)b0 * kHid : nullptr, h2 ? h2 + (size_t)b0 * kHid : nullptr);
    const float *out = reinterpret_cast<const float *>(a);
    if (b < n) {
#pragma unroll
        for (int o = 0; o < kOutPad; o += 4)
            *reinterpret_cast<float4 *>(y + (size_t)b * kOutPad + o) = *reinterpret_cast<const float4 *>(out + lane * kOutS + o);
    }
}

// ---------------------------------------------------------------- backward (activations)
// Batch of n rows (a multiple of 64), loss = mean over n x 12 of (y - t)^2.
constexpr int kLdsBwd = kHid * kWs3 + kHid * kWs2;   // W3 [128][40] + W2 [128][136]

struct GradEpi {   // dZ = (W x dIn)^T . gelu'(z): FP32 rows and bf16 rows + tile
    __bf16 *act;
    const float *gp;     // [64][128] rows of this tile
    float *dz;           // [64][128]
    __bf16 *dzq;         // [64][128]
    int lane;
    __device__ __forceinline__ void operator()(int u, const f32x4 *acc) const
    {
        const int g = lane >> 4, i = lane & 15;
        const int unit = 16 * u + 4 * g;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int row = 16 * t + i;
            const float4 gr = *reinterpret_cast<const float4 *>(gp + (size_t)row * kHid + unit);
            const float d0 = acc[t][0] * gr.x, d1 = acc[t][1] * gr.y, d2 = acc[t][2] * gr.z, d3 = acc[t][3] * gr.w;
            *reinterpret_cast<float4 *>(dz + (size_t)row * kHid + unit) = make_float4(d0, d1, d2, d3);
            bf16x4 q;
            q[0] = (__bf16)d0; q[1] = (__bf16)d1; q[2] = (__bf16)d2; q[3] = (__bf16)d3;
            *reinterpret_cast<bf16x4 *>(act + row * kActS + unit) = q;
            *reinterpret_cast<bf16x4 *>(dzq + (size_t)row * kHid + unit) = q;
        }
    }
};

__global__ __launch_bounds__(64 * kFwdWaves) void k_mlp_backward(const float *y, const float *tq, const int *rows, int n,
                                                                const __bf16 *w, const float *gp1, const float *gp2,
                                                                float *dy, __bf16 *dyq, float *dz2, __bf16 *dz2q,
                                                                float *dz1, __bf16 *dz1q, float *loss_part)
{
    __shared__ __attribute__((aligned(16))) __bf16 lw[kLdsBwd];
    __shared__ __attribute__((aligned(16))) __bf16 act[kFwdWaves][kLdsAct];
    stage_rows(w + kOffW3N, lw, kHid, 2 * kOutPad, kWs3);
    stage_rows(w + kOffW2N, lw + kHid * kWs3, kHid, kHid, kWs2);
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int tile = blockIdx.x * kFwdWaves + wave;
    const int b0 = tile * 64;
    if (b0 >= n) return;
    const int b = b0 + lane;
    const long long r = rows ? rows[b] : b;
    __bf16 *a = act[wave];
    const float scale = 2.0f / ((float)n * (float)kOut);
    float l2 = 0.0f;
    bf16x8 qv[4];
#pragma unroll
    for (int o = 0; o < 2 * kOutPad; ++o) {
        float d = 0.0f;
        if (o < kOut) {
            const float e = y[(size_t)b * kOutPad + o] - tq[r * kOutPad + o];
            l2 += e * e;
            d = scale * e;
        }
        if (o < kOutPad) dy[(size_t)b * kOutPad + o] = d;
        qv[o >> 3][o & 7] = (__bf16)d;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        *reinterpret_cast<bf16x8 *>(a + lane * kActS + 8 * q) = qv[q];
        *reinterpret_cast<bf16x8 *>(dyq + (size_t)b * 2 * kOutPad + 8 * q) = qv[q];
    }
    // per-tile loss partial (fixed butterfly)
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) l2 += __shfl_xor(l2, off, 64);
    if (lane == 0) loss_part[tile] = l2;
    const size_t rb = (size_t)b0 * kHid;
    dense64<kHid / 16, 1>(lw, kWs3, a, kActS, lane, GradEpi{a, gp2 + rb, dz2 + rb, dz2q + rb, lane});
    dense64<kHid / 16, 4>(lw + kHid * kWs3, kWs2, a, kActS, lane, GradEpi{a, gp1 + rb, dz1 + rb, dz1q + rb, lane});
}

// ---------------------------------------------------------------- weight gradients
// Output tile (16 rows of P's columns, 16 of Q's) of dW = P^T Q, P [n][pc],
// Q [n][qc], bf16 rows.  Four waves split the batch; their accumulators are
// added in wave order.
struct WgradJob {
    const __bf16 *P;
    int pc;
    const __bf16 *Q;
    int qc;
    float *dW;      // [pc_used][ldw]
    int ldw;
    int m_tiles, n_tiles;
};

__global__ __launch_bounds__(256) void k_mlp_wgrad(WgradJob j0, WgradJob j1, WgradJob j2, int n)
{
    __shared__ __attribute__((aligned(16))) __bf16 pt[4][16][40];
    __shared__ __attribute__((aligned(16))) __bf16 qt[4][16][40];
    __shared__ float red[4][64][4];
    int t = blockIdx.x;
    const WgradJob *jp = &j0;
    if (t >= j0.m_tiles * j0.n_tiles) {
        t -= j0.m_tiles * j0.n_tiles;
        jp = &j1;
        if (t >= j1.m_tiles * j1.n_tiles) {
            t -= j1.m_tiles * j1.n_tiles;
            jp = &j2;
        }
    }
    const WgradJob &J = *jp;
    const int m0 = (t / J.n_tiles) * 16, n0 = (t % J.n_tiles) * 16;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, i = lane & 15;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    const int slices = n / 32;
    for (int sl = wave; sl < slices; sl += 4) {
        const int rb = sl * 32;
        // stage P[rb..rb+31][m0..m0+15] and Q[..][n0..n0+15] transposed
        {
            const int row = lane >> 1, half = lane & 1;
            const bf16x8 pv = *reinterpret_cast<const bf16x8 *>(J.P + (size_t)(rb + row) * J.pc + m0 + 8 * half);
            const bf16x8 qv = *reinterpret_cast<const bf16x8 *>(J.Q + (size_t)(rb + row) * J.qc + n0 + 8 * half);
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                pt[wave][8 * half + e][row] = pv[e];
                qt[wave][8 * half + e][row] = qv[e];
            }
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const bf16x8 av = *reinterpret_cast<const bf16x8 *>(&pt[wave][i][8 * g]);
        const bf16x8 bv = *reinterpret_cast<const bf16x8 *>(&qt[wave][i][8 * g]);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc, 0, 0, 0);
        __builtin_amdgcn_wave_barrier();
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) red[wave][lane][r] = acc[r];
    __syncthreads();
    if (wave == 0) {
        float o[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) o[r] = ((red[0][lane][r] + red[1][lane][r]) + red[2][lane][r]) + red[3][lane][r];
#pragma unroll
        for (int r = 0; r < 4; ++r) J.dW[(size_t)(m0 + 4 * g + r) * J.ldw + n0 + i] = o[r];
    }
}

// ---------------------------------------------------------------- bias gradients
// Column sums of dy [n][16] (cols 0..15), dz2 [n][128], dz1 [n][128] into
// grad at the bias offsets; 4 threads per column, combined in order.
// Column sums of dY (16), dZ2 (128) and dZ1 (128): 16 columns per block,
// 16 row lanes per column, each with 8 interleaved accumulators (rows
// r = lane + 16 k, accumulator k mod 8), combined in a fixed order.
__global__ __launch_bounds__(256) void k_mlp_bias(const float *dy, const float *dz2, const float *dz1, int n, float *grad)
{
    __shared__ float part[16][17];
    const int col = blockIdx.x * 16 + (threadIdx.x & 15);   // 0..271
    const int rl = threadIdx.x >> 4;
    const float *src = nullptr;
    int ld = 0, c = 0, dst = -1;
    if (col < kOutPad) { src = dy; ld = kOutPad; c = col; dst = kPB3 + col; }
    else if (col < kOutPad + kHid) { src = dz2; ld = kHid; c = col - kOutPad; dst = kPB2 + c; }
    else { src = dz1; ld = kHid; c = col - kOutPad - kHid; dst = kPB1 + c; }
    float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    int r = rl;
    for (; r + 16 * 7 < n; r += 16 * 8) {
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[j] += src[(size_t)(r + 16 * j) * ld + c];
    }
#pragma unroll
    for (int j = 0; j < 8; ++j)
        if (r + 16 * j < n) acc[j] += src[(size_t)(r + 16 * j) * ld + c];
    part[rl][threadIdx.x & 15] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
    __syncthreads();
    if (rl == 0) {
        float t = 0.f;
#pragma unroll
        for (int q = 0; q < 16; ++q) t += part[q][threadIdx.x & 15];
        grad[dst] = t;
    }
}

// ---------------------------------------------------------------- Adam
__global__ void k_mlp_adam(float *P, float *m, float *v, const float *g, float lr, float bc1, float bc2)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= kPTotal) return;
    // padded inputs (W1 rows 26..31) and outputs (W3 cols 12..15, b3 12..15) stay zero
    bool pad = false;
    if (q >= kPW1 && q < kPB1) pad = (q - kPW1) / kHid >= kIn;
    else if (q >= kPW3 && q < kPB3) pad = (q - kPW3) % kOutPad >= kOut;
    else if (q >= kPB3) pad = (q - kPB3) >= kOut;
    if (pad) { P[q] = 0.0f; return; }
    const float gq = g[q];
    const float mq = 0.9f * m[q] + 0.1f * gq;
    const float vq = 0.999f * v[q] + 0.001f * gq * gq;
    m[q] = mq;
    v[q] = vq;
    P[q] -= lr * (mq / bc1) / (sqrtf(vq / bc2) + 1e-8f);
}

// ---------------------------------------------------------------- collect pairs
// For each sampled slot: the local problem of the coming iteration (with the
// pending dual update applied in registers only), its 26 features at the
// start point, and the update of an LM run to convergence (conv_steps).
__global__ __launch_bounds__(256) void k_collect_pairs(DevArrays<float> a, SolverParams sp, const int *slots, int n,
                                                      float *feat, float *delta, int conv_steps)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const long long s = slots[q];
    const int ps = a.pslot[s];
    if (ps < 0) return;
    const int J = a.chunk_cam[s / kChunk];
    const Ctrl &ct = a.ctrl[a.cam_prob[J]];
    const long long S = a.n_slots;
    const double4 cx = a.cons_x[a.ptid[s]];
    double cons[12], u[12];
    float th[12], v[12];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        cons[i] = a.cons_y[(long long)J * kConsY + i];
        th[i] = a.copy_y[i * S + s];
        u[i] = a.dual_y[i * S + s];
    }
    cons[9] = cx.x; cons[10] = cx.y; cons[11] = cx.z;
    const PtCopy<float> xr = a.xrec[ps];
    const PtDual ur = a.urec[ps];
    th[9] = xr.x; th[10] = xr.y; th[11] = xr.z;
    u[9] = ur.x; u[10] = ur.y; u[11] = ur.z;
    if (ct.pending)
#pragma unroll
        for (int i = 0; i < 12; ++i) u[i] = (u[i] + ((double)th[i] - cons[i])) * (i < 9 ? ct.ratio_y : ct.ratio_x);
#pragma unroll
    for (int i = 0; i < 12; ++i) v[i] = (float)(cons[i] - u[i]);
    const float2 z = a.uv[s];
    const Proj<float> p0 = proj_core<float, true>(th, CamAA{});
    float *f = feat + (size_t)q * kIn;
    f[0] = z.x - p0.pu;
    f[1] = z.y - p0.pv;
#pragma unroll
    for (int i = 0; i < 12; ++i) f[2 + i] = (float)((double)th[i] - cons[i]);
#pragma unroll
    for (int i = 0; i < 12; ++i) f[14 + i] = (float)u[i];
    float tc[12];
#pragma unroll
    for (int i = 0; i < 12; ++i) tc[i] = th[i];
    local_lm<float, CamAA>(tc, v, z.x, z.y, (float)ct.rho_x, (float)ct.rho_y, sp.loss, (float)sp.loss_param, conv_steps,
                    (float)sp.lambda0);
#pragma unroll
    for (int i = 0; i < 12; ++i) delta[(size_t)q * kOut + i] = tc[i] - th[i];
}

// ---------------------------------------------------------------- destandardize
// delta = y * std + mean per output, each product and sum rounded on its own
// (no fused multiply-add), as the host-side path of dba_mlp_forward computes.
__global__ void k_mlp_destandardize(const float *y, const float *norm, long long n, float *delta)
{
#pragma clang fp contract(off)
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n * kOut) return;
    const long long r = q / kOut;
    const int o = (int)(q - r * kOut);
    delta[q] = y[r * kOutPad + o] * norm[2 * kIn + kOut + o] + norm[2 * kIn + o];
}

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices];

}  // namespace

// Device address of this GPU's scratch array; the caller has made `device`
// current.  Looked up once per device and kept.
hipError_t noalloc_scratch(int device, void **ptr)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch[device] = p;
    }
    *ptr = g_scratch[device];
    return hipSuccess;
}

hipError_t mlp_destandardize(const float *y, const float *norm, long long n, float *delta, hipStream_t s)
{
    const long long total = n * kOut;
    hipLaunchKernelGGL(k_mlp_destandardize, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, y, norm, n, delta);
    return hipGetLastError();
}

// ---------------------------------------------------------------- launchers
hipError_t mlp_pack(const float *P, __bf16 *w, hipStream_t s)
{
    hipLaunchKernelGGL(k_mlp_pack, dim3((kWTotal + 255) / 256), dim3(256), 0, s, P, w);
    return hipGetLastError();
}

hipError_t mlp_prepare(const float *feat, const float *delta, const float *norm, long long n, __bf16 *xq, float *t,
                       hipStream_t s)
{
    hipLaunchKernelGGL(k_mlp_prepare, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, feat, delta, norm, n, xq, t);
    return hipGetLastError();
}

hipError_t mlp_forward(const __bf16 *xq, const int *rows, int n, const MlpParams &mp, float *y, __bf16 *xb, float *gp1,
                       __bf16 *h1, float *gp2, __bf16 *h2, hipStream_t s)
{
    const int tiles = (n + 63) / 64;
    hipLaunchKernelGGL(k_mlp_forward, dim3((tiles + kFwdWaves - 1) / kFwdWaves), dim3(64 * kFwdWaves), 0, s, xq, rows,
                       n, mp, y, xb, gp1, h1, gp2, h2);
    return hipGetLastError();
}

hipError_t mlp_backward(const float *y, const float *tq, const int *rows, int n, const __bf16 *w, const float *gp1,
                        const float *gp2, float *dy, __bf16 *dyq, float *dz2, __bf16 *dz2q, float *dz1, __bf16 *dz1q,
                        float *loss_part, hipStream_t s)
{
    const int tiles = n / 64;
    hipLaunchKernelGGL(k_mlp_backward, dim3((tiles + kFwdWaves - 1) / kFwdWaves), dim3(64 * kFwdWaves), 0, s, y, tq,
                       rows, n, w, gp1, gp2, dy, dyq, dz2, dz2q, dz1, dz1q, loss_part);
    return hipGetLastError();
}

hipError_t mlp_wgrad(const __bf16 *xb, const __bf16 *h1, const __bf16 *h2, const __bf16 *dyq, const __bf16 *dz2q,
                     const __bf16 *dz1q, int n, float *grad, hipStream_t s)
{
    WgradJob j0{xb, kInPad, dz1q, kHid, grad + kPW1, kHid, kInPad / 16, kHid / 16};
    WgradJob j1{h1, kHid, dz2q, kHid, grad + kPW2, kHid, kHid / 16, kHid / 16};
    WgradJob j2{h2, kHid, dyq, 2 * kOutPad, grad + kPW3, kOutPad, kHid / 16, 1};
    const int tiles = j0.m_tiles * j0.n_tiles + j1.m_tiles * j1.n_tiles + j2.m_tiles * j2.n_tiles;
    hipLaunchKernelGGL(k_mlp_wgrad, dim3(tiles), dim3(256), 0, s, j0, j1, j2, n);
    return hipGetLastError();
}

hipError_t mlp_bias(const float *dy, const float *dz2, const float *dz1, int n, float *grad, hipStream_t s)
{
    hipLaunchKernelGGL(k_mlp_bias, dim3((kOutPad + 2 * kHid) / 16), dim3(256), 0, s, dy, dz2, dz1, n, grad);
    return hipGetLastError();
}

hipError_t mlp_adam(float *P, float *m, float *v, const float *g, float lr, float bc1, float bc2, hipStream_t s)
{
    hipLaunchKernelGGL(k_mlp_adam, dim3((kPTotal + 255) / 256), dim3(256), 0, s, P, m, v, g, lr, bc1, bc2);
    return hipGetLastError();
}

hipError_t collect_pairs(const DevArrays<float> &a, const SolverParams &sp, const int *slots, int n, float *feat,
                         float *delta, int conv_steps, hipStream_t s)
{
    hipLaunchKernelGGL(k_collect_pairs, dim3((n + 255) / 256), dim3(256), 0, s, a, sp, slots, n, feat, delta,
                       conv_steps);
    return hipGetLastError();
}

}  // namespace dba
