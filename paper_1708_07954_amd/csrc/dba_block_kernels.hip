// dba_block_kernels.hip -- gfx950 kernels of the block local updates
// (Ramamurthy et al., "Distributed Bundle Adjustment", Sec. 3.1.4, Eqs. 14-15):
// k_local_block, one camera copy per 64-slot chunk, and k_local_block2,
// blocks of two cameras with one copy per block point.  The rest of the
// iteration (consensus, norms) is in dba_kernels.hip.
//
// A translation unit of its own because these kernels are built with the
// instruction-level-parallelism scheduler (build.py): the two-camera kernel
// runs about 7 % faster under it, while some kernels of dba_kernels.hip run
// slower, so they keep the default one.  The scheduler only orders the same
// instructions: every result is the same under either.
#include "dba_device.h"
#include "block_device.h"

namespace dba {
namespace {

using namespace dev;

// LDS of one wave of the one-camera block kernel: the all-reduce's 64 sums;
// the chunk's camera copy and targets; its consensus, duals and squared
// consensus differences.
template <typename R>
struct BlockLds {
    R red[64];
    R ys[12];
    R vys[12];
    double cyu[27];
};

// Generalised local update of one 64-slot chunk (Sec. 3.1.4, Eqs. 14-15):
// the chunk's observations share one camera copy (copy_yc / dual_yc, per
// chunk) and keep one point copy each.  Deferred dual updates of both, the
// block LM (block_lm), then the chunk's one camera copy goes to the camera
// consensus: cpart = (y + u, y - previous consensus, |y - previous|^2).
template <typename R, typename Cam>
__device__ __forceinline__ void local_block(const DevArrays<R> &a, const SolverParams &sp, int c, int lane,
                                            BlockLds<R> &L)
{
    using R2 = typename Vec<R>::R2;
    const int J = uniform(a.chunk_cam[c]);
    const Ctrl *ct = a.ctrl + uniform(a.chunk_prob[c]);
    const double rho_x = ct->rho_x, rho_y = ct->rho_y;
    const double rat_x = ct->ratio_x, rat_y = ct->ratio_y;
    const int pending = ct->pending;
    const long long s = (long long)c * kChunk + lane;
    const int ps = a.pslot[s];
    const bool active = ps >= 0;
    // lane i < 9 holds camera parameter i: its consensus, the chunk's copy
    // and scaled dual (updated, Eqs. 12-13, and written back); all lanes then
    // read the copy and the targets through the wave's LDS
    if (lane < 9) {
        const double cyi = a.cons_y[(long long)J * kConsY + lane];
        const R ti = a.copy_yc[(long long)c * 9 + lane];
        double uyi = a.dual_yc[(long long)c * 9 + lane];
        if (pending) {
            uyi = (uyi + ((double)ti - cyi)) * rat_y;
            a.dual_yc[(long long)c * 9 + lane] = uyi;
        }
        L.ys[lane] = ti;
        L.vys[lane] = (R)(cyi - uyi);
        L.cyu[lane] = cyi;
        L.cyu[9 + lane] = uyi;
    }
    R th[12], vx[3] = {R(0), R(0), R(0)};
    R2 z;
    z.x = R(0);
    z.y = R(0);
    th[9] = th[10] = th[11] = R(0);
    if (active) {
        const double4 cx = a.cons_x[a.ptid[s]];
        const double cxs[3] = {cx.x, cx.y, cx.z};
        z = a.uv[s];
        const PtCopy<R> xr = a.xrec[ps];
        const PtDual ur = a.urec[ps];
        th[9] = xr.x; th[10] = xr.y; th[11] = xr.z;
        double u[3] = {ur.x, ur.y, ur.z};
        if (pending) {
#pragma unroll
            for (int i = 0; i < 3; ++i) u[i] = (u[i] + ((double)th[9 + i] - cxs[i])) * rat_x;
            a.urec[ps] = PtDual{u[0], u[1], u[2]};
        }
#pragma unroll
        for (int i = 0; i < 3; ++i) vx[i] = (R)(cxs[i] - u[i]);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int i = 0; i < 9; ++i) th[i] = L.ys[i];
    block_lm<R, Cam>(th, L.vys, vx, z.x, z.y, active, (R)rho_x, (R)rho_y, sp.loss, (R)sp.loss_param, sp.lm_steps,
                     (R)sp.lambda0, L.red, lane);
    if (active) {
        a.xrec[ps] = PtCopy<R>{th[9], th[10], th[11]};
    }
    // the chunk's camera copy and consensus partials, a parameter per lane:
    // (y + u, y - previous consensus, |y - previous|^2)
    double *dd2 = L.cyu + 18;
    if (lane < 9) {
        R yi = th[0];
#pragma unroll
        for (int k = 1; k < 9; ++k) yi = lane == k ? th[k] : yi;
        a.copy_yc[(long long)c * 9 + lane] = yi;
        const double t = (double)yi, dd = t - L.cyu[lane];
        double *o = a.cpart + (long long)c * kCpart;
        o[lane] = t + L.cyu[9 + lane];
        o[9 + lane] = dd;
        dd2[lane] = dd * dd;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (lane == 0) {
        double q = 0.0;
#pragma unroll
        for (int i = 0; i < 9; ++i) q += dd2[i];
        a.cpart[(long long)c * kCpart + 18] = q;
    }
    // the LDS is reused by the wave's next chunk
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename R, typename Cam>
__global__ __launch_bounds__(LocalBound<R>::threads) void k_local_block(DevArrays<R> a, SolverParams sp,
                                                                        int persistent)
{
    __shared__ BlockLds<R> lds[LocalBound<R>::threads / 64];
    const int lane = threadIdx.x & 63, wave = wave_id(), wpb = blockDim.x >> 6;
    int c0, c1;
    chunk_range(a.n_chunks, wpb, persistent, c0, c1);
    for (int c = c0 + wave; c < c1; c += wpb) local_block<R, Cam>(a, sp, c, lane, lds[wave]);
}

// Two-camera block b on one wavefront: lane l holds the block's point copy l
// (record blk_rec) and its observations in the chunks of the pair's cameras
// (slot l of each); the camera copies and their duals are per chunk.
template <typename R, typename Cam>
__device__ __forceinline__ void local_block2(const DevArrays<R> &a, const SolverParams &sp, int b, int lane,
                                             R *lds, ProjOf<R, Cam> *pst, R *vys, R *ys, double *cyu)
{
    using R2 = typename Vec<R>::R2;
    // block header: chunk and camera of each pair camera, problem (every
    // per-block and per-lane load below depends on these or on the lane's
    // slot only)
    const int ch[2] = {a.blk_chunk[2 * b], a.blk_chunk[2 * b + 1]};
    const int cam[2] = {a.blk_cam[2 * b], a.blk_cam[2 * b + 1]};
    const int present = (ch[0] >= 0 ? 1 : 0) | (ch[1] >= 0 ? 2 : 0);
    const Ctrl *ct = a.ctrl + a.blk_prob[b];
    const double rho_x = ct->rho_x, rho_y = ct->rho_y;
    const double rat_x = ct->ratio_x, rat_y = ct->ratio_y;
    const int pending = ct->pending;
    // lane i < 18 holds camera parameter i (camera i / 9): its consensus, its
    // copy and its scaled dual (updated, Eqs. 12-13, and written back)
    const int ci = lane < 18 ? lane : 17, cs = ci / 9, cp = ci - 9 * cs;
    const bool cam_lane = lane < 18 && ch[cs] >= 0;
    double cyi = 0.0, uyi = 0.0;
    R ti = R(0);
    if (cam_lane) {
        cyi = a.cons_y[(long long)cam[cs] * kConsY + cp];
        ti = a.copy_yc[(long long)ch[cs] * 9 + cp];
        uyi = a.dual_yc[(long long)ch[cs] * 9 + cp];
        if (pending) {
            uyi = (uyi + ((double)ti - cyi)) * rat_y;
            a.dual_yc[(long long)ch[cs] * 9 + cp] = uyi;
        }
    }
    // the cameras and their targets to every lane through the wave's LDS;
    // each parameter lane's consensus and dual wait there for the end
    if (lane < 18) {
        ys[lane] = ti;
        vys[lane] = cam_lane ? (R)(cyi - uyi) : R(0);
        cyu[lane] = cyi;
        cyu[18 + lane] = uyi;
    }
    const int ps = a.blk_rec[(long long)b * kChunk + lane];
    const int pid = a.blk_pt[(long long)b * kChunk + lane];
    bool act[2];
    R z[4] = {R(0), R(0), R(0), R(0)};
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const long long sl = (long long)(ch[s] >= 0 ? ch[s] : 0) * kChunk + lane;
        act[s] = ch[s] >= 0 && ps >= 0 && a.pslot[sl] >= 0;
        if (act[s]) {
            const R2 zz = a.uv[sl];
            z[2 * s] = zz.x;
            z[2 * s + 1] = zz.y;
        }
    }
    R x[3] = {R(0), R(0), R(0)}, vx[3] = {R(0), R(0), R(0)};
    if (ps >= 0) {
        const double4 cx = a.cons_x[pid];
        const double cxs[3] = {cx.x, cx.y, cx.z};
        const PtCopy<R> xr = a.xrec[ps];
        const PtDual ur = a.urec[ps];
        x[0] = xr.x; x[1] = xr.y; x[2] = xr.z;
        double u[3] = {ur.x, ur.y, ur.z};
        if (pending) {
#pragma unroll
            for (int i = 0; i < 3; ++i) u[i] = (u[i] + ((double)x[i] - cxs[i])) * rat_x;
            a.urec[ps] = PtDual{u[0], u[1], u[2]};
        }
#pragma unroll
        for (int i = 0; i < 3; ++i) vx[i] = (R)(cxs[i] - u[i]);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    R y[18];
#pragma unroll
    for (int i = 0; i < 18; ++i) y[i] = ys[i];
    block_lm2<R, Cam>(y, vys, present, x, vx, act, z, (R)rho_x, (R)rho_y, sp.loss, (R)sp.loss_param, sp.lm_steps,
                      (R)sp.lambda0, lds, pst, lane);
    if (ps >= 0) a.xrec[ps] = PtCopy<R>{x[0], x[1], x[2]};
    // the chunks' camera copies and consensus partials, a parameter per lane:
    // (y + u, y - previous consensus, |y - previous|^2)
    double *dd2 = reinterpret_cast<double *>(lds);
    if (cam_lane) {
        R yi = y[0];
#pragma unroll
        for (int k = 1; k < 18; ++k) yi = ci == k ? y[k] : yi;
        a.copy_yc[(long long)ch[cs] * 9 + cp] = yi;
        const double t = (double)yi, dd = t - cyu[ci];
        double *o = a.cpart + (long long)ch[cs] * kCpart;
        o[cp] = t + cyu[18 + ci];
        o[9 + cp] = dd;
        dd2[ci] = dd * dd;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if ((lane == 0 || lane == 9) && ch[lane / 9] >= 0) {
        double q = 0.0;
#pragma unroll
        for (int i = 0; i < 9; ++i) q += dd2[lane + i];
        a.cpart[(long long)ch[lane / 9] * kCpart + 18] = q;
    }
    // the LDS is reused by the next block of this wave
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr int kBlock2Threads = 256;

// LDS of one wave of the two-camera kernel (dynamic, so a workgroup of w
// waves takes w of these): the reduced system, the camera targets and, in
// FP32, each lane's two projections between LM steps.
template <typename R, typename Cam>
struct Block2Lds {
    R red[kB2Lds];
    R vys[20];
    R ys[20];
    double cyu[36];
    ProjOf<R, Cam> pst[sizeof(R) == 4 ? 128 : 1];
};

// Two waves per SIMD: with the projections in LDS the FP32 kernel fits 256
// registers (the FP64 one spills; it serves the FP64 parity runs).
template <typename R, typename Cam>
__global__ __launch_bounds__(kBlock2Threads, 2) void k_local_block2(DevArrays<R> a, SolverParams sp, int persistent)
{
    extern __shared__ __align__(16) unsigned char b2_lds[];
    const int lane = threadIdx.x & 63, wave = wave_id(), wpb = blockDim.x >> 6;
    Block2Lds<R, Cam> &L = reinterpret_cast<Block2Lds<R, Cam> *>(b2_lds)[wave];
    int b0, b1;
    chunk_range(a.n_blocks2, wpb, persistent, b0, b1);
    for (int b = b0 + wave; b < b1; b += wpb) local_block2<R, Cam>(a, sp, b, lane, L.red, sizeof(R) == 4 ? L.pst : nullptr, L.vys, L.ys, L.cyu);
}

}  // namespace

// ---------------------------------------------------------------- launcher
template <typename R>
hipError_t launch_local_block(const DevArrays<R> &a, const SolverParams &sp, int block_waves, int persistent,
                              int n_cu, hipStream_t s)
{
    if (a.n_blocks2 > 0) {
        // two-camera blocks: one wavefront per block
        if (64 * block_waves > kBlock2Threads) block_waves = kBlock2Threads / 64;
        const int threads = 64 * block_waves;
        int grid;
        if (persistent) {
            grid = n_cu * (8 / block_waves > 0 ? 8 / block_waves : 1);  // two waves per SIMD
            const int need = (a.n_blocks2 + block_waves - 1) / block_waves;
            if (grid > need) grid = need;
        } else {
            grid = (a.n_blocks2 + block_waves - 1) / block_waves;
        }
        if (grid < 1) grid = 1;
        if (sp.camera == 1)
            hipLaunchKernelGGL((k_local_block2<R, CamEuler>), dim3(grid), dim3(threads),
                               block_waves * sizeof(Block2Lds<R, CamEuler>), s, a, sp, persistent);
        else
            hipLaunchKernelGGL((k_local_block2<R, CamAA>), dim3(grid), dim3(threads),
                               block_waves * sizeof(Block2Lds<R, CamAA>), s, a, sp, persistent);
        return hipGetLastError();
    }
    if (64 * block_waves > LocalBound<R>::threads) block_waves = LocalBound<R>::threads / 64;
    const int threads = 64 * block_waves;
    int grid;
    if (persistent) {
        grid = n_cu * (8 / block_waves > 0 ? 8 / block_waves : 1);
        const int need = (a.n_chunks + block_waves - 1) / block_waves;
        if (grid > need) grid = need;
    } else {
        grid = (a.n_chunks + block_waves - 1) / block_waves;
    }
    if (grid < 1) grid = 1;
    if (sp.camera == 1)
        hipLaunchKernelGGL((k_local_block<R, CamEuler>), dim3(grid), dim3(threads), 0, s, a, sp, persistent);
    else
        hipLaunchKernelGGL((k_local_block<R, CamAA>), dim3(grid), dim3(threads), 0, s, a, sp, persistent);
    return hipGetLastError();
}

template hipError_t launch_local_block<float>(const DevArrays<float> &, const SolverParams &, int, int, int,
                                              hipStream_t);
template hipError_t launch_local_block<double>(const DevArrays<double> &, const SolverParams &, int, int, int,
                                               hipStream_t);

}  // namespace dba
