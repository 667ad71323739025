// dba_kernels.hip -- gfx950 kernels of one ADMM bundle-adjustment iteration
// (Ramamurthy et al., "Distributed Bundle Adjustment", Sec. 3.1, Eqs. 9-13).
//
// local      one lane per observation (wave64 = one 64-slot chunk of one
//            camera).  Applies the deferred scaled-dual update of the
//            previous iteration, then minimises the local objective of Eq. (9)
//            in scaled form, F = phi(|z - pi(theta)|^2) + 1/2 (theta - v)^T P
//            (theta - v), by robust Levenberg-Marquardt: the 12x12 normal
//            equations (diagonal plus rank two) are solved in registers.
//            Emits the chunk's sums for the camera consensus with a fixed
//            butterfly.
// consensus  point consensus (Eq. 10): one pass over the records, each
//            point's records in groups of consecutive records (a thread per
//            point, or a thread per group); residual terms summed per wave of
//            points by a fixed butterfly;
//            camera consensus (Eq. 11): one wave per camera, lanes summing
//            strided chunk partials, then a fixed reduce-scatter.  Both FP64.
// norms      one workgroup per problem: primal/dual residual norms, residual
//            balancing of rho, rescale factor for the pending dual update.
// eval       reprojection statistics at the consensus estimate (FP64).
// The block local updates (Sec. 3.1.4) are in dba_block_kernels.hip.
//
// Every reduction has a fixed order that does not depend on the launch
// schedule, so all schedules (and batched vs solo runs) are bitwise equal.
#include "dba_device.h"
#include "mlp_device.h"

namespace dba {
namespace {

using namespace dev;

// ---------------------------------------------------------------- local
// One 64-slot chunk (one camera) per wave; Cam is the camera model.
// LEARNED (9-parameter camera only): the start point is the better of the
// copy and copy + network prediction (ties keep the copy), then
// `learned_steps` LM steps; io/lw are the wave's network I/O tile and the
// staged weights.
template <typename R, bool LEARNED, typename Cam = CamAA, int SOLVER = 0>
__device__ __forceinline__ void local_chunk(const DevArrays<R> &a, const SolverParams &sp, int c, int lane,
                                            const MlpParams *mp = nullptr, const __bf16 *lw = nullptr,
                                            __bf16 *io = nullptr)
{
    using R2 = typename Vec<R>::R2;
    // the chunk's camera and its problem's control block are the same for
    // every lane: scalar registers
    const int J = uniform(a.chunk_cam[c]);
    const Ctrl *ct = a.ctrl + uniform(a.chunk_prob[c]);
    const double rho_x = uniform(ct->rho_x), rho_y = uniform(ct->rho_y);
    const double rat_x = uniform(ct->ratio_x), rat_y = uniform(ct->ratio_y);
    const int pending = uniform(ct->pending);
    const long long S = a.n_slots;
    const long long s = (long long)c * kChunk + lane;
    const int ps = a.pslot[s];
    const bool active = ps >= 0;
    double cy[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) cy[i] = uniform(a.cons_y[(long long)J * kConsY + i]);

    double acc[19];
#pragma unroll
    for (int i = 0; i < 19; ++i) acc[i] = 0.0;

    R th[12], v[12];
    double u[12], cons[12];
    R2 z;
    z.x = R(0);
    z.y = R(0);
    if (active) {
        const double4 cx = a.cons_x[a.ptid[s]];
#pragma unroll
        for (int i = 0; i < 9; ++i) cons[i] = cy[i];
        cons[9] = cx.x; cons[10] = cx.y; cons[11] = cx.z;
        z = a.uv[s];
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            th[i] = a.copy_y[i * S + s];
            u[i] = a.dual_y[i * S + s];
        }
        const PtCopy<R> xr = a.xrec[ps];
        const PtDual ur = a.urec[ps];
        th[9] = xr.x; th[10] = xr.y; th[11] = xr.z;
        u[9] = ur.x; u[10] = ur.y; u[11] = ur.z;
        if (pending) {  // Eqs. (12)-(13) of the previous iteration, then the rho rescale
#pragma unroll
            for (int i = 0; i < 12; ++i)
                u[i] = (u[i] + ((double)th[i] - cons[i])) * (i < 9 ? rat_y : rat_x);
#pragma unroll
            for (int i = 0; i < 9; ++i) a.dual_y[i * S + s] = u[i];
            a.urec[ps] = PtDual{u[9], u[10], u[11]};
        }
#pragma unroll
        for (int i = 0; i < 12; ++i) v[i] = (R)(cons[i] - u[i]);
    }
    const R rx = (R)rho_x, ry = (R)rho_y, lp = (R)sp.loss_param, lam0 = (R)sp.lambda0;
    if constexpr (LEARNED) {
        // features at the start point, standardized (x = f * scale + shift),
        // bf16 into the wave's I/O tile; idle lanes feed zeros
        float f[kIn];
        if (active) {
            const Proj<R> p0 = proj_core<R, false>(th);
            f[0] = (float)(z.x - p0.pu);
            f[1] = (float)(z.y - p0.pv);
#pragma unroll
            for (int i = 0; i < 12; ++i) f[2 + i] = (float)((double)th[i] - cons[i]);
#pragma unroll
            for (int i = 0; i < 12; ++i) f[14 + i] = (float)u[i];
        }
        const float *xf = mp->xform;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            bf16x8 xin;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int k = 8 * q + j;
                xin[j] = (k < kIn && active) ? (__bf16)fmaf(f[k], xf[k], xf[kIn + k]) : (__bf16)0.0f;
            }
            *reinterpret_cast<bf16x8 *>(io + lane * kIoS + 8 * q) = xin;
        }
        mlp_forward64(lw, *mp, io, lane);
        if (active) {
            const float *nm = mp->norm;
            const float *out = reinterpret_cast<const float *>(io) + lane * kOutS;
            R tr[12];
#pragma unroll
            for (int i = 0; i < kOut; ++i) tr[i] = th[i] + (R)(out[i] * nm[2 * kIn + kOut + i] + nm[2 * kIn + i]);
            Proj<R> cur = proj_core<R, true>(th);
            R F = objective<R>(cur, th, v, z.x, z.y, rx, ry, sp.loss, lp);
            const Proj<R> nxt = proj_core<R, true>(tr);
            const R F1 = objective<R>(nxt, tr, v, z.x, z.y, rx, ry, sp.loss, lp);
            if (F1 < F) {  // the guard: keep the prediction only if it lowers F
#pragma unroll
                for (int i = 0; i < 12; ++i) th[i] = tr[i];
                cur = nxt;
                F = F1;
            }
            lm_steps<R, CamAA>(th, cur, F, v, z.x, z.y, rx, ry, sp.loss, lp, sp.learned_steps, lam0);
        }
    } else {
        if (active) local_lm<R, Cam, SOLVER>(th, v, z.x, z.y, rx, ry, sp.loss, lp, sp.lm_steps, lam0);
    }
    if (active) {
#pragma unroll
        for (int i = 0; i < 9; ++i) a.copy_y[i * S + s] = th[i];
        a.xrec[ps] = PtCopy<R>{th[9], th[10], th[11]};
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const double t = (double)th[i];
            const double dd = t - cy[i];
            acc[i] = t + u[i];
            acc[9 + i] = dd;
            acc[18] += dd * dd;
        }
    }
    wave_sum19_store(acc, a.cpart + (long long)c * kCpart, lane);
}

template <typename R, typename Cam, int SOLVER>
__global__ __launch_bounds__(LocalBound<R>::threads) void k_local(DevArrays<R> a, SolverParams sp,
                                                                  int persistent)
{
    const int lane = threadIdx.x & 63, wave = wave_id(), wpb = blockDim.x >> 6;
    int c0, c1;
    chunk_range(a.n_chunks, wpb, persistent, c0, c1);
    for (int c = c0 + wave; c < c1; c += wpb) local_chunk<R, false, Cam, SOLVER>(a, sp, c, lane);
}

// Learned start: the workgroup's waves share the staged weights (one copy
// per CU: 8 waves, 2 per SIMD); each wave has its own network I/O tile.  The
// grid is persistent so the weights are staged once per workgroup.
constexpr int kLearnedWaves = 8;

__global__ __launch_bounds__(64 * kLearnedWaves) void k_local_learned(DevArrays<float> a, SolverParams sp,
                                                                       MlpParams mp, int persistent)
{
    __shared__ __attribute__((aligned(16))) __bf16 lw[kLdsFwd];
    __shared__ __attribute__((aligned(16))) __bf16 io[kLearnedWaves][kLdsIo];
    stage_forward_weights(mp.w, lw);
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = wave_id();
    int c0, c1;
    chunk_range(a.n_chunks, kLearnedWaves, persistent, c0, c1);
    for (int c = c0 + wave; c < c1; c += kLearnedWaves)
        local_chunk<float, true>(a, sp, c, lane, &mp, lw, io[wave]);
}

// ---------------------------------------------------------------- consensus
// Sums of one point's records that the consensus needs: of copy + dual (the
// new consensus times n) and of the copies' offsets d_r from the previous
// consensus, which give sum_r |copy_r - new|^2 = sum |d_r|^2 - 2 e . sum d_r
// + n |e|^2, e = new - previous.
struct PtSums {
    double s0, s1, s2, q0, q1, q2, qq;
    __device__ void clear() { s0 = s1 = s2 = q0 = q1 = q2 = qq = 0.0; }
    template <typename R>
    __device__ void add(const PtCopy<R> &x, const PtDual &u, const double4 &old)
    {
        s0 += (double)x.x + u.x;
        s1 += (double)x.y + u.y;
        s2 += (double)x.z + u.z;
        const double d0 = (double)x.x - old.x, d1 = (double)x.y - old.y, d2 = (double)x.z - old.z;
        q0 += d0;
        q1 += d1;
        q2 += d2;
        qq += d0 * d0 + d1 * d1 + d2 * d2;
    }
    __device__ void add(const PtSums &g)
    {
        s0 += g.s0; s1 += g.s1; s2 += g.s2;
        q0 += g.q0; q1 += g.q1; q2 += g.q2;
        qq += g.qq;
    }
};

// New consensus of point i from its sums (Eq. 10) and its residual terms.
__device__ __forceinline__ void point_finish(double4 *cons_x, int i, const double4 &old, int nrec,
                                             const PtSums &t, double &pri, double &dual)
{
    const double n = (double)nrec;
    const double c0 = t.s0 / n, c1 = t.s1 / n, c2 = t.s2 / n;
    const double e0 = c0 - old.x, e1 = c1 - old.y, e2 = c2 - old.z;
    cons_x[i] = make_double4(c0, c1, c2, 0.0);
    const double ee = e0 * e0 + e1 * e1 + e2 * e2;
    pri = fmax(t.qq - 2.0 * (e0 * t.q0 + e1 * t.q1 + e2 * t.q2) + n * ee, 0.0);
    dual = n * ee;
}

// Point consensus, one wave per consensus wave (at most 64 points whose
// record groups fit the 64 lanes).  Both schedules sum a point's records in
// the order of cons_group -- groups of consecutive records, each in record
// order, then the group sums in group order -- and leave point j's residual
// terms in lane j for a fixed butterfly, so they are bitwise identical.
//   SCHED 1: lane j sums the records of the wave's point j, four loads in
//            flight, closing each group as it goes;
//   SCHED 2: lane l sums one record group (eight loads in flight), the group
//            sums meet in LDS and lane j adds its point's groups in order;
//   SCHED 3: as 2, with the wave's records staged through LDS in tiles
//            loaded with coalesced loads.
constexpr int kStageRecs = 128;
template <typename R, int SCHED>
__device__ __forceinline__ void point_wave(const DevArrays<R> &a, int cw, int w, int lane, double *pd)
{
    const int p0 = a.cw_pt0[cw], np = a.cw_pt0[cw + 1] - p0;
    const bool has = lane < np;
    const int i = p0 + lane;
    int r0 = 0, r1 = 0;
    // lane j's point: its record range and previous consensus, loaded at once
    double4 oldi = make_double4(0.0, 0.0, 0.0, 0.0);
    if (has) {
        r0 = a.pt_off[i];
        r1 = a.pt_off[i + 1];
        oldi = a.cons_x[i];
    }
    double pri = 0.0, dual = 0.0;
    if constexpr (SCHED == 1) {
        if (has) {
            const double4 old = oldi;
            const int K = cons_group(r1 - r0);
            PtSums t, g;
            t.clear();
            g.clear();
            int in_g = 0;
            auto take = [&](const PtCopy<R> &x, const PtDual &u) {
                g.add(x, u, old);
                if (++in_g == K) {
                    t.add(g);
                    g.clear();
                    in_g = 0;
                }
            };
            int r = r0;
            for (; r + 4 <= r1; r += 4) {
                PtCopy<R> x[4];
                PtDual u[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    x[j] = a.xrec[r + j];
                    u[j] = a.urec[r + j];
                }
#pragma unroll
                for (int j = 0; j < 4; ++j) take(x[j], u[j]);
            }
            for (; r < r1; ++r) take(a.xrec[r], a.urec[r]);
            if (in_g > 0) t.add(g);
            point_finish(a.cons_x, i, old, r1 - r0, t, pri, dual);
        }
    } else {
        __shared__ int gpoint[4][64];
        __shared__ PtSums gsum[4][64];
        // lane j: its point's groups start at group `start` (exclusive scan)
        const int G = has ? cons_groups(r1 - r0) : 0;
        int start = G;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int v = __shfl_up(start, off, 64);
            if (lane >= off) start += v;
        }
        start -= G;
        for (int k = 0; k < G; ++k) gpoint[w][start + k] = lane;
        const int n_groups = __shfl(start + G, 63, 64);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // lane l: group l of the wave, records [g0, g1); its point's range,
        // first group and previous consensus come from the point's lane
        const int jg = lane < n_groups ? gpoint[w][lane] : 0;
        const int q0 = __shfl(r0, jg, 64), q1 = __shfl(r1, jg, 64), sj = __shfl(start, jg, 64);
        const double o0 = __shfl(oldi.x, jg, 64), o1 = __shfl(oldi.y, jg, 64), o2 = __shfl(oldi.z, jg, 64);
        int g0 = 0, g1 = 0;
        double4 old = make_double4(0.0, 0.0, 0.0, 0.0);
        if (lane < n_groups) {
            const int K = cons_group(q1 - q0);
            g0 = q0 + (lane - sj) * K;
            g1 = min(g0 + K, q1);
            old = make_double4(o0, o1, o2, 0.0);
        }
        PtSums g;
        g.clear();
        if constexpr (SCHED == 2) {
            for (int r = g0; r < g1; r += 8) {
                PtCopy<R> x[8];
                PtDual u[8];
#pragma unroll
                for (int k = 0; k < 8; ++k)
                    if (r + k < g1) {
                        x[k] = a.xrec[r + k];
                        u[k] = a.urec[r + k];
                    }
#pragma unroll
                for (int k = 0; k < 8; ++k)
                    if (r + k < g1) g.add(x[k], u[k], old);
            }
        } else {
            // the wave's records are contiguous: tiles of kStageRecs staged
            // through LDS with coalesced loads (the next tile's loads in
            // flight while the lanes sum the current one); a record r of
            // the tile sits at 3 (r + r / 8) so that lanes reading records 8
            // apart hit different banks
            constexpr int T = kStageRecs, PER = 3 * T / 64;
            static_assert(3 * T % 64 == 0, "whole values per lane");
            __shared__ R xs[4][3 * (T + T / 8)];
            __shared__ double us[4][3 * (T + T / 8)];
            const int wa = a.pt_off[p0], wb = a.pt_off[p0 + np];
            R xr[PER];
            double ur[PER];
            auto fetch = [&](int t0) {
                const int n3 = 3 * min(T, wb - t0);
                const R *xg = reinterpret_cast<const R *>(a.xrec + t0);
                const double *ug = reinterpret_cast<const double *>(a.urec + t0);
#pragma unroll
                for (int k = 0; k < PER; ++k) {
                    const int q = lane + 64 * k;
                    if (q < n3) {
                        xr[k] = xg[q];
                        ur[k] = ug[q];
                    }
                }
            };
            if (wa < wb) fetch(wa);
            for (int t0 = wa; t0 < wb; t0 += T) {
                const int n3 = 3 * min(T, wb - t0);
#pragma unroll
                for (int k = 0; k < PER; ++k) {
                    const int q = lane + 64 * k;
                    if (q < n3) {
                        const int li = q + 3 * ((q / 3) >> 3);
                        xs[w][li] = xr[k];
                        us[w][li] = ur[k];
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                if (t0 + T < wb) fetch(t0 + T);
                const int lo = max(g0, t0), hi = min(g1, t0 + T);
                for (int r = lo; r < hi; ++r) {
                    const int rl = r - t0, li = 3 * (rl + (rl >> 3));
                    g.add(PtCopy<R>{xs[w][li], xs[w][li + 1], xs[w][li + 2]},
                          PtDual{us[w][li], us[w][li + 1], us[w][li + 2]}, old);
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
        }
        if (lane < n_groups) gsum[w][lane] = g;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (has) {
            PtSums t;
            t.clear();
            for (int k = 0; k < G; ++k) t.add(gsum[w][start + k]);
            point_finish(a.cons_x, i, oldi, r1 - r0, t, pri, dual);
        }
    }
    pri = wave_sum(pri);
    dual = wave_sum(dual);
    if (lane == 0) {
        pd[2 * w] = pri;
        pd[2 * w + 1] = dual;
    }
}

// Consensus kernel: workgroups [0, pt_blocks) hold kConsWaves consensus
// waves each (never two problems' waves: the layout pads each problem to
// whole workgroups) and add their residual terms in wave order; the rest
// four cameras each.
template <typename R, int SCHED>
__global__ __launch_bounds__(256) void k_consensus(DevArrays<R> a, int pt_blocks)
{
    static_assert(kConsWaves == 4, "four waves per workgroup");
    if ((int)blockIdx.x < pt_blocks) {
        __shared__ double pd[2 * kConsWaves];
        const int lane = threadIdx.x & 63, w = wave_id();
        point_wave<R, SCHED>(a, kConsWaves * blockIdx.x + w, w, lane, pd);
        __syncthreads();
        if (threadIdx.x == 0) {
            double pri = 0.0, dual = 0.0;
#pragma unroll
            for (int k = 0; k < kConsWaves; ++k) {
                pri += pd[2 * k];
                dual += pd[2 * k + 1];
            }
            a.ppart[2 * (long long)blockIdx.x] = pri;
            a.ppart[2 * (long long)blockIdx.x + 1] = dual;
        }
    } else {
        // camera consensus: lane l sums chunks k0 + l, k0 + l + 64, ... in
        // order, then a fixed reduce-scatter adds the lanes
        __shared__ double csum[4][kCpart];
        const int lane = threadIdx.x & 63, w = wave_id();
        const int J = (blockIdx.x - pt_blocks) * 4 + w;
        if (J >= a.n_cams) return;  // whole wave; no barrier follows
        const int k0 = a.cam_chunk0[J], k1 = a.cam_chunk0[J + 1];
        double acc[19];
#pragma unroll
        for (int i = 0; i < 19; ++i) acc[i] = 0.0;
        for (int k = k0 + lane; k < k1; k += 64) {
            const double *c = a.cpart + (long long)k * kCpart;
#pragma unroll
            for (int i = 0; i < 19; ++i) acc[i] += c[i];
        }
        wave_sum19_store(acc, csum[w], lane);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (lane == 0) {
            double S[19];
#pragma unroll
            for (int i = 0; i < 19; ++i) S[i] = csum[w][i];
            // copies of the camera: one per observation, or one per chunk
            // with block local updates
            const double M = a.camera_blocks ? (double)(k1 - k0) : (double)a.cam_count[J];
            double *cy = a.cons_y + (long long)J * kConsY;
            double dd = 0.0, dS = 0.0;
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                const double cn = S[i] / M;
                const double del = cn - cy[i];
                cy[i] = cn;
                dd += del * del;
                dS += del * S[9 + i];
            }
            // sum_k |copy_k - new|^2 = sum |d_k|^2 - 2 del . sum d_k + M |del|^2,
            // d_k = copy_k - old consensus
            const double pri = S[18] - 2.0 * dS + M * dd;
            a.campart[2 * (long long)J] = pri > 0.0 ? pri : 0.0;
            a.campart[2 * (long long)J + 1] = M * dd;
        }
    }
}

// ---------------------------------------------------------------- norms
__device__ __forceinline__ void block_sum4(double *v, double (*sh)[kNormThreads])
{
    const int t = threadIdx.x;
#pragma unroll
    for (int k = 0; k < 4; ++k) sh[k][t] = v[k];
    __syncthreads();
    for (int w = kNormThreads / 2; w >= 1; w >>= 1) {
        if (t < w)
#pragma unroll
            for (int k = 0; k < 4; ++k) sh[k][t] += sh[k][t + w];
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = sh[k][0];
}

template <typename R>
__global__ __launch_bounds__(kNormThreads) void k_norms(DevArrays<R> a)
{
    __shared__ double sh[4][kNormThreads];
    const int p = blockIdx.x;
    const ProblemRange pr = a.prob[p];
    double v[4] = {0.0, 0.0, 0.0, 0.0};  // pri_x, dual_x, pri_y, dual_y
    const int b0 = pr.cw0 / kConsWaves, nb = pr.n_cw / kConsWaves;
#pragma unroll 4
    for (int i = threadIdx.x; i < nb; i += kNormThreads) {
        v[0] += a.ppart[2 * (long long)(b0 + i)];
        v[1] += a.ppart[2 * (long long)(b0 + i) + 1];
    }
#pragma unroll 4
    for (int j = threadIdx.x; j < pr.n_cams; j += kNormThreads) {
        v[2] += a.campart[2 * (long long)(pr.cam0 + j)];
        v[3] += a.campart[2 * (long long)(pr.cam0 + j) + 1];
    }
    block_sum4(v, sh);
    if (threadIdx.x == 0) {
        Ctrl &ct = a.ctrl[p];
        const double rx = ct.rho_x, ry = ct.rho_y;
        const double r_pri = sqrt(v[0] + v[2]);
        const double r_dual = sqrt(rx * rx * v[1] + ry * ry * v[3]);
        ct.primal = r_pri;
        ct.dual = r_dual;
        ct.last_rho_x = rx;
        ct.last_rho_y = ry;
        ct.iteration += 1;
        ct.pending = 1;
        if (!isfinite(r_pri) || !isfinite(r_dual)) ct.nonfinite = 1;
        double ratx = 1.0, raty = 1.0;
        if (ct.balancing) {
            double fac = 1.0;
            if (r_pri > ct.rb_mu * r_dual) fac = ct.rb_tau;
            else if (r_dual > ct.rb_mu * r_pri) fac = 1.0 / ct.rb_tau;
            if (fac != 1.0) {
                const double nx = fmin(fmax(rx * fac, ct.rho_min), ct.rho_max);
                const double ny = fmin(fmax(ry * fac, ct.rho_min), ct.rho_max);
                ratx = rx / nx;
                raty = ry / ny;
                ct.rho_x = nx;
                ct.rho_y = ny;
            }
        }
        ct.ratio_x = ratx;
        ct.ratio_y = raty;
    }
}

// ---------------------------------------------------------------- eval
template <typename R, typename Cam>
__global__ __launch_bounds__(256) void k_eval(DevArrays<R> a, SolverParams sp)
{
    const int lane = threadIdx.x & 63;
    const int c = blockIdx.x * 4 + wave_id();
    if (c >= a.n_chunks) return;  // whole wave
    const long long s = (long long)c * kChunk + lane;
    const int ps = a.pslot[s];
    double val[kEpart] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (ps >= 0) {
        const int J = a.chunk_cam[c];
        const double4 cx = a.cons_x[a.ptid[s]];
        double th[12];
#pragma unroll
        for (int i = 0; i < 9; ++i) th[i] = a.cons_y[(long long)J * kConsY + i];
        th[9] = cx.x; th[10] = cx.y; th[11] = cx.z;
        const auto pr = proj_core<double, false>(th, Cam{});
        const typename Vec<R>::R2 z = a.uv[s];
        const double e0 = (double)z.x - pr.pu, e1 = (double)z.y - pr.pv;
        const double s2 = e0 * e0 + e1 * e1;
        double w;
        val[0] = s2;
        val[1] = loss_phi<double>(sp.loss, sp.loss_param, s2, w);
        val[2] = sqrt(s2);
        const bool m = a.mask[s] != 0;
        val[3] = m ? s2 : 0.0;
        val[4] = m ? 1.0 : 0.0;
    }
#pragma unroll
    for (int i = 0; i < kEpart; ++i) val[i] = wave_sum(val[i]);
    if (lane == 0)
#pragma unroll
        for (int i = 0; i < kEpart; ++i) a.epart[(long long)c * kEpart + i] = val[i];
}

template <typename R>
__global__ __launch_bounds__(kNormThreads) void k_eval_reduce(DevArrays<R> a)
{
    __shared__ double sh[4][kNormThreads];
    const int p = blockIdx.x;
    const ProblemRange pr = a.prob[p];
    double v[4] = {0.0, 0.0, 0.0, 0.0}, w4[4] = {0.0, 0.0, 0.0, 0.0};
    for (int c = threadIdx.x; c < pr.n_chunks; c += kNormThreads) {
        const double *e = a.epart + (long long)(pr.chunk0 + c) * kEpart;
        v[0] += e[0]; v[1] += e[1]; v[2] += e[2]; v[3] += e[3];
        w4[0] += e[4];
    }
    block_sum4(v, sh);
    __syncthreads();
    block_sum4(w4, sh);
    if (threadIdx.x == 0) {
        double *o = a.estats + (long long)p * kEpart;
        o[0] = v[0]; o[1] = v[1]; o[2] = v[2]; o[3] = v[3]; o[4] = w4[0];
    }
}

// ---------------------------------------------------------------- state export
template <typename R>
__global__ __launch_bounds__(256) void k_materialize(DevArrays<R> a, int p, double *copies,
                                                      double *duals)
{
    const ProblemRange pr = a.prob[p];
    const long long s = (long long)pr.chunk0 * kChunk + (long long)blockIdx.x * 256 + threadIdx.x;
    if (s >= (long long)(pr.chunk0 + pr.n_chunks) * kChunk) return;
    const int ps = a.pslot[s];
    if (ps < 0) return;
    const long long k = a.slot_orig[s];
    const long long S = a.n_slots;
    const int J = a.chunk_cam[s / kChunk];
    const Ctrl &ct = a.ctrl[p];
    const double4 cx = a.cons_x[a.ptid[s]];
    const PtCopy<R> xr = a.xrec[ps];
    const PtDual ur = a.urec[ps];
    const double xc[3] = {(double)xr.x, (double)xr.y, (double)xr.z};
    const double xu[3] = {ur.x, ur.y, ur.z};
    const double xs[3] = {cx.x, cx.y, cx.z};
    for (int i = 0; i < 12; ++i) {
        double cp, u, cs, rat;
        if (i < 9) {
            const long long cq = (s / kChunk) * 9 + i;
            cp = a.camera_blocks ? (double)a.copy_yc[cq] : (double)a.copy_y[i * S + s];
            u = a.camera_blocks ? a.dual_yc[cq] : a.dual_y[i * S + s];
            cs = a.cons_y[(long long)J * kConsY + i];
            rat = ct.ratio_y;
        } else {
            cp = xc[i - 9];
            u = xu[i - 9];
            cs = xs[i - 9];
            rat = ct.ratio_x;
        }
        if (ct.pending) u = (u + (cp - cs)) * rat;
        if (copies) copies[k * 12 + i] = cp;
        if (duals) duals[k * 12 + i] = u;
    }
}

}  // namespace

// ---------------------------------------------------------------- launchers
template <typename R>
hipError_t launch_local(const DevArrays<R> &a, const SolverParams &sp, int block_waves,
                        int persistent, int n_cu, hipStream_t s)
{
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
    const dim3 g(grid), b(threads);
    // one instantiation per camera model and local solver
    if (sp.camera == 1) {
        if (sp.solver == 2)
            hipLaunchKernelGGL((k_local<R, CamEuler, 2>), g, b, 0, s, a, sp, persistent);
        else if (sp.solver == 1)
            hipLaunchKernelGGL((k_local<R, CamEuler, 1>), g, b, 0, s, a, sp, persistent);
        else
            hipLaunchKernelGGL((k_local<R, CamEuler, 0>), g, b, 0, s, a, sp, persistent);
    } else {
        if (sp.solver == 2)
            hipLaunchKernelGGL((k_local<R, CamAA, 2>), g, b, 0, s, a, sp, persistent);
        else if (sp.solver == 1)
            hipLaunchKernelGGL((k_local<R, CamAA, 1>), g, b, 0, s, a, sp, persistent);
        else
            hipLaunchKernelGGL((k_local<R, CamAA, 0>), g, b, 0, s, a, sp, persistent);
    }
    return hipGetLastError();
}

hipError_t launch_local_learned(const DevArrays<float> &a, const SolverParams &sp, const MlpParams &mp,
                                int persistent, int n_cu, hipStream_t s)
{
    // always persistent: one workgroup per CU stages the weights once
    (void)persistent;
    int grid = n_cu;
    const int need = (a.n_chunks + kLearnedWaves - 1) / kLearnedWaves;
    if (grid > need) grid = need;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(k_local_learned, dim3(grid), dim3(64 * kLearnedWaves), 0, s, a, sp, mp, 1);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_consensus(const DevArrays<R> &a, int schedule, hipStream_t s)
{
    const int pt_blocks = a.n_cw / kConsWaves, cam_blocks = (a.n_cams + 3) / 4;
    const dim3 grid(pt_blocks + cam_blocks), block(256);
    if (schedule == 2)
        hipLaunchKernelGGL((k_consensus<R, 2>), grid, block, 0, s, a, pt_blocks);
    else if (schedule == 3)
        hipLaunchKernelGGL((k_consensus<R, 3>), grid, block, 0, s, a, pt_blocks);
    else
        hipLaunchKernelGGL((k_consensus<R, 1>), grid, block, 0, s, a, pt_blocks);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_norms(const DevArrays<R> &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_norms<R>, dim3(a.n_problems), dim3(kNormThreads), 0, s, a);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_eval(const DevArrays<R> &a, const SolverParams &sp, hipStream_t s)
{
    if (sp.camera == 1)
        hipLaunchKernelGGL((k_eval<R, CamEuler>), dim3((a.n_chunks + 3) / 4), dim3(256), 0, s, a, sp);
    else
        hipLaunchKernelGGL((k_eval<R, CamAA>), dim3((a.n_chunks + 3) / 4), dim3(256), 0, s, a, sp);
    hipLaunchKernelGGL(k_eval_reduce<R>, dim3(a.n_problems), dim3(kNormThreads), 0, s, a);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_materialize(const DevArrays<R> &a, int problem, double *copies, double *duals,
                              hipStream_t s)
{
    // the problem's slots: caller passes the chunk count through a.prob on device;
    // grid covers the largest possible range and threads beyond the problem exit
    hipLaunchKernelGGL(k_materialize<R>, dim3((unsigned)((a.n_slots + 255) / 256)), dim3(256), 0, s,
                       a, problem, copies, duals);
    return hipGetLastError();
}

#define DBA_INSTANTIATE(R)                                                                        \
    template hipError_t launch_local<R>(const DevArrays<R> &, const SolverParams &, int, int, int, \
                                        hipStream_t);                                             \
    template hipError_t launch_consensus<R>(const DevArrays<R> &, int, hipStream_t);              \
    template hipError_t launch_norms<R>(const DevArrays<R> &, hipStream_t);                       \
    template hipError_t launch_eval<R>(const DevArrays<R> &, const SolverParams &, hipStream_t);  \
    template hipError_t launch_materialize<R>(const DevArrays<R> &, int, double *, double *,      \
                                              hipStream_t);
DBA_INSTANTIATE(float)
DBA_INSTANTIATE(double)

}  // namespace dba
