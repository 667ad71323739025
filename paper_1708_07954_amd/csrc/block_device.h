// block_device.h -- generalised local updates (Sec. 3.1.4, Eqs. 14-15) on
// one wavefront: the local problem of a 64-slot camera chunk, one camera copy
// y (9) shared by the chunk and one point copy x_k (3) per observation lane,
//   F = sum_k [phi(|z_k - pi(y, x_k)|^2) + rho_x/2 |x_k - vx_k|^2]
//       + rho_y/2 |y - vy|^2,
// minimised by robust LM with the rules of the per-observation solve (IRLS
// weights, Marquardt damping lambda diag(H), exactly S steps, acceptance on
// a decrease of F or on a predicted decrease below F's rounding resolution).
// The normal equations are reduced to the camera by the Schur complement on
// the points: each lane forms its point block and its contribution to the
// 9x9 camera system -- of rank 2, U M U^T with U the camera part of its two
// Jacobian rows -- a fixed-order all-reduce sums the contributions, every
// lane factors the 9x9 system (LDL^T) and back-solves its own point.
#pragma once
#include "dba_device.h"

namespace dba {
namespace dev {

// Packed upper triangle of a symmetric 9x9 matrix: index of (i, j), i <= j.
__host__ __device__ constexpr int sym9(int i, int j) { return i * 9 - i * (i - 1) / 2 + (j - i); }

// Fixed-order all-reduce of up to 63 values per lane over the wave, as a
// reduce-scatter: at the level with offset o, lanes whose bit o is clear
// keep the first half of their values, the others the second half, each
// adding its partner's copy; after six levels lane l holds the total of
// value l, which goes through 64 entries of LDS to every lane.  The values
// are streamed in increasing index t into the first level (offset 32):
// value t < 32 waits in b[t], value t >= 32 meets value t - 32, so at most
// 32 partial sums are live.
template <typename T>
__device__ __forceinline__ void rs_first_put(T *b, int t, T v)
{
    if (t < 32)
        b[t] = v;
    else
        b[t - 32] = pair_swap_sum<32>(b[t - 32], v);
}

// The remaining five levels and the broadcast: returns the N sums in every
// lane.
template <typename T, int N>
__device__ __forceinline__ void wave_allreduce_tail(const T *b, T *out, T *lds, int lane)
{
    static_assert(N <= 64, "at most 64 values");
    T c[16], d[8], e[4], f[2];
    rs_level<16, 16>(b, c, lane);
    rs_level<8, 8>(c, d, lane);
    rs_level<4, 4>(d, e, lane);
    rs_level<2, 2>(e, f, lane);
    T g;
    rs_level<1, 1>(f, &g, lane);
    lds[lane] = g;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int j = 0; j < N; ++j) out[j] = lds[j];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Solves the symmetric 9x9 system A x = b (packed upper A) by LDL^T; false
// if a pivot is not positive and finite.
template <typename R>
__device__ __forceinline__ bool ldl9_solve(const R *A, const R *b, R *x)
{
    R L[45], D[9], iD[9];
    bool ok = true;
#pragma unroll
    for (int j = 0; j < 9; ++j) {
        // t_k = L(j, k) D_k, then every update of column j is one FMA
        R t[9];
#pragma unroll
        for (int k = 0; k < j; ++k) t[k] = L[sym9(k, j)] * D[k];
        R dj = A[sym9(j, j)];
#pragma unroll
        for (int k = 0; k < j; ++k) dj -= L[sym9(k, j)] * t[k];
        ok = ok && (dj > R(0)) && (dj < Num<R>::inf);
        D[j] = dj;
        const R idj = Num<R>::rcp(dj);
        iD[j] = idj;
#pragma unroll
        for (int i = j + 1; i < 9; ++i) {
            R s = A[sym9(j, i)];
#pragma unroll
            for (int k = 0; k < j; ++k) s -= L[sym9(k, i)] * t[k];
            L[sym9(j, i)] = s * idj;   // L(i, j) stored at (j, i)
        }
    }
    R y[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        R s = b[i];
#pragma unroll
        for (int k = 0; k < i; ++k) s -= L[sym9(k, i)] * y[k];
        y[i] = s;
    }
#pragma unroll
    for (int i = 8; i >= 0; --i) {
        R s = y[i] * iD[i];
#pragma unroll
        for (int k = i + 1; k < 9; ++k) s -= L[sym9(i, k)] * x[k];
        x[i] = s;
    }
    return ok;
}

// One lane's part of the block objective: phi + rho_x/2 |x - vx|^2 at the
// projection o of (y, x); +inf when the depth is <= 1e-6.
template <typename R, typename P>
__device__ __forceinline__ R lane_objective(const P &o, const R *th, const R *vx, R z0, R z1, R rx, int kind,
                                            R lp)
{
    if (!(o.depth > R(1e-6))) return Num<R>::inf;
    const R e0 = z0 - o.pu, e1 = z1 - o.pv;
    R w;
    const R phi = loss_phi<R>(kind, lp, e0 * e0 + e1 * e1, w);
    const R d0 = th[9] - vx[0], d1 = th[10] - vx[1], d2 = th[11] - vx[2];
    return phi + R(0.5) * rx * (d0 * d0 + d1 * d1 + d2 * d2);
}

template <typename R>
__device__ __forceinline__ R camera_penalty(const R *y, const R *vy, R ry)
{
    R p = R(0);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const R d = y[i] - vy[i];
        p += d * d;
    }
    return R(0.5) * ry * p;
}

// Block LM.  th = (y (uniform across the wave), x of this lane); inactive
// lanes (no observation) take part in every reduction with zeros.
template <typename R, typename Cam>
__device__ __forceinline__ void block_lm(R *th, const R *vy, const R *vx, R z0, R z1, bool active, R rx, R ry,
                                         int kind, R lp, int steps, R lam, R *lds, int lane)
{
    using P = decltype(proj_core<R, true>(th, Cam{}));
    P cur;
    R fk = R(0);
    if (active) {
        cur = proj_core<R, true>(th, Cam{});
        fk = lane_objective<R>(cur, th, vx, z0, z1, rx, kind, lp);
    }
    R F = wave_sum<R>(fk) + camera_penalty<R>(th, vy, ry);
    for (int it = 0; it < steps; ++it) {
        // linearisation at (y, x_k): J = [U^T | V^T] with U = (J0_y, J1_y)
        // (9x2) and V = (J0_x, J1_x) (3x2); the lane's blocks of the normal
        // matrix are c U U^T (camera), c U V^T (coupling), c V V^T + rho_x I
        // (point), all of rank 2 besides the penalty
        R U0[9], U1[9], V0[3] = {R(0), R(0), R(0)}, V1[3] = {R(0), R(0), R(0)};
        R e0 = R(0), e1 = R(0), c2 = R(0), fr = R(0);
#pragma unroll
        for (int i = 0; i < 9; ++i) U0[i] = U1[i] = R(0);
        if (active) {
            R J0[12], J1[12];
            proj_jac<R>(cur, th, J0, J1);
            e0 = z0 - cur.pu;
            e1 = z1 - cur.pv;
            R w;
            const R s2 = e0 * e0 + e1 * e1;
            loss_phi<R>(kind, lp, s2, w);
            c2 = R(2) * w;
            fr = Num<R>::sqrt(s2) * (fabs(z0) + fabs(z1) + fabs(th[6]));
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                U0[i] = J0[i];
                U1[i] = J1[i];
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                V0[c] = J0[9 + c];
                V1[c] = J1[9 + c];
            }
        }
        const R fres = F + wave_sum<R>(fr);
        // point block H_xx = c V V^T + rho_x I, damped, inverted (adjugate)
        R hx[6], ngx[3];
        hx[0] = rx + c2 * (V0[0] * V0[0] + V1[0] * V1[0]);
        hx[1] = c2 * (V0[0] * V0[1] + V1[0] * V1[1]);
        hx[2] = c2 * (V0[0] * V0[2] + V1[0] * V1[2]);
        hx[3] = rx + c2 * (V0[1] * V0[1] + V1[1] * V1[1]);
        hx[4] = c2 * (V0[1] * V0[2] + V1[1] * V1[2]);
        hx[5] = rx + c2 * (V0[2] * V0[2] + V1[2] * V1[2]);
#pragma unroll
        for (int c = 0; c < 3; ++c) ngx[c] = active ? c2 * (V0[c] * e0 + V1[c] * e1) - rx * (th[9 + c] - vx[c]) : R(0);
        const R a00 = hx[0] * (R(1) + lam), a11 = hx[3] * (R(1) + lam), a22 = hx[5] * (R(1) + lam);
        const R a01 = hx[1], a02 = hx[2], a12 = hx[4];
        const R m00 = a11 * a22 - a12 * a12, m01 = a02 * a12 - a01 * a22, m02 = a01 * a12 - a02 * a11;
        const R det = a00 * m00 + a01 * m01 + a02 * m02;
        bool okx = true;
        R B[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
        if (active) {
            okx = (det > R(0)) && (det < Num<R>::inf);
            const R idet = Num<R>::rcp(det);
            B[0] = m00 * idet;
            B[1] = m01 * idet;
            B[2] = m02 * idet;
            B[3] = (a00 * a22 - a02 * a02) * idet;
            B[4] = (a01 * a02 - a00 * a12) * idet;
            B[5] = (a00 * a11 - a01 * a01) * idet;
        }
        auto bmul = [&](const R *v, R *o) {
            o[0] = B[0] * v[0] + B[1] * v[1] + B[2] * v[2];
            o[1] = B[1] * v[0] + B[3] * v[1] + B[4] * v[2];
            o[2] = B[2] * v[0] + B[4] * v[1] + B[5] * v[2];
        };
        R BV0[3], BV1[3], Bn[3];
        bmul(V0, BV0);
        bmul(V1, BV1);
        bmul(ngx, Bn);
        // Schur contribution C - W B W^T = U M U^T with the 2x2
        // M = c I - c^2 V^T B V, and ng_y - W B ng_x = U (c (e - V^T B ng_x))
        const R g00 = V0[0] * BV0[0] + V0[1] * BV0[1] + V0[2] * BV0[2];
        const R g01 = V0[0] * BV1[0] + V0[1] * BV1[1] + V0[2] * BV1[2];
        const R g11 = V1[0] * BV1[0] + V1[1] * BV1[1] + V1[2] * BV1[2];
        const R cc = c2 * c2;
        const R M00 = c2 - cc * g00, M01 = -cc * g01, M11 = c2 - cc * g11;
        const R h0 = V0[0] * Bn[0] + V0[1] * Bn[1] + V0[2] * Bn[2];
        const R h1 = V1[0] * Bn[0] + V1[1] * Bn[1] + V1[2] * Bn[2];
        const R r0 = c2 * (e0 - h0), r1 = c2 * (e1 - h1);
        // the lane's 63 values, streamed into the first level of the
        // all-reduce in packed order: the Schur contribution's upper
        // triangle (U0_i q0_j + U1_i q1_j with q = M U^T), c |U_i|^2 (the
        // undamped diagonal of the camera block) and U_i . r
        R q0[9], q1[9];
#pragma unroll
        for (int j = 0; j < 9; ++j) {
            q0[j] = M00 * U0[j] + M01 * U1[j];
            q1[j] = M01 * U0[j] + M11 * U1[j];
        }
        R b32[32];
#pragma unroll
        for (int i = 0; i < 9; ++i)
#pragma unroll
            for (int j = i; j < 9; ++j) rs_first_put<R>(b32, sym9(i, j), U0[i] * q0[j] + U1[i] * q1[j]);
#pragma unroll
        for (int i = 0; i < 9; ++i) rs_first_put<R>(b32, 45 + i, c2 * (U0[i] * U0[i] + U1[i] * U1[i]));
#pragma unroll
        for (int i = 0; i < 9; ++i) rs_first_put<R>(b32, 54 + i, U0[i] * r0 + U1[i] * r1);
        rs_first_put<R>(b32, 63, R(0));
        R sum[63];
        wave_allreduce_tail<R, 63>(b32, sum, lds, lane);
        // camera system: S = A_yy - sum_k W B W^T, rhs = ng_y - sum_k W B ng_x
        R Sy[45], ry9[9], dy[9];
#pragma unroll
        for (int q = 0; q < 45; ++q) Sy[q] = sum[q];
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const R hd = ry + sum[45 + i];                      // diag(H_yy)
            Sy[sym9(i, i)] += ry + lam * hd;
            ry9[i] = sum[54 + i] - ry * (th[i] - vy[i]);        // includes the camera penalty
        }
        const bool oky = ldl9_solve<R>(Sy, ry9, dy);
        const bool ok = oky && (__ballot(!okx) == 0ull);
        // point step dx = B (ng_x - W^T dy) = B ng_x - c B V (U^T dy), and the
        // predicted decrease
        R dx[3] = {R(0), R(0), R(0)};
        R pk = R(0);
        if (active) {
            R u0 = R(0), u1 = R(0);
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                u0 += U0[i] * dy[i];
                u1 += U1[i] * dy[i];
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) dx[c] = Bn[c] - c2 * (BV0[c] * u0 + BV1[c] * u1);
            pk = ngx[0] * dx[0] + ngx[1] * dx[1] + ngx[2] * dx[2] +
                 lam * (hx[0] * dx[0] * dx[0] + hx[3] * dx[1] * dx[1] + hx[5] * dx[2] * dx[2]);
        }
        R gdy = R(0), ddy = R(0);
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            gdy += ry9[i] * dy[i];
            ddy += (ry + sum[45 + i]) * dy[i] * dy[i];
        }
        const R pred = R(0.5) * (wave_sum<R>(pk) + gdy + lam * ddy);
        // trial point and its objective
        R tr[12];
#pragma unroll
        for (int i = 0; i < 9; ++i) tr[i] = th[i] + dy[i];
#pragma unroll
        for (int c = 0; c < 3; ++c) tr[9 + c] = th[9 + c] + dx[c];
        P nxt;
        R fn = R(0);
        if (active && ok) {
            nxt = proj_core<R, true>(tr, Cam{});
            fn = lane_objective<R>(nxt, tr, vx, z0, z1, rx, kind, lp);
        }
        const bool bad = __ballot(!(fn < Num<R>::inf)) != 0ull;
        const R Fn = (ok && !bad) ? wave_sum<R>(fn) + camera_penalty<R>(tr, vy, ry) : Num<R>::inf;
        const bool acc = Fn < Num<R>::inf && (Fn < F || pred <= Num<R>::tie * fres);
#pragma unroll
        for (int i = 0; i < 12; ++i) th[i] = acc ? tr[i] : th[i];
        cur.sel(acc && active, nxt);
        F = acc ? Fn : F;
        lam = acc ? lam_down<R>(lam) : lam_up<R>(lam);
    }
}


// ---------------------------------------------------------------- two cameras
// Blocks of two cameras (Sec. 3.1.4 with kappa = 2): lane l holds point copy
// x_l and up to two observations of it, one per camera of the block, with the
// camera copies y_0, y_1 (18 unknowns, uniform across the wave).  Per LM step
// each lane forms its 3x3 point block and, with U_s the camera rows of its
// observation s (9x2), its contribution U_s M_st U_t^T to the 18x18 reduced
// camera system (M 4x4 from the damped, inverted point block); a fixed-order
// reduction sums the contributions into LDS, lanes 0..17 factor the system
// (LDL^T, a column per lane, pivots and columns broadcast between lanes) and
// solve it, and every lane back-substitutes its point.

// Packed upper triangle of a symmetric 18x18 matrix: index of (i, j), i <= j.
__host__ __device__ constexpr int sym18(int i, int j) { return i * 18 - i * (i - 1) / 2 + (j - i); }

constexpr int kB2Sys = 171;                 // packed 18x18
constexpr int kB2Rhs = kB2Sys;              // 18: reduced right-hand side (ng_y - sum W B ng_x)
constexpr int kB2Ngy = kB2Rhs + 18;         // 18: ng_y, the misfit part of -gradient in y
constexpr int kB2Hd = kB2Ngy + 18;          // 18: misfit part of diag(H_yy)
constexpr int kB2Fres = kB2Hd + 18;         // 1: sum of |e| (|z_1| + |z_2| + f)
constexpr int kB2Vals = kB2Fres + 1;        // 226 reduced values
constexpr int kB2Lds = 256 + 64;            // per wave: the reduced values, then reduction scratch

__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The reduce-scatter levels 16 .. 1 of the streamed values in b: lane l's
// total of value l goes to dst[l].
template <typename T>
__device__ __forceinline__ void wave_reduce_to(const T *b, T *dst, int lane)
{
    T c[16], d[8], e[4], f[2];
    rs_level<16, 16>(b, c, lane);
    rs_level<8, 8>(c, d, lane);
    rs_level<4, 4>(d, e, lane);
    rs_level<2, 2>(e, f, lane);
    T g;
    rs_level<1, 1>(f, &g, lane);
    dst[lane] = g;
}

// Value v of lane l (wave-uniform result).
__device__ __forceinline__ float lane_read(float v, int l)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double lane_read(double v, int l)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

// Solves A x = b for the symmetric 18x18 A (packed upper triangle in the
// wave's LDS a, b at a + kB2Rhs) by LDL^T; x is returned in every lane.
// False if a pivot is not positive and finite.  Lane j < 18 holds column j
// of A (a_ij, i <= j) in registers.  Step k broadcasts the pivot and column
// k (a_ki from lane i) and lane j updates a_ij -= a_ki L_jk, keeping L_jk;
// the forward solve broadcasts z_i as it completes, the backward solve
// reads column j of L, which the lanes write back into LDS, and broadcasts
// x_j.  Lanes past 17 shadow lane 17 (their values are never read).
template <typename R>
__device__ __forceinline__ bool ldl18_lanes(R *a, int lane, R *x)
{
    const int j = lane < 18 ? lane : 17;
    R col[18];
#pragma unroll
    for (int i = 0; i < 18; ++i) col[i] = i <= j ? a[sym18(i, j)] : R(0);
    bool ok = true;
    R rdv[18];
#pragma unroll
    for (int k = 0; k < 18; ++k) {
        const R dk = lane_read(col[k], k);
        ok = ok && (dk > R(0)) && (dk < Num<R>::inf);
        const R rdk = Num<R>::rcp(dk);
        rdv[k] = rdk;
        const R ljk = col[k] * rdk;
#pragma unroll
        for (int i = k + 1; i < 18; ++i) col[i] -= lane_read(col[k], i) * ljk;
        col[k] = ljk;
    }
    // L z = b, z_i broadcast as it completes (lane j > i holds L_ji)
    R z[18], acc = a[kB2Rhs + j];
#pragma unroll
    for (int i = 0; i < 18; ++i) {
        z[i] = lane_read(acc, i);
        acc -= col[i] * z[i];
    }
    // column j of L into LDS at (j, i), i > j, for the backward solve
    wave_lds_sync();
    if (lane < 18)
#pragma unroll
        for (int i = 0; i < 18; ++i)
            if (i < j) a[sym18(i, j)] = col[i];
    wave_lds_sync();
    R lc[18];
#pragma unroll
    for (int i = 0; i < 18; ++i) lc[i] = i > j ? a[sym18(j, i)] : R(0);
    // L^T x = D^-1 z, x_i broadcast from i = 17 down
    acc = R(0);
#pragma unroll
    for (int i = 0; i < 18; ++i) acc = j == i ? z[i] * rdv[i] : acc;
#pragma unroll
    for (int i = 17; i >= 0; --i) {
        x[i] = lane_read(acc, i);
        acc -= lc[i] * x[i];
    }
    return ok;
}

// Projection state of a camera model (Proj or ProjE).
template <typename R, typename Cam>
using ProjOf = decltype(proj_core<R, true>(static_cast<const R *>(nullptr), Cam{}));

// Block LM of a two-camera block.  y: the cameras (18, uniform), present
// bit s: camera s has a copy in the block (an absent camera does not move and
// has no penalty); vy: their targets (18, in the wave's LDS); x, vx: this
// lane's point copy and its target; act[s]: this lane has an observation of
// camera s at pixel (z[2s], z[2s+1]).  lds: the wave's kB2Lds values; pst:
// the wave's LDS for the two projections of each lane between LM steps (FP32;
// nullptr: held in registers), which frees their registers during the
// reduction and the factorisation.
template <typename R, typename Cam>
__device__ __forceinline__ void block_lm2(R *y, const R *vy, int present, R *x, const R *vx, const bool *act,
                                          const R *z, R rx, R ry, int kind, R lp, int steps, R lam, R *lds,
                                          ProjOf<R, Cam> *pst, int lane)
{
    using P = ProjOf<R, Cam>;
    R *red = lds, *scr = lds + 256;
    const bool pt = act[0] || act[1];
    auto theta = [&](int s, R *th) {
#pragma unroll
        for (int i = 0; i < 9; ++i) th[i] = y[9 * s + i];
#pragma unroll
        for (int c = 0; c < 3; ++c) th[9 + c] = x[c];
    };
    auto cam_pen = [&](const R *yy) {
        R q = R(0);
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            if (!(present >> s & 1)) continue;
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                if (!cam_active<Cam>(i)) continue;
                const R d = yy[9 * s + i] - vy[9 * s + i];
                q += d * d;
            }
        }
        return R(0.5) * ry * q;
    };
    auto lane_obj = [&](const P *o, const R *xx) {
        R f = R(0);
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            if (!act[s]) continue;
            if (!(o[s].depth > R(1e-6))) return Num<R>::inf;
            const R e0 = z[2 * s] - o[s].pu, e1 = z[2 * s + 1] - o[s].pv;
            R w;
            f += loss_phi<R>(kind, lp, e0 * e0 + e1 * e1, w);
        }
        if (pt) {
            R q = R(0);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const R d = xx[c] - vx[c];
                q += d * d;
            }
            f += R(0.5) * rx * q;
        }
        return f;
    };
    P cur[2];
#pragma unroll
    for (int s = 0; s < 2; ++s)
        if (act[s]) {
            R th[12];
            theta(s, th);
            cur[s] = proj_core<R, true>(th, Cam{});
            if (pst) pst[2 * lane + s] = cur[s];
        }
    R F = wave_sum<R>(lane_obj(cur, x)) + cam_pen(y);
    for (int it = 0; it < steps; ++it) {
        // linearisation of each observation at (y_s, x)
        R U[2][2][9], V[2][2][3], e[2][2], c2[2], fr = R(0);
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            c2[s] = R(0);
            e[s][0] = e[s][1] = R(0);
#pragma unroll
            for (int i = 0; i < 9; ++i) U[s][0][i] = U[s][1][i] = R(0);
#pragma unroll
            for (int k = 0; k < 3; ++k) V[s][0][k] = V[s][1][k] = R(0);
            if (act[s]) {
                R th[12], J0[12], J1[12];
                theta(s, th);
                const P cs = pst ? pst[2 * lane + s] : cur[s];
                proj_jac<R>(cs, th, J0, J1);
                e[s][0] = z[2 * s] - cs.pu;
                e[s][1] = z[2 * s + 1] - cs.pv;
                R w;
                const R s2 = e[s][0] * e[s][0] + e[s][1] * e[s][1];
                loss_phi<R>(kind, lp, s2, w);
                c2[s] = R(2) * w;
                fr += Num<R>::sqrt(s2) * (fabs(z[2 * s]) + fabs(z[2 * s + 1]) + fabs(y[9 * s + 6]));
#pragma unroll
                for (int i = 0; i < 9; ++i) {
                    U[s][0][i] = J0[i];
                    U[s][1][i] = J1[i];
                }
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    V[s][0][k] = J0[9 + k];
                    V[s][1][k] = J1[9 + k];
                }
            }
        }
        // point block H_xx = sum_s c_s V_s V_s^T + rho_x I, damped, inverted
        R hx[6] = {rx, R(0), R(0), rx, R(0), rx}, ngx[3] = {R(0), R(0), R(0)};
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                const R *v = V[s][a];
                hx[0] += c2[s] * v[0] * v[0];
                hx[1] += c2[s] * v[0] * v[1];
                hx[2] += c2[s] * v[0] * v[2];
                hx[3] += c2[s] * v[1] * v[1];
                hx[4] += c2[s] * v[1] * v[2];
                hx[5] += c2[s] * v[2] * v[2];
#pragma unroll
                for (int k = 0; k < 3; ++k) ngx[k] += c2[s] * v[k] * e[s][a];
            }
        if (pt)
#pragma unroll
            for (int k = 0; k < 3; ++k) ngx[k] -= rx * (x[k] - vx[k]);
        const R a00 = hx[0] * (R(1) + lam), a11 = hx[3] * (R(1) + lam), a22 = hx[5] * (R(1) + lam);
        const R a01 = hx[1], a02 = hx[2], a12 = hx[4];
        const R m00 = a11 * a22 - a12 * a12, m01 = a02 * a12 - a01 * a22, m02 = a01 * a12 - a02 * a11;
        const R det = a00 * m00 + a01 * m01 + a02 * m02;
        const bool okx = !pt || ((det > R(0)) && (det < Num<R>::inf));
        const R idet = Num<R>::rcp(det);
        const R B[6] = {m00 * idet, m01 * idet, m02 * idet, (a00 * a22 - a02 * a02) * idet,
                        (a01 * a02 - a00 * a12) * idet, (a00 * a11 - a01 * a01) * idet};
        auto bmul = [&](const R *v, R *o) {
            o[0] = B[0] * v[0] + B[1] * v[1] + B[2] * v[2];
            o[1] = B[1] * v[0] + B[3] * v[1] + B[4] * v[2];
            o[2] = B[2] * v[0] + B[4] * v[1] + B[5] * v[2];
        };
        R Bn[3];
        bmul(ngx, Bn);
        // M_st = delta_st c_s I - c_s c_t V_s^T B V_t (2x2 blocks, pairs st =
        // 00, 01, 11); r_s = c_s (e_s - V_s^T B ng_x)
        R M[3][2][2], r[2][2];
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int a = 0; a < 2; ++a)
                r[s][a] = c2[s] * (e[s][a] - (V[s][a][0] * Bn[0] + V[s][a][1] * Bn[1] + V[s][a][2] * Bn[2]));
#pragma unroll
        for (int p = 0; p < 3; ++p) {
            const int s = p == 2 ? 1 : 0, t = p == 0 ? 0 : 1;
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    R bv[3];
                    bmul(V[t][b], bv);
                    const R g = V[s][a][0] * bv[0] + V[s][a][1] * bv[1] + V[s][a][2] * bv[2];
                    M[p][a][b] = (s == t && a == b ? c2[s] : R(0)) - c2[s] * c2[t] * g;
                }
        }
        // the lane's 226 values streamed in index order into four batches of
        // 64, each reduced into LDS as it fills
        R b32[32];
        auto put = [&](int t, R v) {
            if (t % 64 == 0 && t > 0) wave_reduce_to<R>(b32, red + t - 64, lane);
            rs_first_put<R>(b32, t % 64, v);
        };
        // entry (i, j), camera rows i of s and j of u: U_si^T M_su U_uj =
        // k0 U[u][0][j] + k1 U[u][1][j] with (k0, k1) = U_si^T M_su
#pragma unroll
        for (int i = 0; i < 18; ++i) {
            const int s = i / 9;
            const R a0 = U[s][0][i % 9], a1 = U[s][1][i % 9];
#pragma unroll
            for (int u = s; u < 2; ++u) {
                const int p = s + u;
                const R k0 = a0 * M[p][0][0] + a1 * M[p][1][0];
                const R k1 = a0 * M[p][0][1] + a1 * M[p][1][1];
#pragma unroll
                for (int j = (u == s ? i : 9 * u); j < 9 * u + 9; ++j)
                    put(sym18(i, j), k0 * U[u][0][j % 9] + k1 * U[u][1][j % 9]);
            }
        }
#pragma unroll
        for (int i = 0; i < 18; ++i) {
            const int s = i / 9;
            put(kB2Rhs + i, U[s][0][i % 9] * r[s][0] + U[s][1][i % 9] * r[s][1]);
        }
#pragma unroll
        for (int i = 0; i < 18; ++i) {
            const int s = i / 9;
            put(kB2Ngy + i, c2[s] * (U[s][0][i % 9] * e[s][0] + U[s][1][i % 9] * e[s][1]));
        }
#pragma unroll
        for (int i = 0; i < 18; ++i) {
            const int s = i / 9;
            put(kB2Hd + i, c2[s] * (U[s][0][i % 9] * U[s][0][i % 9] + U[s][1][i % 9] * U[s][1][i % 9]));
        }
        put(kB2Fres, fr);
#pragma unroll
        for (int t = kB2Vals; t < 256; ++t) put(t, R(0));
        wave_reduce_to<R>(b32, red + 192, lane);
        wave_lds_sync();
        const R fres = F + red[kB2Fres];
        // the camera system: penalty and damping on the diagonal, absent cameras fixed
        if (lane < 18) {
            const int i = lane, s = i / 9;
            if (present >> s & 1) {
                red[sym18(i, i)] += ry + lam * (ry + red[kB2Hd + i]);
                red[kB2Rhs + i] -= ry * (y[i] - vy[i]);
            } else {
                red[sym18(i, i)] = R(1);
                red[kB2Rhs + i] = R(0);
            }
        }
        wave_lds_sync();
        R dy[18];
        const bool oky = ldl18_lanes<R>(red, lane, dy);
        const bool ok = oky && (__ballot(!okx) == 0ull);
        // point step dx = B (ng_x - W^T dy), W_s = c_s U_s V_s^T, and the
        // predicted decrease 1/2 (lambda d^T diag(H) d + ng^T d)
        R dx[3] = {R(0), R(0), R(0)}, pk = R(0);
        if (pt) {
            R wdy[3] = {R(0), R(0), R(0)};
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    R u = R(0);
#pragma unroll
                    for (int i = 0; i < 9; ++i) u += U[s][a][i] * dy[9 * s + i];
#pragma unroll
                    for (int k = 0; k < 3; ++k) wdy[k] += c2[s] * V[s][a][k] * u;
                }
            R t3[3] = {ngx[0] - wdy[0], ngx[1] - wdy[1], ngx[2] - wdy[2]};
            bmul(t3, dx);
            pk = ngx[0] * dx[0] + ngx[1] * dx[1] + ngx[2] * dx[2] +
                 lam * (hx[0] * dx[0] * dx[0] + hx[3] * dx[1] * dx[1] + hx[5] * dx[2] * dx[2]);
        }
        R gdy = R(0), ddy = R(0);
#pragma unroll
        for (int i = 0; i < 18; ++i) {
            if (!(present >> (i / 9) & 1)) continue;
            gdy += (red[kB2Ngy + i] - ry * (y[i] - vy[i])) * dy[i];
            ddy += (ry + red[kB2Hd + i]) * dy[i] * dy[i];
        }
        const R pred = R(0.5) * (wave_sum<R>(pk) + gdy + lam * ddy);
        // trial
        R ty[18], tx[3];
#pragma unroll
        for (int i = 0; i < 18; ++i) ty[i] = (present >> (i / 9) & 1) ? y[i] + dy[i] : y[i];
#pragma unroll
        for (int k = 0; k < 3; ++k) tx[k] = x[k] + dx[k];
        P nxt[2];
        R fn = R(0);
        if (ok) {
#pragma unroll
            for (int s = 0; s < 2; ++s)
                if (act[s]) {
                    R th[12];
#pragma unroll
                    for (int i = 0; i < 9; ++i) th[i] = ty[9 * s + i];
#pragma unroll
                    for (int k = 0; k < 3; ++k) th[9 + k] = tx[k];
                    nxt[s] = proj_core<R, true>(th, Cam{});
                }
            fn = lane_obj(nxt, tx);
        }
        const bool bad = __ballot(!(fn < Num<R>::inf)) != 0ull;
        const R Fn = (ok && !bad) ? wave_sum<R>(fn) + cam_pen(ty) : Num<R>::inf;
        const bool acc = Fn < Num<R>::inf && (Fn < F || pred <= Num<R>::tie * fres);
#pragma unroll
        for (int i = 0; i < 18; ++i) y[i] = acc ? ty[i] : y[i];
#pragma unroll
        for (int k = 0; k < 3; ++k) x[k] = acc ? tx[k] : x[k];
        if (acc) {
#pragma unroll
            for (int s = 0; s < 2; ++s)
                if (act[s]) {
                    if (pst) pst[2 * lane + s] = nxt[s];
                    else cur[s] = nxt[s];
                }
        }
        F = acc ? Fn : F;
        lam = acc ? lam_down<R>(lam) : lam_up<R>(lam);
        wave_lds_sync();
    }
}

}  // namespace dev
}  // namespace dba
