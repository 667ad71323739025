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

// Value of lane l ^ OFF for a 32-bit word, OFF in {1, 2, 4, 8}: DPP quad
// permutations [1,0,3,2] and [2,3,0,1], a swizzle in bit mode (xor mask 4),
// and a rotation by 8 within 16-lane rows, which is xor 8.
template <int OFF>
__device__ __forceinline__ int xor_lane_b32(int v)
{
    static_assert(OFF == 1 || OFF == 2 || OFF == 4 || OFF == 8, "offset");
    if constexpr (OFF == 1) return __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false);
    else if constexpr (OFF == 2) return __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, false);
    else if constexpr (OFF == 4) return __builtin_amdgcn_ds_swizzle(v, 0x101F);
    else return __builtin_amdgcn_update_dpp(0, v, 0x128, 0xF, 0xF, false);
}

template <int OFF>
__device__ __forceinline__ float xor_lane(float v)
{
    return __int_as_float(xor_lane_b32<OFF>(__float_as_int(v)));
}

template <int OFF>
__device__ __forceinline__ double xor_lane(double v)
{
    const int lo = xor_lane_b32<OFF>(__double2loint(v)), hi = xor_lane_b32<OFF>(__double2hiint(v));
    return __hiloint2double(hi, lo);
}

// Exchange of the upper OFF lanes of x with the lower OFF lanes of y within
// each group of 2 OFF lanes (OFF 16 or 32: v_permlane16/32_swap).  Returns
// x[l] + x[l ^ OFF] in lanes whose bit OFF is clear and y[l ^ OFF] + y[l] in
// the others -- both partners add the same two numbers.
template <int OFF>
__device__ __forceinline__ float pair_swap_sum(float x, float y)
{
    static_assert(OFF == 16 || OFF == 32, "offset");
    const unsigned a = __float_as_uint(x), b = __float_as_uint(y);
    if constexpr (OFF == 32) {
        const auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false);
        return __uint_as_float(r[0]) + __uint_as_float(r[1]);
    } else {
        const auto r = __builtin_amdgcn_permlane16_swap(a, b, false, false);
        return __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
}

template <int OFF>
__device__ __forceinline__ double pair_swap_sum(double x, double y)
{
    static_assert(OFF == 16 || OFF == 32, "offset");
    const unsigned xl = __double2loint(x), xh = __double2hiint(x), yl = __double2loint(y), yh = __double2hiint(y);
    unsigned l0, l1, h0, h1;
    if constexpr (OFF == 32) {
        const auto rl = __builtin_amdgcn_permlane32_swap(xl, yl, false, false);
        const auto rh = __builtin_amdgcn_permlane32_swap(xh, yh, false, false);
        l0 = rl[0]; l1 = rl[1]; h0 = rh[0]; h1 = rh[1];
    } else {
        const auto rl = __builtin_amdgcn_permlane16_swap(xl, yl, false, false);
        const auto rh = __builtin_amdgcn_permlane16_swap(xh, yh, false, false);
        l0 = rl[0]; l1 = rl[1]; h0 = rh[0]; h1 = rh[1];
    }
    return __hiloint2double((int)h0, (int)l0) + __hiloint2double((int)h1, (int)l1);
}

// One level of the reduce-scatter with partner l ^ OFF: lanes whose bit OFF
// is clear keep the first H of the 2H values, the others the last H, each
// adding its partner's copy (the same pairing and operand order at every
// level, so the sums never change).
template <int H, int OFF, typename T>
__device__ __forceinline__ void rs_level_x(const T *in, T *out, int lane)
{
    if constexpr (OFF >= 16) {
#pragma unroll
        for (int j = 0; j < H; ++j) out[j] = pair_swap_sum<OFF>(in[j], in[H + j]);
    } else {
        const bool upper = lane & OFF;
#pragma unroll
        for (int j = 0; j < H; ++j) {
            const T keep = upper ? in[H + j] : in[j];
            const T send = upper ? in[j] : in[H + j];
            out[j] = keep + xor_lane<OFF>(send);
        }
    }
}

// Sums v[0..N) (N <= 64) over the wave in a fixed order and returns the sums
// in every lane.  Reduce-scatter: at the level with offset o, lanes whose
// bit o is clear keep the first half of their values, the others the second
// half, each adding its partner's copy; after six levels lane l holds the
// total of value l, which goes through 64 entries of LDS to every lane.
template <typename T, int N>
__device__ __forceinline__ void wave_allreduce(const T *v, T *out, T *lds, int lane)
{
    static_assert(N <= 64, "at most 64 values");
    T a[64];
#pragma unroll
    for (int j = 0; j < 64; ++j) a[j] = j < N ? v[j] : T(0);
    T b[32], c[16], d[8], e[4], f[2];
    rs_level_x<32, 32>(a, b, lane);
    rs_level_x<16, 16>(b, c, lane);
    rs_level_x<8, 8>(c, d, lane);
    rs_level_x<4, 4>(d, e, lane);
    rs_level_x<2, 2>(e, f, lane);
    T g;
    rs_level_x<1, 1>(f, &g, lane);
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

// Butterfly sum over the wave (partners l ^ 32, 16, 8, 4, 2, 1 in that
// order); every lane ends with the same bits.
template <typename T>
__device__ __forceinline__ T wave_sum_t(T v)
{
    v = pair_swap_sum<32>(v, v);
    v = pair_swap_sum<16>(v, v);
    v += xor_lane<8>(v);
    v += xor_lane<4>(v);
    v += xor_lane<2>(v);
    v += xor_lane<1>(v);
    return v;
}

// Solves the symmetric 9x9 system A x = b (packed upper A) by LDL^T; false
// if a pivot is not positive and finite.
template <typename R>
__device__ __forceinline__ bool ldl9_solve(const R *A, const R *b, R *x)
{
    R L[45], D[9];
    bool ok = true;
#pragma unroll
    for (int j = 0; j < 9; ++j) {
        R dj = A[sym9(j, j)];
#pragma unroll
        for (int k = 0; k < j; ++k) dj -= L[sym9(k, j)] * L[sym9(k, j)] * D[k];
        ok = ok && (dj > R(0)) && (dj < Num<R>::inf);
        D[j] = dj;
        const R idj = Num<R>::rcp(dj);
#pragma unroll
        for (int i = j + 1; i < 9; ++i) {
            R s = A[sym9(j, i)];
#pragma unroll
            for (int k = 0; k < j; ++k) s -= L[sym9(k, i)] * L[sym9(k, j)] * D[k];
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
        R s = y[i] * Num<R>::rcp(D[i]);
#pragma unroll
        for (int k = i + 1; k < 9; ++k) s -= L[sym9(i, k)] * x[k];
        x[i] = s;
    }
    return ok;
}

// One lane's part of the block objective: phi + rho_x/2 |x - vx|^2 at the
// projection o of (y, x); +inf when the depth is <= 1e-6.
template <typename R>
__device__ __forceinline__ R lane_objective(const Proj<R> &o, const R *th, const R *vx, R z0, R z1, R rx, int kind,
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
template <typename R>
__device__ __forceinline__ void block_lm(R *th, const R *vy, const R *vx, R z0, R z1, bool active, R rx, R ry,
                                         int kind, R lp, int steps, R lam, R *lds, int lane)
{
    Proj<R> cur;
    R fk = R(0);
    if (active) {
        cur = proj_core<R, true>(th);
        fk = lane_objective<R>(cur, th, vx, z0, z1, rx, kind, lp);
    }
    R F = wave_sum_t<R>(fk) + camera_penalty<R>(th, vy, ry);
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
        const R fres = F + wave_sum_t<R>(fr);
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
        R red[63];
#pragma unroll
        for (int j = 0; j < 9; ++j) {
            const R q0 = M00 * U0[j] + M01 * U1[j], q1 = M01 * U0[j] + M11 * U1[j];
#pragma unroll
            for (int i = 0; i <= j; ++i) red[sym9(i, j)] = U0[i] * q0 + U1[i] * q1;
            red[45 + j] = c2 * (U0[j] * U0[j] + U1[j] * U1[j]);
            red[54 + j] = U0[j] * r0 + U1[j] * r1;
        }
        R sum[63];
        wave_allreduce<R, 63>(red, sum, lds, lane);
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
        const R pred = R(0.5) * (wave_sum_t<R>(pk) + gdy + lam * ddy);
        // trial point and its objective
        R tr[12];
#pragma unroll
        for (int i = 0; i < 9; ++i) tr[i] = th[i] + dy[i];
#pragma unroll
        for (int c = 0; c < 3; ++c) tr[9 + c] = th[9 + c] + dx[c];
        Proj<R> nxt;
        R fn = R(0);
        if (active && ok) {
            nxt = proj_core<R, true>(tr);
            fn = lane_objective<R>(nxt, tr, vx, z0, z1, rx, kind, lp);
        }
        const bool bad = __ballot(!(fn < Num<R>::inf)) != 0ull;
        const R Fn = (ok && !bad) ? wave_sum_t<R>(fn) + camera_penalty<R>(tr, vy, ry) : Num<R>::inf;
        if (Fn < Num<R>::inf && (Fn < F || pred <= Num<R>::tie * fres)) {
#pragma unroll
            for (int i = 0; i < 12; ++i) th[i] = tr[i];
            if (active) cur = nxt;
            F = Fn;
            lam = lam_down<R>(lam);
        } else {
            lam = lam_up<R>(lam);
        }
    }
}

}  // namespace dev
}  // namespace dba
