// dba_device.h -- device-side math shared by the local-solve kernels:
// camera projection and its Jacobian, misfit losses, the local objective of
// Eq. (9) in scaled form, and the robust Levenberg-Marquardt steps whose
// normal equations are factorised as LDL^T in registers.
#pragma once
#include "dba_internal.h"

#include <math.h>

namespace dba {
namespace dev {

template <typename R> struct Num;
template <> struct Num<float> {
    static constexpr float small2 = 0.0625f;  // |w| < 0.25: Rodrigues coefficients by series
    __device__ static float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
    __device__ static float sqrt(float x) { return sqrtf(x); }
    __device__ static float rsqrt(float x) { return rsqrtf(x); }
    __device__ static void sincos(float x, float *s, float *c) { sincosf(x, s, c); }
    __device__ static float log1p(float x) { return log1pf(x); }
    __device__ static float div(float x, float y) { return x * __builtin_amdgcn_rcpf(y); }
    static constexpr float inf = __builtin_huge_valf();
    static constexpr float tie = 1e-6f;       // predicted decrease F cannot resolve
};
template <> struct Num<double> {
    static constexpr double small2 = 1e-4;    // |w| < 1e-2
    __device__ static double rcp(double x) { return 1.0 / x; }
    __device__ static double sqrt(double x) { return ::sqrt(x); }
    __device__ static double rsqrt(double x) { return 1.0 / ::sqrt(x); }
    __device__ static void sincos(double x, double *s, double *c) { ::sincos(x, s, c); }
    __device__ static double log1p(double x) { return ::log1p(x); }
    __device__ static double div(double x, double y) { return x / y; }
    static constexpr double inf = __builtin_huge_val();
    static constexpr double tie = 1e-13;
};


// Rodrigues coefficients of R(w) X = c X + a (w x X) + b (w.X) w and, for the
// Jacobian, a1 = a'(t)/t and b1 = b'(t)/t; 1 - cos t is formed as 2 sin^2(t/2).
template <typename R, bool DERIV>
__device__ __forceinline__ void rot_coeffs(R t2, R &c, R &a, R &b, R &a1, R &b1)
{
    if (t2 < Num<R>::small2) {
        const R t4 = t2 * t2;
        c = R(1) - t2 * R(0.5) + t4 * R(1.0 / 24.0);
        a = R(1) - t2 * R(1.0 / 6.0) + t4 * R(1.0 / 120.0);
        b = R(0.5) - t2 * R(1.0 / 24.0) + t4 * R(1.0 / 720.0);
        if (DERIV) {
            a1 = R(-1.0 / 3.0) + t2 * R(1.0 / 30.0) - t4 * R(1.0 / 840.0);
            b1 = R(-1.0 / 12.0) + t2 * R(1.0 / 180.0) - t4 * R(1.0 / 6720.0);
        }
    } else {
        const R t = Num<R>::sqrt(t2);
        R sh, ch;
        Num<R>::sincos(t * R(0.5), &sh, &ch);
        const R s = R(2) * sh * ch;
        const R omc = R(2) * sh * sh;
        c = R(1) - omc;
        const R it = Num<R>::rcp(t);
        const R it2 = it * it;
        a = s * it;
        b = omc * it2;
        if (DERIV) {
            a1 = (t * c - s) * it2 * it;
            b1 = (t * s - R(2) * omc) * it2 * it2;
        }
    }
}

// Projection pi(theta), theta = (w, t, f, k1, k2, X), with the intermediate
// values the Jacobian needs (so an accepted trial point's projection is
// reused as the next linearisation point).
template <typename R>
struct Proj {
    R c, a, b, a1, b1;      // Rodrigues coefficients
    R cx0, cx1, cx2, wd;    // w x X, w . X
    R iz, p0, p1, r2, d;    // 1/P_3, P_{1,2}/P_3, r^2, distortion factor
    R pu, pv, depth;        // pixel and depth
    // keep this projection (t false) or take n's, each field by a select: an
    // if around a whole-struct copy has the compiler copy every field twice
    // per LM step
    __device__ __forceinline__ void sel(bool t, const Proj &n)
    {
        c = t ? n.c : c; a = t ? n.a : a; b = t ? n.b : b; a1 = t ? n.a1 : a1; b1 = t ? n.b1 : b1;
        cx0 = t ? n.cx0 : cx0; cx1 = t ? n.cx1 : cx1; cx2 = t ? n.cx2 : cx2; wd = t ? n.wd : wd;
        iz = t ? n.iz : iz; p0 = t ? n.p0 : p0; p1 = t ? n.p1 : p1; r2 = t ? n.r2 : r2; d = t ? n.d : d;
        pu = t ? n.pu : pu; pv = t ? n.pv : pv; depth = t ? n.depth : depth;
    }
};

template <typename R, bool DERIV>
__device__ __forceinline__ Proj<R> proj_core(const R *th)
{
    Proj<R> o;
    const R w0 = th[0], w1 = th[1], w2 = th[2];
    const R X0 = th[9], X1 = th[10], X2 = th[11];
    o.a1 = o.b1 = R(0);
    rot_coeffs<R, DERIV>(w0 * w0 + w1 * w1 + w2 * w2, o.c, o.a, o.b, o.a1, o.b1);
    o.cx0 = w1 * X2 - w2 * X1;
    o.cx1 = w2 * X0 - w0 * X2;
    o.cx2 = w0 * X1 - w1 * X0;
    o.wd = w0 * X0 + w1 * X1 + w2 * X2;
    const R bwd = o.b * o.wd;
    const R P0 = o.c * X0 + o.a * o.cx0 + bwd * w0 + th[3];
    const R P1 = o.c * X1 + o.a * o.cx1 + bwd * w1 + th[4];
    const R P2 = o.c * X2 + o.a * o.cx2 + bwd * w2 + th[5];
    o.depth = P2;
    o.iz = Num<R>::rcp(P2);
    o.p0 = P0 * o.iz;
    o.p1 = P1 * o.iz;
    o.r2 = o.p0 * o.p0 + o.p1 * o.p1;
    o.d = R(1) + o.r2 * (th[7] + th[8] * o.r2);
    const R fd = th[6] * o.d;
    o.pu = fd * o.p0;
    o.pv = fd * o.p1;
    return o;
}

// The two rows of d pi / d theta at the point of `o`.  With A = d pi / d P
// (2x3), row r is
//   d/dw = (A_r.q) w + b (A_r.w) X - a (A_r x X) + b (w.X) A_r,
//          q = a1 (w x X) + b1 (w.X) w - a X,
//   d/dt = A_r,   d/dX = c A_r + a (A_r x w) + b (A_r.w) w,
//   d/df = d p_r, d/dk1 = f r^2 p_r, d/dk2 = f r^4 p_r.
template <typename R>
__device__ __forceinline__ void proj_jac(const Proj<R> &o, const R *th, R *J0, R *J1)
{
    const R w0 = th[0], w1 = th[1], w2 = th[2];
    const R X0 = th[9], X1 = th[10], X2 = th[11];
    const R f = th[6], k1 = th[7], k2 = th[8];
    const R c = o.c, a = o.a, b = o.b, d = o.d, r2 = o.r2, p0 = o.p0, p1 = o.p1;
    const R bwd = b * o.wd;
    const R g = R(2) * k1 + R(4) * k2 * r2;
    const R fq = f * o.iz;
    const R dg = d + g * r2;
    const R A00 = fq * (d + g * p0 * p0), A01 = fq * (g * p0 * p1), A02 = -fq * p0 * dg;
    const R A11 = fq * (d + g * p1 * p1), A12 = -fq * p1 * dg;
    const R b1wd = o.b1 * o.wd;
    const R q0 = o.a1 * o.cx0 + b1wd * w0 - a * X0;
    const R q1 = o.a1 * o.cx1 + b1wd * w1 - a * X1;
    const R q2 = o.a1 * o.cx2 + b1wd * w2 - a * X2;
    const R fr2 = f * r2;
    auto row = [&](R *Jr, R Ar0, R Ar1, R Ar2, R pr) {
        const R Aq = Ar0 * q0 + Ar1 * q1 + Ar2 * q2;
        const R bAw = b * (Ar0 * w0 + Ar1 * w1 + Ar2 * w2);
        Jr[0] = Aq * w0 + bAw * X0 - a * (Ar1 * X2 - Ar2 * X1) + bwd * Ar0;
        Jr[1] = Aq * w1 + bAw * X1 - a * (Ar2 * X0 - Ar0 * X2) + bwd * Ar1;
        Jr[2] = Aq * w2 + bAw * X2 - a * (Ar0 * X1 - Ar1 * X0) + bwd * Ar2;
        Jr[3] = Ar0;
        Jr[4] = Ar1;
        Jr[5] = Ar2;
        Jr[6] = d * pr;
        Jr[7] = fr2 * pr;
        Jr[8] = fr2 * r2 * pr;
        Jr[9] = c * Ar0 + a * (Ar1 * w2 - Ar2 * w1) + bAw * w0;
        Jr[10] = c * Ar1 + a * (Ar2 * w0 - Ar0 * w2) + bAw * w1;
        Jr[11] = c * Ar2 + a * (Ar0 * w1 - Ar1 * w0) + bAw * w2;
    };
    row(J0, A00, A01, A02, p0);
    row(J1, A01, A11, A12, p1);
}

// Camera models, as template tags: CamAA the 9-parameter camera (angle-axis
// w, t, f, k1, k2; proj_core / proj_jac above); CamEuler the camera of
// Sec. 2.1, Eq. (1): (alpha, beta, gamma, t) with R = R3(gamma) R2(beta)
// R1(alpha) (rotations about x, y, z), pixels f (P1/P3, P2/P3) with the
// known focal length f in slot 6; slots 7, 8 unused.
struct CamAA {};
struct CamEuler {};

// Whether parameter i of the 12 (camera 0..8, point 9..11) is an unknown of
// the camera model; the others keep their value and drop out of the solve.
template <typename Cam> __host__ __device__ constexpr bool cam_active(int i) { return true; }
template <> __host__ __device__ constexpr bool cam_active<CamEuler>(int i) { return i < 6 || i > 8; }

template <typename R, bool DERIV>
__device__ __forceinline__ Proj<R> proj_core(const R *th, CamAA)
{
    return proj_core<R, DERIV>(th);
}

template <typename R>
struct ProjE {
    R sa, ca, sb, cb, sg, cg;   // sines and cosines of alpha, beta, gamma
    R x1y, x1z, x2x, x2z;       // X1 = R1 X (y, z), X2 = R2 X1 (x, z; X2_y = X1_y)
    R q0, q1;                   // Q = R3 X2 = P - t (x, y)
    R iz, p0, p1;               // 1/P_3, P_{1,2}/P_3
    R pu, pv, depth;            // pixel and depth
    __device__ __forceinline__ void sel(bool t, const ProjE &n)  // as Proj::sel
    {
        sa = t ? n.sa : sa; ca = t ? n.ca : ca; sb = t ? n.sb : sb; cb = t ? n.cb : cb; sg = t ? n.sg : sg; cg = t ? n.cg : cg;
        x1y = t ? n.x1y : x1y; x1z = t ? n.x1z : x1z; x2x = t ? n.x2x : x2x; x2z = t ? n.x2z : x2z;
        q0 = t ? n.q0 : q0; q1 = t ? n.q1 : q1; iz = t ? n.iz : iz; p0 = t ? n.p0 : p0; p1 = t ? n.p1 : p1;
        pu = t ? n.pu : pu; pv = t ? n.pv : pv; depth = t ? n.depth : depth;
    }
};

template <typename R, bool DERIV>
__device__ __forceinline__ ProjE<R> proj_core(const R *th, CamEuler)
{
    ProjE<R> o;
    Num<R>::sincos(th[0], &o.sa, &o.ca);
    Num<R>::sincos(th[1], &o.sb, &o.cb);
    Num<R>::sincos(th[2], &o.sg, &o.cg);
    const R X0 = th[9], X1 = th[10], X2 = th[11];
    o.x1y = o.ca * X1 - o.sa * X2;
    o.x1z = o.sa * X1 + o.ca * X2;
    o.x2x = o.cb * X0 + o.sb * o.x1z;
    o.x2z = o.cb * o.x1z - o.sb * X0;
    o.q0 = o.cg * o.x2x - o.sg * o.x1y;
    o.q1 = o.sg * o.x2x + o.cg * o.x1y;
    const R P0 = o.q0 + th[3], P1 = o.q1 + th[4], P2 = o.x2z + th[5];
    o.depth = P2;
    o.iz = Num<R>::rcp(P2);
    o.p0 = P0 * o.iz;
    o.p1 = P1 * o.iz;
    o.pu = th[6] * o.p0;
    o.pv = th[6] * o.p1;
    return o;
}

// Rows of d pi / d theta for the Euler camera.  With a = A_r (row r of
// d pi / d P = f / P3 [[1, 0, -p0], [0, 1, -p1]]), c = a R3 and b = c R2:
//   d/dgamma = a . (z x Q), d/dbeta = c . (y x X2), d/dalpha = b . (x x X1),
//   d/dt = a, d/dX = b R1 = a R; slots 6..8 have no column.
template <typename R>
__device__ __forceinline__ void proj_jac(const ProjE<R> &o, const R *th, R *J0, R *J1)
{
    const R fq = th[6] * o.iz;
    auto row = [&](R *Jr, R a0, R a1, R a2) {
        const R c0 = a0 * o.cg + a1 * o.sg, c1 = a1 * o.cg - a0 * o.sg, c2 = a2;
        const R b0 = c0 * o.cb - c2 * o.sb, b1 = c1, b2 = c0 * o.sb + c2 * o.cb;
        Jr[0] = b2 * o.x1y - b1 * o.x1z;
        Jr[1] = c0 * o.x2z - c2 * o.x2x;
        Jr[2] = a1 * o.q0 - a0 * o.q1;
        Jr[3] = a0;
        Jr[4] = a1;
        Jr[5] = a2;
        Jr[6] = R(0);
        Jr[7] = R(0);
        Jr[8] = R(0);
        Jr[9] = b0;
        Jr[10] = b1 * o.ca + b2 * o.sa;
        Jr[11] = b2 * o.ca - b1 * o.sa;
    };
    row(J0, fq, R(0), -fq * o.p0);
    row(J1, R(0), fq, -fq * o.p1);
}

// phi(s) and w = phi'(s) of the misfit loss of Eq. (8).
template <typename R>
__device__ __forceinline__ R loss_phi(int kind, R lp, R s, R &w)
{
    if (kind == 1) {
        const R d2 = lp * lp;
        if (s <= d2) { w = R(1); return s; }
        const R r = Num<R>::sqrt(s);
        w = Num<R>::div(lp, r);
        return R(2) * lp * r - d2;
    }
    if (kind == 2) {
        const R q = Num<R>::div(s, lp);
        w = Num<R>::rcp(R(1) + q);
        return lp * Num<R>::log1p(q);
    }
    w = R(1);
    return s;
}

// Local objective of Eq. (9) in scaled form at the point of `o`:
// phi(|z - pi|^2) + 1/2 sum_i P_i (theta_i - v_i)^2, P = (rho_y x9, rho_x x3);
// +inf when the depth is <= 1e-6.
template <typename R, typename Cam = CamAA, typename P>
__device__ __forceinline__ R objective(const P &o, const R *th, const R *v, R z0, R z1,
                                       R rx, R ry, int kind, R lp)
{
    if (!(o.depth > R(1e-6))) return Num<R>::inf;
    const R e0 = z0 - o.pu, e1 = z1 - o.pv;
    R w;
    const R phi = loss_phi<R>(kind, lp, e0 * e0 + e1 * e1, w);
    R pen = R(0);
#pragma unroll
    for (int i = 0; i < 12; ++i) {
        if (!cam_active<Cam>(i)) continue;
        const R dd = th[i] - v[i];
        pen += (i < 9 ? ry : rx) * dd * dd;
    }
    return phi + R(0.5) * pen;
}

template <typename R> __device__ __forceinline__ R lam_down(R l);
template <> __device__ __forceinline__ float lam_down(float l) { return fmaxf(l * 0.1f, 1e-12f); }
template <> __device__ __forceinline__ double lam_down(double l) { return fmax(l / 10.0, 1e-12); }
template <typename R> __device__ __forceinline__ R lam_up(R l) { return l * R(10) < R(1e12) ? l * R(10) : R(1e12); }

// Solves (D + c (J0 J0^T + J1 J1^T)) x = g, D = diag(Dd) > 0, c > 0 -- the
// damped Gauss-Newton system of one local problem.  Returns false when a
// pivot is not positive and finite (the step is then rejected).
//
// LDL^T (Cholesky) factor by two rank-one updates of the diagonal factor
// (Gill, Golub, Murray & Saunders 1974, method C1): A = L1 L2 D2 L2^T L1^T
// with unit lower-triangular L1 = I + low(J0 b1^T), L2 = I + low(q b2^T),
// q = L1^-1 J1; O(12) operations, one reciprocal per row and update.  (The
// Sherman-Morrison-Woodbury form of the same solve, x = D^-1 (g - U y), takes
// 13 % less time in the local-solve kernel, but in FP32 it moves the weakly
// determined parameters -- radial distortion of cameras whose points sit
// near the image centre -- further from FP64: 3e-4 against 1.6e-5 after one
// ADMM iteration of the 2M-observation trajectory.)
template <typename R, typename Cam = CamAA>
__device__ __forceinline__ bool solve_normal(const R *Dd, const R *J0, const R *J1, R c2, const R *ng, R *x)
{
    // rank-one update 1: diag -> L1 D1 L1^T (p = J0); alpha_{j+1} =
    // alpha_j d_j / d1_j, one reciprocal per row
    R b1[12], d1[12], b2[12], q[12], id2[12];
    R al = c2;
#pragma unroll
    for (int j = 0; j < 12; ++j) {
        if (!cam_active<Cam>(j)) continue;  // no unknown: no row
        const R ap = al * J0[j];
        d1[j] = Dd[j] + ap * J0[j];
        const R r = Num<R>::rcp(d1[j]);
        b1[j] = ap * r;
        al = al * Dd[j] * r;
    }
    // rank-one update 2 (z = J1): q = L1^-1 J1, then L2 D2 L2^T
    R S = R(0);
    R al2 = c2;
    bool pos = true;
#pragma unroll
    for (int j = 0; j < 12; ++j) {
        if (!cam_active<Cam>(j)) continue;
        q[j] = J1[j] - J0[j] * S;
        S += b1[j] * q[j];
        const R aq = al2 * q[j];
        const R d2 = d1[j] + aq * q[j];
        pos = pos && (d2 > R(0)) && (d2 < Num<R>::inf);
        const R r = Num<R>::rcp(d2);
        id2[j] = r;
        b2[j] = aq * r;
        al2 = al2 * d1[j] * r;
    }
    const bool ok = pos;
    // solve L1 L2 D2 L2^T L1^T x = -g
    S = R(0);
#pragma unroll
    for (int j = 0; j < 12; ++j) {
        if (!cam_active<Cam>(j)) {
            x[j] = R(0);
            continue;
        }
        x[j] = ng[j] - J0[j] * S;
        S += b1[j] * x[j];
    }
    S = R(0);
#pragma unroll
    for (int j = 0; j < 12; ++j) {
        if (!cam_active<Cam>(j)) continue;
        x[j] = x[j] - q[j] * S;
        S += b2[j] * x[j];
    }
#pragma unroll
    for (int j = 0; j < 12; ++j)
        if (cam_active<Cam>(j)) x[j] *= id2[j];
    S = R(0);
#pragma unroll
    for (int j = 11; j >= 0; --j) {
        if (!cam_active<Cam>(j)) continue;
        x[j] = x[j] - b2[j] * S;
        S += q[j] * x[j];
    }
    S = R(0);
#pragma unroll
    for (int j = 11; j >= 0; --j) {
        if (!cam_active<Cam>(j)) continue;
        x[j] = x[j] - b1[j] * S;
        S += J0[j] * x[j];
    }
    return ok;
}

// Robust LM on the local objective, exactly `steps` steps (rejected ones
// included), Marquardt damping lambda * diag(H).  A trial is accepted if it
// lowers F, or if the model's predicted decrease is below tie times F's
// rounding resolution, F + |e| (|z_1| + |z_2| + f) -- a step that small cannot
// be judged by F in this precision, so the model decides.  A non-finite trial
// (depth <= 1e-6 or a failed factorisation) is rejected.
//
// Normal equations: A = H + lambda diag(H), H = P + 2w J^T J, i.e.
// A = D + c (J0 J0^T + J1 J1^T) with D diagonal and c = 2w, solved in
// registers in O(12) operations (solve_normal).
// GN: Gauss-Newton instead -- no damping (A = H) and every step whose trial
// is finite is taken.
template <typename R, typename Cam, bool GN = false, typename P>
__device__ __forceinline__ void lm_steps(R *th, P &cur, R &F, const R *v, R z0, R z1, R rx,
                                         R ry, int kind, R lp, int steps, R lam)
{
    for (int it = 0; it < steps; ++it) {
        R J0[12], J1[12];
        proj_jac<R>(cur, th, J0, J1);
        const R e0 = z0 - cur.pu, e1 = z1 - cur.pv;
        R w;
        const R s2 = e0 * e0 + e1 * e1;
        loss_phi<R>(kind, lp, s2, w);
        const R c2 = R(2) * w;
        // rounding resolution of F here: e = z - pi loses ~eps |z|
        const R fres = F + Num<R>::sqrt(s2) * (fabs(z0) + fabs(z1) + fabs(th[6]));
        R x[12], ng[12], hd[12], Dd[12];
#pragma unroll
        for (int i = 0; i < 12; ++i) {
            if (!cam_active<Cam>(i)) continue;  // not an unknown of the camera model
            const R Pi = i < 9 ? ry : rx;
            ng[i] = c2 * (J0[i] * e0 + J1[i] * e1) - Pi * (th[i] - v[i]);  // -gradient
            hd[i] = Pi + c2 * (J0[i] * J0[i] + J1[i] * J1[i]);             // diag(H)
            Dd[i] = GN ? Pi : Pi + lam * hd[i];                             // A - c J^T J
        }
        const bool ok = solve_normal<R, Cam>(Dd, J0, J1, c2, ng, x);
        R tr[12];
        R gd = R(0), dd = R(0);
#pragma unroll
        for (int i = 0; i < 12; ++i) {
            if (!cam_active<Cam>(i)) {
                tr[i] = th[i];
                continue;
            }
            tr[i] = th[i] + x[i];
            gd += ng[i] * x[i];
            dd += hd[i] * x[i] * x[i];
        }
        // decrease predicted by the damped Gauss-Newton model
        const R pred = R(0.5) * (lam * dd + gd);
        const P nxt = proj_core<R, true>(tr, Cam{});
        const R Fn = ok ? objective<R, Cam>(nxt, tr, v, z0, z1, rx, ry, kind, lp) : Num<R>::inf;
        // accept a decrease of F, or a step too small for F to judge
        const bool acc = Fn < Num<R>::inf && (GN || Fn < F || pred <= Num<R>::tie * fres);
#pragma unroll
        for (int i = 0; i < 12; ++i) th[i] = acc ? tr[i] : th[i];
        cur.sel(acc, nxt);
        F = acc ? Fn : F;
        lam = acc ? lam_down<R>(lam) : lam_up<R>(lam);
    }
}

// L-BFGS on the local objective (Nocedal & Wright, Alg. 7.4 and 7.5), the
// paper's solver for the Huber misfit: `steps` iterations of d = -H g, where H
// is built from the initial matrix diag(P + 2w J^T J)^-1 at the current iterate
// by the BFGS updates with at most kLbfgsMem curvature pairs; an accepted step's
// pair is s = alpha d, y = g_new - g_old formed as P s + (misfit gradient
// difference), kept only if s.y > 1e-8 s^T P s, the oldest dropped when full.
// The solve ends once the predicted decrease -g.d is at most 1e-13 of F's
// resolution (FP64's tie, in both precisions).  Line search: alpha = 1, 1/2,
// ..., 2^-9; the first trial with finite F' <= F + 1e-4 alpha g.d (Armijo), or
// with both terms of the Gauss-Newton model along the step, -alpha g.d and
// alpha^2/2 d^T (P + 2w J^T J) d, at most tie times F's resolution (too small
// for F to judge, as in the LM), is taken; an iteration with no trial taken
// ends the solve.
//
// The pairs live in registers, newest in slot kLbfgsMem - 1: a new pair
// shifts the others down one slot, so every index is a compile-time constant.
constexpr int kLbfgsMem = 4;
constexpr int kLbfgsTrials = 10;

template <typename R, typename Cam, typename P>
__device__ __forceinline__ void lbfgs_steps(R *th, P &cur, R &F, const R *v, R z0, R z1, R rx,
                                            R ry, int kind, R lp, int steps)
{
    R S[kLbfgsMem][12], Y[kLbfgsMem][12], rk[kLbfgsMem];
    R gm_old[12], sl[12];
    int np = 0;
    bool have = false;
    for (int it = 0; it < steps; ++it) {
        R J0[12], J1[12];
        proj_jac<R>(cur, th, J0, J1);
        const R e0 = z0 - cur.pu, e1 = z1 - cur.pv;
        R w;
        const R s2 = e0 * e0 + e1 * e1;
        loss_phi<R>(kind, lp, s2, w);
        const R c2 = R(2) * w;
        const R fres = F + Num<R>::sqrt(s2) * (fabs(z0) + fabs(z1) + fabs(th[6]));
        R gm[12], g[12], h0[12];
#pragma unroll
        for (int i = 0; i < 12; ++i) {
            if (!cam_active<Cam>(i)) continue;
            const R Pi = i < 9 ? ry : rx;
            gm[i] = -c2 * (J0[i] * e0 + J1[i] * e1);
            g[i] = gm[i] + Pi * (th[i] - v[i]);
            h0[i] = Num<R>::rcp(Pi + c2 * (J0[i] * J0[i] + J1[i] * J1[i]));
        }
        if (have) {
            R y[12], sy = R(0), sps = R(0);
#pragma unroll
            for (int i = 0; i < 12; ++i) {
                if (!cam_active<Cam>(i)) continue;
                const R ps = (i < 9 ? ry : rx) * sl[i];
                y[i] = ps + (gm[i] - gm_old[i]);
                sy += sl[i] * y[i];
                sps += ps * sl[i];
            }
            if (sy > R(1e-8) * sps) {
#pragma unroll
                for (int k = 0; k + 1 < kLbfgsMem; ++k) {
                    rk[k] = rk[k + 1];
#pragma unroll
                    for (int i = 0; i < 12; ++i) {
                        if (!cam_active<Cam>(i)) continue;
                        S[k][i] = S[k + 1][i];
                        Y[k][i] = Y[k + 1][i];
                    }
                }
                rk[kLbfgsMem - 1] = Num<R>::rcp(sy);
#pragma unroll
                for (int i = 0; i < 12; ++i) {
                    if (!cam_active<Cam>(i)) continue;
                    S[kLbfgsMem - 1][i] = sl[i];
                    Y[kLbfgsMem - 1][i] = y[i];
                }
                np = np < kLbfgsMem ? np + 1 : kLbfgsMem;
            }
        }
        // two-loop recursion: d = H g over the valid slots kLbfgsMem - np ..
        R d[12], al[kLbfgsMem];
#pragma unroll
        for (int i = 0; i < 12; ++i)
            if (cam_active<Cam>(i)) d[i] = g[i];
#pragma unroll
        for (int k = kLbfgsMem - 1; k >= 0; --k) {
            if (k < kLbfgsMem - np) continue;
            R sq = R(0);
#pragma unroll
            for (int i = 0; i < 12; ++i)
                if (cam_active<Cam>(i)) sq += S[k][i] * d[i];
            al[k] = rk[k] * sq;
#pragma unroll
            for (int i = 0; i < 12; ++i)
                if (cam_active<Cam>(i)) d[i] -= al[k] * Y[k][i];
        }
#pragma unroll
        for (int i = 0; i < 12; ++i)
            if (cam_active<Cam>(i)) d[i] *= h0[i];
#pragma unroll
        for (int k = 0; k < kLbfgsMem; ++k) {
            if (k < kLbfgsMem - np) continue;
            R yd = R(0);
#pragma unroll
            for (int i = 0; i < 12; ++i)
                if (cam_active<Cam>(i)) yd += Y[k][i] * d[i];
            const R b = al[k] - rk[k] * yd;
#pragma unroll
            for (int i = 0; i < 12; ++i)
                if (cam_active<Cam>(i)) d[i] += S[k][i] * b;
        }
        R gd = R(0), dpd = R(0), jd0 = R(0), jd1 = R(0);
#pragma unroll
        for (int i = 0; i < 12; ++i) {
            if (!cam_active<Cam>(i)) continue;
            d[i] = -d[i];
            gd += g[i] * d[i];
            dpd += (i < 9 ? ry : rx) * d[i] * d[i];
            jd0 += J0[i] * d[i];
            jd1 += J1[i] * d[i];
        }
        if (-gd <= R(1e-13) * fres) break;
        const R dhd = dpd + c2 * (jd0 * jd0 + jd1 * jd1);
        const R tres = Num<R>::tie * fres;
        // backtracking line search
        R alpha = R(1), tr[12], Fn = Num<R>::inf;
        P nxt = cur;
        bool found = false;
        for (int t = 0; t < kLbfgsTrials && !found; ++t) {
            if (t > 0) alpha *= R(0.5);
#pragma unroll
            for (int i = 0; i < 12; ++i) tr[i] = cam_active<Cam>(i) ? th[i] + alpha * d[i] : th[i];
            nxt = proj_core<R, true>(tr, Cam{});
            Fn = objective<R, Cam>(nxt, tr, v, z0, z1, rx, ry, kind, lp);
            const bool small = -alpha * gd <= tres && R(0.5) * alpha * alpha * dhd <= tres;
            found = Fn < Num<R>::inf && (Fn <= F + R(1e-4) * alpha * gd || small);
        }
        if (!found) break;
#pragma unroll
        for (int i = 0; i < 12; ++i) {
            if (!cam_active<Cam>(i)) continue;
            sl[i] = alpha * d[i];
            gm_old[i] = gm[i];
            th[i] = tr[i];
        }
        cur = nxt;
        F = Fn;
        have = true;
    }
}

// Local solve from th: SOLVER 0 robust LM, 1 Gauss-Newton, 2 L-BFGS.
template <typename R, typename Cam, int SOLVER = 0>
__device__ __forceinline__ void local_lm(R *th, const R *v, R z0, R z1, R rx, R ry, int kind,
                                         R lp, int steps, R lam)
{
    auto cur = proj_core<R, true>(th, Cam{});
    R F = objective<R, Cam>(cur, th, v, z0, z1, rx, ry, kind, lp);
    if constexpr (SOLVER == 2)
        lbfgs_steps<R, Cam>(th, cur, F, v, z0, z1, rx, ry, kind, lp, steps);
    else
        lm_steps<R, Cam, SOLVER == 1>(th, cur, F, v, z0, z1, rx, ry, kind, lp, steps, lam);
}

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
__device__ __forceinline__ void rs_level(const T *in, T *out, int lane)
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

// Butterfly sum over the wave (partners l ^ 32, 16, 8, 4, 2, 1 in that
// order); every lane ends with the same bits.
template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
    v = pair_swap_sum<32>(v, v);
    v = pair_swap_sum<16>(v, v);
    v += xor_lane<8>(v);
    v += xor_lane<4>(v);
    v += xor_lane<2>(v);
    v += xor_lane<1>(v);
    return v;
}

// Sums the 19 per-lane values v[0..18] over the 64 lanes of the wave and
// stores sum k to o[k] (one store per value, from the lane that holds it).
// Halving the values at every level needs 21 exchanges instead of 19 x 6.
__device__ __forceinline__ void wave_sum19_store(const double *v, double *o, int lane)
{
    double a[20], b[10], c[6], d[4], e[2];
#pragma unroll
    for (int j = 0; j < 19; ++j) a[j] = v[j];
    a[19] = 0.0;
    const bool b5 = lane & 32, b4 = lane & 16, b3 = lane & 8, b2 = lane & 4, b1 = lane & 2;
    rs_level<10, 32>(a, b, lane);     // values 10 b5 + [0, 10)
    rs_level<5, 16>(b, c, lane);     // + 5 b4 + [0, 5)
    c[5] = 0.0;
    rs_level<3, 8>(c, d, lane);       // + 3 b3 + [0, 3)   (position 5 is padding)
    d[3] = 0.0;
    rs_level<2, 4>(d, e, lane);       // + 2 b2 + [0, 2)   (position 3 is padding)
    double f;
    rs_level<1, 2>(e, &f, lane);      // + b1
    f += xor_lane<1>(f);
    const int inner = 2 * b2 + b1, mid = 3 * b3 + inner;
    const int k = 10 * b5 + 5 * b4 + mid;
    if (!(lane & 1) && inner < 3 && mid < 5 && k < 19) o[k] = f;
}

// Block -> tile mapping that gives each XCD (blocks are dealt round-robin to
// the 8 XCDs) a contiguous range of tiles, so neighbouring cameras share an L2.
// Index of the calling wave in its workgroup, in a scalar register: the
// compiler cannot tell that threadIdx.x / 64 is the same across a wave, and
// without this keeps every per-chunk index, address and uniform load in
// vector registers.
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// A value every lane of the wave holds the same copy of, moved to scalar
// registers (frees the vector registers a uniform load would otherwise hold).
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ double uniform(double v)
{
    const int lo = __builtin_amdgcn_readfirstlane(__double2loint(v));
    const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(v));
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ int xcd_block()
{
    const int G = gridDim.x, b = blockIdx.x;
    const int q = G >> 3, r = G & 7, x = b & 7;
    return x * q + (x < r ? x : r) + (b >> 3);
}

// Workgroup size of the local kernels.  FP32: up to 8 waves per workgroup;
// FP64 needs more than 256 VGPRs, so at most 4 waves (one per SIMD).
template <typename R> struct LocalBound { static constexpr int threads = 512; };
template <> struct LocalBound<double> { static constexpr int threads = 256; };

// The chunks (or blocks) [c0, c1) of this workgroup: wpb of them, or an even
// share of all of them when the grid is persistent; consecutive ranges go to
// one XCD (xcd_block).
__device__ __forceinline__ void chunk_range(int n_chunks, int wpb, int persistent, int &c0, int &c1)
{
    const int lb = xcd_block();
    if (persistent) {
        const int per = (n_chunks + gridDim.x - 1) / gridDim.x;
        c0 = lb * per;
        c1 = min(c0 + per, n_chunks);
    } else {
        c0 = lb * wpb;
        c1 = min(c0 + wpb, n_chunks);
    }
}


}  // namespace dev
}  // namespace dba
