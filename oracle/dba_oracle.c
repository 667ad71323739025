/*
 * dba_oracle.c -- plain, single-threaded FP64 reference implementation of
 * ADMM distributed bundle adjustment ("Distributed Bundle Adjustment",
 * Ramamurthy et al.).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code with
 * the GPU path and the GPU path never calls it.
 *
 * Everything is written for clarity, not speed: one observation at a time,
 * dense 12x12 normal equations solved by Cholesky, sums in ascending
 * observation order.  Readings of the paper that it fixes (camera model,
 * loss definitions, local solver, residual norms, rho balancing) are listed
 * in the header of oracle/__init__.py.
 *
 * Build: gcc -O2 -fno-fast-math -ffp-contract=off -shared -fPIC
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_SMALL_ANGLE 1e-2  /* below: Taylor series for the Rodrigues coefficients */
#define ORC_DEPTH_EPS 1e-6    /* depth at or below this: trial point rejected */
#define ORC_LAMBDA_MIN 1e-12
#define ORC_LAMBDA_MAX 1e12
#define ORC_TIE 1e-13         /* predicted decrease (relative to F's resolution) F cannot judge */
#define ORC_LBFGS_MEM 4       /* L-BFGS: curvature pairs kept */
#define ORC_LS_TRIALS 10      /* L-BFGS: backtracking trials per iteration, alpha = 1, 1/2, .., 2^-9 */
#define ORC_ARMIJO 1e-4       /* L-BFGS: sufficient-decrease constant c1 */
#define ORC_CURV 1e-8         /* L-BFGS: a pair is kept only if s.y > 1e-8 s^T P s */

enum { ORC_L2 = 0, ORC_HUBER = 1, ORC_STUDENT_T = 2 };

/* ------------------------------------------------------------------------ */
/* Rotation by an angle-axis vector w (Rodrigues):                          */
/*   R X = c X + a (w x X) + b (w . X) w,  theta = |w|,                     */
/*   c = cos theta, a = sin theta / theta, b = (1 - cos theta) / theta^2.   */
/* For the Jacobian also a1 = (da/dtheta)/theta, b1 = (db/dtheta)/theta.    */
/* ------------------------------------------------------------------------ */
void orc_rot_coeffs(double theta2, double out[5])
{
    double c, a, b, a1, b1;
    if (theta2 < ORC_SMALL_ANGLE * ORC_SMALL_ANGLE) {
        double t2 = theta2, t4 = theta2 * theta2;
        c = 1.0 - t2 / 2.0 + t4 / 24.0;
        a = 1.0 - t2 / 6.0 + t4 / 120.0;
        b = 0.5 - t2 / 24.0 + t4 / 720.0;
        a1 = -1.0 / 3.0 + t2 / 30.0 - t4 / 840.0;
        b1 = -1.0 / 12.0 + t2 / 180.0 - t4 / 6720.0;
    } else {
        /* 1 - cos t is formed as 2 sin^2(t/2), which keeps its relative
         * accuracy for small t */
        double t = sqrt(theta2);
        double s = sin(t);
        double h = sin(0.5 * t);
        double omc = 2.0 * h * h;
        c = cos(t);
        a = s / t;
        b = omc / theta2;
        a1 = (t * c - s) / (theta2 * t);
        b1 = (t * s - 2.0 * omc) / (theta2 * theta2);
    }
    out[0] = c; out[1] = a; out[2] = b; out[3] = a1; out[4] = b1;
}

static void cross3(const double u[3], const double v[3], double o[3])
{
    o[0] = u[1] * v[2] - u[2] * v[1];
    o[1] = u[2] * v[0] - u[0] * v[2];
    o[2] = u[0] * v[1] - u[1] * v[0];
}

static double dot3(const double u[3], const double v[3])
{
    return u[0] * v[0] + u[1] * v[1] + u[2] * v[2];
}

/* Camera transform P = R(w) X + t. */
void orc_transform(const double cam[9], const double X[3], double P[3])
{
    const double *w = cam;
    double k[5], wx[3];
    orc_rot_coeffs(dot3(w, w), k);
    cross3(w, X, wx);
    double wd = dot3(w, X);
    for (int r = 0; r < 3; ++r)
        P[r] = k[0] * X[r] + k[1] * wx[r] + k[2] * wd * w[r] + cam[3 + r];
}

/* Projection pi(cam, X): perspective division (Eq. 1) with focal length and
 * two radial distortion terms.  Returns the depth P_3. */
double orc_project(const double cam[9], const double X[3], double uv[2])
{
    double P[3];
    orc_transform(cam, X, P);
    double p0 = P[0] / P[2], p1 = P[1] / P[2];
    double r2 = p0 * p0 + p1 * p1;
    double d = 1.0 + cam[7] * r2 + cam[8] * r2 * r2;
    uv[0] = cam[6] * d * p0;
    uv[1] = cam[6] * d * p1;
    return P[2];
}

/* Projection and its analytic Jacobian J (2 x 12, row-major) with respect to
 * theta = (cam[0..8], X[0..2]).  Returns the depth. */
double orc_project_jac(const double cam[9], const double X[3], double uv[2], double J[24])
{
    const double *w = cam;
    double k[5], wx[3], P[3];
    orc_rot_coeffs(dot3(w, w), k);
    const double c = k[0], a = k[1], b = k[2], a1 = k[3], b1 = k[4];
    cross3(w, X, wx);
    double wd = dot3(w, X);
    for (int r = 0; r < 3; ++r)
        P[r] = c * X[r] + a * wx[r] + b * wd * w[r] + cam[3 + r];

    /* R = c I + a [w]x + b w w^T */
    double R[3][3];
    double W[3][3] = {{0, -w[2], w[1]}, {w[2], 0, -w[0]}, {-w[1], w[0], 0}};
    for (int r = 0; r < 3; ++r)
        for (int s = 0; s < 3; ++s)
            R[r][s] = (r == s ? c : 0.0) + a * W[r][s] + b * w[r] * w[s];

    /* dRX/dw = -a X w^T + a1 (w x X) w^T - a [X]x + b1 (w.X) w w^T
     *          + b (w X^T + (w.X) I) */
    double XX[3][3] = {{0, -X[2], X[1]}, {X[2], 0, -X[0]}, {-X[1], X[0], 0}};
    double D[3][3];
    for (int r = 0; r < 3; ++r)
        for (int s = 0; s < 3; ++s)
            D[r][s] = -a * X[r] * w[s] + a1 * wx[r] * w[s] - a * XX[r][s]
                      + b1 * wd * w[r] * w[s] + b * (w[r] * X[s] + (r == s ? wd : 0.0));

    const double f = cam[6], k1 = cam[7], k2 = cam[8];
    double q = 1.0 / P[2];
    double p0 = P[0] / P[2], p1 = P[1] / P[2];
    double r2 = p0 * p0 + p1 * p1;
    double d = 1.0 + k1 * r2 + k2 * r2 * r2;
    uv[0] = f * d * p0;
    uv[1] = f * d * p1;

    /* dpi/dp = f (d I + (2 k1 + 4 k2 r2) p p^T);  dp/dP = q [[1,0,-p0],[0,1,-p1]] */
    double g = 2.0 * k1 + 4.0 * k2 * r2;
    double M[2][2] = {{f * (d + g * p0 * p0), f * g * p0 * p1},
                      {f * g * p1 * p0, f * (d + g * p1 * p1)}};
    double dPdP[2][3] = {{q, 0.0, -q * p0}, {0.0, q, -q * p1}};
    double A[2][3]; /* dpi/dP */
    for (int r = 0; r < 2; ++r)
        for (int s = 0; s < 3; ++s)
            A[r][s] = M[r][0] * dPdP[0][s] + M[r][1] * dPdP[1][s];

    for (int r = 0; r < 2; ++r) {
        double *Jr = J + 12 * r;
        for (int s = 0; s < 3; ++s) {
            Jr[s] = A[r][0] * D[0][s] + A[r][1] * D[1][s] + A[r][2] * D[2][s];
            Jr[3 + s] = A[r][s];
            Jr[9 + s] = A[r][0] * R[0][s] + A[r][1] * R[1][s] + A[r][2] * R[2][s];
        }
        double pr = (r == 0) ? p0 : p1;
        Jr[6] = d * pr;
        Jr[7] = f * r2 * pr;
        Jr[8] = f * r2 * r2 * pr;
    }
    return P[2];
}

/* ------------------------------------------------------------------------ */
/* The paper's camera (Sec. 2.1, Eq. 1): y = (alpha, beta, gamma, t), the    */
/* rotation R = R3(gamma) R2(beta) R1(alpha) with R1, R2, R3 the rotations   */
/* about the x, y and z axes, z~ = R x + t, and pixel coordinates            */
/* f (z~1 / z~3, z~2 / z~3) with the known focal length f (cam[6]).  cam[7]  */
/* and cam[8] are not used; their Jacobian columns are zero, so a local      */
/* solve leaves them at their value (6 camera unknowns).                     */
/* ------------------------------------------------------------------------ */
static void rot_x(double a, double M[3][3])
{
    double c = cos(a), s = sin(a);
    double R[3][3] = {{1, 0, 0}, {0, c, -s}, {0, s, c}};
    memcpy(M, R, sizeof(R));
}
static void rot_y(double a, double M[3][3])
{
    double c = cos(a), s = sin(a);
    double R[3][3] = {{c, 0, s}, {0, 1, 0}, {-s, 0, c}};
    memcpy(M, R, sizeof(R));
}
static void rot_z(double a, double M[3][3])
{
    double c = cos(a), s = sin(a);
    double R[3][3] = {{c, -s, 0}, {s, c, 0}, {0, 0, 1}};
    memcpy(M, R, sizeof(R));
}
/* derivatives of the three rotations with respect to their angle */
static void drot_x(double a, double M[3][3])
{
    double c = cos(a), s = sin(a);
    double R[3][3] = {{0, 0, 0}, {0, -s, -c}, {0, c, -s}};
    memcpy(M, R, sizeof(R));
}
static void drot_y(double a, double M[3][3])
{
    double c = cos(a), s = sin(a);
    double R[3][3] = {{-s, 0, c}, {0, 0, 0}, {-c, 0, -s}};
    memcpy(M, R, sizeof(R));
}
static void drot_z(double a, double M[3][3])
{
    double c = cos(a), s = sin(a);
    double R[3][3] = {{-s, -c, 0}, {c, -s, 0}, {0, 0, 0}};
    memcpy(M, R, sizeof(R));
}
static void mat3_mul(double A[3][3], double B[3][3], double C[3][3])
{
    double T[3][3];
    for (int r = 0; r < 3; ++r)
        for (int s = 0; s < 3; ++s) T[r][s] = A[r][0] * B[0][s] + A[r][1] * B[1][s] + A[r][2] * B[2][s];
    memcpy(C, T, sizeof(T));
}

/* R = R3(gamma) R2(beta) R1(alpha) of an Euler camera */
void orc_euler_rotation(const double cam[9], double R[9])
{
    double R1[3][3], R2[3][3], R3[3][3], T[3][3];
    rot_x(cam[0], R1);
    rot_y(cam[1], R2);
    rot_z(cam[2], R3);
    mat3_mul(R2, R1, T);
    mat3_mul(R3, T, T);
    memcpy(R, T, sizeof(T));
}

double orc_project_euler(const double cam[9], const double X[3], double uv[2])
{
    double R[9], P[3];
    orc_euler_rotation(cam, R);
    for (int r = 0; r < 3; ++r) P[r] = R[3 * r] * X[0] + R[3 * r + 1] * X[1] + R[3 * r + 2] * X[2] + cam[3 + r];
    uv[0] = cam[6] * P[0] / P[2];
    uv[1] = cam[6] * P[1] / P[2];
    return P[2];
}

/* Projection and its Jacobian (2 x 12) with respect to (alpha, beta, gamma,
 * t, f, -, -, X); columns 6..8 are zero (f known, no distortion). */
double orc_project_jac_euler(const double cam[9], const double X[3], double uv[2], double J[24])
{
    double R1[3][3], R2[3][3], R3[3][3], D1[3][3], D2[3][3], D3[3][3], R[3][3], Ra[3][3], Rb[3][3], Rc[3][3], T[3][3];
    rot_x(cam[0], R1);
    rot_y(cam[1], R2);
    rot_z(cam[2], R3);
    drot_x(cam[0], D1);
    drot_y(cam[1], D2);
    drot_z(cam[2], D3);
    mat3_mul(R2, R1, T);
    mat3_mul(R3, T, R);       /* R */
    mat3_mul(R2, D1, T);
    mat3_mul(R3, T, Ra);      /* dR / d alpha */
    mat3_mul(D2, R1, T);
    mat3_mul(R3, T, Rb);      /* dR / d beta */
    mat3_mul(R2, R1, T);
    mat3_mul(D3, T, Rc);      /* dR / d gamma */
    double P[3], dP[3][3];    /* dP[angle][row] */
    for (int r = 0; r < 3; ++r) {
        P[r] = R[r][0] * X[0] + R[r][1] * X[1] + R[r][2] * X[2] + cam[3 + r];
        dP[0][r] = Ra[r][0] * X[0] + Ra[r][1] * X[1] + Ra[r][2] * X[2];
        dP[1][r] = Rb[r][0] * X[0] + Rb[r][1] * X[1] + Rb[r][2] * X[2];
        dP[2][r] = Rc[r][0] * X[0] + Rc[r][1] * X[1] + Rc[r][2] * X[2];
    }
    const double f = cam[6], q = 1.0 / P[2];
    const double p0 = P[0] / P[2], p1 = P[1] / P[2];
    uv[0] = f * P[0] / P[2];
    uv[1] = f * P[1] / P[2];
    /* dpi/dP = f q [[1, 0, -p0], [0, 1, -p1]] */
    double A[2][3] = {{f * q, 0.0, -f * q * p0}, {0.0, f * q, -f * q * p1}};
    for (int r = 0; r < 2; ++r) {
        double *Jr = J + 12 * r;
        for (int a = 0; a < 3; ++a) Jr[a] = A[r][0] * dP[a][0] + A[r][1] * dP[a][1] + A[r][2] * dP[a][2];
        for (int s = 0; s < 3; ++s) {
            Jr[3 + s] = A[r][s];
            Jr[9 + s] = A[r][0] * R[0][s] + A[r][1] * R[1][s] + A[r][2] * R[2][s];
        }
        Jr[6] = Jr[7] = Jr[8] = 0.0;
    }
    return P[2];
}

/* Projection of the camera model `camera` (0: angle-axis + t + f + k1, k2;
 * 1: the Euler camera above). */
double orc_project_cam(int camera, const double cam[9], const double X[3], double uv[2])
{
    return camera == 1 ? orc_project_euler(cam, X, uv) : orc_project(cam, X, uv);
}

double orc_project_jac_cam(int camera, const double cam[9], const double X[3], double uv[2], double J[24])
{
    return camera == 1 ? orc_project_jac_euler(cam, X, uv, J) : orc_project_jac(cam, X, uv, J);
}

/* ------------------------------------------------------------------------ */
/* Misfit loss phi_m of the squared residual norm s = |e|^2 (Eq. 5), and     */
/* its derivative phi'(s).  l2: phi = s.  Huber (delta): phi = s inside,     */
/* 2 delta sqrt(s) - delta^2 outside.  Student-t (nu): nu log(1 + s/nu).     */
/* ------------------------------------------------------------------------ */
void orc_loss(int kind, double param, double s, double out[2])
{
    if (kind == ORC_HUBER) {
        double d2 = param * param;
        if (s <= d2) { out[0] = s; out[1] = 1.0; }
        else { double r = sqrt(s); out[0] = 2.0 * param * r - d2; out[1] = param / r; }
    } else if (kind == ORC_STUDENT_T) {
        out[0] = param * log1p(s / param);
        out[1] = 1.0 / (1.0 + s / param);
    } else {
        out[0] = s; out[1] = 1.0;
    }
}

/* ------------------------------------------------------------------------ */
/* Dense symmetric positive definite solve A x = b by Cholesky (A = L L^T). */
/* Returns 0, or -1 on a non-positive (or non-finite) pivot.                */
/* ------------------------------------------------------------------------ */
int orc_cholesky_solve(int n, const double *A, const double *b, double *x)
{
    double Lm[64 * 64];
    double y[64];
    if (n < 1 || n > 64) return -2;
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j <= i; ++j) {
            double s = A[i * n + j];
            for (int k = 0; k < j; ++k) s -= Lm[i * n + k] * Lm[j * n + k];
            if (i == j) {
                if (!(s > 0.0) || !isfinite(s)) return -1;
                Lm[i * n + i] = sqrt(s);
            } else {
                Lm[i * n + j] = s / Lm[j * n + j];
            }
        }
    }
    for (int i = 0; i < n; ++i) {
        double s = b[i];
        for (int k = 0; k < i; ++k) s -= Lm[i * n + k] * y[k];
        y[i] = s / Lm[i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = y[i];
        for (int k = i + 1; k < n; ++k) s -= Lm[k * n + i] * x[k];
        x[i] = s / Lm[i * n + i];
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Local update (Eq. 9) in scaled form: with u = r / rho, minimise           */
/*   F(theta) = phi(|z - pi(theta)|^2) + 1/2 (theta - v)^T P (theta - v),    */
/*   v = consensus - u,  P = diag(rho_y (x9), rho_x (x3)),                   */
/* by robust Levenberg-Marquardt: IRLS weight w = phi'(s), Gauss-Newton      */
/* matrix H = 2 w J^T J + P, Marquardt damping lambda diag(H), exactly       */
/* `steps` steps (rejected ones included), acceptance if F' < F or if the   */
/* step's predicted decrease is below 1e-13 (F + |e| (|z_1| + |z_2| + f)),  */
/* the rounding resolution of F (too small for F to judge).                  */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t loss;
    double loss_param;
    int32_t lm_steps;
    double lambda0;
    int32_t rho_balancing;
    double rb_mu, rb_tau, rho_min, rho_max;
    int32_t camera;  /* 0: angle-axis camera (9 unknowns), 1: Euler camera (6) */
    int32_t solver;  /* 0: robust LM (reading 4), 1: Gauss-Newton (no damping, every finite step taken),
                        2: L-BFGS (orc_local_solve_lbfgs) */
} orc_opts;

double orc_local_objective(const orc_opts *o, const double z[2], const double v[12],
                           const double theta[12], double rho_x, double rho_y)
{
    double uv[2], ls[2];
    double depth = orc_project_cam(o->camera, theta, theta + 9, uv);
    if (!(depth > ORC_DEPTH_EPS)) return INFINITY;
    double e0 = z[0] - uv[0], e1 = z[1] - uv[1];
    orc_loss(o->loss, o->loss_param, e0 * e0 + e1 * e1, ls);
    double pen = 0.0;
    for (int c = 0; c < 12; ++c) {
        double d = theta[c] - v[c];
        pen += (c < 9 ? rho_y : rho_x) * d * d;
    }
    return ls[0] + 0.5 * pen;
}

/* ------------------------------------------------------------------------ */
/* L-BFGS two-loop recursion (Nocedal & Wright, Numerical Optimization,       */
/* Alg. 7.4): d = H g, where H is the inverse-Hessian approximation obtained  */
/* from diag(h0) by the BFGS updates with the pairs (s_k, y_k) = (S + n k,    */
/* Y + n k), k = 0 (oldest) .. np - 1 (newest).  n <= 64, np <= 64.           */
/* ------------------------------------------------------------------------ */
void orc_lbfgs_apply(int n, int np, const double *S, const double *Y, const double *h0,
                     const double *g, double *d)
{
    double q[64], a[64], rk[64];
    for (int r = 0; r < n; ++r) q[r] = g[r];
    for (int k = np - 1; k >= 0; --k) {
        double sy = 0.0, sq = 0.0;
        for (int r = 0; r < n; ++r) {
            sy += S[n * k + r] * Y[n * k + r];
            sq += S[n * k + r] * q[r];
        }
        rk[k] = 1.0 / sy;
        a[k] = rk[k] * sq;
        for (int r = 0; r < n; ++r) q[r] -= a[k] * Y[n * k + r];
    }
    for (int r = 0; r < n; ++r) d[r] = h0[r] * q[r];
    for (int k = 0; k < np; ++k) {
        double yd = 0.0;
        for (int r = 0; r < n; ++r) yd += Y[n * k + r] * d[r];
        const double b = rk[k] * yd;
        for (int r = 0; r < n; ++r) d[r] += S[n * k + r] * (a[k] - b);
    }
}

/* At theta: the misfit's gradient gm = -2 w J^T e (F's gradient is gm +
 * P (theta - v)), the Jacobian J, w = phi'(s), the inverse diagonal of the
 * Gauss-Newton matrix P + 2 w J^T J, and |e| (for F's resolution). */
static void local_gradient(const orc_opts *o, const double z[2], const double theta[12], double rho_x,
                           double rho_y, double gm[12], double J[24], double *w, double h0[12], double *enorm)
{
    double uv[2], ls[2];
    orc_project_jac_cam(o->camera, theta, theta + 9, uv, J);
    double e0 = z[0] - uv[0], e1 = z[1] - uv[1];
    orc_loss(o->loss, o->loss_param, e0 * e0 + e1 * e1, ls);
    for (int r = 0; r < 12; ++r) {
        gm[r] = -2.0 * ls[1] * (J[r] * e0 + J[12 + r] * e1);
        h0[r] = 1.0 / ((r < 9 ? rho_y : rho_x) + 2.0 * ls[1] * (J[r] * J[r] + J[12 + r] * J[12 + r]));
    }
    *w = ls[1];
    *enorm = sqrt(e0 * e0 + e1 * e1);
}

/* ------------------------------------------------------------------------ */
/* Local update (Eq. 9) by L-BFGS (the paper's solver for the Huber misfit,  */
/* Sec. 3.1; Nocedal & Wright Alg. 7.5), reading 12 of oracle/__init__.py:   */
/*   H0 = diag(P + 2 w J^T J)^-1 at the current iterate (the inverse of the  */
/*   Gauss-Newton matrix's diagonal), recomputed every iteration;            */
/*   at most ORC_LBFGS_MEM pairs, the oldest dropped first; the pair of an   */
/*   accepted step is s = alpha d and y = g_new - g_old, formed as           */
/*   P s + (gm_new - gm_old) (the penalty's part exactly), and kept only if  */
/*   s.y > ORC_CURV s^T P s (so H stays positive definite);                  */
/*   `steps` iterations, each: d = -H g, the solve ending if the predicted   */
/*   decrease -g.d is at most 1e-13 of F's resolution (converged as far as   */
/*   F can tell); backtracking from alpha = 1, halving, at most              */
/*   ORC_LS_TRIALS trials; a trial is taken if F is finite there and         */
/*   F' <= F + c1 alpha g.d (Armijo), or if both terms of the Gauss-Newton   */
/*   model of F along the step, -alpha g.d and alpha^2/2 d^T (P + 2w J^T J) d,*/
/*   are at most 1e-13 of F's resolution (too small for F to judge); an      */
/*   iteration with no trial taken ends the solve.                           */
/* f_trace (optional, steps + 1): F after each iteration; alpha_trace        */
/* (optional, steps): the step taken, 0 once the solve has ended.  Returns   */
/* the number of steps taken.                                                */
/* ------------------------------------------------------------------------ */
int orc_local_solve_lbfgs(const orc_opts *o, const double z[2], const double v[12], double theta[12],
                          double rho_x, double rho_y, int steps, double *f_trace, double *alpha_trace)
{
    double h0[12], S[ORC_LBFGS_MEM * 12], Y[ORC_LBFGS_MEM * 12];
    double g[12], gm[12], gm_old[12], s_last[12], d[12], trial[12], J[24];
    int np = 0, have_step = 0, taken = 0, it = 0;
    double F = orc_local_objective(o, z, v, theta, rho_x, rho_y);
    if (f_trace) f_trace[0] = F;
    for (; it < steps; ++it) {
        double en, w;
        local_gradient(o, z, theta, rho_x, rho_y, gm, J, &w, h0, &en);
        for (int r = 0; r < 12; ++r) g[r] = gm[r] + (r < 9 ? rho_y : rho_x) * (theta[r] - v[r]);
        const double fres = F + en * (fabs(z[0]) + fabs(z[1]) + fabs(theta[6]));
        if (have_step) {
            double y[12], sy = 0.0, sps = 0.0;
            for (int r = 0; r < 12; ++r) {
                const double ps = (r < 9 ? rho_y : rho_x) * s_last[r];
                y[r] = ps + (gm[r] - gm_old[r]);
                sy += s_last[r] * y[r];
                sps += ps * s_last[r];
            }
            if (sy > ORC_CURV * sps) {
                if (np == ORC_LBFGS_MEM) {
                    memmove(S, S + 12, sizeof(double) * 12 * (ORC_LBFGS_MEM - 1));
                    memmove(Y, Y + 12, sizeof(double) * 12 * (ORC_LBFGS_MEM - 1));
                    --np;
                }
                memcpy(S + 12 * np, s_last, sizeof(s_last));
                memcpy(Y + 12 * np, y, sizeof(y));
                ++np;
            }
        }
        orc_lbfgs_apply(12, np, S, Y, h0, g, d);
        double gd = 0.0, dpd = 0.0, jd0 = 0.0, jd1 = 0.0;
        for (int r = 0; r < 12; ++r) {
            d[r] = -d[r];
            gd += g[r] * d[r];
            dpd += (r < 9 ? rho_y : rho_x) * d[r] * d[r];
            jd0 += J[r] * d[r];
            jd1 += J[12 + r] * d[r];
        }
        if (-gd <= ORC_TIE * fres) break;
        const double dhd = dpd + 2.0 * w * (jd0 * jd0 + jd1 * jd1);
        double alpha = 1.0, Fn = INFINITY;
        int found = 0;
        for (int t = 0; t < ORC_LS_TRIALS && !found; ++t) {
            if (t > 0) alpha *= 0.5;
            for (int r = 0; r < 12; ++r) trial[r] = theta[r] + alpha * d[r];
            Fn = orc_local_objective(o, z, v, trial, rho_x, rho_y);
            const int small = -alpha * gd <= ORC_TIE * fres && 0.5 * alpha * alpha * dhd <= ORC_TIE * fres;
            found = isfinite(Fn) && (Fn <= F + ORC_ARMIJO * alpha * gd || small);
        }
        if (!found) break;
        for (int r = 0; r < 12; ++r) {
            s_last[r] = alpha * d[r];
            gm_old[r] = gm[r];
        }
        memcpy(theta, trial, sizeof(trial));
        F = Fn;
        have_step = 1;
        ++taken;
        if (f_trace) f_trace[it + 1] = F;
        if (alpha_trace) alpha_trace[it] = alpha;
    }
    for (; it < steps; ++it) {
        if (f_trace) f_trace[it + 1] = F;
        if (alpha_trace) alpha_trace[it] = 0.0;
    }
    return taken;
}

/* theta: in = start point, out = result.  f_trace (optional, steps+1
 * entries): F after each step (entry 0 = at the start).  Returns the number
 * of accepted steps. */
int orc_local_solve(const orc_opts *o, const double z[2], const double v[12],
                    double theta[12], double rho_x, double rho_y, int steps,
                    double *f_trace)
{
    if (o->solver == 2) return orc_local_solve_lbfgs(o, z, v, theta, rho_x, rho_y, steps, f_trace, NULL);
    double lambda = o->lambda0;
    double F = orc_local_objective(o, z, v, theta, rho_x, rho_y);
    if (f_trace) f_trace[0] = F;
    int accepted = 0;
    for (int it = 0; it < steps; ++it) {
        double uv[2], J[24], ls[2];
        orc_project_jac_cam(o->camera, theta, theta + 9, uv, J);
        double e0 = z[0] - uv[0], e1 = z[1] - uv[1];
        orc_loss(o->loss, o->loss_param, e0 * e0 + e1 * e1, ls);
        double w = ls[1];
        /* resolution of F at theta: rounding of e = z - pi is ~eps |z|, so F
         * carries noise ~eps |e| |z| besides eps F (f stands in for the
         * pixel scale of pi) */
        const double fres = F + sqrt(e0 * e0 + e1 * e1) * (fabs(z[0]) + fabs(z[1]) + fabs(theta[6]));
        double g[12], H[144], A[144], rhs[12], delta[12];
        for (int r = 0; r < 12; ++r) {
            double pr = (r < 9 ? rho_y : rho_x);
            g[r] = -2.0 * w * (J[r] * e0 + J[12 + r] * e1) + pr * (theta[r] - v[r]);
            for (int s = 0; s < 12; ++s)
                H[r * 12 + s] = 2.0 * w * (J[r] * J[s] + J[12 + r] * J[12 + s])
                                + (r == s ? pr : 0.0);
        }
        const int gn = o->solver == 1;
        for (int r = 0; r < 12; ++r) {
            for (int s = 0; s < 12; ++s) A[r * 12 + s] = H[r * 12 + s];
            if (!gn) A[r * 12 + r] += lambda * H[r * 12 + r];
            rhs[r] = -g[r];
        }
        int ok = orc_cholesky_solve(12, A, rhs, delta) == 0;
        double Fn = INFINITY, pred = INFINITY;
        double trial[12];
        if (ok) {
            for (int r = 0; r < 12; ++r) trial[r] = theta[r] + delta[r];
            Fn = orc_local_objective(o, z, v, trial, rho_x, rho_y);
            /* decrease predicted by the damped Gauss-Newton model:
             * -g.delta - 1/2 delta^T H delta = 1/2 (lambda sum H_rr delta_r^2 - g.delta) */
            double gd = 0.0, dd = 0.0;
            for (int r = 0; r < 12; ++r) {
                gd += g[r] * delta[r];
                dd += H[r * 12 + r] * delta[r] * delta[r];
            }
            pred = 0.5 * (lambda * dd - gd);
        }
        /* accept a decrease of F; a step whose predicted decrease is below
         * what F can resolve is accepted on the model's word */
        /* Gauss-Newton takes every step whose trial is finite */
        if (ok && isfinite(Fn) && (gn || Fn < F || pred <= ORC_TIE * fres)) {
            memcpy(theta, trial, sizeof(trial));
            F = Fn;
            lambda = fmax(lambda / 10.0, ORC_LAMBDA_MIN);
            ++accepted;
        } else {
            lambda = fmin(lambda * 10.0, ORC_LAMBDA_MAX);
        }
        if (f_trace) f_trace[it + 1] = F;
    }
    return accepted;
}

/* ------------------------------------------------------------------------ */
/* ADMM iterations (Eqs. 9-13) over the whole problem, state updated in      */
/* place.  Per observation k (camera j = obs_cam[k], point i = obs_pt[k]):   */
/*   copy[12k..12k+11] = (y_j^i (9), x_i^j (3)),  dual = scaled duals u.     */
/* One iteration:                                                            */
/*   1. local solve of every observation (Eq. 9), started at its copy;       */
/*   2. consensus (Eqs. 10, 11): mean over each segment of copy + u, summed  */
/*      in ascending observation order;                                      */
/*   3. scaled dual update (Eqs. 12, 13): u += copy - consensus;             */
/*   4. residual norms r_pri = |copy - consensus|,                           */
/*      r_dual = |rho (consensus - previous consensus)| counted once per     */
/*      copy;                                                                */
/*   5. optional residual balancing of rho, duals rescaled by old/new rho.   */
/* trace (optional, 4 per iteration): r_pri, r_dual, rho_x, rho_y used.      */
/* Returns 0, or -1 on bad input.                                            */
/* ------------------------------------------------------------------------ */
/* ------------------------------------------------------------------------ */
/* Learned start of one local update (an extension, reading R14): the start  */
/* is the better of the base point theta (the previous copy) and            */
/* theta + delta (the network's predicted update) by the local objective F, */
/* ties keep the base; `steps` steps of the local solver follow.  Returns 1 */
/* if the predicted start was kept.                                          */
/* ------------------------------------------------------------------------ */
int orc_learned_local_solve(const orc_opts *o, const double z[2], const double v[12], double theta[12],
                            const double delta[12], double rho_x, double rho_y, int steps)
{
    double trial[12];
    for (int c = 0; c < 12; ++c) trial[c] = theta[c] + delta[c];
    const double F0 = orc_local_objective(o, z, v, theta, rho_x, rho_y);
    const double F1 = orc_local_objective(o, z, v, trial, rho_x, rho_y);
    const int kept = F1 < F0;
    if (kept) memcpy(theta, trial, sizeof(trial));
    orc_local_solve(o, z, v, theta, rho_x, rho_y, steps, NULL);
    return kept;
}

/* Features of the learned start (R14) of every observation k at the current */
/* state: feat[26 k ..] = residual z - pi at the copy (2), camera copy minus */
/* camera consensus (9), point copy minus point consensus (3), camera scaled */
/* dual (9), point scaled dual (3).                                          */
void orc_learned_features(int64_t L, const int32_t *obs_cam, const int32_t *obs_pt, const double *obs_uv,
                          const double *cons_y, const double *cons_x, const double *copy, const double *dual,
                          int camera, double *feat)
{
    for (int64_t k = 0; k < L; ++k) {
        const double *th = copy + 12 * k;
        double uv[2];
        orc_project_cam(camera, th, th + 9, uv);
        double *f = feat + 26 * k;
        f[0] = obs_uv[2 * k] - uv[0];
        f[1] = obs_uv[2 * k + 1] - uv[1];
        for (int c = 0; c < 9; ++c) f[2 + c] = th[c] - cons_y[9 * (size_t)obs_cam[k] + c];
        for (int c = 0; c < 3; ++c) f[11 + c] = th[9 + c] - cons_x[3 * (size_t)obs_pt[k] + c];
        for (int c = 0; c < 12; ++c) f[14 + c] = dual[12 * k + c];
    }
}

static int admm_iterate(int64_t L, int32_t m, int32_t n,
                        const int32_t *obs_cam, const int32_t *obs_pt, const double *obs_uv,
                        double *cons_y, double *cons_x, double *copy, double *dual,
                        double *rho, const orc_opts *o, int32_t n_iters, double *trace,
                        const double *start_delta, int32_t start_steps);

int orc_admm_iterate(int64_t L, int32_t m, int32_t n,
                     const int32_t *obs_cam, const int32_t *obs_pt, const double *obs_uv,
                     double *cons_y, double *cons_x, double *copy, double *dual,
                     double *rho, const orc_opts *o, int32_t n_iters, double *trace)
{
    return admm_iterate(L, m, n, obs_cam, obs_pt, obs_uv, cons_y, cons_x, copy, dual, rho, o, n_iters, trace,
                        NULL, 0);
}

/* One ADMM iteration whose local updates start as orc_learned_local_solve */
/* says, from the predicted updates start_delta [L][12], with start_steps   */
/* local-solver steps; the rest of the iteration as orc_admm_iterate.       */
int orc_admm_iterate_learned(int64_t L, int32_t m, int32_t n,
                             const int32_t *obs_cam, const int32_t *obs_pt, const double *obs_uv,
                             double *cons_y, double *cons_x, double *copy, double *dual,
                             double *rho, const orc_opts *o, const double *start_delta, int32_t start_steps,
                             double *trace)
{
    if (!start_delta || start_steps < 0) return -1;
    return admm_iterate(L, m, n, obs_cam, obs_pt, obs_uv, cons_y, cons_x, copy, dual, rho, o, 1, trace,
                        start_delta, start_steps);
}

static int admm_iterate(int64_t L, int32_t m, int32_t n,
                        const int32_t *obs_cam, const int32_t *obs_pt, const double *obs_uv,
                        double *cons_y, double *cons_x, double *copy, double *dual,
                        double *rho, const orc_opts *o, int32_t n_iters, double *trace,
                        const double *start_delta, int32_t start_steps)
{
    double *cnt_y = calloc((size_t)m, sizeof(double));
    double *cnt_x = calloc((size_t)n, sizeof(double));
    double *sum_y = malloc(sizeof(double) * 9 * (size_t)m);
    double *sum_x = malloc(sizeof(double) * 3 * (size_t)n);
    double *old_y = malloc(sizeof(double) * 9 * (size_t)m);
    double *old_x = malloc(sizeof(double) * 3 * (size_t)n);
    if (!cnt_y || !cnt_x || !sum_y || !sum_x || !old_y || !old_x) return -1;
    for (int64_t k = 0; k < L; ++k) {
        if (obs_cam[k] < 0 || obs_cam[k] >= m || obs_pt[k] < 0 || obs_pt[k] >= n) return -1;
        cnt_y[obs_cam[k]] += 1.0;
        cnt_x[obs_pt[k]] += 1.0;
    }

    for (int32_t it = 0; it < n_iters; ++it) {
        const double rx = rho[0], ry = rho[1];
        /* 1. local updates */
        for (int64_t k = 0; k < L; ++k) {
            const int j = obs_cam[k], i = obs_pt[k];
            double v[12];
            for (int c = 0; c < 9; ++c) v[c] = cons_y[9 * j + c] - dual[12 * k + c];
            for (int c = 0; c < 3; ++c) v[9 + c] = cons_x[3 * i + c] - dual[12 * k + 9 + c];
            if (start_delta)
                orc_learned_local_solve(o, obs_uv + 2 * k, v, copy + 12 * k, start_delta + 12 * k, rx, ry,
                                        start_steps);
            else
                orc_local_solve(o, obs_uv + 2 * k, v, copy + 12 * k, rx, ry, o->lm_steps, NULL);
        }
        /* 2. consensus */
        memcpy(old_y, cons_y, sizeof(double) * 9 * (size_t)m);
        memcpy(old_x, cons_x, sizeof(double) * 3 * (size_t)n);
        memset(sum_y, 0, sizeof(double) * 9 * (size_t)m);
        memset(sum_x, 0, sizeof(double) * 3 * (size_t)n);
        for (int64_t k = 0; k < L; ++k) {
            const int j = obs_cam[k], i = obs_pt[k];
            for (int c = 0; c < 9; ++c) sum_y[9 * j + c] += copy[12 * k + c] + dual[12 * k + c];
            for (int c = 0; c < 3; ++c) sum_x[3 * i + c] += copy[12 * k + 9 + c] + dual[12 * k + 9 + c];
        }
        for (int j = 0; j < m; ++j)
            for (int c = 0; c < 9; ++c) cons_y[9 * j + c] = sum_y[9 * j + c] / cnt_y[j];
        for (int i = 0; i < n; ++i)
            for (int c = 0; c < 3; ++c) cons_x[3 * i + c] = sum_x[3 * i + c] / cnt_x[i];
        /* 3. dual update and 4. primal residual */
        double pri2 = 0.0;
        for (int64_t k = 0; k < L; ++k) {
            const int j = obs_cam[k], i = obs_pt[k];
            for (int c = 0; c < 12; ++c) {
                double cv = (c < 9) ? cons_y[9 * j + c] : cons_x[3 * i + c - 9];
                double d = copy[12 * k + c] - cv;
                dual[12 * k + c] += d;
                pri2 += d * d;
            }
        }
        /* 4. dual residual */
        double dy2 = 0.0, dx2 = 0.0;
        for (int j = 0; j < m; ++j) {
            double s = 0.0;
            for (int c = 0; c < 9; ++c) { double d = cons_y[9 * j + c] - old_y[9 * j + c]; s += d * d; }
            dy2 += cnt_y[j] * s;
        }
        for (int i = 0; i < n; ++i) {
            double s = 0.0;
            for (int c = 0; c < 3; ++c) { double d = cons_x[3 * i + c] - old_x[3 * i + c]; s += d * d; }
            dx2 += cnt_x[i] * s;
        }
        double r_pri = sqrt(pri2);
        double r_dual = sqrt(rx * rx * dx2 + ry * ry * dy2);
        if (trace) {
            trace[4 * it + 0] = r_pri; trace[4 * it + 1] = r_dual;
            trace[4 * it + 2] = rx; trace[4 * it + 3] = ry;
        }
        /* 5. residual balancing */
        if (o->rho_balancing) {
            double fac = 1.0;
            if (r_pri > o->rb_mu * r_dual) fac = o->rb_tau;
            else if (r_dual > o->rb_mu * r_pri) fac = 1.0 / o->rb_tau;
            if (fac != 1.0) {
                double nx = fmin(fmax(rx * fac, o->rho_min), o->rho_max);
                double ny = fmin(fmax(ry * fac, o->rho_min), o->rho_max);
                double sx = rx / nx, sy = ry / ny;
                for (int64_t k = 0; k < L; ++k) {
                    for (int c = 0; c < 9; ++c) dual[12 * k + c] *= sy;
                    for (int c = 9; c < 12; ++c) dual[12 * k + c] *= sx;
                }
                rho[0] = nx; rho[1] = ny;
            }
        }
    }
    free(cnt_y); free(cnt_x); free(sum_y); free(sum_x); free(old_y); free(old_x);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Reprojection statistics at the consensus estimate.                        */
/* out[0] = RMSE over all observations, sqrt(sum |e|^2 / L);                 */
/* out[1] = RMSE over observations with mask[k] != 0 (all if mask == NULL);  */
/* out[2] = robust cost sum phi(|e|^2); out[3] = mean |e| over all.          */
/* ------------------------------------------------------------------------ */
void orc_reprojection_stats(int64_t L, const int32_t *obs_cam, const int32_t *obs_pt,
                            const double *obs_uv, const double *cons_y, const double *cons_x,
                            const uint8_t *mask, int loss, double loss_param, int camera, double out[4])
{
    double s_all = 0.0, s_m = 0.0, cost = 0.0, abs_sum = 0.0;
    int64_t n_m = 0;
    for (int64_t k = 0; k < L; ++k) {
        double uv[2], ls[2];
        orc_project_cam(camera, cons_y + 9 * (size_t)obs_cam[k], cons_x + 3 * (size_t)obs_pt[k], uv);
        double e0 = obs_uv[2 * k] - uv[0], e1 = obs_uv[2 * k + 1] - uv[1];
        double s = e0 * e0 + e1 * e1;
        s_all += s;
        abs_sum += sqrt(s);
        orc_loss(loss, loss_param, s, ls);
        cost += ls[0];
        if (!mask || mask[k]) { s_m += s; ++n_m; }
    }
    out[0] = L > 0 ? sqrt(s_all / (double)L) : 0.0;
    out[1] = n_m > 0 ? sqrt(s_m / (double)n_m) : 0.0;
    out[2] = cost;
    out[3] = L > 0 ? abs_sum / (double)L : 0.0;
}

/* ======================================================================== */
/* Generalised local updates (Sec. 3.1.4, Eqs. 14-15): a local problem      */
/* covers a block of observations that share one camera; the block holds   */
/* one copy y of the camera and one copy x_k of each observation's point.   */
/* ======================================================================== */

/* Dense SPD solve for the block systems (n up to a few hundred). */
static int chol_solve_n(int n, const double *A, const double *b, double *x)
{
    double *Lm = malloc(sizeof(double) * (size_t)n * (size_t)n);
    double *yv = malloc(sizeof(double) * (size_t)n);
    int rc = 0;
    if (!Lm || !yv) { free(Lm); free(yv); return -2; }
    for (int i = 0; i < n && rc == 0; ++i) {
        for (int j = 0; j <= i; ++j) {
            double s = A[(size_t)i * n + j];
            for (int k = 0; k < j; ++k) s -= Lm[(size_t)i * n + k] * Lm[(size_t)j * n + k];
            if (i == j) {
                if (!(s > 0.0) || !isfinite(s)) { rc = -1; break; }
                Lm[(size_t)i * n + i] = sqrt(s);
            } else {
                Lm[(size_t)i * n + j] = s / Lm[(size_t)j * n + j];
            }
        }
    }
    if (rc == 0) {
        for (int i = 0; i < n; ++i) {
            double s = b[i];
            for (int k = 0; k < i; ++k) s -= Lm[(size_t)i * n + k] * yv[k];
            yv[i] = s / Lm[(size_t)i * n + i];
        }
        for (int i = n - 1; i >= 0; --i) {
            double s = yv[i];
            for (int k = i + 1; k < n; ++k) s -= Lm[(size_t)k * n + i] * x[k];
            x[i] = s / Lm[(size_t)i * n + i];
        }
    }
    free(Lm);
    free(yv);
    return rc;
}

/* Block objective: sum_k phi(|z_k - pi(y, x_k)|^2) + rho_y/2 |y - vy|^2
 * + sum_k rho_x/2 |x_k - vx_k|^2; +inf if a depth is <= 1e-6.
 * theta = (y (9), x_1 (3), ..., x_nb (3)). */
double orc_block_objective(const orc_opts *o, int nb, const double *z, const double *vy, const double *vx,
                           const double *theta, double rho_x, double rho_y)
{
    double F = 0.0;
    for (int c = 0; c < 9; ++c) {
        double d = theta[c] - vy[c];
        F += 0.5 * rho_y * d * d;
    }
    for (int k = 0; k < nb; ++k) {
        const double *xk = theta + 9 + 3 * k;
        double uv[2], ls[2];
        double depth = orc_project_cam(o->camera, theta, xk, uv);
        if (!(depth > ORC_DEPTH_EPS)) return INFINITY;
        double e0 = z[2 * k] - uv[0], e1 = z[2 * k + 1] - uv[1];
        orc_loss(o->loss, o->loss_param, e0 * e0 + e1 * e1, ls);
        F += ls[0];
        for (int c = 0; c < 3; ++c) {
            double d = xk[c] - vx[3 * k + c];
            F += 0.5 * rho_x * d * d;
        }
    }
    return F;
}

/* Robust LM on the block objective with the rules of orc_local_solve
 * (IRLS weights, Marquardt damping lambda diag(H), exactly `steps` steps,
 * acceptance on a decrease of F or on a predicted decrease below 1e-13 times
 * F's rounding resolution F + sum_k |e_k| (|z_k1| + |z_k2| + f)).  The
 * normal equations of all 9 + 3 nb unknowns are formed densely and solved by
 * Cholesky.  theta in/out; f_trace optional (steps + 1).  Returns the number
 * of accepted steps, or -2 on allocation failure. */
int orc_block_local_solve(const orc_opts *o, int nb, const double *z, const double *vy, const double *vx,
                          double *theta, double rho_x, double rho_y, int steps, double *f_trace)
{
    const int N = 9 + 3 * nb;
    double *g = malloc(sizeof(double) * N), *H = calloc((size_t)N * N, sizeof(double));
    double *A = malloc(sizeof(double) * (size_t)N * N), *rhs = malloc(sizeof(double) * N);
    double *delta = malloc(sizeof(double) * N), *trial = malloc(sizeof(double) * N);
    if (!g || !H || !A || !rhs || !delta || !trial) {
        free(g); free(H); free(A); free(rhs); free(delta); free(trial);
        return -2;
    }
    double lambda = o->lambda0;
    double F = orc_block_objective(o, nb, z, vy, vx, theta, rho_x, rho_y);
    if (f_trace) f_trace[0] = F;
    int accepted = 0;
    for (int it = 0; it < steps; ++it) {
        memset(H, 0, sizeof(double) * (size_t)N * N);
        for (int c = 0; c < 9; ++c) {
            g[c] = rho_y * (theta[c] - vy[c]);
            H[(size_t)c * N + c] = rho_y;
        }
        double fres = F;
        for (int k = 0; k < nb; ++k) {
            const double *xk = theta + 9 + 3 * k;
            double cam_pt[12], uv[2], J[24], ls[2];
            memcpy(cam_pt, theta, 9 * sizeof(double));
            memcpy(cam_pt + 9, xk, 3 * sizeof(double));
            orc_project_jac_cam(o->camera, cam_pt, cam_pt + 9, uv, J);
            double e0 = z[2 * k] - uv[0], e1 = z[2 * k + 1] - uv[1];
            orc_loss(o->loss, o->loss_param, e0 * e0 + e1 * e1, ls);
            const double w = ls[1];
            fres += sqrt(e0 * e0 + e1 * e1) * (fabs(z[2 * k]) + fabs(z[2 * k + 1]) + fabs(theta[6]));
            /* columns of this observation in the block: camera 0..8, point 9+3k.. */
            int col[12];
            for (int c = 0; c < 9; ++c) col[c] = c;
            for (int c = 0; c < 3; ++c) col[9 + c] = 9 + 3 * k + c;
            for (int c = 0; c < 3; ++c) {
                g[col[9 + c]] = rho_x * (xk[c] - vx[3 * k + c]);
                H[(size_t)col[9 + c] * N + col[9 + c]] += rho_x;
            }
            for (int r = 0; r < 12; ++r) {
                g[col[r]] += -2.0 * w * (J[r] * e0 + J[12 + r] * e1);
                for (int s = 0; s < 12; ++s)
                    H[(size_t)col[r] * N + col[s]] += 2.0 * w * (J[r] * J[s] + J[12 + r] * J[12 + s]);
            }
        }
        for (int r = 0; r < N; ++r) {
            for (int s = 0; s < N; ++s) A[(size_t)r * N + s] = H[(size_t)r * N + s];
            A[(size_t)r * N + r] += lambda * H[(size_t)r * N + r];
            rhs[r] = -g[r];
        }
        int ok = chol_solve_n(N, A, rhs, delta) == 0;
        double Fn = INFINITY, pred = INFINITY;
        if (ok) {
            for (int r = 0; r < N; ++r) trial[r] = theta[r] + delta[r];
            Fn = orc_block_objective(o, nb, z, vy, vx, trial, rho_x, rho_y);
            double gd = 0.0, dd = 0.0;
            for (int r = 0; r < N; ++r) {
                gd += g[r] * delta[r];
                dd += H[(size_t)r * N + r] * delta[r] * delta[r];
            }
            pred = 0.5 * (lambda * dd - gd);
        }
        if (ok && isfinite(Fn) && (Fn < F || pred <= ORC_TIE * fres)) {
            memcpy(theta, trial, sizeof(double) * N);
            F = Fn;
            lambda = fmax(lambda / 10.0, ORC_LAMBDA_MIN);
            ++accepted;
        } else {
            lambda = fmin(lambda * 10.0, ORC_LAMBDA_MAX);
        }
        if (f_trace) f_trace[it + 1] = F;
    }
    free(g); free(H); free(A); free(rhs); free(delta); free(trial);
    return accepted;
}

/* ------------------------------------------------------------------------ */
/* General block of the generalised local update (Sec. 3.1.4, Eqs. 14-15):   */
/* nc cameras and np points with ONE copy each in the block, and nobs        */
/* observations between them (observation q: block camera oc[q], block point */
/* op[q], pixel z[2q..2q+1]).  Objective:                                    */
/*   sum_q phi(|z_q - pi(y_oc[q], x_op[q])|^2)                               */
/*   + rho_y/2 sum_c |y_c - vy_c|^2 + rho_x/2 sum_p |x_p - vx_p|^2;          */
/* +inf if a depth is <= 1e-6.  theta = (y_0 .. y_{nc-1} (9 each),           */
/* x_0 .. x_{np-1} (3 each)).                                                */
/* ------------------------------------------------------------------------ */
double orc_gblock_objective(const orc_opts *o, int nc, int np, int nobs, const int32_t *oc, const int32_t *op,
                            const double *z, const double *vy, const double *vx, const double *theta,
                            double rho_x, double rho_y)
{
    double F = 0.0;
    for (int c = 0; c < 9 * nc; ++c) {
        const double d = theta[c] - vy[c];
        F += 0.5 * rho_y * d * d;
    }
    for (int c = 0; c < 3 * np; ++c) {
        const double d = theta[9 * nc + c] - vx[c];
        F += 0.5 * rho_x * d * d;
    }
    for (int q = 0; q < nobs; ++q) {
        double uv[2], ls[2];
        const double depth = orc_project_cam(o->camera, theta + 9 * oc[q], theta + 9 * nc + 3 * op[q], uv);
        if (!(depth > ORC_DEPTH_EPS)) return INFINITY;
        const double e0 = z[2 * q] - uv[0], e1 = z[2 * q + 1] - uv[1];
        orc_loss(o->loss, o->loss_param, e0 * e0 + e1 * e1, ls);
        F += ls[0];
    }
    return F;
}

/* Robust LM on the general block objective with the rules of
 * orc_block_local_solve (dense normal equations over all 9 nc + 3 np
 * unknowns, Cholesky, exactly `steps` steps, the same acceptance and tie
 * rule).  Returns the number of accepted steps, -2 on allocation failure. */
int orc_gblock_local_solve(const orc_opts *o, int nc, int np, int nobs, const int32_t *oc, const int32_t *op,
                           const double *z, const double *vy, const double *vx, double *theta, double rho_x,
                           double rho_y, int steps)
{
    const int N = 9 * nc + 3 * np;
    double *g = malloc(sizeof(double) * N), *H = malloc(sizeof(double) * (size_t)N * N);
    double *A = malloc(sizeof(double) * (size_t)N * N), *rhs = malloc(sizeof(double) * N);
    double *delta = malloc(sizeof(double) * N), *trial = malloc(sizeof(double) * N);
    if (!g || !H || !A || !rhs || !delta || !trial) {
        free(g); free(H); free(A); free(rhs); free(delta); free(trial);
        return -2;
    }
    double lambda = o->lambda0;
    double F = orc_gblock_objective(o, nc, np, nobs, oc, op, z, vy, vx, theta, rho_x, rho_y);
    int accepted = 0;
    for (int it = 0; it < steps; ++it) {
        memset(H, 0, sizeof(double) * (size_t)N * N);
        for (int r = 0; r < N; ++r) {
            const int cam = r < 9 * nc;
            const double pr = cam ? rho_y : rho_x;
            g[r] = pr * (theta[r] - (cam ? vy[r] : vx[r - 9 * nc]));
            H[(size_t)r * N + r] = pr;
        }
        double fres = F;
        for (int q = 0; q < nobs; ++q) {
            const double *yc = theta + 9 * oc[q], *xp = theta + 9 * nc + 3 * op[q];
            double uv[2], J[24], ls[2];
            orc_project_jac_cam(o->camera, yc, xp, uv, J);
            const double e0 = z[2 * q] - uv[0], e1 = z[2 * q + 1] - uv[1];
            orc_loss(o->loss, o->loss_param, e0 * e0 + e1 * e1, ls);
            const double w = ls[1];
            fres += sqrt(e0 * e0 + e1 * e1) * (fabs(z[2 * q]) + fabs(z[2 * q + 1]) + fabs(yc[6]));
            int col[12];
            for (int c = 0; c < 9; ++c) col[c] = 9 * oc[q] + c;
            for (int c = 0; c < 3; ++c) col[9 + c] = 9 * nc + 3 * op[q] + c;
            for (int r = 0; r < 12; ++r) {
                g[col[r]] += -2.0 * w * (J[r] * e0 + J[12 + r] * e1);
                for (int t = 0; t < 12; ++t)
                    H[(size_t)col[r] * N + col[t]] += 2.0 * w * (J[r] * J[t] + J[12 + r] * J[12 + t]);
            }
        }
        for (int r = 0; r < N; ++r) {
            for (int t = 0; t < N; ++t) A[(size_t)r * N + t] = H[(size_t)r * N + t];
            A[(size_t)r * N + r] += lambda * H[(size_t)r * N + r];
            rhs[r] = -g[r];
        }
        const int ok = chol_solve_n(N, A, rhs, delta) == 0;
        double Fn = INFINITY, pred = INFINITY;
        if (ok) {
            for (int r = 0; r < N; ++r) trial[r] = theta[r] + delta[r];
            Fn = orc_gblock_objective(o, nc, np, nobs, oc, op, z, vy, vx, trial, rho_x, rho_y);
            double gd = 0.0, dd = 0.0;
            for (int r = 0; r < N; ++r) {
                gd += g[r] * delta[r];
                dd += H[(size_t)r * N + r] * delta[r] * delta[r];
            }
            pred = 0.5 * (lambda * dd - gd);
        }
        if (ok && isfinite(Fn) && (Fn < F || pred <= ORC_TIE * fres)) {
            memcpy(theta, trial, sizeof(double) * N);
            F = Fn;
            lambda = fmax(lambda / 10.0, ORC_LAMBDA_MIN);
            ++accepted;
        } else {
            lambda = fmin(lambda * 10.0, ORC_LAMBDA_MAX);
        }
    }
    free(g); free(H); free(A); free(rhs); free(delta); free(trial);
    return accepted;
}

/* ADMM iterations with block local updates.  Blocks: nblk, blk_off[nblk+1]
 * offsets into blk_obs (observation indices of each block in order),
 * blk_cam[nblk] the block's camera.  State: ycopy/ydual [nblk][9] (the
 * block's camera copy and scaled dual), xcopy/xdual [L][3] (per observation
 * point copy and dual).  One iteration:
 *   1. local update of every block (Eqs. 14-15), started at its copies;
 *   2. consensus: camera = mean over its blocks of ycopy + ydual (ascending
 *      block), point = mean over its observations of xcopy + xdual
 *      (ascending observation);
 *   3. scaled dual updates u += copy - consensus;
 *   4. r_pri over all copies, r_dual = |rho (consensus change)| counted once
 *      per copy (a camera has as many copies as blocks);
 *   5. optional residual balancing, duals rescaled by old / new rho.
 * trace (optional, 4 per iteration).  Returns 0, or -1 on bad input. */
int orc_admm_iterate_blocked(int64_t L, int32_t m, int32_t n, const int32_t *obs_cam, const int32_t *obs_pt,
                             const double *obs_uv, int32_t nblk, const int64_t *blk_off, const int64_t *blk_obs,
                             const int32_t *blk_cam, double *cons_y, double *cons_x, double *ycopy, double *ydual,
                             double *xcopy, double *xdual, double *rho, const orc_opts *o, int32_t n_iters,
                             double *trace)
{
    double *cnt_y = calloc((size_t)m, sizeof(double)), *cnt_x = calloc((size_t)n, sizeof(double));
    double *sum_y = malloc(sizeof(double) * 9 * (size_t)m), *sum_x = malloc(sizeof(double) * 3 * (size_t)n);
    double *old_y = malloc(sizeof(double) * 9 * (size_t)m), *old_x = malloc(sizeof(double) * 3 * (size_t)n);
    int64_t maxb = 0;
    for (int32_t b = 0; b < nblk; ++b)
        if (blk_off[b + 1] - blk_off[b] > maxb) maxb = blk_off[b + 1] - blk_off[b];
    double *z = malloc(sizeof(double) * 2 * (size_t)(maxb + 1)), *vx = malloc(sizeof(double) * 3 * (size_t)(maxb + 1));
    double *theta = malloc(sizeof(double) * (9 + 3 * (size_t)(maxb + 1)));
    if (!cnt_y || !cnt_x || !sum_y || !sum_x || !old_y || !old_x || !z || !vx || !theta) return -1;
    for (int32_t b = 0; b < nblk; ++b) {
        if (blk_cam[b] < 0 || blk_cam[b] >= m) return -1;
        cnt_y[blk_cam[b]] += 1.0;
        for (int64_t q = blk_off[b]; q < blk_off[b + 1]; ++q)
            if (obs_cam[blk_obs[q]] != blk_cam[b]) return -1;
    }
    for (int64_t k = 0; k < L; ++k) {
        if (obs_pt[k] < 0 || obs_pt[k] >= n) return -1;
        cnt_x[obs_pt[k]] += 1.0;
    }
    for (int32_t it = 0; it < n_iters; ++it) {
        const double rx = rho[0], ry = rho[1];
        /* 1. block local updates */
        for (int32_t b = 0; b < nblk; ++b) {
            const int j = blk_cam[b];
            const int nb = (int)(blk_off[b + 1] - blk_off[b]);
            double vy[9];
            for (int c = 0; c < 9; ++c) {
                vy[c] = cons_y[9 * j + c] - ydual[9 * (size_t)b + c];
                theta[c] = ycopy[9 * (size_t)b + c];
            }
            for (int q = 0; q < nb; ++q) {
                const int64_t k = blk_obs[blk_off[b] + q];
                const int i = obs_pt[k];
                z[2 * q] = obs_uv[2 * k];
                z[2 * q + 1] = obs_uv[2 * k + 1];
                for (int c = 0; c < 3; ++c) {
                    vx[3 * q + c] = cons_x[3 * i + c] - xdual[3 * k + c];
                    theta[9 + 3 * q + c] = xcopy[3 * k + c];
                }
            }
            orc_block_local_solve(o, nb, z, vy, vx, theta, rx, ry, o->lm_steps, NULL);
            for (int c = 0; c < 9; ++c) ycopy[9 * (size_t)b + c] = theta[c];
            for (int q = 0; q < nb; ++q) {
                const int64_t k = blk_obs[blk_off[b] + q];
                for (int c = 0; c < 3; ++c) xcopy[3 * k + c] = theta[9 + 3 * q + c];
            }
        }
        /* 2. consensus */
        memcpy(old_y, cons_y, sizeof(double) * 9 * (size_t)m);
        memcpy(old_x, cons_x, sizeof(double) * 3 * (size_t)n);
        memset(sum_y, 0, sizeof(double) * 9 * (size_t)m);
        memset(sum_x, 0, sizeof(double) * 3 * (size_t)n);
        for (int32_t b = 0; b < nblk; ++b)
            for (int c = 0; c < 9; ++c) sum_y[9 * blk_cam[b] + c] += ycopy[9 * (size_t)b + c] + ydual[9 * (size_t)b + c];
        for (int64_t k = 0; k < L; ++k)
            for (int c = 0; c < 3; ++c) sum_x[3 * obs_pt[k] + c] += xcopy[3 * k + c] + xdual[3 * k + c];
        for (int j = 0; j < m; ++j)
            for (int c = 0; c < 9; ++c) cons_y[9 * j + c] = sum_y[9 * j + c] / cnt_y[j];
        for (int i = 0; i < n; ++i)
            for (int c = 0; c < 3; ++c) cons_x[3 * i + c] = sum_x[3 * i + c] / cnt_x[i];
        /* 3. duals, 4. residuals */
        double pri2 = 0.0;
        for (int32_t b = 0; b < nblk; ++b)
            for (int c = 0; c < 9; ++c) {
                double d = ycopy[9 * (size_t)b + c] - cons_y[9 * blk_cam[b] + c];
                ydual[9 * (size_t)b + c] += d;
                pri2 += d * d;
            }
        for (int64_t k = 0; k < L; ++k)
            for (int c = 0; c < 3; ++c) {
                double d = xcopy[3 * k + c] - cons_x[3 * obs_pt[k] + c];
                xdual[3 * k + c] += d;
                pri2 += d * d;
            }
        double dy2 = 0.0, dx2 = 0.0;
        for (int j = 0; j < m; ++j) {
            double s = 0.0;
            for (int c = 0; c < 9; ++c) { double d = cons_y[9 * j + c] - old_y[9 * j + c]; s += d * d; }
            dy2 += cnt_y[j] * s;
        }
        for (int i = 0; i < n; ++i) {
            double s = 0.0;
            for (int c = 0; c < 3; ++c) { double d = cons_x[3 * i + c] - old_x[3 * i + c]; s += d * d; }
            dx2 += cnt_x[i] * s;
        }
        double r_pri = sqrt(pri2), r_dual = sqrt(rx * rx * dx2 + ry * ry * dy2);
        if (trace) {
            trace[4 * it + 0] = r_pri; trace[4 * it + 1] = r_dual;
            trace[4 * it + 2] = rx; trace[4 * it + 3] = ry;
        }
        /* 5. residual balancing */
        if (o->rho_balancing) {
            double fac = 1.0;
            if (r_pri > o->rb_mu * r_dual) fac = o->rb_tau;
            else if (r_dual > o->rb_mu * r_pri) fac = 1.0 / o->rb_tau;
            if (fac != 1.0) {
                double nx = fmin(fmax(rx * fac, o->rho_min), o->rho_max);
                double ny = fmin(fmax(ry * fac, o->rho_min), o->rho_max);
                double sx = rx / nx, sy = ry / ny;
                for (int64_t q = 0; q < 9 * (int64_t)nblk; ++q) ydual[q] *= sy;
                for (int64_t q = 0; q < 3 * L; ++q) xdual[q] *= sx;
                rho[0] = nx; rho[1] = ny;
            }
        }
    }
    free(cnt_y); free(cnt_x); free(sum_y); free(sum_x); free(old_y); free(old_x); free(z); free(vx); free(theta);
    return 0;
}
