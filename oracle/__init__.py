"""FP64 CPU oracle for ADMM distributed bundle adjustment.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke``
and by the CPU-baseline leg of ``bench.py``.  The GPU library never imports,
links or calls anything here, and nothing here uses the GPU library.

What it computes (Ramamurthy et al., "Distributed Bundle Adjustment"):
  * camera model: perspective division (Sec. 2.1, Eq. 1) extended to a
    9-parameter camera (angle-axis w, translation t, focal f, radial k1, k2):
    P = R(w) X + t, p = (P1/P3, P2/P3), pi = f (1 + k1 r^2 + k2 r^4) p;
  * the split objective and its augmented Lagrangian (Sec. 3.1, Eqs. 5-8),
    in scaled-dual form u = r / rho;
  * one ADMM iteration (Eqs. 9-13): per-observation local update, point and
    camera consensus, dual update; plus the primal/dual residual norms and
    residual-balancing of rho used to monitor and steer it;
  * reprojection statistics (RMSE, robust cost) at the consensus estimate;
  * ``oracle.mlp``: the warm-start network's forward/backward in FP64.

Readings where the paper is silent or loose (the same on the GPU path):
  R1 camera: 9 parameters as above, all optimised; no principal point; the
     rotation is updated additively in angle-axis form; for |w| < 1e-2 the
     Rodrigues coefficients use their Taylor series to 4th order.
  R2 Huber on the 2-D residual norm: phi(s) = s for s <= delta^2, else
     2 delta sqrt(s) - delta^2 (s = |e|^2); Student-t: nu log(1 + s/nu).
  R3 data term without 1/2, penalty (rho/2)|.|^2, as written in Eq. (8).
  R4 local solver (the paper names Gauss-Newton / L-BFGS): robust LM with
     IRLS weight phi'(s), Gauss-Newton matrix 2 w J^T J + P, Marquardt damping
     lambda*diag, lambda0 = 1e-3, x10 / /10 within [1e-12, 1e12], exactly S
     steps counting rejected ones; a trial is accepted if F' < F, or if the
     damped Gauss-Newton model predicts a decrease below
     1e-13 (F + |e| (|z_1| + |z_2| + f)) -- F's rounding resolution, since
     e = z - pi loses ~eps |z| -- so the model decides instead of rounding;
     a trial with
     depth P3 <= 1e-6 or a non-positive Cholesky pivot is rejected; the solve
     starts from the previous local copy.
  R5 iteration order: local -> consensus -> dual -> norms -> rho update.
  R6 residuals: r_pri = sqrt(sum_k |copy_k - consensus|^2),
     r_dual = sqrt(rho_x^2 sum_i N_i |dx_i|^2 + rho_y^2 sum_j M_j |dy_j|^2).
  R7 residual balancing: mu = 10, tau = 2, rho clamped to [1e-6, 1e6],
     scaled duals multiplied by rho_old / rho_new.
  R8 RMSE = sqrt(sum |e|^2 / L) at the consensus estimate.
  R9 generalised local updates (Sec. 3.1.4, Eqs. 14-15): a block is up to 64
     observations of one camera in ascending point order; it holds one copy
     of the camera and one point copy per observation, and its local problem
     (all 9 + 3 nb unknowns) is solved by the LM of R4 with the block's
     objective summed over its observations; a camera's consensus averages
     its block copies, and its residual weight is its number of blocks.
  R10 the paper's own camera (Sec. 2.1, Eq. 1), ``camera="euler"``: y =
     (alpha, beta, gamma, t), R = R3(gamma) R2(beta) R1(alpha) with R1, R2,
     R3 the right-handed rotations about x, y, z; pixels f (z~1/z~3,
     z~2/z~3) with the known focal length f (Eq. 1 leaves K out; the text
     defines it and calls the focal length known); no distortion.  The
     camera row keeps 9 slots (alpha, beta, gamma, t, f, 0, 0): slots 6-8
     have zero Jacobian columns, so every local solve leaves them at their
     value and exactly the 6 + 3 unknowns of the paper move.
  R11 ``solver="gauss_newton"`` (the paper's local solver for the l2 misfit,
     Sec. 3.1): the steps of R4 without damping, A = 2 w J^T J + P, and every
     step whose trial is finite is taken (no decrease test).
  R12 ``solver="lbfgs"`` (the paper's local solver for the Huber misfit,
     Sec. 3.1; the method as in Nocedal & Wright, Alg. 7.4 and 7.5, which
     the paper cites): S iterations (``lm_steps``) of d = -H g with the
     initial matrix H0_k = diag(P + 2 w J^T J)^-1 at the current iterate (the
     inverse diagonal of the Gauss-Newton matrix, recomputed every iteration;
     P^-1 alone stalls the line search when rho is far below the misfit's
     curvature) and at most 4 curvature pairs, oldest dropped first; an
     accepted step's pair is s = alpha d, y = g_new - g_old formed as P s +
     (misfit gradient difference), kept only if s.y > 1e-8 s^T P s (H stays
     positive definite); the solve ends when -g.d is at most R4's tie
     threshold (converged as far as F can tell); backtracking line search
     alpha = 1, 1/2, ..., 2^-9 with the Armijo test F' <= F + 1e-4 alpha g.d,
     or with both terms of the Gauss-Newton model along the step (-alpha g.d
     and alpha^2/2 d^T (P + 2w J^T J) d) at most the tie threshold (F cannot
     judge it); a trial with depth <= 1e-6 fails the test; an iteration with
     no trial taken ends the solve.  The paper gives none of these
     constants.
  R13 blocks of several cameras (``GeneralBlockADMM``, Sec. 3.1.4): cameras
     in consecutive groups of kappa (frame order on a trajectory); a group's
     observed points in ascending order, in runs of at most pi points; a
     block holds one run, the group's observations of it and the group's
     cameras that make them, with ONE copy of each of its cameras and points;
     its local problem is solved by R4's LM over all 9 kappa' + 3 pi'
     unknowns; a camera's (point's) consensus averages its block copies plus
     their scaled duals.  kappa = 1 gives R9's blocks with one point copy per
     observation.
  R14 learned start (an extension, not in the paper; ``ADMM.iterate_learned``):
     each local update starts from the better, by the local objective F, of
     its previous copy and the copy plus the update a network predicts (ties
     keep the copy), and runs ``learned_steps`` LM steps of R4 from there.
     The network (``oracle.mlp``) sees the observation's residual at the
     copy, camera and point copy minus consensus and the scaled duals, each
     standardised, rounded to bfloat16.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dba_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

LOSS = {"l2": 0, "huber": 1, "student_t": 2}
CAMERA = {"angle_axis": 0, "euler": 1}
SOLVER = {"lm": 0, "gauss_newton": 1, "lbfgs": 2}


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (plain -O2, no fast-math, no FMA
    contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off",
                               "-std=c11", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        _declare(_lib)
    return _lib


_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)
_up = ctypes.POINTER(ctypes.c_uint8)


class OrcOpts(ctypes.Structure):
    _fields_ = [("loss", ctypes.c_int32), ("loss_param", ctypes.c_double),
                ("lm_steps", ctypes.c_int32), ("lambda0", ctypes.c_double),
                ("rho_balancing", ctypes.c_int32), ("rb_mu", ctypes.c_double),
                ("rb_tau", ctypes.c_double), ("rho_min", ctypes.c_double),
                ("rho_max", ctypes.c_double), ("camera", ctypes.c_int32), ("solver", ctypes.c_int32)]


def _declare(L):
    L.orc_rot_coeffs.argtypes = [ctypes.c_double, _dp]
    L.orc_transform.argtypes = [_dp, _dp, _dp]
    L.orc_project.argtypes = [_dp, _dp, _dp]
    L.orc_project.restype = ctypes.c_double
    L.orc_project_jac.argtypes = [_dp, _dp, _dp, _dp]
    L.orc_project_jac.restype = ctypes.c_double
    L.orc_loss.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, _dp]
    L.orc_cholesky_solve.argtypes = [ctypes.c_int, _dp, _dp, _dp]
    L.orc_cholesky_solve.restype = ctypes.c_int
    L.orc_local_objective.argtypes = [ctypes.POINTER(OrcOpts), _dp, _dp, _dp,
                                      ctypes.c_double, ctypes.c_double]
    L.orc_local_objective.restype = ctypes.c_double
    L.orc_local_solve.argtypes = [ctypes.POINTER(OrcOpts), _dp, _dp, _dp,
                                  ctypes.c_double, ctypes.c_double, ctypes.c_int, _dp]
    L.orc_local_solve.restype = ctypes.c_int
    L.orc_lbfgs_apply.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp, _dp, _dp, _dp]
    L.orc_lbfgs_apply.restype = None
    L.orc_local_solve_lbfgs.argtypes = [ctypes.POINTER(OrcOpts), _dp, _dp, _dp, ctypes.c_double,
                                        ctypes.c_double, ctypes.c_int, _dp, _dp]
    L.orc_local_solve_lbfgs.restype = ctypes.c_int
    L.orc_gblock_objective.argtypes = [ctypes.POINTER(OrcOpts), ctypes.c_int, ctypes.c_int, ctypes.c_int, _ip, _ip,
                                       _dp, _dp, _dp, _dp, ctypes.c_double, ctypes.c_double]
    L.orc_gblock_objective.restype = ctypes.c_double
    L.orc_gblock_local_solve.argtypes = [ctypes.POINTER(OrcOpts), ctypes.c_int, ctypes.c_int, ctypes.c_int, _ip,
                                         _ip, _dp, _dp, _dp, _dp, ctypes.c_double, ctypes.c_double, ctypes.c_int]
    L.orc_gblock_local_solve.restype = ctypes.c_int
    L.orc_admm_iterate.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                   _ip, _ip, _dp, _dp, _dp, _dp, _dp, _dp,
                                   ctypes.POINTER(OrcOpts), ctypes.c_int32, _dp]
    L.orc_admm_iterate.restype = ctypes.c_int
    L.orc_admm_iterate_learned.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                           _ip, _ip, _dp, _dp, _dp, _dp, _dp, _dp,
                                           ctypes.POINTER(OrcOpts), _dp, ctypes.c_int32, _dp]
    L.orc_admm_iterate_learned.restype = ctypes.c_int
    L.orc_learned_local_solve.argtypes = [ctypes.POINTER(OrcOpts), _dp, _dp, _dp, _dp, ctypes.c_double,
                                          ctypes.c_double, ctypes.c_int]
    L.orc_learned_local_solve.restype = ctypes.c_int
    L.orc_learned_features.argtypes = [ctypes.c_int64, _ip, _ip, _dp, _dp, _dp, _dp, _dp, ctypes.c_int, _dp]
    L.orc_learned_features.restype = None
    L.orc_reprojection_stats.argtypes = [ctypes.c_int64, _ip, _ip, _dp, _dp, _dp, _up,
                                         ctypes.c_int, ctypes.c_double, ctypes.c_int, _dp]
    L.orc_euler_rotation.argtypes = [_dp, _dp]
    L.orc_project_cam.argtypes = [ctypes.c_int, _dp, _dp, _dp]
    L.orc_project_cam.restype = ctypes.c_double
    L.orc_project_jac_cam.argtypes = [ctypes.c_int, _dp, _dp, _dp, _dp]
    L.orc_project_jac_cam.restype = ctypes.c_double
    L.orc_block_objective.argtypes = [ctypes.POINTER(OrcOpts), ctypes.c_int, _dp, _dp, _dp, _dp,
                                      ctypes.c_double, ctypes.c_double]
    L.orc_block_objective.restype = ctypes.c_double
    L.orc_block_local_solve.argtypes = [ctypes.POINTER(OrcOpts), ctypes.c_int, _dp, _dp, _dp, _dp,
                                        ctypes.c_double, ctypes.c_double, ctypes.c_int, _dp]
    L.orc_block_local_solve.restype = ctypes.c_int
    _lp = ctypes.POINTER(ctypes.c_int64)
    L.orc_admm_iterate_blocked.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, _ip, _ip, _dp,
                                           ctypes.c_int32, _lp, _lp, _ip, _dp, _dp, _dp, _dp, _dp, _dp, _dp,
                                           ctypes.POINTER(OrcOpts), ctypes.c_int32, _dp]
    L.orc_admm_iterate_blocked.restype = ctypes.c_int


def _d(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def _i(a):
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(_ip)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def make_opts(loss="huber", loss_param=2.0, lm_steps=5, lambda0=1e-3,
              rho_balancing=False, rb_mu=10.0, rb_tau=2.0, rho_min=1e-6, rho_max=1e6, camera="angle_axis",
              solver="lm"):
    return OrcOpts(LOSS[loss] if isinstance(loss, str) else int(loss), float(loss_param),
                   int(lm_steps), float(lambda0), int(bool(rho_balancing)), float(rb_mu),
                   float(rb_tau), float(rho_min), float(rho_max), CAMERA[camera], SOLVER[solver])


# ---------------------------------------------------------------- pieces

def rot_coeffs(theta2: float) -> np.ndarray:
    out = np.zeros(5)
    lib().orc_rot_coeffs(float(theta2), _d(out))
    return out


def transform(cam, X):
    cam, X = _f64(cam), _f64(X)
    P = np.zeros(3)
    lib().orc_transform(_d(cam), _d(X), _d(P))
    return P


def project(cam, X, camera="angle_axis"):
    cam, X = _f64(cam), _f64(X)
    uv = np.zeros(2)
    depth = lib().orc_project_cam(CAMERA[camera], _d(cam), _d(X), _d(uv))
    return uv, depth


def project_jac(cam, X, camera="angle_axis"):
    cam, X = _f64(cam), _f64(X)
    uv, J = np.zeros(2), np.zeros((2, 12))
    depth = lib().orc_project_jac_cam(CAMERA[camera], _d(cam), _d(X), _d(uv), _d(J))
    return uv, J, depth


def euler_rotation(cam):
    """R = R3(gamma) R2(beta) R1(alpha) of an Euler camera row."""
    R = np.zeros(9)
    lib().orc_euler_rotation(_d(_f64(cam)), _d(R))
    return R.reshape(3, 3)


def loss(kind, param, s):
    out = np.zeros(2)
    lib().orc_loss(LOSS[kind] if isinstance(kind, str) else int(kind), float(param),
                   float(s), _d(out))
    return out[0], out[1]


def cholesky_solve(A, b):
    A, b = _f64(A), _f64(b)
    n = b.shape[0]
    x = np.zeros(n)
    rc = lib().orc_cholesky_solve(n, _d(A), _d(b), _d(x))
    return x if rc == 0 else None


def local_objective(opts, z, v, theta, rho_x, rho_y):
    return lib().orc_local_objective(ctypes.byref(opts), _d(_f64(z)), _d(_f64(v)),
                                     _d(_f64(theta)), float(rho_x), float(rho_y))


def local_solve(opts, z, v, theta, rho_x, rho_y, steps=None):
    """Returns (theta_out, n_accepted, F trace of length steps+1)."""
    steps = opts.lm_steps if steps is None else int(steps)
    th = _f64(theta).copy()
    tr = np.zeros(steps + 1)
    acc = lib().orc_local_solve(ctypes.byref(opts), _d(_f64(z)), _d(_f64(v)), _d(th),
                                float(rho_x), float(rho_y), steps, _d(tr))
    return th, acc, tr


def lbfgs_apply(S, Y, h0, g):
    """H g for the L-BFGS matrix built from diag(h0) by the pairs (rows of S,
    Y, oldest first), by the two-loop recursion."""
    S = np.ascontiguousarray(S, np.float64).reshape(-1, len(h0))
    Y = np.ascontiguousarray(Y, np.float64).reshape(S.shape)
    d = np.zeros(len(h0))
    lib().orc_lbfgs_apply(len(h0), S.shape[0], _d(S), _d(Y), _d(_f64(h0)), _d(_f64(g)), _d(d))
    return d


def local_solve_lbfgs(opts, z, v, theta, rho_x, rho_y, steps=None):
    """L-BFGS local solve (R12).  Returns (theta_out, n_taken, F trace of
    length steps+1, step lengths alpha of length steps, 0 after the end)."""
    steps = opts.lm_steps if steps is None else int(steps)
    th = _f64(theta).copy()
    tr = np.zeros(steps + 1)
    al = np.zeros(steps)
    n = lib().orc_local_solve_lbfgs(ctypes.byref(opts), _d(_f64(z)), _d(_f64(v)), _d(th),
                                    float(rho_x), float(rho_y), steps, _d(tr), _d(al))
    return th, n, tr, al


# ---------------------------------------------------------------- whole ADMM

@dataclass
class Problem:
    n_cams: int
    n_points: int
    obs_cam: np.ndarray
    obs_point: np.ndarray
    obs_uv: np.ndarray

    @classmethod
    def from_scene(cls, s):
        return cls(s.n_cams, s.n_points, np.ascontiguousarray(s.obs_cam, np.int32),
                   np.ascontiguousarray(s.obs_point, np.int32), _f64(s.obs_uv).reshape(-1, 2))


class ADMM:
    """The plain ADMM iteration on the whole problem, state in numpy arrays:
    ``cons_y`` (m, 9), ``cons_x`` (n, 3), ``copy`` (L, 12) = (y_j^i, x_i^j),
    ``dual`` (L, 12) scaled duals, ``rho`` = [rho_x, rho_y]."""

    def __init__(self, problem: Problem, cams0, points0, *, loss="huber", loss_param=2.0,
                 rho=1.0, rho_x=None, rho_y=None, rho_balancing=False, lm_steps=5,
                 lambda0=1e-3, camera="angle_axis", solver="lm"):
        self.p = problem
        self.opts = make_opts(loss, loss_param, lm_steps, lambda0, rho_balancing, camera=camera, solver=solver)
        self.loss, self.loss_param, self.camera = loss, loss_param, camera
        self.cons_y = _f64(cams0).reshape(-1, 9).copy()
        self.cons_x = _f64(points0).reshape(-1, 3).copy()
        L = problem.obs_cam.shape[0]
        self.copy = np.zeros((L, 12))
        self.copy[:, :9] = self.cons_y[problem.obs_cam]
        self.copy[:, 9:] = self.cons_x[problem.obs_point]
        self.dual = np.zeros((L, 12))
        self.rho = np.array([rho if rho_x is None else rho_x,
                             rho if rho_y is None else rho_y], dtype=np.float64)
        self.iteration = 0

    def iterate(self, n_iters: int) -> np.ndarray:
        """Runs n iterations; returns the trace (n, 4): r_pri, r_dual, rho_x, rho_y."""
        tr = np.zeros((n_iters, 4))
        p = self.p
        rc = lib().orc_admm_iterate(p.obs_cam.shape[0], p.n_cams, p.n_points,
                                    _i(p.obs_cam), _i(p.obs_point), _d(p.obs_uv),
                                    _d(self.cons_y), _d(self.cons_x), _d(self.copy),
                                    _d(self.dual), _d(self.rho), ctypes.byref(self.opts),
                                    int(n_iters), _d(tr))
        if rc != 0:
            raise ValueError("oracle: bad problem indices")
        self.iteration += n_iters
        return tr

    def features(self) -> np.ndarray:
        """Features of the learned start (R14) of every observation, (L, 26)."""
        p = self.p
        f = np.zeros((p.obs_cam.shape[0], 26))
        lib().orc_learned_features(p.obs_cam.shape[0], _i(p.obs_cam), _i(p.obs_point), _d(p.obs_uv),
                                   _d(self.cons_y), _d(self.cons_x), _d(self.copy), _d(self.dual),
                                   CAMERA[self.camera], _d(f))
        return f

    def iterate_learned(self, params, norm, learned_steps: int) -> np.ndarray:
        """One iteration with the learned start (R14): the network of
        ``oracle.mlp`` (weights and activations rounded to bfloat16) on the
        standardised features predicts each local update, the guard keeps
        the better start, ``learned_steps`` LM steps follow; consensus,
        duals, norms and rho as in ``iterate``.  ``params``: the flat FP32
        parameter block of the C ABI; ``norm``: feature mean / std, output
        mean / std (76 values).  Returns the trace row (1, 4)."""
        from . import mlp
        nm = np.asarray(norm, np.float32).astype(np.float64)
        net = mlp.unflatten(np.asarray(params, np.float32).astype(np.float64))
        x = mlp.standardize_input(self.features(), nm[:26], nm[26:52])
        y, _ = mlp.forward(net, x, quantize=True)
        delta = np.ascontiguousarray(y[:, :12] * nm[64:76] + nm[52:64])
        tr = np.zeros((1, 4))
        p = self.p
        rc = lib().orc_admm_iterate_learned(p.obs_cam.shape[0], p.n_cams, p.n_points,
                                            _i(p.obs_cam), _i(p.obs_point), _d(p.obs_uv),
                                            _d(self.cons_y), _d(self.cons_x), _d(self.copy),
                                            _d(self.dual), _d(self.rho), ctypes.byref(self.opts),
                                            _d(delta), int(learned_steps), _d(tr))
        if rc != 0:
            raise ValueError("oracle: bad problem indices or learned steps")
        self.iteration += 1
        return tr

    def stats(self, mask=None):
        """(rmse_all, rmse_masked, robust_cost, mean_abs_error) at consensus."""
        return reprojection_stats(self.p, self.cons_y, self.cons_x, mask,
                                  self.loss, self.loss_param, self.camera)


# ---------------------------------------------------------------- blocks
# Generalised local updates (Sec. 3.1.4, Eqs. 14-15), read as: a block is up
# to `size` observations of one camera, taken in ascending point order (then
# observation order); the block holds one camera copy and one point copy per
# observation.

def _l(a):
    assert a.dtype == np.int64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def make_blocks(obs_cam, obs_point, n_cams, size=64):
    """Returns blk_off (nblk + 1), blk_obs (L), blk_cam (nblk): each camera's
    observations sorted by (point, observation index), cut into runs of at
    most `size`, cameras in ascending order."""
    obs_cam = np.asarray(obs_cam)
    order = np.lexsort((np.arange(obs_cam.shape[0]), np.asarray(obs_point), obs_cam))
    offs, cams = [0], []
    cam_sorted = obs_cam[order]
    for j in range(n_cams):
        lo, hi = np.searchsorted(cam_sorted, j, "left"), np.searchsorted(cam_sorted, j, "right")
        for a in range(lo, hi, size):
            offs.append(min(a + size, hi))
            cams.append(j)
    return (np.asarray(offs, dtype=np.int64), np.ascontiguousarray(order, dtype=np.int64),
            np.asarray(cams, dtype=np.int32))


def block_objective(opts, z, vy, vx, theta, rho_x, rho_y):
    z, vy, vx, theta = _f64(z), _f64(vy), _f64(vx), _f64(theta)
    return lib().orc_block_objective(ctypes.byref(opts), int(z.shape[0]), _d(z), _d(vy), _d(vx), _d(theta),
                                     float(rho_x), float(rho_y))


def block_local_solve(opts, z, vy, vx, theta, rho_x, rho_y, steps):
    """z (nb, 2), vy (9), vx (nb, 3), theta (9 + 3 nb) start; returns
    (theta, accepted, F trace)."""
    z, vy, vx = _f64(z), _f64(vy), _f64(vx)
    th = _f64(theta).copy()
    tr = np.zeros(steps + 1)
    acc = lib().orc_block_local_solve(ctypes.byref(opts), int(z.shape[0]), _d(z), _d(vy), _d(vx), _d(th),
                                      float(rho_x), float(rho_y), int(steps), _d(tr))
    return th, acc, tr


class BlockADMM:
    """ADMM with block local updates: ``ycopy``/``ydual`` (nblk, 9) per block,
    ``xcopy``/``xdual`` (L, 3) per observation, ``cons_y`` (m, 9), ``cons_x``
    (n, 3), ``rho`` = [rho_x, rho_y]."""

    def __init__(self, problem: Problem, cams0, points0, *, block=64, loss="huber", loss_param=2.0, rho=1.0,
                 rho_x=None, rho_y=None, rho_balancing=False, lm_steps=5, lambda0=1e-3, camera="angle_axis"):
        self.p = problem
        self.opts = make_opts(loss, loss_param, lm_steps, lambda0, rho_balancing, camera=camera)
        self.loss, self.loss_param, self.camera = loss, loss_param, camera
        self.blk_off, self.blk_obs, self.blk_cam = make_blocks(problem.obs_cam, problem.obs_point,
                                                               problem.n_cams, block)
        self.cons_y = _f64(cams0).reshape(-1, 9).copy()
        self.cons_x = _f64(points0).reshape(-1, 3).copy()
        self.ycopy = np.ascontiguousarray(self.cons_y[self.blk_cam])
        self.ydual = np.zeros_like(self.ycopy)
        self.xcopy = np.ascontiguousarray(self.cons_x[problem.obs_point])
        self.xdual = np.zeros_like(self.xcopy)
        self.rho = np.array([rho if rho_x is None else rho_x, rho if rho_y is None else rho_y], dtype=np.float64)
        self.iteration = 0

    @property
    def n_blocks(self):
        return int(self.blk_cam.shape[0])

    def iterate(self, n_iters: int) -> np.ndarray:
        tr = np.zeros((n_iters, 4))
        p = self.p
        rc = lib().orc_admm_iterate_blocked(p.obs_cam.shape[0], p.n_cams, p.n_points, _i(p.obs_cam),
                                            _i(p.obs_point), _d(p.obs_uv), self.n_blocks, _l(self.blk_off),
                                            _l(self.blk_obs), _i(self.blk_cam), _d(self.cons_y), _d(self.cons_x),
                                            _d(self.ycopy), _d(self.ydual), _d(self.xcopy), _d(self.xdual),
                                            _d(self.rho), ctypes.byref(self.opts), int(n_iters), _d(tr))
        if rc != 0:
            raise ValueError("oracle: bad blocks")
        self.iteration += n_iters
        return tr

    def copies(self):
        """Per observation (L, 12): its block's camera copy and its point copy."""
        blk_of = np.empty(self.p.obs_cam.shape[0], dtype=np.int64)
        for b in range(self.n_blocks):
            blk_of[self.blk_obs[self.blk_off[b]:self.blk_off[b + 1]]] = b
        return np.hstack([self.ycopy[blk_of], self.xcopy]), np.hstack([self.ydual[blk_of], self.xdual])

    def stats(self, mask=None):
        return reprojection_stats(self.p, self.cons_y, self.cons_x, mask, self.loss, self.loss_param,
                                  self.camera)


def make_general_blocks(obs_cam, obs_point, n_cams, kappa, pi):
    """Blocks of the generalised local update with kappa cameras (reading
    R13): cameras in consecutive groups of kappa; a group's observed points,
    in ascending order, in runs of at most pi; a block holds one run, the
    group's observations of its points (in observation order) and the group's
    cameras that make them.  Returns a list of (cams, points, obs) arrays."""
    obs_cam = np.asarray(obs_cam)
    obs_point = np.asarray(obs_point)
    blocks = []
    for g0 in range(0, n_cams, kappa):
        sel = np.flatnonzero((obs_cam >= g0) & (obs_cam < g0 + kappa))
        pts = np.unique(obs_point[sel])
        for r0 in range(0, len(pts), pi):
            run = pts[r0:r0 + pi]
            obs = sel[np.isin(obs_point[sel], run)]
            blocks.append((np.unique(obs_cam[obs]), run, obs))
    return blocks


class GeneralBlockADMM:
    """ADMM with general block local updates (Sec. 3.1.4, Eqs. 14-15; reading
    R13): a block holds one copy of each of its cameras and of each of its
    points; its local problem (orc_gblock_local_solve) couples them through
    its observations.  Consensus: a camera's (point's) mean over its block
    copies of copy + scaled dual, in block order; duals u += copy -
    consensus.  Fixed rho."""

    def __init__(self, problem: Problem, cams0, points0, *, kappa=2, pi=16, loss="huber", loss_param=2.0, rho=1.0,
                 lm_steps=5, lambda0=1e-3, camera="angle_axis"):
        self.p = problem
        self.opts = make_opts(loss, loss_param, lm_steps, lambda0, False, camera=camera)
        self.loss, self.loss_param, self.camera = loss, loss_param, camera
        self.blocks = make_general_blocks(problem.obs_cam, problem.obs_point, problem.n_cams, kappa, pi)
        self.cons_y = _f64(cams0).reshape(-1, 9).copy()
        self.cons_x = _f64(points0).reshape(-1, 3).copy()
        self.ycam = np.concatenate([b[0] for b in self.blocks])      # camera of each camera copy
        self.xpt = np.concatenate([b[1] for b in self.blocks])       # point of each point copy
        self.ycopy = self.cons_y[self.ycam].copy()
        self.ydual = np.zeros_like(self.ycopy)
        self.xcopy = self.cons_x[self.xpt].copy()
        self.xdual = np.zeros_like(self.xcopy)
        self.rho = float(rho)
        self.ny = np.bincount(self.ycam, minlength=problem.n_cams).astype(np.float64)
        self.nx = np.bincount(self.xpt, minlength=problem.n_points).astype(np.float64)
        self.iteration = 0

    @property
    def n_copies(self):
        return len(self.ycam), len(self.xpt)

    def iterate(self, n_iters: int):
        p, rho = self.p, self.rho
        for _ in range(n_iters):
            y0 = x0 = 0
            for cams, pts, obs in self.blocks:
                nc, npt = len(cams), len(pts)
                ys, xs = slice(y0, y0 + nc), slice(x0, x0 + npt)
                oc = np.ascontiguousarray(np.searchsorted(cams, p.obs_cam[obs]), dtype=np.int32)
                op = np.ascontiguousarray(np.searchsorted(pts, p.obs_point[obs]), dtype=np.int32)
                z = np.ascontiguousarray(p.obs_uv[obs])
                vy = np.ascontiguousarray(self.cons_y[cams] - self.ydual[ys])
                vx = np.ascontiguousarray(self.cons_x[pts] - self.xdual[xs])
                th = np.concatenate([self.ycopy[ys].ravel(), self.xcopy[xs].ravel()])
                lib().orc_gblock_local_solve(ctypes.byref(self.opts), nc, npt, len(obs), _i(oc), _i(op), _d(z),
                                             _d(vy), _d(vx), _d(th), rho, rho, self.opts.lm_steps)
                self.ycopy[ys] = th[:9 * nc].reshape(nc, 9)
                self.xcopy[xs] = th[9 * nc:].reshape(npt, 3)
                y0, x0 = y0 + nc, x0 + npt
            sy = np.zeros_like(self.cons_y)
            sx = np.zeros_like(self.cons_x)
            np.add.at(sy, self.ycam, self.ycopy + self.ydual)
            np.add.at(sx, self.xpt, self.xcopy + self.xdual)
            self.cons_y = sy / self.ny[:, None]
            self.cons_x = sx / self.nx[:, None]
            self.ydual += self.ycopy - self.cons_y[self.ycam]
            self.xdual += self.xcopy - self.cons_x[self.xpt]
            self.iteration += 1

    def stats(self, mask=None):
        return reprojection_stats(self.p, self.cons_y, self.cons_x, mask, self.loss, self.loss_param,
                                  self.camera)


def reprojection_stats(problem: Problem, cams, points, mask=None, loss_kind="l2",
                       loss_param=1.0, camera="angle_axis"):
    out = np.zeros(4)
    cams, points = _f64(cams), _f64(points)
    mp = None
    if mask is not None:
        mk = np.ascontiguousarray(mask, dtype=np.uint8)
        mp = mk.ctypes.data_as(_up)
    lib().orc_reprojection_stats(problem.obs_cam.shape[0], _i(problem.obs_cam),
                                 _i(problem.obs_point), _d(problem.obs_uv), _d(cams),
                                 _d(points), mp, LOSS[loss_kind] if isinstance(loss_kind, str)
                                 else int(loss_kind), float(loss_param), CAMERA[camera], _d(out))
    return out
