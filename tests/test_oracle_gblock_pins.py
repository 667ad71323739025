"""Pins of the oracle's blocks of several cameras (Sec. 3.1.4, Eqs. 14-15;
reading R13): with one camera per block they are the one-camera blocks bit for
bit; the block objective written out; a two-camera block's LM reaches the
minimum found by scipy's BFGS over all its unknowns; the scaled duals of every
camera and point sum to zero; and ADMM with two-camera blocks reaches the
centralised MINPACK optimum."""
import numpy as np
import pytest
from scipy.optimize import minimize

import oracle
from scenes import make_sphere_scene, make_trajectory_scene


def test_one_camera_blocks_are_the_existing_blocks():
    sc = make_trajectory_scene(seed=4, n_cams=30, n_points=700)
    p = oracle.Problem.from_scene(sc)
    kw = dict(loss="huber", loss_param=2.0, rho=1e4)
    a = oracle.BlockADMM(p, sc.cams_init, sc.points_init, block=16, **kw)
    g = oracle.GeneralBlockADMM(p, sc.cams_init, sc.points_init, kappa=1, pi=16, **kw)
    a.iterate(4)
    g.iterate(4)
    assert np.array_equal(g.cons_y, a.cons_y) and np.array_equal(g.cons_x, a.cons_x)


def _two_camera_block(seed=3):
    sc = make_trajectory_scene(seed=seed, n_cams=12, n_points=200)
    blocks = oracle.make_general_blocks(sc.obs_cam, sc.obs_point, sc.n_cams, 2, 6)
    cams, pts, obs = next(b for b in blocks if len(b[0]) == 2 and len(np.unique(sc.obs_point[b[2]])) < len(b[2]))
    oc = np.searchsorted(cams, sc.obs_cam[obs]).astype(np.int32)
    op = np.searchsorted(pts, sc.obs_point[obs]).astype(np.int32)
    return sc, cams, pts, obs, oc, op


def test_block_objective_written_out():
    sc, cams, pts, obs, oc, op = _two_camera_block()
    rng = np.random.default_rng(1)
    vy = sc.cams_init[cams] + rng.normal(0, 1e-3, (len(cams), 9))
    vx = sc.points_init[pts] + rng.normal(0, 1e-2, (len(pts), 3))
    th = np.concatenate([sc.cams_init[cams].ravel(), sc.points_init[pts].ravel()])
    opts = oracle.make_opts("huber", 2.0)
    F = oracle.lib().orc_gblock_objective(opts, len(cams), len(pts), len(obs), oracle._i(oc), oracle._i(op),
                                          oracle._d(np.ascontiguousarray(sc.obs_uv[obs])), oracle._d(vy.ravel()),
                                          oracle._d(vx.ravel()), oracle._d(th), 1e3, 2e3)
    ref = 0.5 * 2e3 * np.sum((sc.cams_init[cams] - vy) ** 2) + 0.5 * 1e3 * np.sum((sc.points_init[pts] - vx) ** 2)
    for q, k in enumerate(obs):
        e = sc.obs_uv[k] - oracle.project(sc.cams_init[cams[oc[q]]], sc.points_init[pts[op[q]]])[0]
        ref += oracle.loss("huber", 2.0, e @ e)[0]
    assert F == pytest.approx(ref, rel=1e-13)


def test_two_camera_block_lm_reaches_the_bfgs_minimum():
    sc, cams, pts, obs, oc, op = _two_camera_block()
    nc, npt = len(cams), len(pts)
    rng = np.random.default_rng(2)
    vy = (sc.cams_init[cams] + rng.normal(0, 1e-3, (nc, 9)) * np.r_[np.ones(6), 10, 1e-3, 1e-3]).ravel()
    vx = (sc.points_init[pts] + rng.normal(0, 1e-2, (npt, 3))).ravel()
    th0 = np.concatenate([sc.cams_init[cams].ravel(), sc.points_init[pts].ravel()])
    opts = oracle.make_opts("huber", 2.0)
    z = np.ascontiguousarray(sc.obs_uv[obs])
    args = (len(cams), len(pts), len(obs), oracle._i(oc), oracle._i(op), oracle._d(z), oracle._d(vy), oracle._d(vx))

    def f(t):
        return oracle.lib().orc_gblock_objective(opts, *args, oracle._d(np.ascontiguousarray(t)), 1e3, 1e3)
    th = th0.copy()
    oracle.lib().orc_gblock_local_solve(opts, *args, oracle._d(th), 1e3, 1e3, 60)
    r = minimize(f, th0, method="BFGS", options=dict(gtol=1e-9, maxiter=50000))
    assert f(th) <= r.fun * (1 + 1e-9) + 1e-9
    assert f(th) < f(th0)


def test_duals_sum_to_zero_per_camera_and_point():
    sc = make_trajectory_scene(seed=5, n_cams=20, n_points=400)
    g = oracle.GeneralBlockADMM(oracle.Problem.from_scene(sc), sc.cams_init, sc.points_init, kappa=2, pi=8,
                                loss="huber", loss_param=2.0, rho=1e4)
    g.iterate(3)
    sy = np.zeros_like(g.cons_y)
    sx = np.zeros_like(g.cons_x)
    np.add.at(sy, g.ycam, g.ydual)
    np.add.at(sx, g.xpt, g.xdual)
    assert np.abs(sy).max() < 1e-10 * (1 + np.abs(g.cons_y).max()) and np.abs(sx).max() < 1e-10
    # fewer point copies than observations: points seen by both cameras of a block share one
    assert g.n_copies[1] < sc.n_obs


def test_two_camera_blocks_reach_the_centralised_optimum():
    from test_oracle_euler_pins import _minpack_lm_euler
    s = make_sphere_scene(seed=7, n_cams=8, n_points=100, radius=8.0, box=3.0, k_lo=8, k_hi=8, camera="euler")
    p = oracle.Problem.from_scene(s)
    cams, pts = _minpack_lm_euler(s)
    opt = oracle.reprojection_stats(p, cams, pts, None, "l2", 1.0, "euler")
    g = oracle.GeneralBlockADMM(p, s.cams_init, s.points_init, kappa=2, pi=25, loss="l2", loss_param=1.0,
                                rho=1e4, camera="euler")
    init = g.stats()
    g.iterate(300)
    assert init[0] > 10 * opt[0]
    assert abs(g.stats()[0] - opt[0]) < 5e-3 * opt[0], (g.stats()[0], opt[0])


def test_two_cameras_per_block_converge_in_fewer_iterations():
    # iterations to the inlier RMSE the per-observation ADMM reaches after 200
    # iterations (within 0.5 %): per observation > one camera per block > two
    # (about a minute: the effect needs a trajectory long enough for the
    # consensus to take many iterations)
    sc = make_trajectory_scene(seed=11, n_cams=60, n_points=3000)
    p = oracle.Problem.from_scene(sc)
    inl = ~sc.outlier
    kw = dict(loss="huber", loss_param=2.0, rho=1e5)
    base = oracle.ADMM(p, sc.cams_init, sc.points_init, **kw)
    base.iterate(200)
    goal = 1.005 * base.stats(inl)[1]

    def iterations(a, cap=200):
        for k in range(1, cap + 1):
            a.iterate(1)
            if a.stats(inl)[1] <= goal:
                return k
        return None
    n1 = iterations(oracle.GeneralBlockADMM(p, sc.cams_init, sc.points_init, kappa=1, pi=16, **kw))
    n2 = iterations(oracle.GeneralBlockADMM(p, sc.cams_init, sc.points_init, kappa=2, pi=16, **kw))
    print("iterations: one camera per block", n1, "two", n2)
    assert n1 is not None and n2 is not None and n2 < 0.8 * n1 < 0.8 * 200
