"""Pins of the oracle's generalised (block) local updates, Sec. 3.1.4,
Eqs. 14-15: a block is up to 64 observations of one camera that share one
camera copy.  Checked against things other than the oracle's own formulas:
the per-observation method it must reduce to with blocks of one observation,
finite differences of the block objective, scipy's BFGS, the ADMM invariants,
the noise-free fixed point and the centralised LM optimum."""
import numpy as np
import pytest
from scipy.optimize import minimize

import oracle
from scenes import make_config0, make_ring_scene
from test_oracle_pins import _minpack_lm


def _block_case(seed, nb, rho, noise=1.0):
    """A block of nb observations of one camera of a ring scene, with the
    consensus perturbed away from the copies."""
    rng = np.random.default_rng(seed)
    s = make_ring_scene(seed=seed, n_cams=3, n_points=max(nb, 1))
    sel = np.flatnonzero(s.obs_cam == 1)[:nb]
    z = s.obs_uv[sel]
    y0 = s.cams_init[1].copy()
    x0 = s.points_init[s.obs_point[sel]].copy()
    vy = y0 + rng.normal(0, 1e-3, 9) * noise
    vx = x0 + rng.normal(0, 1e-3, x0.shape) * noise
    theta = np.concatenate([y0, x0.ravel()])
    return z, vy, vx, theta


def _fd_grad(opts, z, vy, vx, th, rx, ry):
    g = np.zeros_like(th)
    for c in range(th.shape[0]):
        h = 1e-6 * max(1.0, abs(th[c]))
        a, b = th.copy(), th.copy()
        a[c] += h
        b[c] -= h
        g[c] = (oracle.block_objective(opts, z, vy, vx, a, rx, ry) -
                oracle.block_objective(opts, z, vy, vx, b, rx, ry)) / (2 * h)
    return g


def test_blocks_partition_each_camera_in_point_order():
    s = make_ring_scene(seed=2, n_cams=3, n_points=150)
    p = oracle.Problem.from_scene(s)
    off, obs, cam = oracle.make_blocks(p.obs_cam, p.obs_point, p.n_cams, 64)
    assert list(np.diff(off)) == [64, 64, 22] * 3 and list(cam) == [0, 0, 0, 1, 1, 1, 2, 2, 2]
    assert sorted(obs.tolist()) == list(range(p.obs_cam.shape[0]))
    for b in range(len(cam)):
        ks = obs[off[b]:off[b + 1]]
        assert (p.obs_cam[ks] == cam[b]).all() and (np.diff(p.obs_point[ks]) > 0).all()


def test_block_objective_definition():
    z, vy, vx, th = _block_case(3, 5, 1e3)
    o = oracle.make_opts("huber", 2.0)
    nb = z.shape[0]
    F = 0.5 * 1e3 * ((th[:9] - vy) ** 2).sum()
    for k in range(nb):
        uv, _ = oracle.project(th[:9], th[9 + 3 * k:12 + 3 * k])
        F += oracle.loss(1, 2.0, ((z[k] - uv) ** 2).sum())[0]
        F += 0.5 * 2e3 * ((th[9 + 3 * k:12 + 3 * k] - vx[k]) ** 2).sum()
    assert oracle.block_objective(o, z, vy, vx, th, 2e3, 1e3) == pytest.approx(F, rel=1e-13)


def test_single_observation_block_is_the_local_solve():
    z, vy, vx, th = _block_case(4, 1, 1e4)
    o = oracle.make_opts("huber", 2.0)
    tb, ab, fb = oracle.block_local_solve(o, z, vy, vx, th, 1e4, 1e4, 5)
    v = np.concatenate([vy, vx[0]])
    tl, al, fl = oracle.local_solve(o, z[0], v, th, 1e4, 1e4, 5)
    # same steps and decisions; F itself sums its terms in another order
    assert np.array_equal(tb, tl) and ab == al
    np.testing.assert_allclose(fb, fl, rtol=1e-14)


@pytest.mark.parametrize("loss,param", [("l2", 1.0), ("huber", 2.0), ("student_t", 4.0)])
def test_block_lm_is_monotone_and_stationary(loss, param):
    z, vy, vx, th = _block_case(5, 9, 1e3, noise=30.0)
    o = oracle.make_opts(loss, param)
    t, acc, tr = oracle.block_local_solve(o, z, vy, vx, th, 1e3, 1e3, 60)
    assert acc > 0
    assert np.all(np.diff(tr) <= 1e-9 * (1 + np.abs(tr[:-1])))
    g0 = np.linalg.norm(_fd_grad(o, z, vy, vx, th, 1e3, 1e3))
    g = np.linalg.norm(_fd_grad(o, z, vy, vx, t, 1e3, 1e3))
    assert g < 1e-5 * (1 + g0), (g, g0)


def test_block_lm_minimum_matches_bfgs():
    z, vy, vx, th = _block_case(6, 4, 1e3, noise=20.0)
    o = oracle.make_opts("huber", 2.0)
    t, _, tr = oracle.block_local_solve(o, z, vy, vx, th, 1e3, 1e3, 80)
    f = lambda x: oracle.block_objective(o, z, vy, vx, x, 1e3, 1e3)
    r = minimize(f, th, method="BFGS", options=dict(gtol=1e-10, maxiter=20000))
    assert tr[-1] <= r.fun * (1 + 1e-9) + 1e-9
    assert np.abs(t - r.x).max() < 1e-4


def test_blocks_of_one_observation_are_the_per_observation_method():
    s = make_ring_scene(seed=9, n_cams=4, n_points=40)
    p = oracle.Problem.from_scene(s)
    kw = dict(loss="huber", loss_param=2.0, rho=1e4)
    a = oracle.ADMM(p, s.cams_init, s.points_init, **kw)
    b = oracle.BlockADMM(p, s.cams_init, s.points_init, block=1, **kw)
    ta, tb = a.iterate(6), b.iterate(6)
    cb, db = b.copies()
    assert np.array_equal(a.cons_y, b.cons_y) and np.array_equal(a.cons_x, b.cons_x)
    assert np.array_equal(a.copy, cb) and np.array_equal(a.dual, db)
    np.testing.assert_allclose(ta, tb, rtol=1e-13)


def test_block_duals_sum_to_zero_and_consensus_is_the_mean():
    s = make_ring_scene(seed=10, n_cams=5, n_points=150)
    p = oracle.Problem.from_scene(s)
    b = oracle.BlockADMM(p, s.cams_init, s.points_init, block=64, loss="huber", loss_param=2.0, rho=1e3,
                         rho_balancing=True)
    for _ in range(4):
        b.iterate(1)
        for j in range(p.n_cams):
            sel = b.blk_cam == j
            assert np.abs(b.ydual[sel].sum(0)).max() < 1e-12 * max(1, np.abs(b.ydual[sel]).max()) * sel.sum()
            np.testing.assert_allclose(b.cons_y[j], b.ycopy[sel].mean(0), rtol=1e-12, atol=1e-12)
        for i in range(p.n_points):
            sel = p.obs_point == i
            np.testing.assert_allclose(b.cons_x[i], b.xcopy[sel].mean(0), rtol=1e-12, atol=1e-12)


def test_block_noise_free_ground_truth_is_a_fixed_point():
    s = make_config0(noise_px=0.0)
    p = oracle.Problem.from_scene(s)
    b = oracle.BlockADMM(p, s.cams_gt, s.points_gt, block=64, loss="huber", loss_param=2.0, rho=1e4)
    b.iterate(20)
    np.testing.assert_allclose(b.cons_y, s.cams_gt, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(b.cons_x, s.points_gt, rtol=1e-12, atol=1e-12)


def test_block_admm_reaches_the_centralised_lm_optimum():
    s = make_ring_scene(seed=7, n_cams=8, n_points=100, box=3.0, radius=8.0)
    p = oracle.Problem.from_scene(s)
    cams, pts = _minpack_lm(s, "huber", 2.0)
    lm = oracle.reprojection_stats(p, cams, pts, None, "huber", 2.0)
    b = oracle.BlockADMM(p, s.cams_init, s.points_init, block=64, loss="huber", loss_param=2.0, rho=1e4)
    b.iterate(400)
    st = b.stats()
    assert abs(st[0] - lm[0]) < 5e-3 * lm[0], (st[0], lm[0])
