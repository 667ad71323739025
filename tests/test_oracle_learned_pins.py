"""Pins of the oracle's learned start (reading R14: the network's predicted
update, the guard that keeps the better start by the local objective, then
LM steps) against what fixes it independently of the oracle: the features
recomputed with scipy rotations, the special cases that reduce to the plain
method (a network that predicts nothing, a prediction that raises F), and a
prediction equal to the local minimiser found by scipy's BFGS."""
import numpy as np
import pytest
from scipy.optimize import minimize
from scipy.spatial.transform import Rotation

import oracle
from oracle import mlp
from scenes import make_config2


def _scene():
    return make_config2(n_cams=20, n_points=200)


def _admm(sc, **kw):
    base = dict(loss="huber", loss_param=2.0, rho=1e5, rho_balancing=True)
    base.update(kw)
    a = oracle.ADMM(oracle.Problem.from_scene(sc), sc.cams_init, sc.points_init, **base)
    a.opts.rho_min, a.opts.rho_max = 1e5, 1e7
    return a


def _zero_net(mean=None):
    """A network whose output is zero, so the predicted update is the output
    mean of the normalisation block."""
    norm = np.concatenate([np.zeros(26), np.ones(26), np.zeros(12) if mean is None else mean, np.ones(12)])
    return np.zeros(22800, np.float32), norm.astype(np.float32)


def test_features_recomputed_with_scipy():
    sc = _scene()
    a = _admm(sc)
    a.iterate(3)
    f = a.features()
    oc, op = sc.obs_cam, sc.obs_point
    th = a.copy
    P = Rotation.from_rotvec(th[:, :3]).apply(th[:, 9:]) + th[:, 3:6]
    q = P[:, :2] / P[:, 2:3]
    r2 = (q * q).sum(1)
    uv = th[:, 6:7] * (1 + th[:, 7] * r2 + th[:, 8] * r2 * r2)[:, None] * q
    np.testing.assert_allclose(f[:, :2], sc.obs_uv - uv, rtol=0, atol=1e-9)
    np.testing.assert_array_equal(f[:, 2:11], th[:, :9] - a.cons_y[oc])
    np.testing.assert_array_equal(f[:, 11:14], th[:, 9:] - a.cons_x[op])
    np.testing.assert_array_equal(f[:, 14:], a.dual)
    # after iterations the duals and copy - consensus are not zero
    assert np.abs(f[:, 2:]).max() > 0


@pytest.mark.parametrize("steps", [1, 3])
def test_a_network_predicting_nothing_gives_the_plain_iteration(steps):
    """Zero prediction: F(base + 0) = F(base), a tie, so the guard keeps the
    base and the learned iteration is the plain one with the same LM steps,
    bit for bit (consensus, duals, norms and rho included)."""
    sc = _scene()
    plain = _admm(sc, lm_steps=steps)
    learned = _admm(sc, lm_steps=5)
    params, norm = _zero_net()
    for _ in range(4):
        tp = plain.iterate(1)
        tl = learned.iterate_learned(params, norm, steps)
        np.testing.assert_array_equal(tp, tl)
    for name in ("cons_y", "cons_x", "copy", "dual", "rho"):
        np.testing.assert_array_equal(getattr(plain, name), getattr(learned, name))


def test_a_prediction_that_raises_f_is_rejected():
    """A constant predicted update far from every local minimiser raises F
    for every observation: each local update then starts at its previous
    copy, as in the plain iteration."""
    sc = _scene()
    plain = _admm(sc, lm_steps=2)
    learned = _admm(sc)
    params, norm = _zero_net(mean=np.full(12, 0.5))
    plain.iterate(1)
    learned.iterate_learned(params, norm, 2)
    np.testing.assert_array_equal(plain.copy, learned.copy)
    np.testing.assert_array_equal(plain.cons_y, learned.cons_y)


def test_the_guard_keeps_a_prediction_at_the_local_minimiser():
    """With zero LM steps the local update is the start itself: the base when
    the prediction raises F, base + delta when delta is the exact local
    minimiser's offset (computed by scipy's BFGS, not by the oracle's
    solver), which lowers F."""
    sc = _scene()
    opts = oracle.make_opts("huber", 2.0)
    rho = 1e4
    rng = np.random.default_rng(2)
    for k in rng.choice(sc.n_obs, 6, replace=False):
        th0 = np.concatenate([sc.cams_init[sc.obs_cam[k]], sc.points_init[sc.obs_point[k]]])
        v = th0 + rng.normal(0, 1e-2, 12)
        z = sc.obs_uv[k]
        scale = np.maximum(1.0, np.abs(th0))
        fun = lambda y: oracle.local_objective(opts, z, v, y * scale, rho, rho)
        res = minimize(fun, th0 / scale, method="BFGS", options=dict(gtol=1e-10, maxiter=20000))
        best = res.x * scale
        assert res.fun < fun(th0 / scale)
        th = th0.copy()
        kept = oracle.lib().orc_learned_local_solve(oracle.ctypes.byref(opts), oracle._d(z), oracle._d(v),
                                                    oracle._d(th), oracle._d(best - th0), rho, rho, 0)
        assert kept == 1
        np.testing.assert_array_equal(th, th0 + (best - th0))
        th = th0.copy()
        bad = np.full(12, 0.5)
        kept = oracle.lib().orc_learned_local_solve(oracle.ctypes.byref(opts), oracle._d(z), oracle._d(v),
                                                    oracle._d(th), oracle._d(bad), rho, rho, 0)
        assert kept == 0
        np.testing.assert_array_equal(th, th0)


def test_learned_iteration_applies_the_network_prediction():
    """The predicted updates are the output of ``oracle.mlp`` (pinned against
    torch) on the standardised features, de-standardised: the learned
    iteration equals the iteration given those predictions directly, and
    differs from the plain iteration with the same LM steps (some
    predictions pass the guard)."""
    sc = _scene()
    a = _admm(sc)
    a.iterate(2)
    p = mlp.init_params(5)
    flat = mlp.flatten(p).astype(np.float32)
    rng = np.random.default_rng(6)
    norm = np.concatenate([rng.normal(0, 1, 26), rng.uniform(0.5, 2, 26), rng.normal(0, 1e-4, 12),
                           rng.uniform(1e-5, 1e-4, 12)]).astype(np.float32)
    nm = norm.astype(np.float64)
    y, _ = mlp.forward(mlp.unflatten(flat.astype(np.float64)),
                       mlp.standardize_input(a.features(), nm[:26], nm[26:52]), quantize=True)
    delta = y[:, :12] * nm[64:76] + nm[52:64]
    # the same iteration with the prediction supplied directly
    b = _admm(sc)
    b.iterate(2)
    a.iterate_learned(flat, norm, 2)
    tr = np.zeros((1, 4))
    pb = b.p
    rc = oracle.lib().orc_admm_iterate_learned(pb.obs_cam.shape[0], pb.n_cams, pb.n_points, oracle._i(pb.obs_cam),
                                               oracle._i(pb.obs_point), oracle._d(pb.obs_uv), oracle._d(b.cons_y),
                                               oracle._d(b.cons_x), oracle._d(b.copy), oracle._d(b.dual),
                                               oracle._d(b.rho), oracle.ctypes.byref(b.opts),
                                               oracle._d(np.ascontiguousarray(delta)), 2, oracle._d(tr))
    assert rc == 0
    np.testing.assert_array_equal(a.copy, b.copy)
    # and some predictions were kept: the result differs from the plain start
    c = _admm(sc)
    c.iterate(2)
    c.opts.lm_steps = 2
    c.iterate(1)
    assert not np.array_equal(a.copy, c.copy)
