"""Pins of the oracle's L-BFGS local solver (the paper's solver for the Huber
misfit, Sec. 3.1; Nocedal & Wright, Alg. 7.4 and 7.5).

The two-loop recursion is checked against the dense BFGS inverse update
H+ = (I - r s y^T) H (I - r y s^T) + r s s^T (r = 1 / s.y) and the secant
condition.  Seven iterations are checked against a line search written here:
the gradient and the Gauss-Newton diagonal (the initial matrix) by central
differences, the memory of 4 pairs and the curvature rule, the direction from
the dense update, and the largest power of 1/2 that passes the Armijo test.  Further checks: a stationary start stays put and
a converged solve stops,
steps are powers of 1/2 and F never rises,
the iterates reach the minimiser found by scipy's BFGS, the Euler camera's
fixed slots stay put, and ADMM with these local solves reaches the centralised
MINPACK optimum (l2) and the same fixed point as with the LM (Huber)."""
import numpy as np
import pytest
from scipy.optimize import minimize

import oracle
from scenes import make_sphere_scene

ARMIJO = 1e-4


def _dense_bfgs(S, Y, h0):
    H = np.diag(h0)
    I = np.eye(len(h0))
    for s, y in zip(S, Y):
        r = 1.0 / (s @ y)
        H = (I - r * np.outer(s, y)) @ H @ (I - r * np.outer(y, s)) + r * np.outer(s, s)
    return H


def _pairs(rng, n, k):
    # pairs of a random SPD matrix: y = A s, so s.y > 0
    B = rng.normal(size=(n, n))
    A = B @ B.T + n * np.eye(n)
    S = rng.normal(size=(k, n))
    return S, S @ A.T


@pytest.mark.parametrize("n,k", [(12, 0), (12, 1), (12, 4), (5, 7), (9, 3)])
def test_two_loop_equals_dense_bfgs(n, k):
    rng = np.random.default_rng(10 * n + k)
    S, Y = _pairs(rng, n, k)
    h0 = rng.uniform(1e-5, 1e-2, n)
    g = rng.normal(size=n)
    d = oracle.lbfgs_apply(S, Y, h0, g)
    np.testing.assert_allclose(d, _dense_bfgs(S, Y, h0) @ g, rtol=1e-10, atol=1e-14 * np.abs(d).max())
    if k:
        # secant condition of the newest pair
        np.testing.assert_allclose(oracle.lbfgs_apply(S, Y, h0, Y[-1]), S[-1], rtol=1e-9)


def _case(seed, camera="angle_axis", sigma=3.0):
    rng = np.random.default_rng(seed)
    k = (0.0, 0.0) if camera == "euler" else (1e-3, -2e-3)
    cam = np.array([0.2, -0.1, 0.3, 0.1, -0.2, 6.0, 800.0, *k])
    X = np.array([0.3, -0.2, 0.4])
    th = np.concatenate([cam, X])
    z = oracle.project(cam, X, camera)[0] + rng.normal(0, sigma, 2)
    v = th + np.r_[rng.normal(0, 1e-2, 6), 0, 0, 0, rng.normal(0, 1e-2, 3)]
    return z, v, th


def _fd_grad(opts, z, v, th, rx, ry, free):
    g = np.zeros(12)
    for c in free:
        h = 1e-6 * max(1.0, abs(th[c]))
        a, b = th.copy(), th.copy()
        a[c] += h
        b[c] -= h
        g[c] = (oracle.local_objective(opts, z, v, a, rx, ry) - oracle.local_objective(opts, z, v, b, rx, ry)) / (2 * h)
    return g


def _gn_inv_diag(opts, z, th, rx, ry, loss, lp, camera):
    """diag(P + 2 w J^T J)^-1 with J by central differences of the projection
    and w = phi'(s) by a central difference of the loss."""
    J = np.zeros((2, 12))
    for c in range(12):
        h = 1e-6 * max(1.0, abs(th[c]))
        a, b = th.copy(), th.copy()
        a[c] += h
        b[c] -= h
        J[:, c] = (oracle.project(a[:9], a[9:], camera)[0] - oracle.project(b[:9], b[9:], camera)[0]) / (2 * h)
    e = z - oracle.project(th[:9], th[9:], camera)[0]
    s2 = e @ e
    hs = 1e-6 * s2
    w = (oracle.loss(loss, lp, s2 + hs)[0] - oracle.loss(loss, lp, s2 - hs)[0]) / (2 * hs)
    return 1.0 / (np.array([ry] * 9 + [rx] * 3) + 2 * w * (J ** 2).sum(0))


def _armijo_step(opts, z, v, th, d, g, rx, ry):
    F = oracle.local_objective(opts, z, v, th, rx, ry)
    gd = g @ d
    for t in range(10):
        a = 0.5 ** t
        Fn = oracle.local_objective(opts, z, v, th + a * d, rx, ry)
        if Fn <= F + ARMIJO * a * gd:
            # the test's decision is not near its threshold
            assert abs(Fn - F - ARMIJO * a * gd) > 1e-6 * abs(F)
            return a
        assert abs(Fn - F - ARMIJO * a * gd) > 1e-6 * abs(F)
    raise AssertionError("no step")


@pytest.mark.parametrize("loss,lp,camera,rho,seed", [
    ("huber", 2.0, "angle_axis", 1e3, 3), ("huber", 2.0, "euler", 1e2, 3), ("l2", 1.0, "angle_axis", 1e2, 3),
    ("student_t", 4.0, "euler", 1e3, 3), ("student_t", 1.0, "angle_axis", 1e3, 8)])
def test_iterations_by_hand(loss, lp, camera, rho, seed):
    """Seven iterations, each from the oracle's previous iterate: the gradient
    and H0 by central differences, the pairs of the accepted steps kept under
    positive curvature, at most the 4 newest, the direction from the dense BFGS
    update, the step from the Armijo search written here."""
    z, v, th0 = _case(seed, camera)
    rx, ry = rho, 2.0 * rho
    opts = oracle.make_opts(loss, lp, camera=camera, solver="lbfgs")
    free = [c for c in range(12) if camera == "angle_axis" or not 6 <= c <= 8]
    P = np.array([ry] * 9 + [rx] * 3)
    pairs, dropped = [], 0
    th, g_old = th0, None
    for k in range(7):
        g = _fd_grad(opts, z, v, th, rx, ry, free)
        if k:
            s, y = th - th_prev, g - g_old
            thr = 1e-8 * (s * P) @ s
            assert abs(s @ y - thr) > 1e-3 * abs(s @ y)
            if s @ y > thr:
                pairs = (pairs + [(s, y)])[-4:]
            else:
                dropped += 1
        h0 = _gn_inv_diag(opts, z, th, rx, ry, loss, lp, camera)
        S = np.array([p[0][free] for p in pairs]).reshape(-1, len(free))
        Y = np.array([p[1][free] for p in pairs]).reshape(-1, len(free))
        d = np.zeros(12)
        d[free] = -_dense_bfgs(S, Y, h0[free]) @ g[free]
        a = _armijo_step(opts, z, v, th, d, g, rx, ry)
        nxt, n, _, al = oracle.local_solve_lbfgs(opts, z, v, th0, rx, ry, steps=k + 1)
        assert n == k + 1 and al[k] == a, (k, al, a)
        np.testing.assert_allclose(nxt, th + a * d, rtol=0, atol=1e-5 * np.abs(a * d).max())
        th_prev, g_old, th = th, g, nxt
    # the cases cover a full memory and a dropped pair
    assert len(pairs) == 4 or dropped


def test_stationary_start_stays_put():
    # the observation sits on the projection and the start is v: g = 0, so the
    # solve has converged before its first step
    cam = np.array([0.2, -0.1, 0.3, 0.1, -0.2, 6.0, 800.0, 1e-3, -2e-3])
    X = np.array([0.3, -0.2, 0.4])
    th = np.concatenate([cam, X])
    z = oracle.project(cam, X)[0]
    opts = oracle.make_opts("huber", 2.0, solver="lbfgs")
    t1, n, tr, al = oracle.local_solve_lbfgs(opts, z, th, th, 1e3, 1e3, steps=4)
    assert n == 0 and np.all(al == 0.0) and np.array_equal(t1, th) and np.all(tr == 0.0)


def test_stops_once_converged():
    # many iterations: the solve ends once the predicted decrease is below F's
    # resolution, and further iterations change nothing
    z, v, th = _case(5, "angle_axis")
    opts = oracle.make_opts("l2", 1.0, solver="lbfgs")
    t, n, tr, al = oracle.local_solve_lbfgs(opts, z, v, th, 1e5, 1e5, steps=64)
    assert 0 < n < 64 and np.all(al[n:] == 0.0) and np.all(al[:n] > 0)
    t2, n2, _, _ = oracle.local_solve_lbfgs(opts, z, v, th, 1e5, 1e5, steps=n + 10)
    assert n2 == n and np.array_equal(t2, t)


@pytest.mark.parametrize("seed", range(6))
def test_steps_are_halvings_and_f_never_rises(seed):
    camera = "euler" if seed % 2 else "angle_axis"
    z, v, th = _case(seed, camera, sigma=20.0)
    opts = oracle.make_opts(["huber", "l2", "student_t"][seed % 3], 2.0, camera=camera, solver="lbfgs")
    rho = [1e1, 1e2, 1e3][seed % 3]
    t, n, tr, al = oracle.local_solve_lbfgs(opts, z, v, th, rho, rho, steps=25)
    taken = al[al > 0]
    assert n == len(taken)
    k = -np.log2(taken)
    assert np.array_equal(k, np.round(k)) and np.all((0 <= k) & (k <= 9))
    assert np.all(np.diff(tr) <= 1e-12 * np.abs(tr[:-1]))
    assert tr[-1] < tr[0]
    if camera == "euler":
        assert np.array_equal(t[6:9], th[6:9])


@pytest.mark.parametrize("loss,camera", [("huber", "angle_axis"), ("l2", "angle_axis"), ("huber", "euler"),
                                         ("student_t", "angle_axis")])
def test_reaches_the_bfgs_minimiser(loss, camera):
    z, v, th0 = _case(5, camera)
    rho = 1e3
    opts = oracle.make_opts(loss, 4.0 if loss == "student_t" else 2.0, camera=camera, solver="lbfgs")
    th, n, tr, _ = oracle.local_solve_lbfgs(opts, z, v, th0, rho, rho, steps=80)
    free = [c for c in range(12) if camera == "angle_axis" or not 6 <= c <= 8]

    def f(x):
        t = th0.copy()
        t[free] = x
        return oracle.local_objective(opts, z, v, t, rho, rho)
    r = minimize(f, th0[free], method="BFGS", options=dict(gtol=1e-10, maxiter=20000))
    assert abs(tr[-1] - r.fun) <= 1e-8 * abs(r.fun)
    np.testing.assert_allclose(th[free], r.x, atol=2e-4 * np.abs(r.x).max())


def test_admm_with_lbfgs_reaches_the_centralised_l2_optimum():
    # the Euler-camera scene of the LM's pin: 8 cameras, each seeing all 100 points
    from test_oracle_euler_pins import _minpack_lm_euler
    s = make_sphere_scene(seed=7, n_cams=8, n_points=100, radius=8.0, box=3.0, k_lo=8, k_hi=8, camera="euler")
    p = oracle.Problem.from_scene(s)
    cams, pts = _minpack_lm_euler(s)
    opt = oracle.reprojection_stats(p, cams, pts, None, "l2", 1.0, "euler")
    a = oracle.ADMM(p, s.cams_init, s.points_init, loss="l2", loss_param=1.0, rho=1e4, camera="euler",
                    solver="lbfgs")
    init = a.stats()
    a.iterate(400)
    assert init[0] > 10 * opt[0]
    assert abs(a.stats()[0] - opt[0]) < 5e-3 * opt[0], (a.stats()[0], opt[0])


def test_admm_with_lbfgs_and_lm_share_the_huber_fixed_point():
    s = make_sphere_scene(seed=5, n_cams=6, n_points=40, radius=8.0, box=3.0, k_lo=6, k_hi=6, camera="euler")
    p = oracle.Problem.from_scene(s)
    kw = dict(loss="huber", loss_param=2.0, rho=1e4, camera="euler")
    lm = oracle.ADMM(p, s.cams_init, s.points_init, **kw)
    lb = oracle.ADMM(p, s.cams_init, s.points_init, solver="lbfgs", lm_steps=10, **kw)
    lm.iterate(500)
    lb.iterate(500)
    assert abs(lb.stats()[1] - lm.stats()[1]) < 1e-3 * lm.stats()[1]
    np.testing.assert_allclose(lb.cons_x, lm.cons_x, atol=1e-3 * np.abs(lm.cons_x).max())
