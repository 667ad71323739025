"""Pins of the oracle's Gauss-Newton local solver (the paper's solver for the
l2 misfit, Sec. 3.1): one step is the least-squares step of the linearised
local problem, checked with numpy's lstsq on a central-difference Jacobian;
on a noise-free local problem the iterates converge quadratically; every
finite step is taken."""
import numpy as np
import pytest

import oracle


def _fd_jacobian(cam, X, camera):
    th = np.concatenate([cam, X])
    J = np.zeros((2, 12))
    for c in range(12):
        h = 1e-6 * max(1.0, abs(th[c]))
        a, b = th.copy(), th.copy()
        a[c] += h
        b[c] -= h
        J[:, c] = (oracle.project(a[:9], a[9:], camera)[0] - oracle.project(b[:9], b[9:], camera)[0]) / (2 * h)
    return J


def _case(seed, camera):
    rng = np.random.default_rng(seed)
    if camera == "euler":
        cam = np.array([0.2, -0.1, 0.3, 0.1, -0.2, 6.0, 800.0, 0.0, 0.0])
    else:
        cam = np.array([0.2, -0.1, 0.3, 0.1, -0.2, 6.0, 800.0, 1e-3, -2e-3])
    X = np.array([0.3, -0.2, 0.4])
    th = np.concatenate([cam, X])
    z = oracle.project(cam, X, camera)[0] + rng.normal(0, 2.0, 2)
    v = th + np.r_[rng.normal(0, 1e-2, 6), 0, 0, 0, rng.normal(0, 1e-2, 3)]
    return z, v, th


@pytest.mark.parametrize("camera", ["angle_axis", "euler"])
def test_one_step_is_the_least_squares_step(camera):
    z, v, th = _case(1, camera)
    rx = ry = 1e3
    opts = oracle.make_opts("l2", 1.0, camera=camera, solver="gauss_newton")
    t1, acc, _ = oracle.local_solve(opts, z, v, th, rx, ry, steps=1)
    assert acc == 1
    # minimise |sqrt2 (e - J d)|^2 + |sqrt(P) (th + d - v)|^2 over the unknowns
    J = _fd_jacobian(th[:9], th[9:], camera)
    e = z - oracle.project(th[:9], th[9:], camera)[0]
    # the unknowns of the camera model (the Euler camera's focal length is known)
    free = [c for c in range(12) if camera == "angle_axis" or not 6 <= c <= 8]
    P = np.array([ry] * 9 + [rx] * 3)
    A = np.vstack([np.sqrt(2.0) * J[:, free], np.diag(np.sqrt(P[free]))])
    b = np.concatenate([np.sqrt(2.0) * e, -np.sqrt(P[free]) * (th[free] - v[free])])
    d = np.linalg.lstsq(A, b, rcond=None)[0]
    np.testing.assert_allclose(t1[free] - th[free], d, rtol=1e-5, atol=1e-9 * np.abs(th[free]).max())


def test_quadratic_convergence_without_noise():
    cam = np.array([0.2, -0.1, 0.3, 0.1, -0.2, 6.0, 800.0, 1e-3, -2e-3])
    X = np.array([0.3, -0.2, 0.4])
    truth = np.concatenate([cam, X])
    z = oracle.project(cam, X)[0]
    v = truth.copy()
    start = truth + np.r_[1e-3 * np.ones(6), 0, 0, 0, 1e-3 * np.ones(3)]
    opts = oracle.make_opts("l2", 1.0, solver="gauss_newton")
    errs = []
    th = start.copy()
    for _ in range(4):
        th, _, _ = oracle.local_solve(opts, z, v, th, 10.0, 10.0, steps=1)
        errs.append(np.abs(th - truth).max())
    # error ratio e_{k+1} / e_k^2 bounded: quadratic convergence until rounding
    assert errs[1] < 1e-3 * errs[0] and errs[2] < max(1e-3 * errs[1], 1e-12)


def test_takes_every_finite_step():
    z, v, th = _case(2, "angle_axis")
    lm = oracle.make_opts("l2", 1.0, solver="lm")
    gn = oracle.make_opts("l2", 1.0, solver="gauss_newton")
    _, acc_gn, tr = oracle.local_solve(gn, z, v, th, 1e3, 1e3, steps=8)
    assert acc_gn == 8
    _, acc_lm, _ = oracle.local_solve(lm, z, v, th, 1e3, 1e3, steps=8)
    assert acc_lm <= 8
