"""Pins of the oracle's Euler camera (Sec. 2.1, Eq. 1): y = (alpha, beta,
gamma, t), R = R3(gamma) R2(beta) R1(alpha), pixels f (z~1/z~3, z~2/z~3)
with a known focal length.  Checked against scipy's rotations, hand-computed
projections, central differences, BFGS on the 9-unknown local problem, the
noise-free fixed point and a centralised MINPACK LM whose residual uses
scipy's Rotation (independent of the oracle)."""
import numpy as np
import pytest
from scipy.optimize import minimize
from scipy.spatial.transform import Rotation

import oracle
from scenes import make_sphere_scene, make_trajectory_scene


def _rx(a):
    c, s = np.cos(a), np.sin(a)
    return np.array([[1, 0, 0], [0, c, -s], [0, s, c]])


def _ry(a):
    c, s = np.cos(a), np.sin(a)
    return np.array([[c, 0, s], [0, 1, 0], [-s, 0, c]])


def _rz(a):
    c, s = np.cos(a), np.sin(a)
    return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]])


def _cam(a, b, g, t, f=800.0):
    return np.array([a, b, g, t[0], t[1], t[2], f, 0.0, 0.0])


@pytest.mark.parametrize("angles", [(0.3, -0.2, 0.7), (3.0, 0.1, -2.5), (-1.2, 1.1, 0.4)])
def test_rotation_is_r3_r2_r1(angles):
    a, b, g = angles
    R = oracle.euler_rotation(_cam(a, b, g, (0, 0, 0)))
    np.testing.assert_allclose(R, _rz(g) @ _ry(b) @ _rx(a), atol=1e-15)
    np.testing.assert_allclose(R, Rotation.from_euler("xyz", [a, b, g]).as_matrix(), atol=1e-14)


def test_projection_by_hand():
    # identity rotation: pixels f (X + t)_{1,2} / (X + t)_3
    uv, depth = oracle.project(_cam(0, 0, 0, (0, 0, 5)), [1.0, 2.0, 0.0], "euler")
    np.testing.assert_allclose(uv, [160.0, 320.0], rtol=1e-15)
    assert depth == 5.0
    # a quarter turn about z maps x to y: (1, 0, 4) -> (0, 1, 4)
    uv, depth = oracle.project(_cam(0, 0, np.pi / 2, (0, 0, 0), f=100.0), [1.0, 0.0, 4.0], "euler")
    np.testing.assert_allclose(uv, [0.0, 25.0], atol=1e-13)
    # a quarter turn about x maps y to z: (0, 2, 1) -> (0, -1, 2)
    uv, depth = oracle.project(_cam(np.pi / 2, 0, 0, (0, 0, 0), f=10.0), [0.0, 2.0, 1.0], "euler")
    np.testing.assert_allclose(uv, [0.0, -5.0], atol=1e-13)
    assert abs(depth - 2.0) < 1e-15
    # slots 7 and 8 are not part of the model
    cam = _cam(0.2, 0.1, -0.3, (0.1, 0.2, 6))
    cam2 = cam.copy()
    cam2[7:] = [0.5, -0.3]
    assert np.array_equal(oracle.project(cam, [0.3, 0.1, 0.2], "euler")[0],
                          oracle.project(cam2, [0.3, 0.1, 0.2], "euler")[0])


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_jacobian_matches_central_differences(seed):
    rng = np.random.default_rng(seed)
    cam = _cam(*rng.uniform(-1, 1, 3), rng.uniform(-1, 1, 2).tolist() + [8.0])
    X = rng.uniform(-1, 1, 3)
    uv, J, _ = oracle.project_jac(cam, X, "euler")
    np.testing.assert_array_equal(uv, oracle.project(cam, X, "euler")[0])
    th = np.concatenate([cam, X])
    for c in range(12):
        h = 1e-6 * max(1.0, abs(th[c]))
        a, b = th.copy(), th.copy()
        a[c] += h
        b[c] -= h
        fd = (oracle.project(a[:9], a[9:], "euler")[0] - oracle.project(b[:9], b[9:], "euler")[0]) / (2 * h)
        if c in (6, 7, 8):
            # the focal length is known and there is no distortion: no column
            assert np.all(J[:, c] == 0.0)
        else:
            np.testing.assert_allclose(J[:, c], fd, rtol=1e-6, atol=1e-6 * np.abs(J).max())


def test_local_solve_moves_the_nine_unknowns_only_and_minimises():
    rng = np.random.default_rng(5)
    cam = _cam(0.2, -0.1, 0.3, (0.1, -0.2, 6.0))
    X = np.array([0.3, -0.2, 0.4])
    z = oracle.project(cam, X, "euler")[0] + rng.normal(0, 2.0, 2)
    v = np.concatenate([cam, X]) + np.r_[rng.normal(0, 1e-2, 6), 0, 0, 0, rng.normal(0, 1e-2, 3)]
    th0 = np.concatenate([cam, X])
    opts = oracle.make_opts("huber", 2.0, camera="euler")
    th, acc, tr = oracle.local_solve(opts, z, v, th0, 1e3, 1e3, steps=60)
    assert acc > 0 and np.all(np.diff(tr) <= 1e-9 * (1 + np.abs(tr[:-1])))
    assert np.array_equal(th[6:9], th0[6:9])
    free = [0, 1, 2, 3, 4, 5, 9, 10, 11]

    def f(x):
        t = th0.copy()
        t[free] = x
        return oracle.local_objective(opts, z, v, t, 1e3, 1e3)
    r = minimize(f, th0[free], method="BFGS", options=dict(gtol=1e-10, maxiter=20000))
    assert tr[-1] <= r.fun * (1 + 1e-9) + 1e-9
    np.testing.assert_allclose(th[free], r.x, atol=1e-4)


def test_noise_free_ground_truth_is_a_fixed_point():
    s = make_sphere_scene(seed=8, n_cams=12, n_points=300, noise_px=0.0, perturb=False, camera="euler")
    a = oracle.ADMM(oracle.Problem.from_scene(s), s.cams_gt, s.points_gt, loss="huber", loss_param=2.0,
                    rho=1e3, camera="euler")
    a.iterate(20)
    np.testing.assert_allclose(a.cons_y, s.cams_gt, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(a.cons_x, s.points_gt, rtol=1e-12, atol=1e-12)
    assert a.stats()[0] < 1e-9


def _minpack_lm_euler(scene):
    """Centralised l2 bundle adjustment over the 6 camera and 3 point
    unknowns of the Euler model, MINPACK LM, residuals written with scipy's
    Rotation.from_euler."""
    from scipy.optimize import least_squares
    m, n = scene.n_cams, scene.n_points
    oc, op, z = scene.obs_cam, scene.obs_point, scene.obs_uv
    f = scene.cams_init[:, 6]

    def res(th):
        cams = th[:6 * m].reshape(m, 6)
        pts = th[6 * m:].reshape(n, 3)
        P = Rotation.from_euler("xyz", cams[oc, :3]).apply(pts[op]) + cams[oc, 3:6]
        return (z - f[oc, None] * P[:, :2] / P[:, 2:3]).ravel()

    x0 = np.concatenate([scene.cams_init[:, :6].ravel(), scene.points_init.ravel()])
    r = least_squares(res, x0, method="lm", xtol=1e-15, ftol=1e-15, gtol=1e-15, max_nfev=100000)
    cams = scene.cams_init.copy()
    cams[:, :6] = r.x[:6 * m].reshape(m, 6)
    return cams, r.x[6 * m:].reshape(n, 3)


def test_admm_reaches_the_centralised_lm_optimum():
    # 8 cameras on a sphere cap, each seeing all 100 points
    s = make_sphere_scene(seed=7, n_cams=8, n_points=100, radius=8.0, box=3.0, k_lo=8, k_hi=8, camera="euler")
    p = oracle.Problem.from_scene(s)
    cams, pts = _minpack_lm_euler(s)
    lm = oracle.reprojection_stats(p, cams, pts, None, "l2", 1.0, "euler")
    a = oracle.ADMM(p, s.cams_init, s.points_init, loss="l2", loss_param=1.0, rho=1e4, camera="euler")
    init = a.stats()
    # run until both residual norms are below 1e-9 (about 3 000 iterations)
    for _ in range(60):
        tr = a.iterate(100)
        if tr[-1, 0] < 1e-9 and tr[-1, 1] < 1e-9:
            break
    assert tr[-1, 0] < 1e-9 and tr[-1, 1] < 1e-9, (a.iteration, tr[-1])
    ad = a.stats()
    assert init[0] > 10 * lm[0]
    assert abs(ad[0] - lm[0]) < 1e-6 * lm[0], (ad[0], lm[0])
    np.testing.assert_allclose(a.cons_y[:, 6:], s.cams_init[:, 6:], rtol=0, atol=0)


def test_trajectory_scenes_stay_clear_of_gimbal_lock():
    # the Euler parameterisation is singular at beta = +-pi/2; the nadir
    # trajectory and sphere-cap families keep |beta| well below it
    t = make_trajectory_scene(seed=4, n_cams=200, n_points=2000, camera="euler")
    c = make_sphere_scene(seed=8, n_cams=100, n_points=2000, camera="euler")
    assert np.abs(t.cams_init[:, 1]).max() < 0.5 and np.abs(c.cams_init[:, 1]).max() < 1.2
