"""GPU parity of the paper's own camera (Sec. 2.1, Eq. 1: Euler angles and
translation, known focal length, no distortion; camera_model = euler)
against the FP64 oracle on the same seeded scenes: FP64 within 1e-9 on every
parameter, FP32 within 1e-3 and RMSE within 0.5 %, for the per-observation
and the block local updates; the unused camera slots stay bitwise at their
values; state, batched = solo, and validation."""
import numpy as np
import pytest

import oracle
from paper_1708_07954_amd import binding
from scenes import make_sphere_scene, make_trajectory_scene
from _util import param_rel_err, state_rel_err

pytestmark = pytest.mark.gpu

CASES = {
    "sphere_t": (lambda: make_sphere_scene(seed=8, n_cams=20, n_points=700, camera="euler"),
                 dict(loss="student_t", loss_param=4.0, rho=1e3), 12),
    "traj_huber_balancing": (lambda: make_trajectory_scene(seed=4, n_cams=40, n_points=900, camera="euler"),
                             dict(loss="huber", loss_param=2.0, rho=1e4, rho_balancing=True, rho_min=1e4,
                                  rho_max=1e7), 12),
    "sphere_l2": (lambda: make_sphere_scene(seed=9, n_cams=10, n_points=300, k_lo=4, k_hi=8, camera="euler"),
                  dict(loss="l2", loss_param=1.0, rho=1e4), 15),
}


def _oracle(sc, iters, blocks=False, rho_min=1e-6, rho_max=1e6, **kw):
    p = oracle.Problem.from_scene(sc)
    if blocks:
        a = oracle.BlockADMM(p, sc.cams_init, sc.points_init, block=64, camera="euler", **kw)
    else:
        a = oracle.ADMM(p, sc.cams_init, sc.points_init, camera="euler", **kw)
    a.opts.rho_min, a.opts.rho_max = rho_min, rho_max
    tr = a.iterate(iters)
    return a, tr


def _gpu(sc, iters, **kw):
    s = binding.Solver(camera="euler", **kw).set_scene(sc)
    s.iterate(iters)
    return s


@pytest.mark.parametrize("blocks", [False, True])
@pytest.mark.parametrize("case", sorted(CASES))
def test_euler_fp64_parity(case, blocks):
    make, kw, iters = CASES[case]
    sc = make()
    a, tr = _oracle(sc, iters, blocks=blocks, **kw)
    s = _gpu(sc, iters, precision="fp64", camera_blocks=blocks, **kw)
    cams, pts = s.params()
    err = param_rel_err(cams, pts, a.cons_y, a.cons_x)
    r = s.residuals(want_rmse=True)
    print(case, "blocks" if blocks else "per-observation", "max rel err", err, "rmse", r["rmse"], a.stats()[0])
    assert err < 1e-9
    assert r["primal"] == pytest.approx(tr[-1, 0], rel=1e-6)
    assert r["dual"] == pytest.approx(tr[-1, 1], rel=1e-6)
    assert r["rmse"] == pytest.approx(a.stats()[0], rel=1e-9)
    # the focal length and the unused slots never move
    assert np.array_equal(cams[:, 6:], sc.cams_init[:, 6:])
    s.close()


@pytest.mark.parametrize("blocks", [False, True])
@pytest.mark.parametrize("case", ["sphere_t", "traj_huber_balancing"])
def test_euler_fp32_parity(case, blocks):
    make, kw, iters = CASES[case]
    sc = make()
    a, _ = _oracle(sc, iters, blocks=blocks, **kw)
    s = _gpu(sc, iters, precision="fp32", camera_blocks=blocks, **kw)
    cams, pts = s.params()
    err = param_rel_err(cams, pts, a.cons_y, a.cons_x)
    r = s.residuals(want_rmse=True)
    print(case, "blocks" if blocks else "per-observation", "fp32 max rel err", err, "rmse", r["rmse"], a.stats()[0])
    assert err < 1e-3
    assert abs(r["rmse"] - a.stats()[0]) < 5e-3 * a.stats()[0]
    assert np.array_equal(cams[:, 6:], sc.cams_init[:, 6:])
    s.close()


def test_euler_state_parity():
    make, kw, _ = CASES["sphere_t"]
    sc = make()
    a, _ = _oracle(sc, 5, **kw)
    s = _gpu(sc, 5, precision="fp64", **kw)
    copies, duals = s.state()
    assert state_rel_err(copies, a.copy) < 1e-9
    assert state_rel_err(duals, a.dual) < 1e-7
    s.close()


def test_euler_batched_equals_solo_bitwise():
    scenes = [make_sphere_scene(seed=40 + q, n_cams=6 + 2 * q, n_points=150 + 40 * q, camera="euler") for q in range(3)]
    kw = dict(precision="fp32", loss="huber", loss_param=2.0, rho=1e3, camera="euler")
    s = binding.Solver(**kw).set_scenes(scenes)
    s.iterate(6)
    for q, sc in enumerate(scenes):
        solo = binding.Solver(**kw).set_scene(sc)
        solo.iterate(6)
        a, b = s.params(q), solo.params()
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
        solo.close()
    s.close()


def test_euler_validation():
    with pytest.raises(binding.DbaError) as e:
        binding.Solver(precision="fp32", camera="euler", start="learned")
    assert e.value.status == "DBA_E_INVALID_ARG"
    sc = make_sphere_scene(seed=8, n_cams=5, n_points=60, camera="euler")
    for slot, value in ((7, 1e-3), (8, -1e-3), (6, 0.0)):
        cams = sc.cams_init.copy()
        cams[2, slot] = value
        s = binding.Solver(precision="fp64", camera="euler")
        with pytest.raises(binding.DbaError) as e:
            s.set_scene(sc, cams=cams)
        assert e.value.status == "DBA_E_INVALID_ARG", slot
        s.close()
    # a point moved behind its camera at the start
    pts = sc.points_init.copy()
    R = oracle.euler_rotation(sc.cams_init[0])
    c = -R.T @ sc.cams_init[0, 3:6]              # camera centre
    k = int(np.flatnonzero(sc.obs_cam == 0)[0])
    i = sc.obs_point[k]
    pts[i] = c - 1.0 * R[2]                     # one unit behind along the optical axis
    s = binding.Solver(precision="fp64", camera="euler")
    with pytest.raises(binding.DbaError) as e:
        s.set_scene(sc, points=pts)
    assert e.value.status == "DBA_E_BEHIND_CAMERA"
    s.close()


def test_euler_full_size_first_iteration_matches_oracle():
    """One iteration of the 2M-observation trajectory workload with the Euler
    camera (seed 7), in the benchmark's launch configuration, against the
    oracle run at test time: FP64 within 1e-9, FP32 within 1e-3."""
    from scenes import make_config2
    sc = make_config2(seed=7, camera="euler")
    kw = dict(loss="huber", loss_param=2.0, rho=1e5, rho_balancing=True)
    a, _ = _oracle(sc, 1, rho_min=1e5, rho_max=1e7, **kw)
    for precision, tol in (("fp32", 1e-3), ("fp64", 1e-9)):
        s = _gpu(sc, 1, precision=precision, rho_min=1e5, rho_max=1e7, block_waves=1, persistent=0, **kw)
        cams, pts = s.params()
        err = param_rel_err(cams, pts, a.cons_y, a.cons_x)
        print(precision, "Euler full-size 1-iteration max rel err", err)
        assert err < tol
        s.close()


def test_euler_convergence_study_problems_match_the_oracle():
    """Problems of the l2-vs-Huber convergence study (5 cameras, 10 points,
    50 observations, point noise 0.2 .. 1.7), batched, against the oracle run
    on each alone: FP64 within 1e-9 after 15 iterations."""
    scenes = [make_sphere_scene(seed=1000 + q, n_cams=5, n_points=10, k_lo=5, k_hi=5, radius=10.0, box=2.0,
                                rot_sigma=0.1, trans_sigma=0.1, point_sigma=sig, camera="euler")
              for q, sig in enumerate((0.2, 0.8, 1.4, 1.7))]
    for loss, lp in (("l2", 1.0), ("huber", 2.0)):
        s = binding.Solver(precision="fp64", camera="euler", loss=loss, loss_param=lp, rho=100.0).set_scenes(scenes)
        s.iterate(15)
        for q, sc in enumerate(scenes):
            a = oracle.ADMM(oracle.Problem.from_scene(sc), sc.cams_init, sc.points_init, loss=loss, loss_param=lp,
                            rho=100.0, camera="euler")
            a.iterate(15)
            cams, pts = s.params(q)
            err = param_rel_err(cams, pts, a.cons_y, a.cons_x)
            print(loss, q, "max rel err", err)
            assert err < 1e-9
        s.close()


def test_euler_full_size_200_iterations_match_the_stored_oracle():
    """The 2M trajectory with the Euler camera (seed 7), FP32 local solves,
    200 iterations, against the stored FP64 oracle run: every parameter within
    1e-3 (a parameter past it is a stated gap, _util.bar_or_gap, against the
    oracle's own spread under FP32-size perturbations of its start), inlier
    RMSE within 0.5 %, the unused camera slots bitwise unchanged."""
    import os
    from scenes import make_config2
    from _util import FP32_BAR, RMSE_BAR, bar_or_gap, golden_points, param_err_summary
    here = os.path.join(os.path.dirname(__file__), "golden")
    path = os.path.join(here, "trajectory_euler.npz")
    if not os.path.exists(path):
        pytest.skip("stored oracle run not generated (tests/golden/make_golden.py trajectory_euler)")
    g = np.load(path)
    sc = make_config2(seed=7, camera="euler")
    assert str(g["checksum"]) == sc.checksum()
    s = binding.Solver(precision="fp32", camera="euler", loss="huber", loss_param=2.0, rho=1e5, rho_balancing=True,
                       rho_min=1e5, rho_max=1e7).set_scene(sc)
    s.set_eval_mask(~sc.outlier)
    s.iterate(int(g["iterations"]))
    cams, pts = s.params()
    e = param_err_summary(cams, pts[golden_points(g)], g["cams"], g["points"])
    spread = None
    pp = os.path.join(here, "trajectory_euler_perturbed.npz")
    if os.path.exists(pp):
        q = np.load(pp)
        spread = param_err_summary(q["cams"], q["points"], g["cams"], g["points"])
    r = s.residuals(want_rmse=True)
    print("Euler trajectory rel err", e, "inlier rmse", r["rmse_masked"], g["stats"][1], "oracle self-spread", spread)
    assert abs(r["rmse_masked"] - g["stats"][1]) < RMSE_BAR * g["stats"][1]
    assert np.array_equal(cams[:, 6:], sc.cams_init[:, 6:])
    s.close()
    gap = bar_or_gap(e, FP32_BAR, spread, "fp32 Euler trajectory, 200 iterations")
    if gap:
        pytest.xfail(gap)
