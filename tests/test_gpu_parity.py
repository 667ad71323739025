"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the
same seeded inputs.  FP64 path: 1e-9 relative on every parameter; FP32-local
path: 1e-3 relative and RMSE within 0.5%."""
import numpy as np
import pytest

import oracle
from paper_1708_07954_amd import binding
from scenes import make_config0, make_config2, make_ring_scene, make_sphere_scene
from _util import (CAM_FLOOR, FP32_BAR, FP64_BAR, RMSE_BAR, bar_or_gap, golden_points, param_err_summary,
                   param_rel_err, reprojection_gap, state_rel_err, worst_param)

pytestmark = pytest.mark.gpu


def gpu_run(scene, iters, **opts):
    s = binding.Solver(**opts).set_scene(scene)
    s.iterate(iters)
    return s


def oracle_run(scene, iters, *, loss, loss_param, rho, rho_balancing=False, rho_min=1e-6, rho_max=1e6,
               lm_steps=5):
    a = oracle.ADMM(oracle.Problem.from_scene(scene), scene.cams_init, scene.points_init, loss=loss,
                    loss_param=loss_param, rho=rho, rho_balancing=rho_balancing, lm_steps=lm_steps)
    a.opts.rho_min, a.opts.rho_max = rho_min, rho_max
    tr = a.iterate(iters)
    return a, tr


CASES = {
    "ring_huber_rho1e4": (lambda: make_config0(), dict(loss="huber", loss_param=2.0, rho=1e4), 50),
    "ring_huber_rho1": (lambda: make_config0(), dict(loss="huber", loss_param=2.0, rho=1.0), 50),
    "ring7x37_l2": (lambda: make_ring_scene(seed=4, n_cams=7, n_points=37), dict(loss="l2", loss_param=1.0, rho=1e3), 40),
    "sphere_t": (lambda: make_sphere_scene(seed=8, n_cams=20, n_points=700), dict(loss="student_t", loss_param=4.0, rho=1e3), 30),
    "traj_balancing": (lambda: make_config2(n_cams=60, n_points=800),
                       dict(loss="huber", loss_param=2.0, rho=1e4, rho_balancing=True, rho_min=1e4, rho_max=1e7), 30),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_fp64_parity(case):
    make, kw, iters = CASES[case]
    sc = make()
    a, tr = oracle_run(sc, iters, **kw)
    s = gpu_run(sc, iters, precision="fp64", **kw)
    cams, pts = s.params()
    err = param_rel_err(cams, pts, a.cons_y, a.cons_x)
    r = s.residuals(want_rmse=True)
    st = a.stats()
    print(case, "max rel err", err, worst_param(cams, pts, a.cons_y, a.cons_x), "r_pri", r["primal"],
          tr[-1, 0], "r_dual", r["dual"], tr[-1, 1], "rel", abs(r["primal"] / tr[-1, 0] - 1),
          abs(r["dual"] / tr[-1, 1] - 1), "rmse", r["rmse"], st[0])
    assert err < 1e-9
    assert r["iteration"] == iters
    assert r["rho_x"] == tr[-1, 2] and r["rho_y"] == tr[-1, 3]
    assert r["next_rho_x"] == a.rho[0]
    assert r["primal"] == pytest.approx(tr[-1, 0], rel=1e-9)
    assert r["dual"] == pytest.approx(tr[-1, 1], rel=1e-9)
    assert r["rmse"] == pytest.approx(st[0], rel=1e-9)
    assert r["robust_cost"] == pytest.approx(st[2], rel=1e-9)


@pytest.mark.parametrize("case", ["ring7x37_l2", "traj_balancing"])
def test_fp64_state_parity(case):
    make, kw, _ = CASES[case]
    sc = make()
    a, _ = oracle_run(sc, 7, **kw)
    s = gpu_run(sc, 7, precision="fp64", **kw)
    copies, duals = s.state()
    # the scaled duals accumulate copy - consensus, so their rounding is on
    # the scale of the copies: printed against both scales
    du = np.abs(duals - a.dual).max(axis=0)
    print(case, "copies", state_rel_err(copies, a.copy), "duals", state_rel_err(duals, a.dual),
          "duals on the copies' scale", float((du / np.abs(a.copy).max(axis=0)).max()))
    assert state_rel_err(copies, a.copy) < 1e-9
    assert float((du / np.abs(a.copy).max(axis=0)).max()) < 1e-9
    assert state_rel_err(duals, a.dual) < 1e-7


@pytest.mark.parametrize("case", ["ring_huber_rho1e4", "sphere_t", "traj_balancing"])
def test_fp32_parity(case):
    make, kw, iters = CASES[case]
    sc = make()
    a, _ = oracle_run(sc, iters, **kw)
    s = gpu_run(sc, iters, precision="fp32", **kw)
    cams, pts = s.params()
    err = param_rel_err(cams, pts, a.cons_y, a.cons_x)
    r = s.residuals(want_rmse=True)
    st = a.stats()
    print(case, "fp32 max rel err", err, worst_param(cams, pts, a.cons_y, a.cons_x), "rmse", r["rmse"], st[0])
    assert err < 1e-3
    assert abs(r["rmse"] - st[0]) < 5e-3 * st[0]


def test_dual_invariant_on_gpu():
    sc = make_sphere_scene(seed=8, n_cams=20, n_points=700)
    s = gpu_run(sc, 9, precision="fp64", loss="student_t", loss_param=4.0, rho=1e3)
    copies, duals = s.state()
    sy = np.zeros((sc.n_cams, 9))
    np.add.at(sy, sc.obs_cam, duals[:, :9])
    sx = np.zeros((sc.n_points, 3))
    np.add.at(sx, sc.obs_point, duals[:, 9:])
    scale = np.abs(copies).max()
    assert np.abs(sy).max() < 1e-12 * scale * 200
    assert np.abs(sx).max() < 1e-12 * scale * 20
    cams, pts = s.params()
    cy = np.zeros((sc.n_cams, 9))
    np.add.at(cy, sc.obs_cam, copies[:, :9])
    cy /= np.bincount(sc.obs_cam)[:, None]
    np.testing.assert_allclose(cams, cy, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_every_schedule_is_bitwise_identical(precision):
    sc = make_sphere_scene(seed=9, n_cams=30, n_points=900)
    kw = dict(precision=precision, loss="student_t", loss_param=4.0, rho=1e3)
    ref = None
    for bw in (1, 2, 4, 8):
        for pers in (0, 1):
            for graph in (False, True):
                s = gpu_run(sc, 6, block_waves=bw, persistent=pers, use_graph=graph, **kw)
                cams, pts = s.params()
                copies, duals = s.state()
                r = s.residuals()
                got = (cams, pts, copies, duals, r["primal"], r["dual"])
                if ref is None:
                    ref = got
                else:
                    for x, y in zip(got[:4], ref[:4]):
                        np.testing.assert_array_equal(x, y)
                    assert got[4:] == ref[4:]
                s.close()
    # the point-consensus segment schedules (a thread per point; a thread
    # per record group, loading directly or through LDS)
    for sched in (1, 2, 3):
        s = gpu_run(sc, 6, block_waves=4, persistent=0, segment_schedule=sched, **kw)
        assert binding.dba_segment_schedule(s.h) == dict(segment_schedule=sched, tuned=0)
        np.testing.assert_array_equal(s.params()[0], ref[0])
        np.testing.assert_array_equal(s.params()[1], ref[1])
        np.testing.assert_array_equal(s.state()[1], ref[3])
        assert s.residuals()["primal"] == ref[4]
        s.close()
    s = gpu_run(sc, 6, **kw)  # autotuned (tuning runs on real iterations)
    np.testing.assert_array_equal(s.params()[0], ref[0])
    s.iterate(10)
    assert binding.dba_schedule(s.h)["tuned"] > 1
    seg = binding.dba_segment_schedule(s.h)
    assert seg["tuned"] == 3 and seg["segment_schedule"] in (1, 2, 3)


@pytest.mark.parametrize("use_graph", [False, True])
def test_a_caller_stream_gives_the_same_iterates(use_graph):
    # dba_options.stream: the library enqueues on the caller's stream (here a
    # torch stream) instead of creating its own
    import torch
    sc = make_sphere_scene(seed=9, n_cams=30, n_points=900)
    kw = dict(precision="fp64", loss="student_t", loss_param=4.0, rho=1e3, block_waves=4, persistent=0,
              segment_schedule=1)
    ref = gpu_run(sc, 6, **kw)
    want = (*ref.params(), ref.state()[1])
    ref.close()
    st = torch.cuda.Stream()
    s = binding.Solver(stream=st.cuda_stream, use_graph=use_graph, **kw).set_scene(sc)
    s.iterate(6)
    done = torch.cuda.Event()
    done.record(st)
    done.synchronize()
    got = (*s.params(), s.state()[1])
    s.close()
    for x, y in zip(got, want):
        np.testing.assert_array_equal(x, y)


def test_iterate_in_pieces_equals_one_call():
    sc = make_config0()
    kw = dict(precision="fp64", loss="huber", loss_param=2.0, rho=1e4, block_waves=4, persistent=0)
    a = gpu_run(sc, 37, **kw)
    b = binding.Solver(**kw).set_scene(sc)
    for n in (1, 16, 3, 17):
        b.iterate(n)
    np.testing.assert_array_equal(a.params()[0], b.params()[0])
    np.testing.assert_array_equal(a.state()[1], b.state()[1])


def test_input_validation_errors():
    sc = make_ring_scene(seed=1, n_cams=4, n_points=10)
    s = binding.Solver(precision="fp64")
    bad = sc.obs_uv.copy()
    bad[3, 1] = np.nan
    with pytest.raises(binding.DbaError) as e:
        binding.dba_set_problem(s.h, sc.n_cams, sc.n_points, sc.obs_cam, sc.obs_point, bad,
                                sc.cams_init, sc.points_init)
    assert e.value.status == "DBA_E_NONFINITE"
    oc = sc.obs_cam.copy()
    oc[0] = 4
    with pytest.raises(binding.DbaError) as e:
        binding.dba_set_problem(s.h, sc.n_cams, sc.n_points, oc, sc.obs_point, sc.obs_uv,
                                sc.cams_init, sc.points_init)
    assert e.value.status == "DBA_E_INDEX_RANGE"
    keep = sc.obs_point != 3
    with pytest.raises(binding.DbaError) as e:
        binding.dba_set_problem(s.h, sc.n_cams, sc.n_points, sc.obs_cam[keep], sc.obs_point[keep],
                                sc.obs_uv[keep], sc.cams_init, sc.points_init)
    assert e.value.status == "DBA_E_UNOBSERVED"
    cams = sc.cams_init.copy()
    cams[2, 3:6] = 0.0     # camera at the origin of a scene around the origin
    cams[2, :3] = 0.0
    pts = sc.points_init.copy()
    pts[:, 2] = -np.abs(pts[:, 2]) - 1.0
    with pytest.raises(binding.DbaError) as e:
        binding.dba_set_problem(s.h, sc.n_cams, sc.n_points, sc.obs_cam, sc.obs_point, sc.obs_uv, cams, pts)
    assert e.value.status == "DBA_E_BEHIND_CAMERA"
    with pytest.raises(binding.DbaError) as e:
        binding.dba_iterate(s.h, 1)
    assert e.value.status == "DBA_E_STATE"
    # a failed set keeps the previous problem
    s.set_scene(sc)
    s.iterate(2)
    with pytest.raises(binding.DbaError):
        binding.dba_set_problem(s.h, sc.n_cams, sc.n_points, oc, sc.obs_point, sc.obs_uv,
                                sc.cams_init, sc.points_init)
    assert s.residuals()["iteration"] == 2


# ---------------------------------------------------------------- full-size workloads
import os  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _golden(name):
    path = os.path.join(GOLDEN, f"{name}.npz")
    if not os.path.exists(path):
        pytest.skip(f"{name}.npz not generated (tests/golden/make_golden.py {name})")
    return np.load(path)


def _spread(name, g, precision, at=None):
    """The FP64 oracle's own deviation from its stored run `g` when its start
    is perturbed by one rounding unit of `precision` (1e-7 for fp32, 2^-52 for
    fp64; tests/golden/<name>_perturbed[_fp64].npz), after `at` iterations or
    at the end; None if not stored."""
    path = os.path.join(GOLDEN, f"{name}_perturbed{'_fp64' if precision == 'fp64' else ''}.npz")
    if not os.path.exists(path):
        return None
    z = np.load(path)
    assert str(z["checksum"]) == str(g["checksum"]) and z["points"].shape == g["points"].shape
    if at is None:
        return param_err_summary(z["cams"], z["points"], g["cams"], g["points"])
    return param_err_summary(z[f"cams_at{at}"], z[f"points_at{at}"], g[f"cams_at{at}"], g[f"points_at{at}"])


def _check_stored(name, g, s, precision, at, gaps):
    """Every parameter of handle `s` against the stored run (after `at`
    iterations, or at its end); a gap is collected, not passed."""
    cams, pts = s.params()
    ref_c, ref_p = (g["cams"], g["points"]) if at is None else (g[f"cams_at{at}"], g[f"points_at{at}"])
    e = param_err_summary(cams, pts[golden_points(g)], ref_c, ref_p)
    spread = _spread(name, g, precision, at)
    its = int(g["iterations"]) if at is None else at
    print(f"{precision} {name} after {its} iterations: rel err {e}",
          worst_param(cams, pts[golden_points(g)], ref_c, ref_p), "oracle spread", spread, flush=True)
    gap = bar_or_gap(e, FP64_BAR if precision == "fp64" else FP32_BAR, spread, f"{precision} {name}, {its} iterations")
    if gap:
        gaps.append(gap)
    return e


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_sphere_workload_matches_stored_oracle(precision):
    """100 cameras, 20000 points, ~230k observations, Student-t, 100
    iterations, against the stored FP64 oracle run after 20 and after 100
    iterations: every camera and point parameter within the bar (1e-9 FP64,
    1e-3 FP32), RMSE within 0.5 % (FP32) or 1e-9 (FP64); a parameter past the
    bar is a stated gap (_util.bar_or_gap)."""
    from scenes import make_config1
    g = _golden("sphere")
    sc = make_config1()
    assert str(g["checksum"]) == sc.checksum()
    s = gpu_run(sc, 20, precision=precision, loss="student_t", loss_param=4.0, rho=1e3)
    gaps = []
    _check_stored("sphere", g, s, precision, 20, gaps)
    s.iterate(int(g["iterations"]) - 20)
    _check_stored("sphere", g, s, precision, None, gaps)
    r = s.residuals(want_rmse=True)
    print("rmse", r["rmse"], g["stats"][0])
    assert abs(r["rmse"] - g["stats"][0]) < (FP64_BAR if precision == "fp64" else RMSE_BAR) * g["stats"][0]
    if gaps:
        pytest.xfail("; ".join(gaps))


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_trajectory_workload_matches_stored_oracle(precision):
    """The benchmark workload: 1000 cameras, 200000 points, 2.006M
    observations, Huber, rho balancing, 200 iterations, against the stored
    FP64 oracle run after 20 and after 200 iterations: every camera and point
    parameter within the bar (1e-3 with FP32 local solves, 1e-9 in FP64),
    inlier RMSE within 0.5 %; a parameter past the bar is a stated gap
    (_util.bar_or_gap).  The pixel difference between the two estimates'
    predictions is printed."""
    from scenes import make_config2
    g = _golden("trajectory")
    sc = make_config2()
    assert str(g["checksum"]) == sc.checksum()
    s = binding.Solver(precision=precision, loss="huber", loss_param=2.0, rho=1e5, rho_balancing=True,
                       rho_min=1e5, rho_max=1e7).set_scene(sc)
    s.set_eval_mask(~sc.outlier)
    gaps = []
    s.iterate(20)
    _check_stored("trajectory", g, s, precision, 20, gaps)
    s.iterate(int(g["iterations"]) - 20)
    e = _check_stored("trajectory", g, s, precision, None, gaps)
    cams, pts = s.params()
    r = s.residuals(want_rmse=True)
    gap, n_gap = reprojection_gap(sc, cams, pts, g["cams"], g["points"], golden_points(g))
    ec = np.abs(cams - g["cams"]) / np.maximum(np.abs(g["cams"]), CAM_FLOOR)
    print("inlier rmse", r["rmse_masked"], g["stats"][1], "max per camera column", ec.max(0),
          "reprojection gap px", gap, "over", n_gap, "next rho", r["next_rho_x"], g["rho"][0])
    assert abs(r["rmse_masked"] - g["stats"][1]) < RMSE_BAR * g["stats"][1]
    if gaps:
        pytest.xfail("; ".join(gaps))


def test_full_size_first_iterations_match_oracle():
    """The 2.006M-observation workload in the benchmark's launch configuration
    against the oracle run at test time: every camera and point within 1e-3
    (FP32 local solves) after the first iteration, within 1e-9 (FP64) after
    the first and after the fifth.  (Later the workload's weakly determined
    parameters drift apart under any difference of rounding: reading 17 and
    test_trajectory_workload_matches_stored_oracle.)"""
    from scenes import make_config2
    sc = make_config2()
    kw = dict(loss="huber", loss_param=2.0, rho=1e5, rho_balancing=True, rho_min=1e5, rho_max=1e7)
    a, _ = oracle_run(sc, 1, **kw)
    runs = {p: gpu_run(sc, 1, precision=p, block_waves=1, persistent=0, **kw) for p in ("fp32", "fp64")}
    for its, checks in ((1, (("fp32", FP32_BAR), ("fp64", FP64_BAR))), (5, (("fp64", FP64_BAR),))):
        if its > 1:
            a.iterate(its - 1)
        for precision, tol in checks:
            s = runs[precision]
            s.iterate(its - s.residuals()["iteration"])
            cams, pts = s.params()
            e = param_err_summary(cams, pts, a.cons_y, a.cons_x)
            print(precision, f"full-size, {its} iteration(s): rel err", e, worst_param(cams, pts, a.cons_y, a.cons_x),
                  flush=True)
            assert e["max"] < tol
    for s in runs.values():
        s.close()
