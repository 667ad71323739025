"""Batched execution: many problems of uneven size in the same launches.
Each problem keeps its own rho, residuals and iteration count, equals the
same problem run alone bit for bit, and matches the FP64 oracle (stored
results written by tests/golden/make_golden.py from oracle/ only)."""
import os

import numpy as np
import pytest

from paper_1708_07954_amd import binding
from scenes import make_config2, make_config3, make_ring_scene
from _util import FP32_BAR, FP64_BAR, RMSE_BAR, bar_or_gap, param_err_summary, param_rel_err

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _batch(count=16, scale=0.02):
    return make_config3(scale=scale)[:count]


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_batched_equals_solo_bitwise(precision):
    scenes = _batch(8)
    kw = dict(precision=precision, loss="student_t", loss_param=4.0, rho=1e3, block_waves=2, persistent=1)
    b = binding.Solver(**kw).set_scenes(scenes)
    b.iterate(12)
    for q, sc in enumerate(scenes):
        s = binding.Solver(**kw).set_scene(sc)
        s.iterate(12)
        np.testing.assert_array_equal(b.params(q)[0], s.params()[0])
        np.testing.assert_array_equal(b.params(q)[1], s.params()[1])
        np.testing.assert_array_equal(b.state(q)[1], s.state()[1])
        rb, rs = b.residuals(q), s.residuals()
        assert rb["primal"] == rs["primal"] and rb["dual"] == rs["dual"] and rb["iteration"] == 12
        s.close()


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-9), ("fp32", 1e-3)])
def test_batched_matches_stored_oracle(precision, tol):
    g = np.load(os.path.join(GOLDEN, "batch.npz"))
    scenes = _batch(int(g["count"]), float(g["scale"]))
    b = binding.Solver(precision=precision, loss="student_t", loss_param=4.0, rho=1e3).set_scenes(scenes)
    b.iterate(int(g["iterations"]))
    worst = 0.0
    for q, sc in enumerate(scenes):
        assert str(g[f"checksum{q}"]) == sc.checksum()
        cams, pts = b.params(q)
        worst = max(worst, param_rel_err(cams, pts, g[f"cams{q}"], g[f"points{q}"]))
    print(precision, "worst problem rel err", worst)
    assert worst < tol


def test_problems_keep_their_own_rho():
    """Residual balancing acts per problem: a problem far from consensus and a
    converged one get different rho in the same launches."""
    far = make_config2(n_cams=40, n_points=400)
    still = make_ring_scene(seed=2, n_cams=6, n_points=40, noise_px=0.0, perturb=False)
    kw = dict(precision="fp64", loss="huber", loss_param=2.0, rho=1e2, rho_balancing=True, rho_min=1e-6, rho_max=1e9)
    b = binding.Solver(**kw).set_scenes([far, still])
    b.iterate(5)
    r0, r1 = b.residuals(0), b.residuals(1)
    assert r0["next_rho_x"] != r1["next_rho_x"]
    # each problem's chunks read its own control block: both match their solo runs bit for bit
    for q, sc in enumerate((far, still)):
        s = binding.Solver(**kw).set_scene(sc)
        s.iterate(5)
        assert b.residuals(q)["next_rho_x"] == s.residuals()["next_rho_x"]
        np.testing.assert_array_equal(b.params(q)[0], s.params()[0])
        np.testing.assert_array_equal(b.params(q)[1], s.params()[1])
        s.close()
    b.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_full_size_batched_workload_matches_stored_oracle(precision):
    """The batched workload at full size -- 64 problems, 2.98M observations
    in the same launches, autotuned schedule, replayed graphs, 100 iterations
    -- with its smallest, median and largest problem against stored FP64
    oracle runs of each problem alone (tests/golden/batch_full.npz): every
    camera and point parameter within the bar (1e-9 FP64, 1e-3 FP32) and the
    RMSE within 0.5 %; a parameter past the bar is a stated gap against the
    oracle's own spread under a start perturbed by one rounding unit
    (_util.bar_or_gap)."""
    g = np.load(os.path.join(GOLDEN, "batch_full.npz"))
    spread_file = os.path.join(GOLDEN, "batch_full_perturbed" + ("_fp64" if precision == "fp64" else "") + ".npz")
    z = np.load(spread_file) if os.path.exists(spread_file) else None
    scenes = make_config3()
    print(f"{precision}: {len(scenes)} problems, {sum(sc.n_obs for sc in scenes)} observations", flush=True)
    b = binding.Solver(precision=precision, loss="student_t", loss_param=4.0, rho=1e3).set_scenes(scenes)
    b.iterate(int(g["iterations"]))
    sched = binding.dba_schedule(b.h)
    gaps = []
    for q in (int(x) for x in g["members"]):
        sc = scenes[q]
        assert str(g[f"checksum{q}"]) == sc.checksum()
        cams, pts = b.params(q)
        e = param_err_summary(cams, pts, g[f"cams{q}"], g[f"points{q}"])
        spread = None if z is None else param_err_summary(z[f"cams{q}"], z[f"points{q}"], g[f"cams{q}"],
                                                          g[f"points{q}"])
        r = b.residuals(q, want_rmse=True)
        print(f"{precision} problem {q} ({sc.n_obs} observations): rel err {e}, rmse {r['rmse']} "
              f"oracle {g[f'stats{q}'][0]}, oracle spread {spread}, schedule {sched}", flush=True)
        assert abs(r["rmse"] - g[f"stats{q}"][0]) < RMSE_BAR * g[f"stats{q}"][0]
        gap = bar_or_gap(e, FP64_BAR if precision == "fp64" else FP32_BAR, spread, f"{precision} batched problem {q}")
        if gap:
            gaps.append(gap)
    b.close()
    if gaps:
        pytest.xfail("; ".join(gaps))
