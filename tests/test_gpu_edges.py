"""Edge cases of the layout against the FP64 oracle: the smallest problem
(one observation), cameras whose observations fill a 64-slot chunk exactly,
miss it by one or spill one slot into the next, point counts around 256
and 64-lane consensus waves, camera counts around the 4-camera consensus
block, long camera segments and long point tracks (beyond 512 records, where
the consensus groups grow past 8 records); a batch mixing a
one-observation problem with larger ones; empty and degenerate inputs
rejected with the documented status."""
import numpy as np
import pytest

import oracle
from paper_1708_07954_amd import binding
from scenes import make_ring_scene
from _util import param_rel_err

pytestmark = pytest.mark.gpu

KW = dict(loss="huber", loss_param=2.0, rho=1e4)

# (cameras, points): every camera sees every point, so each camera has
# `points` observations and each point `cameras`
EDGES = [(1, 1), (1, 2), (2, 63), (3, 64), (2, 65), (1, 129), (5, 255), (5, 256), (3, 257), (4, 7), (9, 3),
         # long segments: 157 chunks summed into one camera's consensus; point
         # tracks of 300 records (more than a consensus block has threads)
         (2, 10000), (300, 3),
         # tracks of 600 records: more than 512, so the consensus sums them in
         # 60 groups of 10 records
         (600, 2)]


def _oracle(sc, iters):
    a = oracle.ADMM(oracle.Problem.from_scene(sc), sc.cams_init, sc.points_init, **KW)
    a.iterate(iters)
    return a


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("n_cams,n_points", EDGES)
def test_layout_edges_match_the_oracle(n_cams, n_points, precision):
    sc = make_ring_scene(seed=11, n_cams=n_cams, n_points=n_points)
    iters = 12
    a = _oracle(sc, iters)
    s = binding.Solver(precision=precision, **KW).set_scene(sc)
    s.iterate(iters)
    cams, pts = s.params()
    err = param_rel_err(cams, pts, a.cons_y, a.cons_x)
    info = binding.dba_problem_info(s.h)
    r = s.residuals(want_rmse=True)
    s.close()
    print(n_cams, n_points, precision, "max rel err", err, info)
    assert err < (1e-9 if precision == "fp64" else 1e-3)
    assert r["iteration"] == iters and np.isfinite(r["primal"])


@pytest.mark.parametrize("n_cams,n_points", [(300, 3), (600, 2), (2, 10000), (5, 256), (3, 257), (1, 1)])
def test_segment_schedules_agree_bitwise_on_layout_edges(n_cams, n_points):
    # tracks of 300 records (38 groups of 8), of 600 (60 groups of 10), of 2
    # records (a wave of 64 points), consensus waves filled exactly or by one
    # point
    sc = make_ring_scene(seed=11, n_cams=n_cams, n_points=n_points)
    ref = None
    for sched in (1, 2, 3):
        s = binding.Solver(precision="fp64", segment_schedule=sched, **KW).set_scene(sc)
        s.iterate(5)
        got = (*s.params(), s.state()[1], s.residuals()["primal"])
        s.close()
        if ref is None:
            ref = got
            continue
        for x, y in zip(got[:3], ref[:3]):
            np.testing.assert_array_equal(x, y)
        assert got[3] == ref[3]


def test_batch_with_a_one_observation_problem():
    scenes = [make_ring_scene(seed=21, n_cams=3, n_points=70), make_ring_scene(seed=22, n_cams=1, n_points=1),
              make_ring_scene(seed=23, n_cams=2, n_points=65)]
    s = binding.Solver(precision="fp64", **KW).set_scenes(scenes)
    s.iterate(8)
    for q, sc in enumerate(scenes):
        a = _oracle(sc, 8)
        cams, pts = s.params(q)
        assert param_rel_err(cams, pts, a.cons_y, a.cons_x) < 1e-9
    s.close()


def test_empty_and_degenerate_inputs_are_rejected():
    s = binding.Solver(precision="fp64", **KW)
    z = np.zeros(0, np.int32)
    with pytest.raises(binding.DbaError) as e:
        binding.dba_set_problem(s.h, 1, 1, z, z, np.zeros((0, 2)), np.zeros((1, 9)), np.zeros((1, 3)))
    assert e.value.status == "DBA_E_INVALID_ARG"
    with pytest.raises(binding.DbaError) as e:
        binding.dba_set_problems(s.h, [])
    assert e.value.status == "DBA_E_INVALID_ARG"
    sc = make_ring_scene(seed=3, n_cams=2, n_points=4)
    cams = sc.cams_init.copy()
    cams[1, :] = np.inf
    with pytest.raises(binding.DbaError) as e:
        binding.dba_set_problem(s.h, sc.n_cams, sc.n_points, sc.obs_cam, sc.obs_point, sc.obs_uv, cams,
                                sc.points_init)
    assert e.value.status == "DBA_E_NONFINITE"
    s.set_scene(sc)
    with pytest.raises(binding.DbaError) as e:
        binding.dba_iterate(s.h, -1)
    assert e.value.status == "DBA_E_INVALID_ARG"
    s.iterate(0)
    assert s.residuals()["iteration"] == 0
    s.close()
