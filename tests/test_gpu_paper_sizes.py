"""Problems of the sizes of the paper's real-data table (Sec. 4.3, Table 1:
cameras, points and observations of its four datasets, about 2.6-2.9
observations per point), as synthetic trajectories with tracks of 2-4
consecutive frames about 6 degrees apart and no outliers, since the datasets themselves are not
available: FP64 within 1e-9 of the oracle after 20 iterations; FP32 with the
global parameter error within 1e-3 and the RMSE within 0.5 % (the per-parameter
errors, which exceed 1e-3 in weakly determined parameters here, are printed);
one problem at a time and all four batched."""
import numpy as np
import pytest

import oracle
from paper_1708_07954_amd import binding
from scenes import make_trajectory_scene
from _util import param_err_summary, param_rel_err, worst_param

pytestmark = pytest.mark.gpu

SIZES = [(11, 1346), (10, 1382), (25, 2161), (30, 2383)]
KW = dict(loss="huber", loss_param=2.0, rho=1e3)
ITERS = 20


def _scenes():
    # frames 2 units apart at altitude 20 (about 6 degrees of parallax per frame), as
    # in a hand-held or aerial capture; the benchmark trajectory's 0.25-unit spacing
    # would leave 2-4-frame tracks nearly without parallax
    return [make_trajectory_scene(seed=300 + q, n_cams=m, n_points=n, t_max=4, outlier_frac=0.0, speed=2.0,
                                  name=f"paper_table1_{m}x{n}") for q, (m, n) in enumerate(SIZES)]


def _oracle(sc):
    a = oracle.ADMM(oracle.Problem.from_scene(sc), sc.cams_init, sc.points_init, **KW)
    a.iterate(ITERS)
    return a


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_paper_table1_sizes(precision):
    scenes = _scenes()
    print("observations per scene", [sc.n_obs for sc in scenes],
          "per point", [round(sc.n_obs / sc.n_points, 2) for sc in scenes])
    refs = [_oracle(sc) for sc in scenes]
    batched = binding.Solver(precision=precision, **KW).set_scenes(scenes)
    batched.iterate(ITERS)
    for q, (sc, a) in enumerate(zip(scenes, refs)):
        s = binding.Solver(precision=precision, **KW).set_scene(sc)
        s.iterate(ITERS)
        cams, pts = s.params()
        err = param_rel_err(cams, pts, a.cons_y, a.cons_x)
        r = s.residuals(want_rmse=True)
        print(sc.name, precision, "max rel err", err, worst_param(cams, pts, a.cons_y, a.cons_x), "rmse", r["rmse"],
              a.stats()[0])
        if precision == "fp64":
            assert err < 1e-9
        else:
            # 2-4-frame tracks leave some point depths and distortion terms
            # weakly determined: an FP32 local solve settles them on the model's
            # word once F cannot resolve the step (the tie rule), ~1e-4 from
            # where FP64 settles, and ADMM carries that to ~1e-2 in the worst of
            # them after 20 iterations (99th percentile ~1e-3).  The global error
            # and the reprojection RMSE hold the FP32 bar.
            e = param_err_summary(cams, pts, a.cons_y, a.cons_x)
            print("   fp32 error summary", e)
            assert e["glob"] < 1e-3
            assert abs(r["rmse"] - a.stats()[0]) < 5e-3 * a.stats()[0]
        b = batched.params(q)
        assert np.array_equal(b[0], cams) and np.array_equal(b[1], pts)
        s.close()
    batched.close()
