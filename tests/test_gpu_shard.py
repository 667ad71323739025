"""The point partition of the multi-GPU design, on the GPU path: one
iteration of the 2M-observation trajectory on each of 8 point shards (whole
tracks per rank, the cameras that see them) against one iteration of the whole
problem, through the C ABI.  The shards' point consensus equals the whole
problem's bit for bit (the point work is rank-local), and the rank-ordered sum
of the shards' camera partial sums gives the whole problem's camera
consensus."""
import numpy as np
import pytest

from paper_1708_07954_amd import binding
from scenes import make_config2, point_shard

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_point_shards_reproduce_the_whole_iteration(precision):
    sc = make_config2()
    kw = dict(precision=precision, loss="huber", loss_param=2.0, rho=1e5, rho_balancing=True, rho_min=1e5,
              rho_max=1e7)
    s = binding.Solver(**kw).set_scene(sc)
    s.iterate(1)
    cams_full, pts_full = s.params()
    s.close()
    n_ranks = 8
    cam_sum = np.zeros((sc.n_cams, 9))
    cam_cnt = np.zeros(sc.n_cams)
    for r in range(n_ranks):
        sh = point_shard(sc, r, n_ranks)
        s = binding.Solver(**kw).set_scene(sh)
        s.iterate(1)
        cams, pts = s.params()
        s.close()
        assert np.array_equal(pts, pts_full[sh.meta["points"]]), r
        m = np.bincount(sh.obs_cam, minlength=sh.n_cams)
        cam_sum[sh.meta["cams"]] += cams * m[:, None]
        cam_cnt[sh.meta["cams"]] += m
    assert np.array_equal(cam_cnt, np.bincount(sc.obs_cam, minlength=sc.n_cams))
    err = np.abs(cam_sum / cam_cnt[:, None] - cams_full) / np.maximum(np.abs(cams_full), 1e-2)
    print(precision, "camera consensus from the shards' partial sums, max rel err", err.max())
    assert err.max() < 1e-12
