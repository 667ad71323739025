"""The point partition behind the multi-GPU design: each rank keeps whole
point tracks and the cameras that see them.  Checked on the CPU with the
oracle: the shards cover every observation once; one ADMM iteration on a
shard gives its points exactly the consensus of the whole problem (the point
work is rank-local); and the whole problem's camera consensus is the sum of
the ranks' camera partial sums (the one exchange per iteration), added in
rank order."""
import numpy as np
import pytest

import oracle
from scenes import make_trajectory_scene, point_shard

N_RANKS = 4


@pytest.fixture(scope="module")
def scene():
    return make_trajectory_scene(seed=4, n_cams=60, n_points=3000)


def test_shards_cover_every_observation_once(scene):
    seen = np.zeros(scene.n_obs, np.int64)
    for r in range(N_RANKS):
        sh = point_shard(scene, r, N_RANKS)
        cams, pts = sh.meta["cams"], sh.meta["points"]
        assert np.all(pts % N_RANKS == r)
        # back to the original observations: same camera, point and pixel
        orig_cam, orig_pt = cams[sh.obs_cam], pts[sh.obs_point]
        idx = np.flatnonzero(scene.obs_point % N_RANKS == r)
        assert np.array_equal(orig_cam, scene.obs_cam[idx]) and np.array_equal(orig_pt, scene.obs_point[idx])
        assert np.array_equal(sh.obs_uv, scene.obs_uv[idx])
        seen[idx] += 1
        # whole tracks: a kept point keeps all its observations; every kept camera is observed
        assert np.array_equal(np.bincount(sh.obs_point, minlength=sh.n_points),
                              np.bincount(scene.obs_point, minlength=scene.n_points)[pts])
        assert np.all(np.bincount(sh.obs_cam, minlength=sh.n_cams) > 0)
    assert np.all(seen == 1)


def test_one_iteration_point_consensus_is_rank_local_and_cameras_reduce(scene):
    kw = dict(loss="huber", loss_param=2.0, rho=1e4)
    full = oracle.ADMM(oracle.Problem.from_scene(scene), scene.cams_init, scene.points_init, **kw)
    full.iterate(1)
    cam_sum = np.zeros((scene.n_cams, 9))
    cam_cnt = np.zeros(scene.n_cams)
    for r in range(N_RANKS):
        sh = point_shard(scene, r, N_RANKS)
        a = oracle.ADMM(oracle.Problem.from_scene(sh), sh.cams_init, sh.points_init, **kw)
        a.iterate(1)
        # points: the whole problem's consensus, bit for bit
        assert np.array_equal(a.cons_x, full.cons_x[sh.meta["points"]])
        # cameras: this rank's partial sums, gathered in rank order
        m = np.bincount(sh.obs_cam, minlength=sh.n_cams)
        cam_sum[sh.meta["cams"]] += a.cons_y * m[:, None]
        cam_cnt[sh.meta["cams"]] += m
    assert np.array_equal(cam_cnt, np.bincount(scene.obs_cam, minlength=scene.n_cams))
    np.testing.assert_allclose(cam_sum / cam_cnt[:, None], full.cons_y, rtol=1e-13, atol=1e-13)
