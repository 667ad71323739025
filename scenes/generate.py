"""Seeded synthetic scenes for distributed bundle adjustment.

The paper evaluates on synthetic scenes whose cameras move smoothly and whose
points are seen in a few consecutive frames (Sec. 4.1), on a tiny 5-camera /
10-point / 50-observation problem (Sec. 4.2), and on real image sets that are
not available here (Sec. 4.3).  These generators stand in for all of them.

Camera parameter vector (9 values, one row per camera):
    (w_x, w_y, w_z, t_x, t_y, t_z, f, k1, k2)
with ``w`` an angle-axis rotation (world -> camera), ``t`` the translation,
``f`` the focal length in pixels and ``k1, k2`` radial distortion; the
principal point is at the origin.  A point ``X`` maps to ``P = R X + t`` and to
the pixel ``f * (1 + k1 r^2 + k2 r^4) * (P_1/P_3, P_2/P_3)`` with
``r^2 = (P_1^2 + P_2^2)/P_3^2`` (Sec. 2.1, Eq. 1, extended by focal length and
distortion).  Synthesis below uses scipy rotation matrices; it is only the data
recipe and shares nothing with either solver.

Observations are emitted point-major: all observations of point 0 (cameras
ascending), then point 1, and so on.
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass, field

import numpy as np
from scipy.spatial.transform import Rotation

FOCAL = 800.0
IMAGE_HALF = 500.0          # image spans [-500, 500]^2 pixels


@dataclass
class Scene:
    name: str
    seed: int
    n_cams: int
    n_points: int
    obs_cam: np.ndarray       # int32 [L]
    obs_point: np.ndarray     # int32 [L]
    obs_uv: np.ndarray        # float64 [L, 2]
    cams_init: np.ndarray     # float64 [m, 9]
    points_init: np.ndarray   # float64 [n, 3]
    cams_gt: np.ndarray       # float64 [m, 9]
    points_gt: np.ndarray     # float64 [n, 3]
    outlier: np.ndarray       # bool [L]
    meta: dict = field(default_factory=dict)

    @property
    def n_obs(self) -> int:
        return int(self.obs_cam.shape[0])

    def checksum(self) -> str:
        h = hashlib.sha256()
        for a in (self.obs_cam, self.obs_point, self.obs_uv, self.cams_init,
                  self.points_init):
            h.update(np.ascontiguousarray(a).tobytes())
        return h.hexdigest()[:16]


# --------------------------------------------------------------------------
# rigs
# --------------------------------------------------------------------------

def _look_at(centres: np.ndarray, target=np.zeros(3)) -> np.ndarray:
    """World->camera rotation matrices for cameras at ``centres`` looking at
    ``target`` with world up +z (fallback +x near the pole); image y points
    down."""
    R = np.empty((centres.shape[0], 3, 3))
    for j, c in enumerate(centres):
        z = target - c
        z = z / np.linalg.norm(z)
        up = np.array([0.0, 0.0, 1.0])
        if abs(z @ up) > 0.999:
            up = np.array([1.0, 0.0, 0.0])
        x = np.cross(z, up)
        x /= np.linalg.norm(x)
        y = np.cross(z, x)
        R[j] = np.stack([x, y, z])
    return R


def _synth_pixels(R, t, f, k1, k2, X, cam, pt):
    """Pixel coordinates and depth of points ``pt`` seen by cameras ``cam``
    (data synthesis only)."""
    P = np.einsum("kij,kj->ki", R[cam], X[pt]) + t[cam]
    depth = P[:, 2]
    p = P[:, :2] / depth[:, None]
    r2 = (p * p).sum(1)
    d = 1.0 + k1[cam] * r2 + k2[cam] * r2 * r2
    return f[cam, None] * d[:, None] * p, depth


def _assemble(name, seed, rng, R_gt, C, X_gt, obs_cam, obs_pt, *,
              noise_px=1.0, perturb=True, outlier_frac=0.0,
              rot_sigma=0.05, trans_sigma=0.2, point_sigma=0.1, meta=None, camera="angle_axis"):
    """camera "angle_axis": rows (w, t, f, k1, k2); "euler": the paper's
    camera, rows (alpha, beta, gamma, t, f, 0, 0) with R = Rz(gamma)
    Ry(beta) Rx(alpha), no distortion, the rotation perturbed in the Euler
    angles.  Both draw the same random numbers in the same order."""
    m = R_gt.shape[0]
    t_gt = -np.einsum("jik,jk->ji", R_gt, C)
    f = np.full(m, FOCAL)
    k1 = rng.uniform(-1e-2, 1e-2, m)
    k2 = rng.uniform(-1e-2, 1e-2, m)
    euler = camera == "euler"
    if euler:
        k1 = np.zeros(m)
        k2 = np.zeros(m)
        w_gt = Rotation.from_matrix(R_gt).as_euler("xyz")
    else:
        w_gt = Rotation.from_matrix(R_gt).as_rotvec()
    cams_gt = np.column_stack([w_gt, t_gt, f, k1, k2])

    uv, depth = _synth_pixels(R_gt, t_gt, f, k1, k2, X_gt, obs_cam, obs_pt)
    if noise_px > 0:
        uv = uv + rng.normal(0.0, noise_px, uv.shape)
    L = obs_cam.shape[0]
    outlier = np.zeros(L, dtype=bool)
    if outlier_frac > 0:
        k = int(round(outlier_frac * L))
        idx = rng.choice(L, size=k, replace=False)
        outlier[idx] = True
        uv[idx] = rng.uniform(-IMAGE_HALF, IMAGE_HALF, (k, 2))

    if perturb:
        dw = rng.normal(0.0, rot_sigma, (m, 3))
        if euler:
            w_init = w_gt + dw
        else:
            R_init = Rotation.from_rotvec(dw) * Rotation.from_matrix(R_gt)
            w_init = R_init.as_rotvec()
        t_init = t_gt + rng.normal(0.0, trans_sigma, (m, 3))
        X_init = X_gt + rng.normal(0.0, point_sigma, X_gt.shape)
    else:
        w_init, t_init, X_init = w_gt.copy(), t_gt.copy(), X_gt.copy()
    cams_init = np.column_stack([w_init, t_init, f, k1, k2])

    return Scene(name=name, seed=seed, n_cams=m, n_points=X_gt.shape[0],
                 obs_cam=obs_cam.astype(np.int32), obs_point=obs_pt.astype(np.int32),
                 obs_uv=np.ascontiguousarray(uv, dtype=np.float64),
                 cams_init=np.ascontiguousarray(cams_init),
                 points_init=np.ascontiguousarray(X_init),
                 cams_gt=cams_gt, points_gt=X_gt.copy(), outlier=outlier,
                 meta=dict(meta or {}, min_depth_gt=float(depth.min())))


# --------------------------------------------------------------------------
# scene families
# --------------------------------------------------------------------------

def make_ring_scene(seed=0, n_cams=10, n_points=200, radius=10.0, box=2.0,
                    name="ring", **kw) -> Scene:
    """Cameras evenly spaced on a horizontal circle looking at the origin,
    points uniform in a cube, every point seen by every camera."""
    rng = np.random.default_rng(seed)
    a = 2 * np.pi * np.arange(n_cams) / n_cams
    C = radius * np.column_stack([np.cos(a), np.sin(a), np.zeros(n_cams)])
    R = _look_at(C)
    X = rng.uniform(-box, box, (n_points, 3))
    obs_pt = np.repeat(np.arange(n_points), n_cams)
    obs_cam = np.tile(np.arange(n_cams), n_points)
    return _assemble(name, seed, rng, R, C, X, obs_cam, obs_pt, **kw)


def _choose_visibility(rng, n_points, n_cams, k_lo, k_hi):
    """For every point a uniformly random set of K ~ U{k_lo..k_hi} distinct
    cameras, returned point-major with cameras ascending."""
    K = rng.integers(k_lo, k_hi + 1, n_points)
    order = rng.random((n_points, n_cams)).argsort(axis=1)
    take = np.arange(n_cams)[None, :] < K[:, None]
    chosen = np.where(take, order, n_cams)          # n_cams sorts last
    chosen.sort(axis=1)
    obs_pt = np.repeat(np.arange(n_points), K)
    obs_cam = chosen[take]                          # row-major = point-major
    return obs_cam, obs_pt


def make_sphere_scene(seed=1, n_cams=100, n_points=20000, k_lo=8, k_hi=15,
                      radius=30.0, max_polar_deg=60.0, box=5.0, name="sphere",
                      **kw) -> Scene:
    """Cameras area-uniform on a spherical cap looking at the origin; each
    point seen by a random 8..15 of them."""
    rng = np.random.default_rng(seed)
    cz = rng.uniform(np.cos(np.radians(max_polar_deg)), 1.0, n_cams)
    phi = rng.uniform(0, 2 * np.pi, n_cams)
    sz = np.sqrt(1 - cz * cz)
    C = radius * np.column_stack([sz * np.cos(phi), sz * np.sin(phi), cz])
    R = _look_at(C)
    X = rng.uniform(-box, box, (n_points, 3))
    k_lo, k_hi = min(k_lo, n_cams), min(k_hi, n_cams)
    obs_cam, obs_pt = _choose_visibility(rng, n_points, n_cams, k_lo, k_hi)
    return _assemble(name, seed, rng, R, C, X, obs_cam, obs_pt, **kw)


def _zipf_lengths(rng, size, t_min=2, t_max=60, alpha=1.4675):
    T = np.arange(t_min, t_max + 1)
    p = T.astype(np.float64) ** -alpha
    p /= p.sum()
    return rng.choice(T, size=size, p=p)


def make_trajectory_scene(seed=2, n_cams=1000, n_points=200000, t_max=60,
                          outlier_frac=0.05, altitude=20.0, speed=0.25,
                          name="trajectory", **kw) -> Scene:
    """Nadir cameras along a smoothed random walk; each point seen in a window
    of T consecutive frames, T from a truncated Zipf law on {2..t_max}; a
    fraction of observations replaced by uniform outliers."""
    rng = np.random.default_rng(seed)
    m = n_cams
    turn = np.zeros(m)
    for j in range(1, m):
        turn[j] = 0.95 * turn[j - 1] + rng.normal(0.0, 0.004)
    heading = rng.uniform(0, 2 * np.pi) + np.cumsum(turn)
    step = speed * np.column_stack([np.cos(heading), np.sin(heading)])
    xy = np.cumsum(step, axis=0)
    C = np.column_stack([xy, altitude + rng.normal(0.0, 0.05, m)])
    xc = np.column_stack([np.cos(heading), np.sin(heading), np.zeros(m)])
    zc = np.tile([0.0, 0.0, -1.0], (m, 1))
    yc = np.cross(zc, xc)
    R0 = np.stack([xc, yc, zc], axis=1)
    tilt = Rotation.from_rotvec(rng.normal(0.0, 0.05, (m, 3)))
    R = (tilt * Rotation.from_matrix(R0)).as_matrix()
    t = -np.einsum("jik,jk->ji", R, C)

    n = n_points
    T = _zipf_lengths(rng, n, 2, min(t_max, m))
    s = rng.integers(0, m - T + 1)
    # mean camera centre of each window via prefix sums
    cs = np.vstack([np.zeros((1, 3)), np.cumsum(C, axis=0)])
    centre = (cs[s + T] - cs[s]) / T[:, None]
    obs_pt = np.repeat(np.arange(n), T)
    starts = np.repeat(s, T)
    within = np.arange(obs_pt.shape[0]) - np.repeat(np.cumsum(T) - T, T)
    obs_cam = starts + within

    f = np.full(m, FOCAL)
    zero = np.zeros(m)
    X = np.empty((n, 3))
    todo = np.arange(n)
    spread = 4.0
    for attempt in range(200):
        k = todo.shape[0]
        X[todo, :2] = centre[todo, :2] + rng.uniform(-spread, spread, (k, 2))
        X[todo, 2] = rng.uniform(-2.0, 2.0, k)
        sel = np.isin(obs_pt, todo)
        uv, depth = _synth_pixels(R, t, f, zero, zero, X, obs_cam[sel], obs_pt[sel])
        bad_obs = (np.abs(uv) > 0.97 * IMAGE_HALF).any(1) | (depth < 1.0)
        bad_pts = np.unique(obs_pt[sel][bad_obs])
        if bad_pts.size == 0:
            break
        todo = bad_pts
        if attempt % 20 == 19:
            spread *= 0.7
    else:
        raise RuntimeError("trajectory scene: could not place all points")
    return _assemble(name, seed, rng, R, C, X, obs_cam, obs_pt,
                     outlier_frac=outlier_frac, **kw)


# --------------------------------------------------------------------------
# the named workloads
# --------------------------------------------------------------------------

def make_tiny_paper_scene(seed=0, **kw) -> Scene:
    """The size of the paper's convergence study: 5 cameras, 10 points, all
    50 observations (Sec. 4.2)."""
    return make_ring_scene(seed=seed, n_cams=5, n_points=10, name="tiny5x10", **kw)


def make_config0(seed=0, **kw) -> Scene:
    """10 cameras on a radius-10 circle, 200 points in [-2,2]^3, all 2000
    observations."""
    return make_ring_scene(seed=seed, n_cams=10, n_points=200, radius=10.0,
                           box=2.0, name="ring10x200", **kw)


def make_config1(seed=1, n_cams=100, n_points=20000, **kw) -> Scene:
    """100 cameras on a sphere cap, 20000 points in [-5,5]^3, 8..15 cameras
    per point (about 230k observations)."""
    return make_sphere_scene(seed=seed, n_cams=n_cams, n_points=n_points,
                             name=f"sphere{n_cams}x{n_points}", **kw)


def make_config2(seed=2, n_cams=1000, n_points=200000, **kw) -> Scene:
    """1000 cameras on a random-walk trajectory, 200000 points, Zipf track
    lengths 2..60 (about 2M observations), 5% uniform outliers."""
    return make_trajectory_scene(seed=seed, n_cams=n_cams, n_points=n_points,
                                 name=f"trajectory{n_cams}x{n_points}", **kw)


def point_shard(scene: Scene, rank: int, n_ranks: int) -> Scene:
    """One rank's share under a partition of the observations by point:
    the points with index % n_ranks == rank keep their whole tracks, and
    the cameras that see any of them are kept (renumbered in their order);
    observations keep their relative order.  meta["cams"] / meta["points"]
    hold the kept original indices."""
    keep_pt = np.arange(scene.n_points) % n_ranks == rank
    obs = np.flatnonzero(keep_pt[scene.obs_point])
    cams = np.unique(scene.obs_cam[obs])
    pts = np.flatnonzero(keep_pt)
    cam_new = np.full(scene.n_cams, -1, np.int64)
    cam_new[cams] = np.arange(len(cams))
    pt_new = np.full(scene.n_points, -1, np.int64)
    pt_new[pts] = np.arange(len(pts))
    return Scene(name=f"{scene.name}_shard{rank}of{n_ranks}", seed=scene.seed, n_cams=len(cams),
                 n_points=len(pts), obs_cam=cam_new[scene.obs_cam[obs]].astype(np.int32),
                 obs_point=pt_new[scene.obs_point[obs]].astype(np.int32),
                 obs_uv=np.ascontiguousarray(scene.obs_uv[obs]), cams_init=scene.cams_init[cams].copy(),
                 points_init=scene.points_init[pts].copy(), cams_gt=scene.cams_gt[cams].copy(),
                 points_gt=scene.points_gt[pts].copy(), outlier=scene.outlier[obs].copy(),
                 meta=dict(scene.meta, cams=cams, points=pts, rank=rank, n_ranks=n_ranks))


def make_config3(seeds=range(1000, 1064), scale=1.0):
    """64 independent sphere-cap problems of uneven size: camera counts
    log-uniform in [5, 300], observation targets log-uniform in [2e3, 3e5].
    ``scale`` shrinks the observation targets for quick tests."""
    out = []
    for sd in seeds:
        rng = np.random.default_rng(sd)
        m = int(round(np.exp(rng.uniform(np.log(5), np.log(300)))))
        l_target = np.exp(rng.uniform(np.log(2e3), np.log(3e5))) * scale
        k_lo, k_hi = min(8, m), min(15, m)
        n = int(np.clip(round(l_target / (0.5 * (k_lo + k_hi))), 100, 30000))
        out.append(make_sphere_scene(seed=sd, n_cams=m, n_points=n, k_lo=k_lo,
                                     k_hi=k_hi, name=f"batch{sd}_{m}x{n}"))
    return out
