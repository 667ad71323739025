"""Shared helpers of the test suite (comparison metrics only)."""
import numpy as np

CAM_FLOOR = np.array([1, 1, 1, 1, 1, 1, 1, 1e-2, 1e-2], dtype=np.float64)


def golden_points(g):
    """Indexes of the points a stored oracle run holds (every point unless it
    stores a sample ``points_idx``)."""
    return g["points_idx"] if "points_idx" in g.files else slice(None)


def param_rel_err(cams, pts, cams_ref, pts_ref):
    """Max over components of |a - b| / max(|b|, floor): floor 1 for rotation,
    translation, focal and points, 1e-2 for the distortion terms."""
    ec = np.abs(cams - cams_ref) / np.maximum(np.abs(cams_ref), CAM_FLOOR)
    ep = np.abs(pts - pts_ref) / np.maximum(np.abs(pts_ref), 1.0)
    return float(max(ec.max(), ep.max()))


def state_rel_err(a, b):
    """Max |a - b| over a (L, 12) state, relative to the per-column scale of b."""
    scale = np.maximum(np.abs(b).max(axis=0), 1e-300)
    return float((np.abs(a - b) / scale).max())


def worst_param(cams, pts, cams_ref, pts_ref):
    """(kind, index, component, value, reference) of the largest relative error."""
    ec = np.abs(cams - cams_ref) / np.maximum(np.abs(cams_ref), CAM_FLOOR)
    ep = np.abs(pts - pts_ref) / np.maximum(np.abs(pts_ref), 1.0)
    if ec.max() >= ep.max():
        j, c = np.unravel_index(ec.argmax(), ec.shape)
        return ("cam", int(j), int(c), float(cams[j, c]), float(cams_ref[j, c]))
    i, c = np.unravel_index(ep.argmax(), ep.shape)
    return ("point", int(i), int(c), float(pts[i, c]), float(pts_ref[i, c]))


def param_err_summary(cams, pts, cams_ref, pts_ref):
    """Per-component relative errors (floors as param_rel_err): max, 99th and
    99.9th percentile, and the global |a - b| / |b| over all parameters."""
    ec = np.abs(cams - cams_ref) / np.maximum(np.abs(cams_ref), CAM_FLOOR)
    ep = np.abs(pts - pts_ref) / np.maximum(np.abs(pts_ref), 1.0)
    e = np.concatenate([ec.ravel(), ep.ravel()])
    a = np.concatenate([cams.ravel(), pts.ravel()])
    b = np.concatenate([cams_ref.ravel(), pts_ref.ravel()])
    return dict(max=float(e.max()), p99=float(np.percentile(e, 99)), p999=float(np.percentile(e, 99.9)),
                glob=float(np.linalg.norm(a - b) / np.linalg.norm(b)))


def reprojection_gap(sc, cams, pts, cams_ref, pts_ref, idx, limit=20000):
    """Largest pixel difference between the predictions of two estimates
    (FP64 oracle projection) over observations of the points idx; pts is the
    full point array, pts_ref holds the points idx."""
    import oracle
    if isinstance(idx, slice):
        idx = np.arange(len(pts_ref))
    sel = np.flatnonzero(np.isin(sc.obs_point, idx))[:limit]
    where = {int(p): q for q, p in enumerate(idx)}
    gap = 0.0
    for k in sel:
        j, i = int(sc.obs_cam[k]), int(sc.obs_point[k])
        a, _ = oracle.project(cams[j], pts[i])
        b, _ = oracle.project(cams_ref[j], pts_ref[where[i]])
        gap = max(gap, float(np.abs(a - b).max()))
    return gap, len(sel)


# Parity bars against the FP64 oracle (frozen; a change needs its own commit
# and a written reading): every parameter within FP64_BAR (FP64 path) or
# FP32_BAR (FP32 local solves and the learned start), relative per component
# as param_rel_err; reprojection RMSE within RMSE_BAR.
FP64_BAR, FP32_BAR, RMSE_BAR = 1e-9, 1e-3, 5e-3
# A parameter past its bar after many iterations is a stated gap, not a pass:
# the test reports it (pytest xfail, with the numbers) only when the oracle
# moves that far itself -- at every quantile of the per-parameter error (99th,
# 99.9th percentile, maximum) and for the global error, within SPREAD_FACTOR
# times the deviation of the FP64 oracle from its own stored run when its
# start is perturbed by one rounding unit of the precision
# (tests/golden/*_perturbed*.npz), or within the bar.  The GPU rounds
# differently at every iteration, the perturbed oracle only at the start, so
# the factor allows for the accumulation over the iterations (measured: 13.5
# on the sphere workload in FP64 after 100 iterations).  Anything beyond it
# fails.
SPREAD_FACTOR = 30.0


def bar_or_gap(e, bar, spread=None, what=""):
    """Checks a param_err_summary against its bar.  Returns None when every
    parameter meets the bar.  Otherwise each of p99, p99.9, max and the
    global error must be within the bar or within SPREAD_FACTOR times the
    same statistic of the oracle's own spread; then returns the gap's
    description for pytest.xfail.  Raises AssertionError in every other
    case (no stored spread included)."""
    if e["max"] < bar:
        return None
    assert spread is not None, (what, "over the bar with no stored oracle spread", e)
    for k in ("p99", "p999", "max", "glob"):
        assert e[k] < max(bar, SPREAD_FACTOR * spread[k]), (what, k, e, "oracle spread", spread)
    return (f"{what}: gap -- max parameter error {e['max']:.3g} exceeds the bar {bar:g} "
            f"(p99 {e['p99']:.2g}, p99.9 {e['p999']:.2g}, global {e['glob']:.2g}); the FP64 oracle itself "
            f"moves {spread['max']:.3g} (p99 {spread['p99']:.2g}, p99.9 {spread['p999']:.2g}) when its start "
            f"is perturbed by one rounding unit")
