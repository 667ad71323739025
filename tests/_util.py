"""Shared helpers of the test suite (comparison metrics only)."""
import numpy as np

CAM_FLOOR = np.array([1, 1, 1, 1, 1, 1, 1, 1e-2, 1e-2], dtype=np.float64)


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
    sel = np.flatnonzero(np.isin(sc.obs_point, idx))[:limit]
    where = {int(p): q for q, p in enumerate(idx)}
    gap = 0.0
    for k in sel:
        j, i = int(sc.obs_cam[k]), int(sc.obs_point[k])
        a, _ = oracle.project(cams[j], pts[i])
        b, _ = oracle.project(cams_ref[j], pts_ref[where[i]])
        gap = max(gap, float(np.abs(a - b).max()))
    return gap, len(sel)


# FP32-local parity against the FP64 oracle after many iterations: 99 % of
# the parameters and the global relative error within 1e-3.  The tail is
# bounded by what the workload itself determines: e_self is the deviation of
# the FP64 oracle from its own stored run when started from a start
# perturbed at FP32 rounding size (1 +- 1e-7); a parameter the workload does
# not pin to 1e-3 under such a perturbation may differ by up to three times
# the oracle's own spread (99.9th percentile and maximum) -- FP32 rounds at
# every operation of every iteration, the reference perturbs only the start.
# Without e_self the maximum is bounded at 1e-1.
FP32_P99, FP32_GLOBAL, FP32_MAX, FP32_SPREAD = 1e-3, 1e-3, 1e-1, 3.0


def fp32_parity_ok(e, e_self=None):
    ok = e["p99"] < FP32_P99 and e["glob"] < FP32_GLOBAL
    if e_self is None:
        return ok and e["max"] < FP32_MAX
    return (ok and e["p999"] < max(FP32_P99, FP32_SPREAD * e_self["p999"])
            and e["max"] < max(FP32_P99, FP32_SPREAD * e_self["max"]))
