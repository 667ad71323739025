"""ctypes binding of libdba.so: the C ABI of include/dba.h under the same
names, plus a small ``Solver`` convenience wrapper.  Argument marshalling
only: every step of the iteration runs in the library's HIP kernels.  There
is no fallback -- if the library is missing, or no GPU is visible, calls
raise."""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdba.so")

DBA_OK = 0
CAMERA = {"angle_axis": 0, "euler": 1}
SOLVER = {"lm": 0, "gauss_newton": 1, "lbfgs": 2}
STATUS = {0: "DBA_OK", -1: "DBA_E_INVALID_ARG", -2: "DBA_E_INDEX_RANGE", -3: "DBA_E_UNOBSERVED",
          -4: "DBA_E_NONFINITE", -5: "DBA_E_BEHIND_CAMERA", -6: "DBA_E_DEVICE", -7: "DBA_E_STATE"}
LOSS = {"l2": 0, "huber": 1, "student_t": 2}
PRECISION = {"fp64": 0, "fp32": 1}
START = {"plain": 0, "learned": 1}
KERNELS = ("local", "consensus", "norms", "learned")


class DbaError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code
        self.status = STATUS.get(code, str(code))


class dba_options(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("stream", ctypes.c_void_p),
                ("precision", ctypes.c_int32), ("loss", ctypes.c_int32),
                ("loss_param", ctypes.c_double), ("rho_x", ctypes.c_double),
                ("rho_y", ctypes.c_double), ("rho_balancing", ctypes.c_int32),
                ("rb_mu", ctypes.c_double), ("rb_tau", ctypes.c_double),
                ("rho_min", ctypes.c_double), ("rho_max", ctypes.c_double),
                ("lm_steps", ctypes.c_int32), ("lm_lambda0", ctypes.c_double),
                ("start", ctypes.c_int32), ("learned_lm_steps", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("block_waves", ctypes.c_int32),
                ("persistent", ctypes.c_int32), ("camera_blocks", ctypes.c_int32),
                ("block_points", ctypes.c_int32), ("camera_model", ctypes.c_int32),
                ("local_solver", ctypes.c_int32), ("block_cameras", ctypes.c_int32),
                ("segment_schedule", ctypes.c_int32)]


class dba_problem_desc(ctypes.Structure):
    _fields_ = [("n_cams", ctypes.c_int32), ("n_points", ctypes.c_int32),
                ("n_obs", ctypes.c_int64), ("obs_cam", ctypes.c_void_p),
                ("obs_point", ctypes.c_void_p), ("obs_uv", ctypes.c_void_p),
                ("cams", ctypes.c_void_p), ("points", ctypes.c_void_p)]


class dba_residual_report(ctypes.Structure):
    _fields_ = [("primal", ctypes.c_double), ("dual", ctypes.c_double),
                ("rho_x", ctypes.c_double), ("rho_y", ctypes.c_double),
                ("next_rho_x", ctypes.c_double), ("next_rho_y", ctypes.c_double),
                ("rmse", ctypes.c_double), ("rmse_masked", ctypes.c_double),
                ("robust_cost", ctypes.c_double), ("mean_error", ctypes.c_double),
                ("iteration", ctypes.c_int64), ("nonfinite", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


# exported symbols of include/dba.h
EXPORTS = ("dba_default_options", "dba_create", "dba_destroy", "dba_last_error",
           "dba_set_problem", "dba_set_problems", "dba_iterate", "dba_residuals",
           "dba_set_eval_mask", "dba_get_params", "dba_get_state", "dba_problem_info",
           "dba_set_kernel_timing", "dba_kernel_times", "dba_schedule", "dba_segment_schedule", "dba_set_mlp", "dba_get_mlp",
           "dba_set_start", "dba_mlp_forward", "dba_mlp_forward_noalloc", "dba_mlp_loss_grad", "dba_collect_pairs", "dba_mlp_train",
           "dba_mlp_apply_gradient", "dba_mlp_adam_state")
MLP_PARAMS, MLP_NORM = 22800, 76

_lib = None


def load(path: Optional[str] = None) -> ctypes.CDLL:
    """Loads libdba.so (build it with ``python -m paper_1708_07954_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run python -m paper_1708_07954_amd.build")
    # One HIP runtime per process: the library's libamdhip64.so.7 resolves to
    # whichever copy is loaded first.  Where PyTorch is installed its bundled
    # runtime must be that copy -- with the system one loaded first, PyTorch's
    # device initialisation fails (hipErrorNoDevice) -- so it is imported
    # before the library.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(path)
    P = ctypes.POINTER
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    L.dba_default_options.argtypes = [P(dba_options)]
    L.dba_create.argtypes = [P(dba_options), P(vp)]
    L.dba_destroy.argtypes = [vp]
    L.dba_destroy.restype = None
    L.dba_last_error.argtypes = [vp]
    L.dba_last_error.restype = ctypes.c_char_p
    L.dba_set_problem.argtypes = [vp, i32, i32, i64, vp, vp, vp, vp, vp]
    L.dba_set_problems.argtypes = [vp, i32, P(dba_problem_desc)]
    L.dba_iterate.argtypes = [vp, i32]
    L.dba_residuals.argtypes = [vp, i32, i32, P(dba_residual_report)]
    L.dba_set_eval_mask.argtypes = [vp, i32, vp]
    L.dba_get_params.argtypes = [vp, i32, vp, vp]
    L.dba_get_state.argtypes = [vp, i32, vp, vp]
    L.dba_problem_info.argtypes = [vp, i32, P(i32), P(i32), P(i64)]
    L.dba_set_kernel_timing.argtypes = [vp, i32]
    L.dba_kernel_times.argtypes = [vp, P(dbl), P(i64)]
    L.dba_schedule.argtypes = [vp, P(i32), P(i32), P(i32)]
    L.dba_segment_schedule.argtypes = [vp, P(i32), P(i32)]
    if hasattr(L, "dba_set_mlp"):
        _declare_learned(L)
    _lib = L
    return L


def _declare_learned(L):
    vp, i32, i64, dbl, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_uint64
    L.dba_set_mlp.argtypes = [vp, vp, vp]
    L.dba_get_mlp.argtypes = [vp, vp, vp]
    L.dba_set_start.argtypes = [vp, i32, i32]
    L.dba_mlp_forward.argtypes = [vp, vp, i64, vp]
    L.dba_mlp_forward_noalloc.argtypes = [vp, vp, i64, vp]
    L.dba_mlp_loss_grad.argtypes = [vp, vp, vp, i32, vp, vp, vp]
    L.dba_collect_pairs.argtypes = [vp, i32, i32, u64, i32, vp, vp]
    L.dba_mlp_train.argtypes = [vp, vp, vp, i64, i32, i32, dbl, u64, vp]
    L.dba_mlp_apply_gradient.argtypes = [vp, vp, dbl]
    L.dba_mlp_adam_state.argtypes = [vp, vp, vp, ctypes.POINTER(i64)]


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def _check(h, rc):
    if rc != DBA_OK:
        msg = load().dba_last_error(h).decode() if h else ""
        raise DbaError(rc, msg)


def make_options(*, device=0, stream=None, precision="fp64", loss="huber", loss_param=2.0, rho=1.0,
                 rho_x=None, rho_y=None, rho_balancing=False, rb_mu=10.0, rb_tau=2.0,
                 rho_min=1e-6, rho_max=1e6, lm_steps=5, lm_lambda0=1e-3, start="plain",
                 learned_lm_steps=2, use_graph=True, block_waves=0, persistent=-1,
                 camera_blocks=False, block_points=0, camera="angle_axis", solver="lm",
                 block_cameras=1, segment_schedule=0) -> dba_options:
    """dba_options from keywords: enum fields by name (precision "fp64" /
    "fp32"; loss "l2" / "huber" / "student_t"; start "plain" / "learned";
    camera "angle_axis" / "euler"; solver "lm" / "gauss_newton" / "lbfgs"),
    the rest as in dba.h (lm_steps counts L-BFGS iterations for "lbfgs")."""
    o = dba_options()
    _check(None, load().dba_default_options(ctypes.byref(o)))
    o.device = device
    o.stream = stream
    o.precision = PRECISION[precision] if isinstance(precision, str) else int(precision)
    o.loss = LOSS[loss] if isinstance(loss, str) else int(loss)
    o.loss_param = float(loss_param)
    o.rho_x = float(rho if rho_x is None else rho_x)
    o.rho_y = float(rho if rho_y is None else rho_y)
    o.rho_balancing = int(bool(rho_balancing))
    o.rb_mu, o.rb_tau, o.rho_min, o.rho_max = float(rb_mu), float(rb_tau), float(rho_min), float(rho_max)
    o.lm_steps = int(lm_steps)
    o.lm_lambda0 = float(lm_lambda0)
    o.start = START[start] if isinstance(start, str) else int(start)
    o.learned_lm_steps = int(learned_lm_steps)
    o.use_graph = int(bool(use_graph))
    o.block_waves = int(block_waves)
    o.persistent = int(persistent)
    o.camera_blocks = int(bool(camera_blocks))
    o.block_points = int(block_points)
    o.camera_model = CAMERA[camera]
    o.local_solver = SOLVER[solver]
    o.block_cameras = int(block_cameras)
    o.segment_schedule = int(segment_schedule)
    return o


# ---------------------------------------------------------------- C-ABI names

def dba_create(opt: dba_options) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    _check(None, load().dba_create(ctypes.byref(opt), ctypes.byref(h)))
    return h


def dba_destroy(h):
    load().dba_destroy(h)


def _problem_arrays(obs_cam, obs_point, obs_uv, cams, points):
    oc = np.ascontiguousarray(obs_cam, dtype=np.int32)
    op = np.ascontiguousarray(obs_point, dtype=np.int32)
    uv = np.ascontiguousarray(obs_uv, dtype=np.float64).reshape(-1)
    cm = np.ascontiguousarray(cams, dtype=np.float64).reshape(-1)
    pt = np.ascontiguousarray(points, dtype=np.float64).reshape(-1)
    return oc, op, uv, cm, pt


def dba_set_problem(h, n_cams, n_points, obs_cam, obs_point, obs_uv, cams, points):
    oc, op, uv, cm, pt = _problem_arrays(obs_cam, obs_point, obs_uv, cams, points)
    _check(h, load().dba_set_problem(h, int(n_cams), int(n_points), oc.shape[0], _ptr(oc), _ptr(op),
                                     _ptr(uv), _ptr(cm), _ptr(pt)))


def dba_set_problems(h, problems: Sequence[dict]):
    keep, descs = [], (dba_problem_desc * len(problems))()
    for q, p in enumerate(problems):
        arrs = _problem_arrays(p["obs_cam"], p["obs_point"], p["obs_uv"], p["cams"], p["points"])
        keep.append(arrs)
        oc, op, uv, cm, pt = arrs
        descs[q] = dba_problem_desc(int(p["n_cams"]), int(p["n_points"]), oc.shape[0], oc.ctypes.data,
                                    op.ctypes.data, uv.ctypes.data, cm.ctypes.data, pt.ctypes.data)
    _check(h, load().dba_set_problems(h, len(problems), descs))


def dba_iterate(h, n_iters: int):
    _check(h, load().dba_iterate(h, int(n_iters)))


def dba_residuals(h, problem=0, want_rmse=False) -> dict:
    r = dba_residual_report()
    _check(h, load().dba_residuals(h, int(problem), int(bool(want_rmse)), ctypes.byref(r)))
    return r.as_dict()


def dba_set_eval_mask(h, problem, mask):
    m = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
    _check(h, load().dba_set_eval_mask(h, int(problem), _ptr(m)))


def dba_problem_info(h, problem=0):
    m, n, L = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
    _check(h, load().dba_problem_info(h, int(problem), ctypes.byref(m), ctypes.byref(n), ctypes.byref(L)))
    return m.value, n.value, L.value


def dba_get_params(h, problem=0):
    m, n, _ = dba_problem_info(h, problem)
    cams, pts = np.zeros((m, 9)), np.zeros((n, 3))
    _check(h, load().dba_get_params(h, int(problem), _ptr(cams), _ptr(pts)))
    return cams, pts


def dba_get_state(h, problem=0):
    _, _, L = dba_problem_info(h, problem)
    copies, duals = np.zeros((L, 12)), np.zeros((L, 12))
    _check(h, load().dba_get_state(h, int(problem), _ptr(copies), _ptr(duals)))
    return copies, duals


def dba_set_kernel_timing(h, enable, local_only=False, sampled=False):
    """enable: time every kernel; local_only: the local solve only; sampled:
    the local solve only, in the first iteration of each graph replay."""
    _check(h, load().dba_set_kernel_timing(h, (3 if sampled else 2 if local_only else 1) if enable else 0))


def dba_kernel_times(h) -> dict:
    ms = (ctypes.c_double * 4)()
    n = (ctypes.c_int64 * 4)()
    _check(h, load().dba_kernel_times(h, ms, n))
    return {k: (ms[q], n[q]) for q, k in enumerate(KERNELS)}


def dba_schedule(h):
    bw, pe, tu = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(h, load().dba_schedule(h, ctypes.byref(bw), ctypes.byref(pe), ctypes.byref(tu)))
    return dict(block_waves=bw.value, persistent=pe.value, tuned=tu.value)


def dba_segment_schedule(h):
    sl, tu = ctypes.c_int32(), ctypes.c_int32()
    _check(h, load().dba_segment_schedule(h, ctypes.byref(sl), ctypes.byref(tu)))
    return dict(segment_schedule=sl.value, tuned=tu.value)


def _f32(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float32)
    if shape is not None and a.shape != shape:
        a = a.reshape(shape)
    return a


def dba_set_mlp(h, params, norm):
    p, n = _f32(params).reshape(-1), _f32(norm).reshape(-1)
    assert p.size == MLP_PARAMS and n.size == MLP_NORM
    _check(h, load().dba_set_mlp(h, _ptr(p), _ptr(n)))


def dba_get_mlp(h):
    p, n = np.zeros(MLP_PARAMS, np.float32), np.zeros(MLP_NORM, np.float32)
    _check(h, load().dba_get_mlp(h, _ptr(p), _ptr(n)))
    return p, n


def dba_set_start(h, start, learned_lm_steps=2):
    _check(h, load().dba_set_start(h, START[start] if isinstance(start, str) else int(start), int(learned_lm_steps)))


def dba_mlp_forward(h, features):
    f = _f32(features).reshape(-1, 26)
    out = np.zeros((f.shape[0], 12), np.float32)
    _check(h, load().dba_mlp_forward(h, _ptr(f), f.shape[0], _ptr(out)))
    return out


def dba_mlp_forward_noalloc(h, features_ptr: int, n: int, delta_ptr: int):
    """Allocation-free evaluation on device buffers: features_ptr points to
    [n][26] FP32, delta_ptr to [n][12] FP32 (device addresses, e.g. a torch
    tensor's data_ptr()); enqueued on the handle's stream, not synchronised."""
    _check(h, load().dba_mlp_forward_noalloc(h, ctypes.c_void_p(int(features_ptr)), int(n),
                                             ctypes.c_void_p(int(delta_ptr))))


def dba_mlp_loss_grad(h, x_std, t_std):
    x, t = _f32(x_std).reshape(-1, 32), _f32(t_std).reshape(-1, 16)
    n = x.shape[0]
    loss = np.zeros(1, np.float32)
    grad = np.zeros(MLP_PARAMS, np.float32)
    y = np.zeros((n, 16), np.float32)
    _check(h, load().dba_mlp_loss_grad(h, _ptr(x), _ptr(t), n, _ptr(loss), _ptr(grad), _ptr(y)))
    return float(loss[0]), grad, y


def dba_collect_pairs(h, n_iters, per_iter, seed=0, conv_steps=30):
    f = np.zeros((n_iters * per_iter, 26), np.float32)
    d = np.zeros((n_iters * per_iter, 12), np.float32)
    _check(h, load().dba_collect_pairs(h, int(n_iters), int(per_iter), int(seed), int(conv_steps), _ptr(f), _ptr(d)))
    return f, d


def dba_mlp_train(h, features, deltas, epochs=10, batch=4096, lr=1e-3, seed=0):
    f, d = _f32(features).reshape(-1, 26), _f32(deltas).reshape(-1, 12)
    assert f.shape[0] == d.shape[0]
    el = np.zeros(int(epochs), np.float32)
    _check(h, load().dba_mlp_train(h, _ptr(f), _ptr(d), f.shape[0], int(epochs), int(batch), float(lr), int(seed),
                                   _ptr(el)))
    return el


def dba_mlp_apply_gradient(h, grad, lr):
    g = _f32(grad).reshape(-1)
    assert g.shape[0] == MLP_PARAMS
    _check(h, load().dba_mlp_apply_gradient(h, _ptr(g), float(lr)))


def dba_mlp_adam_state(h):
    """(m, v, step) of the network's Adam optimiser."""
    m = np.zeros(MLP_PARAMS, np.float32)
    v = np.zeros(MLP_PARAMS, np.float32)
    step = ctypes.c_int64(0)
    _check(h, load().dba_mlp_adam_state(h, _ptr(m), _ptr(v), ctypes.byref(step)))
    return m, v, int(step.value)


# ---------------------------------------------------------------- convenience

class Solver:
    """One handle: ``Solver(**options).set_scene(scene).iterate(n)``."""

    def __init__(self, **options):
        self.opt = make_options(**options)
        self.h = dba_create(self.opt)

    def close(self):
        if self.h:
            dba_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_scene(self, s, cams=None, points=None):
        dba_set_problem(self.h, s.n_cams, s.n_points, s.obs_cam, s.obs_point, s.obs_uv,
                        s.cams_init if cams is None else cams,
                        s.points_init if points is None else points)
        return self

    def set_scenes(self, scenes):
        dba_set_problems(self.h, [dict(n_cams=s.n_cams, n_points=s.n_points, obs_cam=s.obs_cam,
                                       obs_point=s.obs_point, obs_uv=s.obs_uv, cams=s.cams_init,
                                       points=s.points_init) for s in scenes])
        return self

    def iterate(self, n):
        dba_iterate(self.h, n)
        return self

    def residuals(self, problem=0, want_rmse=False):
        return dba_residuals(self.h, problem, want_rmse)

    def params(self, problem=0):
        return dba_get_params(self.h, problem)

    def state(self, problem=0):
        return dba_get_state(self.h, problem)

    def set_eval_mask(self, mask, problem=0):
        dba_set_eval_mask(self.h, problem, mask)
