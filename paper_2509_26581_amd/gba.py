"""Python binding of the gfx950 bundle-adjustment library (libgba.so).

Argument marshalling only: every function forwards to the C ABI of the same
name declared in include/gba.h; all arithmetic runs in the HIP kernels.  The
library is required: importing a function that needs it raises GbaError when
libgba.so has not been built (python -m paper_2509_26581_amd.build).

PyTorch is used only as plumbing: `torch_allocator()` hands the library
PyTorch's caching allocator and `torch_stream()` the current HIP stream.
"""
import ctypes
import os

import numpy as np

LIB_PATH = os.environ.get("GBA_LIBRARY") or os.path.join(
    os.path.dirname(os.path.abspath(__file__)), "libgba.so")

GBA_OK = 0
ERRORS = {-1: "INVALID_ARG", -2: "UNKNOWN_ID", -3: "DUPLICATE_ID", -4: "NONFINITE",
          -5: "OOM", -6: "HIP", -7: "STATE", -8: "UNSUPPORTED", -9: "BUDGET"}
GBA_PENDING = 1

GBA_FP64, GBA_MIXED_FP32, GBA_MIXED_BF16 = 0, 1, 2
GBA_LOSS_SQUARED, GBA_LOSS_HUBER = 0, 1
GBA_PRECOND_IDENTITY, GBA_PRECOND_BLOCK_JACOBI = 0, 1
GBA_ACC_AUTO, GBA_ACC_LDS, GBA_ACC_CAMERA_PASS, GBA_ACC_CAMERA_BLOCKS = 0, 1, 2, 3
GBA_PCG_AUTO, GBA_PCG_CHUNKED, GBA_PCG_PERSISTENT = 0, 1, 2
GBA_JACOBIAN_ANALYTIC, GBA_JACOBIAN_AUTODIFF, GBA_JACOBIAN_DYNAMIC = 0, 1, 2
GBA_SOLVER_SCHUR, GBA_SOLVER_FULL = 0, 1
GBA_VI_PRE_STRIDE = 148
TERMINATION = {0: "NONE", 1: "MAX_ITERS", 2: "COST_TOL", 3: "STEP_TOL",
               4: "LAMBDA_OVERFLOW", 5: "NUMERICAL_FAILURE", 6: "NO_WORK"}


class GbaError(RuntimeError):
    def __init__(self, status, message=""):
        super().__init__(f"gba error {status} ({ERRORS.get(status, '?')}): {message}")
        self.status = status


class gba_options(ctypes.Structure):
    _fields_ = [("initial_lambda", ctypes.c_double), ("min_diag", ctypes.c_double),
                ("max_diag", ctypes.c_double), ("pcg_max_iters", ctypes.c_int),
                ("pcg_tol", ctypes.c_double), ("pcg_tol_relative", ctypes.c_int),
                ("pcg_rejection_ratio", ctypes.c_double), ("precond", ctypes.c_int),
                ("timing", ctypes.c_int), ("accumulation", ctypes.c_int),
                ("tiles_per_block", ctypes.c_int), ("deterministic", ctypes.c_int),
                ("jacobi_scaling", ctypes.c_int), ("pcg_schedule", ctypes.c_int),
                ("jacobian", ctypes.c_int), ("solver", ctypes.c_int)]


class gba_report(ctypes.Structure):
    _fields_ = [("initial_cost", ctypes.c_double), ("final_cost", ctypes.c_double),
                ("final_lambda", ctypes.c_double), ("trials", ctypes.c_int),
                ("accepted", ctypes.c_int), ("pcg_iters_total", ctypes.c_int),
                ("termination", ctypes.c_int), ("ms_total", ctypes.c_double),
                ("ms_linearize", ctypes.c_double), ("ms_precond", ctypes.c_double),
                ("ms_pcg", ctypes.c_double), ("ms_other", ctypes.c_double),
                ("ms_matvec", ctypes.c_double), ("matvec_count", ctypes.c_int),
                ("reserved_i", ctypes.c_int), ("workspace_bytes", ctypes.c_size_t)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved_i"}
        d["termination_name"] = TERMINATION.get(self.termination, "?")
        return d


class gba_trial(ctypes.Structure):
    _fields_ = [("cost", ctypes.c_double), ("candidate_cost", ctypes.c_double),
                ("lambda_", ctypes.c_double), ("model_decrease", ctypes.c_double),
                ("step_norm", ctypes.c_double), ("accepted", ctypes.c_int),
                ("pcg_iters", ctypes.c_int)]


class gba_problem(ctypes.Structure):
    _fields_ = [("n_cams", ctypes.c_int32), ("n_pts", ctypes.c_int32), ("n_edges", ctypes.c_int64),
                ("cams", ctypes.c_void_p), ("pts", ctypes.c_void_p), ("cam_idx", ctypes.c_void_p),
                ("pt_idx", ctypes.c_void_p), ("uv", ctypes.c_void_p), ("info", ctypes.c_void_p),
                ("cam_fixed", ctypes.c_void_p), ("pt_fixed", ctypes.c_void_p),
                ("max_iters", ctypes.c_int32), ("reserved", ctypes.c_int32), ("tol", ctypes.c_double)]


class gba_result(ctypes.Structure):
    _fields_ = [("cams", ctypes.c_void_p), ("pts", ctypes.c_void_p), ("report", gba_report),
                ("latency_ms", ctypes.c_double), ("queue_ms", ctypes.c_double),
                ("batch_peak", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class gba_server_config(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("device", ctypes.c_int),
                ("hbm_budget_bytes", ctypes.c_size_t), ("max_slots", ctypes.c_int),
                ("loss", ctypes.c_int), ("delta", ctypes.c_double), ("options", gba_options),
                ("tune_db", ctypes.c_char_p), ("tiles_per_block", ctypes.c_int),
                ("edges_per_block", ctypes.c_int), ("pts_per_block", ctypes.c_int),
                ("pcg_sync_every", ctypes.c_int), ("reserved", ctypes.c_int * 8)]


class gba_serving_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("admitted", ctypes.c_int64),
                ("rejected", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("collected", ctypes.c_int64), ("in_flight", ctypes.c_int64),
                ("queued", ctypes.c_int64), ("trials_run", ctypes.c_int64),
                ("repacks", ctypes.c_int64), ("mean_batch", ctypes.c_double),
                ("p50_latency_ms", ctypes.c_double), ("p99_latency_ms", ctypes.c_double),
                ("p50_service_ms", ctypes.c_double), ("p99_service_ms", ctypes.c_double),
                ("solves_per_s", ctypes.c_double), ("bytes_in_use", ctypes.c_size_t),
                ("bytes_peak", ctypes.c_size_t), ("budget", ctypes.c_size_t),
                ("tiles_per_block", ctypes.c_int), ("edges_per_block", ctypes.c_int),
                ("pts_per_block", ctypes.c_int), ("pcg_sync_every", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)

_lib = None
_P = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)
_I64 = ctypes.POINTER(ctypes.c_int64)

class gba_vi_problem(ctypes.Structure):
    _fields_ = [("n_kf", ctypes.c_int32), ("reserved0", ctypes.c_int32),
                ("n_pts", ctypes.c_int64), ("n_obs", ctypes.c_int64),
                ("states", ctypes.c_void_p), ("pts", ctypes.c_void_p), ("kf", ctypes.c_void_p),
                ("pt", ctypes.c_void_p), ("obs", ctypes.c_void_p), ("intr", ctypes.c_void_p),
                ("pre", ctypes.c_void_p), ("sigma_px", ctypes.c_double),
                ("huber_delta2", ctypes.c_double), ("sigma_gw", ctypes.c_double),
                ("sigma_aw", ctypes.c_double)]


class gba_vi_options(ctypes.Structure):
    _fields_ = [("pcg_max_iters", ctypes.c_int), ("solver", ctypes.c_int),
                ("pcg_tol", ctypes.c_double), ("initial_lambda", ctypes.c_double),
                ("min_diag", ctypes.c_double), ("max_diag", ctypes.c_double),
                ("precision", ctypes.c_int), ("reserved1", ctypes.c_int),
                ("pcg_rejection_ratio", ctypes.c_double)]


_SIGS = {
    "gba_default_options": (None, [ctypes.POINTER(gba_options)]),
    "gba_create": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ALLOC_FN, FREE_FN, _P,
                                  ctypes.POINTER(_P)]),
    "gba_set_stream": (ctypes.c_int, [_P, _P]),
    "gba_reserve": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64]),
    "gba_add_cameras": (ctypes.c_int, [_P, ctypes.c_int64, _I64, _D]),
    "gba_add_points": (ctypes.c_int, [_P, ctypes.c_int64, _I64, _D]),
    "gba_add_edges": (ctypes.c_int, [_P, ctypes.c_int64, _I64, _I64, _D, _D]),
    "gba_set_fixed": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int64, ctypes.c_int]),
    "gba_set_edge_active": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_int]),
    "gba_set_robust_kernel": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_double]),
    "gba_set_options": (ctypes.c_int, [_P, ctypes.POINTER(gba_options)]),
    "gba_prepare": (ctypes.c_int, [_P]),
    "gba_solve": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_double, ctypes.POINTER(gba_report)]),
    "gba_reset": (ctypes.c_int, [_P]),
    "gba_get_cost": (ctypes.c_int, [_P, _D]),
    "gba_get_cameras": (ctypes.c_int, [_P, _D]),
    "gba_get_points": (ctypes.c_int, [_P, _D]),
    "gba_get_trials": (ctypes.c_int, [_P, ctypes.c_int, ctypes.POINTER(gba_trial),
                                      ctypes.POINTER(ctypes.c_int)]),
    "gba_eval_edges": (ctypes.c_int, [_P, _D, _D, _D, _D]),
    "gba_eval_edges_noalloc": (ctypes.c_int, [_P, _D, _D, _D, _D]),
    "gba_eval_normal_equations": (ctypes.c_int, [_P, _D, _D, _D, _D]),
    "gba_eval_step": (ctypes.c_int, [_P, ctypes.c_double, _D, _D, ctypes.POINTER(ctypes.c_int)]),
    "gba_time_matvec": (ctypes.c_int, [_P, ctypes.c_double, ctypes.c_int, _D]),
    "gba_hbm_probe": (ctypes.c_int, [ctypes.c_int, _P, ctypes.c_size_t, _P, ctypes.c_int, _P, _D]),
    "gba_vi_preintegrate": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _P, _D, _D, ctypes.c_double,
                                           _D, ctypes.c_double, ctypes.c_double, _D]),
    "gba_vi_eval_inertial": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _D, _D, _D, _D]),
    "gba_vi_eval_stereo": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _D, ctypes.c_int64, _D,
                                          ctypes.c_int64, _P, _P, _D, _D, _D, _D]),
    "gba_vi_default_options": (None, [ctypes.POINTER(gba_vi_options)]),
    "gba_vi_solve": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(gba_vi_problem), ctypes.c_int,
                                    ctypes.c_double, ctypes.POINTER(gba_vi_options),
                                    ctypes.POINTER(gba_report), _P, ctypes.c_int,
                                    ctypes.POINTER(ctypes.c_int)]),
    "gba_last_error": (ctypes.c_char_p, [_P]),
    "gba_destroy": (None, [_P]),
    "gba_server_default_config": (None, [ctypes.POINTER(gba_server_config)]),
    "gba_server_create": (ctypes.c_int, [ctypes.POINTER(gba_server_config), ALLOC_FN, FREE_FN, _P,
                                         ctypes.POINTER(_P)]),
    "gba_server_submit": (ctypes.c_int, [_P, ctypes.POINTER(gba_problem),
                                         ctypes.POINTER(ctypes.c_uint64)]),
    "gba_server_poll": (ctypes.c_int, [_P, ctypes.c_uint64, ctypes.c_int, ctypes.POINTER(gba_result)]),
    "gba_server_stats": (ctypes.c_int, [_P, ctypes.POINTER(gba_serving_stats)]),
    "gba_server_last_error": (ctypes.c_char_p, [_P]),
    "gba_server_destroy": (None, [_P]),
}


def load(path=LIB_PATH):
    """Load libgba.so; raise GbaError if it is absent (no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise GbaError(-8, f"{path} is not built; run python -m paper_2509_26581_amd.build")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def exported_symbols():
    return list(_SIGS)


def _ptr(a, dtype=np.float64):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(np.ctypeslib.as_ctypes_type(dtype)))


def _arr(a, dtype, shape_tail=None):
    a = np.ascontiguousarray(a, dtype=dtype)
    if shape_tail is not None:
        a = a.reshape((-1,) + tuple(shape_tail))
    return a


def _check(h, status):
    if status != GBA_OK:
        msg = load().gba_last_error(h)
        raise GbaError(status, msg.decode() if msg else "")


# ---------------------------------------------------------------- C names
def gba_default_options():
    o = gba_options()
    load().gba_default_options(ctypes.byref(o))
    return o


class _Allocator:
    """Keeps ctypes callbacks alive for the lifetime of a graph."""

    def __init__(self, alloc_fn, free_fn):
        self.alloc = ALLOC_FN(alloc_fn)
        self.free = FREE_FN(free_fn)


def torch_allocator(device=0):
    """PyTorch caching-allocator callbacks (device memory plumbing only)."""
    import torch

    def _alloc(nbytes, ctx):
        stream = torch.cuda.current_stream(device).cuda_stream
        return torch.cuda.caching_allocator_alloc(int(nbytes), device, stream)

    def _free(ptr, ctx):
        torch.cuda.caching_allocator_delete(ptr)

    return _Allocator(_alloc, _free)


def torch_stream(device=0):
    import torch
    return torch.cuda.current_stream(device).cuda_stream


def gba_create(precision=GBA_FP64, device=0, allocator=None):
    lib = load()
    h = _P()
    a = allocator.alloc if allocator else ALLOC_FN(0)
    f = allocator.free if allocator else FREE_FN(0)
    st = lib.gba_create(int(precision), int(device), a, f, None, ctypes.byref(h))
    if st != GBA_OK:
        raise GbaError(st, "gba_create failed")
    return h


def gba_set_stream(h, stream):
    _check(h, load().gba_set_stream(h, _P(stream)))


def gba_reserve(h, n_cams, n_pts, n_edges):
    _check(h, load().gba_reserve(h, int(n_cams), int(n_pts), int(n_edges)))


def gba_add_cameras(h, ids, params):
    ids = _arr(ids, np.int64)
    params = _arr(params, np.float64, (9,))
    _check(h, load().gba_add_cameras(h, len(ids), _ptr(ids, np.int64), _ptr(params)))


def gba_add_points(h, ids, xyz):
    ids = _arr(ids, np.int64)
    xyz = _arr(xyz, np.float64, (3,))
    _check(h, load().gba_add_points(h, len(ids), _ptr(ids, np.int64), _ptr(xyz)))


def gba_add_edges(h, cam_ids, pt_ids, uv, info=None):
    c = _arr(cam_ids, np.int64)
    p = _arr(pt_ids, np.int64)
    uv = _arr(uv, np.float64, (2,))
    inf = None if info is None else _arr(info, np.float64, (3,))
    _check(h, load().gba_add_edges(h, len(c), _ptr(c, np.int64), _ptr(p, np.int64), _ptr(uv),
                                   _ptr(inf)))


def gba_set_fixed(h, kind, vid, fixed=True):
    _check(h, load().gba_set_fixed(h, int(kind), int(vid), 1 if fixed else 0))


def gba_set_edge_active(h, edge_index, active=True):
    _check(h, load().gba_set_edge_active(h, int(edge_index), 1 if active else 0))


def gba_set_robust_kernel(h, loss, delta=1.0):
    _check(h, load().gba_set_robust_kernel(h, int(loss), float(delta)))


def gba_set_options(h, opts):
    _check(h, load().gba_set_options(h, ctypes.byref(opts)))


def gba_prepare(h):
    _check(h, load().gba_prepare(h))


def gba_solve(h, max_iters, tol=0.0):
    rep = gba_report()
    _check(h, load().gba_solve(h, int(max_iters), float(tol), ctypes.byref(rep)))
    return rep


def gba_reset(h):
    _check(h, load().gba_reset(h))


def gba_get_cost(h):
    c = ctypes.c_double()
    _check(h, load().gba_get_cost(h, ctypes.byref(c)))
    return c.value


def gba_get_cameras(h, n_cams):
    out = np.empty((n_cams, 9))
    _check(h, load().gba_get_cameras(h, _ptr(out)))
    return out


def gba_get_points(h, n_pts):
    out = np.empty((n_pts, 3))
    _check(h, load().gba_get_points(h, _ptr(out)))
    return out


def gba_get_trials(h, max_entries=100000):
    buf = (gba_trial * max_entries)()
    n = ctypes.c_int()
    _check(h, load().gba_get_trials(h, max_entries, buf, ctypes.byref(n)))
    return [dict(cost=t.cost, candidate_cost=t.candidate_cost, lam=t.lambda_,
                 model_decrease=t.model_decrease, step_norm=t.step_norm,
                 accepted=bool(t.accepted), pcg_iters=t.pcg_iters)
            for t in buf[:min(n.value, max_entries)]]


def gba_eval_edges(h, n_edges):
    r = np.empty((n_edges, 2))
    jc = np.empty((n_edges, 2, 9))
    jp = np.empty((n_edges, 2, 3))
    w = np.empty(n_edges)
    _check(h, load().gba_eval_edges(h, _ptr(r), _ptr(jc), _ptr(jp), _ptr(w)))
    return r, jc, jp, w


def gba_eval_edges_noalloc(h, n_edges):
    r = np.empty((n_edges, 2))
    jc = np.empty((n_edges, 2, 9))
    jp = np.empty((n_edges, 2, 3))
    w = np.empty(n_edges)
    _check(h, load().gba_eval_edges_noalloc(h, _ptr(r), _ptr(jc), _ptr(jp), _ptr(w)))
    return r, jc, jp, w


GBA_NOALLOC_MAX_EDGES = 65536


def gba_eval_normal_equations(h, n_cams, n_pts):
    hcc = np.empty((n_cams, 9, 9))
    bc = np.empty((n_cams, 9))
    hpp = np.empty((n_pts, 3, 3))
    bp = np.empty((n_pts, 3))
    _check(h, load().gba_eval_normal_equations(h, _ptr(hcc), _ptr(bc), _ptr(hpp), _ptr(bp)))
    return hcc, bc, hpp, bp


def gba_eval_step(h, lam, n_cams, n_pts):
    dc = np.empty((n_cams, 9))
    dp = np.empty((n_pts, 3))
    it = ctypes.c_int()
    _check(h, load().gba_eval_step(h, float(lam), _ptr(dc), _ptr(dp), ctypes.byref(it)))
    return dc, dp, it.value


def gba_time_matvec(h, lam, launches):
    t = ctypes.c_double()
    _check(h, load().gba_time_matvec(h, float(lam), int(launches), ctypes.byref(t)))
    return t.value


def gba_hbm_probe(device, buf_ptr, nbytes, sink_ptr, launches, stream=None):
    """Streaming read of nbytes at the device address buf_ptr, `launches`
    times; returns the average microseconds per launch (marshalling only)."""
    t = ctypes.c_double()
    st = load().gba_hbm_probe(int(device), ctypes.c_void_p(buf_ptr), ctypes.c_size_t(nbytes),
                              ctypes.c_void_p(sink_ptr), int(launches),
                              ctypes.c_void_p(stream) if stream else None, ctypes.byref(t))
    if st != 0:
        raise GbaError(st, "gba_hbm_probe failed")
    return t.value


def _vi_check(st, what):
    if st != 0:
        raise GbaError(st, what + " failed")


def gba_vi_preintegrate(device, sample_off, gyro, acc, dt, bias0, sigma_g=0.0, sigma_a=0.0):
    """IMU preintegration of len(sample_off) - 1 intervals; returns (n, 148)."""
    off = np.ascontiguousarray(sample_off, np.int64)
    n = len(off) - 1
    g = np.ascontiguousarray(gyro, np.float64)
    a = np.ascontiguousarray(acc, np.float64)
    b = np.ascontiguousarray(bias0, np.float64)
    out = np.empty((max(n, 0), GBA_VI_PRE_STRIDE))
    _vi_check(load().gba_vi_preintegrate(int(device), n, off.ctypes.data, _ptr(g), _ptr(a), float(dt),
                                         _ptr(b), float(sigma_g), float(sigma_a), _ptr(out)),
              "gba_vi_preintegrate")
    return out


def gba_vi_eval_inertial(device, states, pre):
    """Residuals (n_kf - 1, 9) and Jacobians (n_kf - 1, 9, 24)."""
    st = np.ascontiguousarray(states, np.float64)
    pr = np.ascontiguousarray(pre, np.float64)
    n = max(len(st) - 1, 0)
    r = np.empty((n, 9))
    J = np.empty((n, 9, 24))
    _vi_check(load().gba_vi_eval_inertial(int(device), len(st), _ptr(st), _ptr(pr), _ptr(r), _ptr(J)),
              "gba_vi_eval_inertial")
    return r, J


def gba_vi_eval_stereo(device, states, pts, kf, pt, obs, intr):
    """Residuals (n, 3) and Jacobians (n, 3, 9)."""
    st = np.ascontiguousarray(states, np.float64)
    P = np.ascontiguousarray(pts, np.float64)
    k = np.ascontiguousarray(kf, np.int64)
    q = np.ascontiguousarray(pt, np.int64)
    o = np.ascontiguousarray(obs, np.float64)
    it = np.ascontiguousarray(intr, np.float64)
    n = len(k)
    r = np.empty((n, 3))
    J = np.empty((n, 3, 9))
    _vi_check(load().gba_vi_eval_stereo(int(device), len(st), _ptr(st), len(P), _ptr(P), n,
                                        k.ctypes.data, q.ctypes.data, _ptr(o), _ptr(it), _ptr(r),
                                        _ptr(J)), "gba_vi_eval_stereo")
    return r, J


def vi_options(**kw):
    o = gba_vi_options()
    load().gba_vi_default_options(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def gba_vi_solve(device, states, pts, kf, pt, obs, intr, pre, max_iters, tol=0.0,
                 sigma_px=1.0, huber_delta2=0.0, sigma_gw=1e-4, sigma_aw=1e-3, options=None,
                 max_log=1000):
    """Visual-inertial LM solve (marshalling only).  Returns (states (K, 15),
    points (N, 3), report dict, trial log)."""
    st = np.array(states, np.float64, order="C", copy=True)
    P = np.array(pts, np.float64, order="C", copy=True).reshape(-1, 3)
    k = np.ascontiguousarray(kf, np.int64)
    q = np.ascontiguousarray(pt, np.int64)
    o = np.ascontiguousarray(obs, np.float64)
    it = np.ascontiguousarray(intr, np.float64)
    pr = np.ascontiguousarray(pre, np.float64)
    prob = gba_vi_problem(n_kf=len(st), n_pts=len(P), n_obs=len(k), states=st.ctypes.data,
                          pts=P.ctypes.data, kf=k.ctypes.data, pt=q.ctypes.data,
                          obs=o.ctypes.data, intr=it.ctypes.data, pre=pr.ctypes.data,
                          sigma_px=sigma_px, huber_delta2=huber_delta2, sigma_gw=sigma_gw,
                          sigma_aw=sigma_aw)
    rep = gba_report()
    buf = (gba_trial * max(1, max_log))()
    n = ctypes.c_int()
    _vi_check(load().gba_vi_solve(int(device), ctypes.byref(prob), int(max_iters), float(tol),
                                  ctypes.byref(options) if options is not None else None,
                                  ctypes.byref(rep), ctypes.cast(buf, _P), int(max_log),
                                  ctypes.byref(n)), "gba_vi_solve")
    log = [dict(cost=t.cost, candidate_cost=t.candidate_cost, lam=t.lambda_,
                model_decrease=t.model_decrease, step_norm=t.step_norm,
                accepted=bool(t.accepted), pcg_iters=t.pcg_iters) for t in buf[:n.value]]
    return st, P, rep.as_dict(), log


def gba_last_error(h):
    m = load().gba_last_error(h)
    return m.decode() if m else ""


def gba_destroy(h):
    if h:
        load().gba_destroy(h)


# ------------------------------------------------------ convenience wrapper
class Graph:
    """Owns one gba_graph handle; builds it from arrays (marshalling only)."""

    def __init__(self, precision=GBA_FP64, device=0, use_torch=False):
        self.allocator = torch_allocator(device) if use_torch else None
        self.h = gba_create(precision, device, self.allocator)
        if use_torch:
            gba_set_stream(self.h, torch_stream(device))
        self.n_cams = self.n_pts = self.n_edges = 0

    @classmethod
    def from_arrays(cls, cams, pts, cam_idx, pt_idx, obs, info=None, loss=GBA_LOSS_SQUARED,
                    delta=1.0, precision=GBA_FP64, options=None, cam_fixed=None,
                    pt_fixed=None, edge_active=None, device=0, use_torch=False):
        g = cls(precision, device, use_torch)
        cams = np.asarray(cams, np.float64)
        pts = np.asarray(pts, np.float64)
        gba_reserve(g.h, len(cams), len(pts), len(cam_idx))
        gba_add_cameras(g.h, np.arange(len(cams)), cams)
        gba_add_points(g.h, np.arange(len(pts)), pts)
        gba_add_edges(g.h, cam_idx, pt_idx, obs, info)
        g.n_cams, g.n_pts, g.n_edges = len(cams), len(pts), len(cam_idx)
        gba_set_robust_kernel(g.h, loss, delta)
        if options is not None:
            gba_set_options(g.h, options)
        if cam_fixed is not None:
            for i in np.flatnonzero(cam_fixed):
                gba_set_fixed(g.h, 0, int(i), True)
        if pt_fixed is not None:
            for j in np.flatnonzero(pt_fixed):
                gba_set_fixed(g.h, 1, int(j), True)
        if edge_active is not None:
            for e in np.flatnonzero(~np.asarray(edge_active, bool)):
                gba_set_edge_active(g.h, int(e), False)
        return g

    def solve(self, max_iters, tol=0.0):
        return gba_solve(self.h, max_iters, tol)

    def cameras(self):
        return gba_get_cameras(self.h, self.n_cams)

    def points(self):
        return gba_get_points(self.h, self.n_pts)

    def cost(self):
        return gba_get_cost(self.h)

    def trials(self):
        return gba_get_trials(self.h)

    def close(self):
        if self.h:
            gba_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def options(**kw):
    o = gba_default_options()
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


# ------------------------------------------------------------------ serving
def gba_server_default_config():
    c = gba_server_config()
    load().gba_server_default_config(ctypes.byref(c))
    return c


def _check_s(s, status):
    if status != GBA_OK:
        msg = load().gba_server_last_error(s)
        raise GbaError(status, msg.decode() if msg else "")


def gba_server_create(cfg, allocator=None):
    lib = load()
    h = _P()
    a = allocator.alloc if allocator else ALLOC_FN(0)
    f = allocator.free if allocator else FREE_FN(0)
    st = lib.gba_server_create(ctypes.byref(cfg), a, f, None, ctypes.byref(h))
    if st != GBA_OK:
        raise GbaError(st, "gba_server_create failed")
    return h


def gba_server_submit(s, req):
    """req: dict with cams [nc,9], pts [np,3], cam_idx, pt_idx, uv [ne,2] and
    optional info [ne,3], cam_fixed, pt_fixed, max_iters, tol."""
    keep = {
        "cams": _arr(req["cams"], np.float64, (9,)),
        "pts": _arr(req["pts"], np.float64, (3,)),
        "cam_idx": _arr(req["cam_idx"], np.int32),
        "pt_idx": _arr(req["pt_idx"], np.int32),
        "uv": _arr(req["uv"], np.float64, (2,)),
    }
    if req.get("info") is not None:
        keep["info"] = _arr(req["info"], np.float64, (3,))
    for k in ("cam_fixed", "pt_fixed"):
        if req.get(k) is not None:
            keep[k] = _arr(np.asarray(req[k]).astype(bool), np.uint8)
    p = gba_problem()
    p.n_cams, p.n_pts, p.n_edges = len(keep["cams"]), len(keep["pts"]), len(keep["cam_idx"])
    for k, v in keep.items():
        setattr(p, k, v.ctypes.data)
    p.max_iters = int(req.get("max_iters", 10))
    p.tol = float(req.get("tol", 0.0))
    t = ctypes.c_uint64()
    _check_s(s, load().gba_server_submit(s, ctypes.byref(p), ctypes.byref(t)))
    return t.value


def gba_server_poll(s, ticket, n_cams, n_pts, wait=True):
    """Returns None while pending (wait=False), else a dict with the result."""
    cams = np.empty((n_cams, 9))
    pts = np.empty((n_pts, 3))
    r = gba_result()
    r.cams = cams.ctypes.data
    r.pts = pts.ctypes.data
    st = load().gba_server_poll(s, ctypes.c_uint64(ticket), 1 if wait else 0, ctypes.byref(r))
    if st == GBA_PENDING:
        return None
    _check_s(s, st)
    return {"cams": cams, "pts": pts, "report": r.report.as_dict(), "latency_ms": r.latency_ms,
            "queue_ms": r.queue_ms, "batch_peak": r.batch_peak}


def gba_server_stats(s):
    st = gba_serving_stats()
    _check_s(s, load().gba_server_stats(s, ctypes.byref(st)))
    return st.as_dict()


def gba_server_last_error(s):
    m = load().gba_server_last_error(s)
    return m.decode() if m else ""


def gba_server_destroy(s):
    if s:
        load().gba_server_destroy(s)


class Server:
    """Owns one gba_server handle (marshalling only)."""

    def __init__(self, precision=GBA_MIXED_FP32, budget_bytes=4 << 30, max_slots=64,
                 loss=GBA_LOSS_HUBER, delta=1.0, tune_db=None, device=0, **overrides):
        cfg = gba_server_default_config()
        cfg.precision = precision
        cfg.device = device
        cfg.hbm_budget_bytes = int(budget_bytes)
        cfg.max_slots = int(max_slots)
        cfg.loss = loss
        cfg.delta = float(delta)
        self._db = tune_db.encode() if tune_db else None
        cfg.tune_db = self._db
        for k, v in overrides.items():
            if hasattr(cfg.options, k):
                setattr(cfg.options, k, v)
            elif hasattr(cfg, k):
                setattr(cfg, k, v)
            else:
                raise KeyError(k)
        self.h = gba_server_create(cfg)
        self.sizes = {}

    def submit(self, req):
        t = gba_server_submit(self.h, req)
        self.sizes[t] = (len(req["cams"]), len(req["pts"]))
        return t

    def poll(self, ticket, wait=True):
        nc, np_ = self.sizes[ticket]
        r = gba_server_poll(self.h, ticket, nc, np_, wait)
        if r is not None:
            del self.sizes[ticket]
        return r

    def stats(self):
        return gba_server_stats(self.h)

    def close(self):
        if self.h:
            gba_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
