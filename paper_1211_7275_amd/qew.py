"""ctypes binding of libqew (declared in include/qew.h): argument marshalling only.

Every step of the path runs in the HIP library.  PyTorch supplies the device
memory (the workspace is a uint8 tensor) and the stream.  Importing this
module loads ``lib/libqew.so`` after torch (so both share one HIP runtime) and
raises ImportError if the library was not built.
"""
import ctypes
import os

import numpy as np
import torch  # noqa: F401  (loads the HIP runtime the library binds to)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libqew.so")

QEW_OK = 0
QEW_EINVAL = -1
QEW_ENOMEM = -2
QEW_EDEVICE = -3
QEW_EUNSUPPORTED = -4

QEW_RF_CR_UNIFORM = 0
QEW_RB_CR_GAUSS = 1
QEW_RB_LIN_GAUSS = 2
QEW_RF_PC_GAUSS = 3
QEW_FP64_PLAIN = 0
QEW_FP32_SPLIT = 1
QEW_ONE_STEP = 0
QEW_FUSED = 1
QEW_FLAG_NO_GRAPH = 1
QEW_FLAG_TIMING = 2
QEW_FLAG_FUSED_DENSE = 4
QEW_FLAG_FUSED_SPARSE = 8

EXPORTS = ("qew_plan", "qew_workspace_bytes", "qew_plan_info_get", "qew_autotune", "qew_run",
           "qew_run_noalloc", "qew_ensemble", "qew_sq_get", "qew_run_stats_get", "qew_read_state", "qew_write_state",
           "qew_debug_philox_fill", "qew_debug_force_eval", "qew_critical_force", "qew_plan_destroy",
           "qew_last_error")

ENSEMBLE_ROWS = ("v", "v_se", "w2", "w2_se", "ubar", "ubar_se", "w2_about_ensemble_ubar")


class qew_problem(ctypes.Structure):
    _fields_ = [
        ("n_samples", ctypes.c_int32), ("kind", ctypes.c_int32),
        ("L", ctypes.POINTER(ctypes.c_int64)), ("f", ctypes.POINTER(ctypes.c_double)),
        ("disorder_id", ctypes.POINTER(ctypes.c_uint32)),
        ("c", ctypes.c_double), ("dt", ctypes.c_double), ("strength", ctypes.c_double),
        ("seed", ctypes.c_uint64), ("n_steps", ctypes.c_int64),
        ("meas_steps", ctypes.POINTER(ctypes.c_int64)), ("n_meas", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("path", ctypes.c_int32), ("k", ctypes.c_int32),
        ("tile", ctypes.c_int32), ("flags", ctypes.c_int32), ("period", ctypes.c_int32),
        ("sq_bins", ctypes.c_int32), ("sq_edges", ctypes.POINTER(ctypes.c_int64)),
    ]


class qew_plan_info(ctypes.Structure):
    _fields_ = [
        ("total_sites", ctypes.c_int64), ("padded_sites", ctypes.c_int64),
        ("n_tiles", ctypes.c_int32), ("n_meas_tiles", ctypes.c_int32), ("k", ctypes.c_int32),
        ("tile", ctypes.c_int32), ("autotuned", ctypes.c_int32), ("pad_", ctypes.c_int32),
        ("cur_step", ctypes.c_int64),
    ]


class qew_run_stats(ctypes.Structure):
    _fields_ = [
        ("total_ms", ctypes.c_double), ("step_ms", ctypes.c_double), ("meas_ms", ctypes.c_double),
        ("step_launches", ctypes.c_int64), ("meas_launches", ctypes.c_int64),
        ("site_updates", ctypes.c_int64), ("graph_launches", ctypes.c_int64),
        ("sparse_launches", ctypes.c_int64), ("fused_ms", ctypes.c_double),
        ("fused_launches", ctypes.c_int64), ("fused_steps", ctypes.c_int64),
        ("node_refreshes", ctypes.c_int64),
    ]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libqew.so is not built ({LIB_PATH}); run __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH, mode=ctypes.RTLD_GLOBAL)
    vp, sz, st = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32
    dp = ctypes.POINTER(ctypes.c_double)
    lib.qew_plan.argtypes = [ctypes.POINTER(qew_problem), ctypes.POINTER(vp)]
    lib.qew_plan.restype = st
    lib.qew_workspace_bytes.argtypes = [vp]
    lib.qew_workspace_bytes.restype = sz
    lib.qew_plan_info_get.argtypes = [vp, ctypes.POINTER(qew_plan_info)]
    lib.qew_plan_info_get.restype = st
    lib.qew_autotune.argtypes = [vp, vp, sz, vp]
    lib.qew_autotune.restype = st
    lib.qew_run.argtypes = [vp, vp, sz, vp, ctypes.c_int32, dp, dp, dp]
    lib.qew_run.restype = st
    lib.qew_run_noalloc.argtypes = [vp, vp, sz, vp, ctypes.c_int32, dp, dp, dp]
    lib.qew_run_noalloc.restype = st
    lib.qew_ensemble.argtypes = [vp, vp, vp, dp]
    lib.qew_ensemble.restype = st
    lib.qew_sq_get.argtypes = [vp, vp, vp, dp]
    lib.qew_sq_get.restype = st
    lib.qew_run_stats_get.argtypes = [vp, ctypes.POINTER(qew_run_stats)]
    lib.qew_run_stats_get.restype = st
    lib.qew_read_state.argtypes = [vp, vp, vp, ctypes.c_int32, dp, ctypes.POINTER(ctypes.c_int64)]
    lib.qew_read_state.restype = st
    lib.qew_write_state.argtypes = [vp, vp, vp, ctypes.c_int32, dp, ctypes.c_int64]
    lib.qew_write_state.restype = st
    lib.qew_debug_philox_fill.argtypes = [vp, ctypes.c_uint64, vp, ctypes.c_int64, vp]
    lib.qew_debug_philox_fill.restype = st
    lib.qew_debug_force_eval.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_uint64,
                                         ctypes.c_int32, ctypes.c_int32, vp, vp, vp, vp, vp,
                                         ctypes.c_int64, vp]
    lib.qew_debug_force_eval.restype = st
    lib.qew_critical_force.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_uint64, ctypes.c_int32,
                                       ctypes.c_double, ctypes.c_int32, ctypes.c_int32, vp, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int64,
                                       vp, vp, vp, vp]
    lib.qew_critical_force.restype = st
    lib.qew_plan_destroy.argtypes = [vp]
    lib.qew_plan_destroy.restype = None
    lib.qew_last_error.argtypes = []
    lib.qew_last_error.restype = ctypes.c_char_p
    return lib


_lib = _load()


class QewError(RuntimeError):
    def __init__(self, status, where):
        msg = _lib.qew_last_error().decode(errors="replace")
        super().__init__(f"{where} failed with status {status}: {msg}")
        self.status = status


def _check(status, where):
    if status != QEW_OK:
        raise QewError(status, where)


def lib():
    return _lib


# ------------------------------------------------------------ raw calls ---

def qew_last_error():
    return _lib.qew_last_error().decode(errors="replace")


def qew_plan(problem):
    """problem: qew_problem (ctypes) or a workloads dict; returns (plan handle, keepalive)."""
    h = ctypes.c_void_p()
    _check(_lib.qew_plan(ctypes.byref(problem), ctypes.byref(h)), "qew_plan")
    return h


def qew_workspace_bytes(plan):
    return int(_lib.qew_workspace_bytes(plan))


def qew_plan_info_get(plan):
    info = qew_plan_info()
    _check(_lib.qew_plan_info_get(plan, ctypes.byref(info)), "qew_plan_info_get")
    return info


def qew_autotune(plan, ws, stream=None):
    _check(_lib.qew_autotune(plan, ws.data_ptr(), ws.numel(), _stream_ptr(stream)), "qew_autotune")


def qew_run(plan, ws, stream, resume, h_v, h_w2, h_ubar):
    _check(_lib.qew_run(plan, ws.data_ptr(), ws.numel(), _stream_ptr(stream), int(resume),
                        _dptr(h_v), _dptr(h_w2), _dptr(h_ubar)), "qew_run")


def qew_run_noalloc(plan, ws, stream, resume, h_v, h_w2, h_ubar):
    _check(_lib.qew_run_noalloc(plan, ws.data_ptr(), ws.numel(), _stream_ptr(stream), int(resume),
                                _dptr(h_v), _dptr(h_w2), _dptr(h_ubar)), "qew_run_noalloc")


def qew_ensemble(plan, ws, n_meas, stream=None):
    """Disorder averages on the device: dict of ENSEMBLE_ROWS -> [n_meas] arrays."""
    out = np.zeros((7, int(n_meas)), np.float64)
    _check(_lib.qew_ensemble(plan, ws.data_ptr(), _stream_ptr(stream), _dptr(out)), "qew_ensemble")
    return dict(zip(ENSEMBLE_ROWS, out))


def qew_sq_get(plan, ws, n_meas, n_bins, stream=None):
    """Disorder-averaged binned structure factor [n_meas][n_bins] (Eq. (6))."""
    out = np.zeros((int(n_meas), int(n_bins)), np.float64)
    _check(_lib.qew_sq_get(plan, ws.data_ptr(), _stream_ptr(stream), _dptr(out)), "qew_sq_get")
    return out


def qew_run_stats_get(plan):
    s = qew_run_stats()
    _check(_lib.qew_run_stats_get(plan, ctypes.byref(s)), "qew_run_stats_get")
    return s


def qew_read_state(plan, ws, sample, L, stream=None):
    u = np.zeros(int(L), np.float64)
    step = ctypes.c_int64()
    _check(_lib.qew_read_state(plan, ws.data_ptr(), _stream_ptr(stream), int(sample), _dptr(u),
                               ctypes.byref(step)), "qew_read_state")
    return u, int(step.value)


def qew_write_state(plan, ws, sample, u, step, stream=None):
    u = np.ascontiguousarray(u, np.float64)
    _check(_lib.qew_write_state(plan, ws.data_ptr(), _stream_ptr(stream), int(sample), _dptr(u),
                                int(step)), "qew_write_state")


def qew_debug_philox_fill(d_ctr, seed, d_out, stream=None):
    n = d_ctr.numel() // 4
    _check(_lib.qew_debug_philox_fill(d_ctr.data_ptr(), int(seed) & 0xFFFFFFFFFFFFFFFF,
                                      d_out.data_ptr(), n, _stream_ptr(stream)),
           "qew_debug_philox_fill")


def qew_debug_force_eval(kind, strength, seed, precision, d_did, d_j, d_cell, d_frac, d_out,
                         stream=None, period=0):
    _check(_lib.qew_debug_force_eval(int(kind), float(strength), int(seed), int(period), int(precision),
                                     d_did.data_ptr(), d_j.data_ptr(), d_cell.data_ptr(),
                                     d_frac.data_ptr(), d_out.data_ptr(), d_out.numel(),
                                     _stream_ptr(stream)), "qew_debug_force_eval")


def qew_critical_force(kind, strength, seed, period, c, d_did, f_lo, f_hi, tol_f, tol_force, max_sweeps,
                       d_u, d_f, d_status, stream=None):
    """d_did: [S] uint32, d_u: [S, L] float64 (start in, pinned configuration out),
    d_f: [S, 2] float64 out, d_status: [S, 2] int64 out (device tensors)."""
    S, L = d_u.shape
    _check(_lib.qew_critical_force(int(kind), float(strength), int(seed) & 0xFFFFFFFFFFFFFFFF, int(period),
                                   float(c), int(S), int(L), d_did.data_ptr(), float(f_lo), float(f_hi),
                                   float(tol_f), float(tol_force), int(max_sweeps), d_u.data_ptr(),
                                   d_f.data_ptr(), d_status.data_ptr(), _stream_ptr(stream)),
           "qew_critical_force")


def qew_plan_destroy(plan):
    _lib.qew_plan_destroy(plan)


def _dptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _stream_ptr(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# ------------------------------------------------------ convenience API ---

def make_problem(p, precision=QEW_FP32_SPLIT, path=QEW_FUSED, k=0, tile=0, flags=0):
    """qew_problem from a workloads dict; returns (struct, keepalive arrays)."""
    L = np.ascontiguousarray(p["L"], np.int64)
    f = np.ascontiguousarray(p["f"], np.float64)
    did = np.ascontiguousarray(p["disorder_id"], np.uint32)
    meas = np.ascontiguousarray(p["meas_steps"], np.int64)
    edges = p.get("sq_edges")
    edges = None if edges is None else np.ascontiguousarray(edges, np.int64)
    keep = (L, f, did, meas, edges)
    pr = qew_problem(
        n_samples=L.size, kind=int(p["kind"]),
        L=L.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
        f=f.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
        disorder_id=did.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
        c=float(p["c"]), dt=float(p["dt"]), strength=float(p["strength"]),
        seed=int(p["seed"]) & 0xFFFFFFFFFFFFFFFF, n_steps=int(p["n_steps"]),
        meas_steps=meas.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)) if meas.size else None,
        n_meas=meas.size, precision=int(precision), path=int(path), k=int(k), tile=int(tile),
        flags=int(flags), period=int(p.get("period", 0)),
        sq_bins=0 if edges is None else edges.size - 1,
        sq_edges=None if edges is None else edges.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    return pr, keep


class Simulation:
    """A plan plus its device workspace (a torch uint8 tensor on `device`)."""

    def __init__(self, problem, precision=QEW_FP32_SPLIT, path=QEW_FUSED, k=0, tile=0, flags=0,
                 device="cuda"):
        self.problem = problem
        self._pr, self._keep = make_problem(problem, precision, path, k, tile, flags)
        self.plan = qew_plan(self._pr)
        nbytes = qew_workspace_bytes(self.plan)
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        off = (-self.ws.data_ptr()) % 256
        self.ws = self.ws[off: off + nbytes]
        self.S = len(problem["L"])
        self.n_meas = len(problem["meas_steps"])
        edges = problem.get("sq_edges")
        self.sq_bins = 0 if edges is None else len(edges) - 1

    def close(self):
        if self.plan:
            qew_plan_destroy(self.plan)
            self.plan = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        return qew_plan_info_get(self.plan)

    def autotune(self, stream=None):
        qew_autotune(self.plan, self.ws, stream)

    def run(self, resume=False, stream=None):
        """Run to n_steps; returns per-sample series dict v, w2, ubar [S][n_meas]."""
        if stream is None:
            stream = torch.cuda.current_stream()
        v = np.full((self.S, self.n_meas), np.nan)
        w2 = np.full_like(v, np.nan)
        ub = np.full_like(v, np.nan)
        qew_run(self.plan, self.ws, stream, resume, v, w2, ub)
        return {"v": v, "w2": w2, "ubar": ub}

    def ensemble(self, stream=None):
        """Disorder average and standard errors of the series (computed on the device)."""
        return qew_ensemble(self.plan, self.ws, self.n_meas, stream)

    def structure_factor(self, stream=None):
        """Binned S_q averaged over samples at every measurement: [n_meas][sq_bins]."""
        return qew_sq_get(self.plan, self.ws, self.n_meas, self.sq_bins, stream)

    def stats(self):
        return qew_run_stats_get(self.plan)

    def read_state(self, s):
        return qew_read_state(self.plan, self.ws, s, self.problem["L"][s])

    def write_state(self, s, u, step):
        qew_write_state(self.plan, self.ws, s, u, step)
