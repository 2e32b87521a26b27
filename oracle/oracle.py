"""ctypes binding of the FP64 CPU oracle (``qew_oracle.c``).

TEST INFRASTRUCTURE ONLY: used by ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py``; the GPU library never imports it.

Every function follows the paper (arXiv:1211.7275): Eq. (1) integrated by the
explicit Euler method on a periodic chain (Sec. III B), pinning force from
random values at integer u with a cubic spline (Sec. III B; RB force is minus
the derivative of the potential, Sec. II), observables of Eqs. (3)-(5).
"""
import ctypes
import os

import numpy as np

from . import build as _build

RF = 0        # random field, uniform force values, Catmull-Rom
RB = 1        # random bond, Gaussian potential, Catmull-Rom
RB_LIN = 2    # random bond, Gaussian potential, linear spline (Case 3)
RF_PC = 3     # random field, Gaussian forces, no interpolation (Case 4)

_lib = None


def lib():
    """Load ``liboracle.so``, building it first if it is absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_build.LIB):
        _build.build()
    L = ctypes.CDLL(_build.LIB)
    u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
    f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
    i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
    c_int, c_i64, c_u64, c_u32, c_d = (ctypes.c_int, ctypes.c_int64, ctypes.c_uint64,
                                       ctypes.c_uint32, ctypes.c_double)
    L.qo_philox4x32_10.argtypes = [u32p, u32p, u32p]
    L.qo_philox_many.argtypes = [u32p, c_u64, u32p, c_i64]
    L.qo_node.argtypes = [c_int, c_u64, c_u32, c_i64, c_i64, c_i64]
    L.qo_node.restype = c_d
    L.qo_cr_value.argtypes = [f64p, c_d]
    L.qo_cr_value.restype = c_d
    L.qo_cr_slope.argtypes = [f64p, c_d]
    L.qo_cr_slope.restype = c_d
    L.qo_pinning.argtypes = [c_int, c_d, c_u64, c_u32, c_i64, c_d, c_i64]
    L.qo_pinning.restype = c_d
    L.qo_potential.argtypes = [c_int, c_d, c_u64, c_u32, c_i64, c_d, c_i64]
    L.qo_potential.restype = c_d
    L.qo_forces.argtypes = [c_int, c_d, c_u64, c_u32, c_i64, c_i64, c_d, c_d, f64p, f64p]
    L.qo_measure.argtypes = [c_i64, f64p, f64p, ctypes.POINTER(c_d), ctypes.POINTER(c_d),
                             ctypes.POINTER(c_d)]
    L.qo_euler.argtypes = [c_i64, c_d, f64p, f64p, f64p]
    L.qo_run.argtypes = [c_int, c_d, c_u64, c_u32, c_i64, c_i64, c_d, c_d, c_d, c_i64, c_i64,
                         i64p, ctypes.c_int32, f64p, f64p, f64p, f64p]
    L.qo_run.restype = c_int
    L.qo_run_window.argtypes = [c_int, c_d, c_u64, c_u32, c_i64, c_i64, c_i64, c_i64, c_d, c_d,
                                c_d, c_i64, f64p]
    L.qo_run_window.restype = c_int
    L.qo_relax.argtypes = [c_int, c_d, c_u64, c_u32, c_i64, c_i64, c_d, c_d, c_d, f64p, f64p,
                           c_i64, c_d, ctypes.POINTER(c_i64)]
    L.qo_relax.restype = c_int
    L.qo_mean_node.argtypes = [c_int, c_u64, c_u32, c_i64, c_i64]
    L.qo_mean_node.restype = c_d
    L.qo_set_threads.argtypes = [c_int]
    L.qo_get_threads.restype = c_int
    _lib = L
    return L


def set_threads(n):
    lib().qo_set_threads(int(n))


def get_threads():
    return int(lib().qo_get_threads())


def philox(ctr, key):
    """Philox4x32-10 of one counter (4 words) under one key (2 words)."""
    out = np.zeros(4, np.uint32)
    lib().qo_philox4x32_10(np.ascontiguousarray(ctr, np.uint32),
                           np.ascontiguousarray(key, np.uint32), out)
    return out


def philox_many(ctr, seed):
    ctr = np.ascontiguousarray(ctr, np.uint32).reshape(-1, 4)
    out = np.zeros_like(ctr)
    lib().qo_philox_many(ctr, int(seed), out, ctr.shape[0])
    return out


def node(kind, seed, did, j, n, period=0):
    """Unscaled disorder value at integer u = n of column j."""
    return lib().qo_node(int(kind), int(seed), int(did), int(j), int(n), int(period))


def cr_value(p, s):
    return lib().qo_cr_value(np.ascontiguousarray(p, np.float64), float(s))


def cr_slope(p, s):
    return lib().qo_cr_slope(np.ascontiguousarray(p, np.float64), float(s))


def pinning(kind, strength, seed, did, j, u, period=0):
    return lib().qo_pinning(int(kind), float(strength), int(seed), int(did), int(j), float(u),
                            int(period))


def potential(strength, seed, did, j, u, kind=RB, period=0):
    return lib().qo_potential(int(kind), float(strength), int(seed), int(did), int(j), float(u),
                              int(period))


def forces(kind, strength, seed, did, c, f, u, period=0):
    u = np.ascontiguousarray(u, np.float64)
    F = np.zeros_like(u)
    lib().qo_forces(int(kind), float(strength), int(seed), int(did), int(period), u.size,
                    float(c), float(f), u, F)
    return F


def measure(u, F):
    u = np.ascontiguousarray(u, np.float64)
    F = np.ascontiguousarray(F, np.float64)
    v, ub, w2 = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    lib().qo_measure(u.size, u, F, ctypes.byref(v), ctypes.byref(ub), ctypes.byref(w2))
    return v.value, ub.value, w2.value


def euler(dt, u, F):
    u = np.ascontiguousarray(u, np.float64)
    F = np.ascontiguousarray(F, np.float64)
    out = np.zeros_like(u)
    lib().qo_euler(u.size, float(dt), u, F, out)
    return out


def run_sample(kind, strength, seed, did, L, c, dt, f, n_steps, meas_steps,
               u0=None, step0=0, period=0):
    """Evolve one sample; returns dict(v, ubar, w2, u) (u = state at n_steps)."""
    meas = np.ascontiguousarray(meas_steps, np.int64)
    u = np.zeros(int(L), np.float64) if u0 is None else np.array(u0, np.float64, copy=True)
    v = np.full(meas.size, np.nan)
    ub = np.full(meas.size, np.nan)
    w2 = np.full(meas.size, np.nan)
    rc = lib().qo_run(int(kind), float(strength), int(seed), int(did), int(period), int(L),
                      float(c), float(dt), float(f), int(step0), int(n_steps), meas,
                      int(meas.size), u, v, ub, w2)
    if rc != 0:
        raise ValueError("oracle qo_run rejected its input")
    return {"v": v, "ubar": ub, "w2": w2, "u": u}


def site_after(kind, strength, seed, did, L, j, c, dt, f, n_steps, period=0):
    """u_j after n_steps from the flat start on the periodic chain of length L,
    computed on the light-cone window of sites j - n_steps - 1 .. j + n_steps + 1."""
    half = int(n_steps) + 1
    W = 2 * half + 1
    if W >= L:
        r = run_sample(kind, strength, seed, did, L, c, dt, f, n_steps, [], period=period)
        return r["u"][int(j)]
    u = np.zeros(W, np.float64)
    rc = lib().qo_run_window(int(kind), float(strength), int(seed), int(did), int(period),
                             int(L), int(j) - half, W, float(c), float(dt), float(f),
                             int(n_steps), u)
    if rc != 0:
        raise ValueError("oracle qo_run_window rejected its input")
    return u[half]


def mean_node(kind, seed, did, L, n):
    return lib().qo_mean_node(int(kind), int(seed), int(did), int(L), int(n))


def run(problem, u0=None, step0=0):
    """Run every sample of a problem dict (see paper_1211_7275_amd.workloads).

    Returns per-sample series [S][n_meas] for v, ubar, w2 and the final states
    (list of arrays).  Ensemble averages give each sample equal weight.
    """
    S = len(problem["L"])
    meas = np.asarray(problem["meas_steps"], np.int64)
    out = {k: np.zeros((S, meas.size)) for k in ("v", "ubar", "w2")}
    states = []
    for s in range(S):
        r = run_sample(problem["kind"], problem["strength"], problem["seed"],
                       problem["disorder_id"][s], problem["L"][s], problem["c"],
                       problem["dt"], problem["f"][s], problem["n_steps"], meas,
                       None if u0 is None else u0[s], step0, problem.get("period", 0))
        for k in ("v", "ubar", "w2"):
            out[k][s] = r[k]
        states.append(r["u"])
    out["u"] = states
    return out


# --------------------------------------------------------------------------
# Structure factor, Eq. (6): S_q(t) = overbar |L^-1 sum_x u(x,t) e^{-iqx}|^2,
# q = 2 pi n / L.  numpy's FFT is the library step; for real u the modes n and
# L - n are equal, so n = 1 .. L/2 is returned.
# --------------------------------------------------------------------------

def structure_factor(u):
    """S_n of one chain for n = 1 .. L//2 (index n - 1)."""
    u = np.asarray(u, np.float64)
    L = u.size
    U = np.fft.rfft(u)
    return (np.abs(U[1:L // 2 + 1]) / L) ** 2


def sq_binned(S, edges):
    """Mean of S_n over the modes n in [edges[b], edges[b+1]) for each bin b."""
    edges = np.asarray(edges, np.int64)
    return np.array([S[edges[b] - 1:edges[b + 1] - 1].mean() for b in range(edges.size - 1)])


def states_at(problem, s, steps):
    """States of sample s at the given increasing steps (flat start), by
    running the chain segment by segment (the disorder does not depend on
    time, so a continued run equals an uninterrupted one)."""
    u = np.zeros(int(problem["L"][s]), np.float64)
    out, now = [], 0
    for m in steps:
        if m > now:
            u = run_sample(problem["kind"], problem["strength"], problem["seed"],
                           problem["disorder_id"][s], problem["L"][s], problem["c"],
                           problem["dt"], problem["f"][s], int(m), [], u0=u,
                           step0=now, period=problem.get("period", 0))["u"]
            now = int(m)
        out.append(u.copy())
    return out


def sq_series(problem, edges):
    """Disorder-averaged binned S_q at every measurement step: [n_meas][n_bins]."""
    meas = np.asarray(problem["meas_steps"], np.int64)
    S = len(problem["L"])
    acc = np.zeros((meas.size, len(edges) - 1))
    for s in range(S):
        for i, u in enumerate(states_at(problem, s, meas)):
            acc[i] += sq_binned(structure_factor(u), edges)
    return acc / S


# --------------------------------------------------------------------------
# Critical force and configuration of a sample periodic in u (Sec. III A): the
# pinned solution of c d2u/dx2 + F_p + f = 0 with the largest f, by bisection
# on f.  Each trial relaxes from the last pinned configuration found (below
# the critical one, where the line moves forward only), and the trial decides
# pinned (all forces below tol) or depinned (the line advanced by a full
# period M, impossible while a pinned configuration exists).
# --------------------------------------------------------------------------

PINNED, DEPINNED, UNDECIDED = 0, 1, 2


def relax(kind, strength, seed, did, M, c, dt, f, u, u_ref, max_steps, tol):
    """One relaxation (see qo_relax); returns (status, steps) and updates u in place."""
    steps = ctypes.c_int64()
    rc = lib().qo_relax(int(kind), float(strength), int(seed), int(did), int(M), u.size,
                        float(c), float(dt), float(f), u, np.ascontiguousarray(u_ref, np.float64),
                        int(max_steps), float(tol), ctypes.byref(steps))
    if rc < 0:
        raise ValueError("oracle qo_relax rejected its input")
    return rc, int(steps.value)


def critical_force(kind, strength, seed, did, L, M, c=1.0, dt=0.05, f_lo=0.0, f_hi=5.0,
                   tol_f=1e-6, tol_force=1e-10, max_steps=10_000_000):
    """Bisection for f_c^s of one sample.  Returns dict(f_lo, f_hi, u_c, trials)
    with f_c^s in [f_lo, f_hi), f_hi - f_lo < tol_f, u_c the pinned
    configuration at f_lo and trials the (f, status, steps) of every relaxation."""
    u = np.zeros(int(L), np.float64)
    trials = []
    st, n = relax(kind, strength, seed, did, M, c, dt, f_lo, u, np.full(u.size, np.inf), max_steps,
                  tol_force)
    trials.append((f_lo, st, n))
    if st != PINNED:
        raise ValueError("no pinned configuration at the lower drive")
    while f_hi - f_lo >= tol_f:
        f_mid = 0.5 * (f_lo + f_hi)
        v = u.copy()
        st, n = relax(kind, strength, seed, did, M, c, dt, f_mid, v, u, max_steps, tol_force)
        trials.append((f_mid, st, n))
        if st == PINNED:
            f_lo, u = f_mid, v
        elif st == DEPINNED:
            f_hi = f_mid
        else:
            raise ValueError("relaxation undecided within max_steps")
    return {"f_lo": f_lo, "f_hi": f_hi, "u_c": u, "trials": trials}
