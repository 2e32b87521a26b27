"""Seeded synthetic workloads (inputs only: no arithmetic of the method).

The paper's disorder is synthetic by construction (random values generated at
the integer points of u and x, Sec. III B), so a workload is fully given by
its sizes, drives, disorder kind and strength, seed and measurement times.
Both the GPU library and the CPU oracle consume the dicts built here; this
module holds none of the method's arithmetic (no generator of the disorder,
no spline, no integrator).

Problem dict keys: kind (0 = RF Catmull-Rom uniform, 1 = RB Catmull-Rom
Gaussian, 2 = RB linear-spline Gaussian, 3 = RF Gaussian without
interpolation), strength, seed, c, dt, n_steps, L [S], f [S], disorder_id [S],
meas_steps [n_meas], and optionally period (transverse period M, 0 = none)
and sq_edges (mode bins of the structure factor, see sq_edges_full / sq_edges_log).
"""
import numpy as np

RF = 0        # random field, uniform force values, Catmull-Rom
RB = 1        # random bond, Gaussian potential, Catmull-Rom
RB_LIN = 2    # random bond, Gaussian potential, linear spline (Case 3)
RF_PC = 3     # random field, Gaussian forces, no interpolation (Case 4)

SEED_BASE = 0x51EDC0DE00


def log_steps(n_steps, n_points):
    """n_points distinct measurement steps in [1, n_steps], log-spaced.

    n_0 = 1, n_i = max(n_{i-1} + 1, round(n_steps ** (i / (n_points - 1)))),
    so the last one is n_steps.
    """
    n_steps = int(n_steps)
    n_points = int(n_points)
    if n_points < 1 or n_steps < 1:
        return np.zeros(0, np.int64)
    if n_points == 1:
        return np.array([n_steps], np.int64)
    if n_points > n_steps:
        raise ValueError("more measurement points than steps")
    out = []
    prev = 0
    for i in range(n_points):
        target = int(round(n_steps ** (i / (n_points - 1))))
        cur = max(prev + 1, target)
        out.append(cur)
        prev = cur
    out = np.array(out, np.int64)
    if out[-1] != n_steps:
        raise ValueError("log spacing overshoots the horizon; use fewer points")
    return out


def _problem(kind, L, f, did, n_steps, n_meas, seed, c=1.0, dt=0.05, strength=1.0):
    L = np.asarray(L, np.int64)
    return {
        "kind": int(kind), "strength": float(strength), "seed": int(seed),
        "c": float(c), "dt": float(dt), "n_steps": int(n_steps),
        "L": L, "f": np.asarray(f, np.float64),
        "disorder_id": np.asarray(did, np.uint32),
        "meas_steps": log_steps(n_steps, n_meas),
    }


def config0(n_steps=10_000, n_meas=50, samples=4, L=1024):
    """Small plain case: L=1024, 4 RF samples, 10^4 steps, 50 log-spaced points."""
    S = samples
    return _problem(RF, [L] * S, [1.0] * S, np.arange(S), n_steps, n_meas, SEED_BASE + 0)


def config1(n_steps=100_000, n_meas=100, disorders=64, L=1 << 16, drives=(0.8, 1.0, 1.2)):
    """RB Gaussian, L=2^16, 64 disorders x drives {0.8,1.0,1.2} sharing disorder ids."""
    did = np.tile(np.arange(disorders), len(drives))
    f = np.repeat(np.asarray(drives, np.float64), disorders)
    return _problem(RB, [L] * did.size, f, did, n_steps, n_meas, SEED_BASE + 1)


def config2_sizes(samples=512, seed=SEED_BASE + 2):
    """Per-sample chain lengths L_s = 2^e, e uniform in {10..16}, drawn by numpy's
    PCG64 from the config seed (an input draw, not part of the method)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return (1 << rng.integers(10, 17, size=samples)).astype(np.int64)


def config2(n_steps=20_000, n_meas=100, samples=512):
    """Batched uneven sizes: 512 RF samples, L_s in {2^10..2^16}, f=1.0."""
    L = config2_sizes(samples)
    return _problem(RF, L, [1.0] * samples, np.arange(samples), n_steps, n_meas, SEED_BASE + 2)


def config3(n_steps=1_000_000, n_meas=200, samples=4, L=1 << 22):
    """Large chain: L=2^22, 4 RF samples, f=1.0, 10^6 steps, 200 log-spaced points."""
    return _problem(RF, [L] * samples, [1.0] * samples, np.arange(samples), n_steps, n_meas,
                    SEED_BASE + 3)


# Largest drive whose velocity still dies in the f-scan at L = 2^16 (4 disorders,
# 10^5 steps, drives 0.02 apart, `python -m paper_1211_7275_amd.std`): the
# threshold of the unit-strength disorder lies between this drive and the next.
C4_FCENTER = {RF: 0.363, RB: 1.937}


def config4(kind, f_center=None, n_steps=1_000_000, n_meas=200, L=1 << 25, spacing=0.02):
    """Paper scale: L=2^25, one disorder, 5 drives spaced 0.02 around f_center
    (default: the f-scan's last dying drive for this kind)."""
    if f_center is None:
        f_center = C4_FCENTER[kind]
    f = f_center + spacing * np.arange(-2, 3)
    return _problem(kind, [L] * 5, f, np.zeros(5, np.uint32), n_steps, n_meas,
                    SEED_BASE + 4 + int(kind))


def sq_edges_full(L):
    """One structure-factor bin per mode n = 1 .. L/2."""
    return np.arange(1, int(L) // 2 + 2, dtype=np.int64)


def sq_edges_log(L, n_bins):
    """At most n_bins bins of the modes 1 .. L/2, log-spaced, distinct integer edges."""
    top = int(L) // 2 + 1
    e = np.unique(np.round(np.logspace(0, np.log10(top), int(n_bins) + 1)).astype(np.int64))
    e[0], e[-1] = 1, top
    return np.unique(e)


def config_sq(n_steps=10_000, n_meas=30, samples=64, L=8192, f=1.0, kind=RF):
    """Structure factor during relaxation at the shape of Fig. 4 (L = 8192), with a
    smaller ensemble: every mode n = 1 .. L/2 at log-spaced times."""
    p = _problem(kind, [L] * samples, [f] * samples, np.arange(samples), n_steps, n_meas,
                 SEED_BASE + 8)
    p["sq_edges"] = sq_edges_full(L)
    return p


def custom(kind, L, f, n_steps, meas_steps, seed, disorder_id=None, c=1.0, dt=0.05,
           strength=1.0, period=0, sq_edges=None):
    L = np.atleast_1d(np.asarray(L, np.int64))
    f = np.broadcast_to(np.asarray(f, np.float64), L.shape).copy()
    did = np.arange(L.size) if disorder_id is None else disorder_id
    return {
        "kind": int(kind), "strength": float(strength), "seed": int(seed),
        "c": float(c), "dt": float(dt), "n_steps": int(n_steps), "L": L, "f": f,
        "disorder_id": np.asarray(did, np.uint32),
        "meas_steps": np.asarray(meas_steps, np.int64),
        "period": int(period),
        "sq_edges": None if sq_edges is None else np.asarray(sq_edges, np.int64),
    }
