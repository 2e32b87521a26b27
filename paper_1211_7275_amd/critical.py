"""Critical force f_c^s and critical configuration of samples periodic in u
(Sec. III A), on the GPU.

A sample of L columns whose disorder repeats with period M in u (the
transverse period of the library's disorder) has a largest drive f_c^s at
which a pinned solution of c d2u/dx2 + F_p(u, x) + f = 0 exists.  Every
sample of a batch is bisected on f independently, and every trial of a round
runs in one FP64 batch through the library:

- a trial relaxes the chain from the last pinned configuration found (below
  the critical one, so the line only moves forward) at the trial drive, in
  chunks of Euler steps;
- it is pinned when no site moved by more than chunk * dt * tol_force during
  a chunk (the mean force per site over the chunk is below tol_force);
- it is depinned when every site has advanced by at least M: a forward-moving
  line never passes a pinned configuration, and the translates by M of a
  pinned configuration are pinned too, so none exists at that drive.

The host only compares states between chunks (no force is evaluated here);
every Euler step and measurement runs in the library's kernels.
"""
import numpy as np

from . import qew, workloads

PINNED, DEPINNED, UNDECIDED = 0, 1, 2


def _relax(kind, L, M, f, dids, u, u_ref, seed, strength, c, dt, chunk, max_steps, tol_force):
    """Relax every sample at its drive f[s] from u[s] (in place).  Returns the
    status per sample and the steps taken by the batch."""
    S = len(f)
    p = workloads.custom(kind, [L] * S, f, chunk, [chunk], seed, disorder_id=dids, c=c, dt=dt,
                         strength=strength, period=M)
    sim = qew.Simulation(p, precision=qew.QEW_FP64_PLAIN, path=qew.QEW_ONE_STEP)
    status = np.full(S, UNDECIDED)
    steps = 0
    tol_move = chunk * dt * tol_force
    try:
        while steps < max_steps:
            for s in range(S):
                sim.write_state(s, u[s], 0)
            sim.run(resume=True)
            steps += chunk
            for s in range(S):
                new = sim.read_state(s)[0]
                if status[s] == UNDECIDED:
                    if np.max(np.abs(new - u[s])) <= tol_move:
                        status[s] = PINNED
                    elif u_ref is not None and np.min(new - u_ref[s]) >= M:
                        status[s] = DEPINNED
                u[s] = new
            if np.all(status != UNDECIDED):
                break
    finally:
        sim.close()
    return status, steps


def critical_forces(kind, L, M, disorder_ids, seed, f_lo=0.0, f_hi=5.0, tol_f=1e-6,
                    tol_force=1e-10, strength=1.0, c=1.0, dt=0.05, chunk=2048,
                    max_steps=4_000_000):
    """Bisect f_c^s of every sample (disorder id) of length L and period M.
    Returns dict(f_lo [S], f_hi [S], u_c [S][L], rounds, steps): f_c^s lies in
    [f_lo, f_hi) with f_hi - f_lo < tol_f, u_c is the pinned configuration at
    f_lo, steps the Euler steps run per sample over all rounds."""
    dids = np.asarray(disorder_ids, np.uint32)
    S = dids.size
    lo = np.full(S, float(f_lo))
    hi = np.full(S, float(f_hi))
    u = np.zeros((S, int(L)))
    status, steps = _relax(kind, L, M, lo, dids, u, None, seed, strength, c, dt, chunk,
                           max_steps, tol_force)
    if np.any(status != PINNED):
        raise RuntimeError("no pinned configuration at the lower drive for some sample")
    total, rounds = steps, 0
    while np.any(hi - lo >= tol_f):
        active = hi - lo >= tol_f
        mid = np.where(active, 0.5 * (lo + hi), lo)
        trial = u.copy()
        status, steps = _relax(kind, L, M, mid, dids, trial, u, seed, strength, c, dt, chunk,
                               max_steps, tol_force)
        total += steps
        rounds += 1
        if np.any(status[active] == UNDECIDED):
            raise RuntimeError("a relaxation was undecided within max_steps")
        pinned = active & (status == PINNED)
        lo[pinned] = mid[pinned]
        u[pinned] = trial[pinned]
        depinned = active & (status == DEPINNED)
        hi[depinned] = mid[depinned]
    return {"f_lo": lo, "f_hi": hi, "u_c": u, "rounds": rounds, "steps": total}


def main(argv=None):
    """Critical forces of a batch of periodic samples; prints one JSON line with
    the forces, their mean and spread, the time, and the roughness exponent
    fitted to the structure factor of the critical configurations."""
    import argparse
    import json
    import time

    import torch

    from . import std
    ap = argparse.ArgumentParser(description="f_c^s of periodic samples (bisection on the GPU)")
    ap.add_argument("--kind", type=int, default=1)
    ap.add_argument("--L", type=int, default=256)
    ap.add_argument("--M", type=int, default=256)
    ap.add_argument("--samples", type=int, default=32)
    ap.add_argument("--tol-f", type=float, default=1e-5)
    ap.add_argument("--f-hi", type=float, default=4.0)
    ap.add_argument("--seed", type=int, default=workloads.SEED_BASE + 9)
    a = ap.parse_args(argv)
    t0 = time.perf_counter()
    r = critical_forces(a.kind, a.L, a.M, np.arange(a.samples), a.seed, f_hi=a.f_hi, tol_f=a.tol_f)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # structure factor of the critical configurations, on the device
    edges = workloads.sq_edges_full(a.L)
    p = workloads.custom(a.kind, [a.L] * a.samples, r["f_lo"], 0, [0], a.seed,
                         disorder_id=np.arange(a.samples), period=a.M, sq_edges=edges)
    sim = qew.Simulation(p, precision=qew.QEW_FP64_PLAIN, path=qew.QEW_ONE_STEP)
    try:
        for s in range(a.samples):
            sim.write_state(s, r["u_c"][s], 0)
        sim.run(resume=True)
        sq = sim.structure_factor()[0]
    finally:
        sim.close()
    q = 2 * np.pi * np.arange(1, a.L // 2 + 1) / a.L
    n_fit = max(a.L // 16, 4)
    _, slope = std.power_law_fit(q[:n_fit], sq[:n_fit])
    print(json.dumps({"kind": a.kind, "L": a.L, "M": a.M, "samples": a.samples,
                      "f_c_mean": float(r["f_lo"].mean()), "f_c_std": float(r["f_lo"].std()),
                      "f_c": r["f_lo"].tolist(), "rounds": r["rounds"], "steps": r["steps"],
                      "seconds": round(wall, 2),
                      "site_updates_per_s": a.L * a.samples * r["steps"] / wall,
                      "zeta_from_sq": round((-slope - 1) / 2, 4), "sq_fit_modes": n_fit}))


if __name__ == "__main__":
    main()
