"""Critical force f_c^s and critical configuration of samples periodic in u
(Sec. III A), on the GPU.

A sample of L columns whose disorder repeats with period M in u (the
transverse period of the library's disorder) has a largest drive f_c^s at
which a pinned solution of c d2u/dx2 + F_p(u, x) + f = 0 exists.

`critical_forces` calls the library's no-passing solver (qew_critical_force):
every sample is bisected on f on the device in one launch, each trial drive
decided by moving sites forward to the first zeros of their own forces (which
never passes a pinned configuration) until the line is pinned or has advanced
by M.  Nothing is integrated in time and nothing returns to the host between
trials.

`critical_forces_euler` is the earlier driver kept for comparison: the same
bisection, each trial an Euler relaxation of Eq. (1) through qew_run in chunks
of steps, decided on the host between chunks:
- pinned when no site moved by more than chunk * dt * tol_force during a
  chunk (the mean force per site over the chunk is below tol_force);
- depinned when every site has advanced by at least M.
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


STATUS = {0: "done", 1: "no pinned configuration at the lower drive",
          2: "a trial undecided within max_sweeps", 3: "out of bisection rounds"}


def critical_forces(kind, L, M, disorder_ids, seed, f_lo=0.0, f_hi=5.0, tol_f=1e-6,
                    tol_force=1e-10, strength=1.0, c=1.0, max_sweeps=2_000_000, u0=None):
    """f_c^s of every sample (disorder id) of length L and period M by the
    library's no-passing solver.  Returns dict(f_lo [S], f_hi [S], u_c [S][L],
    sweeps [S]): f_c^s lies in [f_lo, f_hi) with f_hi - f_lo < tol_f, u_c is the
    pinned configuration at f_lo.  u0: start configurations (default flat)."""
    import torch
    dids = np.asarray(disorder_ids, np.uint32)
    S = dids.size
    dev = torch.device("cuda")
    d_did = torch.from_numpy(dids.view(np.int32).copy()).to(dev)  # the uint32 ids, bit for bit
    u = np.zeros((S, int(L))) if u0 is None else np.array(u0, np.float64).reshape(S, int(L))
    d_u = torch.from_numpy(np.ascontiguousarray(u)).to(dev)
    d_f = torch.zeros((S, 2), dtype=torch.float64, device=dev)
    d_st = torch.zeros((S, 2), dtype=torch.int64, device=dev)
    qew.qew_critical_force(kind, strength, seed, M, c, d_did, f_lo, f_hi, tol_f, tol_force, max_sweeps,
                           d_u, d_f, d_st, torch.cuda.current_stream())
    torch.cuda.synchronize()
    st = d_st.cpu().numpy()
    bad = st[:, 0] != 0
    if np.any(bad):
        s = int(np.flatnonzero(bad)[0])
        raise RuntimeError(f"critical force of sample {s}: {STATUS.get(int(st[s, 0]), st[s, 0])}")
    f = d_f.cpu().numpy()
    return {"f_lo": f[:, 0], "f_hi": f[:, 1], "u_c": d_u.cpu().numpy(), "sweeps": st[:, 1]}


def critical_forces_euler(kind, L, M, disorder_ids, seed, f_lo=0.0, f_hi=5.0, tol_f=1e-6,
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
    ap = argparse.ArgumentParser(description="f_c^s of periodic samples on the GPU")
    ap.add_argument("--kind", type=int, default=1)
    ap.add_argument("--L", type=int, default=256)
    ap.add_argument("--M", type=int, default=256)
    ap.add_argument("--samples", type=int, default=32)
    ap.add_argument("--tol-f", type=float, default=1e-5)
    ap.add_argument("--f-hi", type=float, default=4.0)
    ap.add_argument("--seed", type=int, default=workloads.SEED_BASE + 9)
    ap.add_argument("--method", choices=("no-passing", "euler"), default="no-passing")
    a = ap.parse_args(argv)
    solve = critical_forces if a.method == "no-passing" else critical_forces_euler
    solve(a.kind, min(a.L, 64), min(a.M, 64), np.arange(1), a.seed, f_hi=a.f_hi, tol_f=1e-2)  # warm-up: library and kernels
    t0 = time.perf_counter()
    r = solve(a.kind, a.L, a.M, np.arange(a.samples), a.seed, f_hi=a.f_hi, tol_f=a.tol_f)
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
    work = ({"sweeps_per_sample": r["sweeps"].tolist()} if a.method == "no-passing" else
            {"rounds": r["rounds"], "euler_steps": r["steps"]})
    print(json.dumps({"method": a.method, "kind": a.kind, "L": a.L, "M": a.M, "samples": a.samples,
                      "tol_f": a.tol_f, "f_c_mean": float(r["f_lo"].mean()), "f_c_std": float(r["f_lo"].std()),
                      "f_c": r["f_lo"].tolist(), "seconds": round(wall, 3), **work,
                      "zeta_from_sq": round((-slope - 1) / 2, 4), "sq_fit_modes": n_fit}))


if __name__ == "__main__":
    main()
