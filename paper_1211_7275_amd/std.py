"""Short-time-dynamics (STD) analysis of the disorder-averaged series (Sec. IV).

Host-side numpy on the series the library returns (t = step * dt):

- gamma(t) = w(t) / (t v(t)), which is constant in the critical regime because
  beta = nu (z - zeta) (Sec. IV B); its plateau marks where pure power laws
  hold;
- pure power-law fits y = A t^e on a time range, and the windowed exponents of
  procedure (c) of Sec. IV E (fits on [t0, 4 t0] for many t0);
- corrected power laws y = A t^e [1 + (t / t_c)^-alpha] (the corrected width
  and velocity of Sec. IV D, and the gamma fit with e = 0);
- the f-scan that brackets the critical force (Sec. IV A): at f < f_c the
  velocity dies, at f > f_c it saturates, and at f_c it decays as
  t^(-beta/(nu z)); `fscan` runs all drives as one batch on the GPU, sharing
  disorder ids across drives.
"""
import numpy as np
from scipy.optimize import curve_fit


def gamma(t, w2, v):
    """gamma(t) = w / (t v) with w = sqrt(w2)."""
    t = np.asarray(t, np.float64)
    return np.sqrt(np.asarray(w2, np.float64)) / (t * np.asarray(v, np.float64))


def _window(t, y, t_lo, t_hi):
    t = np.asarray(t, np.float64)
    y = np.asarray(y, np.float64)
    sel = (t > 0) & (y > 0)
    if t_lo is not None:
        sel &= t >= t_lo
    if t_hi is not None:
        sel &= t <= t_hi
    return t[sel], y[sel]


def power_law_fit(t, y, t_lo=None, t_hi=None):
    """Least-squares fit of log y = log A + e log t on t_lo <= t <= t_hi.
    Returns (A, e)."""
    tt, yy = _window(t, y, t_lo, t_hi)
    if tt.size < 2:
        raise ValueError("a power-law fit needs at least two positive points in the window")
    e, logA = np.polyfit(np.log(tt), np.log(yy), 1)
    return float(np.exp(logA)), float(e)


def window_exponents(t, y, t0s, factor=4.0):
    """Exponent of pure power-law fits on [t0, factor * t0] for each t0 (procedure (c))."""
    out = []
    for t0 in t0s:
        tt, _ = _window(t, y, t0, factor * t0)
        out.append(power_law_fit(t, y, t0, factor * t0)[1] if tt.size >= 2 else np.nan)
    return np.array(out)


def _corrected(logt, logA, e, log_tc, alpha):
    return logA + e * logt + np.log1p(np.exp(-alpha * (logt - log_tc)))


def corrected_fit(t, y, t_mic, p0=None, t_hi=None):
    """Fit y = A t^e [1 + (t / t_c)^-alpha] for t >= t_mic (least squares in log y).
    Returns dict(A, e, t_c, alpha)."""
    tt, yy = _window(t, y, t_mic, t_hi)
    if tt.size < 5:
        raise ValueError("a corrected fit needs at least five positive points")
    if p0 is None:
        A0, e0 = power_law_fit(tt[tt.size // 2:], yy[yy.size // 2:])
        p0 = (np.log(A0), e0, np.log(tt[0]), 0.7)
    else:
        p0 = (np.log(p0[0]), p0[1], np.log(p0[2]), p0[3])
    popt, _ = curve_fit(_corrected, np.log(tt), np.log(yy), p0=p0, maxfev=20000)
    return {"A": float(np.exp(popt[0])), "e": float(popt[1]), "t_c": float(np.exp(popt[2])),
            "alpha": float(popt[3])}


def gamma_fit(t, g, t_mic, p0=None):
    """Fit gamma = G0 [1 + (t / t_g)^-alpha_g] for t >= t_mic.  Returns dict(G0, t_g, alpha_g)."""
    tt, gg = _window(t, g, t_mic, None)
    if tt.size < 4:
        raise ValueError("the gamma fit needs at least four positive points")
    f = lambda lt, lG, ltg, a: _corrected(lt, lG, 0.0, ltg, a)  # noqa: E731
    p = (np.log(gg[-1]), np.log(tt[0]), 0.5) if p0 is None else (np.log(p0[0]), np.log(p0[1]), p0[2])
    popt, _ = curve_fit(f, np.log(tt), np.log(gg), p0=p, maxfev=20000)
    return {"G0": float(np.exp(popt[0])), "t_g": float(np.exp(popt[1])), "alpha_g": float(popt[2])}


def late_slope(t, v, decades=1.0):
    """Exponent of a pure power-law fit of v over the last `decades` decades of t."""
    t = np.asarray(t, np.float64)
    return power_law_fit(t, v, t[-1] / 10.0 ** decades)[1]


def classify_drive(t, v, decades=1.0, critical_slope=0.128, v_floor=1e-5):
    """+1 if v(t) saturates (f above the threshold), -1 if it dies.

    At f = f_c the velocity decays as t^(-beta/(nu z)), with beta/(nu z) = 0.128
    (Sec. IV E); a late log-slope above -critical_slope means the curve bends
    towards saturation, below it towards zero.  A velocity that has fallen
    below v_floor (a pinned line, down to the rounding of its arithmetic) dies."""
    v = np.asarray(v, np.float64)
    if not np.all(np.isfinite(v)) or v[-1] <= v_floor:
        return -1
    return 1 if late_slope(t, v, decades) > -critical_slope else -1


def bracket_fc(drives, t, v_by_drive, decades=1.0, critical_slope=0.128, v_floor=1e-5):
    """Classify every drive (`classify_drive`) and return (f_lo, f_hi, signs):
    f_lo the largest drive whose v dies, f_hi the smallest whose v saturates
    (None where no drive qualifies)."""
    drives = np.asarray(drives, np.float64)
    signs = np.array([classify_drive(t, v, decades, critical_slope, v_floor) for v in v_by_drive])
    dying = drives[signs < 0]
    saturating = drives[signs > 0]
    f_lo = float(dying.max()) if dying.size else None
    f_hi = float(saturating.min()) if saturating.size else None
    return f_lo, f_hi, signs


def fscan(kind, L, drives, n_steps, n_meas, seed, disorders=1, precision=None, path=None,
          strength=1.0, dt=0.05, c=1.0, decades=1.0):
    """f-scan on the GPU: len(drives) x disorders samples of length L in one
    batch (disorder ids 0..disorders-1 shared by every drive), series averaged
    over the disorders of each drive, then `bracket_fc`.
    Returns dict(t, drives, v, w2, f_lo, f_hi, signs)."""
    from . import qew, workloads
    drives = np.asarray(drives, np.float64)
    did = np.tile(np.arange(disorders), drives.size)
    f = np.repeat(drives, disorders)
    meas = workloads.log_steps(n_steps, n_meas)
    p = workloads.custom(kind, [L] * f.size, f, n_steps, meas, seed, disorder_id=did, c=c, dt=dt,
                         strength=strength)
    precision = qew.QEW_FP32_SPLIT if precision is None else precision
    path = (qew.QEW_FUSED if precision == qew.QEW_FP32_SPLIT else qew.QEW_ONE_STEP) if path is None else path
    sim = qew.Simulation(p, precision=precision, path=path)
    try:
        out = sim.run()
    finally:
        sim.close()
    v = out["v"].reshape(drives.size, disorders, -1).mean(1)
    w2 = out["w2"].reshape(drives.size, disorders, -1).mean(1)
    t = meas * dt
    f_lo, f_hi, signs = bracket_fc(drives, t, v, decades)
    return {"t": t, "drives": drives, "v": v, "w2": w2, "f_lo": f_lo, "f_hi": f_hi, "signs": signs}


def exponents(t, v, w2, t0s=(1.0, 10.0, 100.0, 1000.0, 10000.0), t_mic=2.0):
    """The exponent estimates of Sec. IV E for one drive's series: beta/(nu z)
    from v and 1 - zeta/z from w = sqrt(w2), by pure power laws on [t0, 4 t0]
    (procedure (c)) and by the corrected forms for t >= t_mic (procedure (a)),
    with gamma(t) at the end of each window."""
    t = np.asarray(t, np.float64)
    w = np.sqrt(np.asarray(w2, np.float64))
    t0s = [t0 for t0 in t0s if 4 * t0 <= t[-1]]
    out = {"t0": list(t0s),
           "beta_over_nu_z": (-window_exponents(t, v, t0s)).tolist(),
           "one_minus_zeta_over_z": (1.0 - window_exponents(t, w, t0s)).tolist(),
           "gamma": [float(np.interp(4 * t0, t, gamma(t, w2, v))) for t0 in t0s]}
    try:
        out["corrected_beta_over_nu_z"] = -corrected_fit(t, v, t_mic)["e"]
        out["corrected_one_minus_zeta_over_z"] = 1.0 - corrected_fit(t, w, t_mic)["e"]
    except (RuntimeError, ValueError):
        pass
    return out


def main(argv=None):
    """Command line f-scan: a geometric coarse scan over [--f-min, --f-max]
    locates the threshold, then a scan in steps of --f-step between the last
    dying and the first saturating coarse drive brackets it.  Prints one JSON
    line (bracket, drives, classes, late slopes, last velocities)."""
    import argparse
    import json
    from . import workloads
    ap = argparse.ArgumentParser(description="STD f-scan on the GPU (bracket of the critical force)")
    ap.add_argument("--kind", type=int, default=0)
    ap.add_argument("--L", type=int, default=1 << 16)
    ap.add_argument("--f-min", type=float, default=0.05)
    ap.add_argument("--f-max", type=float, default=5.0)
    ap.add_argument("--coarse", type=int, default=24, help="drives of the coarse scan")
    ap.add_argument("--f-step", type=float, default=0.02)
    ap.add_argument("--steps", type=int, default=100_000)
    ap.add_argument("--points", type=int, default=100)
    ap.add_argument("--disorders", type=int, default=1)
    ap.add_argument("--seed", type=int, default=workloads.SEED_BASE + 4)
    ap.add_argument("--decay", type=float, nargs="+", metavar="F",
                    help="instead of a scan: run these drives and report the exponents of v and w")
    a = ap.parse_args(argv)
    if a.decay:
        r = fscan(a.kind, a.L, a.decay, a.steps, a.points, a.seed, disorders=a.disorders)
        res = []
        for i, f in enumerate(r["drives"]):
            e = exponents(r["t"], r["v"][i], r["w2"][i])
            e["f"] = float(f)
            e["class"] = int(r["signs"][i])
            res.append(e)
        print(json.dumps({"kind": a.kind, "L": a.L, "steps": a.steps, "disorders": a.disorders,
                          "drives": res}))
        return

    def describe(r):
        late = [late_slope(r["t"], v) if v[-1] > 0 else None for v in r["v"]]
        return {"f_lo": r["f_lo"], "f_hi": r["f_hi"], "drives": np.round(r["drives"], 6).tolist(),
                "signs": r["signs"].tolist(), "late_slope": late, "v_last": r["v"][:, -1].tolist()}

    coarse = np.geomspace(a.f_min, a.f_max, a.coarse)
    rc = fscan(a.kind, a.L, coarse, a.steps, a.points, a.seed, disorders=a.disorders)
    out = {"kind": a.kind, "L": a.L, "steps": a.steps, "disorders": a.disorders,
           "coarse": describe(rc)}
    if rc["f_lo"] is not None and rc["f_hi"] is not None and rc["f_lo"] < rc["f_hi"]:
        fine = np.round(np.arange(rc["f_lo"], rc["f_hi"], a.f_step), 10)
        fine = np.append(fine[fine < rc["f_hi"] - 1e-9], rc["f_hi"])
        rf = fscan(a.kind, a.L, fine, a.steps, a.points, a.seed, disorders=a.disorders)
        out["fine"] = describe(rf)
        out["f_lo"], out["f_hi"] = rf["f_lo"], rf["f_hi"]
    print(json.dumps(out))


if __name__ == "__main__":
    main()
