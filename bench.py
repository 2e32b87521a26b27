"""Benchmark of the QEW hot path on one MI355X.

Workload: L = 2^22 sites x 4 random-field samples (uniform values, Catmull-Rom
spline), c = 1, dt = 0.05, f = 1.0, flat start, 10^6 Euler steps with 200
log-spaced measurements of v, ubar and w2.  The timed region is that whole
run: a benchmark "step" is 1/K of the 10^6-step horizon (K = --steps), so the
K timed steps are the complete workload with every measurement.  Inputs are
synthetic and generated on the device (the disorder is counter-based; the
state starts flat).

The timed path is the FP32-split fused (temporally blocked) kernel; the FP64
plain one-step kernel is timed beside it on a window of the same workload with
the same measurement density (its cost per Euler step does not depend on the
state: it regenerates every node of every site at every step).  The FP64
oracle is timed on the host on a bounded stretch of sample 0, and the GPU
states and series at the end of that stretch are compared with it.
Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_1211_7275_amd import workloads  # noqa: E402

# MI355X (gfx950) figures used for the rooflines.
CUS = 256
CLOCK_HZ = 2.4e9
# FP32 vector peak 157.3 TFLOP/s = 78.6e12 FMAs/s: 256 CUs x 4 SIMDs x 32 lanes x 2.4 GHz
# 32-bit VALU lane-operations per second.
VALU_LANE_OPS = CUS * 4 * 32 * CLOCK_HZ
HBM_PEAK_GBS = 8000.0

# Algorithmic VALU operations of one FP32 split site update:
# Laplacian on (cell, offset) 7, Catmull-Rom from the four cached nodes 12,
# total force 2, Euler 1, renormalisation 7.
OPS_SITE_UPDATE_RF = 29
OPS_SITE_UPDATE_RB = 28
# One node: Philox4x32-10 (10 rounds x (2 64-bit products + 2 three-input
# xors + 2 key adds)) = 60, plus the value conversion (RF 3, RB 8).
OPS_NODE_RF = 63
OPS_NODE_RB = 68
# The benchmark workload: horizon and measurement points of the 10^6-step run.
HORIZON = 1_000_000
N_POINTS = 200
# Launch geometry of the benchmark line (steps per fused launch, sites per
# workgroup tile): the autotuner's choice on this workload.  Its candidates
# around the optimum are within about 1 % of each other and swap from box to
# box, so the benchmark fixes the geometry its profiles were taken with;
# --k 0 --tile 0 lets the autotuner choose.
BENCH_K = 56
BENCH_TILE = 2048

TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "hbm_traffic_fused_L2e22x4.md")


def _elf_sections(data):
    """{name: (addr, offset, size)} of a little-endian ELF64 image."""
    import struct
    shoff, = struct.unpack_from("<Q", data, 0x28)
    shentsize, shnum, shstrndx = struct.unpack_from("<HHH", data, 0x3A)
    hdr = [struct.unpack_from("<IIQQQQIIQQ", data, shoff + i * shentsize) for i in range(shnum)]
    stroff = hdr[shstrndx][4]
    out = {}
    for h in hdr:
        name = data[stroff + h[0]:data.index(b"\0", stroff + h[0])].decode()
        out[name] = (h[3], h[4], h[5], h)
    return out


# Kernels whose measured traffic the bench line carries, by symbol pattern:
# every dense fused instantiation, and the FP64 one-step kernel of the
# benchmark's disorder (random field) without measurement.
FUSED_SYMBOLS = rb"k_step_fusedILi\d+ELi\d+ELb0E"
PLAIN_SYMBOLS = rb"k_step_plainILi0ELb0E"


def kernel_source_hash(pattern=FUSED_SYMBOLS):
    """sha256 (first 16 hex) of the machine code of the kernels whose symbols
    match `pattern` (default: every dense k_step_fused instantiation) in the
    gfx950 code object of the built library: it changes exactly when those
    kernels' compiled code does."""
    import hashlib
    import re
    import struct
    lib = os.path.join(ROOT, "paper_1211_7275_amd", "lib", "libqew.so")
    with open(lib, "rb") as fh:
        data = fh.read()
    _, off, size, _ = _elf_sections(data)[".hip_fatbin"]
    blob = data[off:off + size]
    assert blob[:24] == b"__CLANG_OFFLOAD_BUNDLE__", "unexpected device code bundle"
    n, = struct.unpack_from("<Q", blob, 24)
    pos, code = 32, None
    for _ in range(n):
        eoff, esize, tlen = struct.unpack_from("<QQQ", blob, pos)
        triple = blob[pos + 24:pos + 24 + tlen].decode()
        pos += 24 + tlen
        if "gfx950" in triple:
            code = blob[eoff:eoff + esize]
    assert code is not None, "no gfx950 code object in the library"
    secs = _elf_sections(code)
    text_addr, text_off, _, _ = secs[".text"]
    _, sym_off, sym_size, sym_hdr = secs[".symtab"]
    _, str_off, _, _ = secs[".strtab"]
    h = hashlib.sha256()
    syms = []
    for i in range(sym_size // 24):
        st_name, st_info, st_other, st_shndx, st_value, st_size = struct.unpack_from(
            "<IBBHQQ", code, sym_off + 24 * i)
        name = code[str_off + st_name:code.index(b"\0", str_off + st_name)]
        if re.search(pattern, name) and st_size > 0 and not name.endswith(b".kd"):
            syms.append((name, st_value, st_size))
    for name, value, size in sorted(syms):
        start = text_off + (value - text_addr)
        h.update(name)
        h.update(code[start:start + size])
    return h.hexdigest()[:16]


def committed_traffic(k=None, tile=None, plain=False):
    """HBM bytes per launch measured by rocprofv3 (FETCH_SIZE/WRITE_SIZE,
    copy-calibrated) for this kernel code (and fused geometry), else None."""
    if not os.path.exists(TRAFFIC_SUMMARY):
        return None
    if plain:
        want = f"plain source={kernel_source_hash(PLAIN_SYMBOLS)}"
    else:
        want = f"fused k={k} tile={tile} source={kernel_source_hash()}"
    for ln in open(TRAFFIC_SUMMARY):
        if ln.startswith("traffic_per_launch ") and want in ln:
            for tok in ln.split():
                if tok.startswith("bytes="):
                    return int(tok[6:])
    return None


def bench_problem(steps, L=1 << 22, samples=4):
    """The benchmark workload cut to its first `steps` Euler steps, with the
    measurements of the 10^6-step cadence that fall inside them."""
    p = workloads.config3(n_steps=HORIZON, n_meas=N_POINTS, samples=samples, L=L)
    meas = p["meas_steps"]
    p["n_steps"] = int(steps)
    p["meas_steps"] = meas[meas <= steps]
    return p


def window_problem(steps, L=1 << 22, samples=4):
    """The benchmark workload over a window of `steps` Euler steps with the
    full run's measurement density (N_POINTS per HORIZON steps), log-spaced."""
    p = workloads.config3(n_steps=HORIZON, n_meas=N_POINTS, samples=samples, L=L)
    n = max(1, int(round(N_POINTS * steps / HORIZON)))
    p["n_steps"] = int(steps)
    p["meas_steps"] = workloads.log_steps(steps, n)
    return p


def time_path(qew, p, precision, path, warm_steps, k=0, tile=0, flags=0):
    """Warm-up run of `warm_steps` Euler steps (geometry autotuned there when
    k or tile is 0), then the timed run of p from the flat start."""
    import torch

    pw = dict(p, n_steps=int(warm_steps), meas_steps=p["meas_steps"][p["meas_steps"] <= warm_steps])
    warm = qew.Simulation(pw, precision=precision, path=path, k=k, tile=tile, flags=flags)
    warm.run()
    info = warm.info()
    warm.close()
    sim = qew.Simulation(p, precision=precision, path=path, k=info.k if path else 0,
                         tile=info.tile if path else 0, flags=qew.QEW_FLAG_TIMING | flags)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = sim.run()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = sim.stats()
    info = sim.info()
    sim.close()
    return out, st, info, t1 - t0


def fused_roofline(kind, st, info, out, steps):
    """ALU roofline of the fused kernel (the dominant one) from the HIP-event
    durations of the run's fused segments: algorithmic operations of the site
    updates those launches made, divided by their time."""
    sites = info.total_sites
    # Cells entered per site update (physics, not implementation): the centre
    # of mass advanced by ubar(last) - ubar(0) cells over the timed steps.
    ub = out["ubar"]
    adv = float(np.nanmean(ub[:, -1])) if ub.shape[1] else 0.0
    entries_per_update = max(adv, 0.0) / max(steps, 1)
    per_update = (OPS_SITE_UPDATE_RF if kind == 0 else OPS_SITE_UPDATE_RB) + \
        (OPS_NODE_RF if kind == 0 else OPS_NODE_RB) * entries_per_update
    launches = max(int(st.fused_launches), 1)
    launch_ms = st.fused_ms / launches
    updates_per_launch = sites * int(st.fused_steps) / launches
    achieved = per_update * updates_per_launch / (launch_ms * 1e-3) / 1e12
    peak = VALU_LANE_OPS / 1e12
    return {"bound": "alu", "achieved": round(achieved, 3), "peak": round(peak, 3),
            "unit": "TOP/s", "frac": round(achieved / peak, 4),
            "traffic": committed_traffic(info.k, info.tile),
            "ops_per_update": round(per_update, 3), "launch_ms": round(launch_ms, 5),
            "launches": int(st.fused_launches), "euler_steps": int(st.fused_steps),
            "one_step_launches": int(st.step_launches - st.fused_launches),
            "node_refreshes": int(st.node_refreshes), "kernel": "k_step_fused (dense)",
            "k": info.k, "tile": info.tile}


def plain_roofline(st, info, steps):
    """HBM roofline of the FP64 plain one-step kernel (16 B per site update)."""
    launch_ms = st.step_ms / max(st.step_launches, 1)
    bytes_per_launch = 16.0 * info.total_sites * steps / max(st.step_launches, 1)
    gbs = bytes_per_launch / (launch_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": committed_traffic(plain=True),
            "launch_ms": round(launch_ms, 5), "launches": int(st.step_launches)}


def cpu_model():
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(p, seconds_target=15.0):
    """The oracle on sample 0 of the workload (full length) from the flat
    start, for as many Euler steps as fit the time target, with the workload's
    measurements inside that stretch.  Returns the baseline entry of the bench
    line and the oracle's run (steps, measurement steps, series, final state)."""
    from oracle import oracle

    threads = oracle.get_threads()
    kind, strength, seed, c, dt = p["kind"], p["strength"], p["seed"], p["c"], p["dt"]
    L, did, f = int(p["L"][0]), int(p["disorder_id"][0]), float(p["f"][0])
    # the step time from a 4-step run after a 1-step warm-up of the threads
    oracle.run_sample(kind, strength, seed, did, L, c, dt, f, 1, [])
    t0 = time.perf_counter()
    oracle.run_sample(kind, strength, seed, did, L, c, dt, f, 4, [])
    per_step = (time.perf_counter() - t0) / 4
    steps = max(1, int(seconds_target / max(per_step, 1e-6)))
    meas = p["meas_steps"][p["meas_steps"] <= steps]
    t0 = time.perf_counter()
    ref = oracle.run_sample(kind, strength, seed, did, L, c, dt, f, steps, meas)
    wall = time.perf_counter() - t0
    # the same sample on one core, a few steps
    oracle.set_threads(1)
    try:
        t1 = time.perf_counter()
        oracle.run_sample(kind, strength, seed, did, L, c, dt, f, 4, [])
        single = L * 4 / (time.perf_counter() - t1)
    finally:
        oracle.set_threads(threads)
    entry = {"value": round(L * steps / wall, 1), "unit": "site-updates/s", "cores": threads,
             "kind": "oracle",
             "sample": f"sample 0 of 4 (L=2^22), Euler steps 1..{steps} from the flat start with the "
                       f"{len(meas)} measurements of the 10^6-step cadence inside them, FP64, OpenMP "
                       f"over sites on {threads} threads, {wall:.1f} s",
             "cpu_model": cpu_model(), "single_core_value": round(single, 1)}
    return entry, {"steps": steps, "meas": meas, "ref": ref}


def _rel(a, b, floor):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), floor))) if a.size else 0.0


def c3_parity(qew, p, oracle_run, k, tile):
    """Error against the oracle of both GPU paths on the benchmark workload:
    sample 0 after the oracle's stretch of Euler steps (every site), and its
    v, ubar, w2 at every measurement of that stretch.  The fused path runs in
    the benchmark's launch geometry."""
    steps, meas, ref = oracle_run["steps"], oracle_run["meas"], oracle_run["ref"]
    pp = dict(p, n_steps=int(steps), meas_steps=np.asarray(meas, np.int64))
    res = {"workload": f"the benchmark workload, Euler steps 1..{steps}, sample 0 (all "
                       f"{int(p['L'][0])} sites) and its {len(meas)} measurements"}
    for name, prec, path, kk, tt in (("fp32_split_fused", qew.QEW_FP32_SPLIT, qew.QEW_FUSED, k, tile),
                                     ("fp64_plain", qew.QEW_FP64_PLAIN, qew.QEW_ONE_STEP, 0, 0)):
        sim = qew.Simulation(pp, precision=prec, path=path, k=kk, tile=tt)
        try:
            out = sim.run()
            u = sim.read_state(0)[0]
        finally:
            sim.close()
        d = np.abs(u - ref["u"])
        w2_mask = ref["w2"] > 0  # w2(0) = 0 exactly on the flat start
        res[name] = {"max_site_abs_err": float(d.max()), "p999_site_abs_err": float(np.quantile(d, 0.999)),
                     "max_v_rel_err": _rel(out["v"][0], ref["v"], 1e-3),
                     "max_ubar_rel_err": _rel(out["ubar"][0], ref["ubar"], 1e-3),
                     "max_w2_rel_err": _rel(out["w2"][0][w2_mask], ref["w2"][w2_mask], 1e-12)}
    return res


def summarize_profile(run_dir, copy_dir_fetch=None, copy_dir_write=None):
    """Markdown summary of rocprofv3 CSV output of a bench.py run (kernel trace
    and/or FETCH_SIZE / WRITE_SIZE / SQ counters), for profiles/."""
    import csv
    import glob
    import statistics

    def rows(pattern):
        out = []
        for fn in glob.glob(os.path.join(run_dir, "**", pattern), recursive=True):
            out += list(csv.DictReader(open(fn)))
        return out

    def short(n):
        return n.replace("(anonymous namespace)::", "").split("(")[0].replace("void ", "")

    lines = []
    stats = rows("*kernel_stats.csv")
    if stats:
        lines += ["| kernel | calls | total ms | average us |", "|---|---|---|---|"]
        for r in stats[:8]:
            lines.append(f"| `{short(r['Name'])}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.2f} "
                         f"| {float(r['AverageNs']) / 1e3:.1f} |")
    trace = rows("*kernel_trace.csv")
    if trace:
        trace.sort(key=lambda r: int(r["Start_Timestamp"]))
        # The timed run of a path starts at its last initialisation kernel and
        # runs until the other path's first initialisation after it (or the end).
        for init, other in (("k_init_split", "k_init_plain"), ("k_init_plain", "k_init_split")):
            idx = [i for i, r in enumerate(trace) if init in r["Kernel_Name"]]
            if not idx:
                continue
            seg = []
            for r in trace[idx[-1] + 1:]:
                if other in r["Kernel_Name"]:
                    break
                seg.append(r)
            by_name = {}  # each kernel (e.g. each variant of the fused kernel) on its own line
            for r in seg:
                by_name.setdefault(short(r["Kernel_Name"]), []).append(
                    (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6)
            for name, d in by_name.items():
                lines.append(f"\ntimed run: `{name}` {len(d)} launches, average {sum(d) / len(d):.5f} ms, "
                             f"total {sum(d):.3f} ms")
    counters = rows("*counter_collection.csv")
    if counters:
        # one record per dispatch: name, duration, counter sums
        disp = {}
        for r in counters:
            d = disp.setdefault(int(r["Dispatch_Id"]), {
                "name": short(r["Kernel_Name"]),
                "ns": int(r["End_Timestamp"]) - int(r["Start_Timestamp"]), "c": {}})
            d["c"][r["Counter_Name"]] = d["c"].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
        order = sorted(disp)
        lines += ["", "Timed runs only (dispatches after the last initialisation kernel of each path):", "",
                  "| kernel | counter | dispatches | median per dispatch | sum | kernel ms (sum) |",
                  "|---|---|---|---|---|---|"]
        for init, tag in (("k_init_split", "k_step_fused"), ("k_init_plain", "k_step_plain")):
            inits = [i for i in order if init in disp[i]["name"]]
            if not inits:
                continue
            groups = {}
            for i in order:
                if i > inits[-1] and tag in disp[i]["name"]:
                    groups.setdefault(disp[i]["name"], []).append(disp[i])
            for name, seg in groups.items():
                ms = sum(d["ns"] for d in seg) / 1e6
                for cn in sorted(seg[0]["c"]):
                    v = [d["c"].get(cn, 0.0) for d in seg]
                    lines.append(f"| `{name}` | {cn} | {len(v)} | {statistics.median(v):.6g} "
                                 f"| {sum(v):.6g} | {ms:.3f} |")
        copies = [d for d in disp.values() if "copyBuffer" in d["name"]]
        if copies:
            for cn in sorted(copies[0]["c"]):
                v = [d["c"].get(cn, 0.0) for d in copies]
                lines.append(f"| `{copies[0]['name']}` (runtime copies) | {cn} | {len(v)} "
                             f"| {statistics.median(v):.6g} | {sum(v):.6g} | |")
    return "\n".join(lines)


# Workloads besides the benchmark line: name -> (description, builder(steps)).
# The drives of the L = 2^25 workloads sit around the critical force bracketed
# by the f-scan of `paper_1211_7275_amd.std` (workloads.C4_FCENTER).
OTHER_WORKLOADS = {
    "c1": ("L=2^16 RB Catmull-Rom Gaussian, 64 disorders x f in {0.8, 1.0, 1.2}",
           lambda n: workloads.config1(n_steps=n)),
    "c2": ("512 RF samples, L_s = 2^10..2^16 (uneven batch), f=1.0",
           lambda n: workloads.config2(n_steps=n)),
    "c4rf": ("L=2^25 x 5 drives around f_c, RF Catmull-Rom uniform, one disorder",
             lambda n: workloads.config4(0, n_steps=n)),
    "c4rb": ("L=2^25 x 5 drives around f_c, RB Catmull-Rom Gaussian, one disorder",
             lambda n: workloads.config4(1, n_steps=n)),
    "c3ref": ("the benchmark workload (L=2^22 x 4 RF) timed on this horizon like the other "
              "workloads (reference for c3sq)", lambda n: bench_problem(n)),
    "c3sq": ("the benchmark workload (L=2^22 x 4 RF) with the structure factor in 64 log-spaced "
             "mode bins at every measurement",
             lambda n: dict(bench_problem(n), sq_edges=workloads.sq_edges_log(1 << 22, 64))),
    "sq8192": ("structure factor at the shape of Fig. 4: L=8192 x 64 RF samples, every mode, "
               "30 log-spaced measurements",
               lambda n: workloads.config_sq(n_steps=n)),
}


def copy_bandwidth(nbytes, reps=5):
    """Device-to-device copy rate (read + write bytes per second) of a buffer of nbytes."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    rate = 2.0 * a.numel() * 4 * reps / (time.perf_counter() - t0)
    del a, b
    torch.cuda.empty_cache()
    return rate


def plain_without_disorder(qew, args, small=False):
    """The FP64 one-step kernel with no pinning force (a pure stencil, 16 B of
    HBM traffic per site update) on the L = 2^25 x 5 shape (small: the
    benchmark's 2^22 x 4, whose two 128 MiB buffers come close to the 256 MB
    Infinity Cache), against the copy bandwidth of a buffer of the same size."""
    base = workloads.config3(n_steps=args.steps) if small else workloads.config4(0, n_steps=args.steps)
    p = dict(base, strength=0.0)
    p["meas_steps"] = np.array([args.steps])
    out, st, info, wall = time_path(qew, p, qew.QEW_FP64_PLAIN, qew.QEW_ONE_STEP, args.warmup)
    roof = plain_roofline(st, info, args.steps)
    copy = copy_bandwidth(int(info.total_sites) * 8)
    return {"metric": "FP64 one-step stencil without disorder, HBM GB/s", "value": roof["achieved"],
            "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "site_updates_per_s": round(info.total_sites * args.steps / wall, 1),
            "copy_gbs": round(copy / 1e9, 1), "of_copy": round(roof["achieved"] * 1e9 / copy, 4),
            "config": {"workload": ("L=2^22 x 4" if small else "L=2^25 x 5") +
                       ", strength 0, FP64 plain one-step", "buffer_bytes":
                       int(info.total_sites) * 8}, "roofline": roof}


def other_workload(qew, args):
    if args.workload in ("plain0", "plain0small"):
        return plain_without_disorder(qew, args, small=args.workload == "plain0small")
    desc, build = OTHER_WORKLOADS[args.workload]
    steps = args.steps
    p = build(steps)
    variant = {"auto": 0, "dense": qew.QEW_FLAG_FUSED_DENSE,
               "sparse": qew.QEW_FLAG_FUSED_SPARSE}[args.fused_variant]
    out, st, info, wall = time_path(qew, p, qew.QEW_FP32_SPLIT, qew.QEW_FUSED, args.warmup,
                                    k=args.k, tile=args.tile, flags=variant)
    value = info.total_sites * steps / wall
    roof = fused_roofline(p["kind"], st, info, out, steps)
    roof["traffic"] = None  # the committed traffic summary covers the benchmark workload only
    return {"metric": "site-updates/s (FP32 split, fused)", "value": round(value, 1),
            "unit": "site-updates/s", "n_gpus": 1, "steps": steps, "warmup": args.warmup,
            "ms_per_step": round(wall * 1e3 / steps, 6), "higher_is_better": True,
            "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"{args.workload}: {desc}", "samples": len(p["L"]),
                       "total_sites": int(info.total_sites),
                       "measurements": int(len(p["meas_steps"])), "k": info.k, "tile": info.tile,
                       "fused_variant": args.fused_variant},
            "roofline": roof, "sparse_launches": int(st.sparse_launches),
            "meas_ms_per_measurement": round(st.meas_ms / max(st.meas_launches, 1), 4),
            "v_last_mean": float(np.nanmean(out["v"][:, -1])) if out["v"].shape[1] else None}


def progress(*a):
    """Phase lines on stderr (the JSON line alone goes to stdout)."""
    print("[bench]", *a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20,
                    help="benchmark line: number of benchmark steps, each 1/steps of the 10^6-step "
                         "horizon (the timed run is always the whole horizon); other workloads: "
                         "Euler steps")
    ap.add_argument("--warmup", type=int, default=5,
                    help="benchmark steps of untimed warm-up (capped at one horizon)")
    ap.add_argument("--horizon", type=int, default=HORIZON,
                    help="Euler steps of the benchmark run (the workload's is 10^6)")
    ap.add_argument("--plain-window", type=int, default=20_000,
                    help="Euler steps the FP64 plain leg is timed on (0: the whole horizon)")
    ap.add_argument("--skip-plain", action="store_true")
    ap.add_argument("--only-plain", action="store_true",
                    help="time only the FP64 plain leg (profiler runs of that kernel)")
    ap.add_argument("--skip-cpu", action="store_true",
                    help="skip the oracle leg (and with it the error against the oracle)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--k", type=int, default=None, help=f"steps per fused launch (default {BENCH_K}; 0: autotune)")
    ap.add_argument("--tile", type=int, default=None, help=f"sites per fused tile (default {BENCH_TILE}; 0: autotune)")
    ap.add_argument("--no-graph", action="store_true",
                    help="launch every kernel directly instead of replaying hipGraphs (the same "
                         "kernels and dispatches; for profiler counter runs)")
    ap.add_argument("--fused-variant", default="auto", choices=("auto", "dense", "sparse"),
                    help="other workloads: the fused kernel variant (auto: chosen from the "
                         "measured velocities before each stretch between measurements)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device copy (HBM counter calibration) and exit")
    ap.add_argument("--summarize-profile", metavar="DIR",
                    help="print a markdown summary of rocprofv3 CSV output under DIR and exit")
    ap.add_argument("--source-hash", action="store_true",
                    help="print the hashes of the fused and the plain kernels' machine code and exit")
    ap.add_argument("--workload", default="c3", choices=sorted(OTHER_WORKLOADS) + ["c3", "plain0", "plain0small"],
                    help="c3 (default): the benchmark line; others print one line for that "
                         "workload's FP32 split fused throughput (--steps sets the horizon)")
    args = ap.parse_args()

    if args.summarize_profile:
        print(summarize_profile(args.summarize_profile))
        return
    if args.source_hash:
        print(f"fused source={kernel_source_hash()} plain source={kernel_source_hash(PLAIN_SYMBOLS)}")
        return

    if args.gpus != 1:
        print(json.dumps({"error": "bench.py runs on one GPU only; "
                                   "run with --gpus 1 (multi-GPU sharding is not implemented)"}))
        sys.exit(2)
    if args.steps < 1 or args.warmup < 0 or args.horizon < 1:
        print(json.dumps({"error": "need --steps >= 1, --warmup >= 0 and --horizon >= 1"}))
        sys.exit(2)

    import torch

    if args.copy_calibration:
        n = 1 << 28
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": n * 4, "copy_calibration_bytes_written": n * 4,
                          "launches": 5}))
        return

    from paper_1211_7275_amd import qew

    if args.workload != "c3":
        if args.k is None:
            args.k = 0
        if args.tile is None:
            args.tile = 0
        print(json.dumps(other_workload(qew, args)), flush=True)
        return

    if args.only_plain:
        H = int(args.horizon)
        gflags = qew.QEW_FLAG_NO_GRAPH if args.no_graph else 0
        print(json.dumps({"metric": "FP64 plain one-step path on the benchmark workload (window)",
                          "fp64_plain": plain_leg(qew, args, H, gflags)}), flush=True)
        return

    k = BENCH_K if args.k is None else args.k
    tile = BENCH_TILE if args.tile is None else args.tile
    H = int(args.horizon)
    p = bench_problem(H)
    line_extra = {}
    # 1. The oracle on the host: its rate, and the reference for the error of both paths.
    oracle_run = None
    if not args.skip_cpu:
        progress("oracle on the host cores")
        line_extra["cpu_baseline"], oracle_run = cpu_baseline(p, args.cpu_seconds)
        progress("error of both GPU paths against the oracle,", oracle_run["steps"], "steps")
        line_extra["error_vs_oracle"] = c3_parity(qew, p, oracle_run, k, tile)
    # 2. The timed run: the whole horizon after the warm-up, fused FP32 split.
    warm_steps = min(H, int(round(args.warmup * H / args.steps)))
    gflags = qew.QEW_FLAG_NO_GRAPH if args.no_graph else 0
    progress("warm-up of", warm_steps, "Euler steps, then the timed run of", H)
    out, st, info, wall = time_path(qew, p, qew.QEW_FP32_SPLIT, qew.QEW_FUSED, max(warm_steps, 1),
                                    k=k, tile=tile, flags=gflags)
    sites = info.total_sites
    value = sites * H / wall
    roof = fused_roofline(p["kind"], st, info, out, H)
    line = {
        "metric": "site-updates/s FP32-split batched vs FP64 plain at L=2^22; % VALU/HBM roofline",
        "value": round(value, 1),
        "unit": "site-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (counter-based Philox disorder generated on the device, flat start)",
        "config": {
            "workload": "L=2^22 x 4 samples, random field uniform(-1,1) Catmull-Rom, c=1, dt=0.05, "
                        "f=1.0, flat start, 10^6 Euler steps with 200 log-spaced measurements",
            "L": int(p["L"][0]), "samples": len(p["L"]), "euler_steps_timed": H,
            "euler_steps_per_step": H / args.steps, "warmup_euler_steps": warm_steps,
            "measurements": int(len(p["meas_steps"])),
            "path": "fp32-split fused temporally blocked", "k": info.k, "tile": info.tile,
            "autotuned": bool(info.autotuned), "graphs": not args.no_graph,
        },
        "roofline": roof,
    }
    progress("timed run:", round(wall, 3), "s")
    # 3. The FP64 plain one-step path on a window with the same measurement density.
    if not args.skip_plain:
        line["fp64_plain"] = plain_leg(qew, args, H, gflags)
        line["speedup_vs_fp64_plain"] = round(value / line["fp64_plain"]["value"], 3)
    line.update(line_extra)
    print(json.dumps(line), flush=True)


def plain_leg(qew, args, H, gflags):
    """The FP64 plain one-step path timed on a window of the workload with
    the full run's measurement density."""
    win = H if args.plain_window <= 0 else min(int(args.plain_window), H)
    progress("FP64 plain path over", win, "Euler steps")
    pp = bench_problem(H) if win == H else window_problem(win)
    out2, st2, info2, wall2 = time_path(qew, pp, qew.QEW_FP64_PLAIN, qew.QEW_ONE_STEP, 64, flags=gflags)
    return {
        "value": round(info2.total_sites * win / wall2, 1), "unit": "site-updates/s", "euler_steps_timed": win,
        "measurements": int(len(pp["meas_steps"])),
        "window": "the whole horizon" if win == H else
                  f"Euler steps 1..{win} of the workload with {len(pp['meas_steps'])} log-spaced "
                  f"measurements (the full run's 200 per 10^6 steps); the plain kernel's cost per "
                  f"step does not depend on the state, so the rate holds for the whole horizon",
        "ms_per_euler_step": round(wall2 * 1e3 / win, 6),
        "roofline": plain_roofline(st2, info2, win),
    }


if __name__ == "__main__":
    main()
