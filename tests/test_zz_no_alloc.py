"""qew_run_noalloc (the entry point that allocates nothing) against qew_run,
through the C ABI: two calls in a row on one GPU, the second with a smaller
problem, each compared with qew_run on the same problem.  Both entry points
run the same kernels in the same order, so the series, the final states and
the device ensemble averages must be equal bit for bit."""
import sys

import numpy as np
import pytest

from paper_1211_7275_amd import workloads

pytestmark = pytest.mark.gpu

SEED = workloads.SEED_BASE + 90


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def qew():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_1211_7275_amd import qew as q
    return q


def _run(qew, p, precision, path, k, tile, noalloc, resume_from=None):
    """Run p with either entry point; returns series, states and ensemble."""
    import torch
    sim = qew.Simulation(p, precision=precision, path=path, k=k, tile=tile)
    try:
        S, n = len(p["L"]), len(p["meas_steps"])
        v, w2, ub = (np.full((S, n), np.nan) for _ in range(3))
        resume = 0
        if resume_from is not None:
            step, states = resume_from
            for s, u in enumerate(states):
                sim.write_state(s, u, step)
            resume = 1
        call = qew.qew_run_noalloc if noalloc else qew.qew_run
        call(sim.plan, sim.ws, torch.cuda.current_stream(), resume, v, w2, ub)
        return {"v": v, "w2": w2, "ubar": ub, "u": [sim.read_state(s)[0] for s in range(S)],
                "ens": sim.ensemble(), "stats": sim.stats()}
    finally:
        sim.close()


def _same(a, b):
    for key in ("v", "w2", "ubar"):
        assert np.array_equal(a[key], b[key], equal_nan=True), key
    for s in range(len(a["u"])):
        assert np.array_equal(a["u"][s], b["u"][s]), s
    for key, val in a["ens"].items():
        assert np.array_equal(val, b["ens"][key], equal_nan=True), key


CASES = [
    # (name, problem, precision, path, k, tile)
    ("fused RF, 3 chains up to 70000 sites",
     workloads.custom(0, [5000, 70000, 1024], [0.9, 1.0, 1.3], 300, [0, 1, 2, 7, 33, 150, 299, 300], SEED),
     1, 1, 16, 1024),
    ("fused RB, 2 chains (smaller)",
     workloads.custom(1, [777, 3000], [2.0, 2.5], 120, [0, 5, 60, 120], SEED + 1), 1, 1, 8, 1024),
]


def test_noalloc_twice_in_a_row_matches_qew_run(qew):
    for name, p, prec, path, k, tile in CASES:
        say("noalloc vs qew_run:", name)
        ref = _run(qew, p, prec, path, k, tile, noalloc=False)
        got = _run(qew, p, prec, path, k, tile, noalloc=True)
        assert got["stats"].graph_launches == 0 and got["stats"].sparse_launches == 0
        _same(got, ref)


def test_noalloc_one_step_paths_and_resume(qew):
    """Both precisions of the one-step path, a larger and then a smaller
    problem, and a resumed run (the series before the restored step stay as
    the workspace held them)."""
    big = workloads.custom(3, [4096, 9000], 1.2, 200, workloads.log_steps(200, 12), SEED + 2)
    small = workloads.custom(2, [100], 1.7, 50, [0, 10, 50], SEED + 3)
    for prec in (0, 1):
        for p in (big, small):
            say("noalloc one-step precision", prec, "sites", int(np.sum(p["L"])))
            _same(_run(qew, p, prec, 0, 0, 0, noalloc=True), _run(qew, p, prec, 0, 0, 0, noalloc=False))
    half = _run(qew, dict(big, n_steps=90, meas_steps=big["meas_steps"][big["meas_steps"] <= 90]), 0, 0, 0, 0,
                noalloc=False)
    a = _run(qew, big, 0, 0, 0, 0, noalloc=True, resume_from=(90, half["u"]))
    b = _run(qew, big, 0, 0, 0, 0, noalloc=False, resume_from=(90, half["u"]))
    _same(a, b)
    assert np.all(np.isnan(a["v"][:, big["meas_steps"] < 90]))
