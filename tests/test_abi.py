"""CPU checks of the C ABI: the library loads, exports every function the
header declares, and qew_plan validates problems on the host (no GPU call)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1211_7275_amd import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qew.h")

qew = pytest.importorskip("paper_1211_7275_amd.qew", reason="libqew.so not built")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(qew_[a-z_]+)\s*\(", text)
    return sorted(set(names))


def test_header_functions_exported():
    names = _declared_functions()
    assert len(names) >= 12
    lib = qew.lib()
    for n in names:
        assert hasattr(lib, n), f"{n} declared in qew.h but not exported"
    assert set(names) == set(qew.EXPORTS)


def test_library_is_gfx950_hip():
    out = os.popen(f"/opt/rocm/llvm/bin/llvm-readelf -S {qew.LIB_PATH} 2>/dev/null").read()
    assert ".hip_fatbin" in out or "hip_fatbin" in out


def _plan_status(p, **kw):
    pr, keep = qew.make_problem(p, **kw)
    h = ctypes.c_void_p()
    st = qew.lib().qew_plan(ctypes.byref(pr), ctypes.byref(h))
    if st == 0:
        qew.lib().qew_plan_destroy(h)
    return st, qew.qew_last_error()


def _base():
    return workloads.custom(0, [64, 100], 1.0, 100, [0, 10, 100], 123)


def test_plan_accepts_valid_problem():
    st, _ = _plan_status(_base())
    assert st == 0
    st, _ = _plan_status(_base(), precision=qew.QEW_FP64_PLAIN, path=qew.QEW_ONE_STEP)
    assert st == 0


@pytest.mark.parametrize("mutate,expect", [
    (lambda p: p.update(L=np.array([2, 64])), qew.QEW_EINVAL),
    (lambda p: p.update(L=np.array([64, 2**31])), qew.QEW_EINVAL),
    (lambda p: p.update(c=0.0), qew.QEW_EINVAL),
    (lambda p: p.update(dt=-0.1), qew.QEW_EINVAL),
    (lambda p: p.update(dt=0.6), qew.QEW_EINVAL),           # c*dt > 1/2
    (lambda p: p.update(strength=-1.0), qew.QEW_EINVAL),
    (lambda p: p.update(strength=float("nan")), qew.QEW_EINVAL),
    (lambda p: p.update(kind=7), qew.QEW_EINVAL),
    (lambda p: p.update(n_steps=-1), qew.QEW_EINVAL),
    (lambda p: p.update(meas_steps=np.array([0, 10, 10])), qew.QEW_EINVAL),
    (lambda p: p.update(meas_steps=np.array([5, 3])), qew.QEW_EINVAL),
    (lambda p: p.update(meas_steps=np.array([0, 101])), qew.QEW_EINVAL),
    (lambda p: p.update(f=np.array([1.0, np.inf])), qew.QEW_EINVAL),
])
def test_plan_rejects_bad_problems(mutate, expect):
    p = _base()
    mutate(p)
    st, msg = _plan_status(p)
    assert st == expect
    assert msg


def test_plan_rejects_bad_path_options():
    p = _base()
    assert _plan_status(p, precision=qew.QEW_FP64_PLAIN, path=qew.QEW_FUSED)[0] == qew.QEW_EUNSUPPORTED
    assert _plan_status(p, k=129)[0] == qew.QEW_EINVAL
    assert _plan_status(p, tile=700)[0] == qew.QEW_EINVAL
    assert _plan_status(p, k=64, tile=1024)[0] == 0
    assert _plan_status(p, k=128, tile=2048)[0] == 0
    assert _plan_status(p, tile=512)[0] == qew.QEW_EINVAL
    assert _plan_status(p, k=130, tile=4096)[0] == qew.QEW_EINVAL
    assert _plan_status(p, flags=64)[0] == qew.QEW_EINVAL
    assert _plan_status(p, precision=5)[0] == qew.QEW_EINVAL
    assert _plan_status(p, flags=qew.QEW_FLAG_FUSED_DENSE)[0] == 0
    assert _plan_status(p, flags=qew.QEW_FLAG_FUSED_SPARSE)[0] == 0
    assert _plan_status(p, flags=qew.QEW_FLAG_FUSED_DENSE | qew.QEW_FLAG_FUSED_SPARSE)[0] == qew.QEW_EINVAL
    # the variant flags belong to the fused path
    for fl in (qew.QEW_FLAG_FUSED_DENSE, qew.QEW_FLAG_FUSED_SPARSE):
        for prec in (qew.QEW_FP32_SPLIT, qew.QEW_FP64_PLAIN):
            st, msg = _plan_status(p, precision=prec, path=qew.QEW_ONE_STEP, flags=fl)
            assert st == qew.QEW_EINVAL and "fused path only" in msg


def test_plan_null_arguments():
    lib = qew.lib()
    h = ctypes.c_void_p()
    assert lib.qew_plan(None, ctypes.byref(h)) == qew.QEW_EINVAL
    pr, keep = qew.make_problem(_base())
    assert lib.qew_plan(ctypes.byref(pr), None) == qew.QEW_EINVAL
    pr.L = None
    assert lib.qew_plan(ctypes.byref(pr), ctypes.byref(h)) == qew.QEW_EINVAL
    assert lib.qew_workspace_bytes(None) == 0
    lib.qew_plan_destroy(None)


def test_plan_info_and_workspace_size():
    p = workloads.custom(0, [1024, 3000, 70000], 1.0, 10, [10], 1)
    pr, keep = qew.make_problem(p, k=16, tile=1024)  # 1024-site workgroup tiles
    plan = qew.qew_plan(pr)
    try:
        info = qew.qew_plan_info_get(plan)
        assert info.total_sites == 1024 + 3000 + 70000
        assert info.padded_sites == 1024 + 3008 + 70016
        V = 1024 - 32
        assert info.n_tiles == sum(-(-L // V) for L in (1024, 3000, 70000))
        assert info.n_meas_tiles == 1 + 1 + 18
        assert info.k == 16 and info.tile == 1024
        ws = qew.qew_workspace_bytes(plan)
        # state (2 x 8 B) + node cache (2 x 16 B) per padded site, plus tables
        assert ws >= info.padded_sites * 48
        assert ws < info.padded_sites * 48 + 1 << 20
    finally:
        qew.qew_plan_destroy(plan)


def test_run_rejects_small_or_missing_workspace():
    p = _base()
    pr, keep = qew.make_problem(p, precision=qew.QEW_FP64_PLAIN, path=qew.QEW_ONE_STEP)
    plan = qew.qew_plan(pr)
    try:
        lib = qew.lib()
        need = qew.qew_workspace_bytes(plan)
        assert lib.qew_run(plan, None, need, None, 0, None, None, None) == qew.QEW_EINVAL
        assert lib.qew_run(plan, 256, need - 1, None, 0, None, None, None) == qew.QEW_ENOMEM
        assert lib.qew_run(plan, 257, need, None, 0, None, None, None) == qew.QEW_EINVAL
        assert lib.qew_run(plan, 256, need, None, 1, None, None, None) == qew.QEW_EINVAL  # no state
        assert lib.qew_debug_philox_fill(None, 0, None, -1, None) == qew.QEW_EINVAL
        assert lib.qew_debug_philox_fill(None, 0, None, 5, None) == qew.QEW_EINVAL
    finally:
        qew.qew_plan_destroy(plan)


def test_plan_structure_factor_options():
    """S_q needs equal power-of-two lengths and valid mode bins; it adds the
    FFT buffers and the [n_meas][bins] series to the workspace."""
    good = workloads.custom(0, [64, 64], 1.0, 100, [0, 10, 100], 123, sq_edges=[1, 2, 5, 33])
    assert _plan_status(good)[0] == 0
    assert _plan_status(good, precision=qew.QEW_FP64_PLAIN, path=qew.QEW_ONE_STEP)[0] == 0
    for L, edges in (([64, 32], [1, 5]),          # unequal lengths
                     ([48, 48], [1, 5]),          # not a power of two
                     ([4, 4], [1, 2]),            # below 8
                     ([64, 64], [0, 5]),          # mode 0
                     ([64, 64], [1, 34]),         # beyond L/2 + 1
                     ([64, 64], [1, 5, 5]),       # empty bin
                     ([64, 64], [3, 2])):         # decreasing
        bad = workloads.custom(0, L, 1.0, 100, [0, 10, 100], 123, sq_edges=edges)
        st, msg = _plan_status(bad)
        assert st == qew.QEW_EINVAL and msg, (L, edges)
    plain = workloads.custom(0, [1024] * 3, 1.0, 100, [0, 10, 100], 123)
    with_sq = dict(plain, sq_edges=workloads.sq_edges_full(1024))
    sizes = []
    for p in (plain, with_sq):
        pr, keep = qew.make_problem(p, precision=qew.QEW_FP64_PLAIN, path=qew.QEW_ONE_STEP)
        h = qew.qew_plan(pr)
        sizes.append(qew.qew_workspace_bytes(h))
        qew.qew_plan_destroy(h)
    # two complex FP64 buffers of L/2 per sample, plus 3 x 513 bins
    assert sizes[1] - sizes[0] >= 2 * 3 * 512 * 16 + 3 * 513 * 8


def test_run_noalloc_rejects_before_any_device_work():
    """qew_run_noalloc refuses, on the host and before touching a device, a
    fused plan without a fixed geometry, a plan with structure-factor bins,
    and a plan whose tables, partials and series exceed its 8 MiB scratch."""
    lib = qew.lib()
    assert lib.qew_run_noalloc(None, None, 0, None, 0, None, None, None) == qew.QEW_EINVAL

    def status(p, **kw):
        pr, keep = qew.make_problem(p, **kw)
        h = ctypes.c_void_p()
        assert lib.qew_plan(ctypes.byref(pr), ctypes.byref(h)) == 0
        try:
            st = lib.qew_run_noalloc(h, None, 0, None, 0, None, None, None)
            return st, qew.qew_last_error()
        finally:
            lib.qew_plan_destroy(h)

    st, msg = status(_base())  # fused, k = tile = 0
    assert st == qew.QEW_EINVAL and "fixed fused geometry" in msg
    sq = workloads.custom(0, [64], 1.0, 10, [10], 1, sq_edges=workloads.sq_edges_full(64))
    st, msg = status(sq, k=8, tile=1024)
    assert st == qew.QEW_EUNSUPPORTED and "structure factor" in msg
    big = workloads.custom(0, [64] * 64, 1.0, 6000, np.arange(1, 6001), 1)  # 9.2 MB of series
    st, msg = status(big, precision=qew.QEW_FP64_PLAIN, path=qew.QEW_ONE_STEP)
    assert st == qew.QEW_ENOMEM and "scratch array holds 8388608" in msg


def test_critical_force_argument_checks():
    """qew_critical_force validates on the host before any device call."""
    lib = qew.lib()
    ptr = ctypes.c_void_p(256)  # never dereferenced: every case fails validation first

    def st(kind=1, strength=1.0, period=64, c=1.0, S=1, L=64, f_lo=0.0, f_hi=4.0, tol_f=1e-4,
           tol_force=1e-10, max_sweeps=1000, null=False):
        p = None if null else ptr
        return lib.qew_critical_force(kind, strength, 1, period, c, S, L, p, f_lo, f_hi, tol_f, tol_force,
                                      max_sweeps, p, p, p, None)

    assert st(kind=2) == qew.QEW_EUNSUPPORTED and "Catmull-Rom" in qew.qew_last_error()
    assert st(kind=3) == qew.QEW_EUNSUPPORTED
    assert st(period=0) == qew.QEW_EINVAL and "periodic" in qew.qew_last_error()
    assert st(strength=-1.0) == qew.QEW_EINVAL
    assert st(c=0.0) == qew.QEW_EINVAL
    assert st(S=0) == qew.QEW_EINVAL
    assert st(L=2) == qew.QEW_EINVAL and st(L=4097) == qew.QEW_EINVAL
    assert st(f_lo=1.0, f_hi=1.0) == qew.QEW_EINVAL
    assert st(f_hi=float("inf")) == qew.QEW_EINVAL
    assert st(tol_f=0.0) == qew.QEW_EINVAL and st(tol_force=-1.0) == qew.QEW_EINVAL
    assert st(max_sweeps=3) == qew.QEW_EINVAL
    assert st(tol_f=1e-300) == qew.QEW_EINVAL and "200" in qew.qew_last_error()
    assert st(null=True) == qew.QEW_EINVAL
