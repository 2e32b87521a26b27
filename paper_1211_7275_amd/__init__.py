"""MI355X-native quenched Edwards-Wilkinson relaxation engine (arXiv:1211.7275).

The hot path -- explicit Euler integration of the discretised QEW chain with
on-the-fly Philox/Catmull-Rom disorder and FP64 v(t), w^2(t) reductions -- runs
in the HIP library ``libqew.so`` behind the C ABI declared in
``include/qew.h``.  ``paper_1211_7275_amd.qew`` is the thin ctypes binding;
``paper_1211_7275_amd.workloads`` builds the seeded synthetic inputs.

Importing this package loads nothing; import ``qew`` to load the library.
"""
__all__ = ["qew", "workloads"]
