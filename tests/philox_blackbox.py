"""Independent Philox4x32-10 engine used as a black box to pin the oracle.

PyTorch ships a header-only Philox4x32-10 engine (``ATen/core/PhiloxRNGEngine.h``)
whose key is the 64-bit seed and whose counter is (offset, subsequence).  A
tiny C++ driver, compiled here at test time and never linked into anything
else, feeds it arbitrary (counter, key) pairs and prints the four output
words.  Nothing of that header is copied: it is only compiled and run.
"""
import os
import shutil
import subprocess
import tempfile

import numpy as np

_DRIVER = r"""
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdio>
#include <cstdint>
int main() {
  unsigned c0, c1, c2, c3, k0, k1;
  while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    uint64_t seed = (uint64_t)k0 | ((uint64_t)k1 << 32);
    uint64_t subsequence = (uint64_t)c2 | ((uint64_t)c3 << 32);
    uint64_t offset = (uint64_t)c0 | ((uint64_t)c1 << 32);
    at::philox_engine eng(seed, subsequence, offset);
    unsigned o0 = eng(), o1 = eng(), o2 = eng(), o3 = eng();
    std::printf("%08x %08x %08x %08x\n", o0, o1, o2, o3);
  }
  return 0;
}
"""

_exe = None


def _torch_include():
    try:
        import torch.utils.cpp_extension as ce
        incs = ce.include_paths()
    except Exception:
        return None
    for d in incs:
        if os.path.exists(os.path.join(d, "ATen", "core", "PhiloxRNGEngine.h")):
            return d
    return None


def available():
    return _torch_include() is not None and shutil.which("g++") is not None


def _build():
    global _exe
    if _exe is not None:
        return _exe
    d = tempfile.mkdtemp(prefix="philox_bb_")
    src = os.path.join(d, "bb.cpp")
    exe = os.path.join(d, "bb")
    with open(src, "w") as fh:
        fh.write(_DRIVER)
    subprocess.run(["g++", "-O1", "-std=c++17", "-I", _torch_include(), src, "-o", exe],
                   check=True)
    _exe = exe
    return exe


def philox(ctr, key):
    """ctr: [n][4] uint32, key: [n][2] uint32 -> [n][4] uint32."""
    ctr = np.asarray(ctr, np.uint32).reshape(-1, 4)
    key = np.asarray(key, np.uint32).reshape(-1, 2)
    lines = "\n".join(" ".join("%08x" % w for w in (*c, *k)) for c, k in zip(ctr, key))
    res = subprocess.run([_build()], input=lines + "\n", capture_output=True, text=True,
                         check=True)
    out = np.array([[int(w, 16) for w in ln.split()] for ln in res.stdout.strip().splitlines()],
                   dtype=np.uint32)
    return out.reshape(-1, 4)
