"""Build libpsatd.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_1812_07357_amd.build_lib [--incremental]  (or build() from Python).
Objects are compiled in parallel into _build/ and linked into
paper_1812_07357_amd/libpsatd.so.
"""

from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libpsatd.so")

ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")

# Packed FP32 instructions are disabled: the compiler forms them from plain
# float code, and some of their forms are not trusted on this hardware.
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
    f"-I{os.path.join(ROOT, 'include')}",
]

# (source, object name, extra flags).  passes.hip is compiled once per
# (pass, precision) unit, the run-time z kernels in four units, so that the large pass
# kernels build in parallel.
_PASS_UNITS = [(u, name, prec) for u, name in ((1, "xfwd"), (2, "ypass"), (3, "zpush"), (4, "zpush_batch"),
                                               (5, "xinv"), (6, "zpush_two_stage"), (7, "zpush_multi"),
                                               (8, "zpush_pml"), (9, "zpush_pml_multi"))
               for prec in ("float", "double")]
SOURCES = [("passes.hip", f"passes_{name}_{prec}", [f"-DPSATD_UNIT={u}", f"-DPSATD_REAL={prec}"])
           for u, name, prec in _PASS_UNITS]
SOURCES += [(src, os.path.splitext(src)[0], []) for src in ("tables.hip", "guards.hip", "plan.hip", "mlp.hip", "pic.hip", "pml.hip")]


def _compile(unit) -> str:
    src, name, extra = unit
    obj = os.path.join(BUILD, name + ".o")
    cmd = [HIPCC, *FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src} ({name}):\n{r.stderr[-8000:]}")
    return obj


def _stale(unit) -> bool:
    """True if the unit's object is missing or older than its source or any header."""
    src, name, _ = unit
    obj = os.path.join(BUILD, name + ".o")
    if not os.path.exists(obj):
        return True
    deps = [os.path.join(CSRC, src)] + [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hpp")]
    deps.append(os.path.join(ROOT, "include", "psatd.h"))
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(d) > t for d in deps)


def build(verbose: bool = True, incremental: bool = False) -> str:
    """Compile every unit (or, with ``incremental``, only the stale ones) and link the library."""
    os.makedirs(BUILD, exist_ok=True)
    units = [u for u in SOURCES if not incremental or _stale(u)]
    jobs = min(max(1, len(units)), max(1, (os.cpu_count() or 2)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        list(ex.map(_compile, units))
    objs = [os.path.join(BUILD, name + ".o") for _, name, _ in SOURCES]
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-8000:]}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}", file=sys.stderr)
    return LIB


if __name__ == "__main__":
    build(incremental="--incremental" in sys.argv[1:])
