"""Host-instrumented build of libpsatd for CPU checks (AddressSanitizer + UndefinedBehaviorSanitizer).

Every unit is compiled for the host side only (``--offload-host-only``) with the
sanitizers on the host pass, so the library's host code -- argument checks, the
schedule builder, the autotuner cache reader, the resource hooks -- runs
instrumented on a machine without a GPU.  No kernel is compiled: the units'
references to their device code objects are bound to empty placeholders, so this
build can never launch anything and is only for host-side checks.  Then the C
driver ``host_abi_check.c`` is built against it.

Usage: python tests/sanitizer/build_host_san.py OUTDIR  (prints the driver path)
"""

from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_1812_07357_amd", "csrc")
HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang"

SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]
FLAGS = ["-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "--offload-host-only",
         f"-I{os.path.join(ROOT, 'include')}"]


def _units():
    out = []
    for u in range(1, 10):
        for prec in ("float", "double"):
            out.append(("passes.hip", f"passes_{u}_{prec}", [f"-DPSATD_UNIT={u}", f"-DPSATD_REAL={prec}"]))
    for src in ("tables.hip", "guards.hip", "plan.hip", "mlp.hip", "pic.hip", "pml.hip"):
        out.append((src, os.path.splitext(src)[0], []))
    return out


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"{' '.join(cmd[:3])} ... failed:\n{r.stderr[-4000:]}")
    return r.stdout


def build(outdir: str) -> str:
    os.makedirs(outdir, exist_ok=True)

    def one(unit):
        src, name, extra = unit
        obj = os.path.join(outdir, name + ".o")
        _run([HIPCC, *FLAGS, *SAN, *extra, "-c", os.path.join(CSRC, src), "-o", obj])
        return obj

    jobs = max(1, min(16, os.cpu_count() or 2))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(one, _units()))
    # placeholders for the device code objects that were not built
    syms = set()
    for o in objs:
        for line in _run(["nm", "-u", o]).splitlines():
            parts = line.split()
            if parts and parts[-1].startswith("__hip_fatbin"):
                syms.add(parts[-1])
    stub_c = os.path.join(outdir, "no_device_code.c")
    with open(stub_c, "w") as f:
        f.write("/* host-only build: no device code objects */\n")
        for s in sorted(syms):
            f.write(f"const unsigned char {s}[64] __attribute__((aligned(4096))) = {{0}};\n")
    stub_o = os.path.join(outdir, "no_device_code.o")
    _run(["gcc", "-c", "-fPIC", stub_c, "-o", stub_o])
    lib = os.path.join(outdir, "libpsatd_hostsan.so")
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *SAN, "-o", lib, *objs, stub_o])
    drv = os.path.join(outdir, "host_abi_check")
    _run([CLANG, "-g", "-O1", "-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=undefined",
          f"-I{os.path.join(ROOT, 'include')}", os.path.join(HERE, "host_abi_check.c"), "-o", drv,
          f"-L{outdir}", "-lpsatd_hostsan", f"-Wl,-rpath,{outdir}"])
    return drv


if __name__ == "__main__":
    print(build(sys.argv[1] if len(sys.argv) > 1 else os.path.join(ROOT, "_build_hostsan")))
