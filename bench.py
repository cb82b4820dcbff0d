#!/usr/bin/env python3
"""Benchmark of one PSATD step (guard fill + FFT + k-space push + inverse FFT + merge) on one MI355X.

Workload: one group of the hybrid solver on one GPU -- a 512 x 256 x 256 cell
periodic grid G1 with 32 guard cells per side and axis (box 576 x 320 x 320),
order p = 100 modified wavenumbers, dt = dx / (2c), FP32.  Inputs are seeded
and synthetic: a Gaussian laser pulse (wavelength 16 dx, waist 40 dx, length
3 wavelengths) plus N(0, 0.01) noise on E and B, J and rho from 1e6
random-walk macro-particles deposited with cloud-in-cell weights.

One step = one psatd_step_g1 call on inputs already resident in HBM.  The same
workload is also timed in FP64.  Prints ONE JSON line (rank 0, N = 1).
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "cell-updates/s per PSATD step (FP32 vs FP64) + % HBM roofline, 1 MI355X"
INTERIOR = (512, 256, 256)  # x, y, z
NGUARD = 32
ORDER = 100
DX = 1.0
DT = 0.5
PASSES = ("x_fwd_fill", "y_fwd", "z_push", "y_inv", "x_inv_merge")
# Kernels of each pass: the run-time-schedule kernel, or the one compiled for the two-stage
# line schedule (the plan reports which one each pass uses).
KERNELS = {"x_fwd_fill": ("k_xfwd", "k_xfwd2"), "y_fwd": ("k_ypass<-1>", "k_ypass2<-1>"),
           "z_push": ("k_zpush", "k_zpush2"), "y_inv": ("k_ypass<1>", "k_ypass2<1>"),
           "x_inv_merge": ("k_xinv", "k_xinv2")}


def pass_of_kernel(name):
    """The step pass a single-box pass kernel belongs to (None for other kernels)."""
    import re

    m = re.search(r"k_(xfwd|ypass|zpush|xinv)(2?)(_b)?<(-?1)?", name)
    if not m or m.group(3):
        return None
    kind = m.group(1)
    if kind == "ypass":
        return "y_fwd" if m.group(4) == "-1" else "y_inv"
    return {"xfwd": "x_fwd_fill", "zpush": "z_push", "xinv": "x_inv_merge"}[kind]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_inputs(interior, d, dt, seed_stream=0):
    """(11, NZ, NY, NX) float64 host array of the seeded laser + noise + macro-particle workload."""
    import synth

    nx, ny, nz = interior
    shape = (nz, ny, nx)
    rng = synth.rng_for(2, seed_stream)
    lam = 16.0 * d
    out = np.empty((11,) + shape)
    E, B = synth.laser_pulse(shape, d, wavelength=lam, waist=40.0 * d, length=3 * lam, x_center=0.5 * nx * d)
    out[0:3] = E
    out[3:6] = B
    del E, B
    for i in range(6):
        out[i] += rng.normal(0.0, 0.01, size=shape)
    J, rho_old, rho_new = synth.macro_particle_deposit(rng, shape, d, dt, 1_000_000, q=0.1)
    out[6:9] = J
    out[9] = rho_old
    out[10] = rho_new
    return out


def algorithmic_bytes(box, interior, ng, s):
    """Bytes each pass must move per launch (reads + writes), s = bytes per real.

    Units: NX*NY*NZ box cells, npts = (NX/2+1)*NY*NZ half-spectrum points.
    x_fwd_fill reads 11 real fields over the box and writes 11 half spectra;
    y_fwd reads and writes 11 half spectra; z_push reads 11 half spectra and the
    5 coefficient tables and writes 6 half spectra for the interior z range;
    y_inv reads those and writes the interior (y, z) lines; x_inv_merge reads
    them and writes the interior cells of 6 fields.
    """
    NX, NY, NZ = box
    nx, ny, nz = interior
    nxh = NX // 2 + 1
    c = 2 * s
    npts = nxh * NY * NZ
    return {
        "x_fwd_fill": 11 * NX * NY * NZ * s + 11 * npts * c,
        "y_fwd": 2 * 11 * npts * c,
        "z_push": 11 * npts * c + 5 * npts * s + 6 * nxh * NY * nz * c,
        "y_inv": 6 * nxh * NY * nz * c + 6 * nxh * ny * nz * c,
        "x_inv_merge": 6 * nxh * ny * nz * c + 6 * nx * ny * nz * s,
    }


def compulsory_bytes(box, s):
    """Bytes one step cannot avoid: read E, B, J, rho_old, rho_new (11 arrays) and write E, B (6)
    once per box cell, 17 s per cell (68 B in FP32, 136 B in FP64)."""
    return 17 * s * box[0] * box[1] * box[2]


def source_digest():
    """Digest of the pass kernels' source with comments and blank space removed."""
    import re

    h = hashlib.sha256()
    for name in ("passes.hip", "fft_lds.hpp", "cplx.hpp", "internal.hpp", "gmem.hpp"):
        with open(os.path.join(ROOT, "paper_1812_07357_amd", "csrc", name)) as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def traffic_from_profile(kernel_pass, digest):
    """HBM bytes per launch measured by rocprofv3 counters, if taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic_config2_fp32.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_digest") != digest:
        return None
    entry = rec.get("passes", {}).get(kernel_pass)
    return None if entry is None else entry.get("bytes_per_launch")


def run_gpu(precision, inputs_host, steps, warmup, staggered=False):
    import torch

    from paper_1812_07357_amd import psatd

    nx, ny, nz = INTERIOR
    dtype = torch.float64 if precision == "fp64" else torch.float32
    plan = psatd.Plan(nx, ny, nz, nguard=NGUARD, order=ORDER, dx=DX, dt=DT, precision=precision,
                      staggered=staggered)
    plan.autotune()
    schedule = {"xyz"[a]: plan.schedule(a) for a in range(3)}
    schedule["two_stage_passes"] = [PASSES[i] for i in range(5) if (plan.query(psatd.Q_TWO_STAGE) >> i) & 1]
    g1 = torch.as_tensor(inputs_host, dtype=dtype).to("cuda")
    origin = (0, 0, 0)
    for _ in range(warmup):
        plan.step_g1(g1, origin)
    torch.cuda.synchronize()
    plan.set_timing(True)
    plan.pass_times()  # discard anything recorded so far
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.step_g1(g1, origin)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    passes, nrec = plan.pass_times()
    plan.set_timing(False)
    ms = (t1 - t0) * 1e3 / steps
    mask = plan.query(psatd.Q_TWO_STAGE)
    kernels = {pas: KERNELS[pas][(mask >> i) & 1] for i, pas in enumerate(PASSES)}
    res = {"ms_per_step": ms, "passes_ms": passes, "recorded_steps": nrec, "box": plan.box, "kernels": kernels,
           "workspace_bytes": plan.query(psatd.Q_WORKSPACE_BYTES), "schedule": schedule}
    fields = g1[0:6].clone()
    plan.close()
    del g1
    torch.cuda.empty_cache()
    return res, fields


def host_cpu():
    """(model name, logical cores usable by this process) of the host."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    return model, cores


def cpu_baseline(nsteps=2, runs=3):
    """The FP64 oracle on a half-scale copy of the workload: ``nsteps`` local steps of a
    256 x 128 x 128 grid with 16 guards (box 288 x 160 x 160, same box/interior ratio),
    its library FFTs on every host core; the median of ``runs`` timed runs."""
    import oracle.step
    from oracle import domain

    model, cores = host_cpu()
    oracle.step.WORKERS = cores
    interior = (256, 128, 128)
    g1 = make_inputs(interior, DX, DT, seed_stream=7)
    box = {"origin": (0, 0, 0), "interior": interior, "nguard": 16, "order": ORDER}
    times = []
    for _ in range(runs):
        t0 = time.perf_counter()
        domain.local_steps(g1, [box], nsteps, DX, DT)
        times.append(time.perf_counter() - t0)
    t = float(np.median(times))
    cells = interior[0] * interior[1] * interior[2] * nsteps
    return {"value": cells / t, "unit": "cell-updates/s", "cores": cores, "kind": "oracle",
            "cpu_model": model, "runs_s": [round(v, 2) for v in times],
            "sample": f"median of {runs} runs of {nsteps} FP64 oracle steps (complex FFTs on {cores} threads, "
                      f"numpy push on one) on a 256x128x128 grid + 16 guards (box 288x160x160, same "
                      f"box/interior ratio as the workload), {t:.1f} s each"}


def run_batch(steps):
    """64 uneven boxes (edges 32..96 + guards 8..64, orders 16..64), FP32: graph of `steps` steps vs eager."""
    import torch

    import synth
    from paper_1812_07357_amd import psatd

    rng = synth.rng_for(3, 0)
    gdims, boxes = synth.uneven_decomposition(rng)
    # fields seeded like the 32^3 case: plane waves on the global grid and a Gaussian current
    host = synth.plane_waves_and_blob(synth.rng_for(3, 1), gdims[::-1], DX, 4, mmax=8).astype(np.float32)
    batch = psatd.Batch(boxes, gdims, dx=DX, dt=DT)
    batch.autotune()
    g = torch.as_tensor(host, device="cuda")
    batch.run(g, steps)                     # capture + first replay (warm-up)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batch.run(g, steps)
    torch.cuda.synchronize()
    t_graph = (time.perf_counter() - t0) / steps
    t0 = time.perf_counter()
    for _ in range(steps):
        batch.step(g)
    torch.cuda.synchronize()
    t_eager = (time.perf_counter() - t0) / steps
    interior = batch.query(psatd.QB_INTERIOR_CELLS)
    boxc = batch.query(psatd.QB_BOX_CELLS)
    batch.close()
    five = comp = 0
    for b in boxes:
        ng = b["nguard"]
        bx = tuple(n + 2 * ng for n in b["interior"])
        five += sum(algorithmic_bytes(bx, b["interior"], ng, 4).values())
        comp += compulsory_bytes(bx, 4)
    return {"boxes": len(boxes), "global": list(gdims), "steps_per_graph": steps, "box_cells": boxc,
            "interior_cell_updates_per_s": interior / t_graph, "box_cell_updates_per_s": boxc / t_graph,
            "ms_per_step_graph": t_graph * 1e3, "ms_per_step_eager": t_eager * 1e3,
            "step_compulsory_hbm_frac": round(comp / t_graph / 1e9 / HBM_PEAK_GBS, 4),
            "step_5pass_hbm_frac": round(five / t_graph / 1e9 / HBM_PEAK_GBS, 4)}


def pic_particles(ppc, u_rms, seed=4):
    """Cell-ordered warm plasma on the benchmark grid, drawn on the GPU: particle p sits in
    cell p // ppc (x fastest) at a uniform position inside it, with Gaussian momenta."""
    import torch

    nx, ny, nz = INTERIOR
    n = ppc * nx * ny * nz
    gen = torch.Generator(device="cuda").manual_seed(seed)
    cell = torch.arange(n, device="cuda", dtype=torch.int64) // ppc
    x = torch.empty((3, n), dtype=torch.float32, device="cuda")
    x[0] = (cell % nx).float()
    x[1] = ((cell // nx) % ny).float()
    x[2] = (cell // (nx * ny)).float()
    del cell
    x += torch.rand((3, n), generator=gen, device="cuda")
    x *= DX
    top = torch.tensor([nx * DX, ny * DX, nz * DX], device="cuda")[:, None]
    x = torch.minimum(x, torch.nextafter(top, torch.zeros_like(top)))
    u = u_rms * torch.randn((3, n), generator=gen, device="cuda")
    return x.contiguous(), u.contiguous()


def run_pic(inputs_host, steps, warmup, ppc=2):
    """PIC cycle on the benchmark group, FP32: gather + Boris push, deposit through 8^3 D1
    tiles, the PSATD step on the 576x320x320 FFT box (D2), each timed with HIP events."""
    import torch

    from paper_1812_07357_amd import psatd

    nx, ny, nz = INTERIOR
    ncell = nx * ny * nz
    plan = psatd.Plan(nx, ny, nz, nguard=NGUARD, order=ORDER, dx=DX, dt=DT, precision="fp32")
    plan.autotune()
    x, u = pic_particles(ppc, 0.05)
    n = x.shape[1]
    pic = psatd.Pic(INTERIOR, dx=DX, dt=DT, q=-0.01 / ppc, q_over_m=-1.0, max_particles=n, tile=8)
    g1 = torch.as_tensor(inputs_host, dtype=torch.float32).to("cuda")
    xo = torch.empty_like(x)
    origin = (0, 0, 0)
    for _ in range(warmup):
        pic.push(g1, x, u, xo)
        pic.deposit(g1, xo, x, u)
        plan.step_g1(g1, origin)
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]
    t0 = time.perf_counter()
    for k in range(steps):
        ev[k][0].record()
        pic.push(g1, x, u, xo)
        ev[k][1].record()
        pic.deposit(g1, xo, x, u)
        ev[k][2].record()
        plan.step_g1(g1, origin)
        ev[k][3].record()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    push = sum(e[0].elapsed_time(e[1]) for e in ev) / steps
    dep = sum(e[1].elapsed_time(e[2]) for e in ev) / steps
    stp = sum(e[2].elapsed_time(e[3]) for e in ev) / steps
    plan.close()
    pic.close()
    # push and deposit of the wider B-spline shapes (degree 2, 3), each on a fresh copy of the
    # initial particles (those of the cycle above have been accelerated by the laser)
    shapes = {}
    del x, u
    torch.cuda.empty_cache()
    for shape in (2, 3):
        x, u = pic_particles(ppc, 0.05)
        ps = psatd.Pic(INTERIOR, dx=DX, dt=DT, q=-0.01 / ppc, q_over_m=-1.0, max_particles=n, tile=8, shape=shape)
        ps.push(g1, x, u, xo)
        ps.deposit(g1, xo, x, u)
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(3)]
        for e in evs:
            e[0].record()
            ps.push(g1, x, u, xo)
            e[1].record()
            ps.deposit(g1, xo, x, u)
            e[2].record()
        torch.cuda.synchronize()
        shapes[f"degree_{shape}"] = {"push_ms": round(sum(e[0].elapsed_time(e[1]) for e in evs) / 3, 4),
                                     "deposit_ms": round(sum(e[1].elapsed_time(e[2]) for e in evs) / 3, 4)}
        ps.close()
    del g1, x, u, xo
    torch.cuda.empty_cache()
    s = 4
    # compulsory bytes: push reads x, u and writes x, u, x_old (15 s per particle) and reads E, B once
    # (6 s per cell); deposit reads x_old, x, u (9 s per particle) and writes J, rho_old, rho_new once
    push_bytes = 15 * s * n + 6 * s * ncell
    dep_bytes = 9 * s * n + 5 * s * ncell
    return {"particles": n, "ppc": ppc, "tile": 8, "ms_per_cycle": ms, "push_ms": round(push, 4),
            "deposit_ms": round(dep, 4), "maxwell_step_ms": round(stp, 4),
            "particle_pushes_per_s": n / (ms * 1e-3),
            "push_hbm_frac": round(push_bytes / (push * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "deposit_hbm_frac": round(dep_bytes / (dep * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "higher_order_shapes": shapes,
            "note": "cell-ordered warm plasma (u_rms 0.05 c), ppc particles per cell of the 512x256x256 grid; "
                    "the cycle uses degree-1 (cloud-in-cell) shapes"}


def run_pml(steps, warmup=2, width=32):
    """Two-step PML step (12 split parts) on the 576x320x320 box with layers of `width` cells at
    both ends of every axis, FP32; the split parts start as the laser recipe's E, B in set A."""
    import torch

    from paper_1812_07357_amd import psatd

    box = (INTERIOR[0] + 2 * NGUARD, INTERIOR[1] + 2 * NGUARD, INTERIOR[2] + 2 * NGUARD)
    plan = psatd.Plan(*box, nguard=0, order=ORDER, dx=DX, dt=DT, precision="fp32")
    plan.autotune()
    plan.pml_set((width, width, width), 3.0 * np.log(1e4) / (2 * width * DX), 2.0)
    shape = plan.box_shape
    gen = torch.Generator(device="cuda").manual_seed(5)
    parts = torch.zeros((12,) + shape, device="cuda")
    parts[0:6] = 0.01 * torch.randn((6,) + shape, generator=gen, device="cuda")
    src = torch.zeros((5,) + shape, device="cuda")
    for _ in range(warmup):
        plan.pml_step(parts, src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.pml_step(parts, src)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    plan.close()
    del parts, src
    torch.cuda.empty_cache()
    cells = box[0] * box[1] * box[2]
    return {"box": list(box), "layer_cells": width, "ms_per_step": ms, "box_cell_updates_per_s": cells / (ms * 1e-3),
            "note": "12 split parts: forward x, y and z passes once (the z pass writes both split sets), "
                    "inverse y and x passes per set, plus the sum and damping kernels"}


def summarize_pmc(directory, steps, out_json):
    """HBM traffic per launch of each pass from rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE runs of this script.

    Both counters are in KiB per dispatch.  They are calibrated by the 1 GiB
    read + 1 GiB write of the --calibration-copy kernel (torch.neg) in the same
    runs; only the last ``steps`` dispatches of each pass kernel (the timed
    steps, after autotuning and warm-up) are averaged.
    """
    import csv
    import glob

    per = {"FETCH_SIZE": {}, "WRITE_SIZE": {}}
    calib = {}
    for path in glob.glob(os.path.join(directory, "**", "*counter_collection.csv"), recursive=True):
        with open(path) as f:
            for r in csv.DictReader(f):
                c = r["Counter_Name"]
                if c not in per:
                    continue
                k = r["Kernel_Name"]
                v = float(r["Counter_Value"])
                if "neg_kernel" in k:
                    calib[c] = v
                    continue
                pas = pass_of_kernel(k)
                if pas is not None:
                    per[c].setdefault(pas, []).append((int(r["Dispatch_Id"]), v))
    if set(calib) != {"FETCH_SIZE", "WRITE_SIZE"}:
        raise SystemExit("calibration kernel (neg) not found in both counter runs")
    gib_kib = float(1 << 20)
    factor = {c: gib_kib / calib[c] for c in calib}
    alg = algorithmic_bytes(tuple(n + 2 * NGUARD for n in INTERIOR), INTERIOR, NGUARD, 4)
    passes = {}
    for pas in PASSES:
        vals = {}
        for c in per:
            d = sorted(per[c].get(pas, []))[-steps:]
            vals[c] = sum(v for _, v in d) / len(d) if d else float("nan")
        b = 1024.0 * (vals["FETCH_SIZE"] * factor["FETCH_SIZE"] + vals["WRITE_SIZE"] * factor["WRITE_SIZE"])
        passes[pas] = {"fetch_kib": vals["FETCH_SIZE"], "write_kib": vals["WRITE_SIZE"],
                       "bytes_per_launch": round(b), "algorithmic_bytes": alg[pas], "ratio": round(b / alg[pas], 4)}
    rec = {"source_digest": source_digest(), "workload": "512x256x256 + 32 guards, order 100, FP32",
           "calibration": {"kernel": "torch.neg over 1 GiB (reads 1 GiB, writes 1 GiB)",
                           "fetch_kib": calib["FETCH_SIZE"], "write_kib": calib["WRITE_SIZE"],
                           "fetch_factor": round(factor["FETCH_SIZE"], 4),
                           "write_factor": round(factor["WRITE_SIZE"], 4)},
           "passes": passes}
    with open(out_json, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec, indent=1))


def run_extra(steps=20):
    """Timing of the other workloads (parity cases, not the headline) and of rocFFT on the same transforms.

    - 32^3 periodic grid, exact k (order 0), no guards, FP64 (launch-bound);
    - 1024x512x512 + 16 guards (box 1056x544x544), order 32, FP32 and FP64;
    - the 17 real 3D transforms of the 576x320x320 box alone (11 forward
      R2C, 6 inverse C2R) through torch.fft, i.e. rocFFT: a timing comparison,
      never part of the path.
    """
    import torch

    from paper_1812_07357_amd import psatd

    def time_plan(interior, ng, order, precision, nsteps):
        nx, ny, nz = interior
        plan = psatd.Plan(nx, ny, nz, nguard=ng, order=order, dx=DX, dt=DT, precision=precision)
        dtype = torch.float64 if precision == "fp64" else torch.float32
        g = torch.randn((11, nz, ny, nx), dtype=dtype, device="cuda")
        for _ in range(3):
            plan.step_g1(g, (0, 0, 0))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(nsteps):
            plan.step_g1(g, (0, 0, 0))
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / nsteps
        box = plan.box
        plan.close()
        del g
        torch.cuda.empty_cache()
        return {"ms_per_step": ms, "interior_cell_updates_per_s": nx * ny * nz / (ms * 1e-3),
                "box_cell_updates_per_s": box[0] * box[1] * box[2] / (ms * 1e-3)}

    out = {"32^3 exact k FP64": time_plan((32, 32, 32), 0, 0, "fp64", 10 * steps)}
    for prec in ("fp32", "fp64"):
        out[f"1024x512x512+16 p=32 {prec.upper()}"] = time_plan((1024, 512, 512), 16, 32, prec, steps)
    nx, ny, nz = (n + 2 * NGUARD for n in INTERIOR)
    for prec, dtype in (("FP32", torch.float32), ("FP64", torch.float64)):
        a = torch.randn((11, nz, ny, nx), dtype=dtype, device="cuda")
        for _ in range(2):
            spec = torch.fft.rfftn(a, dim=(1, 2, 3))
            back = torch.fft.irfftn(spec[0:6], s=(nz, ny, nx), dim=(1, 2, 3))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            spec = torch.fft.rfftn(a, dim=(1, 2, 3))
            back = torch.fft.irfftn(spec[0:6], s=(nz, ny, nx), dim=(1, 2, 3))
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        out[f"rocFFT 17 transforms of the 576x320x320 box {prec}"] = {
            "ms": ms, "note": "transforms only (no push, no guard fill/merge), torch.fft on ROCm"}
        del a, spec, back
        torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-staggered", action="store_true")
    ap.add_argument("--no-pic", action="store_true")
    ap.add_argument("--no-pml", action="store_true")
    ap.add_argument("--calibration-copy", action="store_true",
                    help="run one plain 1 GiB device copy first (reference for HBM byte counters)")
    ap.add_argument("--extra", action="store_true",
                    help="also time the 32^3 and 1024x512x512 workloads and rocFFT on the same transforms")
    ap.add_argument("--summarize-pmc", metavar="DIR",
                    help="write profiles/hbm_traffic_config2_fp32.json from rocprofv3 --pmc runs under DIR and exit")
    args = ap.parse_args()
    if args.summarize_pmc:
        summarize_pmc(args.summarize_pmc, args.steps,
                      os.path.join(ROOT, "profiles", "hbm_traffic_config2_fp32.json"))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the PSATD step of one group runs on a single MI355X "
              "(multi-GPU groups are not part of this build); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    log("generating inputs")
    host = make_inputs(INTERIOR, DX, DT)
    nx, ny, nz = INTERIOR
    interior_cells = nx * ny * nz

    if args.calibration_copy:
        # A plain streaming kernel that reads 1 GiB and writes 1 GiB (b = -a):
        # under a counter profiler its FETCH_SIZE / WRITE_SIZE calibrate the
        # counters against known bytes.
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.neg(a, out=b)
        torch.cuda.synchronize()
        del a, b
        log("calibration copy of 1 GiB done")

    log("fp32 run")
    r32, f32 = run_gpu("fp32", host, args.steps, args.warmup)
    box = r32["box"]
    box_cells = box[0] * box[1] * box[2]
    value = interior_cells / (r32["ms_per_step"] * 1e-3)

    digest = source_digest()
    alg = algorithmic_bytes(box, INTERIOR, NGUARD, 4)
    dom = max(PASSES, key=lambda k: r32["passes_ms"][k])
    dom_ms = r32["passes_ms"][dom]
    achieved = alg[dom] / (dom_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic_from_profile(dom, digest),
                "kernel": r32["kernels"][dom], "pass": dom, "kernel_ms": round(dom_ms, 4),
                "algorithmic_bytes_per_launch": alg[dom]}
    step_alg = sum(alg.values())

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r32["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "PSATD step of one group: 512x256x256 interior + 32 guards per side "
                               "(box 576x320x320), order 100, dt=dx/2c, FP32, fused guard fill/merge",
                   "interior": list(INTERIOR), "nguard": NGUARD, "order": ORDER, "box": list(box), "dt": DT},
        "roofline": roofline,
        "box_cell_updates_per_s": box_cells / (r32["ms_per_step"] * 1e-3),
        "passes_ms_fp32": {k: round(v, 4) for k, v in r32["passes_ms"].items()},
        # compulsory bytes: read the 11 input arrays and write E, B once per box cell (68 B in FP32)
        "step_compulsory_hbm_frac_fp32": round(compulsory_bytes(box, 4) / (r32["ms_per_step"] * 1e-3) / 1e9
                                               / HBM_PEAK_GBS, 4),
        # the five passes' own reads and writes (intermediate spectra included)
        "step_5pass_hbm_frac_fp32": round(step_alg / (r32["ms_per_step"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "source_digest": digest,
        "schedule_fp32": r32["schedule"],
    }

    if not args.no_fp64:
        log("fp64 run")
        r64, f64 = run_gpu("fp64", host, args.steps, args.warmup)
        alg64 = algorithmic_bytes(box, INTERIOR, NGUARD, 8)
        out["fp64"] = {
            "value": interior_cells / (r64["ms_per_step"] * 1e-3),
            "ms_per_step": r64["ms_per_step"],
            "passes_ms": {k: round(v, 4) for k, v in r64["passes_ms"].items()},
            "step_compulsory_hbm_frac": round(compulsory_bytes(box, 8) / (r64["ms_per_step"] * 1e-3) / 1e9
                                              / HBM_PEAK_GBS, 4),
            "step_5pass_hbm_frac": round(sum(alg64.values()) / (r64["ms_per_step"] * 1e-3) / 1e9
                                         / HBM_PEAK_GBS, 4),
        }
        out["fp32_speedup_over_fp64"] = r64["ms_per_step"] / r32["ms_per_step"]
        # FP32 vs FP64 error after warmup + steps steps of the same input, per vector field
        e = (f32.double() - f64)
        out["fp32_vs_fp64_rel_l2"] = {
            "steps": args.warmup + args.steps,
            "E": float(e[0:3].norm() / f64[0:3].norm()),
            "B": float(e[3:6].norm() / f64[3:6].norm()),
        }
        del f64, e
    del f32

    if not args.no_staggered:
        log("fp32 staggered-grid run")
        rs, fs = run_gpu("fp32", host, args.steps, args.warmup, staggered=True)
        del fs
        out["staggered_fp32"] = {"value": interior_cells / (rs["ms_per_step"] * 1e-3), "ms_per_step": rs["ms_per_step"],
                                 "passes_ms": {k: round(v, 4) for k, v in rs["passes_ms"].items()},
                                 "note": "same workload on the staggered (Yee) grid, PSATD_FLAG_STAGGERED"}

    if not args.no_pic:
        log("fp32 PIC cycle (push, deposit, step)")
        out["pic_fp32"] = run_pic(host, min(args.steps, 20), 2)

    if not args.no_pml:
        log("fp32 two-step PML step")
        out["pml_fp32"] = run_pml(min(args.steps, 20))

    if not args.no_batch:
        log("batch run (64 uneven boxes, hipGraph)")
        out["batch_fp32"] = run_batch(50)

    if args.extra:
        log("extra workloads and rocFFT comparison")
        out["extra"] = run_extra()

    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
