"""GPU: the precision study on the 1024 x 512 x 512 + 16 guard box with sources.

Workload: order p = 32, dt = dx / 2c, 200 steps; E and B are 16 seeded plane
waves of the global grid, polarised orthogonally to their order-p wave vector
K_p (so div_p E = 0), and J is a seeded Gaussian current (sigma 3 cells, peak
0.1) held constant.  The charge follows continuity with the solver's own K_p
(rho_{n+1} = rho_n - dt div_p J, rho_0 = 0), advanced between steps, so the
push (Sec. 1.1 of arXiv:1812.07357: analytic integration, Gauss's law kept) is
fed consistent sources.

Three-way comparison:
* full size: FP32 against the FP64 GPU path after 200 steps, relative L2 per
  vector field, and the Gauss residual ||i K_p . E^ - rho^/eps0|| / ||rho^/eps0||
  of both (the local solve's box wraps onto the periodic grid, so the residual
  is the guard truncation error at the seam, not round-off);
* a 128^3 grid with one box of 16 guards (160^3), same order, plane waves and
  Gaussian current, sources fixed: the FP64 GPU path against the FP64 CPU
  oracle after 10 steps (<= 1e-12) and 200 steps (<= 1e-11), and the FP32 path
  against both.  The oracle results are stored by
  tests/golden/make_oracle_expected.py (200 oracle steps take minutes).
"""

import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def _golden_module():
    import importlib.util

    spec = importlib.util.spec_from_file_location("make_oracle_expected",
                                                  os.path.join(HERE, "golden", "make_oracle_expected.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _full_size_inputs(gshape, d, order, nmodes, rng):
    """(11, ...) FP64 GPU tensor: transverse plane waves (w.r.t. K_p) + Gaussian J; rho zero."""
    import torch

    from oracle import kspace

    nz, ny, nx = gshape
    dims = np.array([nx, ny, nz])
    pw = synth.plane_wave_modes(rng, gshape, nmodes, mmax=16)
    kvec = 2 * np.pi * pw["m"] / (dims * d)
    kp = np.stack([kspace.modified_k_at(kvec[:, a], d, order) for a in range(3)], axis=1)
    x = torch.arange(nx, dtype=torch.float64, device="cuda") * d
    y = torch.arange(ny, dtype=torch.float64, device="cuda") * d
    z = torch.arange(nz, dtype=torch.float64, device="cuda") * d
    g = torch.zeros((11,) + tuple(gshape), dtype=torch.float64, device="cuda")
    for j in range(nmodes):
        khat = kp[j] / np.linalg.norm(kp[j])
        e = synth.transverse_unit(pw["u"][j], khat) * pw["amp"][j]
        b = np.cross(khat, e)
        ph = (kvec[j, 0] * x)[None, None, :] + (kvec[j, 1] * y)[None, :, None] + (kvec[j, 2] * z)[:, None, None]
        cs = torch.cos(ph + pw["phase"][j])
        for c in range(3):
            g[c] += float(e[c]) * cs
            g[3 + c] += float(b[c]) * cs
        del ph, cs
    direction = rng.normal(size=3)
    direction /= np.linalg.norm(direction)
    r2 = ((x - 0.5 * nx * d) ** 2)[None, None, :] + ((y - 0.5 * ny * d) ** 2)[None, :, None] \
        + ((z - 0.5 * nz * d) ** 2)[:, None, None]
    blob = 0.1 * torch.exp(-r2 / (2 * 3.0 ** 2))
    for c in range(3):
        g[6 + c] = float(direction[c]) * blob
    return g


def _k_half(gshape, d, order):
    import torch

    from oracle import kspace

    nz, ny, nx = gshape
    kx = torch.as_tensor(kspace.modified_k(nx, d, order)[: nx // 2 + 1], device="cuda")[None, None, :]
    ky = torch.as_tensor(kspace.modified_k(ny, d, order), device="cuda")[None, :, None]
    kz = torch.as_tensor(kspace.modified_k(nz, d, order), device="cuda")[:, None, None]
    return kx, ky, kz


def _div(fields3, K):
    """Spectral order-p divergence i K . F^ of three real FP64 arrays (half spectrum)."""
    import torch

    out = None
    for c in range(3):
        t = 1j * K[c] * torch.fft.rfftn(fields3[c].double())
        out = t if out is None else out + t
        del t
    return out


def test_full_size_fp32_vs_fp64_with_sources_200_steps(lib):
    import torch

    interior, ng, order, d, dt, nsteps = (1024, 512, 512), 16, 32, 1.0, 0.5, 200
    nx, ny, nz = interior
    gshape = (nz, ny, nx)
    g64 = _full_size_inputs(gshape, d, order, 16, synth.rng_for(4, 2))
    K = _k_half(gshape, d, order)
    # dt div_p J, computed spectrally with the solver's own K_p
    dq = torch.fft.irfftn(dt * _div(g64[6:9], K), s=gshape)
    g64[10] = -dq
    res = {}
    for precision in ("fp64", "fp32"):
        plan = lib.Plan(nx, ny, nz, nguard=ng, order=order, dx=d, dt=dt, precision=precision)
        g = g64.to(plan.dtype, copy=True).contiguous()
        dqp = dq.to(plan.dtype)
        print(f"precision study {precision}: {nsteps} steps with continuity-advanced charge", flush=True)
        for _ in range(nsteps):
            plan.step_g1(g, (0, 0, 0))
            g[9].copy_(g[10])
            g[10].sub_(dqp)
        torch.cuda.synchronize()
        plan.close()
        rho = torch.fft.rfftn(g[9].double())
        gauss = float((_div(g[0:3], K) - rho).abs().norm() / rho.abs().norm())
        res[precision] = (g[0:6].double().clone(), gauss)
        del g, rho, dqp
        torch.cuda.empty_cache()
    e = res["fp32"][0] - res["fp64"][0]
    rel_e = float(e[0:3].norm() / res["fp64"][0][0:3].norm())
    rel_b = float(e[3:6].norm() / res["fp64"][0][3:6].norm())
    print(f"  FP32 vs FP64 after {nsteps} steps: E {rel_e:.2e} B {rel_b:.2e}; Gauss residual "
          f"FP64 {res['fp64'][1]:.2e} FP32 {res['fp32'][1]:.2e}", flush=True)
    assert rel_e <= 2e-5 and rel_b <= 2e-5, (rel_e, rel_b)
    assert np.isfinite(res["fp64"][1]) and np.isfinite(res["fp32"][1])
    # FP32 adds round-off to the guard truncation residual, not a new error source
    assert abs(res["fp32"][1] - res["fp64"][1]) <= 1e-4 + 0.05 * res["fp64"][1]


def test_three_way_on_the_128_cubed_box(lib):
    import torch

    gm = _golden_module()
    rec = dict(np.load(os.path.join(HERE, "golden", "box128.npz"), allow_pickle=False))
    interior, ng, order, g1 = gm.box128_case()
    w = [torch.as_tensor(a, device="cuda") for a in gm.weights(g1.shape[1:])]
    out = {}
    for precision in ("fp64", "fp32"):
        plan = lib.Plan(*interior, nguard=ng, order=order, dx=gm.D, dt=gm.DT, precision=precision)
        g = torch.as_tensor(g1, dtype=plan.dtype, device="cuda")
        print(f"128^3 + 16 box, order 32, {precision}: 200 steps", flush=True)
        for n in range(1, 201):
            plan.step_g1(g, (0, 0, 0))
            if n in (10, 200):
                out[(precision, n)] = g[0:6].double().clone()
        torch.cuda.synchronize()
        plan.close()
        del g
    report = {}
    for (precision, n), f6 in out.items():
        key = f"s{n}_"
        smax = float(np.abs(rec[key + "vals"]).max())
        worst_p = worst_s = 0.0
        c = torch.as_tensor(rec[key + "cells"][0], device="cuda")
        for f in range(6):
            for q in range(len(w)):
                p = float((w[q] * f6[f]).sum())
                worst_p = max(worst_p, abs(p - rec[key + "proj"][0, f, q])
                              / (rec[key + "wnorm"][0, q] * rec[key + "norm"][0, f]))
            got = f6[f][c[:, 0], c[:, 1], c[:, 2]].cpu().numpy()
            worst_s = max(worst_s, float(np.abs(got - rec[key + "vals"][0, f]).max()) / smax)
        report[(precision, n)] = (worst_p, worst_s)
        print(f"  {precision} vs oracle after {n} steps: projection {worst_p:.2e} sample {worst_s:.2e}", flush=True)
    e = out[("fp32", 200)] - out[("fp64", 200)]
    rel_e = float(e[0:3].norm() / out[("fp64", 200)][0:3].norm())
    rel_b = float(e[3:6].norm() / out[("fp64", 200)][3:6].norm())
    print(f"  FP32 vs FP64 GPU after 200 steps: E {rel_e:.2e} B {rel_b:.2e}", flush=True)
    assert max(report[("fp64", 10)]) <= 1e-12
    assert max(report[("fp64", 200)]) <= 1e-11
    assert report[("fp32", 10)][0] <= 2e-6 and report[("fp32", 10)][1] <= 2e-5
    assert report[("fp32", 200)][0] <= 2e-5 and report[("fp32", 200)][1] <= 2e-4
    assert rel_e <= 2e-5 and rel_b <= 2e-5
