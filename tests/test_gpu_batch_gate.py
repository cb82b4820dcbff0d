"""GPU: the batched 64-box step against the oracle on every box, and the FP32 accuracy gate.

Sec. 1.3 and Fig. 1(a) of arXiv:1812.07357: many sub-domains, each with guard
cells and its own FFT, advanced independently every step.  The decomposition is
the 4 x 4 x 4 uneven split of a 268 x 257 x 224 grid (widths 32..96, guards
in {8, 16, 32, 64}, orders in {16, 32, 64}) that bench.py times.

* One batched step on dense N(0, 1) fields, FP64 and FP32, against the oracle's
  local step on every one of the 64 boxes.  The oracle result is stored by
  tests/golden/make_oracle_expected.py (it takes minutes on the CPU): per box
  and field, projections on two seeded random weight arrays plus 64 sampled
  cells.  A projection moves with any element of the box, so a wrong column,
  tile or box shows.  FP64: projections within 1e-12 of |w| |f| (Cauchy-Schwarz
  scale), samples within 1e-12 of the largest sample; FP32: 2e-6 and 2e-5.
* The accuracy target of the FP32 batched path: 100 steps replayed from the
  captured graph, FP32 against the FP64 batch on the same inputs (seeded plane
  waves and a Gaussian current, as bench.py), relative L2 <= 1e-5 per vector
  field (E and B separately) over the grid.
"""

import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "batch64_step1.npz")


def _golden_module():
    import importlib.util

    spec = importlib.util.spec_from_file_location("make_oracle_expected",
                                                  os.path.join(HERE, "golden", "make_oracle_expected.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _check_against_golden(out6, rec, w, tol_proj, tol_sample):
    """Compare a (6, NZ, NY, NX) float64 torch tensor on the GPU with a stored oracle summary."""
    import torch

    worst_p, worst_s = 0.0, 0.0
    smax = float(np.abs(rec["vals"]).max())
    for r in range(rec["lo"].shape[0]):
        lo, hi = rec["lo"][r], rec["hi"][r]
        sl = (slice(lo[2], hi[2]), slice(lo[1], hi[1]), slice(lo[0], hi[0]))
        c = torch.as_tensor(rec["cells"][r], device="cuda")
        for f in range(6):
            a = out6[f][sl]
            for q in range(len(w)):
                p = float((w[q][sl] * a).sum())
                scale = rec["wnorm"][r, q] * rec["norm"][r, f]
                worst_p = max(worst_p, abs(p - rec["proj"][r, f, q]) / scale)
            got = out6[f][c[:, 0], c[:, 1], c[:, 2]].cpu().numpy()
            worst_s = max(worst_s, float(np.abs(got - rec["vals"][r, f]).max()) / smax)
    assert worst_p <= tol_proj, worst_p
    assert worst_s <= tol_sample, worst_s
    return worst_p, worst_s


@pytest.mark.parametrize("precision,tol_proj,tol_sample", [("fp64", 1e-12, 1e-12), ("fp32", 2e-6, 2e-5)])
def test_every_box_of_the_64_box_batch_matches_the_oracle(lib, precision, tol_proj, tol_sample):
    import torch

    gm = _golden_module()
    rec = dict(np.load(GOLDEN, allow_pickle=False))
    gdims, boxes, g1 = gm.batch64_case()
    w = [torch.as_tensor(a, device="cuda") for a in gm.weights(g1.shape[1:])]
    batch = lib.Batch(boxes, gdims, dx=gm.D, dt=gm.DT, precision=precision)
    g = torch.as_tensor(g1, dtype=batch.dtype, device="cuda")
    print(f"64-box batch, one step, {precision}", flush=True)
    batch.step(g)
    torch.cuda.synchronize()
    batch.close()
    out6 = g[0:6].double()
    del g
    wp, ws = _check_against_golden(out6, rec, w, tol_proj, tol_sample)
    print(f"  worst projection error {wp:.2e}, worst sample error {ws:.2e}", flush=True)


def test_fp32_batch_meets_the_accuracy_target_over_100_steps(lib):
    import torch

    gdims, boxes = synth.uneven_decomposition(synth.rng_for(3, 0))
    host = synth.plane_waves_and_blob(synth.rng_for(3, 1), gdims[::-1], 1.0, 4, mmax=8)
    res = {}
    for precision in ("fp64", "fp32"):
        batch = lib.Batch(boxes, gdims, dx=1.0, dt=0.5, precision=precision)
        g = torch.as_tensor(host, dtype=batch.dtype, device="cuda")
        print(f"64-box batch, 100 steps from the graph, {precision}", flush=True)
        batch.run(g, 100)
        torch.cuda.synchronize()
        batch.close()
        res[precision] = g[0:6].double()
        del g
    e = res["fp32"] - res["fp64"]
    rel_e = float(e[0:3].norm() / res["fp64"][0:3].norm())
    rel_b = float(e[3:6].norm() / res["fp64"][3:6].norm())
    print(f"  FP32 vs FP64 after 100 steps: E {rel_e:.2e}, B {rel_b:.2e}", flush=True)
    assert np.isfinite(rel_e) and np.isfinite(rel_b)
    assert rel_e <= 1e-5 and rel_b <= 1e-5, (rel_e, rel_b)
