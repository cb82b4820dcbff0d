"""Writes the stored oracle results that the large-case GPU tests compare against.

Every value in the files written here comes from the FP64 CPU oracle
(``oracle/``) run on inputs from the seeded generators (``synth``); nothing is
taken from the GPU path.  The cases are too slow for the oracle to run inside a
GPU test, so the expected outputs are kept in compressed form:

* for each output field (Ex..Bz) and each region (a sub-domain interior, or the
  whole grid), its L2 norm and its projections on two seeded N(0, 1) weight
  arrays over the global grid, sum_cells w * f;
* the field values at seeded sample cells.

A projection on random weights changes with any element of the field, so a
mistake confined to a few columns, a tile or one box still shows.

Cases (``python tests/golden/make_oracle_expected.py [name ...]``):

* ``batch64_step1``: the 64-box uneven decomposition (per-axis widths 32..96,
  guards in {8, 16, 32, 64}, orders in {16, 32, 64}) of a 268 x 257 x 224 grid,
  dense N(0, 1) fields on every array, one local step (Jacobi order);
  regions = the 64 interiors.
* ``box128``: a 128^3 periodic grid with one box of 16 guards per side
  (160^3), order 32, dt = dx / 2c; 16 seeded plane waves in E, B and a Gaussian
  current (sigma 3 cells, peak 0.1), sources held fixed; results after 10 and
  200 steps; region = the whole grid.
"""

from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402

D, DT = 1.0, 0.5
NSAMPLE = 64


def weights(gshape):
    """The two seeded weight arrays of the projections (shared with the tests)."""
    return [synth.rng_for(114, k).normal(0.0, 1.0, size=gshape) for k in range(2)]


def batch64_case():
    """(gdims, boxes, inputs) of the 64-box case."""
    gdims, boxes = synth.uneven_decomposition(synth.rng_for(3, 0))
    g1 = synth.random_fields(synth.rng_for(113, 0), gdims[::-1])
    return gdims, boxes, g1


def box128_case():
    """(interior, nguard, order, inputs) of the 128^3 + 16 case."""
    interior = (128, 128, 128)
    g1 = synth.plane_waves_and_blob(synth.rng_for(4, 1), interior[::-1], D, 16)
    return interior, 16, 32, g1


def sample_cells(rng, lo, hi, n):
    """n cells (k, j, i) drawn uniformly in the box [lo, hi) given as (x, y, z) triples."""
    i = rng.integers(lo[0], hi[0], size=n)
    j = rng.integers(lo[1], hi[1], size=n)
    k = rng.integers(lo[2], hi[2], size=n)
    return np.stack([k, j, i], axis=1)


def summarize(out6, regions, w, rng):
    """Norms, projections and samples of the six output fields over each region (lo, hi)."""
    nreg = len(regions)
    proj = np.zeros((nreg, 6, len(w)))
    norm = np.zeros((nreg, 6))
    wnorm = np.zeros((nreg, len(w)))
    cells = np.zeros((nreg, NSAMPLE, 3), dtype=np.int64)
    vals = np.zeros((nreg, 6, NSAMPLE))
    for r, (lo, hi) in enumerate(regions):
        sl = (slice(lo[2], hi[2]), slice(lo[1], hi[1]), slice(lo[0], hi[0]))
        for q in range(len(w)):
            wnorm[r, q] = np.linalg.norm(w[q][sl])
        for f in range(6):
            a = out6[f][sl]
            norm[r, f] = np.linalg.norm(a)
            for q in range(len(w)):
                proj[r, f, q] = float(np.sum(w[q][sl] * a))
        c = sample_cells(rng, lo, hi, NSAMPLE)
        cells[r] = c
        vals[r] = out6[:, c[:, 0], c[:, 1], c[:, 2]]
    return {"lo": np.array([r[0] for r in regions]), "hi": np.array([r[1] for r in regions]), "proj": proj,
            "norm": norm, "wnorm": wnorm, "cells": cells, "vals": vals}


def make_batch64():
    from oracle import domain

    gdims, boxes, g1 = batch64_case()
    t0 = time.perf_counter()
    out = domain.local_step(g1, boxes, D, DT)
    print(f"batch64_step1: oracle {time.perf_counter() - t0:.1f} s", flush=True)
    regions = [(b["origin"], tuple(o + n for o, n in zip(b["origin"], b["interior"]))) for b in boxes]
    rec = summarize(out[0:6], regions, weights(g1.shape[1:]), synth.rng_for(115, 0))
    np.savez_compressed(os.path.join(HERE, "batch64_step1.npz"), **rec)


def make_box128():
    from oracle import domain

    interior, ng, order, g1 = box128_case()
    box = [{"origin": (0, 0, 0), "interior": interior, "nguard": ng, "order": order}]
    w = weights(g1.shape[1:])
    region = [((0, 0, 0), interior)]
    f = g1
    recs = {}
    t0 = time.perf_counter()
    for n in range(1, 201):
        f = domain.local_step(f, box, D, DT)
        if n in (10, 200):
            rec = summarize(f[0:6], region, w, synth.rng_for(115, n))
            recs.update({f"s{n}_{k}": v for k, v in rec.items()})
            print(f"box128: {n} steps, {time.perf_counter() - t0:.1f} s", flush=True)
    np.savez_compressed(os.path.join(HERE, "box128.npz"), **recs)


CASES = {"batch64_step1": make_batch64, "box128": make_box128}

if __name__ == "__main__":
    for name in sys.argv[1:] or list(CASES):
        CASES[name]()
