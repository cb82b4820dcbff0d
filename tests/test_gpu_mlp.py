"""GPU: the guard-width surrogate's kernels (psatd_mlp_*) against the FP64 oracle.

Forward, gradient and Adam run through the C ABI on bfloat16 weights; the
oracle (oracle/mlp.py) runs in FP64 on the same bfloat16-rounded weights and
standardised inputs.  Gates: forward 1e-5 relative (max norm), gradient 1e-5
relative (2-norm per parameter tensor), Adam 1e-6 relative on the master
weights, bfloat16 copy bit-exact with the oracle's rounding of the master
weights.  The solver-generated label is checked against the oracle's own
local-vs-global run.
"""

import numpy as np
import pytest

import synth
from oracle import domain, mlp as omlp

pytestmark = pytest.mark.gpu

MEAN = np.array([0.05, 3.5, 0.6, 25.0, 0.17, 4.5], dtype=np.float32)
SCALE = np.array([12.0, 0.8, 4.0, 0.1, 14.0, 1.2], dtype=np.float32)
OUT_MEAN, OUT_SCALE = -6.0, 3.0


def _inputs(seed, n):
    rng = np.random.default_rng(seed)
    X = (MEAN + rng.normal(size=(n, 6)) / SCALE).astype(np.float32)
    t = rng.normal(OUT_MEAN, OUT_SCALE, size=n).astype(np.float32)
    return X, t


def _std(X):
    return (X.astype(np.float64) - MEAN.astype(np.float64)) * SCALE.astype(np.float64)


def _make(lib, seed=0, max_batch=1024):
    from paper_1812_07357_amd import guard_model

    init = guard_model.init_params(np.random.default_rng(seed))
    return lib.Mlp(init, MEAN, SCALE, OUT_MEAN, OUT_SCALE, max_batch=max_batch)


def _tensor_groups(v):
    p = omlp.unpack(np.asarray(v, dtype=np.float64))
    return {k: p[k].ravel() for k, _ in omlp.SHAPES}


@pytest.mark.parametrize("n", [1, 31, 32, 1000])
def test_forward_matches_oracle(lib, n):
    import torch

    net = _make(lib, seed=1)
    X, _ = _inputs(2, n)
    y = net.predict(torch.as_tensor(X, device="cuda")).cpu().numpy().astype(np.float64)
    _, wbf = net.params()
    ref, _ = omlp.forward(wbf.astype(np.float64), _std(X))
    ref = OUT_MEAN + OUT_SCALE * ref
    assert np.max(np.abs(y - ref)) <= 1e-5 * max(1.0, np.abs(ref).max())
    net.close()


def test_bf16_copy_is_rounded_master(lib):
    net = _make(lib, seed=3)
    master, wbf = net.params()
    assert np.array_equal(omlp.bf16_round(master).view(np.uint32), wbf.view(np.uint32))
    net.close()


@pytest.mark.parametrize("n,batch,with_idx", [(777, 300, True), (64, 64, False), (40, 1, False)])
def test_gradient_matches_oracle(lib, n, batch, with_idx):
    import torch

    net = _make(lib, seed=4)
    X, t = _inputs(5, n)
    rng = np.random.default_rng(6)
    idx = None
    if with_idx:
        idx = rng.integers(0, n, size=batch).astype(np.int32)
        idx[7] = idx[3]     # a repeated sample counts twice
        idx[11] = n + 5     # out of range: contributes nothing
        sel = np.array([i for i in idx if 0 <= i < n])
    else:
        sel = np.arange(batch)
    g, loss = net.grad(torch.as_tensor(X, device="cuda"), torch.as_tensor(t, device="cuda"),
                       None if idx is None else torch.as_tensor(idx, device="cuda"), batch=batch)
    _, wbf = net.params()
    tn = (t.astype(np.float64) - OUT_MEAN) / OUT_SCALE
    L, gref = omlp.loss_and_grad(wbf.astype(np.float64), _std(X[sel]), tn[sel])
    # the kernels divide by the batch size, masked samples included
    f = len(sel) / batch
    gref *= f
    L *= f
    assert abs(float(loss.cpu()) - L) <= 1e-5 * L
    got = _tensor_groups(g.cpu().numpy())
    exp = _tensor_groups(gref)
    for k in got:
        assert np.linalg.norm(got[k] - exp[k]) <= 1e-5 * np.linalg.norm(exp[k]), k
    net.close()


def test_adam_matches_oracle(lib):
    import torch

    net = _make(lib, seed=7)
    X, t = _inputs(8, 256)
    Xg, tg = torch.as_tensor(X, device="cuda"), torch.as_tensor(t, device="cuda")
    m = np.zeros(omlp.NPARAM)
    v = np.zeros(omlp.NPARAM)
    for step in range(1, 4):
        master, _ = net.params()
        g, _ = net.grad(Xg, tg)
        net.adam(lr=1e-3)
        new, wbf = net.params()
        ref, m, v = omlp.adam(master.astype(np.float64), g.cpu().numpy().astype(np.float64), m, v, step)
        assert np.max(np.abs(new - ref)) <= 1e-6 * max(1.0, np.abs(ref).max())
        assert np.array_equal(omlp.bf16_round(new).view(np.uint32), wbf.view(np.uint32))
    net.close()


def test_training_fits_a_smooth_target(lib):
    import torch

    rng = np.random.default_rng(9)
    n = 4096
    X = (MEAN + rng.normal(size=(n, 6)) / SCALE).astype(np.float32)
    z = _std(X)
    t = (OUT_MEAN + OUT_SCALE * (np.tanh(z[:, 0] - 0.5 * z[:, 1]) + 0.3 * z[:, 5] ** 2 - 0.2 * z[:, 2])).astype(
        np.float32)
    net = _make(lib, seed=10, max_batch=256)
    Xg, tg = torch.as_tensor(X, device="cuda"), torch.as_tensor(t, device="cuda")
    idx = torch.as_tensor(rng.integers(0, n, size=2000 * 256).astype(np.int32), device="cuda")
    hist = net.train(Xg, tg, idx, 2000, 256, lr=2e-3).cpu().numpy()
    assert np.all(np.isfinite(hist))
    assert hist[-50:].mean() < 0.05 * hist[:10].mean(), (hist[:10].mean(), hist[-50:].mean())
    net.close()


def test_label_matches_oracle_local_vs_global(lib):
    """One solver-generated training label (FP64 GPU) against the oracle's own local and global runs."""
    from paper_1812_07357_amd import guard_model

    lvg = guard_model.LocalVsGlobal(domain=32, split=2, precision="fp64")
    run = guard_model.Run(order=8, cdt=0.5, lam=10.0, width=0.2)
    g1 = lvg.fields(run, synth.rng_for(500, 0), nmodes=8)
    got = lvg.errors(g1, run, [2, 4], [2, 4])
    g1 = g1.cpu().numpy()
    for ng in (2, 4):
        boxes = lvg.boxes(ng, run.order)
        for k, e in zip((2, 4), got[ng]):
            loc = domain.local_steps(g1, boxes, k, 1.0, run.cdt)
            glo = domain.global_steps(g1, k, 1.0, run.cdt, run.order)
            ref = omlp.truncation_error(loc[0:6], glo[0:6])
            assert ref > -12.0  # a real truncation error, far above round-off
            assert abs(e - ref) <= 1e-6 * abs(ref) + 1e-9, (ng, k, e, ref)
