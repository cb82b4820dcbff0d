"""Learned guard width: training data from the solver, training, and the choice of n_g.

The paper asks for a model that gives the number of guard cells n_g a local
solver needs as a function of its order, time step and cell size (Sec. 1.4;
n_g sets the memory and cost of the local and hybrid solvers, Sec. 2.2).  This
module builds one:

* ``LocalVsGlobal`` runs the solver itself (``psatd.Batch`` for the local
  solve on split^3 sub-domains with guards, ``psatd.Plan`` for the global
  periodic solve) and measures the truncation error of the local solve:
  log10 of max |local - global| / max |global| over every cell and the six
  components of E and B, floored at -16.
* ``generate`` draws runs (order, c dt/dx, laser wavelength, spectral width),
  runs each with a few guard widths and records the error at several step
  counts: one sample per (run, n_g, steps).
* ``train`` fits the network of ``psatd.Mlp`` (6 -> 64 -> 64 -> 1, bfloat16
  weights, trained by the library's own forward/backward/Adam kernels).
* ``choose_guard`` picks the smallest candidate n_g whose predicted error,
  plus a safety margin taken from held-out residuals, meets a tolerance.
  ``choose_checked`` then lets the plain local-vs-global comparison judge
  that choice and steps n_g up until the comparison passes (fallback);
  ``plain_scan`` is the method without the network (try n_g upwards).

Random numbers (run parameters, fields, initial weights, minibatches) are
drawn on the host from an explicit numpy Generator and passed in.
"""

from __future__ import annotations

import math
import time
from dataclasses import dataclass

import numpy as np

from . import psatd

# Candidate guard widths.  With 32-cell sub-domains of a 64-cell periodic
# training grid, n_g = 16 or 48 would make the box (32 + 2 n_g) an exact
# multiple of the grid period, so the local solve would reproduce the global
# one exactly -- an artifact of the small training grid -- and they are left
# out; every box edge left factors into the transform's small radices.
GUARDS = (4, 6, 8, 10, 12, 14, 20, 24, 28, 32, 40, 44)
CHECKPOINTS = (8, 12, 16, 24, 32, 48, 64)
FLOOR = -16.0


@dataclass
class Run:
    order: int        # stencil order p (0 = infinite)
    cdt: float        # c dt / dx
    lam: float        # laser wavelength / dx
    width: float      # relative spectral width 1 / (k0 L)


def draw_run(rng: np.random.Generator) -> Run:
    """p = 2 round(2^u), u ~ U[2, 7] (10 % infinite order); c dt/dx ~ U[0.25, 1]; lambda/dx ~ U[10, 40]; width ~ U[0.05, 0.3]."""
    if rng.uniform() < 0.1:
        order = 0
    else:
        order = 2 * int(round(2.0 ** rng.uniform(2.0, 7.0)))
    return Run(order=order, cdt=float(rng.uniform(0.25, 1.0)), lam=float(rng.uniform(10.0, 40.0)),
               width=float(rng.uniform(0.05, 0.3)))


def features(order, nguard, cdt, lam, width, steps) -> np.ndarray:
    """Network inputs (n, 6) float32: 2/p (0 for infinite order), log2 n_g, c dt/dx, lambda/dx, width, log2 steps."""
    order = np.asarray(order, dtype=np.float64)
    inv_p = np.where(order > 0, 2.0 / np.maximum(order, 1.0), 0.0)
    cols = [inv_p, np.log2(np.asarray(nguard, dtype=np.float64)), np.asarray(cdt, dtype=np.float64),
            np.asarray(lam, dtype=np.float64), np.asarray(width, dtype=np.float64),
            np.log2(np.asarray(steps, dtype=np.float64))]
    return np.stack(np.broadcast_arrays(*cols), axis=-1).astype(np.float32)


class LocalVsGlobal:
    """Truncation error of the local solver with guards against the global periodic solve.

    The global grid is ``domain``^3 cells, split into ``split``^3 equal
    sub-domains; fields are a laser-like vacuum packet (E, B; J = rho = 0).
    """

    def __init__(self, domain: int = 64, split: int = 2, precision: str = "fp64", d: float = 1.0, c: float = 1.0):
        if domain % split:
            raise ValueError("domain must be a multiple of split")
        self.domain, self.split, self.precision, self.d, self.c = domain, split, precision, d, c
        self.sub = domain // split

    def fields(self, run: Run, rng: np.random.Generator, nmodes: int = 16):
        """(11, n, n, n) float64 GPU tensor: a laser-like vacuum packet in E, B; J = rho = 0."""
        import torch

        import synth

        n = self.domain
        lm = synth.laser_modes(rng, (n, n, n), self.d, run.lam * self.d, run.width, nmodes=nmodes, c=self.c)
        g1 = torch.zeros((11, n, n, n), dtype=torch.float64, device="cuda")
        x = torch.arange(n, dtype=torch.float64, device="cuda") * self.d
        for j in range(len(lm["amp"])):
            k = 2.0 * np.pi * lm["m"][j] / (n * self.d)
            ph = ((k[2] * x)[:, None, None] + (k[1] * x)[None, :, None] + (k[0] * x)[None, None, :]
                  + lm["phase"][j])
            cs = torch.cos(ph) * lm["amp"][j]
            for c in range(3):
                g1[c] += lm["evec"][j][c] * cs
                g1[3 + c] += lm["bvec"][j][c] * cs
            del ph, cs
        return g1

    def boxes(self, nguard: int, order: int):
        s = self.sub
        return [{"origin": (i * s, j * s, k * s), "interior": (s, s, s), "nguard": nguard, "order": order}
                for k in range(self.split) for j in range(self.split) for i in range(self.split)]

    def reference(self, g1, run: Run, checkpoints, stream=None):
        """Global periodic solve: (initial fields in the working precision, {steps: E and B after steps})."""
        import torch

        dtype = torch.float64 if self.precision == "fp64" else torch.float32
        n = self.domain
        checkpoints = sorted(int(k) for k in checkpoints)
        g0 = torch.as_tensor(g1).to(device="cuda", dtype=dtype).contiguous()
        plan = psatd.Plan(n, n, n, nguard=0, order=run.order, dx=self.d, dt=run.cdt * self.d / self.c, c=self.c,
                          precision=self.precision)
        g = g0.clone()
        ref = {}
        for k in range(1, checkpoints[-1] + 1):
            plan.step_g1(g, (0, 0, 0), stream)
            if k in checkpoints:
                ref[k] = g[0:6].clone()
        plan.close()
        return g0, ref

    def local_errors(self, g0, ref, run: Run, nguard: int, stream=None):
        """log10 error of the local solve with guard width ``nguard`` at each step count of ``ref`` (sorted)."""
        n = self.domain
        batch = psatd.Batch(self.boxes(int(nguard), run.order), (n, n, n), dx=self.d, dt=run.cdt * self.d / self.c,
                            c=self.c, precision=self.precision)
        g = g0.clone()
        pairs = []
        for k in range(1, max(ref) + 1):
            batch.step(g, stream)
            if k in ref:
                pairs.append(((g[0:6] - ref[k]).abs().max(), ref[k].abs().max()))
        batch.close()
        vals = []
        for num, den in pairs:
            e = float(num) / float(den) if float(den) > 0 else 0.0
            vals.append(max(FLOOR, math.log10(e)) if e > 0 else FLOOR)
        return vals

    def errors(self, g1, run: Run, guards, checkpoints, stream=None):
        """{n_g: [log10 error after each checkpoint step count]} for the fields g1 (11, n, n, n)."""
        g0, ref = self.reference(g1, run, checkpoints, stream)
        return {int(ng): self.local_errors(g0, ref, run, int(ng), stream) for ng in guards}

    def judge(self, g1, run: Run, steps: int):
        """The plain comparison as a function n_g -> measured log10 error after ``steps`` steps (memoised)."""
        g0, ref = self.reference(g1, run, [steps])
        cache = {}

        def judge(ng):
            if ng not in cache:
                cache[ng] = self.local_errors(g0, ref, run, int(ng))[0]
            return cache[ng]

        judge.cache = cache
        return judge


def generate(nruns: int, rng: np.random.Generator, lvg: LocalVsGlobal | None = None, guards_per_run: int = 3,
             guards=GUARDS, checkpoints=CHECKPOINTS, log=None):
    """Solver-generated samples: returns dict with X (n, 6) float32, y (n,) float32, run (n,) int, timing."""
    lvg = lvg or LocalVsGlobal()
    X, y, rid = [], [], []
    t0 = time.perf_counter()
    for r in range(nruns):
        run = draw_run(rng)
        g1 = lvg.fields(run, rng)
        gs = sorted(int(v) for v in rng.choice(np.asarray(guards), size=guards_per_run, replace=False))
        errs = lvg.errors(g1, run, gs, checkpoints)
        for ng in gs:
            for k, e in zip(sorted(checkpoints), errs[ng]):
                X.append(features(run.order, ng, run.cdt, run.lam, run.width, k))
                y.append(e)
                rid.append(r)
        if log and (r + 1) % max(1, nruns // 20) == 0:
            log(f"runs {r + 1}/{nruns}  samples {len(y)}  {time.perf_counter() - t0:.1f} s")
    return {"X": np.stack(X).astype(np.float32), "y": np.asarray(y, dtype=np.float32),
            "run": np.asarray(rid, dtype=np.int32), "seconds": time.perf_counter() - t0}


def init_params(rng: np.random.Generator) -> np.ndarray:
    """Initial weights: N(0, 1/fan_in) weights (He-like for SiLU), zero biases; flat layout of psatd.Mlp."""
    w1 = rng.normal(0.0, math.sqrt(1.0 / 6.0), size=(64, 6))
    w2 = rng.normal(0.0, math.sqrt(1.0 / 64.0), size=(64, 64))
    w3 = rng.normal(0.0, math.sqrt(1.0 / 64.0), size=64)
    return np.concatenate([w1.ravel(), np.zeros(64), w2.ravel(), np.zeros(64), w3, np.zeros(1)]).astype(np.float32)


def split_runs(run_ids: np.ndarray, rng: np.random.Generator, frac=(0.8, 0.1, 0.1)):
    """Train / validation / test masks, split by run so no run contributes to two sets."""
    runs = np.unique(run_ids)
    perm = rng.permutation(runs)
    n1 = int(round(frac[0] * len(runs)))
    n2 = n1 + int(round(frac[1] * len(runs)))
    sets = (set(perm[:n1].tolist()), set(perm[n1:n2].tolist()), set(perm[n2:].tolist()))
    return tuple(np.isin(run_ids, np.fromiter(s, dtype=run_ids.dtype, count=len(s))) for s in sets)


@dataclass
class Model:
    mlp: "psatd.Mlp"
    margin: float          # safety margin (log10 units) added to predictions when choosing n_g
    metrics: dict


# Labels above this are capped: an error as large as the field itself means the
# run is unusable (at infinite order and large c dt/dx the local solve can even
# grow without bound), and how far beyond that it goes does not matter for the
# choice of n_g.
LABEL_CAP = 0.0


def train(X: np.ndarray, y: np.ndarray, run_ids: np.ndarray, rng: np.random.Generator, steps: int = 4000,
          batch: int = 512, lr: float = 1e-3, quantile: float = 0.95):
    """Fit the network on the training runs; the margin is the ``quantile`` of held-out under-predictions."""
    import torch

    y = np.minimum(np.asarray(y, dtype=np.float32), np.float32(LABEL_CAP))
    tr, va, te = split_runs(run_ids, rng)
    mean = X[tr].mean(axis=0)
    std = X[tr].std(axis=0)
    std = np.where(std > 1e-6, std, 1.0)
    ym, ys = float(y[tr].mean()), float(max(y[tr].std(), 1e-3))
    mlp = psatd.Mlp(init_params(rng), mean, 1.0 / std, ym, ys, max_batch=batch)
    dev = "cuda"
    Xt = torch.as_tensor(X[tr], device=dev)
    yt = torch.as_tensor(y[tr], device=dev)
    idx = torch.as_tensor(rng.integers(0, int(tr.sum()), size=steps * batch).astype(np.int32), device=dev)
    t0 = time.perf_counter()
    hist = mlp.train(Xt, yt, idx, steps, batch, lr=lr)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0

    def resid(mask):
        if not mask.any():
            return np.zeros(0)
        p = mlp.predict(torch.as_tensor(X[mask], device=dev)).cpu().numpy()
        return y[mask] - p

    r_tr, r_va, r_te = resid(tr), resid(va), resid(te)
    margin = float(np.quantile(r_va, quantile)) if r_va.size else 1.0
    rms = lambda r: float(np.sqrt(np.mean(r * r))) if r.size else float("nan")  # noqa: E731
    metrics = {"rmse_train": rms(r_tr), "rmse_val": rms(r_va), "rmse_test": rms(r_te), "margin": margin,
               "loss_first": float(hist[0]), "loss_last": float(hist[-1]), "train_seconds": train_s,
               "steps": steps, "batch": batch, "samples_train": int(tr.sum()), "samples_val": int(va.sum()),
               "samples_test": int(te.sum())}
    return Model(mlp, max(margin, 0.0), metrics), (tr, va, te)


def save(path: str, model: Model):
    master, _ = model.mlp.params()
    mean, scale, om, os_ = model.mlp.norm
    np.savez(path, master=master, in_mean=mean, in_scale=scale, out_mean=np.float32(om), out_scale=np.float32(os_),
             margin=np.float32(model.margin))


def load(path: str) -> Model:
    z = np.load(path, allow_pickle=False)
    mlp = psatd.Mlp(z["master"], z["in_mean"], z["in_scale"], float(z["out_mean"]), float(z["out_scale"]),
                    max_batch=64)
    return Model(mlp, float(z["margin"]), {})


def predict(model: Model, run: Run, steps: int, guards=GUARDS) -> np.ndarray:
    """Predicted log10 error for each candidate guard width."""
    import torch

    f = features(run.order, np.asarray(guards), run.cdt, run.lam, run.width, steps)
    return model.mlp.predict(torch.as_tensor(f, device="cuda")).cpu().numpy().astype(np.float64)


def pick_guard(pred, margin: float, tol: float, guards=GUARDS) -> int:
    """Smallest candidate whose predicted log10 error plus ``margin`` is at most log10(tol) (largest if none)."""
    ok = [g for g, p in zip(guards, pred) if p + margin <= math.log10(tol)]
    return int(ok[0]) if ok else int(guards[-1])


def choose_guard(model: Model, run: Run, steps: int, tol: float, guards=GUARDS) -> int:
    """The network's choice of n_g for a run (no solver call)."""
    return pick_guard(predict(model, run, steps, guards), model.margin, tol, guards)


def judged(start: int, judge, tol: float, guards=GUARDS):
    """Plain local-vs-global comparison as judge: from ``start`` upwards, the first n_g that passes.

    ``judge(ng)`` returns the measured log10 error.  Returns (n_g or None, judge calls, measured log10 error).
    """
    calls = 0
    for cand in [c for c in guards if c >= start]:
        calls += 1
        e = judge(cand)
        if e <= math.log10(tol):
            return int(cand), calls, e
    return None, calls, None


def choose_checked(model: Model, judge, run: Run, steps: int, tol: float, guards=GUARDS):
    """The network's choice, judged by the plain comparison, stepping n_g up until it passes (fallback)."""
    return judged(choose_guard(model, run, steps, tol, guards), judge, tol, guards)


def plain_scan(judge, tol: float, guards=GUARDS):
    """The method without the network: try guard widths upwards from the smallest until the comparison passes."""
    return judged(guards[0], judge, tol, guards)


# ---------------------------------------------------------------- evaluation
def box_cells(lvg: LocalVsGlobal, ng: int) -> int:
    """Cells transformed per local step with guard width ng (all sub-domains)."""
    return (lvg.sub + 2 * int(ng)) ** 3 * lvg.split**3


def compare(model: Model, lvg: LocalVsGlobal, run: Run, g1, steps: int, tol: float, guards=GUARDS):
    """The network's choice (judged, with fallback) against the plain scan and the largest candidate."""
    judge = lvg.judge(g1, run, steps)
    t0 = time.perf_counter()
    pick = choose_guard(model, run, steps, tol, guards)
    t_pick = time.perf_counter() - t0
    g_model, calls_model, e_model = judged(pick, judge, tol, guards)
    g_plain, calls_plain, e_plain = plain_scan(judge, tol, guards)
    out = {"run": run.__dict__, "steps": steps, "tol": tol, "pick": pick, "pick_seconds": t_pick,
           "model": {"nguard": g_model, "judge_calls": calls_model, "log10_err": e_model},
           "plain": {"nguard": g_plain, "judge_calls": calls_plain, "log10_err": e_plain},
           "measured": {int(k): float(v) for k, v in sorted(judge.cache.items())}}
    if g_model is not None:
        out["cells_ratio_vs_largest"] = box_cells(lvg, g_model) / box_cells(lvg, guards[-1])
    return out


def _main(argv=None):
    import argparse
    import json
    import sys

    import torch

    import synth

    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    g = sub.add_parser("generate", help="solver-generated training samples")
    g.add_argument("--runs", type=int, default=950)
    g.add_argument("--stream", type=int, default=0)
    g.add_argument("--out", required=True)
    t = sub.add_parser("train", help="train the network on generated samples")
    t.add_argument("--data", required=True)
    t.add_argument("--out", required=True)
    t.add_argument("--report", required=True)
    t.add_argument("--steps", type=int, default=6000)
    t.add_argument("--batch", type=int, default=512)
    t.add_argument("--lr", type=float, default=1e-3)
    e = sub.add_parser("evaluate", help="network + judge vs plain scan on fresh 64^3 runs")
    e.add_argument("--model", required=True)
    e.add_argument("--runs", type=int, default=12)
    e.add_argument("--tol", type=float, default=1e-6)
    e.add_argument("--steps", type=int, default=32)
    e.add_argument("--report", required=True)
    c = sub.add_parser("check", help="choose n_g for a large FP32 run and judge it against the global solve")
    c.add_argument("--model", required=True)
    c.add_argument("--domain", type=int, default=512)
    c.add_argument("--split", type=int, default=4)
    c.add_argument("--precision", default="fp32")
    c.add_argument("--order", type=int, default=100)
    c.add_argument("--cdt", type=float, default=0.5)
    c.add_argument("--lam", type=float, default=16.0)
    c.add_argument("--width", type=float, default=1.0 / (2.0 * np.pi * 3.0))
    c.add_argument("--steps", type=int, default=32)
    c.add_argument("--tol", type=float, default=1e-4)
    c.add_argument("--report", required=True)
    a = ap.parse_args(argv)

    def log(msg):
        print(f"[guard_model] {msg}", file=sys.stderr, flush=True)

    if a.cmd == "generate":
        d = generate(a.runs, synth.rng_for(5, a.stream), log=log)
        np.savez(a.out, X=d["X"], y=d["y"], run=d["run"])
        log(f"{len(d['y'])} samples from {a.runs} runs in {d['seconds']:.1f} s -> {a.out}")
    elif a.cmd == "train":
        z = np.load(a.data, allow_pickle=False)
        model, _ = train(z["X"], z["y"], z["run"], synth.rng_for(5, 1000), steps=a.steps, batch=a.batch, lr=a.lr)
        save(a.out, model)
        with open(a.report, "w") as f:
            json.dump(model.metrics, f, indent=1)
        log(json.dumps(model.metrics))
    elif a.cmd == "evaluate":
        model = load(a.model)
        lvg = LocalVsGlobal()
        rng = synth.rng_for(5, 2000)
        rows = []
        for i in range(a.runs):
            run = draw_run(rng)
            r = compare(model, lvg, run, lvg.fields(run, rng), a.steps, a.tol)
            rows.append(r)
            log(f"run {i}: pick {r['pick']} -> {r['model']['nguard']} ({r['model']['judge_calls']} calls); "
                f"plain {r['plain']['nguard']} ({r['plain']['judge_calls']} calls)")
        ok = [r for r in rows if r["plain"]["nguard"] is not None]
        summary = {
            "runs": len(rows), "tol": a.tol, "steps": a.steps,
            "judge_calls_model": float(np.mean([r["model"]["judge_calls"] for r in rows])),
            "judge_calls_plain": float(np.mean([r["plain"]["judge_calls"] for r in rows])),
            "first_pick_passed": float(np.mean([r["model"]["judge_calls"] == 1 and r["model"]["nguard"] is not None
                                                for r in rows])),
            "same_as_plain": float(np.mean([r["model"]["nguard"] == r["plain"]["nguard"] for r in ok])) if ok else None,
            "mean_cells_ratio_vs_largest": float(np.mean([r.get("cells_ratio_vs_largest", 1.0) for r in rows])),
        }
        with open(a.report, "w") as f:
            json.dump({"summary": summary, "rows": rows}, f, indent=1)
        log(json.dumps(summary))
    else:
        model = load(a.model)
        lvg = LocalVsGlobal(a.domain, a.split, a.precision)
        run = Run(order=a.order, cdt=a.cdt, lam=a.lam, width=a.width)
        g1 = lvg.fields(run, synth.rng_for(5, 3000))
        r = compare(model, lvg, run, g1, a.steps, a.tol)
        r.update({"domain": a.domain, "split": a.split, "precision": a.precision})
        with open(a.report, "w") as f:
            json.dump(r, f, indent=1)
        log(json.dumps(r))
        del g1
        torch.cuda.empty_cache()


if __name__ == "__main__":
    _main()
