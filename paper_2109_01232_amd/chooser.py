"""Learned parameter chooser for GMRES-IR: features -> MLP -> (m, inner cap, degree).

The paper's restart-length study (Section "Choosing a Restart Size for
GMRES-IR") shows that the fastest restart length depends on the problem:
small m wins when orthogonalisation dominates, large m stalls the fp32 inner
solve; polynomial preconditioning shifts the cost toward SpMV (Section
"Convergence and Kernel Speedup for Preconditioned GMRES vs GMRES-IR").  The
chooser learns that mapping from solver sweeps the method itself generates.

Pipeline (every numerical step runs in the library's HIP kernels):

* ``gmresir_features``: 16 fp32 features of (A, b).
* ``sweep``: per system, the default (m = 50, cap = m, degree 0) and 16
  grid points drawn at random, each timed end to end (polynomial set-up
  included) and cut off at twice the incumbent's time (an iteration budget
  from the per-iteration byte model); the label is the fastest configuration
  reaching the fp64 residual target.
* ``train``: Adam on the mean squared error of the encoded label
  (log2 m, log2(cap/m), degree/40) with ``gmresir_mlp_train_step``.
* ``choose``: features -> ``gmresir_mlp_forward`` -> snap to the grid.
  ``solve_with_chooser`` falls back to the defaults whenever the predicted
  configuration does not reach the target.

Command line (GPU): ``python -m paper_2109_01232_amd.chooser sweep|train|evaluate ...``.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

from . import binding as B
from . import problems as P

M_GRID = (10, 20, 30, 50, 75, 100, 150, 200)
CAP_GRID = (1, 2, 4)
DEG_GRID = (0, 5, 10, 20, 30, 40)
DEFAULT = (50, 1, 0)
RTOL = 1e-10
WEIGHTS_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "chooser_weights.json")


def encode(m: int, capm: int, deg: int) -> np.ndarray:
    return np.array([math.log2(m), math.log2(capm), deg / 40.0])


def snap(y) -> tuple:
    m = min(M_GRID, key=lambda v: abs(math.log2(v) - y[0]))
    c = min(CAP_GRID, key=lambda v: abs(math.log2(v) - y[1]))
    d = min(DEG_GRID, key=lambda v: abs(v / 40.0 - y[2]))
    return (m, c, d)


def grid() -> list:
    return [(m, c, d) for m in M_GRID for c in CAP_GRID for d in DEG_GRID]


class Runner:
    """Times solves of one system on the GPU (inputs resident before timing)."""

    def __init__(self, system, device="cuda"):
        import torch

        self.torch = torch
        self.system = system
        self.M = B.Matrix.from_csr(system.A, device)
        self.b = torch.from_numpy(system.b).to(device)
        self.x = torch.zeros_like(self.b)
        self.ws = B.Workspace(device)
        self.roots = {}

    def features(self) -> np.ndarray:
        return B.gmresir_features(self.M, self.b, ws=self.ws)

    def run(self, cfg, max_iters=200000) -> dict:
        torch = self.torch
        m, capm, deg = cfg
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        roots = None
        if deg > 0:
            roots = B.gmresir_poly_setup(self.M, deg, seed=12345, ws=self.ws)
        self.x.zero_()
        p = B.make_params(restart=m, inner="fp32", rtol=RTOL, inner_cap=m * capm, poly_degree=deg,
                          max_iters=max(int(max_iters), 1), check_mode=1)
        try:
            st, d, _ = B.gmresir_solve(self.M, self.b, self.x, p, poly_roots=roots, ws=self.ws)
        except B.GmresirError as e:
            st, d = e.status, {"iters": 0, "rel_resid_true": float("nan")}
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        return {"cfg": list(cfg), "status": int(st), "time": t, "iters": int(d["iters"]),
                "resid": float(d["rel_resid_true"]), "ok": st == B.OK}


def _iter_cost(cfg, n, nnz):
    """Relative cost per inner iteration (bytes model) used to turn a time
    budget into an iteration budget."""
    m, capm, deg = cfg
    spmv = 8.0 * nnz + 12.0 * n
    return (deg + 1) * spmv + 3.0 * 4.0 * n * (m / 2.0 + 1) + 16.0 * n


def sweep_system(seed: int, n_random: int, rng: np.random.Generator, n_max: float = 2e6) -> dict:
    sysm = P.chooser_system(seed, n_max=n_max)
    R = Runner(sysm)
    feats = R.features()
    R.run(DEFAULT, max_iters=200)  # warm-up (kernels, allocator)
    base = R.run(DEFAULT)
    runs = [base]
    best = base if base["ok"] else None
    t_it = base["time"] / max(base["iters"], 1)
    cost0 = _iter_cost(DEFAULT, sysm.A.n, sysm.A.nnz)
    cands = [c for c in grid() if c != DEFAULT]
    idx = rng.choice(len(cands), size=min(n_random, len(cands)), replace=False)
    for cfg in [cands[i] for i in idx]:
        budget_t = 2.0 * (best["time"] if best else base["time"] * 4)
        per_it = t_it * _iter_cost(cfg, sysm.A.n, sysm.A.nnz) / cost0
        r = R.run(cfg, max_iters=max(10, int(budget_t / per_it)))
        runs.append(r)
        if r["ok"] and (best is None or r["time"] < best["time"]):
            best = r
    return {"seed": seed, "n": sysm.A.n, "nnz": sysm.A.nnz, "meta": sysm.meta, "features": feats.tolist(),
            "runs": runs, "best": best["cfg"] if best else None,
            "best_time": best["time"] if best else None, "default_time": base["time"] if base["ok"] else None}


def cmd_sweep(args):
    rng = np.random.default_rng(args.rng_seed + args.start)
    with open(args.out, "a") as f:
        for seed in range(args.start, args.stop):
            t0 = time.time()
            rec = sweep_system(seed, args.n_random, rng, args.n_max)
            f.write(json.dumps(rec) + "\n")
            f.flush()
            print(f"[sweep] seed {seed} n={rec['n']} default={rec['default_time']} best={rec['best']} "
                  f"{rec['best_time']} ({time.time() - t0:.1f}s)", flush=True)


def load_records(paths):
    recs = []
    for p in paths:
        with open(p) as f:
            recs += [json.loads(line) for line in f if line.strip()]
    recs = [r for r in recs if r["best"] is not None]
    recs.sort(key=lambda r: r["seed"])
    return recs


def train(recs, steps=4000, lr=3e-3, batch=256, seed=0, device="cuda"):
    """Adam on the GPU through gmresir_mlp_train_step; returns the weight record."""
    import torch

    X = np.array([r["features"] for r in recs], dtype=np.float64)
    Y = np.array([encode(*r["best"]) for r in recs], dtype=np.float64)
    shift = X.mean(axis=0)
    sd = X.std(axis=0)
    scale = np.where(sd > 1e-12, 1.0 / np.where(sd > 1e-12, sd, 1.0), 0.0)
    rng = np.random.default_rng(seed)
    layers = []
    for fi, fo in ((16, 64), (64, 64), (64, 3)):
        lim = math.sqrt(6.0 / (fi + fo))
        layers.append((rng.uniform(-lim, lim, (fi, fo)), np.zeros(fo)))
    p0 = np.concatenate([np.concatenate([W.ravel(), b]) for W, b in layers]).astype(np.float32)
    f32 = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(device)
    Pd, Md, Vd = f32(p0), torch.zeros(len(p0), device=device), torch.zeros(len(p0), device=device)
    Xd, Yd, sh, sc = f32(X), f32(Y), f32(shift), f32(scale)
    loss = torch.zeros(1, device=device)
    n = len(recs)
    hist = []
    for step in range(1, steps + 1):
        if n > batch:
            ix = torch.from_numpy(rng.choice(n, batch, replace=False)).to(device)
            xb, yb = Xd[ix].contiguous(), Yd[ix].contiguous()
        else:
            xb, yb = Xd, Yd
        cur_lr = lr * (0.5 * (1 + math.cos(math.pi * step / steps)) * 0.95 + 0.05)
        B.gmresir_mlp_train_step(Pd, Md, Vd, sh, sc, xb, yb, cur_lr, step, loss)
        if step % 500 == 0 or step == 1:
            hist.append((step, float(loss.item())))
    return {"params": Pd.cpu().numpy().tolist(), "shift": shift.astype(np.float32).tolist(),
            "scale": scale.astype(np.float32).tolist(), "loss_history": hist, "n_train": n}


class Chooser:
    def __init__(self, weights: dict, device="cuda"):
        import torch

        self.torch = torch
        f32 = lambda a: torch.tensor(np.asarray(a, dtype=np.float32), device=device)
        self.P = f32(weights["params"])
        self.shift = f32(weights["shift"])
        self.scale = f32(weights["scale"])
        self.device = device

    @classmethod
    def load(cls, path=WEIGHTS_PATH, device="cuda"):
        with open(path) as f:
            return cls(json.load(f), device)

    def predict_raw(self, feats: np.ndarray) -> np.ndarray:
        torch = self.torch
        X = torch.tensor(np.atleast_2d(feats).astype(np.float32), device=self.device)
        Y = torch.empty((X.shape[0], 3), dtype=torch.float32, device=self.device)
        B.gmresir_mlp_forward(self.P, self.shift, self.scale, X, Y)
        return Y.cpu().numpy()

    def choose(self, feats: np.ndarray) -> tuple:
        return snap(self.predict_raw(feats)[0])


def solve_with_chooser(runner: Runner, chooser: Chooser, budget_factor: float = 1.0):
    """Predicted configuration, with the fixed defaults as fallback when it
    does not reach the target.  Returns (result of the accepted run, total
    time, configuration used, time of the choice).  The total includes the
    features (row statistics and a 10-step fp32 Arnoldi process) and the
    network's forward pass, which the fixed configurations do not pay, and any
    wasted attempt."""
    torch = runner.torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    feats = runner.features()
    cfg = chooser.choose(feats)
    t_choice = time.perf_counter() - t0
    r = runner.run(cfg)
    if r["ok"]:
        return r, t_choice + r["time"], cfg, t_choice
    d = runner.run(DEFAULT)
    return d, t_choice + r["time"] + d["time"], DEFAULT, t_choice


def cmd_train(args):
    recs = load_records(args.data)
    train_recs = [r for r in recs if r["seed"] < args.holdout_start]
    w = train(train_recs, steps=args.steps, lr=args.lr)
    w["grid"] = {"m": M_GRID, "cap_over_m": CAP_GRID, "degree": DEG_GRID}
    w["default"] = DEFAULT
    with open(args.out, "w") as f:
        json.dump(w, f)
    print(f"[train] {len(train_recs)} systems, loss history {w['loss_history']}", flush=True)


def cmd_evaluate(args):
    chooser = Chooser.load(args.weights)
    out = []
    for seed in range(args.start, args.stop):
        sysm = P.chooser_system(seed, n_max=args.n_max)
        R = Runner(sysm)
        R.run(DEFAULT, max_iters=200)
        base = R.run(DEFAULT)
        chooser.choose(R.features())  # warm-up of the feature and network kernels
        r, total, cfg, t_choice = solve_with_chooser(R, chooser)
        rec = {"seed": seed, "n": sysm.A.n, "family": sysm.meta.get("family"), "default": base, "chosen": list(cfg),
               "chosen_run": r,
               "choice_time": t_choice, "chosen_total": total,
               "speedup": (base["time"] / total) if base["ok"] else None}
        for fixed in args.also:
            fc = tuple(int(v) for v in fixed.split(","))
            fr = R.run(fc)
            ft = fr["time"] if fr["ok"] else fr["time"] + base["time"]
            rec["fixed_" + fixed] = {"run": fr, "speedup": (base["time"] / ft) if base["ok"] else None}
        out.append(rec)
        print(f"[eval] seed {seed} n={sysm.A.n} default {base['time']:.4f}s chosen {cfg} {total:.4f}s "
              f"ok={r['ok']} speedup={rec['speedup']}", flush=True)
    with open(args.out, "w") as f:
        for rec in out:
            f.write(json.dumps(rec) + "\n")
    sp = np.array([r["speedup"] for r in out if r["speedup"] is not None])
    if len(sp):
        summary = {"systems": len(sp), "geomean_speedup": float(np.exp(np.log(sp).mean())),
                   "median_speedup": float(np.median(sp)), "frac_improved": float(np.mean(sp > 1.0)),
                   "worst": float(sp.min()), "best": float(sp.max()),
                   "fallbacks": int(sum(1 for r in out if not r["chosen_run"]["ok"])),
                   "median_choice_time_s": float(np.median([r["choice_time"] for r in out]))}
        for fixed in args.also:
            fs = np.array([r["fixed_" + fixed]["speedup"] for r in out if r["fixed_" + fixed]["speedup"]])
            summary["fixed_" + fixed + "_geomean_speedup"] = float(np.exp(np.log(fs).mean()))
        print(json.dumps(summary), flush=True)


def main(argv=None):
    ap = argparse.ArgumentParser(prog="python -m paper_2109_01232_amd.chooser")
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("sweep")
    s.add_argument("--start", type=int, required=True)
    s.add_argument("--stop", type=int, required=True)
    s.add_argument("--n-random", type=int, default=16)
    s.add_argument("--n-max", type=float, default=2e6)
    s.add_argument("--rng-seed", type=int, default=2024)
    s.add_argument("--out", required=True)
    t = sub.add_parser("train")
    t.add_argument("--data", nargs="+", required=True)
    t.add_argument("--holdout-start", type=int, default=1800)
    t.add_argument("--steps", type=int, default=4000)
    t.add_argument("--lr", type=float, default=3e-3)
    t.add_argument("--out", default=WEIGHTS_PATH)
    e = sub.add_parser("evaluate")
    e.add_argument("--weights", default=WEIGHTS_PATH)
    e.add_argument("--start", type=int, default=1800)
    e.add_argument("--stop", type=int, default=2000)
    e.add_argument("--n-max", type=float, default=2e6)
    e.add_argument("--out", required=True)
    e.add_argument("--also", nargs="*", default=[], help="fixed configurations m,cap,deg timed beside, e.g. 50,1,10")
    args = ap.parse_args(argv)
    {"sweep": cmd_sweep, "train": cmd_train, "evaluate": cmd_evaluate}[args.cmd](args)


if __name__ == "__main__":
    main()
