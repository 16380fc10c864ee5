"""Training and evaluation of the learned CG start (driver around the library).

Training pairs (descriptor of column j, s_j on the orbitals of the 12 atoms
nearest to atom(j)) come from the library's own CG solves (FP64, tolerance
1e-12) on training geometries; the network is trained by the library's FP32
forward/backward/Adam kernels.  PyTorch only holds the device arrays and the
shuffled index batches; the standardisation of inputs and targets is computed
on the host.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

from . import Context, default_opts, STATS
from . import synth


def collect_pairs(ctx: Context, tb, cols=None, cg_tol=1e-12):
    """Descriptors and converged s_j coefficients for columns of `tb` (device)."""
    import torch
    ctx.build_tb(tb)
    sh = ctx.mlp_shape()
    cols = np.arange(tb.M, dtype=np.int32) if cols is None else np.asarray(cols, np.int32)
    n = len(cols)
    feat = torch.empty(n * sh["n_in"], dtype=torch.float32, device="cuda")
    ctx.column_features(cols, feat)
    sj = torch.empty(n * sh["n_out"], dtype=torch.float32, device="cuda")
    # the CG alone is needed: smallest subspace (p = 1, q = 0)
    ctx.solve_columns(cols, 1, 0, mu=0.0, kT=tb.kT, opts=default_opts(cg_tol=cg_tol, use_graph=0),
                      sj_near=sj)
    torch.cuda.synchronize()
    return feat.view(n, sh["n_in"]), sj.view(n, sh["n_out"])


def train(ctx: Context, X, T, epochs=20, batch=1024, lr=1e-3, seed=0, log=None):
    """Adam on the mean squared error with standardised inputs and targets
    (per feature / output: zero mean, unit spread, computed on the host).
    Both standardisations are folded into the first and last layers
    afterwards, so the network maps raw descriptors to s_j coefficients.
    Returns the mean (standardised) loss of every epoch."""
    import torch
    n = X.shape[0]
    Xh = X.cpu().numpy().astype(np.float64)
    Th = T.cpu().numpy().astype(np.float64)
    xm, xs = Xh.mean(0), Xh.std(0, ddof=1)
    xs = np.where(xs > 1e-6, xs, 1.0)
    mean, std = Th.mean(0), np.maximum(Th.std(0, ddof=1), 1e-6)
    Xs = torch.from_numpy(((Xh - xm) / xs).astype(np.float32)).cuda()
    Ts = torch.from_numpy(((Th - mean) / std).astype(np.float32)).cuda()
    del Xh, Th
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    history = []
    for ep in range(epochs):
        perm = torch.randperm(n, generator=gen, device="cuda").to(torch.int32)
        losses = []
        for b in range(0, n - batch + 1, batch):
            losses.append(ctx.mlp_train_step(Xs, Ts, batch, lr, idx=perm[b:b + batch]))
        history.append(float(np.mean(losses)))
        if log:
            log(f"epoch {ep}: loss {history[-1]:.3e}")
    # fold x' = (x - xm) / xs into W1 (n_in x n_hidden, row-major) and b1, and
    # y = std * y' + mean into W3 (n_hidden x n_out) and b3
    sh = ctx.mlp_shape()
    p = ctx.mlp_get_params().astype(np.float64)
    ni, no, nh = sh["n_in"], sh["n_out"], sh["n_hidden"]
    xmn, xsn = xm, xs
    w1 = p[:ni * nh].reshape(ni, nh)
    b1 = p[ni * nh:ni * nh + nh] - (xmn / xsn) @ w1
    p[:ni * nh] = (w1 / xsn[:, None]).ravel()
    p[ni * nh:ni * nh + nh] = b1
    sd, mu = std, mean
    w3 = p[-no - nh * no:-no].reshape(nh, no) * sd[None, :]
    b3 = p[-no:] * sd + mu
    p[-no - nh * no:-no] = w3.ravel()
    p[-no:] = b3
    ctx.mlp_set_params(p.astype(np.float32))
    return history


def save(ctx: Context, path: str, meta: dict):
    p = ctx.mlp_get_params()
    np.save(path + ".npy", p)
    with open(path + ".json", "w") as f:
        json.dump(dict(meta, shape=ctx.mlp_shape()), f, indent=1)


def load(ctx: Context, path: str):
    ctx.mlp_set_params(np.load(path + ".npy"))
    with open(path + ".json") as f:
        return json.load(f)


def cg_stats(ctx: Context, tb, start: str, cg_tol=1e-8, precision="fp64", reps=3, mu=None):
    """Solve all columns of `tb` (already built) with the given start: CG
    iterations (mean, p95), FP64 residual checks, fallbacks, columns/s (best
    of reps, graph replay)."""
    import torch
    stats = torch.zeros(tb.M * STATS, dtype=torch.int32, device="cuda")
    o = tb.n_orb
    rho = torch.zeros(tb.nblk * o * o, dtype=torch.float64, device="cuda")
    opts = default_opts(cg_tol=cg_tol, precision=precision, start=start)
    mu = math.nan if mu is None else mu
    best, res = math.inf, None
    for _ in range(reps):
        r = ctx.solve_columns(None, tb.p, tb.q, mu=mu, kT=tb.kT, opts=opts, rho=rho, col_stats=stats)
        if r.elapsed_ms < best:
            best, res = r.elapsed_ms, r
    st = stats.cpu().numpy().reshape(tb.M, STATS)
    return dict(cg_mean=float(st[:, 1].mean()), cg_p95=float(np.percentile(st[:, 1], 95)),
                judge_mean=float(st[:, 2].mean()), fallback=float(np.mean(st[:, 4] == 2)),
                learned=float(np.mean(st[:, 4] == 1)), ms=best, cols_per_s=tb.M / (best * 1e-3),
                energy=res.energy, mu=res.mu, rho=rho.cpu().numpy())


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--model", default="sp3", choices=["sp3", "spd"],
                    help="sp3: train on diamond cells, evaluate on disordered cells; spd: train "
                         "on small fcc spd cells, evaluate on a larger fcc spd cell")
    ap.add_argument("--train-seeds", default="")
    ap.add_argument("--eval-seeds", default="")
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--cg-tol", type=float, default=1e-8)
    ap.add_argument("--precision", default="mixed_f64acc")
    ap.add_argument("--eval-atoms", type=int, default=8000)
    ap.add_argument("--eval-cells", default="16,16,16")
    ap.add_argument("--save", default="")
    ap.add_argument("--json", default="")
    args = ap.parse_args(argv)
    spd = args.model == "spd"
    train_seeds = args.train_seeds or ("5101-5112" if spd else "2101-2112")
    eval_seeds = args.eval_seeds or ("5000-5000" if spd else "3001-3005")

    def rng(s):
        a, b = (int(v) for v in s.split("-"))
        return list(range(a, b + 1))

    def log(*a):
        print("[learned]", *a, flush=True)

    ctx = Context(0)
    t0 = time.perf_counter()
    Xs, Ts = [], []
    if spd:
        train_systems = [lambda sd=sd: synth.config_fcc_spd(sd, cells=(8, 8, 8))
                         for sd in rng(train_seeds)]
    else:
        train_systems = [lambda: synth.config_diamond64(1001)] + \
                        [lambda sd=sd: synth.config_diamond4096(sd) for sd in rng(train_seeds)]
    for make in train_systems:
        X, T = collect_pairs(ctx, make())
        Xs.append(X)
        Ts.append(T)
    import torch
    X = torch.cat(Xs).contiguous()
    T = torch.cat(Ts).contiguous()
    log(f"{X.shape[0]} training pairs in {time.perf_counter() - t0:.1f}s")
    ctx.mlp_init(seed=7)
    t0 = time.perf_counter()
    hist = train(ctx, X, T, epochs=args.epochs, batch=args.batch, lr=args.lr, log=log)
    train_s = time.perf_counter() - t0
    log(f"trained {args.epochs} epochs in {train_s:.1f}s, final loss {hist[-1]:.3e}")
    if args.save:
        save(ctx, args.save, dict(model=args.model, train_seeds=train_seeds, epochs=args.epochs,
                                  loss=hist[-1]))
    results = []
    cells = tuple(int(v) for v in args.eval_cells.split(","))
    for seed in rng(eval_seeds):
        tb = (synth.config_fcc_spd(seed, cells=cells) if spd
              else synth.config_disordered8000(seed, n_atoms=args.eval_atoms))
        ctx.build_tb(tb)
        ref = cg_stats(ctx, tb, "zero", 1e-12, "fp64", reps=1)
        z = cg_stats(ctx, tb, "zero", args.cg_tol, args.precision, mu=ref["mu"])
        l = cg_stats(ctx, tb, "learned", args.cg_tol, args.precision, mu=ref["mu"])
        ez = float(np.abs(z["rho"] - ref["rho"]).max())
        el = float(np.abs(l["rho"] - ref["rho"]).max())
        row = dict(seed=seed, system=tb.name, zero={k: v for k, v in z.items() if k != "rho"},
                   learned={k: v for k, v in l.items() if k != "rho"},
                   rho_err_zero=ez, rho_err_learned=el)
        log(f"{tb.name} seed {seed}: CG iterations {z['cg_mean']:.2f} -> {l['cg_mean']:.2f} "
            f"(p95 {z['cg_p95']:.0f} -> {l['cg_p95']:.0f}), FP64 residual checks "
            f"{z['judge_mean']:.2f} -> {l['judge_mean']:.2f}, fallback {l['fallback']:.3f}, "
            f"columns/s {z['cols_per_s']:.4g} -> {l['cols_per_s']:.4g}, "
            f"max|rho - rho(FP64, tol 1e-12)| zero {ez:.2e} learned {el:.2e}")
        results.append(row)
    out = dict(model=args.model, train_pairs=int(X.shape[0]), train_s=train_s, loss_history=hist,
               eval=results, cg_tol=args.cg_tol, precision=args.precision)
    if args.json:
        with open(args.json, "w") as f:
            json.dump(out, f, indent=1)
    return out


if __name__ == "__main__":
    main()
