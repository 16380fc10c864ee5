#!/usr/bin/env python3
"""Throughput of the per-column multiple Arnoldi solve on one MI355X.

One step = one ma_solve_columns call over every column of the workload: inner
CG, S-orthonormal multiple-Krylov basis, Galerkin pair, reduced eigenproblem,
chemical-potential bisection, Fermi-weighted rho/pi and the scalar band energy
and electron count.  The system (H, S, regions) is built and resident in HBM
before the timed region; its build time is reported separately.

Prints one JSON line (rank 0).  Only one GPU is supported.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Green's-fn columns/s at fixed ρ_ij error; learned vs zero-start CG; HBM %peak"

# MI355X published peaks
PEAK_HBM_GBS = 8000.0
PEAK_FP64_VECTOR_TFLOPS = 78.6


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def workload(name):
    from paper_1202_0098_amd import synth
    if name == "diamond4096":
        return synth.config_diamond4096()
    if name == "diamond64":
        return synth.config_diamond64()
    if name == "disordered8000":
        return synth.config_disordered8000()
    if name == "fcc_spd":
        return synth.config_fcc_spd()
    if name == "fcc_spd16384":
        return synth.config_fcc_spd(cells=(16, 16, 16))
    raise SystemExit(f"unknown workload {name}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="fcc_spd",
                    help="fcc_spd (default: the 262,144-atom spd cell), fcc_spd16384, "
                         "diamond4096, disordered8000, diamond64")
    ap.add_argument("--precision", default=None, choices=["fp64", "mixed", "mixed_f64acc"],
                    help="default: mixed_f64acc for the spd cells, fp64 otherwise")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--tuning", default="",
                    help="fixed launch shape 'SLOTS_PER_CU,SCHEDULE[,BASIS_KERNEL[,PIPELINE]]' "
                         "instead of the autotuner")
    ap.add_argument("--no-graph", action="store_true", help="launch without hipGraph replay")
    ap.add_argument("--pipeline", type=int, default=-1,
                    help="chunks pipelining the eigensolver beside the basis kernel (default: "
                         "the autotuned choice, else 4; 0 = chunks in sequence, one chunk "
                         "replayed as hipGraphs)")
    ap.add_argument("--chunk-columns", type=int, default=0,
                    help="columns per chunk of the solve (0: the library's choice)")
    ap.add_argument("--basis-kernel", default="auto",
                    choices=["auto", "onchip", "workspace", "group", "atom"],
                    help="basis kernel: on-chip basis (regions up to 512 orbitals) or workspace")
    ap.add_argument("--copy-calib", type=int, default=0, metavar="MIB",
                    help="after the timed steps, run a plain device copy of MIB MiB five times "
                         "(reference kernel for HBM byte counters)")
    ap.add_argument("--cpu-sample", type=int, default=-1,
                    help="columns of the oracle CPU baseline sample (0 = skip, -1 = whole "
                         "workload up to 16,384 columns)")
    ap.add_argument("--region-buckets", type=int, default=0, metavar="N",
                    help="after the timed steps, solve the columns of N groups of atoms of "
                         "ascending region size one group at a time (at the bisected mu) and "
                         "report columns/s per group")
    ap.add_argument("--updates", type=int, default=0, metavar="K",
                    help="after the timed steps, K MD-style geometry updates (Gaussian steps "
                         "of 0.02 A, pattern rebuilt), each solved from the zero start and "
                         "from the s_j kept at the previous geometry")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import torch
    import paper_1202_0098_amd as ma

    if args.precision is None:
        args.precision = "mixed_f64acc" if args.workload.startswith("fcc_spd") else "fp64"
    if not torch.cuda.is_available():
        raise SystemExit("no GPU visible")
    t_gen = time.perf_counter()
    s = workload(args.workload)
    log(f"workload {s.name}: atoms={s.n_atoms} M={s.M} blocks={s.nblk} p={s.p} q={s.q} "
        f"(generated in {time.perf_counter() - t_gen:.1f} s)")
    ctx = ma.Context(0)
    t0 = time.perf_counter()
    ctx.build_tb(s)
    build_s = time.perf_counter() - t0
    info = ctx.info()
    log(f"built in {build_s:.2f}s: {info}")
    o = s.n_orb
    nu = s.p + s.q
    dev = "cuda"
    rho = torch.zeros(s.nblk * o * o, dtype=torch.float64, device=dev)
    pi = torch.zeros_like(rho)
    stats = torch.zeros(s.M * ma.STATS, dtype=torch.int32, device=dev)
    opts = ma.default_opts(precision=args.precision, use_graph=0 if args.no_graph else 1,
                           basis_kernel=args.basis_kernel)
    if args.pipeline >= 0:
        opts.pipeline = args.pipeline
    if args.chunk_columns > 0:
        opts.chunk_columns = args.chunk_columns
    tuning = None
    if args.tuning:
        parts = args.tuning.split(",")
        slots, sched = parts[:2]
        kern = parts[2] if len(parts) >= 3 else args.basis_kernel
        pipe = int(parts[3]) if len(parts) >= 4 else -1
        ctx.set_tuning(s.p, s.q, args.precision, int(slots), sched, kern, pipe)
        tuning = {"slots_per_cu": int(slots), "schedule": sched, "basis_kernel": kern,
                  "pipeline": pipe}
        log(f"fixed tuning {tuning}")
    elif not args.no_autotune:
        t0 = time.perf_counter()
        # large systems: tune on every column of a compact block of atoms
        # (about 65,536 columns: the atoms nearest to a seeded atom; whole
        # atoms, as the atom-lockstep kernels process all columns of an atom
        # together).  The schedules differ mostly in how much the regions of
        # the atoms in flight together overlap, which a sample spread over
        # the cell would not show.
        tcols = None
        if s.M > 65536:
            na = 65536 // o
            box = np.asarray(s.box, float)
            c = s.pos[np.random.default_rng(99).integers(s.n_atoms)]
            d = s.pos - c
            d -= box * np.round(d / box)
            atoms = np.sort(np.argsort((d * d).sum(1), kind="stable")[:na])
            tcols = (atoms[:, None] * o + np.arange(o)).ravel().astype(np.int32)
        first = ctx.solve_columns(tcols, s.p, s.q, mu=math.nan, kT=s.kT, opts=opts)
        log(f"first solve {first.elapsed_ms:.1f} ms (mu {first.mu:.6f}); autotuning")
        tuning = ctx.autotune(tcols, s.p, s.q, mu=first.mu, kT=s.kT, opts=opts, reps=2)
        log(f"autotune ({time.perf_counter() - t0:.1f}s): {tuning['basis_kernel']} basis kernel, "
            f"{tuning['slots_per_cu']} slots/CU, schedule {tuning['schedule']}, pipeline "
            f"{tuning['pipeline']}, {tuning['best_ms']:.2f} ms; tried "
            f"{[(k, a, b, pl, round(c, 2)) for (a, b, c, k), pl in zip(tuning['tried'], tuning['tried_pipeline'])]}")

    def step():
        return ctx.solve_columns(None, s.p, s.q, mu=math.nan, kT=s.kT, opts=opts,
                                 rho=rho, pi=pi, col_stats=stats)

    log("warmup")
    for w in range(args.warmup):
        r = step()
        log(f"warmup {w}: {r.elapsed_ms:.2f} ms (basis {r.kernel_ms:.2f} ms, eig {r.eig_ms:.2f} ms) E={r.energy:.6f} "
            f"N={r.n_elec:.6f} mu={r.mu:.9f}")
    torch.cuda.synchronize()
    kernel_ms, eig_ms = [], []
    t0 = time.perf_counter()
    for k in range(args.steps):
        r = step()
        kernel_ms.append(r.kernel_ms)
        eig_ms.append(r.eig_ms)
        if s.M > 65536:
            log(f"step {k}: {r.elapsed_ms:.1f} ms")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = 1e3 * wall / args.steps
    cols_per_s = s.M / (wall / args.steps)
    st = stats.cpu().numpy().reshape(s.M, ma.STATS)
    log(f"timed {args.steps} steps: {ms_per_step:.3f} ms/step, {cols_per_s:.4g} columns/s; "
        f"nu_eff mean {st[:, 0].mean():.2f}, CG iters mean {st[:, 1].mean():.2f}")
    if args.copy_calib > 0:
        # a plain elementwise copy: reads and writes exactly MIB MiB per launch
        n = args.copy_calib * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        for _ in range(5):
            torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        log(f"copy calibration: 5 launches of {args.copy_calib} MiB read + {args.copy_calib} MiB written")
        del a, b

    buckets = region_buckets(ctx, s, opts, r.mu, args.region_buckets) \
        if args.region_buckets > 0 else None
    updates = geometry_updates(ctx, s, opts, args.updates) if args.updates > 0 else None
    if updates is not None:
        ctx.build_tb(s)

    # ---- roofline of the column kernel -------------------------------------
    k_ms = float(np.mean(kernel_ms))
    reg_atoms, loc_blocks = ctx.region_sizes(s.n_atoms)
    counts = kernel_model(s, st, reg_atoms, loc_blocks, args.precision)
    achieved_gbs = counts["bytes"] / (k_ms * 1e-3) / 1e9
    copy_gbs = copy_bandwidth(torch)
    log(f"measured copy bandwidth {copy_gbs:.0f} GB/s")
    roofline = {
        "bound": "hbm",
        "achieved": round(achieved_gbs, 2),
        "peak": PEAK_HBM_GBS,
        "unit": "GB/s",
        "frac": round(achieved_gbs / PEAK_HBM_GBS, 5),
        "traffic": measured_traffic(s.name, args.precision),
        "algorithmic_bytes": round(counts["bytes"]),
        "operator_applications_per_column": round(counts["n_app"], 3),
        "measured_copy_peak": round(copy_gbs, 1),
        "frac_of_measured_copy": round(achieved_gbs / copy_gbs, 5),
        "kernel": "basis kernel",
        "kernel_ms": round(k_ms, 4),
        "eig_kernel_ms": round(float(np.mean(eig_ms)), 4),
        "fp64_tflops": round(counts["flops"] / (k_ms * 1e-3) / 1e12, 4),
    }

    # ---- CPU baseline: the oracle on a bounded sample ----------------------
    cpu = None
    default_sample = 16384 if s.n_orb <= 4 else 4096   # about 10-30 s on 16 host cores
    sample = min(s.M, default_sample) if args.cpu_sample < 0 else min(args.cpu_sample, s.M)
    if sample > 0:
        import oracle
        cols = np.sort(np.random.default_rng(12345).choice(s.M, sample,
                                                           replace=False)).astype(np.int32)
        oracle.build()
        t0 = time.perf_counter()
        res = oracle.solve(s, cols=cols)
        dt = time.perf_counter() - t0
        cpu = {"value": round(len(cols) / dt, 2), "unit": "columns/s",
               "cores": oracle.num_threads(), "kind": "oracle",
               "sample": f"{len(cols)} seeded random columns of the same workload "
                         f"(regions, CG, basis, eigensolve, bisection over the sample), "
                         f"{dt:.1f} s"}
        log(f"cpu oracle: {cpu}")

    out = {
        "metric": METRIC,
        "value": round(cols_per_s, 2),
        "unit": "columns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": s.name, "atoms": s.n_atoms, "columns": s.M, "p": s.p, "q": s.q,
                   "kT": s.kT, "mu": "bisected at half filling", "precision": args.precision,
                   "build_s": round(build_s, 3),
                   "launch": launch_form(opts, tuning, s.M, args.no_graph),
                   "basis_kernel": args.basis_kernel,
                   "tuning": None if tuning is None else {
                       "slots_per_cu": tuning["slots_per_cu"], "schedule": tuning["schedule"],
                       "basis_kernel": tuning["basis_kernel"],
                       "pipeline": tuning["pipeline"]}},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    if buckets is not None:
        out["region_buckets"] = buckets
    if updates is not None:
        out["geometry_updates"] = updates
    print(json.dumps(out), flush=True)


def launch_form(opts, tuning, ncols, no_graph):
    """How the library launches a solve of ncols columns with these options
    (the pipeline option: explicit, else the tuned one, else 4)."""
    pipe = opts.pipeline if opts.pipeline >= 0 else (
        tuning["pipeline"] if tuning is not None and tuning.get("pipeline", -1) >= 0 else 4)
    if pipe >= 2 and ncols >= pipe * 2048:
        return "eager, eigensolver pipelined beside the basis kernel"
    if no_graph:
        return "eager, chunks in sequence"
    return "chunks in sequence on one stream (one chunk: hipGraph replay)"


def region_buckets(ctx, s, opts, mu, nb, reps=3):
    """Columns/s by region size: the atoms sorted by region size and cut
    into nb groups of equal atom count; each group's columns solved alone
    (mu given, the launch shape of the full solve), best of reps by device
    time."""
    import paper_1202_0098_amd as ma
    o = s.n_orb
    reg_atoms, _ = ctx.region_sizes(s.n_atoms)
    order = np.argsort(reg_atoms, kind="stable")
    out = []
    for g in np.array_split(order, nb):
        cols = (np.sort(g)[:, None] * o + np.arange(o)).ravel().astype(np.int32)
        best = math.inf
        for _ in range(reps):
            r = ctx.solve_columns(cols, s.p, s.q, mu=mu, kT=s.kT, opts=opts)
            best = min(best, r.elapsed_ms)
        out.append({"region_atoms": [int(reg_atoms[g].min()), int(reg_atoms[g].max())],
                    "mean_region_atoms": round(float(reg_atoms[g].mean()), 1),
                    "columns": len(cols), "ms": round(best, 3),
                    "columns_per_s": round(len(cols) / (best * 1e-3), 1)})
        log(f"region bucket {out[-1]}")
    return out


def geometry_updates(ctx, s, opts, k_updates, sigma=0.02):
    """k_updates MD-style updates of the workload (Gaussian steps of sigma,
    seeds seed + k, pattern and regions rebuilt); each update is solved from
    the zero start and from the s_j kept at the previous geometry.  Returns
    per update: device ms, mean CG iterations and columns/s of both starts."""
    import torch
    import paper_1202_0098_amd as ma
    from paper_1202_0098_amd import synth
    o = s.n_orb
    st = torch.zeros(s.M * ma.STATS, dtype=torch.int32, device="cuda")
    keep = type(opts).from_buffer_copy(opts)
    keep.keep_sj = 1
    ctx.solve_columns(None, s.p, s.q, mu=math.nan, kT=s.kT, opts=keep)
    out = []
    cur = s
    for k in range(1, k_updates + 1):
        t0 = time.perf_counter()
        cur = synth.md_updates(cur, 1, sigma, seed0=s.seed + k - 1)[0]
        gen_s = time.perf_counter() - t0
        t0 = time.perf_counter()
        ctx.build_tb(cur)
        build_s = time.perf_counter() - t0
        rec = {"update": k, "seed": int(cur.seed), "generate_s": round(gen_s, 2),
               "build_s": round(build_s, 3)}
        for name, start in (("zero", 0), ("previous", 2)):
            o2 = type(opts).from_buffer_copy(opts)
            o2.start = start
            o2.keep_sj = 1 if start == 2 else 0
            r = ctx.solve_columns(None, cur.p, cur.q, mu=math.nan, kT=cur.kT, opts=o2,
                                  col_stats=st)
            torch.cuda.synchronize()
            a = st.cpu().numpy().reshape(cur.M, ma.STATS)
            rec[name] = {"ms": round(r.elapsed_ms, 2), "basis_ms": round(r.kernel_ms, 2),
                         "cg_iters_mean": round(float(a[:, 1].mean()), 3),
                         "columns_per_s": round(cur.M / (r.elapsed_ms * 1e-3), 1),
                         "energy": r.energy, "mu": r.mu}
        log(f"update {rec}")
        out.append(rec)
    return out


def device_source_digest():
    """SHA-256 over the device sources of the library (sorted by name)."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_1202_0098_amd", "csrc")
    h = hashlib.sha256()
    for fn in sorted(os.listdir(csrc)):
        if fn.endswith(".hip") or fn in ("ma_device.h", "ma_internal.h"):
            with open(os.path.join(csrc, fn), "rb") as f:
                h.update(fn.encode() + b"\0" + f.read())
    return h.hexdigest()


def measured_traffic(workload_name, precision):
    """HBM bytes per step of the basis kernel (summed over its launches in a
    step) from the committed counter summary of this workload and precision
    (FETCH_SIZE + WRITE_SIZE, each scaled by the same counter on a plain copy
    of known size), or None when there is none or the kernel source has
    changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"k_basis_{workload_name}_{precision}_traffic.md")
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as f:
        for line in f:
            if line.startswith("- ") and ": " in line:
                k, v = line[2:].split(": ", 1)
                fields[k.strip()] = v.strip().strip("`")
    if fields.get("kernel source sha256") != device_source_digest():
        return None
    try:
        return float(fields["HBM bytes per step"])
    except (KeyError, ValueError):
        return None


def kernel_model(s, st, reg_atoms, loc_blocks, precision):
    """Algorithmic bytes and flops of the basis kernel over one step
    (operator-streaming model).

    Per column j of atom A, with nb local operator blocks (o x o each, H and S
    share the pattern), L accepted basis vectors and c CG iterations:
      n_app  = 2 L + c (+1 when the learned start was used: its residual
               check) operator applications -- H and S once per basis vector,
               S once per CG iteration; the H product of the block-2 chain
               rides in the same operator pass and streams nothing extra
      bytes  = n_app nb (o^2 v + 4) / o + 16 |pattern(j)|: every application
               streams the region operator once (v = 8 bytes per FP64 value,
               4 per FP32 value, 4 bytes of block index), shared by the o
               columns of the atom, and rho and pi are written once (FP64)
      flops  = 2 o^2 nb per application and column, plus ~8 n L^2 FP64
               flops of Gram-Schmidt and projection
    """
    o = s.n_orb
    a = np.arange(s.M) // o
    L = st[:, 0].astype(float)
    c = st[:, 1].astype(float) + (st[:, 4] == 1).astype(float)
    nb = loc_blocks[a].astype(float)
    npat = np.diff(s.blk_ptr)[a].astype(float) * o
    n = reg_atoms[a].astype(float) * o
    apps = 2 * L + c
    vbytes = 8 if precision == "fp64" else 4
    bytes_ = float(np.sum(apps * nb * (o * o * vbytes + 4) / o + 16 * npat))
    flops = float(np.sum(2 * o * o * nb * apps + 8 * n * L * L))
    return {"flops": flops, "bytes": bytes_, "n_app": float(np.mean(apps))}


def copy_bandwidth(torch, mib=2048, reps=10):
    """Measured HBM bandwidth of a plain elementwise copy (read + write of
    MIB MiB each), timed with events on the current stream: the achievable
    second denominator beside the published peak."""
    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.mul(a, 1.0, out=b)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        torch.mul(a, 1.0, out=b)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2 * n * 8 / (ms * 1e-3) / 1e9


if __name__ == "__main__":
    main()
