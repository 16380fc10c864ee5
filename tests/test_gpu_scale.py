"""Parity at the benchmark sizes, in the launch form bench.py times.

Every column of the workload is solved in one call with the default options
(pipelined chunks, chemical potential bisected on the device).  The oracle
then solves a seeded sample of columns; their Ritz values, rho and pi (at the
GPU's chemical potential) must match to the precision mode's tolerance, and
the electron count N(mu) rebuilt from every column's Ritz values
and weights must equal the target.

Tolerances as in test_gpu_parity: FP64 max-abs rho/pi <= 1e-10; mixed_f64acc
max-abs rho <= 1e-5.
"""

import math
import sys

import numpy as np
import pytest

from paper_1202_0098_amd import synth

pytestmark = pytest.mark.gpu

RHO_TOL = {"fp64": 1e-10, "mixed_f64acc": 1e-5}
# Ritz values (eV).  FP64: rounding of the eigensolve.  mixed_f64acc: the
# basis SpMVs use FP32 operator values (rounding u = 6e-8 relative per entry,
# a perturbation of about u ||H||_inf = 4e-6 eV on the spd cell, whose rows sum
# to 67 eV in absolute value) and s_j comes from FP32 CG passes judged in FP64
# at the inner tolerance, which moves the block-2 Krylov space; measured
# 1.9e-5 eV on the sampled columns.  The stated tolerances of the method are
# those on rho and the band energy; this check bounds the Ritz values at 1e-4.
# FP64: the two sides' bases are rounded independently, and with p = q = 20
# the last vectors of a 40-dimensional space are close to dependent (the
# breakdown threshold is 1e-10), so the upper Ritz values carry the rounding
# amplified by the conditioning of the projected overlap: 1.6e-9 eV measured
# on the disordered cell; bounded at 1e-8 eV (5e-10 of ||H||_inf ~ 20 eV).
EPS_TOL = {"fp64": 1e-8, "mixed_f64acc": 1e-4}


def _say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _solve_all(torch, ctx, s, prec, autotune=False, **opt):
    import paper_1202_0098_amd as ma
    o = s.n_orb
    nu = s.p + s.q
    _say(f"{s.name} build")
    ctx.build_tb(s)
    rho = torch.zeros(s.nblk * o * o, dtype=torch.float64, device="cuda")
    pi = torch.zeros_like(rho)
    eps = torch.zeros(s.M * nu, dtype=torch.float64, device="cuda")
    wts = torch.zeros_like(eps)
    st = torch.zeros(s.M * ma.STATS, dtype=torch.int32, device="cuda")
    opts = ma.default_opts(precision=prec, **opt)
    if autotune:
        first = ctx.solve_columns(None, s.p, s.q, mu=math.nan, kT=s.kT, opts=opts)
        tun = ctx.autotune(None, s.p, s.q, mu=first.mu, kT=s.kT, opts=opts, reps=1)
        _say(f"{s.name} autotuned: {tun['basis_kernel']} kernel, {tun['slots_per_cu']} "
             f"slots/CU, schedule {tun['schedule']}")
    _say(f"{s.name} {prec}: all {s.M} columns, pipeline {opts.pipeline}")
    res = ctx.solve_columns(None, s.p, s.q, mu=math.nan, kT=s.kT, opts=opts, rho=rho, pi=pi,
                            eps=eps, wts=wts, col_stats=st)
    torch.cuda.synchronize()
    return res, rho, pi, eps, wts, st


def _full_solve_sampled(torch, s, prec, nsample, seed, extra_cols=(), autotune=False,
                        ctx=None, out=None):
    import oracle
    import paper_1202_0098_amd as ma
    o = s.n_orb
    nu = s.p + s.q
    if out is None:
        own = ctx is None
        if own:
            ctx = ma.Context(0)
        try:
            out = _solve_all(torch, ctx, s, prec, autotune)
        finally:
            if own:
                ctx.close()
    res, rho, pi, eps, wts, st = out
    rho = rho.view(s.nblk, o, o)
    pi = pi.view(s.nblk, o, o)
    eps = eps.view(s.M, nu)
    wts = wts.view(s.M, nu)
    st = st.view(s.M, ma.STATS)
    assert int((st[:, 3] != 0).sum()) == 0, "a column failed"

    # electron count at the returned mu, from every column's Ritz data (FP64,
    # on the device: 1/(1 + exp((eps - mu)/kT)) as a logistic)
    valid = torch.arange(nu, device="cuda")[None, :] < st[:, :1]
    x = (torch.where(valid, eps, torch.zeros_like(eps)) - res.mu) / s.kT
    f = torch.where(valid, torch.sigmoid(-x), torch.zeros_like(x))
    n_mu = float((f * torch.where(valid, wts, torch.zeros_like(wts))).sum())   # per spin
    _say(f"mu={res.mu:.12f} N(mu) per spin={n_mu:.9f} target={s.n_target}")
    assert abs(n_mu - s.n_target) <= 1e-6 * s.n_target

    cols = np.random.default_rng(seed).choice(s.M, nsample, replace=False)
    cols = np.unique(np.concatenate([cols, np.asarray(extra_cols, np.int64)])).astype(np.int32)
    _say(f"oracle on {len(cols)} sampled columns")
    raw = oracle.solve_raw(s, cols)
    assert raw["rc"] == 0
    tc = torch.from_numpy(cols.astype(np.int64)).cuda()
    nu_eff = st[tc, 0].cpu().numpy()
    assert np.array_equal(nu_eff, raw["nu_eff"]), "nu_eff differs"
    eps_s = eps[tc].cpu().numpy()
    ok = np.arange(nu)[None, :] < nu_eff[:, None]
    assert np.all(np.isfinite(eps_s[ok]))
    d_eps = float(np.max(np.where(ok, np.abs(eps_s - np.where(ok, raw["eps"], 0.0)), 0.0)))
    rr, pp, _, _ = oracle.outputs(s, raw, res.mu, s.kT)
    d_rho = d_pi = 0.0
    pi_scale = 1.0
    for c, j in enumerate(cols):
        A, r = divmod(int(j), o)
        k0, k1 = int(s.blk_ptr[A]), int(s.blk_ptr[A + 1])
        npat = (k1 - k0) * o
        g_rho = rho[k0:k1, r, :].reshape(-1).cpu().numpy()
        g_pi = pi[k0:k1, r, :].reshape(-1).cpu().numpy()
        d_rho = max(d_rho, float(np.abs(g_rho - rr[c, :npat]).max()))
        d_pi = max(d_pi, float(np.abs(g_pi - pp[c, :npat]).max()))
        pi_scale = max(pi_scale, float(np.abs(pp[c, :npat]).max()))
    _say(f"sampled: max|deps|={d_eps:.3e} max|drho|={d_rho:.3e} max|dpi|={d_pi:.3e}")
    assert d_eps <= EPS_TOL[prec]
    assert d_rho <= RHO_TOL[prec]
    assert d_pi <= RHO_TOL[prec] * pi_scale


def test_diamond4096_fp64_all_columns_pipelined(torch_cuda):
    """The 4,096-atom diamond cell, FP64, every column, as bench.py runs it."""
    _full_solve_sampled(torch_cuda, synth.config_diamond4096(), "fp64", 96, 21)


def test_fcc_spd262144_mixed_f64acc_all_columns_pipelined(torch_cuda):
    """The 262,144-atom spd fcc cell (2,359,296 columns), mixed precision with
    FP64 accumulation, every column, as bench.py runs it."""
    _full_solve_sampled(torch_cuda, synth.config_fcc_spd(), "mixed_f64acc", 32, 23)


def test_disordered8000_fp64_all_columns_autotuned(torch_cuda):
    """The 8,000-atom disordered cell (32,000 columns, regions of 60..260
    atoms, p = q = 20), FP64, every column after autotuning, in the default
    pipelined launch; the sample holds every column of the 4 atoms with the
    smallest and the 4 with the largest regions."""
    s = synth.config_disordered8000()
    order = np.argsort(s.region_nrp, kind="stable")
    atoms = np.concatenate([order[:4], order[-4:]])
    extra = (atoms[:, None] * s.n_orb + np.arange(s.n_orb)).ravel()
    _say(f"extreme regions: {s.region_nrp[order[:4]]} .. {s.region_nrp[order[-4:]]} atoms")
    _full_solve_sampled(torch_cuda, s, "fp64", 64, 31, extra_cols=extra, autotune=True)


def test_fcc_spd262144_geometry_update(torch_cuda):
    """One MD-style update of the 262,144-atom spd cell (Gaussian steps of
    0.02 A, pattern and regions rebuilt), solved from the s_j kept at the
    first geometry (start "previous") in the default launch; sampled columns
    against the oracle on the new geometry."""
    import paper_1202_0098_amd as ma
    s0 = synth.config_fcc_spd()
    ctx = ma.Context(0)
    try:
        _say("geometry 0: every column, keep s_j")
        r0 = _solve_all(torch_cuda, ctx, s0, "mixed_f64acc", keep_sj=1)
        it0 = float(r0[5].view(s0.M, ma.STATS)[:, 1].double().mean())
        del r0
        s1 = synth.md_updates(s0, 1, 0.02, seed0=5000)[0]
        del s0
        out = _solve_all(torch_cuda, ctx, s1, "mixed_f64acc", start="previous")
        st = out[5].view(s1.M, ma.STATS)
        it1 = float(st[:, 1].double().mean())
        used = np.bincount(st[:, 4].cpu().numpy(), minlength=5)
        _say(f"CG iterations: geometry 0 (zero start) {it0:.2f}, update 1 (previous) {it1:.2f}; "
             f"starts used {used}")
        assert used[3] >= 0.99 * s1.M
        assert it1 < it0
    finally:
        ctx.close()
    _full_solve_sampled(torch_cuda, s1, "mixed_f64acc", 32, 29, out=out)
