"""The allocation-free entry point (GPU): ma_solve_columns_noalloc against
ma_solve_columns on the same inputs, two calls in a row (the second smaller,
so it runs on what the first left in the shared scratch), to the FP64 bar of
the oracle parity tests (max-abs rho/pi 1e-10, relative energy 1e-12; the
kernels are the same, so the results agree to rounding)."""

import math
import sys

import numpy as np
import pytest

from paper_1202_0098_amd import synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def _run(torch, ma, ctx, s, cols, mu, noalloc, **opt):
    o = s.n_orb
    nu = s.p + s.q
    ncols = len(cols)
    rho = torch.zeros(s.nblk * o * o, dtype=torch.float64, device="cuda")
    pi = torch.zeros_like(rho)
    eps = torch.zeros(ncols * nu, dtype=torch.float64, device="cuda")
    st = torch.zeros(ncols * ma.STATS, dtype=torch.int32, device="cuda")
    res = ctx.solve_columns(cols, s.p, s.q, mu=mu, kT=s.kT, opts=ma.default_opts(**opt),
                            rho=rho, pi=pi, eps=eps, col_stats=st, noalloc=noalloc)
    torch.cuda.synchronize()
    return (res, rho.cpu().numpy(), pi.cpu().numpy(), eps.cpu().numpy(),
            st.cpu().numpy().reshape(ncols, ma.STATS))


def _agree(a, b):
    assert np.array_equal(a[4][:, 0], b[4][:, 0]) and np.all(a[4][:, 3] == 0)
    assert np.abs(a[1] - b[1]).max() <= 1e-10
    assert np.abs(a[2] - b[2]).max() <= 1e-10 * max(1.0, np.abs(b[2]).max())
    assert np.allclose(a[3], b[3], atol=1e-10, rtol=0, equal_nan=True)
    assert abs(a[0].mu - b[0].mu) <= 1e-10 * max(1.0, abs(b[0].mu))
    assert abs(a[0].energy - b[0].energy) <= 1e-12 * abs(b[0].energy)


def test_noalloc_matches_solve_columns_twice():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1202_0098_amd as ma
    ctx = ma.Context(0)
    try:
        s = synth.config_diamond4096()
        ctx.build_tb(s)
        rng = np.random.default_rng(71)
        big = np.sort(rng.choice(s.M, 6000, replace=False)).astype(np.int32)
        small = np.sort(rng.choice(s.M, 700, replace=False)).astype(np.int32)
        for name, cols, mu in [("6000 columns, mu bisected", big, math.nan),
                               ("700 columns, mu given", small, 0.93)]:
            _say(f"noalloc diamond4096 {name}")
            got = _run(torch, ma, ctx, s, cols, mu, True)
            _say(f"solve_columns diamond4096 {name}")
            ref = _run(torch, ma, ctx, s, cols, mu, False)
            _say(f"mu {got[0].mu:.12f} vs {ref[0].mu:.12f}, E {got[0].energy:.10f} vs "
                 f"{ref[0].energy:.10f}, max|drho| {np.abs(got[1] - ref[1]).max():.2e}")
            _agree(got, ref)
        # options the allocation-free path does not support are refused before any launch
        with pytest.raises(ma.MarnoldiError) as ei:
            ctx.solve_columns(None, s.p, s.q, mu=math.nan, kT=s.kT, noalloc=True,
                              opts=ma.default_opts(start="learned"))
        assert ei.value.status == ma.MA_EINVAL
    finally:
        ctx.close()
