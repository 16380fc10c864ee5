"""Reuse of s_j (GPU, through the C interface).

Within one MD step the overlap matrix does not change, so S^-1 e_j is needed
only once per step (the charge-self-consistency remark of Sec. 2): a solve
with keep_sj keeps every solved column's s_j, and a later solve with start
"previous" on the same geometry starts its CG there and needs no iteration.
Across geometry updates the kept s_j, mapped onto the column's current region
atom by atom, is the CG start (an extension: the start only moves where the CG
begins).  Parity: the oracle run from the same start vector, mapped here on
the host from the oracle's own s_j of the previous geometry, follows the same
CG path, so the FP64 results agree to the usual 1e-10; a start that the FP64
residual judge rejects falls back to the zero start.
"""

import sys

import numpy as np
import pytest

from paper_1202_0098_amd import synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1202_0098_amd as ma
    ctx = ma.Context(0)
    yield torch, ma, ctx
    ctx.close()


def _solve(torch, ma, ctx, s, cols, mu, **opt):
    o = s.n_orb
    n = s.M if cols is None else len(cols)
    rho = torch.zeros(s.nblk * o * o, dtype=torch.float64, device="cuda")
    st = torch.zeros(n * ma.STATS, dtype=torch.int32, device="cuda")
    r = ctx.solve_columns(cols, s.p, s.q, mu=mu, kT=s.kT, rho=rho, col_stats=st,
                          opts=ma.default_opts(**opt))
    torch.cuda.synchronize()
    return r, rho.cpu().numpy(), st.cpu().numpy().reshape(n, ma.STATS)


def _map_start(old_sys, new_sys, cols, sj_old):
    """The kept s_j of each column on its current region: the value of the
    same orbital of the same atom in the old region, zero for new atoms."""
    o = new_sys.n_orb
    reg = {}
    rows = []
    for c, j in enumerate(cols):
        A = int(j) // o
        if A not in reg:
            a = oracle_region(old_sys, A)
            b = oracle_region(new_sys, A)
            reg[A] = (a, b)
        a, b = reg[A]
        pos = {int(x): k for k, x in enumerate(a)}
        v = np.zeros(len(b) * o)
        for t, B in enumerate(b):
            k = pos.get(int(B))
            if k is not None:
                v[t * o:(t + 1) * o] = sj_old[c, k * o:(k + 1) * o]
        rows.append(v)
    n = max(len(v) for v in rows)
    x0 = np.zeros((len(cols), n))
    for c, v in enumerate(rows):
        x0[c, :len(v)] = v
    return x0


def oracle_region(s, A):
    import oracle
    nrp = 0 if s.region_nrp is None else int(s.region_nrp[A])
    return oracle.region_of(s.pos, s.box, A, s.region_mode, s.region_radius, nrp)


@pytest.mark.parametrize("precision,kernel", [("fp64", "workspace"), ("fp64", "onchip"),
                                              ("mixed_f64acc", "workspace"),
                                              ("mixed_f64acc", "atom")])
def test_previous_start_across_updates(env, precision, kernel):
    torch, ma, ctx = env
    import oracle
    s0 = synth.config_diamond4096()
    ups = synth.md_updates(s0, 2, 0.02, seed0=70)
    rng = np.random.default_rng(5)
    atoms = np.sort(rng.choice(s0.n_atoms, 40, replace=False))
    cols = (atoms[:, None] * s0.n_orb + np.arange(s0.n_orb)).ravel().astype(np.int32)
    mu = 0.95
    _say(f"{precision}/{kernel}: geometry 0, 160 columns, keep s_j")
    ctx.build_tb(s0)
    _, rho0, st0 = _solve(torch, ma, ctx, s0, cols, mu, precision=precision,
                          basis_kernel=kernel, keep_sj=1)
    assert np.all(st0[:, 4] == 0)
    # same geometry again (S unchanged): the kept s_j is already converged
    _, rho_again, st_again = _solve(torch, ma, ctx, s0, cols, mu, precision=precision,
                                    basis_kernel=kernel, start="previous")
    _say(f"same geometry: CG iterations zero start {st0[:, 1].mean():.2f}, previous start "
         f"{st_again[:, 1].mean():.2f}; max|drho| {np.abs(rho_again - rho0).max():.1e}")
    assert np.all(st_again[:, 4] == 3)
    assert np.all(st_again[:, 1] == 0)
    assert np.abs(rho_again - rho0).max() <= 1e-13
    tol = 1e-10 if precision == "fp64" else 1e-5
    ora_prev = oracle.solve_raw(s0, cols, want_sj=True)
    moved = 0
    prev = s0
    for k, s in enumerate(ups, 1):
        x0 = _map_start(prev, s, cols, ora_prev["sj"])
        moved += sum(int(not np.array_equal(oracle_region(prev, int(A)), oracle_region(s, int(A))))
                     for A in atoms)
        ctx.build_tb(s)
        _say(f"{precision}/{kernel}: update {k}, zero and previous starts")
        _, rho_z, st_z = _solve(torch, ma, ctx, s, cols, mu, precision=precision,
                                basis_kernel=kernel)
        _, rho_p, st_p = _solve(torch, ma, ctx, s, cols, mu, precision=precision,
                                basis_kernel=kernel, start="previous", keep_sj=1)
        ref_z = oracle.solve(s, cols=cols, mu=mu)
        ref_p = oracle.solve(s, cols=cols, mu=mu, x0=x0, want_sj=True)
        rz = oracle.scatter_slots(s, cols, ref_z["rho"]).ravel()
        rp = oracle.scatter_slots(s, cols, ref_p["rho"]).ravel()
        dz, dp = np.abs(rho_z - rz).max(), np.abs(rho_p - rp).max()
        _say(f"update {k}: CG iterations zero {st_z[:, 1].mean():.2f} previous "
             f"{st_p[:, 1].mean():.2f} (oracle {ref_p['raw']['cg_iters'].mean():.2f}; starts "
             f"used {np.bincount(st_p[:, 4], minlength=5)}); max|drho| zero {dz:.2e} "
             f"previous {dp:.2e}; the two oracle starts differ by {np.abs(rz - rp).max():.1e}")
        assert dz <= tol and dp <= tol
        assert np.all(st_p[:, 4] == 3)
        if precision == "fp64":
            assert np.array_equal(st_p[:, 1], ref_p["raw"]["cg_iters"])
        assert st_p[:, 1].mean() < st_z[:, 1].mean()
        ora_prev = ref_p["raw"]
        prev = s
    assert moved > 0    # regions changed: the atom-by-atom mapping was exercised


def test_unkept_columns_start_from_zero(env):
    """Columns not solved by the keeping solve get a zero start, which the
    residual judge rejects (start code 4) and replaces by the usual zero
    start: results unchanged."""
    torch, ma, ctx = env
    s = synth.config_diamond4096()
    ctx.build_tb(s)
    _solve(torch, ma, ctx, s, np.arange(0, 64, dtype=np.int32), 0.95, keep_sj=1)
    cols = np.arange(32, 96, dtype=np.int32)
    _, rho_p, st_p = _solve(torch, ma, ctx, s, cols, 0.95, start="previous")
    _, rho_z, st_z = _solve(torch, ma, ctx, s, cols, 0.95)
    assert np.all(st_p[:32, 4] == 3) and np.all(st_p[32:, 4] == 4)
    assert np.all(st_p[32:, 1] == st_z[32:, 1])
    assert np.abs(rho_p - rho_z).max() <= 1e-10


def test_previous_start_errors(env):
    torch, ma, ctx = env
    s = synth.config_diamond64()
    ctx.build_tb(s)
    # a fresh context has kept nothing
    ctx2 = ma.Context(0)
    try:
        ctx2.build_tb(s)
        with pytest.raises(ma.MarnoldiError) as ei:
            _solve(torch, ma, ctx2, s, None, 0.9, start="previous")
        assert ei.value.status == ma.MA_EINVAL
    finally:
        ctx2.close()
    with pytest.raises(ma.MarnoldiError) as ei:
        _solve(torch, ma, ctx, s, None, 0.9, basis_kernel="group", keep_sj=1)
    assert ei.value.status == ma.MA_EINVAL
    o = s.n_orb
    rho = torch.zeros(s.nblk * o * o, dtype=torch.float64, device="cuda")
    with pytest.raises(ma.MarnoldiError) as ei:
        ctx.solve_columns(None, s.p, s.q, mu=0.9, kT=s.kT, rho=rho,
                          opts=ma.default_opts(keep_sj=1), noalloc=True)
    assert ei.value.status == ma.MA_EINVAL
