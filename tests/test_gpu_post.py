"""Forces, density of states and the subspace Green's function from the
column outputs (GPU, through the C interface) against the oracle.

Forces (Sec. 2, the partial sums F_K^(j)): the library's force kernel on the
library's rho and pi against the oracle's forces on the oracle's rho and pi
(FP64 mode: the outputs agree to 1e-10, so the forces agree to 1e-9 of their
scale), and the force kernel alone on the oracle's rho and pi (1e-12).
DOS and G(z) (Eqs. 11-12): against the oracle on the same Ritz data (1e-10),
and G(z) against the resolvent (zS - H)^-1 with a complete subspace.
"""

import math
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


def _solve(torch, ma, ctx, s, mu=math.nan, **opt):
    o = s.n_orb
    rho = torch.zeros(s.nblk * o * o, dtype=torch.float64, device="cuda")
    pi = torch.zeros_like(rho)
    res = ctx.solve_columns(None, s.p, s.q, mu=mu, kT=s.kT, opts=ma.default_opts(**opt),
                            rho=rho, pi=pi)
    torch.cuda.synchronize()
    return res, rho, pi


@pytest.mark.parametrize("cfg", ["diamond64", "diamond4096", "fcc_spd_4x4x4"])
def test_forces_match_oracle(env, cfg):
    torch, ma, ctx = env
    import oracle
    s = {"diamond64": synth.config_diamond64, "diamond4096": synth.config_diamond4096,
         "fcc_spd_4x4x4": lambda: synth.config_fcc_spd(cells=(4, 4, 4))}[cfg]()
    _say(f"{cfg}: build and solve every column (fp64, mu bisected)")
    ctx.build_tb(s)
    res, rho, pi = _solve(torch, ma, ctx, s)
    dH, dS = synth.derivative_blocks(s)
    dHd = torch.from_numpy(np.ascontiguousarray(dH)).cuda()
    dSd = torch.from_numpy(np.ascontiguousarray(dS)).cuda()
    F = torch.zeros(s.n_atoms * 3, dtype=torch.float64, device="cuda")
    ctx.forces(dHd, dSd, rho, pi, F)
    torch.cuda.synchronize()
    Fg = F.cpu().numpy().reshape(-1, 3)
    _say(f"{cfg}: oracle solve of every column")
    ora = oracle.solve(s, mu=res.mu)
    Fo = oracle.forces(s, ora["raw"]["cols"], ora["rho"], ora["pi"], dH, dS)
    scale = max(1.0, np.abs(Fo).max())
    d = np.abs(Fg - Fo).max()
    _say(f"{cfg}: max|F| {np.abs(Fo).max():.3f} eV/A, max|dF| {d:.3e}, |sum F| {np.abs(Fg.sum(0)).max():.2e}")
    assert d <= 1e-9 * scale
    assert np.abs(Fg.sum(0)).max() <= 1e-9 * scale * math.sqrt(s.n_atoms)
    # the force kernel alone, on the oracle's rho and pi
    rho_o = torch.from_numpy(oracle.scatter_slots(s, ora["raw"]["cols"], ora["rho"]).ravel()).cuda()
    pi_o = torch.from_numpy(oracle.scatter_slots(s, ora["raw"]["cols"], ora["pi"]).ravel()).cuda()
    ctx.forces(dHd, dSd, rho_o, pi_o, F)
    torch.cuda.synchronize()
    assert np.abs(F.cpu().numpy().reshape(-1, 3) - Fo).max() <= 1e-12 * scale


def test_dos_matches_oracle(env):
    torch, ma, ctx = env
    import oracle
    s = synth.config_diamond64()
    ctx.build_tb(s)
    _say("diamond64 solve for the DOS")
    _solve(torch, ma, ctx, s)
    E = np.linspace(-25.0, 25.0, 1001)
    got = ctx.dos(E, eta=0.1)
    raw = oracle.solve_raw(s)
    ref = oracle.dos(raw, E, eta=0.1)
    _say(f"DOS: max {ref.max():.3f} states/eV, max rel diff {np.abs(got - ref).max() / ref.max():.2e}")
    assert np.abs(got - ref).max() <= 1e-10 * ref.max()


@pytest.mark.parametrize("z", [0.4 + 0.1j, -3.0 + 0.5j])
def test_green_matches_oracle(env, z):
    torch, ma, ctx = env
    import oracle
    s = synth.config_diamond64()
    ctx.build_tb(s)
    _solve(torch, ma, ctx, s)
    o = s.n_orb
    gr = torch.zeros(s.nblk * o * o, dtype=torch.float64, device="cuda")
    gi = torch.zeros_like(gr)
    ctx.green(z, gr, gi)
    torch.cuda.synchronize()
    raw = oracle.solve_raw(s)
    G = oracle.green(s, raw, z)
    ref_r = oracle.scatter_slots(s, raw["cols"], G.real).ravel()
    ref_i = oracle.scatter_slots(s, raw["cols"], G.imag).ravel()
    d = max(np.abs(gr.cpu().numpy() - ref_r).max(), np.abs(gi.cpu().numpy() - ref_i).max())
    _say(f"G({z}): max|dG| {d:.2e}")
    assert d <= 1e-10 * max(1.0, np.abs(ref_r).max(), np.abs(ref_i).max())


def test_green_complete_subspace_is_the_resolvent(env):
    torch, ma, ctx = env
    P = synth.random_pencil(4, 4, seed=13)
    n = P.M
    P.p, P.q = n - 5, 5
    ctx.build_tb(P)
    _solve(torch, ma, ctx, P)
    o = P.n_orb
    z = 0.3 + 0.05j
    gr = torch.zeros(P.nblk * o * o, dtype=torch.float64, device="cuda")
    gi = torch.zeros_like(gr)
    ctx.green(z, gr, gi)
    torch.cuda.synchronize()
    Hd, Sd = P.dense()
    R = np.linalg.solve(z * Sd - Hd, np.eye(n))
    g = (gr.cpu().numpy() + 1j * gi.cpu().numpy()).reshape(P.nblk, o, o)
    d = 0.0
    for A in range(P.n_atoms):
        for k in range(P.blk_ptr[A], P.blk_ptr[A + 1]):
            B = P.blk_col[k]
            # slot (k, r, c) holds element (i = (B, c), j = (A, r))
            d = max(d, np.abs(g[k] - R[B * o:(B + 1) * o, A * o:(A + 1) * o].T).max())
    assert d <= 1e-9


def test_post_needs_a_solve(env):
    torch, ma, ctx = env
    s = synth.config_diamond64()
    ctx.build_tb(s)
    with pytest.raises(ma.MarnoldiError) as ei:
        ctx.dos(np.zeros(3), eta=0.1)
    assert ei.value.status == ma.MA_ESTATE
    _solve(torch, ma, ctx, s, mu=0.9)   # given mu: no amplitudes kept
    with pytest.raises(ma.MarnoldiError) as ei:
        ctx.green(0.1 + 0.1j)
    assert ei.value.status == ma.MA_ESTATE
    assert np.all(np.isfinite(ctx.dos(np.linspace(-5, 5, 11), eta=0.2)))
