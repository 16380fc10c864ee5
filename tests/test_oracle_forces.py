"""Pins of the oracle's forces and Green's function (CPU).

Forces (Sec. 2, the partial sums F_K^(j)): with a complete subspace the
method's rho and pi are those of exact diagonalisation, and F_K must equal
minus the derivative of the grand potential
Omega(mu) = -spin kT sum_k ln(1 + exp(-(lambda_k - mu)/kT)) of the pencil
(H(R), S(R)) at fixed mu, taken by central finite differences of positions
with the pattern rebuilt.  The derivative blocks (complex step) are pinned by
finite differences of the generator itself.  Newton's third law holds for
any subspace.

Green's function (Eqs. 11-12): with a complete subspace,
G(z) e_j = (zS - H)^-1 e_j from a dense solve; the density of states
integrates to the electron count at full occupation.
"""

import numpy as np
import pytest
import scipy.linalg as sl

from paper_1202_0098_amd import synth


def _cluster(seed, n=6, kind="sp3"):
    """n atoms in a compact random cluster inside a large box (no periodic
    images within the cutoff): each atom bonded to one placed before it, no
    pair within 0.05 A of the cutoff."""
    rng = np.random.default_rng(seed)
    prm = synth.SP3_PARAMS if kind == "sp3" else synth.SPD_PARAMS
    rc = prm["rcut"]
    box = np.array([40.0, 40.0, 40.0])
    pts = [np.array([20.0, 20.0, 20.0])]
    while len(pts) < n:
        p = pts[rng.integers(len(pts))] + rng.normal(0, 1.0, 3) * 1.6
        d = np.linalg.norm(np.array(pts) - p, axis=1)
        if 0.85 * prm["d0"] < d.min() < rc - 0.1 and np.all(np.abs(d - rc) > 0.05):
            pts.append(p)
    s = synth.build_tb(np.array(pts), box, prm, "cluster")
    return s


def _omega(s, mu, kT, spin):
    Hd, Sd = s.dense()
    lam = sl.eigh(Hd, Sd, eigvals_only=True)
    x = -(lam - mu) / kT
    return -spin * kT * np.sum(np.logaddexp(0.0, x))


def test_derivative_blocks_match_finite_differences():
    s = _cluster(3)
    dH, dS = synth.derivative_blocks(s)
    rows = np.repeat(np.arange(s.n_atoms), np.diff(s.blk_ptr))
    h = 1e-6
    for k in np.nonzero(rows != s.blk_col)[0][:6]:
        B = int(s.blk_col[k])
        d0 = synth.min_image(s.pos[B] - s.pos[rows[k]], s.box)
        for c in range(3):
            e = np.zeros(3)
            e[c] = h
            fd = (synth.sk_blocks((d0 + e)[None], s.params)[0]
                  - synth.sk_blocks((d0 - e)[None], s.params)[0]) / (2 * h)
            assert np.abs(dH[k, c] - fd).max() < 1e-7
            assert np.abs(dS[k, c] - s.params["c_overlap"] * fd / s.params["V_ref"]).max() < 1e-8


@pytest.mark.parametrize("seed,kind", [(5, "sp3"), (6, "sp3"), (7, "spd")])
def test_complete_subspace_forces_are_minus_grand_potential_gradient(oracle_mod, seed, kind):
    s = _cluster(seed, n=5 if kind == "spd" else 6, kind=kind)
    n = s.M
    mu, kT, spin = 0.5, 0.3, 2.0
    # more subspace than dimensions: whatever block 1 misses, block 2 adds,
    # and the breakdown rule drops the excess
    p, q = n, min(n, 64 - n)
    res = oracle_mod.solve(s, mu=mu, kT=kT, p=p, q=q)
    assert np.all(res["raw"]["nu_eff"] == n)
    # complete up to directions dropped by the breakdown rule (relative size
    # below 1e-10: the spd cluster's Krylov spaces exhaust before n), so rho
    # and pi are the exact ones to that level
    Hd, Sd = s.dense()
    lam, phi = sl.eigh(Hd, Sd)
    f = 1.0 / (1.0 + np.exp((lam - mu) / kT))
    R = np.zeros((n, n))
    o = s.n_orb
    for c, j in enumerate(res["raw"]["cols"]):
        A = int(j) // o
        k0, k1 = s.blk_ptr[A], s.blk_ptr[A + 1]
        rows = np.concatenate([np.arange(b * o, (b + 1) * o) for b in s.blk_col[k0:k1]])
        R[rows, j] = res["rho"][c, :len(rows)]
    rho_ex = (phi * f) @ phi.T
    mask = R != 0
    assert np.abs(R[mask] - rho_ex[mask]).max() < 1e-8
    dH, dS = synth.derivative_blocks(s)
    F = oracle_mod.forces(s, res["raw"]["cols"], res["rho"], res["pi"], dH, dS, spin)
    h = 1e-5
    Ffd = np.zeros_like(F)
    for K in range(s.n_atoms):
        for c in range(3):
            pos_p, pos_m = s.pos.copy(), s.pos.copy()
            pos_p[K, c] += h
            pos_m[K, c] -= h
            sp, sm = synth.rebuild(s, pos_p), synth.rebuild(s, pos_m)
            assert sp.nblk == s.nblk == sm.nblk
            Ffd[K, c] = -(_omega(sp, mu, kT, spin) - _omega(sm, mu, kT, spin)) / (2 * h)
    assert np.abs(F - Ffd).max() < 1e-6 * max(1.0, np.abs(Ffd).max())
    assert np.abs(F.sum(0)).max() < 1e-10


def test_forces_obey_newtons_third_law_for_any_subspace(oracle_mod):
    s = synth.config_diamond64()
    res = oracle_mod.solve(s)
    dH, dS = synth.derivative_blocks(s)
    F = oracle_mod.forces(s, res["raw"]["cols"], res["rho"], res["pi"], dH, dS)
    assert np.abs(F).max() > 0.1
    assert np.abs(F.sum(0)).max() < 1e-10 * np.abs(F).max() * s.n_atoms


@pytest.mark.parametrize("z", [0.3 + 0.05j, -4.0 + 0.4j, 2.5 - 0.2j])
def test_complete_subspace_green_function_is_the_resolvent(oracle_mod, z):
    P = synth.random_pencil(4, 4, seed=13)
    n = P.M
    raw = oracle_mod.solve_raw(P, p=n - 5, q=5)
    assert np.all(raw["nu_eff"] == n)
    G = oracle_mod.green(P, raw, z)
    Hd, Sd = P.dense()
    R = np.linalg.solve(z * Sd - Hd, np.eye(n))      # (zS - H)^-1, column j = x_j(z)
    o = P.n_orb
    for c, j in enumerate(raw["cols"]):
        A, r = divmod(int(j), o)
        k0, k1 = P.blk_ptr[A], P.blk_ptr[A + 1]
        rows = np.concatenate([np.arange(b * o, (b + 1) * o) for b in P.blk_col[k0:k1]])
        assert np.abs(G[c, :len(rows)] - R[rows, j]).max() < 1e-10


def test_dos_integrates_to_the_column_count(oracle_mod):
    s = synth.config_diamond64()
    raw = oracle_mod.solve_raw(s)
    E = np.linspace(-60.0, 60.0, 240001)
    D = oracle_mod.dos(raw, E, eta=0.05, spin=2.0)
    integral = np.trapezoid(D, E)
    # sum_j sum_a w_a = sum_j N_j(full occupation) = M per spin, minus the
    # Lorentzian tails outside [-60, 60] (2 eta / (pi * 50) per unit weight)
    assert abs(integral / (2.0 * s.M) - 1.0) < 2e-3
    # the Lorentzian peaks sit on the Ritz values: D is largest near them
    ok = np.arange(raw["eps"].shape[1])[None, :] < raw["nu_eff"][:, None]
    lo, hi = raw["eps"][ok].min(), raw["eps"][ok].max()
    assert D[(E > lo - 0.5) & (E < hi + 0.5)].sum() > 0.99 * D.sum()
