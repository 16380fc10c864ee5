"""Synthetic input generator: structure of H and S, reproducibility, sizes."""

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from paper_1202_0098_amd import synth


def _check_structure(s):
    o = s.n_orb
    assert s.blk_ptr[0] == 0 and s.blk_ptr[-1] == s.nblk
    for a in range(s.n_atoms):
        cols = s.blk_col[s.blk_ptr[a]:s.blk_ptr[a + 1]]
        assert np.all(np.diff(cols) > 0) and a in cols
    # block transpose symmetry (pattern and values)
    key = {}
    for a in range(s.n_atoms):
        for k in range(s.blk_ptr[a], s.blk_ptr[a + 1]):
            key[(a, int(s.blk_col[k]))] = k
    for (a, b), k in key.items():
        kt = key[(b, a)]
        assert np.array_equal(s.H[k], s.H[kt].T)
        assert np.array_equal(s.S[k], s.S[kt].T)
        if a == b:
            assert np.array_equal(s.S[k], np.eye(o))


def test_diamond64_structure_and_spd():
    s = synth.config_diamond64()
    assert (s.n_atoms, s.M, s.n_orb) == (64, 256, 4)
    # cutoff 3.0 A: self + 4 nearest neighbours (second shell at 3.84 A)
    assert np.all(np.diff(s.blk_ptr) == 5)
    _check_structure(s)
    Hd, Sd = s.dense()
    w = np.linalg.eigvalsh(Sd)
    assert 0.5 < w.min() and w.max() < 1.5


def test_reproducible_seeds():
    a = synth.config_diamond64(seed=1001)
    b = synth.config_diamond64(seed=1001)
    c = synth.config_diamond64(seed=1002)
    assert np.array_equal(a.H, b.H) and np.array_equal(a.pos, b.pos)
    assert not np.array_equal(a.pos, c.pos)


def test_diamond4096_sizes():
    s = synth.config_diamond4096()
    assert (s.n_atoms, s.M) == (4096, 16384)
    assert s.nblk == 5 * 4096
    assert np.all(s.region_nrp == 120)


def test_fcc_spd_small_structure():
    s = synth.config_fcc_spd(cells=(4, 4, 4))
    assert s.n_orb == 9 and s.n_atoms == 256
    per_row = np.diff(s.blk_ptr)
    # cutoff 5.0 sits just above the third fcc shell (4.96 A): ~43 blocks/row
    assert 30 <= per_row.mean() <= 48
    _check_structure(s)
    Hd, Sd = s.dense()
    assert np.linalg.eigvalsh(Sd).min() > 0.3


@pytest.mark.parametrize("prm", [synth.SP3_PARAMS, synth.SPD_PARAMS])
def test_slater_koster_rotational_invariance(prm):
    """A rotated cluster has the same spectrum: the blocks transform as the
    s, p, d orbitals do."""
    rng = np.random.default_rng(0)
    pos = rng.uniform(0, 4.0, size=(6, 3))
    R = Rotation.random(random_state=3).as_matrix()
    prm = dict(prm, rcut=6.0, lam=100.0)

    def spec(P):
        s = synth.build_tb(P + 50, [200, 200, 200], prm)
        return np.linalg.eigvalsh(s.dense()[0])
    e1, e2 = spec(pos), spec(pos @ R.T)
    assert np.abs(e1 - e2).max() < 1e-12 * np.abs(e1).max()


def test_slater_koster_bond_along_z():
    """For a bond along z the block is diagonal in m with the bond integrals."""
    prm = synth.SPD_PARAMS
    d0 = prm["d0"]
    E = synth.sk_blocks(np.array([[0.0, 0.0, d0]]), prm)[0]
    V = prm["V0"]
    s, x, y, z, xy, yz, zx, x2, z2 = range(9)
    exp = {(s, s): V["sss"], (s, z): V["sps"], (z, z): V["pps"], (x, x): V["ppp"],
           (y, y): V["ppp"], (s, z2): V["sds"], (z, z2): V["pds"], (x, zx): V["pdp"],
           (y, yz): V["pdp"], (z2, z2): V["dds"], (zx, zx): V["ddp"], (yz, yz): V["ddp"],
           (xy, xy): V["ddd"], (x2, x2): V["ddd"]}
    M = np.zeros((9, 9))
    for (a, b), v in exp.items():
        M[a, b] = v
        # parity of the reversed pair: odd for s-p and p-d
        la = 0 if a == 0 else (1 if a < 4 else 2)
        lb = 0 if b == 0 else (1 if b < 4 else 2)
        M[b, a] = v * (-1) ** (la + lb)
    assert np.abs(E - M).max() < 1e-14


def test_rsa_minimum_distance_and_density():
    rng = np.random.default_rng(5)
    box = (1000 / 0.04997) ** (1 / 3)
    pos = synth.rsa_positions(1000, box, 2.2, 0.2, rng)
    d = pos[:, None] - pos[None]
    d -= box * np.round(d / box)
    r = np.sqrt((d ** 2).sum(-1)) + np.eye(len(pos)) * 100
    assert r.min() >= 2.2
    assert len(pos) == 1000
