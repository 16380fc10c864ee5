"""Pins of the oracle's real-space projection and Fermi weighting.

The region of an atom (Sec. 3, real-space projection of H and S around the
atom of basis j) is pinned by crystallography and by brute force:
  * on perfect diamond and fcc lattices every atom sees the textbook
    coordination shells, so a radius between two shells admits exactly the
    cumulative shell count (diamond 5/17/29/35/47/71/87/99/123 atoms with the
    centre, fcc 13/19/43/55/79/87);
  * on displaced cells the region equals a brute-force enumeration of the 27
    periodic images of every atom (no rounding-based minimum image);
  * the radius is strict (d < r), ties in the nearest-k rule go to the lower
    atom index, and the minimum image holds in a box just over 2r wide.
The Fermi function (the occupation of Eqs. 13-14) is pinned by its exact
values at 0 and +-ln 3, its symmetry, an independently written logistic, the
large-argument asymptotics and the (eps - mu)/kT scale of the occupations.
"""

import math

import numpy as np
import pytest

from paper_1202_0098_amd import synth

# coordination shells (squared distance in units of (a/4)^2 for diamond and
# (a/2)^2 for fcc, number of atoms): textbook crystallography
DIAMOND_SHELLS = [(3, 4), (8, 12), (11, 12), (16, 6), (19, 12), (24, 24), (27, 16), (32, 12),
                  (35, 24)]
FCC_SHELLS = [(2, 12), (4, 6), (6, 24), (8, 12), (10, 24), (12, 8)]


def _lattice(basis, n, a):
    """n x n x n conventional cells of edge a, written out here (not from the
    input generators)."""
    pts = []
    for i in range(n):
        for j in range(n):
            for k in range(n):
                for b in basis:
                    pts.append([(i + b[0]) * a, (j + b[1]) * a, (k + b[2]) * a])
    return np.array(pts, float)


FCC_BASIS = [(0, 0, 0), (0, .5, .5), (.5, 0, .5), (.5, .5, 0)]
DIAMOND_BASIS = FCC_BASIS + [(x + .25, y + .25, z + .25) for x, y, z in FCC_BASIS]


def _radii_between(shells, unit):
    """(radius midway between shell k and k+1, cumulative count through k)."""
    out = []
    cum = 1
    for k, (d2, cnt) in enumerate(shells):
        cum += cnt
        if k + 1 < len(shells):
            r = 0.5 * (math.sqrt(d2) + math.sqrt(shells[k + 1][0])) * unit
            out.append((r, cum))
    return out


@pytest.mark.parametrize("kind", ["diamond", "fcc"])
def test_radius_regions_count_the_coordination_shells(oracle_mod, kind):
    a = 5.43 if kind == "diamond" else 4.05
    basis, shells, unit = ((DIAMOND_BASIS, DIAMOND_SHELLS, a / 4) if kind == "diamond"
                           else (FCC_BASIS, FCC_SHELLS, a / 2))
    n = 4
    pos = _lattice(basis, n, a)
    box = np.full(3, n * a)
    for r, cum in _radii_between(shells, unit):
        assert 2 * r < n * a   # the sphere fits the periodic box
        for A in range(0, len(pos), 7):
            reg = oracle_mod.region_of(pos, box, A, "radius", r)
            assert len(reg) == cum, (kind, r, A, len(reg))
            assert A in reg and np.all(np.diff(reg) > 0)


def test_fcc_7A_region(oracle_mod):
    """The 262,144-atom cell's 7 A radius sits just inside the 87-atom shell
    (7.015 A): 79 atoms on the perfect lattice; thermal displacements admit
    part of the next shell."""
    a = 4.05
    pos = _lattice(FCC_BASIS, 4, a)
    box = np.full(3, 4 * a)
    assert all(len(oracle_mod.region_of(pos, box, A, "radius", 7.0)) == 79 for A in range(0, 256, 17))
    s = synth.config_fcc_spd(cells=(4, 4, 4))
    sizes = [len(oracle_mod.region_of(s.pos, s.box, A, "radius", 7.0)) for A in range(s.n_atoms)]
    assert 79 <= np.mean(sizes) <= 87 and min(sizes) >= 70 and max(sizes) <= 96


def _brute_d2(pos, box, A):
    """Squared distance to the nearest periodic image of every atom, by
    enumerating the 27 image shifts."""
    best = np.full(len(pos), np.inf)
    for sx in (-1, 0, 1):
        for sy in (-1, 0, 1):
            for sz in (-1, 0, 1):
                d = pos + np.array([sx, sy, sz]) * box - pos[A]
                best = np.minimum(best, np.einsum("ij,ij->i", d, d))
    return best


@pytest.mark.parametrize("cfg", ["diamond4096", "disordered", "fcc"])
def test_regions_match_brute_force_images(oracle_mod, cfg):
    if cfg == "diamond4096":
        s = synth.config_diamond4096()
    elif cfg == "disordered":
        s = synth.config_disordered8000(n_atoms=2000)
    else:
        s = synth.config_fcc_spd(cells=(4, 4, 8))
    pos = synth.wrap(s.pos, s.box)
    for A in np.random.default_rng(3).choice(s.n_atoms, 12, replace=False):
        d2 = _brute_d2(pos, s.box, int(A))
        if s.region_mode == "radius":
            want = np.nonzero(d2 < s.region_radius ** 2)[0]
        else:
            k = int(s.region_nrp[A])
            order = sorted(range(s.n_atoms), key=lambda b: (d2[b], b))
            want = np.sort(order[:k])
        got = oracle_mod.region_of(s.pos, s.box, int(A), s.region_mode, s.region_radius,
                                   0 if s.region_nrp is None else int(s.region_nrp[A]))
        assert np.array_equal(got, want), (cfg, A)


def test_diamond4096_regions_hold_120_atoms(oracle_mod):
    s = synth.config_diamond4096()
    for A in range(0, s.n_atoms, 97):
        reg = oracle_mod.region_of(s.pos, s.box, A, "nearest", 0.0, 120)
        assert len(reg) == 120 and A in reg


def _simple_cubic(n):
    """Simple cubic lattice with spacing 1 A: every squared distance is an
    exact integer."""
    g = np.stack(np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij"), -1)
    return g.reshape(-1, 3).astype(float), np.full(3, float(n))


def test_radius_is_strict(oracle_mod):
    pos, box = _simple_cubic(10)
    A = 555
    # d^2 < 4: 1 + 6 + 12 + 8 = 27 atoms; the 6 atoms at exactly 2 A are out
    assert len(oracle_mod.region_of(pos, box, A, "radius", 2.0)) == 27
    assert len(oracle_mod.region_of(pos, box, A, "radius", 2.0 + 1e-9)) == 33


def test_nearest_ties_go_to_the_lower_atom_index(oracle_mod):
    pos, box = _simple_cubic(6)
    for A in [0, 43, 129, 215]:
        d2 = _brute_d2(pos, box, A)
        first = np.nonzero(np.abs(d2 - 1.0) < 1e-12)[0]
        assert len(first) == 6
        for k in range(1, 7):
            reg = oracle_mod.region_of(pos, box, A, "nearest", 0.0, 1 + k)
            assert np.array_equal(reg, np.sort(np.concatenate([[A], first[:k]])))


def test_minimum_image_in_a_box_just_over_twice_the_radius(oracle_mod):
    box = np.array([10.0, 30.0, 30.0])
    pos = np.array([[0.2, 15.0, 15.0],     # A
                    [9.9, 15.0, 15.0],     # 0.3 A away through the boundary
                    [5.15, 15.0, 15.0],    # 4.95 A directly, 5.05 A through it
                    [5.25, 15.0, 15.0]])   # 5.05 A directly, 4.95 A through it
    assert list(oracle_mod.region_of(pos, box, 0, "radius", 4.96)) == [0, 1, 2, 3]
    assert list(oracle_mod.region_of(pos, box, 0, "radius", 4.94)) == [0, 1]
    assert list(oracle_mod.region_of(pos, box, 0, "nearest", 0.0, 2)) == [0, 1]


# ---------------------------------------------------------------------------
# Fermi weighting
# ---------------------------------------------------------------------------

def test_fermi_exact_values_and_symmetry(oracle_mod):
    f = oracle_mod.fermi
    assert f(np.array([0.0]))[0] == 0.5
    assert abs(f(np.array([math.log(3.0)]))[0] - 0.25) < 1e-16
    assert abs(f(np.array([-math.log(3.0)]))[0] - 0.75) < 1e-16
    x = np.linspace(-40.0, 40.0, 801)
    assert np.abs(f(x) + f(-x) - 1.0).max() < 1e-15


def test_fermi_against_an_independent_logistic(oracle_mod):
    x = np.linspace(-30.0, 30.0, 601)
    ref = np.array([1.0 / (1.0 + math.exp(v)) for v in x])
    assert np.abs(oracle_mod.fermi(x) - ref).max() <= 1e-15
    # far tails: no overflow, f(x) -> exp(-x) for large x, 1 for very negative x
    big = np.array([700.0, 745.0, 1e6])
    got = oracle_mod.fermi(big)
    assert np.all(np.isfinite(got))
    assert abs(got[0] / math.exp(-700.0) - 1.0) < 1e-12
    assert got[2] == 0.0
    assert np.all(oracle_mod.fermi(np.array([-800.0, -1e6])) == 1.0)
    # derivative identity f' = -f (1 - f), by central differences
    h = 1e-5
    xs = np.linspace(-8, 8, 33)
    fd = (oracle_mod.fermi(xs + h) - oracle_mod.fermi(xs - h)) / (2 * h)
    fx = oracle_mod.fermi(xs)
    assert np.abs(fd + fx * (1 - fx)).max() < 1e-9


def test_occupation_scale_and_electron_count(oracle_mod):
    """f((eps - mu)/kT): a level kT ln 3 above mu holds 1/4, one kT ln 3 below
    it 3/4; the electron count sums f w over the kept Ritz pairs only."""
    kT, mu = 0.2, -1.3
    raw = {"eps": np.array([[mu + kT * math.log(3.0), mu - kT * math.log(3.0), mu, 99.0]]),
           "nu_eff": np.array([3]),
           "vj": np.array([[1.0, 2.0, 0.5, 7.0]]),
           "svj": np.array([[0.5, 0.25, 2.0, 7.0]])}
    f, mask = oracle_mod.occupations(raw, mu, kT)
    assert np.allclose(f[0], [0.25, 0.75, 0.5, 0.0], rtol=0, atol=1e-15)
    assert list(mask[0]) == [True, True, True, False]
    # w = vj * svj = 0.5, 0.5, 1.0 -> N = 0.25*0.5 + 0.75*0.5 + 0.5*1.0
    assert abs(oracle_mod.electron_count(raw, mu, kT) - 1.0) < 1e-15
