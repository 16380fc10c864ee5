"""Seeded synthetic tight-binding systems (input generation only).

This module produces the inputs of the per-column solve: atom positions in a
periodic orthorhombic box, and the Hamiltonian H and overlap S as atom-block
sparse matrices (block CSR, one ``o x o`` block per interacting atom pair,
``o`` orbitals per atom).  It contains none of the solver's arithmetic; both the
HIP path and the CPU oracle consume what it returns.

Hamiltonian model (two-centre Slater-Koster form).  For a bond vector
``d = r_B - r_A`` of length ``|d| < r_c`` with direction cosines (l, m, n) the
block ``H[(A, a), (B, b)]`` is the Slater-Koster element ``E_ab(l, m, n)``
built from bond integrals ``V = V0 * (d0/|d|)**2 * exp(-(|d| - d0)/lam)``.
On-site blocks are ``diag(eps_s, eps_p x3 [, eps_d x5])``.  The overlap is the
identity on atom-diagonal blocks and ``c * H_AB / V_ref`` off the diagonal
(``V_ref`` a fixed constant, the largest ``|V0|``), so S has H's pattern.

The paper's own workloads (NRL gold, the extended-Hueckel polymer) are not
available; these synthetic sp3 (diamond / disordered) and spd (fcc) systems
stand in for them with the sparsity, neighbourhood sizes and S ~ I structure
the method expects (S positive definite and close to the identity, which is
what makes the inner conjugate-gradient loop converge in a few tens of steps).
"""

from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np
from scipy.spatial import cKDTree

SQ3 = math.sqrt(3.0)

# ---------------------------------------------------------------------------
# parameter sets
# ---------------------------------------------------------------------------

#: sp3 parameters (eV, Angstrom) of the diamond-lattice Si-like model.
SP3_PARAMS = dict(
    orbitals="sp3",
    eps=dict(s=-5.2, p=1.2),
    V0=dict(sss=-1.9, sps=1.7, pps=3.0, ppp=-0.8),
    d0=5.43 * math.sqrt(3.0) / 4.0,   # ideal diamond nearest-neighbour distance
    lam=0.5,
    rcut=3.0,
    c_overlap=0.08,
    V_ref=3.0,
)

#: spd parameters (eV, Angstrom) of the fcc metal model.  The values are
#: synthetic: a d band near the half-filling chemical potential, s and p bands
#: above it, with Slater-Koster signs of a late transition metal.
SPD_PARAMS = dict(
    orbitals="spd",
    eps=dict(s=0.0, p=5.0, d=-2.0),
    V0=dict(sss=-1.2, sps=1.4, sds=-0.7, pps=2.0, ppp=-0.5, pds=-0.9,
            pdp=0.35, dds=-0.8, ddp=0.4, ddd=-0.06),
    d0=4.05 / math.sqrt(2.0),         # ideal fcc nearest-neighbour distance
    lam=0.6,
    rcut=5.0,
    c_overlap=0.05,
    V_ref=2.0,
)


def n_orbitals(kind: str) -> int:
    return {"s": 1, "sp3": 4, "spd": 9}[kind]


# ---------------------------------------------------------------------------
# lattices and geometries
# ---------------------------------------------------------------------------

def diamond_positions(nx: int, ny: int, nz: int, a: float) -> np.ndarray:
    """Diamond lattice: 8 atoms per conventional cubic cell of edge a."""
    fcc = np.array([[0, 0, 0], [0, .5, .5], [.5, 0, .5], [.5, .5, 0]], float)
    basis = np.concatenate([fcc, fcc + 0.25])
    return _tile(basis, nx, ny, nz, a)


def fcc_positions(nx: int, ny: int, nz: int, a: float) -> np.ndarray:
    """fcc lattice: 4 atoms per conventional cubic cell of edge a."""
    basis = np.array([[0, 0, 0], [0, .5, .5], [.5, 0, .5], [.5, .5, 0]], float)
    return _tile(basis, nx, ny, nz, a)


def _tile(basis, nx, ny, nz, a):
    g = np.stack(np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz),
                             indexing="ij"), -1).reshape(-1, 3)
    pos = (g[:, None, :] + basis[None, :, :]).reshape(-1, 3) * a
    return pos


def wrap(pos: np.ndarray, box: np.ndarray) -> np.ndarray:
    return np.mod(pos, box)


def min_image(d: np.ndarray, box: np.ndarray) -> np.ndarray:
    return d - box * np.round(d / box)


def rsa_positions(n: int, box: float, dmin: float, amp: float,
                  rng: np.random.Generator, batch: int = 4096) -> np.ndarray:
    """Random sequential addition in a periodic cube with a density modulation.

    A trial point r is accepted with probability (1 + amp*m(r)) / (1 + amp) and
    only if it keeps at least ``dmin`` from every accepted point.  m is a sum of
    four lowest-wavevector plane waves with seeded amplitudes and phases,
    scaled so that max |m| = 1 on a 32^3 grid.
    """
    ks = np.array([[1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 0]], float)
    coef = rng.uniform(0.5, 1.0, size=4)
    phase = rng.uniform(0, 2 * np.pi, size=4)

    def field(r):
        arg = 2 * np.pi * (r @ ks.T) / box + phase
        return np.cos(arg) @ coef

    g = (np.arange(32) + 0.5) / 32 * box
    grid = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    scale = np.abs(field(grid)).max()
    boxv = np.array([box, box, box])
    pts = np.zeros((0, 3))
    tree = None
    while len(pts) < n:
        cand = rng.uniform(0, box, size=(batch, 3))
        keep = rng.uniform(0, 1, size=batch) < (1 + amp * field(cand) / scale) / (1 + amp)
        cand = cand[keep]
        if tree is not None and len(cand):
            dist, _ = tree.query(cand, k=1)
            cand = cand[dist >= dmin]
        acc = []
        for c in cand:
            if acc:
                dd = min_image(np.asarray(acc) - c, boxv)
                if np.min(np.einsum("ij,ij->i", dd, dd)) < dmin * dmin:
                    continue
            acc.append(c)
            if len(pts) + len(acc) >= n:
                break
        if acc:
            pts = np.concatenate([pts, np.asarray(acc)])
            tree = cKDTree(pts, boxsize=boxv)
    return pts[:n]


# ---------------------------------------------------------------------------
# Slater-Koster two-centre blocks
# ---------------------------------------------------------------------------

def _bond_integrals(dist, prm):
    f = (prm["d0"] / dist) ** 2 * np.exp(-(dist - prm["d0"]) / prm["lam"])
    return {k: v * f for k, v in prm["V0"].items()}


def sk_blocks(dvec: np.ndarray, prm: dict) -> np.ndarray:
    """Slater-Koster blocks E_ab for bond vectors dvec (n, 3) -> (n, o, o).

    Orbital order: s, x, y, z [, xy, yz, zx, x2-y2, 3z2-r2].  Row index is the
    orbital on the origin atom, column the orbital on the atom at +dvec.
    """
    # written with analytic operations only, so that a complex bond vector
    # gives the complex-step derivative (sk_block_derivs)
    dist = np.sqrt(np.sum(dvec * dvec, axis=1))
    l, m, n = (dvec / dist[:, None]).T
    V = _bond_integrals(dist, prm)
    kind = prm["orbitals"]
    o = n_orbitals(kind)
    E = np.zeros((len(dist), o, o), dtype=np.result_type(dvec.dtype, np.float64))
    # s-s, s-p, p-p
    E[:, 0, 0] = V["sss"]
    dc = (l, m, n)
    for a in range(3):
        E[:, 0, 1 + a] = dc[a] * V["sps"]
        E[:, 1 + a, 0] = -dc[a] * V["sps"]
        for b in range(3):
            if a == b:
                E[:, 1 + a, 1 + b] = dc[a] ** 2 * V["pps"] + (1 - dc[a] ** 2) * V["ppp"]
            else:
                E[:, 1 + a, 1 + b] = dc[a] * dc[b] * (V["pps"] - V["ppp"])
    if kind == "sp3":
        return E
    if kind != "spd":
        raise ValueError(kind)
    l2, m2, n2 = l * l, m * m, n * n
    lm2 = l2 - m2
    zr = n2 - 0.5 * (l2 + m2)
    XY, YZ, ZX, X2, Z2 = 4, 5, 6, 7, 8
    # s-d (even parity: the d-s element equals the s-d element)
    sd = {XY: SQ3 * l * m, YZ: SQ3 * m * n, ZX: SQ3 * n * l,
          X2: 0.5 * SQ3 * lm2, Z2: zr}
    for b, f in sd.items():
        E[:, 0, b] = f * V["sds"]
        E[:, b, 0] = f * V["sds"]
    s, p = V["pds"], V["pdp"]
    lmn = l * m * n
    pd = {
        (1, XY): SQ3 * l2 * m * s + m * (1 - 2 * l2) * p,
        (1, YZ): SQ3 * lmn * s - 2 * lmn * p,
        (1, ZX): SQ3 * l2 * n * s + n * (1 - 2 * l2) * p,
        (2, XY): SQ3 * m2 * l * s + l * (1 - 2 * m2) * p,
        (2, YZ): SQ3 * m2 * n * s + n * (1 - 2 * m2) * p,
        (2, ZX): SQ3 * lmn * s - 2 * lmn * p,
        (3, XY): SQ3 * lmn * s - 2 * lmn * p,
        (3, YZ): SQ3 * n2 * m * s + m * (1 - 2 * n2) * p,
        (3, ZX): SQ3 * n2 * l * s + l * (1 - 2 * n2) * p,
        (1, X2): 0.5 * SQ3 * l * lm2 * s + l * (1 - lm2) * p,
        (2, X2): 0.5 * SQ3 * m * lm2 * s - m * (1 + lm2) * p,
        (3, X2): 0.5 * SQ3 * n * lm2 * s - n * lm2 * p,
        (1, Z2): l * zr * s - SQ3 * l * n2 * p,
        (2, Z2): m * zr * s - SQ3 * m * n2 * p,
        (3, Z2): n * zr * s + SQ3 * n * (l2 + m2) * p,
    }
    # p-d (odd parity: the d-p element is minus the p-d element)
    for (a, b), f in pd.items():
        E[:, a, b] = f
        E[:, b, a] = -f
    s, p, d = V["dds"], V["ddp"], V["ddd"]
    dd = {
        (XY, XY): 3 * l2 * m2 * s + (l2 + m2 - 4 * l2 * m2) * p + (n2 + l2 * m2) * d,
        (YZ, YZ): 3 * m2 * n2 * s + (m2 + n2 - 4 * m2 * n2) * p + (l2 + m2 * n2) * d,
        (ZX, ZX): 3 * n2 * l2 * s + (n2 + l2 - 4 * n2 * l2) * p + (m2 + n2 * l2) * d,
        (XY, YZ): 3 * l * m2 * n * s + l * n * (1 - 4 * m2) * p + l * n * (m2 - 1) * d,
        (YZ, ZX): 3 * m * n2 * l * s + m * l * (1 - 4 * n2) * p + m * l * (n2 - 1) * d,
        (ZX, XY): 3 * n * l2 * m * s + n * m * (1 - 4 * l2) * p + n * m * (l2 - 1) * d,
        (XY, X2): 1.5 * l * m * lm2 * s - 2 * l * m * lm2 * p + 0.5 * l * m * lm2 * d,
        (YZ, X2): 1.5 * m * n * lm2 * s - m * n * (1 + 2 * lm2) * p + m * n * (1 + 0.5 * lm2) * d,
        (ZX, X2): 1.5 * n * l * lm2 * s + n * l * (1 - 2 * lm2) * p - n * l * (1 - 0.5 * lm2) * d,
        (XY, Z2): SQ3 * l * m * zr * s - 2 * SQ3 * l * m * n2 * p + 0.5 * SQ3 * l * m * (1 + n2) * d,
        (YZ, Z2): SQ3 * m * n * zr * s + SQ3 * m * n * (l2 + m2 - n2) * p - 0.5 * SQ3 * m * n * (l2 + m2) * d,
        (ZX, Z2): SQ3 * l * n * zr * s + SQ3 * l * n * (l2 + m2 - n2) * p - 0.5 * SQ3 * l * n * (l2 + m2) * d,
        (X2, X2): 0.75 * lm2 ** 2 * s + (l2 + m2 - lm2 ** 2) * p + (n2 + 0.25 * lm2 ** 2) * d,
        (X2, Z2): 0.5 * SQ3 * lm2 * zr * s - SQ3 * n2 * lm2 * p + 0.25 * SQ3 * (1 + n2) * lm2 * d,
        (Z2, Z2): zr ** 2 * s + 3 * n2 * (l2 + m2) * p + 0.75 * (l2 + m2) ** 2 * d,
    }
    for (a, b), f in dd.items():
        E[:, a, b] = f
        E[:, b, a] = f
    return E


def sk_block_derivs(dvec: np.ndarray, prm: dict) -> np.ndarray:
    """d E_ab / d dvec_c for bond vectors dvec (n, 3) -> (n, 3, o, o), by
    complex-step differentiation (Squire and Trapp, SIAM Rev. 40, 1998): the
    imaginary part of E(dvec + i h e_c) / h, exact to rounding for h = 1e-30."""
    h = 1e-30
    out = []
    for c in range(3):
        dz = np.asarray(dvec, float).astype(complex)
        dz[:, c] += 1j * h
        out.append(sk_blocks(dz, prm).imag / h)
    return np.stack(out, 1)


def onsite_block(prm: dict) -> np.ndarray:
    kind = prm["orbitals"]
    e = prm["eps"]
    diag = [e["s"]]
    if kind in ("sp3", "spd"):
        diag += [e["p"]] * 3
    if kind == "spd":
        diag += [e["d"]] * 5
    return np.diag(diag)


# ---------------------------------------------------------------------------
# block-sparse H and S
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class TBSystem:
    """A periodic tight-binding system in atom-block CSR form.

    blk_ptr[a]..blk_ptr[a+1] index the blocks of block-row a; blk_col holds the
    column atom of each block (ascending within a row, diagonal included);
    H[k] and S[k] are the o x o blocks, row orbitals on the row atom.
    """
    pos: np.ndarray            # (n_atoms, 3) Angstrom, wrapped into the box
    box: np.ndarray            # (3,) orthorhombic periodic box lengths
    n_orb: int
    blk_ptr: np.ndarray        # int64 (n_atoms + 1)
    blk_col: np.ndarray        # int32 (nblk)
    H: np.ndarray              # float64 (nblk, o, o)
    S: np.ndarray              # float64 (nblk, o, o)
    name: str = ""
    # solve parameters of the workload
    region_mode: str = "all"   # "all" | "radius" | "nearest"
    region_radius: float = 0.0
    region_nrp: Optional[np.ndarray] = None   # int32 per atom for "nearest"
    p: int = 8
    q: int = 8
    kT: float = 0.1
    seed: int = 0
    params: Optional[dict] = None   # the generator parameters (for rebuilds and derivatives)

    @property
    def n_atoms(self) -> int:
        return int(self.pos.shape[0])

    @property
    def M(self) -> int:
        return self.n_atoms * self.n_orb

    @property
    def nblk(self) -> int:
        return int(self.blk_col.shape[0])

    @property
    def n_target(self) -> float:
        """Half filling: the column-summed electron number per spin, M/2."""
        return 0.5 * self.M

    def dense(self):
        """Dense (M x M) H and S; only for small systems."""
        o = self.n_orb
        Hd = np.zeros((self.M, self.M))
        Sd = np.zeros((self.M, self.M))
        for a in range(self.n_atoms):
            for k in range(self.blk_ptr[a], self.blk_ptr[a + 1]):
                b = self.blk_col[k]
                Hd[a * o:(a + 1) * o, b * o:(b + 1) * o] = self.H[k]
                Sd[a * o:(a + 1) * o, b * o:(b + 1) * o] = self.S[k]
        return Hd, Sd


def neighbour_pairs(pos: np.ndarray, box: np.ndarray, rcut: float):
    """All ordered pairs (i, j), i != j, with minimum-image distance < rcut."""
    tree = cKDTree(pos, boxsize=box)
    pairs = tree.query_pairs(rcut, output_type="ndarray")   # rows (a, b), a < b
    i = np.concatenate([pairs[:, 0], pairs[:, 1]])
    j = np.concatenate([pairs[:, 1], pairs[:, 0]])
    d = min_image(pos[j] - pos[i], box)
    return i.astype(np.int64), j.astype(np.int64), d


def build_tb(pos: np.ndarray, box, prm: dict, name: str = "") -> TBSystem:
    box = np.asarray(box, float)
    if np.any(prm["rcut"] >= box / 2):
        raise ValueError("cutoff must be below half the box")
    pos = wrap(np.asarray(pos, float), box)
    n = len(pos)
    o = n_orbitals(prm["orbitals"])
    i, j, d = neighbour_pairs(pos, box, prm["rcut"])
    # neighbour_pairs lists each unordered pair twice: first (a, b) with a < b,
    # then (b, a) in the same order.  Evaluate the first half only and mirror
    # it, H_ba = H_ab^T (the Slater-Koster parity relation for the reversed bond).
    npair = len(i) // 2
    Eh = sk_blocks(d[:npair], prm)
    E = np.concatenate([Eh, np.transpose(Eh, (0, 2, 1))])
    rows = np.concatenate([np.arange(n), i])
    cols = np.concatenate([np.arange(n), j])
    H = np.concatenate([np.broadcast_to(onsite_block(prm), (n, o, o)), E])
    Soff = prm["c_overlap"] * E / prm["V_ref"]
    S = np.concatenate([np.broadcast_to(np.eye(o), (n, o, o)), Soff])
    srt = np.lexsort((cols, rows))
    rows, cols = rows[srt], cols[srt]
    H = np.ascontiguousarray(H[srt])
    S = np.ascontiguousarray(S[srt])
    blk_ptr = np.zeros(n + 1, np.int64)
    np.add.at(blk_ptr, rows + 1, 1)
    blk_ptr = np.cumsum(blk_ptr)
    return TBSystem(pos=pos, box=box, n_orb=o, blk_ptr=blk_ptr,
                    blk_col=cols.astype(np.int32), H=H, S=S, name=name, params=prm)


def derivative_blocks(s: TBSystem):
    """dH, dS of shape (nblk, 3, o, o): the derivative of block k = (A, B) with
    respect to the position of its column atom B (zero on the atom-diagonal
    blocks, which do not depend on the geometry); the derivative with respect
    to R_A is its negative."""
    prm = s.params
    rows = np.repeat(np.arange(s.n_atoms), np.diff(s.blk_ptr))
    off = rows != s.blk_col
    d = min_image(s.pos[s.blk_col[off]] - s.pos[rows[off]], s.box)
    o = s.n_orb
    dH = np.zeros((s.nblk, 3, o, o))
    dH[off] = sk_block_derivs(d, prm)
    dS = prm["c_overlap"] * dH / prm["V_ref"]
    return dH, dS


def rebuild(s: TBSystem, pos: np.ndarray, name: str = "") -> TBSystem:
    """The same workload (generator, regions, p, q, kT) at new positions; the
    pattern is rebuilt from the cutoff."""
    t = build_tb(pos, s.box, s.params, name or s.name)
    t.region_mode, t.region_radius, t.region_nrp = s.region_mode, s.region_radius, s.region_nrp
    t.p, t.q, t.kT, t.seed = s.p, s.q, s.kT, s.seed
    return t


def md_updates(s: TBSystem, n_steps: int, sigma: float, seed0: int):
    """Successive geometry updates of an MD-style sequence: step k adds
    i.i.d. N(0, sigma^2) displacements (seed seed0 + k) to the previous
    positions and rebuilds the pattern."""
    out = []
    cur = s
    for k in range(1, n_steps + 1):
        rng = np.random.default_rng(seed0 + k)
        pos = cur.pos + rng.normal(0, sigma, size=cur.pos.shape)
        cur = rebuild(cur, pos, f"{s.name}_update{k}")
        cur.seed = seed0 + k
        out.append(cur)
    return out


# ---------------------------------------------------------------------------
# the workloads
# ---------------------------------------------------------------------------

def config_diamond64(seed: int = 1001) -> TBSystem:
    """64-atom diamond cell (2x2x2 conventional, a = 5.43), sigma 0.05, whole-cell
    regions, p = q = 8, kT = 0.1 eV.  M = 256."""
    rng = np.random.default_rng(seed)
    a = 5.43
    pos = diamond_positions(2, 2, 2, a)
    pos = pos + rng.normal(0, 0.05, size=pos.shape)
    s = build_tb(pos, [2 * a] * 3, SP3_PARAMS, name="diamond64")
    s.region_mode, s.p, s.q, s.kT, s.seed = "all", 8, 8, 0.1, seed
    return s


def config_diamond4096(seed: int = 2001, nrp: int = 120) -> TBSystem:
    """4,096-atom diamond supercell (8x8x8 conventional), sigma 0.05, regions of
    the 120 nearest atoms (480 orbitals), p = q = 15, kT = 0.1 eV.  M = 16,384."""
    rng = np.random.default_rng(seed)
    a = 5.43
    pos = diamond_positions(8, 8, 8, a)
    pos = pos + rng.normal(0, 0.05, size=pos.shape)
    s = build_tb(pos, [8 * a] * 3, SP3_PARAMS, name="diamond4096")
    s.region_mode = "nearest"
    s.region_nrp = np.full(s.n_atoms, nrp, np.int32)
    s.p, s.q, s.kT, s.seed = 15, 15, 0.1, seed
    return s


def config_disordered8000(seed: int = 3001, n_atoms: int = 8000) -> TBSystem:
    """Disordered cell by random sequential addition (d_min 2.2, mean density
    0.04997 / A^3 modulated by +-20 %), sp3 model, per-atom region sizes drawn
    uniformly from 60..260 atoms, p = q = 20, kT = 0.1 eV."""
    rng = np.random.default_rng(seed)
    box = (n_atoms / 0.04997) ** (1.0 / 3.0)
    pos = rsa_positions(n_atoms, box, 2.2, 0.2, rng)
    s = build_tb(pos, [box] * 3, SP3_PARAMS, name=f"disordered{n_atoms}")
    s.region_mode = "nearest"
    s.region_nrp = rng.integers(60, 261, size=n_atoms).astype(np.int32)
    s.p, s.q, s.kT, s.seed = 20, 20, 0.1, seed
    return s


def config_fcc_spd(seed: int = 5000, cells=(32, 32, 64), sigma: float = 0.08,
                   radius: float = 7.0) -> TBSystem:
    """spd fcc metal, a = 4.05: the default 32x32x64 conventional cells hold
    262,144 atoms (M = 2,359,296); sigma 0.08, cutoff 5.0, regions of radius
    7.0, p = q = 15, kT = 0.2 eV.  Smaller ``cells`` give the same local
    structure at a smaller size."""
    rng = np.random.default_rng(seed)
    a = 4.05
    pos = fcc_positions(*cells, a)
    pos = pos + rng.normal(0, sigma, size=pos.shape)
    s = build_tb(pos, np.array(cells, float) * a, SPD_PARAMS,
                 name=f"fcc_spd{len(pos)}")
    s.region_mode, s.region_radius = "radius", radius
    s.p, s.q, s.kT, s.seed = 15, 15, 0.2, seed
    return s


def random_pencil(n_atoms: int, n_orb: int, seed: int, s_scale: float = 0.05,
                  h_scale: float = 1.0) -> TBSystem:
    """Tiny dense random pencil (every block present): random symmetric H and
    S = I + small random symmetric, positive definite.  Geometry is a line of
    atoms; use with whole-system regions."""
    rng = np.random.default_rng(seed)
    M = n_atoms * n_orb
    A = rng.normal(size=(M, M)) * h_scale
    Hd = 0.5 * (A + A.T)
    B = rng.normal(size=(M, M)) * s_scale
    Sd = np.eye(M) + 0.5 * (B + B.T)
    w = np.linalg.eigvalsh(Sd)
    if w.min() <= 0.2:
        raise ValueError("random S not safely positive definite")
    o = n_orb
    rows = np.repeat(np.arange(n_atoms), n_atoms)
    cols = np.tile(np.arange(n_atoms), n_atoms)
    H = np.stack([Hd[r * o:(r + 1) * o, c * o:(c + 1) * o] for r, c in zip(rows, cols)])
    S = np.stack([Sd[r * o:(r + 1) * o, c * o:(c + 1) * o] for r, c in zip(rows, cols)])
    pos = np.stack([np.arange(n_atoms) * 1.0, np.zeros(n_atoms), np.zeros(n_atoms)], 1)
    blk_ptr = np.arange(n_atoms + 1, dtype=np.int64) * n_atoms
    return TBSystem(pos=pos, box=np.array([1e3, 1e3, 1e3]), n_orb=o,
                    blk_ptr=blk_ptr, blk_col=cols.astype(np.int32),
                    H=np.ascontiguousarray(H), S=np.ascontiguousarray(S),
                    name=f"pencil{M}", region_mode="all", seed=seed)


CONFIGS = {
    "diamond64": config_diamond64,
    "diamond4096": config_diamond4096,
    "disordered8000": config_disordered8000,
    "fcc_spd": config_fcc_spd,
}
