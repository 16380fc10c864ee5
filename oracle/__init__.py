"""CPU oracle of the per-column multiple Arnoldi solve (arXiv:1202.0098, Sec. 2).

TEST INFRASTRUCTURE ONLY: the tests, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may use it; the HIP library never does, and the
two share no code.  Everything is FP64.

Split of the work:
  * ``ma_oracle.c`` (plain C + OpenMP, built by :func:`build`): per column the
    region operator, the inner CG for s_j = S^-1 e_j, the S-orthonormal basis
    of K_p(H; e_j) + K_q(H; s_j) (Eqs. 4, 6-9), the Galerkin pair (H~, S~)
    and its eigenpairs, and the Ritz vectors at the rows the outputs need.
  * this module (numpy): the real-space regions (Sec. 3), the Fermi-weighted
    density and energy-density matrices (Eqs. 13-14), the column energies
    (Eq. 17), the electron count Tr[rho S] and the bisection for the chemical
    potential (Sec. 2, last paragraph before Eq. 19), the atomic forces from
    the column outputs (Sec. 2, the force partial sums), and the subspace
    Green's function at complex energies with the density of states
    (Eqs. 11-12).

Conventions shared with the library's interface (an interface, not code):
  * a column j is a global orbital index, atom(j) = j // o, orbital j % o;
  * outputs live in the block-slot layout of the input: slot (k, r, c) of block
    k in block-row A holds the element (i, j) with j = (A, r) and
    i = (blk_col[k], c), i.e. block-row A stores columns j of atom A;
  * the electron count per column is N_j = sum_i rho_ij S_ji and the band
    energy per column E_j = sum_i rho_ij H_ji; both are per spin.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ma_oracle.c")
_LIB = os.path.join(_HERE, "libma_oracle.so")
_lib = None

STATUS = {0: "ok", -2: "no memory", -4: "not positive definite",
          -5: "CG not converged", -7: "pattern outside region"}


def build() -> str:
    """Compile the C part of the oracle with gcc (always rebuilds)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
           "-o", _LIB, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    i32, i64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.ora_solve_columns.restype = ctypes.c_int
    lib.ora_solve_columns.argtypes = [
        i32, i32, P, P, P, P, P, P, i32, P, i32, i32, f64, f64, P, i64, i32,
        P, P, P, P, P, P, P, P, i64, P, P]
    lib.ora_num_threads.restype = ctypes.c_int
    lib.ora_gen_eig.restype = ctypes.c_int
    lib.ora_gen_eig.argtypes = [i32, P, P, P, P]
    _lib = lib
    return lib


def num_threads() -> int:
    return int(_load().ora_num_threads())


def gen_eig(Ht, St):
    """The oracle's dense generalised eigensolver (Cholesky + cyclic Jacobi)."""
    n = Ht.shape[0]
    Ht = np.ascontiguousarray(Ht, np.float64)
    St = np.ascontiguousarray(St, np.float64)
    C = np.zeros((n, n))
    ev = np.zeros(n)
    rc = _load().ora_gen_eig(n, _ptr(Ht), _ptr(St), _ptr(C), _ptr(ev))
    if rc != 0:
        raise RuntimeError(STATUS.get(rc, rc))
    return ev, C


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


# ---------------------------------------------------------------------------
# regions (Sec. 3: real-space projection around the atom of basis j)
# ---------------------------------------------------------------------------

def region_of(pos, box, A, mode, radius=0.0, nrp=0):
    """Atoms of the region of atom A, ascending.

    mode "all": every atom.  "radius": atoms with minimum-image squared
    distance below radius**2.  "nearest": the nrp nearest atoms (A itself
    included), ties broken by the lower atom index.
    """
    n = len(pos)
    if mode == "all":
        return np.arange(n, dtype=np.int32)
    d = pos - pos[A]
    d = d - box * np.round(d / box)
    d2 = d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1] + d[:, 2] * d[:, 2]
    if mode == "radius":
        sel = np.nonzero(d2 < radius * radius)[0]
    elif mode == "nearest":
        order = np.lexsort((np.arange(n), d2))
        sel = np.sort(order[:int(nrp)])
    else:
        raise ValueError(mode)
    return sel.astype(np.int32)


def regions(sys, atoms=None):
    """CSR of regions (reg_ptr over all atoms, empty for atoms not listed)."""
    n = sys.n_atoms
    atoms = np.arange(n) if atoms is None else np.unique(np.asarray(atoms))
    lists = {}
    for A in atoms:
        nrp = 0 if sys.region_nrp is None else sys.region_nrp[A]
        lists[int(A)] = region_of(sys.pos, sys.box, int(A), sys.region_mode,
                                  sys.region_radius, nrp)
    cnt = np.zeros(n + 1, np.int64)
    for A, l in lists.items():
        cnt[A + 1] = len(l)
    reg_ptr = np.cumsum(cnt)
    reg_atoms = np.zeros(max(int(reg_ptr[-1]), 1), np.int32)
    for A, l in lists.items():
        reg_atoms[reg_ptr[A]:reg_ptr[A + 1]] = l
    return reg_ptr, reg_atoms


# ---------------------------------------------------------------------------
# the per-column solve (C)
# ---------------------------------------------------------------------------

def solve_raw(sys, cols=None, p=None, q=None, cg_tol=1e-12, tau=1e-10,
              x0=None, want_sj=False, want_reduced=False, reg=None):
    """Run the C part on the listed columns (all if None).

    Returns a dict with per-column arrays: eps, vj, svj (nu each), vpat
    (maxpat x nu), nu_eff, cg_iters, status, and optionally sj (local s_j),
    ht/st (reduced matrices).
    """
    lib = _load()
    o = sys.n_orb
    p = sys.p if p is None else p
    q = sys.q if q is None else q
    nu = p + q
    cols = np.arange(sys.M, dtype=np.int32) if cols is None else np.asarray(cols, np.int32)
    ncols = len(cols)
    if reg is None:
        reg = regions(sys, cols // o)
    reg_ptr, reg_atoms = reg
    rowlen = np.diff(sys.blk_ptr)
    maxpat = int(rowlen.max()) * o
    blk_ptr = np.ascontiguousarray(sys.blk_ptr, np.int64)
    blk_col = np.ascontiguousarray(sys.blk_col, np.int32)
    H = np.ascontiguousarray(sys.H, np.float64)
    S = np.ascontiguousarray(sys.S, np.float64)
    out = dict(
        nu_eff=np.zeros(ncols, np.int32), cg_iters=np.zeros(ncols, np.int32),
        status=np.zeros(ncols, np.int32), eps=np.zeros((ncols, nu)),
        vj=np.zeros((ncols, nu)), svj=np.zeros((ncols, nu)),
        vpat=np.zeros((ncols, maxpat, nu)))
    nloc_max = int(np.max(np.diff(reg_ptr))) * o
    sj = np.zeros((ncols, nloc_max)) if want_sj else None
    ht = np.zeros((ncols, nu, nu)) if want_reduced else None
    st = np.zeros((ncols, nu, nu)) if want_reduced else None
    x0a = None
    x0_stride = 0
    if x0 is not None:
        x0a = np.ascontiguousarray(x0, np.float64)
        x0_stride = x0a.shape[1]
    rc = lib.ora_solve_columns(
        sys.n_atoms, o, _ptr(blk_ptr), _ptr(blk_col), _ptr(H), _ptr(S),
        _ptr(reg_ptr), _ptr(reg_atoms), ncols, _ptr(cols), p, q,
        float(cg_tol), float(tau), _ptr(x0a), x0_stride, maxpat,
        _ptr(out["nu_eff"]), _ptr(out["cg_iters"]), _ptr(out["status"]),
        _ptr(out["eps"]), _ptr(out["vj"]), _ptr(out["svj"]), _ptr(out["vpat"]),
        _ptr(sj), nloc_max, _ptr(ht), _ptr(st))
    out["rc"] = rc
    out["cols"] = cols
    out["maxpat"] = maxpat
    out["nu"] = nu
    if want_sj:
        out["sj"] = sj
    if want_reduced:
        out["ht"], out["st"] = ht, st
    return out


# ---------------------------------------------------------------------------
# Fermi weighting and outputs (Eqs. 13, 14, 17), electron count, bisection
# ---------------------------------------------------------------------------

def fermi(x):
    """Fermi-Dirac occupation 1 / (1 + exp(x)), evaluated without overflow."""
    x = np.asarray(x, float)
    out = np.empty_like(x)
    neg = x <= 0
    out[neg] = 1.0 / (1.0 + np.exp(x[neg]))
    e = np.exp(-x[~neg])
    out[~neg] = e / (1.0 + e)
    return out


def occupations(raw, mu, kT):
    """f(eps_a) per column; zero for padded (dropped) Ritz slots."""
    eps = raw["eps"]
    mask = np.arange(eps.shape[1])[None, :] < raw["nu_eff"][:, None]
    f = np.zeros_like(eps)
    f[mask] = fermi((eps[mask] - mu) / kT)
    return f, mask


def column_weights(raw):
    """w_a^(j) = V_ja (S V)_ja: the weight of Ritz state a in N_j."""
    return raw["vj"] * raw["svj"]


def electron_count(raw, mu, kT):
    """sum_j N_j(mu) = sum_j sum_a f(eps_a) V_ja (S V)_ja  (per spin)."""
    f, _ = occupations(raw, mu, kT)
    return float(np.sum(f * column_weights(raw)))


def find_mu(raw, kT, n_target, max_iter=200):
    """Bisection for mu with sum_j N_j(mu) = n_target.

    Bracket [min eps - 50 kT, max eps + 50 kT]; stop when the bracket is below
    1e-13 max(1, |mu|) or after max_iter halvings; return the midpoint.
    """
    eps = raw["eps"]
    mask = np.arange(eps.shape[1])[None, :] < raw["nu_eff"][:, None]
    lo = float(eps[mask].min()) - 50 * kT
    hi = float(eps[mask].max()) + 50 * kT
    for _ in range(max_iter):
        mid = 0.5 * (lo + hi)
        if hi - lo <= 1e-13 * max(1.0, abs(mid)):
            break
        if electron_count(raw, mid, kT) < n_target:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def outputs(sys, raw, mu, kT):
    """rho_ij, pi_ij at the pattern slots of each column, and E_j, N_j.

    Returns (rho, pi, E, N): rho/pi of shape (ncols, maxpat) in the block-slot
    order of column j's block-row (slot t = block index within the row * o +
    column orbital), E and N of shape (ncols,).
    """
    o = sys.n_orb
    f, _ = occupations(raw, mu, kT)
    eps = np.where(np.isnan(raw["eps"]), 0.0, raw["eps"])
    t_rho = f * raw["vj"]                   # f_a V_ja
    t_pi = f * eps * raw["vj"]              # f_a eps_a V_ja
    rho = np.einsum("cta,ca->ct", raw["vpat"], t_rho)
    pi = np.einsum("cta,ca->ct", raw["vpat"], t_pi)
    cols = raw["cols"]
    E = np.zeros(len(cols))
    N = np.zeros(len(cols))
    for c, j in enumerate(cols):
        A, r = divmod(int(j), o)
        k0, k1 = sys.blk_ptr[A], sys.blk_ptr[A + 1]
        hrow = sys.H[k0:k1, r, :].reshape(-1)   # H_ji for i in the pattern
        srow = sys.S[k0:k1, r, :].reshape(-1)
        npat = len(hrow)
        E[c] = float(np.dot(rho[c, :npat], hrow))
        N[c] = float(np.dot(rho[c, :npat], srow))
    return rho, pi, E, N


def scatter_slots(sys, cols, vals):
    """Place per-column slot values into a full block-slot array (nblk, o, o)."""
    o = sys.n_orb
    out = np.zeros((sys.nblk, o, o))
    for c, j in enumerate(np.asarray(cols)):
        A, r = divmod(int(j), o)
        k0, k1 = sys.blk_ptr[A], sys.blk_ptr[A + 1]
        out[k0:k1, r, :] = vals[c, :(k1 - k0) * o].reshape(k1 - k0, o)
    return out


def solve(sys, cols=None, mu=None, kT=None, spin=2.0, **kw):
    """Full oracle pass: raw solve, mu (bisected at half filling if None),
    rho/pi per column, and the scalars E_band = g_s sum_j E_j,
    N_e = g_s sum_j N_j."""
    kT = sys.kT if kT is None else kT
    raw = solve_raw(sys, cols, **kw)
    if raw["rc"] != 0:
        bad = np.nonzero(raw["status"])[0]
        raise RuntimeError(f"oracle failed: {STATUS.get(int(raw['rc']), raw['rc'])} "
                           f"at column {int(raw['cols'][bad[0]])}")
    if mu is None:
        mu = find_mu(raw, kT, sys.n_target)
    rho, pi, E, N = outputs(sys, raw, mu, kT)
    return dict(raw=raw, mu=mu, rho=rho, pi=pi, E=E, N=N,
                energy=spin * float(np.sum(E)), n_elec=spin * float(np.sum(N)))


# ---------------------------------------------------------------------------
# atomic forces (Sec. 2: F_K as a sum of partial sums over the columns j)
# ---------------------------------------------------------------------------

def forces(sys, cols, rho, pi, dH, dS, spin=2.0):
    """F_K = -spin sum_j sum_i [rho_ij dH_ji/dR_K - pi_ij dS_ji/dR_K].

    rho, pi: per-column pattern slots as returned by :func:`outputs` (row c
    belongs to column cols[c]); dH, dS: (nblk, 3, o, o), the derivative of
    block k = (A, B) with respect to the position of its column atom B (its
    derivative with respect to R_A is the negative).  H_ji with j = (A, r) and
    i = (B, c) is element (r, c) of block (A, B), so column j contributes
    -spin g to F_B and +spin g to F_A, where
    g = sum_c [rho_ij dH_k[:, r, c] - pi_ij dS_k[:, r, c]].  The sign of the
    overlap term is that of the derivative of the grand potential with
    S-normalised eigenvectors (a reading: the paper prints both terms with
    the same sign).  Returns (n_atoms, 3), summed over the listed columns.
    """
    o = sys.n_orb
    F = np.zeros((sys.n_atoms, 3))
    for c, j in enumerate(np.asarray(cols)):
        A, r = divmod(int(j), o)
        k0, k1 = int(sys.blk_ptr[A]), int(sys.blk_ptr[A + 1])
        for kk in range(k1 - k0):
            k = k0 + kk
            B = int(sys.blk_col[k])
            if B == A:
                continue
            rv = rho[c, kk * o:(kk + 1) * o]
            pv = pi[c, kk * o:(kk + 1) * o]
            g = dH[k][:, r, :] @ rv - dS[k][:, r, :] @ pv
            F[B] -= spin * g
            F[A] += spin * g
    return F


# ---------------------------------------------------------------------------
# subspace Green's function at complex z and the density of states (Eqs. 11-12)
# ---------------------------------------------------------------------------

def green(sys, raw, z):
    """G_ij(z) = sum_a v_ia v_ja / (z - eps_a) at the pattern slots of every
    column (Eq. 12, the subspace Green's function applied to e_j, Eq. 11):
    complex array (ncols, maxpat)."""
    nu_eff = raw["nu_eff"]
    eps = raw["eps"]
    mask = np.arange(eps.shape[1])[None, :] < nu_eff[:, None]
    w = np.where(mask, 1.0 / (z - np.where(mask, eps, 0.0)), 0.0)
    return np.einsum("cta,ca->ct", raw["vpat"], w * raw["vj"])


def dos(raw, energies, eta, spin=2.0):
    """Density of states with Lorentzian broadening eta:
    D(E) = -spin/pi Im sum_j sum_a w_a / (E + i eta - eps_a), w_a = v_ja (S v_a)_j,
    the S-weighted trace of the subspace Green's functions (per column it
    integrates to N_j at full occupation)."""
    nu_eff = raw["nu_eff"]
    eps = raw["eps"]
    mask = np.arange(eps.shape[1])[None, :] < nu_eff[:, None]
    e = eps[mask]
    w = (raw["vj"] * raw["svj"])[mask]
    E = np.asarray(energies, float)[:, None]
    return spin / np.pi * np.sum(w[None, :] * eta / ((E - e[None, :]) ** 2 + eta * eta), axis=1)
