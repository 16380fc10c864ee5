"""MI355X-native multiple Arnoldi solver (arXiv:1202.0098): Python binding.

A thin ctypes layer over ``libmarnoldi.so`` (HIP, gfx950), whose C interface
is ``include/marnoldi.h``.  This module only marshals arguments: every step of
the solve runs in the library's kernels.  PyTorch supplies device memory and
the stream.  If the library has not been built, importing works but every
call raises: there is no other code path.
"""

from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmarnoldi.so")

MA_OK, MA_EINVAL, MA_ENOMEM, MA_EDEVICE, MA_ENOTPD, MA_ENOCONV, MA_ESTATE = 0, -1, -2, -3, -4, -5, -6
REGION_MODES = {"all": 0, "radius": 1, "nearest": 2}
PREC = {"fp64": 0, "mixed": 1, "mixed_f64acc": 2}

# the functions include/marnoldi.h declares
API_FUNCTIONS = ("ma_version", "ma_default_opts", "ma_create", "ma_destroy", "ma_last_error",
                 "ma_build_system", "ma_system_info", "ma_region_sizes", "ma_region_atoms",
                 "ma_solve_columns", "ma_autotune", "ma_set_tuning", "ma_mlp_shape_of",
                 "ma_mlp_init", "ma_mlp_set_params", "ma_mlp_get_params", "ma_column_features",
                 "ma_mlp_forward", "ma_mlp_loss_grad", "ma_mlp_train_step", "ma_find_mu",
                 "ma_workspace_size", "ma_set_workspace", "ma_solve_columns_noalloc",
                 "ma_forces", "ma_dos", "ma_green")


class MarnoldiError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"[{status}] {msg}")
        self.status = status


class _System(ctypes.Structure):
    _fields_ = [("n_atoms", ctypes.c_int32), ("n_orb", ctypes.c_int32),
                ("blk_ptr", ctypes.c_void_p), ("blk_col", ctypes.c_void_p),
                ("H", ctypes.c_void_p), ("S", ctypes.c_void_p),
                ("xyz", ctypes.c_void_p), ("box", ctypes.c_void_p)]


class _Region(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("radius", ctypes.c_double),
                ("n_rp", ctypes.c_int32), ("n_rp_atom", ctypes.c_void_p)]


class _Opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("cg_tol", ctypes.c_double),
                ("inner_tol", ctypes.c_double), ("max_refine", ctypes.c_int32),
                ("breakdown_tau", ctypes.c_double), ("spin", ctypes.c_double),
                ("n_target", ctypes.c_double), ("start", ctypes.c_int32),
                ("slots_per_cu", ctypes.c_int32), ("schedule", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("basis_kernel", ctypes.c_int32),
                ("chunk_columns", ctypes.c_int32), ("pipeline", ctypes.c_int32),
                ("keep_sj", ctypes.c_int32)]


class _Tuning(ctypes.Structure):
    _fields_ = [("slots_per_cu", ctypes.c_int32), ("schedule", ctypes.c_int32),
                ("best_ms", ctypes.c_double), ("n_tried", ctypes.c_int32),
                ("tried_slots", ctypes.c_int32 * 64), ("tried_schedule", ctypes.c_int32 * 64),
                ("tried_ms", ctypes.c_double * 64), ("basis_kernel", ctypes.c_int32),
                ("tried_kernel", ctypes.c_int32 * 64), ("pipeline", ctypes.c_int32),
                ("tried_pipeline", ctypes.c_int32 * 64)]


SCHEDULES = {"lpt": 0, "input": 1, "xcd_input": 2, "xcd_lpt": 3, "spatial": 4}
BASIS_KERNELS = {"auto": 0, "onchip": 1, "workspace": 2, "group": 3, "atom": 4}


class _Result(ctypes.Structure):
    _fields_ = [("rho", ctypes.c_void_p), ("pi", ctypes.c_void_p), ("eps", ctypes.c_void_p),
                ("wts", ctypes.c_void_p), ("col_stats", ctypes.c_void_p),
                ("energy", ctypes.c_double), ("n_elec", ctypes.c_double),
                ("mu", ctypes.c_double), ("elapsed_ms", ctypes.c_double),
                ("kernel_ms", ctypes.c_double), ("sj_near", ctypes.c_void_p),
                ("eig_ms", ctypes.c_double)]


class _MlpShape(ctypes.Structure):
    _fields_ = [("n_in", ctypes.c_int32), ("n_hidden", ctypes.c_int32),
                ("n_out", ctypes.c_int32), ("n_params", ctypes.c_int64)]


STATS = 8   # per-column statistics (see ma_result.col_stats)


_lib = None


def library_available() -> bool:
    return os.path.exists(LIB_PATH)


def load_library():
    """Load libmarnoldi.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise MarnoldiError(MA_ESTATE, f"{LIB_PATH} is missing: run __graft_entry__.build() "
                            "(or python paper_1202_0098_amd/build.py)")
    # torch first: the library then binds to the HIP runtime torch has loaded,
    # so the process holds one runtime (and the caller's streams are its streams)
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    P, i32, i64, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.ma_version.restype = ctypes.c_char_p
    lib.ma_default_opts.argtypes = [ctypes.POINTER(_Opts)]
    lib.ma_create.argtypes = [ctypes.POINTER(P), i32, P]
    lib.ma_destroy.argtypes = [P]
    lib.ma_last_error.argtypes = [P]
    lib.ma_last_error.restype = ctypes.c_char_p
    lib.ma_build_system.argtypes = [P, ctypes.POINTER(_System), ctypes.POINTER(_Region)]
    lib.ma_system_info.argtypes = [P, P, P, P, P]
    lib.ma_solve_columns.argtypes = [P, i64, P, i32, i32, f64, f64, ctypes.POINTER(_Opts),
                                     ctypes.POINTER(_Result)]
    lib.ma_region_sizes.argtypes = [P, P, P]
    lib.ma_region_sizes.restype = ctypes.c_int
    lib.ma_region_atoms.argtypes = [ctypes.POINTER(_System), ctypes.POINTER(_Region), i32, P, i64]
    lib.ma_region_atoms.restype = ctypes.c_int64
    lib.ma_autotune.argtypes = [P, i64, P, i32, i32, f64, f64, ctypes.POINTER(_Opts), i32,
                                ctypes.POINTER(_Tuning)]
    lib.ma_set_tuning.argtypes = [P, i32, i32, i32, i32, i32, i32, i32]
    lib.ma_mlp_shape_of.argtypes = [P, ctypes.POINTER(_MlpShape)]
    lib.ma_mlp_init.argtypes = [P, ctypes.c_uint64]
    lib.ma_mlp_set_params.argtypes = [P, P, i64]
    lib.ma_mlp_get_params.argtypes = [P, P, i64]
    lib.ma_column_features.argtypes = [P, i64, P, P]
    lib.ma_mlp_forward.argtypes = [P, P, i64, P, i32]
    lib.ma_mlp_loss_grad.argtypes = [P, P, P, i64, P, i64, P, P]
    lib.ma_mlp_train_step.argtypes = [P, P, P, i64, P, i64, ctypes.c_float, P]
    lib.ma_find_mu.argtypes = [P, f64, f64, f64, ctypes.POINTER(_Result)]
    lib.ma_find_mu.restype = ctypes.c_int
    lib.ma_workspace_size.argtypes = [P, i64, P, i32, i32, f64, ctypes.POINTER(_Opts)]
    lib.ma_workspace_size.restype = ctypes.c_size_t
    lib.ma_set_workspace.argtypes = [P, P, ctypes.c_size_t]
    lib.ma_set_workspace.restype = ctypes.c_int
    lib.ma_solve_columns_noalloc.argtypes = [P, i64, P, i32, i32, f64, f64,
                                             ctypes.POINTER(_Opts), ctypes.POINTER(_Result)]
    lib.ma_solve_columns_noalloc.restype = ctypes.c_int
    lib.ma_forces.argtypes = [P, P, P, P, P, f64, P]
    lib.ma_forces.restype = ctypes.c_int
    lib.ma_dos.argtypes = [P, i64, P, f64, f64, P]
    lib.ma_dos.restype = ctypes.c_int
    lib.ma_green.argtypes = [P, f64, f64, P, P]
    lib.ma_green.restype = ctypes.c_int
    for name in ("ma_mlp_shape_of", "ma_mlp_init", "ma_mlp_set_params", "ma_mlp_get_params",
                 "ma_column_features", "ma_mlp_forward", "ma_mlp_loss_grad", "ma_mlp_train_step"):
        getattr(lib, name).restype = ctypes.c_int
    for name in ("ma_create", "ma_destroy", "ma_build_system", "ma_system_info",
                 "ma_solve_columns", "ma_autotune", "ma_set_tuning", "ma_mlp_shape_of",
                 "ma_mlp_init", "ma_mlp_set_params", "ma_mlp_get_params", "ma_column_features",
                 "ma_mlp_forward", "ma_mlp_loss_grad", "ma_mlp_train_step", "ma_find_mu",
                 "ma_set_workspace", "ma_solve_columns_noalloc"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def version() -> str:
    return load_library().ma_version().decode()


def default_opts(**kw) -> _Opts:
    o = _Opts()
    load_library().ma_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if k == "precision" and isinstance(v, str):
            v = PREC[v]
        if k == "schedule" and isinstance(v, str):
            v = SCHEDULES[v]
        if k == "start" and isinstance(v, str):
            v = {"zero": 0, "learned": 1, "previous": 2}[v]
        if k == "basis_kernel" and isinstance(v, str):
            v = BASIS_KERNELS[v]
        setattr(o, k, v)
    return o


def _ptr(a) -> Optional[int]:
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        return a.data_ptr()
    return a.ctypes.data


def region_atoms(tb, atom: int) -> np.ndarray:
    """The library's region of `atom` for a TBSystem-like input (host only)."""
    lib = load_library()
    blk_ptr = np.ascontiguousarray(tb.blk_ptr, np.int64)
    blk_col = np.ascontiguousarray(tb.blk_col, np.int32)
    H = np.ascontiguousarray(tb.H, np.float64)
    xyz = np.ascontiguousarray(tb.pos, np.float64)
    box = np.ascontiguousarray(tb.box, np.float64)
    nrp = None if tb.region_nrp is None else np.ascontiguousarray(tb.region_nrp, np.int32)
    sysd = _System(tb.n_atoms, tb.n_orb, _ptr(blk_ptr), _ptr(blk_col), _ptr(H), _ptr(H),
                   _ptr(xyz), _ptr(box))
    reg = _Region(REGION_MODES[tb.region_mode], float(tb.region_radius), 0, _ptr(nrp))
    out = np.zeros(tb.n_atoms, np.int32)
    n = lib.ma_region_atoms(ctypes.byref(sysd), ctypes.byref(reg), int(atom), _ptr(out),
                            tb.n_atoms)
    if n < 0:
        raise MarnoldiError(int(n), "ma_region_atoms: invalid arguments")
    return out[:n].copy()


@dataclass
class SolveResult:
    energy: float
    n_elec: float
    mu: float
    elapsed_ms: float
    kernel_ms: float
    eig_ms: float = 0.0


class Context:
    """One library context bound to a device and a stream (torch's current
    stream by default)."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        lib = load_library()
        self._lib = lib
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = ctypes.c_void_p()
        st = lib.ma_create(ctypes.byref(h), device, ctypes.c_void_p(stream.cuda_stream))
        if st != MA_OK:
            raise MarnoldiError(st, "ma_create failed")
        self._h = h
        self._keep = None

    def close(self):
        if getattr(self, "_h", None):
            self._lib.ma_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st: int):
        if st != MA_OK:
            raise MarnoldiError(st, self._lib.ma_last_error(self._h).decode())

    def build_system(self, n_atoms, n_orb, blk_ptr, blk_col, H, S, xyz=None, box=None,
                     region="all", radius=0.0, n_rp=0, n_rp_atom=None):
        """Upload a block-sparse pencil and build the regions (host arrays)."""
        arrs = dict(blk_ptr=np.ascontiguousarray(blk_ptr, np.int64),
                    blk_col=np.ascontiguousarray(blk_col, np.int32),
                    H=np.ascontiguousarray(H, np.float64),
                    S=np.ascontiguousarray(S, np.float64),
                    xyz=None if xyz is None else np.ascontiguousarray(xyz, np.float64),
                    box=None if box is None else np.ascontiguousarray(box, np.float64),
                    nrp=None if n_rp_atom is None else np.ascontiguousarray(n_rp_atom, np.int32))
        sysd = _System(int(n_atoms), int(n_orb), _ptr(arrs["blk_ptr"]), _ptr(arrs["blk_col"]),
                       _ptr(arrs["H"]), _ptr(arrs["S"]), _ptr(arrs["xyz"]), _ptr(arrs["box"]))
        reg = _Region(REGION_MODES[region], float(radius), int(n_rp), _ptr(arrs["nrp"]))
        self._check(self._lib.ma_build_system(self._h, ctypes.byref(sysd), ctypes.byref(reg)))

    def build_tb(self, tb):
        """build_system from a :class:`synth.TBSystem`-like object."""
        self.build_system(tb.n_atoms, tb.n_orb, tb.blk_ptr, tb.blk_col, tb.H, tb.S,
                          xyz=tb.pos, box=tb.box, region=tb.region_mode,
                          radius=tb.region_radius, n_rp=0, n_rp_atom=tb.region_nrp)

    def info(self):
        M, nblk = ctypes.c_int64(), ctypes.c_int64()
        nmax, maxpat = ctypes.c_int32(), ctypes.c_int32()
        self._check(self._lib.ma_system_info(self._h, ctypes.byref(M), ctypes.byref(nblk),
                                             ctypes.byref(nmax), ctypes.byref(maxpat)))
        return dict(M=M.value, nblk=nblk.value, nmax=nmax.value, maxpat=maxpat.value)

    def region_sizes(self, n_atoms: int):
        """(atoms per region, local operator blocks) for every atom."""
        ra = np.zeros(n_atoms, np.int32)
        lb = np.zeros(n_atoms, np.int64)
        self._check(self._lib.ma_region_sizes(self._h, _ptr(ra), _ptr(lb)))
        return ra, lb

    def autotune(self, cols, p, q, mu, kT, opts=None, reps=2):
        """Search basis kernel x slots per CU x schedule (and pipelining on or
        off) on the whole solve's device time; the best configuration is kept
        for (p, q, precision).  Returns a dict; `tried` holds (slots,
        schedule, ms, kernel) and `tried_pipeline` the pipeline option of
        each."""
        if cols is None:
            cptr, n = None, 0
        else:
            cols = np.ascontiguousarray(cols, np.int32)
            cptr, n = _ptr(cols), len(cols)
        o = opts if opts is not None else default_opts()
        t = _Tuning()
        self._check(self._lib.ma_autotune(self._h, n, cptr, int(p), int(q), float(mu), float(kT),
                                          ctypes.byref(o), int(reps), ctypes.byref(t)))
        names = {v: k for k, v in SCHEDULES.items()}
        knames = {v: k for k, v in BASIS_KERNELS.items()}
        return dict(slots_per_cu=t.slots_per_cu, schedule=names[t.schedule], best_ms=t.best_ms,
                    basis_kernel=knames[t.basis_kernel], pipeline=t.pipeline,
                    tried=[(t.tried_slots[i], names[t.tried_schedule[i]], t.tried_ms[i],
                            knames[t.tried_kernel[i]]) for i in range(t.n_tried)],
                    tried_pipeline=[t.tried_pipeline[i] for i in range(t.n_tried)])

    def set_tuning(self, p, q, precision, slots_per_cu, schedule, basis_kernel="auto",
                   pipeline=-1):
        prec = PREC[precision] if isinstance(precision, str) else int(precision)
        sch = SCHEDULES[schedule] if isinstance(schedule, str) else int(schedule)
        kern = BASIS_KERNELS[basis_kernel] if isinstance(basis_kernel, str) else int(basis_kernel)
        self._check(self._lib.ma_set_tuning(self._h, int(p), int(q), prec, int(slots_per_cu), sch,
                                            kern, int(pipeline)))

    # ---- learned CG start ----------------------------------------------------
    def mlp_shape(self):
        sh = _MlpShape()
        self._check(self._lib.ma_mlp_shape_of(self._h, ctypes.byref(sh)))
        return dict(n_in=sh.n_in, n_hidden=sh.n_hidden, n_out=sh.n_out, n_params=sh.n_params)

    def mlp_init(self, seed: int = 0):
        self._check(self._lib.ma_mlp_init(self._h, ctypes.c_uint64(seed)))

    def mlp_set_params(self, params):
        params = np.ascontiguousarray(params, np.float32)
        self._check(self._lib.ma_mlp_set_params(self._h, _ptr(params), len(params)))

    def mlp_get_params(self):
        n = self.mlp_shape()["n_params"]
        out = np.zeros(n, np.float32)
        self._check(self._lib.ma_mlp_get_params(self._h, _ptr(out), n))
        return out

    def column_features(self, cols, feat):
        cols = np.ascontiguousarray(cols, np.int32)
        self._check(self._lib.ma_column_features(self._h, len(cols), _ptr(cols), _ptr(feat)))

    def mlp_forward(self, x, n, y, bf16=True):
        self._check(self._lib.ma_mlp_forward(self._h, _ptr(x), int(n), _ptr(y), int(bool(bf16))))

    def _rows(self, x, n_rows):
        if n_rows is not None:
            return int(n_rows)
        return int(x.numel() // self.mlp_shape()["n_in"])

    def mlp_loss_grad(self, x, t, n, idx=None, want_grad=True, n_rows=None):
        """Loss and gradient on n rows (idx: rows of the tables x, t; n_rows:
        rows of the tables, default from x's size)."""
        loss = ctypes.c_double()
        g = np.zeros(self.mlp_shape()["n_params"], np.float32) if want_grad else None
        self._check(self._lib.ma_mlp_loss_grad(self._h, _ptr(x), _ptr(t), self._rows(x, n_rows),
                                               _ptr(idx), int(n), ctypes.byref(loss), _ptr(g)))
        return loss.value, g

    def mlp_train_step(self, x, t, n, lr, idx=None, n_rows=None):
        loss = ctypes.c_double()
        self._check(self._lib.ma_mlp_train_step(self._h, _ptr(x), _ptr(t), self._rows(x, n_rows),
                                                _ptr(idx), int(n), ctypes.c_float(lr),
                                                ctypes.byref(loss)))
        return loss.value

    def solve_columns(self, cols, p, q, mu=math.nan, kT=0.1, opts=None, rho=None, pi=None,
                      eps=None, wts=None, col_stats=None, sj_near=None,
                      noalloc=False) -> SolveResult:
        """Solve the listed columns (None = all).  rho/pi/eps/wts/col_stats are
        optional torch device tensors (float64 / int32) written by the library.
        noalloc=True calls the allocation-free entry point."""
        if cols is None:
            cptr, n = None, 0
        else:
            cols = np.ascontiguousarray(cols, np.int32)
            cptr, n = _ptr(cols), len(cols)
        o = opts if opts is not None else default_opts()
        res = _Result(_ptr(rho), _ptr(pi), _ptr(eps), _ptr(wts), _ptr(col_stats), 0.0, 0.0, 0.0,
                      0.0, 0.0, _ptr(sj_near), 0.0)
        fn = self._lib.ma_solve_columns_noalloc if noalloc else self._lib.ma_solve_columns
        self._check(fn(self._h, n, cptr, int(p), int(q), float(mu), float(kT), ctypes.byref(o),
                       ctypes.byref(res)))
        return SolveResult(res.energy, res.n_elec, res.mu, res.elapsed_ms, res.kernel_ms,
                           res.eig_ms)

    def find_mu(self, n_target, kT, spin=2.0, rho=None, pi=None) -> SolveResult:
        """Bisect mu again on the last bisected solve's Ritz data and rewrite
        rho/pi (optional torch device tensors) without re-solving."""
        res = _Result(_ptr(rho), _ptr(pi), None, None, None, 0.0, 0.0, 0.0, 0.0, 0.0, None, 0.0)
        self._check(self._lib.ma_find_mu(self._h, float(n_target), float(kT), float(spin),
                                         ctypes.byref(res)))
        return SolveResult(res.energy, res.n_elec, res.mu, res.elapsed_ms, 0.0, 0.0)

    def forces(self, dH, dS, rho, pi, forces, spin=2.0):
        """Atomic forces (device tensors: dH, dS nblk*3*o*o, rho, pi nblk*o*o,
        forces n_atoms*3)."""
        self._check(self._lib.ma_forces(self._h, _ptr(dH), _ptr(dS), _ptr(rho), _ptr(pi),
                                        float(spin), _ptr(forces)))

    def dos(self, energies, eta, spin=2.0) -> np.ndarray:
        """Density of states of the last solve at the given energies (host)."""
        e = np.ascontiguousarray(energies, np.float64)
        out = np.zeros_like(e)
        self._check(self._lib.ma_dos(self._h, len(e), _ptr(e), float(eta), float(spin), _ptr(out)))
        return out

    def green(self, z, g_re=None, g_im=None):
        """G_ij(z) at the pattern slots of the last (bisected) solve's columns."""
        self._check(self._lib.ma_green(self._h, float(z.real), float(z.imag), _ptr(g_re),
                                       _ptr(g_im)))

    def workspace_size(self, cols, p, q, mu=math.nan, opts=None) -> int:
        """Bytes of caller workspace a solve with these arguments needs."""
        if cols is None:
            cptr, n = None, 0
        else:
            cols = np.ascontiguousarray(cols, np.int32)
            cptr, n = _ptr(cols), len(cols)
        o = opts if opts is not None else default_opts()
        nbytes = self._lib.ma_workspace_size(self._h, n, cptr, int(p), int(q), float(mu),
                                             ctypes.byref(o))
        if nbytes == 0:
            raise MarnoldiError(MA_EINVAL, self._lib.ma_last_error(self._h).decode())
        return int(nbytes)

    def set_workspace(self, buf=None):
        """Use a caller-owned device buffer (a torch tensor, 256-byte aligned)
        for the per-solve buffers; None goes back to the library's own."""
        if buf is None:
            self._check(self._lib.ma_set_workspace(self._h, None, 0))
            self._keep = None
        else:
            self._check(self._lib.ma_set_workspace(self._h, buf.data_ptr(),
                                                   buf.numel() * buf.element_size()))
            self._keep = buf
