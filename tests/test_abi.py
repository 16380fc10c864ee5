"""The C interface without a GPU: exported symbols and host-side logic."""

import ctypes
import os
import re

import numpy as np
import pytest

from paper_1202_0098_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = []
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            names += re.findall(r"MA_API\s+[\w\s\*]+?\b(ma_\w+)\s*\(", txt)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    import paper_1202_0098_amd as ma
    if not ma.library_available():
        pytest.fail("libmarnoldi.so is not built (run __graft_entry__.build())")
    return ma.load_library()


def test_library_exports_every_declared_function(lib):
    import paper_1202_0098_amd as ma
    declared = _declared_functions()
    assert len(declared) >= 9
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(ma.API_FUNCTIONS) == declared


def test_version_and_defaults(lib):
    import paper_1202_0098_amd as ma
    assert "gfx950" in ma.version()
    o = ma.default_opts()
    assert o.precision == 0 and o.cg_tol == 1e-12 and o.breakdown_tau == 1e-10
    assert o.spin == 2.0 and np.isnan(o.n_target)


def test_null_context_calls_fail_cleanly(lib):
    assert lib.ma_destroy(None) == -1
    assert lib.ma_last_error(None) == b"null context"


@pytest.mark.parametrize("name,atoms", [
    ("diamond4096", [0, 1, 7, 2044, 3000, 4095]),
    ("disordered", list(range(0, 2000, 97))),
    ("fcc_spd", [0, 5, 100, 511]),
])
def test_library_regions_match_oracle_regions(name, atoms):
    import oracle
    import paper_1202_0098_amd as ma
    if name == "diamond4096":
        s = synth.config_diamond4096()
    elif name == "disordered":
        s = synth.config_disordered8000(n_atoms=2000)
    else:
        s = synth.config_fcc_spd(cells=(4, 4, 8))
    for A in atoms:
        lib_reg = ma.region_atoms(s, A)
        nrp = 0 if s.region_nrp is None else s.region_nrp[A]
        ora_reg = oracle.region_of(s.pos, s.box, A, s.region_mode, s.region_radius, nrp)
        assert np.array_equal(lib_reg, ora_reg), (name, A)


def test_region_query_rejects_bad_arguments():
    import paper_1202_0098_amd as ma
    s = synth.config_diamond64()
    s.region_mode = "nearest"
    s.region_nrp = np.full(s.n_atoms, 0, np.int32)
    with pytest.raises(ma.MarnoldiError):
        ma.region_atoms(s, 0)
    s.region_nrp = np.full(s.n_atoms, 10, np.int32)
    with pytest.raises(ma.MarnoldiError):
        ma.region_atoms(s, s.n_atoms)
    assert len(ma.region_atoms(s, 3)) == 10
