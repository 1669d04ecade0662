"""The C-ABI library builds, loads and exports every symbol include/geoflood.h
declares (no device calls: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "geoflood.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gf_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_symbols()
    for need in ["gf_create", "gf_set_bathymetry", "gf_fill_ghosts", "gf_step", "gf_tag", "gf_regrid", "gf_mass"]:
        assert need in names


def test_library_exports_every_declared_symbol():
    import paper_2403_15435_amd as gf
    lib = ctypes.CDLL(gf.LIB_PATH)
    for name in declared_symbols():
        assert hasattr(lib, name), name
    assert set(gf.EXPORTS) == set(declared_symbols())


def test_version_and_null_context():
    import paper_2403_15435_amd as gf
    L = gf.load()
    assert L.gf_version().startswith(b"geoflood")
    assert L.gf_step(None, 1, None, None) == gf.GF_E_INVALID
    assert L.gf_mass(None, 0, None, None, None) == gf.GF_E_INVALID
    assert L.gf_create(None, None) == gf.GF_E_INVALID
    assert L.gf_step_plain(None, 1, None, None) == gf.GF_E_INVALID
    assert L.gf_profile_patches(None, None, None) == gf.GF_E_INVALID
    assert L.gf_run(None, 1, 0, 4, 16, None) == gf.GF_E_INVALID
    assert L.gf_net_collect(None, 16, 4, None, None, 0, None) == gf.GF_E_INVALID
