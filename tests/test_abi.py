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
    assert L.gf_profile_enable(None, 1) == gf.GF_E_INVALID
    assert L.gf_profile_read(None, None, None) == gf.GF_E_INVALID
    assert L.gf_run(None, 1, 0, 4, 16, None) == gf.GF_E_INVALID
    assert L.gf_net_collect(None, 16, 4, None, None, 0, None) == gf.GF_E_INVALID
    assert L.gf_set_gauges(None, 0, None, None, 1) == gf.GF_E_INVALID
    assert L.gf_step_lts(None, 1, None, None) == gf.GF_E_INVALID
    assert L.gf_get_gauges(None, 0, None, 0, None) == gf.GF_E_INVALID
    assert L.gf_tag(None, gf.GF_TAG_PLAIN, None, 0, None) == gf.GF_E_INVALID
    assert L.gf_set_initial(None, 0, gf.GF_IC_FN(0), None, 0) == gf.GF_E_INVALID
    assert L.gf_net_train_step_dev(None, None, None, 1, None, 0.1, None) == gf.GF_E_INVALID


def test_struct_layouts_match_the_header(tmp_path):
    """The binding's ctypes structures have the sizes and field offsets the C
    compiler gives the header's structures."""
    import subprocess
    import paper_2403_15435_amd as gf
    structs = {"gf_config": gf.gf_config, "gf_step_stats": gf.gf_step_stats, "gf_run_stats": gf.gf_run_stats,
               "gf_scenario_desc": gf.gf_scenario_desc}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "geoflood.h"', 'int main(void) {']
    for name, cls in structs.items():
        lines.append(f'printf("{name} size %zu\\n", sizeof({name}));')
        for fname, _ in cls._fields_:
            lines.append(f'printf("{name} {fname} %zu\\n", offsetof({name}, {fname}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    out = subprocess.check_output([str(exe)], text=True).split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for name, cls in structs.items():
        assert got[(name, "size")] == ctypes.sizeof(cls), name
        for fname, _ in cls._fields_:
            assert got[(name, fname)] == getattr(cls, fname).offset, (name, fname)


@pytest.mark.parametrize("bad", ["u", "q", "n_regions", "region_box", "region_levels", "region_fraction",
                                 "n_grades", "grade_quantity", "grade_threshold", "grade_level", "null_regions",
                                 "limiter", "transverse"])
def test_create_rejects_invalid_refinement_rules(bad):
    """Rules are checked before anything touches the device."""
    import paper_2403_15435_amd as gf
    L = gf.load()
    regions = (ctypes.c_double * 30)(*([10.0, 10.0, 20.0, 20.0, 1.0, 2.0] * 5))
    grades = (ctypes.c_double * 15)(*([0.0, 0.5, 1.0] * 5))
    d = gf.gf_scenario_desc(x0=0.0, y0=0.0, x1=100.0, y1=100.0, mi=1, mj=1, min_level=0, max_level=2,
                            manning_n=0.0, inflow_side=-1, tag_h_refine=0.1, tag_eta_refine=0.05, t_end=1.0,
                            n_regions=1, regions=regions, n_grades=1, grades=grades)
    if bad == "u":
        d.tag_u_refine = -1.0
    elif bad == "q":
        d.tag_q_refine = float("nan")
    elif bad == "n_regions":
        d.n_regions = 5
    elif bad == "region_box":
        regions[2] = 5.0                  # x1 < x0
    elif bad == "region_levels":
        regions[4], regions[5] = 3.0, 2.0  # min above max
    elif bad == "region_fraction":
        regions[4] = 1.5
    elif bad == "n_grades":
        d.n_grades = 5
    elif bad == "grade_quantity":
        grades[0] = 2.0
    elif bad == "grade_threshold":
        grades[1] = -0.5
    elif bad == "grade_level":
        grades[2] = -1.0
    elif bad == "null_regions":
        d.regions = None
    cfg = gf.gf_config(precision=gf.GF_FP64, m=16, g=9.81, dry_tol=1e-4, cfl_desired=0.9, cfl_max=1.0, n_scen=1,
                       scen=ctypes.pointer(d), max_patches=16, hip_stream=None)
    if bad == "limiter":
        cfg.limiter = 5
    elif bad == "transverse":
        cfg.transverse = 2
    out = ctypes.c_void_p()
    assert L.gf_create(ctypes.byref(cfg), ctypes.byref(out)) == gf.GF_E_INVALID
    assert not out.value
