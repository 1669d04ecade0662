"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer:
the sanitized build (every report fatal) driven through each of its entry
points -- ghost fill, the adaptive step on a mesh with coarse/fine faces,
friction, inflow and outflow rules, tagging with regions and grades, regrids,
local time stepping, the mass budget -- on small scenarios, in a child
process started with the sanitizer runtime preloaded.  Its results must also
equal the plain build's bit for bit (the sanitizers change no arithmetic)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DRIVER = r'''
import sys
import numpy as np
sys.path.insert(0, ROOT)
sys.path.insert(0, ROOT + "/tests")
import oracle
from paper_2403_15435_amd import inputs
from helpers import init_oracle


def run(variant):
    out = []
    # AMR reservoir: fractal bed, friction, walls; refinement passes, steps
    # and regrids, then local time stepping
    sc = inputs.reservoir_fractal(level=2, m=16, L=2000.0, seed=3, radius=500.0)
    sc.min_level, sc.max_level, sc.init_level = 1, 3, 1
    o = oracle.Oracle(sc, variant=variant)
    init_oracle(o, sc)
    for _ in range(2):
        o.regrid(o.tag())
        init_oracle(o, sc)
    for _ in range(3):
        o.advance(5)
        o.regrid(o.tag())
    o.advance(2)
    out += [o.state(), o.mass(), o.leaves()]
    o.fill_ghosts()
    out.append(o.get_ghosted(0, 0))
    o2 = oracle.Oracle(sc, variant=variant, leaves=o.leaves())
    o2.set_state(o.state())
    o2.set_time(o.t, o.dt)
    o2.advance(2, lts=True)
    out += [o2.state(), o2.mass()]
    # inflow hydrograph, outflow, FP32 bed, a region and a grade
    v = inputs.v_valley(level_max=2, m=16, mi=4, mj=2, lx=4000.0, ly=2000.0, dem_level=2)
    v.regions = [(0.0, 900.0, 200.0, 1100.0, 1, 2)]
    v.grades = [(0, 0.5, 1)]
    o3 = oracle.Oracle(v, variant=variant)
    o3.set_bathy_f32(True)
    init_oracle(o3, v)
    o3.regrid(o3.tag())
    init_oracle(o3, v)
    o3.advance(6)
    out += [o3.state(), o3.mass(), np.array([o3.t, o3.dt, oracle.cbrt(3.0), o3.hydrograph(1800.0)])]
    return out


if __name__ == "__main__":
    got = run("asan")
    ref = run(None)
    assert len(got) == len(ref)
    for k, (a, b) in enumerate(zip(got, ref)):
        assert np.array_equal(np.asarray(a), np.asarray(b)), k
    print("sanitized oracle ok", len(got))
'''


def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    import oracle
    rt = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    if not os.path.isabs(rt) or not os.path.exists(rt):
        pytest.skip("gcc has no AddressSanitizer runtime here")
    oracle.build(force=False, variant="asan")
    oracle.build(force=False)
    script = tmp_path / "drive.py"
    script.write_text(f"ROOT = {ROOT!r}\n" + DRIVER)
    env = dict(os.environ)
    env["LD_PRELOAD"] = rt
    # the interpreter's own allocations are not the oracle's: no leak report
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:exitcode=86"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1:exitcode=87"
    env["OMP_NUM_THREADS"] = "2"
    r = subprocess.run([sys.executable, str(script)], env=env, capture_output=True, text=True, timeout=600)
    print(r.stdout[-2000:], r.stderr[-4000:])
    assert r.returncode == 0, r.stderr[-4000:]
    assert "sanitized oracle ok" in r.stdout
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
