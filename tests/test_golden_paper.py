"""Values the paper prints, held as fixtures under tests/golden/ with their
citation, against the synthetic inputs and the oracle: the floodplain
benchmark of Section 5.1 (domain, inlet segment, trapezoid inflow
hydrograph, friction, tolerances, final time).  The paper prints no worked
example of a step, so these pin the workload's definition, not a result."""
import json
import os

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def paper():
    with open(os.path.join(HERE, "golden", "floodplain_section5.json")) as f:
        return json.load(f)


def test_floodplain_inputs_follow_the_paper(paper):
    from paper_2403_15435_amd import inputs
    sc = inputs.flood_speed()
    d = paper["domain_m"]
    assert (sc.x0, sc.x1, sc.y0, sc.y1) == (d["x"][0], d["x"][1], d["y"][0], d["y"][1])
    assert sc.inflow_side == 0 and sc.bc[0] == inputs.BC_INFLOW
    assert all(b == inputs.BC_WALL for b in sc.bc[1:])
    assert (sc.inflow_lo, sc.inflow_hi) == (paper["inlet"]["y_lo_m"], paper["inlet"]["y_hi_m"])
    assert sc.inflow_hi - sc.inflow_lo == paper["inlet"]["length_m"]
    assert sc.manning_n == paper["manning_n"]
    assert sc.t_end == paper["final_time_h"] * 3600.0
    assert not np.any(sc.dem) and sc.dem.min() == 0.0     # flat bed
    # the paper's grid: 5 m, 200 x 400 cells; level 0 here is 6 x 12 trees of
    # 32^2 cells (5.2 m), since no power-of-two patch divides 200
    g = paper["uniform_grid"]
    assert g["cells"][0] * g["dx_m"] == d["x"][1] and g["cells"][1] * g["dx_m"] == d["y"][1]
    assert (sc.x1 - sc.x0) / (sc.mi * sc.m) == pytest.approx(1000.0 / 192)


def test_oracle_hydrograph_is_the_printed_trapezoid(paper):
    import oracle
    from paper_2403_15435_amd import inputs
    hy = paper["hydrograph_total_discharge"]
    q, r, p, f = hy["peak_m3_per_s"], 60.0 * hy["rise_min"], 60.0 * hy["plateau_min"], 60.0 * hy["fall_min"]
    o = oracle.Oracle(inputs.flood_speed(level_max=1))
    # linear rise from 0, plateau, linear fall to 0, then nothing
    for t, want in [(0.0, 0.0), (r / 4, q / 4), (r / 2, q / 2), (r, q), (r + p / 2, q), (r + p, q),
                    (r + p + f / 4, 0.75 * q), (r + p + f / 2, q / 2), (r + p + f, 0.0), (r + p + f + 600.0, 0.0)]:
        assert o.hydrograph(t) == pytest.approx(want, abs=1e-12), t
    # the total inflow volume: the trapezoid's area
    ts = np.linspace(0.0, r + p + f, 30001)
    vals = np.array([o.hydrograph(t) for t in ts])
    vol = float(np.sum((vals[1:] + vals[:-1]) * np.diff(ts)) / 2)
    assert vol == pytest.approx(q * (p + (r + f) / 2), rel=1e-9)


def test_oracle_defaults_follow_the_paper(paper):
    import oracle
    assert oracle.TAU_DEFAULT == paper["dry_tolerance_m"]
    # the adaptive step targets the paper's CFL number of 0.9
    import inspect
    sig = inspect.signature(oracle.Oracle.__init__)
    assert sig.parameters["cfl_desired"].default == paper["cfl_max"]
