"""gf_mass_static, the mass budget for callers that cannot allocate, against
gf_mass: equal bit for bit, on two calls in a row (the second on a smaller
context, so the shared static scratch holds more entries than it reads), and
again on the first context; too many patches are refused."""
import numpy as np
import pytest

import paper_2403_15435_amd as gf
from paper_2403_15435_amd import inputs

pytestmark = pytest.mark.gpu


def _check_all(ctx, n_scen, what):
    for k in range(n_scen):
        a = ctx.mass(k)
        b = ctx.mass_static(k)
        assert np.array_equal(a, b), (what, k, a, b)
    print(f"{what}: {n_scen} scenarios, mass_static equals mass bit for bit", flush=True)


def test_mass_static_equals_mass_on_two_calls():
    # call 1: 24 ensemble dam breaks (FP32, clamped volumes after 30 steps)
    scs = inputs.ensemble_dambreaks(24)
    big = gf.Context(scs, precision=gf.GF_FP32)
    for k in range(len(scs)):
        big.set_initial(k)
    big.step(30)
    n_big = sum(big.leaves(k).shape[0] for k in range(len(scs)))
    _check_all(big, len(scs), f"ensemble, {n_big} patches")
    # call 2: a smaller context (FP64 valley with inflow and outflow volumes)
    sc = inputs.v_valley(level_max=2, m=16, min_level=1)
    small = gf.Context([sc], precision=gf.GF_FP64, max_patches=2048)
    small.set_initial(0)
    small.set_time(0, 4000.0)
    small.step(20)
    n_small = small.leaves(0).shape[0]
    assert n_small < n_big
    m, c, b = small.mass_static(0)
    assert b != 0.0
    _check_all(small, 1, f"valley, {n_small} patches")
    # the first context again, after more steps
    big.step(5)
    _check_all(big, len(scs), "ensemble again")


def test_mass_static_refuses_more_patches_than_its_scratch():
    sc = inputs.Scenario(name="wide", x0=0.0, y0=0.0, x1=5000.0, y1=4000.0, mi=5, mj=4, m=16, min_level=6,
                         max_level=6, manning_n=0.0, init_level=6)
    sc.dem = np.zeros((4 * 16 + 1, 5 * 16 + 1))
    sc.dem_level = 0
    sc.eta_fn = lambda X, Y, b: 1.0 + 0.0 * b
    ctx = gf.Context([sc], precision=gf.GF_FP32, max_patches=5 * 4 * 4 ** 6)
    assert ctx.leaves(0).shape[0] == 81920
    with pytest.raises(gf.GFError) as e:
        ctx.mass_static(0)
    assert e.value.code == gf.GF_E_INVALID
    assert "65536" in str(e.value)
    ctx.mass(0)   # the allocating form still serves
