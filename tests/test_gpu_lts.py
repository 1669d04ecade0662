"""Local time stepping on the GPU (gf_step_lts, reading R40) against the
oracle's: the same macro steps, rejections, clocks and states."""
import numpy as np
import pytest

import paper_2403_15435_amd as gf
from paper_2403_15435_amd import inputs
from helpers import check_fp32, init_oracle
from test_gpu_parity import amr_mesh_16

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def orc():
    import oracle
    oracle.build(force=False)
    return oracle


def _pair(orc, sc, leaves, prec=gf.GF_FP64, cap=256):
    f32 = prec == gf.GF_FP32
    o = orc.Oracle(sc, leaves=leaves)
    if f32:
        o.set_bathy_f32(True)
    init_oracle(o, sc, "f32" if f32 else "f64")
    ctx = gf.Context([sc], precision=prec, max_patches=cap)
    ctx.set_leaves(0, o.leaves())
    st = o.state()
    ctx.set_state(0, (st.astype(np.float32).astype(np.float64) if f32 else st)[:, :3])
    return o, ctx


def test_single_level_equals_gf_step(orc):
    sc = inputs.reservoir_fractal(level=2, m=16, L=2000.0, seed=3, radius=500.0)
    o, a = _pair(orc, sc, sc.uniform_leaves(2))
    b = gf.Context([sc], precision=gf.GF_FP64, max_patches=64)
    b.set_state(0, o.state()[:, :3])
    sa = a.step(20, lts=True)
    b.step(20)
    o.advance(20, lts=True)
    assert sa.steps == 20
    assert np.array_equal(a.state(0), b.state(0))
    assert np.array_equal(a.state(0)[:, :3], o.state()[:, :3])
    assert a.time(0) == b.time(0)


@pytest.mark.parametrize("sched", [-1, 0])
def test_amr_macro_steps_bit_exact(orc, sched):
    """Dam break on levels 1..3 (four ticks per macro step): 20 adaptive macro
    steps with their rejections, bit for bit with the oracle, on the resident
    and on the one-workgroup-per-patch schedule."""
    sc = inputs.reservoir_fractal(level=2, m=16, L=2000.0, seed=3, radius=500.0)
    sc.min_level, sc.max_level = 1, 3
    o, ctx = _pair(orc, sc, amr_mesh_16())
    ctx.set_schedule(sched)
    m0 = ctx.mass(0)[0]
    st = ctx.step(20, lts=True)
    o.advance(20, lts=True)
    t, dt, steps, rej = ctx.time(0)
    print(f"lts amr: t {t:.4f} s, {steps} macro steps, {rej} rejected (oracle {o.rejected})", flush=True)
    assert (t, dt, steps, rej) == (o.t, o.dt, o.steps, o.rejected)
    assert o.rejected > 0
    assert np.array_equal(ctx.state(0)[:, :3], o.state()[:, :3])
    lv = ctx.leaves(0)
    assert st.cell_updates == 20 * sum(16 * 16 << (l - 1) for l in lv[:, 1])
    M, cl, bd = ctx.mass(0)
    assert abs(M - m0 - cl - bd) <= 1e-12 * m0


def test_inflow_amr_with_regrids_bit_exact(orc):
    """The floodplain on levels 0..2 from the dry start: ten cycles of tag,
    regrid and 3 macro steps, bit for bit with the oracle (inflow at the tick
    times, three levels, regrids between calls)."""
    sc = inputs.flood_speed(level_max=2, m=16, mi=6, mj=12)
    o = orc.Oracle(sc)
    init_oracle(o, sc)
    ctx = gf.Context([sc], precision=gf.GF_FP64, max_patches=4096)
    ctx.set_state(0, o.state()[:, :3])
    for cycle in range(10):
        fo = o.tag()
        assert np.array_equal(ctx.tag(), fo), cycle
        o.regrid(fo)
        ctx.regrid(None)
        _, dts = o.advance(3, return_dt=True, lts=True)
        ctx.step(len(dts), dts, lts=True)
        assert np.array_equal(ctx.state(0)[:, :3], o.state()[:, :3]), cycle
    assert len(set(o.leaves()[:, 1].tolist())) == 3
    M, cl, bd = ctx.mass(0)
    assert bd > 0 and abs(M - cl - bd) <= 1e-12 * M


def test_fp32_amr_within_bars(orc):
    sc = inputs.reservoir_fractal(level=2, m=16, L=2000.0, seed=3, radius=500.0)
    sc.min_level, sc.max_level = 1, 3
    o, ctx = _pair(orc, sc, amr_mesh_16(), gf.GF_FP32)
    _, dts = o.advance(10, return_dt=True, lts=True)
    ctx.step(len(dts), dts, lts=True)
    rel, front = check_fp32(sc, o.leaves(), ctx.state(0), o.state(), 3)
    print(f"fp32 lts amr 10 macro steps: rel away from fronts {rel:.3e}, front abs {front:.3e}", flush=True)
    assert rel <= 2e-5 and front <= 1e-3


def test_fixed_macro_step_above_cfl_keeps_state(orc):
    sc = inputs.reservoir_fractal(level=2, m=16, L=2000.0, seed=3, radius=500.0)
    sc.min_level, sc.max_level = 1, 3
    o, ctx = _pair(orc, sc, amr_mesh_16())
    ctx.step(3, lts=True)
    s0, t0 = ctx.state(0), ctx.time(0)
    with pytest.raises(gf.GFError) as e:
        ctx.step(1, [500.0], lts=True)
    assert e.value.code == gf.GF_E_CFL
    assert np.array_equal(ctx.state(0), s0)
    assert ctx.time(0)[0] == t0[0] and ctx.time(0)[2] == t0[2]


def test_lts_then_gf_step_continues(orc):
    """After macro steps every patch is back in the common buffer: the plain
    clock continues from the same state as the oracle."""
    sc = inputs.reservoir_fractal(level=2, m=16, L=2000.0, seed=3, radius=500.0)
    sc.min_level, sc.max_level = 1, 3
    o, ctx = _pair(orc, sc, amr_mesh_16())
    _, d1 = o.advance(5, return_dt=True, lts=True)
    ctx.step(len(d1), d1, lts=True)
    _, d2 = o.advance(5, return_dt=True)
    ctx.step(len(d2), d2)
    assert np.array_equal(ctx.state(0)[:, :3], o.state()[:, :3])


def test_two_scenarios_with_different_level_spans(orc):
    """One context, two scenarios: a three-level AMR dam break (four ticks per
    macro step) and a single-level reservoir (one tick): each follows its own
    oracle bit for bit, clocks and rejections included."""
    a = inputs.reservoir_fractal(level=2, m=16, L=2000.0, seed=3, radius=500.0)
    a.min_level, a.max_level = 1, 3
    b = inputs.reservoir_fractal(level=2, m=16, L=2000.0, seed=8, radius=300.0)
    oa = orc.Oracle(a, leaves=amr_mesh_16())
    ob = orc.Oracle(b)
    init_oracle(oa, a)
    init_oracle(ob, b)
    ctx = gf.Context([a, b], precision=gf.GF_FP64, max_patches=256)
    ctx.set_leaves(0, oa.leaves())
    ctx.set_state(0, oa.state()[:, :3])
    ctx.set_state(1, ob.state()[:, :3])
    ctx.step(12, lts=True)
    oa.advance(12, lts=True)
    ob.advance(12, lts=True)
    for k, o in ((0, oa), (1, ob)):
        t, dt, steps, rej = ctx.time(k)
        assert (t, dt, steps, rej) == (o.t, o.dt, o.steps, o.rejected), k
        assert np.array_equal(ctx.state(k)[:, :3], o.state()[:, :3]), k


def test_gauges_record_each_macro_step(orc):
    """A gauge in a fine leaf and one in a coarse leaf: one record per
    accepted macro step, equal to the oracle's cell after that macro step."""
    from test_gpu_parity import _gauge_cell
    sc = inputs.reservoir_fractal(level=2, m=16, L=2000.0, seed=3, radius=500.0)
    sc.min_level, sc.max_level = 1, 3
    o, ctx = _pair(orc, sc, amr_mesh_16())
    pts = [(0, 310.0, 1720.0), (0, 1500.0, 600.0), (0, 1000.0, 1000.0)]
    ctx.set_gauges(pts, cap=32)
    want = [[] for _ in pts]
    for k in range(8):
        _, d = o.advance(1, return_dt=True, lts=True)
        ctx.step(1, list(d), lts=True)
        for g, (_, x, y) in enumerate(pts):
            want[g].append((o.t,) + _gauge_cell(sc, o.leaves(), o.state(), x, y))
    for g in range(len(pts)):
        assert np.array_equal(ctx.gauge(g), np.array(want[g])), g


def test_valley_outflow_amr_and_t_end(orc):
    """The small inflow valley (extrapolation outflow) refined by the plain
    tagger to levels 1 and 2, then macro steps to a t_end that truncates the
    last one: clocks, budget and state bit for bit with the oracle."""
    sc = inputs.v_valley(level_max=2, m=16, mi=4, mj=2, lx=4000.0, ly=2000.0, dem_level=2, init_level=0)
    sc.min_level = 0
    o = orc.Oracle(sc)
    init_oracle(o, sc)
    for _ in range(2):
        o.regrid(o.tag())
        init_oracle(o, sc)
    assert len(set(o.leaves()[:, 1].tolist())) == 2
    o.set_time(4000.0)
    t_end = 4000.0 + 37.3
    sc2 = inputs.v_valley(level_max=2, m=16, mi=4, mj=2, lx=4000.0, ly=2000.0, dem_level=2, init_level=0)
    sc2.min_level, sc2.t_end = 0, t_end
    o2 = orc.Oracle(sc2, leaves=o.leaves())
    o2.set_state(o.state())
    o2.set_time(4000.0)
    ctx = gf.Context([sc2], precision=gf.GF_FP64, max_patches=512)
    ctx.set_leaves(0, o2.leaves())
    ctx.set_state(0, o2.state()[:, :3])
    ctx.set_time(0, 4000.0)
    m0 = ctx.mass(0)
    st = ctx.step(1000, lts=True)
    o2.advance(1000, lts=True)
    t, dt, steps, rej = ctx.time(0)
    assert t == t_end == o2.t
    assert (steps, rej) == (o2.steps, o2.rejected)
    assert st.steps == steps
    assert np.array_equal(ctx.state(0)[:, :3], o2.state()[:, :3])
    M = ctx.mass(0)
    assert M[2] - m0[2] != 0.0
    assert abs((M[0] - m0[0]) - (M[1] - m0[1]) - (M[2] - m0[2])) <= 1e-12 * M[0]
