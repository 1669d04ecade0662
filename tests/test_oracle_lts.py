"""Pins of the oracle's local time stepping (reading R40: each level steps at
its own Courant-limited length, coarse ghosts of a fine substep interpolated
in time, fine fluxes summed over the substeps when refluxing), against what
the method fixes without it: the single-level case, steady and resting
states, the volume budget, and the plain AMR scheme it must stay close to."""
import numpy as np

from paper_2403_15435_amd import inputs
from helpers import init_oracle, to_finest


def _half_refined(sc):
    """Left half of one tree at level 2, right half at level 3 (16^2 patches)."""
    rows = []
    for iy in range(4):
        for ix in range(4):
            if ix >= 2:
                rows += [(0, 3, 2 * ix + a, 2 * iy + b) for b in range(2) for a in range(2)]
            else:
                rows.append((0, 2, ix, iy))
    return np.array(rows, np.int32)


def test_single_level_equals_the_plain_step(oracle_mod):
    """With one level there is one tick per step: the same results bit for bit."""
    sc = inputs.reservoir_fractal(level=2, m=16, L=2000.0, seed=3, radius=500.0)
    a = oracle_mod.Oracle(sc)
    b = oracle_mod.Oracle(sc)
    init_oracle(a, sc)
    init_oracle(b, sc)
    a.advance(20)
    b.advance(20, lts=True)
    assert a.t == b.t and a.steps == b.steps and a.rejected == b.rejected
    assert np.array_equal(a.state(), b.state())


def test_free_stream_and_lake_at_rest_on_amr(oracle_mod):
    """Uniform frictionless flow with open sides stays uniform bit for bit
    across coarse/fine faces (the fine records summed over two substeps equal
    the coarse record, so refluxing changes nothing); a deep lake over fractal
    terrain on three levels keeps its momentum at round-off."""
    h0, u0, v0 = 2.0, 1.5, -0.8
    sc = inputs.Scenario(name="stream", x0=0.0, y0=0.0, x1=320.0, y1=320.0, mi=1, mj=1, m=16,
                         min_level=0, max_level=2, manning_n=0.0, bc=(1, 1, 1, 1), init_level=1)
    sc.dem = np.zeros((17, 17)); sc.dem_level = 0
    sc.eta_fn = lambda X, Y, b: h0 + 0.0 * X
    sc.uv_fn = lambda X, Y, h: (h * u0, h * v0)
    lv = np.array([(0, 1, 0, 0), (0, 1, 1, 0), (0, 1, 0, 1)] + [(0, 2, 2 + a, 2 + b) for b in range(2) for a in range(2)],
                  np.int32)
    o = oracle_mod.Oracle(sc, leaves=lv)
    init_oracle(o, sc)
    o.advance(25, [0.6] * 25, lts=True)
    st = o.state()
    assert np.all(st[:, 0] == h0) and np.all(st[:, 1] == h0 * u0) and np.all(st[:, 2] == h0 * v0)

    lake = inputs.lake_at_rest(level=2, m=16, eta0=300.0, seed=7)
    lake.min_level, lake.max_level = 1, 3
    o = oracle_mod.Oracle(lake)
    fl = np.zeros(o.n_leaves, np.int8)
    fl[[2, 5, 9]] = 1
    fl[12:16] = -1
    o.regrid(fl)
    assert len(set(o.leaves()[:, 1].tolist())) == 2
    init_oracle(o, o.sc)
    o.advance(50, lts=True)
    assert np.abs(o.state()[:, 1:3]).max() <= 1e-10


def test_volume_budget_and_step_count(oracle_mod):
    """Dam break on three levels: the budget closes to round-off through
    rejected and accepted macro steps, and a macro step spans between 1.5
    and 2^(L1 - L0) = 4 plain steps of the same mesh (4 when the fastest
    waves sit on the finest level; here the coarse quadrants flood too)."""
    from test_gpu_parity import amr_mesh_16
    sc = inputs.reservoir_fractal(level=2, m=16, L=2000.0, seed=3, radius=500.0)
    sc.min_level, sc.max_level = 1, 3
    a = oracle_mod.Oracle(sc, leaves=amr_mesh_16())
    init_oracle(a, sc)
    m0 = a.mass()[0]
    a.advance(20, lts=True)
    M, cl, bd = a.mass()
    assert abs(M - m0 - cl - bd) <= 1e-13 * m0
    sc2 = inputs.reservoir_fractal(level=2, m=16, L=2000.0, seed=3, radius=500.0)
    sc2.min_level, sc2.max_level = 1, 3
    sc2.t_end = a.t
    c = oracle_mod.Oracle(sc2, leaves=amr_mesh_16())
    init_oracle(c, sc2)
    c.advance(100000)
    assert c.t == a.t
    ratio = c.steps / a.steps
    assert 1.5 <= ratio <= 4.0, ratio


def test_time_interpolation_on_an_accelerating_plane(oracle_mod):
    """Uniform flow down a plane (slope 1/1024, no friction) accelerates at
    g h S, linearly in time; the coarse ghosts of a fine substep halfway
    through the coarse step are then exact, and the run stays within 4e-4 m
    of the plain AMR run over the same time (holding the coarse state fixed
    over its step instead lags by g h S dt / 2 and departs by 1e-3 m)."""
    m, L, S, h0, u0 = 16, 2000.0, 1.0 / 1024, 2.0, 1.0

    def run(lts):
        sc = inputs.Scenario(name="plane", x0=0.0, y0=0.0, x1=L, y1=L, mi=1, mj=1, m=m, min_level=2, max_level=3,
                             manning_n=0.0, bc=(1, 1, 1, 1), init_level=2)
        nn = m * 8 + 1
        xs = np.linspace(0.0, L, nn)
        sc.dem = np.ascontiguousarray(np.tile(100.0 - S * xs, (nn, 1)))
        sc.dem_level = 3
        sc.eta_fn = lambda X, Y, b: b + h0
        sc.uv_fn = lambda X, Y, h: (h * u0, 0.0 * h)
        o = oracle_mod.Oracle(sc, leaves=_half_refined(sc))
        init_oracle(o, sc)
        if lts:
            o.advance(5, [2.0] * 5, lts=True)
        else:
            o.advance(10, [1.0] * 10)
        assert o.t == 10.0
        return to_finest(sc, o.leaves(), o.state(), 0, 3)
    d = np.abs(run(True) - run(False))[8:120, 24:104].max()
    assert d <= 4e-4, d


def test_moving_hump_accuracy(oracle_mod):
    """A hump crossing from the level-2 half into the level-3 half, to t = 60
    s, against a uniform level-4 run: the LTS error (mean |h - ref| on the
    level-3 grid) is no larger than 1.1 times that of plain AMR on the same
    mesh, with half as many steps."""
    def hump(lo, hi):
        sc = inputs.Scenario(name="hump", x0=0.0, y0=0.0, x1=2000.0, y1=2000.0, mi=1, mj=1, m=16, min_level=lo,
                             max_level=hi, manning_n=0.0, init_level=lo, t_end=60.0)
        sc.dem = np.zeros((17, 17)); sc.dem_level = 0
        sc.eta_fn = lambda X, Y, b: 10.0 + 0.5 * np.exp(-((X - 700) ** 2 + (Y - 1000) ** 2) / 150.0 ** 2) + 0.0 * b
        return sc
    ref = hump(4, 4)
    o = oracle_mod.Oracle(ref)
    init_oracle(o, ref)
    o.advance(100000)
    R = to_finest(ref, o.leaves(), o.state(), 0, 4).reshape(128, 2, 128, 2).mean(axis=(1, 3))
    sc = hump(2, 3)
    err, steps = {}, {}
    for lts in (False, True):
        o = oracle_mod.Oracle(sc, leaves=_half_refined(sc))
        init_oracle(o, sc)
        o.advance(100000, lts=lts)
        assert o.t == 60.0
        err[lts] = np.abs(to_finest(sc, o.leaves(), o.state(), 0, 3) - R).mean()
        steps[lts] = o.steps
    assert err[True] <= 1.1 * err[False], err
    assert steps[True] * 2 <= steps[False] + 2, steps
