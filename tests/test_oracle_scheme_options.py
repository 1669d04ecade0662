"""The scheme options of the boundary (gf_config.limiter, .transverse) in the
oracle, pinned to what the textbook limiters and the 2D extension fix: the
limiter functions on the Sweby diagram's defining points and properties, the
order of accuracy each limiter gives on a smooth problem, the first-order
method without limiting, and the transverse terms vanishing on
one-dimensional data while keeping the unsplit run stable (Section 3.2)."""
import math

import numpy as np
import pytest

from paper_2403_15435_amd import inputs
from helpers import assemble, init_oracle

MC, MINMOD, SUPERBEE, VANLEER, NONE = 0, 1, 2, 3, 4


@pytest.fixture(scope="module")
def oracle_mod():
    import oracle
    oracle.build(force=False)
    return oracle


def test_limiter_functions(oracle_mod):
    """Points of the Sweby diagram and the defining properties: phi = 0 for
    theta <= 0; phi(1) = 1 (second order on smooth data); inside the TVD
    region 0 <= phi <= min(2 theta, 2); symmetric, phi(theta)/theta =
    phi(1/theta); minmod and superbee bound the second-order TVD region from
    below and above; the named values of each."""
    lim = oracle_mod.wave_limiter
    for L in (MC, MINMOD, SUPERBEE, VANLEER):
        for th in (-3.0, -0.5, 0.0):
            assert lim(L, th) == 0.0
        assert lim(L, 1.0) == 1.0
        for th in np.linspace(0.01, 20.0, 400):
            phi = lim(L, th)
            assert 0.0 <= phi <= min(2.0 * th, 2.0) + 1e-15
            assert phi / th == pytest.approx(lim(L, 1.0 / th), rel=1e-12)
            if L != MINMOD:
                assert lim(MINMOD, th) <= phi + 1e-15 and phi <= lim(SUPERBEE, th) + 1e-15
    assert lim(NONE, 0.7) == 0.0 and lim(NONE, 2.0) == 0.0
    # minmod: theta on [0, 1], then 1
    assert [lim(MINMOD, t) for t in (0.25, 0.5, 3.0)] == [0.25, 0.5, 1.0]
    # superbee: 2 theta to 1/2, 1 on [1/2, 1], theta on [1, 2], then 2
    assert [lim(SUPERBEE, t) for t in (0.25, 0.75, 1.5, 5.0)] == [0.5, 1.0, 1.5, 2.0]
    # MC: 2 theta to 1/3, (1 + theta)/2 on [1/3, 3], then 2
    assert [lim(MC, t) for t in (0.25, 1.0 / 3.0, 2.0, 4.0)] == pytest.approx([0.5, 2.0 / 3.0, 1.5, 2.0], rel=1e-15)
    # van Leer: 2 theta / (1 + theta), tending to 2
    assert lim(VANLEER, 3.0) == 1.5 and lim(VANLEER, 1e6) == pytest.approx(2.0, rel=1e-5)


def _hump(level, L=2000.0, h0=10.0, amp=0.05, sigma=150.0):
    m = 16
    sc = inputs.Scenario(name="hump", x0=0.0, y0=0.0, x1=L, y1=L, mi=1, mj=1, m=m, min_level=level,
                         max_level=level, manning_n=0.0, bc=(0, 0, 0, 0), t_end=30.0, init_level=level)
    n = m * (1 << level)
    sc.dem = np.zeros((n + 1, n + 1))
    sc.dem_level = level
    sc.eta_fn = lambda X, Y, b: h0 + amp * np.exp(-((X - L / 2) ** 2 + (Y - L / 2) ** 2) / (2 * sigma ** 2))
    return sc


def _run(oracle_mod, level, limiter=MC, transverse=0, cfl=0.9, t_end=30.0):
    sc = _hump(level)
    sc.t_end = t_end
    o = oracle_mod.Oracle(sc, cfl_desired=cfl, limiter=limiter, transverse=transverse)
    init_oracle(o, sc)
    o.advance(100000)
    assert o.t == t_end
    return assemble(sc, o.leaves(), o.state(), 0)


@pytest.mark.parametrize("limiter,lo,hi", [(MINMOD, 1.8, 2.3), (SUPERBEE, 1.8, 2.3), (VANLEER, 1.8, 2.3),
                                           (NONE, 0.9, 1.5)])
def test_order_of_accuracy_by_limiter(oracle_mod, limiter, lo, hi):
    """The smooth hump to t = 30 s at CFL 0.9, 64^2 and 128^2 cells against
    512^2 with the same limiter: a limited second-order method converges at
    about second order (measured 1.95-2.03), the method without corrections at
    first order (a pure first-order error shows 1.22 against this reference;
    measured 1.37)."""
    ref = _run(oracle_mod, 5, limiter)
    errs = []
    for level in (2, 3):
        h = _run(oracle_mod, level, limiter)
        r = ref.shape[0] // h.shape[0]
        errs.append(float(np.abs(h - ref.reshape(h.shape[0], r, h.shape[1], r).mean(axis=(1, 3))).mean()))
        assert np.array_equal(h, h.T)
    order = math.log2(errs[0] / errs[1])
    assert lo <= order <= hi, (errs, order)


def test_transverse_terms(oracle_mod):
    """Without transverse terms the unsplit 2D update is stable only to a
    Courant number of about 1/2: the hump at CFL 0.9 grows far past its
    amplitude, at CFL 0.45 it stays bounded; with them it is bounded at 0.9.
    On data that does not vary in y the transverse fluxes cancel exactly, so
    both forms give the same bits."""
    # 256^2 cells to t = 30 s (measured: 1.94 m at CFL 0.9 without the
    # transverse terms, 0.014 m at CFL 0.45 and with them)
    bad = _run(oracle_mod, 4, transverse=1, cfl=0.9)
    good = _run(oracle_mod, 4, transverse=0, cfl=0.9)
    half = _run(oracle_mod, 4, transverse=1, cfl=0.45)
    assert np.abs(good - 10.0).max() <= 0.05 and np.abs(half - 10.0).max() <= 0.05
    assert not np.isfinite(bad).all() or np.abs(bad - 10.0).max() > 0.5
    sc = inputs.ritter_dambreak(n_cells=64, m=16)
    sts = []
    for tr in (0, 1):
        o = oracle_mod.Oracle(sc, transverse=tr)
        init_oracle(o, sc)
        o.advance(40)
        sts.append(o.state())
    assert np.array_equal(sts[0], sts[1])
