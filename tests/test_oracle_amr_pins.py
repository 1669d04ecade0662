"""Pins of the oracle parts that the single-level pins do not reach: the cube
root of the friction term, the transverse form (grouped per cell against per
edge), coarse-to-fine ghost interpolation on a tilted free surface, the
adaptive mesh against the Ritter closed form, the momentum behaviour of
refluxing, and the independence of the results from the oracle's thread
count.  None of the expected values comes from the oracle itself."""
import math
from fractions import Fraction

import numpy as np
import pytest

from paper_2403_15435_amd import inputs
from exact_swe import ritter
from helpers import init_oracle, to_finest

G = 9.81


# ----------------------------------------------------------------- cube root
def test_cube_root_within_one_ulp(oracle_mod):
    """The friction term's h^(1/3) (eq. (manning), reading R8) is a Newton
    iteration after an exact reduction x = f 2^(3k + r); every residue r of
    the exponent takes its own branch.  Against numpy's cube root on 10^6
    log-uniform depths in [1e-8, 1e4] m it is within one ulp, and on a
    sample it brackets the exact root in rational arithmetic:
    (y - ulp)^3 < x < (y + ulp)^3."""
    rng = np.random.default_rng(11)
    x = np.exp(rng.uniform(math.log(1e-8), math.log(1e4), 1_000_000))
    # every branch of the reduction: exponents of all residues mod 3
    e = np.frexp(x)[1]
    assert set(np.unique(e % 3)) == {0, 1, 2}
    cb = oracle_mod.lib().orc_cbrt
    y = np.fromiter((cb(float(v)) for v in x), dtype=np.float64, count=x.size)
    ref = np.cbrt(x)
    ulps = np.abs(y - ref) / np.spacing(ref)
    assert ulps.max() <= 1.0, ulps.max()
    for v, r in zip(x[:3000], y[:3000]):
        u = Fraction(float(np.spacing(r)))
        X, Y = Fraction(float(v)), Fraction(float(r))
        assert (Y - u) ** 3 < X < (Y + u) ** 3
    # exact cubes come back exactly
    for k in (-9, -3, 0, 1, 2, 5):
        for base in (1.0, 1.5, 3.0, 7.0):
            v = base * 2.0 ** k
            assert cb(v ** 3) == v


# ----------------------------------------------------------- transverse form
def _forced_pair(oracle_mod, sc, nsteps):
    a = oracle_mod.Oracle(sc)
    b = oracle_mod.Oracle(sc, variant="per_edge")
    init_oracle(a, sc)
    init_oracle(b, sc)
    _, dts = a.advance(nsteps, return_dt=True)
    b.advance(len(dts), dts)
    return a.state(), b.state()


def _rel_errors(sa, sb):
    w = sa[:, 0] >= 1e-2
    rel_h = float((np.abs(sa[:, 0] - sb[:, 0])[w] / sa[:, 0][w]).max())
    rel_m = max(float(np.abs(sa[:, f] - sb[:, f]).max() / np.abs(sa[:, f]).max()) for f in (1, 2))
    return rel_h, rel_m


def test_transverse_grouped_equals_per_edge(oracle_mod):
    """Reading R11': the oracle splits each cell's net normal increment
    (A+dQ - F of its left edge plus A-dQ + F of its right edge) with the Roe
    state of the cell and its transverse neighbour.  The transverse solver is
    linear in the increment and both edges share that state, so this equals
    splitting each edge's increment on its own (the per-edge form, built from
    the same source with ORC_TRANSVERSE_PER_EDGE) up to rounding.  Fully wet
    terrain, 100 steps: per cell 1e-12 relative in h, 1e-12 of the field's
    largest value in hu, hv.  With wet/dry fronts the rounding difference of
    a single step is the same size, and it is amplified by the front's
    wet/dry decisions over later steps (reported, bounded at 10 steps)."""
    sc = inputs.wet_dambreak(level=3, m=16, L=2000.0, seed=2, radius=300.0)
    rel_h, rel_m = _rel_errors(*_forced_pair(oracle_mod, sc, 100))
    print(f"fully wet, 100 steps: {rel_h:.2e} in h, {rel_m:.2e} in momentum")
    assert rel_h <= 1e-12 and rel_m <= 1e-12
    sc = inputs.reservoir_fractal(level=3, m=16, L=2000.0, seed=2, radius=300.0)
    for n, bar in ((1, 1e-14), (10, 1e-12)):
        rel_h, rel_m = _rel_errors(*_forced_pair(oracle_mod, sc, n))
        print(f"reservoir with fronts, {n} steps: {rel_h:.2e} in h, {rel_m:.2e} in momentum")
        assert rel_h <= bar and rel_m <= bar


# ------------------------------------------- coarse-to-fine interpolation
def _tilted(level=2, m=16, L=2000.0):
    """Linear bed and linear free surface and momenta on a flat square, so
    that every limited slope equals the exact difference."""
    sc = inputs.Scenario(name="tilted", x0=0.0, y0=0.0, x1=L, y1=L, mi=1, mj=1, m=m, min_level=0,
                         max_level=6, manning_n=0.0, init_level=level)
    n = m + 1
    X, Y = np.meshgrid(np.linspace(0.0, L, n), np.linspace(0.0, L, n))
    sc.dem = 1.0 + 0.003 * X - 0.001 * Y
    sc.dem_level = 0
    eta = lambda X, Y: 10.0 + 0.01 * X + 0.02 * Y
    hu = lambda X, Y: 0.5 + 0.001 * X - 0.002 * Y
    hv = lambda X, Y: -0.3 + 0.0015 * X + 0.0005 * Y
    return sc, eta, hu, hv


def _cover(sc, lv, l, I, J):
    """Index of the leaf holding the level-l cell (I, J)."""
    m = sc.m
    for k, (t, ll, ix, iy) in enumerate(lv):
        s = 1 << (l - ll) if ll <= l else None
        if s is None:
            continue
        if ix * m * s <= I < (ix + 1) * m * s and iy * m * s <= J < (iy + 1) * m * s:
            return k
    return -1


def test_coarse_to_fine_ghosts_on_tilted_surface(oracle_mod):
    """Reading R14 on a linear free surface eta = 10 + 0.01x + 0.02y with
    linear momenta: the minmod slopes of the coarse parent equal the exact
    differences, so a fine ghost cell gets the exact linear value at its own
    coordinate along every direction in which the parent has both
    neighbours inside the coarse leaf, and the parent's coordinate along a
    direction in which it has not (the stencil stays inside that leaf).
    h + b must equal eta there, hu and hv the linear momenta, to round-off.
    The x and y slopes differ, so a swapped offset sign or a slope from the
    wrong neighbours is off by a quarter coarse cell's change.  Coarse ghost
    cells next to finer leaves (4-child means) must also reproduce the
    linear fields at their own centres."""
    sc, eta, hu_f, hv_f = _tilted()
    o = oracle_mod.Oracle(sc)
    fl = np.zeros(o.n_leaves, np.int8)
    fl[[3, 6, 9, 12]] = 1          # a few level-2 patches refined, mixed faces and corners
    o.regrid(fl)
    lv = o.leaves()
    assert set(lv[:, 1]) == {2, 3}
    # exact linear state on every leaf, from the oracle's own cell beds
    for k in range(lv.shape[0]):
        X, Y = sc.cell_centres(lv[k])
        b = o.get_field(k, 3)
        o.set_field(k, 0, eta(X, Y) - b)
        o.set_field(k, 1, hu_f(X, Y))
        o.set_field(k, 2, hv_f(X, Y))
    o.fill_ghosts()
    m = sc.m
    checked = {"fine_t": 0, "fine_both": 0, "coarse": 0}
    worst = 0.0
    for k, (t, l, ix, iy) in enumerate(lv):
        gh = [o.get_ghosted(k, f) for f in range(4)]
        dx, dy = sc.dx(l), sc.dy(l)
        NI = sc.mi * m << l
        for j in range(-2, m + 2):
            for i in range(-2, m + 2):
                if 0 <= i < m and 0 <= j < m:
                    continue
                I, J = ix * m + i, iy * m + j
                if not (0 <= I < NI and 0 <= J < NI):
                    continue
                src = _cover(sc, lv, l, I, J)
                if src < 0:
                    # covered by finer leaves: a coarse ghost, 4-child means
                    xs, ys = (I + 0.5) * dx, (J + 0.5) * dy
                    checked["coarse"] += 1
                else:
                    sl = int(lv[src, 1])
                    if sl == l:
                        continue
                    assert sl == l - 1
                    Ic, Jc = I >> 1, J >> 1
                    ci, cj = Ic - int(lv[src, 2]) * m, Jc - int(lv[src, 3]) * m
                    hasx = 1 <= ci <= m - 2
                    hasy = 1 <= cj <= m - 2
                    dxc, dyc = sc.dx(sl), sc.dy(sl)
                    xs = (I + 0.5) * dx if hasx else (Ic + 0.5) * dxc
                    ys = (J + 0.5) * dy if hasy else (Jc + 0.5) * dyc
                    checked["fine_both" if (hasx and hasy) else "fine_t"] += int(hasx or hasy)
                g = (j + 2, i + 2)
                err = max(abs(gh[0][g] + gh[3][g] - eta(xs, ys)), abs(gh[1][g] - hu_f(xs, ys)),
                          abs(gh[2][g] - hv_f(xs, ys)))
                worst = max(worst, err)
    print(f"ghost cells checked {checked}, worst error {worst:.2e}")
    assert worst <= 1e-11
    assert checked["fine_t"] >= 100 and checked["coarse"] >= 100


# ------------------------------------------------------ AMR against Ritter
def _ritter_run(oracle_mod, level, band=None):
    """Ritter dam break (2000 m box, 16x16 patches) on a uniform level, or on
    that level with the patch columns whose x range lies in `band` refined
    once."""
    sc = inputs.ritter_dambreak(16 << level, 16)
    sc.min_level, sc.max_level = level, level + 1
    o = oracle_mod.Oracle(sc)
    if band is not None:
        lv = o.leaves()
        w = sc.m * sc.dx(level)
        fl = np.array([1 if band[0] <= ix * w and (ix + 1) * w <= band[1] else 0 for _, _, ix, _ in lv], np.int8)
        o.regrid(fl)
    init_oracle(o, sc)
    o.advance(100000)
    assert o.t == 50.0
    return sc, o


def test_amr_band_against_ritter(oracle_mod):
    """The dry-bed dam break with a refined band of patch columns over the
    dam (x in [750, 1500] m: level 4 inside, level 3 outside).  The
    rarefaction crosses both coarse/fine faces.  Inside the band the
    adaptive run differs from the uniform level-4 run by at most twice the
    uniform run's own error against the closed form (Section 4: refinement
    must not cost accuracy where the fine level covers the flow), the
    solution stays y-invariant bit for bit with no transverse momentum, and
    the volume budget closes."""
    band = (750.0, 1500.0)
    sc4, o4 = _ritter_run(oracle_mod, 4)
    sca, oa = _ritter_run(oracle_mod, 3, band)
    assert set(oa.leaves()[:, 1]) == {3, 4}
    Ha = to_finest(sca, oa.leaves(), oa.state(), 0, 4)
    HVa = to_finest(sca, oa.leaves(), oa.state(), 2, 4)
    H4 = to_finest(sc4, o4.leaves(), o4.state(), 0, 4)
    assert np.all(Ha == Ha[0:1, :]) and np.all(HVa == 0.0)
    dx = sc4.dx(4)
    x = (np.arange(Ha.shape[1]) + 0.5) * dx
    hR, _ = ritter(x, 50.0, 1000.0, 10.0)
    inb = (x > band[0]) & (x < band[1])
    e_uni = np.abs(H4[0][inb] - hR[inb]).sum() * dx
    d_amr = np.abs(Ha[0][inb] - H4[0][inb]).sum() * dx
    e_amr = np.abs(Ha[0][inb] - hR[inb]).sum() * dx
    print(f"band L1: uniform-fine vs Ritter {e_uni:.3f}, AMR vs uniform-fine {d_amr:.3f}, AMR vs Ritter {e_amr:.3f}")
    assert d_amr <= 2.0 * e_uni
    M, clamp, bnd = oa.mass()
    M0 = 10.0 * 1000.0 * 2000.0
    assert abs(M - M0 - clamp - bnd) <= 1e-12 * M0


# --------------------------------------------------- refluxing and momentum
def _hump(level, L=4000.0, m=16, h0=10.0, amp=0.5, xc=1250.0, yc=2000.0, sig=200.0):
    """A right-moving linear wave on a still lake over a flat bed: the
    momentum hu = c (h - h0) sits in the hump, the lake around it is at rest,
    and nothing reaches the walls during the run."""
    sc = inputs.Scenario(name="hump", x0=0.0, y0=0.0, x1=L, y1=L, mi=1, mj=1, m=m, min_level=0, max_level=8,
                         manning_n=0.0, init_level=level, t_end=60.0)
    sc.dem = np.zeros((m + 1, m + 1))
    sc.dem_level = 0
    c = math.sqrt(G * h0)
    sc.eta_fn = lambda X, Y, b: h0 + amp * np.exp(-((X - xc) ** 2 + (Y - yc) ** 2) / sig ** 2) + 0.0 * b
    sc.uv_fn = lambda X, Y, h: (c * (h - h0), 0.0 * h)
    return sc


def _momentum_drift(oracle_mod, level, band):
    sc = _hump(level)
    o = oracle_mod.Oracle(sc)
    if band:
        lv = o.leaves()
        w = sc.m * sc.dx(level)
        o.regrid(np.array([1 if 1500.0 <= ix * w and (ix + 1) * w <= 2500.0 else 0 for _, _, ix, _ in lv], np.int8))
    init_oracle(o, sc)

    def P():
        st, lv = o.state(), o.leaves()
        return sum(st[k, 1].sum() * sc.dx(l) * sc.dy(l) for k, (_, l, _, _) in enumerate(lv))
    p0 = P()
    o.advance(100000)
    assert o.t == 60.0
    return (P() - p0) / p0, len(set(o.leaves()[:, 1]))


def test_reflux_momentum_drift_bound(oracle_mod):
    """Reading R17' corrects the coarse face cell's depth to the fine side's
    volume flux and keeps its velocity; momentum fluxes at coarse/fine faces
    are not matched, so the total momentum of a wave crossing a refined band
    drifts.  On a uniform mesh the scheme conserves it to round-off (flat
    bed, walls untouched); on the band the drift stays below 1% of the
    wave's momentum and falls at first order when both levels are refined
    (error ratio >= 1.8 per doubling)."""
    for lvl in (3, 4):
        d, nl = _momentum_drift(oracle_mod, lvl, False)
        assert nl == 1 and abs(d) <= 1e-10
    d3, nl3 = _momentum_drift(oracle_mod, 3, True)
    d4, nl4 = _momentum_drift(oracle_mod, 4, True)
    print(f"momentum drift on the band: {d3:.3e} (levels 3-4), {d4:.3e} (levels 4-5)")
    assert nl3 == 2 and nl4 == 2
    assert abs(d3) <= 1e-2 and abs(d4) <= 1e-2
    assert abs(d3) / abs(d4) >= 1.8


# ------------------------------------------------------------- threads
def test_thread_count_does_not_change_results(oracle_mod):
    """The loops over leaves run on OpenMP threads; each writes only its own
    leaf and budget partials are summed in leaf order, so one thread and
    several give the same bits: state, step lengths, budgets, flags and
    leaves over an adaptive run with inflow, clamping and regrids."""
    out = []
    for nt in (1, 4):
        oracle_mod.set_threads(nt)
        assert oracle_mod.threads() == nt
        sc = inputs.v_valley(level_max=3, m=16, min_level=1)
        o = oracle_mod.Oracle(sc, leaves=sc.uniform_leaves(sc.init_level))
        init_oracle(o, sc)
        dts = []
        flags = []
        for cycle in range(3):
            dts.append(o.advance(4, return_dt=True)[1])
            f = o.tag()
            flags.append(f)
            o.regrid(f)
        out.append((o.state(), np.concatenate(dts), o.mass(), np.concatenate(flags), o.leaves()))
    oracle_mod.set_threads(0)
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)
