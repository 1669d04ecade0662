"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module holds input recipes only (terrain nodes, initial conditions,
scenario parameters).  None of the method's arithmetic lives here: the
bathymetry pyramid, ghost filling, the Riemann solver and the update are
implemented separately by the library and by the CPU oracle.

Terrain: value noise with quintic smoothstep interpolation of lattice values,
lattice values drawn from SplitMix64(seed, octave, ix, iy) mapped to [-1, 1],
5 octaves, lacunarity 2, persistence 0.5, base wavelength L/4.  The paper
measures on real DEMs (the Malpasset CADAM terrain, Section 6) and on the
UK Environment Agency benchmark geometries (Section 5); seeded fractal
terrain of the same scale stands in for them here.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, List, Optional, Sequence, Tuple

import numpy as np

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def splitmix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser (Steele, Lea, Flood 2014) on uint64 arrays."""
    with np.errstate(over="ignore"):
        z = (x + np.uint64(0x9E3779B97F4A7C15)) & _M64
        z = ((z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)) & _M64
        z = ((z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)) & _M64
        return z ^ (z >> np.uint64(31))


def lattice_uniform(seed: int, octave: int, ix: np.ndarray, iy: np.ndarray) -> np.ndarray:
    """U[-1, 1] lattice value from SplitMix64 of (seed, octave, ix, iy)."""
    with np.errstate(over="ignore"):
        k = splitmix64(np.uint64(seed & 0xFFFFFFFFFFFFFFFF) * np.ones_like(ix, dtype=np.uint64))
        k = splitmix64(k ^ np.uint64(octave))
        k = splitmix64(k ^ ix.astype(np.int64).astype(np.uint64))
        k = splitmix64(k ^ iy.astype(np.int64).astype(np.uint64))
    # top 53 bits -> [0, 1)
    u = (k >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    return 2.0 * u - 1.0


def _quintic(t: np.ndarray) -> np.ndarray:
    return t * t * t * (t * (t * 6.0 - 15.0) + 10.0)


def value_noise(x: np.ndarray, y: np.ndarray, seed: int, octaves: int = 5,
                base_wavelength: float = 1.0, lacunarity: float = 2.0,
                persistence: float = 0.5) -> np.ndarray:
    """Fractal value noise at points (x, y); x, y broadcast together."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    if x.ndim == 2 and y.ndim == 2 and x.shape[0] == 1 and y.shape[1] == 1:
        return _value_noise_grid(x[0], y[:, 0], seed, octaves, base_wavelength, lacunarity, persistence)
    x, y = np.broadcast_arrays(x, y)
    out = np.zeros(x.shape, dtype=np.float64)
    amp = 1.0
    wl = base_wavelength
    for o in range(octaves):
        gx = x / wl
        gy = y / wl
        ix = np.floor(gx)
        iy = np.floor(gy)
        tx = _quintic(gx - ix)
        ty = _quintic(gy - iy)
        ix = ix.astype(np.int64)
        iy = iy.astype(np.int64)
        v00 = lattice_uniform(seed, o, ix, iy)
        v10 = lattice_uniform(seed, o, ix + 1, iy)
        v01 = lattice_uniform(seed, o, ix, iy + 1)
        v11 = lattice_uniform(seed, o, ix + 1, iy + 1)
        a = v00 + (v10 - v00) * tx
        b = v01 + (v11 - v01) * tx
        out += amp * (a + (b - a) * ty)
        amp *= persistence
        wl /= lacunarity
    return out


def _value_noise_grid(xr: np.ndarray, yc: np.ndarray, seed: int, octaves: int, base_wavelength: float,
                      lacunarity: float, persistence: float) -> np.ndarray:
    """value_noise on the grid (yc[j], xr[i]): the lattice values are drawn once
    per lattice point and gathered; every grid value is formed by the same
    operations as in value_noise, so the result is identical."""
    out = np.zeros((yc.shape[0], xr.shape[0]), dtype=np.float64)
    amp = 1.0
    wl = base_wavelength
    for o in range(octaves):
        gx = xr / wl
        gy = yc / wl
        ix = np.floor(gx)
        iy = np.floor(gy)
        tx = _quintic(gx - ix)[None, :]
        ty = _quintic(gy - iy)[:, None]
        ix = ix.astype(np.int64)
        iy = iy.astype(np.int64)
        i0, j0 = int(ix.min()), int(iy.min())
        li = np.arange(i0, int(ix.max()) + 2, dtype=np.int64)
        lj = np.arange(j0, int(iy.max()) + 2, dtype=np.int64)
        lat = lattice_uniform(seed, o, np.broadcast_to(li[None, :], (lj.shape[0], li.shape[0])),
                              np.broadcast_to(lj[:, None], (lj.shape[0], li.shape[0])))
        cx, cy = ix - i0, iy - j0
        v00 = lat[np.ix_(cy, cx)]
        v10 = lat[np.ix_(cy, cx + 1)]
        v01 = lat[np.ix_(cy + 1, cx)]
        v11 = lat[np.ix_(cy + 1, cx + 1)]
        a = v00 + (v10 - v00) * tx
        b = v01 + (v11 - v01) * tx
        out += amp * (a + (b - a) * ty)
        amp *= persistence
        wl /= lacunarity
    return out


def fractal_dem_nodes(nx_nodes: int, ny_nodes: int, lx: float, ly: float, seed: int,
                      base: float = 100.0, amp: float = 50.0, norm: str = "max") -> np.ndarray:
    """Terrain node values on an (ny_nodes, nx_nodes) lattice covering [0,lx]x[0,ly].

    norm="max": base + amp * r / max|r|;  norm="rms": base + amp * r / rms(r).
    Returned array is indexed [j][i] (y outer), float64.
    """
    xs = np.linspace(0.0, lx, nx_nodes)
    ys = np.linspace(0.0, ly, ny_nodes)
    L = max(lx, ly)
    r = value_noise(xs[None, :], ys[:, None], seed, base_wavelength=L / 4.0)
    if norm == "max":
        s = np.max(np.abs(r))
    else:
        s = math.sqrt(float(np.mean(r * r)))
    return np.ascontiguousarray(base + amp * r / s)


# ---------------------------------------------------------------------------
# Scenario descriptions (plain parameter records; both implementations read them)
# ---------------------------------------------------------------------------

BC_WALL, BC_EXTRAP, BC_INFLOW = 0, 1, 2


@dataclass
class Scenario:
    name: str
    x0: float
    y0: float
    x1: float
    y1: float
    mi: int
    mj: int
    m: int
    min_level: int
    max_level: int
    manning_n: float
    bc: Tuple[int, int, int, int] = (BC_WALL, BC_WALL, BC_WALL, BC_WALL)
    inflow_side: int = -1
    inflow_lo: float = 0.0
    inflow_hi: float = 0.0
    hydro: Optional[List[Tuple[float, float]]] = None
    tag_h_refine: float = 0.1
    tag_eta_refine: float = 0.05
    t_end: float = 1e300
    tag_u_refine: float = 0.0              # speed threshold [m/s] (0: off)
    tag_q_refine: float = 0.0              # velocity-depth product threshold [m^2/s] (0: off)
    regions: Optional[List[Tuple[float, float, float, float, int, int]]] = None  # x0 y0 x1 y1 min max
    grades: Optional[List[Tuple[int, float, int]]] = None                        # quantity threshold level
    dem: Optional[np.ndarray] = None       # node values [ny][nx] at level dem_level corners
    dem_level: int = 0
    init_level: int = 0
    eta_fn: Optional[Callable] = None      # (x, y, b) -> eta (free surface); h = max(eta - b, 0)
    uv_fn: Optional[Callable] = None       # (x, y, h) -> (hu, hv)

    def dx(self, level: int) -> float:
        return (self.x1 - self.x0) / (self.mi * self.m * (1 << level))

    def dy(self, level: int) -> float:
        return (self.y1 - self.y0) / (self.mj * self.m * (1 << level))

    def uniform_leaves(self, level: int) -> np.ndarray:
        """All patches of one level, as rows (tree, level, ix, iy), tree row-major,
        Morton (z) order within each tree (x is the low bit)."""
        n = 1 << level
        rows = []
        for tj in range(self.mj):
            for ti in range(self.mi):
                t = tj * self.mi + ti
                cells = [(morton2(ix, iy), ix, iy) for iy in range(n) for ix in range(n)]
                cells.sort()
                for _, ix, iy in cells:
                    rows.append((t, level, ix, iy))
        return np.asarray(rows, dtype=np.int32).reshape(-1, 4)

    def cell_centres(self, leaf: Sequence[int]) -> Tuple[np.ndarray, np.ndarray]:
        t, l, ix, iy = (int(v) for v in leaf)
        ti, tj = t % self.mi, t // self.mi
        dx, dy = self.dx(l), self.dy(l)
        PI = ti * (1 << l) + ix
        PJ = tj * (1 << l) + iy
        xc = self.x0 + (PI * self.m + np.arange(self.m) + 0.5) * dx
        yc = self.y0 + (PJ * self.m + np.arange(self.m) + 0.5) * dy
        return np.meshgrid(xc, yc)  # [j][i]


def morton2(ix: int, iy: int) -> int:
    """Z-order key with x in the low bit."""
    k = 0
    for b in range(31):
        k |= ((ix >> b) & 1) << (2 * b)
        k |= ((iy >> b) & 1) << (2 * b + 1)
    return k


def initial_state(sc: Scenario, leaf, b: np.ndarray, precision: str = "f64"):
    """Initial (h, hu, hv) on one leaf from the scenario's free-surface recipe.

    b is the cell bathymetry the implementation under test uses for that leaf
    (interior, [j][i]).  For precision "f32" the state is formed in float32
    from float32 b: h = max(eta32 - b32, 0), so that h + b == eta exactly
    wherever eta lies in [b, 2b] (Sterbenz).
    """
    X, Y = sc.cell_centres(leaf)
    eta = sc.eta_fn(X, Y, b)
    if precision == "f32":
        b32 = np.asarray(b, dtype=np.float32)
        e32 = np.asarray(eta, dtype=np.float32)
        h = np.maximum(e32 - b32, np.float32(0.0)).astype(np.float32)
        if sc.uv_fn is not None:
            hu, hv = sc.uv_fn(X, Y, h.astype(np.float64))
            hu = np.asarray(hu, dtype=np.float32)
            hv = np.asarray(hv, dtype=np.float32)
        else:
            hu = np.zeros_like(h)
            hv = np.zeros_like(h)
        return h, hu, hv
    h = np.maximum(eta - b, 0.0)
    if sc.uv_fn is not None:
        hu, hv = sc.uv_fn(X, Y, h)
    else:
        hu = np.zeros_like(h)
        hv = np.zeros_like(h)
    return h, np.asarray(hu, dtype=np.float64), np.asarray(hv, dtype=np.float64)


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

def ritter_dambreak(n_cells: int = 128, m: int = 16, h0: float = 10.0) -> Scenario:
    """Dry-bed dam break in a 2000 m box: h0 left of x = 1000 m, dry right,
    flat bed, no friction, walls, run to t = 50 s."""
    level = int(round(math.log2(n_cells // m)))
    assert (m << level) == n_cells
    sc = Scenario(name=f"ritter{n_cells}", x0=0.0, y0=0.0, x1=2000.0, y1=2000.0,
                  mi=1, mj=1, m=m, min_level=level, max_level=level, manning_n=0.0,
                  t_end=50.0, init_level=level)
    sc.dem = np.zeros((m + 1, m + 1))
    sc.dem_level = 0
    sc.eta_fn = lambda X, Y, b: np.where(X < 1000.0, h0, 0.0) + 0.0 * b
    return sc


def reservoir_fractal(level: int = 6, m: int = 32, seed: int = 2, radius: float = 400.0,
                      h_res: float = 20.0, L: float = 10000.0, manning_n: float = 0.033,
                      dem_level: Optional[int] = None, centre: Optional[Tuple[float, float]] = None) -> Scenario:
    """Square L x L domain, uniform level, fractal terrain 100 +/- 50 m, a
    circular reservoir of depth h_res (h = 20 m for r <= radius, else dry)
    centred at `centre` (default: the domain centre)."""
    if dem_level is None:
        dem_level = level
    sc = Scenario(name=f"reservoir_l{level}_m{m}", x0=0.0, y0=0.0, x1=L, y1=L, mi=1, mj=1, m=m,
                  min_level=level, max_level=level, manning_n=manning_n, init_level=level)
    nn = m * (1 << dem_level) + 1
    sc.dem = fractal_dem_nodes(nn, nn, L, L, seed, base=100.0, amp=50.0, norm="max")
    sc.dem_level = dem_level
    cx, cy = (0.5 * L, 0.5 * L) if centre is None else centre

    def eta(X, Y, b):
        r = np.hypot(X - cx, Y - cy)
        return np.where(r <= radius, b + h_res, -1e9)
    sc.eta_fn = eta
    return sc


def adaptive_reservoir(seed: int, L: float = 4000.0, m: int = 16, max_level: int = 3, dem_level: int = 3,
                       radius: float = 250.0) -> Scenario:
    """The reservoir on AMR levels 0..max_level with its centre drawn from
    U[L/4, 3L/4]^2 by the seed (the learned-tagger workload, scaled)."""
    rng = np.random.default_rng(seed)
    c = (float(rng.uniform(0.25 * L, 0.75 * L)), float(rng.uniform(0.25 * L, 0.75 * L)))
    sc = reservoir_fractal(level=max_level, m=m, L=L, seed=seed, radius=radius, dem_level=dem_level, centre=c)
    sc.name = f"adaptive_reservoir_{seed}"
    sc.min_level, sc.max_level, sc.init_level = 0, max_level, 1
    return sc


def wet_dambreak(level: int = 6, m: int = 32, seed: int = 2, radius: float = 400.0,
                 eta0: float = 155.0, eta1: float = 165.0, L: float = 10000.0,
                 manning_n: float = 0.033) -> Scenario:
    """The reservoir terrain (100 +/- 50 m) under a lake at eta0 = 155 m, so
    every cell is wet, with a column raised to eta1 within `radius` of the
    centre: a dam break on fully wet terrain."""
    sc = Scenario(name=f"wet_dambreak_l{level}_m{m}", x0=0.0, y0=0.0, x1=L, y1=L, mi=1, mj=1, m=m,
                  min_level=level, max_level=level, manning_n=manning_n, init_level=level)
    nn = m * (1 << level) + 1
    sc.dem = fractal_dem_nodes(nn, nn, L, L, seed, base=100.0, amp=50.0, norm="max")
    sc.dem_level = level
    cx = cy = 0.5 * L

    def eta(X, Y, b):
        r = np.hypot(X - cx, Y - cy)
        return np.where(r <= radius, eta1, eta0) + 0.0 * b
    sc.eta_fn = eta
    return sc


def lake_at_rest(level: int = 3, m: int = 16, seed: int = 7, eta0: float = 110.0,
                 L: float = 2000.0) -> Scenario:
    """Fractal terrain 100 +/- 50 m with a flat free surface eta0: dry islands
    where b > eta0.  Used for the well-balancing invariant."""
    sc = Scenario(name="lake", x0=0.0, y0=0.0, x1=L, y1=L, mi=1, mj=1, m=m,
                  min_level=level, max_level=level, manning_n=0.033, init_level=level)
    nn = m * (1 << level) + 1
    sc.dem = fractal_dem_nodes(nn, nn, L, L, seed)
    sc.dem_level = level
    sc.eta_fn = lambda X, Y, b: np.full_like(b, eta0)
    return sc


def trapezoid_hydrograph(q_peak: float, t_rise: float, t_plateau: float, t_fall: float):
    return [(0.0, 0.0), (t_rise, q_peak), (t_rise + t_plateau, q_peak),
            (t_rise + t_plateau + t_fall, 0.0)]


def v_valley(level_max: int = 6, m: int = 32, seed: int = 3, min_level: int = 0,
             dem_level: int = 4, q_peak: float = 5000.0, manning_n: float = 0.04,
             mi: int = 16, mj: int = 8, lx: float = 20000.0, ly: float = 10000.0,
             init_level: Optional[int] = None) -> Scenario:
    """V-shaped valley: b = 100 + 1e-3 (lx - x) + 0.05 |y - ly/2| + r(x, y) with
    r fractal at 2 m rms; inflow over |y - ly/2| <= 100 m at x = 0 following a
    trapezoid hydrograph that reaches q_peak; outflow (extrapolation) at x = lx;
    walls elsewhere.  Initial state: a normal-depth flood along the axis."""
    sc = Scenario(name="v_valley", x0=0.0, y0=0.0, x1=lx, y1=ly, mi=mi, mj=mj, m=m,
                  min_level=min_level, max_level=level_max, manning_n=manning_n,
                  bc=(BC_INFLOW, BC_EXTRAP, BC_WALL, BC_WALL), inflow_side=0,
                  inflow_lo=ly / 2 - 100.0, inflow_hi=ly / 2 + 100.0,
                  hydro=trapezoid_hydrograph(q_peak, 3600.0, 10800.0, 3600.0),
                  init_level=min_level if init_level is None else init_level)
    nx = mi * m * (1 << dem_level) + 1
    ny = mj * m * (1 << dem_level) + 1
    xs = np.linspace(0.0, lx, nx)
    ys = np.linspace(0.0, ly, ny)
    r = value_noise(xs[None, :], ys[:, None], seed, base_wavelength=max(lx, ly) / 4.0)
    r = 2.0 * r / math.sqrt(float(np.mean(r * r)))
    sc.dem = np.ascontiguousarray(100.0 + 1e-3 * (lx - xs[None, :]) + 0.05 * np.abs(ys[:, None] - ly / 2) + r)
    sc.dem_level = dem_level
    # normal depth for Q in a V channel of side slope 0.05: A = 20 d^2, R ~ d/2
    S0 = 1e-3
    d_n = (q_peak * manning_n / (20.0 * math.sqrt(S0)) * 2.0 ** (2.0 / 3.0)) ** (3.0 / 8.0)
    u_n = q_peak / (20.0 * d_n * d_n)

    def eta(X, Y, b):
        return 100.0 + 1e-3 * (lx - X) + d_n + 0.0 * b

    def uv(X, Y, h):
        return h * u_n, np.zeros_like(h)
    sc.eta_fn = eta
    sc.uv_fn = uv
    return sc


def flood_speed(level_max: int = 3, m: int = 32, min_level: int = 0, mi: int = 6, mj: int = 12,
                q_peak: float = 20.0, manning_n: float = 0.03, tag_h: float = 0.05) -> Scenario:
    """Speed of flood propagation over an extended floodplain: flat bed at 0 m,
    x in [0, 1000] m, y in [0, 2000] m, dry start; inflow over 990 <= y <= 1010
    at x = 0 following a trapezoid hydrograph 0 -> q_peak m^3/s (60 min rise,
    180 min plateau, 60 min fall), walls elsewhere; n = manning_n; run to 6 h.
    Level-0 cells are 1000 / (mi m) m wide (5.2 m for 6 x 12 trees of 32^2:
    a 5 m grid has 200 cells across, which no power-of-two patch divides).
    Tagging: depth above tag_h, and a flood-source region over the inlet held
    at the finest level."""
    lx, ly = 1000.0, 2000.0
    sc = Scenario(name="flood_speed", x0=0.0, y0=0.0, x1=lx, y1=ly, mi=mi, mj=mj, m=m,
                  min_level=min_level, max_level=level_max, manning_n=manning_n,
                  bc=(BC_INFLOW, BC_WALL, BC_WALL, BC_WALL), inflow_side=0, inflow_lo=990.0, inflow_hi=1010.0,
                  hydro=trapezoid_hydrograph(q_peak, 3600.0, 10800.0, 3600.0), tag_h_refine=tag_h,
                  t_end=6 * 3600.0, init_level=min_level,
                  regions=[(0.0, 980.0, 20.0, 1020.0, level_max, level_max)])
    sc.dem = np.zeros((mj * m + 1, mi * m + 1))
    sc.dem_level = 0

    def eta(X, Y, b):
        return b - 1.0
    sc.eta_fn = eta
    return sc


def ensemble_dambreaks(n_scen: int = 256, master_seed: int = 4000, m: int = 32,
                       dx: float = 10.0, sizes=(64, 128, 256, 512)) -> List[Scenario]:
    """Independent dam-break scenarios: N_k ~ U{sizes}, L = dx N_k, fractal
    terrain 100 +/- 50 (L / 10 km) m, a 2-cell dam strip at x in [L/3, L/3+20)
    raised by 50 m except a breach |y - L/2| <= w/2, w ~ U[50, 500] m (clipped
    to 0.8 L); reservoir x < L/3 at eta0 = median(upstream b) + 20 m; dry
    downstream; n ~ U[0.02, 0.06]; walls."""
    out = []
    for k in range(n_scen):
        rng = np.random.default_rng(master_seed + k)
        N = int(rng.choice(np.asarray(sizes)))
        L = dx * N
        w = min(float(rng.uniform(50.0, 500.0)), 0.8 * L)
        n_man = float(rng.uniform(0.02, 0.06))
        level = int(round(math.log2(N // m)))
        sc = Scenario(name=f"ens{k}", x0=0.0, y0=0.0, x1=L, y1=L, mi=1, mj=1, m=m,
                      min_level=level, max_level=level, manning_n=n_man, init_level=level)
        nn = N + 1
        xs = np.linspace(0.0, L, nn)
        ys = np.linspace(0.0, L, nn)
        dem = fractal_dem_nodes(nn, nn, L, L, master_seed + k, base=100.0, amp=50.0 * (L / 10000.0))
        xd0 = L / 3.0
        strip = (xs[None, :] >= xd0) & (xs[None, :] < xd0 + 2 * dx)
        breach = np.abs(ys[:, None] - L / 2) <= w / 2
        dem = dem + np.where(strip & ~breach, 50.0, 0.0)
        sc.dem = np.ascontiguousarray(dem)
        sc.dem_level = level
        up = dem[:, xs < xd0]
        eta0 = float(np.median(up)) + 20.0

        def eta(X, Y, b, eta0=eta0, xd0=xd0):
            return np.where(X < xd0, eta0, -1e9) + 0.0 * b
        sc.eta_fn = eta
        out.append(sc)
    return out


# ---------------------------------------------------------------------------
# Learned tagger: initial weights (drawn here once, passed to both sides)
# ---------------------------------------------------------------------------
CNN_PARAM_SHAPES = [("W1", (16, 3, 3, 4)), ("b1", (16,)), ("W2", (32, 3, 3, 16)), ("b2", (32,)),
                    ("W3", (32, 3, 3, 32)), ("b3", (32,)), ("Wf", (3, 32)), ("bf", (3,))]


def cnn_init_params(seed: int = 0) -> np.ndarray:
    """He-normal initial weights (std sqrt(2 / fan_in)), zero biases, as one
    float32-representable vector in the layout W1, b1, W2, b2, W3, b3, Wf, bf."""
    rng = np.random.default_rng(seed)
    parts = []
    for name, shape in CNN_PARAM_SHAPES:
        if name.startswith("W"):
            fan_in = int(np.prod(shape[1:]))
            parts.append(rng.standard_normal(int(np.prod(shape))) * math.sqrt(2.0 / fan_in))
        else:
            parts.append(np.zeros(int(np.prod(shape))))
    return np.concatenate(parts).astype(np.float32).astype(np.float64)
