"""Shared test helpers: scenario builders and global-array assembly."""
import numpy as np

from paper_2403_15435_amd import inputs


def row_scenario(n_cells, hL, uL, hR, uR, length=1000.0, m=16, t_end=1e300):
    """One row of patches (y-invariant problem) with a jump at the middle."""
    mi = n_cells // m
    dx = length / n_cells
    sc = inputs.Scenario(name="row", x0=0.0, y0=0.0, x1=length, y1=m * dx, mi=mi, mj=1, m=m,
                         min_level=0, max_level=0, manning_n=0.0, t_end=t_end, init_level=0)
    sc.dem = np.zeros((m + 1, mi * m + 1))
    sc.dem_level = 0
    x0 = 0.5 * length
    sc.eta_fn = lambda X, Y, b: np.where(X < x0, hL, hR) + 0.0 * b
    sc.uv_fn = lambda X, Y, h: (np.where(X < x0, hL * uL, hR * uR) + 0.0 * h, 0.0 * h)
    return sc


def assemble(sc, leaves, st, field, level=None):
    """Global array [J][I] of one field for a uniform mesh (all leaves on one level)."""
    lv = np.asarray(leaves)
    if level is None:
        level = int(lv[0, 1])
    m = sc.m
    NI = sc.mi * m << level
    NJ = sc.mj * m << level
    out = np.zeros((NJ, NI), dtype=st.dtype)
    for k, (t, l, ix, iy) in enumerate(lv):
        assert l == level
        PI = (t % sc.mi) * (1 << l) + ix
        PJ = (t // sc.mi) * (1 << l) + iy
        out[PJ * m:(PJ + 1) * m, PI * m:(PI + 1) * m] = st[k, field]
    return out


def to_finest(sc, leaves, st, field, level):
    """Piecewise-constant projection of an AMR field onto a uniform level."""
    lv = np.asarray(leaves)
    m = sc.m
    NI = sc.mi * m << level
    NJ = sc.mj * m << level
    out = np.zeros((NJ, NI))
    for k, (t, l, ix, iy) in enumerate(lv):
        r = 1 << (level - l)
        PI = (t % sc.mi) * (1 << l) + ix
        PJ = (t // sc.mi) * (1 << l) + iy
        blk = np.kron(st[k, field], np.ones((r, r)))
        out[PJ * m * r:(PJ + 1) * m * r, PI * m * r:(PI + 1) * m * r] = blk
    return out


def init_oracle(o, sc, precision="f64"):
    """Initial state from the scenario recipe on every oracle leaf, formed from
    the oracle's own bathymetry."""
    from paper_2403_15435_amd.inputs import initial_state
    lv = o.leaves()
    for k in range(lv.shape[0]):
        b = o.get_field(k, 3)
        h, hu, hv = initial_state(sc, lv[k], b, precision)
        o.set_field(k, 0, np.asarray(h, dtype=np.float64))
        o.set_field(k, 1, np.asarray(hu, dtype=np.float64))
        o.set_field(k, 2, np.asarray(hv, dtype=np.float64))


def _dilate(mask, r):
    pad = np.pad(mask, r, mode="edge")
    out = np.zeros_like(mask)
    for dj in range(2 * r + 1):
        for di in range(2 * r + 1):
            out |= pad[dj:dj + mask.shape[0], di:di + mask.shape[1]]
    return out


def check_fp32(sc, leaves, g, o, level):
    """Max relative h error away from fronts and max absolute error at front
    cells, on the mesh projected to `level`.  A cell is at a front when a cell
    of depth <= 1e-2 m (in either solution) lies within 2 cells of the cell's
    own level (a 5x5 neighbourhood on a uniform mesh)."""
    Ho = to_finest(sc, leaves, o, 0, level)
    Hg = to_finest(sc, leaves, g, 0, level)
    shallow = (Ho <= 1e-2) | (Hg <= 1e-2)
    lvl = np.full(Ho.shape, level)
    m = sc.m
    for t, l, ix, iy in np.asarray(leaves):
        rr = 1 << (level - l)
        PI = (t % sc.mi) * (1 << l) + ix
        PJ = (t // sc.mi) * (1 << l) + iy
        lvl[PJ * m * rr:(PJ + 1) * m * rr, PI * m * rr:(PI + 1) * m * rr] = l
    near = np.zeros_like(shallow)
    for l in np.unique(lvl):
        near |= _dilate(shallow, 2 << (level - l)) & (lvl == l)
    away = ~near
    rel = np.abs(Hg - Ho)[away] / Ho[away] if away.any() else np.zeros(1)
    front = np.abs(Hg - Ho)[near] if near.any() else np.zeros(1)
    return float(rel.max()), float(front.max())


def oracle_refine_passes(o, sc, passes, precision="f64"):
    """The oracle's counterpart of gf_set_initial with refinement passes: the
    recipe on every leaf, then up to `passes` rounds of plain tagging,
    regridding and the recipe again (stopping when nothing is flagged)."""
    init_oracle(o, sc, precision)
    for _ in range(passes):
        f = o.tag()
        if not f.any():
            break
        o.regrid(f)
        init_oracle(o, sc, precision)


def _dilate_sep(mask, r):
    """Chebyshev dilation by r cells, as a row pass then a column pass."""
    out = mask.copy()
    for d in range(1, r + 1):
        out[:, d:] |= mask[:, :-d]
        out[:, :-d] |= mask[:, d:]
    tmp = out.copy()
    for d in range(1, r + 1):
        out[d:, :] |= tmp[:-d, :]
        out[:-d, :] |= tmp[d:, :]
    return out


def check_fp32_large(sc, leaves, g, o, finest):
    """check_fp32 for meshes too large to project onto the finest level with
    per-level dilations: the same bar and front rule (a cell is at a front
    when a cell of depth <= 1e-2 m in either solution lies within 2 cells of
    the cell's own level), with a finer cell counted at a coarser level
    through its parent (any shallow child makes the parent shallow: at least
    as many front cells as the exact rule).  Returns (max relative h error
    away from fronts, max absolute error at fronts, cells away, cells at
    fronts)."""
    lv = np.asarray(leaves)
    m = sc.m
    L = int(finest)
    S = np.zeros((sc.mj * m << L, sc.mi * m << L), dtype=bool)

    def origin(t, l, ix, iy):
        return (t // sc.mi) * (1 << l) + iy, (t % sc.mi) * (1 << l) + ix
    for k, (t, l, ix, iy) in enumerate(lv):
        sh = (o[k, 0] <= 1e-2) | (g[k, 0] <= 1e-2)
        if not sh.any():
            continue
        PJ, PI = origin(t, l, ix, iy)
        r = 1 << (L - l)
        S[PJ * m * r:(PJ + 1) * m * r, PI * m * r:(PI + 1) * m * r] = np.repeat(np.repeat(sh, r, 0), r, 1)
    near = {}
    levels = sorted(set(int(l) for l in lv[:, 1]), reverse=True)
    cur, cl = S, L
    for l in range(L, min(levels) - 1, -1):
        if l < cl:
            cur = cur.reshape(cur.shape[0] // 2, 2, cur.shape[1] // 2, 2).any(axis=(1, 3))
            cl = l
        if l in levels:
            near[l] = _dilate_sep(cur, 2)
    rel, front, n_away, n_front = 0.0, 0.0, 0, 0
    for k, (t, l, ix, iy) in enumerate(lv):
        PJ, PI = origin(t, l, ix, iy)
        nm = near[int(l)][PJ * m:(PJ + 1) * m, PI * m:(PI + 1) * m]
        d = np.abs(g[k, 0] - o[k, 0])
        if (~nm).any():
            rel = max(rel, float((d[~nm] / o[k, 0][~nm]).max()))
            n_away += int((~nm).sum())
        if nm.any():
            front = max(front, float(d[nm].max()))
            n_front += int(nm.sum())
    return rel, front, n_away, n_front
