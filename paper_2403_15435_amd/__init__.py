"""MI355X shallow-water patch library (GeoFlood method) -- Python binding.

Thin ctypes marshalling over the C ABI declared in include/geoflood.h; every
step of the computation runs in the HIP library libgeoflood.so.  Importing
this package fails loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgeoflood.so")

GF_OK, GF_E_INVALID, GF_E_NOMEM, GF_E_HIP, GF_E_STATE, GF_E_CFL, GF_E_NUMERIC, GF_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5, -6, -7
GF_FP64, GF_FP32 = 0, 1
_ERRNAME = {-1: "GF_E_INVALID", -2: "GF_E_NOMEM", -3: "GF_E_HIP", -4: "GF_E_STATE", -5: "GF_E_CFL",
            -6: "GF_E_NUMERIC", -7: "GF_E_UNSUPPORTED"}


class gf_scenario_desc(C.Structure):
    _fields_ = [("x0", C.c_double), ("y0", C.c_double), ("x1", C.c_double), ("y1", C.c_double),
                ("mi", C.c_int32), ("mj", C.c_int32), ("min_level", C.c_int32), ("max_level", C.c_int32),
                ("manning_n", C.c_double), ("bc", C.c_int32 * 4), ("inflow_side", C.c_int32),
                ("inflow_lo", C.c_double), ("inflow_hi", C.c_double), ("hydro", C.POINTER(C.c_double)),
                ("n_hydro", C.c_int32), ("tag_h_refine", C.c_double), ("tag_eta_refine", C.c_double),
                ("t_end", C.c_double), ("tag_u_refine", C.c_double), ("tag_q_refine", C.c_double),
                ("n_regions", C.c_int32), ("regions", C.POINTER(C.c_double)),
                ("n_grades", C.c_int32), ("grades", C.POINTER(C.c_double))]


class gf_config(C.Structure):
    _fields_ = [("precision", C.c_int32), ("m", C.c_int32), ("g", C.c_double), ("dry_tol", C.c_double),
                ("cfl_desired", C.c_double), ("cfl_max", C.c_double), ("n_scen", C.c_int32),
                ("scen", C.POINTER(gf_scenario_desc)), ("max_patches", C.c_int64), ("hip_stream", C.c_void_p),
                ("autotune_cache", C.c_char_p), ("limiter", C.c_int32), ("transverse", C.c_int32)]


class gf_step_stats(C.Structure):
    _fields_ = [("steps", C.c_int64), ("rejected", C.c_int64), ("cell_updates", C.c_int64),
                ("t_min", C.c_double), ("t_max", C.c_double), ("dt_min", C.c_double), ("dt_max", C.c_double),
                ("cfl_max", C.c_double), ("seconds", C.c_double)]


class gf_run_stats(C.Structure):
    _fields_ = [("steps", C.c_int64), ("regrids", C.c_int64), ("forced_regrids", C.c_int64), ("checks", C.c_int64),
                ("misses", C.c_int64), ("leaf_steps", C.c_int64), ("seconds", C.c_double)]


GF_RUN_PLAIN, GF_RUN_SPARSE, GF_RUN_LEARNED = 0, 1, 2
GF_TAG_PLAIN, GF_TAG_LEARNED = 0, 1
GF_LIMITER_MC, GF_LIMITER_MINMOD, GF_LIMITER_SUPERBEE, GF_LIMITER_VANLEER, GF_LIMITER_NONE = 0, 1, 2, 3, 4
GF_TRANSVERSE_CORRECTED, GF_TRANSVERSE_NONE = 0, 1

# void ic(user, scen, level, x0, y0, dx, dy, nx, ny, const double *b, double *h, double *hu, double *hv)
GF_IC_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_int32, C.c_int32, C.c_double, C.c_double, C.c_double, C.c_double,
                       C.c_int32, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double),
                       C.POINTER(C.c_double))
NET_PARAMS = 14579
NET_FEATURES = 2304

EXPORTS = ["gf_create", "gf_destroy", "gf_set_bathymetry", "gf_set_initial", "gf_set_leaves", "gf_get_leaves", "gf_set_patch",
           "gf_get_patch", "gf_set_state", "gf_get_state", "gf_fill_ghosts", "gf_get_ghosted", "gf_step", "gf_step_plain", "gf_step_lts",
           "gf_tag", "gf_regrid", "gf_set_gauges", "gf_get_gauges", "gf_mass", "gf_mass_static", "gf_time", "gf_set_time", "gf_set_step_threads",
           "gf_get_step_threads", "gf_set_step_pad", "gf_set_schedule", "gf_autotune", "gf_autotune_trials", "gf_profile_enable", "gf_profile_read", "gf_profile_kernel", "gf_probe_triad", "gf_profile_patches", "gf_net_set_params", "gf_net_get_params", "gf_net_features",
           "gf_net_forward", "gf_net_train_step", "gf_net_train_step_dev", "gf_net_predict", "gf_net_collect", "gf_run", "gf_last_error", "gf_version"]

_lib = None


def load(path: str = LIB_PATH):
    """Load libgeoflood.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with paper_2403_15435_amd.build.build()")
    # Load torch first: it maps its own HIP runtime, and the library then binds
    # to that same runtime (one runtime per process, shared streams).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(path)
    vp, i32, i64, dp = C.c_void_p, C.c_int32, C.c_int64, C.POINTER(C.c_double)
    L.gf_create.argtypes = [C.POINTER(gf_config), C.POINTER(vp)]
    L.gf_destroy.argtypes = [vp]
    L.gf_destroy.restype = None
    L.gf_set_bathymetry.argtypes = [vp, i32, dp, i64, i64, i32]
    L.gf_set_leaves.argtypes = [vp, i32, C.POINTER(i32), i64]
    L.gf_set_gauges.argtypes = [vp, i32, C.POINTER(i32), dp, i64]
    L.gf_get_gauges.argtypes = [vp, i32, dp, i64, C.POINTER(i64)]
    L.gf_get_leaves.argtypes = [vp, i32, C.POINTER(i32), i64, C.POINTER(i64)]
    L.gf_set_patch.argtypes = [vp, i32, i64, i32, dp]
    L.gf_get_patch.argtypes = [vp, i32, i64, i32, dp]
    L.gf_set_state.argtypes = [vp, i32, dp]
    L.gf_get_state.argtypes = [vp, i32, dp]
    L.gf_fill_ghosts.argtypes = [vp]
    L.gf_get_ghosted.argtypes = [vp, i32, i64, i32, dp]
    L.gf_step.argtypes = [vp, i32, dp, C.POINTER(gf_step_stats)]
    L.gf_step_plain.argtypes = [vp, i32, dp, C.POINTER(gf_step_stats)]
    L.gf_step_lts.argtypes = [vp, i32, dp, C.POINTER(gf_step_stats)]
    L.gf_tag.argtypes = [vp, i32, C.POINTER(C.c_int8), i64, C.POINTER(i64)]
    L.gf_set_initial.argtypes = [vp, i32, GF_IC_FN, vp, i32]
    L.gf_regrid.argtypes = [vp, C.POINTER(C.c_int8), C.POINTER(i64)]
    L.gf_mass.argtypes = [vp, i32, dp, dp, dp]
    L.gf_mass_static.argtypes = [vp, i32, dp, dp, dp]
    L.gf_time.argtypes = [vp, i32, dp, dp, C.POINTER(i64), C.POINTER(i64)]
    L.gf_set_time.argtypes = [vp, i32, C.c_double, C.c_double]
    L.gf_set_step_threads.argtypes = [vp, i32]
    L.gf_get_step_threads.argtypes = [vp, C.POINTER(i32)]
    L.gf_set_schedule.argtypes = [vp, i32]
    L.gf_autotune.argtypes = [vp, i32, C.c_char_p, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32), dp]
    L.gf_autotune_trials.argtypes = [vp, C.POINTER(i32), dp, i64, C.POINTER(i64)]
    L.gf_set_step_pad.argtypes = [vp, i32]
    L.gf_profile_enable.argtypes = [vp, i32]
    L.gf_profile_read.argtypes = [vp, C.POINTER(i64), dp]
    L.gf_profile_kernel.argtypes = [vp, C.POINTER(i64), dp]
    L.gf_probe_triad.argtypes = [vp, vp, vp, i64, C.c_float, vp]
    L.gf_profile_patches.argtypes = [vp, C.POINTER(i64), C.POINTER(i64)]
    i8p = C.POINTER(C.c_int8)
    L.gf_net_set_params.argtypes = [vp, dp, i64]
    L.gf_net_get_params.argtypes = [vp, dp, i64]
    L.gf_net_features.argtypes = [vp, dp, i64, C.POINTER(i64)]
    L.gf_net_forward.argtypes = [vp, dp, i32, dp]
    L.gf_net_train_step.argtypes = [vp, dp, i8p, i32, dp, C.c_double, dp, dp]
    L.gf_net_train_step_dev.argtypes = [vp, vp, vp, i32, dp, C.c_double, dp]
    L.gf_net_predict.argtypes = [vp, i8p, i64, C.POINTER(i64)]
    L.gf_net_collect.argtypes = [vp, i32, i32, dp, i8p, i64, C.POINTER(i64)]
    L.gf_run.argtypes = [vp, i32, i32, i32, i32, C.POINTER(gf_run_stats)]
    L.gf_last_error.argtypes = [vp]
    L.gf_last_error.restype = C.c_char_p
    L.gf_version.restype = C.c_char_p
    for name in EXPORTS:
        if name not in ("gf_destroy", "gf_last_error", "gf_version"):
            getattr(L, name).restype = C.c_int
    _lib = L
    return L


def probe_triad(a, b, c, s: float = 3.0, stream=None):
    """One launch of the library's HBM triad probe on torch float32 tensors
    (c = a + s b), on `stream` (default: torch's current stream)."""
    n = a.numel()
    if not (b.numel() == n and c.numel() == n):
        raise ValueError("a, b, c need the same size")
    L = load()
    h = stream if stream is not None else _stream_handle()
    rc = L.gf_probe_triad(C.c_void_p(a.data_ptr()), C.c_void_p(b.data_ptr()), C.c_void_p(c.data_ptr()), n, s, h)
    if rc != 0:
        raise GFError(rc, "triad probe launch failed")


class GFError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_ERRNAME.get(code, code)}: {msg}")
        self.code = code


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _stream_handle():
    try:
        import torch
        if torch.cuda.is_available():
            return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    except Exception:
        pass
    return C.c_void_p(None)


class Context:
    """A library context over one or more scenarios (inputs.Scenario objects)."""

    def __init__(self, scenarios: Sequence, precision: int = GF_FP64, max_patches: Optional[int] = None,
                 g: float = 9.81, dry_tol: float = 1e-4, cfl_desired: float = 0.9, cfl_max: float = 1.0,
                 stream=None, autotune_cache: Optional[str] = None, limiter: int = GF_LIMITER_MC,
                 transverse: int = GF_TRANSVERSE_CORRECTED):
        L = load()
        self.L = L
        self.scenarios = list(scenarios)
        self.m = self.scenarios[0].m
        self.precision = precision
        self._hydro = []
        descs = (gf_scenario_desc * len(self.scenarios))()
        for k, sc in enumerate(self.scenarios):
            d = descs[k]
            d.x0, d.y0, d.x1, d.y1 = sc.x0, sc.y0, sc.x1, sc.y1
            d.mi, d.mj, d.min_level, d.max_level = sc.mi, sc.mj, sc.min_level, sc.max_level
            d.manning_n = sc.manning_n
            for s in range(4):
                d.bc[s] = sc.bc[s]
            d.inflow_side, d.inflow_lo, d.inflow_hi = sc.inflow_side, sc.inflow_lo, sc.inflow_hi
            hy = np.ascontiguousarray(np.asarray(sc.hydro if sc.hydro else [(0.0, 0.0)], dtype=np.float64).reshape(-1))
            self._hydro.append(hy)
            d.hydro = _dptr(hy)
            d.n_hydro = len(sc.hydro) if sc.hydro else 0
            d.tag_h_refine, d.tag_eta_refine = sc.tag_h_refine, sc.tag_eta_refine
            d.t_end = sc.t_end
            d.tag_u_refine, d.tag_q_refine = sc.tag_u_refine, sc.tag_q_refine
            rg = np.ascontiguousarray(np.asarray(sc.regions if sc.regions else [(0.0,) * 6], dtype=np.float64).reshape(-1))
            gr = np.ascontiguousarray(np.asarray(sc.grades if sc.grades else [(0.0,) * 3], dtype=np.float64).reshape(-1))
            self._hydro += [rg, gr]
            d.n_regions, d.regions = (len(sc.regions) if sc.regions else 0), _dptr(rg)
            d.n_grades, d.grades = (len(sc.grades) if sc.grades else 0), _dptr(gr)
        if max_patches is None:
            max_patches = 0
            for sc in self.scenarios:
                max_patches += sc.mi * sc.mj * 4 ** sc.max_level
            max_patches = int(min(max_patches, 200000))
        cfg = gf_config(precision=precision, m=self.m, g=g, dry_tol=dry_tol, cfl_desired=cfl_desired,
                        cfl_max=cfl_max, n_scen=len(self.scenarios), scen=descs, max_patches=max_patches,
                        hip_stream=stream if stream is not None else _stream_handle(),
                        autotune_cache=autotune_cache.encode() if autotune_cache else None,
                        limiter=limiter, transverse=transverse)
        self._p = C.c_void_p()
        rc = L.gf_create(C.byref(cfg), C.byref(self._p))
        if rc != 0:
            raise GFError(rc, "gf_create failed: " + L.gf_last_error(None).decode())
        for k, sc in enumerate(self.scenarios):
            if sc.dem is not None:
                self.set_bathymetry(k, sc.dem, sc.dem_level)
                self.set_leaves(k, sc.uniform_leaves(sc.init_level))

    def _chk(self, rc: int):
        if rc != 0:
            raise GFError(rc, self.L.gf_last_error(self._p).decode())

    def close(self):
        if getattr(self, "_p", None):
            self.L.gf_destroy(self._p)
            self._p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- ABI
    def set_bathymetry(self, scen: int, dem: np.ndarray, dem_level: int):
        a = np.ascontiguousarray(dem, dtype=np.float64)
        self._chk(self.L.gf_set_bathymetry(self._p, scen, _dptr(a), a.shape[1], a.shape[0], dem_level))

    def set_leaves(self, scen: int, leaves: np.ndarray):
        a = np.ascontiguousarray(np.asarray(leaves, dtype=np.int32).reshape(-1, 4))
        self._chk(self.L.gf_set_leaves(self._p, scen, a.ctypes.data_as(C.POINTER(C.c_int32)), a.shape[0]))

    def leaves(self, scen: int = 0) -> np.ndarray:
        n = C.c_int64()
        self._chk(self.L.gf_get_leaves(self._p, scen, None, 0, C.byref(n)))
        out = np.zeros((n.value, 4), dtype=np.int32)
        self._chk(self.L.gf_get_leaves(self._p, scen, out.ctypes.data_as(C.POINTER(C.c_int32)), n.value, C.byref(n)))
        return out

    def set_patch(self, scen: int, leaf: int, field: int, a: np.ndarray):
        a = np.ascontiguousarray(a, dtype=np.float64)
        self._chk(self.L.gf_set_patch(self._p, scen, leaf, field, _dptr(a)))

    def get_patch(self, scen: int, leaf: int, field: int) -> np.ndarray:
        out = np.zeros((self.m, self.m))
        self._chk(self.L.gf_get_patch(self._p, scen, leaf, field, _dptr(out)))
        return out

    def set_state(self, scen: int, st: np.ndarray):
        a = np.ascontiguousarray(np.asarray(st, dtype=np.float64)[:, :3])
        self._chk(self.L.gf_set_state(self._p, scen, _dptr(a)))

    def state(self, scen: int = 0) -> np.ndarray:
        n = self.leaves(scen).shape[0]
        out = np.zeros((n, 4, self.m, self.m))
        self._chk(self.L.gf_get_state(self._p, scen, _dptr(out)))
        return out

    def fill_ghosts(self):
        self._chk(self.L.gf_fill_ghosts(self._p))

    def ghosted(self, scen: int, leaf: int, field: int) -> np.ndarray:
        out = np.zeros((self.m + 4, self.m + 4))
        self._chk(self.L.gf_get_ghosted(self._p, scen, leaf, field, _dptr(out)))
        return out

    def step(self, nsteps: int, dt_fixed: Optional[Sequence[float]] = None, plain: bool = False,
             lts: bool = False) -> gf_step_stats:
        """nsteps accepted steps by the fused path (gf_step), by the plain
        comparator path (gf_step_plain) when plain is set, or nsteps macro
        steps of local time stepping (gf_step_lts) when lts is set."""
        st = gf_step_stats()
        fn = self.L.gf_step_plain if plain else (self.L.gf_step_lts if lts else self.L.gf_step)
        if dt_fixed is not None:
            d = np.ascontiguousarray(dt_fixed, dtype=np.float64)
            if d.shape[0] < nsteps:
                raise ValueError("dt_fixed needs one entry per step")
            self._chk(fn(self._p, nsteps, _dptr(d), C.byref(st)))
        else:
            self._chk(fn(self._p, nsteps, None, C.byref(st)))
        return st

    def tag(self, mode: int = GF_TAG_PLAIN) -> np.ndarray:
        """Flags of every leaf: the plain criteria (GF_TAG_PLAIN) or the network (GF_TAG_LEARNED)."""
        n = C.c_int64()
        cap = sum(self.leaves(k).shape[0] for k in range(len(self.scenarios)))
        out = np.zeros(max(cap, 1), dtype=np.int8)
        self._chk(self.L.gf_tag(self._p, mode, out.ctypes.data_as(C.POINTER(C.c_int8)), cap, C.byref(n)))
        return out[:n.value].copy()

    def set_gauges(self, points, cap: int = 4096):
        """Gauges at points [(scenario, x, y)], up to cap records each."""
        pts = list(points)
        sc = np.ascontiguousarray([int(p[0]) for p in pts] or [0], dtype=np.int32)
        xy = np.ascontiguousarray([(float(p[1]), float(p[2])) for p in pts] or [(0.0, 0.0)], dtype=np.float64)
        self._chk(self.L.gf_set_gauges(self._p, len(pts), sc.ctypes.data_as(C.POINTER(C.c_int32)), _dptr(xy), cap))
        self._gauge_cap = cap

    def gauge(self, g: int) -> np.ndarray:
        """Records of gauge g as rows (t, h, hu, hv, b)."""
        n = C.c_int64()
        self._chk(self.L.gf_get_gauges(self._p, g, None, 0, C.byref(n)))
        k = min(n.value, self._gauge_cap)
        out = np.zeros((max(k, 1), 5))
        self._chk(self.L.gf_get_gauges(self._p, g, _dptr(out), k, C.byref(n)))
        return out[:k]

    def regrid(self, flags: Optional[np.ndarray] = None) -> int:
        n = C.c_int64()
        if flags is None:
            self._chk(self.L.gf_regrid(self._p, None, C.byref(n)))
        else:
            f = np.ascontiguousarray(flags, dtype=np.int8)
            self._chk(self.L.gf_regrid(self._p, f.ctypes.data_as(C.POINTER(C.c_int8)), C.byref(n)))
        return n.value

    def mass(self, scen: int = 0):
        m, c, b = C.c_double(), C.c_double(), C.c_double()
        self._chk(self.L.gf_mass(self._p, scen, C.byref(m), C.byref(c), C.byref(b)))
        return np.array([m.value, c.value, b.value])

    def mass_static(self, scen: int = 0):
        """gf_mass_static: the mass budget without any allocation (static device scratch)."""
        m, c, b = C.c_double(), C.c_double(), C.c_double()
        self._chk(self.L.gf_mass_static(self._p, scen, C.byref(m), C.byref(c), C.byref(b)))
        return np.array([m.value, c.value, b.value])

    def time(self, scen: int = 0):
        t, dt = C.c_double(), C.c_double()
        s, r = C.c_int64(), C.c_int64()
        self._chk(self.L.gf_time(self._p, scen, C.byref(t), C.byref(dt), C.byref(s), C.byref(r)))
        return t.value, dt.value, s.value, r.value

    def set_time(self, scen: int, t: float, dt_next: float = 0.0):
        self._chk(self.L.gf_set_time(self._p, scen, t, dt_next))

    def set_step_threads(self, nt: int):
        self._chk(self.L.gf_set_step_threads(self._p, nt))

    def set_schedule(self, workgroups: int = -1):
        """-1: resident persistent grid; k > 0: k persistent workgroups; 0: one per patch."""
        self._chk(self.L.gf_set_schedule(self._p, int(workgroups)))

    def autotune(self, steps: int = 5, cache: Optional[str] = None):
        """Time the step kernel's shapes on the current state and keep the
        fastest (state unchanged).  Returns (threads, schedule, us_per_step);
        the padding chosen is in autotune_choice()."""
        nt, sc, pad, us = C.c_int32(), C.c_int32(), C.c_int32(), C.c_double()
        self._chk(self.L.gf_autotune(self._p, steps, cache.encode() if cache else None,
                                     C.byref(nt), C.byref(sc), C.byref(pad), C.byref(us)))
        self._tuned = (nt.value, sc.value, pad.value, us.value)
        return nt.value, sc.value, us.value

    def autotune_choice(self):
        """(threads, schedule, padding, us_per_step) of the last autotune."""
        return getattr(self, "_tuned", None)

    def autotune_trials(self):
        """The last timed autotune's trials: rows (threads, schedule, padding, us per step)."""
        n = C.c_int64()
        self._chk(self.L.gf_autotune_trials(self._p, None, None, 0, C.byref(n)))
        sh = np.zeros((max(n.value, 1), 3), dtype=np.int32)
        us = np.zeros(max(n.value, 1))
        self._chk(self.L.gf_autotune_trials(self._p, sh.ctypes.data_as(C.POINTER(C.c_int32)), _dptr(us), n.value,
                                            C.byref(n)))
        return [(int(a), int(b), int(c), float(u)) for (a, b, c), u in zip(sh[:n.value], us[:n.value])]

    def set_step_pad(self, pad: int):
        self._chk(self.L.gf_set_step_pad(self._p, pad))

    def step_threads(self) -> int:
        n = C.c_int32()
        self._chk(self.L.gf_get_step_threads(self._p, C.byref(n)))
        return n.value

    def profile_enable(self, on: bool = True, patches: bool = False, kernel: bool = False):
        """Time steps with an event pair per stretch of launches (on), have the
        kernels count patches (patches), time each step-kernel launch alone
        with its own event pair (kernel)."""
        self._chk(self.L.gf_profile_enable(self._p, (1 if on else 0) | (2 if patches else 0) | (4 if kernel else 0)))

    def profile_kernel(self):
        """(timed step-kernel launches, their summed ms) since the last read."""
        n, ms = C.c_int64(), C.c_double()
        self._chk(self.L.gf_profile_kernel(self._p, C.byref(n), C.byref(ms)))
        return n.value, ms.value

    def profile_read(self):
        n, ms = C.c_int64(), C.c_double()
        self._chk(self.L.gf_profile_read(self._p, C.byref(n), C.byref(ms)))
        return n.value, ms.value

    # --------------------------------------------------------- learned tagger
    def net_set_params(self, params: np.ndarray):
        p = np.ascontiguousarray(params, dtype=np.float64)
        self._chk(self.L.gf_net_set_params(self._p, _dptr(p), p.size))

    def net_params(self) -> np.ndarray:
        out = np.zeros(NET_PARAMS)
        self._chk(self.L.gf_net_get_params(self._p, _dptr(out), NET_PARAMS))
        return out

    def net_features(self) -> np.ndarray:
        """(n_leaves, 24, 24, 4) feature tiles of all scenarios' leaves (FP32 values)."""
        n = C.c_int64()
        self._chk(self.L.gf_net_features(self._p, None, 0, C.byref(n)))
        out = np.zeros((n.value, 24, 24, 4))
        self._chk(self.L.gf_net_features(self._p, _dptr(out), out.size, C.byref(n)))
        return out

    def net_forward(self, x: np.ndarray) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, NET_FEATURES)
        out = np.zeros((x.shape[0], 3))
        self._chk(self.L.gf_net_forward(self._p, _dptr(x), x.shape[0], _dptr(out)))
        return out

    def net_train_step(self, x: np.ndarray, y: np.ndarray, class_w, lr: float, want_grad: bool = False):
        x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, NET_FEATURES)
        y = np.ascontiguousarray(y, dtype=np.int8)
        cw = np.ascontiguousarray(class_w, dtype=np.float64)
        loss = C.c_double()
        g = np.zeros(NET_PARAMS) if want_grad else None
        self._chk(self.L.gf_net_train_step(self._p, _dptr(x), y.ctypes.data_as(C.POINTER(C.c_int8)), x.shape[0],
                                           _dptr(cw), lr, C.byref(loss), _dptr(g) if want_grad else None))
        return (loss.value, g) if want_grad else loss.value

    def net_train_step_dev(self, x_bf16, y, class_w, lr: float, want_loss: bool = True):
        """One training step on a batch in device memory: x_bf16 a torch int16 /
        uint16 / bfloat16 tensor of n x 2304 values, y a torch int8 tensor of n
        labels, both on the context's device."""
        n = int(y.numel())
        if x_bf16.numel() != n * NET_FEATURES:
            raise ValueError("x_bf16 needs n x 2304 values")
        if not (x_bf16.is_contiguous() and y.is_contiguous()):
            raise ValueError("x_bf16 and y must be contiguous")
        if x_bf16.element_size() != 2 or y.element_size() != 1:
            raise ValueError("x_bf16 holds 16-bit values and y 8-bit labels")
        cw = np.ascontiguousarray(class_w, dtype=np.float64)
        loss = C.c_double()
        self._chk(self.L.gf_net_train_step_dev(self._p, C.c_void_p(x_bf16.data_ptr()), C.c_void_p(y.data_ptr()), n,
                                               _dptr(cw), lr, C.byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    def net_predict(self) -> np.ndarray:
        n = C.c_int64()
        cap = sum(self.leaves(k).shape[0] for k in range(len(self.scenarios)))
        out = np.zeros(cap, dtype=np.int8)
        self._chk(self.L.gf_net_predict(self._p, out.ctypes.data_as(C.POINTER(C.c_int8)), cap, C.byref(n)))
        return out[:n.value]

    def net_collect(self, window: int = 16, check_every: int = 4):
        """Features and labels (class 0 coarsen, 1 keep, 2 refine) of one window; regrids after it."""
        n = C.c_int64()
        cap = sum(self.leaves(k).shape[0] for k in range(len(self.scenarios)))
        F = np.zeros((cap, 24, 24, 4))
        y = np.zeros(cap, dtype=np.int8)
        self._chk(self.L.gf_net_collect(self._p, window, check_every, _dptr(F), y.ctypes.data_as(C.POINTER(C.c_int8)),
                                        cap, C.byref(n)))
        return F[:n.value], y[:n.value].copy()

    def run(self, nsteps: int, mode: int, check_every: int = 4, regrid_every: int = 16) -> "gf_run_stats":
        st = gf_run_stats()
        self._chk(self.L.gf_run(self._p, nsteps, mode, check_every, regrid_every, C.byref(st)))
        return st

    def profile_patches(self):
        """(patches through the full update, stable dry patches skipped) since profile_enable(patches=True)."""
        a, b = C.c_int64(), C.c_int64()
        self._chk(self.L.gf_profile_patches(self._p, C.byref(a), C.byref(b)))
        return a.value, b.value

    # ------------------------------------------------------------ helpers
    def set_initial_fn(self, scen: int, fn, max_passes: int = 0):
        """gf_set_initial with a Python callback fn(level, x0, y0, dx, dy, b) ->
        (h, hu, hv), b and the results m x m arrays [j][i]."""
        m = self.m

        def ic(user, s, level, x0, y0, dx, dy, nx, ny, b, h, hu, hv):
            bb = np.ctypeslib.as_array(b, shape=(ny, nx)).copy()
            H, HU, HV = fn(level, x0, y0, dx, dy, bb)
            for ptr, v in ((h, H), (hu, HU), (hv, HV)):
                np.ctypeslib.as_array(ptr, shape=(ny, nx))[:] = np.asarray(v, dtype=np.float64).reshape(ny, nx)
        cb = GF_IC_FN(ic)
        self._chk(self.L.gf_set_initial(self._p, scen, cb, None, int(max_passes)))

    def set_initial(self, scen: int = 0, precision: Optional[str] = None, max_passes: int = 0):
        """Initial state from the scenario recipe (inputs.initial_state, formed
        from this library's own bed) through gf_set_initial; max_passes rounds
        of plain tagging and regridding around it.  Returns the state."""
        from .inputs import initial_state
        if precision is None:
            precision = "f32" if self.precision == GF_FP32 else "f64"
        sc = self.scenarios[scen]
        m = self.m

        def fn(level, x0, y0, dx, dy, b):
            # the leaf (tree, level, ix, iy) from its corner
            PI = int(round((x0 - sc.x0) / (dx * m)))
            PJ = int(round((y0 - sc.y0) / (dy * m)))
            n = 1 << level
            leaf = ((PJ // n) * sc.mi + PI // n, level, PI % n, PJ % n)
            return initial_state(sc, leaf, b, precision)
        self.set_initial_fn(scen, fn, max_passes)
        return self.state(scen)
