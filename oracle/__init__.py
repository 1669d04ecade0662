"""CPU oracle for the GeoFlood patch update -- TEST INFRASTRUCTURE ONLY.

Plain FP64 C code (geoflood_oracle.c) wrapped with ctypes.  Only tests/,
__graft_entry__.smoke() and the CPU-baseline leg of bench.py may use it; the
library under test never imports it and shares no code with it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "geoflood_oracle.c")
_LIB = os.path.join(_HERE, "libgeoflood_oracle.so")

G_DEFAULT = 9.81
TAU_DEFAULT = 1e-4

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)


# Compile-time variants of the oracle, for pins that compare two written-out
# forms of one step.  "per_edge": the transverse solver splits each edge's
# increment into the neighbouring cell separately (the form as first written
# in the cited CTU method) instead of the cell's net normal increment.
# "asan": AddressSanitizer and UndefinedBehaviorSanitizer, every report
# fatal; loaded only by a process started with the sanitizer runtime
# preloaded (a check of the oracle itself, not of the method).
VARIANTS = {None: [], "per_edge": ["-DORC_TRANSVERSE_PER_EDGE"],
            "asan": ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                     "-fno-sanitize-recover=all"]}


def _lib_path(variant=None) -> str:
    return _LIB if variant is None else os.path.join(_HERE, f"libgeoflood_oracle_{variant}.so")


def build(force: bool = True, variant=None) -> str:
    """Compile the oracle with gcc (no FMA contraction, plain -O2, OpenMP)."""
    path = _lib_path(variant)
    if force or not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
        tmp = path + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-ffp-contract=off", "-fopenmp", "-fPIC",
                               "-shared", *VARIANTS[variant], "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, path)
    return path


_libs = {}


def lib(variant=None):
    if variant not in _libs:
        build(force=False, variant=variant)
        L = C.CDLL(_lib_path(variant))
        L.orc_create.restype = C.c_void_p
        L.orc_create.argtypes = [_dp, _ip, _dp, C.c_int]
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_set_dem.argtypes = [C.c_void_p, _dp, C.c_long, C.c_long, C.c_int]
        L.orc_set_leaves.argtypes = [C.c_void_p, _ip, C.c_int]
        L.orc_num_leaves.argtypes = [C.c_void_p]
        L.orc_get_leaves.argtypes = [C.c_void_p, _ip]
        L.orc_set_field.argtypes = [C.c_void_p, C.c_int, C.c_int, _dp]
        L.orc_get_field.argtypes = [C.c_void_p, C.c_int, C.c_int, _dp]
        L.orc_get_ghosted.argtypes = [C.c_void_p, C.c_int, C.c_int, _dp]
        L.orc_fill_ghosts.argtypes = [C.c_void_p]
        L.orc_max_speed.argtypes = [C.c_void_p]
        L.orc_max_speed.restype = C.c_double
        L.orc_step.argtypes = [C.c_void_p, C.c_double]
        L.orc_step.restype = C.c_double
        L.orc_advance.argtypes = [C.c_void_p, C.c_int, _dp, _dp, _dp]
        L.orc_advance_lts.argtypes = [C.c_void_p, C.c_int, _dp, _dp, _dp]
        L.orc_set_bathy_f32.argtypes = [C.c_void_p, C.c_int]
        L.orc_set_scheme.argtypes = [C.c_void_p, C.c_int, C.c_int]
        L.orc_wave_limiter.argtypes = [C.c_int, C.c_double]
        L.orc_wave_limiter.restype = C.c_double
        L.orc_mass.argtypes = [C.c_void_p, _dp]
        L.orc_tag.argtypes = [C.c_void_p, C.POINTER(C.c_byte)]
        L.orc_set_tag_rules.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_int, _dp, C.c_int, _dp]
        L.orc_regrid.argtypes = [C.c_void_p, C.POINTER(C.c_byte)]
        L.orc_time.argtypes = [C.c_void_p]
        L.orc_time.restype = C.c_double
        L.orc_dt.argtypes = [C.c_void_p]
        L.orc_dt.restype = C.c_double
        L.orc_steps.argtypes = [C.c_void_p]
        L.orc_steps.restype = C.c_long
        L.orc_rejected.argtypes = [C.c_void_p]
        L.orc_rejected.restype = C.c_long
        L.orc_set_time.argtypes = [C.c_void_p, C.c_double, C.c_double]
        L.orc_bathy.argtypes = [C.c_void_p, C.c_int, C.c_long, C.c_long]
        L.orc_bathy.restype = C.c_double
        L.orc_riemann.argtypes = [C.c_double] * 8 + [C.c_double, C.c_double, _dp, _dp, _dp, _dp]
        L.orc_riemann.restype = C.c_int
        L.orc_mirror_middle_depth.argtypes = [C.c_double, C.c_double, C.c_double]
        L.orc_mirror_middle_depth.restype = C.c_double
        L.orc_inflow_depth.argtypes = [C.c_double] * 5
        L.orc_inflow_depth.restype = C.c_double
        L.orc_hydrograph.argtypes = [C.c_void_p, C.c_double]
        L.orc_hydrograph.restype = C.c_double
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_get_threads.restype = C.c_int
        L.orc_cbrt.argtypes = [C.c_double]
        L.orc_cbrt.restype = C.c_double
        _libs[variant] = L
    return _libs[variant]


def set_threads(n: int) -> int:
    """Threads for the oracle's loops over leaves (n < 1: every core).  The
    results do not depend on it.  Returns the count now in effect."""
    lib().orc_set_threads(int(n))
    return lib().orc_get_threads()


def threads() -> int:
    return lib().orc_get_threads()


def wave_limiter(lim: int, theta: float) -> float:
    """phi(theta) of limiter `lim` (0 MC, 1 minmod, 2 superbee, 3 van Leer, 4 none)."""
    return lib().orc_wave_limiter(lim, theta)


def cbrt(x: float) -> float:
    """The oracle's cube root (used by the friction term)."""
    return lib().orc_cbrt(float(x))


def _d(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def riemann(hl, ml, tl, bl, hr, mr, tr, br, g=G_DEFAULT, tau=TAU_DEFAULT):
    """One normal Riemann problem: returns (s[3], z[3,3], amdq[3], apdq[3], wall)."""
    s = np.zeros(3)
    z = np.zeros(9)
    am = np.zeros(3)
    ap = np.zeros(3)
    w = lib().orc_riemann(hl, ml, tl, bl, hr, mr, tr, br, g, tau, _d(s), _d(z), _d(am), _d(ap))
    return s, z.reshape(3, 3), am, ap, w


def mirror_middle_depth(h, u, g=G_DEFAULT):
    return lib().orc_mirror_middle_depth(h, u, g)


def inflow_depth(qbar, hint, mint, g=G_DEFAULT, tau=TAU_DEFAULT):
    return lib().orc_inflow_depth(qbar, hint, mint, g, tau)


class Oracle:
    """One scenario on the CPU oracle.  `sc` is an inputs.Scenario."""

    def __init__(self, sc, g: float = G_DEFAULT, tau: float = TAU_DEFAULT,
                 cfl_desired: float = 0.9, cfl_max: float = 1.0, leaves: Optional[np.ndarray] = None,
                 variant=None, limiter: int = 0, transverse: int = 0):
        self.sc = sc
        self.m = sc.m
        self._L = lib(variant)
        dp = np.array([sc.x0, sc.y0, sc.x1, sc.y1, g, tau, sc.manning_n, cfl_desired, cfl_max,
                       sc.inflow_lo, sc.inflow_hi, sc.tag_h_refine, sc.tag_eta_refine, sc.t_end], dtype=np.float64)
        ip = np.array([sc.mi, sc.mj, sc.m, sc.min_level, sc.max_level, *sc.bc, sc.inflow_side], dtype=np.int32)
        hy = np.array(sc.hydro if sc.hydro else [(0.0, 0.0)], dtype=np.float64).reshape(-1)
        nh = len(sc.hydro) if sc.hydro else 0
        L = self._L
        self._p = L.orc_create(_d(dp), ip.ctypes.data_as(_ip), _d(hy), nh)
        # limiter: 0 MC, 1 minmod, 2 superbee, 3 van Leer, 4 none; transverse: 0 corrected, 1 none
        L.orc_set_scheme(self._p, limiter, transverse)
        rg = np.asarray(sc.regions if sc.regions else [(0.0,) * 6], dtype=np.float64).reshape(-1)
        gr = np.asarray(sc.grades if sc.grades else [(0.0,) * 3], dtype=np.float64).reshape(-1)
        L.orc_set_tag_rules(self._p, sc.tag_u_refine, sc.tag_q_refine, len(sc.regions) if sc.regions else 0, _d(rg),
                            len(sc.grades) if sc.grades else 0, _d(gr))
        dem = np.ascontiguousarray(sc.dem, dtype=np.float64)
        rc = L.orc_set_dem(self._p, _d(dem), dem.shape[1], dem.shape[0], sc.dem_level)
        if rc != 0:
            raise ValueError("DEM shape does not match the scenario at dem_level")
        if leaves is None:
            leaves = sc.uniform_leaves(sc.init_level)
        self.set_leaves(leaves)

    def __del__(self):
        try:
            if self._p:
                self._L.orc_destroy(self._p)
                self._p = None
        except Exception:
            pass

    # mesh -------------------------------------------------------------
    def set_leaves(self, leaves: np.ndarray):
        a = np.ascontiguousarray(np.asarray(leaves, dtype=np.int32).reshape(-1, 4))
        self._L.orc_set_leaves(self._p, a.ctypes.data_as(_ip), a.shape[0])

    @property
    def n_leaves(self) -> int:
        return self._L.orc_num_leaves(self._p)

    def leaves(self) -> np.ndarray:
        out = np.zeros((self.n_leaves, 4), dtype=np.int32)
        self._L.orc_get_leaves(self._p, out.ctypes.data_as(_ip))
        return out

    # fields -----------------------------------------------------------
    def set_field(self, leaf: int, field: int, a: np.ndarray):
        a = np.ascontiguousarray(a, dtype=np.float64).reshape(self.m, self.m)
        if self._L.orc_set_field(self._p, leaf, field, _d(a)) != 0:
            raise IndexError
    def get_field(self, leaf: int, field: int) -> np.ndarray:
        out = np.zeros((self.m, self.m))
        if self._L.orc_get_field(self._p, leaf, field, _d(out)) != 0:
            raise IndexError
        return out

    def get_ghosted(self, leaf: int, field: int) -> np.ndarray:
        out = np.zeros((self.m + 4, self.m + 4))
        self._L.orc_get_ghosted(self._p, leaf, field, _d(out))
        return out

    def state(self) -> np.ndarray:
        """(n_leaves, 4, m, m) array of h, hu, hv, b."""
        n = self.n_leaves
        out = np.zeros((n, 4, self.m, self.m))
        for k in range(n):
            for f in range(4):
                out[k, f] = self.get_field(k, f)
        return out

    def set_state(self, st: np.ndarray):
        for k in range(st.shape[0]):
            for f in range(3):
                self.set_field(k, f, st[k, f])

    # time stepping ----------------------------------------------------
    def fill_ghosts(self):
        self._L.orc_fill_ghosts(self._p)

    def max_speed(self) -> float:
        return self._L.orc_max_speed(self._p)

    def step(self, dt: float) -> float:
        """One step of length dt; returns max|s|/dx.  Does not advance the clock."""
        return self._L.orc_step(self._p, dt)

    def advance(self, nsteps: int, dt_fixed: Optional[Sequence[float]] = None, return_dt: bool = False,
                lts: bool = False):
        """Advance with adaptive or fixed steps; returns the Courant numbers of the
        accepted steps (and their lengths if return_dt).  lts: each step is a
        macro step of local time stepping (dt that of the coarsest level)."""
        nu = np.zeros(max(nsteps, 1))
        dts = np.zeros(max(nsteps, 1))
        s0 = self.steps
        if dt_fixed is not None:
            d = np.ascontiguousarray(dt_fixed, dtype=np.float64)
            rc = (self._L.orc_advance_lts if lts else self._L.orc_advance)(self._p, nsteps, _d(d), _d(nu), _d(dts))
        else:
            rc = (self._L.orc_advance_lts if lts else self._L.orc_advance)(self._p, nsteps, None, _d(nu), _d(dts))
        if rc != 0:
            raise RuntimeError(f"oracle advance failed ({rc})")
        k = self.steps - s0
        return (nu[:k], dts[:k]) if return_dt else nu[:k]

    def set_bathy_f32(self, on: bool = True):
        """Hold the bathymetry rounded to float32 (FP32-path judging)."""
        self._L.orc_set_bathy_f32(self._p, 1 if on else 0)

    @property
    def t(self) -> float:
        return self._L.orc_time(self._p)

    @property
    def dt(self) -> float:
        return self._L.orc_dt(self._p)

    @property
    def steps(self) -> int:
        return self._L.orc_steps(self._p)

    @property
    def rejected(self) -> int:
        return self._L.orc_rejected(self._p)

    def set_time(self, t: float, dt: float = 0.0):
        self._L.orc_set_time(self._p, t, dt)

    def mass(self):
        out = np.zeros(3)
        self._L.orc_mass(self._p, _d(out))
        return out  # mass, clamp mass, boundary inflow volume

    # AMR --------------------------------------------------------------
    def tag(self) -> np.ndarray:
        out = np.zeros(self.n_leaves, dtype=np.int8)
        self._L.orc_tag(self._p, out.ctypes.data_as(C.POINTER(C.c_byte)))
        return out

    def regrid(self, flags: np.ndarray) -> int:
        f = np.ascontiguousarray(flags, dtype=np.int8)
        return self._L.orc_regrid(self._p, f.ctypes.data_as(C.POINTER(C.c_byte)))

    def bathy(self, level: int, I: int, J: int) -> float:
        return self._L.orc_bathy(self._p, level, I, J)

    def hydrograph(self, t: float) -> float:
        return self._L.orc_hydrograph(self._p, t)
