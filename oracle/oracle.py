"""ctypes wrapper of the FP64 CPU reference (test infrastructure only)."""

from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pd_oracle.c")
_SO = os.path.join(_HERE, "libpdoracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain IEEE double, no contraction)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fPIC", "-shared", "-std=c11", "-ffp-contract=off",
               "-fno-fast-math", "-fopenmp", "-Wall", "-Wno-unused-function",
               _SRC, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_SO)
        P = C.c_void_p
        i64, i32, dbl = C.c_int64, C.c_int, C.c_double
        L.orc_create.restype = P
        L.orc_create.argtypes = [i64, i32, P, dbl, P, dbl, P, P, i32]
        L.orc_free.argtypes = [P]
        L.orc_n_bonds.restype = i64
        L.orc_n_bonds.argtypes = [P]
        for name in ("orc_get_bonds", "orc_get_bond_geom"):
            getattr(L, name).argtypes = [P, P, P]
        for name in ("orc_get_m", "orc_get_theta", "orc_get_rho", "orc_set_rho",
                     "orc_get_break_step", "orc_damage"):
            getattr(L, name).argtypes = [P, P]
        L.orc_get_step.restype = i64
        L.orc_get_step.argtypes = [P]
        L.orc_set_step.argtypes = [P, i64]
        L.orc_min_margin.restype = dbl
        L.orc_min_margin.argtypes = [P]
        L.orc_n_close.restype = i64
        L.orc_n_close.argtypes = [P]
        L.orc_reset_margin.argtypes = [P]
        L.orc_track_bond_margins.argtypes = [P, i32]
        L.orc_get_bond_margins.restype = i32
        L.orc_get_bond_margins.argtypes = [P, P]
        L.orc_constants.argtypes = [i32, dbl, dbl, P]
        L.orc_critical_stretch.restype = dbl
        L.orc_critical_stretch.argtypes = [i32, dbl, dbl, dbl, dbl, i32]
        L.orc_set_specimen.restype = i32
        L.orc_set_specimen.argtypes = [P, i32, i32, dbl, dbl, dbl, dbl, dbl]
        L.orc_apply_cuts.restype = i64
        L.orc_apply_cuts.argtypes = [P, P, i32]
        L.orc_force.argtypes = [P, P, P, P]
        L.orc_strain_energy.restype = dbl
        L.orc_strain_energy.argtypes = [P, P]
        L.orc_strain_energy_last.restype = dbl
        L.orc_strain_energy_last.argtypes = [P]
        L.orc_run.restype = i32
        L.orc_run.argtypes = [P, i64, P, P, P, P, i64, P]
        L.orc_lambda_max.restype = dbl
        L.orc_lambda_max.argtypes = [P, P, i32, C.c_uint64]
        L.orc_set_finite.restype = None
        L.orc_set_finite.argtypes = [P, i32]
        L.orc_adr_density.restype = None
        L.orc_adr_density.argtypes = [P, dbl, P]
        L.orc_adr_run.restype = i32
        L.orc_adr_run.argtypes = [P, i64, P, P, P, P, P, P, P, i64, dbl, P]
        L.orc_num_threads.restype = i32
        L.orc_set_num_threads.argtypes = [i32]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def constants(mode: int, E: float, nu: float) -> dict:
    out = np.zeros(5)
    lib().orc_constants(mode, E, nu, _p(out))
    return dict(kappa=out[0], mu=out[1], A=out[2], K=out[3], G=out[4])


def critical_stretch(mode: int, E: float, nu: float, G0: Optional[float], delta: float,
                     variant: int = 0) -> float:
    g = float("nan") if G0 is None else float(G0)
    return lib().orc_critical_stretch(mode, E, nu, g, delta, variant)


class Oracle:
    """FP64 reference model of one workload (all specimens)."""

    def __init__(self, w, search: str = "auto", s0: Optional[np.ndarray] = None,
                 dt: Optional[np.ndarray] = None, apply_cuts: bool = True):
        L = lib()
        self.w = w
        self.n = w.n
        if search == "auto":
            search = "brute" if w.n <= 4000 else "cells"
        self._lat = np.ascontiguousarray(w.lat, dtype=np.int32)
        self._origin = np.ascontiguousarray(w.origin, dtype=np.float64)
        self._vol = np.ascontiguousarray(w.vol, dtype=np.float64)
        self._spec = np.ascontiguousarray(w.specimen, dtype=np.int32)
        self.h = L.orc_create(w.n, w.dim, _p(self._lat), w.dx, _p(self._origin), w.delta,
                              _p(self._vol), _p(self._spec), 1 if search == "cells" else 0)
        if not self.h:
            raise RuntimeError("orc_create failed")
        self.nb = int(L.orc_n_bonds(self.h))
        mode = w.mode_id()
        ns = w.n_specimens
        dts = np.asarray(w.dt if dt is None else dt, dtype=np.float64).reshape(-1)
        if dts.size == 1 and ns > 1:
            dts = np.full(ns, dts[0])
        self.s0 = np.zeros(ns)
        for k, mat in enumerate(w.materials):
            s = critical_stretch(mode, mat.E, mat.nu, mat.G0, w.delta, w.s0_variant) \
                if s0 is None else float(np.asarray(s0).reshape(-1)[k])
            self.s0[k] = s
            L.orc_set_specimen(self.h, k, mode, mat.E, mat.nu, mat.rho, s, float(dts[k]))
        self.dt = dts
        self.n_cut = 0
        if apply_cuts and len(w.cuts):
            ct = np.ascontiguousarray(w.cut_table())
            self.n_cut = int(L.orc_apply_cuts(self.h, _p(ct), ct.shape[0]))
        self._bc = np.ascontiguousarray(w.bc, dtype=np.uint8)
        self._fext = np.ascontiguousarray(w.fext, dtype=np.float64)

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().orc_free(self.h)
                self.h = None
        except Exception:
            pass

    # ---- accessors -----------------------------------------------------
    def bonds(self):
        bi = np.empty(self.nb, np.int32)
        bj = np.empty(self.nb, np.int32)
        lib().orc_get_bonds(self.h, _p(bi), _p(bj))
        return bi, bj

    def bond_geom(self):
        xl = np.empty(self.nb)
        M = np.empty((self.nb, 3))
        lib().orc_get_bond_geom(self.h, _p(xl), _p(M))
        return xl, M

    def m(self):
        out = np.empty(self.n)
        lib().orc_get_m(self.h, _p(out))
        return out

    def theta(self):
        out = np.empty(self.n)
        lib().orc_get_theta(self.h, _p(out))
        return out

    def rho(self):
        out = np.empty(self.nb, np.uint8)
        lib().orc_get_rho(self.h, _p(out))
        return out

    def set_rho(self, r):
        r = np.ascontiguousarray(r, dtype=np.uint8)
        lib().orc_set_rho(self.h, _p(r))

    def break_step(self):
        out = np.empty(self.nb, np.int32)
        lib().orc_get_break_step(self.h, _p(out))
        return out

    @property
    def step(self) -> int:
        return int(lib().orc_get_step(self.h))

    @step.setter
    def step(self, s: int):
        lib().orc_set_step(self.h, int(s))

    def min_margin(self) -> float:
        return float(lib().orc_min_margin(self.h))

    def n_close(self) -> int:
        return int(lib().orc_n_close(self.h))

    def reset_margin(self):
        lib().orc_reset_margin(self.h)

    def track_bond_margins(self, on: bool = True):
        """Start (or stop) recording, per bond, the smallest |s - s_c| / s_c
        seen while the bond was intact."""
        lib().orc_track_bond_margins(self.h, 1 if on else 0)

    def bond_margins(self) -> np.ndarray:
        out = np.empty(self.nb)
        if lib().orc_get_bond_margins(self.h, _p(out)) != 0:
            raise RuntimeError("bond margins are not tracked (call track_bond_margins first)")
        return out

    # ---- operators -----------------------------------------------------
    def force(self, u: np.ndarray):
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(self.n, 3)
        f = np.empty((self.n, 3))
        th = np.empty(self.n)
        lib().orc_force(self.h, _p(u), _p(f), _p(th))
        return f, th

    def strain_energy(self, u: np.ndarray) -> float:
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(self.n, 3)
        return float(lib().orc_strain_energy(self.h, _p(u)))

    def damage(self) -> np.ndarray:
        out = np.empty(self.n)
        lib().orc_damage(self.h, _p(out))
        return out

    def initial_state(self):
        u = np.zeros((self.n, 3))
        v = np.ascontiguousarray(self.w.v0, dtype=np.float64).copy()
        return u, v

    def run(self, nsteps: int, u: np.ndarray, v: np.ndarray, want_force: bool = False):
        """Advance in place; returns the internal force of the last step if asked."""
        assert u.flags.c_contiguous and v.flags.c_contiguous
        assert u.dtype == np.float64 and v.dtype == np.float64
        f = np.empty((self.n, 3)) if want_force else None
        lib().orc_run(self.h, int(nsteps), _p(u), _p(v), _p(self._bc), _p(self._fext),
                      int(self.w.ramp_steps), _p(f) if f is not None else None)
        return f

    def set_finite(self, finite: bool):
        """Select the finite extension and deformed force direction (Eqs.
        1.10, 1.13) instead of the linearized ones (Eqs. 2.4, 2.7)."""
        lib().orc_set_finite(self.h, 1 if finite else 0)

    def adr_density(self, dt: float = 1.0) -> np.ndarray:
        """Fictitious density of the relaxation (n x 3) for the current bond
        status."""
        lam = np.empty((self.n, 3))
        lib().orc_adr_density(self.h, float(dt), _p(lam))
        return lam

    def adr_start(self, dt: float = 1.0):
        """Relaxation state: (u, v, fprev, iteration counter, lambda)."""
        u, v = self.initial_state()
        return dict(u=u, v=v, fprev=np.zeros((self.n, 3)), it=np.zeros(1, np.int64), lam=self.adr_density(dt),
                    dt=float(dt), stats=np.zeros(4))

    def adr_run(self, nsteps: int, st: dict):
        """Advance a relaxation state in place by nsteps iterations."""
        lib().orc_adr_run(self.h, int(nsteps), _p(st["u"]), _p(st["v"]), _p(st["fprev"]), _p(st["it"]),
                          _p(st["lam"]), _p(self._bc), _p(self._fext), int(self.w.ramp_steps), st["dt"],
                          _p(st["stats"]))

    def lambda_max(self, iters: int = 500, seed: int = 0) -> float:
        return float(lib().orc_lambda_max(self.h, _p(self._bc), int(iters), C.c_uint64(seed)))


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(t: int):
    lib().orc_set_num_threads(int(t))
