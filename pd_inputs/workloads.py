"""Workload generators (geometry, boundary conditions, loads, notches, materials).

Conventions shared by every consumer of these inputs:

* Nodes sit on a uniform lattice.  Node ``p`` has integer lattice coordinates
  ``lat[p]`` and physical position ``origin + dx * lat[p]``.  All examples of
  the paper are discretised on uniform grids with an m-ratio delta/dx of 3
  (Section 4 opening); the workloads use delta = 3.015 dx so that no lattice
  distance lies on the horizon sphere.
* Node volume is dx^3 in 3D and dx^2 * h in 2D with thickness h = 1 m.
* ``bc[p]`` bit c set means displacement component c of node p is prescribed:
  its velocity is held at ``v0[p, c]`` for the whole run and its displacement
  advances by dt * v0 each step (a fixed component simply has v0 = 0).
* ``fext[p]`` is the nodal external force at full load.  The load applied at
  step n is ``fext * r(n)`` with ``r(n) = min(1, n / ramp_steps)``, or
  ``r = 1`` when ``ramp_steps == 0``.
* A cut (notch) removes, before the first step, every bond whose straight
  segment properly crosses the notch patch.
* Specimens: ``specimen[p]`` is the specimen id of node p; bonds never join
  nodes of different specimens, and every specimen has its own material,
  time step and critical stretch.
"""

from __future__ import annotations

import json
import math
import os
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
PARAMS_PATH = os.path.join(_HERE, "params.json")

M_RATIO = 3.015  # delta / dx for every workload


@dataclass
class Material:
    E: float          # Young's modulus [Pa]
    nu: float         # Poisson's ratio
    rho: float        # mass density [kg/m^3]
    G0: Optional[float] = None  # fracture energy [J/m^2]; None = bonds never break


@dataclass
class Cut:
    """A notch patch.

    kind 'segment2d': straight segment from p0=(x,y) to p1=(x,y).
    kind 'rect3d'   : planar parallelogram {c + s*a + t*b : s, t in [0, 1]}.
    kind 'helicoid' : helicoidal strip about the z axis through (0, 0):
                      z - zc = pitch * theta, r_in <= r <= r_out,
                      th0 <= theta <= th1 (theta = atan2(y, x) in (-pi, pi]).
    ``specimen`` restricts the cut to one specimen (-1 = every specimen).
    """

    kind: str
    p: List[float] = field(default_factory=list)
    specimen: int = -1

    def as_row(self) -> List[float]:
        """Fixed 12-slot record: [kind_id, specimen, 10 parameters]."""
        kid = {"segment2d": 0, "rect3d": 1, "helicoid": 2}[self.kind]
        vals = list(self.p) + [0.0] * (10 - len(self.p))
        return [float(kid), float(self.specimen)] + vals


@dataclass
class Workload:
    name: str
    dim: int
    mode: str                     # '3d', 'plane_stress' or 'plane_strain'
    lat: np.ndarray               # (n, dim) int32
    dx: float
    origin: np.ndarray            # (3,) float64
    delta: float
    vol: np.ndarray               # (n,) float64
    specimen: np.ndarray          # (n,) int32
    materials: List[Material]     # indexed by specimen id
    bc: np.ndarray                # (n,) uint8
    v0: np.ndarray                # (n, 3) float64
    fext: np.ndarray              # (n, 3) float64
    ramp_steps: int
    cuts: List[Cut]
    steps: int
    dt: np.ndarray                # (n_specimens,) float64
    s0_variant: int = 0           # 0: 3D beta' as printed, 1: re-derived
    notes: str = ""

    @property
    def n(self) -> int:
        return int(self.lat.shape[0])

    @property
    def n_specimens(self) -> int:
        return len(self.materials)

    def positions(self) -> np.ndarray:
        """(n, 3) physical coordinates (z = 0 in 2D)."""
        x = np.zeros((self.n, 3))
        x[:, : self.dim] = self.lat.astype(np.float64) * self.dx
        x += self.origin[None, :]
        return x

    def cut_table(self) -> np.ndarray:
        return np.array([c.as_row() for c in self.cuts], dtype=np.float64).reshape(-1, 12)

    def mode_id(self) -> int:
        return {"3d": 0, "plane_stress": 1, "plane_strain": 2}[self.mode]


# --------------------------------------------------------------------------
# parameter table (time steps and torsion rates), written by the CPU reference
# --------------------------------------------------------------------------

def load_params() -> dict:
    if not os.path.exists(PARAMS_PATH):
        return {}
    with open(PARAMS_PATH) as f:
        return json.load(f)


def _param(key: str, default=None):
    p = load_params()
    return p.get(key, default)


def _box(shape) -> np.ndarray:
    grids = np.meshgrid(*[np.arange(s, dtype=np.int32) for s in shape], indexing="ij")
    return np.stack([g.ravel() for g in grids], axis=1).astype(np.int32)


def _finish(w: Workload, dt_key: Optional[str]) -> Workload:
    if dt_key is not None and w.dt is None:
        v = _param(dt_key)
        w.dt = np.array(v if isinstance(v, list) else [v if v is not None else np.nan],
                        dtype=np.float64)
    return w


# --------------------------------------------------------------------------
# workload 1: 3D cantilever, no damage
# --------------------------------------------------------------------------

def cantilever3d(nx: int = 20, ny: int = 4, nz: int = 4, dx: float = 1e-3,
                 steps: int = 2000, load: float = 1000.0, ramp_steps: int = 50,
                 fixed_layers: int = 3, dt: Optional[float] = None) -> Workload:
    """Cantilever beam clamped over its first three lattice layers (x index
    0..2) with a total tip force ``load`` in -z spread evenly over the last
    layer, ramped linearly over ``ramp_steps`` steps and then held."""
    lat = _box((nx, ny, nz))
    n = lat.shape[0]
    bc = np.where(lat[:, 0] < fixed_layers, 7, 0).astype(np.uint8)
    tip = lat[:, 0] == nx - 1
    fext = np.zeros((n, 3))
    fext[tip, 2] = -load / float(tip.sum())
    key = "cantilever3d" if (nx, ny, nz, dx) == (20, 4, 4, 1e-3) else None
    w = Workload(
        name="cantilever3d", dim=3, mode="3d", lat=lat, dx=dx, origin=np.zeros(3),
        delta=M_RATIO * dx, vol=np.full(n, dx ** 3), specimen=np.zeros(n, np.int32),
        materials=[Material(E=200e9, nu=0.3, rho=7850.0, G0=None)], bc=bc,
        v0=np.zeros((n, 3)), fext=fext, ramp_steps=ramp_steps, cuts=[], steps=steps,
        dt=None if dt is None else np.array([dt]),
        notes="3D cantilever 20x4x4, 1 kN tip load in -z ramped over 50 steps",
    )
    if w.dt is None and key is None:
        raise ValueError("non-default cantilever needs an explicit dt")
    return _finish(w, key)


# --------------------------------------------------------------------------
# workload 2: 2D plane-stress edge-notched plate under tension
# --------------------------------------------------------------------------

def plate2d(nx: int = 200, ny: int = 80, dx: float = 0.5e-3, steps: int = 1500,
            sigma: float = 1.0e6, E: float = 72e9, nu: float = 0.22, rho: float = 2440.0,
            G0: Optional[float] = 3.8, notch_row: Optional[int] = None,
            notch_tip: Optional[float] = None, mode: str = "plane_stress",
            dt: Optional[float] = None) -> Workload:
    """Rectangular plate, notch along the half-lattice line between rows
    ``notch_row`` and ``notch_row + 1`` from outside the left edge to
    x = notch_tip (in lattice units), uniform traction ``sigma`` pulling the
    bottom (j = 0) and top (j = ny-1) rows outward."""
    lat = _box((nx, ny))
    n = lat.shape[0]
    h = 1.0
    if notch_row is None:
        notch_row = ny // 2 - 1
    if notch_tip is None:
        notch_tip = (nx // 2 - 1) + 0.37
    fext = np.zeros((n, 3))
    fext[lat[:, 1] == 0, 1] = -sigma * dx * h
    fext[lat[:, 1] == ny - 1, 1] = +sigma * dx * h
    yc = (notch_row + 0.5) * dx
    cut = Cut("segment2d", [-0.5 * dx, yc, notch_tip * dx, yc])
    key = "plate2d" if (nx, ny, dx, E, nu, sigma) == (200, 80, 0.5e-3, 72e9, 0.22, 1.0e6) else None
    w = Workload(
        name="plate2d", dim=2, mode=mode, lat=lat, dx=dx, origin=np.zeros(3),
        delta=M_RATIO * dx, vol=np.full(n, dx * dx * h), specimen=np.zeros(n, np.int32),
        materials=[Material(E=E, nu=nu, rho=rho, G0=G0)], bc=np.zeros(n, np.uint8),
        v0=np.zeros((n, 3)), fext=fext, ramp_steps=0, cuts=[cut], steps=steps,
        dt=None if dt is None else np.array([dt]),
        notes=f"2D {mode} plate {nx}x{ny}, notch to x={notch_tip:.2f}dx, {sigma/1e6:g} MPa",
    )
    if w.dt is None and key is None:
        raise ValueError("non-default plate needs an explicit dt")
    return _finish(w, key)


# --------------------------------------------------------------------------
# workload 3: 3D double-notched plate, edge impact by prescribed velocity
# --------------------------------------------------------------------------

def impact3d(nx: int = 200, ny: int = 200, nz: int = 9, dx: float = 1e-3,
             steps: int = 2000, v_imp: float = 16.5, dt: Optional[float] = None) -> Workload:
    """Plate with two through-thickness notches parallel to x, starting
    outside the x = 0 edge and ending a quarter of the way in; the three
    lattice layers i <= 2 of the rows between the notches are driven at
    ``v_imp`` along +x (only the x component is prescribed)."""
    lat = _box((nx, ny, nz))
    n = lat.shape[0]
    # notch planes on half-lattice lines; scaled with ny so that reduced
    # variants keep the geometry (200 -> rows 75.5 and 125.5)
    y1 = int(round(ny * 75.5 / 200.0 - 0.5)) + 0.5
    y2 = int(round(ny * 125.5 / 200.0 - 0.5)) + 0.5
    tip = int(round(nx * 50.0 / 200.0)) + 0.37
    cuts = []
    for yc in (y1, y2):
        c = [-0.5 * dx, yc * dx, -0.5 * dx]
        a = [(tip + 0.5) * dx, 0.0, 0.0]
        b = [0.0, 0.0, (nz - 1 + 1.0) * dx]
        cuts.append(Cut("rect3d", c + a + b))
    between = (lat[:, 1] > y1) & (lat[:, 1] < y2)
    driven = between & (lat[:, 0] <= 2)
    bc = np.where(driven, 1, 0).astype(np.uint8)
    v0 = np.zeros((n, 3))
    v0[driven, 0] = v_imp
    key = "impact3d" if (nx, ny, nz, dx) == (200, 200, 9, 1e-3) else None
    w = Workload(
        name="impact3d", dim=3, mode="3d", lat=lat, dx=dx, origin=np.zeros(3),
        delta=M_RATIO * dx, vol=np.full(n, dx ** 3), specimen=np.zeros(n, np.int32),
        materials=[Material(E=191e9, nu=0.3, rho=8000.0, G0=22170.0)], bc=bc, v0=v0,
        fext=np.zeros((n, 3)), ramp_steps=0, cuts=cuts, steps=steps,
        dt=None if dt is None else np.array([dt]),
        notes=f"3D {nx}x{ny}x{nz} double-notched plate, {v_imp} m/s edge impact",
    )
    if w.dt is None and key is None:
        raise ValueError("non-default impact plate needs an explicit dt")
    return _finish(w, key)


# --------------------------------------------------------------------------
# workload 4: notched cylinder under end twist
# --------------------------------------------------------------------------

def cylinder_lattice(r: float, L: float, dx: float) -> np.ndarray:
    """Cell-centred nodes ((i+1/2)dx - r, (j+1/2)dx - r, (k+1/2)dx) inside
    the disk x^2 + y^2 <= r^2 and 0 < z <= L."""
    ni = int(math.floor(2.0 * r / dx - 0.5)) + 1
    nk = int(math.floor(L / dx - 0.5)) + 1
    i = np.arange(ni)
    xc = (i + 0.5) * dx - r
    X, Y = np.meshgrid(xc, xc, indexing="ij")
    inside = (X * X + Y * Y) <= r * r
    I, J = np.nonzero(inside)
    disk = np.stack([I, J], axis=1).astype(np.int32)
    nd = disk.shape[0]
    lat = np.empty((nd * nk, 3), dtype=np.int32)
    for k in range(nk):
        lat[k * nd:(k + 1) * nd, :2] = disk
        lat[k * nd:(k + 1) * nd, 2] = k
    return lat


def cylinder3d(dx: float = 0.6e-3, r: float = 25e-3, L: float = 100e-3, steps: int = 5000,
               dt: Optional[float] = None, twist_rate: Optional[float] = None,
               notch_depth: float = 5e-3, zc: Optional[float] = None) -> Workload:
    """Cylinder along z with a helicoidal notch of 45 degree pitch at the
    outer radius (z - zc = r * theta), radial depth ``notch_depth`` and a
    half-turn angular span; the three end layers at each end are driven with
    the linearised rigid rotation u = +-(phi(t)/2) e_z x (x, y, 0), u_z = 0,
    phi(t) = twist_rate * t (all three components prescribed)."""
    lat = cylinder_lattice(r, L, dx)
    n = lat.shape[0]
    origin = np.array([0.5 * dx - r, 0.5 * dx - r, 0.5 * dx])
    nk = int(lat[:, 2].max()) + 1
    if zc is None:
        zc = 50.37e-3 * (L / 100e-3)
    key = None
    if (dx, r, L) == (0.6e-3, 25e-3, 100e-3):
        key = "cylinder3d"
    elif (dx, r, L) == (0.5e-3, 25e-3, 100e-3):
        key = "cylinder3d_dx05"
    if twist_rate is None:
        if key is None:
            raise ValueError("non-default cylinder needs an explicit twist_rate")
        twist_rate = _param(key + "_twist_rate")
        if twist_rate is None:
            twist_rate = float("nan")
    pos = lat.astype(np.float64) * dx + origin[None, :]
    bot = lat[:, 2] < 3
    top = lat[:, 2] >= nk - 3
    bc = np.where(bot | top, 7, 0).astype(np.uint8)
    v0 = np.zeros((n, 3))
    sgn = np.where(top, 0.5, np.where(bot, -0.5, 0.0)) * twist_rate
    v0[:, 0] = -sgn * pos[:, 1]
    v0[:, 1] = sgn * pos[:, 0]
    cut = Cut("helicoid", [zc, r, r - notch_depth, 10.0 * r, -0.5 * math.pi, 0.5 * math.pi])
    w = Workload(
        name="cylinder3d", dim=3, mode="3d", lat=lat, dx=dx, origin=origin,
        delta=M_RATIO * dx, vol=np.full(n, dx ** 3), specimen=np.zeros(n, np.int32),
        materials=[Material(E=30e9, nu=0.2, rho=2400.0, G0=100.0)], bc=bc, v0=v0,
        fext=np.zeros((n, 3)), ramp_steps=0, cuts=[cut], steps=steps,
        dt=None if dt is None else np.array([dt]),
        notes=f"3D cylinder r={r*1e3:g} mm L={L*1e3:g} mm dx={dx*1e3:g} mm, helical notch, end twist",
    )
    if w.dt is None and key is None:
        raise ValueError("non-default cylinder needs an explicit dt")
    return _finish(w, key)


# --------------------------------------------------------------------------
# workload 5: batch of random 2D plane-stress plates
# --------------------------------------------------------------------------

def batch_draws(n_plates: int = 256, seed: int = 2309) -> List[dict]:
    """The random plate parameters, drawn in a fixed order per plate."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(n_plates):
        nx = int(rng.integers(50, 401))
        ny = int(rng.integers(50, 161))
        E = float(rng.uniform(50e9, 200e9))
        nu = float(rng.uniform(0.15, 0.35))
        notch_frac = float(rng.uniform(0.2, 0.6))
        row_frac = float(rng.uniform(0.3, 0.7))
        sigma = float(rng.uniform(0.5e6, 2.0e6))
        out.append(dict(nx=nx, ny=ny, E=E, nu=nu, notch_frac=notch_frac,
                        row_frac=row_frac, sigma=sigma))
    return out


def batch2d(n_plates: int = 256, seed: int = 2309, steps: int = 1000, dx: float = 0.5e-3,
            rho: float = 2440.0, G0: float = 3.8, first: int = 0,
            dt: Optional[np.ndarray] = None) -> Workload:
    """Plates ``first .. first+n_plates-1`` of the seeded batch, stacked along
    y with an 8-row gap (wider than the horizon) between neighbours."""
    draws = batch_draws(first + n_plates, seed)[first:]
    lats, specs, fexts, cuts, mats = [], [], [], [], []
    y_off = 0
    h = 1.0
    for k, d in enumerate(draws):
        nx, ny = d["nx"], d["ny"]
        lat = _box((nx, ny))
        lat[:, 1] += y_off
        notch_len = d["notch_frac"] * nx * dx
        row = int(math.floor(d["row_frac"] * ny))
        yc = (y_off + row + 0.5) * dx
        tipx = (math.floor(notch_len / dx) + 0.37) * dx
        cuts.append(Cut("segment2d", [-0.5 * dx, yc, tipx, yc], specimen=k))
        f = np.zeros((lat.shape[0], 3))
        f[lat[:, 1] == y_off, 1] = -d["sigma"] * dx * h
        f[lat[:, 1] == y_off + ny - 1, 1] = +d["sigma"] * dx * h
        lats.append(lat)
        fexts.append(f)
        specs.append(np.full(lat.shape[0], k, np.int32))
        mats.append(Material(E=d["E"], nu=d["nu"], rho=rho, G0=G0))
        y_off += ny + 8
    lat = np.concatenate(lats).astype(np.int32)
    n = lat.shape[0]
    if dt is None:
        table = _param("batch2d_dt")
        if table is not None and len(table) >= first + n_plates and seed == 2309 \
                and dx == 0.5e-3:
            dt = np.array(table[first:first + n_plates], dtype=np.float64)
        else:
            dt = np.full(n_plates, np.nan)
    return Workload(
        name="batch2d", dim=2, mode="plane_stress", lat=lat, dx=dx, origin=np.zeros(3),
        delta=M_RATIO * dx, vol=np.full(n, dx * dx * h), specimen=np.concatenate(specs),
        materials=mats, bc=np.zeros(n, np.uint8), v0=np.zeros((n, 3)),
        fext=np.concatenate(fexts), ramp_steps=0, cuts=cuts, steps=steps,
        dt=np.asarray(dt, dtype=np.float64),
        notes=f"{n_plates} random plane-stress plates (seed {seed}), {n} nodes",
    )


WORKLOAD_NAMES = ("cantilever3d", "plate2d", "impact3d", "cylinder3d", "batch2d")


def workload(name: str, **kw) -> Workload:
    return {
        "cantilever3d": cantilever3d,
        "plate2d": plate2d,
        "impact3d": impact3d,
        "cylinder3d": cylinder3d,
        "batch2d": batch2d,
    }[name](**kw)
