"""Python binding of libpd: argument marshalling between numpy/torch and the C
ABI of include/pd.h.  Every step of the solver runs in the library's HIP
kernels; this module only builds the argument structs, owns the device
buffers (torch tensors) and converts between caller and internal node order.
"""

from __future__ import annotations

import ctypes as C
from typing import Optional

import numpy as np
import torch

from . import _abi as A

_MODE = {"3d": A.PD_3D, "plane_stress": A.PD_PLANE_STRESS, "plane_strain": A.PD_PLANE_STRAIN}


def _np(a) -> C.c_void_p:
    return a.ctypes.data_as(C.c_void_p)


def _tp(t: Optional[torch.Tensor]):
    return C.c_void_p(t.data_ptr()) if t is not None else None


class Context:
    def __init__(self, device: int = 0):
        L = A.load()
        torch.cuda.set_device(device)
        self.device = device
        self.stream = torch.cuda.current_stream(device)
        h = C.c_void_p()
        st = L.pd_ctx_create(C.byref(h), device, C.c_void_p(self.stream.cuda_stream))
        A.check("pd_ctx_create", st)
        self.h = h

    def __del__(self):
        try:
            if getattr(self, "h", None):
                A.load().pd_ctx_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def check(self, fn, status):
        A.check(fn, status, self.h)


def critical_stretch(mode: str, E: float, nu: float, G0, delta: float, variant: int = 0) -> float:
    out = C.c_double()
    g = float("nan") if G0 is None else float(G0)
    A.check("pd_critical_stretch", A.load().pd_critical_stretch(_MODE[mode], E, nu, g, delta, variant,
                                                                  C.byref(out)))
    return out.value


def specimen_params(mode: str, E, nu, rho, s0, dt) -> A.pd_spec:
    sp = A.pd_spec()
    A.check("pd_specimen_params", A.load().pd_specimen_params(_MODE[mode], E, nu, rho, s0, dt, C.byref(sp)))
    return sp


class FamilyHost:
    """Result of pd_build_family (host arrays, internal order)."""

    def __init__(self, lat, dx, origin, delta, vol, specimen=None, cuts=None):
        L = A.load()
        lat = np.ascontiguousarray(lat, dtype=np.int32)
        n, dim = lat.shape
        self._lat = lat
        self._vol = np.ascontiguousarray(vol, dtype=np.float64)
        self._spec = None if specimen is None else np.ascontiguousarray(specimen, dtype=np.int32)
        body = A.pd_body()
        body.n, body.dim = n, dim
        body.lat = _np(self._lat)
        body.dx = float(dx)
        for c in range(3):
            body.origin[c] = float(origin[c])
        body.delta = float(delta)
        body.vol = _np(self._vol)
        body.specimen = _np(self._spec) if self._spec is not None else None
        cuts = list(cuts or [])
        carr = (A.pd_cut * max(1, len(cuts)))()
        for k, ct in enumerate(cuts):
            carr[k].kind = {"segment2d": 0, "rect3d": 1, "helicoid": 2}[ct.kind]
            carr[k].specimen = int(ct.specimen)
            for q, v in enumerate(ct.p):
                carr[k].p[q] = float(v)
        sizes = A.pd_family_sizes()
        A.check("pd_build_family", L.pd_build_family(C.byref(body), C.cast(carr, C.c_void_p), len(cuts),
                                                     C.byref(sizes), None))
        s = sizes
        self.sizes = s
        self.perm = np.empty(s.n_pad, np.int32)
        self.row_of = np.empty(s.n, np.int32)
        self.slice_ptr = np.empty(s.n_slices + 1, np.int64)
        self.words = np.empty(s.n_words, np.uint32)
        self.mask = np.empty(s.n_mask, np.uint64)
        self.stencil = np.empty(s.n_stencil * 4, np.float64)
        self.stencil_off = np.empty(s.n_stencil * 3, np.int32)
        self.vol = np.empty(s.n_pad, np.float64)
        self.inv_m = np.empty(s.n_pad, np.float64)
        self.spec = np.empty(s.n_pad, np.int32)
        self.lat4 = np.empty(s.n_pad * 4, np.int32)
        self.tile_org = np.empty(s.n_tiles * 4, np.int32)
        self.tile_nbr = np.empty(s.n_tiles * 27, np.int32)
        self.ktab = np.empty(128 * 20, np.uint32)
        self.halo_map = np.empty(max(1, s.n_halo), np.int16)
        self.halo_pos = np.empty(max(1, s.n_box), np.int32)
        hb = A.pd_family_host(_np(self.perm), _np(self.row_of), _np(self.slice_ptr), _np(self.words),
                              _np(self.mask), _np(self.stencil), _np(self.stencil_off), _np(self.vol),
                              _np(self.inv_m), _np(self.spec), _np(self.lat4), _np(self.tile_org),
                              _np(self.tile_nbr), _np(self.ktab), _np(self.halo_map),
                              _np(self.halo_pos))
        self._hb = hb
        A.check("pd_build_family", L.pd_build_family(C.byref(body), C.cast(carr, C.c_void_p), len(cuts),
                                                     C.byref(sizes), C.byref(hb)))

        self.supertiles()

    def supertiles(self):
        """pd_build_supertiles: st_tiles, st_nbr, st_pos, st_ktab (None where the
        family has no super-tiles: tiles other than 4x4x4 in 3D or 8x8 in 2D,
        or reach above 3)."""
        self.st_tiles = self.st_nbr = self.st_pos = self.st_ktab = None
        self.n_st, self.st_n_pos = 0, 0
        L = A.load()
        ss = A.pd_st_sizes()
        st = L.pd_build_supertiles(C.byref(self.sizes), C.byref(self._hb), C.byref(ss), None, None, None, None)
        if st == -5:  # PD_ERR_UNSUPPORTED
            return
        A.check("pd_build_supertiles", st)
        self.st_tiles = np.empty(4 * ss.n_st, np.int32)
        self.st_nbr = np.empty(48 * ss.n_st, np.int32)
        self.st_pos = np.empty(ss.n_pos, np.int32)
        self.st_ktab = np.empty(128 * 8, np.uint32)
        A.check("pd_build_supertiles", L.pd_build_supertiles(C.byref(self.sizes), C.byref(self._hb), C.byref(ss),
                                                             _np(self.st_tiles), _np(self.st_nbr),
                                                             _np(self.st_pos), _np(self.st_ktab)))
        self.n_st, self.st_n_pos = int(ss.n_st), int(ss.n_pos)

    @property
    def n(self):
        return int(self.sizes.n)

    def bond_table(self):
        """Every directed bond as (row, k, caller i, caller j, stencil id) arrays."""
        s = self.sizes
        rows, ks, wi = [], [], []
        for sl in range(s.n_slices):
            b0, b1 = self.slice_ptr[sl], self.slice_ptr[sl + 1]
            L = (b1 - b0) // 64
            if L == 0:
                continue
            # groups of four words per lane: index (k // 4, lane, k % 4)
            w = self.words[b0:b1].reshape(L // 4, 64, 4)
            g, lane, c = np.nonzero((w & 127) != 127)
            k = 4 * g + c
            rows.append(sl * 64 + lane)
            ks.append(k)
            wi.append(b0 + g * 256 + lane * 4 + c)
        rows = np.concatenate(rows) if rows else np.zeros(0, np.int64)
        ks = np.concatenate(ks) if ks else np.zeros(0, np.int64)
        wi = np.concatenate(wi) if wi else np.zeros(0, np.int64)
        words = self.words[wi]
        j = (words >> 7).astype(np.int64)
        return rows.astype(np.int64), ks.astype(np.int64), self.perm[rows], self.perm[j], (words & 127)

    def status_index(self, bi: np.ndarray, bj: np.ndarray):
        """Where the status bit of each unique bond (caller nodes bi < bj)
        sits: (mask word index, bit lane) of its directed copy i -> j."""
        rows, ks, ci, cj, _ = self.bond_table()
        fwd = ci < cj
        n = int(max(int(ci.max(initial=0)), int(cj.max(initial=0)))) + 1
        key = ci[fwd].astype(np.int64) * n + cj[fwd]
        want = np.asarray(bi, np.int64) * n + np.asarray(bj, np.int64)
        order = np.argsort(key, kind="stable")
        pos = order[np.clip(np.searchsorted(key[order], want), 0, max(0, key.size - 1))]
        if key.size == 0 or not np.array_equal(key[pos], want):
            raise KeyError("a bond is not in the family")
        r, k = rows[fwd][pos], ks[fwd][pos]
        return self.slice_ptr[r // 64] // 64 + k, (r % 64).astype(np.uint64)

    def cleared_keys(self, mask0: np.ndarray, mask: np.ndarray) -> np.ndarray:
        """Sorted keys i * n + j (caller nodes, i < j) of the bonds whose
        status bits are set in mask0 and clear in mask; raises if the two
        directed copies of such a bond disagree."""
        cleared = mask0 & ~mask
        wi = np.nonzero(cleared)[0]
        if wi.size == 0:
            return np.zeros(0, np.int64)
        bits = (cleared[wi][:, None] >> np.arange(64, dtype=np.uint64)[None, :]) & np.uint64(1)
        wsel, lane = np.nonzero(bits)
        word = wi[wsel].astype(np.int64)
        first = self.slice_ptr // 64
        sl = np.searchsorted(first, word, side="right") - 1
        k = word - first[sl]
        widx = self.slice_ptr[sl] + (k >> 2) * 256 + lane * 4 + (k & 3)
        row = sl * 64 + lane
        ci = self.perm[row].astype(np.int64)
        cj = self.perm[(self.words[widx] >> 7).astype(np.int64)].astype(np.int64)
        n = self.n
        key = np.minimum(ci, cj) * n + np.maximum(ci, cj)
        u, cnt = np.unique(key, return_counts=True)
        if np.any(cnt != 2):
            raise AssertionError("directed bond copies disagree on their status")
        return u

    def bond_status(self, mask: np.ndarray):
        """Status of every unique bond, sorted by caller (i, j) with i < j.

        Returns (bi, bj, status) and raises if the two directed copies of a
        bond disagree."""
        rows, ks, ci, cj, _ = self.bond_table()
        slice_of = rows // 64
        lane = rows % 64
        widx = self.slice_ptr[slice_of] // 64 + ks
        bit = ((mask[widx] >> lane.astype(np.uint64)) & np.uint64(1)).astype(np.uint8)
        lo, hi = np.minimum(ci, cj), np.maximum(ci, cj)
        order = np.lexsort((hi, lo))
        lo, hi, bit, fwd = lo[order], hi[order], bit[order], (ci < cj)[order]
        # pairs appear twice (once per direction), adjacent after sorting
        a_lo, a_hi, a_bit = lo[0::2], hi[0::2], bit[0::2]
        if not (np.array_equal(a_lo, lo[1::2]) and np.array_equal(a_hi, hi[1::2])):
            raise AssertionError("directed bond copies are not paired")
        if not np.array_equal(a_bit, bit[1::2]):
            raise AssertionError("directed bond copies disagree on their status")
        return a_lo.astype(np.int32), a_hi.astype(np.int32), a_bit


class Solver:
    """One workload on one GPU: family, problem, state (and optionally K)."""

    def __init__(self, w, device: int = 0, s0: Optional[np.ndarray] = None,
                 dt: Optional[np.ndarray] = None, fp32_state: bool = True, ctx: Optional[Context] = None,
                 u0: Optional[np.ndarray] = None, family: Optional[FamilyHost] = None):
        self.w = w
        self.ctx = ctx or Context(device)
        self.dev = torch.device("cuda", self.ctx.device)
        self.fam = family or FamilyHost(w.lat, w.dx, w.origin, w.delta, w.vol, w.specimen, w.cuts)
        s = self.fam.sizes
        self.n, self.n_pad = int(s.n), int(s.n_pad)
        d = self.dev
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(d)
        self.slice_ptr = t(self.fam.slice_ptr)
        self.words = t(self.fam.words.view(np.int32))
        self.stencil = t(self.fam.stencil)
        self.vol = t(self.fam.vol)
        self.inv_m = t(self.fam.inv_m)
        self.lat4 = t(self.fam.lat4)
        self.perm = t(self.fam.perm)
        self.spec_rows = t(self.fam.spec)
        self.mask0 = self.fam.mask.copy()
        # specimen table
        ns = max(w.n_specimens, int(s.n_specimens))
        dts = np.asarray(w.dt if dt is None else dt, dtype=np.float64).reshape(-1)
        if dts.size == 1 and ns > 1:
            dts = np.full(ns, dts[0])
        self.s0 = np.zeros(ns)
        spec = (A.pd_spec * ns)()
        for k in range(ns):
            mat = w.materials[k]
            sk = critical_stretch(w.mode, mat.E, mat.nu, mat.G0, w.delta, w.s0_variant) \
                if s0 is None else float(np.asarray(s0).reshape(-1)[k])
            self.s0[k] = sk
            spec[k] = specimen_params(w.mode, mat.E, mat.nu, mat.rho, sk, float(dts[k]))
        self.dt = dts
        self.spec = t(np.frombuffer(bytes(spec), dtype=np.float64).copy())
        self.aux = torch.zeros(self.n_pad, dtype=torch.int32, device=d)
        self.fext = torch.zeros(self.n_pad * 4, dtype=torch.float64, device=d)
        P = A.pd_problem_dev()
        P.n_pad, P.n_slices, P.dim = self.n_pad, int(s.n_slices), int(s.dim)
        P.n_stencil, P.n_specimens = int(s.n_stencil), ns
        P.slice_ptr, P.words, P.stencil = _tp(self.slice_ptr), _tp(self.words), _tp(self.stencil)
        P.vol, P.inv_m, P.lat4, P.spec = _tp(self.vol), _tp(self.inv_m), _tp(self.lat4), _tp(self.spec)
        P.aux, P.fext = _tp(self.aux), _tp(self.fext)
        P.ramp_steps = int(w.ramp_steps)
        self.stencil_off = t(self.fam.stencil_off)
        self.tile_nbr = t(self.fam.tile_nbr)
        P.stencil_off, P.tile_nbr = _tp(self.stencil_off), _tp(self.tile_nbr)
        self.ktab = t(self.fam.ktab.view(np.int32))
        P.ktab = _tp(self.ktab)
        self.halo_map = t(self.fam.halo_map)
        P.halo_map = _tp(self.halo_map)
        self.halo_pos = t(self.fam.halo_pos)
        P.halo_pos = _tp(self.halo_pos)
        P.n_pos = int(s.n_box)
        P.vol_uniform = float(s.vol_uniform)
        for c in range(3):
            P.tile[c] = int(s.tile[c])
        P.reach = int(s.reach)
        if self.fam.st_tiles is not None:
            self.st_tiles, self.st_nbr = t(self.fam.st_tiles), t(self.fam.st_nbr)
            self.st_pos, self.st_ktab = t(self.fam.st_pos), t(self.fam.st_ktab.view(np.int32))
            P.st_tiles, P.st_nbr = _tp(self.st_tiles), _tp(self.st_nbr)
            P.st_pos, P.st_ktab = _tp(self.st_pos), _tp(self.st_ktab)
            P.n_st, P.st_n_pos = self.fam.n_st, self.fam.st_n_pos
        self.P = P
        # state
        self.uv = [torch.zeros(self.n_pad * 4, dtype=torch.float64, device=d) for _ in range(2)]
        self.vel = torch.zeros(self.n_pad * 4, dtype=torch.float64, device=d)
        self.qr = torch.zeros(self.n_pad * 2, dtype=torch.float64, device=d)
        self.mask = t(self.mask0.view(np.int64))
        self.ush = [torch.zeros(self.n_pad * 4, dtype=torch.int32, device=d) for _ in range(2)] \
            if fp32_state else [None, None]
        self.qr32 = torch.zeros(self.n_pad * 2, dtype=torch.float32, device=d) if fp32_state else None
        self.dsum = torch.zeros(self.n_pad * 4, dtype=torch.float64, device=d) if fp32_state else None
        self.fe32 = torch.zeros(self.n_pad * 4, dtype=torch.float32, device=d) if fp32_state else None
        self.qv32 = torch.zeros(self.n_pad * 2, dtype=torch.float32, device=d) if fp32_state else None
        self.fe64 = torch.zeros(self.n_pad * 4, dtype=torch.float64, device=d)
        self.ctl = torch.zeros(A.PD_CTL_BYTES // 8, dtype=torch.int64, device=d)
        S = A.pd_state_dev()
        S.uv[0], S.uv[1] = self.uv[0].data_ptr(), self.uv[1].data_ptr()
        S.vel, S.qr, S.mask = _tp(self.vel), _tp(self.qr), _tp(self.mask)
        S.fe64 = _tp(self.fe64)
        if fp32_state:
            S.ush[0], S.ush[1] = self.ush[0].data_ptr(), self.ush[1].data_ptr()
            S.qr32 = _tp(self.qr32)
            S.dsum = _tp(self.dsum)
            S.fe32 = _tp(self.fe32)
            S.qv32 = _tp(self.qv32)
        S.ctl = _tp(self.ctl)
        S.cur = 0
        self.S = S
        self.K = None
        self.F = None
        self.reset(u0=u0)

    # ---- state -----------------------------------------------------------
    def reset(self, u0: Optional[np.ndarray] = None, v0: Optional[np.ndarray] = None, start_step: int = 0,
              mask: Optional[np.ndarray] = None):
        d = self.dev
        w = self.w
        u0t = None if u0 is None else torch.from_numpy(np.ascontiguousarray(u0, np.float64).reshape(-1)).to(d)
        v0a = w.v0 if v0 is None else v0
        v0t = torch.from_numpy(np.ascontiguousarray(v0a, np.float64).reshape(-1)).to(d)
        bct = torch.from_numpy(np.ascontiguousarray(w.bc, np.uint8)).to(d)
        ft = torch.from_numpy(np.ascontiguousarray(w.fext, np.float64).reshape(-1)).to(d)
        self._init_keep = (u0t, v0t, bct, ft)
        m = self.mask0 if mask is None else mask
        self.mask.copy_(torch.from_numpy(np.ascontiguousarray(m).view(np.int64)).to(d))
        self.S.cur = 0
        L = A.load()
        self.ctx.check("pd_state_init", L.pd_state_init(
            self.ctx.h, C.byref(self.P), _tp(self.perm), self.n, _tp(u0t), _tp(v0t), _tp(bct), _tp(ft),
            _tp(self.spec_rows), _tp(self.aux), _tp(self.fext), C.byref(self.S), int(start_step)))
        if self.K is not None:
            self.K.assembled = 0
        if self.F is not None:
            self.F.assembled = 0

    def read(self):
        d = self.dev
        u = torch.empty(self.n * 3, dtype=torch.float64, device=d)
        v = torch.empty(self.n * 3, dtype=torch.float64, device=d)
        self.ctx.check("pd_state_read", A.load().pd_state_read(self.ctx.h, C.byref(self.P), _tp(self.perm),
                                                                 self.n, C.byref(self.S), _tp(u), _tp(v)))
        torch.cuda.synchronize(d)
        return u.cpu().numpy().reshape(self.n, 3), v.cpu().numpy().reshape(self.n, 3)

    def step_count(self) -> int:
        out = C.c_int64()
        self.ctx.check("pd_get_step", A.load().pd_get_step(self.ctx.h, C.byref(self.S), C.byref(out)))
        return int(out.value)

    def broken_keys(self) -> np.ndarray:
        """Sorted keys i * n + j (caller nodes, i < j) of the bonds broken by
        the steps since the initial status (notch cuts excluded)."""
        return self.fam.cleared_keys(self.mask0, self.mask_host())

    def mask_host(self) -> np.ndarray:
        torch.cuda.synchronize(self.dev)
        return self.mask.cpu().numpy().view(np.uint64).copy()

    def bond_status(self):
        return self.fam.bond_status(self.mask_host())

    # ---- operators ---------------------------------------------------------
    def _to_caller(self, t4: torch.Tensor) -> np.ndarray:
        a = t4.view(self.n_pad, 4)[:, :3].cpu().numpy()
        out = np.empty((self.n, 3))
        real = self.fam.perm >= 0
        out[self.fam.perm[real]] = a[real]
        return out

    def _rows_to_caller(self, t1: torch.Tensor) -> np.ndarray:
        a = t1.cpu().numpy()
        out = np.empty(self.n)
        real = self.fam.perm >= 0
        out[self.fam.perm[real]] = a[real]
        return out

    def force(self, precision: str = "fp64"):
        """Internal force and dilatation of the current state (caller order)."""
        f = torch.zeros(self.n_pad * 4, dtype=torch.float64, device=self.dev)
        th = torch.zeros(self.n_pad, dtype=torch.float64, device=self.dev)
        prec = {"fp64": A.PD_FP64, "fp32": A.PD_FP32_RECHECK}[precision]
        self.ctx.check("pd_force", A.load().pd_force(self.ctx.h, C.byref(self.P), C.byref(self.S), prec,
                                                       _tp(f), _tp(th)))
        torch.cuda.synchronize(self.dev)
        return self._to_caller(f), self._rows_to_caller(th)

    def force_finite(self):
        """Force and dilatation with the finite extension (Eqs. 1.10, 1.13)."""
        f = torch.zeros(self.n_pad * 4, dtype=torch.float64, device=self.dev)
        th = torch.zeros(self.n_pad, dtype=torch.float64, device=self.dev)
        self.ctx.check("pd_force_finite", A.load().pd_force_finite(self.ctx.h, C.byref(self.P), C.byref(self.S),
                                                                     _tp(f), _tp(th)))
        torch.cuda.synchronize(self.dev)
        return self._to_caller(f), self._rows_to_caller(th)

    def autotune(self, precision: str = "fp32", trial_steps: int = 20, cache: Optional[str] = None) -> dict:
        """Pick the fastest kernel variant / block size (pd_autotune).  With a
        cache path, results are stored in a JSON file keyed by
        (gfx arch, dim, tile shape, stencil size, precision) and reused.
        Tuning advances the state; the state is reset afterwards."""
        import json
        import os
        s = self.fam.sizes
        key = f"gfx950/d{int(s.dim)}/t{'x'.join(str(int(v)) for v in s.tile)}/s{int(s.n_stencil)}/{precision}"
        data = {}
        if cache and os.path.exists(cache):
            with open(cache) as f:
                data = json.load(f)
            if key in data:
                return data[key]
        r = A.pd_tune_result()
        prec = {"fp64": A.PD_FP64, "fp32": A.PD_FP32_RECHECK}[precision]
        self.ctx.check("pd_autotune", A.load().pd_autotune(self.ctx.h, C.byref(self.P), C.byref(self.S), prec,
                                                             int(trial_steps), C.byref(r)))
        res = dict(kernel={0: "auto", 1: "gather", 2: "tiled", 3: "super", 4: "tiled1"}[r.kernel], block=int(r.block),
                   ms_per_step=r.ms_per_step,
                   candidates=[dict(kernel=int(r.cand_kernel[i]), block=int(r.cand_block[i]),
                                    ms=r.cand_ms[i]) for i in range(r.n_candidates)])
        self.reset()
        if cache:
            data[key] = res
            os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
            with open(cache, "w") as f:
                json.dump(data, f, indent=1)
        return res

    def tiled_supported(self, precision: str = "fp32") -> bool:
        """Whether kernel='auto' runs the LDS-staged tile kernels (pd_tile_kernels_apply)."""
        yes = C.c_int32(0)
        self.ctx.check("pd_tile_kernels_apply", A.load().pd_tile_kernels_apply(
            C.byref(self.P), C.byref(self.S), {"fp64": A.PD_FP64, "fp32": A.PD_FP32_RECHECK}[precision],
            C.byref(yes)))
        return bool(yes.value)

    def profile_read(self, reset: bool = True) -> dict:
        p = A.pd_profile_stats()
        self.ctx.check("pd_profile_read", A.load().pd_profile_read(self.ctx.h, C.byref(p), 1 if reset else 0))
        return dict(steps=p.steps, ms_pass1=p.ms_pass1, ms_pass2=p.ms_pass2, ms_extra=p.ms_extra)

    def step(self, nsteps: int, precision: str = "fp64", form: str = "mf", graph_chunk: int = 0,
             block: int = 0, check_every: int = 0, report: bool = True, profile: bool = False,
             kernel: str = "auto", extension: str = "linear", energy_check: bool = False,
             energy_growth: float = 0.0):
        o = A.pd_step_opts()
        o.precision = {"fp64": A.PD_FP64, "fp32": A.PD_FP32_RECHECK}[precision]
        o.form = {"mf": A.PD_MATRIX_FREE, "bsr": A.PD_BSR, "fac": A.PD_FACTORED}[form]
        o.graph_chunk, o.block, o.check_every = int(graph_chunk), int(block), int(check_every)
        o.profile = 1 if profile else 0
        o.kernel = {"auto": 0, "gather": 1, "tiled": 2, "super": 3, "tiled1": 4}[kernel]
        o.extension = {"linear": 0, "finite": 1}[extension]
        o.energy_check = 1 if energy_check else 0
        o.energy_growth = float(energy_growth)
        rep = A.pd_step_report()
        if form == "fac":
            Fp = C.byref(self.F) if self.F is not None else None
            self.ctx.check("pd_fac_step", A.load().pd_fac_step(self.ctx.h, C.byref(self.P), C.byref(self.S),
                                                               int(nsteps), C.byref(o), Fp,
                                                               C.byref(rep) if report else None))
        else:
            Kp = C.byref(self.K) if self.K is not None else None
            self.ctx.check("pd_step", A.load().pd_step(self.ctx.h, C.byref(self.P), C.byref(self.S), int(nsteps),
                                                         C.byref(o), Kp, C.byref(rep) if report else None))
        if not report:
            return None
        return dict(step=rep.step, broken_total=rep.broken_total, rechecks=rep.rechecks,
                    nonfinite=rep.nonfinite, umax=rep.umax, min_margin=rep.min_margin, kinetic=rep.kinetic,
                    strain=rep.strain, energy_step=rep.energy_step)

    def damage(self) -> np.ndarray:
        phi = torch.zeros(self.n_pad, dtype=torch.float64, device=self.dev)
        self.ctx.check("pd_damage", A.load().pd_damage(self.ctx.h, C.byref(self.P), _tp(self.mask), _tp(phi)))
        torch.cuda.synchronize(self.dev)
        return self._rows_to_caller(phi)

    def energy(self):
        f = torch.zeros(self.n_pad * 4, dtype=torch.float64, device=self.dev)
        k, s = C.c_double(), C.c_double()
        self.ctx.check("pd_energy", A.load().pd_energy(self.ctx.h, C.byref(self.P), C.byref(self.S), _tp(f),
                                                         C.byref(k), C.byref(s)))
        return k.value, s.value

    def energy_noalloc(self, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """pd_energy_noalloc: (kinetic, strain) into a device tensor of two
        doubles, enqueued on the context's stream without synchronising."""
        if out is None:
            out = torch.empty(2, dtype=torch.float64, device=self.dev)
        self.ctx.check("pd_energy_noalloc", A.load().pd_energy_noalloc(self.ctx.h, C.byref(self.P),
                                                                         C.byref(self.S), _tp(out)))
        return out

    def stable_dt(self, iters: int = 500, seed: int = 0) -> float:
        f = torch.zeros(self.n_pad * 4, dtype=torch.float64, device=self.dev)
        out = C.c_double()
        self.ctx.check("pd_stable_dt", A.load().pd_stable_dt(self.ctx.h, C.byref(self.P), C.byref(self.S),
                                                               _tp(f), int(iters), C.c_uint64(seed),
                                                               C.byref(out)))
        return out.value

    # ---- block-sparse stiffness --------------------------------------------
    def build_K(self, fp32: bool = False):
        L = A.load()
        bs = A.pd_bsr_sizes()
        A.check("pd_bsr_pattern", L.pd_bsr_pattern(C.byref(self.fam.sizes), C.byref(self.fam._hb), C.byref(bs),
                                                     None, None))
        row_ptr = np.empty(self.n_pad + 1, np.int64)
        col = np.empty(max(1, bs.nnzb), np.int32)
        A.check("pd_bsr_pattern", L.pd_bsr_pattern(C.byref(self.fam.sizes), C.byref(self.fam._hb), C.byref(bs),
                                                     _np(row_ptr), _np(col)))
        d = self.dev
        dim = int(self.fam.sizes.dim)
        self.K_row_ptr = torch.from_numpy(row_ptr).to(d)
        self.K_col = torch.from_numpy(col).to(d)
        self.K_vals = torch.zeros(max(1, bs.nnzb) * dim * dim, dtype=torch.float32 if fp32 else torch.float64,
                                  device=d)
        self.K_bc = torch.zeros(self.n_pad * 8, dtype=torch.float64, device=d)
        self.K_dirty = torch.zeros(self.n_pad, dtype=torch.int32, device=d)
        K = A.pd_bsr_dev()
        K.nnzb, K.dim, K.fp32 = bs.nnzb, dim, 1 if fp32 else 0
        K.max_row_blocks, K.reach = bs.max_row_blocks, bs.reach
        K.row_ptr, K.col, K.vals = _tp(self.K_row_ptr), _tp(self.K_col), _tp(self.K_vals)
        K.bc, K.dirty = _tp(self.K_bc), _tp(self.K_dirty)
        self.K = K
        self.K_sizes = bs
        return bs

    def assemble_K(self):
        self.ctx.check("pd_assemble_K", A.load().pd_assemble_K(self.ctx.h, C.byref(self.P), _tp(self.mask),
                                                                 C.byref(self.K)))

    def static_solve(self, tol: float = 1e-12, max_iter: int = 20000, check_every: int = 50,
                     matrix_free: bool = False, use_K: bool = True) -> dict:
        """Static equilibrium from the current state with the assembled
        double K (pd_static_solve); the solution replaces u.  matrix_free:
        the CG products by the double force kernels; use_K=False (with
        matrix_free) passes no K at all."""
        L = A.load()
        nw = int(L.pd_static_workspace(self.n_pad))
        if getattr(self, "_cg_work", None) is None or self._cg_work.numel() < nw:
            self._cg_work = torch.zeros(nw, dtype=torch.float64, device=self.dev)
        o = A.pd_cg_opts(float(tol), int(max_iter), int(check_every), 1 if matrix_free else 0, 0)
        rep = A.pd_cg_report()
        Kp = C.byref(self.K) if use_K else None
        self.ctx.check("pd_static_solve", L.pd_static_solve(self.ctx.h, C.byref(self.P), Kp,
                                                              C.byref(self.S), C.byref(o), _tp(self._cg_work),
                                                              C.byref(rep)))
        return dict(iterations=rep.iterations, converged=bool(rep.converged), rel_residual=rep.rel_residual)

    def newmark_step(self, nsteps: int, dt: float, breaking: bool = False, tol: float = 1e-12,
                     max_iter: int = 20000, check_every: int = 50, matrix_free: bool = False,
                     use_K: bool = True) -> dict:
        """nsteps implicit average-acceleration Newmark steps with the
        assembled double K (pd_newmark_step); the state advances in place."""
        L = A.load()
        nw = int(L.pd_newmark_workspace(self.n_pad))
        if getattr(self, "_nm_work", None) is None or self._nm_work.numel() < nw:
            self._nm_work = torch.zeros(nw, dtype=torch.float64, device=self.dev)
        o = A.pd_newmark_opts(float(dt), A.pd_cg_opts(float(tol), int(max_iter), int(check_every),
                                                    1 if matrix_free else 0, 0),
                              1 if breaking else 0, 0)
        rep = A.pd_cg_report()
        Kp = C.byref(self.K) if use_K else None
        self.ctx.check("pd_newmark_step", L.pd_newmark_step(self.ctx.h, C.byref(self.P), Kp,
                                                              C.byref(self.S), int(nsteps), C.byref(o),
                                                              _tp(self._nm_work), C.byref(rep)))
        return dict(iterations=rep.iterations, converged=bool(rep.converged), rel_residual=rep.rel_residual)

    def bsr_apply(self):
        f = torch.zeros(self.n_pad * 4, dtype=torch.float64, device=self.dev)
        self.ctx.check("pd_bsr_apply", A.load().pd_bsr_apply(self.ctx.h, C.byref(self.P), C.byref(self.K),
                                                               C.byref(self.S), _tp(f)))
        torch.cuda.synchronize(self.dev)
        return self._to_caller(f)

    # ---- factored matrix scheme ------------------------------------------
    def build_factored(self):
        """Bond numbering and index arrays (pd_fac_pattern), device buffers of
        the four operators; call assemble_factored() afterwards."""
        L = A.load()
        fs = A.pd_fac_sizes()
        A.check("pd_fac_pattern", L.pd_fac_pattern(C.byref(self.fam.sizes), C.byref(self.fam._hb), C.byref(fs),
                                                     None, None, None))
        nb, nw = int(fs.nb), int(fs.n_words)
        bond_ij = np.empty(2 * max(1, nb), np.int32)
        bond_pos = np.empty(2 * max(1, nb), np.int32)
        bid = np.empty(nw, np.int32)
        A.check("pd_fac_pattern", L.pd_fac_pattern(C.byref(self.fam.sizes), C.byref(self.fam._hb), C.byref(fs),
                                                     _np(bond_ij), _np(bond_pos), _np(bid)))
        d, dim = self.dev, int(self.fam.sizes.dim)
        f64 = dict(dtype=torch.float64, device=d)
        self.F_bond_ij = torch.from_numpy(bond_ij).to(d)
        self.F_bond_pos = torch.from_numpy(bond_pos).to(d)
        self.F_bid = torch.from_numpy(bid).to(d)
        self.F_ce = torch.zeros(2 * dim * max(1, nb), **f64)
        self.F_xi = torch.zeros(max(1, nb), **f64)
        self.F_cth = torch.zeros(nw, **f64)
        self.F_ke = torch.zeros(dim * nw, **f64)
        self.F_kth = torch.zeros(dim * nw, **f64)
        self.F_kdiag = torch.zeros(4 * self.n_pad, **f64)
        self.F_E = torch.zeros(max(1, nb), **f64)
        self.F_theta = torch.zeros(self.n_pad, **f64)
        self.F_dirty = torch.zeros(self.n_pad, dtype=torch.int32, device=d)
        F = A.pd_fac_dev()
        F.nb, F.n_words, F.dim = nb, nw, dim
        F.bond_ij, F.bond_pos, F.bid = _tp(self.F_bond_ij), _tp(self.F_bond_pos), _tp(self.F_bid)
        F.ce, F.xi, F.cth, F.ke = _tp(self.F_ce), _tp(self.F_xi), _tp(self.F_cth), _tp(self.F_ke)
        F.kth, F.kth_diag = _tp(self.F_kth), _tp(self.F_kdiag)
        F.E, F.theta, F.dirty = _tp(self.F_E), _tp(self.F_theta), _tp(self.F_dirty)
        self.F = F
        self.F_sizes = fs
        return fs

    def assemble_factored(self):
        self.ctx.check("pd_fac_assemble", A.load().pd_fac_assemble(self.ctx.h, C.byref(self.P), _tp(self.mask),
                                                                     C.byref(self.F)))

    def fac_apply(self):
        """(f, theta, E) of the factored products for the current state: f and
        theta in caller order, E per bond in the library's bond numbering."""
        f = torch.zeros(self.n_pad * 4, dtype=torch.float64, device=self.dev)
        self.ctx.check("pd_fac_apply", A.load().pd_fac_apply(self.ctx.h, C.byref(self.P), C.byref(self.F),
                                                               C.byref(self.S), _tp(f)))
        torch.cuda.synchronize(self.dev)
        nb = int(self.F.nb)
        return self._to_caller(f), self._rows_to_caller(self.F_theta), self.F_E[:nb].cpu().numpy()

    def fac_bonds(self):
        """Caller node pair (i, j) of every bond in the library's numbering."""
        nb = int(self.F.nb)
        ij = self.F_bond_ij[:2 * nb].cpu().numpy().reshape(nb, 2)
        return self.fam.perm[ij[:, 0]], self.fam.perm[ij[:, 1]]

    # ---- adaptive dynamic relaxation -------------------------------------
    def adr_setup(self, dt: float = 1.0):
        """Buffers of the relaxation and its fictitious density for the
        current bond status (pd_adr_density); the next adr_step starts the
        relaxation.  The state (u, v) is whatever reset() left."""
        d, n4 = self.dev, self.n_pad * 4
        f64 = dict(dtype=torch.float64, device=d)
        self.R_lambda = torch.zeros(n4, **f64)
        self.R_fprev = torch.zeros(n4, **f64)
        self.R_fint = torch.zeros(n4, **f64)
        self.R_partial = torch.zeros(4 * ((self.n_pad + 255) // 256), **f64)
        self.R_stats = torch.zeros(8, **f64)
        R = A.pd_adr_dev()
        R.dt = float(dt)
        R.lambda_, R.f_prev, R.f_int = _tp(self.R_lambda), _tp(self.R_fprev), _tp(self.R_fint)
        R.partial, R.stats = _tp(self.R_partial), _tp(self.R_stats)
        self.R = R
        self.ctx.check("pd_adr_density", A.load().pd_adr_density(self.ctx.h, C.byref(self.P), _tp(self.mask),
                                                                   C.byref(self.R)))

    def adr_step(self, nsteps: int, graph_chunk: int = 0, kernel: str = "auto", report: bool = True,
                 profile: bool = False, check_every: int = 0, extension: str = "linear"):
        o = A.pd_step_opts()
        o.precision, o.form = A.PD_FP64, A.PD_MATRIX_FREE
        o.extension = {"linear": 0, "finite": 1}[extension]
        o.graph_chunk, o.check_every = int(graph_chunk), int(check_every)
        o.profile = 1 if profile else 0
        o.kernel = {"auto": 0, "gather": 1, "tiled": 2, "super": 3, "tiled1": 4}[kernel]
        rep = A.pd_step_report()
        self.ctx.check("pd_adr_step", A.load().pd_adr_step(self.ctx.h, C.byref(self.P), C.byref(self.S),
                                                             int(nsteps), C.byref(o), C.byref(self.R),
                                                             C.byref(rep) if report else None))
        if not report:
            return None
        return dict(step=rep.step, broken_total=rep.broken_total, nonfinite=rep.nonfinite)

    def adr_stats(self) -> dict:
        torch.cuda.synchronize(self.dev)
        s = self.R_stats.cpu().numpy()
        return dict(c=s[0], ukU=s[1], uu=s[2], res2=s[3], first=s[4], iterations=int(s[5]))

    def adr_lambda(self) -> np.ndarray:
        torch.cuda.synchronize(self.dev)
        return self._to_caller(self.R_lambda)
