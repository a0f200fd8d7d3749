"""CPU-side checks of libpd: it loads, exports every declared entry point,
and its host-side set-up (family search, notch cuts, weighted volume,
constants, block pattern, argument checks) agrees with the CPU reference.
No GPU compute call is made here."""

import ctypes as C
import math
import os
import re

import numpy as np
import pytest

import oracle
from oracle import Oracle
from pd_inputs import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_2309_11273_amd import _abi
    if not os.path.exists(_abi.LIB_PATH):
        from paper_2309_11273_amd import build
        build.build()
    return _abi.load()


def test_exports_every_declared_symbol(lib):
    hdr = open(os.path.join(ROOT, "include", "pd.h")).read()
    names = set(re.findall(r"\b(pd_[a-z_A-Z0-9]+)\s*\(", hdr))
    assert len(names) >= 19
    for n in sorted(names):
        assert hasattr(lib, n), n
    from paper_2309_11273_amd import _abi
    assert names == set(_abi.SIGNATURES), names ^ set(_abi.SIGNATURES)


def _family(w):
    from paper_2309_11273_amd.solver import FamilyHost
    return FamilyHost(w.lat, w.dx, w.origin, w.delta, w.vol, w.specimen, w.cuts)


CASES = {
    "cantilever": lambda: W.cantilever3d(),
    "plate": lambda: W.plate2d(),
    "impact_small": lambda: W.impact3d(nx=40, ny=40, dt=1e-7),
    "cylinder_small": lambda: W.cylinder3d(dx=2e-3, dt=1e-7, twist_rate=1.0),
    "batch3": lambda: W.batch2d(n_plates=3, dt=np.ones(3)),
    "plane_strain": lambda: W.plate2d(nx=30, ny=20, dt=1e-7, mode="plane_strain", notch_row=9,
                                      notch_tip=14.37),
    "plate_16x4": lambda: W.plate2d(nx=64, ny=20, dt=1e-7, notch_row=9, notch_tip=31.37),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_family_matches_reference(lib, case):
    """Same unique bonds, same notch-cut bonds, same weighted volume (Eq. 1.9)."""
    w = CASES[case]()
    f = _family(w)
    o = Oracle(w)
    bi, bj, st = f.bond_status(f.mask)
    obi, obj = o.bonds()
    np.testing.assert_array_equal(bi, obi)
    np.testing.assert_array_equal(bj, obj)
    np.testing.assert_array_equal(st, o.rho())
    assert int(f.sizes.n_cut) == o.n_cut
    assert int(f.sizes.n_bonds) == o.nb
    real = f.perm >= 0
    m = np.empty(w.n)
    m[f.perm[real]] = 1.0 / f.inv_m[real]
    np.testing.assert_allclose(m, o.m(), rtol=1e-14)
    # per-bond geometry from the stencil equals the reference's xi/x and x
    rows, ks, ci, cj, sid = f.bond_table()
    sten = f.stencil.reshape(-1, 4)
    xl, M = o.bond_geom()
    key = np.minimum(ci, cj).astype(np.int64) * w.n + np.maximum(ci, cj)
    idx = np.searchsorted(obi.astype(np.int64) * w.n + obj, key)
    sign = np.where(ci < cj, 1.0, -1.0)
    assert np.array_equal(sten[sid, 3], xl[idx])
    assert np.array_equal(sten[sid, :3], M[idx] * sign[:, None])
    # interleaved layout: a slice's word k for all lanes is contiguous
    assert f.slice_ptr[-1] == f.sizes.n_words
    assert np.all(np.diff(f.slice_ptr) % 64 == 0)


@pytest.mark.parametrize("case", ["cantilever", "plate", "cylinder_small"])
def test_stencil_order_shortest_first_in_mirror_pairs(lib, case):
    """Stencil entries by length, each offset followed by its opposite with
    exactly negated M and the same x (the tile kernels take a bond and its
    mirror together and use entry 0 as a shortest bond)."""
    w = CASES[case]()
    f = _family(w)
    ns = int(f.sizes.n_stencil)
    off = f.stencil_off.reshape(-1, 3)[:ns].astype(np.int64)
    sten = f.stencil.reshape(-1, 4)[:ns]
    n2 = (off ** 2).sum(axis=1)
    assert ns % 2 == 0 and np.all(np.diff(n2) >= 0)
    assert np.array_equal(off[1::2], -off[0::2])
    assert np.array_equal(sten[1::2, :3], -sten[0::2, :3])
    assert np.array_equal(sten[1::2, 3], sten[0::2, 3])
    assert sten[0, 3] == sten[:, 3].min()
    # the single-precision table rows of a pair: M/x and x M negated, x^2 equal
    kt1 = f.ktab[1536:1536 + 8 * ns].reshape(ns, 8).view(np.float32)
    for c in (0, 1, 3, 4, 6, 7):
        assert np.array_equal(kt1[1::2, c], -kt1[0::2, c]), c
    assert np.array_equal(kt1[1::2, 2], kt1[0::2, 2])


def test_uniform_volume_flag(lib):
    """The family reports one node volume (as float) when every node has it,
    else 0, which keeps the FP32 tile kernels on the staged volumes."""
    w = CASES["cylinder_small"]()
    f = _family(w)
    assert f.sizes.vol_uniform == np.float32(w.vol[0]) and f.sizes.vol_uniform > 0
    w.vol = w.vol.copy()
    w.vol[len(w.vol) // 2] *= 1.01
    assert _family(w).sizes.vol_uniform == 0.0


def _halo_rows(f, tile):
    """Emulation of the LDS-staged kernels' halo gather: global row of every
    slot of the (T0+2R)(T1+2R)(T2+2R) box around 'tile' (-1 = no tile).  In
    3D with 4-wide tiles the x pitch is padded up to 4 mod 8."""
    s = f.sizes
    T0, T1, T2 = list(s.tile)
    R = int(s.reach)
    dim = int(s.dim)
    Bx, By = T0 + 2 * R, T1 + 2 * R
    if dim == 3 and T0 == 4:
        Bx += (12 - Bx % 8) % 8
    Pz = Bx * By
    Bz = T2 + 2 * R if dim == 3 else 1
    tn = f.tile_nbr[27 * tile: 27 * tile + 27]
    out = np.full(Pz * Bz, -1, np.int64)
    for slot in range(Pz * Bz):
        bx, by, bz = (slot % Pz) % Bx, (slot % Pz) // Bx, slot // Pz
        p = [bx - R, by - R, (bz - R) if dim == 3 else 0]
        if p[0] >= T0 + R or p[1] >= T1 + R:
            continue
        T = [T0, T1, T2]
        d = [(-1 if p[c] < 0 else (1 if p[c] >= T[c] else 0)) for c in range(3)]
        nt = tn[(d[2] + 1) * 9 + (d[1] + 1) * 3 + (d[0] + 1)]
        if nt >= 0:
            loc = [p[c] - d[c] * T[c] for c in range(3)]
            out[slot] = nt * 64 + loc[0] + T0 * (loc[1] + T1 * loc[2])
    return out, (Bx, Pz, Bz)


@pytest.mark.parametrize("case", ["cantilever", "cylinder_small", "batch3", "plate", "plate_16x4"])
def test_tile_halo_addressing_matches_bond_words(lib, case):
    """The tile kernels find neighbour k of lane l at halo slot
    slot(l) + soff[k]; that slot must hold exactly the row the bond word
    names, for every present bond (and stay inside the halo box)."""
    w = CASES[case]()
    f = _family(w)
    s = f.sizes
    T0, T1, T2 = list(s.tile)
    R = int(s.reach)
    assert min(T0, T1) >= R and (s.dim == 2 or T2 >= R)
    off = f.stencil_off.reshape(-1, 3)
    L4 = int(s.words_per_row)
    rng = np.random.default_rng(0)
    tiles = rng.choice(int(s.n_tiles), size=min(40, int(s.n_tiles)), replace=False)
    for t in tiles:
        rows, (Bx, Pz, Bz) = _halo_rows(f, int(t))
        soff = off[:, 0] + Bx * off[:, 1] + Pz * off[:, 2]
        hm = f.halo_map.astype(np.int64)
        tn = f.tile_nbr[27 * int(t): 27 * int(t) + 27]
        assert len(hm) == Pz * Bz == int(s.n_halo)
        nt = np.where(hm >= 0, tn[np.maximum(hm, 0) >> 6], -1)
        rows_map = np.where((hm >= 0) & (nt >= 0), nt * 64 + (hm & 63), -1)
        assert np.array_equal(rows_map, rows)
        ns_ = len(soff)
        kt1 = f.ktab[:1024].view(np.int32).reshape(128, 8)
        kt2 = f.ktab[1024:1536].view(np.int32).reshape(128, 4)
        assert np.array_equal(kt1[:ns_, 4], soff) and np.array_equal(kt2[:ns_, 3], soff)
        assert not kt1[ns_:].any() and not kt2[ns_:].any() and not kt1[:, 6:].any()
        kf1 = f.ktab[:1024].view(np.float32).reshape(128, 8)
        kf2 = f.ktab[1024:1536].view(np.float32).reshape(128, 4)
        sten = f.stencil.reshape(-1, 4)
        assert np.array_equal(kf1[:ns_, :4], sten.astype(np.float32))
        assert np.array_equal(kf1[:ns_, 5], (1.0 / sten[:, 3]).astype(np.float32))
        assert np.array_equal(kf2[:ns_, :3], (sten[:, 3:4] * sten[:, :3]).astype(np.float32))
        base = f.slice_ptr[t]
        for lane in range(64):
            l0, l1, l2 = lane % T0, (lane // T0) % T1, lane // (T0 * T1)
            my = (l0 + R) + Bx * (l1 + R) + Pz * ((l2 + R) if s.dim == 3 else 0)
            assert rows[my] == t * 64 + lane
            for k in range(int(s.n_stencil)):
                wd = f.words[base + (k // 4) * 256 + lane * 4 + (k % 4)]
                slot = my + soff[k]
                assert 0 <= slot < Pz * Bz
                if (wd & 127) != 127:
                    assert (wd & 127) == k
                    assert rows[slot] == (wd >> 7)
            for k in range(int(s.n_stencil), L4):
                assert (f.words[base + (k // 4) * 256 + lane * 4 + (k % 4)] & 127) == 127


def _box1_pitches(T, R, dim):
    """Pitches of the single-precision pass-1 box: 64 distinct LDS banks
    (mod 64) over a tile's lanes when padded, unpadded if the padded box
    exceeds the kernel's array stride."""
    e0, e1, e2 = T[0] + 2 * R, T[1] + 2 * R, (T[2] + 2 * R) if dim == 3 else 1
    p0, p1 = e0, e1
    if dim == 3 and T[0] == 4 and T[1] == 4 and e0 <= 12:
        p0 = p1 = 12
    elif dim == 2 and T[0] == 8 and e0 <= 24:
        p0 = 24
    stride = 1472 if dim == 3 else (336 if e0 * e1 * e2 <= 256 else 1024)
    if p0 * p1 * e2 > stride:
        p0, p1 = e0, e1
    return p0, p1, e2


@pytest.mark.parametrize("case", ["cantilever", "cylinder_small", "batch3", "plate", "plate_16x4"])
def test_pass1_box_addressing_matches_bond_words(lib, case):
    """The single-precision pass 1 stages the unpadded box point by point
    (halo_pos) into a padded box and finds neighbour k of lane l at
    slot(l) + soff1[k] (third table); that slot must receive exactly the row
    the bond word names.  Its third-table entries are M/x, x^2 and x M."""
    w = CASES[case]()
    f = _family(w)
    s = f.sizes
    T = list(s.tile)
    R, dim = int(s.reach), int(s.dim)
    p0, p1, e2 = _box1_pitches(T, R, dim)
    e0, e1 = T[0] + 2 * R, T[1] + 2 * R
    # the staged points: exactly the box points a stencil entry of a tile point reaches
    off3 = f.stencil_off.reshape(-1, 3)
    reached = set()
    for l in range(64):
        lp = (l % T[0], (l // T[0]) % T[1], l // (T[0] * T[1]) if dim == 3 else 0)
        reached.add((lp[0] + R, lp[1] + R, lp[2] + (R if dim == 3 else 0)))
        for o in off3:
            reached.add((lp[0] + o[0] + R, lp[1] + o[1] + R, lp[2] + (o[2] + R if dim == 3 else 0)))
    assert int(s.n_box) == len(reached) <= e0 * e1 * e2
    if dim == 3 and T[:2] == [4, 4] and e0 <= 12:
        # the lanes of a tile hit 64 distinct banks (4-byte elements)
        lanes = [(l % 4) + p0 * ((l // 4) % 4) + p0 * p1 * (l // 16) for l in range(64)]
        assert len({v % 64 for v in lanes}) == 64
    if dim == 2 and T[:2] == [8, 8] and p0 == 24:
        # 8-byte elements: each half-wave's 32 lanes hit 32 distinct bank pairs
        lanes = [(l % 8) + p0 * (l // 8) for l in range(64)]
        for h in (lanes[:32], lanes[32:]):
            assert len({v % 32 for v in h}) == 32
    hp = f.halo_pos[: int(s.n_box)].astype(np.int64)
    off = f.stencil_off.reshape(-1, 3)
    ns_ = int(s.n_stencil)
    kt = f.ktab[1536:].view(np.int32).reshape(128, 8)
    kf = f.ktab[1536:].view(np.float32).reshape(128, 8)
    soff1 = off[:, 0] + p0 * off[:, 1] + p0 * p1 * off[:, 2]
    assert np.array_equal(kt[:ns_, 5], soff1) and not kt[ns_:].any()
    sten = f.stencil.reshape(-1, 4)
    mx = (sten[:, :3] / sten[:, 3:4]).astype(np.float32)
    xm = (sten[:, 3:4] * sten[:, :3]).astype(np.float32)
    assert np.array_equal(kf[:ns_, [0, 1, 6]], mx)
    assert np.array_equal(kf[:ns_, 2], (sten[:, 3] * sten[:, 3]).astype(np.float32))
    assert np.array_equal(kf[:ns_, [3, 4, 7]], xm)
    # every box point lands on a distinct slot of the padded box
    slots = hp >> 11
    assert len(np.unique(slots)) == len(slots) and slots.max() < p0 * p1 * e2
    rng = np.random.default_rng(1)
    tiles = rng.choice(int(s.n_tiles), size=min(40, int(s.n_tiles)), replace=False)
    for t in tiles:
        tn = f.tile_nbr[27 * int(t): 27 * int(t) + 27]
        rows = np.full(p0 * p1 * e2, -1, np.int64)
        nt = tn[(hp & 2047) >> 6]
        rows[slots] = np.where(nt >= 0, nt * 64 + (hp & 63), -1)
        base = f.slice_ptr[t]
        for lane in range(64):
            l0, l1, l2 = lane % T[0], (lane // T[0]) % T[1], lane // (T[0] * T[1])
            my = (l0 + R) + p0 * (l1 + R) + p0 * p1 * ((l2 + R) if dim == 3 else 0)
            assert rows[my] == t * 64 + lane
            for k in range(ns_):
                wd = f.words[base + (k // 4) * 256 + lane * 4 + (k % 4)]
                slot = my + soff1[k]
                assert 0 <= slot < p0 * p1 * e2
                if (wd & 127) != 127:
                    assert rows[slot] == (wd >> 7)


@pytest.mark.parametrize("case", ["cantilever", "cylinder_small", "batch3", "plate", "plate_16x4"])
def test_halo_pos_agrees_with_halo_map(lib, case):
    """halo_pos and halo_map describe the same box points: the slot of the
    halo box (pitches of halo_map) that a halo_pos entry's direction and
    local position give is the one halo_map maps back to them."""
    w = CASES[case]()
    f = _family(w)
    s = f.sizes
    T = list(s.tile)
    R, dim = int(s.reach), int(s.dim)
    Bx = T[0] + 2 * R
    if dim == 3 and T[0] == 4:
        Bx += (12 - Bx % 8) % 8
    Pz = Bx * (T[1] + 2 * R)
    hm = f.halo_map.astype(np.int64)
    s0, s1 = T[0].bit_length() - 1, T[1].bit_length() - 1
    for h in f.halo_pos[: int(s.n_box)].astype(np.int64):
        d, l = (h & 2047) >> 6, h & 63
        dx, dy, dz = d % 3 - 1, (d // 3) % 3 - 1, d // 9 - 1
        bx = T[0] * dx + (l & (T[0] - 1)) + R
        by = T[1] * dy + ((l >> s0) & (T[1] - 1)) + R
        bz = T[2] * dz + (l >> (s0 + s1)) + R if dim == 3 else 0
        slot = bx + Bx * by + Pz * bz
        assert 0 <= slot < len(hm) and hm[slot] == (h & 2047)


def test_internal_order_is_tile_major(lib):
    w = W.impact3d(nx=16, ny=16, nz=8, dt=1e-7)
    f = _family(w)
    lat = w.lat[f.perm[: w.n]]
    for s in range(w.n // 64):
        tile = lat[64 * s: 64 * s + 64] // 4
        assert np.all(tile == tile[0])


def test_constants_match_reference(lib):
    from paper_2309_11273_amd.solver import critical_stretch, specimen_params
    for mode, mid in (("3d", 0), ("plane_stress", 1), ("plane_strain", 2)):
        for E, nu in ((200e9, 0.3), (72e9, 0.22), (30e9, 0.2), (190e9, 0.25)):
            k = oracle.constants(mid, E, nu)
            sp = specimen_params(mode, E, nu, 2000.0, 1.0, 1e-8)
            assert sp.kp == pytest.approx(k["K"] - k["G"] / 3, rel=1e-14)
            assert sp.G == pytest.approx(k["G"], rel=1e-14)
            assert sp.A == pytest.approx(k["A"], rel=1e-14)
            for var in (0, 1):
                a = critical_stretch(mode, E, nu, 50.0, 1.5e-3, var)
                b = oracle.critical_stretch(mid, E, nu, 50.0, 1.5e-3, var)
                assert a == pytest.approx(b, rel=1e-14)
    assert math.isinf(critical_stretch("3d", 200e9, 0.3, None, 1e-3))


def test_bsr_pattern_is_two_hop_closure(lib):
    """Row i of K holds exactly the nodes q != i joined to i by one or two
    bonds (Eq. 2.14: the dilatation of a neighbour reaches 2 delta)."""
    from paper_2309_11273_amd import _abi as A
    for w in (W.plate2d(nx=20, ny=12, dt=1e-8, notch_row=5, notch_tip=8.37), W.cantilever3d()):
        f = _family(w)
        o = Oracle(w)
        bi, bj = o.bonds()
        n = w.n
        adj = [set() for _ in range(n)]
        for a, b in zip(bi, bj):
            adj[a].add(b)
            adj[b].add(a)
        bs = A.pd_bsr_sizes()
        A.check("pd_bsr_pattern", lib.pd_bsr_pattern(C.byref(f.sizes), C.byref(f._hb), C.byref(bs), None, None))
        rp = np.empty(f.sizes.n_pad + 1, np.int64)
        col = np.empty(bs.nnzb, np.int32)
        A.check("pd_bsr_pattern", lib.pd_bsr_pattern(C.byref(f.sizes), C.byref(f._hb), C.byref(bs),
                                                     rp.ctypes.data_as(C.c_void_p),
                                                     col.ctypes.data_as(C.c_void_p)))
        total = 0
        for r in np.nonzero(f.perm >= 0)[0]:
            p = f.perm[r]
            want = set(adj[p])
            for j in adj[p]:
                want |= adj[j]
            want.discard(p)
            got = set(f.perm[col[rp[r]:rp[r + 1]]].tolist())
            assert got == want
            total += len(want)
        assert total == bs.nnzb


def _fac_pattern(lib, f):
    from paper_2309_11273_amd import _abi as A
    fs = A.pd_fac_sizes()
    A.check("pd_fac_pattern", lib.pd_fac_pattern(C.byref(f.sizes), C.byref(f._hb), C.byref(fs), None, None, None))
    nb = int(fs.nb)
    ij = np.empty(2 * max(1, nb), np.int32)
    pos = np.empty(2 * max(1, nb), np.int32)
    bid = np.full(int(fs.n_words), -7, np.int32)
    v = lambda a: a.ctypes.data_as(C.c_void_p)
    A.check("pd_fac_pattern", lib.pd_fac_pattern(C.byref(f.sizes), C.byref(f._hb), C.byref(fs), v(ij), v(pos),
                                                 v(bid)))
    return fs, ij[:2 * nb].reshape(nb, 2), pos[:2 * nb].reshape(2, nb).T, bid


@pytest.mark.parametrize("case", ["cantilever", "plate", "batch3", "plate_16x4", "cylinder_small"])
def test_factored_bond_numbering(lib, case):
    """Columns of C_e (bond end rows), the owner / reverse word positions and
    the bond id of every directed position (the column of C_theta and K_e)
    describe exactly the reference's unique bonds, each once."""
    w = CASES[case]()
    f = _family(w)
    o = Oracle(w)
    fs, ij, pos, bid = _fac_pattern(lib, f)
    nb = int(fs.nb)
    assert nb == o.nb == int(f.sizes.n_bonds)
    assert int(fs.n_words) == int(f.sizes.n_words)
    # the unordered caller pairs are the reference's bonds
    ci, cj = f.perm[ij[:, 0]], f.perm[ij[:, 1]]
    assert (ci >= 0).all() and (cj >= 0).all()
    lo, hi = np.minimum(ci, cj).astype(np.int64), np.maximum(ci, cj).astype(np.int64)
    obi, obj = o.bonds()
    np.testing.assert_array_equal(np.sort(lo * w.n + hi), obi.astype(np.int64) * w.n + obj)
    # owner and reverse positions hold the two directed words of the bond
    words = f.words
    assert (np.diff(pos[:, 0]) > 0).all()  # numbered in word order
    wo, wr = words[pos[:, 0]], words[pos[:, 1]]
    np.testing.assert_array_equal(wo >> 7, ij[:, 1].astype(np.uint32))
    np.testing.assert_array_equal(wr >> 7, ij[:, 0].astype(np.uint32))
    off = f.stencil_off.reshape(-1, 3)
    np.testing.assert_array_equal(off[wo & 127], -off[wr & 127])
    assert ((wo & 127) < (wr & 127)).all()
    # the row of a position follows the interleaved layout
    rows, ks, _, _, _ = f.bond_table()
    slice_of = rows // 64
    widx = f.slice_ptr[slice_of] + (ks // 4) * 256 + (rows % 64) * 4 + ks % 4
    row_at = np.full(f.sizes.n_words, -1, np.int64)
    row_at[widx] = rows
    np.testing.assert_array_equal(row_at[pos[:, 0]], ij[:, 0])
    np.testing.assert_array_equal(row_at[pos[:, 1]], ij[:, 1])
    # every directed position names its bond; padding positions name bond 0
    b = bid[widx]
    assert (b >= 0).all() and (b < nb).all()
    j_at = (words[widx] >> 7).astype(np.int64)
    ok = ((ij[b, 0] == rows) & (ij[b, 1] == j_at)) | ((ij[b, 1] == rows) & (ij[b, 0] == j_at))
    assert ok.all()
    pad = np.ones(f.sizes.n_words, bool)
    pad[widx] = False
    assert (bid[pad] == 0).all()
    # each bond is named by exactly two positions
    np.testing.assert_array_equal(np.bincount(b, minlength=nb), np.full(nb, 2))


def test_argument_errors(lib):
    from paper_2309_11273_amd import _abi as A
    s0 = C.c_double()
    assert lib.pd_critical_stretch(0, -1.0, 0.3, 1.0, 1e-3, 0, C.byref(s0)) == -1
    assert lib.pd_critical_stretch(0, 1e9, 0.5, 1.0, 1e-3, 0, C.byref(s0)) == -1
    assert lib.pd_critical_stretch(0, 1e9, 0.3, 1.0, 1e-3, 2, C.byref(s0)) == -1
    assert lib.pd_critical_stretch(0, 1e9, 0.3, 1.0, 1e-3, 0, None) == -1
    sp = A.pd_spec()
    assert lib.pd_specimen_params(0, 1e9, 0.3, 0.0, 1.0, 1e-8, C.byref(sp)) == -1
    assert lib.pd_specimen_params(0, 1e9, 0.3, 1.0, float("nan"), 1e-8, C.byref(sp)) == -1
    sizes = A.pd_family_sizes()
    assert lib.pd_build_family(None, None, 0, C.byref(sizes), None) == -1
    lat = np.zeros((2, 2), np.int32)  # duplicate lattice point
    vol = np.ones(2)
    body = A.pd_body(n=2, dim=2, lat=lat.ctypes.data_as(C.c_void_p), dx=1.0, delta=3.0,
                     vol=vol.ctypes.data_as(C.c_void_p))
    assert lib.pd_build_family(C.byref(body), None, 0, C.byref(sizes), None) == -1
    body.n = 0
    assert lib.pd_build_family(C.byref(body), None, 0, C.byref(sizes), None) == -2
    lat2 = np.array([[0, 0], [1, 0]], np.int32)
    body = A.pd_body(n=2, dim=2, lat=lat2.ctypes.data_as(C.c_void_p), dx=1.0, delta=3.0,
                     vol=vol.ctypes.data_as(C.c_void_p))
    bad = A.pd_cut(kind=1)  # a 3D patch in 2D
    assert lib.pd_build_family(C.byref(body), C.byref(bad), 1, C.byref(sizes), None) == -1
    assert lib.pd_build_family(C.byref(body), None, 0, C.byref(sizes), None) == 0
    assert sizes.n_bonds == 1 and sizes.n_pad == 64
    # calls without a context are rejected before any device work
    st = A.pd_state_dev()
    pr = A.pd_problem_dev()
    assert lib.pd_step(None, C.byref(pr), C.byref(st), 1, None, None, None) == -1
    assert lib.pd_force(None, C.byref(pr), C.byref(st), 0, None, None) == -1
    assert lib.pd_damage(None, C.byref(pr), None, None) == -1
    ps = A.pd_profile_stats()
    assert lib.pd_profile_read(None, C.byref(ps), 0) == -1
    o = A.pd_newmark_opts(1e-6, A.pd_cg_opts(1e-10, 10, 5, 1, 0), 0, 0)
    rep = A.pd_cg_report()
    assert lib.pd_newmark_step(None, C.byref(pr), None, C.byref(st), 1, C.byref(o), None, C.byref(rep)) == -1
    assert lib.pd_static_solve(None, C.byref(pr), None, C.byref(st), C.byref(o.cg), None, C.byref(rep)) == -1


def test_solver_workspace_sizes(lib):
    """The static solve's workspace holds five double4 vectors, the 3x3
    block inverses (12 doubles a row), two partial sums per 256 rows and 16
    scalars; the implicit step's adds a_n (double4) and the mass per row
    after a 32-byte boundary."""
    for n in (64, 128, 256 * 7 + 64, 911360):
        nb = (n + 255) // 256
        st = 5 * 4 * n + 12 * n + 2 * nb + 16
        assert lib.pd_static_workspace(n) == st
        assert lib.pd_newmark_workspace(n) == ((st + 3) // 4) * 4 + 5 * n
    assert lib.pd_newmark_workspace(-1) == 0 and lib.pd_static_workspace(0) == 0


# --------------------------------------------------------------------------
# inputs: grid conventions and notch geometry
# --------------------------------------------------------------------------

def test_table1_node_counts_vertex_lattice_plus_three_layers():
    """Node counts of the 2D cantilever grids (Sec. 4.1 table): a vertex
    lattice of the 48 x 12 m beam plus 3 constrained layers beyond the
    clamped end; and 386,984 nodes for the 3D beam (48 x 12 x 5 m)."""
    import json
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_values.json")))
    t1 = gold["table1_cantilever_2d"]
    counts = []
    for delta in t1["horizon_m"]:
        dx = delta / 3
        counts.append((round(t1["beam_m"]["L"] / dx) + 1 + 3) * (round(t1["beam_m"]["H"] / dx) + 1))
    assert counts == t1["nodes"]
    c3 = gold["cantilever_3d_nodes"]
    dx = c3["dx_m"]
    b = c3["beam_m"]
    assert (round(b["L"] / dx) + 1 + 3) * (round(b["H"] / dx) + 1) * (round(b["W"] / dx) + 1) == c3["value"]


def test_workload_sizes():
    assert W.cantilever3d().n == 320
    assert W.plate2d().n == 16000
    assert W.cylinder_lattice(25e-3, 100e-3, 0.6e-3).shape[0] == 911319
    assert W.cylinder_lattice(25e-3, 100e-3, 0.5e-3).shape[0] == 1572000
    d = W.batch_draws(256)
    assert len(d) == 256
    assert sum(x["nx"] * x["ny"] for x in d) == 5800669
    p = W.load_params()
    for k in ("cantilever3d", "plate2d", "impact3d", "cylinder3d", "cylinder3d_dx05"):
        assert p[k] > 0
    assert len(p["batch2d_dt"]) == 256


def _min_node_distance_to_segment(P, A, B):
    AB = B - A
    t = np.clip(((P - A) @ AB) / (AB @ AB), 0, 1)
    return np.linalg.norm(P - (A + t[:, None] * AB), axis=1)


@pytest.mark.parametrize("name", ["plate2d", "impact3d", "batch2d"])
def test_notches_have_no_ties(name):
    """No node lies on a notch and no lattice bond passes within 1e-6 dx of
    a notch tip: every cut decision is far from a floating-point tie."""
    if name == "plate2d":
        w = W.plate2d()
    elif name == "impact3d":
        w = W.impact3d(nx=40, ny=40, dt=1e-7)
    else:
        w = W.batch2d(n_plates=8, dt=np.ones(8))
    X = w.positions()
    for c in w.cuts:
        if c.kind == "segment2d":
            A, B = np.array(c.p[:2]), np.array(c.p[2:4])
            d = _min_node_distance_to_segment(X[:, :2], A, B)
            assert d.min() > 1e-6 * w.dx
            tip = B
        else:
            cc, a = np.array(c.p[:3]), np.array(c.p[3:6])
            assert np.all(np.abs(X[:, 1] - cc[1]) > 1e-6 * w.dx)
            tip = (cc + a)[:2]
        # bonds crossing the notch line near the tip: crossing abscissae lie on
        # multiples of dx/k (k <= 6) from a node; the tip sits at 0.37 dx
        frac = (tip[0] / w.dx) % 1.0
        for k in range(1, 7):
            for q in range(0, k + 1):
                assert abs(frac - q / k) > 1e-6


def test_xcd_tile_order_is_a_bijection():
    """The tile kernels hand workgroup b tile x*q + min(x, r) + b // 8 with
    x = b % 8, n = 8q + r (every XCD a contiguous range); that must visit
    every tile exactly once for any tile count."""
    for n in list(range(1, 70)) + [15666, 95030, 7500]:
        b = np.arange(n)
        q, r, x = n // 8, n % 8, b % 8
        t = x * q + np.minimum(x, r) + b // 8
        assert np.array_equal(np.sort(t), b)



@pytest.mark.parametrize("case", ["plate", "cylinder"])
def test_cleared_keys_and_status_index(lib, case):
    """The host helpers that map bond-status bits back to caller bonds:
    clearing both directed copies of chosen reference bonds reports exactly
    those bonds, and the status index of every reference bond points at a
    bit of its own directed copy."""
    if case == "plate":
        w = W.plate2d(nx=30, ny=18, dt=1e-7, notch_row=8, notch_tip=14.37, steps=10)
    else:
        w = W.cylinder3d(dx=5e-3, dt=2.4e-7, twist_rate=10.0, steps=10)
    fam = _family(w)
    o = Oracle(w, search="brute")
    bi, bj = o.bonds()
    rows, ks, ci, cj, _ = fam.bond_table()
    widx, lane = fam.status_index(bi, bj)
    # the indexed bit belongs to a directed entry i -> j of that bond
    word_of = {}
    first = fam.slice_ptr // 64
    for r, k, a, b in zip(rows, ks, ci, cj):
        word_of[(int(first[r // 64] + k), int(r % 64))] = (int(a), int(b))
    for q in np.random.default_rng(0).choice(bi.size, 200, replace=False):
        assert word_of[(int(widx[q]), int(lane[q]))] == (int(bi[q]), int(bj[q]))
    rng = np.random.default_rng(1)
    pick = np.sort(rng.choice(bi.size, 25, replace=False))
    m = fam.mask.copy()
    for q in pick:
        for a, b in ((bi[q], bj[q]), (bj[q], bi[q])):
            sel = np.nonzero((ci == a) & (cj == b))[0][0]
            r, k = rows[sel], ks[sel]
            m[first[r // 64] + k] &= ~np.uint64(1 << int(r % 64))
    keys = fam.cleared_keys(fam.mask, m)
    want = bi[pick].astype(np.int64) * w.n + bj[pick]
    # bonds already cut by the notch were 0 in the initial status
    init = ((fam.mask[widx[pick]] >> lane[pick]) & np.uint64(1)).astype(bool)
    assert np.array_equal(keys, np.sort(want[init]))
    # one copy only: the helper refuses
    q = pick[init][0]
    sel = np.nonzero((ci == bi[q]) & (cj == bj[q]))[0][0]
    m2 = fam.mask.copy()
    m2[first[rows[sel] // 64] + ks[sel]] &= ~np.uint64(1 << int(rows[sel] % 64))
    with pytest.raises(AssertionError):
        fam.cleared_keys(fam.mask, m2)


@pytest.mark.parametrize("case", ["cantilever", "impact_small", "cylinder_small", "short_reach", "plate", "batch3"])
def test_supertile_box_addressing_matches_bond_words(lib, case):
    """Super-tiles group the tiles 2 x 2 (x 1) (4x4x4 tiles in 3D, 8x8 in
    2D): every tile is in exactly one quadrant of one super-tile, at its
    place; the shared box (pitches 16 and 228 in 3D, 40 in 2D) receives, at
    slot(l) + soff[k] of lane l of quadrant q, exactly the row the bond word
    of bond k names; the lanes of a quadrant hit 64 distinct LDS banks; the
    table holds M/x, x^2, x M of every entry."""
    if case == "short_reach":
        w = W.impact3d(nx=24, ny=24, nz=8, dt=1e-7)
        w.delta = 2.015 * w.dx
    else:
        w = CASES[case]()
    f = _family(w)
    s = f.sizes
    R = int(s.reach)
    dim = int(s.dim)
    assert f.st_tiles is not None and list(s.tile) == ([4, 4, 4] if dim == 3 else [8, 8, 1])
    nst = f.n_st
    st = f.st_tiles.reshape(nst, 4)
    assert np.array_equal(np.sort(st[st >= 0]), np.arange(int(s.n_tiles)))
    org = f.tile_org.reshape(-1, 4)
    for q in range(4):
        for sidx in np.nonzero(st[:, q] >= 0)[0][:50]:
            t0 = st[sidx][st[sidx] >= 0][0]
            t = st[sidx, q]
            assert org[t, 3] == org[t0, 3] and org[t, 2] == org[t0, 2]
    if dim == 3:
        P0, P1, nslot = 16, 228, 228 * (4 + 2 * R)

        def own(q, l):
            return ((l & 3) + 4 * (q & 1) + R) + P0 * (((l >> 2) & 3) + 4 * (q >> 1) + R) + P1 * ((l >> 4) + R)
    else:
        P0, P1, nslot = 40, 0, 40 * (16 + 2 * R)

        def own(q, l):
            return ((l & 7) + 8 * (q & 1) + R) + P0 * ((l >> 3) + 8 * (q >> 1) + R)
    for q in range(4):
        assert len({(own(q, l) - own(q, 0)) % 64 for l in range(64)}) == 64
    ns_ = int(s.n_stencil)
    off = f.stencil_off.reshape(-1, 3)
    kt = f.st_ktab.view(np.int32).reshape(128, 8)
    kf = f.st_ktab.view(np.float32).reshape(128, 8)
    soff = off[:, 0] + P0 * off[:, 1] + P1 * off[:, 2]
    assert np.array_equal(kt[:ns_, 5], soff) and not kt[ns_:].any()
    k1 = f.ktab[1536:].view(np.float32).reshape(128, 8)
    assert np.array_equal(kf[:ns_, [0, 1, 2, 3, 4, 6, 7]], k1[:ns_, [0, 1, 2, 3, 4, 6, 7]])
    hp = f.st_pos.astype(np.int64)
    slots = hp >> 12
    assert len(np.unique(slots)) == len(slots) and slots.max() < nslot
    assert f.st_n_pos <= (512 if dim == 2 else 2048)
    rng = np.random.default_rng(2)
    for sidx in rng.choice(nst, size=min(25, nst), replace=False):
        nb = f.st_nbr[48 * sidx: 48 * sidx + 48]
        if dim == 2:
            assert (nb[:16] == -1).all() and (nb[32:] == -1).all()
        rows = np.full(nslot, -1, np.int64)
        nt = nb[(hp & 4095) >> 6]
        rows[slots] = np.where(nt >= 0, nt * 64 + (hp & 63), -1)
        for q in range(4):
            t = st[sidx, q]
            if t < 0:
                continue
            base = f.slice_ptr[t]
            for lane in range(64):
                my = own(q, lane)
                assert rows[my] == t * 64 + lane
                for k in range(ns_):
                    wd = f.words[base + (k // 4) * 256 + lane * 4 + (k % 4)]
                    if (wd & 127) != 127:
                        assert rows[my + soff[k]] == (wd >> 7)


def test_supertiles_need_square_tiles(lib):
    """A 2D family of 16x4 tiles has no super-tiles (its kernels are the tile
    kernels)."""
    f = _family(CASES["plate_16x4"]())
    assert list(f.sizes.tile) == [16, 4, 1]
    assert f.st_tiles is None and f.n_st == 0
