// LDS-staged ("tiled") kernels of the single-precision matrix-free step.
//
// The builder lays every specimen's lattice out in tiles of 64 lattice
// points (4x4x4 in 3D, 8x8 or 16x4 in 2D, every edge at least the largest
// stencil offset component R); tile t owns rows 64t .. 64t+63 and lane l of
// the tile sits on local lattice position (l % T0, (l / T0) % T1,
// l / (T0 T1)).  Bond k of every row is stencil entry k.  A workgroup of
// four waves takes one tile (in 2D with short stencils, four tiles, one per
// wave):
//   1. stages what the pass needs of the tile plus an R-wide halo -- a box
//      gathered from the tile and its 3^dim neighbour tiles, point by point
//      from the halo_pos table -- into LDS as separate float arrays at a
//      fixed stride (pass 1: the fixed-point displacement shadow relative to
//      a reference point of the tile, V and G Q r V; pass 2: (K - G/3) theta/m
//      and V), all of a thread's loads issued before any is consumed.  The
//      box pitches are padded so that the 64 lanes of a tile, each reading
//      the element at the same offset from its own point, hit 64 distinct
//      LDS banks;
//   2. every wave sweeps a quarter of the stencil for all 64 rows (pass 1:
//      every fourth group of four entries, so that each wave gets bonds of
//      every length; pass 2: a contiguous quarter), four entries at a time,
//      a bond and its mirror (the opposite offset, the next entry) summed as
//      one term: the neighbour of row l through entry k is point
//      slot(l) + soff[k], soff[k] the same for every lane, so one address
//      per bond serves all arrays (their distance is a multiple of 256
//      bytes: one ds_read2st64 per pair).  The entry's table row and bond-
//      status word are wave-uniform scalar loads, the status word used
//      directly as the lane mask; the status words of the next group are
//      requested once the current group's LDS data are in registers;
//   3. the four partial sums of each row are added in wave order and wave 0
//      writes the row's result (and, in pass 2, the explicit update, whose
//      inputs it requests before the staging).
//
// The arithmetic follows the gather kernels of kernels_f32.hip (same
// fixed-point shadow, same double recheck of near-threshold bonds, same
// difference form of the dilatation term) with the shadow scale Q factored
// out of the per-bond work: the bond strain is carried in units of Q,
// e' = (M / x) . (a_j - a_i) with a the staged shadow, and Q enters once per
// row (the breaking threshold becomes s_c / Q, the deviatoric modulus G Q),
// and with the pair force split between the passes: pass 1, which has the
// strain, sums the deviatoric part; pass 2 only the dilatational part.  Rows
// next to a shadow sentinel (a displacement too large for the fixed-point
// range) take the double gather path bond by bond; the per-bond test is
// compiled only into the sweep used when the tile's halo holds a sentinel.
// Every row of a tile belongs to one specimen, so the material constants
// are wave-uniform and folded into the staged values.
#include <hip/hip_runtime.h>

#include <cmath>
#include <type_traits>

#include "kernels.h"
#include "tile_common.h"

namespace pdk {

// LDS of one tile in pass 1: the staged box (per point: the shadow
// components relative to the tile's reference point, V, and G Q r V with
// r = 1/m) at the fixed stride S (pd_box1_stride); with TPW = 1 the partial
// sums (4 floats and 3 doubles per thread) reuse it after the sweep; then the
// 27 neighbour tiles.  3D: five float arrays, read per point with two
// ds_read2st64 and one ds_read (array distances are multiples of 256 bytes),
// or four when every node has the same volume (UV: V is then a constant, the
// box a fifth smaller, and a compute unit holds six workgroups instead of
// five); 2D: two float2 arrays, (x, y) and (V, G Q r V), read with two 8-byte
// reads from one address, which keeps the box of a one-wave tile small.
template <int DIM, int TPW, bool UV = false>
struct Lay1 {
    // super-tile box: 3D 16 x 14 x 10 slots at pitches 16 and 228 (2280
    // slots), 2D 40 x 22 (880)
    static constexpr int S = TPW == 0 ? (DIM == 3 ? 2304 : 896) : (DIM == 3 ? 1472 : (TPW == 4 ? 336 : 1024));
    // box points staged per thread: 3D boxes of up to 1024 points (R <= 3),
    // 3D super-tile boxes up to 2048, 2D up to 256 per wave (TPW = 4) or 512
    // per workgroup (one tile per workgroup or a super-tile)
    static constexpr int MP = TPW == 0 ? (DIM == 3 ? 8 : 2) : (DIM == 3 ? 4 : (TPW == 4 ? 4 : 2));
    static constexpr int BOX = DIM == 3 ? (UV ? 4 : 5) * S * 4 : 2 * S * 8;
    static constexpr int SUMS = TPW == 1 ? PD_TILE_WAVES * 64 * (4 * 4 + 3 * 8) : 0;
    static constexpr int AREA = BOX > SUMS ? BOX : SUMS;
    // then the neighbour tiles (27, or 48 for a super-tile), for a
    // super-tile the shared reference point, and the box's largest staged
    // magnitude (word 31, or 63 for a super-tile)
    static constexpr int BYTES = AREA + (TPW == 0 ? 64 : 32) * 4;
    static_assert(DIM == 2 || (S % 64 == 0 && 4 * S * 4 / 256 <= 255), "array offsets fit the st64 encoding");
    static_assert(TPW != 0 || (DIM == 3 ? 228 * 10 <= S : 40 * 22 <= S), "super-tile box fits the stride");
};

// access to the staged pass-1 box of Lay1 (UV: no V array, V = Vu)
template <int DIM, int S, bool UV = false>
struct View1 {
    float *b;
    float Vu;
    __device__ __forceinline__ void put(int slot, float x, float y, float z, float V, float h) const {
        if constexpr (DIM == 3) {
            b[slot] = x;
            b[S + slot] = y;
            b[2 * S + slot] = z;
            if constexpr (UV) {
                b[3 * S + slot] = h;
            } else {
                b[3 * S + slot] = V;
                b[4 * S + slot] = h;
            }
        } else {
            float2 *q = reinterpret_cast<float2 *>(b);
            q[slot] = make_float2(x, y);
            q[S + slot] = make_float2(V, h);
        }
    }
    __device__ __forceinline__ void pos(int slot, float &x, float &y, float &z) const {
        if constexpr (DIM == 3) {
            x = b[slot];
            y = b[S + slot];
            z = b[2 * S + slot];
        } else {
            const float2 t = reinterpret_cast<const float2 *>(b)[slot];
            x = t.x;
            y = t.y;
            z = 0.0f;
        }
    }
    __device__ __forceinline__ void get(int slot, float &x, float &y, float &z, float &V, float &h) const {
        if constexpr (DIM == 3) {
            pos(slot, x, y, z);
            if constexpr (UV) {
                V = Vu;
                h = b[3 * S + slot];
            } else {
                V = b[3 * S + slot];
                h = b[4 * S + slot];
            }
        } else {
            const float2 *q = reinterpret_cast<const float2 *>(b);
            const float2 t = q[slot], u = q[S + slot];
            x = t.x;
            y = t.y;
            z = 0.0f;
            V = u.x;
            h = u.y;
        }
    }
};

// ---------------------------------------------------------------------------
// pass 1: breaking (with double recheck), dilatation, deviatoric pair force
// ---------------------------------------------------------------------------
// The pair force of Eq. 2.2 is the sum of a dilatational part,
// (K - G/3) x (q_i + q_j) M V_i V_j, which needs the dilatation of both ends
// and is summed in pass 2, and a deviatoric part, G e (1/m_i + 1/m_j) M V_i V_j,
// which needs only the extension and the bond status after this step's
// breaking, and is summed here where e is at hand (fe32, without the V_i).
//
// Per bond the kernel forms e' = (M / x) . (a_j - a_i), the bond strain e / x
// in units of the shadow scale Q, from the staged floats a = fl(s - s_ref)
// (s the fixed-point shadow, s_ref the tile's reference point; s - s_ref is
// an exact integer, rounded only if its magnitude exceeds 2^24).  With
// u = 2^-24: each staged component is off by at most u |a| if |a| >= 2^24 and
// not at all below; the difference a_j - a_i of two such integers is exact
// when it is below 2^24 and off by at most u |a_j - a_i| above; the
// three-term product with the rounded table entries M/x and the later
// product with x add at most 6 u sum_c |a_jc - a_ic|.  With the shadow's own
// rounding (half a unit per component of each end, at most sqrt(3) after the
// product with the unit vector M), in units of Q:
//     |e' x - e / Q| <= sqrt(3) + 2^-21 D + 2^-24 A,
// D = sum_c |a_jc - a_ic|, A = the sum of the |a| at least 2^24 of both ends.
// The screen passes every bond with e' >= thr_lo, thr_lo = s_c / Q minus
// (sqrt(3) + 2^-21 * 6 a + 2^-24 * 6 a) / x_min, a the largest |a| staged
// for a node point of the box (the last term only if a >= 2^24): every D of
// the box's bonds is at most 6 a and every A at most 6 a, so no bond that
// can reach the critical stretch escapes it; a screened bond whose
// e' x + 2^-20 D + 2^-23 A reaches s_c x / Q - sqrt(3) is decided from the
// double state.
template <int DIM, bool BREAK, int TPW, bool UV = false>
__global__ __launch_bounds__(PD_TILE_THREADS) void k_tpass1_f32(StepArgs a, int cur,
                                                                const KEnt *__restrict__ kt,
                                                                const KEnt1 *__restrict__ kn) {
    extern __shared__ __align__(16) unsigned char smem[];
    static_assert(!UV || DIM == 3, "a constant volume is taken in 3D only");
    using GR = Grp<DIM, TPW>;
    using LY = Lay1<DIM, TPW, UV>;
    constexpr int S = LY::S;
    constexpr int MS = LY::MP;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int gt = TPW <= 1 ? tid : lane;  // thread within its box's group
    const int sub = TPW == 1 ? 0 : wv;     // tile of the workgroup this wave serves
    const int kq = TPW == 1 ? wv : 0;      // stencil part of this wave
    constexpr int HB = TPW == 0 ? 12 : 11;  // bits of the point code in a box-point entry
    constexpr int NNB = TPW == 0 ? 48 : 27;  // neighbour tiles of the box
    bool valid;
    int64_t stid = 0;
    const int64_t tile = TPW == 0 ? super_tile(a, sub, stid, valid) : group_tile<TPW>(a.n_slices, sub, valid);
    const int64_t base = a.slice_ptr[tile];
    const int L4 = (int)((a.slice_ptr[tile + 1] - base) >> 6);
    unsigned char *reg = smem + (TPW == 4 ? sub * LY::BYTES : 0);
    const View1<DIM, S, UV> box{reinterpret_cast<float *>(reg), a.vol_uniform};
    int *stn = reinterpret_cast<int *>(reg + LY::AREA);
    int32_t B1[4];
    pd_tile_box1(a.tile, a.reach, DIM, B1);
    const int npts = TPW == 0 ? a.st_n_pos : a.n_pos;  // box points the stencil reaches
    const int32_t *hpos = TPW == 0 ? a.st_pos : a.halo_pos;
    pd_ctl *ctl = a.ctl;
    const double Q = ctl->qs[cur];
    const int4 *__restrict__ sh = a.ush[cur];
    const float2 *__restrict__ qr = a.qr32;
    const double4 *__restrict__ uv = a.uv[cur];
    const double4 *__restrict__ sten = reinterpret_cast<const double4 *>(a.stencil);
    uint64_t *mrow = a.mask + (base >> 6);
    // the tile's status words through the scalar cache: a wave reads each of
    // its words once, before it rewrites that word, and no other wave reads it
    const cu64_t *mks = (const cu64_t *)mrow;
    const int64_t row = tile * 64 + lane;
    // the loads that depend on the tile alone, requested together before any
    // of them is waited for (unconditional, in-bounds indexes): the staging
    // then waits for one memory round trip before its gathers
    const int nbv = TPW == 0 ? a.st_nbr[48 * stid + min(gt, NNB - 1)] : a.tile_nbr[27 * tile + min(gt, NNB - 1)];
    const uint32_t auxv = a.aux[row];
    const int4 own = sh[row];
    const float ri = qr[row].y;
    // box points of this thread; threads past the last point redo it (the
    // same value into the same slot)
    // (act[i]: some thread of this wave has a point in round i)
    int hp[MS];
    bool act[MS];
#pragma unroll
    for (int i = 0; i < MS; i++) {
        act[i] = (gt & ~63) + i * GR::NT < npts;
        hp[i] = hpos[min(gt + i * GR::NT, npts - 1)];
    }
    if (gt < NNB) stn[gt] = nbv;
    // largest |a| of the staged box points (float bits), reduced in LDS
    unsigned int *amw = reinterpret_cast<unsigned int *>(stn) + (TPW == 0 ? 63 : 31);
    if (gt == 0) *amw = 0u;
    // the tile's bond range and the shadow scale arrive with the loads above
    // (not requested later, next to their first use)
    asm volatile("" ::"s"(base), "s"(L4), "s"(Q));
    const int G4 = L4 >> 2;
    // this wave's groups of entries: kq, kq + SPLIT, ... (interleaved, so
    // that every wave gets bonds of every length and direction, and the
    // rechecks of a strained direction are shared among the waves)
    constexpr int GS = GR::SPLIT;
    const int g0 = kq;
    uint64_t mw[4];  // this wave's first status words (requested with the gathers)
    const uint32_t spi = tile_specimen(auxv);
    // reference point: the shadow of the tile's centre lattice point, or of
    // its first node if the centre is padding (V = 0); zero if a sentinel
    // (every component read, so that the row's record is one load)
    const uint64_t nodes = __ballot(own.w != 0);
    const int lc = (a.tile[0] >> 1) + a.tile[0] * ((a.tile[1] >> 1) + a.tile[1] * (a.tile[2] >> 1));
    const int lr = ((nodes >> lc) & 1ull) || !nodes ? lc : (int)__builtin_ctzll(nodes);
    const int r0 = __builtin_amdgcn_readlane(own.x, lr);
    const int r1 = __builtin_amdgcn_readlane(own.y, lr);
    const int r2 = DIM == 3 ? __builtin_amdgcn_readlane(own.z, lr) : 0;
    const bool rsent = r0 == PD_SENTINEL_T;
    int rx = rsent ? 0 : r0;
    int ry = rsent ? 0 : r1;
    int rz = rsent ? 0 : r2;
    int *rfl = stn + NNB;
    if constexpr (TPW == 0) {
        // one reference for the shared box: that of the first quadrant with a
        // tile (a wave without a tile took that tile's rows, so any wave with
        // the first tile can write it)
        if (valid && lane == 0 && tile == first_st_tile(a, stid)) {
            rfl[0] = rx;
            rfl[1] = ry;
            rfl[2] = rz;
        }
    }
    tile_sync<TPW>();
    // every load issued so far has arrived (they were requested together):
    // said explicitly, so that the gathers below, issued round by round, are
    // not held up by waits the compiler would otherwise place for them
    __builtin_amdgcn_s_waitcnt(0);
    if constexpr (TPW == 0) {
        rx = rfl[0];
        ry = rfl[1];
        rz = rfl[2];
    }
    bool sent = false;
    // the specimen's constants, requested before the gathers (so that their
    // wait does not include them)
    const pd_spec sp = a.spec[spi];
    {
        uint32_t rw[MS];
#pragma unroll
        for (int i = 0; i < MS; i++) {
            const int h = hp[i] & ((1 << HB) - 1);
            const int nt = act[i] ? stn[h >> 6] : 0;
            // no tile in that direction: any row of this tile (finite values on a
            // point no intact bond reaches)
            rw[i] = (uint32_t)(nt < 0 ? (int)tile : nt) * 64u + (uint32_t)(h & 63);
        }
        int4 v[MS];
        float r[MS];
#pragma unroll
        for (int i = 0; i < MS; i++) {
            if (!act[i]) continue;
            v[i] = sh[rw[i]];
            r[i] = qr[rw[i]].y;
        }
        // the first status words of the sweep, requested once the gathers are
        // in flight (scalar reads in flight would hold up every wait for LDS
        // data before them)
#pragma unroll
        for (int c = 0; c < 4; c++) mw[c] = g0 < G4 ? mks[4 * g0 + c] : 0ull;
        const float GQ = (float)(sp.G * Q);  // extension carried in units of Q
        float amx = 0.0f;  // largest |a| of this thread's node points (sentinels aside)
        bool badv = false;  // UV: a staged node volume other than the constant
#pragma unroll
        for (int i = 0; i < MS; i++) {
            if (!act[i]) continue;
            const bool st = v[i].x == PD_SENTINEL_T;
            sent |= st;
            const float Vv = __int_as_float(v[i].w);
            const float ax = idiff(v[i].x, rx), ay = idiff(v[i].y, ry), az = DIM == 3 ? idiff(v[i].z, rz) : 0.0f;
            // padding points (V = 0) end no bond
            if (!st && Vv != 0.0f) amx = fmaxf(amx, fmaxf(fabsf(ax), fmaxf(fabsf(ay), fabsf(az))));
            if (UV) badv |= Vv != 0.0f && Vv != box.Vu;
            box.put(hp[i] >> HB, st ? __builtin_inff() : ax, ay, az, Vv, GQ * r[i] * Vv);
        }
        const unsigned int wam = wave_max_bits(amx);
        if (lane == 0) atomicMax(amw, wam);
        if (UV && __ballot(badv) && lane == 0) atomicOr(&ctl->flags, PD_CTL_VOLUME);
    }
    const bool anysent = tile_sync_or<TPW>(sent);
    // a super-tile quadrant without a tile has nothing more to do (no later
    // workgroup barrier in this mode)
    if (TPW == 0 && !valid) return;
    if (BREAK && valid && tile == 0 && (TPW == 1 ? gt < 64 : true)) {
        // one whole wave: the next shadow's scale from this shadow's maximum,
        // and the next maximum cleared for pass 2
        const unsigned int um = umax_wave(ctl, cur, lane);
        umax_clear_wave(ctl, cur ^ 1, lane);
        if (lane == 0) {
            ctl->s1 = ctl->s2;
            ctl->qs[cur ^ 1] = shadow_scale_t(um);
        }
    }
    const float GQ = (float)(sp.G * Q);  // extension carried in units of Q
    const int my = TPW == 0 ? own_slot_st<DIM>(a.reach, sub, lane) : own_slot1<DIM>(a.tile, a.reach, B1, lane);
    float aix, aiy, aiz;
    box.pos(my, aix, aiy, aiz);
    const float big_i = big_abs(aix) + big_abs(aiy) + big_abs(aiz);
    const float rpi = GQ * ri;
    const double s0 = sp.s0;
    // breaking threshold in units of Q, widened by the float rounding of the test
    const double invQ = inv_pow2(Q);
    const float thrQ = (float)(s0 * invQ) * (1.0f - 1e-6f);
    // screen on e': below thr_lo no bond of the box can reach the threshold.
    // With a the largest staged |a| of a node point of the box, D <= 6 a
    // and A <= 6 a (A only if a >= 2^24), so the band of every bond is at
    // most (sqrt(3) + 2^-21 6 a + 2^-24 6 a) / x; entry 0 is a shortest
    // bond of the stencil (the bound widened for its own float rounding)
    const float am = __uint_as_float(*amw);
    const float band = 1.7320509f + 2.8610229e-6f * am + (am >= 16777216.0f ? 3.5762787e-7f * am : 0.0f);
    const float thr_lo = thrQ * (1.0f - 9.5367432e-7f) - (band * 1.001f + 1.0f) * kt[0].ix;
    float acc = 0.0f, fx = 0.0f, fy = 0.0f, fz = 0.0f;
    uint32_t nbroken = 0, nrecheck = 0, nfall = 0;
    double dd0 = 0.0, dd1 = 0.0, dd2 = 0.0;
    float mmin = __builtin_inff();  // smallest |s - s_c| / s_c decided in double

    // double bond strain e / x of bond k of this row (canonical order, from
    // the double state); a break takes the bond out of the row's D_i
    auto decide = [&](int k, bool &broke) -> double {
        const uint32_t w = a.words[pd_widx(base, k, lane)];
        const double4 ui = uv[row], uj = uv[w >> 7];
        const double4 sd = sten[k];
        const double e64 = ext_canonical_t(sd.x, sd.y, DIM == 3 ? sd.z : 0.0, uj.x - ui.x, uj.y - ui.y,
                                           DIM == 3 ? uj.z - ui.z : 0.0);
        const double st = e64 / sd.w;
        if (BREAK) mmin = fminf(mmin, (float)(fabs(st - s0) / s0));
        if (BREAK && st >= s0) {
            broke = true;
            const double xv = sd.w * uj.w;
            dd0 += xv * sd.x;
            dd1 += xv * sd.y;
            dd2 += xv * sd.z;
        }
        return st;
    };

    // one group of four stencil entries with its status words mm; requests
    // the status words of group gn into mn
    auto group = [&](auto chk, int gg, const uint64_t(&mm)[4], uint64_t(&mn)[4], int gn) {
        constexpr bool CHK = decltype(chk)::value;
        {
            KEnt1 e[4];
            float ajx[4], ajy[4], ajz[4], vj[4], hj[4], evs[4];
#pragma unroll
            for (int c = 0; c < 4; c++) e[c] = kn[4 * gg + c];  // a 4 KiB table: scalar-cache hits
            // the mirror rows' x^2 and x M are not used; naming them keeps the
            // four rows two whole 64-byte scalar loads, waited for once
            // before the LDS reads (a partial row would be loaded piecewise,
            // and a later wait would hold the LDS reads issued before it)
            asm volatile("" ::"s"(e[1].x2), "s"(e[1].xm0), "s"(e[1].xm1), "s"(e[1].xm2), "s"(e[3].x2),
                         "s"(e[3].xm0), "s"(e[3].xm1), "s"(e[3].xm2));
#pragma unroll
            for (int c = 0; c < 4; c++) box.get(my + e[c].soff, ajx[c], ajy[c], ajz[c], vj[c], hj[c]);
#pragma unroll
            for (int c = 0; c < 4; c++) {
                const float fdx = ajx[c] - aix, fdy = ajy[c] - aiy;
                const float fdz = DIM == 3 ? ajz[c] - aiz : 0.0f;
                float ev = e[c].mx0 * fdx + e[c].mx1 * fdy;  // e / (x Q)
                if (DIM == 3) ev += e[c].mx2 * fdz;
                evs[c] = ev;
            }
            // the next group's status words (inside this wave's range), requested
            // only once this group's LDS reads have been consumed: scalar and
            // LDS reads share one completion counter, so a scalar read in
            // flight would hold up the wait for the LDS data (the empty asm
            // pins the strains and the staged values here and keeps the
            // scalar reads after them)
            if constexpr (UV) {  // (V a constant: not pinned, or it would be copied per entry)
                asm volatile("" : "+v"(evs[0]), "+v"(evs[1]), "+v"(evs[2]), "+v"(evs[3]), "+v"(hj[0]), "+v"(hj[1]),
                             "+v"(hj[2]), "+v"(hj[3])::"memory");
            } else {
                asm volatile("" : "+v"(evs[0]), "+v"(evs[1]), "+v"(evs[2]), "+v"(evs[3]), "+v"(vj[0]), "+v"(vj[1]),
                             "+v"(vj[2]), "+v"(vj[3]), "+v"(hj[0]), "+v"(hj[1]), "+v"(hj[2]), "+v"(hj[3])::"memory");
            }
#pragma unroll
            for (int c = 0; c < 4; c++) mn[c] = mks[4 * gn + c];
            uint64_t live[4], fbm[4];
#pragma unroll
            for (int c = 0; c < 4; c++) {
                live[c] = mm[c];
                fbm[c] = 0ull;
            }
            if (CHK) {
#pragma unroll
                for (int c = 0; c < 4; c++) {
                    // intact bonds next to a sentinel: strain (and decision) from the
                    // double state, taken out of the screen below
                    int so = e[c].soff;
                    asm volatile("" : "+s"(so));
                    float bx, by, bz;
                    box.pos(my + so, bx, by, bz);
                    fbm[c] = __ballot(__builtin_isinf(aix) || __builtin_isinf(bx)) & live[c];
                    if (fbm[c]) {
                        nfall += __popcll(fbm[c]);
                        bool broke = false;
                        if (lane_bit(fbm[c])) evs[c] = (float)(decide(4 * gg + c, broke) * invQ);
                        const uint64_t bb = BREAK ? __ballot(broke) : 0ull;
                        if (bb) {
                            live[c] &= ~bb;
                            if (lane == 0 && valid) mrow[4 * gg + c] = live[c];
                            nbroken += __popcll(bb);
                        }
                    }
                }
            }
            if (BREAK) {
                // the screen of the four entries, one branch for the group
                uint64_t maybe[4];
#pragma unroll
                for (int c = 0; c < 4; c++) maybe[c] = __ballot(evs[c] >= thr_lo) & live[c] & ~fbm[c];
                if (maybe[0] | maybe[1] | maybe[2] | maybe[3]) {
#pragma unroll
                    for (int c = 0; c < 4; c++) {
                        if (!maybe[c]) continue;
                        const int k = 4 * gg + c;
                        // the neighbour's staged values read again (through an
                        // opaque offset: not kept in registers for this rare test)
                        int so = e[c].soff;
                        asm volatile("" : "+s"(so));
                        float bx, by, bz;
                        box.pos(my + so, bx, by, bz);
                        const float xk = kt[k].x;
                        const float sd = fabsf(bx - aix) + fabsf(by - aiy) + (DIM == 3 ? fabsf(bz - aiz) : 0.0f);
                        const float sa = big_abs(bx) + big_abs(by) + (DIM == 3 ? big_abs(bz) : 0.0f) + big_i;
                        const float lim = thrQ * xk - 1.7320509f;
                        const bool need = lane_bit(maybe[c]) &&
                                          fmaf(1.1920929e-7f, sa, fmaf(9.5367432e-7f, sd, evs[c] * xk)) >= lim;
                        const uint64_t needm = __ballot(need);
                        if (needm) {
                            nrecheck += __popcll(needm);
                            bool broke = false;
                            if (need) (void)decide(k, broke);
                            const uint64_t bb = __ballot(broke);
                            if (bb) {
                                live[c] &= ~bb;
                                if (lane == 0 && valid) mrow[k] = live[c];
                                nbroken += __popcll(bb);
                            }
                        }
                    }
                }
            }
            // entries c and c + 1 are a bond and its mirror (the opposite
            // offset: the same x^2, x M negated), summed as one term
#pragma unroll
            for (int c = 0; c < 4; c += 2) {
                const float ea = lane_bit(live[c]) ? evs[c] : 0.0f;  // broken bonds carry nothing
                const float eb = lane_bit(live[c + 1]) ? evs[c + 1] : 0.0f;
                // dilatation: x V_j e = x^2 V_j e'
                acc = fmaf(e[c].x2, fmaf(vj[c + 1], eb, vj[c] * ea), acc);
                // deviatoric force: G e (1/m_i + 1/m_j) V_j M, with M of the mirror = -M
                const float te = ea * fmaf(rpi, vj[c], hj[c]) - eb * fmaf(rpi, vj[c + 1], hj[c + 1]);
                fx = fmaf(te, e[c].xm0, fx);
                fy = fmaf(te, e[c].xm1, fy);
                if (DIM == 3) fz = fmaf(te, e[c].xm2, fz);
            }
        }
    };
    // groups in pairs with two sets of status words, so that the words in
    // flight are never copied (a copy would wait for them)
    auto sweep = [&](auto chk) {
        uint64_t ma[4], mb[4];
#pragma unroll
        for (int c = 0; c < 4; c++) ma[c] = mw[c];
        for (int gg = g0; gg < G4; gg += 2 * GS) {
            const int g2 = gg + GS;  // the group after gg (if any: else gg's words again)
            group(chk, gg, ma, mb, g2 < G4 ? g2 : gg);
            if (g2 < G4) group(chk, g2, mb, ma, g2 + GS < G4 ? g2 + GS : g2);
        }
    };
    if (anysent) sweep(std::true_type{});
    else sweep(std::false_type{});

    if (BREAK && valid) {
        if (lane == 0 && nbroken) atomicAdd(&ctl->broken, (unsigned long long)nbroken);
        if (lane == 0 && nrecheck) atomicAdd(&ctl->rechecks, (unsigned long long)nrecheck);
        if (lane == 0 && nfall) atomicAdd(&ctl->fallbacks, (unsigned long long)nfall);
        if (nrecheck | nfall) margin_merge(mmin, &ctl->margin_key);
    }
    float tot[4] = {acc, fx, fy, fz};
    double d[3] = {dd0, dd1, dd2};
    if constexpr (TPW == 1) {
        __syncthreads();  // every wave is done with the staged box
        float *red = reinterpret_cast<float *>(smem);                                              // [4][waves][64]
        double *redd = reinterpret_cast<double *>(smem + 4 * PD_TILE_WAVES * 64 * sizeof(float));  // [3][waves][64]
#pragma unroll
        for (int v = 0; v < 4; v++) red[(v * PD_TILE_WAVES + wv) * 64 + lane] = tot[v];
        if (BREAK) {
#pragma unroll
            for (int v = 0; v < 3; v++) redd[(v * PD_TILE_WAVES + wv) * 64 + lane] = d[v];
        }
        __syncthreads();
        if (wv != 0) return;
#pragma unroll
        for (int v = 0; v < 4; v++) {
            tot[v] = red[v * PD_TILE_WAVES * 64 + lane];
            for (int q = 1; q < PD_TILE_WAVES; q++) tot[v] += red[(v * PD_TILE_WAVES + q) * 64 + lane];
        }
        if (BREAK) {
            // bonds of this row broken in this step leave D_i, in wave order
#pragma unroll
            for (int v = 0; v < 3; v++) {
                d[v] = 0.0;
                for (int q = 0; q < PD_TILE_WAVES; q++) d[v] += redd[(v * PD_TILE_WAVES + q) * 64 + lane];
            }
        }
    }
    if (!valid) return;
    if (BREAK && (d[0] != 0.0 || d[1] != 0.0 || d[2] != 0.0)) {
        double4 D = ldv(a.dsum, DIM, row);
        D.x -= d[0];
        D.y -= d[1];
        D.z -= d[2];
        stv(a.dsum, DIM, row, D);
    }
    // theta_i / m_i = A r_i^2 sum_j x V_j e_j, the sum carried in units of Q;
    // pass 2 stages it with V_i
    const double accQ = (double)tot[0] * Q;
    const float qi = (float)((double)sp.A * (double)ri * (double)ri * accQ);
    // (the gather kernels' qr32.x is not needed: pass 2 here reads qv32)
    a.qv32[row] = make_float2(qi, __int_as_float(own.w));
    if (a.theta_out) a.theta_out[row] = (double)sp.A * (double)ri * accQ;
    stvf(a.fe32, DIM, row, make_float4(tot[1], tot[2], tot[3], 0.0f));
}

// ---------------------------------------------------------------------------
// pass 2: dilatational pair force, explicit update, next shadow
// ---------------------------------------------------------------------------
// LDS of one tile in pass 2: (K - G/3) theta/m and V per point in the
// layout of pass 1's box (3D: two float arrays, read with one
// ds_read2st64; 2D: one float2 array), with TPW = 1 the partial sums (3
// floats per thread), then the 27 neighbour tiles.
template <int DIM, int TPW>
struct Lay2 {
    static constexpr int S = Lay1<DIM, TPW>::S;
    static constexpr int BOX = 2 * S * 4;
    static constexpr int SUMS = TPW == 1 ? 3 * PD_TILE_WAVES * 64 * 4 : 0;
    static constexpr int BYTES = BOX + SUMS + (TPW == 0 ? 64 : 32) * 4;
};

template <int DIM, bool UPDATE, int TPW>
__global__ __launch_bounds__(PD_TILE_THREADS) void k_tpass2_f32(StepArgs a, int cur,
                                                                const KEnt1 *__restrict__ kn) {
    extern __shared__ __align__(16) unsigned char smem[];
    using GR = Grp<DIM, TPW>;
    using LY = Lay2<DIM, TPW>;
    constexpr int S = LY::S;
    constexpr int MS = Lay1<DIM, TPW>::MP;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int gt = TPW <= 1 ? tid : lane;
    const int sub = TPW == 1 ? 0 : wv;
    const int kq = TPW == 1 ? wv : 0;
    constexpr int HB = TPW == 0 ? 12 : 11;
    constexpr int NNB = TPW == 0 ? 48 : 27;
    bool valid;
    int64_t stid = 0;
    const int64_t tile = TPW == 0 ? super_tile(a, sub, stid, valid) : group_tile<TPW>(a.n_slices, sub, valid);
    const int64_t base = a.slice_ptr[tile];
    const int L4 = (int)((a.slice_ptr[tile + 1] - base) >> 6);
    unsigned char *reg = smem + (TPW == 4 ? sub * LY::BYTES : 0);
    float *hb = reinterpret_cast<float *>(reg);  // [2][S]: (K - G/3) theta_j/m_j, V_j
    float *red = reinterpret_cast<float *>(reg + LY::BOX);  // TPW = 1: [3][waves][64]
    int *stn = reinterpret_cast<int *>(reg + LY::BOX + LY::SUMS);
    int32_t B1[4];
    pd_tile_box1(a.tile, a.reach, DIM, B1);
    const int npts = TPW == 0 ? a.st_n_pos : a.n_pos;  // box points the stencil reaches
    const int32_t *hpos = TPW == 0 ? a.st_pos : a.halo_pos;
    pd_ctl *ctl = a.ctl;
    const float2 *__restrict__ qvs = a.qv32;
    const int64_t row = tile * 64 + lane;
    const cu64_t *mks = (const cu64_t *)(a.mask + (base >> 6));
    // (act[i]: some thread of this wave has a point in round i)
    int hp[MS];
    bool act[MS];
#pragma unroll
    for (int i = 0; i < MS; i++) {
        act[i] = (gt & ~63) + i * GR::NT < npts;
        hp[i] = act[i] ? hpos[min(gt + i * GR::NT, npts - 1)] : 0;
    }
    if (gt < NNB) stn[gt] = TPW == 0 ? a.st_nbr[48 * stid + gt] : a.tile_nbr[27 * tile + gt];
    const int G4 = L4 >> 2;
    const int gper = (G4 + GR::SPLIT - 1) / GR::SPLIT;
    const int g0 = kq * gper, g1 = min(G4, g0 + gper);
    uint64_t mw[4];
#pragma unroll
    for (int c = 0; c < 4; c++) mw[c] = g0 < g1 ? mks[4 * g0 + c] : 0ull;
    const uint32_t aux = a.aux[row];
    const pd_spec sp = a.spec[tile_specimen(aux)];
    const float kp = (float)sp.kp;
    // the row's own data for the update, requested now by the wave that
    // finishes the rows, so that it arrives during the staging and the sweep
    double4 ui = make_double4(0.0, 0.0, 0.0, 0.0), D = ui, v = ui;
    float4 fe = make_float4(0.f, 0.f, 0.f, 0.f);
    if (kq == 0 && valid) {
        ui = a.uv[cur][row];
        D = ldv(a.dsum, DIM, row);
        fe = ldvf(a.fe32, DIM, row);
        if (UPDATE) v = ldv(a.vel, DIM, row);
    }
    tile_sync<TPW>();
    {
        uint32_t rw[MS];
#pragma unroll
        for (int i = 0; i < MS; i++) {
            const int h = hp[i] & ((1 << HB) - 1);
            const int nt = act[i] ? stn[h >> 6] : 0;
            rw[i] = (uint32_t)(nt < 0 ? (int)tile : nt) * 64u + (uint32_t)(h & 63);
        }
        float2 qv[MS];  // (theta/m, V) of the point, one 8-byte record
#pragma unroll
        for (int i = 0; i < MS; i++)
            if (act[i]) qv[i] = qvs[rw[i]];
#pragma unroll
        for (int i = 0; i < MS; i++) {
            if (!act[i]) continue;
            const int slot = hp[i] >> HB;
            if constexpr (DIM == 3) {
                hb[slot] = kp * qv[i].x;
                hb[S + slot] = qv[i].y;
            } else {
                reinterpret_cast<float2 *>(hb)[slot] = make_float2(kp * qv[i].x, qv[i].y);
            }
        }
    }
    tile_sync<TPW>();
    if (TPW == 0 && !valid) return;  // no later workgroup barrier in this mode
    const int my = TPW == 0 ? own_slot_st<DIM>(a.reach, sub, lane) : own_slot1<DIM>(a.tile, a.reach, B1, lane);
    const float qi = DIM == 3 ? hb[my] : reinterpret_cast<const float2 *>(hb)[my].x;
    float fx = 0.f, fy = 0.f, fz = 0.f;
    {
        auto group = [&](int gg, const uint64_t(&mm)[4], uint64_t(&mn)[4], int gn) {
            float xm0[4], xm1[4], xm2[4], qj[4], vj[4];
            KEnt1 r[4];
#pragma unroll
            for (int c = 0; c < 4; c++) r[c] = kn[4 * gg + c];  // a 4 KiB table: scalar-cache hits
            // every field named, so that the four rows come in two 64-byte
            // scalar loads, waited for once before the LDS reads
            asm volatile("" ::"s"(r[0].mx0), "s"(r[0].mx1), "s"(r[0].x2), "s"(r[0].mx2), "s"(r[1].mx0),
                         "s"(r[1].mx1), "s"(r[1].x2), "s"(r[1].xm0), "s"(r[1].xm1), "s"(r[1].mx2), "s"(r[1].xm2),
                         "s"(r[2].mx0), "s"(r[2].mx1), "s"(r[2].x2), "s"(r[2].mx2), "s"(r[3].mx0), "s"(r[3].mx1),
                         "s"(r[3].x2), "s"(r[3].xm0), "s"(r[3].xm1), "s"(r[3].mx2), "s"(r[3].xm2));
#pragma unroll
            for (int c = 0; c < 4; c++) {
                const KEnt1 &e = r[c];
                xm0[c] = e.xm0;
                xm1[c] = e.xm1;
                xm2[c] = e.xm2;
                if constexpr (DIM == 3) {
                    qj[c] = hb[my + e.soff];
                    vj[c] = hb[S + my + e.soff];
                } else {
                    const float2 t = reinterpret_cast<const float2 *>(hb)[my + e.soff];
                    qj[c] = t.x;
                    vj[c] = t.y;
                }
            }
            // next group's status words once this group's LDS reads are consumed
            // (scalar and LDS reads share one completion counter)
            asm volatile("" : "+v"(qj[0]), "+v"(qj[1]), "+v"(qj[2]), "+v"(qj[3]), "+v"(vj[0]), "+v"(vj[1]),
                         "+v"(vj[2]), "+v"(vj[3])::"memory");
#pragma unroll
            for (int c = 0; c < 4; c++) mn[c] = mks[4 * gn + c];
            // entries c and c + 1 are a bond and its mirror (x M negated)
#pragma unroll
            for (int c = 0; c < 4; c += 2) {
                // (K - G/3) (q_j - q_i) V_j, times x M from the table
                float ta = (qj[c] - qi) * vj[c], tb = (qj[c + 1] - qi) * vj[c + 1];
                ta = lane_bit(mm[c]) ? ta : 0.0f;
                tb = lane_bit(mm[c + 1]) ? tb : 0.0f;
                const float t = ta - tb;
                fx = fmaf(t, xm0[c], fx);
                fy = fmaf(t, xm1[c], fy);
                if (DIM == 3) fz = fmaf(t, xm2[c], fz);
            }
        };
        // groups in pairs with two sets of status words (no copy of words in flight)
        uint64_t ma[4], mb[4];
#pragma unroll
        for (int c = 0; c < 4; c++) ma[c] = mw[c];
        for (int gg = g0; gg < g1; gg += 2) {
            group(gg, ma, mb, min(gg + 1, g1 - 1));
            if (gg + 1 < g1) group(gg + 1, mb, ma, min(gg + 2, g1 - 1));
        }
    }
    float sx = fx, sy = fy, sz = fz;
    if constexpr (TPW == 1) {
        red[(0 * PD_TILE_WAVES + wv) * 64 + lane] = fx;
        red[(1 * PD_TILE_WAVES + wv) * 64 + lane] = fy;
        red[(2 * PD_TILE_WAVES + wv) * 64 + lane] = fz;
        __syncthreads();
        if (wv != 0) return;
        sx = red[lane];
        sy = red[PD_TILE_WAVES * 64 + lane];
        sz = red[2 * PD_TILE_WAVES * 64 + lane];
        for (int q = 1; q < PD_TILE_WAVES; q++) {
            sx += red[q * 64 + lane];
            sy += red[(PD_TILE_WAVES + q) * 64 + lane];
            sz += red[(2 * PD_TILE_WAVES + q) * 64 + lane];
        }
    }
    if (!valid) return;
    // dilatational sum in difference form plus its row constant 2 (K - G/3) q_i D_i,
    // deviatoric sum from pass 1; all times V_i
    const double c2 = 2.0 * (double)qi;
    double Fx = ((double)sx + (double)fe.x + c2 * D.x) * ui.w;
    double Fy = ((double)sy + (double)fe.y + c2 * D.y) * ui.w;
    double Fz = ((double)sz + (double)fe.z + c2 * D.z) * ui.w;
    if (!UPDATE) {
        a.f_out[row] = make_double4(Fx, Fy, Fz, 0.0);
        return;
    }
    const int64_t n = ctl->s1;
    if (tile == 0 && (TPW == 1 ? gt == 0 : lane == 0)) {
        ctl->s2 = n + 1;
        // the next shadow written below describes the new state
        ctl->sh_step = n + 1;
        ctl->sh_cur = cur ^ 1;
    }
    const double Qn = ctl->qs[cur ^ 1];
    double r = 1.0;
    if (a.ramp_steps > 0) r = n >= a.ramp_steps ? 1.0 : (double)n / (double)a.ramp_steps;
    if (aux & 8u) {
        const double4 fx4 = a.fext[row];
        Fx += fx4.x * r;
        Fy += fx4.y * r;
        Fz += fx4.z * r;
    }
    const double mass = sp.rho * ui.w;
    const double ax = (aux & 1u) ? 0.0 : Fx / mass;
    const double ay = (aux & 2u) ? 0.0 : Fy / mass;
    const double az = (aux & 4u) ? 0.0 : Fz / mass;
    v.x = v.x + sp.dt * ax;
    v.y = v.y + sp.dt * ay;
    v.z = v.z + sp.dt * az;
    double4 u = ui;
    u.x = u.x + sp.dt * v.x;
    u.y = u.y + sp.dt * v.y;
    u.z = u.z + sp.dt * v.z;
    a.uv[cur ^ 1][row] = u;
    stv(a.vel, DIM, row, v);
    const double invQn = inv_pow2(Qn);
    bool bad = false;
    int4 s;
    s.x = quantise_t(u.x, invQn, bad);
    s.y = quantise_t(u.y, invQn, bad);
    s.z = quantise_t(u.z, invQn, bad);
    s.w = __float_as_int((float)ui.w);
    if (bad) s.x = PD_SENTINEL_T;
    a.ush[cur ^ 1][row] = s;
    float m = (float)fmax(fabs(u.x), fmax(fabs(u.y), fabs(u.z)));
    const bool finite = isfinite(u.x) && isfinite(u.y) && isfinite(u.z);
    if (!finite) m = 0.0f;
    m = __uint_as_float(__float_as_uint(m) + 1u);
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
    // into the slot of this tile's class: the slots spread the tiles' atomics
    // over 64 lines, so no read of the running maximum has to filter them
    if (lane == 0) atomicMax(&ctl->umax_slot[cur ^ 1][(tile % PD_UMAX_SLOTS) * PD_UMAX_STRIDE], __float_as_uint(m));
    if (__ballot(!finite) && lane == 0) atomicOr(&ctl->flags, PD_CTL_NONFINITE);
    if (__ballot(bad) && lane == 0) atomicOr(&ctl->flags, PD_CTL_FALLBACK);
}

// ---------------------------------------------------------------------------
// D_i = sum over intact bonds of x M V_j (double precision), the row constant
// of the difference form of the dilatation term
// ---------------------------------------------------------------------------
template <int DIM>
__global__ __launch_bounds__(PD_TILE_THREADS) void k_tdsum(StepArgs a, int cur, const KEnt *__restrict__ kt,
                                                           const double4 *__restrict__ sten) {
    extern __shared__ __align__(16) unsigned char smem[];
    if (a.ctl->sh_skip) return;
    constexpr int MS = StageCap<DIM>::value;
    const Box g = make_box(a, DIM);
    const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const int tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t base = a.slice_ptr[tile];
    const int L4 = (int)((a.slice_ptr[tile + 1] - base) >> 6);
    double *hv = reinterpret_cast<double *>(smem);
    uint64_t *smask = reinterpret_cast<uint64_t *>(hv + g.nslot);
    double *red = reinterpret_cast<double *>(smask + 128);
    int *stn = reinterpret_cast<int *>(red + 3 * PD_TILE_WAVES * 64);
    const double4 *__restrict__ uv = a.uv[cur];
    int hmv[MS];
#pragma unroll
    for (int i = 0; i < MS; i++) {
        const int s = tid + i * PD_TILE_THREADS;
        hmv[i] = s < g.nslot ? a.halo_map[s] : -1;
    }
    if (tid < 27) stn[tid] = a.tile_nbr[27 * tile + tid];
    const uint64_t mword = tid < L4 ? a.mask[(base >> 6) + tid] : 0ull;
    __syncthreads();
    {
        int64_t rw[MS];
        double v[MS];
#pragma unroll
        for (int i = 0; i < MS; i++) {
            rw[i] = halo_row_of(hmv[i], stn);
        }
#pragma unroll
        for (int i = 0; i < MS; i++) v[i] = rw[i] >= 0 ? uv[rw[i]].w : 0.0;
#pragma unroll
        for (int i = 0; i < MS; i++) {
            const int s = tid + i * PD_TILE_THREADS;
            if (s < g.nslot) hv[s] = v[i];
        }
    }
    if (tid < 128) smask[tid] = mword;
    __syncthreads();
    const int my = own_slot<DIM>(g, lane);
    const int G4 = L4 >> 2;
    const int gper = (G4 + PD_TILE_WAVES - 1) / PD_TILE_WAVES;
    const int g0 = wv * gper, g1 = min(G4, g0 + gper);
    double d0 = 0.0, d1 = 0.0, d2 = 0.0;
    const int ns = a.n_stencil;
    for (int k = 4 * g0; k < 4 * g1; k++) {
        const double Vj = hv[my + kt[k].soff];
        const double4 sd = sten[min(k, ns - 1)];  // entries past n_stencil are padding (status bits 0)
        const double xv = lane_bit(uni64_t(smask[k])) ? sd.w * Vj : 0.0;
        d0 += xv * sd.x;
        d1 += xv * sd.y;
        if (DIM == 3) d2 += xv * sd.z;
    }
    red[(0 * PD_TILE_WAVES + wv) * 64 + lane] = d0;
    red[(1 * PD_TILE_WAVES + wv) * 64 + lane] = d1;
    red[(2 * PD_TILE_WAVES + wv) * 64 + lane] = d2;
    __syncthreads();
    if (wv != 0) return;
    double s0 = red[lane], s1 = red[PD_TILE_WAVES * 64 + lane], s2 = red[2 * PD_TILE_WAVES * 64 + lane];
    for (int q = 1; q < PD_TILE_WAVES; q++) {
        s0 += red[q * 64 + lane];
        s1 += red[(PD_TILE_WAVES + q) * 64 + lane];
        s2 += red[(2 * PD_TILE_WAVES + q) * 64 + lane];
    }
    stv(a.dsum, DIM, tile * 64 + lane, make_double4(s0, s1, s2, 0.0));
}

static size_t tdsum_lds(const StepArgs &a) {
    int32_t B[4];
    pd_tile_box(a.tile, a.reach, a.dim, B);
    const size_t nslot = (size_t)B[3] * B[2];
    return nslot * sizeof(double) + 128 * sizeof(uint64_t) + 3 * PD_TILE_WAVES * 64 * sizeof(double) +
           32 * sizeof(int);
}

hipError_t launch_tdsum(const StepArgs &a, int cur, hipStream_t s) {
    const dim3 g((unsigned)a.n_slices), b(PD_TILE_THREADS);
    const KEnt *kt = reinterpret_cast<const KEnt *>(a.ktab);
    const double4 *sten = reinterpret_cast<const double4 *>(a.stencil);
    if (a.dim == 3) hipLaunchKernelGGL((k_tdsum<3>), g, b, tdsum_lds(a), s, a, cur, kt, sten);
    else hipLaunchKernelGGL((k_tdsum<2>), g, b, tdsum_lds(a), s, a, cur, kt, sten);
    return hipGetLastError();
}

static int box_slots(const StepArgs &a) {
    int32_t B[4];
    pd_tile_box(a.tile, a.reach, a.dim, B);
    return B[3] * B[2];
}

static int box_points(const StepArgs &a) { return pd_box_points(a.tile, a.reach, a.dim); }

static_assert(Lay1<3, 1>::S == 1472 && Lay1<2, 4>::S == 336 && Lay1<2, 1>::S == 1024,
              "pass-1 array strides follow pd_box1_stride");

static size_t tiled_lds(const StepArgs &a, int pass, int tpw) {
    if (pass == 1 && a.dim == 3) return a.vol_uniform > 0.0f ? Lay1<3, 1, true>::BYTES : Lay1<3, 1>::BYTES;
    if (pass == 1) return tpw == 4 ? 4 * Lay1<2, 4>::BYTES : Lay1<2, 1>::BYTES;
    return a.dim == 3 ? Lay2<3, 1>::BYTES : (tpw == 4 ? 4 * Lay2<2, 4>::BYTES : Lay2<2, 1>::BYTES);
}

bool tiled_supported(const StepArgs &a) {
    if (!a.tile_nbr || !a.ktab || !a.halo_map || !a.halo_pos || !a.qv32) return false;
    if (a.tile[0] * a.tile[1] * a.tile[2] != 64) return false;
    for (int c = 0; c < 3; c++)
        if (a.tile[c] < 1 || (a.tile[c] & (a.tile[c] - 1))) return false;  // powers of two
    if (a.reach < 1 || a.tile[0] < a.reach || a.tile[1] < a.reach) return false;
    if (a.dim == 3 && a.tile[2] < a.reach) return false;
    if (a.dim == 2 && a.tile[2] != 1) return false;
    if (a.n_stencil > 124) return false;  // groups of four inside the 128-row table
    const int ns = box_slots(a), np = a.n_pos;
    if (np < 1 || np > box_points(a)) return false;
    const int tpw = tiles_per_group(a, box_points(a));
    const int cap = a.dim == 3 ? Grp<3, 1>::CAP : (tpw == 4 ? Grp<2, 4>::CAP : Grp<2, 1>::CAP);
    if (ns > cap || np > cap || np < 1) return false;
    int32_t B1[4];
    pd_tile_box1(a.tile, a.reach, a.dim, B1);
    if (B1[3] * B1[2] > pd_box1_stride(a.dim, box_points(a))) return false;
    const int cap1 = a.dim == 3 ? 256 * Lay1<3, 1>::MP : (tpw == 4 ? 64 * Lay1<2, 4>::MP : 256 * Lay1<2, 1>::MP);
    if (np > cap1) return false;
    if (a.n_pad >= (int64_t(1) << 31)) return false;  // 32-bit row numbers in the staging
    return tiled_lds(a, 1, tpw) <= 64 * 1024 && tiled_lds(a, 2, tpw) <= 64 * 1024;
}

bool supertiles_supported(const StepArgs &a) {
    if (!tiled_supported(a)) return false;  // the tile path's tables and limits
    if (!a.st_tiles || !a.st_nbr || !a.st_pos || !a.st_ktab || a.n_st < 1 || a.n_st >= (int64_t(1) << 31))
        return false;
    if (a.reach < 1 || a.reach > 3) return false;
    if (a.dim == 3) {
        if (a.tile[0] != 4 || a.tile[1] != 4 || a.tile[2] != 4) return false;
        if (a.st_n_pos < 1 || a.st_n_pos > Grp<3, 0>::CAP ||
            a.st_n_pos > (8 + 2 * a.reach) * (8 + 2 * a.reach) * (4 + 2 * a.reach))
            return false;
        return Lay1<3, 0>::BYTES <= 64 * 1024 && Lay2<3, 0>::BYTES <= 64 * 1024;
    }
    if (a.tile[0] != 8 || a.tile[1] != 8 || a.tile[2] != 1) return false;
    return a.st_n_pos >= 1 && a.st_n_pos <= Grp<2, 0>::CAP && a.st_n_pos <= (16 + 2 * a.reach) * (16 + 2 * a.reach);
}

template <int DIM>
static hipError_t spass1(const StepArgs &a, int cur, bool brk, hipStream_t s) {
    const dim3 g((unsigned)a.n_st), b(PD_TILE_THREADS);
    const KEnt *kt = reinterpret_cast<const KEnt *>(a.ktab);
    const KEnt1 *kn = reinterpret_cast<const KEnt1 *>(a.st_ktab);
    if constexpr (DIM == 3) {
        if (a.vol_uniform > 0.0f) {
            constexpr size_t lds = Lay1<3, 0, true>::BYTES;
            if (brk) hipLaunchKernelGGL((k_tpass1_f32<3, true, 0, true>), g, b, lds, s, a, cur, kt, kn);
            else hipLaunchKernelGGL((k_tpass1_f32<3, false, 0, true>), g, b, lds, s, a, cur, kt, kn);
            return hipGetLastError();
        }
    }
    constexpr size_t lds = Lay1<DIM, 0>::BYTES;
    if (brk) hipLaunchKernelGGL((k_tpass1_f32<DIM, true, 0>), g, b, lds, s, a, cur, kt, kn);
    else hipLaunchKernelGGL((k_tpass1_f32<DIM, false, 0>), g, b, lds, s, a, cur, kt, kn);
    return hipGetLastError();
}

template <int DIM>
static hipError_t spass2(const StepArgs &a, int cur, bool update, hipStream_t s) {
    const dim3 g((unsigned)a.n_st), b(PD_TILE_THREADS);
    const KEnt1 *kn = reinterpret_cast<const KEnt1 *>(a.st_ktab);
    constexpr size_t lds = Lay2<DIM, 0>::BYTES;
    if (update) hipLaunchKernelGGL((k_tpass2_f32<DIM, true, 0>), g, b, lds, s, a, cur, kn);
    else hipLaunchKernelGGL((k_tpass2_f32<DIM, false, 0>), g, b, lds, s, a, cur, kn);
    return hipGetLastError();
}

hipError_t launch_spass1_f32(const StepArgs &a, int cur, bool brk, hipStream_t s) {
    return a.dim == 3 ? spass1<3>(a, cur, brk, s) : spass1<2>(a, cur, brk, s);
}

hipError_t launch_spass2_f32(const StepArgs &a, int cur, bool update, hipStream_t s) {
    return a.dim == 3 ? spass2<3>(a, cur, update, s) : spass2<2>(a, cur, update, s);
}

hipError_t launch_tpass1_f32(const StepArgs &a, int cur, bool brk, hipStream_t s) {
    const int tpw = tiles_per_group(a, box_points(a));
    const size_t lds = tiled_lds(a, 1, tpw);
    const dim3 g((unsigned)((a.n_slices + tpw - 1) / tpw)), b(PD_TILE_THREADS);
    const KEnt *kt = reinterpret_cast<const KEnt *>(a.ktab);
    const KEnt1 *kn = reinterpret_cast<const KEnt1 *>(a.ktab + 1536);
    if (a.dim == 3 && a.vol_uniform > 0.0f) {
        if (brk) hipLaunchKernelGGL((k_tpass1_f32<3, true, 1, true>), g, b, lds, s, a, cur, kt, kn);
        else hipLaunchKernelGGL((k_tpass1_f32<3, false, 1, true>), g, b, lds, s, a, cur, kt, kn);
    } else if (a.dim == 3) {
        if (brk) hipLaunchKernelGGL((k_tpass1_f32<3, true, 1>), g, b, lds, s, a, cur, kt, kn);
        else hipLaunchKernelGGL((k_tpass1_f32<3, false, 1>), g, b, lds, s, a, cur, kt, kn);
    } else if (tpw == 4) {
        if (brk) hipLaunchKernelGGL((k_tpass1_f32<2, true, 4>), g, b, lds, s, a, cur, kt, kn);
        else hipLaunchKernelGGL((k_tpass1_f32<2, false, 4>), g, b, lds, s, a, cur, kt, kn);
    } else {
        if (brk) hipLaunchKernelGGL((k_tpass1_f32<2, true, 1>), g, b, lds, s, a, cur, kt, kn);
        else hipLaunchKernelGGL((k_tpass1_f32<2, false, 1>), g, b, lds, s, a, cur, kt, kn);
    }
    return hipGetLastError();
}

hipError_t launch_tpass2_f32(const StepArgs &a, int cur, bool update, hipStream_t s) {
    const int tpw = tiles_per_group(a, box_points(a));
    const size_t lds = tiled_lds(a, 2, tpw);
    const dim3 g((unsigned)((a.n_slices + tpw - 1) / tpw)), b(PD_TILE_THREADS);
    const KEnt1 *kn = reinterpret_cast<const KEnt1 *>(a.ktab + 1536);
    if (a.dim == 3) {
        if (update) hipLaunchKernelGGL((k_tpass2_f32<3, true, 1>), g, b, lds, s, a, cur, kn);
        else hipLaunchKernelGGL((k_tpass2_f32<3, false, 1>), g, b, lds, s, a, cur, kn);
    } else if (tpw == 4) {
        if (update) hipLaunchKernelGGL((k_tpass2_f32<2, true, 4>), g, b, lds, s, a, cur, kn);
        else hipLaunchKernelGGL((k_tpass2_f32<2, false, 4>), g, b, lds, s, a, cur, kn);
    } else {
        if (update) hipLaunchKernelGGL((k_tpass2_f32<2, true, 1>), g, b, lds, s, a, cur, kn);
        else hipLaunchKernelGGL((k_tpass2_f32<2, false, 1>), g, b, lds, s, a, cur, kn);
    }
    return hipGetLastError();
}

}  // namespace pdk
