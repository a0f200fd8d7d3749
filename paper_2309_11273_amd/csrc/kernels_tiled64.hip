// LDS-staged ("tiled") kernels of the double-precision matrix-free step.
//
// Same tile layout and workgroup organisation as the single-precision tile
// kernels (kernels_tiled.hip): one workgroup of four waves per 64-point
// tile, the tile plus its R-wide halo staged in LDS, every wave sweeping a
// quarter of the stencil for all 64 rows with wave-uniform entry data, and
// the pair force split between the passes (pass 1 sums the deviatoric part
// G e (1/m_i + 1/m_j) M V_j, which needs the extension; pass 2 the
// dilatational part (K - G/3) x (q_i + q_j) M V_j, q = theta/m).
//
// Everything is double.  The extension is evaluated in the canonical order
// (M1 eta1 + M2 eta2) + M3 eta3 without contraction, so the breaking
// decision s = e/x >= s_c sees exactly the bits the other double paths see;
// a cheap pre-filter e >= s_c (1 - 1e-9) x skips the division for all bonds
// that are clearly below the threshold.
//
// With FIN the kernels evaluate the finite model of Eqs. 1.10, 1.13 instead:
// e = |Y| - x with Y = x M + (u_j - u_i) (|Y|^2 summed (Y1^2 + Y2^2) + Y3^2
// without contraction), both force parts along Y / |Y|; pass 2 then stages
// the displacements as well, to rebuild Y.  |Y| itself is the correctly
// rounded square root (it decides breaking); the direction takes the
// hardware reciprocal square root refined by one Newton step, which costs a
// fraction of a double divide and is accurate to about 1e-13.
//
// LDS holds the staged quantities as separate arrays of doubles at a fixed
// stride (a multiple of 64 elements), so that one address serves all of a
// slot's arrays and pairs of them are fetched by one two-address LDS read.
#include <hip/hip_runtime.h>

#include <cmath>

#include "finite.h"
#include "kernels.h"
#include "tile_common.h"

namespace pdk {

// LDS of one tile: NA arrays of doubles at the fixed stride S (room for every
// slot the tile's thread group can stage, a multiple of 64 elements), then the
// tile's 128 status words and 27 neighbour tiles.  With TPW = 1 the partial
// sums of the four waves reuse the arrays after the sweep.
template <int DIM, int TPW, int NA>
struct Lay64 {
    static constexpr int S = Grp<DIM, TPW>::CAP;
    static constexpr int BYTES = NA * S * 8 + 128 * 8 + 32 * 4;
};
// pass 1: G V/m, u_x, u_y, (u_z,) V;  pass 2: (K - G/3) theta/m, V
// staging and stencil split of the double pass 1 with W waves per workgroup
// (one tile per workgroup: the W waves share the tile's box and its stencil)
template <int DIM, int TPW, int W>
struct Grp64 {
    using G = Grp<DIM, TPW>;
    static constexpr int SPLIT = TPW == 1 ? W : G::SPLIT;
    static constexpr int NT = TPW == 1 ? 64 * W : G::NT;
    static constexpr int MS = TPW == 1 ? (G::CAP + NT - 1) / NT : G::MS;
    static_assert(NT * MS >= G::CAP, "the staging covers the box capacity");
};
template <int DIM>
struct NA1 {
    static constexpr int value = DIM == 3 ? 5 : 4;
};

__device__ __forceinline__ double ext_canonical64(double m1, double m2, double m3, double e1, double e2,
                                                  double e3) {
#pragma clang fp contract(off)
    double a = m1 * e1;
    double b = m2 * e2;
    double c = m3 * e3;
    return (a + b) + c;
}

// deformed bond Y = x M + (dx, dy, dz) and |Y|^2 (finite model)
__device__ __forceinline__ double deformed64(const double4 &sd, double dx, double dy, double dz, double &y1,
                                             double &y2, double &y3) {
#pragma clang fp contract(off)
    y1 = sd.w * sd.x + dx;
    y2 = sd.w * sd.y + dy;
    y3 = sd.w * sd.z + dz;
    return (y1 * y1 + y2 * y2) + y3 * y3;
}

// 1/sqrt(s) for the force direction, where no decision depends on the last
// bits: the hardware estimate refined by one Newton-Raphson step for the
// reciprocal square root, r <- r (3 - s r^2) / 2 (relative error about the
// square of the estimate's)
__device__ __forceinline__ double rsqrt_refined(double s) {
    const double r = __builtin_amdgcn_rsq(s);
    return r * fma(-0.5 * s, r * r, 1.5);
}

// ---------------------------------------------------------------------------
// pass 1: breaking, dilatation, deviatoric pair force
// ---------------------------------------------------------------------------
// W waves per workgroup: with one tile per workgroup (TPW = 1) they split the
// staging and the stencil between them (eight in 3D, where the five staged
// double arrays hold a compute unit to three workgroups)
template <int DIM, bool BREAK, int TPW, bool FIN = false, int W = PD_TILE_WAVES>
__global__ __launch_bounds__(64 * W) void k_tpass1_f64(StepArgs a, int cur, const KEnt *__restrict__ kt,
                                                       const double4 *__restrict__ sten) {
    extern __shared__ __align__(16) unsigned char smem[];
    static_assert(TPW == 1 || W == PD_TILE_WAVES, "several tiles per workgroup take four waves");
    using GR = Grp64<DIM, TPW, W>;
    constexpr int MS = GR::MS;
    constexpr int NA = NA1<DIM>::value;
    using LY = Lay64<DIM, TPW, NA>;
    constexpr int S = LY::S;
    constexpr int IV = NA - 1;  // index of the V array
    const Box g = make_box(a, DIM);
    const int tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int gt = TPW == 1 ? tid : lane;
    const int sub = TPW == 1 ? 0 : wv;
    const int kq = TPW == 1 ? wv : 0;
    bool valid;
    const int64_t tile = group_tile<TPW>(a.n_slices, sub, valid);
    const int64_t base = a.slice_ptr[tile];
    const int L4 = (int)((a.slice_ptr[tile + 1] - base) >> 6);
    double *hA = reinterpret_cast<double *>(smem + sub * LY::BYTES);
    uint64_t *smask = reinterpret_cast<uint64_t *>(hA + NA * S);
    int *stn = reinterpret_cast<int *>(smask + 128);
    pd_ctl *ctl = a.ctl;
    const double4 *__restrict__ uv = a.uv[cur];
    const double2 *__restrict__ qr = a.qr;
    uint64_t *mrow = a.mask + (base >> 6);
    const int64_t row = tile * 64 + lane;
    // the loads that depend on the tile alone, requested together before any
    // of them is waited for (unconditional, in-bounds indexes)
    const int nbv = a.tile_nbr[27 * tile + min(gt, 26)];
    const uint32_t auxv = a.aux[row];
    int hmv[MS];
#pragma unroll
    for (int i = 0; i < MS; i++) {
        const int s = gt + i * GR::NT;
        hmv[i] = s < g.nslot ? a.halo_map[s] : -1;
    }
    if (gt < 27) stn[gt] = nbv;
    asm volatile("" ::"s"(base), "s"(L4));  // the bond range arrives with the loads above
    const uint32_t spi = tile_specimen(auxv);
    __syncthreads();
    const pd_spec sp = a.spec[spi];
    const double G = sp.G;
    uint64_t mw0, mw1;
    {
        int64_t rw[MS];
        double4 u[MS];
        double r[MS];
#pragma unroll
        for (int i = 0; i < MS; i++) {
            rw[i] = halo_row_of(hmv[i], stn);
        }
#pragma unroll
        for (int i = 0; i < MS; i++) {
            u[i] = rw[i] >= 0 ? uv[rw[i]] : make_double4(0.0, 0.0, 0.0, 0.0);
            r[i] = rw[i] >= 0 ? qr[rw[i]].y : 0.0;
        }
        // the tile's status words, requested with the gathers
        mw0 = gt < L4 ? mrow[gt] : 0ull;
        mw1 = (TPW != 1 && gt + 64 < L4) ? mrow[gt + 64] : 0ull;
#pragma unroll
        for (int i = 0; i < MS; i++) {
            const int s = gt + i * GR::NT;
            if (s < g.nslot) {
                hA[s] = G * r[i] * u[i].w;
                hA[S + s] = u[i].x;
                hA[2 * S + s] = u[i].y;
                if (DIM == 3) hA[3 * S + s] = u[i].z;
                hA[IV * S + s] = u[i].w;
            }
        }
    }
    if (gt < 128) smask[gt] = mw0;
    if (TPW != 1) smask[gt + 64] = mw1;
    __syncthreads();
    if (BREAK && valid && tile == 0 && gt == 0) ctl->s1 = ctl->s2;
    const int my = own_slot<DIM>(g, lane);
    const double uix = hA[S + my], uiy = hA[2 * S + my], uiz = DIM == 3 ? hA[3 * S + my] : 0.0;
    const double ri = qr[row].y;
    const double rpi = G * ri;
    const double s0 = sp.s0;
    const double thr_scale = s0 * (1.0 - 1e-9);  // pre-filter, exact test below
    const int ns = a.n_stencil;
    const int G4 = L4 >> 2;
    const int gper = (G4 + GR::SPLIT - 1) / GR::SPLIT;
    const int g0 = kq * gper, g1 = min(G4, g0 + gper);
    double acc = 0.0, fx = 0.0, fy = 0.0, fz = 0.0;
    uint32_t nbroken = 0;
    for (int gg = g0; gg < g1; gg++) {
        double rv[4], ux[4], uy[4], uz[4], vj[4], evk[4];
        double4 sd[4];
        uint64_t mm[4];
#pragma unroll
        for (int c = 0; c < 4; c++) {
            const int k = 4 * gg + c;
            const int slot = my + kt[k].soff;
            sd[c] = sten[min(k, ns - 1)];  // entries past n_stencil are padding (status bits 0)
            rv[c] = hA[slot];
            ux[c] = hA[S + slot];
            uy[c] = hA[2 * S + slot];
            uz[c] = DIM == 3 ? hA[3 * S + slot] : 0.0;
            vj[c] = hA[IV * S + slot];
            mm[c] = uni64_t(smask[k]);
        }
#pragma unroll
        for (int c = 0; c < 4; c++) {
            const int k = 4 * gg + c;
            const double dx = ux[c] - uix, dy = uy[c] - uiy, dz = DIM == 3 ? uz[c] - uiz : 0.0;
            double ev, n1 = sd[c].x, n2 = sd[c].y, n3 = sd[c].z;
            if constexpr (FIN) {
                double y1, y2, y3;
                const double yy = deformed64(sd[c], dx, dy, dz, y1, y2, y3);
                const double yl = sqrt(yy);  // correctly rounded: it decides breaking
                ev = yl - sd[c].w;
                // the deformed direction, taken only for bonds that carry force
                const bool use = lane_bit(mm[c]);
                const double iy = rsqrt_refined(yy);
                n1 = use ? y1 * iy : 0.0;
                n2 = use ? y2 * iy : 0.0;
                n3 = use ? y3 * iy : 0.0;
            } else {
                ev = DIM == 3 ? ext_canonical64(sd[c].x, sd[c].y, sd[c].z, dx, dy, dz)
                              : ext_canonical64(sd[c].x, sd[c].y, 0.0, dx, dy, 0.0);
            }
            uint64_t live = mm[c];
            if (BREAK) {
                const bool need = lane_bit(live) && ev >= thr_scale * sd[c].w;
                const uint64_t needm = __ballot(need);
                if (needm) {
                    const uint64_t bb = __ballot(need && ev / sd[c].w >= s0);
                    if (bb) {
                        live &= ~bb;
                        if (lane == 0 && valid) mrow[k] = live;
                        nbroken += __popcll(bb);
                    }
                }
            }
            if constexpr (FIN) {
                const bool intact = lane_bit(live);
                // dilatation: x V_j e;  deviatoric force: G e (1/m_i + 1/m_j) V_j
                const double xv = sd[c].w * vj[c];
                acc = fma(intact ? xv : 0.0, ev, acc);
                const double te = intact ? ev * fma(rpi, vj[c], rv[c]) : 0.0;
                fx = fma(te, n1, fx);
                fy = fma(te, n2, fy);
                if (DIM == 3) fz = fma(te, n3, fz);
            } else {
                evk[c] = lane_bit(live) ? ev : 0.0;  // broken bonds carry nothing
            }
        }
        if constexpr (!FIN) {
            // entries c and c + 1 are a bond and its mirror (the opposite
            // offset: the same x, M negated), summed as one term
#pragma unroll
            for (int c = 0; c < 4; c += 2) {
                // dilatation: x V_j e;  deviatoric force: G e (1/m_i + 1/m_j) V_j M
                acc = fma(sd[c].w, fma(vj[c + 1], evk[c + 1], vj[c] * evk[c]), acc);
                const double te =
                    evk[c] * fma(rpi, vj[c], rv[c]) - evk[c + 1] * fma(rpi, vj[c + 1], rv[c + 1]);
                fx = fma(te, sd[c].x, fx);
                fy = fma(te, sd[c].y, fy);
                if (DIM == 3) fz = fma(te, sd[c].z, fz);
            }
        }
    }
    if (BREAK && valid && lane == 0 && nbroken) atomicAdd(&ctl->broken, (unsigned long long)nbroken);
    double tot[4] = {acc, fx, fy, fz};
    if constexpr (TPW == 1) {
        __syncthreads();  // every wave is done with the staged box: reuse it for the sums
        double *red = hA;
#pragma unroll
        for (int v = 0; v < 4; v++) red[(v * W + wv) * 64 + lane] = tot[v];
        __syncthreads();
        if (wv != 0) return;
#pragma unroll
        for (int v = 0; v < 4; v++) {
            tot[v] = red[v * W * 64 + lane];
            for (int q = 1; q < W; q++) tot[v] += red[(v * W + q) * 64 + lane];
        }
    }
    if (!valid) return;
    // theta_i = A / m_i * acc; store theta_i / m_i
    a.qr[row].x = sp.A * ri * tot[0] * ri;
    if (a.theta_out) a.theta_out[row] = sp.A * ri * tot[0];
    stv(a.fe64, DIM, row, make_double4(tot[1], tot[2], tot[3], 0.0));
}

// ---------------------------------------------------------------------------
// pass 2: dilatational pair force, explicit update
// ---------------------------------------------------------------------------
template <int DIM, bool UPDATE, int TPW, bool FIN = false>
__global__ __launch_bounds__(PD_TILE_THREADS) void k_tpass2_f64(StepArgs a, int cur, const KEnt *__restrict__ kt,
                                                                const double4 *__restrict__ sten) {
    extern __shared__ __align__(16) unsigned char smem[];
    using GR = Grp<DIM, TPW>;
    constexpr int MS = GR::MS;
    // (K - G/3) theta/m, V; with FIN also u_x, u_y (, u_z)
    constexpr int NA = FIN ? (DIM == 3 ? 5 : 4) : 2;
    using LY = Lay64<DIM, TPW, NA>;
    constexpr int S = LY::S;
    const Box g = make_box(a, DIM);
    const int tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int gt = TPW == 1 ? tid : lane;
    const int sub = TPW == 1 ? 0 : wv;
    const int kq = TPW == 1 ? wv : 0;
    bool valid;
    const int64_t tile = group_tile<TPW>(a.n_slices, sub, valid);
    const int64_t base = a.slice_ptr[tile];
    const int L4 = (int)((a.slice_ptr[tile + 1] - base) >> 6);
    // [0] (K - G/3) theta_j / m_j, [1] V_j; reused for the partial sums
    double *hB = reinterpret_cast<double *>(smem + sub * LY::BYTES);
    uint64_t *smask = reinterpret_cast<uint64_t *>(hB + NA * S);
    int *stn = reinterpret_cast<int *>(smask + 128);
    pd_ctl *ctl = a.ctl;
    const double4 *__restrict__ uv = a.uv[cur];
    const double2 *__restrict__ qr = a.qr;
    const int64_t row = tile * 64 + lane;
    const uint32_t aux = a.aux[row];
    const uint64_t *mrow = a.mask + (base >> 6);
    // the loads that depend on the tile alone, requested together before any
    // of them is waited for (unconditional, in-bounds indexes)
    const int nbv = a.tile_nbr[27 * tile + min(gt, 26)];
    int hmv[MS];
#pragma unroll
    for (int i = 0; i < MS; i++) {
        const int s = gt + i * GR::NT;
        hmv[i] = s < g.nslot ? a.halo_map[s] : -1;
    }
    if (gt < 27) stn[gt] = nbv;
    asm volatile("" ::"s"(base), "s"(L4));  // the bond range arrives with the loads above
    const uint32_t spi = tile_specimen(aux);
    __syncthreads();
    const pd_spec sp = a.spec[spi];
    const double kp = sp.kp;
    uint64_t mw0, mw1;
    {
        int64_t rw[MS];
        double q[MS];
        double4 u[MS];
#pragma unroll
        for (int i = 0; i < MS; i++) {
            rw[i] = halo_row_of(hmv[i], stn);
        }
#pragma unroll
        for (int i = 0; i < MS; i++) {
            q[i] = rw[i] >= 0 ? qr[rw[i]].x : 0.0;
            u[i] = rw[i] >= 0 ? uv[rw[i]] : make_double4(0.0, 0.0, 0.0, 0.0);
        }
        // the tile's status words, requested with the gathers
        mw0 = gt < L4 ? mrow[gt] : 0ull;
        mw1 = (TPW != 1 && gt + 64 < L4) ? mrow[gt + 64] : 0ull;
#pragma unroll
        for (int i = 0; i < MS; i++) {
            const int s = gt + i * GR::NT;
            if (s < g.nslot) {
                hB[s] = kp * q[i];
                hB[S + s] = u[i].w;
                if constexpr (FIN) {
                    hB[2 * S + s] = u[i].x;
                    hB[3 * S + s] = u[i].y;
                    if (DIM == 3) hB[4 * S + s] = u[i].z;
                }
            }
        }
    }
    if (gt < 128) smask[gt] = mw0;
    if (TPW != 1) smask[gt + 64] = mw1;
    __syncthreads();
    const int my = own_slot<DIM>(g, lane);
    const double qi = hB[my];
    double uix = 0.0, uiy = 0.0, uiz = 0.0;
    if constexpr (FIN) {
        uix = hB[2 * S + my];
        uiy = hB[3 * S + my];
        if (DIM == 3) uiz = hB[4 * S + my];
    }
    const int ns = a.n_stencil;
    const int G4 = L4 >> 2;
    const int gper = (G4 + GR::SPLIT - 1) / GR::SPLIT;
    const int g0 = kq * gper, g1 = min(G4, g0 + gper);
    double fx = 0.0, fy = 0.0, fz = 0.0;
    for (int gg = g0; gg < g1; gg++) {
        double qj[4], vj[4], uj[4][3];
        double4 sd[4];
        uint64_t mm[4];
#pragma unroll
        for (int c = 0; c < 4; c++) {
            const int k = 4 * gg + c;
            const int slot = my + kt[k].soff;
            sd[c] = sten[min(k, ns - 1)];
            qj[c] = hB[slot];
            vj[c] = hB[S + slot];
            if constexpr (FIN) {
                uj[c][0] = hB[2 * S + slot];
                uj[c][1] = hB[3 * S + slot];
                uj[c][2] = DIM == 3 ? hB[4 * S + slot] : 0.0;
            }
            mm[c] = uni64_t(smask[k]);
        }
        if constexpr (!FIN) {
            // entries c and c + 1 are a bond and its mirror (the same x, M
            // negated): (K - G/3) x [(q_i + q_j) V_j - (q_i + q_j') V_j'] M
#pragma unroll
            for (int c = 0; c < 4; c += 2) {
                const double ta = lane_bit(mm[c]) ? (qi + qj[c]) * vj[c] : 0.0;
                const double tb = lane_bit(mm[c + 1]) ? (qi + qj[c + 1]) * vj[c + 1] : 0.0;
                const double t = (ta - tb) * sd[c].w;
                fx = fma(t, sd[c].x, fx);
                fy = fma(t, sd[c].y, fy);
                if (DIM == 3) fz = fma(t, sd[c].z, fz);
            }
            continue;
        }
#pragma unroll
        for (int c = 0; c < 4; c++) {
            // (K - G/3) x (q_i + q_j) V_j
            double t = (qi + qj[c]) * vj[c] * sd[c].w;
            const bool use = lane_bit(mm[c]);
            t = use ? t : 0.0;
            double n1 = sd[c].x, n2 = sd[c].y, n3 = sd[c].z;
            if constexpr (FIN) {
                double y1, y2, y3;
                const double yy = deformed64(sd[c], uj[c][0] - uix, uj[c][1] - uiy,
                                             DIM == 3 ? uj[c][2] - uiz : 0.0, y1, y2, y3);
                const double iy = rsqrt_refined(yy);
                n1 = use ? y1 * iy : 0.0;
                n2 = use ? y2 * iy : 0.0;
                n3 = use ? y3 * iy : 0.0;
            }
            fx = fma(t, n1, fx);
            fy = fma(t, n2, fy);
            if (DIM == 3) fz = fma(t, n3, fz);
        }
    }
    double sx = fx, sy = fy, sz = fz;
    if constexpr (TPW == 1) {
        __syncthreads();
        double *red = hB;
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
    const double4 ui = uv[row];
    const double4 fe = ldv(a.fe64, DIM, row);
    double Fx = (sx + fe.x) * ui.w;
    double Fy = (sy + fe.y) * ui.w;
    double Fz = (sz + fe.z) * ui.w;
    if (!UPDATE) {
        a.f_out[row] = make_double4(Fx, Fy, Fz, 0.0);
        return;
    }
    const int64_t n = ctl->s1;
    if (tile == 0 && gt == 0) ctl->s2 = n + 1;
    double r = 1.0;
    if (a.ramp_steps > 0) r = n >= a.ramp_steps ? 1.0 : (double)n / (double)a.ramp_steps;
    if (aux & 8u) {
        const double4 fx4 = a.fext[row];
        Fx += fx4.x * r;
        Fy += fx4.y * r;
        Fz += fx4.z * r;
    }
    const double mass = sp.rho * ui.w;
    double4 v = ldv(a.vel, DIM, row);
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
    const bool bad = !(isfinite(u.x) && isfinite(u.y) && isfinite(u.z));
    if (__ballot(bad) && lane == 0) atomicOr(&ctl->flags, PD_CTL_NONFINITE);
}

static int box_slots64(const StepArgs &a) {
    int32_t B[4];
    pd_tile_box(a.tile, a.reach, a.dim, B);
    return B[3] * B[2];
}

// pass 3 stands for pass 2 of the finite model (as many arrays as pass 1)
static size_t tiled64_lds(int dim, int pass, int tpw) {
    const bool big = pass != 2;
    if (dim == 3) return big ? Lay64<3, 1, 5>::BYTES : Lay64<3, 1, 2>::BYTES;
    if (tpw == 4) return 4 * (size_t)(big ? Lay64<2, 4, 4>::BYTES : Lay64<2, 4, 2>::BYTES);
    return big ? Lay64<2, 1, 4>::BYTES : Lay64<2, 1, 2>::BYTES;
}

bool tiled64_supported(const StepArgs &a) {
    if (!a.fe64 || !a.tile_nbr || !a.ktab || !a.halo_map) return false;
    if (a.tile[0] * a.tile[1] * a.tile[2] != 64) return false;
    for (int c = 0; c < 3; c++)
        if (a.tile[c] < 1 || (a.tile[c] & (a.tile[c] - 1))) return false;  // powers of two
    if (a.reach < 1 || a.tile[0] < a.reach || a.tile[1] < a.reach) return false;
    if (a.dim == 3 && a.tile[2] < a.reach) return false;
    if (a.dim == 2 && a.tile[2] != 1) return false;
    if (a.n_stencil > 124) return false;  // groups of four inside the 128-row table
    if (a.n_pad >= (int64_t(1) << 31)) return false;
    const int cap = a.dim == 3 ? Grp<3, 1>::CAP
                               : (tiles_per_group(a, box_slots64(a)) == 4 ? Grp<2, 4>::CAP : Grp<2, 1>::CAP);
    if (box_slots64(a) > cap) return false;
    const int tpw = tiles_per_group(a, box_slots64(a));
    // the partial sums of TPW = 1 reuse the staged arrays (2 of them in pass 2)
    if (tpw == 1 && 2 * (a.dim == 3 ? Grp<3, 1>::CAP : Grp<2, 1>::CAP) < 3 * PD_TILE_WAVES * 64) return false;
    return tiled64_lds(a.dim, 1, tpw) <= 64 * 1024 && tiled64_lds(a.dim, 2, tpw) <= 64 * 1024;
}

hipError_t launch_tpass1_f64(const StepArgs &a, int cur, bool brk, hipStream_t s) {
    const int tpw = tiles_per_group(a, box_slots64(a));
    const size_t lds = tiled64_lds(a.dim, 1, tpw);
    const dim3 g((unsigned)((a.n_slices + tpw - 1) / tpw)), b(PD_TILE_THREADS);
    const KEnt *kt = reinterpret_cast<const KEnt *>(a.ktab);
    const double4 *sten = reinterpret_cast<const double4 *>(a.stencil);
    if (a.dim == 3) {
        const dim3 b8(64 * 8);
        if (brk) hipLaunchKernelGGL((k_tpass1_f64<3, true, 1, false, 8>), g, b8, lds, s, a, cur, kt, sten);
        else hipLaunchKernelGGL((k_tpass1_f64<3, false, 1, false, 8>), g, b8, lds, s, a, cur, kt, sten);
    } else if (tpw == 4) {
        if (brk) hipLaunchKernelGGL((k_tpass1_f64<2, true, 4>), g, b, lds, s, a, cur, kt, sten);
        else hipLaunchKernelGGL((k_tpass1_f64<2, false, 4>), g, b, lds, s, a, cur, kt, sten);
    } else {
        if (brk) hipLaunchKernelGGL((k_tpass1_f64<2, true, 1>), g, b, lds, s, a, cur, kt, sten);
        else hipLaunchKernelGGL((k_tpass1_f64<2, false, 1>), g, b, lds, s, a, cur, kt, sten);
    }
    return hipGetLastError();
}

hipError_t launch_tpass2_f64(const StepArgs &a, int cur, bool update, hipStream_t s) {
    const int tpw = tiles_per_group(a, box_slots64(a));
    const size_t lds = tiled64_lds(a.dim, 2, tpw);
    const dim3 g((unsigned)((a.n_slices + tpw - 1) / tpw)), b(PD_TILE_THREADS);
    const KEnt *kt = reinterpret_cast<const KEnt *>(a.ktab);
    const double4 *sten = reinterpret_cast<const double4 *>(a.stencil);
    if (a.dim == 3) {
        if (update) hipLaunchKernelGGL((k_tpass2_f64<3, true, 1>), g, b, lds, s, a, cur, kt, sten);
        else hipLaunchKernelGGL((k_tpass2_f64<3, false, 1>), g, b, lds, s, a, cur, kt, sten);
    } else if (tpw == 4) {
        if (update) hipLaunchKernelGGL((k_tpass2_f64<2, true, 4>), g, b, lds, s, a, cur, kt, sten);
        else hipLaunchKernelGGL((k_tpass2_f64<2, false, 4>), g, b, lds, s, a, cur, kt, sten);
    } else {
        if (update) hipLaunchKernelGGL((k_tpass2_f64<2, true, 1>), g, b, lds, s, a, cur, kt, sten);
        else hipLaunchKernelGGL((k_tpass2_f64<2, false, 1>), g, b, lds, s, a, cur, kt, sten);
    }
    return hipGetLastError();
}

bool tiled64_fin_supported(const StepArgs &a) {
    if (!tiled64_supported(a)) return false;
    return tiled64_lds(a.dim, 3, tiles_per_group(a, box_slots64(a))) <= 64 * 1024;
}

hipError_t launch_tpass1_f64_fin(const StepArgs &a, int cur, bool brk, hipStream_t s) {
    const int tpw = tiles_per_group(a, box_slots64(a));
    const size_t lds = tiled64_lds(a.dim, 1, tpw);
    const dim3 g((unsigned)((a.n_slices + tpw - 1) / tpw)), b(PD_TILE_THREADS);
    const KEnt *kt = reinterpret_cast<const KEnt *>(a.ktab);
    const double4 *sten = reinterpret_cast<const double4 *>(a.stencil);
#define PD_FT1(D, B, T) hipLaunchKernelGGL((k_tpass1_f64<D, B, T, true>), g, b, lds, s, a, cur, kt, sten)
    if (a.dim == 3) {
        const dim3 b8(64 * 8);
        if (brk) hipLaunchKernelGGL((k_tpass1_f64<3, true, 1, true, 8>), g, b8, lds, s, a, cur, kt, sten);
        else hipLaunchKernelGGL((k_tpass1_f64<3, false, 1, true, 8>), g, b8, lds, s, a, cur, kt, sten);
    }
    else if (tpw == 4) { if (brk) PD_FT1(2, true, 4); else PD_FT1(2, false, 4); }
    else { if (brk) PD_FT1(2, true, 1); else PD_FT1(2, false, 1); }
#undef PD_FT1
    return hipGetLastError();
}

hipError_t launch_tpass2_f64_fin(const StepArgs &a, int cur, bool update, hipStream_t s) {
    const int tpw = tiles_per_group(a, box_slots64(a));
    const size_t lds = tiled64_lds(a.dim, 3, tpw);
    const dim3 g((unsigned)((a.n_slices + tpw - 1) / tpw)), b(PD_TILE_THREADS);
    const KEnt *kt = reinterpret_cast<const KEnt *>(a.ktab);
    const double4 *sten = reinterpret_cast<const double4 *>(a.stencil);
#define PD_FT2(D, U, T) hipLaunchKernelGGL((k_tpass2_f64<D, U, T, true>), g, b, lds, s, a, cur, kt, sten)
    if (a.dim == 3) { if (update) PD_FT2(3, true, 1); else PD_FT2(3, false, 1); }
    else if (tpw == 4) { if (update) PD_FT2(2, true, 4); else PD_FT2(2, false, 4); }
    else { if (update) PD_FT2(2, true, 1); else PD_FT2(2, false, 1); }
#undef PD_FT2
    return hipGetLastError();
}

}  // namespace pdk
