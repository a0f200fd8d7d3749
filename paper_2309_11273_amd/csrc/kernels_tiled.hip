// LDS-staged ("tiled") kernels of the single-precision matrix-free step.
//
// The builder lays every specimen's lattice out in tiles of 64 lattice
// points (4x4x4 in 3D, 8x8 or 16x4 in 2D, every edge at least the largest
// stencil offset component R); tile t owns rows 64t .. 64t+63 and lane l of
// the tile sits on local lattice position (l % T0, (l / T0) % T1,
// l / (T0 T1)).  Bond k of every row is stencil entry k.  A workgroup of
// four waves takes one tile:
//   1. stages what the pass needs of the tile plus an R-wide halo -- a box
//      gathered from the tile and its 3^dim neighbour tiles -- into LDS
//      (pass 1: the fixed-point displacement shadow, V and G Q V / m; pass 2:
//      (K - G/3) theta/m and V), all of a thread's slot loads issued before
//      any is consumed, together with the tile's bond-status words;
//   2. every wave sweeps a quarter of the stencil for all 64 rows, four
//      entries at a time: the neighbour of row l through entry k is LDS slot
//      slot(l) + soff[k], soff[k] the same for every lane, and the float bond
//      geometry, soff and status word of entry k are wave-uniform (scalar)
//      values, the status word used directly as the lane mask;
//   3. the four partial sums of each row are added in wave order and wave 0
//      writes the row's result (and, in pass 2, the explicit update).
//
// The arithmetic follows the gather kernels of kernels_f32.hip (same
// fixed-point shadow and error band, same double recheck of near-threshold
// bonds, same difference form of the dilatation term) with the shadow scale
// Q factored out of the per-bond work: the float extension is carried in
// units of Q, e' = M . (s_j - s_i), and Q enters once per row (the breaking
// threshold becomes s_c x / Q, the deviatoric modulus G Q), and with the
// pair force split between the passes: pass 1, which has the extension,
// sums the deviatoric part; pass 2 only the dilatational part.  Rows next
// to a shadow sentinel (a displacement too large for the fixed-point range)
// take the double gather path bond by bond; the per-bond test is compiled
// only into the sweep used when the tile's halo holds a sentinel.  Every row
// of a tile belongs to one specimen, so the material constants are
// wave-uniform and folded into the staged values.
#include <hip/hip_runtime.h>

#include <cmath>
#include <type_traits>

#include "kernels.h"
#include "tile_common.h"

namespace pdk {

// LDS of one tile in pass 1: the staged box (shadow + G Q V / m per slot) --
// with TPW = 1 the partial sums (4 floats and 3 doubles per thread) reuse it
// after the sweep, so it is at least that large -- then the tile's 128 status
// words and its 27 neighbour tiles
template <int TPW>
__host__ __device__ inline int tile1_box_bytes(int nslot) {
    const int box = (nslot * 16 + ((nslot + 1) & ~1) * 4 + 15) & ~15;
    const int sums = PD_TILE_WAVES * 64 * (4 * 4 + 3 * 8);
    return (TPW == 1 && sums > box) ? sums : box;
}
template <int TPW>
__host__ __device__ inline int tile1_bytes(int nslot) {
    return tile1_box_bytes<TPW>(nslot) + 128 * 8 + 32 * 4;
}
// pass 2: the staged box ((K - G/3) theta/m, V per slot), status words,
// neighbour tiles, and with TPW = 1 the partial sums
template <int TPW>
__host__ __device__ inline int tile2_box_bytes(int nslot) {
    return (((nslot + 1) & ~1) * 8 + 15) & ~15;
}
template <int TPW>
__host__ __device__ inline int tile2_bytes(int nslot) {
    return tile2_box_bytes<TPW>(nslot) + 128 * 8 + 32 * 4 + (TPW == 1 ? 3 * PD_TILE_WAVES * 64 * 4 : 0);
}

// ---------------------------------------------------------------------------
// pass 1: breaking (with double recheck), dilatation, deviatoric pair force
// ---------------------------------------------------------------------------
// The pair force of Eq. 2.2 is the sum of a dilatational part,
// (K - G/3) x (q_i + q_j) M V_i V_j, which needs the dilatation of both ends
// and is summed in pass 2, and a deviatoric part, G e (1/m_i + 1/m_j) M V_i V_j,
// which needs only the extension and the bond status after this step's
// breaking, and is summed here where e is at hand (fe32, without the V_i).
template <int DIM, bool BREAK, int TPW>
__global__ __launch_bounds__(PD_TILE_THREADS) void k_tpass1_f32(StepArgs a, int cur,
                                                                const KEnt *__restrict__ kt) {
    extern __shared__ __align__(16) unsigned char smem[];
    using GR = Grp<DIM, TPW>;
    constexpr int MS = GR::MS;
    const Box g = make_box(a, DIM);
    const int tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int gt = TPW == 1 ? tid : lane;  // thread within its tile's group
    const int sub = TPW == 1 ? 0 : wv;     // tile of the workgroup this wave serves
    const int kq = TPW == 1 ? wv : 0;      // stencil part of this wave
    bool valid;
    const int64_t tile = group_tile<TPW>(a.n_slices, sub, valid);
    const int64_t base = a.slice_ptr[tile];
    const int L4 = (int)((a.slice_ptr[tile + 1] - base) >> 6);
    unsigned char *reg = smem + sub * tile1_bytes<TPW>(g.nslot);
    int4 *halo = reinterpret_cast<int4 *>(reg);                  // shadow, V bits
    float *hrv = reinterpret_cast<float *>(halo + g.nslot);      // G Q V_j / m_j
    uint64_t *smask = reinterpret_cast<uint64_t *>(reg + tile1_box_bytes<TPW>(g.nslot));
    int *stn = reinterpret_cast<int *>(smask + 128);
    pd_ctl *ctl = a.ctl;
    const double Q = ctl->qs[cur];
    const int4 *__restrict__ sh = a.ush[cur];
    const float2 *__restrict__ qr = a.qr32;
    const double4 *__restrict__ uv = a.uv[cur];
    const double4 *__restrict__ sten = reinterpret_cast<const double4 *>(a.stencil);
    uint64_t *mrow = a.mask + (base >> 6);
    const int64_t row = tile * 64 + lane;
    int hmv[MS];
#pragma unroll
    for (int i = 0; i < MS; i++) {
        const int s = gt + i * GR::NT;
        hmv[i] = s < g.nslot ? a.halo_map[s] : -1;
    }
    if (gt < 27) stn[gt] = a.tile_nbr[27 * tile + gt];
    const uint64_t mw0 = gt < L4 ? mrow[gt] : 0ull;
    const uint64_t mw1 = (TPW != 1 && gt + 64 < L4) ? mrow[gt + 64] : 0ull;
    const pd_spec sp = a.spec[tile_specimen(a.aux[row])];
    const float GQ = (float)(sp.G * Q);  // extension carried in units of Q
    __syncthreads();
    bool sent = false;
    {
        int64_t rw[MS];
        int4 v[MS];
        float r[MS];
#pragma unroll
        for (int i = 0; i < MS; i++) {
            rw[i] = halo_row_of(hmv[i], stn);
        }
#pragma unroll
        for (int i = 0; i < MS; i++) {
            v[i] = rw[i] >= 0 ? sh[rw[i]] : make_int4(0, 0, 0, 0);
            r[i] = rw[i] >= 0 ? qr[rw[i]].y : 0.0f;
        }
#pragma unroll
        for (int i = 0; i < MS; i++) {
            const int s = gt + i * GR::NT;
            if (s < g.nslot) {
                halo[s] = v[i];
                hrv[s] = GQ * r[i] * __int_as_float(v[i].w);
                sent |= v[i].x == PD_SENTINEL_T;
            }
        }
    }
    if (gt < 128) smask[gt] = mw0;
    if (TPW != 1) smask[gt + 64] = mw1;
    const bool anysent = __syncthreads_or(sent);
    if (BREAK && valid && tile == 0 && gt == 0) {
        ctl->s1 = ctl->s2;
        ctl->qs[cur ^ 1] = shadow_scale_t(ctl->umax_bits[cur]);
        ctl->umax_bits[cur ^ 1] = 0u;
    }
    const int my = own_slot<DIM>(g, lane);
    const int4 si = halo[my];
    const float ri = qr[row].y;
    const float rpi = GQ * ri;
    const double s0 = sp.s0;
    // breaking threshold in units of Q, widened by the float rounding of the test
    const double invQ = inv_pow2(Q);
    const float thrQ = (float)(s0 * invQ) * (1.0f - 1e-6f);
    // screen on e/x: the float extension is off by at most sqrt(3) + 2^-20 * 3 * 2^31
    // (|shadow| < 2^30), so no bond with e/x below thr_lo can reach the threshold;
    // entry 0 is the shortest bond of the stencil
    const float thr_lo = thrQ * (1.0f - 9.5367432e-7f) - 6200.0f * kt[0].ix;
    const int G4 = L4 >> 2;
    const int gper = (G4 + GR::SPLIT - 1) / GR::SPLIT;
    const int g0 = kq * gper, g1 = min(G4, g0 + gper);
    float acc = 0.0f, fx = 0.0f, fy = 0.0f, fz = 0.0f;
    uint32_t nbroken = 0, nrecheck = 0, nfall = 0;
    double dd0 = 0.0, dd1 = 0.0, dd2 = 0.0;

    // double extension of bond k of this row (canonical order, from the
    // double state); a break takes the bond out of the row's D_i
    auto decide = [&](int k, bool brk_ok, bool &broke) -> double {
        const uint32_t w = a.words[pd_widx(base, k, lane)];
        const double4 ui = uv[row], uj = uv[w >> 7];
        const double4 sd = sten[k];
        const double e64 = ext_canonical_t(sd.x, sd.y, DIM == 3 ? sd.z : 0.0, uj.x - ui.x, uj.y - ui.y,
                                           DIM == 3 ? uj.z - ui.z : 0.0);
        if (BREAK && brk_ok && e64 / sd.w >= s0) {
            broke = true;
            const double xv = sd.w * uj.w;
            dd0 += xv * sd.x;
            dd1 += xv * sd.y;
            dd2 += xv * sd.z;
        }
        return e64;
    };

    // byte offsets of this row's own slot in the two staged arrays
    const int o_halo = my * 16, o_rv = g.nslot * 16 + my * 4;
    auto sweep = [&](auto chk) {
        constexpr bool CHK = decltype(chk)::value;
        KEnt en[4];
#pragma unroll
        for (int c = 0; c < 4; c++) en[c] = kt[4 * g0 + c];
        for (int gg = g0; gg < g1; gg++) {
            KEnt e[4];
            int4 sj[4];
            float rvj[4];
            uint64_t mm[4];
#pragma unroll
            for (int c = 0; c < 4; c++) {
                e[c] = en[c];
                sj[c] = *reinterpret_cast<const int4 *>(reg + o_halo + 16 * e[c].soff);
                rvj[c] = *reinterpret_cast<const float *>(reg + o_rv + 4 * e[c].soff);
                mm[c] = uni64_t(smask[4 * gg + c]);
            }
            // next group's table rows (row index stays inside the 128-row table)
            const int gn = min(gg + 1, 31);
#pragma unroll
            for (int c = 0; c < 4; c++) en[c] = kt[4 * gn + c];
#pragma unroll
            for (int c = 0; c < 4; c++) {
                const int k = 4 * gg + c;
                uint64_t live = mm[c];
                // (a sentinel makes these differences meaningless; such bonds are redone below)
                const float fdx = idiff(sj[c].x, si.x), fdy = idiff(sj[c].y, si.y);
                const float fdz = DIM == 3 ? idiff(sj[c].z, si.z) : 0.0f;
                float ev = e[c].m0 * fdx + e[c].m1 * fdy;
                if (DIM == 3) ev += e[c].m2 * fdz;
                if (BREAK) {
                    const uint64_t maybe = __ballot(ev * e[c].ix >= thr_lo) & live;
                    if (maybe) {
                        // |ev - e64 / Q| <= sqrt(3) + 2^-20 sum |d|: decide in double when
                        // ev + that bound reaches the threshold
                        const float lim = thrQ * e[c].x - 1.7320509f;
                        const float sdd = fabsf(fdx) + fabsf(fdy) + fabsf(fdz);
                        const bool need = lane_bit(maybe) && fmaf(9.5367432e-7f, sdd, ev) >= lim;
                        const uint64_t needm = __ballot(need);
                        if (needm) {
                            nrecheck += __popcll(needm);
                            bool broke = false;
                            if (need) (void)decide(k, true, broke);
                            const uint64_t bb = __ballot(broke);
                            if (bb) {
                                live &= ~bb;
                                if (lane == 0 && valid) mrow[k] = live;
                                nbroken += __popcll(bb);
                            }
                        }
                    }
                }
                if (CHK) {
                    // intact bonds next to a sentinel: extension (and decision) from the double state
                    const uint64_t fbm = __ballot(si.x == PD_SENTINEL_T || sj[c].x == PD_SENTINEL_T) & live;
                    if (fbm) {
                        nfall += __popcll(fbm);
                        bool broke = false;
                        if (lane_bit(fbm)) ev = (float)(decide(k, true, broke) * invQ);
                        const uint64_t bb = BREAK ? __ballot(broke) : 0ull;
                        if (bb) {
                            live &= ~bb;
                            if (lane == 0 && valid) mrow[k] = live;
                            nbroken += __popcll(bb);
                        }
                    }
                }
                const float evm = lane_bit(live) ? ev : 0.0f;  // broken bonds carry nothing
                const float Vj = __int_as_float(sj[c].w);
                // dilatation: x V_j e;  deviatoric force: G e (1/m_i + 1/m_j) V_j
                acc = fmaf(e[c].x * Vj, evm, acc);
                const float te = evm * fmaf(rpi, Vj, rvj[c]);
                fx = fmaf(te, e[c].m0, fx);
                fy = fmaf(te, e[c].m1, fy);
                if (DIM == 3) fz = fmaf(te, e[c].m2, fz);
            }
        }
    };
    if (anysent) sweep(std::true_type{});
    else sweep(std::false_type{});

    if (BREAK && valid) {
        if (lane == 0 && nbroken) atomicAdd(&ctl->broken, (unsigned long long)nbroken);
        if (lane == 0 && nrecheck) atomicAdd(&ctl->rechecks, (unsigned long long)nrecheck);
        if (lane == 0 && nfall) atomicAdd(&ctl->fallbacks, (unsigned long long)nfall);
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
        double4 D = a.dsum[row];
        D.x -= d[0];
        D.y -= d[1];
        D.z -= d[2];
        a.dsum[row] = D;
    }
    // theta_i / m_i = A r_i^2 Q sum_j x V_j e'_j
    const double accQ = (double)tot[0] * Q;
    a.qr32[row].x = (float)((double)sp.A * (double)ri * (double)ri * accQ);
    if (a.theta_out) a.theta_out[row] = (double)sp.A * (double)ri * accQ;
    a.fe32[row] = make_float4(tot[1], tot[2], tot[3], 0.0f);
}

// ---------------------------------------------------------------------------
// pass 2: dilatational pair force, explicit update, next shadow
// ---------------------------------------------------------------------------
template <int DIM, bool UPDATE, int TPW>
__global__ __launch_bounds__(PD_TILE_THREADS) void k_tpass2_f32(StepArgs a, int cur,
                                                                const KEnt2 *__restrict__ kt,
                                                                const uint64_t *__restrict__ kmask) {
    extern __shared__ __align__(16) unsigned char smem[];
    using GR = Grp<DIM, TPW>;
    constexpr int MS = GR::MS;
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
    unsigned char *reg = smem + sub * tile2_bytes<TPW>(g.nslot);
    float2 *hq = reinterpret_cast<float2 *>(reg);  // ((K - G/3) theta_j/m_j, V_j)
    uint64_t *smask = reinterpret_cast<uint64_t *>(reg + tile2_box_bytes<TPW>(g.nslot));
    int *stn = reinterpret_cast<int *>(smask + 128);
    float *red = reinterpret_cast<float *>(stn + 32);  // TPW = 1: [3][waves][64]
    pd_ctl *ctl = a.ctl;
    const int4 *__restrict__ sh = a.ush[cur];
    const float2 *__restrict__ qr = a.qr32;
    const int64_t row = tile * 64 + lane;
    const uint32_t aux = a.aux[row];
    const uint64_t *__restrict__ mrow = kmask + (base >> 6);
    int hmv[MS];
#pragma unroll
    for (int i = 0; i < MS; i++) {
        const int s = gt + i * GR::NT;
        hmv[i] = s < g.nslot ? a.halo_map[s] : -1;
    }
    if (gt < 27) stn[gt] = a.tile_nbr[27 * tile + gt];
    const uint64_t mw0 = gt < L4 ? mrow[gt] : 0ull;
    const uint64_t mw1 = (TPW != 1 && gt + 64 < L4) ? mrow[gt + 64] : 0ull;
    const pd_spec sp = a.spec[tile_specimen(aux)];
    const float kp = (float)sp.kp;
    __syncthreads();
    {
        int64_t rw[MS];
        float q[MS];
        int vb[MS];
#pragma unroll
        for (int i = 0; i < MS; i++) {
            rw[i] = halo_row_of(hmv[i], stn);
        }
#pragma unroll
        for (int i = 0; i < MS; i++) {
            q[i] = rw[i] >= 0 ? qr[rw[i]].x : 0.0f;
            vb[i] = rw[i] >= 0 ? sh[rw[i]].w : 0;
        }
#pragma unroll
        for (int i = 0; i < MS; i++) {
            const int s = gt + i * GR::NT;
            if (s < g.nslot) hq[s] = make_float2(kp * q[i], __int_as_float(vb[i]));
        }
    }
    if (gt < 128) smask[gt] = mw0;
    if (TPW != 1) smask[gt + 64] = mw1;
    __syncthreads();
    const int my = own_slot<DIM>(g, lane);
    const float qi = hq[my].x;
    const int o_q = my * 8;  // byte offset of this row's own slot
    const int G4 = L4 >> 2;
    const int gper = (G4 + GR::SPLIT - 1) / GR::SPLIT;
    const int g0 = kq * gper, g1 = min(G4, g0 + gper);
    float fx = 0.f, fy = 0.f, fz = 0.f;
    {
        KEnt2 en[4];
#pragma unroll
        for (int c = 0; c < 4; c++) en[c] = kt[4 * g0 + c];
        for (int gg = g0; gg < g1; gg++) {
            KEnt2 e[4];
            float2 qj[4];
            uint64_t mm[4];
#pragma unroll
            for (int c = 0; c < 4; c++) {
                e[c] = en[c];
                qj[c] = *reinterpret_cast<const float2 *>(reg + o_q + 8 * e[c].soff);
                mm[c] = uni64_t(smask[4 * gg + c]);
            }
            const int gn = min(gg + 1, 31);
#pragma unroll
            for (int c = 0; c < 4; c++) en[c] = kt[4 * gn + c];
#pragma unroll
            for (int c = 0; c < 4; c++) {
                // (K - G/3) (q_j - q_i) V_j, times x M from the table
                float t = (qj[c].x - qi) * qj[c].y;
                t = lane_bit(mm[c]) ? t : 0.0f;
                fx = fmaf(t, e[c].xm0, fx);
                fy = fmaf(t, e[c].xm1, fy);
                if (DIM == 3) fz = fmaf(t, e[c].xm2, fz);
            }
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
    const double4 ui = a.uv[cur][row];
    const double4 D = a.dsum[row];
    const float4 fe = a.fe32[row];
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
    if (tile == 0 && gt == 0) ctl->s2 = n + 1;
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
    double4 v = a.vel[row];
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
    a.vel[row] = v;
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
    // merge into the global maximum only when this tile exceeds what is there
    if (lane == 0 && __float_as_uint(m) > __atomic_load_n(&ctl->umax_bits[cur ^ 1], __ATOMIC_RELAXED))
        atomicMax(&ctl->umax_bits[cur ^ 1], __float_as_uint(m));
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
    a.dsum[tile * 64 + lane] = make_double4(s0, s1, s2, 0.0);
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

static size_t tiled_lds(const StepArgs &a, int pass, int tpw) {
    const int ns = box_slots(a);
    if (tpw == 1) return pass == 1 ? tile1_bytes<1>(ns) : tile2_bytes<1>(ns);
    return (size_t)tpw * (pass == 1 ? tile1_bytes<4>(ns) : tile2_bytes<4>(ns));
}

bool tiled_supported(const StepArgs &a) {
    if (!a.tile_nbr || !a.ktab || !a.halo_map) return false;
    if (a.tile[0] * a.tile[1] * a.tile[2] != 64) return false;
    for (int c = 0; c < 3; c++)
        if (a.tile[c] < 1 || (a.tile[c] & (a.tile[c] - 1))) return false;  // powers of two
    if (a.reach < 1 || a.tile[0] < a.reach || a.tile[1] < a.reach) return false;
    if (a.dim == 3 && a.tile[2] < a.reach) return false;
    if (a.dim == 2 && a.tile[2] != 1) return false;
    if (a.n_stencil > 124) return false;  // groups of four inside the 128-row table
    const int ns = box_slots(a);
    const int tpw = tiles_per_group(a.dim, ns);
    const int cap = a.dim == 3 ? Grp<3, 1>::CAP : (tpw == 4 ? Grp<2, 4>::CAP : Grp<2, 1>::CAP);
    if (ns > cap) return false;
    return tiled_lds(a, 1, tpw) <= 64 * 1024 && tiled_lds(a, 2, tpw) <= 64 * 1024;
}

hipError_t launch_tpass1_f32(const StepArgs &a, int cur, bool brk, hipStream_t s) {
    const int tpw = tiles_per_group(a.dim, box_slots(a));
    const size_t lds = tiled_lds(a, 1, tpw);
    const dim3 g((unsigned)((a.n_slices + tpw - 1) / tpw)), b(PD_TILE_THREADS);
    const KEnt *kt = reinterpret_cast<const KEnt *>(a.ktab);
    if (a.dim == 3) {
        if (brk) hipLaunchKernelGGL((k_tpass1_f32<3, true, 1>), g, b, lds, s, a, cur, kt);
        else hipLaunchKernelGGL((k_tpass1_f32<3, false, 1>), g, b, lds, s, a, cur, kt);
    } else if (tpw == 4) {
        if (brk) hipLaunchKernelGGL((k_tpass1_f32<2, true, 4>), g, b, lds, s, a, cur, kt);
        else hipLaunchKernelGGL((k_tpass1_f32<2, false, 4>), g, b, lds, s, a, cur, kt);
    } else {
        if (brk) hipLaunchKernelGGL((k_tpass1_f32<2, true, 1>), g, b, lds, s, a, cur, kt);
        else hipLaunchKernelGGL((k_tpass1_f32<2, false, 1>), g, b, lds, s, a, cur, kt);
    }
    return hipGetLastError();
}

hipError_t launch_tpass2_f32(const StepArgs &a, int cur, bool update, hipStream_t s) {
    const int tpw = tiles_per_group(a.dim, box_slots(a));
    const size_t lds = tiled_lds(a, 2, tpw);
    const dim3 g((unsigned)((a.n_slices + tpw - 1) / tpw)), b(PD_TILE_THREADS);
    const KEnt2 *kt = reinterpret_cast<const KEnt2 *>(a.ktab + 1024);
    const uint64_t *km = a.mask;
    if (a.dim == 3) {
        if (update) hipLaunchKernelGGL((k_tpass2_f32<3, true, 1>), g, b, lds, s, a, cur, kt, km);
        else hipLaunchKernelGGL((k_tpass2_f32<3, false, 1>), g, b, lds, s, a, cur, kt, km);
    } else if (tpw == 4) {
        if (update) hipLaunchKernelGGL((k_tpass2_f32<2, true, 4>), g, b, lds, s, a, cur, kt, km);
        else hipLaunchKernelGGL((k_tpass2_f32<2, false, 4>), g, b, lds, s, a, cur, kt, km);
    } else {
        if (update) hipLaunchKernelGGL((k_tpass2_f32<2, true, 1>), g, b, lds, s, a, cur, kt, km);
        else hipLaunchKernelGGL((k_tpass2_f32<2, false, 1>), g, b, lds, s, a, cur, kt, km);
    }
    return hipGetLastError();
}

}  // namespace pdk
