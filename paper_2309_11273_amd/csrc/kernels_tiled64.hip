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
// LDS holds the staged quantities as separate arrays of doubles at a fixed
// stride (a multiple of 64 elements), so that one address serves all of a
// slot's arrays and pairs of them are fetched by one two-address LDS read.
#include <hip/hip_runtime.h>

#include <cmath>

#include "kernels.h"
#include "tile_common.h"

namespace pdk {

// fixed array stride in the LDS box (doubles): room for every slot a
// workgroup can stage
template <int DIM>
struct Stride64 {
    static constexpr int value = StageCap<DIM>::value * PD_TILE_THREADS;
};

__device__ __forceinline__ double ext_canonical64(double m1, double m2, double m3, double e1, double e2,
                                                  double e3) {
#pragma clang fp contract(off)
    double a = m1 * e1;
    double b = m2 * e2;
    double c = m3 * e3;
    return (a + b) + c;
}

// ---------------------------------------------------------------------------
// pass 1: breaking, dilatation, deviatoric pair force
// ---------------------------------------------------------------------------
template <int DIM, bool BREAK>
__global__ __launch_bounds__(PD_TILE_THREADS) void k_tpass1_f64(StepArgs a, int cur, const KEnt *__restrict__ kt,
                                                                const double4 *__restrict__ sten) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int MS = StageCap<DIM>::value;
    constexpr int S = Stride64<DIM>::value;
    const Box g = make_box(a, DIM);
    const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const int tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t base = a.slice_ptr[tile];
    const int L4 = (int)((a.slice_ptr[tile + 1] - base) >> 6);
    // [0] G V_j / m_j, [1..3] u_j, [4] V_j; reused for the partial sums
    double *hA = reinterpret_cast<double *>(smem);
    uint64_t *smask = reinterpret_cast<uint64_t *>(hA + 5 * S);
    int *stn = reinterpret_cast<int *>(smask + 128);
    pd_ctl *ctl = a.ctl;
    const double4 *__restrict__ uv = a.uv[cur];
    const double2 *__restrict__ qr = a.qr;
    uint64_t *mrow = a.mask + (base >> 6);
    const int64_t row = tile * 64 + lane;
    int hmv[MS];
#pragma unroll
    for (int i = 0; i < MS; i++) {
        const int s = tid + i * PD_TILE_THREADS;
        hmv[i] = s < g.nslot ? a.halo_map[s] : -1;
    }
    if (tid < 27) stn[tid] = a.tile_nbr[27 * tile + tid];
    const uint64_t mword = tid < L4 ? mrow[tid] : 0ull;
    const pd_spec sp = a.spec[tile_specimen(a.aux[row])];
    const double G = sp.G;
    __syncthreads();
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
#pragma unroll
        for (int i = 0; i < MS; i++) {
            const int s = tid + i * PD_TILE_THREADS;
            if (s < g.nslot) {
                hA[s] = G * r[i] * u[i].w;
                hA[S + s] = u[i].x;
                hA[2 * S + s] = u[i].y;
                if (DIM == 3) hA[3 * S + s] = u[i].z;
                hA[4 * S + s] = u[i].w;
            }
        }
    }
    if (tid < 128) smask[tid] = mword;
    __syncthreads();
    if (BREAK && tile == 0 && tid == 0) ctl->s1 = ctl->s2;
    const int my = own_slot<DIM>(g, lane);
    const double uix = hA[S + my], uiy = hA[2 * S + my], uiz = DIM == 3 ? hA[3 * S + my] : 0.0;
    const double ri = qr[row].y;
    const double rpi = G * ri;
    const double s0 = sp.s0;
    const double thr_scale = s0 * (1.0 - 1e-9);  // pre-filter, exact test below
    const int ns = a.n_stencil;
    const int G4 = L4 >> 2;
    const int gper = (G4 + PD_TILE_WAVES - 1) / PD_TILE_WAVES;
    const int g0 = wv * gper, g1 = min(G4, g0 + gper);
    double acc = 0.0, fx = 0.0, fy = 0.0, fz = 0.0;
    uint32_t nbroken = 0;
    for (int gg = g0; gg < g1; gg++) {
        double rv[4], ux[4], uy[4], uz[4], vj[4];
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
            vj[c] = hA[4 * S + slot];
            mm[c] = uni64_t(smask[k]);
        }
#pragma unroll
        for (int c = 0; c < 4; c++) {
            const int k = 4 * gg + c;
            const double dx = ux[c] - uix, dy = uy[c] - uiy, dz = DIM == 3 ? uz[c] - uiz : 0.0;
            const double ev = DIM == 3 ? ext_canonical64(sd[c].x, sd[c].y, sd[c].z, dx, dy, dz)
                                       : ext_canonical64(sd[c].x, sd[c].y, 0.0, dx, dy, 0.0);
            bool intact = lane_bit(mm[c]);
            if (BREAK) {
                bool broke = false;
                if (intact && ev >= thr_scale * sd[c].w) {
                    if (ev / sd[c].w >= s0) {
                        intact = false;
                        broke = true;
                    }
                }
                const uint64_t bb = __ballot(broke);
                if (bb) {
                    if (lane == 0) mrow[k] = mm[c] & ~bb;
                    nbroken += __popcll(bb);
                }
            }
            // dilatation: x V_j e;  deviatoric force: G e (1/m_i + 1/m_j) V_j
            const double xv = sd[c].w * vj[c];
            acc = fma(intact ? xv : 0.0, ev, acc);
            const double te = intact ? ev * fma(rpi, vj[c], rv[c]) : 0.0;
            fx = fma(te, sd[c].x, fx);
            fy = fma(te, sd[c].y, fy);
            if (DIM == 3) fz = fma(te, sd[c].z, fz);
        }
    }
    if (BREAK && lane == 0 && nbroken) atomicAdd(&ctl->broken, (unsigned long long)nbroken);
    __syncthreads();  // every wave is done with the staged box: reuse it for the sums
    double *red = hA;
    red[(0 * PD_TILE_WAVES + wv) * 64 + lane] = acc;
    red[(1 * PD_TILE_WAVES + wv) * 64 + lane] = fx;
    red[(2 * PD_TILE_WAVES + wv) * 64 + lane] = fy;
    red[(3 * PD_TILE_WAVES + wv) * 64 + lane] = fz;
    __syncthreads();
    if (wv != 0) return;
    double tot[4];
#pragma unroll
    for (int v = 0; v < 4; v++) {
        tot[v] = red[v * PD_TILE_WAVES * 64 + lane];
        for (int q = 1; q < PD_TILE_WAVES; q++) tot[v] += red[(v * PD_TILE_WAVES + q) * 64 + lane];
    }
    // theta_i = A / m_i * acc; store theta_i / m_i
    a.qr[row].x = sp.A * ri * tot[0] * ri;
    if (a.theta_out) a.theta_out[row] = sp.A * ri * tot[0];
    a.fe64[row] = make_double4(tot[1], tot[2], tot[3], 0.0);
}

// ---------------------------------------------------------------------------
// pass 2: dilatational pair force, explicit update
// ---------------------------------------------------------------------------
template <int DIM, bool UPDATE>
__global__ __launch_bounds__(PD_TILE_THREADS) void k_tpass2_f64(StepArgs a, int cur, const KEnt *__restrict__ kt,
                                                                const double4 *__restrict__ sten) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int MS = StageCap<DIM>::value;
    constexpr int S = Stride64<DIM>::value;
    const Box g = make_box(a, DIM);
    const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const int tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t base = a.slice_ptr[tile];
    const int L4 = (int)((a.slice_ptr[tile + 1] - base) >> 6);
    // [0] (K - G/3) theta_j / m_j, [1] V_j; reused for the partial sums
    double *hB = reinterpret_cast<double *>(smem);
    uint64_t *smask = reinterpret_cast<uint64_t *>(hB + 2 * S);
    int *stn = reinterpret_cast<int *>(smask + 128);
    pd_ctl *ctl = a.ctl;
    const double4 *__restrict__ uv = a.uv[cur];
    const double2 *__restrict__ qr = a.qr;
    const int64_t row = tile * 64 + lane;
    const uint32_t aux = a.aux[row];
    int hmv[MS];
#pragma unroll
    for (int i = 0; i < MS; i++) {
        const int s = tid + i * PD_TILE_THREADS;
        hmv[i] = s < g.nslot ? a.halo_map[s] : -1;
    }
    if (tid < 27) stn[tid] = a.tile_nbr[27 * tile + tid];
    const uint64_t mword = tid < L4 ? a.mask[(base >> 6) + tid] : 0ull;
    const pd_spec sp = a.spec[tile_specimen(aux)];
    const double kp = sp.kp;
    __syncthreads();
    {
        int64_t rw[MS];
        double q[MS], v[MS];
#pragma unroll
        for (int i = 0; i < MS; i++) {
            rw[i] = halo_row_of(hmv[i], stn);
        }
#pragma unroll
        for (int i = 0; i < MS; i++) {
            q[i] = rw[i] >= 0 ? qr[rw[i]].x : 0.0;
            v[i] = rw[i] >= 0 ? uv[rw[i]].w : 0.0;
        }
#pragma unroll
        for (int i = 0; i < MS; i++) {
            const int s = tid + i * PD_TILE_THREADS;
            if (s < g.nslot) {
                hB[s] = kp * q[i];
                hB[S + s] = v[i];
            }
        }
    }
    if (tid < 128) smask[tid] = mword;
    __syncthreads();
    const int my = own_slot<DIM>(g, lane);
    const double qi = hB[my];
    const int ns = a.n_stencil;
    const int G4 = L4 >> 2;
    const int gper = (G4 + PD_TILE_WAVES - 1) / PD_TILE_WAVES;
    const int g0 = wv * gper, g1 = min(G4, g0 + gper);
    double fx = 0.0, fy = 0.0, fz = 0.0;
    for (int gg = g0; gg < g1; gg++) {
        double qj[4], vj[4];
        double4 sd[4];
        uint64_t mm[4];
#pragma unroll
        for (int c = 0; c < 4; c++) {
            const int k = 4 * gg + c;
            const int slot = my + kt[k].soff;
            sd[c] = sten[min(k, ns - 1)];
            qj[c] = hB[slot];
            vj[c] = hB[S + slot];
            mm[c] = uni64_t(smask[k]);
        }
#pragma unroll
        for (int c = 0; c < 4; c++) {
            // (K - G/3) x (q_i + q_j) V_j
            double t = (qi + qj[c]) * vj[c] * sd[c].w;
            t = lane_bit(mm[c]) ? t : 0.0;
            fx = fma(t, sd[c].x, fx);
            fy = fma(t, sd[c].y, fy);
            if (DIM == 3) fz = fma(t, sd[c].z, fz);
        }
    }
    __syncthreads();
    double *red = hB;
    red[(0 * PD_TILE_WAVES + wv) * 64 + lane] = fx;
    red[(1 * PD_TILE_WAVES + wv) * 64 + lane] = fy;
    red[(2 * PD_TILE_WAVES + wv) * 64 + lane] = fz;
    __syncthreads();
    if (wv != 0) return;
    double sx = red[lane], sy = red[PD_TILE_WAVES * 64 + lane], sz = red[2 * PD_TILE_WAVES * 64 + lane];
    for (int q = 1; q < PD_TILE_WAVES; q++) {
        sx += red[q * 64 + lane];
        sy += red[(PD_TILE_WAVES + q) * 64 + lane];
        sz += red[(2 * PD_TILE_WAVES + q) * 64 + lane];
    }
    const double4 ui = uv[row];
    const double4 fe = a.fe64[row];
    double Fx = (sx + fe.x) * ui.w;
    double Fy = (sy + fe.y) * ui.w;
    double Fz = (sz + fe.z) * ui.w;
    if (!UPDATE) {
        a.f_out[row] = make_double4(Fx, Fy, Fz, 0.0);
        return;
    }
    const int64_t n = ctl->s1;
    if (tile == 0 && tid == 0) ctl->s2 = n + 1;
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
    const bool bad = !(isfinite(u.x) && isfinite(u.y) && isfinite(u.z));
    if (__ballot(bad) && lane == 0) atomicOr(&ctl->flags, PD_CTL_NONFINITE);
}

static size_t tiled64_lds(int dim, int pass) {
    const size_t S = dim == 3 ? Stride64<3>::value : Stride64<2>::value;
    return (pass == 1 ? 5 : 2) * S * sizeof(double) + 128 * sizeof(uint64_t) + 32 * sizeof(int);
}

bool tiled64_supported(const StepArgs &a) {
    if (!a.fe64 || !tiled_supported(a)) return false;
    // the partial sums reuse the staged arrays
    if (tiled64_lds(a.dim, 2) < 3 * PD_TILE_WAVES * 64 * sizeof(double) + 128 * sizeof(uint64_t)) return false;
    return tiled64_lds(a.dim, 1) <= 64 * 1024;
}

hipError_t launch_tpass1_f64(const StepArgs &a, int cur, bool brk, hipStream_t s) {
    const size_t lds = tiled64_lds(a.dim, 1);
    const dim3 g((unsigned)a.n_slices), b(PD_TILE_THREADS);
    const KEnt *kt = reinterpret_cast<const KEnt *>(a.ktab);
    const double4 *sten = reinterpret_cast<const double4 *>(a.stencil);
    if (a.dim == 3) {
        if (brk) hipLaunchKernelGGL((k_tpass1_f64<3, true>), g, b, lds, s, a, cur, kt, sten);
        else hipLaunchKernelGGL((k_tpass1_f64<3, false>), g, b, lds, s, a, cur, kt, sten);
    } else {
        if (brk) hipLaunchKernelGGL((k_tpass1_f64<2, true>), g, b, lds, s, a, cur, kt, sten);
        else hipLaunchKernelGGL((k_tpass1_f64<2, false>), g, b, lds, s, a, cur, kt, sten);
    }
    return hipGetLastError();
}

hipError_t launch_tpass2_f64(const StepArgs &a, int cur, bool update, hipStream_t s) {
    const size_t lds = tiled64_lds(a.dim, 2);
    const dim3 g((unsigned)a.n_slices), b(PD_TILE_THREADS);
    const KEnt *kt = reinterpret_cast<const KEnt *>(a.ktab);
    const double4 *sten = reinterpret_cast<const double4 *>(a.stencil);
    if (a.dim == 3) {
        if (update) hipLaunchKernelGGL((k_tpass2_f64<3, true>), g, b, lds, s, a, cur, kt, sten);
        else hipLaunchKernelGGL((k_tpass2_f64<3, false>), g, b, lds, s, a, cur, kt, sten);
    } else {
        if (update) hipLaunchKernelGGL((k_tpass2_f64<2, true>), g, b, lds, s, a, cur, kt, sten);
        else hipLaunchKernelGGL((k_tpass2_f64<2, false>), g, b, lds, s, a, cur, kt, sten);
    }
    return hipGetLastError();
}

}  // namespace pdk
