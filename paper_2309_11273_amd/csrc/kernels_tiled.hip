// LDS-staged ("tiled") kernels of the single-precision matrix-free step.
//
// The builder lays every specimen's lattice out in tiles of 64 lattice
// points (4x4x4 in 3D, 8x8 or 16x4 in 2D, every edge at least the largest
// stencil offset component R); tile t owns rows 64t .. 64t+63 and lane l of
// the tile sits on local lattice position (l % T0, (l / T0) % T1,
// l / (T0 T1)).  Bond k of every row is stencil entry k.  A workgroup of
// four waves takes one tile:
//   1. stages the fixed-point displacement shadow (and, in pass 2, theta/m
//      and 1/m) of the tile plus an R-wide halo -- a (T0+2R)(T1+2R)(T2+2R)
//      box gathered from the tile and its 3^dim neighbour tiles -- into LDS;
//   2. every wave sweeps a quarter of the stencil for all 64 rows: the
//      neighbour of row l through stencil entry k is LDS slot
//      slot(l) + soff[k], with soff[k] the same for every lane, and the bond
//      geometry (M Q, x) is one broadcast LDS read per k;
//   3. the four partial sums of each row are added in wave order and wave 0
//      writes the row's result (and, in pass 2, the explicit update).
// The arithmetic per bond is that of the gather kernels of kernels_f32.hip
// (same shadow, same error band, same double recheck of near-threshold
// bonds and same difference form of the dilatation term); only the source
// of the neighbour data changes: LDS instead of L2 gathers, and no bond
// word stream (the word is read only on the rare fallback paths).
#include <hip/hip_runtime.h>

#include <cmath>

#include "kernels.h"

namespace pdk {

#define PD_SENTINEL_T ((int)0x80000000)
#define PD_TILE_WAVES 4

__device__ __forceinline__ double ext_canonical_t(double m1, double m2, double m3, double e1, double e2,
                                                  double e3) {
#pragma clang fp contract(off)
    double a = m1 * e1;
    double b = m2 * e2;
    double c = m3 * e3;
    return (a + b) + c;
}

__device__ __forceinline__ double shadow_scale_t(unsigned int mbits) {
    const float m = __uint_as_float(mbits);
    if (!(m > 0.0f) || !isfinite(m)) return ldexp(1.0, -100);
    const int e = ilogb((double)m);
    return ldexp(1.0, max(e - 27, -100));
}

__device__ __forceinline__ int quantise_t(double u, double invQ, bool &bad) {
    const double t = u * invQ;
    if (!(fabs(t) < 1073741824.0)) {
        bad = true;
        return 0;
    }
    return (int)rint(t);
}

struct TileShape {
    int T0, T1, T2, R, Bx, By, Bz, nslot;
};

template <int DIM>
__device__ __forceinline__ TileShape tile_shape(const StepArgs &a) {
    TileShape t;
    t.T0 = a.tile[0];
    t.T1 = a.tile[1];
    t.T2 = a.tile[2];
    t.R = a.reach;
    t.Bx = t.T0 + 2 * t.R;
    t.By = t.T1 + 2 * t.R;
    t.Bz = DIM == 3 ? t.T2 + 2 * t.R : 1;
    t.nslot = t.Bx * t.By * t.Bz;
    return t;
}

// global row of halo slot s of tile 'tile' (-1: no tile there)
template <int DIM>
__device__ __forceinline__ int64_t halo_row(const TileShape &g, const int32_t *tn, int s) {
    const int bx = s % g.Bx, byz = s / g.Bx, by = byz % g.By, bz = byz / g.By;
    const int p0 = bx - g.R, p1 = by - g.R, p2 = DIM == 3 ? bz - g.R : 0;
    const int d0 = p0 < 0 ? -1 : (p0 >= g.T0 ? 1 : 0);
    const int d1 = p1 < 0 ? -1 : (p1 >= g.T1 ? 1 : 0);
    const int d2 = DIM == 3 ? (p2 < 0 ? -1 : (p2 >= g.T2 ? 1 : 0)) : 0;
    const int nt = tn[(d2 + 1) * 9 + (d1 + 1) * 3 + (d0 + 1)];
    if (nt < 0) return -1;
    return (int64_t)nt * 64 + (p0 - d0 * g.T0) + g.T0 * ((p1 - d1 * g.T1) + g.T1 * (p2 - d2 * g.T2));
}

__device__ __forceinline__ void stage_tables(const StepArgs &a, const TileShape &g, double Q, float4 *sst, int *soff,
                                             uint64_t *smask, int64_t mbase, int L4) {
    for (int s = threadIdx.x; s < 128; s += blockDim.x) {
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        int o = 0;
        if (s < a.n_stencil) {
            v = make_float4((float)(a.stencil[4 * s] * Q), (float)(a.stencil[4 * s + 1] * Q),
                            (float)(a.stencil[4 * s + 2] * Q), (float)a.stencil[4 * s + 3]);
            const int *so = a.stencil_off + 3 * s;
            o = so[0] + g.Bx * (so[1] + g.By * so[2]);
        }
        sst[s] = v;
        soff[s] = o;
    }
    for (int k = threadIdx.x; k < L4; k += blockDim.x) smask[k] = a.mask[mbase + k];
}

// ---------------------------------------------------------------------------
// pass 1: breaking (with double recheck) and dilatation
// ---------------------------------------------------------------------------
template <int DIM, bool BREAK>
__global__ __launch_bounds__(256) void k_tpass1_f32(StepArgs a, int cur) {
    extern __shared__ __align__(16) unsigned char smem[];
    const TileShape g = tile_shape<DIM>(a);
    const int64_t tile = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t base = a.slice_ptr[tile];
    const int L4 = (int)((a.slice_ptr[tile + 1] - base) >> 6);
    int4 *halo = reinterpret_cast<int4 *>(smem);
    float4 *sst = reinterpret_cast<float4 *>(halo + g.nslot);
    int *soff = reinterpret_cast<int *>(sst + 128);
    uint64_t *smask = reinterpret_cast<uint64_t *>(soff + 128);
    float *red = reinterpret_cast<float *>(smask + L4);
    pd_ctl *ctl = a.ctl;
    const double Q = ctl->qs[cur];
    const int4 *__restrict__ sh = a.ush[cur];
    const double4 *__restrict__ uv = a.uv[cur];
    const double4 *__restrict__ sten = reinterpret_cast<const double4 *>(a.stencil);
    stage_tables(a, g, Q, sst, soff, smask, base >> 6, L4);
    const int32_t *tn = a.tile_nbr + 27 * tile;
    for (int s = tid; s < g.nslot; s += blockDim.x) {
        const int64_t r = halo_row<DIM>(g, tn, s);
        halo[s] = r >= 0 ? sh[r] : make_int4(0, 0, 0, 0);
    }
    __syncthreads();
    if (BREAK && tile == 0 && tid == 0) {
        ctl->s1 = ctl->s2;
        ctl->qs[cur ^ 1] = shadow_scale_t(ctl->umax_bits[cur]);
        ctl->umax_bits[cur ^ 1] = 0u;
    }
    const int l0 = lane % g.T0, l1 = (lane / g.T0) % g.T1, l2 = lane / (g.T0 * g.T1);
    const int my = (l0 + g.R) + g.Bx * ((l1 + g.R) + g.By * (DIM == 3 ? l2 + g.R : 0));
    const int64_t row = tile * 64 + lane;
    const int4 si = halo[my];
    const uint32_t aux = a.aux[row];
    const pd_spec sp = a.spec[aux >> 8];
    const double s0 = sp.s0;
    const float s0f = (float)s0 * (1.0f - 1e-6f);
    const float Qf = (float)Q;
    const float band0 = Qf * 1.7320509f;
    const float band1 = Qf * 9.5367432e-7f;  // 2^-20
    const int ns = a.n_stencil;
    const int kper = (ns + PD_TILE_WAVES - 1) / PD_TILE_WAVES;
    const int k0 = wv * kper, k1 = min(ns, k0 + kper);
    float acc = 0.0f;
    uint32_t nbroken = 0, nrecheck = 0, nfall = 0;
    double dd0 = 0.0, dd1 = 0.0, dd2 = 0.0;
    for (int k = k0; k < k1; k++) {
        const uint64_t m64 = smask[k];
        if (m64 == 0) continue;
        const int4 sj = halo[my + soff[k]];
        const float4 st = sst[k];
        bool intact = (m64 >> lane) & 1ull;
        bool broke = false;
        float e;
        if (__builtin_expect(si.x == PD_SENTINEL_T || sj.x == PD_SENTINEL_T, 0)) {
            e = 0.0f;
            const uint32_t w = a.words[pd_widx(base, k, lane)];
            if ((w & 127u) != PD_PAD_ID) {
                const double4 ui = uv[row], uj = uv[w >> 7];
                const double4 sd = sten[k];
                const double e64 = ext_canonical_t(sd.x, sd.y, DIM == 3 ? sd.z : 0.0, uj.x - ui.x, uj.y - ui.y,
                                                   DIM == 3 ? uj.z - ui.z : 0.0);
                if (intact) nfall++;
                if (BREAK && intact && e64 / sd.w >= s0) {
                    intact = false;
                    broke = true;
                    const double xv = sd.w * uj.w;
                    dd0 += xv * sd.x;
                    dd1 += xv * sd.y;
                    dd2 += xv * sd.z;
                }
                e = (float)e64;
            }
        } else {
            const float fdx = (float)(sj.x - si.x), fdy = (float)(sj.y - si.y);
            const float fdz = DIM == 3 ? (float)(sj.z - si.z) : 0.0f;
            e = st.x * fdx + st.y * fdy;
            if (DIM == 3) e += st.z * fdz;
            if (BREAK && intact) {
                const float band = band0 + band1 * (fabsf(fdx) + fabsf(fdy) + fabsf(fdz));
                if (e + band >= s0f * st.w) {
                    const uint32_t w = a.words[pd_widx(base, k, lane)];
                    const double4 ui = uv[row], uj = uv[w >> 7];
                    const double4 sd = sten[k];
                    const double e64 = ext_canonical_t(sd.x, sd.y, DIM == 3 ? sd.z : 0.0, uj.x - ui.x,
                                                       uj.y - ui.y, DIM == 3 ? uj.z - ui.z : 0.0);
                    nrecheck++;
                    if (e64 / sd.w >= s0) {
                        intact = false;
                        broke = true;
                        const double xv = sd.w * uj.w;
                        dd0 += xv * sd.x;
                        dd1 += xv * sd.y;
                        dd2 += xv * sd.z;
                    }
                }
            }
        }
        if (BREAK) {
            const uint64_t bb = __ballot(broke);
            if (bb) {
                if (lane == 0) a.mask[(base >> 6) + k] = m64 & ~bb;
                nbroken += __popcll(bb);
            }
        }
        if (intact) acc += st.w * __int_as_float(sj.w) * e;
    }
    red[wv * 64 + lane] = acc;
    if (BREAK) {
        if (dd0 != 0.0 || dd1 != 0.0 || dd2 != 0.0) {
            double *D = reinterpret_cast<double *>(a.dsum + row);
            atomicAdd(D, -dd0);
            atomicAdd(D + 1, -dd1);
            atomicAdd(D + 2, -dd2);
        }
        if (lane == 0 && nbroken) atomicAdd(&ctl->broken, (unsigned long long)nbroken);
        unsigned long long rc = nrecheck, fb = nfall;
        for (int o = 32; o > 0; o >>= 1) {
            rc += __shfl_xor(rc, o);
            fb += __shfl_xor(fb, o);
        }
        if (lane == 0 && rc) atomicAdd(&ctl->rechecks, rc);
        if (lane == 0 && fb) atomicAdd(&ctl->fallbacks, fb);
    }
    __syncthreads();
    if (wv != 0) return;
    float tot = red[lane];
    for (int q = 1; q < PD_TILE_WAVES; q++) tot += red[q * 64 + lane];
    const float2 qri = a.qr32[row];
    const double acc64 = (double)tot;
    a.qr32[row].x = (float)((double)sp.A * (double)qri.y * (double)qri.y * acc64);
    if (a.theta_out) a.theta_out[row] = (double)sp.A * (double)qri.y * acc64;
}

// ---------------------------------------------------------------------------
// pass 2: pair force, explicit update, next shadow
// ---------------------------------------------------------------------------
template <int DIM, bool UPDATE>
__global__ __launch_bounds__(256) void k_tpass2_f32(StepArgs a, int cur) {
    extern __shared__ __align__(16) unsigned char smem[];
    const TileShape g = tile_shape<DIM>(a);
    const int64_t tile = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t base = a.slice_ptr[tile];
    const int L4 = (int)((a.slice_ptr[tile + 1] - base) >> 6);
    int4 *halo = reinterpret_cast<int4 *>(smem);
    float2 *hqr = reinterpret_cast<float2 *>(halo + g.nslot);
    float4 *sst = reinterpret_cast<float4 *>(hqr + ((g.nslot + 1) & ~1));
    int *soff = reinterpret_cast<int *>(sst + 128);
    uint64_t *smask = reinterpret_cast<uint64_t *>(soff + 128);
    float *red = reinterpret_cast<float *>(smask + L4);
    pd_ctl *ctl = a.ctl;
    const double Q = ctl->qs[cur];
    const int4 *__restrict__ sh = a.ush[cur];
    const double4 *__restrict__ uv = a.uv[cur];
    const float2 *__restrict__ qr = a.qr32;
    const double4 *__restrict__ sten = reinterpret_cast<const double4 *>(a.stencil);
    stage_tables(a, g, Q, sst, soff, smask, base >> 6, L4);
    const int32_t *tn = a.tile_nbr + 27 * tile;
    for (int s = tid; s < g.nslot; s += blockDim.x) {
        const int64_t r = halo_row<DIM>(g, tn, s);
        if (r >= 0) {
            halo[s] = sh[r];
            hqr[s] = qr[r];
        } else {
            halo[s] = make_int4(0, 0, 0, 0);
            hqr[s] = make_float2(0.f, 0.f);
        }
    }
    __syncthreads();
    const int l0 = lane % g.T0, l1 = (lane / g.T0) % g.T1, l2 = lane / (g.T0 * g.T1);
    const int my = (l0 + g.R) + g.Bx * ((l1 + g.R) + g.By * (DIM == 3 ? l2 + g.R : 0));
    const int64_t row = tile * 64 + lane;
    const int4 si = halo[my];
    const float2 qri = hqr[my];
    const uint32_t aux = a.aux[row];
    const pd_spec sp = a.spec[aux >> 8];
    const float kp = (float)sp.kp, G = (float)sp.G;
    const int ns = a.n_stencil;
    const int kper = (ns + PD_TILE_WAVES - 1) / PD_TILE_WAVES;
    const int k0 = wv * kper, k1 = min(ns, k0 + kper);
    float fx = 0.f, fy = 0.f, fz = 0.f;
    for (int k = k0; k < k1; k++) {
        const uint64_t m64 = smask[k];
        if (m64 == 0) continue;
        const int slot = my + soff[k];
        const int4 sj = halo[slot];
        const float2 qrj = hqr[slot];
        const float4 st = sst[k];
        float e, Vj;
        if (__builtin_expect(si.x == PD_SENTINEL_T || sj.x == PD_SENTINEL_T, 0)) {
            e = 0.0f;
            Vj = 0.0f;
            const uint32_t w = a.words[pd_widx(base, k, lane)];
            if ((w & 127u) != PD_PAD_ID) {
                const double4 ui = uv[row], uj = uv[w >> 7];
                const double4 sd = sten[k];
                double e64 = sd.x * (uj.x - ui.x) + sd.y * (uj.y - ui.y);
                if (DIM == 3) e64 += sd.z * (uj.z - ui.z);
                e = (float)e64;
                Vj = (float)uj.w;
            }
        } else {
            e = st.x * (float)(sj.x - si.x) + st.y * (float)(sj.y - si.y);
            if (DIM == 3) e += st.z * (float)(sj.z - si.z);
            Vj = __int_as_float(sj.w);
        }
        // [(K - G/3) x (q_j - q_i) + G e (1/m_i + 1/m_j)] V_j, q = theta/m
        const float t = (kp * st.w * (qrj.x - qri.x) + G * e * (qri.y + qrj.y)) * Vj;
        if ((m64 >> lane) & 1ull) {
            fx += t * st.x;
            fy += t * st.y;
            if (DIM == 3) fz += t * st.z;
        }
    }
    red[(0 * PD_TILE_WAVES + wv) * 64 + lane] = fx;
    red[(1 * PD_TILE_WAVES + wv) * 64 + lane] = fy;
    red[(2 * PD_TILE_WAVES + wv) * 64 + lane] = fz;
    __syncthreads();
    if (wv != 0) return;
    float sx = red[lane], sy = red[PD_TILE_WAVES * 64 + lane], sz = red[2 * PD_TILE_WAVES * 64 + lane];
    for (int q = 1; q < PD_TILE_WAVES; q++) {
        sx += red[q * 64 + lane];
        sy += red[(PD_TILE_WAVES + q) * 64 + lane];
        sz += red[(2 * PD_TILE_WAVES + q) * 64 + lane];
    }
    const double4 ui = uv[row];
    const double4 D = a.dsum[row];
    const double invQ = 1.0 / Q;
    const double c2 = 2.0 * sp.kp * (double)qri.x;
    double Fx = ((double)sx * invQ + c2 * D.x) * ui.w;
    double Fy = ((double)sy * invQ + c2 * D.y) * ui.w;
    double Fz = ((double)sz * invQ + c2 * D.z) * ui.w;
    if (!UPDATE) {
        a.f_out[row] = make_double4(Fx, Fy, Fz, 0.0);
        return;
    }
    const int64_t n = ctl->s1;
    if (tile == 0 && tid == 0) ctl->s2 = n + 1;
    const double Qn = ctl->qs[cur ^ 1];
    double r = 1.0;
    if (a.ramp_steps > 0) r = n >= a.ramp_steps ? 1.0 : (double)n / (double)a.ramp_steps;
    if (aux & 8u) {
        const double4 fe = a.fext[row];
        Fx += fe.x * r;
        Fy += fe.y * r;
        Fz += fe.z * r;
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
    const double invQn = 1.0 / Qn;
    bool bad = false;
    int4 s;
    s.x = quantise_t(u.x, invQn, bad);
    s.y = quantise_t(u.y, invQn, bad);
    s.z = quantise_t(u.z, invQn, bad);
    s.w = si.w;
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

static size_t tiled_lds(const StepArgs &a, int pass) {
    const int Bx = a.tile[0] + 2 * a.reach, By = a.tile[1] + 2 * a.reach;
    const int Bz = a.dim == 3 ? a.tile[2] + 2 * a.reach : 1;
    const size_t nslot = (size_t)Bx * By * Bz;
    const size_t L4 = (size_t)((a.n_stencil + 3) / 4 * 4);
    size_t b = nslot * sizeof(int4);
    if (pass == 2) b += ((nslot + 1) & ~(size_t)1) * sizeof(float2);
    b += 128 * sizeof(float4) + 128 * sizeof(int) + L4 * sizeof(uint64_t);
    b += (pass == 2 ? 3 : 1) * PD_TILE_WAVES * 64 * sizeof(float);
    return b;
}

bool tiled_supported(const StepArgs &a) {
    if (!a.tile_nbr || !a.stencil_off) return false;
    if (a.tile[0] * a.tile[1] * a.tile[2] != 64) return false;
    if (a.reach < 1 || a.tile[0] < a.reach || a.tile[1] < a.reach) return false;
    if (a.dim == 3 && a.tile[2] < a.reach) return false;
    if (a.dim == 2 && a.tile[2] != 1) return false;
    return tiled_lds(a, 2) <= 64 * 1024;
}

hipError_t launch_tpass1_f32(const StepArgs &a, int cur, bool brk, hipStream_t s) {
    const size_t lds = tiled_lds(a, 1);
    const dim3 g((unsigned)a.n_slices), b(64 * PD_TILE_WAVES);
    if (a.dim == 3) {
        if (brk) hipLaunchKernelGGL((k_tpass1_f32<3, true>), g, b, lds, s, a, cur);
        else hipLaunchKernelGGL((k_tpass1_f32<3, false>), g, b, lds, s, a, cur);
    } else {
        if (brk) hipLaunchKernelGGL((k_tpass1_f32<2, true>), g, b, lds, s, a, cur);
        else hipLaunchKernelGGL((k_tpass1_f32<2, false>), g, b, lds, s, a, cur);
    }
    return hipGetLastError();
}

hipError_t launch_tpass2_f32(const StepArgs &a, int cur, bool update, hipStream_t s) {
    const size_t lds = tiled_lds(a, 2);
    const dim3 g((unsigned)a.n_slices), b(64 * PD_TILE_WAVES);
    if (a.dim == 3) {
        if (update) hipLaunchKernelGGL((k_tpass2_f32<3, true>), g, b, lds, s, a, cur);
        else hipLaunchKernelGGL((k_tpass2_f32<3, false>), g, b, lds, s, a, cur);
    } else {
        if (update) hipLaunchKernelGGL((k_tpass2_f32<2, true>), g, b, lds, s, a, cur);
        else hipLaunchKernelGGL((k_tpass2_f32<2, false>), g, b, lds, s, a, cur);
    }
    return hipGetLastError();
}

}  // namespace pdk
