// gfx950 kernels of the matrix-free step with single-precision force sums
// and double-precision state ("FP32 + FP64 recheck" path).
//
// Neighbour displacements are gathered from a fixed-point shadow of the
// double-precision displacement: ush[r] = (round(u_x/Q), round(u_y/Q),
// round(u_z/Q), float bits of V) with one global power-of-two scale Q per
// shadow buffer.  The difference u_j - u_i of two shadows is then an exact
// integer, so the extension e = M.(u_j - u_i) suffers no cancellation even
// when the whole neighbourhood has moved far (an impacted edge), and its
// error is bounded by a known band:
//     |e32 - e64| <= Q * (sqrt(3) + 2^-20 * sum_c |d_c|)
// (quantisation <= Q/2 per node and component, rounding of float(d), of
// M*Q and of three products and two sums).  A bond whose float extension
// lies inside that band below the breaking threshold is decided again in
// double precision from the double displacements, by the same expression
// and order as the double path, so the breaking decisions are exact for
// the state the solver holds.
//
// The dilatation part of the pair force is summed in difference form:
//   sum_j (K-G/3) x (q_i + q_j) M V_j
//     = (K-G/3) [ sum_j x (q_j - q_i) M V_j + 2 q_i D_i ],  D_i = sum_j x M V_j
// (q = theta/m, sums over intact bonds).  D_i vanishes for a complete
// symmetric family and is kept in double precision (set up at the start of
// a call, updated when a bond of the row breaks), so the float sum only
// carries the small differences q_j - q_i instead of the large
// row-constant q_i that cancels over the family.
//
// Q is chosen from the largest displacement component m of the state the
// shadow represents: Q = 2^(floor(log2 m) - 27), so |u|/Q < 2^28.  Pass 2
// writes the next shadow with the scale chosen by pass 1 of the same step
// from max|u^n|; a node whose new displacement would exceed 2^30 Q (a
// jump of more than 4x in one step) is stored as a sentinel and read from
// the double state by every consumer instead.
#include <hip/hip_runtime.h>

#include <cmath>

#include "kernels.h"

namespace pdk {

#define PD_SENTINEL ((int)0x80000000)

__device__ __forceinline__ double ext_canonical32(double m1, double m2, double m3, double e1, double e2,
                                                  double e3) {
#pragma clang fp contract(off)
    double a = m1 * e1;
    double b = m2 * e2;
    double c = m3 * e3;
    return (a + b) + c;
}

__device__ __forceinline__ uint64_t uniform64b(uint64_t v) {
    uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Power-of-two scale for a shadow of displacements bounded by m.  The
// scale is kept >= 2^-100 so that the float table M*Q and the float force
// accumulated along M*Q stay normal numbers; displacements beyond 2^30 Q
// then fall back to the double state.
__device__ __forceinline__ double shadow_scale(unsigned int mbits) {
    const float m = __uint_as_float(mbits);
    if (!(m > 0.0f) || !isfinite(m)) return ldexp(1.0, -100);
    const int e = ilogb((double)m);
    return ldexp(1.0, max(e - 27, -100));
}

__device__ __forceinline__ int quantise(double u, double invQ, bool &bad) {
    const double t = u * invQ;
    if (!(fabs(t) < 1073741824.0)) {  // 2^30
        bad = true;
        return 0;
    }
    return (int)rint(t);
}

// Wave minimum of a non-negative margin, merged into *key as ~(float bits)
// (larger key = smaller margin; a zero key means no margin yet).  Called by
// every lane of the wave.
__device__ __forceinline__ void margin_merge_g(float m, unsigned int *key) {
    for (int o = 32; o > 0; o >>= 1) m = fminf(m, __shfl_xor(m, o));
    if ((threadIdx.x & 63) == 0 && m < __builtin_inff()) atomicMax(key, ~__float_as_uint(m));
}

// Wave maximum of a non-negative float, merged into *dst.  The atomic is
// issued only when the wave's value exceeds what is already there (a plain
// read that may be stale, which only costs an extra atomic), so tens of
// thousands of waves do not serialise on one address.
__device__ __forceinline__ void wave_max_atomic(float v, unsigned int *dst) {
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    if ((threadIdx.x & 63) == 0) {
        const unsigned int bits = __float_as_uint(v);
        if (bits > __atomic_load_n(dst, __ATOMIC_RELAXED)) atomicMax(dst, bits);
    }
}

__device__ __forceinline__ void load_stencil_scaled(float4 *sst, const double *stencil, int n_stencil, double Q) {
    for (int s = threadIdx.x; s < 128; s += blockDim.x) {
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (s < n_stencil)
            v = make_float4((float)(stencil[4 * s] * Q), (float)(stencil[4 * s + 1] * Q),
                            (float)(stencil[4 * s + 2] * Q), (float)stencil[4 * s + 3]);
        sst[s] = v;
    }
}

// ---------------------------------------------------------------------------
// set-up at the start of a call: shadow scale and shadow, D_i
// ---------------------------------------------------------------------------
// The shadow, its scale and D_i persist between calls: the set-up is skipped
// when they still describe the current state (same buffer, same step
// counter, same kind of set-up), so a trajectory does not depend on how its
// steps are split across calls.  'force' redoes it regardless.
__global__ void k_shadow_begin(pd_ctl *ctl, int k, int kind, int force) {
    // one wave (the maximum's slots are cleared lane by lane)
    const bool current = !force && ctl->sh_kind == kind && ctl->sh_cur == k && ctl->sh_step == ctl->s2;
    if (threadIdx.x == 0) ctl->sh_skip = current ? 1 : 0;
    if (!current) umax_clear_wave(ctl, k, threadIdx.x & 63);
}

__global__ void k_shadow_invalidate(pd_ctl *ctl) {
    if (threadIdx.x == 0) ctl->sh_kind = 0;
}

hipError_t launch_shadow_invalidate(pd_ctl *ctl, hipStream_t s) {
    hipLaunchKernelGGL(k_shadow_invalidate, dim3(1), dim3(64), 0, s, ctl);
    return hipGetLastError();
}

__global__ void k_shadow_end(pd_ctl *ctl, int k, int kind) {
    if (threadIdx.x == 0) {
        ctl->sh_kind = kind;
        ctl->sh_cur = k;
        ctl->sh_step = ctl->s2;
    }
}

// grid-stride maximum: one block maximum (and at most one atomic) per block
__global__ __launch_bounds__(256) void k_umax(int64_t n_pad, const double4 *uv, pd_ctl *ctl, int k) {
    __shared__ float wm[4];
    if (ctl->sh_skip) return;
    float m = 0.0f;
    for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < n_pad; r += (int64_t)gridDim.x * 256) {
        const double4 u = uv[r];
        float v = (float)fmax(fabs(u.x), fmax(fabs(u.y), fabs(u.z)));
        // round up so that the float bound is not below the double value
        v = __uint_as_float(__float_as_uint(v) + 1u);
        m = fmaxf(m, v);
    }
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
    if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        m = fmaxf(fmaxf(wm[0], wm[1]), fmaxf(wm[2], wm[3]));
        const unsigned int bits = __float_as_uint(m);
        if (bits > __atomic_load_n(&ctl->umax_bits[k], __ATOMIC_RELAXED)) atomicMax(&ctl->umax_bits[k], bits);
    }
}

__global__ __launch_bounds__(256) void k_shadow_write(int64_t n_pad, const double4 *uv, int4 *ush, pd_ctl *ctl,
                                                      int k) {
    if (ctl->sh_skip) return;
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const double Q = shadow_scale(ctl->umax_bits[k]);
    if (r == 0) ctl->qs[k] = Q;
    if (r >= n_pad) return;
    const double invQ = 1.0 / Q;
    const double4 u = uv[r];
    bool bad = false;
    int4 s;
    s.x = quantise(u.x, invQ, bad);
    s.y = quantise(u.y, invQ, bad);
    s.z = quantise(u.z, invQ, bad);
    s.w = __float_as_int((float)u.w);
    if (bad) s.x = PD_SENTINEL;
    ush[r] = s;
}

// D_i = sum over intact bonds of x M V_j (double precision)
template <int DIM>
__global__ __launch_bounds__(256) void k_dsum(StepArgs a, int cur) {
    if (a.ctl->sh_skip) return;
    const int lane = threadIdx.x & 63;
    const int64_t slice = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (slice >= a.n_slices) return;
    const int64_t row = slice * 64 + lane;
    const int64_t base = a.slice_ptr[slice];
    const int64_t L = (a.slice_ptr[slice + 1] - base) >> 6;
    const double4 *__restrict__ uv = a.uv[cur];
    const double4 *__restrict__ sten = reinterpret_cast<const double4 *>(a.stencil);
    double d0 = 0.0, d1 = 0.0, d2 = 0.0;
    for (int64_t k = 0; k < L; k++) {
        const uint64_t m64 = uniform64b(a.mask[(base >> 6) + k]);
        if (!((m64 >> lane) & 1ull)) continue;
        const uint32_t w = a.words[pd_widx(base, k, lane)];
        const double4 sd = sten[w & 127u];
        const double xv = sd.w * uv[w >> 7].w;
        d0 += xv * sd.x;
        d1 += xv * sd.y;
        if (DIM == 3) d2 += xv * sd.z;
    }
    stv(a.dsum, DIM, row, make_double4(d0, d1, d2, 0.0));
}

// ---------------------------------------------------------------------------
// pass 1 (FP32): breaking with FP64 recheck, dilatation
// ---------------------------------------------------------------------------
template <int DIM, bool BREAK>
__global__ __launch_bounds__(256) void k_pass1_f32(StepArgs a, int cur) {
    __shared__ float4 sst[128];
    pd_ctl *ctl = a.ctl;
    const double Q = ctl->qs[cur];
    load_stencil_scaled(sst, a.stencil, a.n_stencil, Q);
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int64_t slice = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (slice >= a.n_slices) return;
    if (BREAK && blockIdx.x == 0 && threadIdx.x < 64) {
        // the first wave: the next shadow's scale from this shadow's maximum
        // (its word and the tile kernels' slots), the next maximum cleared
        const unsigned int um = umax_wave(ctl, cur, lane);
        umax_clear_wave(ctl, cur ^ 1, lane);
        if (lane == 0) {
            ctl->s1 = ctl->s2;
            ctl->qs[cur ^ 1] = shadow_scale(um);
        }
    }
    const int64_t row = slice * 64 + lane;
    const int64_t base = a.slice_ptr[slice];
    const int64_t L = (a.slice_ptr[slice + 1] - base) >> 6;
    const int4 *__restrict__ sh = a.ush[cur];
    const double4 *__restrict__ uv = a.uv[cur];
    const double4 *__restrict__ sten = reinterpret_cast<const double4 *>(a.stencil);
    const int4 si = sh[row];
    const uint32_t aux = a.aux[row];
    const pd_spec sp = a.spec[aux >> 8];
    const double s0 = sp.s0;
    const float s0f = (float)s0 * (1.0f - 1e-6f);
    const float Qf = (float)Q;
    const float band0 = Qf * 1.7320509f;
    const float band1 = Qf * 9.5367432e-7f;  // 2^-20
    float acc = 0.0f;
    uint32_t nbroken = 0, nrecheck = 0, nfall = 0;
    double dd0 = 0.0, dd1 = 0.0, dd2 = 0.0;  // x M V_j of the bonds this row breaks now
    float mmin = __builtin_inff();           // smallest |s - s_c| / s_c decided in double
    const uint4 *__restrict__ wg = reinterpret_cast<const uint4 *>(a.words + base) + lane;
    const uint4 *__restrict__ mg = reinterpret_cast<const uint4 *>(a.mask + (base >> 6));
    const int64_t G = L >> 2;
    uint4 wn = G > 0 ? wg[0] : make_uint4(0u, 0u, 0u, 0u);
    for (int64_t g = 0; g < G; g++) {
      const uint4 w4 = wn;
      if (g + 1 < G) wn = wg[(g + 1) * 64];
      const uint4 ma = mg[2 * g], mb = mg[2 * g + 1];
      const uint64_t mm[4] = {uniform64b(((uint64_t)ma.y << 32) | ma.x), uniform64b(((uint64_t)ma.w << 32) | ma.z),
                              uniform64b(((uint64_t)mb.y << 32) | mb.x), uniform64b(((uint64_t)mb.w << 32) | mb.z)};
      if ((mm[0] | mm[1] | mm[2] | mm[3]) == 0) continue;
      const uint32_t ws[4] = {w4.x, w4.y, w4.z, w4.w};
      int4 sjs[4];
#pragma unroll
      for (int c = 0; c < 4; c++) sjs[c] = sh[ws[c] >> 7];
#pragma unroll
      for (int c = 0; c < 4; c++) {
        const int64_t k = 4 * g + c;
        const uint64_t m64 = mm[c];
        const uint32_t w = ws[c];
        const int64_t j = w >> 7;
        const float4 st = sst[w & 127u];
        const int4 sj = sjs[c];
        bool intact = (m64 >> lane) & 1ull;
        bool broke = false;
        float e;
        if (__builtin_expect(si.x == PD_SENTINEL || sj.x == PD_SENTINEL, 0)) {
            // shadow unavailable: exact double extension and decision
            e = 0.0f;
            if ((w & 127u) != PD_PAD_ID) {
                const double4 ui = uv[row], uj = uv[j];
                const double4 sd = sten[w & 127u];
                const double e64 = ext_canonical32(sd.x, sd.y, DIM == 3 ? sd.z : 0.0, uj.x - ui.x,
                                                   uj.y - ui.y, DIM == 3 ? uj.z - ui.z : 0.0);
                if (intact) nfall++;
                if (BREAK && intact) mmin = fminf(mmin, (float)(fabs(e64 / sd.w - s0) / s0));
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
            const int dx = sj.x - si.x, dy = sj.y - si.y, dz = DIM == 3 ? sj.z - si.z : 0;
            const float fdx = (float)dx, fdy = (float)dy, fdz = (float)dz;
            e = st.x * fdx + st.y * fdy;
            if (DIM == 3) e += st.z * fdz;
            if (BREAK && intact) {
                const float band = band0 + band1 * (fabsf(fdx) + fabsf(fdy) + fabsf(fdz));
                if (e + band >= s0f * st.w) {
                    const double4 ui = uv[row], uj = uv[j];
                    const double4 sd = sten[w & 127u];
                    const double e64 = ext_canonical32(sd.x, sd.y, DIM == 3 ? sd.z : 0.0, uj.x - ui.x,
                                                       uj.y - ui.y, DIM == 3 ? uj.z - ui.z : 0.0);
                    nrecheck++;
                    mmin = fminf(mmin, (float)(fabs(e64 / sd.w - s0) / s0));
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
    }
    // (M Q) . (du / Q) is the physical extension: theta_i / m_i = A r_i^2 acc
    const float2 qri = a.qr32[row];
    const double acc64 = (double)acc;
    a.qr32[row].x = (float)((double)sp.A * (double)qri.y * (double)qri.y * acc64);
    if (a.theta_out) a.theta_out[row] = (double)sp.A * (double)qri.y * acc64;
    if (BREAK) {
        if (dd0 != 0.0 || dd1 != 0.0 || dd2 != 0.0) {
            double4 D = ldv(a.dsum, DIM, row);
            D.x -= dd0;
            D.y -= dd1;
            D.z -= dd2;
            stv(a.dsum, DIM, row, D);
        }
        if (lane == 0 && nbroken) atomicAdd(&ctl->broken, (unsigned long long)nbroken);
        unsigned long long rc = nrecheck, fb = nfall;
        for (int o = 32; o > 0; o >>= 1) {
            rc += __shfl_xor(rc, o);
            fb += __shfl_xor(fb, o);
        }
        if (lane == 0 && rc) atomicAdd(&ctl->rechecks, rc);
        if (lane == 0 && fb) atomicAdd(&ctl->fallbacks, fb);
        if (rc | fb) margin_merge_g(mmin, &ctl->margin_key);
    }
}

// ---------------------------------------------------------------------------
// pass 2 (FP32 force, FP64 update, next shadow)
// ---------------------------------------------------------------------------
template <int DIM, bool UPDATE>
__global__ __launch_bounds__(256) void k_pass2_f32(StepArgs a, int cur) {
    __shared__ float4 sst[128];
    pd_ctl *ctl = a.ctl;
    const double Q = ctl->qs[cur];
    load_stencil_scaled(sst, a.stencil, a.n_stencil, Q);
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int64_t slice = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (slice >= a.n_slices) return;
    const int64_t row = slice * 64 + lane;
    const int64_t base = a.slice_ptr[slice];
    const int64_t L = (a.slice_ptr[slice + 1] - base) >> 6;
    const int4 *__restrict__ sh = a.ush[cur];
    const double4 *__restrict__ uv = a.uv[cur];
    const float2 *__restrict__ qr = a.qr32;
    const double4 *__restrict__ sten = reinterpret_cast<const double4 *>(a.stencil);
    const int4 si = sh[row];
    const float2 qri = qr[row];
    const uint32_t aux = a.aux[row];
    const pd_spec sp = a.spec[aux >> 8];
    const float kp = (float)sp.kp, G = (float)sp.G;
    float fx = 0.f, fy = 0.f, fz = 0.f;
    const uint4 *__restrict__ wg = reinterpret_cast<const uint4 *>(a.words + base) + lane;
    const uint4 *__restrict__ mg = reinterpret_cast<const uint4 *>(a.mask + (base >> 6));
    const int64_t G4 = L >> 2;
    uint4 wn = G4 > 0 ? wg[0] : make_uint4(0u, 0u, 0u, 0u);
    for (int64_t g = 0; g < G4; g++) {
      const uint4 w4 = wn;
      if (g + 1 < G4) wn = wg[(g + 1) * 64];
      const uint4 ma = mg[2 * g], mb = mg[2 * g + 1];
      const uint64_t mm[4] = {uniform64b(((uint64_t)ma.y << 32) | ma.x), uniform64b(((uint64_t)ma.w << 32) | ma.z),
                              uniform64b(((uint64_t)mb.y << 32) | mb.x), uniform64b(((uint64_t)mb.w << 32) | mb.z)};
      if ((mm[0] | mm[1] | mm[2] | mm[3]) == 0) continue;
      const uint32_t ws[4] = {w4.x, w4.y, w4.z, w4.w};
      int4 sjs[4];
      float2 qrjs[4];
#pragma unroll
      for (int c = 0; c < 4; c++) {
        sjs[c] = sh[ws[c] >> 7];
        qrjs[c] = qr[ws[c] >> 7];
      }
#pragma unroll
      for (int c = 0; c < 4; c++) {
        const uint64_t m64 = mm[c];
        const uint32_t w = ws[c];
        const int64_t j = w >> 7;
        const float4 st = sst[w & 127u];
        const int4 sj = sjs[c];
        const float2 qrj = qrjs[c];
        float e, Vj;
        if (__builtin_expect(si.x == PD_SENTINEL || sj.x == PD_SENTINEL, 0)) {
            e = 0.0f;
            Vj = 0.0f;
            if ((w & 127u) != PD_PAD_ID) {
                const double4 ui = uv[row], uj = uv[j];
                const double4 sd = sten[w & 127u];
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
    }
    const double4 ui = uv[row];
    const double4 D = ldv(a.dsum, DIM, row);
    // the direction was accumulated as M Q: divide by Q (a power of two);
    // add the row-constant dilatation term 2 (K - G/3) q_i D_i
    const double invQ = 1.0 / Q;
    const double c2 = 2.0 * sp.kp * (double)qri.x;
    double Fx = ((double)fx * invQ + c2 * D.x) * ui.w;
    double Fy = ((double)fy * invQ + c2 * D.y) * ui.w;
    double Fz = ((double)fz * invQ + c2 * D.z) * ui.w;
    if (!UPDATE) {
        a.f_out[row] = make_double4(Fx, Fy, Fz, 0.0);
        return;
    }
    const int64_t n = ctl->s1;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctl->s2 = n + 1;
        // the next shadow written below describes the new state
        ctl->sh_step = n + 1;
        ctl->sh_cur = cur ^ 1;
    }
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
    const double invQn = 1.0 / Qn;
    bool bad = false;
    int4 s;
    s.x = quantise(u.x, invQn, bad);
    s.y = quantise(u.y, invQn, bad);
    s.z = quantise(u.z, invQn, bad);
    s.w = si.w;
    if (bad) s.x = PD_SENTINEL;
    a.ush[cur ^ 1][row] = s;
    float m = (float)fmax(fabs(u.x), fmax(fabs(u.y), fabs(u.z)));
    const bool finite = isfinite(u.x) && isfinite(u.y) && isfinite(u.z);
    if (!finite) m = 0.0f;
    m = __uint_as_float(__float_as_uint(m) + 1u);
    wave_max_atomic(m, &ctl->umax_bits[cur ^ 1]);
    if (__ballot(!finite) && lane == 0) atomicOr(&ctl->flags, PD_CTL_NONFINITE);
    if (__ballot(bad) && lane == 0) atomicOr(&ctl->flags, PD_CTL_FALLBACK);
}

hipError_t launch_shadow_prep(const StepArgs &a, int cur, bool tiled, bool force, hipStream_t s) {
    const int kind = tiled ? 1 : 2;
    hipLaunchKernelGGL(k_shadow_begin, dim3(1), dim3(64), 0, s, a.ctl, cur, kind, force ? 1 : 0);
    const int64_t nb = (a.n_pad + 255) / 256;
    hipLaunchKernelGGL(k_umax, dim3((unsigned)(nb < 1024 ? nb : 1024)), dim3(256), 0, s, a.n_pad, a.uv[cur], a.ctl,
                       cur);
    hipLaunchKernelGGL(k_shadow_write, dim3((unsigned)nb), dim3(256), 0, s, a.n_pad, a.uv[cur], a.ush[cur], a.ctl,
                       cur);
    hipError_t e;
    if (tiled) {
        if ((e = launch_tdsum(a, cur, s)) != hipSuccess) return e;
    } else {
        const dim3 g((unsigned)((a.n_slices + 3) / 4));
        if (a.dim == 3) hipLaunchKernelGGL((k_dsum<3>), g, dim3(256), 0, s, a, cur);
        else hipLaunchKernelGGL((k_dsum<2>), g, dim3(256), 0, s, a, cur);
    }
    hipLaunchKernelGGL(k_shadow_end, dim3(1), dim3(64), 0, s, a.ctl, cur, kind);
    return hipGetLastError();
}

hipError_t launch_pass1_f32(const StepArgs &a, int cur, bool brk, int block, hipStream_t s) {
    const int64_t per = block / 64;
    dim3 g((unsigned)((a.n_slices + per - 1) / per));
    if (a.dim == 3) {
        if (brk) hipLaunchKernelGGL((k_pass1_f32<3, true>), g, dim3(block), 0, s, a, cur);
        else hipLaunchKernelGGL((k_pass1_f32<3, false>), g, dim3(block), 0, s, a, cur);
    } else {
        if (brk) hipLaunchKernelGGL((k_pass1_f32<2, true>), g, dim3(block), 0, s, a, cur);
        else hipLaunchKernelGGL((k_pass1_f32<2, false>), g, dim3(block), 0, s, a, cur);
    }
    return hipGetLastError();
}

hipError_t launch_pass2_f32(const StepArgs &a, int cur, bool update, int block, hipStream_t s) {
    const int64_t per = block / 64;
    dim3 g((unsigned)((a.n_slices + per - 1) / per));
    if (a.dim == 3) {
        if (update) hipLaunchKernelGGL((k_pass2_f32<3, true>), g, dim3(block), 0, s, a, cur);
        else hipLaunchKernelGGL((k_pass2_f32<3, false>), g, dim3(block), 0, s, a, cur);
    } else {
        if (update) hipLaunchKernelGGL((k_pass2_f32<2, true>), g, dim3(block), 0, s, a, cur);
        else hipLaunchKernelGGL((k_pass2_f32<2, false>), g, dim3(block), 0, s, a, cur);
    }
    return hipGetLastError();
}

}  // namespace pdk
