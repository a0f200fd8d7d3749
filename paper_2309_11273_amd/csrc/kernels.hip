// gfx950 kernels of the matrix-free linearized OSB-PD step (double precision
// path) and the per-row utility kernels.
//
// Layout (internal row order, 64-row slices, one wave64 per slice):
//   uv[r]   double4 (u_x, u_y, u_z, V)       displacement and node volume
//   vel[r]  double4 (v_x, v_y, v_z, 0)
//   qr[r]   double2 (theta/m, 1/m)
//   words   uint32 (j << 7 | stencil id), word k of all 64 rows of a slice
//           stored contiguously: lanes read 256 consecutive bytes per k
//   mask    uint64 per (slice, k): bit lane = bond status of that word
//   stencil double4 (M1, M2, M3, x) per bond offset, staged in LDS
// The per-bond loops gather neighbour rows from L2 (rows of a slice form a
// lattice tile, so neighbouring slices share most of their neighbours).
// Summation inside a row follows the bond order (sorted by neighbour row),
// so results do not depend on the launch shape.
#include <hip/hip_runtime.h>

#include <cmath>

#include "kernels.h"

namespace pdk {

// Extension e = M . eta evaluated as (M1 eta1 + M2 eta2) + M3 eta3 without
// contraction, so that both directed copies of a bond (and the CPU
// reference) obtain the same bits from the same displacements.
__device__ __forceinline__ double ext_canonical(double m1, double m2, double m3, double e1, double e2,
                                                double e3) {
#pragma clang fp contract(off)
    double a = m1 * e1;
    double b = m2 * e2;
    double c = m3 * e3;
    return (a + b) + c;
}

__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
    uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ void load_stencil_lds(double4 *sst, const double *stencil, int n_stencil) {
    for (int s = threadIdx.x; s < 128; s += blockDim.x) {
        double4 v = make_double4(0.0, 0.0, 0.0, 0.0);
        if (s < n_stencil) v = make_double4(stencil[4 * s], stencil[4 * s + 1], stencil[4 * s + 2], stencil[4 * s + 3]);
        sst[s] = v;
    }
}

// ---------------------------------------------------------------------------
// pass 1: breaking (Eqs. 1.17, 1.30) and dilatation (Eq. 2.3)
// ---------------------------------------------------------------------------
template <int DIM, bool BREAK>
__global__ __launch_bounds__(256) void k_pass1_f64(StepArgs a, int cur) {
    __shared__ double4 sst[128];
    load_stencil_lds(sst, a.stencil, a.n_stencil);
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int64_t slice = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (slice >= a.n_slices) return;
    if (BREAK && blockIdx.x == 0 && threadIdx.x == 0) a.ctl->s1 = a.ctl->s2;
    const int64_t row = slice * 64 + lane;
    const int64_t base = a.slice_ptr[slice];
    const int64_t L = (a.slice_ptr[slice + 1] - base) >> 6;
    const double4 *__restrict__ uv = a.uv[cur];
    const double4 ui = uv[row];
    const uint32_t aux = a.aux[row];
    const pd_spec sp = a.spec[aux >> 8];
    const double s0 = sp.s0;
    const double thr_scale = s0 * (1.0 - 1e-9);  // cheap pre-filter, exact test below
    double acc = 0.0;
    uint32_t nbroken = 0;
    // groups of four bond words per lane: one 16-byte load per group, the next
    // group's words are requested before this group's neighbours are gathered
    const uint4 *__restrict__ wg = reinterpret_cast<const uint4 *>(a.words + base) + lane;
    const uint4 *__restrict__ mg = reinterpret_cast<const uint4 *>(a.mask + (base >> 6));
    const int64_t G = L >> 2;
    uint4 wn = G > 0 ? wg[0] : make_uint4(0u, 0u, 0u, 0u);
    for (int64_t g = 0; g < G; g++) {
        const uint4 w4 = wn;
        if (g + 1 < G) wn = wg[(g + 1) * 64];
        const uint4 ma = mg[2 * g], mb = mg[2 * g + 1];
        uint64_t m[4] = {uniform64(((uint64_t)ma.y << 32) | ma.x), uniform64(((uint64_t)ma.w << 32) | ma.z),
                         uniform64(((uint64_t)mb.y << 32) | mb.x), uniform64(((uint64_t)mb.w << 32) | mb.z)};
        if ((m[0] | m[1] | m[2] | m[3]) == 0) continue;
        const uint32_t ws[4] = {w4.x, w4.y, w4.z, w4.w};
        double4 uj[4];
#pragma unroll
        for (int c = 0; c < 4; c++) uj[c] = uv[ws[c] >> 7];
#pragma unroll
        for (int c = 0; c < 4; c++) {
            const double4 st = sst[ws[c] & 127u];
            const double e = ext_canonical(st.x, st.y, DIM == 3 ? st.z : 0.0, uj[c].x - ui.x, uj[c].y - ui.y,
                                           DIM == 3 ? uj[c].z - ui.z : 0.0);
            bool intact = (m[c] >> lane) & 1ull;
            bool broke = false;
            if (BREAK && intact && e >= thr_scale * st.w) {
                if (e / st.w >= s0) {
                    intact = false;
                    broke = true;
                }
            }
            if (BREAK) {
                const uint64_t bb = __ballot(broke);
                if (bb) {
                    if (lane == 0) a.mask[(base >> 6) + 4 * g + c] = m[c] & ~bb;
                    nbroken += __popcll(bb);
                }
            }
            if (intact) acc += st.w * uj[c].w * e;  // w x V_j e, w = 1
        }
    }
    const double2 qri = a.qr[row];
    // theta_i = A / m_i * acc; store theta_i / m_i
    a.qr[row].x = sp.A * qri.y * acc * qri.y;
    if (a.theta_out) a.theta_out[row] = sp.A * qri.y * acc;
    if (BREAK && lane == 0 && nbroken) atomicAdd(&a.ctl->broken, (unsigned long long)nbroken);
}

// ---------------------------------------------------------------------------
// pass 2: pair force (Eq. 2.2) and explicit update (Eqs. 2.11, 2.12)
// ---------------------------------------------------------------------------
template <int DIM, bool UPDATE>
__global__ __launch_bounds__(256) void k_pass2_f64(StepArgs a, int cur) {
    __shared__ double4 sst[128];
    load_stencil_lds(sst, a.stencil, a.n_stencil);
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int64_t slice = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (slice >= a.n_slices) return;
    const int64_t row = slice * 64 + lane;
    const int64_t base = a.slice_ptr[slice];
    const int64_t L = (a.slice_ptr[slice + 1] - base) >> 6;
    const double4 *__restrict__ uv = a.uv[cur];
    const double2 *__restrict__ qr = a.qr;
    const double4 ui = uv[row];
    const double2 qri = qr[row];
    const uint32_t aux = a.aux[row];
    const pd_spec sp = a.spec[aux >> 8];
    double fx = 0.0, fy = 0.0, fz = 0.0;
    const uint4 *__restrict__ wg = reinterpret_cast<const uint4 *>(a.words + base) + lane;
    const uint4 *__restrict__ mg = reinterpret_cast<const uint4 *>(a.mask + (base >> 6));
    const int64_t G = L >> 2;
    uint4 wn = G > 0 ? wg[0] : make_uint4(0u, 0u, 0u, 0u);
    for (int64_t g = 0; g < G; g++) {
        const uint4 w4 = wn;
        if (g + 1 < G) wn = wg[(g + 1) * 64];
        const uint4 ma = mg[2 * g], mb = mg[2 * g + 1];
        const uint64_t m[4] = {uniform64(((uint64_t)ma.y << 32) | ma.x), uniform64(((uint64_t)ma.w << 32) | ma.z),
                               uniform64(((uint64_t)mb.y << 32) | mb.x), uniform64(((uint64_t)mb.w << 32) | mb.z)};
        if ((m[0] | m[1] | m[2] | m[3]) == 0) continue;
        const uint32_t ws[4] = {w4.x, w4.y, w4.z, w4.w};
        double4 uj[4];
        double2 qrj[4];
#pragma unroll
        for (int c = 0; c < 4; c++) {
            uj[c] = uv[ws[c] >> 7];
            qrj[c] = qr[ws[c] >> 7];
        }
#pragma unroll
        for (int c = 0; c < 4; c++) {
            const double4 st = sst[ws[c] & 127u];
            double e = st.x * (uj[c].x - ui.x) + st.y * (uj[c].y - ui.y);
            if (DIM == 3) e += st.z * (uj[c].z - ui.z);
            // [(K - G/3) x (theta_i/m_i + theta_j/m_j) + G e (1/m_i + 1/m_j)] V_j
            const double t = (sp.kp * st.w * (qri.x + qrj[c].x) + sp.G * e * (qri.y + qrj[c].y)) * uj[c].w;
            if ((m[c] >> lane) & 1ull) {
                fx += t * st.x;
                fy += t * st.y;
                if (DIM == 3) fz += t * st.z;
            }
        }
    }
    fx *= ui.w;
    fy *= ui.w;
    fz *= ui.w;
    if (!UPDATE) {
        a.f_out[row] = make_double4(fx, fy, fz, 0.0);
        return;
    }
    const int64_t n = a.ctl->s1;
    if (blockIdx.x == 0 && threadIdx.x == 0) a.ctl->s2 = n + 1;
    double r = 1.0;
    if (a.ramp_steps > 0) r = n >= a.ramp_steps ? 1.0 : (double)n / (double)a.ramp_steps;
    if (aux & 8u) {
        const double4 fe = a.fext[row];
        fx += fe.x * r;
        fy += fe.y * r;
        fz += fe.z * r;
    }
    const double mass = sp.rho * ui.w;
    double4 v = a.vel[row];
    const double ax = (aux & 1u) ? 0.0 : fx / mass;
    const double ay = (aux & 2u) ? 0.0 : fy / mass;
    const double az = (aux & 4u) ? 0.0 : fz / mass;
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
    if (__ballot(bad) && lane == 0) atomicOr(&a.ctl->flags, PD_CTL_NONFINITE);
}

// ---------------------------------------------------------------------------
// utility kernels
// ---------------------------------------------------------------------------
__global__ void k_state_init(InitArgs a) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r == 0) {
        pd_ctl *c = a.ctl;
        c->s1 = a.start_step;
        c->s2 = a.start_step;
        c->broken = 0;
        c->rechecks = 0;
        c->flags = 0;
        c->umax_bits[0] = c->umax_bits[1] = 0;
        c->qs[0] = c->qs[1] = 0.0;
        c->fallbacks = 0;
        for (int k = 0; k < 8; k++) c->red[k] = 0.0;
        c->dirty[0] = c->dirty[1] = 0;
    }
    if (r >= a.n_pad) return;
    const int32_t p = a.perm[r];
    double u[3] = {0, 0, 0}, v[3] = {0, 0, 0}, f[3] = {0, 0, 0};
    uint32_t bc = 7;
    uint32_t spec = 0;
    if (p >= 0) {
        for (int c = 0; c < 3; c++) {
            if (a.u0) u[c] = a.u0[3 * (int64_t)p + c];
            if (a.v0) v[c] = a.v0[3 * (int64_t)p + c];
            if (a.f0) f[c] = a.f0[3 * (int64_t)p + c];
        }
        bc = a.bc ? (a.bc[p] & 7u) : 0u;
        spec = (uint32_t)a.spec_rows[r];
    }
    const bool load = (f[0] != 0.0) || (f[1] != 0.0) || (f[2] != 0.0);
    a.aux[r] = bc | (load ? 8u : 0u) | (spec << 8);
    a.fext[r] = make_double4(f[0], f[1], f[2], 0.0);
    const double V = a.vol[r];
    a.uv[r] = make_double4(u[0], u[1], u[2], V);
    a.vel[r] = make_double4(v[0], v[1], v[2], 0.0);
    a.qr[r] = make_double2(0.0, a.inv_m[r]);
    if (a.qr32) a.qr32[r] = make_float2(0.0f, (float)a.inv_m[r]);
}

__global__ void k_state_read(const int32_t *perm, int64_t n_pad, const double4 *uv, const double4 *vel,
                             double *u_out, double *v_out) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_pad) return;
    const int32_t p = perm[r];
    if (p < 0) return;
    if (u_out) {
        const double4 u = uv[r];
        u_out[3 * (int64_t)p] = u.x;
        u_out[3 * (int64_t)p + 1] = u.y;
        u_out[3 * (int64_t)p + 2] = u.z;
    }
    if (v_out) {
        const double4 v = vel[r];
        v_out[3 * (int64_t)p] = v.x;
        v_out[3 * (int64_t)p + 1] = v.y;
        v_out[3 * (int64_t)p + 2] = v.z;
    }
}

// Damage (Eq. 1.31): phi = 1 - sum intact V_j / sum V_j over the family.
__global__ __launch_bounds__(256) void k_damage(DamageArgs a) {
    const int lane = threadIdx.x & 63;
    const int64_t slice = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (slice >= a.n_slices) return;
    const int64_t row = slice * 64 + lane;
    const int64_t base = a.slice_ptr[slice];
    const int64_t L = (a.slice_ptr[slice + 1] - base) >> 6;
    double num = 0.0, den = 0.0;
    for (int64_t k = 0; k < L; k++) {
        const uint64_t m64 = uniform64(a.mask[(base >> 6) + k]);
        const uint32_t w = a.words[pd_widx(base, k, lane)];
        if ((w & 127u) == PD_PAD_ID) continue;
        const double Vj = a.vol[w >> 7];
        den += Vj;
        if ((m64 >> lane) & 1ull) num += Vj;
    }
    a.phi[row] = den > 0.0 ? 1.0 - num / den : 0.0;
}

// Block-wide sums of u.f, rho V v.v for the energies; one double atomic per
// block into red[0], red[1].
__global__ __launch_bounds__(256) void k_energy(int64_t n_pad, const double4 *uv, const double4 *vel,
                                                const double4 *f, const uint32_t *aux, const pd_spec *spec,
                                                double *red) {
    __shared__ double s0[256], s1[256];
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double uf = 0.0, kin = 0.0;
    if (r < n_pad) {
        const double4 u = uv[r], v = vel[r], ff = f[r];
        const pd_spec sp = spec[aux[r] >> 8];
        uf = u.x * ff.x + u.y * ff.y + u.z * ff.z;
        kin = sp.rho * u.w * (v.x * v.x + v.y * v.y + v.z * v.z);
    }
    s0[threadIdx.x] = uf;
    s1[threadIdx.x] = kin;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            s0[threadIdx.x] += s0[threadIdx.x + o];
            s1[threadIdx.x] += s1[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomicAdd(&red[0], s0[0]);
        atomicAdd(&red[1], s1[0]);
    }
}

__global__ void k_zero_red(pd_ctl *ctl) {
    if (threadIdx.x < 8) ctl->red[threadIdx.x] = 0.0;
}

// Power iteration helpers for the stable time step.
// x := seeded random vector on free components (counter-based hash).
__global__ void k_pi_init(int64_t n_pad, int dim, const uint32_t *aux, double4 *uv, uint64_t seed) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_pad) return;
    double x[3];
    for (int c = 0; c < 3; c++) {
        uint64_t z = seed + 0x9E3779B97F4A7C15ull * (uint64_t)(3 * r + c + 1);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z = z ^ (z >> 31);
        x[c] = (double)(z >> 11) * (1.0 / 9007199254740992.0) - 0.5;
        if (c >= dim || ((aux[r] >> c) & 1u)) x[c] = 0.0;
    }
    double4 u = uv[r];
    uv[r] = make_double4(x[0], x[1], x[2], u.w);
}

// y = M^-1 (-f) on free components; accumulate x.Kx, x.Mx, y.My.
__global__ __launch_bounds__(256) void k_pi_step(int64_t n_pad, int dim, const uint32_t *aux, const pd_spec *spec,
                                                 const double4 *uv, const double4 *f, double4 *y,
                                                 double *red) {
    __shared__ double s[3][256];
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double xkx = 0, xmx = 0, ymy = 0;
    if (r < n_pad) {
        const double4 x = uv[r], ff = f[r];
        const uint32_t ax = aux[r];
        const double mass = spec[ax >> 8].rho * x.w;
        double xv[3] = {x.x, x.y, x.z}, fv[3] = {ff.x, ff.y, ff.z}, yv[3] = {0, 0, 0};
        for (int c = 0; c < dim; c++) {
            if ((ax >> c) & 1u) continue;
            if (!(mass > 0.0)) continue;
            const double kx = -fv[c];
            xkx += xv[c] * kx;
            xmx += xv[c] * mass * xv[c];
            yv[c] = kx / mass;
            ymy += yv[c] * yv[c] * mass;
        }
        y[r] = make_double4(yv[0], yv[1], yv[2], x.w);
    }
    s[0][threadIdx.x] = xkx;
    s[1][threadIdx.x] = xmx;
    s[2][threadIdx.x] = ymy;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            for (int q = 0; q < 3; q++) s[q][threadIdx.x] += s[q][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int q = 0; q < 3; q++) atomicAdd(&red[q], s[q][0]);
}

__global__ void k_pi_scale(int64_t n_pad, const double4 *y, double4 *uv, const double *red) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_pad) return;
    const double nrm = sqrt(red[2]);
    const double s = nrm > 0.0 ? 1.0 / nrm : 0.0;
    const double4 v = y[r];
    uv[r] = make_double4(v.x * s, v.y * s, v.z * s, v.w);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline dim3 grid_for_slices(int64_t n_slices, int block) {
    const int64_t per = block / 64;
    return dim3((unsigned)((n_slices + per - 1) / per));
}

hipError_t launch_pass1_f64(const StepArgs &a, int cur, bool brk, int block, hipStream_t s) {
    dim3 g = grid_for_slices(a.n_slices, block);
    if (a.dim == 3) {
        if (brk) hipLaunchKernelGGL((k_pass1_f64<3, true>), g, dim3(block), 0, s, a, cur);
        else hipLaunchKernelGGL((k_pass1_f64<3, false>), g, dim3(block), 0, s, a, cur);
    } else {
        if (brk) hipLaunchKernelGGL((k_pass1_f64<2, true>), g, dim3(block), 0, s, a, cur);
        else hipLaunchKernelGGL((k_pass1_f64<2, false>), g, dim3(block), 0, s, a, cur);
    }
    return hipGetLastError();
}

hipError_t launch_pass2_f64(const StepArgs &a, int cur, bool update, int block, hipStream_t s) {
    dim3 g = grid_for_slices(a.n_slices, block);
    if (a.dim == 3) {
        if (update) hipLaunchKernelGGL((k_pass2_f64<3, true>), g, dim3(block), 0, s, a, cur);
        else hipLaunchKernelGGL((k_pass2_f64<3, false>), g, dim3(block), 0, s, a, cur);
    } else {
        if (update) hipLaunchKernelGGL((k_pass2_f64<2, true>), g, dim3(block), 0, s, a, cur);
        else hipLaunchKernelGGL((k_pass2_f64<2, false>), g, dim3(block), 0, s, a, cur);
    }
    return hipGetLastError();
}

hipError_t launch_state_init(const InitArgs &a, hipStream_t s) {
    const int64_t nb = (a.n_pad + 255) / 256;
    hipLaunchKernelGGL(k_state_init, dim3((unsigned)nb), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_state_read(const int32_t *perm, int64_t n_pad, const double4 *uv, const double4 *vel,
                             double *u_out, double *v_out, hipStream_t s) {
    const int64_t nb = (n_pad + 255) / 256;
    hipLaunchKernelGGL(k_state_read, dim3((unsigned)nb), dim3(256), 0, s, perm, n_pad, uv, vel, u_out, v_out);
    return hipGetLastError();
}

hipError_t launch_damage(const DamageArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_damage, grid_for_slices(a.n_slices, 256), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_energy(int64_t n_pad, const double4 *uv, const double4 *vel, const double4 *f,
                         const uint32_t *aux, const pd_spec *spec, pd_ctl *ctl, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_red, dim3(1), dim3(64), 0, s, ctl);
    const int64_t nb = (n_pad + 255) / 256;
    hipLaunchKernelGGL(k_energy, dim3((unsigned)nb), dim3(256), 0, s, n_pad, uv, vel, f, aux, spec, ctl->red);
    return hipGetLastError();
}

hipError_t launch_pi_init(int64_t n_pad, int dim, const uint32_t *aux, double4 *uv, uint64_t seed,
                          hipStream_t s) {
    const int64_t nb = (n_pad + 255) / 256;
    hipLaunchKernelGGL(k_pi_init, dim3((unsigned)nb), dim3(256), 0, s, n_pad, dim, aux, uv, seed);
    return hipGetLastError();
}

hipError_t launch_pi_step(int64_t n_pad, int dim, const uint32_t *aux, const pd_spec *spec, double4 *uv,
                          const double4 *f, double4 *y, pd_ctl *ctl, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_red, dim3(1), dim3(64), 0, s, ctl);
    const int64_t nb = (n_pad + 255) / 256;
    hipLaunchKernelGGL(k_pi_step, dim3((unsigned)nb), dim3(256), 0, s, n_pad, dim, aux, spec, uv, f, y, ctl->red);
    hipLaunchKernelGGL(k_pi_scale, dim3((unsigned)nb), dim3(256), 0, s, n_pad, y, uv, ctl->red);
    return hipGetLastError();
}

}  // namespace pdk
