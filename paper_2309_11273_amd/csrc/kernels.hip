// gfx950 kernels of the matrix-free linearized OSB-PD step (double precision
// path) and the per-row utility kernels.
//
// Layout (internal row order, 64-row slices, one wave64 per slice):
//   uv[r]   double4 (u_x, u_y, u_z, V)       displacement and node volume
//   vel     per row (v_x, v_y, v_z) packed in 3D, (v_x, v_y) in 2D
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
#include <cstddef>

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
    double4 v = ldv(a.vel, DIM, row);
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
    stv(a.vel, DIM, row, v);
    const bool bad = !(isfinite(u.x) && isfinite(u.y) && isfinite(u.z));
    if (__ballot(bad) && lane == 0) atomicOr(&a.ctl->flags, PD_CTL_NONFINITE);
}

// ---------------------------------------------------------------------------
// utility kernels
// ---------------------------------------------------------------------------
__global__ void k_state_init(InitArgs a) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // the control block: step counter (words 0, 1) set, every other word cleared
    if (r >= 2 && r < (int64_t)(sizeof(pd_ctl) / 8)) reinterpret_cast<unsigned long long *>(a.ctl)[r] = 0ull;
    static_assert(offsetof(pd_ctl, s2) == 8, "step counter in the first two words");
    if (r == 0) {
        a.ctl->s1 = a.start_step;
        a.ctl->s2 = a.start_step;
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
    stv(a.vel, a.dim, r, make_double4(v[0], v[1], v[2], 0.0));
    a.qr[r] = make_double2(0.0, a.inv_m[r]);
    if (a.qr32) a.qr32[r] = make_float2(0.0f, (float)a.inv_m[r]);
}

__global__ void k_state_read(const int32_t *perm, int64_t n_pad, int dim, const double4 *uv, const double *vel,
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
        const double4 v = ldv(vel, dim, r);
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

// ---------------------------------------------------------------------------
// energies (Eq. 1.20) and the power iteration, reduced in a fixed order
// ---------------------------------------------------------------------------
// Sums over a block of 256 threads, NQ values each, in a fixed tree: the
// result does not depend on the order in which waves run.  Thread 0 holds
// the totals afterwards.  Every thread of the block must call it.
template <int NQ>
__device__ __forceinline__ void block_sum_fixed(double (&v)[NQ], double (*sh)[256]) {
    const int t = threadIdx.x;
#pragma unroll
    for (int q = 0; q < NQ; q++) sh[q][t] = v[q];
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (t < o) {
#pragma unroll
            for (int q = 0; q < NQ; q++) sh[q][t] += sh[q][t + o];
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < NQ; q++) v[q] = sh[q][0];
}

// Per row: the kinetic energy 1/2 rho V_i v.v and V_i W_i with the strain
// energy density of Eq. 1.20 in the constants of Eqs. 1.8, 1.15, 1.16,
//   W_i = (K - G/3) / (2 A) theta_i^2 + G / (2 m_i) sum_j rho_ij e_ij^2 V_j,
//   theta_i = (A / m_i) sum_j rho_ij x e_ij V_j               (Eq. 2.3, w = 1),
// with the linearized extension (Eqs. 2.4, 2.7) or, FIN, the finite one
// (e = |x M + u_j - u_i| - x, Eq. 1.10).  One partial (kinetic, strain) per
// block of four slices.
template <int DIM, bool FIN>
__global__ __launch_bounds__(256) void k_energy_rows(StepArgs a, int cur, double4 *part) {
    __shared__ double4 sst[128];
    __shared__ double red[2][256];
    load_stencil_lds(sst, a.stencil, a.n_stencil);
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int64_t slice = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    double v[2] = {0.0, 0.0};
    if (slice < a.n_slices) {
        const int64_t row = slice * 64 + lane;
        const double4 *__restrict__ uv = a.uv[cur];
        const double4 ui = uv[row];
        const int64_t base = a.slice_ptr[slice];
        const int64_t L = (a.slice_ptr[slice + 1] - base) >> 6;
        double at = 0.0, ae = 0.0;
        for (int64_t k = 0; k < L; k++) {
            const uint64_t m64 = uniform64(a.mask[(base >> 6) + k]);
            if (!((m64 >> lane) & 1ull)) continue;
            const uint32_t w = a.words[pd_widx(base, k, lane)];
            const double4 uj = uv[w >> 7];
            const double4 sd = sst[w & 127u];
            const double h0 = uj.x - ui.x, h1 = uj.y - ui.y, h2 = DIM == 3 ? uj.z - ui.z : 0.0;
            double e;
            if (FIN) {
                const double y0 = sd.w * sd.x + h0, y1 = sd.w * sd.y + h1, y2 = sd.w * sd.z + h2;
                e = sqrt((y0 * y0 + y1 * y1) + y2 * y2) - sd.w;
            } else {
                e = ext_canonical(sd.x, sd.y, DIM == 3 ? sd.z : 0.0, h0, h1, h2);
            }
            at += sd.w * e * uj.w;
            ae += e * e * uj.w;
        }
        if (ui.w > 0.0) {
            const pd_spec sp = a.spec[a.aux[row] >> 8];
            const double r = a.inv_m[row];
            const double th = sp.A * r * at;
            const double W = sp.kp / (2.0 * sp.A) * th * th + 0.5 * sp.G * r * ae;
            const double4 vv = ldv(a.vel, DIM, row);
            v[0] = 0.5 * sp.rho * ui.w * (vv.x * vv.x + vv.y * vv.y + vv.z * vv.z);
            v[1] = ui.w * W;
        }
    }
    block_sum_fixed<2>(v, red);
    if (threadIdx.x == 0) part[blockIdx.x] = make_double4(v[0], v[1], 0.0, 0.0);
}

// One block adds n partials: thread t takes t, t + 256, ... in index order,
// then the fixed tree.  Writes the four sums to out, or, with rec, records
// them as the energy check of the state (the previous check's total kept).
__global__ __launch_bounds__(256) void k_sum_partials(const double4 *part, int64_t n, double *out, int nout,
                                                      pd_ctl *rec) {
    __shared__ double red[4][256];
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t i = threadIdx.x; i < n; i += 256) {
        const double4 p = part[i];
        v[0] += p.x;
        v[1] += p.y;
        v[2] += p.z;
        v[3] += p.w;
    }
    block_sum_fixed<4>(v, red);
    if (threadIdx.x != 0) return;
    if (rec) {
        rec->en[2] = rec->en[0] + rec->en[1];
        rec->en[0] = v[0];
        rec->en[1] = v[1];
        rec->en[3] = (double)(rec->s2 + 1);  // 0 = no check yet
    } else {
        for (int q = 0; q < nout; q++) out[q] = v[q];
    }
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

// y = M^-1 (-f) on free components; block partials of x.Kx, x.Mx, y.My.
__global__ __launch_bounds__(256) void k_pi_step(int64_t n_pad, int dim, const uint32_t *aux, const pd_spec *spec,
                                                 const double4 *uv, const double4 *f, double4 *y,
                                                 double4 *part) {
    __shared__ double s[3][256];
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double acc[3] = {0.0, 0.0, 0.0};
    if (r < n_pad) {
        const double4 x = uv[r], ff = f[r];
        const uint32_t ax = aux[r];
        const double mass = spec[ax >> 8].rho * x.w;
        double xv[3] = {x.x, x.y, x.z}, fv[3] = {ff.x, ff.y, ff.z}, yv[3] = {0, 0, 0};
        for (int c = 0; c < dim; c++) {
            if ((ax >> c) & 1u) continue;
            if (!(mass > 0.0)) continue;
            const double kx = -fv[c];
            acc[0] += xv[c] * kx;
            acc[1] += xv[c] * mass * xv[c];
            yv[c] = kx / mass;
            acc[2] += yv[c] * yv[c] * mass;
        }
        y[r] = make_double4(yv[0], yv[1], yv[2], x.w);
    }
    block_sum_fixed<3>(acc, s);
    if (threadIdx.x == 0) part[blockIdx.x] = make_double4(acc[0], acc[1], acc[2], 0.0);
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
    // one thread per row and at least one per word of the control block
    const int64_t ctl_words = (int64_t)(sizeof(pd_ctl) / 8);
    const int64_t nb = ((a.n_pad > ctl_words ? a.n_pad : ctl_words) + 255) / 256;
    hipLaunchKernelGGL(k_state_init, dim3((unsigned)nb), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_state_read(const int32_t *perm, int64_t n_pad, int dim, const double4 *uv, const double *vel,
                             double *u_out, double *v_out, hipStream_t s) {
    const int64_t nb = (n_pad + 255) / 256;
    hipLaunchKernelGGL(k_state_read, dim3((unsigned)nb), dim3(256), 0, s, perm, n_pad, dim, uv, vel, u_out, v_out);
    return hipGetLastError();
}

hipError_t launch_damage(const DamageArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_damage, grid_for_slices(a.n_slices, 256), dim3(256), 0, s, a);
    return hipGetLastError();
}

int64_t reduce_parts(int64_t n_pad) { return (n_pad + 255) / 256; }

hipError_t launch_energy(const StepArgs &a, int cur, bool finite, double4 *part, double *out, int nout, pd_ctl *rec,
                         hipStream_t s) {
    const int64_t nb = reduce_parts(a.n_pad);
    const dim3 g((unsigned)nb), b(256);
    if (a.dim == 3) {
        if (finite) hipLaunchKernelGGL((k_energy_rows<3, true>), g, b, 0, s, a, cur, part);
        else hipLaunchKernelGGL((k_energy_rows<3, false>), g, b, 0, s, a, cur, part);
    } else {
        if (finite) hipLaunchKernelGGL((k_energy_rows<2, true>), g, b, 0, s, a, cur, part);
        else hipLaunchKernelGGL((k_energy_rows<2, false>), g, b, 0, s, a, cur, part);
    }
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, part, nb, out, nout, rec);
    return hipGetLastError();
}

hipError_t launch_pi_init(int64_t n_pad, int dim, const uint32_t *aux, double4 *uv, uint64_t seed,
                          hipStream_t s) {
    const int64_t nb = (n_pad + 255) / 256;
    hipLaunchKernelGGL(k_pi_init, dim3((unsigned)nb), dim3(256), 0, s, n_pad, dim, aux, uv, seed);
    return hipGetLastError();
}

hipError_t launch_pi_step(int64_t n_pad, int dim, const uint32_t *aux, const pd_spec *spec, double4 *uv,
                          const double4 *f, double4 *y, pd_ctl *ctl, double4 *part, hipStream_t s) {
    const int64_t nb = reduce_parts(n_pad);
    hipLaunchKernelGGL(k_pi_step, dim3((unsigned)nb), dim3(256), 0, s, n_pad, dim, aux, spec, uv, f, y, part);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, part, nb, ctl->red, 3, (pd_ctl *)nullptr);
    hipLaunchKernelGGL(k_pi_scale, dim3((unsigned)nb), dim3(256), 0, s, n_pad, y, uv, ctl->red);
    return hipGetLastError();
}

}  // namespace pdk
