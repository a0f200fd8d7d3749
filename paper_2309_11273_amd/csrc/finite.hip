// Finite-deformation form of the OSB-PD force (Eqs. 1.10, 1.13): the
// extension is e = |Y| - x with the deformed bond Y = x M + (u_j - u_i), and
// the pair force of Eq. 2.2 acts along Y / |Y| instead of the reference
// direction M.  The dilatation (Eq. 1.6), the critical-stretch test
// (Eqs. 1.17, 1.30) and the update are those of the linearized step.
//
// Bond-list (gather) kernels in double precision, laid out like the
// linearized gather kernels: one wave per 64-row slice, bond words in groups
// of four per lane, neighbour rows gathered through L2, the stencil table in
// LDS.  |Y|^2 is summed as (Y1^2 + Y2^2) + Y3^2 without contraction, so both
// directed copies of a bond (Y_ji = -Y_ij exactly) get the same e and take
// the same breaking decision.
#include <hip/hip_runtime.h>

#include <cmath>

#include "finite.h"

namespace pdk {

namespace {

// deformed bond length |x M + eta| (correctly rounded: it decides breaking)
// and, with DIR, the direction Y / |Y| from the hardware reciprocal square
// root refined by one Newton step, r <- r (3 - s r^2) / 2 (relative error
// about 1e-13, a fraction of the cost of three double divides)
template <bool DIR>
__device__ __forceinline__ double deformed_length(const double4 &st, double e1, double e2, double e3, double *dir) {
#pragma clang fp contract(off)
    const double y1 = st.w * st.x + e1;
    const double y2 = st.w * st.y + e2;
    const double y3 = st.w * st.z + e3;
    const double yy = (y1 * y1 + y2 * y2) + y3 * y3;
    if (DIR) {
        const double r = __builtin_amdgcn_rsq(yy);
        const double iy = r * fma(-0.5 * yy, r * r, 1.5);
        dir[0] = y1 * iy;
        dir[1] = y2 * iy;
        dir[2] = y3 * iy;
    }
    return sqrt(yy);
}

__device__ __forceinline__ uint64_t wave_uniform64(uint64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ void stage_stencil(double4 *sst, const double *stencil, int n_stencil) {
    for (int s = threadIdx.x; s < 128; s += blockDim.x) {
        double4 v = make_double4(0.0, 0.0, 0.0, 0.0);
        if (s < n_stencil) v = make_double4(stencil[4 * s], stencil[4 * s + 1], stencil[4 * s + 2], stencil[4 * s + 3]);
        sst[s] = v;
    }
}

}  // namespace

// pass 1: breaking and dilatation with the finite extension
template <int DIM, bool BREAK>
__global__ __launch_bounds__(256) void k_fin_pass1(StepArgs a, int cur) {
    __shared__ double4 sst[128];
    stage_stencil(sst, a.stencil, a.n_stencil);
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int64_t slice = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (slice >= a.n_slices) return;
    if (BREAK && blockIdx.x == 0 && threadIdx.x == 0) a.ctl->s1 = a.ctl->s2;
    const int64_t row = slice * 64 + lane;
    const int64_t base = a.slice_ptr[slice];
    const int64_t G = (a.slice_ptr[slice + 1] - base) >> 8;
    const double4 *__restrict__ uv = a.uv[cur];
    const double4 ui = uv[row];
    const pd_spec sp = a.spec[a.aux[row] >> 8];
    double acc = 0.0;
    uint32_t nbroken = 0;
    const uint4 *__restrict__ wg = reinterpret_cast<const uint4 *>(a.words + base) + lane;
    const uint4 *__restrict__ mg = reinterpret_cast<const uint4 *>(a.mask + (base >> 6));
    for (int64_t g = 0; g < G; g++) {
        const uint4 w4 = wg[g * 64];
        const uint4 ma = mg[2 * g], mb = mg[2 * g + 1];
        const uint64_t m[4] = {wave_uniform64(((uint64_t)ma.y << 32) | ma.x),
                               wave_uniform64(((uint64_t)ma.w << 32) | ma.z),
                               wave_uniform64(((uint64_t)mb.y << 32) | mb.x),
                               wave_uniform64(((uint64_t)mb.w << 32) | mb.z)};
        if ((m[0] | m[1] | m[2] | m[3]) == 0) continue;
        const uint32_t ws[4] = {w4.x, w4.y, w4.z, w4.w};
        double4 uj[4];
#pragma unroll
        for (int c = 0; c < 4; c++) uj[c] = uv[ws[c] >> 7];
#pragma unroll
        for (int c = 0; c < 4; c++) {
            const double4 st = sst[ws[c] & 127u];
            const double y = deformed_length<false>(st, uj[c].x - ui.x, uj[c].y - ui.y,
                                                    DIM == 3 ? uj[c].z - ui.z : 0.0, nullptr);
            const double e = y - st.w;
            bool intact = (m[c] >> lane) & 1ull;
            bool broke = false;
            if (BREAK && intact && e / st.w >= sp.s0) {
                intact = false;
                broke = true;
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
    const double ri = a.qr[row].y;
    a.qr[row].x = sp.A * ri * acc * ri;  // theta_i / m_i
    if (a.theta_out) a.theta_out[row] = sp.A * ri * acc;
    if (BREAK && lane == 0 && nbroken) atomicAdd(&a.ctl->broken, (unsigned long long)nbroken);
}

// pass 2: pair force along the deformed bond; UPDATE: the explicit update
template <int DIM, bool UPDATE>
__global__ __launch_bounds__(256) void k_fin_pass2(StepArgs a, int cur) {
    __shared__ double4 sst[128];
    stage_stencil(sst, a.stencil, a.n_stencil);
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int64_t slice = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (slice >= a.n_slices) return;
    const int64_t row = slice * 64 + lane;
    const int64_t base = a.slice_ptr[slice];
    const int64_t G = (a.slice_ptr[slice + 1] - base) >> 8;
    const double4 *__restrict__ uv = a.uv[cur];
    const double2 *__restrict__ qr = a.qr;
    const double4 ui = uv[row];
    const double2 qri = qr[row];
    const uint32_t aux = a.aux[row];
    const pd_spec sp = a.spec[aux >> 8];
    double f[3] = {0.0, 0.0, 0.0};
    const uint4 *__restrict__ wg = reinterpret_cast<const uint4 *>(a.words + base) + lane;
    const uint4 *__restrict__ mg = reinterpret_cast<const uint4 *>(a.mask + (base >> 6));
    for (int64_t g = 0; g < G; g++) {
        const uint4 w4 = wg[g * 64];
        const uint4 ma = mg[2 * g], mb = mg[2 * g + 1];
        const uint64_t m[4] = {wave_uniform64(((uint64_t)ma.y << 32) | ma.x),
                               wave_uniform64(((uint64_t)ma.w << 32) | ma.z),
                               wave_uniform64(((uint64_t)mb.y << 32) | mb.x),
                               wave_uniform64(((uint64_t)mb.w << 32) | mb.z)};
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
            if (!((m[c] >> lane) & 1ull)) continue;
            const double4 st = sst[ws[c] & 127u];
            double dir[3];
            const double y = deformed_length<true>(st, uj[c].x - ui.x, uj[c].y - ui.y,
                                                   DIM == 3 ? uj[c].z - ui.z : 0.0, dir);
            const double e = y - st.w;
            // [(K - G/3) x (theta_i/m_i + theta_j/m_j) + G e (1/m_i + 1/m_j)] V_j
            const double t = (sp.kp * st.w * (qri.x + qrj[c].x) + sp.G * e * (qri.y + qrj[c].y)) * uj[c].w;
            for (int q = 0; q < DIM; q++) f[q] += t * dir[q];
        }
    }
    double fx = f[0] * ui.w, fy = f[1] * ui.w, fz = f[2] * ui.w;
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
    if (!(isfinite(u.x) && isfinite(u.y) && isfinite(u.z))) atomicOr(&a.ctl->flags, PD_CTL_NONFINITE);
}

hipError_t launch_fin_pass1(const StepArgs &a, int cur, bool brk, int block, hipStream_t s) {
    const int wpb = block / 64;
    const dim3 g((unsigned)((a.n_slices + wpb - 1) / wpb));
#define PD_F1(D, B) hipLaunchKernelGGL((k_fin_pass1<D, B>), g, dim3(block), 0, s, a, cur)
    if (a.dim == 3) { if (brk) PD_F1(3, true); else PD_F1(3, false); }
    else { if (brk) PD_F1(2, true); else PD_F1(2, false); }
#undef PD_F1
    return hipGetLastError();
}

hipError_t launch_fin_pass2(const StepArgs &a, int cur, bool update, int block, hipStream_t s) {
    const int wpb = block / 64;
    const dim3 g((unsigned)((a.n_slices + wpb - 1) / wpb));
#define PD_F2(D, U) hipLaunchKernelGGL((k_fin_pass2<D, U>), g, dim3(block), 0, s, a, cur)
    if (a.dim == 3) { if (update) PD_F2(3, true); else PD_F2(3, false); }
    else { if (update) PD_F2(2, true); else PD_F2(2, false); }
#undef PD_F2
    return hipGetLastError();
}

}  // namespace pdk
