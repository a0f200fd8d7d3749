// Adaptive dynamic relaxation of the linearized OSB-PD equations (the
// quasi-static solver of the paper's Example 4, in Kilic and Madenci's
// form).  One iteration is the FP64 force kernels without their update
// (breaking, dilatation, pair force into f_int), then three kernels here:
//   k_adr_sums    F = f_int + F_ext r(n); per row the local-stiffness terms
//                 u k u with k_r = -(F_r - F_r^prev) / (lambda_r dt v_r) and
//                 u^2 over the free components, and |F|^2; per-workgroup
//                 sums (a fixed tree, so the result does not depend on
//                 timing); F kept as the next iteration's F^prev
//   k_adr_reduce  one workgroup adds the per-workgroup sums in a fixed order
//                 and forms the damping c = 2 sqrt(sum u k u / sum u^2)
//   k_adr_update  v = ((2 - c dt) v + 2 dt F / lambda) / (2 + c dt) (first
//                 iteration: v = dt F / (2 lambda)), u += dt v
// The fictitious density comes from an upper bound of the row sums of |K|
// (k_adr_gamma, k_adr_lambda), so that lambda >= dt^2/4 sum_j |K_ij|.
#include <hip/hip_runtime.h>

#include "adr.h"

namespace pdk {

struct AdrArgs {
    double dt;
    double *lambda;
    double *f_prev;
    double *f_int;
    double *partial;
    double *stats;
    const double *vol;
    const double *inv_m;
};

static AdrArgs adr_args(const pd_problem_dev *p, const pd_adr_dev *R) {
    AdrArgs r{};
    r.dt = R->dt;
    r.lambda = R->lambda;
    r.f_prev = R->f_prev;
    r.f_int = R->f_int;
    r.partial = R->partial;
    r.stats = R->stats;
    r.vol = p->vol;
    r.inv_m = p->inv_m;
    return r;
}

// per row: B_i = sum_j b_ij M_ij into f_int[4i..4i+2], Gam_i = 2 sum_k
// gamma_ik |M_ik|_1 into f_int[4i+3] (intact bonds); one lane per row
template <int DIM>
__global__ __launch_bounds__(256) void k_adr_gamma(StepArgs a, AdrArgs r) {
    const int lane = threadIdx.x & 63;
    const int64_t slice = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (slice >= a.n_slices) return;
    const int64_t row = slice * 64 + lane;
    const int64_t base = a.slice_ptr[slice];
    const int64_t L = (a.slice_ptr[slice + 1] - base) >> 6;
    const pd_spec sp = a.spec[a.aux[row] >> 8];
    const double Vi = r.vol[row], ri = r.inv_m[row];
    double B[3] = {0.0, 0.0, 0.0}, gam = 0.0;
    for (int64_t k = 0; k < L; k++) {
        if (!((a.mask[(base >> 6) + k] >> lane) & 1ull)) continue;
        const uint32_t w = a.words[pd_widx(base, k, lane)];
        const int64_t j = w >> 7;
        const double *st = a.stencil + 4 * (w & 127u);
        const double x = st[3], Vj = r.vol[j];
        const double bij = sp.kp * x * Vi * Vj;
        double m1 = 0.0;
        for (int c = 0; c < DIM; c++) {
            B[c] += bij * st[c];
            m1 += fabs(st[c]);
        }
        gam += 2.0 * (sp.A * x * Vj * ri * ri) * m1;
    }
    r.f_int[4 * row + 0] = B[0];
    r.f_int[4 * row + 1] = B[1];
    r.f_int[4 * row + 2] = B[2];
    r.f_int[4 * row + 3] = gam;
}

// lambda from the bound of the row sums; f_prev and stats cleared
template <int DIM>
__global__ __launch_bounds__(256) void k_adr_lambda(StepArgs a, AdrArgs r) {
    const int lane = threadIdx.x & 63;
    const int64_t slice = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (slice >= a.n_slices) return;
    if (blockIdx.x == 0 && threadIdx.x < 8) r.stats[threadIdx.x] = 0.0;
    const int64_t row = slice * 64 + lane;
    const int64_t base = a.slice_ptr[slice];
    const int64_t L = (a.slice_ptr[slice + 1] - base) >> 6;
    const pd_spec sp = a.spec[a.aux[row] >> 8];
    const double Vi = r.vol[row], ri = r.inv_m[row];
    double acc[3] = {0.0, 0.0, 0.0};
    for (int64_t k = 0; k < L; k++) {
        if (!((a.mask[(base >> 6) + k] >> lane) & 1ull)) continue;
        const uint32_t w = a.words[pd_widx(base, k, lane)];
        const int64_t j = w >> 7;
        const double *st = a.stencil + 4 * (w & 127u);
        const double x = st[3], Vj = r.vol[j], rj = r.inv_m[j];
        const double cij = sp.G * Vi * Vj * (ri + rj);
        const double bij = fabs(sp.kp * x * Vi * Vj);
        const double gj = r.f_int[4 * j + 3];
        double m1 = 0.0;
        for (int c = 0; c < DIM; c++) m1 += fabs(st[c]);
        for (int c = 0; c < DIM; c++) acc[c] += 2.0 * cij * fabs(st[c]) * m1 + bij * fabs(st[c]) * gj;
    }
    const double gi = r.f_int[4 * row + 3];
    const double q = 0.25 * r.dt * r.dt;
    for (int c = 0; c < 4; c++) {
        const double l = c < DIM ? q * (acc[c] + fabs(r.f_int[4 * row + c]) * gi) : 0.0;
        r.lambda[4 * row + c] = l > 0.0 ? l : 1.0;
        r.f_prev[4 * row + c] = 0.0;
    }
}

// fixed-shape tree sum of 256 values per workgroup
__device__ __forceinline__ double block_sum(double v, double *sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    const double out = sh[0];
    __syncthreads();
    return out;
}

template <int DIM>
__global__ __launch_bounds__(256) void k_adr_sums(StepArgs a, AdrArgs r, int cur) {
    __shared__ double sh[256];
    const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool first = r.stats[5] == 0.0;
    double num = 0.0, den = 0.0, res = 0.0;
    if (row < a.n_pad) {
        const int64_t n = a.ctl->s1;
        double rr = 1.0;
        if (a.ramp_steps > 0) rr = n >= a.ramp_steps ? 1.0 : (double)n / (double)a.ramp_steps;
        const uint32_t aux = a.aux[row];
        const double4 fi = reinterpret_cast<const double4 *>(r.f_int)[row];
        double F[3] = {fi.x, fi.y, fi.z};
        if (aux & 8u) {
            const double4 fe = a.fext[row];
            F[0] += fe.x * rr;
            F[1] += fe.y * rr;
            F[2] += fe.z * rr;
        }
        const double4 u4 = a.uv[cur][row];
        const double4 v4 = ldv(a.vel, DIM, row);
        const double u[3] = {u4.x, u4.y, u4.z}, v[3] = {v4.x, v4.y, v4.z};
        const double *lam = r.lambda + 4 * row;
        const double *fp = r.f_prev + 4 * row;
        for (int c = 0; c < DIM; c++) {
            if (aux & (1u << c)) continue;
            res += F[c] * F[c];
            if (!first && v[c] != 0.0) {
                const double k = -(F[c] / lam[c] - fp[c] / lam[c]) / (r.dt * v[c]);
                num += u[c] * k * u[c];
            }
            den += u[c] * u[c];
        }
        reinterpret_cast<double4 *>(r.f_prev)[row] = make_double4(F[0], F[1], F[2], 0.0);
    }
    num = block_sum(num, sh);
    den = block_sum(den, sh);
    res = block_sum(res, sh);
    if (threadIdx.x == 0) {
        r.partial[4 * blockIdx.x + 0] = num;
        r.partial[4 * blockIdx.x + 1] = den;
        r.partial[4 * blockIdx.x + 2] = res;
    }
}

__global__ __launch_bounds__(256) void k_adr_reduce(AdrArgs r, int nblocks) {
    __shared__ double sh[256];
    double s[3] = {0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x)
        for (int q = 0; q < 3; q++) s[q] += r.partial[4 * b + q];
    for (int q = 0; q < 3; q++) s[q] = block_sum(s[q], sh);
    if (threadIdx.x == 0) {
        const bool first = r.stats[5] == 0.0;
        double c = 0.0;
        if (!first && s[1] > 0.0 && s[0] > 0.0) c = 2.0 * sqrt(s[0] / s[1]);
        r.stats[0] = c;
        r.stats[1] = s[0];
        r.stats[2] = s[1];
        r.stats[3] = s[2];
        r.stats[4] = first ? 1.0 : 0.0;
        r.stats[5] = r.stats[5] + 1.0;
    }
}

template <int DIM>
__global__ __launch_bounds__(256) void k_adr_update(StepArgs a, AdrArgs r, int cur) {
    const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (row == 0) a.ctl->s2 = a.ctl->s1 + 1;
    if (row >= a.n_pad) return;
    const bool first = r.stats[4] != 0.0;
    const double c = r.stats[0], dt = r.dt;
    const uint32_t aux = a.aux[row];
    const double4 F = reinterpret_cast<const double4 *>(r.f_prev)[row];
    const double4 lam = reinterpret_cast<const double4 *>(r.lambda)[row];
    double4 v = ldv(a.vel, DIM, row);
    double4 u = a.uv[cur][row];
    const double Fc[3] = {F.x, F.y, F.z}, lc[3] = {lam.x, lam.y, lam.z};
    double vc[3] = {v.x, v.y, v.z};
    for (int q = 0; q < DIM; q++) {
        if (aux & (1u << q)) continue;
        if (first) vc[q] = dt * Fc[q] / (2.0 * lc[q]);
        else vc[q] = ((2.0 - c * dt) * vc[q] + 2.0 * dt * Fc[q] / lc[q]) / (2.0 + c * dt);
    }
    v.x = vc[0];
    v.y = vc[1];
    v.z = vc[2];
    u.x = u.x + dt * v.x;
    u.y = u.y + dt * v.y;
    u.z = u.z + dt * v.z;
    a.uv[cur ^ 1][row] = u;
    stv(a.vel, DIM, row, v);
    if (!(isfinite(u.x) && isfinite(u.y) && isfinite(u.z))) atomicOr(&a.ctl->flags, PD_CTL_NONFINITE);
}

int adr_blocks(int64_t n_pad) { return (int)((n_pad + 255) / 256); }

hipError_t launch_adr_density(const StepArgs &a, const pd_problem_dev *p, const pd_adr_dev *R, hipStream_t s) {
    const AdrArgs r = adr_args(p, R);
    const dim3 g((unsigned)((a.n_slices + 3) / 4));
    if (a.dim == 3) hipLaunchKernelGGL((k_adr_gamma<3>), g, dim3(256), 0, s, a, r);
    else hipLaunchKernelGGL((k_adr_gamma<2>), g, dim3(256), 0, s, a, r);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (a.dim == 3) hipLaunchKernelGGL((k_adr_lambda<3>), g, dim3(256), 0, s, a, r);
    else hipLaunchKernelGGL((k_adr_lambda<2>), g, dim3(256), 0, s, a, r);
    return hipGetLastError();
}

hipError_t launch_adr_iteration(const StepArgs &a, const pd_problem_dev *p, const pd_adr_dev *R, int cur,
                                hipStream_t s) {
    const AdrArgs r = adr_args(p, R);
    const int nb = adr_blocks(a.n_pad);
    if (a.dim == 3) hipLaunchKernelGGL((k_adr_sums<3>), dim3(nb), dim3(256), 0, s, a, r, cur);
    else hipLaunchKernelGGL((k_adr_sums<2>), dim3(nb), dim3(256), 0, s, a, r, cur);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_adr_reduce, dim3(1), dim3(256), 0, s, r, nb);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (a.dim == 3) hipLaunchKernelGGL((k_adr_update<3>), dim3(nb), dim3(256), 0, s, a, r, cur);
    else hipLaunchKernelGGL((k_adr_update<2>), dim3(nb), dim3(256), 0, s, a, r, cur);
    return hipGetLastError();
}

}  // namespace pdk
