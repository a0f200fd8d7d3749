// Static equilibrium with the assembled block-sparse stiffness (Eq. 2.14):
// preconditioned conjugate gradients on the free components.
//
// With the restoring force in difference form f_i = sum_q Kt_iq (u_q - u_i)
// (bsr.hip), the stiffness is K = -df/du: K_iq = -Kt_iq (q != i) and
// K_ii = sum_q Kt_iq.  Starting from the current displacement u0 (its
// prescribed components held), the solver finds du with du = 0 on the
// prescribed components and
//   K_ff du_f = F_ext,f + f(u0)_f        (the out-of-balance force),
// then writes u0 + du.  The preconditioner is block Jacobi, P D^-1 P with
// D_i = K_ii inverted per node and P the projection on the free components.
//
// One iteration: q = K p (one wave per row, like the block product of the
// explicit step), the p.q sum, alpha; x += alpha p, r -= alpha q,
// z = P D^-1 P r with the r.z and r.r sums; beta; p = z + beta p.  Sums are
// per-workgroup partials (a fixed tree) added in a fixed order by one
// workgroup, so a solve gives the same bits on every run.
#include <hip/hip_runtime.h>

#include <cmath>

#include "cg.h"

namespace pdk {

namespace {

struct CgArgs {
    const int64_t *row_ptr;
    const int32_t *col;
    const double *vals;
    double4 *r, *z, *p, *q, *x;
    double *dinv;  // 12 per row: the 3x3 inverse (row-major), 3 unused
    double *partial;
    double *scal;  // rz, alpha, beta, rr, rr0, rel, iterations
};

__device__ __forceinline__ double block_sum256(double v, double *sh) {
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

// wave-per-row difference product s_i = sum_q Kt_iq (v_q - v_i)
template <int DIM>
__device__ __forceinline__ void row_product(const CgArgs &c, int64_t row, const double4 *v, double out[3]) {
    constexpr int NV = DIM * DIM;
    const int lane = threadIdx.x & 63;
    const double4 vi = v[row];
    const int64_t rp0 = c.row_ptr[row], nblk = c.row_ptr[row + 1] - rp0;
    double f[3] = {0.0, 0.0, 0.0};
#pragma unroll 2
    for (int64_t t = lane; t < nblk; t += 64) {
        const double4 vq = v[c.col[rp0 + t]];
        const double d[3] = {vq.x - vi.x, vq.y - vi.y, DIM == 3 ? vq.z - vi.z : 0.0};
        // entry (a, b) of the block at (a DIM + b) nblk (component-major rows)
        const double *K = c.vals + (size_t)rp0 * NV + t;
        for (int a = 0; a < DIM; a++)
            for (int b = 0; b < DIM; b++) f[a] += K[(a * DIM + b) * nblk] * d[b];
    }
    for (int o = 32; o > 0; o >>= 1)
        for (int a = 0; a < 3; a++) f[a] += __shfl_xor(f[a], o);
    for (int a = 0; a < 3; a++) out[a] = f[a];
}

__device__ __forceinline__ double4 masked(double4 v, uint32_t aux) {
    if (aux & 1u) v.x = 0.0;
    if (aux & 2u) v.y = 0.0;
    if (aux & 4u) v.z = 0.0;
    v.w = 0.0;
    return v;
}

__device__ __forceinline__ double4 precondition(const double *Di, double4 r, uint32_t aux) {
    r = masked(r, aux);
    double4 z = make_double4(Di[0] * r.x + Di[1] * r.y + Di[2] * r.z, Di[3] * r.x + Di[4] * r.y + Di[5] * r.z,
                             Di[6] * r.x + Di[7] * r.y + Di[8] * r.z, 0.0);
    return masked(z, aux);
}

}  // namespace

// D_i = sum_q Kt_iq and its inverse (identity where D_i is singular, e.g.
// padding rows); one thread per row
template <int DIM>
__global__ __launch_bounds__(256) void k_cg_dinv(StepArgs a, CgArgs c) {
    constexpr int NV = DIM * DIM;
    const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= a.n_pad) return;
    double D[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    const int64_t rp0 = c.row_ptr[row], nblk = c.row_ptr[row + 1] - rp0;
    for (int64_t t = 0; t < nblk; t++) {
        const double *K = c.vals + (size_t)rp0 * NV + t;
        for (int i = 0; i < DIM; i++)
            for (int j = 0; j < DIM; j++) D[3 * i + j] += K[(i * DIM + j) * nblk];
    }
    if (DIM == 2) D[8] = 1.0;
    const double c00 = D[4] * D[8] - D[5] * D[7], c01 = D[5] * D[6] - D[3] * D[8], c02 = D[3] * D[7] - D[4] * D[6];
    const double det = D[0] * c00 + D[1] * c01 + D[2] * c02;
    double inv[9];
    double scale = 0.0;
    for (int k = 0; k < 9; k++) scale = fmax(scale, fabs(D[k]));
    if (!(fabs(det) > 1e-300) || !(fabs(det) > 1e-12 * scale * scale * scale)) {
        for (int k = 0; k < 9; k++) inv[k] = (k % 4 == 0) ? 1.0 : 0.0;
    } else {
        const double id = 1.0 / det;
        inv[0] = c00 * id;
        inv[1] = (D[2] * D[7] - D[1] * D[8]) * id;
        inv[2] = (D[1] * D[5] - D[2] * D[4]) * id;
        inv[3] = c01 * id;
        inv[4] = (D[0] * D[8] - D[2] * D[6]) * id;
        inv[5] = (D[2] * D[3] - D[0] * D[5]) * id;
        inv[6] = c02 * id;
        inv[7] = (D[1] * D[6] - D[0] * D[7]) * id;
        inv[8] = (D[0] * D[4] - D[1] * D[3]) * id;
    }
    if (DIM == 2) inv[2] = inv[5] = inv[6] = inv[7] = inv[8] = 0.0;
    for (int k = 0; k < 9; k++) c.dinv[12 * row + k] = inv[k];
}

// r = F_ext + f(u0) on the free components (one wave per row)
template <int DIM>
__global__ __launch_bounds__(256) void k_cg_residual(StepArgs a, CgArgs c, int cur) {
    const int64_t row = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (row >= a.n_pad) return;
    double f[3];
    row_product<DIM>(c, row, a.uv[cur], f);
    if ((threadIdx.x & 63) != 0) return;
    const uint32_t aux = a.aux[row];
    double4 r = make_double4(f[0], f[1], f[2], 0.0);
    if (aux & 8u) {
        const double4 fe = a.fext[row];
        r.x += fe.x;
        r.y += fe.y;
        r.z += fe.z;
    }
    c.r[row] = masked(r, aux);
}

// q = K p = -(difference product of p) on the free components
template <int DIM>
__global__ __launch_bounds__(256) void k_cg_matvec(StepArgs a, CgArgs c) {
    const int64_t row = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (row >= a.n_pad) return;
    double f[3];
    row_product<DIM>(c, row, c.p, f);
    if ((threadIdx.x & 63) != 0) return;
    c.q[row] = masked(make_double4(-f[0], -f[1], -f[2], 0.0), a.aux[row]);
}

// mode 0 (start): x = 0, z = M r, p = z, sums r.z and r.r
// mode 1: sum p.q
// mode 2: x += alpha p, r -= alpha q, z = M r, sums r.z and r.r
__global__ __launch_bounds__(256) void k_cg_vec(StepArgs a, CgArgs c, int mode) {
    __shared__ double sh[256];
    const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double s0 = 0.0, s1 = 0.0;
    if (row < a.n_pad) {
        const uint32_t aux = a.aux[row];
        if (mode == 1) {
            const double4 p = c.p[row], q = c.q[row];
            s0 = p.x * q.x + p.y * q.y + p.z * q.z;
        } else {
            double4 r = c.r[row];
            if (mode == 0) {
                c.x[row] = make_double4(0.0, 0.0, 0.0, 0.0);
            } else {
                const double al = c.scal[1];
                const double4 p = c.p[row], q = c.q[row];
                double4 x = c.x[row];
                x.x += al * p.x;
                x.y += al * p.y;
                x.z += al * p.z;
                c.x[row] = x;
                r.x -= al * q.x;
                r.y -= al * q.y;
                r.z -= al * q.z;
                c.r[row] = r;
            }
            const double4 z = precondition(c.dinv + 12 * row, r, aux);
            c.z[row] = z;
            if (mode == 0) c.p[row] = z;
            s0 = r.x * z.x + r.y * z.y + r.z * z.z;
            s1 = r.x * r.x + r.y * r.y + r.z * r.z;
        }
    }
    s0 = block_sum256(s0, sh);
    s1 = block_sum256(s1, sh);
    if (threadIdx.x == 0) {
        c.partial[2 * blockIdx.x] = s0;
        c.partial[2 * blockIdx.x + 1] = s1;
    }
}

// one workgroup: add the partial sums in a fixed order, then
// mode 0: rz, rr0 = rr; mode 1: alpha = rz / pq; mode 2: beta, rz, residual
__global__ __launch_bounds__(256) void k_cg_scalars(CgArgs c, int nblocks, int mode) {
    __shared__ double sh[256];
    double s0 = 0.0, s1 = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) {
        s0 += c.partial[2 * b];
        s1 += c.partial[2 * b + 1];
    }
    s0 = block_sum256(s0, sh);
    s1 = block_sum256(s1, sh);
    if (threadIdx.x != 0) return;
    double *S = c.scal;
    if (mode == 0) {
        S[0] = s0;
        S[3] = s1;
        S[4] = s1;
        S[5] = s1 > 0.0 ? 1.0 : 0.0;
        S[6] = 0.0;
    } else if (mode == 1) {
        S[1] = (s0 > 0.0 && S[0] != 0.0) ? S[0] / s0 : 0.0;
    } else {
        S[2] = S[0] != 0.0 ? s0 / S[0] : 0.0;
        S[0] = s0;
        S[3] = s1;
        S[5] = S[4] > 0.0 ? sqrt(s1 / S[4]) : 0.0;
        S[6] += 1.0;
    }
}

// p = z + beta p
__global__ __launch_bounds__(256) void k_cg_direction(StepArgs a, CgArgs c) {
    const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= a.n_pad) return;
    const double be = c.scal[2];
    const double4 z = c.z[row];
    double4 p = c.p[row];
    p.x = z.x + be * p.x;
    p.y = z.y + be * p.y;
    p.z = z.z + be * p.z;
    c.p[row] = p;
}

// u = u0 + x
__global__ __launch_bounds__(256) void k_cg_finish(StepArgs a, CgArgs c, int cur) {
    const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= a.n_pad) return;
    const double4 x = c.x[row];
    double4 u = a.uv[cur][row];
    u.x += x.x;
    u.y += x.y;
    u.z += x.z;
    a.uv[cur][row] = u;
    if (!(isfinite(u.x) && isfinite(u.y) && isfinite(u.z))) atomicOr(&a.ctl->flags, PD_CTL_NONFINITE);
}

int64_t cg_workspace_doubles(int64_t n_pad) {
    const int64_t nb = (n_pad + 255) / 256;
    return 5 * 4 * n_pad + 12 * n_pad + 2 * nb + 16;
}

static CgArgs cg_args(const pd_bsr_dev *K, double *work, int64_t n_pad) {
    CgArgs c{};
    c.row_ptr = K->row_ptr;
    c.col = K->col;
    c.vals = reinterpret_cast<const double *>(K->vals);
    double *w = work;
    c.r = reinterpret_cast<double4 *>(w);
    w += 4 * n_pad;
    c.z = reinterpret_cast<double4 *>(w);
    w += 4 * n_pad;
    c.p = reinterpret_cast<double4 *>(w);
    w += 4 * n_pad;
    c.q = reinterpret_cast<double4 *>(w);
    w += 4 * n_pad;
    c.x = reinterpret_cast<double4 *>(w);
    w += 4 * n_pad;
    c.dinv = w;
    w += 12 * n_pad;
    c.partial = w;
    w += 2 * ((n_pad + 255) / 256);
    c.scal = w;
    return c;
}

hipError_t launch_cg_start(const StepArgs &a, const pd_bsr_dev *K, double *work, int cur, hipStream_t s) {
    const CgArgs c = cg_args(K, work, a.n_pad);
    const unsigned nrow = (unsigned)((a.n_pad + 255) / 256), nwave = (unsigned)((a.n_pad + 3) / 4);
    if (a.dim == 3) {
        hipLaunchKernelGGL((k_cg_dinv<3>), dim3(nrow), dim3(256), 0, s, a, c);
        hipLaunchKernelGGL((k_cg_residual<3>), dim3(nwave), dim3(256), 0, s, a, c, cur);
    } else {
        hipLaunchKernelGGL((k_cg_dinv<2>), dim3(nrow), dim3(256), 0, s, a, c);
        hipLaunchKernelGGL((k_cg_residual<2>), dim3(nwave), dim3(256), 0, s, a, c, cur);
    }
    hipLaunchKernelGGL(k_cg_vec, dim3(nrow), dim3(256), 0, s, a, c, 0);
    hipLaunchKernelGGL(k_cg_scalars, dim3(1), dim3(256), 0, s, c, (int)nrow, 0);
    return hipGetLastError();
}

hipError_t launch_cg_iteration(const StepArgs &a, const pd_bsr_dev *K, double *work, hipStream_t s) {
    const CgArgs c = cg_args(K, work, a.n_pad);
    const unsigned nrow = (unsigned)((a.n_pad + 255) / 256), nwave = (unsigned)((a.n_pad + 3) / 4);
    if (a.dim == 3) hipLaunchKernelGGL((k_cg_matvec<3>), dim3(nwave), dim3(256), 0, s, a, c);
    else hipLaunchKernelGGL((k_cg_matvec<2>), dim3(nwave), dim3(256), 0, s, a, c);
    hipLaunchKernelGGL(k_cg_vec, dim3(nrow), dim3(256), 0, s, a, c, 1);
    hipLaunchKernelGGL(k_cg_scalars, dim3(1), dim3(256), 0, s, c, (int)nrow, 1);
    hipLaunchKernelGGL(k_cg_vec, dim3(nrow), dim3(256), 0, s, a, c, 2);
    hipLaunchKernelGGL(k_cg_scalars, dim3(1), dim3(256), 0, s, c, (int)nrow, 2);
    hipLaunchKernelGGL(k_cg_direction, dim3(nrow), dim3(256), 0, s, a, c);
    return hipGetLastError();
}

hipError_t launch_cg_finish(const StepArgs &a, const pd_bsr_dev *K, double *work, int cur, hipStream_t s) {
    const CgArgs c = cg_args(K, work, a.n_pad);
    hipLaunchKernelGGL(k_cg_finish, dim3((unsigned)((a.n_pad + 255) / 256)), dim3(256), 0, s, a, c, cur);
    return hipGetLastError();
}

const double *cg_scalars(double *work, int64_t n_pad) {
    return work + 5 * 4 * n_pad + 12 * n_pad + 2 * ((n_pad + 255) / 256);
}

}  // namespace pdk
