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
//
// Implicit dynamics (the counterpart of the explicit update of Eq. 2.11,
// whose cost with the wide-band K Remark 1 of Sec. 3.3 weighs): the
// average-acceleration Newmark rule (beta = 1/4, gamma = 1/2) with the lumped
// mass m_i = rho V_i.  One step from (u_n, v_n):
//   a_n = M^-1 (F_ext + f(u_n))               on the free components,
//   u*  = u_n, prescribed components advanced by dt v_n,
//   (K_ff + (4/dt^2) M) du_f = F_ext + f(u*) + M (4 v_n / dt + a_n)   (free),
//   u_{n+1} = u* + du,  a_{n+1} = (4/dt^2)(du - dt v_n) - a_n,
//   v_{n+1} = v_n + dt/2 (a_n + a_{n+1})      on the free components.
// The solve is the same preconditioned CG with the mass term added to the
// operator and to the block-Jacobi diagonal.  a_n is taken from the equation
// of motion at the start of each step (it equals the previous step's a_{n+1}
// when that solve converged and no bond broke).
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
    // implicit dynamics: lumped mass per row (nullptr for the static solve),
    // the operator's mass factor 4/dt^2, a_n per row
    double *mass;
    double shift;
    double4 *acc;
    // the state's displacements (volume V in .w): p carries V in .w too, so
    // that the force kernels can take p as a displacement field
    const double4 *uvc;
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

// the inverse of a diagonal block D (row-major 3x3; identity where D is
// singular, e.g. padding rows) into dinv
template <int DIM>
__device__ __forceinline__ void store_block_inverse(const CgArgs &c, int64_t row, double D[9]) {
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

__device__ __forceinline__ uint64_t wave_u64(uint64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

}  // namespace

// D_i = sum_q Kt_iq (plus the Newmark mass term) and its inverse (identity
// where D_i is singular, e.g. padding rows); one wave per row, the lanes
// striding over the row's blocks like the block product
template <int DIM>
__global__ __launch_bounds__(256) void k_cg_dinv(StepArgs a, CgArgs c) {
    constexpr int NV = DIM * DIM;
    const int64_t row = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (row >= a.n_pad) return;
    const int lane = threadIdx.x & 63;
    double D[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    const int64_t rp0 = c.row_ptr[row], nblk = c.row_ptr[row + 1] - rp0;
    for (int64_t t = lane; t < nblk; t += 64) {
        const double *K = c.vals + (size_t)rp0 * NV + t;
        for (int i = 0; i < DIM; i++)
            for (int j = 0; j < DIM; j++) D[3 * i + j] += K[(i * DIM + j) * nblk];
    }
    for (int o = 32; o > 0; o >>= 1)
        for (int k = 0; k < 9; k++) D[k] += __shfl_xor(D[k], o);
    if (lane != 0) return;
    if (c.mass) {
        const double sm = c.shift * c.mass[row];
        D[0] += sm;
        D[4] += sm;
        D[8] += sm;
    }
    store_block_inverse<DIM>(c, row, D);
}

// The diagonal block of K = -df/du without the stored K, from the force of
// Eq. 2.2 with q = theta / m (Eq. 1.8: q_i = A r_i^2 sum_k x V_k e_ik,
// r = 1/m, w = 1):
//   f_i = V_i sum_j V_j [kp x (q_i + q_j) + G e_ij (r_i + r_j)] M_ij,
// and u_i enters e_ij (de_ij/du_i = -M), q_i (dq_i/du_i = -A r_i^2 b_i,
// b_i = sum_j x V_j M_ij) and every neighbour's q_j (through e_ji:
// dq_j/du_i = -A r_j^2 x V_i M_ij), so
//   D_i = V_i [kp A r_i^2 b_i b_i^T
//              + sum_j V_j (kp A r_j^2 V_i x^2 + G (r_i + r_j)) M M^T]
// over the intact bonds; plus the Newmark mass term.  One wave per 64-row
// slice, each lane its own row, bond words and status bits as in the
// bond-list kernels.
template <int DIM>
__global__ __launch_bounds__(256) void k_cg_dinv_mf(StepArgs a, CgArgs c) {
    const int lane = threadIdx.x & 63;
    const int64_t slice = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (slice >= a.n_slices) return;
    const int64_t row = slice * 64 + lane;
    const int64_t base = a.slice_ptr[slice];
    const int64_t L = (a.slice_ptr[slice + 1] - base) >> 6;
    const double Vi = c.uvc[row].w, ri = a.qr[row].y;
    const pd_spec sp = a.spec[a.aux[row] >> 8];
    double S[6] = {0, 0, 0, 0, 0, 0}, b[3] = {0, 0, 0};
    for (int64_t k = 0; k < L; k++) {
        const uint64_t m64 = wave_u64(a.mask[(base >> 6) + k]);
        if (!((m64 >> lane) & 1ull)) continue;
        const uint32_t w = a.words[pd_widx(base, k, lane)];
        const int64_t j = w >> 7;
        const double *st = a.stencil + 4 * (w & 127u);
        const double x = st[3], Vj = c.uvc[j].w, rj = a.qr[j].y;
        const double cj = Vj * (sp.kp * sp.A * rj * rj * Vi * x * x + sp.G * (ri + rj));
        S[0] += cj * st[0] * st[0];
        S[1] += cj * st[0] * st[1];
        S[2] += cj * st[0] * st[2];
        S[3] += cj * st[1] * st[1];
        S[4] += cj * st[1] * st[2];
        S[5] += cj * st[2] * st[2];
        for (int q = 0; q < 3; q++) b[q] += Vj * x * st[q];
    }
    const double g = sp.kp * sp.A * ri * ri;
    double D[9] = {Vi * (S[0] + g * b[0] * b[0]), Vi * (S[1] + g * b[0] * b[1]), Vi * (S[2] + g * b[0] * b[2]),
                   Vi * (S[1] + g * b[1] * b[0]), Vi * (S[3] + g * b[1] * b[1]), Vi * (S[4] + g * b[1] * b[2]),
                   Vi * (S[2] + g * b[2] * b[0]), Vi * (S[4] + g * b[2] * b[1]), Vi * (S[5] + g * b[2] * b[2])};
    if (c.mass) {
        const double sm = c.shift * c.mass[row];
        D[0] += sm;
        D[4] += sm;
        D[8] += sm;
    }
    store_block_inverse<DIM>(c, row, D);
}

// r = F_ext + f(u0) on the free components (one wave per row)
// (MF: f(u0) already in q, written by the force kernels)
template <int DIM, bool MF>
__global__ __launch_bounds__(256) void k_cg_residual(StepArgs a, CgArgs c, int cur) {
    const int64_t row = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (row >= a.n_pad) return;
    double f[3];
    if (MF) {
        const double4 fq = c.q[row];
        f[0] = fq.x, f[1] = fq.y, f[2] = fq.z;
    } else {
        row_product<DIM>(c, row, a.uv[cur], f);
    }
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

// q = K p = -(difference product of p) on the free components, plus
// (4/dt^2) M p for implicit dynamics
template <int DIM>
__global__ __launch_bounds__(256) void k_cg_matvec(StepArgs a, CgArgs c) {
    const int64_t row = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (row >= a.n_pad) return;
    double f[3];
    row_product<DIM>(c, row, c.p, f);
    if ((threadIdx.x & 63) != 0) return;
    double4 q = make_double4(-f[0], -f[1], -f[2], 0.0);
    if (c.mass) {
        const double sm = c.shift * c.mass[row];
        const double4 pr = c.p[row];
        q.x += sm * pr.x;
        q.y += sm * pr.y;
        q.z += sm * pr.z;
    }
    c.q[row] = masked(q, a.aux[row]);
}

// matrix-free product: the force kernels have written f(p) (the restoring
// force of the direction taken as a displacement field, Eq. 2.2 summed) into
// q; q = -f(p) on the free components, plus (4/dt^2) M p for the implicit step
__global__ __launch_bounds__(256) void k_cg_mf_fix(StepArgs a, CgArgs c) {
    const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= a.n_pad) return;
    const double4 f = c.q[row];
    double4 q = make_double4(-f.x, -f.y, -f.z, 0.0);
    if (c.mass) {
        const double sm = c.shift * c.mass[row];
        const double4 pr = c.p[row];
        q.x += sm * pr.x;
        q.y += sm * pr.y;
        q.z += sm * pr.z;
    }
    c.q[row] = masked(q, a.aux[row]);
}

// Newmark start: m_i = rho V_i and a_n = (F_ext + f(u_n)) / m_i on the free
// components (zero for padding rows, whose mass is zero)
// (MF: f(u_n) already in q, written by the force kernels)
template <int DIM, bool MF>
__global__ __launch_bounds__(256) void k_nm_accel(StepArgs a, CgArgs c, int cur) {
    const int64_t row = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (row >= a.n_pad) return;
    double f[3];
    if (MF) {
        const double4 fq = c.q[row];
        f[0] = fq.x, f[1] = fq.y, f[2] = fq.z;
    } else {
        row_product<DIM>(c, row, a.uv[cur], f);
    }
    if ((threadIdx.x & 63) != 0) return;
    const uint32_t aux = a.aux[row];
    const double m = a.spec[aux >> 8].rho * a.uv[cur][row].w;
    double4 g = make_double4(f[0], f[1], f[2], 0.0);
    if (aux & 8u) {
        const double4 fe = a.fext[row];
        g.x += fe.x;
        g.y += fe.y;
        g.z += fe.z;
    }
    const double im = m > 0.0 ? 1.0 / m : 0.0;
    c.mass[row] = m;
    c.acc[row] = masked(make_double4(g.x * im, g.y * im, g.z * im, 0.0), aux);
}

// u* = u_n with the prescribed components advanced by dt v_n, into the other
// displacement buffer
__global__ __launch_bounds__(256) void k_nm_predict(StepArgs a, double dt, int cur) {
    const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= a.n_pad) return;
    if (row == 0) a.ctl->s1 = a.ctl->s2;
    const uint32_t aux = a.aux[row];
    double4 u = a.uv[cur][row];
    const double4 v = ldv(a.vel, a.dim, row);
    if (aux & 1u) u.x += dt * v.x;
    if (aux & 2u) u.y += dt * v.y;
    if (aux & 4u) u.z += dt * v.z;
    a.uv[cur ^ 1][row] = u;
}

// right-hand side F_ext + f(u*) + M (4 v_n / dt + a_n) on the free components
// (MF: f(u*) already in q)
template <int DIM, bool MF>
__global__ __launch_bounds__(256) void k_nm_rhs(StepArgs a, CgArgs c, double dt, int cur) {
    const int64_t row = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (row >= a.n_pad) return;
    double f[3];
    if (MF) {
        const double4 fq = c.q[row];
        f[0] = fq.x, f[1] = fq.y, f[2] = fq.z;
    } else {
        row_product<DIM>(c, row, a.uv[cur ^ 1], f);
    }
    if ((threadIdx.x & 63) != 0) return;
    const uint32_t aux = a.aux[row];
    const double m = c.mass[row];
    const double4 v = ldv(a.vel, DIM, row), an = c.acc[row];
    const double k4 = 4.0 / dt;
    double4 r = make_double4(f[0] + m * (k4 * v.x + an.x), f[1] + m * (k4 * v.y + an.y),
                             f[2] + m * (k4 * v.z + an.z), 0.0);
    if (aux & 8u) {
        const double4 fe = a.fext[row];
        r.x += fe.x;
        r.y += fe.y;
        r.z += fe.z;
    }
    c.r[row] = masked(r, aux);
}

// u_{n+1} = u* + du, a_{n+1} and v_{n+1} on the free components; the
// prescribed velocities are kept
__global__ __launch_bounds__(256) void k_nm_finish(StepArgs a, CgArgs c, double dt, int cur) {
    const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= a.n_pad) return;
    if (row == 0) a.ctl->s2 = a.ctl->s1 + 1;
    const uint32_t aux = a.aux[row];
    const double4 du = c.x[row], an = c.acc[row];
    double4 u = a.uv[cur ^ 1][row];
    u.x += du.x;
    u.y += du.y;
    u.z += du.z;
    a.uv[cur ^ 1][row] = u;
    double4 v = ldv(a.vel, a.dim, row);
    const double h = 0.5 * dt;
    if (!(aux & 1u)) v.x += h * (an.x + (c.shift * (du.x - dt * v.x) - an.x));
    if (!(aux & 2u)) v.y += h * (an.y + (c.shift * (du.y - dt * v.y) - an.y));
    if (!(aux & 4u)) v.z += h * (an.z + (c.shift * (du.z - dt * v.z) - an.z));
    stv(a.vel, a.dim, row, v);
    if (!(isfinite(u.x) && isfinite(u.y) && isfinite(u.z) && isfinite(v.x) && isfinite(v.y) && isfinite(v.z)))
        atomicOr(&a.ctl->flags, PD_CTL_NONFINITE);
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
            if (mode == 0) c.p[row] = make_double4(z.x, z.y, z.z, c.uvc[row].w);
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
    p.w = c.uvc[row].w;
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

// the Newmark arrays start at a 32-byte boundary after the solver's (a_n is
// read as double4)
static int64_t nm_base(int64_t n_pad) { return (cg_workspace_doubles(n_pad) + 3) & ~int64_t(3); }

int64_t nm_workspace_doubles(int64_t n_pad) { return nm_base(n_pad) + 5 * n_pad; }

// dt > 0: the Newmark operator K + (4/dt^2) M, with a_n and the mass after
// the solver's arrays
static CgArgs cg_args(const StepArgs &a, const pd_bsr_dev *K, double *work, int cur, double dt = 0.0) {
    const int64_t n_pad = a.n_pad;
    CgArgs c{};
    c.uvc = a.uv[cur];
    if (K) {
        c.row_ptr = K->row_ptr;
        c.col = K->col;
        c.vals = reinterpret_cast<const double *>(K->vals);
    }
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
    if (dt > 0.0) {
        double *e = work + nm_base(n_pad);
        c.acc = reinterpret_cast<double4 *>(e);
        c.mass = e + 4 * n_pad;
        c.shift = 4.0 / (dt * dt);
    }
    return c;
}

// restoring force f(uv[buf]) (Eq. 2.2 summed, no breaking, no update) into
// q by the double force kernels
static hipError_t force_into_q(const StepArgs &a, const CgArgs &c, int buf, hipStream_t s) {
    StepArgs af = a;
    af.f_out = c.q;
    af.theta_out = nullptr;
    const bool tiled = tiled64_supported(af);
    hipError_t e = tiled ? launch_tpass1_f64(af, buf, false, s) : launch_pass1_f64(af, buf, false, 256, s);
    if (e != hipSuccess) return e;
    return tiled ? launch_tpass2_f64(af, buf, false, s) : launch_pass2_f64(af, buf, false, 256, s);
}

// block-Jacobi diagonal: from the stored K when there is one, else from the
// bonds (k_cg_dinv_mf)
static void launch_dinv(const StepArgs &a, const pd_bsr_dev *K, const CgArgs &c, hipStream_t s) {
    const unsigned nwave = (unsigned)((a.n_pad + 3) / 4), nsl = (unsigned)((a.n_slices + 3) / 4);
    if (K) {
        if (a.dim == 3) hipLaunchKernelGGL((k_cg_dinv<3>), dim3(nwave), dim3(256), 0, s, a, c);
        else hipLaunchKernelGGL((k_cg_dinv<2>), dim3(nwave), dim3(256), 0, s, a, c);
    } else {
        if (a.dim == 3) hipLaunchKernelGGL((k_cg_dinv_mf<3>), dim3(nsl), dim3(256), 0, s, a, c);
        else hipLaunchKernelGGL((k_cg_dinv_mf<2>), dim3(nsl), dim3(256), 0, s, a, c);
    }
}

hipError_t launch_cg_start(const StepArgs &a, const pd_bsr_dev *K, double *work, int cur, bool mf, hipStream_t s) {
    const CgArgs c = cg_args(a, K, work, cur);
    const unsigned nrow = (unsigned)((a.n_pad + 255) / 256), nwave = (unsigned)((a.n_pad + 3) / 4);
    hipError_t e;
    if (mf && (e = force_into_q(a, c, cur, s)) != hipSuccess) return e;
    launch_dinv(a, K, c, s);
    if (a.dim == 3) {
        if (mf) hipLaunchKernelGGL((k_cg_residual<3, true>), dim3(nwave), dim3(256), 0, s, a, c, cur);
        else hipLaunchKernelGGL((k_cg_residual<3, false>), dim3(nwave), dim3(256), 0, s, a, c, cur);
    } else {
        if (mf) hipLaunchKernelGGL((k_cg_residual<2, true>), dim3(nwave), dim3(256), 0, s, a, c, cur);
        else hipLaunchKernelGGL((k_cg_residual<2, false>), dim3(nwave), dim3(256), 0, s, a, c, cur);
    }
    hipLaunchKernelGGL(k_cg_vec, dim3(nrow), dim3(256), 0, s, a, c, 0);
    hipLaunchKernelGGL(k_cg_scalars, dim3(1), dim3(256), 0, s, c, (int)nrow, 0);
    return hipGetLastError();
}


hipError_t launch_nm_start(const StepArgs &a, const pd_bsr_dev *K, double *work, double dt, int cur, bool mf,
                           hipStream_t s) {
    const CgArgs c = cg_args(a, K, work, cur, dt);
    const unsigned nrow = (unsigned)((a.n_pad + 255) / 256), nwave = (unsigned)((a.n_pad + 3) / 4);
    hipError_t e;
    if (mf && (e = force_into_q(a, c, cur, s)) != hipSuccess) return e;
#define PD_NM(KN, ...)                                                                                 \
    do {                                                                                               \
        if (a.dim == 3) {                                                                              \
            if (mf) hipLaunchKernelGGL((KN<3, true>), dim3(nwave), dim3(256), 0, s, __VA_ARGS__);      \
            else hipLaunchKernelGGL((KN<3, false>), dim3(nwave), dim3(256), 0, s, __VA_ARGS__);        \
        } else {                                                                                       \
            if (mf) hipLaunchKernelGGL((KN<2, true>), dim3(nwave), dim3(256), 0, s, __VA_ARGS__);      \
            else hipLaunchKernelGGL((KN<2, false>), dim3(nwave), dim3(256), 0, s, __VA_ARGS__);        \
        }                                                                                              \
    } while (0)
    PD_NM(k_nm_accel, a, c, cur);
    hipLaunchKernelGGL(k_nm_predict, dim3(nrow), dim3(256), 0, s, a, dt, cur);
    if (mf && (e = force_into_q(a, c, cur ^ 1, s)) != hipSuccess) return e;
    PD_NM(k_nm_rhs, a, c, dt, cur);
#undef PD_NM
    launch_dinv(a, K, c, s);
    hipLaunchKernelGGL(k_cg_vec, dim3(nrow), dim3(256), 0, s, a, c, 0);
    hipLaunchKernelGGL(k_cg_scalars, dim3(1), dim3(256), 0, s, c, (int)nrow, 0);
    return hipGetLastError();
}

hipError_t launch_nm_finish(const StepArgs &a, const pd_bsr_dev *K, double *work, double dt, int cur,
                            hipStream_t s) {
    const CgArgs c = cg_args(a, K, work, cur, dt);
    hipLaunchKernelGGL(k_nm_finish, dim3((unsigned)((a.n_pad + 255) / 256)), dim3(256), 0, s, a, c, dt, cur);
    return hipGetLastError();
}

hipError_t launch_cg_iteration(const StepArgs &a, const pd_bsr_dev *K, double *work, double dt, int cur, bool mf,
                               hipStream_t s) {
    const CgArgs c = cg_args(a, K, work, cur, dt);
    const unsigned nrow = (unsigned)((a.n_pad + 255) / 256), nwave = (unsigned)((a.n_pad + 3) / 4);
    if (mf) {
        // K p = -f(p): the double force kernels (no breaking, no update) on
        // p as the displacement field, then the sign, mask and mass term
        StepArgs am = a;
        am.uv[0] = c.p;
        am.f_out = c.q;
        am.theta_out = nullptr;
        const bool tiled = tiled64_supported(am);
        hipError_t e = tiled ? launch_tpass1_f64(am, 0, false, s) : launch_pass1_f64(am, 0, false, 256, s);
        if (e != hipSuccess) return e;
        e = tiled ? launch_tpass2_f64(am, 0, false, s) : launch_pass2_f64(am, 0, false, 256, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_cg_mf_fix, dim3(nrow), dim3(256), 0, s, am, c);
    } else if (a.dim == 3) {
        hipLaunchKernelGGL((k_cg_matvec<3>), dim3(nwave), dim3(256), 0, s, a, c);
    } else {
        hipLaunchKernelGGL((k_cg_matvec<2>), dim3(nwave), dim3(256), 0, s, a, c);
    }
    hipLaunchKernelGGL(k_cg_vec, dim3(nrow), dim3(256), 0, s, a, c, 1);
    hipLaunchKernelGGL(k_cg_scalars, dim3(1), dim3(256), 0, s, c, (int)nrow, 1);
    hipLaunchKernelGGL(k_cg_vec, dim3(nrow), dim3(256), 0, s, a, c, 2);
    hipLaunchKernelGGL(k_cg_scalars, dim3(1), dim3(256), 0, s, c, (int)nrow, 2);
    hipLaunchKernelGGL(k_cg_direction, dim3(nrow), dim3(256), 0, s, a, c);
    return hipGetLastError();
}

hipError_t launch_cg_finish(const StepArgs &a, const pd_bsr_dev *K, double *work, int cur, hipStream_t s) {
    const CgArgs c = cg_args(a, K, work, cur);
    hipLaunchKernelGGL(k_cg_finish, dim3((unsigned)((a.n_pad + 255) / 256)), dim3(256), 0, s, a, c, cur);
    return hipGetLastError();
}

const double *cg_scalars(double *work, int64_t n_pad) {
    return work + 5 * 4 * n_pad + 12 * n_pad + 2 * ((n_pad + 255) / 256);
}

}  // namespace pdk
