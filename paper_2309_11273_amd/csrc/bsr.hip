// Block-sparse stiffness form of the linearized OSB-PD internal force.
//
// With g_l = theta_l / m_l = sum_k gamma_lk M_lk . (u_k - u_l),
// gamma_lk = A x_lk V_k / m_l^2 (Eqs. 1.6, 2.3), the force of Eq. 2.2 is
//   f_i = sum_j c_ij M_ij M_ij^T (u_j - u_i)                     (deviatoric)
//       + sum_j b_ij M_ij (g_i + g_j)                             (volumetric)
// with c_ij = G V_i V_j (1/m_i + 1/m_j) and b_ij = (K - G/3) x_ij V_i V_j.
// Writing every displacement difference relative to u_i gives the
// difference form f_i = sum_{q != i} Kt_iq (u_q - u_i) with 3x3 blocks
//   Kt_iq = [q in H_i] ( c_iq M M^T + gamma_iq B_i M^T - b_iq M C_q^T )
//         + sum_{j in H_i, q in H_j, q != i} b_ij gamma_jq M_ij M_jq^T
// where B_i = sum_j b_ij M_ij and C_l = sum_k gamma_lk M_lk (all sums over
// intact bonds).  This is F_int = (K^v + K^d) U of Eq. 2.14 with
// K^v = K_theta C_theta C_e and K^d = K_e C_e; the second sum is why the
// pattern reaches two bonds (2 delta).  Using differences keeps the product
// free of the rigid-motion cancellation of K u when u is large.
//
// Storage: the values of row i occupy the range [row_ptr[i], row_ptr[i+1])
// of blocks, entry (r, s) of block slot t at
// vals[row_ptr[i] * NV + (r * DIM + s) * nblk_i + t] (component-major within
// the row), so the 64 lanes of a wave that take consecutive blocks of one
// row read consecutive values for each entry.
//
// Assembly: one workgroup per row accumulates its blocks in LDS.  The
// one-bond terms touch distinct blocks; the two-bond terms are added one
// neighbour j at a time (distinct q for a fixed j, barrier between j), so
// the sums are deterministic.  After a step breaks bonds, only the rows
// within one bond of a broken bond are re-assembled.
#include <hip/hip_runtime.h>

#include <cmath>

#include "kernels.h"

namespace pdk {

struct BsrArgs {
    const int64_t *row_ptr;
    const int32_t *col;
    void *vals;
    double *bc;
    uint32_t *dirty;
    const int32_t *lat4;
    const double *vol;
    const double *inv_m;
    int32_t max_row_blocks;
    int32_t reach;
};

__device__ __forceinline__ uint64_t uni64(uint64_t v) {
    uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// per-node sums B_i, C_i (bc[8 i + 0..2] = B, bc[8 i + 4..6] = C)
template <int DIM>
__global__ __launch_bounds__(256) void k_bsr_prep(StepArgs a, BsrArgs b, int all, int par) {
    const int lane = threadIdx.x & 63;
    const int64_t slice = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (slice >= a.n_slices) return;
    if (!all && a.ctl->dirty[par] == 0) return;
    const int64_t row = slice * 64 + lane;
    const bool mine = all || b.dirty[row];
    if (!all && !__ballot(mine)) return;
    const int64_t base = a.slice_ptr[slice];
    const int64_t L = (a.slice_ptr[slice + 1] - base) >> 6;
    const pd_spec sp = a.spec[a.aux[row] >> 8];
    const double Vi = b.vol[row], ri = b.inv_m[row];
    double B[3] = {0, 0, 0}, C[3] = {0, 0, 0};
    for (int64_t k = 0; k < L; k++) {
        const uint64_t m64 = uni64(a.mask[(base >> 6) + k]);
        if (!((m64 >> lane) & 1ull)) continue;
        const uint32_t w = a.words[pd_widx(base, k, lane)];
        const int64_t j = w >> 7;
        const double *st = a.stencil + 4 * (w & 127u);
        const double x = st[3], Vj = b.vol[j];
        const double bij = sp.kp * x * Vi * Vj;
        const double gij = sp.A * x * Vj * ri * ri;
        for (int c = 0; c < DIM; c++) {
            B[c] += bij * st[c];
            C[c] += gij * st[c];
        }
    }
    if (!mine) return;
    double *o = b.bc + 8 * row;
    for (int c = 0; c < 3; c++) {
        o[c] = B[c];
        o[4 + c] = C[c];
    }
}

template <int DIM>
__device__ __forceinline__ int map_index(const int4 &d, int reach) {
    const int S = 2 * reach + 1;
    if (DIM == 3) return ((d.x + reach) * S + (d.y + reach)) * S + (d.z + reach);
    return (d.x + reach) * S + (d.y + reach);
}

// one row of the assembly, the whole workgroup (LDS smem)
template <int DIM, bool FP32V>
__device__ void assemble_row(const StepArgs &a, const BsrArgs &b, int64_t i, int all, double *smem) {
    constexpr int NV = DIM * DIM;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int64_t rp0 = b.row_ptr[i];
    const int nblk = (int)(b.row_ptr[i + 1] - rp0);
    double *acc = smem;
    double *sst = acc + (size_t)b.max_row_blocks * NV;
    short *map = reinterpret_cast<short *>(sst + 4 * 128);
    const int S = 2 * b.reach + 1;
    const int nmap = DIM == 3 ? S * S * S : S * S;
    for (int t = tid; t < nblk * NV; t += nt) acc[t] = 0.0;
    for (int t = tid; t < nmap; t += nt) map[t] = -1;
    for (int t = tid; t < 4 * 128; t += nt) sst[t] = t < 4 * a.n_stencil ? a.stencil[t] : 0.0;
    __syncthreads();
    const int4 li = reinterpret_cast<const int4 *>(b.lat4)[i];
    for (int t = tid; t < nblk; t += nt) {
        const int4 lq = reinterpret_cast<const int4 *>(b.lat4)[b.col[rp0 + t]];
        const int4 d = make_int4(lq.x - li.x, lq.y - li.y, lq.z - li.z, 0);
        map[map_index<DIM>(d, b.reach)] = (short)t;
    }
    __syncthreads();
    const pd_spec sp = a.spec[a.aux[i] >> 8];
    const double Vi = b.vol[i], ri = b.inv_m[i];
    const double *Bi = b.bc + 8 * i;
    const int64_t si = i >> 6;
    const int li_lane = (int)(i & 63);
    const int64_t base_i = a.slice_ptr[si];
    const int64_t Li = (a.slice_ptr[si + 1] - base_i) >> 6;
    // one-bond terms
    for (int64_t k = tid; k < Li; k += nt) {
        const uint32_t w = a.words[pd_widx(base_i, k, li_lane)];
        if ((w & 127u) == PD_PAD_ID) continue;
        if (!((a.mask[(base_i >> 6) + k] >> li_lane) & 1ull)) continue;
        const int64_t q = w >> 7;
        const double *st = sst + 4 * (w & 127u);
        const double x = st[3], Vq = b.vol[q], rq = b.inv_m[q];
        const double *Cq = b.bc + 8 * q + 4;
        const double c = sp.G * Vi * Vq * (ri + rq);
        const double g = sp.A * x * Vq * ri * ri;
        const double bb = sp.kp * x * Vi * Vq;
        const int4 lq = reinterpret_cast<const int4 *>(b.lat4)[q];
        const int slot = map[map_index<DIM>(make_int4(lq.x - li.x, lq.y - li.y, lq.z - li.z, 0), b.reach)];
        if (slot < 0) continue;
        double *blk = acc + (size_t)slot * NV;
        for (int r = 0; r < DIM; r++)
            for (int s = 0; s < DIM; s++)
                blk[r * DIM + s] += c * st[r] * st[s] + g * Bi[r] * st[s] - bb * st[r] * Cq[s];
    }
    __syncthreads();
    // two-bond terms, one neighbour j at a time
    for (int64_t k = 0; k < Li; k++) {
        const uint32_t w = a.words[pd_widx(base_i, k, li_lane)];
        const bool use = ((w & 127u) != PD_PAD_ID) && ((a.mask[(base_i >> 6) + k] >> li_lane) & 1ull);
        if (use) {
            const int64_t j = w >> 7;
            const double *sij = sst + 4 * (w & 127u);
            const double bij = sp.kp * sij[3] * Vi * b.vol[j];
            const double rj = b.inv_m[j];
            const int64_t sj = j >> 6;
            const int lj = (int)(j & 63);
            const int64_t base_j = a.slice_ptr[sj];
            const int64_t Lj = (a.slice_ptr[sj + 1] - base_j) >> 6;
            for (int64_t kk = tid; kk < Lj; kk += nt) {
                const uint32_t w2 = a.words[pd_widx(base_j, kk, lj)];
                if ((w2 & 127u) == PD_PAD_ID) continue;
                const int64_t q = w2 >> 7;
                if (q == i) continue;
                if (!((a.mask[(base_j >> 6) + kk] >> lj) & 1ull)) continue;
                const double *sjq = sst + 4 * (w2 & 127u);
                const double g = sp.A * sjq[3] * b.vol[q] * rj * rj;
                const int4 lq = reinterpret_cast<const int4 *>(b.lat4)[q];
                const int slot =
                    map[map_index<DIM>(make_int4(lq.x - li.x, lq.y - li.y, lq.z - li.z, 0), b.reach)];
                if (slot < 0) continue;
                double *blk = acc + (size_t)slot * NV;
                const double f = bij * g;
                for (int r = 0; r < DIM; r++)
                    for (int s = 0; s < DIM; s++) blk[r * DIM + s] += f * sij[r] * sjq[s];
            }
        }
        __syncthreads();
    }
    for (int t = tid; t < nblk * NV; t += nt) {
        // acc holds block-major entries; the row is stored component-major
        const int k = t / nblk, slot = t - k * nblk;
        const double v = acc[(size_t)slot * NV + k];
        if (FP32V) reinterpret_cast<float *>(b.vals)[(size_t)rp0 * NV + t] = (float)v;
        else reinterpret_cast<double *>(b.vals)[(size_t)rp0 * NV + t] = v;
    }
    if (!all && tid == 0) b.dirty[i] = 0u;
}

// all = 1: one workgroup per row.  all = 0 (after a step): a fixed grid
// strides over the rows and re-assembles those flagged; when no bond broke
// every workgroup returns at once.
template <int DIM, bool FP32V>
__global__ void k_bsr_assemble(StepArgs a, BsrArgs b, int all, int par) {
    extern __shared__ double smem[];
    if (all) {
        assemble_row<DIM, FP32V>(a, b, blockIdx.x, 1, smem);
        return;
    }
    if (a.ctl->dirty[par] == 0) return;
    for (int64_t i = blockIdx.x; i < a.n_pad; i += gridDim.x) {
        if (!b.dirty[i]) continue;
        assemble_row<DIM, FP32V>(a, b, i, 0, smem);
        __syncthreads();
    }
}

// pass 1 variant for the block form: breaking only, marking the rows that
// must be re-assembled (the row of a broken bond and its whole family)
template <int DIM>
__global__ __launch_bounds__(256) void k_break_mark(StepArgs a, BsrArgs b, int cur) {
    __shared__ double4 sst[128];
    for (int s = threadIdx.x; s < 128; s += blockDim.x) {
        double4 v = make_double4(0.0, 0.0, 0.0, 0.0);
        if (s < a.n_stencil)
            v = make_double4(a.stencil[4 * s], a.stencil[4 * s + 1], a.stencil[4 * s + 2], a.stencil[4 * s + 3]);
        sst[s] = v;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int64_t slice = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (slice >= a.n_slices) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.ctl->s1 = a.ctl->s2;
        a.ctl->dirty[cur ^ 1] = 0;
    }
    const int64_t row = slice * 64 + lane;
    const int64_t base = a.slice_ptr[slice];
    const int64_t L = (a.slice_ptr[slice + 1] - base) >> 6;
    const double4 *__restrict__ uv = a.uv[cur];
    const double4 ui = uv[row];
    const pd_spec sp = a.spec[a.aux[row] >> 8];
    const double s0 = sp.s0;
    const double thr_scale = s0 * (1.0 - 1e-9);
    uint32_t nbroken = 0;
    bool any = false;
    for (int64_t k = 0; k < L; k++) {
        const uint64_t m64 = uni64(a.mask[(base >> 6) + k]);
        if (m64 == 0) continue;
        const uint32_t w = a.words[pd_widx(base, k, lane)];
        const double4 st = sst[w & 127u];
        const double4 uj = uv[w >> 7];
        double e;
        {
#pragma clang fp contract(off)
            const double p1 = st.x * (uj.x - ui.x);
            const double p2 = st.y * (uj.y - ui.y);
            const double p3 = DIM == 3 ? st.z * (uj.z - ui.z) : 0.0;
            e = (p1 + p2) + p3;
        }
        bool broke = false;
        if (((m64 >> lane) & 1ull) && e >= thr_scale * st.w && e / st.w >= s0) broke = true;
        const uint64_t bb = __ballot(broke);
        if (bb) {
            if (lane == 0) a.mask[(base >> 6) + k] = m64 & ~bb;
            nbroken += __popcll(bb);
        }
        any |= broke;
    }
    if (lane == 0 && nbroken) atomicAdd(&a.ctl->broken, (unsigned long long)nbroken);
    if (any) {
        b.dirty[row] = 1u;
        for (int64_t k = 0; k < L; k++) {
            const uint32_t w = a.words[pd_widx(base, k, lane)];
            if ((w & 127u) != PD_PAD_ID) b.dirty[w >> 7] = 1u;
        }
        atomicAdd(&a.ctl->dirty[cur], 1ull);
    }
}

// f_i = sum_q Kt_iq (u_q - u_i), one wave per row; optional update
template <int DIM, bool FP32V, bool UPDATE>
__global__ __launch_bounds__(256) void k_bsr_spmv(StepArgs a, BsrArgs b, int cur) {
    constexpr int NV = DIM * DIM;
    const int lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (row >= a.n_pad) return;
    const double4 *__restrict__ uv = a.uv[cur];
    const double4 ui = uv[row];
    const int64_t rp0 = b.row_ptr[row], rp1 = b.row_ptr[row + 1];
    const int64_t nblk = rp1 - rp0;
    double f[3] = {0, 0, 0};
    float ff[3] = {0, 0, 0};
#pragma unroll 2
    for (int64_t t = lane; t < nblk; t += 64) {
        const double4 uq = uv[b.col[rp0 + t]];
        const double d[3] = {uq.x - ui.x, uq.y - ui.y, DIM == 3 ? uq.z - ui.z : 0.0};
        if (FP32V) {
            const float *K = reinterpret_cast<const float *>(b.vals) + (size_t)rp0 * NV + t;
            const float df[3] = {(float)d[0], (float)d[1], (float)d[2]};
            for (int r = 0; r < DIM; r++)
                for (int s = 0; s < DIM; s++) ff[r] += K[(r * DIM + s) * nblk] * df[s];
        } else {
            const double *K = reinterpret_cast<const double *>(b.vals) + (size_t)rp0 * NV + t;
            for (int r = 0; r < DIM; r++)
                for (int s = 0; s < DIM; s++) f[r] += K[(r * DIM + s) * nblk] * d[s];
        }
    }
    if (FP32V)
        for (int r = 0; r < 3; r++) f[r] = (double)ff[r];
    for (int o = 32; o > 0; o >>= 1)
        for (int r = 0; r < 3; r++) f[r] += __shfl_xor(f[r], o);
    if (!UPDATE) {
        if (lane == 0) a.f_out[row] = make_double4(f[0], f[1], f[2], 0.0);
        return;
    }
    const int64_t n = a.ctl->s1;
    if (blockIdx.x == 0 && threadIdx.x == 0) a.ctl->s2 = n + 1;
    bool bad = false;
    if (lane == 0) {
        const uint32_t aux = a.aux[row];
        const pd_spec sp = a.spec[aux >> 8];
        double r = 1.0;
        if (a.ramp_steps > 0) r = n >= a.ramp_steps ? 1.0 : (double)n / (double)a.ramp_steps;
        double fx = f[0], fy = f[1], fz = f[2];
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
        bad = !(isfinite(u.x) && isfinite(u.y) && isfinite(u.z));
        if (bad) atomicOr(&a.ctl->flags, PD_CTL_NONFINITE);
    }
}

static BsrArgs bsr_args(const pd_problem_dev *p, const pd_bsr_dev *K) {
    BsrArgs b{};
    b.row_ptr = K->row_ptr;
    b.col = K->col;
    b.vals = K->vals;
    b.bc = K->bc;
    b.dirty = K->dirty;
    b.lat4 = p->lat4;
    b.vol = p->vol;
    b.inv_m = p->inv_m;
    b.max_row_blocks = K->max_row_blocks;
    b.reach = K->reach;
    return b;
}

size_t bsr_assemble_lds(int dim, int max_row_blocks, int reach) {
    const int S = 2 * reach + 1;
    const size_t nmap = dim == 3 ? (size_t)S * S * S : (size_t)S * S;
    return ((size_t)max_row_blocks * dim * dim + 4 * 128) * sizeof(double) + nmap * sizeof(short);
}

hipError_t launch_bsr_prep_assemble(const StepArgs &a, const pd_problem_dev *p, const pd_bsr_dev *K, bool all,
                                    int par, hipStream_t s) {
    BsrArgs b = bsr_args(p, K);
    const int64_t nb = (a.n_slices + 3) / 4;
    if (a.dim == 3) hipLaunchKernelGGL((k_bsr_prep<3>), dim3((unsigned)nb), dim3(256), 0, s, a, b, (int)all, par);
    else hipLaunchKernelGGL((k_bsr_prep<2>), dim3((unsigned)nb), dim3(256), 0, s, a, b, (int)all, par);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t lds = bsr_assemble_lds(a.dim, K->max_row_blocks, K->reach);
    const int nt = a.dim == 3 ? 128 : 64;
    const dim3 g((unsigned)(all ? a.n_pad : std::min<int64_t>(a.n_pad, 2048)));
    if (a.dim == 3) {
        if (K->fp32) hipLaunchKernelGGL((k_bsr_assemble<3, true>), g, dim3(nt), lds, s, a, b, (int)all, par);
        else hipLaunchKernelGGL((k_bsr_assemble<3, false>), g, dim3(nt), lds, s, a, b, (int)all, par);
    } else {
        if (K->fp32) hipLaunchKernelGGL((k_bsr_assemble<2, true>), g, dim3(nt), lds, s, a, b, (int)all, par);
        else hipLaunchKernelGGL((k_bsr_assemble<2, false>), g, dim3(nt), lds, s, a, b, (int)all, par);
    }
    return hipGetLastError();
}

hipError_t set_bsr_lds_limit(int dim, bool fp32, size_t lds) {
    const void *f;
    if (dim == 3) f = fp32 ? (const void *)k_bsr_assemble<3, true> : (const void *)k_bsr_assemble<3, false>;
    else f = fp32 ? (const void *)k_bsr_assemble<2, true> : (const void *)k_bsr_assemble<2, false>;
    return hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

hipError_t launch_break_mark(const StepArgs &a, const pd_problem_dev *p, const pd_bsr_dev *K, int cur,
                             hipStream_t s) {
    BsrArgs b = bsr_args(p, K);
    const int64_t nb = (a.n_slices + 3) / 4;
    if (a.dim == 3) hipLaunchKernelGGL((k_break_mark<3>), dim3((unsigned)nb), dim3(256), 0, s, a, b, cur);
    else hipLaunchKernelGGL((k_break_mark<2>), dim3((unsigned)nb), dim3(256), 0, s, a, b, cur);
    return hipGetLastError();
}

hipError_t launch_bsr_spmv(const StepArgs &a, const pd_problem_dev *p, const pd_bsr_dev *K, int cur, bool update,
                           hipStream_t s) {
    BsrArgs b = bsr_args(p, K);
    const dim3 g((unsigned)((a.n_pad + 3) / 4));
    const dim3 blk(256);
#define PD_SPMV(D, F, U) hipLaunchKernelGGL((k_bsr_spmv<D, F, U>), g, blk, 0, s, a, b, cur)
    if (a.dim == 3) {
        if (K->fp32) { if (update) PD_SPMV(3, true, true); else PD_SPMV(3, true, false); }
        else { if (update) PD_SPMV(3, false, true); else PD_SPMV(3, false, false); }
    } else {
        if (K->fp32) { if (update) PD_SPMV(2, true, true); else PD_SPMV(2, true, false); }
        else { if (update) PD_SPMV(2, false, true); else PD_SPMV(2, false, false); }
    }
#undef PD_SPMV
    return hipGetLastError();
}

}  // namespace pdk
