// The factored matrix scheme of the linearized OSB-PD internal force.
//
// Four global operators are stored as sparse matrices and applied in the
// order of the paper's solver loop (Appendix B):
//   E     = C_e U                 C_e      N_b x dim N   (Eqs. 2.4, 2.7)
//   Theta = C_theta E             C_theta  N x N_b       (Eqs. 2.6, 2.10)
//   F     = K_theta Theta + K_e E K_theta  dim N x N,  K_e dim N x N_b
//                                                        (Eqs. 2.5, 2.8, 2.9)
// With w = 1 and M the unit vector from i to j, bond b = (i, j) gives
//   C_e row b:        -M at node i, +M at node j
//   C_theta:          A x V_j / m_i at (i, b), A x V_i / m_j at (j, b)
//   K_e column b:     g M at node i, -g M at node j, g = G V_i V_j (1/m_i + 1/m_j)
//   K_theta:          c M / m_i at (i, i) and c M / m_j at (i, j) for row i,
//                     mirrored with -M for row j, c = (K - G/3) x V_i V_j.
// Every directed entry i -> j of row i therefore carries the row-i values
// with M = M_ij, which is how the row kernels below assemble them.
//
// The dilatation product maps workgroups to slices so that each XCD works
// through a contiguous range of tiles: its own L2 then serves the E gathers
// of neighbouring rows (measured faster; the other products stream their
// operator and are not helped by it).
//
// Layout for the GPU: the bond words of the family already place the
// directed entries of 64 rows (one tile) in a slice, interleaved in groups of
// four per lane.  C_theta, K_e and K_theta use those positions as their
// storage (sliced ELL, one lane per row): lane l reads four consecutive
// values of its row per group, so the 64 lanes of a wave read contiguous
// memory.  C_e is stored bond-major (one thread per row of C_e), bonds
// numbered in the word order of their owning entry so that consecutive bonds
// sit on consecutive lanes of one slice.  Values are double, as in the paper.
//
// Breaking (Eq. 1.30) is tested on E_b / x_b as the first product computes
// it; a broken bond gets E_b = 0, which removes it from C_theta E and K_e E.
// Its contribution to K_theta does not go through E, so the K_theta rows of
// both ends are re-assembled (from the geometry and the bond status) before
// the dilatation product of the same step.
#include <hip/hip_runtime.h>

#include "factored.h"
#include "tile_common.h"

namespace pdk {

struct FacArgs {
    int64_t nb;
    int64_t nw;
    const int32_t *bond_ij;
    const int32_t *bond_pos;
    const int32_t *bid;
    double *ce;
    double *xi;
    double *cth;
    double *ke;
    double *kth;
    double *kdiag;
    double *E;
    double *theta;
    uint32_t *dirty;
    const double *vol;
    const double *inv_m;
};

static FacArgs fac_args(const pd_problem_dev *p, const pd_fac_dev *F) {
    FacArgs f{};
    f.nb = F->nb;
    f.nw = F->n_words;
    f.bond_ij = F->bond_ij;
    f.bond_pos = F->bond_pos;
    f.bid = F->bid;
    f.ce = F->ce;
    f.xi = F->xi;
    f.cth = F->cth;
    f.ke = F->ke;
    f.kth = F->kth;
    f.kdiag = F->kth_diag;
    f.E = F->E;
    f.theta = F->theta;
    f.dirty = F->dirty;
    f.vol = p->vol;
    f.inv_m = p->inv_m;
    return f;
}

// bond status word (index into the mask) and bit of the directed entry at
// word position p of row 'row'
__device__ __forceinline__ int64_t status_word(const StepArgs &a, int64_t row, int64_t p) {
    const int64_t base = a.slice_ptr[row >> 6];
    const int64_t q = p - base;
    return (base >> 6) + ((q >> 8) << 2) + (q & 3);
}

// C_e rows and bond lengths (independent of the bond status)
template <int DIM>
__global__ __launch_bounds__(256) void k_fac_bonds(StepArgs a, FacArgs f) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= f.nb) return;
    const uint32_t t = a.words[f.bond_pos[b]] & 127u;
    const double *st = a.stencil + 4 * t;
    for (int c = 0; c < DIM; c++) {
        f.ce[c * f.nb + b] = -st[c];
        f.ce[(DIM + c) * f.nb + b] = st[c];
    }
    f.xi[b] = st[3];
}

// Rows of C_theta and K_e (all = 1 only) and of K_theta, one lane per row.
// all = 0: only the rows flagged in f.dirty (K_theta only), flags cleared.
template <int DIM>
__global__ __launch_bounds__(256) void k_fac_rows(StepArgs a, FacArgs f, int all, int par) {
    const int lane = threadIdx.x & 63;
    const int64_t slice = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (slice >= a.n_slices) return;
    if (!all && a.ctl->dirty[par] == 0) return;
    const int64_t row = slice * 64 + lane;
    const bool mine = all || f.dirty[row] != 0u;
    if (!__ballot(mine)) return;
    if (!mine) return;
    const int64_t base = a.slice_ptr[slice];
    const int64_t L = (a.slice_ptr[slice + 1] - base) >> 6;
    const pd_spec sp = a.spec[a.aux[row] >> 8];
    const double Vi = f.vol[row], ri = f.inv_m[row];
    double dg[3] = {0.0, 0.0, 0.0};
    for (int64_t k = 0; k < L; k++) {
        const int64_t p = pd_widx(base, k, lane);
        const uint32_t w = a.words[p];
        if ((w & 127u) == PD_PAD_ID) {
            if (all) {
                f.cth[p] = 0.0;
                for (int c = 0; c < DIM; c++) {
                    f.ke[c * f.nw + p] = 0.0;
                    f.kth[c * f.nw + p] = 0.0;
                }
            }
            continue;
        }
        const int64_t j = w >> 7;
        const double *st = a.stencil + 4 * (w & 127u);
        const double x = st[3], Vj = f.vol[j], rj = f.inv_m[j];
        if (all) {
            f.cth[p] = sp.A * x * Vj * ri;
            const double g = sp.G * Vi * Vj * (ri + rj);
            for (int c = 0; c < DIM; c++) f.ke[c * f.nw + p] = g * st[c];
        }
        const bool intact = (a.mask[(base >> 6) + k] >> lane) & 1ull;
        const double cb = intact ? sp.kp * x * Vi * Vj : 0.0;
        for (int c = 0; c < DIM; c++) {
            f.kth[c * f.nw + p] = cb * rj * st[c];
            dg[c] += cb * ri * st[c];
        }
    }
    for (int c = 0; c < 3; c++) f.kdiag[4 * row + c] = c < DIM ? dg[c] : 0.0;
    f.kdiag[4 * row + 3] = 0.0;
    if (!all) f.dirty[row] = 0u;
}

// E = C_e U, one thread per bond (row of C_e); with BREAK the breaking test
// of Eq. 1.30 on E_b / x_b, and E_b = 0 for every broken bond.
template <int DIM, bool BREAK>
__global__ __launch_bounds__(256) void k_fac_extension(StepArgs a, FacArgs f, int cur) {
    if (BREAK && blockIdx.x == 0 && threadIdx.x == 0) {
        a.ctl->s1 = a.ctl->s2;
        a.ctl->dirty[cur ^ 1] = 0;
    }
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= f.nb) return;
    const int2 ij = reinterpret_cast<const int2 *>(f.bond_ij)[b];
    const int32_t pown = f.bond_pos[b];
    const double4 *__restrict__ uv = a.uv[cur];
    const double4 ui = uv[ij.x], uj = uv[ij.y];
    const double *ce = f.ce + b;
    const int64_t nb = f.nb;
    double e = ce[0] * ui.x;
    e += ce[nb] * ui.y;
    if (DIM == 3) e += ce[2 * nb] * ui.z;
    e += ce[DIM * nb] * uj.x;
    e += ce[(DIM + 1) * nb] * uj.y;
    if (DIM == 3) e += ce[(DIM + 2) * nb] * uj.z;
    const int64_t wi = status_word(a, ij.x, pown);
    bool intact = (a.mask[wi] >> (ij.x & 63)) & 1ull;
    if (BREAK && intact) {
        const pd_spec sp = a.spec[a.aux[ij.x] >> 8];
        if (e / f.xi[b] >= sp.s0) {
            intact = false;
            atomicAnd(reinterpret_cast<unsigned long long *>(a.mask + wi), ~(1ull << (ij.x & 63)));
            const int64_t wj = status_word(a, ij.y, f.bond_pos[nb + b]);
            atomicAnd(reinterpret_cast<unsigned long long *>(a.mask + wj), ~(1ull << (ij.y & 63)));
            f.dirty[ij.x] = 1u;
            f.dirty[ij.y] = 1u;
            atomicAdd(&a.ctl->broken, 2ull);
            atomicAdd(&a.ctl->dirty[cur], 1ull);
        }
    }
    f.E[b] = intact ? e : 0.0;
}

// Theta = C_theta E.  One workgroup of four waves per slice: wave q takes
// the groups q, q + 4, ... of all 64 rows (lane = row), and the partial sums
// are added in wave order through LDS.
__global__ __launch_bounds__(256) void k_fac_dilatation(StepArgs a, FacArgs f) {
    __shared__ double part[4][64];
    const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int64_t slice = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t row = slice * 64 + lane;
    const int64_t base = a.slice_ptr[slice];
    const int64_t G = (a.slice_ptr[slice + 1] - base) >> 8;
    const double *__restrict__ E = f.E;
    double th = 0.0;
    for (int64_t g = q; g < G; g += 4) {
        const int64_t p0 = base + (g << 8) + 4 * lane;
        const int4 b4 = *reinterpret_cast<const int4 *>(f.bid + p0);
        const double2 c01 = *reinterpret_cast<const double2 *>(f.cth + p0);
        const double2 c23 = *reinterpret_cast<const double2 *>(f.cth + p0 + 2);
        th += c01.x * E[b4.x];
        th += c01.y * E[b4.y];
        th += c23.x * E[b4.z];
        th += c23.y * E[b4.w];
    }
    part[q][lane] = th;
    __syncthreads();
    if (q != 0) return;
    th = ((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane];
    f.theta[row] = th;
    if (a.theta_out) a.theta_out[row] = th;
}

// F = K_theta Theta + K_e E, one workgroup of four waves per slice as in the
// dilatation product; UPDATE: wave 0 applies the explicit update (Eqs. 2.11,
// 2.12) instead of writing F.
template <int DIM, bool UPDATE>
__global__ __launch_bounds__(256) void k_fac_force(StepArgs a, FacArgs f, int cur) {
    __shared__ double part[4][2 * DIM][64];
    const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int64_t slice = blockIdx.x;
    const int64_t row = slice * 64 + lane;
    const int64_t base = a.slice_ptr[slice];
    const int64_t G = (a.slice_ptr[slice + 1] - base) >> 8;
    const double *__restrict__ E = f.E;
    const double *__restrict__ th = f.theta;
    double fk[DIM], fe[DIM];
    for (int c = 0; c < DIM; c++) fk[c] = fe[c] = 0.0;
    for (int64_t g = q; g < G; g += 4) {
        const int64_t p0 = base + (g << 8) + 4 * lane;
        const uint4 w4 = *reinterpret_cast<const uint4 *>(a.words + p0);
        const int4 b4 = *reinterpret_cast<const int4 *>(f.bid + p0);
        const double t[4] = {th[w4.x >> 7], th[w4.y >> 7], th[w4.z >> 7], th[w4.w >> 7]};
        const double e[4] = {E[b4.x], E[b4.y], E[b4.z], E[b4.w]};
        for (int c = 0; c < DIM; c++) {
            const double2 k01 = *reinterpret_cast<const double2 *>(f.kth + c * f.nw + p0);
            const double2 k23 = *reinterpret_cast<const double2 *>(f.kth + c * f.nw + p0 + 2);
            const double2 e01 = *reinterpret_cast<const double2 *>(f.ke + c * f.nw + p0);
            const double2 e23 = *reinterpret_cast<const double2 *>(f.ke + c * f.nw + p0 + 2);
            fk[c] += k01.x * t[0];
            fk[c] += k01.y * t[1];
            fk[c] += k23.x * t[2];
            fk[c] += k23.y * t[3];
            fe[c] += e01.x * e[0];
            fe[c] += e01.y * e[1];
            fe[c] += e23.x * e[2];
            fe[c] += e23.y * e[3];
        }
    }
    for (int c = 0; c < DIM; c++) {
        part[q][c][lane] = fk[c];
        part[q][DIM + c][lane] = fe[c];
    }
    __syncthreads();
    if (q != 0) return;
    const double thi = th[row];
    double fv[3] = {0.0, 0.0, 0.0};
    for (int c = 0; c < DIM; c++) {
        const double sk = f.kdiag[4 * row + c] * thi +
                          (((part[0][c][lane] + part[1][c][lane]) + part[2][c][lane]) + part[3][c][lane]);
        const double se = ((part[0][DIM + c][lane] + part[1][DIM + c][lane]) + part[2][DIM + c][lane]) +
                          part[3][DIM + c][lane];
        fv[c] = sk + se;
    }
    const double fx = fv[0], fy = fv[1], fz = fv[2];
    if (!UPDATE) {
        a.f_out[row] = make_double4(fx, fy, fz, 0.0);
        return;
    }
    const int64_t n = a.ctl->s1;
    if (blockIdx.x == 0 && threadIdx.x == 0) a.ctl->s2 = n + 1;
    const double4 ui = a.uv[cur][row];
    const uint32_t aux = a.aux[row];
    const pd_spec sp = a.spec[aux >> 8];
    double r = 1.0;
    if (a.ramp_steps > 0) r = n >= a.ramp_steps ? 1.0 : (double)n / (double)a.ramp_steps;
    double gx = fx, gy = fy, gz = fz;
    if (aux & 8u) {
        const double4 fx4 = a.fext[row];
        gx += fx4.x * r;
        gy += fx4.y * r;
        gz += fx4.z * r;
    }
    const double mass = sp.rho * ui.w;
    double4 v = ldv(a.vel, DIM, row);
    const double ax = (aux & 1u) ? 0.0 : gx / mass;
    const double ay = (aux & 2u) ? 0.0 : gy / mass;
    const double az = (aux & 4u) ? 0.0 : gz / mass;
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

hipError_t launch_fac_assemble(const StepArgs &a, const pd_problem_dev *p, const pd_fac_dev *F, hipStream_t s) {
    const FacArgs f = fac_args(p, F);
    if (f.nb > 0) {
        const dim3 g((unsigned)((f.nb + 255) / 256));
        if (a.dim == 3) hipLaunchKernelGGL((k_fac_bonds<3>), g, dim3(256), 0, s, a, f);
        else hipLaunchKernelGGL((k_fac_bonds<2>), g, dim3(256), 0, s, a, f);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const dim3 g((unsigned)((a.n_slices + 3) / 4));
    if (a.dim == 3) hipLaunchKernelGGL((k_fac_rows<3>), g, dim3(256), 0, s, a, f, 1, 0);
    else hipLaunchKernelGGL((k_fac_rows<2>), g, dim3(256), 0, s, a, f, 1, 0);
    return hipGetLastError();
}

hipError_t launch_fac_extension(const StepArgs &a, const pd_problem_dev *p, const pd_fac_dev *F, int cur, bool brk,
                                hipStream_t s) {
    const FacArgs f = fac_args(p, F);
    const dim3 g((unsigned)std::max<int64_t>(1, (f.nb + 255) / 256));
#define PD_EXT(D, B) hipLaunchKernelGGL((k_fac_extension<D, B>), g, dim3(256), 0, s, a, f, cur)
    if (a.dim == 3) { if (brk) PD_EXT(3, true); else PD_EXT(3, false); }
    else { if (brk) PD_EXT(2, true); else PD_EXT(2, false); }
#undef PD_EXT
    return hipGetLastError();
}

hipError_t launch_fac_kth_dirty(const StepArgs &a, const pd_problem_dev *p, const pd_fac_dev *F, int par,
                                hipStream_t s) {
    const FacArgs f = fac_args(p, F);
    const dim3 g((unsigned)((a.n_slices + 3) / 4));
    if (a.dim == 3) hipLaunchKernelGGL((k_fac_rows<3>), g, dim3(256), 0, s, a, f, 0, par);
    else hipLaunchKernelGGL((k_fac_rows<2>), g, dim3(256), 0, s, a, f, 0, par);
    return hipGetLastError();
}

hipError_t launch_fac_dilatation(const StepArgs &a, const pd_problem_dev *p, const pd_fac_dev *F, hipStream_t s) {
    const FacArgs f = fac_args(p, F);
    hipLaunchKernelGGL(k_fac_dilatation, dim3((unsigned)a.n_slices), dim3(256), 0, s, a, f);
    return hipGetLastError();
}

hipError_t launch_fac_force(const StepArgs &a, const pd_problem_dev *p, const pd_fac_dev *F, int cur, bool update,
                            hipStream_t s) {
    const FacArgs f = fac_args(p, F);
    const dim3 g((unsigned)a.n_slices);
#define PD_FRC(D, U) hipLaunchKernelGGL((k_fac_force<D, U>), g, dim3(256), 0, s, a, f, cur)
    if (a.dim == 3) { if (update) PD_FRC(3, true); else PD_FRC(3, false); }
    else { if (update) PD_FRC(2, true); else PD_FRC(2, false); }
#undef PD_FRC
    return hipGetLastError();
}

}  // namespace pdk
