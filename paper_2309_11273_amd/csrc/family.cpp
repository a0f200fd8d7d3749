// Host-side set-up of the linearized OSB-PD solver: horizon search, internal
// row order, interleaved bond words, bond-offset stencil, weighted volume and
// notch cuts.
//
// Family H_i = { j : 0 < |xi_ij| <= delta } (Sec. 2.1); bond geometry
// xi = x_j - x_i, x = |xi|, M = xi / x (Eqs. 1.2-1.5 and the linearized
// unit state below Eq. 1.13); weighted volume m_i = sum_j w x^2 V_j with
// w = 1 (Eq. 1.9).  Nodes lie on a uniform lattice, so every bond is one of
// a small set of lattice offsets: the geometry is stored once per offset
// (the "stencil") and each bond stores the neighbour row and the offset id.
#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <numeric>
#include <thread>
#include <unordered_map>
#include <vector>

#include "pd.h"
#include "pd_internal.h"

namespace {

struct Stencil {
    int32_t off[3];
    double M[3];
    double x;
};

// Bond length of lattice offset o: xi_c = dx * o_c, x = sqrt(sum xi_c^2)
// accumulated in component order.
double offset_length(double dx, const int32_t *o, double xi[3]) {
    double s = 0.0;
    for (int c = 0; c < 3; c++) {
        xi[c] = dx * (double)o[c];
        s += xi[c] * xi[c];
    }
    return std::sqrt(s);
}

// Lattice offsets of the family, shortest first; every offset is followed by
// its opposite (entry 2m+1 = -entry 2m, with exactly negated M), so that
// the tile kernels can take a bond and its mirror together and entry 0 is
// a shortest bond.
std::vector<Stencil> make_stencil(int dim, double dx, double delta) {
    std::vector<Stencil> st;
    int R = (int)std::floor(delta / dx) + 1;
    int Rz = dim == 3 ? R : 0;
    for (int a = -R; a <= R; a++)
        for (int b = -R; b <= R; b++)
            for (int c = -Rz; c <= Rz; c++) {
                int32_t o[3] = {a, b, c};
                double xi[3];
                double x = offset_length(dx, o, xi);
                if (!(x > 0.0) || !(x <= delta)) continue;
                Stencil s;
                for (int k = 0; k < 3; k++) {
                    s.off[k] = o[k];
                    s.M[k] = xi[k] / x;
                }
                s.x = x;
                st.push_back(s);
            }
    // order: |o|^2, then the pair (represented by its lexicographically
    // larger member), then the larger member first
    auto n2 = [](const Stencil &a) {
        return (int64_t)a.off[0] * a.off[0] + (int64_t)a.off[1] * a.off[1] + (int64_t)a.off[2] * a.off[2];
    };
    auto rep = [](const Stencil &a) {
        const std::array<int32_t, 3> p{a.off[0], a.off[1], a.off[2]}, m{-a.off[0], -a.off[1], -a.off[2]};
        return std::max(p, m);
    };
    std::sort(st.begin(), st.end(), [&](const Stencil &a, const Stencil &b) {
        const int64_t na = n2(a), nb = n2(b);
        if (na != nb) return na < nb;
        const auto ra = rep(a), rb = rep(b);
        if (ra != rb) return ra < rb;
        return std::array<int32_t, 3>{a.off[0], a.off[1], a.off[2]} > std::array<int32_t, 3>{b.off[0], b.off[1], b.off[2]};
    });
    return st;
}

// Lattice point -> caller node index.
struct Lookup {
    int32_t lo[3] = {0, 0, 0}, ext[3] = {1, 1, 1};
    std::vector<int32_t> dense;
    std::unordered_map<uint64_t, int32_t> sparse;
    bool use_dense = true;

    static uint64_t key(const int32_t *l) {
        return ((uint64_t)(uint32_t)(l[0] + (1 << 20)) << 42) ^
               ((uint64_t)(uint32_t)(l[1] + (1 << 20)) << 21) ^ (uint64_t)(uint32_t)(l[2] + (1 << 20));
    }
    bool build(const std::vector<int32_t> &lat, int64_t n) {
        int32_t hi[3];
        for (int c = 0; c < 3; c++) { lo[c] = INT32_MAX; hi[c] = INT32_MIN; }
        for (int64_t p = 0; p < n; p++)
            for (int c = 0; c < 3; c++) {
                lo[c] = std::min(lo[c], lat[3 * p + c]);
                hi[c] = std::max(hi[c], lat[3 * p + c]);
            }
        double vol = 1.0;
        for (int c = 0; c < 3; c++) {
            ext[c] = hi[c] - lo[c] + 1;
            vol *= (double)ext[c];
        }
        use_dense = vol <= (double)(1LL << 30) && vol <= 64.0 * (double)n + (double)(1 << 24);
        if (use_dense) {
            dense.assign((size_t)vol, -1);
            for (int64_t p = 0; p < n; p++) {
                size_t k = idx(&lat[3 * p]);
                if (dense[k] >= 0) return false;
                dense[k] = (int32_t)p;
            }
        } else {
            sparse.reserve((size_t)n * 2);
            for (int64_t p = 0; p < n; p++) {
                if (!sparse.emplace(key(&lat[3 * p]), (int32_t)p).second) return false;
            }
        }
        return true;
    }
    size_t idx(const int32_t *l) const {
        return ((size_t)(l[0] - lo[0]) * ext[1] + (size_t)(l[1] - lo[1])) * ext[2] + (size_t)(l[2] - lo[2]);
    }
    int32_t find(const int32_t *l) const {
        if (use_dense) {
            for (int c = 0; c < 3; c++)
                if (l[c] < lo[c] || l[c] >= lo[c] + ext[c]) return -1;
            return dense[idx(l)];
        }
        auto it = sparse.find(key(l));
        return it == sparse.end() ? -1 : it->second;
    }
};

// ---- notch tests (proper crossing, no ties by construction of the inputs)

double cross2(double ax, double ay, double bx, double by) { return ax * by - ay * bx; }

bool crosses_segment(const double *P, const double *Q, const double *c) {
    double d1 = cross2(c[2] - c[0], c[3] - c[1], P[0] - c[0], P[1] - c[1]);
    double d2 = cross2(c[2] - c[0], c[3] - c[1], Q[0] - c[0], Q[1] - c[1]);
    double d3 = cross2(Q[0] - P[0], Q[1] - P[1], c[0] - P[0], c[1] - P[1]);
    double d4 = cross2(Q[0] - P[0], Q[1] - P[1], c[2] - P[0], c[3] - P[1]);
    return (d1 * d2 < 0.0) && (d3 * d4 < 0.0);
}

bool crosses_parallelogram(const double *P, const double *Q, const double *p) {
    const double *c = p, *a = p + 3, *b = p + 6;
    double nrm[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
    double sp = 0, sq = 0;
    for (int k = 0; k < 3; k++) {
        sp += nrm[k] * (P[k] - c[k]);
        sq += nrm[k] * (Q[k] - c[k]);
    }
    if (!(sp * sq < 0.0)) return false;
    double t = sp / (sp - sq);
    double r[3];
    for (int k = 0; k < 3; k++) r[k] = P[k] + t * (Q[k] - P[k]) - c[k];
    double aa = 0, ab = 0, bb = 0, ra = 0, rb = 0;
    for (int k = 0; k < 3; k++) {
        aa += a[k] * a[k]; ab += a[k] * b[k]; bb += b[k] * b[k];
        ra += r[k] * a[k]; rb += r[k] * b[k];
    }
    double det = aa * bb - ab * ab;
    double s = (ra * bb - rb * ab) / det;
    double u = (rb * aa - ra * ab) / det;
    return s > 0.0 && s < 1.0 && u > 0.0 && u < 1.0;
}

double helix_level(const double *X, const double *p) { return (X[2] - p[0]) - p[1] * std::atan2(X[1], X[0]); }

bool crosses_helicoid(const double *P, const double *Q, const double *p) {
    double fp = helix_level(P, p), fq = helix_level(Q, p);
    if (!(fp * fq < 0.0)) return false;
    double t = fp / (fp - fq);
    double X[3];
    for (int k = 0; k < 3; k++) X[k] = P[k] + t * (Q[k] - P[k]);
    double r = std::sqrt(X[0] * X[0] + X[1] * X[1]);
    double th = std::atan2(X[1], X[0]);
    return r > p[2] && r < p[3] && th > p[4] && th < p[5];
}

template <class F>
void parallel_for(int64_t n, F &&f) {
    unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    if (n < 4096 || nt == 1) {
        f(0, n);
        return;
    }
    std::vector<std::thread> th;
    int64_t chunk = (n + nt - 1) / nt;
    for (unsigned t = 0; t < nt; t++) {
        int64_t a = t * chunk, b = std::min(n, a + chunk);
        if (a >= b) break;
        th.emplace_back([&, a, b] { f(a, b); });
    }
    for (auto &x : th) x.join();
}

}  // namespace

extern "C" pd_status pd_build_family(const pd_body *body, const pd_cut *cuts, int32_t ncuts,
                                     pd_family_sizes *sizes, pd_family_host *out) {
    if (!body || !sizes || !body->lat || !body->vol) return PD_ERR_ARG;
    const int64_t n = body->n;
    const int dim = body->dim;
    if (n < 1 || n > PD_MAX_NODES) return PD_ERR_SIZE;
    if (dim != 2 && dim != 3) return PD_ERR_ARG;
    if (!(body->dx > 0.0) || !(body->delta > 0.0) || !std::isfinite(body->delta)) return PD_ERR_ARG;
    if (ncuts < 0 || ncuts > PD_MAX_CUTS || (ncuts > 0 && !cuts)) return PD_ERR_ARG;
    for (int k = 0; k < ncuts; k++)
        if (cuts[k].kind < 0 || cuts[k].kind > 2 || (cuts[k].kind != 0 && dim == 2) ||
            (cuts[k].kind == 0 && dim == 3))
            return PD_ERR_ARG;

    std::vector<int32_t> lat((size_t)3 * n, 0);
    std::vector<int32_t> spec((size_t)n, 0);
    int32_t nspec = 1;
    for (int64_t p = 0; p < n; p++) {
        for (int c = 0; c < dim; c++) lat[3 * p + c] = body->lat[dim * p + c];
        if (!(body->vol[p] > 0.0)) return PD_ERR_ARG;
        if (body->specimen) {
            int32_t s = body->specimen[p];
            if (s < 0 || s >= PD_MAX_SPECIMENS) return PD_ERR_ARG;
            spec[p] = s;
            nspec = std::max(nspec, s + 1);
        }
    }
    std::vector<Stencil> st = make_stencil(dim, body->dx, body->delta);
    if ((int)st.size() > PD_MAX_STENCIL) return PD_ERR_SIZE;
    if (st.empty()) return PD_ERR_ARG;

    Lookup look;
    if (!look.build(lat, n)) return PD_ERR_ARG;  // duplicate lattice point

    // ---- tiles of 64 lattice points, per specimen --------------------------
    std::vector<int32_t> slo((size_t)3 * nspec, INT32_MAX), shi((size_t)3 * nspec, INT32_MIN);
    for (int64_t p = 0; p < n; p++)
        for (int c = 0; c < 3; c++) {
            slo[3 * spec[p] + c] = std::min(slo[3 * spec[p] + c], lat[3 * p + c]);
            shi[3 * spec[p] + c] = std::max(shi[3 * spec[p] + c], lat[3 * p + c]);
        }
    for (int s = 0; s < nspec; s++)
        for (int c = 0; c < 3; c++)
            if (slo[3 * s + c] != INT32_MAX && (int64_t)shi[3 * s + c] - slo[3 * s + c] >= (1 << 20))
                return PD_ERR_SIZE;
    auto tile_key = [&](int64_t p, const int *T, int32_t *t, int32_t *r) {
        for (int c = 0; c < 3; c++) {
            const int32_t rel = lat[3 * p + c] - slo[3 * spec[p] + c];
            t[c] = rel / T[c];
            r[c] = rel - t[c] * T[c];
        }
        return ((uint64_t)spec[p] << 48) | ((uint64_t)t[2] << 32) | ((uint64_t)t[1] << 16) | (uint64_t)t[0];
    };
    static const int shapes3[][3] = {{4, 4, 4}, {8, 4, 2}, {8, 8, 1}, {16, 4, 1}};
    static const int shapes2[][3] = {{8, 8, 1}, {16, 4, 1}, {32, 2, 1}};
    const int nshape = dim == 3 ? 4 : 3;
    int T[3] = {0, 0, 0};
    std::vector<uint64_t> tkeys;
    int reach = 0;
    for (const Stencil &sv : st)
        for (int c = 0; c < dim; c++) reach = std::max(reach, std::abs(sv.off[c]));
    {
        size_t best = SIZE_MAX;
        std::vector<uint64_t> keys((size_t)n);
        for (int k = 0; k < 2 * nshape; k++) {
            // first pass: shapes whose every edge is at least the largest
            // stencil offset component (a tile's family then lies in its
            // 3^dim neighbour tiles); second pass only if none qualifies
            if (k == nshape && best != SIZE_MAX) break;
            const int *Tk = dim == 3 ? shapes3[k % nshape] : shapes2[k % nshape];
            bool fits = true;
            if (k < nshape)
                for (int c = 0; c < dim; c++)
                    if (Tk[c] < reach) fits = false;
            // tiles per axis must fit in 16 bits
            for (int s = 0; s < nspec && fits; s++)
                for (int c = 0; c < 3; c++)
                    if (slo[3 * s + c] != INT32_MAX && (shi[3 * s + c] - slo[3 * s + c]) / Tk[c] >= 65535) fits = false;
            if (!fits) continue;
            parallel_for(n, [&](int64_t a, int64_t b) {
                int32_t t[3], r[3];
                for (int64_t p = a; p < b; p++) keys[p] = tile_key(p, Tk, t, r);
            });
            std::vector<uint64_t> u = keys;
            std::sort(u.begin(), u.end());
            u.erase(std::unique(u.begin(), u.end()), u.end());
            if (u.size() < best) {
                best = u.size();
                for (int c = 0; c < 3; c++) T[c] = Tk[c];
                tkeys.swap(u);
            }
        }
        if (best == SIZE_MAX) return PD_ERR_SIZE;
    }
    const int64_t n_tiles = (int64_t)tkeys.size();
    const int64_t n_pad = n_tiles * 64;
    const int64_t n_slices = n_tiles;
    if (n_pad >= PD_MAX_NODES) return PD_ERR_SIZE;
    std::vector<int64_t> node_of_row((size_t)n_pad, -1);
    std::vector<int32_t> row_of((size_t)n);
    parallel_for(n, [&](int64_t a, int64_t b) {
        int32_t t[3], r[3];
        for (int64_t p = a; p < b; p++) {
            const uint64_t key = tile_key(p, T, t, r);
            const int64_t tid = std::lower_bound(tkeys.begin(), tkeys.end(), key) - tkeys.begin();
            const int64_t row = tid * 64 + r[0] + T[0] * (r[1] + T[1] * r[2]);
            row_of[p] = (int32_t)row;
            node_of_row[row] = p;
        }
    });

    // ---- per row: neighbours in stencil order, weighted volume, notch cuts ---
    const int ns = (int)st.size();
    const int L4 = (ns + 3) / 4 * 4;
    std::vector<double> m((size_t)n_pad, 0.0);
    std::vector<uint64_t> cutbits((size_t)n_pad * 2, 0);  // one bit per stencil entry (<= 127)
    std::vector<int32_t> deg((size_t)n_pad, 0), ncutr((size_t)n_pad, 0);
    auto pos = [&](int64_t p, double *X) {
        for (int c = 0; c < 3; c++) X[c] = body->origin[c] + body->dx * (double)lat[3 * p + c];
    };
    auto neighbour = [&](int64_t p, int s) -> int64_t {
        int32_t q[3];
        for (int c = 0; c < 3; c++) q[c] = lat[3 * p + c] + st[s].off[c];
        const int32_t qi = look.find(q);
        return (qi < 0 || spec[qi] != spec[p]) ? -1 : qi;
    };
    parallel_for(n_pad, [&](int64_t a, int64_t b) {
        for (int64_t r = a; r < b; r++) {
            const int64_t p = node_of_row[r];
            if (p < 0) continue;
            double msum = 0.0;
            for (int s = 0; s < ns; s++) {
                const int64_t q = neighbour(p, s);
                if (q < 0) continue;
                deg[r]++;
                msum += st[s].x * st[s].x * body->vol[q];
                if (ncuts > 0) {
                    const int64_t lo = std::min(p, q), hi = std::max(p, q);
                    double P[3], Q[3];
                    pos(lo, P);
                    pos(hi, Q);
                    for (int c = 0; c < ncuts; c++) {
                        if (cuts[c].specimen >= 0 && spec[p] != cuts[c].specimen) continue;
                        bool hit;
                        if (cuts[c].kind == 0) hit = crosses_segment(P, Q, cuts[c].p);
                        else if (cuts[c].kind == 1) hit = crosses_parallelogram(P, Q, cuts[c].p);
                        else hit = crosses_helicoid(P, Q, cuts[c].p);
                        if (hit) {
                            cutbits[2 * r + (s >> 6)] |= 1ull << (s & 63);
                            ncutr[r]++;
                            break;
                        }
                    }
                }
            }
            m[r] = msum;
        }
    });
    int32_t max_row = 0;
    int64_t nnz = 0, ncut_dir = 0;
    for (int64_t r = 0; r < n_pad; r++) {
        nnz += deg[r];
        ncut_dir += ncutr[r];
        max_row = std::max(max_row, deg[r]);
    }
    const int64_t n_words = n_pad * L4;

    sizes->n = n;
    sizes->n_pad = n_pad;
    sizes->n_slices = n_slices;
    sizes->n_words = n_words;
    sizes->n_mask = n_words / 64;
    sizes->nnz = nnz;
    sizes->n_bonds = nnz / 2;
    sizes->n_cut = ncut_dir / 2;
    sizes->n_stencil = ns;
    sizes->max_row = max_row;
    sizes->dim = dim;
    sizes->n_specimens = nspec;
    sizes->n_tiles = n_tiles;
    for (int c = 0; c < 3; c++) sizes->tile[c] = T[c];
    sizes->words_per_row = L4;
    sizes->reach = reach;
    // one volume for every node: the FP32 tile kernels then take it as a
    // constant (compared as the float the shadow carries)
    {
        bool same = n > 0;
        for (int64_t p = 1; p < n && same; p++) same = (float)body->vol[p] == (float)body->vol[0];
        sizes->vol_uniform = same ? (float)body->vol[0] : 0.0f;
        sizes->pad_vu = 0;
    }
    {
        int32_t B[4];
        pd_tile_box(T, reach, dim, B);
        sizes->n_halo = B[3] * B[2];
    }
    // points of the box that some stencil entry of some tile point reaches (the
    // corners of the box beyond the horizon are never read)
    std::vector<uint8_t> reached(pd_box_points(T, reach, dim), 0);
    {
        const int32_t e0 = T[0] + 2 * reach, e1 = T[1] + 2 * reach;
        for (int s = 0; s < ns; s++)
            for (int32_t l = 0; l < T[0] * T[1] * T[2]; l++) {
                const int32_t q[3] = {l % T[0] + st[s].off[0] + reach, (l / T[0]) % T[1] + st[s].off[1] + reach,
                                      dim == 3 ? l / (T[0] * T[1]) + st[s].off[2] + reach : 0};
                reached[q[0] + e0 * (q[1] + e1 * q[2])] = 1;
            }
        for (int32_t l = 0; l < T[0] * T[1] * T[2]; l++) {  // the tile's own points
            const int32_t q[3] = {l % T[0] + reach, (l / T[0]) % T[1] + reach, dim == 3 ? l / (T[0] * T[1]) + reach : 0};
            reached[q[0] + e0 * (q[1] + e1 * q[2])] = 1;
        }
        int32_t nr = 0;
        for (uint8_t r : reached) nr += r;
        sizes->n_box = nr;
    }
    if (!out) return PD_OK;
    if (!out->perm || !out->row_of || !out->slice_ptr || !out->words || !out->mask || !out->stencil ||
        !out->stencil_off || !out->vol || !out->inv_m || !out->spec || !out->lat4 || !out->tile_org ||
        !out->tile_nbr || !out->ktab || !out->halo_map || !out->halo_pos)
        return PD_ERR_ARG;

    for (int64_t r = 0; r < n_pad; r++) out->perm[r] = (int32_t)node_of_row[r];
    for (int64_t p = 0; p < n; p++) out->row_of[p] = row_of[p];
    for (int64_t s = 0; s <= n_slices; s++) out->slice_ptr[s] = s * 64 * L4;
    int32_t box[4];
    pd_tile_box(T, reach, dim, box);
    for (int32_t s = 0; s < box[3] * box[2]; s++) {
        const int32_t b[3] = {(s % box[3]) % box[0], (s % box[3]) / box[0], s / box[3]};
        int32_t p[3], d[3];
        for (int c = 0; c < 3; c++) {
            p[c] = (c < dim) ? b[c] - reach : 0;
            d[c] = p[c] < 0 ? -1 : (p[c] >= T[c] ? 1 : 0);
        }
        if (p[0] >= T[0] + reach || p[1] >= T[1] + reach) {
            out->halo_map[s] = -1;  // pitch padding
            continue;
        }
        const int32_t dir = (d[2] + 1) * 9 + (d[1] + 1) * 3 + (d[0] + 1);
        const int32_t loc = (p[0] - d[0] * T[0]) + T[0] * ((p[1] - d[1] * T[1]) + T[1] * (p[2] - d[2] * T[2]));
        out->halo_map[s] = (int16_t)(64 * dir + loc);
    }
    // the unpadded box point by point, with its slot in the pass-1 box
    int32_t box1[4];
    pd_tile_box1(T, reach, dim, box1);
    {
        const int32_t e0 = T[0] + 2 * reach, e1 = T[1] + 2 * reach;
        const int32_t nb = pd_box_points(T, reach, dim);
        int32_t np = 0;
        for (int32_t b = 0; b < nb; b++) {
            if (!reached[b]) continue;
            const int32_t bx = b % e0, by = (b / e0) % e1, bz = b / (e0 * e1);
            const int32_t p[3] = {bx - reach, by - reach, dim == 3 ? bz - reach : 0};
            int32_t d[3];
            for (int c = 0; c < 3; c++) d[c] = p[c] < 0 ? -1 : (p[c] >= T[c] ? 1 : 0);
            const int32_t dir = (d[2] + 1) * 9 + (d[1] + 1) * 3 + (d[0] + 1);
            const int32_t loc = (p[0] - d[0] * T[0]) + T[0] * ((p[1] - d[1] * T[1]) + T[1] * (p[2] - d[2] * T[2]));
            const int32_t slot = bx + box1[0] * by + box1[3] * bz;
            out->halo_pos[np++] = (slot << 11) | (64 * dir + loc);
        }
    }
    for (int q = 0; q < 20 * 128; q++) out->ktab[q] = 0u;
    auto fbits = [](double v) {
        const float f = (float)v;
        uint32_t b;
        std::memcpy(&b, &f, 4);
        return b;
    };
    for (int s = 0; s < ns; s++) {
        for (int c = 0; c < 3; c++) {
            out->stencil[4 * s + c] = st[s].M[c];
            out->ktab[8 * s + c] = fbits(st[s].M[c]);
            out->stencil_off[3 * s + c] = st[s].off[c];
        }
        out->stencil[4 * s + 3] = st[s].x;
        out->ktab[8 * s + 3] = fbits(st[s].x);
        const int32_t so = st[s].off[0] + box[0] * st[s].off[1] + box[3] * st[s].off[2];
        out->ktab[8 * s + 4] = (uint32_t)so;
        out->ktab[8 * s + 5] = fbits(1.0 / st[s].x);
        for (int c = 0; c < 3; c++) out->ktab[1024 + 4 * s + c] = fbits(st[s].x * st[s].M[c]);
        out->ktab[1024 + 4 * s + 3] = (uint32_t)so;
        uint32_t *k1 = out->ktab + 1536 + 8 * s;
        k1[0] = fbits(st[s].M[0] / st[s].x);
        k1[1] = fbits(st[s].M[1] / st[s].x);
        k1[2] = fbits(st[s].x * st[s].x);
        k1[3] = fbits(st[s].x * st[s].M[0]);
        k1[4] = fbits(st[s].x * st[s].M[1]);
        k1[5] = (uint32_t)(st[s].off[0] + box1[0] * st[s].off[1] + box1[3] * st[s].off[2]);
        k1[6] = fbits(st[s].M[2] / st[s].x);
        k1[7] = fbits(st[s].x * st[s].M[2]);
    }
    parallel_for(n_slices, [&](int64_t a, int64_t b) {
        for (int64_t sl = a; sl < b; sl++) {
            const int64_t base = sl * 64 * L4;
            for (int k = 0; k < L4; k++) {
                uint64_t bits = 0;
                for (int lane = 0; lane < 64; lane++) {
                    const int64_t r = 64 * sl + lane;
                    const int64_t p = node_of_row[r];
                    uint32_t w = ((uint32_t)r << 7) | 127u;
                    if (p >= 0 && k < ns) {
                        const int64_t q = neighbour(p, k);
                        if (q >= 0) {
                            w = ((uint32_t)row_of[q] << 7) | (uint32_t)k;
                            if (!((cutbits[2 * r + (k >> 6)] >> (k & 63)) & 1ull)) bits |= 1ull << lane;
                        }
                    }
                    out->words[pd_widx(base, k, lane)] = w;
                }
                out->mask[base / 64 + k] = bits;
            }
        }
    });
    for (int64_t r = 0; r < n_pad; r++) {
        const int64_t p = node_of_row[r];
        const bool real = p >= 0;
        out->vol[r] = real ? body->vol[p] : 0.0;
        out->inv_m[r] = (real && m[r] > 0.0) ? 1.0 / m[r] : 0.0;
        out->spec[r] = real ? spec[p] : 0;
        for (int c = 0; c < 3; c++) out->lat4[4 * r + c] = real ? lat[3 * p + c] : 0;
        out->lat4[4 * r + 3] = 0;
    }
    for (int64_t t = 0; t < n_tiles; t++) {
        const uint64_t key = tkeys[t];
        const int32_t sp = (int32_t)(key >> 48);
        const int32_t tc[3] = {(int32_t)(key & 0xffff), (int32_t)((key >> 16) & 0xffff), (int32_t)((key >> 32) & 0xffff)};
        for (int c = 0; c < 3; c++) out->tile_org[4 * t + c] = slo[3 * sp + c] + tc[c] * T[c];
        out->tile_org[4 * t + 3] = sp;
        for (int dz = -1; dz <= 1; dz++)
            for (int dy = -1; dy <= 1; dy++)
                for (int dx = -1; dx <= 1; dx++) {
                    const int32_t q[3] = {tc[0] + dx, tc[1] + dy, tc[2] + dz};
                    int32_t id = -1;
                    if (q[0] >= 0 && q[1] >= 0 && q[2] >= 0) {
                        const uint64_t k2 = ((uint64_t)sp << 48) | ((uint64_t)q[2] << 32) | ((uint64_t)q[1] << 16) |
                                            (uint64_t)q[0];
                        auto it = std::lower_bound(tkeys.begin(), tkeys.end(), k2);
                        if (it != tkeys.end() && *it == k2) id = (int32_t)(it - tkeys.begin());
                    }
                    out->tile_nbr[27 * t + (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)] = id;
                }
    }
    return PD_OK;
}

// Block pattern of the stiffness: q is in row i iff q != i and q is a
// neighbour of i or a neighbour of a neighbour of i (rows of real nodes).
extern "C" pd_status pd_bsr_pattern(const pd_family_sizes *sz, const pd_family_host *fam, pd_bsr_sizes *out,
                                    int64_t *row_ptr, int32_t *col) {
    if (!sz || !fam || !out || !fam->slice_ptr || !fam->words || !fam->lat4) return PD_ERR_ARG;
    const int64_t n_pad = sz->n_pad;
    std::vector<std::vector<int32_t>> rows((size_t)n_pad);
    auto row_len = [&](int64_t r) { return (fam->slice_ptr[r / 64 + 1] - fam->slice_ptr[r / 64]) / 64; };
    auto word = [&](int64_t r, int64_t k) { return fam->words[pd_widx(fam->slice_ptr[r / 64], k, (int)(r % 64))]; };
    std::vector<int32_t> reach_rows((size_t)n_pad, 0);
    parallel_for(n_pad, [&](int64_t a, int64_t b) {
        std::vector<int32_t> tmp;
        for (int64_t r = a; r < b; r++) {
            tmp.clear();
            int64_t L = row_len(r);
            for (int64_t k = 0; k < L; k++) {
                uint32_t w = word(r, k);
                if ((w & 127u) == 127u) continue;
                int32_t j = (int32_t)(w >> 7);
                tmp.push_back(j);
                int64_t Lj = row_len(j);
                for (int64_t kk = 0; kk < Lj; kk++) {
                    uint32_t w2 = word(j, kk);
                    if ((w2 & 127u) == 127u) continue;
                    int32_t q = (int32_t)(w2 >> 7);
                    if (q != r) tmp.push_back(q);
                }
            }
            std::sort(tmp.begin(), tmp.end());
            tmp.erase(std::unique(tmp.begin(), tmp.end()), tmp.end());
            int32_t rc = 0;
            for (int32_t q : tmp)
                for (int c = 0; c < 3; c++)
                    rc = std::max(rc, std::abs(fam->lat4[4 * (int64_t)q + c] - fam->lat4[4 * r + c]));
            reach_rows[r] = rc;
            rows[r] = tmp;
        }
    });
    int64_t total = 0;
    int32_t mx = 0, reach = 0;
    for (int64_t r = 0; r < n_pad; r++) {
        total += (int64_t)rows[r].size();
        mx = std::max(mx, (int32_t)rows[r].size());
        reach = std::max(reach, reach_rows[r]);
    }
    out->nnzb = total;
    out->max_row_blocks = mx;
    out->reach = reach;
    if (!col) return PD_OK;
    if (!row_ptr) return PD_ERR_ARG;
    row_ptr[0] = 0;
    for (int64_t r = 0; r < n_pad; r++) row_ptr[r + 1] = row_ptr[r] + (int64_t)rows[r].size();
    parallel_for(n_pad, [&](int64_t a, int64_t b) {
        for (int64_t r = a; r < b; r++)
            if (!rows[r].empty())  // padding rows have no blocks (and no data pointer)
                std::memcpy(col + row_ptr[r], rows[r].data(), sizeof(int32_t) * rows[r].size());
    });
    return PD_OK;
}

// Bond numbering of the factored scheme.  Bond k of a row is stencil entry
// k, so the reverse of entry k of row i is entry rev[k] of row j; the entry
// with the smaller stencil id owns the bond.  Owners are numbered in word
// order, slice by slice, so that consecutive bonds sit on consecutive lanes.
extern "C" pd_status pd_fac_pattern(const pd_family_sizes *sz, const pd_family_host *fam, pd_fac_sizes *out,
                                    int32_t *bond_ij, int32_t *bond_pos, int32_t *bid) {
    if (!sz || !fam || !out || !fam->slice_ptr || !fam->words || !fam->stencil_off) return PD_ERR_ARG;
    if (sz->n_words >= ((int64_t)1 << 31)) return PD_ERR_SIZE;
    const int ns = sz->n_stencil;
    const int64_t n_slices = sz->n_slices;
    std::vector<int32_t> rev((size_t)ns, -1);
    for (int a = 0; a < ns; a++)
        for (int b = 0; b < ns; b++) {
            const int32_t *oa = fam->stencil_off + 3 * a, *ob = fam->stencil_off + 3 * b;
            if (oa[0] == -ob[0] && oa[1] == -ob[1] && oa[2] == -ob[2]) rev[a] = b;
        }
    for (int a = 0; a < ns; a++)
        if (rev[a] < 0 || rev[a] == a) return PD_ERR_ARG;
    auto owner = [&](uint32_t w) { return (w & 127u) != 127u && (int)(w & 127u) < rev[w & 127u]; };
    std::vector<int64_t> first((size_t)n_slices + 1, 0);
    parallel_for(n_slices, [&](int64_t a, int64_t b) {
        for (int64_t sl = a; sl < b; sl++) {
            int64_t c = 0;
            for (int64_t p = fam->slice_ptr[sl]; p < fam->slice_ptr[sl + 1]; p++) c += owner(fam->words[p]);
            first[sl + 1] = c;
        }
    });
    for (int64_t sl = 0; sl < n_slices; sl++) first[sl + 1] += first[sl];
    out->nb = first[n_slices];
    out->n_words = sz->n_words;
    if (!bond_ij) return PD_OK;
    if (!bond_pos || !bid) return PD_ERR_ARG;
    auto pos_of = [&](int64_t row, int k) { return pd_widx(fam->slice_ptr[row / 64], k, (int)(row % 64)); };
    std::atomic<bool> asym{false};
    parallel_for(n_slices, [&](int64_t a, int64_t b) {
        for (int64_t sl = a; sl < b; sl++) {
            int64_t nb = first[sl];
            const int64_t base = fam->slice_ptr[sl];
            for (int64_t p = base; p < fam->slice_ptr[sl + 1]; p++) {
                const uint32_t w = fam->words[p];
                if (!owner(w)) continue;
                const int64_t q = p - base;
                const int64_t row = 64 * sl + ((q & 255) >> 2);
                const int64_t j = w >> 7;
                const int64_t pr = pos_of(j, rev[w & 127u]);
                if (fam->words[pr] != (((uint32_t)row << 7) | (uint32_t)rev[w & 127u])) asym = true;
                bond_ij[2 * nb] = (int32_t)row;
                bond_ij[2 * nb + 1] = (int32_t)j;
                bond_pos[nb] = (int32_t)p;
                bond_pos[out->nb + nb] = (int32_t)pr;
                bid[p] = (int32_t)nb;
                nb++;
            }
        }
    });
    if (asym) return PD_ERR_ARG;
    parallel_for(n_slices, [&](int64_t a, int64_t b) {
        for (int64_t sl = a; sl < b; sl++) {
            const int64_t base = fam->slice_ptr[sl];
            for (int64_t p = base; p < fam->slice_ptr[sl + 1]; p++) {
                const uint32_t w = fam->words[p];
                if ((w & 127u) == 127u) bid[p] = 0;
                else if (!owner(w)) bid[p] = bid[pos_of(w >> 7, rev[w & 127u])];
            }
        }
    });
    return PD_OK;
}

// Super-tiles: 2 x 2 (x 1) groups of tiles sharing one halo box -- 4x4x4
// tiles in 3D (box pitches 16 and 228), 8x8 tiles in 2D (x pitch 40).  The
// tile coordinates follow from the tile origins: per specimen the smallest
// origin is the tile grid's origin.
extern "C" pd_status pd_build_supertiles(const pd_family_sizes *sz, const pd_family_host *fam, pd_st_sizes *out,
                                         int32_t *st_tiles, int32_t *st_nbr, int32_t *st_pos, uint32_t *st_ktab) {
    if (!sz || !fam || !out || !fam->tile_org || !fam->stencil || !fam->stencil_off) return PD_ERR_ARG;
    const int dim = sz->dim;
    const bool ok3 = dim == 3 && sz->tile[0] == 4 && sz->tile[1] == 4 && sz->tile[2] == 4;
    const bool ok2 = dim == 2 && sz->tile[0] == 8 && sz->tile[1] == 8 && sz->tile[2] == 1;
    if (!(ok3 || ok2) || sz->reach < 1 || sz->reach > 3 || sz->n_stencil < 1 || sz->n_stencil > 124)
        return PD_ERR_UNSUPPORTED;
    const int64_t nt = sz->n_tiles;
    const int R = sz->reach;
    const int ns = sz->n_stencil;
    const int T = sz->tile[0];              // tile edge in x and y (4 in 3D, 8 in 2D)
    const int TZ = dim == 3 ? 4 : 1;
    const int P0 = dim == 3 ? 16 : 40;     // box pitches (x extent 2T + 2R <= 22)
    const int P1 = dim == 3 ? 228 : 0;
    // tile coordinates per specimen
    std::unordered_map<int32_t, std::array<int32_t, 3>> lo;
    for (int64_t t = 0; t < nt; t++) {
        const int32_t sp = fam->tile_org[4 * t + 3];
        auto it = lo.find(sp);
        if (it == lo.end()) {
            lo[sp] = {fam->tile_org[4 * t], fam->tile_org[4 * t + 1], fam->tile_org[4 * t + 2]};
        } else {
            for (int c = 0; c < 3; c++) it->second[c] = std::min(it->second[c], fam->tile_org[4 * t + c]);
        }
    }
    auto tkey = [](int64_t sp, int64_t x, int64_t y, int64_t z) {
        return (uint64_t)((sp << 48) | ((z + 1) << 32) | ((y + 1) << 16) | (x + 1));
    };
    std::unordered_map<uint64_t, int32_t> tile_at;
    std::vector<uint64_t> skeys;
    tile_at.reserve((size_t)nt * 2);
    for (int64_t t = 0; t < nt; t++) {
        const int32_t sp = fam->tile_org[4 * t + 3];
        const auto &l = lo[sp];
        const int32_t tc[3] = {(fam->tile_org[4 * t] - l[0]) / T, (fam->tile_org[4 * t + 1] - l[1]) / T,
                               (fam->tile_org[4 * t + 2] - l[2]) / TZ};
        tile_at[tkey(sp, tc[0], tc[1], tc[2])] = (int32_t)t;
        skeys.push_back(((uint64_t)sp << 48) | ((uint64_t)tc[2] << 32) | ((uint64_t)(tc[1] >> 1) << 16) |
                        (uint64_t)(tc[0] >> 1));
    }
    std::sort(skeys.begin(), skeys.end());
    skeys.erase(std::unique(skeys.begin(), skeys.end()), skeys.end());
    // reached points of the box (2T + 2R) x (2T + 2R) x (TZ + 2R in 3D)
    const int e0 = 2 * T + 2 * R, e1 = 2 * T + 2 * R, e2 = dim == 3 ? TZ + 2 * R : 1;
    std::vector<uint8_t> reached((size_t)e0 * e1 * e2, 0);
    for (int q = 0; q < 4; q++)
        for (int l = 0; l < 64; l++)
            for (int s = -1; s < ns; s++) {
                int32_t o[3] = {0, 0, 0};
                if (s >= 0)
                    for (int c = 0; c < dim; c++) o[c] = fam->stencil_off[3 * s + c];
                const int bx = T * (q & 1) + (l % T) + o[0] + R, by = T * (q >> 1) + (l / T) % T + o[1] + R,
                          bz = dim == 3 ? l / (T * T) + o[2] + R : 0;
                if (bx < 0 || by < 0 || bz < 0 || bx >= e0 || by >= e1 || bz >= e2) return PD_ERR_UNSUPPORTED;
                reached[bx + e0 * (by + e1 * bz)] = 1;
            }
    int32_t npos = 0;
    for (uint8_t r : reached) npos += r;
    out->n_st = (int64_t)skeys.size();
    out->n_pos = npos;
    out->pad0 = 0;
    if (!st_tiles) return PD_OK;
    if (!st_nbr || !st_pos || !st_ktab) return PD_ERR_ARG;
    for (size_t s = 0; s < skeys.size(); s++) {
        const int64_t sp = (int64_t)(skeys[s] >> 48), z = (int64_t)((skeys[s] >> 32) & 0xffff),
                      sy = (int64_t)((skeys[s] >> 16) & 0xffff), sx = (int64_t)(skeys[s] & 0xffff);
        auto find = [&](int64_t x, int64_t y, int64_t zz) -> int32_t {
            if (x < 0 || y < 0 || zz < 0) return -1;
            auto it = tile_at.find(tkey(sp, x, y, zz));
            return it == tile_at.end() ? -1 : it->second;
        };
        for (int q = 0; q < 4; q++) st_tiles[4 * s + q] = find(2 * sx + (q & 1), 2 * sy + (q >> 1), z);
        for (int dz = 0; dz < 3; dz++)
            for (int dy = 0; dy < 4; dy++)
                for (int dx = 0; dx < 4; dx++)
                    st_nbr[48 * s + dx + 4 * dy + 16 * dz] =
                        (dim == 2 && dz != 1) ? -1 : find(2 * sx - 1 + dx, 2 * sy - 1 + dy, z - 1 + dz);
    }
    int32_t np = 0;
    for (int bz = 0; bz < e2; bz++)
        for (int by = 0; by < e1; by++)
            for (int bx = 0; bx < e0; bx++) {
                if (!reached[bx + e0 * (by + e1 * bz)]) continue;
                const int p[3] = {bx - R, by - R, dim == 3 ? bz - R : 0};
                const int Tc[3] = {T, T, TZ};
                int d[3], l[3];
                for (int c = 0; c < 3; c++) {
                    d[c] = (p[c] + Tc[c]) / Tc[c];  // tile offset + 1 (p >= -R >= -T)
                    l[c] = p[c] - Tc[c] * (d[c] - 1);
                }
                const int32_t slot = bx + P0 * by + P1 * bz;
                st_pos[np++] = (slot << 12) | (64 * (d[0] + 4 * d[1] + 16 * d[2]) + l[0] + T * (l[1] + T * l[2]));
            }
    auto fbits = [](double v) {
        const float f = (float)v;
        uint32_t b;
        std::memcpy(&b, &f, 4);
        return b;
    };
    for (int q = 0; q < 128 * 8; q++) st_ktab[q] = 0u;
    for (int s = 0; s < ns; s++) {
        const double *S = fam->stencil + 4 * s;  // M1, M2, M3, x
        const int32_t *o = fam->stencil_off + 3 * s;
        uint32_t *k1 = st_ktab + 8 * s;
        k1[0] = fbits(S[0] / S[3]);
        k1[1] = fbits(S[1] / S[3]);
        k1[2] = fbits(S[3] * S[3]);
        k1[3] = fbits(S[3] * S[0]);
        k1[4] = fbits(S[3] * S[1]);
        k1[5] = (uint32_t)(o[0] + P0 * o[1] + P1 * (dim == 3 ? o[2] : 0));
        k1[6] = fbits(S[2] / S[3]);
        k1[7] = fbits(S[3] * S[2]);
    }
    return PD_OK;
}
