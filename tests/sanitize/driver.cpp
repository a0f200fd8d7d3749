// Host-code sanitizer run (test infrastructure): the family builder of the
// library (family.cpp) and the CPU reference (oracle/pd_oracle.c), built
// with AddressSanitizer and UndefinedBehaviorSanitizer, on small workloads
// of every kind the solver takes: a 3D box, notched 2D plates (plane
// stress, a wide horizon, three specimens), a double-notched 3D plate and a
// notched cylinder.  Each workload goes through pd_build_family (both
// phases), pd_bsr_pattern and pd_fac_pattern, and through the reference's
// set-up, notch cuts, explicit steps, force, energy, damage, relaxation,
// power iteration, finite model and breaking-margin tracking; the argument
// errors of pd_build_family are exercised too.  Prints one line per
// workload and "sanitize: ok" at the end; the sanitizers abort on the first
// finding.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "pd.h"

extern "C" {
typedef struct orc_model orc_model;
orc_model *orc_create(int64_t n, int dim, const int32_t *lat, double dx, const double *origin, double delta,
                      const double *vol, const int32_t *spec, int search);
void orc_free(orc_model *o);
int64_t orc_n_bonds(const orc_model *o);
int orc_set_specimen(orc_model *o, int s, int mode, double E, double nu, double rho, double s0, double dt);
int64_t orc_apply_cuts(orc_model *o, const double *cuts, int ncut);
double orc_critical_stretch(int mode, double E, double nu, double G0, double delta, int variant);
int orc_run(orc_model *o, int64_t nsteps, double *u, double *v, const uint8_t *bc, const double *fext,
            int64_t ramp_steps, double *f_out);
void orc_force(orc_model *o, const double *u, double *f, double *theta_out);
double orc_strain_energy(orc_model *o, const double *u);
void orc_damage(const orc_model *o, double *phi);
void orc_adr_density(const orc_model *o, double dt, double *lam);
int orc_adr_run(orc_model *o, int64_t nsteps, double *u, double *v, double *fprev, int64_t *iter,
                const double *lam, const uint8_t *bc, const double *fext, int64_t ramp_steps, double dt,
                double *stats);
double orc_lambda_max(orc_model *o, const uint8_t *bc, int iters, uint64_t seed);
void orc_set_finite(orc_model *o, int finite);
void orc_track_bond_margins(orc_model *o, int on);
int orc_get_bond_margins(const orc_model *o, double *out);
}

namespace {

struct Case {
    const char *name;
    int dim;
    int mode;
    double dx, delta;
    std::vector<int32_t> lat;
    std::vector<int32_t> spec;
    std::vector<pd_cut> cuts;
};

void fail(const char *what, int code) {
    std::fprintf(stderr, "sanitize: %s failed (%d)\n", what, code);
    std::exit(1);
}

Case box3(const char *name, int nx, int ny, int nz, double m) {
    Case c{name, 3, 0, 1e-3, m * 1e-3, {}, {}, {}};
    for (int k = 0; k < nz; k++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) c.lat.insert(c.lat.end(), {i, j, k});
    return c;
}

Case plates2(const char *name, int nplates, int nx, int ny, double m) {
    Case c{name, 2, 1, 0.5e-3, m * 0.5e-3, {}, {}, {}};
    int y0 = 0;
    for (int s = 0; s < nplates; s++) {
        const int w = nx + 7 * s, h = ny + 3 * s;
        for (int j = 0; j < h; j++)
            for (int i = 0; i < w; i++) {
                c.lat.insert(c.lat.end(), {i, y0 + j});
                c.spec.push_back(s);
            }
        pd_cut ct{};
        ct.kind = 0;
        ct.specimen = s;
        const double yc = (y0 + h / 2 - 1 + 0.5) * c.dx;
        const double p[4] = {-0.5 * c.dx, yc, (w / 2 - 1 + 0.37) * c.dx, yc};
        for (int q = 0; q < 4; q++) ct.p[q] = p[q];
        c.cuts.push_back(ct);
        y0 += h + 8;
    }
    return c;
}

Case notched_plate3() {
    Case c = box3("impact plate 36x36x9, two notches", 36, 36, 9, 3.015);
    for (double yc : {13.5, 22.5}) {
        pd_cut ct{};
        ct.kind = 1;
        ct.specimen = -1;
        const double p[9] = {-0.5e-3, yc * 1e-3, -0.5e-3, 9.87e-3, 0, 0, 0, 0, 9e-3};
        for (int q = 0; q < 9; q++) ct.p[q] = p[q];
        c.cuts.push_back(ct);
    }
    return c;
}

Case cylinder() {
    const double dx = 2.5e-3, r = 25e-3, L = 100e-3;
    Case c{"cylinder dx 2.5 mm, helicoidal notch", 3, 0, dx, 3.015 * dx, {}, {}, {}};
    const int ni = (int)std::floor(2 * r / dx - 0.5) + 1, nk = (int)std::floor(L / dx - 0.5) + 1;
    for (int k = 0; k < nk; k++)
        for (int i = 0; i < ni; i++)
            for (int j = 0; j < ni; j++) {
                const double x = (i + 0.5) * dx - r, y = (j + 0.5) * dx - r;
                if (x * x + y * y <= r * r) c.lat.insert(c.lat.end(), {i, j, k});
            }
    pd_cut ct{};
    ct.kind = 2;
    ct.specimen = -1;
    const double p[6] = {50.37e-3, r, r - 5e-3, 10 * r, -0.5 * M_PI, 0.5 * M_PI};
    for (int q = 0; q < 6; q++) ct.p[q] = p[q];
    c.cuts.push_back(ct);
    return c;
}

void run_case(const Case &c) {
    const int64_t n = (int64_t)c.lat.size() / c.dim;
    const double vol1 = c.dim == 3 ? c.dx * c.dx * c.dx : c.dx * c.dx;
    std::vector<double> vol((size_t)n, vol1);
    double origin[3] = {0, 0, 0};
    if (c.name[0] == 'c') origin[0] = origin[1] = 0.5 * c.dx - 25e-3, origin[2] = 0.5 * c.dx;
    // library: pd_build_family, both phases, then the two pattern builders
    pd_body b{};
    b.n = n;
    b.dim = c.dim;
    b.lat = c.lat.data();
    b.dx = c.dx;
    for (int q = 0; q < 3; q++) b.origin[q] = origin[q];
    b.delta = c.delta;
    b.vol = vol.data();
    b.specimen = c.spec.empty() ? nullptr : c.spec.data();
    pd_family_sizes sz{};
    pd_status st = pd_build_family(&b, c.cuts.data(), (int32_t)c.cuts.size(), &sz, nullptr);
    if (st != PD_OK) fail("pd_build_family sizes", st);
    std::vector<int32_t> perm(sz.n_pad), row_of(sz.n), spec(sz.n_pad), lat4(sz.n_pad * 4), tile_org(sz.n_tiles * 4),
        tile_nbr(sz.n_tiles * 27), stoff(sz.n_stencil * 3), hpos(std::max<int32_t>(1, sz.n_box));
    std::vector<int64_t> sptr(sz.n_slices + 1);
    std::vector<uint32_t> words(sz.n_words), ktab(128 * 20);
    std::vector<uint64_t> mask(sz.n_mask);
    std::vector<double> sten(sz.n_stencil * 4), fvol(sz.n_pad), invm(sz.n_pad);
    std::vector<int16_t> hmap(std::max<int32_t>(1, sz.n_halo));
    pd_family_host h{perm.data(), row_of.data(), sptr.data(), words.data(), mask.data(), sten.data(),
                     stoff.data(), fvol.data(), invm.data(), spec.data(), lat4.data(), tile_org.data(),
                     tile_nbr.data(), ktab.data(), hmap.data(), hpos.data()};
    if ((st = pd_build_family(&b, c.cuts.data(), (int32_t)c.cuts.size(), &sz, &h)) != PD_OK)
        fail("pd_build_family", st);
    pd_bsr_sizes bs{};
    if ((st = pd_bsr_pattern(&sz, &h, &bs, nullptr, nullptr)) != PD_OK) fail("pd_bsr_pattern sizes", st);
    std::vector<int64_t> rp(sz.n_pad + 1);
    std::vector<int32_t> col(bs.nnzb);
    if ((st = pd_bsr_pattern(&sz, &h, &bs, rp.data(), col.data())) != PD_OK) fail("pd_bsr_pattern", st);
    pd_fac_sizes fs{};
    if ((st = pd_fac_pattern(&sz, &h, &fs, nullptr, nullptr, nullptr)) != PD_OK) fail("pd_fac_pattern sizes", st);
    std::vector<int32_t> bij(2 * fs.nb), bpos(2 * fs.nb), bid(fs.n_words);
    if ((st = pd_fac_pattern(&sz, &h, &fs, bij.data(), bpos.data(), bid.data())) != PD_OK) fail("pd_fac_pattern", st);

    // reference: set-up, cuts, steps, force, energy, damage, relaxation,
    // power iteration, finite model, margins
    orc_model *o = orc_create(n, c.dim, c.lat.data(), c.dx, origin, c.delta, vol.data(),
                              c.spec.empty() ? nullptr : c.spec.data(), n > 3000 ? 1 : 0);
    if (!o) fail("orc_create", 0);
    const int64_t nb = orc_n_bonds(o);
    if (nb != sz.n_bonds) fail("bond count", (int)(nb - sz.n_bonds));
    const int nspec = c.spec.empty() ? 1 : c.spec.back() + 1;
    for (int s = 0; s < nspec; s++) {
        const double E = 70e9 + 10e9 * s, nu = 0.22, G0 = 3.8;
        const double s0 = orc_critical_stretch(c.mode, E, nu, G0, c.delta, 0);
        if (orc_set_specimen(o, s, c.mode, E, nu, 2440.0, s0 * 0.2, 1e-8) != 0) fail("orc_set_specimen", s);
    }
    std::vector<double> cuts;
    for (const pd_cut &ct : c.cuts) {
        cuts.push_back(ct.kind);
        cuts.push_back(ct.specimen);
        for (int q = 0; q < 10; q++) cuts.push_back(ct.p[q]);
    }
    const int64_t ncut = orc_apply_cuts(o, cuts.data(), (int)c.cuts.size());
    if (ncut != sz.n_cut) fail("cut count", (int)(ncut - sz.n_cut));
    std::vector<double> u((size_t)3 * n, 0.0), v((size_t)3 * n, 0.0), f((size_t)3 * n), th((size_t)n),
        fext((size_t)3 * n, 0.0), phi((size_t)n), lam((size_t)3 * n), fprev((size_t)3 * n, 0.0), marg((size_t)nb);
    std::vector<uint8_t> bc((size_t)n, 0);
    for (int64_t p = 0; p < n; p++) {
        v[3 * p] = 1e-3 * std::sin(0.1 * (double)p);
        if (c.lat[c.dim * p] == 0) bc[p] = 7;
        fext[3 * p + 1] = (p % 7 == 0) ? 1e3 : 0.0;
    }
    orc_track_bond_margins(o, 1);
    orc_run(o, 20, u.data(), v.data(), bc.data(), fext.data(), 5, f.data());
    if (orc_get_bond_margins(o, marg.data()) != 0) fail("orc_get_bond_margins", 0);
    orc_force(o, u.data(), f.data(), th.data());
    const double W = orc_strain_energy(o, u.data());
    orc_damage(o, phi.data());
    orc_adr_density(o, 1.0, lam.data());
    int64_t it = 0;
    double stats[4] = {0, 0, 0, 0};
    orc_adr_run(o, 5, u.data(), v.data(), fprev.data(), &it, lam.data(), bc.data(), fext.data(), 0, 1.0, stats);
    const double lmax = orc_lambda_max(o, bc.data(), 5, 7);
    orc_set_finite(o, 1);
    orc_run(o, 3, u.data(), v.data(), bc.data(), fext.data(), 0, nullptr);
    orc_track_bond_margins(o, 0);
    orc_free(o);
    std::printf("%s: n %lld, bonds %lld, cut %lld, K blocks %lld, energy %.3e, lambda %.3e\n", c.name, (long long)n,
                (long long)nb, (long long)ncut, (long long)bs.nnzb, W, lmax);
}

void argument_errors() {
    int32_t lat[6] = {0, 0, 0, 0, 0, 0};  // a duplicate point
    double vol[2] = {1.0, 1.0};
    pd_body b{};
    b.n = 2;
    b.dim = 3;
    b.lat = lat;
    b.dx = 1.0;
    b.delta = 3.015;
    b.vol = vol;
    pd_family_sizes sz{};
    if (pd_build_family(&b, nullptr, 0, &sz, nullptr) != PD_ERR_ARG) fail("duplicate point error", 0);
    b.n = 0;
    if (pd_build_family(&b, nullptr, 0, &sz, nullptr) != PD_ERR_SIZE) fail("empty body error", 0);
    b.n = 2;
    b.dim = 4;
    if (pd_build_family(&b, nullptr, 0, &sz, nullptr) != PD_ERR_ARG) fail("dimension error", 0);
    b.dim = 3;
    lat[3] = 1;
    pd_cut ct{};
    ct.kind = 7;
    if (pd_build_family(&b, &ct, 1, &sz, nullptr) != PD_ERR_ARG) fail("cut kind error", 0);
}

}  // namespace

int main() {
    argument_errors();
    run_case(box3("cantilever 20x4x4", 20, 4, 4, 3.015));
    run_case(plates2("notched plate 48x24", 1, 48, 24, 3.015));
    run_case(plates2("three plates, horizon 5.015 dx", 3, 40, 20, 5.015));
    run_case(notched_plate3());
    run_case(cylinder());
    std::printf("sanitize: ok\n");
    return 0;
}
