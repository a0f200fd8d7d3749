/*
 * pd_oracle.c -- CPU reference ("oracle") for linearized ordinary state-based
 * peridynamics (OSB-PD), double precision, plain loops.
 *
 * TEST INFRASTRUCTURE ONLY.  This file exists to check the GPU library.  Only
 * the test suite, the smoke check and the CPU-baseline leg of the benchmark
 * may load it.  It shares no code, header or table with the GPU library.
 *
 * What it computes, in the paper's notation (Ni, Zaccariotto, Zhu, Galvanetto,
 * "Matrix-based implementation and GPU acceleration of linearized ordinary
 * state-based peridynamic models in MATLAB"):
 *
 *   family          H_i = { j : 0 < |xi_ij| <= delta }              (Sec. 2.1, def. of H_x)
 *   bond geometry   xi = x_j - x_i, x = |xi|, M = xi / x            (Eqs. 1.2-1.5, 1.13 linearized)
 *   weighted volume m_i = sum_j w x^2 V_j, w = 1                    (Eq. 1.9, Sec. 2.3 w=1)
 *   extension       e_ij = M_ij . (u_j - u_i)                       (Eqs. 2.4, 2.7)
 *                   or, for the finite model, e = |x M + u_j - u_i| - x with
 *                   force direction (x M + u_j - u_i)/|...|          (Eqs. 1.10, 1.13)
 *   stretch         s = e / x ; bond status rho = 1 iff s < s_c     (Eqs. 1.17, 1.30)
 *   dilatation      theta_i = (A/m_i) sum_j rho w x e V_j           (Eqs. 1.6, 2.3)
 *   pair force      f_i = sum_j rho [(K-G/3) x (theta_i/m_i + theta_j/m_j)
 *                                  + G e (1/m_i + 1/m_j)] w M_ij V_i V_j     (Eq. 2.2)
 *   update          v += dt a, u += dt v, a = (f + F_ext)/(rho V)   (Eqs. 2.11, 2.12)
 *   damage          phi_i = 1 - sum rho w V_j / sum w V_j           (Eq. 1.31)
 *   quasi-static    adaptive dynamic relaxation (the solver of Sec. 4
 *                   Example 4; its formulas are Kilic and Madenci's, cited
 *                   there, restated below with a Gershgorin density)
 *   constants       A (Eq. 1.8), K (Eq. 1.15), G (Eq. 1.16)
 *   critical stretch s_c (Eqs. 1.26-1.29)
 *
 * Readings where the paper is silent (each is listed with its reason in the
 * design notes of the repository):
 *   - m is computed once over the full geometric family, notch bonds included.
 *   - Breaking is irreversible; the check runs at the start of each force
 *     evaluation, before the dilatation, and s = s_c breaks.
 *   - The internal force f is the restoring force of Eq. 2.2 and the
 *     acceleration is (F_ext + f)/(rho V), as in the solver listing of the
 *     matrix scheme (residual = external + peridynamic force).
 *   - Prescribed displacement components have zero acceleration: their
 *     velocity keeps its initial value and u advances by dt * v.
 *   - The extension is evaluated as (M1*eta1 + M2*eta2) + M3*eta3 with no
 *     fused multiply-add (the file is compiled with -ffp-contract=off).
 *
 * Pins (the CPU test suite checks this file against facts that do not come
 * from these formulas): the bond count the paper prints for a 10x10 grid and
 * the 28 / 122 interior family sizes; rigid motion gives zero force; momentum
 * balance; a uniform dilatation gives theta = A eps; the equibiaxial energy is
 * the classical one; f = -grad E of the stored energy; the paper's matrix form
 * equals the loop form; the stiffness is symmetric positive semi-definite with
 * the rigid-motion null space; the beta constants by quadrature; the 3D
 * critical stretch from the energy released across a crack; the two-node
 * oscillator and the break step in closed form; the discrete energy invariant
 * of the update; the cantilever's first bending frequency; notch cuts against
 * sampled crossings of every bond segment; for the finite model, zero force
 * under a finite rigid rotation, the force as the energy gradient and the
 * first-order agreement with the linearized model; for the relaxation, a
 * density that bounds every row of |K|, convergence to the direct static
 * solution and damping that approaches twice the slowest frequency.
 * Parity unpinned: the 2D critical stretch (Eq. 1.28, taken as printed; the
 * paper prints no value of it, and it is not what the 2D stored energy gives),
 * and the crack paths of the fracture workloads (nothing outside this file
 * predicts them).
 *
 * Build: gcc -O2 -fPIC -shared -ffp-contract=off -fno-fast-math -fopenmp
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAX_SPEC 4096

typedef struct {
    /* per-specimen constants */
    double E, nu, rho, s0, dt;
    double kappa, mu, A, K, G;
} orc_spec;

typedef struct {
    int64_t n;
    int dim;
    int mode;           /* 0 3D, 1 plane stress, 2 plane strain */
    double dx, delta;
    double *X;          /* n*3 reference positions */
    int32_t *lat;       /* n*3 lattice coordinates (z = 0 in 2D) */
    double *V;          /* n */
    int32_t *sp;        /* n specimen id */
    /* unique bonds i < j, sorted by (i, j) */
    int64_t nb;
    int32_t *bi, *bj;
    double *xl;         /* nb bond length x */
    double *M;          /* nb*3 unit vector xi/x, xi = x_j - x_i */
    uint8_t *rho;       /* nb bond status (Eq. 1.30) */
    int32_t *brk;       /* nb step at which the bond broke (-1 intact, -2 cut) */
    double *e;          /* nb scratch: extension */
    int finite;         /* 0: linearized extension (Eqs. 2.4, 2.7); 1: finite (Eqs. 1.10, 1.13) */
    double *My;         /* nb*3 scratch: deformed direction Y/|Y| (finite model) */
    /* node -> incident bonds, sorted by the other node */
    int64_t *aptr;
    int64_t *abond;
    double *m;          /* n weighted volume */
    double *theta;      /* n dilatation */
    int nspec;
    orc_spec spec[ORC_MAX_SPEC];
    int64_t step;       /* index n of the next step */
    /* breaking diagnostics of the last run */
    double min_margin;  /* min |s - s_c| / s_c over evaluated intact bonds */
    int64_t n_close6;   /* evaluations with margin < 1e-6 */
    double *bmargin;    /* nb running min of |s - s_c| / s_c per bond over the
                           evaluations made while it was intact (the breaking
                           evaluation included); NULL = not tracked */
} orc_model;

/* ------------------------------------------------------------------------ */
/* family search                                                            */
/* ------------------------------------------------------------------------ */

typedef struct { int32_t i, j; } pair_t;

static int cmp_pair(const void *a, const void *b) {
    const pair_t *p = (const pair_t *)a, *q = (const pair_t *)b;
    if (p->i != q->i) return p->i < q->i ? -1 : 1;
    if (p->j != q->j) return p->j < q->j ? -1 : 1;
    return 0;
}

/* Bond length of the lattice offset d (in lattice units) scaled by dx. */
static double bond_len(const orc_model *o, const int32_t *li, const int32_t *lj) {
    double s = 0.0;
    for (int c = 0; c < 3; c++) {
        double xi = o->dx * (double)(lj[c] - li[c]);
        s += xi * xi;
    }
    return sqrt(s);
}

static int in_family(const orc_model *o, int64_t i, int64_t j) {
    if (i == j) return 0;
    if (o->sp[i] != o->sp[j]) return 0;
    double x = bond_len(o, o->lat + 3 * i, o->lat + 3 * j);
    return x <= o->delta;
}

/* Brute force O(n^2): every pair is tested. */
static int64_t search_brute(orc_model *o, pair_t **out) {
    int64_t cap = 1024, cnt = 0;
    pair_t *p = (pair_t *)malloc(sizeof(pair_t) * cap);
    for (int64_t i = 0; i < o->n; i++)
        for (int64_t j = i + 1; j < o->n; j++)
            if (in_family(o, i, j)) {
                if (cnt == cap) { cap *= 2; p = (pair_t *)realloc(p, sizeof(pair_t) * cap); }
                p[cnt].i = (int32_t)i; p[cnt].j = (int32_t)j; cnt++;
            }
    *out = p;
    return cnt;
}

/* Cell list: lattice cells of edge c = ceil(delta/dx) lattice units; a
 * node's family lies in its own and the adjacent cells. */
static int64_t search_cells(orc_model *o, pair_t **out) {
    int64_t n = o->n;
    int32_t lo[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, hi[3] = {INT32_MIN, INT32_MIN, INT32_MIN};
    for (int64_t p = 0; p < n; p++)
        for (int c = 0; c < 3; c++) {
            if (o->lat[3 * p + c] < lo[c]) lo[c] = o->lat[3 * p + c];
            if (o->lat[3 * p + c] > hi[c]) hi[c] = o->lat[3 * p + c];
        }
    int32_t cw = (int32_t)ceil(o->delta / o->dx);
    if (cw < 1) cw = 1;
    int64_t nc[3];
    for (int c = 0; c < 3; c++) nc[c] = (hi[c] - lo[c]) / cw + 1;
    int64_t ncell = nc[0] * nc[1] * nc[2];
    int64_t *cstart = (int64_t *)calloc(ncell + 1, sizeof(int64_t));
    int64_t *cell = (int64_t *)malloc(sizeof(int64_t) * n);
    for (int64_t p = 0; p < n; p++) {
        int64_t a = (o->lat[3 * p] - lo[0]) / cw, b = (o->lat[3 * p + 1] - lo[1]) / cw,
                d = (o->lat[3 * p + 2] - lo[2]) / cw;
        cell[p] = (a * nc[1] + b) * nc[2] + d;
        cstart[cell[p] + 1]++;
    }
    for (int64_t k = 0; k < ncell; k++) cstart[k + 1] += cstart[k];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * ncell);
    memcpy(fill, cstart, sizeof(int64_t) * ncell);
    int64_t *members = (int64_t *)malloc(sizeof(int64_t) * n);
    for (int64_t p = 0; p < n; p++) members[fill[cell[p]]++] = p;
    free(fill);

    /* count per node, then fill (two passes keep it parallel and ordered) */
    int64_t *cnt = (int64_t *)calloc(n + 1, sizeof(int64_t));
    for (int pass = 0; pass < 2; pass++) {
        pair_t *buf = pass ? *out : NULL;
        #pragma omp parallel for schedule(dynamic, 256)
        for (int64_t i = 0; i < n; i++) {
            int64_t a = (o->lat[3 * i] - lo[0]) / cw, b = (o->lat[3 * i + 1] - lo[1]) / cw,
                    d = (o->lat[3 * i + 2] - lo[2]) / cw;
            int64_t k = pass ? cnt[i] : 0;
            for (int64_t da = -1; da <= 1; da++)
                for (int64_t db = -1; db <= 1; db++)
                    for (int64_t dd = -1; dd <= 1; dd++) {
                        int64_t A = a + da, B = b + db, D = d + dd;
                        if (A < 0 || B < 0 || D < 0 || A >= nc[0] || B >= nc[1] || D >= nc[2]) continue;
                        int64_t cc = (A * nc[1] + B) * nc[2] + D;
                        for (int64_t q = cstart[cc]; q < cstart[cc + 1]; q++) {
                            int64_t j = members[q];
                            if (j <= i) continue;
                            if (!in_family(o, i, j)) continue;
                            if (pass) { buf[k].i = (int32_t)i; buf[k].j = (int32_t)j; }
                            k++;
                        }
                    }
            if (!pass) cnt[i + 1] = k;
        }
        if (!pass) {
            for (int64_t i = 0; i < n; i++) cnt[i + 1] += cnt[i];
            /* cnt[i] is now the first slot of node i */
            *out = (pair_t *)malloc(sizeof(pair_t) * (cnt[n] > 0 ? cnt[n] : 1));
        }
    }
    int64_t total = cnt[n];
    /* each node's pairs were gathered cell by cell; sort globally */
    qsort(*out, total, sizeof(pair_t), cmp_pair);
    free(cnt); free(members); free(cell); free(cstart);
    return total;
}

/* ------------------------------------------------------------------------ */
/* model creation                                                           */
/* ------------------------------------------------------------------------ */

void orc_free(orc_model *o);

/* lat: n*dim integer lattice coordinates; origin[3]; vol[n]; spec[n] (or NULL).
 * search: 0 brute force, 1 cell list. */
orc_model *orc_create(int64_t n, int dim, const int32_t *lat, double dx, const double *origin,
                      double delta, const double *vol, const int32_t *spec, int search) {
    orc_model *o = (orc_model *)calloc(1, sizeof(orc_model));
    o->n = n; o->dim = dim; o->dx = dx; o->delta = delta;
    o->X = (double *)malloc(sizeof(double) * 3 * n);
    o->lat = (int32_t *)calloc(3 * n, sizeof(int32_t));
    o->V = (double *)malloc(sizeof(double) * n);
    o->sp = (int32_t *)calloc(n, sizeof(int32_t));
    for (int64_t p = 0; p < n; p++) {
        for (int c = 0; c < dim; c++) o->lat[3 * p + c] = lat[dim * p + c];
        for (int c = 0; c < 3; c++) o->X[3 * p + c] = origin[c] + dx * (double)o->lat[3 * p + c];
        o->V[p] = vol[p];
        if (spec) o->sp[p] = spec[p];
    }
    pair_t *pairs = NULL;
    o->nb = search ? search_cells(o, &pairs) : search_brute(o, &pairs);
    int64_t nb = o->nb;
    o->bi = (int32_t *)malloc(sizeof(int32_t) * (nb + 1));
    o->bj = (int32_t *)malloc(sizeof(int32_t) * (nb + 1));
    o->xl = (double *)malloc(sizeof(double) * (nb + 1));
    o->M = (double *)malloc(sizeof(double) * 3 * (nb + 1));
    o->rho = (uint8_t *)malloc(nb + 1);
    o->brk = (int32_t *)malloc(sizeof(int32_t) * (nb + 1));
    o->e = (double *)calloc(nb + 1, sizeof(double));
    o->My = (double *)calloc(3 * (nb + 1), sizeof(double));
    #pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < nb; b++) {
        int64_t i = pairs[b].i, j = pairs[b].j;
        o->bi[b] = (int32_t)i; o->bj[b] = (int32_t)j;
        double xi[3];
        for (int c = 0; c < 3; c++) xi[c] = dx * (double)(o->lat[3 * j + c] - o->lat[3 * i + c]);
        double x = sqrt(xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2]);
        o->xl[b] = x;
        for (int c = 0; c < 3; c++) o->M[3 * b + c] = xi[c] / x;
        o->rho[b] = 1;
        o->brk[b] = -1;
    }
    free(pairs);
    /* adjacency */
    o->aptr = (int64_t *)calloc(n + 1, sizeof(int64_t));
    for (int64_t b = 0; b < nb; b++) { o->aptr[o->bi[b] + 1]++; o->aptr[o->bj[b] + 1]++; }
    for (int64_t p = 0; p < n; p++) o->aptr[p + 1] += o->aptr[p];
    o->abond = (int64_t *)malloc(sizeof(int64_t) * (2 * nb + 1));
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (n + 1));
    memcpy(fill, o->aptr, sizeof(int64_t) * (n + 1));
    /* Bonds are sorted by (i, j).  For node p the incident bonds with p as
     * the larger end (other < p) come first in increasing other, then those
     * with p as the smaller end (other > p), also increasing. */
    for (int64_t b = 0; b < nb; b++) o->abond[fill[o->bj[b]]++] = b;
    for (int64_t b = 0; b < nb; b++) o->abond[fill[o->bi[b]]++] = b;
    free(fill);
    /* weighted volume (Eq. 1.9) over the full geometric family, w = 1 */
    o->m = (double *)calloc(n, sizeof(double));
    o->theta = (double *)calloc(n, sizeof(double));
    #pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < n; p++) {
        double s = 0.0;
        for (int64_t k = o->aptr[p]; k < o->aptr[p + 1]; k++) {
            int64_t b = o->abond[k];
            int64_t q = (o->bi[b] == p) ? o->bj[b] : o->bi[b];
            s += o->xl[b] * o->xl[b] * o->V[q];
        }
        o->m[p] = s;
    }
    o->nspec = 0;
    o->step = 0;
    o->min_margin = INFINITY;
    return o;
}

void orc_free(orc_model *o) {
    if (!o) return;
    free(o->X); free(o->lat); free(o->V); free(o->sp);
    free(o->bi); free(o->bj); free(o->xl); free(o->M); free(o->rho); free(o->brk); free(o->e); free(o->My);
    free(o->aptr); free(o->abond); free(o->m); free(o->theta); free(o->bmargin);
    free(o);
}

int64_t orc_n_bonds(const orc_model *o) { return o->nb; }

void orc_get_bonds(const orc_model *o, int32_t *bi, int32_t *bj) {
    memcpy(bi, o->bi, sizeof(int32_t) * o->nb);
    memcpy(bj, o->bj, sizeof(int32_t) * o->nb);
}
void orc_get_bond_geom(const orc_model *o, double *xl, double *M) {
    memcpy(xl, o->xl, sizeof(double) * o->nb);
    memcpy(M, o->M, sizeof(double) * 3 * o->nb);
}
void orc_get_m(const orc_model *o, double *m) { memcpy(m, o->m, sizeof(double) * o->n); }
void orc_get_theta(const orc_model *o, double *t) { memcpy(t, o->theta, sizeof(double) * o->n); }
void orc_get_rho(const orc_model *o, uint8_t *r) { memcpy(r, o->rho, o->nb); }
void orc_set_rho(orc_model *o, const uint8_t *r) { memcpy(o->rho, r, o->nb); }
void orc_get_break_step(const orc_model *o, int32_t *s) { memcpy(s, o->brk, sizeof(int32_t) * o->nb); }
int64_t orc_get_step(const orc_model *o) { return o->step; }
void orc_set_step(orc_model *o, int64_t s) { o->step = s; }
double orc_min_margin(const orc_model *o) { return o->min_margin; }
int64_t orc_n_close(const orc_model *o) { return o->n_close6; }
void orc_reset_margin(orc_model *o) { o->min_margin = INFINITY; o->n_close6 = 0; }

/* Per-bond breaking margins (a diagnostic: how close each bond came to the
 * critical stretch of Eq. 1.30; the arithmetic of a step is unchanged).
 * on != 0 starts tracking from +inf, on == 0 stops and frees the array. */
void orc_track_bond_margins(orc_model *o, int on) {
    free(o->bmargin);
    o->bmargin = NULL;
    if (!on) return;
    o->bmargin = (double *)malloc(sizeof(double) * (o->nb + 1));
    for (int64_t b = 0; b < o->nb; b++) o->bmargin[b] = INFINITY;
}
/* Copies the running minima into out[nb]; returns 0, or -1 if not tracked. */
int orc_get_bond_margins(const orc_model *o, double *out) {
    if (!o->bmargin) return -1;
    memcpy(out, o->bmargin, sizeof(double) * o->nb);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* material constants and critical stretch                                  */
/* ------------------------------------------------------------------------ */

/* A (Eq. 1.8), K (Eq. 1.15), G (Eq. 1.16); kappa, mu are the bulk and shear
 * moduli of (E, nu). out[5] = {kappa, mu, A, K, G}. */
void orc_constants(int mode, double E, double nu, double *out) {
    double kappa = E / (3.0 * (1.0 - 2.0 * nu));
    double mu = E / (2.0 * (1.0 + nu));
    double A, K, G;
    if (mode == 0) {
        A = 3.0;
        K = 3.0 * kappa;
        G = 15.0 * mu;
    } else if (mode == 1) {
        A = 2.0 * (1.0 - 2.0 * nu) / (1.0 - nu);
        K = 2.0 * kappa * (1.0 - 2.0 * nu) / (1.0 - nu)
            - (2.0 / 3.0) * mu * (1.0 + nu) * (1.0 - 3.0 * nu) / ((1.0 - nu) * (1.0 - 2.0 * nu));
        G = 8.0 * mu;
    } else {
        A = 2.0;
        K = 2.0 * kappa - (2.0 / 3.0) * mu;
        G = 8.0 * mu;
    }
    out[0] = kappa; out[1] = mu; out[2] = A; out[3] = K; out[4] = G;
}

/* Critical stretch s_c.  3D: Eq. 1.26 with beta, beta' of Eq. 1.27
 * (variant 0: beta' as printed, 5 delta / (24 pi); variant 1: 5 delta / 24,
 * the value the same quadrature that gives beta yields).  2D: Eq. 1.28 with
 * Eq. 1.29.  G0 <= 0 or not finite means "never breaks" (returns +inf). */
double orc_critical_stretch(int mode, double E, double nu, double G0, double delta, int variant) {
    if (!(G0 > 0.0) || !isfinite(G0)) return INFINITY;
    double k[5];
    orc_constants(mode, E, nu, k);
    double kappa = k[0], mu = k[1], A = k[2];
    const double pi = 3.14159265358979323846;
    if (mode == 0) {
        double beta = 125.0 * delta / 1848.0;
        double betap = variant ? 5.0 * delta / 24.0 : 5.0 * delta / (24.0 * pi);
        return sqrt(G0 / ((9.0 * kappa - 15.0 * mu) * beta + 15.0 * mu * betap));
    }
    double kp = (mode == 1) ? kappa + mu / 9.0 * ((1.0 + nu) / (1.0 - 2.0 * nu)) * ((1.0 + nu) / (1.0 - 2.0 * nu))
                            : kappa + mu / 9.0;
    double beta = 1087.0 * delta / (1250.0 * pi * pi);
    double betap = 4.0 * delta / (5.0 * pi);
    return sqrt(G0 / (A * A * (kp - 8.0 / 9.0 * mu) * beta + 8.0 * mu * betap));
}

/* Material of specimen s. */
int orc_set_specimen(orc_model *o, int s, int mode, double E, double nu, double rho, double s0, double dt) {
    if (s < 0 || s >= ORC_MAX_SPEC) return -1;
    o->mode = mode;
    orc_spec *p = &o->spec[s];
    double k[5];
    orc_constants(mode, E, nu, k);
    p->E = E; p->nu = nu; p->rho = rho; p->s0 = s0; p->dt = dt;
    p->kappa = k[0]; p->mu = k[1]; p->A = k[2]; p->K = k[3]; p->G = k[4];
    if (s + 1 > o->nspec) o->nspec = s + 1;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* notches                                                                  */
/* ------------------------------------------------------------------------ */

static double cross2(double ax, double ay, double bx, double by) { return ax * by - ay * bx; }

/* Proper crossing of bond P-Q with segment A-B (2D). */
static int cut_segment(const double *P, const double *Q, const double *c) {
    double Ax = c[0], Ay = c[1], Bx = c[2], By = c[3];
    double d1 = cross2(Bx - Ax, By - Ay, P[0] - Ax, P[1] - Ay);
    double d2 = cross2(Bx - Ax, By - Ay, Q[0] - Ax, Q[1] - Ay);
    double d3 = cross2(Q[0] - P[0], Q[1] - P[1], Ax - P[0], Ay - P[1]);
    double d4 = cross2(Q[0] - P[0], Q[1] - P[1], Bx - P[0], By - P[1]);
    return (d1 * d2 < 0.0) && (d3 * d4 < 0.0);
}

/* Bond P-Q crosses the parallelogram {c + s a + t b}, 0 < s, t < 1. */
static int cut_rect(const double *P, const double *Q, const double *prm) {
    const double *c = prm, *a = prm + 3, *b = prm + 6;
    double nrm[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
    double sp = 0, sq = 0;
    for (int k = 0; k < 3; k++) { sp += nrm[k] * (P[k] - c[k]); sq += nrm[k] * (Q[k] - c[k]); }
    if (!(sp * sq < 0.0)) return 0;
    double t = sp / (sp - sq);
    double r[3];
    for (int k = 0; k < 3; k++) r[k] = P[k] + t * (Q[k] - P[k]) - c[k];
    /* solve r = s a + u b in the plane (Gram system) */
    double aa = 0, ab = 0, bb = 0, ra = 0, rb = 0;
    for (int k = 0; k < 3; k++) { aa += a[k] * a[k]; ab += a[k] * b[k]; bb += b[k] * b[k]; ra += r[k] * a[k]; rb += r[k] * b[k]; }
    double det = aa * bb - ab * ab;
    double s = (ra * bb - rb * ab) / det;
    double u = (rb * aa - ra * ab) / det;
    return s > 0.0 && s < 1.0 && u > 0.0 && u < 1.0;
}

/* Helicoidal strip z - zc = p * theta about the z axis: the level set
 * psi = (z - zc) - p * atan2(y, x) changes sign along the bond and the
 * linearly interpolated crossing lies inside r_in < r < r_out,
 * th0 < theta < th1. prm = {zc, p, r_in, r_out, th0, th1}. */
static double helix_psi(const double *X, const double *prm) {
    return (X[2] - prm[0]) - prm[1] * atan2(X[1], X[0]);
}
static int cut_helicoid(const double *P, const double *Q, const double *prm) {
    double fp = helix_psi(P, prm), fq = helix_psi(Q, prm);
    if (!(fp * fq < 0.0)) return 0;
    double t = fp / (fp - fq);
    double Xs[3];
    for (int k = 0; k < 3; k++) Xs[k] = P[k] + t * (Q[k] - P[k]);
    double r = sqrt(Xs[0] * Xs[0] + Xs[1] * Xs[1]);
    double th = atan2(Xs[1], Xs[0]);
    return r > prm[2] && r < prm[3] && th > prm[4] && th < prm[5];
}

/* cuts: ncut records of 12 doubles {kind, specimen, p0..p9}.  Bonds that a
 * notch crosses start broken (rho = 0, break step -2).  Returns the count. */
int64_t orc_apply_cuts(orc_model *o, const double *cuts, int ncut) {
    int64_t total = 0;
    #pragma omp parallel for schedule(static) reduction(+ : total)
    for (int64_t b = 0; b < o->nb; b++) {
        const double *P = o->X + 3 * (int64_t)o->bi[b];
        const double *Q = o->X + 3 * (int64_t)o->bj[b];
        for (int k = 0; k < ncut; k++) {
            const double *c = cuts + 12 * k;
            int kind = (int)c[0], spc = (int)c[1];
            if (spc >= 0 && o->sp[o->bi[b]] != spc) continue;
            int hit = 0;
            if (kind == 0) hit = cut_segment(P, Q, c + 2);
            else if (kind == 1) hit = cut_rect(P, Q, c + 2);
            else if (kind == 2) hit = cut_helicoid(P, Q, c + 2);
            if (hit) { o->rho[b] = 0; o->brk[b] = -2; total++; break; }
        }
    }
    return total;
}

/* ------------------------------------------------------------------------ */
/* force evaluation                                                         */
/* ------------------------------------------------------------------------ */

/* Extension of bond b.  Linearized (Eqs. 2.4, 2.7): e = M . (u_j - u_i).
 * Finite (Eqs. 1.10, 1.13): Y = x M + (u_j - u_i), e = |Y| - x, and the
 * force direction becomes Y / |Y| (stored in My); |Y|^2 is summed as
 * (Y1^2 + Y2^2) + Y3^2. */
static double extension(orc_model *o, int64_t b, const double *u) {
    const double *M = o->M + 3 * b;
    int64_t i = o->bi[b], j = o->bj[b];
    double eta0 = u[3 * j] - u[3 * i];
    double eta1 = u[3 * j + 1] - u[3 * i + 1];
    double eta2 = u[3 * j + 2] - u[3 * i + 2];
    if (!o->finite) return (M[0] * eta0 + M[1] * eta1) + M[2] * eta2;
    double x = o->xl[b];
    double Y0 = x * M[0] + eta0, Y1 = x * M[1] + eta1, Y2 = x * M[2] + eta2;
    double y = sqrt((Y0 * Y0 + Y1 * Y1) + Y2 * Y2);
    double *my = o->My + 3 * b;
    my[0] = Y0 / y;
    my[1] = Y1 / y;
    my[2] = Y2 / y;
    return y - x;
}

void orc_set_finite(orc_model *o, int finite) { o->finite = finite ? 1 : 0; }

/* Breaking check (Eqs. 1.17, 1.30) at step 'step'. */
static void break_bonds(orc_model *o, const double *u, int64_t step) {
    double mm = INFINITY;
    int64_t close = 0;
    #pragma omp parallel for schedule(static) reduction(min : mm) reduction(+ : close)
    for (int64_t b = 0; b < o->nb; b++) {
        double e = extension(o, b, u);
        o->e[b] = e;
        if (!o->rho[b]) continue;
        double s0 = o->spec[o->sp[o->bi[b]]].s0;
        if (!isfinite(s0)) continue;
        double s = e / o->xl[b];
        double margin = fabs(s - s0) / s0;
        if (margin < mm) mm = margin;
        if (margin < 1e-6) close++;
        if (o->bmargin && margin < o->bmargin[b]) o->bmargin[b] = margin;
        if (s >= s0) { o->rho[b] = 0; o->brk[b] = (int32_t)step; }
    }
    if (mm < o->min_margin) o->min_margin = mm;
    o->n_close6 += close;
}

static void compute_extensions(orc_model *o, const double *u) {
    #pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < o->nb; b++) o->e[b] = extension(o, b, u);
}

/* Dilatation (Eqs. 1.6, 2.3) and pair force (Eq. 2.2) from the extensions
 * in o->e and the bond status in o->rho. */
static void dilatation_and_force(orc_model *o, double *f) {
    int64_t n = o->n;
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        const orc_spec *sp = &o->spec[o->sp[i]];
        double acc = 0.0;
        for (int64_t k = o->aptr[i]; k < o->aptr[i + 1]; k++) {
            int64_t b = o->abond[k];
            if (!o->rho[b]) continue;
            int64_t j = (o->bi[b] == i) ? o->bj[b] : o->bi[b];
            acc += o->xl[b] * o->e[b] * o->V[j];   /* w = 1 */
        }
        o->theta[i] = sp->A / o->m[i] * acc;
    }
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        const orc_spec *sp = &o->spec[o->sp[i]];
        double fi[3] = {0.0, 0.0, 0.0};
        for (int64_t k = o->aptr[i]; k < o->aptr[i + 1]; k++) {
            int64_t b = o->abond[k];
            if (!o->rho[b]) continue;
            int i_is_first = (o->bi[b] == i);
            int64_t j = i_is_first ? o->bj[b] : o->bi[b];
            double x = o->xl[b], e = o->e[b];
            double th_t = o->theta[i] / o->m[i] + o->theta[j] / o->m[j];
            double e_t = e / o->m[i] + e / o->m[j];
            double t = ((sp->K - sp->G / 3.0) * th_t * x + sp->G * e_t) * o->V[i] * o->V[j];
            /* M<xi_ij> points from i to j */
            double sgn = i_is_first ? 1.0 : -1.0;
            const double *Md = o->finite ? o->My : o->M;
            for (int c = 0; c < 3; c++) fi[c] += t * sgn * Md[3 * b + c];
        }
        for (int c = 0; c < 3; c++) f[3 * i + c] = fi[c];
    }
}

/* Internal force f(u) for the current bond status (no breaking). */
void orc_force(orc_model *o, const double *u, double *f, double *theta_out) {
    compute_extensions(o, u);
    dilatation_and_force(o, f);
    if (theta_out) memcpy(theta_out, o->theta, sizeof(double) * o->n);
}

/* Strain energy sum_i V_i W_i with W_i = (K-G/3)/(2A) theta_i^2
 * + G/(2 m_i) sum_j rho w e^2 V_j (Eq. 1.20 written with K, G, A of
 * Eqs. 1.8, 1.15, 1.16). Uses the extensions and dilatations of the last
 * force evaluation. */
double orc_strain_energy_last(const orc_model *o) {
    double W = 0.0;
    #pragma omp parallel for schedule(static) reduction(+ : W)
    for (int64_t i = 0; i < o->n; i++) {
        const orc_spec *sp = &o->spec[o->sp[i]];
        double s = 0.0;
        for (int64_t k = o->aptr[i]; k < o->aptr[i + 1]; k++) {
            int64_t b = o->abond[k];
            if (!o->rho[b]) continue;
            int64_t j = (o->bi[b] == i) ? o->bj[b] : o->bi[b];
            s += o->e[b] * o->e[b] * o->V[j];
        }
        double Wi = (sp->K - sp->G / 3.0) / (2.0 * sp->A) * o->theta[i] * o->theta[i]
                    + sp->G / (2.0 * o->m[i]) * s;
        W += o->V[i] * Wi;
    }
    return W;
}

double orc_strain_energy(orc_model *o, const double *u) {
    compute_extensions(o, u);
    double *f = (double *)malloc(sizeof(double) * 3 * o->n);
    dilatation_and_force(o, f);
    free(f);
    return orc_strain_energy_last(o);
}

/* ------------------------------------------------------------------------ */
/* explicit time stepping                                                   */
/* ------------------------------------------------------------------------ */

/* Advance nsteps steps from step index o->step.  u, v: n*3 (in/out).
 * bc[n]: bit c = component c prescribed (zero acceleration).
 * fext: n*3 external force at full load; ramp_steps: r(n) = min(1, n/ramp)
 * (0: r = 1).  f_out (optional): internal force of the last step.
 * Each step: breaking check, dilatation, force, update (Eqs. 1.30, 2.3, 2.2,
 * 2.11, 2.12). */
int orc_run(orc_model *o, int64_t nsteps, double *u, double *v, const uint8_t *bc,
            const double *fext, int64_t ramp_steps, double *f_out) {
    int64_t n = o->n;
    double *f = (double *)malloc(sizeof(double) * 3 * n);
    for (int64_t it = 0; it < nsteps; it++) {
        int64_t step = o->step;
        double r = 1.0;
        if (ramp_steps > 0) r = step >= ramp_steps ? 1.0 : (double)step / (double)ramp_steps;
        break_bonds(o, u, step);
        dilatation_and_force(o, f);
        #pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; i++) {
            const orc_spec *sp = &o->spec[o->sp[i]];
            double mass = sp->rho * o->V[i];
            for (int c = 0; c < 3; c++) {
                double a = (f[3 * i + c] + fext[3 * i + c] * r) / mass;
                if (bc[i] & (1u << c)) a = 0.0;
                v[3 * i + c] = v[3 * i + c] + sp->dt * a;
                u[3 * i + c] = u[3 * i + c] + sp->dt * v[3 * i + c];
            }
        }
        o->step = step + 1;
    }
    if (f_out) memcpy(f_out, f, sizeof(double) * 3 * n);
    free(f);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* adaptive dynamic relaxation (quasi-static loading, Sec. 4 Example 4)      */
/* ------------------------------------------------------------------------ */

/* Fictitious density of the relaxation, one value per component.  The
 * relaxation is stable when lambda_ii >= dt^2/4 sum_j |K_ij| (the Gershgorin
 * condition of Kilic and Madenci's method), K = -df/du.  Writing the force
 * of Eq. 2.2 as
 *   f_i = sum_j c_ij M (M . (u_j - u_i)) + sum_j b_ij M (g_i + g_j),
 *   g_l = theta_l / m_l = sum_k gamma_lk M_lk . (u_k - u_l)        (Eq. 2.3)
 * with c_ij = G V_i V_j (1/m_i + 1/m_j), b_ij = (K - G/3) x V_i V_j and
 * gamma_lk = A x V_k / m_l^2 (w = 1, intact bonds), the triangle inequality
 * bounds the row sums of |K| term by term:
 *   lambda_(i,a) = dt^2/4 [ 2 sum_j c_ij |M_a| |M|_1 + |B_(i,a)| Gam_i
 *                           + sum_j |b_ij| |M_a| Gam_j ]
 * (K - G/3 is negative for small Poisson ratios),
 *   B_i = sum_j b_ij M_ij,  Gam_l = 2 sum_k gamma_lk |M_lk|_1.
 * A component whose bound is zero gets lambda = 1.  lam: n*3. */
void orc_adr_density(const orc_model *o, double dt, double *lam) {
    int64_t n = o->n;
    double *B = (double *)calloc(3 * n, sizeof(double));
    double *Gam = (double *)calloc(n, sizeof(double));
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        const orc_spec *sp = &o->spec[o->sp[i]];
        for (int64_t k = o->aptr[i]; k < o->aptr[i + 1]; k++) {
            int64_t b = o->abond[k];
            if (!o->rho[b]) continue;
            int64_t j = (o->bi[b] == i) ? o->bj[b] : o->bi[b];
            double sgn = (o->bi[b] == i) ? 1.0 : -1.0;
            const double *M = o->M + 3 * b;
            double x = o->xl[b];
            double bij = (sp->K - sp->G / 3.0) * x * o->V[i] * o->V[j];
            double gam = sp->A * x * o->V[j] / (o->m[i] * o->m[i]);
            double m1 = fabs(M[0]) + fabs(M[1]) + fabs(M[2]);
            for (int c = 0; c < 3; c++) B[3 * i + c] += bij * sgn * M[c];
            Gam[i] += 2.0 * gam * m1;
        }
    }
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        const orc_spec *sp = &o->spec[o->sp[i]];
        double acc[3] = {0.0, 0.0, 0.0};
        for (int64_t k = o->aptr[i]; k < o->aptr[i + 1]; k++) {
            int64_t b = o->abond[k];
            if (!o->rho[b]) continue;
            int64_t j = (o->bi[b] == i) ? o->bj[b] : o->bi[b];
            const double *M = o->M + 3 * b;
            double x = o->xl[b];
            double cij = sp->G * o->V[i] * o->V[j] * (1.0 / o->m[i] + 1.0 / o->m[j]);
            double bij = (sp->K - sp->G / 3.0) * x * o->V[i] * o->V[j];
            double m1 = fabs(M[0]) + fabs(M[1]) + fabs(M[2]);
            for (int c = 0; c < 3; c++) acc[c] += 2.0 * cij * fabs(M[c]) * m1 + fabs(bij) * fabs(M[c]) * Gam[j];
        }
        for (int c = 0; c < 3; c++) {
            double l = 0.25 * dt * dt * (acc[c] + fabs(B[3 * i + c]) * Gam[i]);
            lam[3 * i + c] = l > 0.0 ? l : 1.0;
        }
    }
    free(B);
    free(Gam);
}

/* Adaptive dynamic relaxation (Kilic and Madenci's form of the method of
 * Underwood), nsteps iterations of fictitious time step dt from (u, v):
 *   F^n = f(u^n) + F_ext r(n)        (breaking first, as in orc_run)
 *   first iteration (*iter == 0):  v = dt F^n / (2 lambda)
 *   later:  k_r = -(F_r^n - F_r^(n-1)) / (lambda_r dt v_r)   (v_r != 0)
 *           c = 2 sqrt(sum u_r k_r u_r / sum u_r^2) when positive, else 0
 *           v = ((2 - c dt) v + 2 dt F^n / lambda) / (2 + c dt)
 *   u += dt v
 * over the free components r; prescribed components keep v and advance u by
 * dt v (as in orc_run).  fprev (n*3) carries F^(n-1) between calls, *iter
 * the number of iterations done.  stats (4): c, sum u k u, sum u^2 and
 * sum F^2 over the free components, of the last iteration. */
int orc_adr_run(orc_model *o, int64_t nsteps, double *u, double *v, double *fprev, int64_t *iter,
                const double *lam, const uint8_t *bc, const double *fext, int64_t ramp_steps, double dt,
                double *stats) {
    int64_t n = o->n;
    double *f = (double *)malloc(sizeof(double) * 3 * n);
    for (int64_t it = 0; it < nsteps; it++) {
        int64_t step = o->step;
        double r = 1.0;
        if (ramp_steps > 0) r = step >= ramp_steps ? 1.0 : (double)step / (double)ramp_steps;
        break_bonds(o, u, step);
        dilatation_and_force(o, f);
        int first = (*iter == 0);
        double num = 0.0, den = 0.0, res = 0.0;
        /* serial, in component order: the damping is sensitive to rounding,
         * so the reference sums in one fixed order */
        for (int64_t q = 0; q < 3 * n; q++) {
            f[q] += fext[q] * r;
            if (bc[q / 3] & (1u << (q % 3))) continue;
            res += f[q] * f[q];
            if (!first && v[q] != 0.0) {
                double k = -(f[q] / lam[q] - fprev[q] / lam[q]) / (dt * v[q]);
                num += u[q] * k * u[q];
            }
            den += u[q] * u[q];
        }
        double c = 0.0;
        if (!first && den > 0.0 && num > 0.0) c = 2.0 * sqrt(num / den);
        #pragma omp parallel for schedule(static)
        for (int64_t q = 0; q < 3 * n; q++) {
            if (!(bc[q / 3] & (1u << (q % 3)))) {
                if (first) v[q] = dt * f[q] / (2.0 * lam[q]);
                else v[q] = ((2.0 - c * dt) * v[q] + 2.0 * dt * f[q] / lam[q]) / (2.0 + c * dt);
            }
            u[q] = u[q] + dt * v[q];
            fprev[q] = f[q];
        }
        stats[0] = c;
        stats[1] = num;
        stats[2] = den;
        stats[3] = res;
        *iter += 1;
        o->step = step + 1;
    }
    free(f);
    return 0;
}

/* Damage (Eq. 1.31), w = 1. */
void orc_damage(const orc_model *o, double *phi) {
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < o->n; i++) {
        double num = 0.0, den = 0.0;
        for (int64_t k = o->aptr[i]; k < o->aptr[i + 1]; k++) {
            int64_t b = o->abond[k];
            int64_t j = (o->bi[b] == i) ? o->bj[b] : o->bi[b];
            den += o->V[j];
            if (o->rho[b]) num += o->V[j];
        }
        phi[i] = den > 0.0 ? 1.0 - num / den : 0.0;
    }
}

/* ------------------------------------------------------------------------ */
/* largest eigenvalue of M^-1 K on the free degrees of freedom              */
/* ------------------------------------------------------------------------ */

static uint64_t splitmix64(uint64_t *s) {
    uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* Power iteration on K x = lambda M x, M = diag(rho V), K = -df/du, with
 * prescribed components held at zero.  Returns the final Rayleigh quotient
 * x'Kx / x'Mx (a lower bound of lambda_max that converges to it). */
double orc_lambda_max(orc_model *o, const uint8_t *bc, int iters, uint64_t seed) {
    int64_t n = o->n;
    double *x = (double *)malloc(sizeof(double) * 3 * n);
    double *f = (double *)malloc(sizeof(double) * 3 * n);
    uint64_t s = seed;
    for (int64_t k = 0; k < 3 * n; k++) {
        int c = (int)(k % 3);
        int64_t i = k / 3;
        double r = (double)(splitmix64(&s) >> 11) * (1.0 / 9007199254740992.0) - 0.5;
        x[k] = (c < o->dim && !(bc[i] & (1u << c))) ? r : 0.0;
    }
    double lam = 0.0;
    for (int it = 0; it < iters; it++) {
        orc_force(o, x, f, NULL);
        double xKx = 0.0, xMx = 0.0, nrm = 0.0;
        for (int64_t i = 0; i < n; i++) {
            double mass = o->spec[o->sp[i]].rho * o->V[i];
            for (int c = 0; c < 3; c++) {
                int64_t k = 3 * i + c;
                double kx = (c < o->dim && !(bc[i] & (1u << c))) ? -f[k] : 0.0;
                xKx += x[k] * kx;
                xMx += x[k] * mass * x[k];
                f[k] = kx / mass;          /* y = M^-1 K x */
                nrm += f[k] * f[k] * mass;
            }
        }
        lam = xKx / xMx;
        nrm = sqrt(nrm);
        if (!(nrm > 0.0)) break;
        for (int64_t k = 0; k < 3 * n; k++) x[k] = f[k] / nrm;
    }
    free(x); free(f);
    return lam;
}

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int t) {
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}
