/*
 * pd.h -- C ABI of the MI355X (gfx950) linearized ordinary state-based
 * peridynamics (OSB-PD) explicit solver.
 *
 * The operation the library performs is the explicit time stepping of the
 * discretized OSB-PD equation of motion of Ni, Zaccariotto, Zhu, Galvanetto,
 * "Matrix-based implementation and GPU acceleration of linearized ordinary
 * state-based peridynamic models in MATLAB": per step, bond stretch and the
 * critical-stretch breaking rule (Eqs. 1.17, 1.30), the nodal dilatation
 * (Eqs. 1.6, 2.3), the pair forces (Eq. 2.2) and the explicit update
 * (Eqs. 2.11, 2.12).  The internal force is available in three forms: a
 * matrix-free two-pass kernel over a bond list, the block-sparse global
 * stiffness matrix of Eq. 2.14 applied to the displacement, and the
 * paper's factored matrix scheme (four stored sparse operators C_e,
 * C_theta, K_theta, K_e of Eqs. 2.4-2.10 applied in turn).
 *
 * Conventions
 *  - Every function returns a pd_status; PD_OK = 0, errors are negative.
 *    No exception, abort or exit crosses the ABI.  On error a message is
 *    kept in the context (pd_last_error).  Argument errors are detected
 *    before any device work is enqueued.
 *  - Host pointers are marked [host], device pointers [device].  The caller
 *    owns every buffer it passes; the library owns only the pd_ctx object
 *    (stream handle, captured graphs, a small pinned report buffer and a
 *    small device scratch block) and frees it in pd_ctx_destroy.
 *  - Device work is enqueued on the stream given to pd_ctx_create and is
 *    asynchronous unless stated otherwise.
 *  - Nodes are given in the caller's order; pd_build_family chooses an
 *    internal row order (tile-major) and returns the permutation.  All
 *    device arrays are in internal row order and padded to n_pad rows
 *    (a multiple of 64); padding rows carry no bonds and no mass.
 *  - Units are SI.  2D problems use a thickness of 1 m (volumes dx^2 * 1).
 *  - The influence function is w = 1 (the paper's choice, Sec. 2.3).
 */
#ifndef PD_H
#define PD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PD_OK = 0,
    PD_ERR_ARG = -1,         /* invalid argument (null pointer, bad value)       */
    PD_ERR_SIZE = -2,        /* size mismatch or a size above a stated maximum   */
    PD_ERR_HIP = -3,         /* a HIP runtime call failed                        */
    PD_ERR_UNSTABLE = -4,    /* non-finite displacement detected                 */
    PD_ERR_UNSUPPORTED = -5, /* option combination not implemented              */
    PD_ERR_STATE = -6        /* call out of order (e.g. K not assembled)         */
} pd_status;

typedef enum { PD_3D = 0, PD_PLANE_STRESS = 1, PD_PLANE_STRAIN = 2 } pd_mode;
typedef enum { PD_FP64 = 0, PD_FP32_RECHECK = 1 } pd_precision;
typedef enum { PD_MATRIX_FREE = 0, PD_BSR = 1, PD_FACTORED = 2 } pd_form;

/* Largest supported sizes. */
#define PD_MAX_NODES (1LL << 25)  /* node index is stored in 25 bits            */
#define PD_MAX_STENCIL 127        /* distinct bond offsets; id 127 = padding    */
#define PD_MAX_SPECIMENS 65535
#define PD_MAX_CUTS 65536

typedef struct pd_ctx pd_ctx;

/* ------------------------------------------------------------------------ */
/* context                                                                  */
/* ------------------------------------------------------------------------ */

/* Create a context bound to HIP device 'device' and stream 'hip_stream'
 * (a hipStream_t; NULL = the default stream).  Returns PD_ERR_HIP if the
 * device cannot be selected or is not gfx950. */
pd_status pd_ctx_create(pd_ctx **ctx, int device, void *hip_stream);
pd_status pd_ctx_destroy(pd_ctx *ctx);
/* Last error message of the context ("" if none); valid until the next call. */
const char *pd_last_error(const pd_ctx *ctx);
/* Library version string. */
const char *pd_version(void);

/* ------------------------------------------------------------------------ */
/* material constants (host)                                                */
/* ------------------------------------------------------------------------ */

/* Critical stretch s_c.  3D: Eq. 1.26 with beta = 125 delta / 1848 and
 * beta' of Eq. 1.27 (variant 0: as printed, 5 delta / (24 pi); variant 1:
 * 5 delta / 24, the value the varpi quadrature gives).  Plane stress and
 * plane strain: Eq. 1.28 with Eq. 1.29.  G0 <= 0, NaN or inf gives
 * *s0 = +inf (bonds never break).  PD_ERR_ARG for nu outside (-1, 0.5),
 * E <= 0, delta <= 0 or s0 == NULL. */
pd_status pd_critical_stretch(pd_mode mode, double E, double nu, double G0, double delta,
                              int variant, double *s0);

/* Per-specimen constants as the kernels read them (64 bytes, device table
 * of n_specimens entries, built with pd_specimen_params). */
typedef struct pd_spec {
    double kp;   /* K - G/3 with K of Eq. 1.15, G of Eq. 1.16          */
    double G;    /* G of Eq. 1.16                                       */
    double A;    /* A of Eq. 1.8                                        */
    double rho;  /* mass density                                        */
    double s0;   /* critical stretch (Eq. 1.30 threshold; inf = never)  */
    double dt;   /* time step of this specimen                          */
    double pad[2];
} pd_spec;

/* Fill *out from (mode, E, nu, rho, s0, dt): kp, G, A from Eqs. 1.8,
 * 1.15, 1.16 with kappa = E/(3(1-2nu)), mu = E/(2(1+nu)).  PD_ERR_ARG on
 * E <= 0, nu outside (-1, 0.5), rho <= 0, dt <= 0 or NaN s0. */
pd_status pd_specimen_params(pd_mode mode, double E, double nu, double rho, double s0,
                             double dt, pd_spec *out);

/* ------------------------------------------------------------------------ */
/* family (host, set-up)                                                    */
/* ------------------------------------------------------------------------ */

/* The body: nodes on a uniform lattice (all examples of the paper use
 * uniform grids, Sec. 4).  Node p sits at origin + dx * lat[p]. */
typedef struct pd_body {
    int64_t n;                 /* number of nodes (1 .. PD_MAX_NODES)                  */
    int32_t dim;               /* 2 or 3                                               */
    int32_t pad0;
    const int32_t *lat;        /* [host] n*dim integer lattice coordinates             */
    double dx;                 /* lattice spacing > 0                                   */
    double origin[3];          /* position of lattice point (0,0,0)                     */
    double delta;              /* horizon radius > 0 (family: 0 < |xi| <= delta, Sec. 2.1) */
    const double *vol;         /* [host] n node volumes > 0                            */
    const int32_t *specimen;   /* [host] n specimen ids in [0, PD_MAX_SPECIMENS) or NULL (all 0);
                                  bonds never join different specimens               */
} pd_body;

/* A notch: bonds whose straight segment properly crosses the patch start
 * broken (bond status 0 of Eq. 1.30).
 *   kind 0 segment (2D):    p = {ax, ay, bx, by}
 *   kind 1 parallelogram:   p = {c(3), a(3), b(3)}, patch {c + s a + t b : 0 < s,t < 1}
 *   kind 2 helicoidal strip about the z axis: p = {zc, pitch, r_in, r_out, th0, th1};
 *          crossing of psi = (z - zc) - pitch * atan2(y, x) along the bond, with
 *          the linearly interpolated crossing inside r_in < r < r_out, th0 < theta < th1.
 * specimen >= 0 restricts the notch to that specimen. */
typedef struct pd_cut {
    int32_t kind;
    int32_t specimen;
    double p[10];
} pd_cut;

typedef struct pd_family_sizes {
    int64_t n;          /* nodes                                                  */
    int64_t n_pad;      /* rows incl. padding (multiple of 64)                    */
    int64_t n_slices;   /* n_pad / 64                                              */
    int64_t n_words;    /* bond words incl. padding                                */
    int64_t n_mask;     /* 64-bit bond-status words = n_words / 64                 */
    int64_t nnz;        /* directed bonds                                          */
    int64_t n_bonds;    /* unique bonds = nnz / 2                                  */
    int64_t n_cut;      /* unique bonds removed by notches                         */
    int32_t n_stencil;  /* distinct bond offsets                                   */
    int32_t max_row;    /* largest family size                                     */
    int32_t dim;
    int32_t n_specimens;/* 1 + largest specimen id                                 */
    int64_t n_tiles;    /* lattice tiles = n_slices                                */
    int32_t tile[3];    /* tile edge lengths in lattice units (product 64)         */
    int32_t words_per_row; /* bond words per row = n_stencil rounded up to 4      */
    int32_t reach;      /* largest |component| of a stencil offset                 */
    int32_t n_halo;     /* slots of a tile's LDS halo box (tile + reach on every
                           side, x pitch padded; see pd_family_host.halo_map)      */
    int32_t n_box;      /* points of that box (tile + reach on every side) that
                           some stencil entry of some tile point reaches; see
                           pd_family_host.halo_pos                                 */
    float vol_uniform;  /* the node volume as float when every node has the same
                           one (then the FP32 tile kernels take it as a constant
                           instead of staging it per point), else 0               */
    int32_t pad_vu;
} pd_family_sizes;

/* Output arrays of pd_build_family, all [host], allocated by the caller
 * with the sizes from the query call. */
typedef struct pd_family_host {
    int32_t *perm;        /* [n_pad] caller node of internal row r, -1 for padding   */
    int32_t *row_of;      /* [n] internal row of caller node p                       */
    int64_t *slice_ptr;   /* [n_slices+1] first bond word of each 64-row slice       */
    uint32_t *words;      /* [n_words] (j << 7) | stencil id; id 127 = padding       */
    uint64_t *mask;       /* [n_mask] initial bond status, bit lane of word k of a
                             slice = status of bond k of row 64*slice + lane         */
    double *stencil;      /* [n_stencil*4] M1, M2, M3, x per bond offset (Eqs. 1.5, 1.13) */
    int32_t *stencil_off; /* [n_stencil*3] lattice offset of each stencil entry:
                             shortest first, entry 2m+1 the opposite of entry 2m    */
    double *vol;          /* [n_pad] node volume (0 for padding)                     */
    double *inv_m;        /* [n_pad] 1 / m, m of Eq. 1.9 over the full family        */
    int32_t *spec;        /* [n_pad] specimen id (0 for padding)                     */
    int32_t *lat4;        /* [n_pad*4] lattice coordinates x,y,z,0 per row           */
    int32_t *tile_org;    /* [n_tiles*4] lattice origin x,y,z of each tile, specimen */
    int32_t *tile_nbr;    /* [n_tiles*27] tile at offset (dx,dy,dz) in {-1,0,1}^3,
                             index (dz+1)*9 + (dy+1)*3 + (dx+1); -1 if absent        */
    uint32_t *ktab;       /* [128*20] per-entry tables of the LDS-staged kernels, zero
                             beyond n_stencil.  Rows 0-127, 8 words each: M1, M2, M3,
                             x as float, the int32 offset of the entry's neighbour in
                             the tile's LDS halo box, 1/x as float, 0, 0.  Then rows
                             of 4 words from word 1024: x M1, x M2, x M3 as float, the
                             same int32 offset.  Then rows of 8 words from word 1536:
                             M1/x, M2/x, x^2, x M1, x M2 as float, the int32 offset
                             of the neighbour in the single-precision box (the
                             pitches of halo_pos), M3/x, x M3 as float               */
    int16_t *halo_map;    /* [n_halo] for slot s of the LDS halo box (x fastest):
                             64 * d + l, the point at local position l of the
                             neighbour tile in direction d (tile_nbr index), or -1
                             for x-pitch padding; the same for every tile          */
    int32_t *halo_pos;    /* [n_box] for each point of the unpadded box that a
                             stencil entry of a tile point reaches, in box order
                             (x fastest): (slot << 11) | (64 * d + l), d and l as
                             in halo_map and
                             slot the point's place in the single-precision pass-1
                             box, whose x and y pitches are padded so that the 64
                             lanes of a tile read 64 distinct LDS banks            */
} pd_family_host;

/* Horizon search and bond-list construction (Sec. 2.1 family; Eqs. 1.2-1.5,
 * 1.9, 1.13 per bond; notch cuts).  Two-phase: with bufs == NULL only
 * *sizes is filled; call again with every array of bufs allocated.
 * The lattice of each specimen is cut into tiles of 64 lattice points
 * (tile[0] x tile[1] x tile[2], chosen among a few shapes to leave the
 * fewest empty points); every tile holding a node is one 64-row slice,
 * row 64*t + (x + tile[0]*(y + tile[1]*z)) for local lattice position
 * (x, y, z), so a wave64 owns one tile and lanes sit on lattice points.
 * Empty points are padding rows.  Bond k of every row is stencil entry k
 * (a fixed lattice offset), present or not: absent neighbours are padding
 * words (status bit 0).  Within a slice the words are interleaved in
 * groups of four per lane (see the kernels), so a wave reads 1 KiB of
 * consecutive memory per group.  Errors: PD_ERR_ARG (null/invalid body,
 * duplicate lattice points, unknown cut kind), PD_ERR_SIZE (n, stencil or
 * lattice extent above the maxima). */
pd_status pd_build_family(const pd_body *body, const pd_cut *cuts, int32_t ncuts,
                          pd_family_sizes *sizes, pd_family_host *bufs);

/* Super-tiles of a family of 4x4x4 tiles (3D) or 8x8 tiles (2D) with
 * stencil reach <= 3: the tiles grouped 2 x 2 (x 1) (same specimen, same
 * tile layer), so that one workgroup stages one halo box for four tiles
 * (8 x 8 x 4 or 16 x 16 lattice points plus the reach on every side) and
 * each of its four waves sweeps the whole stencil for its own tile.  Two-phase like pd_build_family (with
 * st_tiles == NULL only *out is set).  Outputs [host]:
 *   st_tiles [4 n_st]   tile of quadrant q (x offset 4 (q & 1), y offset
 *                       4 (q >> 1)) of super-tile s at 4 s + q, -1 if none;
 *                       super-tiles in (specimen, z, y, x) order
 *   st_nbr  [48 n_st]   tile at tile offset (dx, dy, dz) in {-1..2}^2 x {-1..1}
 *                       from the super-tile's first tile, index
 *                       (dx + 1) + 4 (dy + 1) + 16 (dz + 1), -1 if none (2D:
 *                       only dz = 0)
 *   st_pos  [n_pos]     the box points some stencil entry of some tile point
 *                       reaches, x fastest: (slot << 12) | (64 d + l), d the
 *                       st_nbr index of the point's tile and l its place in it,
 *                       slot = x + 16 y + 228 z in the 3D box, x + 40 y in the
 *                       2D box (pitches chosen so that the lanes of a tile
 *                       reading the same offset hit distinct LDS banks)
 *   st_ktab [128*8]     per stencil entry: M1/x, M2/x, x^2, x M1, x M2 as float,
 *                       the int32 offset of the neighbour in that box, M3/x,
 *                       x M3 as float (zero beyond n_stencil)
 * Errors: PD_ERR_ARG (NULL arguments), PD_ERR_UNSUPPORTED (tiles other than
 * 4x4x4 in 3D or 8x8 in 2D, or reach above 3). */
typedef struct pd_st_sizes {
    int64_t n_st;            /* super-tiles                                        */
    int32_t n_pos;           /* reached box points                                 */
    int32_t pad0;
} pd_st_sizes;

pd_status pd_build_supertiles(const pd_family_sizes *sizes, const pd_family_host *fam, pd_st_sizes *out,
                              int32_t *st_tiles, int32_t *st_nbr, int32_t *st_pos, uint32_t *st_ktab);

/* ------------------------------------------------------------------------ */
/* device descriptors                                                       */
/* ------------------------------------------------------------------------ */

/* The problem: family arrays uploaded by the caller, plus per-row data. */
typedef struct pd_problem_dev {
    int64_t n_pad;
    int64_t n_slices;
    int32_t dim;
    int32_t n_stencil;
    int32_t n_specimens;
    int32_t pad0;
    const int64_t *slice_ptr; /* [device] n_slices+1                              */
    const uint32_t *words;    /* [device] n_words                                 */
    const double *stencil;    /* [device] n_stencil*4                             */
    const double *vol;        /* [device] n_pad                                   */
    const double *inv_m;      /* [device] n_pad                                   */
    const int32_t *lat4;      /* [device] n_pad*4 (needed by pd_assemble_K only)   */
    const pd_spec *spec;      /* [device] n_specimens                             */
    const uint32_t *aux;      /* [device] n_pad, written by pd_state_init          */
    const double *fext;       /* [device] n_pad*4 external force at full load      */
    int64_t ramp_steps;       /* load factor r(n) = min(1, n / ramp_steps); 0: r = 1 */
    /* tile description for the LDS-staged kernels (NULL tile_nbr: not used) */
    const int32_t *stencil_off; /* [device] n_stencil*3 lattice offsets            */
    const int32_t *tile_nbr;    /* [device] n_slices*27 neighbour tiles            */
    int32_t tile[3];            /* tile edge lengths (pd_family_sizes.tile)        */
    int32_t reach;              /* pd_family_sizes.reach                           */
    const uint32_t *ktab;       /* [device] 128*20 words, pd_family_host.ktab      */
    const int16_t *halo_map;    /* [device] n_halo, pd_family_host.halo_map        */
    const int32_t *halo_pos;    /* [device] n_box, pd_family_host.halo_pos         */
    int32_t n_pos;              /* pd_family_sizes.n_box                           */
    float vol_uniform;          /* pd_family_sizes.vol_uniform, or 0 (every kernel
                                   reads the volumes); if nonzero it must equal the
                                   float of every node's vol: the FP32 tile kernels
                                   check the points they stage, and a mismatch fails
                                   the next report or check of pd_step (PD_ERR_ARG) */
    /* super-tiles (pd_build_supertiles; NULL st_tiles: not used)                 */
    const int32_t *st_tiles;    /* [device] 4 n_st                                 */
    const int32_t *st_nbr;      /* [device] 48 n_st                                */
    const int32_t *st_pos;      /* [device] st_n_pos                               */
    const uint32_t *st_ktab;    /* [device] 128*8 words                            */
    int64_t n_st;
    int32_t st_n_pos;
    int32_t pad2;
} pd_problem_dev;

/* Device control block (step counter, diagnostics, the shadow maxima of the
 * FP32 path spread over 128 cache lines).  Size in bytes, 256-aligned: */
#define PD_CTL_BYTES 16640

/* Solver state, [device] arrays in internal row order. */
typedef struct pd_state_dev {
    double *uv[2];      /* n_pad*4: (u_x, u_y, u_z, V) ping-pong                   */
    double *vel;        /* n_pad*4 allocated: per row (v_x, v_y, v_z) packed in the
                           first n_pad*3 in 3D, (v_x, v_y) in the first n_pad*2 in
                           2D (the per-row vectors below marked "per row, by dim"
                           follow the same rule)                                     */
    double *qr;         /* n_pad*2: (theta/m, 1/m)                                  */
    uint64_t *mask;     /* n_mask bond status bits (mutable: bonds break)           */
    int32_t *ush[2];    /* n_pad*4 fixed-point displacement shadow (FP32 path)      */
    float *qr32;        /* n_pad*2 (theta/m, 1/m) in FP32 (FP32 path)               */
    double *dsum;       /* n_pad*4 sum over intact bonds of x M V_j, per row, by dim
                           (FP32 path)                                               */
    float *fe32;        /* n_pad*4 deviatoric part of the pair force of the step,
                           carried from pass 1 to pass 2, per row, by dim (FP32
                           LDS-staged path)                                          */
    double *fe64;       /* n_pad*4 the same for the FP64 LDS-staged path, per row, by
                           dim (NULL: the FP64 path uses the gather kernels)        */
    float *qv32;        /* n_pad*2 (theta/m, V) of the step in FP32, written by the
                           FP32 LDS-staged pass 1 for its pass 2 (NULL: the FP32
                           path uses the gather kernels)                             */
    void *ctl;          /* PD_CTL_BYTES control block                               */
    int32_t cur;        /* index of uv (and ush) holding the current state          */
    int32_t pad0;
} pd_state_dev;

/* Initialise a state and the per-row aux/fext arrays from caller-order
 * inputs [device]: u0, v0, fext0 (n*3 doubles each, any may be NULL = 0),
 * bc (n bytes: bit c set = displacement component c prescribed: zero
 * acceleration, velocity held at v0), perm (n_pad, from pd_build_family).
 * aux and fext are the arrays later referenced by prob->aux / prob->fext
 * (passed here as writable pointers).  Sets the step counter to
 * 'start_step'.  The mask is not touched (copy the initial mask in). */
pd_status pd_state_init(pd_ctx *ctx, const pd_problem_dev *prob, const int32_t *perm,
                        int64_t n, const double *u0, const double *v0, const uint8_t *bc,
                        const double *fext0, const int32_t *spec_rows, uint32_t *aux_out,
                        double *fext_out, pd_state_dev *st, int64_t start_step);

/* Copy the current displacement and velocity back to caller order [device]
 * (n*3 doubles each; either may be NULL). */
pd_status pd_state_read(pd_ctx *ctx, const pd_problem_dev *prob, const int32_t *perm,
                        int64_t n, const pd_state_dev *st, double *u_out, double *v_out);

/* Read the step counter (synchronises the stream). */
pd_status pd_get_step(pd_ctx *ctx, const pd_state_dev *st, int64_t *step);

/* Whether pd_step / pd_force with opts.kernel = 0 run the LDS-staged tile
 * kernels for this problem, state and precision (*yes = 1) or the gather
 * kernels (*yes = 0).  Host only, no device work. */
pd_status pd_tile_kernels_apply(const pd_problem_dev *prob, const pd_state_dev *st, int32_t precision,
                                int32_t *yes);

/* ------------------------------------------------------------------------ */
/* the force operator                                                       */
/* ------------------------------------------------------------------------ */

/* Internal force f = F(u) (Eqs. 2.3 then 2.2) for the current displacement
 * of 'st' and bond status 'mask', without breaking and without updating.
 * Outputs [device], internal order: f (n_pad*4, f_x f_y f_z 0) and theta
 * (n_pad, dilatation of Eq. 1.6); theta may be NULL.  precision selects
 * the double kernels or the single-precision force kernels of the
 * FP32_RECHECK path (which then also rebuild the shadow state st->ush,
 * st->qr32 and st->dsum from the double displacement).  Uses st->qr and
 * st->fe64 (or st->qr32 and st->fe32) as scratch. */
pd_status pd_force(pd_ctx *ctx, const pd_problem_dev *prob, pd_state_dev *st, int32_t precision,
                   double *f, double *theta);

/* The same force with the finite extension and the deformed direction of
 * Eqs. 1.10, 1.13 (e = |Y| - x, Y = x M + u_j - u_i, pair force of Eq. 2.2
 * along Y/|Y|), in double precision (tile kernels when the family allows
 * them and st->fe64 is set, else gather kernels).  Uses st->qr and st->fe64
 * as scratch.  Errors as pd_force. */
pd_status pd_force_finite(pd_ctx *ctx, const pd_problem_dev *prob, pd_state_dev *st, double *f, double *theta);

/* ------------------------------------------------------------------------ */
/* explicit stepping                                                        */
/* ------------------------------------------------------------------------ */

typedef struct pd_step_opts {
    int32_t precision;   /* pd_precision                                             */
    int32_t form;        /* pd_form                                                  */
    int32_t graph_chunk; /* >0: capture this many steps in a hipGraph and replay it   */
    int32_t block;       /* threads per block (64, 128 or 256) or 0 = 256           */
    int32_t check_every; /* >0: check the non-finite flag every this many steps (sync) */
    int32_t profile;     /* 1: time every kernel with HIP events on the stream (eager
                            launches, one synchronisation per step); see pd_profile_read */
    int32_t kernel;      /* matrix-free kernels: 0 = LDS-staged tile kernels when the
                            family allows them (tile edges >= stencil reach; FP64 also
                            needs st->fe64), else gather kernels; 1 = gather kernels;
                            2 = tile kernels, one tile per workgroup (3D) or per
                            wave (2D) (error if not possible); 3 = FP32 super-tile
                            kernels (four tiles per workgroup sharing one halo box,
                            pd_build_supertiles; error if not possible; the FP64
                            path then uses the tile kernels); 4 = tile kernels with
                            one tile per workgroup in 2D too (its four waves split
                            the stencil; in 3D the same as 2)                       */
    int32_t extension;   /* 0: linearized e = M.(u_j - u_i) along M (Eqs. 2.4, 2.7);
                            1: finite e = |x M + u_j - u_i| - x with the pair force
                            along the deformed bond (Eqs. 1.10, 1.13): PD_FP64,
                            PD_MATRIX_FREE; double tile kernels or, with kernel = 1
                            or a family they do not fit, gather kernels            */
    int32_t energy_check;/* 1: at every check (every check_every steps, and at the end
                            of the call) compute the kinetic energy 1/2 sum rho V v.v
                            and the strain energy sum V_i W_i of Eq. 1.20 (in double,
                            from the double state, with the extension of the step;
                            fixed-order reductions, so the values are the same on
                            every run), and stop with PD_ERR_UNSTABLE when their sum
                            exceeds energy_growth times the sum of the previous
                            check of this state (pd_state_init clears the history).
                            The first use allocates a small reduction buffer in the
                            context (4 doubles per 256 rows).  0: no energies      */
    int32_t pad0;
    double energy_growth;/* growth factor of the energy check; <= 0 means 1e3. An
                            explicit step beyond the stability limit multiplies the
                            energy of its unstable mode several times per step, while
                            loading grows it like a low power of time          */
} pd_step_opts;

/* Kernel timings gathered by pd_step with opts->profile = 1 (milliseconds,
 * summed over the profiled steps).  pass1: breaking + dilatation kernel
 * (breaking-only kernel in the block form); pass2: force + update kernel
 * (block product + update in the block form); extra: everything else the
 * steps launched (block re-assembly). */
typedef struct pd_profile_stats {
    int64_t steps;
    double ms_pass1;
    double ms_pass2;
    double ms_extra;
} pd_profile_stats;

/* Read (and with reset != 0 clear) the context's accumulated timings. */
pd_status pd_profile_read(pd_ctx *ctx, pd_profile_stats *out, int32_t reset);

/* Launch-shape tuning of the matrix-free step.  Candidates: the LDS-staged
 * tile kernels (when the family allows them) and the gather kernels at 64,
 * 128 and 256 threads per block, in the given precision.  Each candidate
 * runs 2 untimed and 'trial_steps' timed steps (HIP events on the stream)
 * on the given state, which therefore advances by 2 + trial_steps per
 * candidate (reset it afterwards).  The gather kernels give results
 * independent of the block size; tile and gather kernels differ in the
 * order of the force sums.  out->kernel / out->block are the pd_step_opts
 * values to use. */
typedef struct pd_tune_result {
    int32_t kernel;            /* best pd_step_opts.kernel                        */
    int32_t block;             /* best pd_step_opts.block                         */
    int32_t n_candidates;
    int32_t pad0;
    double ms_per_step;        /* best time                                       */
    int32_t cand_kernel[8];
    int32_t cand_block[8];
    double cand_ms[8];         /* time per step of each candidate                 */
} pd_tune_result;

pd_status pd_autotune(pd_ctx *ctx, const pd_problem_dev *prob, pd_state_dev *st, int32_t precision,
                      int32_t trial_steps, pd_tune_result *out);

typedef struct pd_step_report {
    int64_t step;           /* step counter after the call                           */
    int64_t broken_total;   /* directed bond-status bits cleared by breaking so far   */
    int64_t rechecks;       /* FP64 rechecks performed by the FP32 path so far        */
    int32_t nonfinite;      /* 1 if a non-finite displacement was produced            */
    int32_t pad0;
    double umax;            /* max |u| component at the end                           */
    double min_margin;      /* smallest |s - s_c| / s_c (Eqs. 1.17, 1.30) among the bonds
                               whose breaking the FP32 path decided in double precision
                               (rechecks and shadow fallbacks) since pd_state_init,
                               rounded to float; +inf if none (and on the FP64 paths,
                               whose every decision is taken in double)               */
    double kinetic;         /* energies of the last energy check (opts.energy_check),  */
    double strain;          /* Eq. 1.20; 0 if none since pd_state_init                 */
    int64_t energy_step;    /* step counter at that check; -1 if none                  */
} pd_step_report;

/* Advance 'nsteps' explicit steps.  Each step n (t_n = n dt):
 *   1. breaking: for every intact bond, e = M.(u_j - u_i) (Eqs. 2.4, 2.7),
 *      s = e/x (Eq. 1.17); s >= s0 clears the bond status (Eq. 1.30) for
 *      good.  FP64: decided in double with e evaluated as
 *      (M1 eta1 + M2 eta2) + M3 eta3 without contraction.  FP32_RECHECK:
 *      decided in float outside a proven error band around s0, by the same
 *      double expression inside it.
 *   2. dilatation theta_i (Eq. 2.3 summed over intact bonds);
 *   3. force f_i (Eq. 2.2), or with PD_BSR f = K u with K of Eq. 2.14
 *      (assembled by pd_assemble_K, re-assembled on rows near new breaks);
 *   4. update (Eqs. 2.11, 2.12): a = (f + F_ext r(n)) / (rho V), zero on
 *      prescribed components; v += dt a; u += dt v.
 * 'rep' (may be NULL) is filled after synchronising the stream; with
 * rep == NULL, check_every == 0 and energy_check == 0 the call is fully
 * asynchronous.  The FP32_RECHECK matrix-free path keeps its fixed-point
 * displacement shadow, the shadow scale and the row constants D_i in the
 * state between calls, so a trajectory is the same bits however its steps
 * are split across calls (for one kernel kind); they are rebuilt from the
 * double state whenever another path, pd_state_init, a solve or a kernel
 * kind change has touched the state since.  After changing the state or
 * the bond status from the host, call pd_state_init.
 * Errors: PD_ERR_ARG, PD_ERR_UNSUPPORTED (PD_BSR without K, unknown
 * option, PD_FACTORED: use pd_fac_step), PD_ERR_UNSTABLE (non-finite state
 * seen at a check, or energy growth beyond opts.energy_growth at an energy
 * check; the state is left as the last step produced it), PD_ERR_HIP. */
struct pd_bsr_dev;
pd_status pd_step(pd_ctx *ctx, const pd_problem_dev *prob, pd_state_dev *st, int64_t nsteps,
                  const pd_step_opts *opts, struct pd_bsr_dev *K, pd_step_report *rep);

/* ------------------------------------------------------------------------ */
/* block-sparse stiffness (Eq. 2.14)                                        */
/* ------------------------------------------------------------------------ */

/* Block pattern of K (host): row i holds a block for every node q != i that
 * is reachable through at most two bonds (the dilatation of a neighbour
 * couples nodes up to 2 delta apart, Eqs. 2.8, 2.10, 2.14).  Two-phase like
 * pd_build_family: with col == NULL only *sizes is set.  row_ptr [n_pad+1],
 * col [nnzb] (sorted per row), both [host]. */
typedef struct pd_bsr_sizes {
    int64_t nnzb;            /* blocks                                               */
    int32_t max_row_blocks;  /* largest row                                          */
    int32_t reach;           /* largest |lattice offset component| of a block        */
} pd_bsr_sizes;

pd_status pd_bsr_pattern(const pd_family_sizes *sizes, const pd_family_host *fam,
                         pd_bsr_sizes *out, int64_t *row_ptr, int32_t *col);

typedef struct pd_bsr_dev {
    int64_t nnzb;
    int32_t dim;            /* block size (2 or 3)                                     */
    int32_t fp32;           /* values stored as float (1) or double (0)                */
    int32_t max_row_blocks; /* from pd_bsr_pattern                                     */
    int32_t reach;          /* from pd_bsr_pattern                                     */
    const int64_t *row_ptr; /* [device] n_pad+1                                        */
    const int32_t *col;     /* [device] nnzb                                           */
    void *vals;             /* [device] nnzb*dim*dim; the blocks of row i fill entries
                               [row_ptr[i], row_ptr[i+1]) * dim*dim, entry (r, s) of the
                               row's block slot t at row_ptr[i]*dim*dim
                               + (r*dim + s)*nblk_i + t (component-major by row)       */
    double *bc;             /* [device] n_pad*8 scratch: per-node sums B_i, C_i        */
    uint32_t *dirty;        /* [device] n_pad flags of rows to re-assemble (zeroed)     */
    int32_t assembled;      /* set by pd_assemble_K                                    */
    int32_t pad0;
} pd_bsr_dev;

/* Assemble the off-diagonal blocks Kt_iq of the restoring operator in
 * difference form, f_i = sum_{q != i} Kt_iq (u_q - u_i), which equals
 * F_int = (K^v + K^d) U of Eq. 2.14 (K^v from Eqs. 2.8, 2.10, 2.7 and K^d
 * from Eqs. 2.9, 2.7) for the bond status 'mask'.  Every row is assembled.
 * Device-side and asynchronous; K->vals etc. caller-allocated. */
pd_status pd_assemble_K(pd_ctx *ctx, const pd_problem_dev *prob, const uint64_t *mask,
                        pd_bsr_dev *K);

/* f = Kt u for the current displacement of st (internal order, n_pad*4). */
pd_status pd_bsr_apply(pd_ctx *ctx, const pd_problem_dev *prob, const pd_bsr_dev *K,
                       const pd_state_dev *st, double *f);

/* ------------------------------------------------------------------------ */
/* factored matrix scheme (Eqs. 2.4-2.10; solver loop of Appendix B)        */
/* ------------------------------------------------------------------------ */

/* The four global operators of the matrix-based scheme, stored as sparse
 * matrices and applied in the paper's order every step:
 *   E     = C_e U              (N_b x dim N; Eqs. 2.4, 2.7)
 *   Theta = C_theta E          (N x N_b;     Eqs. 2.6, 2.10)
 *   F     = K_theta Theta + K_e E  (dim N x N and dim N x N_b; Eqs. 2.5, 2.8, 2.9)
 * Bonds are numbered 0..N_b-1 in the order of their owning directed entry
 * (the entry whose stencil id k is below that of its reverse) in the bond
 * word layout of the family.  Layouts (internal row order):
 *   C_e      row b: blocks at columns i = bond_ij[2b], j = bond_ij[2b+1]
 *            (owner row i), values ce[c*nb + b] for c < dim (block i, = -M)
 *            and ce[(dim+c)*nb + b] (block j, = +M), M the unit vector i->j.
 *   C_theta, K_e  share one pattern: row i holds one entry per directed bond
 *            position p of row i (the family's bond words, padding positions
 *            included with value 0); its column is the bond id bid[p];
 *            values cth[p] and ke[c*n_words + p].
 *   K_theta  diagonal block kth_diag[4 i + c] plus one off-diagonal entry per
 *            directed position p of row i with column words[p] >> 7 (the
 *            neighbour row) and values kth[c*n_words + p].
 * Breaking (Eq. 1.30) clears the bond status bits and zeroes E_b; C_theta
 * and K_e then need no change, while the rows of K_theta of both ends of a
 * newly broken bond are re-assembled in the same step. */
typedef struct pd_fac_sizes {
    int64_t nb;              /* unique bonds N_b                                     */
    int64_t n_words;         /* directed positions (pd_family_sizes.n_words)          */
} pd_fac_sizes;

/* Bond numbering and index arrays (host, two-phase like pd_build_family:
 * with bond_ij == NULL only *out is set).  bond_ij [2 nb]: owner row and
 * neighbour row of each bond; bond_pos [2 nb]: word position of the owner
 * entry of bond b at b, of its reverse entry at nb + b (the step reads the
 * first half only); bid [n_words]: bond id of every position
 * (0 at padding positions).  Errors: PD_ERR_ARG (NULL arrays, a family whose
 * bond words are not symmetric), PD_ERR_SIZE (n_words >= 2^31). */
pd_status pd_fac_pattern(const pd_family_sizes *sizes, const pd_family_host *fam, pd_fac_sizes *out,
                         int32_t *bond_ij, int32_t *bond_pos, int32_t *bid);

typedef struct pd_fac_dev {
    int64_t nb;              /* unique bonds, from pd_fac_pattern                     */
    int64_t n_words;         /* directed positions, from pd_fac_pattern               */
    int32_t dim;             /* 2 or 3                                                 */
    int32_t assembled;       /* set by pd_fac_assemble                                 */
    const int32_t *bond_ij;  /* [device] 2 nb   (pattern)                              */
    const int32_t *bond_pos; /* [device] 2 nb   (pattern)                              */
    const int32_t *bid;      /* [device] n_words (pattern)                             */
    double *ce;              /* [device] 2 dim nb   C_e values                         */
    double *xi;              /* [device] nb         bond lengths |xi| (Eq. 1.5)         */
    double *cth;             /* [device] n_words    C_theta values                     */
    double *ke;              /* [device] dim n_words K_e values                        */
    double *kth;             /* [device] dim n_words K_theta off-diagonal values        */
    double *kth_diag;        /* [device] 4 n_pad    K_theta diagonal blocks             */
    double *E;               /* [device] max(1, nb) extension vector E                  */
    double *theta;           /* [device] n_pad      dilatation vector Theta             */
    uint32_t *dirty;         /* [device] n_pad flags of K_theta rows to re-assemble,
                                zero-initialised by the caller                         */
} pd_fac_dev;

/* Assemble the values of the four operators (w = 1) for the bond status
 * 'mask' (K_theta carries the status; C_e, C_theta and K_e do not, since a
 * broken bond's E_b is zero).  Device-side, asynchronous; needs prob->aux
 * (pd_state_init).  Errors: PD_ERR_ARG (NULL arrays, dim mismatch),
 * PD_ERR_SIZE (nb or n_words inconsistent with the problem). */
pd_status pd_fac_assemble(pd_ctx *ctx, const pd_problem_dev *prob, const uint64_t *mask, pd_fac_dev *F);

/* One evaluation of the factored products for the current displacement of
 * st and its bond status (no breaking, no update): E, Theta into F->E and
 * F->theta, and f = K_theta Theta + K_e E into f [device] (n_pad*4,
 * f_x f_y f_z 0, internal order).  Errors as pd_fac_assemble, plus
 * PD_ERR_STATE if F is not assembled. */
pd_status pd_fac_apply(pd_ctx *ctx, const pd_problem_dev *prob, pd_fac_dev *F, const pd_state_dev *st,
                       double *f);

/* pd_step with the factored form: per step E = C_e U with the breaking
 * test on E / |xi| (Eq. 1.30; newly broken bonds get E_b = 0 and their
 * K_theta rows re-assembled), Theta = C_theta E, F = K_theta Theta + K_e E,
 * then the update of pd_step.  opts->form must be PD_FACTORED and
 * opts->precision PD_FP64 (the values are stored in double); the other
 * options, the report and the errors are those of pd_step. */
pd_status pd_fac_step(pd_ctx *ctx, const pd_problem_dev *prob, pd_state_dev *st, int64_t nsteps,
                      const pd_step_opts *opts, pd_fac_dev *F, pd_step_report *rep);

/* ------------------------------------------------------------------------ */
/* adaptive dynamic relaxation (quasi-static loading, Sec. 4 Example 4)      */
/* ------------------------------------------------------------------------ */

/* The paper solves its quasi-static example by adaptive dynamic relaxation;
 * the method (Kilic and Madenci's, cited there) is restated here.  Per
 * iteration n, with fictitious time step dt and fictitious density lambda
 * (one value per displacement component):
 *   F^n = f(u^n) + F_ext r(n)   (breaking first, as in pd_step; FP64 force)
 *   k_r = -(F_r^n - F_r^(n-1)) / (lambda_r dt v_r)     (free r with v_r != 0)
 *   c   = 2 sqrt(sum u_r k_r u_r / sum u_r^2) if that is positive, else 0
 *   v   = ((2 - c dt) v + 2 dt F^n / lambda) / (2 + c dt)
 *         (first iteration after pd_adr_density: v = dt F^n / (2 lambda))
 *   u  += dt v
 * over the free components (sums included); prescribed components keep v
 * and advance u by dt v, as in pd_step. */
typedef struct pd_adr_dev {
    double dt;          /* fictitious time step > 0                                    */
    double *lambda;     /* [device] n_pad*4 fictitious density (pd_adr_density)          */
    double *f_prev;     /* [device] n_pad*4 F of the previous iteration                  */
    double *f_int;      /* [device] n_pad*4 scratch: internal force of the iteration      */
    double *partial;    /* [device] 4 ceil(n_pad/256) per-workgroup sums                 */
    double *stats;      /* [device] 8: of the last iteration c, sum u k u, sum u^2,
                           sum F^2 over free components; [4] 1 if it was the first;
                           [5] iterations since pd_adr_density                           */
} pd_adr_dev;

/* Fictitious density for the bond status 'mask': lambda_(i,a) = dt^2/4
 * times an upper bound of the row sum of |K| (K = -df/du of Eq. 2.2), the
 * condition under which the relaxation is stable:
 *   2 sum_j c_ij |M_a| |M|_1 + |B_(i,a)| Gam_i + sum_j |b_ij| |M_a| Gam_j
 * with c_ij = G V_i V_j (1/m_i + 1/m_j), b_ij = (K - G/3) x V_i V_j,
 * B_i = sum_j b_ij M_ij, Gam_l = 2 sum_k A x V_k / m_l^2 |M_lk|_1 (intact
 * bonds, w = 1); components with a zero bound get 1.  Also restarts the
 * relaxation (stats and f_prev cleared).  Device-side, asynchronous.
 * Errors: PD_ERR_ARG (NULL arrays, dt <= 0). */
pd_status pd_adr_density(pd_ctx *ctx, const pd_problem_dev *prob, const uint64_t *mask, pd_adr_dev *R);

/* nsteps relaxation iterations on st (u = st->uv[st->cur], v = st->vel).
 * opts: precision PD_FP64 and form PD_MATRIX_FREE (the force kernels of
 * pd_force); graph_chunk, block, kernel, check_every and the report as in
 * pd_step.  The step counter advances once per iteration (it drives the
 * load ramp r(n)).  With profile = 1, pass1 times the breaking and
 * dilatation kernel, pass2 the force kernel and extra the relaxation's own
 * kernels.  Errors: as pd_step, PD_ERR_UNSUPPORTED for other options. */
pd_status pd_adr_step(pd_ctx *ctx, const pd_problem_dev *prob, pd_state_dev *st, int64_t nsteps,
                      const pd_step_opts *opts, pd_adr_dev *R, pd_step_report *rep);

/* ------------------------------------------------------------------------ */
/* static solve and implicit step with the block-sparse stiffness (Eq. 2.14) */
/* ------------------------------------------------------------------------ */

/* Remark 1 (Sec. 3.3) notes that the band of the global stiffness of
 * Eq. 2.14 is wide, which makes an implicit solve costly in memory and time
 * (it turns to coupling with finite elements instead).  Here K stays in the
 * block-sparse form and is only multiplied: no factorisation, no fill-in.
 * pd_static_solve
 * finds static equilibrium f(u) + F_ext = 0 by preconditioned conjugate
 * gradients (block Jacobi) on the free components: from the current u0 of
 * st (prescribed components held), K_ff du = F_ext + f(u0) with
 * K = -df/du (the double-precision K of pd_assemble_K, for the bond status
 * it was assembled with), then u = u0 + du is written to st->uv[st->cur].
 * The full external load is used (no ramp).  Synchronises every
 * opts->check_every iterations to test |r| <= tol |r0|. */
typedef struct pd_cg_opts {
    double tol;            /* relative residual |r| / |r0| to stop at (> 0)           */
    int32_t max_iter;      /* iteration limit (> 0)                                   */
    int32_t check_every;   /* iterations between convergence checks (> 0)             */
    int32_t matrix_free;   /* 0: products with the stored K; 1: every product K x    */
                           /* (the CG's, and those of pd_newmark_step's a_n and right- */
                           /* hand side) taken as -f(x) by the double force kernels    */
                           /* (the force of Eq. 2.2 is linear in u); K then serves     */
                           /* the preconditioner's diagonal only, and may be NULL:     */
                           /* the diagonal blocks are then summed from the bonds and   */
                           /* the implicit step's breaking test is the force pass's   */
    int32_t reserved;      /* 0                                                        */
} pd_cg_opts;

typedef struct pd_cg_report {
    int32_t iterations;    /* iterations done                                          */
    int32_t converged;     /* 1 if the tolerance was met                               */
    double rel_residual;   /* |r| / |r0| at the end                                    */
} pd_cg_report;

/* Doubles of device workspace pd_static_solve needs for n_pad rows. */
int64_t pd_static_workspace(int64_t n_pad);

/* Errors: PD_ERR_ARG (NULL pointers, K NULL without matrix_free, bad
 * options), PD_ERR_STATE (K not assembled), PD_ERR_UNSUPPORTED (K stores
 * float values), PD_ERR_UNSTABLE (non-finite solution), PD_ERR_HIP. */
pd_status pd_static_solve(pd_ctx *ctx, const pd_problem_dev *prob, const struct pd_bsr_dev *K, pd_state_dev *st,
                          const pd_cg_opts *opts, double *work, pd_cg_report *rep);

/* Implicit dynamics with the assembled double K: nsteps steps of the
 * average-acceleration Newmark rule (beta = 1/4, gamma = 1/2, unconditionally
 * stable for the linear model), the implicit counterpart of the explicit
 * update of Eq. 2.11 whose cost Remark 1 (Sec. 3.3) weighs, solved
 * iteratively as above.  Lumped mass m_i = rho V_i.  Per step, from (u_n, v_n) in st:
 *   with opts->breaking = 1, the critical-stretch test of Eqs. 1.17, 1.30 at
 *   u_n marks broken bonds in prob->mask and K is re-assembled around them;
 *   a_n = (F_ext + f(u_n)) / m on the free components;
 *   u* = u_n with the prescribed components advanced by dt v_n;
 *   (K_ff + 4/dt^2 M) du = F_ext + f(u*) + M (4 v_n / dt + a_n) on the free
 *   components, by the block-Jacobi preconditioned CG of pd_static_solve
 *   (opts->cg; |r| <= tol |r0| per step);
 *   u_{n+1} = u* + du, v_{n+1} = v_n + dt/2 (a_n + a_{n+1}) with
 *   a_{n+1} = 4/dt^2 (du - dt v_n) - a_n on the free components (prescribed
 *   velocities kept).
 * The full external load is used (no ramp); st->cur flips every step.
 * work [device] pd_newmark_workspace(n_pad) doubles, 32-byte aligned, owned
 * by the caller, no state kept in it between calls.  rep (may be NULL):
 * iterations summed over the steps, converged = 1 if every step met the
 * tolerance, rel_residual the largest final one.  Synchronises every
 * opts->cg.check_every iterations.  K may be NULL with
 * opts->cg.matrix_free = 1.  Errors: PD_ERR_ARG (NULL pointers, K NULL
 * without matrix_free, dt <= 0, bad options, nsteps < 0), PD_ERR_STATE (K not assembled),
 * PD_ERR_UNSUPPORTED (K stores float values), PD_ERR_UNSTABLE (non-finite
 * residual), PD_ERR_HIP. */
typedef struct pd_newmark_opts {
    double dt;             /* time step (> 0)                                          */
    pd_cg_opts cg;         /* solver of each step                                      */
    int32_t breaking;      /* 1: breaking test and re-assembly at the start of a step  */
    int32_t reserved;      /* 0                                                        */
} pd_newmark_opts;

/* Doubles of device workspace pd_newmark_step needs for n_pad rows. */
int64_t pd_newmark_workspace(int64_t n_pad);

pd_status pd_newmark_step(pd_ctx *ctx, const pd_problem_dev *prob, const struct pd_bsr_dev *K, pd_state_dev *st,
                          int32_t nsteps, const pd_newmark_opts *opts, double *work, pd_cg_report *rep);

/* ------------------------------------------------------------------------ */
/* outputs                                                                  */
/* ------------------------------------------------------------------------ */

/* Damage phi_i = 1 - sum rho w V_j / sum w V_j over the geometric family
 * (Eq. 1.31), internal order, phi [device] n_pad (0 for padding rows). */
pd_status pd_damage(pd_ctx *ctx, const pd_problem_dev *prob, const uint64_t *mask, double *phi);

/* Energies of the current state (synchronises): kinetic 1/2 sum rho V v.v
 * and strain sum V_i W_i with W_i of Eq. 1.20 (in the constants of Eqs.
 * 1.8, 1.15, 1.16, linearized extension; for this quadratic energy it equals
 * 1/2 u.(-f(u)), its gradient being the force of Eq. 2.2), in double with
 * fixed-order reductions (the same bits on every run).  f_scratch [device]
 * n_pad*4 doubles, 32-byte aligned: work space of the reductions. */
pd_status pd_energy(pd_ctx *ctx, const pd_problem_dev *prob, pd_state_dev *st,
                    double *f_scratch, double *kinetic, double *strain);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * energies of pd_energy, the same bits, written to out [device] (2 doubles:
 * kinetic, strain), with no allocation and no synchronisation (stream-
 * ordered on the context's stream, so it can be captured).  The reduction
 * partials live in a fixed array of the library on each GPU (65536 entries
 * of 32 bytes, 2 MiB, held until the process ends), which limits n_pad to
 * PD_NOALLOC_MAX_ROWS rows (PD_ERR_SIZE beyond, before any device work).
 * Every call on one GPU shares that array: calls that overlap on one GPU
 * (from several streams, contexts or threads) race, and the caller must
 * order them.  Errors: PD_ERR_ARG (NULL or misaligned out, state without
 * aux), PD_ERR_SIZE, PD_ERR_HIP. */
#define PD_NOALLOC_PARTS 65536
#define PD_NOALLOC_MAX_ROWS (PD_NOALLOC_PARTS * 256LL)
pd_status pd_energy_noalloc(pd_ctx *ctx, const pd_problem_dev *prob, const pd_state_dev *st, double *out);

/* Largest stable time step 2/omega_max of the explicit update for
 * specimen-uniform material, omega_max^2 = largest eigenvalue of
 * M^-1 K on the free degrees of freedom, by power iteration from a
 * seeded start (iters iterations), intact bonds 'mask'.  Uses st as
 * scratch (u and v are overwritten).  Synchronises. */
pd_status pd_stable_dt(pd_ctx *ctx, const pd_problem_dev *prob, pd_state_dev *st,
                       double *f_scratch, int32_t iters, uint64_t seed, double *dt_crit);

#ifdef __cplusplus
}
#endif

#endif /* PD_H */
