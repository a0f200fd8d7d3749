// Kernel argument blocks and launchers (device side of libpd).
#pragma once

#include <hip/hip_runtime.h>

#include "pd_internal.h"

namespace pdk {

struct StepArgs {
    int64_t n_pad;
    int64_t n_slices;
    int32_t dim;
    int32_t n_stencil;
    int64_t ramp_steps;
    const int64_t *slice_ptr;
    const uint32_t *words;
    const double *stencil;
    const double *inv_m;
    const pd_spec *spec;
    const uint32_t *aux;
    const double4 *fext;
    double4 *uv[2];
    double *vel;        // per row: 3D three packed doubles, 2D double2 (ldv/stv)
    double2 *qr;
    uint64_t *mask;
    pd_ctl *ctl;
    double4 *f_out;     // force-only mode
    double *theta_out;  // optional dilatation output
    // FP32 path
    int4 *ush[2];
    float2 *qr32;
    double *dsum;       // per row, as vel
    float *fe32;        // per row: 3D three packed floats, 2D float2 (ldvf/stvf)
    double *fe64;       // per row, as vel
    float2 *qv32;
    // BSR path
    uint32_t *dirty;
    // tile description (LDS-staged kernels)
    const int32_t *stencil_off;
    const int32_t *tile_nbr;
    int32_t tile[3];
    int32_t reach;
    const uint32_t *ktab;
    const int16_t *halo_map;
    const int32_t *halo_pos;
    int32_t n_pos;
    // super-tiles (four tiles per workgroup sharing one box; NULL: not used)
    const int32_t *st_tiles;
    const int32_t *st_nbr;
    const int32_t *st_pos;
    const uint32_t *st_ktab;
    int64_t n_st;
    int32_t st_n_pos;
    // one tile per workgroup in 2D too (four waves splitting its stencil)
    int32_t one_tile_per_group;
    // every node's volume as float when they are all equal, else 0
    float vol_uniform;
};

struct InitArgs {
    int64_t n_pad;
    int64_t start_step;
    const int32_t *perm;
    const int32_t *spec_rows;
    const double *vol;
    const double *inv_m;
    const double *u0;
    const double *v0;
    const double *f0;
    const uint8_t *bc;
    uint32_t *aux;
    double4 *fext;
    double4 *uv;
    double *vel;
    double2 *qr;
    float2 *qr32;
    pd_ctl *ctl;
    int32_t dim;
};

struct DamageArgs {
    int64_t n_slices;
    const int64_t *slice_ptr;
    const uint32_t *words;
    const uint64_t *mask;
    const double *vol;
    double *phi;
};

hipError_t launch_pass1_f64(const StepArgs &a, int cur, bool brk, int block, hipStream_t s);
hipError_t launch_pass2_f64(const StepArgs &a, int cur, bool update, int block, hipStream_t s);
hipError_t launch_pass1_f32(const StepArgs &a, int cur, bool brk, int block, hipStream_t s);
hipError_t launch_pass2_f32(const StepArgs &a, int cur, bool update, int block, hipStream_t s);
hipError_t launch_shadow_prep(const StepArgs &a, int cur, bool tiled, bool force, hipStream_t s);
bool tiled_supported(const StepArgs &a);
bool supertiles_supported(const StepArgs &a);
hipError_t launch_spass1_f32(const StepArgs &a, int cur, bool brk, hipStream_t s);
hipError_t launch_spass2_f32(const StepArgs &a, int cur, bool update, hipStream_t s);
hipError_t launch_tpass1_f32(const StepArgs &a, int cur, bool brk, hipStream_t s);
hipError_t launch_tpass2_f32(const StepArgs &a, int cur, bool update, hipStream_t s);
hipError_t launch_tdsum(const StepArgs &a, int cur, hipStream_t s);
bool tiled64_supported(const StepArgs &a);
hipError_t launch_tpass1_f64(const StepArgs &a, int cur, bool brk, hipStream_t s);
hipError_t launch_tpass2_f64(const StepArgs &a, int cur, bool update, hipStream_t s);
hipError_t launch_state_init(const InitArgs &a, hipStream_t s);
hipError_t launch_state_read(const int32_t *perm, int64_t n_pad, int dim, const double4 *uv, const double *vel,
                             double *u_out, double *v_out, hipStream_t s);
hipError_t launch_damage(const DamageArgs &a, hipStream_t s);
// partials (double4 each) of the fixed-order reductions for n_pad rows
int64_t reduce_parts(int64_t n_pad);
// kinetic and strain energy (Eq. 1.20) of state buffer cur into out[0..nout-1]
// (nout <= 4; out[2..3] = 0), or with rec != NULL recorded as the state's
// energy check; part holds reduce_parts(n_pad) partials
hipError_t launch_energy(const StepArgs &a, int cur, bool finite, double4 *part, double *out, int nout, pd_ctl *rec,
                         hipStream_t s);
hipError_t launch_pi_init(int64_t n_pad, int dim, const uint32_t *aux, double4 *uv, uint64_t seed,
                          hipStream_t s);
size_t bsr_assemble_lds(int dim, int max_row_blocks, int reach);
hipError_t set_bsr_lds_limit(int dim, bool fp32, size_t lds);
hipError_t launch_bsr_prep_assemble(const StepArgs &a, const pd_problem_dev *p, const pd_bsr_dev *K, bool all,
                                    int par, hipStream_t s);
hipError_t launch_break_mark(const StepArgs &a, const pd_problem_dev *p, const pd_bsr_dev *K, int cur,
                             hipStream_t s);
hipError_t launch_bsr_spmv(const StepArgs &a, const pd_problem_dev *p, const pd_bsr_dev *K, int cur, bool update,
                           hipStream_t s);
hipError_t launch_pi_step(int64_t n_pad, int dim, const uint32_t *aux, const pd_spec *spec, double4 *uv,
                          const double4 *f, double4 *y, pd_ctl *ctl, double4 *part, hipStream_t s);
hipError_t launch_shadow_invalidate(pd_ctl *ctl, hipStream_t s);

}  // namespace pdk
