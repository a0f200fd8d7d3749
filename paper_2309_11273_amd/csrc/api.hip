// C ABI entry points of libpd (host side): context, constants, state set-up,
// force evaluation, explicit stepping with optional hipGraph replay, damage,
// energies and the stable time step.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstddef>
#include <cstring>
#include <string>
#include <vector>

#include "adr.h"
#include "cg.h"
#include "factored.h"
#include "finite.h"
#include "kernels.h"
#include "pd.h"
#include "pd_internal.h"

// the control block without the shadow-maximum slots (what most reads need)
static constexpr size_t kCtlHead = offsetof(pd_ctl, umax_slot);

struct pd_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;  // private stream used only for graph capture
    std::string err;
    pd_ctl *host_ctl = nullptr;        // pinned copy of the control block
    hipGraphExec_t gexec = nullptr;
    std::vector<unsigned char> gkey;  // launch parameters the graph was captured with
    int gsteps = 0;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};  // profiling events
    pd_profile_stats prof{};
    double4 *part = nullptr;           // partials of the fixed-order reductions
    int64_t part_n = 0;
    double4 *scratch_dev = nullptr;    // this device's address of 'scratch' (pd_energy_noalloc)
};

// Reduction partials of pd_energy_noalloc: a fixed array on every GPU the
// library runs on (2 MiB, held until the process ends), so that the call
// allocates nothing.  Host code reaches it only through the per-device
// address that pd_ctx_create looks up (scratch_dev); every call on one GPU
// shares it.  Each call writes the partials it reads, so nothing in it has
// to start at zero.
static __device__ __align__(256) double4 scratch[PD_NOALLOC_PARTS];

namespace {

pd_status fail(pd_ctx *c, pd_status s, const char *fmt, ...) {
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof(buf), fmt, ap);
        va_end(ap);
        c->err = buf;
    }
    return s;
}

#define HIP_TRY(ctx, call)                                                                   \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail((ctx), PD_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_));   \
    } while (0)

pd_status check_problem(pd_ctx *c, const pd_problem_dev *p) {
    if (!p) return fail(c, PD_ERR_ARG, "problem is NULL");
    if (p->dim != 2 && p->dim != 3) return fail(c, PD_ERR_ARG, "dim must be 2 or 3");
    if (p->n_pad <= 0 || p->n_pad % 64 || p->n_slices != p->n_pad / 64)
        return fail(c, PD_ERR_SIZE, "n_pad must be a positive multiple of 64 and n_slices = n_pad/64");
    if (p->n_stencil < 1 || p->n_stencil > PD_MAX_STENCIL) return fail(c, PD_ERR_SIZE, "bad n_stencil");
    if (p->n_specimens < 1 || p->n_specimens > PD_MAX_SPECIMENS) return fail(c, PD_ERR_SIZE, "bad n_specimens");
    if (!p->slice_ptr || !p->words || !p->stencil || !p->vol || !p->inv_m || !p->spec)
        return fail(c, PD_ERR_ARG, "problem has a NULL family array");
    if (p->ramp_steps < 0) return fail(c, PD_ERR_ARG, "ramp_steps < 0");
    return PD_OK;
}

pdk::StepArgs make_args(const pd_problem_dev *p, const pd_state_dev *st) {
    pdk::StepArgs a{};
    a.n_pad = p->n_pad;
    a.n_slices = p->n_slices;
    a.dim = p->dim;
    a.n_stencil = p->n_stencil;
    a.ramp_steps = p->ramp_steps;
    a.slice_ptr = p->slice_ptr;
    a.words = p->words;
    a.stencil = p->stencil;
    a.inv_m = p->inv_m;
    a.spec = p->spec;
    a.aux = p->aux;
    a.fext = reinterpret_cast<const double4 *>(p->fext);
    a.uv[0] = reinterpret_cast<double4 *>(st->uv[0]);
    a.uv[1] = reinterpret_cast<double4 *>(st->uv[1]);
    a.vel = st->vel;
    a.qr = reinterpret_cast<double2 *>(st->qr);
    a.mask = st->mask;
    a.ctl = reinterpret_cast<pd_ctl *>(st->ctl);
    a.ush[0] = reinterpret_cast<int4 *>(st->ush[0]);
    a.ush[1] = reinterpret_cast<int4 *>(st->ush[1]);
    a.qr32 = reinterpret_cast<float2 *>(st->qr32);
    a.dsum = st->dsum;
    a.fe32 = st->fe32;
    a.fe64 = st->fe64;
    a.qv32 = reinterpret_cast<float2 *>(st->qv32);
    a.stencil_off = p->stencil_off;
    a.tile_nbr = p->tile_nbr;
    for (int c = 0; c < 3; c++) a.tile[c] = p->tile[c];
    a.reach = p->reach;
    a.ktab = p->ktab;
    a.halo_map = p->halo_map;
    a.halo_pos = p->halo_pos;
    a.n_pos = p->n_pos;
    a.st_tiles = p->st_tiles;
    a.st_nbr = p->st_nbr;
    a.st_pos = p->st_pos;
    a.st_ktab = p->st_ktab;
    a.n_st = p->n_st;
    a.st_n_pos = p->st_n_pos;
    a.vol_uniform = p->vol_uniform;
    return a;
}

pd_status check_state(pd_ctx *c, const pd_state_dev *st, bool need_f32) {
    if (!st) return fail(c, PD_ERR_ARG, "state is NULL");
    if (!st->uv[0] || !st->uv[1] || !st->vel || !st->qr || !st->mask || !st->ctl)
        return fail(c, PD_ERR_ARG, "state has a NULL array");
    if (st->cur != 0 && st->cur != 1) return fail(c, PD_ERR_ARG, "state cur must be 0 or 1");
    if (need_f32 && (!st->ush[0] || !st->ush[1] || !st->qr32 || !st->dsum || !st->fe32))
        return fail(c, PD_ERR_ARG, "FP32 path needs ush[0], ush[1], qr32, dsum and fe32");
    return PD_OK;
}


// The context's reduction buffer, grown to hold the partials of n_pad rows.
pd_status need_parts(pd_ctx *c, int64_t n_pad) {
    const int64_t n = pdk::reduce_parts(n_pad) + 1;
    if (n <= c->part_n) return PD_OK;
    if (c->part) {
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        HIP_TRY(c, hipFree(c->part));
        c->part = nullptr;
        c->part_n = 0;
    }
    HIP_TRY(c, hipMalloc(reinterpret_cast<void **>(&c->part), sizeof(double4) * n));
    c->part_n = n;
    return PD_OK;
}

}  // namespace

extern "C" {

const char *pd_version(void) { return "pdx 0.1 (gfx950)"; }

pd_status pd_ctx_create(pd_ctx **out, int device, void *stream) {
    if (!out) return PD_ERR_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return PD_ERR_HIP;
    if (hipSetDevice(device) != hipSuccess) return PD_ERR_HIP;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return PD_ERR_HIP;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return PD_ERR_HIP;
    pd_ctx *c = new pd_ctx();
    c->device = device;
    c->stream = reinterpret_cast<hipStream_t>(stream);
    // this device's copy of the no-allocation scratch array (device current)
    if (hipGetSymbolAddress(reinterpret_cast<void **>(&c->scratch_dev), HIP_SYMBOL(scratch)) != hipSuccess ||
        !c->scratch_dev) {
        delete c;
        return PD_ERR_HIP;
    }
    if (hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        delete c;
        return PD_ERR_HIP;
    }
    if (hipHostMalloc(reinterpret_cast<void **>(&c->host_ctl), sizeof(pd_ctl), hipHostMallocDefault) != hipSuccess) {
        (void)hipStreamDestroy(c->cap_stream);
        delete c;
        return PD_ERR_HIP;
    }
    *out = c;
    return PD_OK;
}

pd_status pd_ctx_destroy(pd_ctx *c) {
    if (!c) return PD_OK;
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    for (int k = 0; k < 4; k++)
        if (c->ev[k]) (void)hipEventDestroy(c->ev[k]);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->host_ctl) (void)hipHostFree(c->host_ctl);
    if (c->part) (void)hipFree(c->part);
    delete c;
    return PD_OK;
}

const char *pd_last_error(const pd_ctx *c) { return c ? c->err.c_str() : "no context"; }

pd_status pd_profile_read(pd_ctx *c, pd_profile_stats *out, int32_t reset) {
    if (!c || !out) return PD_ERR_ARG;
    *out = c->prof;
    if (reset) c->prof = pd_profile_stats{};
    return PD_OK;
}

pd_status pd_critical_stretch(pd_mode mode, double E, double nu, double G0, double delta, int variant,
                              double *s0) {
    if (!s0 || !(E > 0.0) || !(nu > -1.0 && nu < 0.5) || !(delta > 0.0)) return PD_ERR_ARG;
    if (mode < PD_3D || mode > PD_PLANE_STRAIN || (variant != 0 && variant != 1)) return PD_ERR_ARG;
    if (!(G0 > 0.0) || !std::isfinite(G0)) {
        *s0 = INFINITY;
        return PD_OK;
    }
    const double pi = 3.14159265358979323846;
    const double kappa = E / (3.0 * (1.0 - 2.0 * nu));
    const double mu = E / (2.0 * (1.0 + nu));
    if (mode == PD_3D) {
        // Eqs. 1.26, 1.27
        const double beta = 125.0 * delta / 1848.0;
        const double betap = variant ? 5.0 * delta / 24.0 : 5.0 * delta / (24.0 * pi);
        *s0 = std::sqrt(G0 / ((9.0 * kappa - 15.0 * mu) * beta + 15.0 * mu * betap));
        return PD_OK;
    }
    // Eqs. 1.28, 1.29 with A of Eq. 1.8
    const double A = mode == PD_PLANE_STRESS ? 2.0 * (1.0 - 2.0 * nu) / (1.0 - nu) : 2.0;
    const double g = (1.0 + nu) / (1.0 - 2.0 * nu);
    const double kp = mode == PD_PLANE_STRESS ? kappa + mu / 9.0 * g * g : kappa + mu / 9.0;
    const double beta = 1087.0 * delta / (1250.0 * pi * pi);
    const double betap = 4.0 * delta / (5.0 * pi);
    *s0 = std::sqrt(G0 / (A * A * (kp - 8.0 / 9.0 * mu) * beta + 8.0 * mu * betap));
    return PD_OK;
}

pd_status pd_specimen_params(pd_mode mode, double E, double nu, double rho, double s0, double dt, pd_spec *out) {
    if (!out || !(E > 0.0) || !(nu > -1.0 && nu < 0.5) || !(rho > 0.0) || !(dt > 0.0) || std::isnan(s0))
        return PD_ERR_ARG;
    if (mode < PD_3D || mode > PD_PLANE_STRAIN) return PD_ERR_ARG;
    const double kappa = E / (3.0 * (1.0 - 2.0 * nu));
    const double mu = E / (2.0 * (1.0 + nu));
    double A, K, G;
    if (mode == PD_3D) {  // Eqs. 1.8, 1.15, 1.16
        A = 3.0;
        K = 3.0 * kappa;
        G = 15.0 * mu;
    } else if (mode == PD_PLANE_STRESS) {
        A = 2.0 * (1.0 - 2.0 * nu) / (1.0 - nu);
        K = 2.0 * kappa * (1.0 - 2.0 * nu) / (1.0 - nu) -
            2.0 / 3.0 * mu * (1.0 + nu) * (1.0 - 3.0 * nu) / ((1.0 - nu) * (1.0 - 2.0 * nu));
        G = 8.0 * mu;
    } else {
        A = 2.0;
        K = 2.0 * kappa - 2.0 / 3.0 * mu;
        G = 8.0 * mu;
    }
    std::memset(out, 0, sizeof(*out));
    out->kp = K - G / 3.0;
    out->G = G;
    out->A = A;
    out->rho = rho;
    out->s0 = s0;
    out->dt = dt;
    return PD_OK;
}

pd_status pd_state_init(pd_ctx *c, const pd_problem_dev *p, const int32_t *perm, int64_t n, const double *u0,
                        const double *v0, const uint8_t *bc, const double *fext0, const int32_t *spec_rows,
                        uint32_t *aux_out, double *fext_out, pd_state_dev *st, int64_t start_step) {
    if (!c) return PD_ERR_ARG;
    pd_status s = check_problem(c, p);
    if (s != PD_OK) return s;
    if ((s = check_state(c, st, false)) != PD_OK) return s;
    if (!perm || !spec_rows || !aux_out || !fext_out) return fail(c, PD_ERR_ARG, "NULL perm/spec/aux/fext");
    if (n < 1 || n > p->n_pad) return fail(c, PD_ERR_SIZE, "n out of range");
    if (start_step < 0) return fail(c, PD_ERR_ARG, "start_step < 0");
    HIP_TRY(c, hipSetDevice(c->device));
    pdk::InitArgs a{};
    a.n_pad = p->n_pad;
    a.start_step = start_step;
    a.perm = perm;
    a.spec_rows = spec_rows;
    a.vol = p->vol;
    a.inv_m = p->inv_m;
    a.u0 = u0;
    a.v0 = v0;
    a.f0 = fext0;
    a.bc = bc;
    a.aux = aux_out;
    a.fext = reinterpret_cast<double4 *>(fext_out);
    a.uv = reinterpret_cast<double4 *>(st->uv[st->cur]);
    a.vel = st->vel;
    a.dim = p->dim;
    a.qr = reinterpret_cast<double2 *>(st->qr);
    a.qr32 = reinterpret_cast<float2 *>(st->qr32);
    a.ctl = reinterpret_cast<pd_ctl *>(st->ctl);
    HIP_TRY(c, pdk::launch_state_init(a, c->stream));
    // the other displacement buffer carries the node volumes too
    HIP_TRY(c, hipMemcpyAsync(st->uv[st->cur ^ 1], st->uv[st->cur], sizeof(double) * 4 * p->n_pad,
                              hipMemcpyDeviceToDevice, c->stream));
    return PD_OK;
}

pd_status pd_state_read(pd_ctx *c, const pd_problem_dev *p, const int32_t *perm, int64_t n, const pd_state_dev *st,
                        double *u_out, double *v_out) {
    if (!c) return PD_ERR_ARG;
    pd_status s = check_problem(c, p);
    if (s != PD_OK) return s;
    if ((s = check_state(c, st, false)) != PD_OK) return s;
    if (!perm) return fail(c, PD_ERR_ARG, "perm is NULL");
    if (n < 1 || n > p->n_pad) return fail(c, PD_ERR_SIZE, "n out of range");
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, pdk::launch_state_read(perm, p->n_pad, p->dim, reinterpret_cast<const double4 *>(st->uv[st->cur]),
                                      st->vel, u_out, v_out, c->stream));
    return PD_OK;
}

pd_status pd_tile_kernels_apply(const pd_problem_dev *p, const pd_state_dev *st, int32_t precision, int32_t *yes) {
    if (!p || !st || !yes) return PD_ERR_ARG;
    if (precision != PD_FP64 && precision != PD_FP32_RECHECK) return PD_ERR_ARG;
    pd_state_dev tmp = *st;
    const pdk::StepArgs a = make_args(p, &tmp);
    *yes = (precision == PD_FP64 ? pdk::tiled64_supported(a) : pdk::tiled_supported(a)) ? 1 : 0;
    return PD_OK;
}

pd_status pd_get_step(pd_ctx *c, const pd_state_dev *st, int64_t *step) {
    if (!c || !st || !st->ctl || !step) return PD_ERR_ARG;
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, hipMemcpyAsync(c->host_ctl, st->ctl, kCtlHead, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    *step = c->host_ctl->s2;
    return PD_OK;
}

pd_status pd_force(pd_ctx *c, const pd_problem_dev *p, pd_state_dev *st, int32_t precision, double *f,
                   double *theta) {
    if (!c) return PD_ERR_ARG;
    pd_status s = check_problem(c, p);
    if (s != PD_OK) return s;
    if (precision != PD_FP64 && precision != PD_FP32_RECHECK) return fail(c, PD_ERR_ARG, "unknown precision");
    if ((s = check_state(c, st, precision == PD_FP32_RECHECK)) != PD_OK) return s;
    if (!f) return fail(c, PD_ERR_ARG, "f is NULL");
    if (!p->aux) return fail(c, PD_ERR_ARG, "aux is NULL (call pd_state_init first)");
    HIP_TRY(c, hipSetDevice(c->device));
    pdk::StepArgs a = make_args(p, st);
    a.f_out = reinterpret_cast<double4 *>(f);
    a.theta_out = theta;
    if (precision == PD_FP64) {
        const bool tiled = pdk::tiled64_supported(a);
        if (tiled) HIP_TRY(c, pdk::launch_tpass1_f64(a, st->cur, false, c->stream));
        else HIP_TRY(c, pdk::launch_pass1_f64(a, st->cur, false, 256, c->stream));
        a.theta_out = nullptr;
        if (tiled) HIP_TRY(c, pdk::launch_tpass2_f64(a, st->cur, false, c->stream));
        else HIP_TRY(c, pdk::launch_pass2_f64(a, st->cur, false, 256, c->stream));
    } else {
        const bool tiled = pdk::tiled_supported(a);
        HIP_TRY(c, pdk::launch_shadow_prep(a, st->cur, tiled, true, c->stream));
        if (tiled) HIP_TRY(c, pdk::launch_tpass1_f32(a, st->cur, false, c->stream));
        else HIP_TRY(c, pdk::launch_pass1_f32(a, st->cur, false, 256, c->stream));
        a.theta_out = nullptr;
        if (tiled) HIP_TRY(c, pdk::launch_tpass2_f32(a, st->cur, false, c->stream));
        else HIP_TRY(c, pdk::launch_pass2_f32(a, st->cur, false, 256, c->stream));
    }
    return PD_OK;
}

static pd_status check_bsr(pd_ctx *c, const pd_problem_dev *p, const pd_bsr_dev *K);
static pd_status check_fac(pd_ctx *c, const pd_problem_dev *p, const pd_fac_dev *F);

// one explicit step on 'stream' starting from displacement buffer 'cur'
static hipError_t enqueue_step(const pdk::StepArgs &a, const pd_step_opts &o, int cur, hipStream_t s,
                               const pd_problem_dev *p, const pd_bsr_dev *K, const pd_fac_dev *F,
                               const pd_adr_dev *R, hipEvent_t *ev = nullptr) {
    hipError_t e;
    const int block = o.block > 0 ? o.block : 256;
    if (ev && (e = hipEventRecord(ev[0], s)) != hipSuccess) return e;
    if (R) {
        // relaxation: FP64 force without its update, then the relaxation kernels
        pdk::StepArgs af = a;
        af.f_out = reinterpret_cast<double4 *>(R->f_int);
        const bool tiled = o.kernel != 1 && (o.extension ? pdk::tiled64_fin_supported(af) : pdk::tiled64_supported(af));
        if (o.extension)
            e = tiled ? pdk::launch_tpass1_f64_fin(af, cur, true, s) : pdk::launch_fin_pass1(af, cur, true, block, s);
        else e = tiled ? pdk::launch_tpass1_f64(af, cur, true, s) : pdk::launch_pass1_f64(af, cur, true, block, s);
        if (e != hipSuccess) return e;
        if (ev && (e = hipEventRecord(ev[1], s)) != hipSuccess) return e;
        if (o.extension)
            e = tiled ? pdk::launch_tpass2_f64_fin(af, cur, false, s) : pdk::launch_fin_pass2(af, cur, false, block, s);
        else e = tiled ? pdk::launch_tpass2_f64(af, cur, false, s) : pdk::launch_pass2_f64(af, cur, false, block, s);
        if (e != hipSuccess) return e;
        if (ev && (e = hipEventRecord(ev[2], s)) != hipSuccess) return e;
        if ((e = pdk::launch_adr_iteration(a, p, R, cur, s)) != hipSuccess) return e;
    } else if (o.form == PD_FACTORED) {
        if ((e = pdk::launch_fac_extension(a, p, F, cur, true, s)) != hipSuccess) return e;
        if (ev && (e = hipEventRecord(ev[1], s)) != hipSuccess) return e;
        if ((e = pdk::launch_fac_kth_dirty(a, p, F, cur, s)) != hipSuccess) return e;
        if ((e = pdk::launch_fac_dilatation(a, p, F, s)) != hipSuccess) return e;
        if (ev && (e = hipEventRecord(ev[2], s)) != hipSuccess) return e;
        if ((e = pdk::launch_fac_force(a, p, F, cur, true, s)) != hipSuccess) return e;
    } else if (o.form == PD_BSR) {
        if ((e = pdk::launch_break_mark(a, p, K, cur, s)) != hipSuccess) return e;
        if (ev && (e = hipEventRecord(ev[1], s)) != hipSuccess) return e;
        if ((e = pdk::launch_bsr_prep_assemble(a, p, K, false, cur, s)) != hipSuccess) return e;
        if (ev && (e = hipEventRecord(ev[2], s)) != hipSuccess) return e;
        if ((e = pdk::launch_bsr_spmv(a, p, K, cur, true, s)) != hipSuccess) return e;
    } else if (o.extension) {
        // the double tile kernels unless the gather kernels are asked for
        const bool tiled = o.kernel != 1 && pdk::tiled64_fin_supported(a);
        e = tiled ? pdk::launch_tpass1_f64_fin(a, cur, true, s) : pdk::launch_fin_pass1(a, cur, true, block, s);
        if (e != hipSuccess) return e;
        if (ev && (e = hipEventRecord(ev[1], s)) != hipSuccess) return e;
        if (ev && (e = hipEventRecord(ev[2], s)) != hipSuccess) return e;
        e = tiled ? pdk::launch_tpass2_f64_fin(a, cur, true, s) : pdk::launch_fin_pass2(a, cur, true, block, s);
        if (e != hipSuccess) return e;
    } else {
        // LDS-staged tile kernels unless the gather kernels are asked for;
        // the FP32 super-tile kernels when asked for (kernel 3)
        const bool fp64 = o.precision == PD_FP64;
        const bool tiled = o.kernel != 1 && (fp64 ? pdk::tiled64_supported(a) : pdk::tiled_supported(a));
        const bool super = !fp64 && o.kernel == 3 && pdk::supertiles_supported(a);
        if (fp64) e = tiled ? pdk::launch_tpass1_f64(a, cur, true, s) : pdk::launch_pass1_f64(a, cur, true, block, s);
        else if (super) e = pdk::launch_spass1_f32(a, cur, true, s);
        else e = tiled ? pdk::launch_tpass1_f32(a, cur, true, s) : pdk::launch_pass1_f32(a, cur, true, block, s);
        if (e != hipSuccess) return e;
        if (ev && (e = hipEventRecord(ev[1], s)) != hipSuccess) return e;
        if (ev && (e = hipEventRecord(ev[2], s)) != hipSuccess) return e;
        if (fp64) e = tiled ? pdk::launch_tpass2_f64(a, cur, true, s) : pdk::launch_pass2_f64(a, cur, true, block, s);
        else if (super) e = pdk::launch_spass2_f32(a, cur, true, s);
        else e = tiled ? pdk::launch_tpass2_f32(a, cur, true, s) : pdk::launch_pass2_f32(a, cur, true, block, s);
        if (e != hipSuccess) return e;
    }
    if (ev && (e = hipEventRecord(ev[3], s)) != hipSuccess) return e;
    return hipSuccess;
}

static pd_status step_impl(pd_ctx *c, const pd_problem_dev *p, pd_state_dev *st, int64_t nsteps,
                           const pd_step_opts *opts, pd_bsr_dev *K, pd_fac_dev *F, pd_adr_dev *R,
                           pd_step_report *rep) {
    if (!c) return PD_ERR_ARG;
    pd_status s = check_problem(c, p);
    if (s != PD_OK) return s;
    pd_step_opts o{};
    if (opts) o = *opts;
    if (o.precision != PD_FP64 && o.precision != PD_FP32_RECHECK) return fail(c, PD_ERR_ARG, "unknown precision");
    if (o.form != PD_MATRIX_FREE && o.form != PD_BSR && o.form != PD_FACTORED)
        return fail(c, PD_ERR_ARG, "unknown form");
    if ((o.form == PD_FACTORED) != (F != nullptr))
        return fail(c, PD_ERR_UNSUPPORTED, "the factored form runs through pd_fac_step (and only it)");
    if (o.block != 0 && o.block != 64 && o.block != 128 && o.block != 256)
        return fail(c, PD_ERR_ARG, "block must be 0, 64, 128 or 256");
    if (o.graph_chunk < 0 || o.check_every < 0) return fail(c, PD_ERR_ARG, "negative option");
    if (o.profile != 0 && o.profile != 1) return fail(c, PD_ERR_ARG, "profile must be 0 or 1");
    if (o.kernel < 0 || o.kernel > 4) return fail(c, PD_ERR_ARG, "kernel must be 0 to 4");
    if (o.extension != 0 && o.extension != 1) return fail(c, PD_ERR_ARG, "extension must be 0 or 1");
    if (o.extension && (o.precision != PD_FP64 || o.form != PD_MATRIX_FREE))
        return fail(c, PD_ERR_UNSUPPORTED, "the finite extension runs with PD_FP64 and PD_MATRIX_FREE");
    if (o.extension && (o.kernel == 2 || o.kernel == 4)) {
        pd_state_dev tmp = *st;
        pdk::StepArgs ta = make_args(p, &tmp);
        ta.one_tile_per_group = o.kernel == 4;
        if (!pdk::tiled64_fin_supported(ta))
            return fail(c, PD_ERR_UNSUPPORTED, "the finite model's tile kernels do not fit this family");
    }
    if (o.kernel == 3 && o.form == PD_MATRIX_FREE && o.precision == PD_FP32_RECHECK && !o.extension) {
        pd_state_dev tmp = *st;
        if (!pdk::supertiles_supported(make_args(p, &tmp)))
            return fail(c, PD_ERR_UNSUPPORTED,
                        "super-tile kernels need 4x4x4 (3D) or 8x8 (2D) tiles, reach <= 3 and the tables of pd_build_supertiles");
    }
    if ((o.kernel == 2 || o.kernel == 3 || o.kernel == 4) && o.form == PD_MATRIX_FREE) {
        pd_state_dev tmp = *st;
        pdk::StepArgs ta = make_args(p, &tmp);
        ta.one_tile_per_group = o.kernel == 4;
        if (o.precision == PD_FP32_RECHECK ? !pdk::tiled_supported(ta) : !pdk::tiled64_supported(ta))
            return fail(c, PD_ERR_UNSUPPORTED,
                        "tile kernels need tile edges >= the stencil reach (and qv32 for FP32, fe64 for FP64)");
    }
    if (o.profile && !c->ev[0]) {
        for (int k = 0; k < 4; k++) HIP_TRY(c, hipEventCreate(&c->ev[k]));
    }
    if ((s = check_state(c, st, o.precision == PD_FP32_RECHECK && o.form == PD_MATRIX_FREE)) != PD_OK) return s;
    if (!p->aux || !p->fext) return fail(c, PD_ERR_ARG, "aux/fext are NULL (call pd_state_init first)");
    if (nsteps < 0) return fail(c, PD_ERR_ARG, "nsteps < 0");
    if (o.form == PD_BSR) {
        if (!K || !K->assembled) return fail(c, PD_ERR_UNSUPPORTED, "PD_BSR needs an assembled K");
        if ((s = check_bsr(c, p, K)) != PD_OK) return s;
        if ((o.precision == PD_FP32_RECHECK) != (K->fp32 != 0))
            return fail(c, PD_ERR_UNSUPPORTED, "BSR precision must match the K value type");
        if (!K->dirty || !K->bc || !p->lat4) return fail(c, PD_ERR_ARG, "BSR needs dirty, bc and lat4");
    }
    if (R) {
        if (o.form != PD_MATRIX_FREE || o.precision != PD_FP64)
            return fail(c, PD_ERR_UNSUPPORTED, "the relaxation uses the FP64 matrix-free force (PD_FP64, PD_MATRIX_FREE)");
        if (!R->lambda || !R->f_prev || !R->f_int || !R->partial || !R->stats)
            return fail(c, PD_ERR_ARG, "R has a NULL array");
        if (!(R->dt > 0.0)) return fail(c, PD_ERR_ARG, "relaxation dt must be > 0");
    }
    if (o.form == PD_FACTORED) {
        if ((s = check_fac(c, p, F)) != PD_OK) return s;
        if (!F->assembled) return fail(c, PD_ERR_STATE, "the factored operators are not assembled");
        if (o.precision != PD_FP64)
            return fail(c, PD_ERR_UNSUPPORTED, "the factored form stores double values (precision PD_FP64)");
    }
    if (o.energy_check != 0 && o.energy_check != 1) return fail(c, PD_ERR_ARG, "energy_check must be 0 or 1");
    if (std::isnan(o.energy_growth)) return fail(c, PD_ERR_ARG, "energy_growth is NaN");
    HIP_TRY(c, hipSetDevice(c->device));
    const double growth = o.energy_growth > 0.0 ? o.energy_growth : 1e3;
    if (o.energy_check && (s = need_parts(c, p->n_pad)) != PD_OK) return s;
    pdk::StepArgs a = make_args(p, st);
    a.one_tile_per_group = o.kernel == 4;
    int cur = st->cur;
    if (o.precision == PD_FP32_RECHECK && o.form == PD_MATRIX_FREE)
        HIP_TRY(c, pdk::launch_shadow_prep(a, cur, o.kernel != 1 && pdk::tiled_supported(a), false, c->stream));

    int64_t done = 0;
    const int64_t check = o.check_every > 0 ? o.check_every : nsteps;
    while (done < nsteps) {
        int64_t todo = std::min<int64_t>(check, nsteps - done);
        int64_t chunk = (o.graph_chunk > 0 && !o.profile) ? ((int64_t)o.graph_chunk + 1) / 2 * 2 : 0;
        if (chunk > 0 && todo >= chunk) {
            // Everything a captured launch bakes in by value: the argument
            // block, the problem descriptor, the options, the starting
            // buffer, the chunk and the operator descriptors (by content, not
            // by address).  Compared byte for byte, so a new problem or a
            // rebuilt operator never replays a stale graph.
            std::vector<unsigned char> key;
            auto add = [&key](const void *q, size_t nb) {
                const unsigned char *b = static_cast<const unsigned char *>(q);
                key.insert(key.end(), b, b + nb);
            };
            add(&a, sizeof(a));
            add(p, sizeof(*p));
            add(&o, sizeof(o));
            add(&cur, sizeof(cur));
            add(&chunk, sizeof(chunk));
            const unsigned char present[3] = {(unsigned char)(K != nullptr), (unsigned char)(F != nullptr),
                                              (unsigned char)(R != nullptr)};
            add(present, sizeof(present));
            if (K) add(K, sizeof(*K));
            if (F) add(F, sizeof(*F));
            if (R) add(R, sizeof(*R));
            if (!c->gexec || c->gkey != key) {
                if (c->gexec) {
                    (void)hipGraphExecDestroy(c->gexec);
                    c->gexec = nullptr;
                }
                hipGraph_t g;
                HIP_TRY(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
                hipError_t ce = hipSuccess;
                for (int64_t i = 0; i < chunk && ce == hipSuccess; i++)
                    ce = enqueue_step(a, o, (cur + (int)i) & 1, c->cap_stream, p, K, F, R);
                hipError_t ee = hipStreamEndCapture(c->cap_stream, &g);
                if (ce != hipSuccess) return fail(c, PD_ERR_HIP, "capture launch: %s", hipGetErrorString(ce));
                if (ee != hipSuccess) return fail(c, PD_ERR_HIP, "end capture: %s", hipGetErrorString(ee));
                hipError_t ie = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
                (void)hipGraphDestroy(g);
                if (ie != hipSuccess) return fail(c, PD_ERR_HIP, "graph instantiate: %s", hipGetErrorString(ie));
                c->gkey = key;
                c->gsteps = (int)chunk;
            }
            while (todo >= chunk) {
                HIP_TRY(c, hipGraphLaunch(c->gexec, c->stream));
                todo -= chunk;
                done += chunk;
            }
        }
        for (int64_t i = 0; i < todo; i++) {
            hipError_t e = enqueue_step(a, o, cur, c->stream, p, K, F, R, o.profile ? c->ev : nullptr);
            if (e != hipSuccess) return fail(c, PD_ERR_HIP, "step launch: %s", hipGetErrorString(e));
            if (o.profile) {
                float t1 = 0, t2 = 0, t3 = 0;
                HIP_TRY(c, hipEventSynchronize(c->ev[3]));
                HIP_TRY(c, hipEventElapsedTime(&t1, c->ev[0], c->ev[1]));
                HIP_TRY(c, hipEventElapsedTime(&t2, c->ev[1], c->ev[2]));
                HIP_TRY(c, hipEventElapsedTime(&t3, c->ev[2], c->ev[3]));
                c->prof.steps++;
                c->prof.ms_pass1 += t1;
                // the relaxation records pass 2 before its own kernels
                c->prof.ms_extra += R ? t3 : t2;
                c->prof.ms_pass2 += R ? t2 : t3;
            }
            cur ^= 1;
            done++;
        }
        const bool last = done == nsteps;
        if (o.check_every > 0 || (o.energy_check && last)) {
            st->cur = cur;
            if (o.energy_check)
                HIP_TRY(c, pdk::launch_energy(a, cur, o.extension != 0, c->part, nullptr, 0,
                                              reinterpret_cast<pd_ctl *>(st->ctl), c->stream));
            HIP_TRY(c, hipMemcpyAsync(c->host_ctl, st->ctl, kCtlHead, hipMemcpyDeviceToHost, c->stream));
            HIP_TRY(c, hipStreamSynchronize(c->stream));
            const pd_ctl *h = c->host_ctl;
            if (h->flags & PD_CTL_VOLUME)
                return fail(c, PD_ERR_ARG, "vol_uniform does not match the node volumes");
            if (h->flags & PD_CTL_NONFINITE)
                return fail(c, PD_ERR_UNSTABLE, "non-finite displacement before step %lld", (long long)h->s2);
            if (o.energy_check) {
                const double now = h->en[0] + h->en[1], before = h->en[2];
                if (before > 0.0 && !(now <= growth * before))
                    return fail(c, PD_ERR_UNSTABLE,
                                "energy grew from %.6g to %.6g (more than %.3g times) by step %lld", before, now,
                                growth, (long long)h->s2);
            }
        }
    }
    st->cur = cur;
    if (rep) {
        HIP_TRY(c, hipMemcpyAsync(c->host_ctl, st->ctl, sizeof(pd_ctl), hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        const pd_ctl *h = c->host_ctl;
        if (h->flags & PD_CTL_VOLUME) return fail(c, PD_ERR_ARG, "vol_uniform does not match the node volumes");
        rep->step = h->s2;
        rep->broken_total = (int64_t)h->broken;
        rep->rechecks = (int64_t)h->rechecks;
        rep->nonfinite = (h->flags & PD_CTL_NONFINITE) ? 1 : 0;
        float um;
        unsigned int bits = h->umax_bits[cur];
        for (int q = 0; q < PD_UMAX_SLOTS; q++) bits = std::max(bits, h->umax_slot[cur][q * PD_UMAX_STRIDE]);
        std::memcpy(&um, &bits, 4);
        rep->umax = (double)um;
        if (h->margin_key) {
            float mg;
            const unsigned int mb = ~h->margin_key;
            std::memcpy(&mg, &mb, 4);
            rep->min_margin = (double)mg;
        } else {
            rep->min_margin = INFINITY;
        }
        rep->kinetic = h->en[0];
        rep->strain = h->en[1];
        rep->energy_step = h->en[3] > 0.0 ? (int64_t)h->en[3] - 1 : -1;
        if (rep->nonfinite) return fail(c, PD_ERR_UNSTABLE, "non-finite displacement");
    }
    return PD_OK;
}

pd_status pd_step(pd_ctx *c, const pd_problem_dev *p, pd_state_dev *st, int64_t nsteps, const pd_step_opts *opts,
                  pd_bsr_dev *K, pd_step_report *rep) {
    return step_impl(c, p, st, nsteps, opts, K, nullptr, nullptr, rep);
}

pd_status pd_fac_step(pd_ctx *c, const pd_problem_dev *p, pd_state_dev *st, int64_t nsteps,
                      const pd_step_opts *opts, pd_fac_dev *F, pd_step_report *rep) {
    if (!c) return PD_ERR_ARG;
    if (!F) return fail(c, PD_ERR_ARG, "F is NULL");
    if (opts && opts->form != PD_FACTORED) return fail(c, PD_ERR_ARG, "pd_fac_step needs opts->form = PD_FACTORED");
    pd_step_opts o{};
    if (opts) o = *opts;
    o.form = PD_FACTORED;
    return step_impl(c, p, st, nsteps, &o, nullptr, F, nullptr, rep);
}

pd_status pd_force_finite(pd_ctx *c, const pd_problem_dev *p, pd_state_dev *st, double *f, double *theta) {
    if (!c) return PD_ERR_ARG;
    pd_status s = check_problem(c, p);
    if (s != PD_OK) return s;
    if ((s = check_state(c, st, false)) != PD_OK) return s;
    if (!f) return fail(c, PD_ERR_ARG, "f is NULL");
    if (!p->aux) return fail(c, PD_ERR_ARG, "aux is NULL (call pd_state_init first)");
    HIP_TRY(c, hipSetDevice(c->device));
    pdk::StepArgs a = make_args(p, st);
    a.f_out = reinterpret_cast<double4 *>(f);
    a.theta_out = theta;
    const bool tiled = pdk::tiled64_fin_supported(a);
    if (tiled) HIP_TRY(c, pdk::launch_tpass1_f64_fin(a, st->cur, false, c->stream));
    else HIP_TRY(c, pdk::launch_fin_pass1(a, st->cur, false, 256, c->stream));
    a.theta_out = nullptr;
    if (tiled) HIP_TRY(c, pdk::launch_tpass2_f64_fin(a, st->cur, false, c->stream));
    else HIP_TRY(c, pdk::launch_fin_pass2(a, st->cur, false, 256, c->stream));
    return PD_OK;
}

pd_status pd_adr_step(pd_ctx *c, const pd_problem_dev *p, pd_state_dev *st, int64_t nsteps,
                      const pd_step_opts *opts, pd_adr_dev *R, pd_step_report *rep) {
    if (!c) return PD_ERR_ARG;
    if (!R) return fail(c, PD_ERR_ARG, "R is NULL");
    return step_impl(c, p, st, nsteps, opts, nullptr, nullptr, R, rep);
}

pd_status pd_adr_density(pd_ctx *c, const pd_problem_dev *p, const uint64_t *mask, pd_adr_dev *R) {
    if (!c) return PD_ERR_ARG;
    pd_status s = check_problem(c, p);
    if (s != PD_OK) return s;
    if (!R || !R->lambda || !R->f_prev || !R->f_int || !R->partial || !R->stats)
        return fail(c, PD_ERR_ARG, "R or one of its arrays is NULL");
    if (!(R->dt > 0.0)) return fail(c, PD_ERR_ARG, "relaxation dt must be > 0");
    if (!mask || !p->aux || !p->vol || !p->inv_m) return fail(c, PD_ERR_ARG, "NULL mask, aux, vol or inv_m");
    HIP_TRY(c, hipSetDevice(c->device));
    pd_state_dev tmp{};
    tmp.mask = const_cast<uint64_t *>(mask);
    pdk::StepArgs a = make_args(p, &tmp);
    HIP_TRY(c, pdk::launch_adr_density(a, p, R, c->stream));
    return PD_OK;
}

static pd_status check_fac(pd_ctx *c, const pd_problem_dev *p, const pd_fac_dev *F) {
    if (!F) return fail(c, PD_ERR_ARG, "F is NULL");
    if (!F->bond_ij || !F->bond_pos || !F->bid || !F->ce || !F->xi || !F->cth || !F->ke || !F->kth ||
        !F->kth_diag || !F->E || !F->theta || !F->dirty)
        return fail(c, PD_ERR_ARG, "F has a NULL array");
    if (F->dim != p->dim) return fail(c, PD_ERR_ARG, "F dim differs from the problem");
    if (F->nb < 0 || F->n_words <= 0 || F->n_words >= ((int64_t)1 << 31) || p->n_slices <= 0 ||
        F->n_words % (256 * p->n_slices) != 0 || 2 * F->nb > F->n_words)
        return fail(c, PD_ERR_SIZE, "F sizes do not fit the problem (nb %lld, n_words %lld)", (long long)F->nb,
                    (long long)F->n_words);
    const void *al[] = {F->ce, F->cth, F->ke, F->kth, F->kth_diag, F->bid, F->bond_ij, F->bond_pos};
    for (const void *q : al)
        if (reinterpret_cast<uintptr_t>(q) % 32 != 0) return fail(c, PD_ERR_ARG, "F arrays must be 32-byte aligned");
    if (!p->vol || !p->inv_m) return fail(c, PD_ERR_ARG, "problem vol/inv_m is NULL");
    return PD_OK;
}

pd_status pd_fac_assemble(pd_ctx *c, const pd_problem_dev *p, const uint64_t *mask, pd_fac_dev *F) {
    if (!c) return PD_ERR_ARG;
    pd_status s = check_problem(c, p);
    if (s != PD_OK) return s;
    if ((s = check_fac(c, p, F)) != PD_OK) return s;
    if (!mask || !p->aux) return fail(c, PD_ERR_ARG, "NULL mask or aux (call pd_state_init first)");
    HIP_TRY(c, hipSetDevice(c->device));
    pd_state_dev tmp{};
    tmp.mask = const_cast<uint64_t *>(mask);
    pdk::StepArgs a = make_args(p, &tmp);
    HIP_TRY(c, pdk::launch_fac_assemble(a, p, F, c->stream));
    F->assembled = 1;
    return PD_OK;
}

pd_status pd_fac_apply(pd_ctx *c, const pd_problem_dev *p, pd_fac_dev *F, const pd_state_dev *st, double *f) {
    if (!c) return PD_ERR_ARG;
    pd_status s = check_problem(c, p);
    if (s != PD_OK) return s;
    if ((s = check_fac(c, p, F)) != PD_OK) return s;
    if ((s = check_state(c, st, false)) != PD_OK) return s;
    if (!F->assembled) return fail(c, PD_ERR_STATE, "the factored operators are not assembled");
    if (!f) return fail(c, PD_ERR_ARG, "f is NULL");
    if (!p->aux) return fail(c, PD_ERR_ARG, "aux is NULL (call pd_state_init first)");
    HIP_TRY(c, hipSetDevice(c->device));
    pdk::StepArgs a = make_args(p, st);
    a.f_out = reinterpret_cast<double4 *>(f);
    HIP_TRY(c, pdk::launch_fac_extension(a, p, F, st->cur, false, c->stream));
    HIP_TRY(c, pdk::launch_fac_dilatation(a, p, F, c->stream));
    HIP_TRY(c, pdk::launch_fac_force(a, p, F, st->cur, false, c->stream));
    return PD_OK;
}

static pd_status check_bsr(pd_ctx *c, const pd_problem_dev *p, const pd_bsr_dev *K) {
    if (!K) return fail(c, PD_ERR_ARG, "K is NULL");
    if (!K->row_ptr || !K->col || !K->vals || !K->bc || !K->dirty) return fail(c, PD_ERR_ARG, "K has a NULL array");
    if (K->dim != p->dim) return fail(c, PD_ERR_ARG, "K dim differs from the problem");
    if (!p->lat4) return fail(c, PD_ERR_ARG, "problem lat4 is NULL");
    if (K->max_row_blocks < 0 || K->reach < 0 || K->reach > 64) return fail(c, PD_ERR_SIZE, "bad K pattern sizes");
    const size_t lds = pdk::bsr_assemble_lds(p->dim, K->max_row_blocks, K->reach);
    if (lds > 160 * 1024) return fail(c, PD_ERR_UNSUPPORTED, "a row of K does not fit in LDS (%zu bytes)", lds);
    return PD_OK;
}

pd_status pd_assemble_K(pd_ctx *c, const pd_problem_dev *p, const uint64_t *mask, pd_bsr_dev *K) {
    if (!c) return PD_ERR_ARG;
    pd_status s = check_problem(c, p);
    if (s != PD_OK) return s;
    if ((s = check_bsr(c, p, K)) != PD_OK) return s;
    if (!mask || !p->aux) return fail(c, PD_ERR_ARG, "NULL mask or aux (call pd_state_init first)");
    HIP_TRY(c, hipSetDevice(c->device));
    pd_state_dev tmp{};
    tmp.mask = const_cast<uint64_t *>(mask);
    pdk::StepArgs a = make_args(p, &tmp);
    const size_t lds = pdk::bsr_assemble_lds(p->dim, K->max_row_blocks, K->reach);
    HIP_TRY(c, pdk::set_bsr_lds_limit(p->dim, K->fp32 != 0, lds));
    HIP_TRY(c, pdk::launch_bsr_prep_assemble(a, p, K, true, 0, c->stream));
    K->assembled = 1;
    return PD_OK;
}

pd_status pd_bsr_apply(pd_ctx *c, const pd_problem_dev *p, const pd_bsr_dev *K, const pd_state_dev *st, double *f) {
    if (!c) return PD_ERR_ARG;
    pd_status s = check_problem(c, p);
    if (s != PD_OK) return s;
    if ((s = check_bsr(c, p, K)) != PD_OK) return s;
    if ((s = check_state(c, st, false)) != PD_OK) return s;
    if (!K->assembled) return fail(c, PD_ERR_STATE, "K is not assembled");
    if (!f) return fail(c, PD_ERR_ARG, "f is NULL");
    HIP_TRY(c, hipSetDevice(c->device));
    pdk::StepArgs a = make_args(p, st);
    a.f_out = reinterpret_cast<double4 *>(f);
    HIP_TRY(c, pdk::launch_bsr_spmv(a, p, K, st->cur, false, c->stream));
    return PD_OK;
}

int64_t pd_static_workspace(int64_t n_pad) { return n_pad > 0 ? pdk::cg_workspace_doubles(n_pad) : 0; }

pd_status pd_static_solve(pd_ctx *c, const pd_problem_dev *p, const pd_bsr_dev *K, pd_state_dev *st,
                          const pd_cg_opts *o, double *work, pd_cg_report *rep) {
    if (!c) return PD_ERR_ARG;
    pd_status s = check_problem(c, p);
    if (s != PD_OK) return s;
    if (!o || !work) return fail(c, PD_ERR_ARG, "NULL options or workspace");
    if (!K && o->matrix_free != 1) return fail(c, PD_ERR_ARG, "K is NULL (allowed with matrix_free = 1 only)");
    if (K && (s = check_bsr(c, p, K)) != PD_OK) return s;
    if ((s = check_state(c, st, false)) != PD_OK) return s;
    if (K && !K->assembled) return fail(c, PD_ERR_STATE, "K is not assembled");
    if (K && K->fp32) return fail(c, PD_ERR_UNSUPPORTED, "the static solve needs K in double");
    if (!(o->tol > 0.0) || o->max_iter <= 0 || o->check_every <= 0 || (o->matrix_free != 0 && o->matrix_free != 1))
        return fail(c, PD_ERR_ARG, "bad solver options");
    if (reinterpret_cast<uintptr_t>(work) % 32 != 0) return fail(c, PD_ERR_ARG, "workspace must be 32-byte aligned");
    if (!p->aux || !p->fext) return fail(c, PD_ERR_ARG, "aux/fext are NULL (call pd_state_init first)");
    HIP_TRY(c, hipSetDevice(c->device));
    pdk::StepArgs a = make_args(p, st);
    const int cur = st->cur;
    HIP_TRY(c, pdk::launch_cg_start(a, K, work, cur, o->matrix_free != 0, c->stream));
    const double *scal = pdk::cg_scalars(work, p->n_pad);
    double h[8] = {0};
    int it = 0;
    bool conv = false;
    HIP_TRY(c, hipMemcpyAsync(h, scal, sizeof(h), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    conv = h[4] == 0.0;  // zero residual: u0 is already in equilibrium
    while (!conv && it < o->max_iter) {
        const int chunk = std::min(o->check_every, o->max_iter - it);
        for (int k = 0; k < chunk; k++)
            HIP_TRY(c, pdk::launch_cg_iteration(a, K, work, 0.0, cur, o->matrix_free != 0, c->stream));
        it += chunk;
        HIP_TRY(c, hipMemcpyAsync(h, scal, sizeof(h), hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        if (!std::isfinite(h[5])) return fail(c, PD_ERR_UNSTABLE, "non-finite residual in the static solve");
        conv = h[5] <= o->tol;
    }
    HIP_TRY(c, pdk::launch_cg_finish(a, K, work, cur, c->stream));
    HIP_TRY(c, pdk::launch_shadow_invalidate(reinterpret_cast<pd_ctl *>(st->ctl), c->stream));
    if (rep) {
        rep->iterations = (int32_t)h[6];
        rep->converged = conv ? 1 : 0;
        rep->rel_residual = h[5];
    }
    return PD_OK;
}

int64_t pd_newmark_workspace(int64_t n_pad) { return n_pad > 0 ? pdk::nm_workspace_doubles(n_pad) : 0; }

pd_status pd_newmark_step(pd_ctx *c, const pd_problem_dev *p, const pd_bsr_dev *K, pd_state_dev *st, int32_t nsteps,
                          const pd_newmark_opts *o, double *work, pd_cg_report *rep) {
    if (!c) return PD_ERR_ARG;
    pd_status s = check_problem(c, p);
    if (s != PD_OK) return s;
    if (!o || !work) return fail(c, PD_ERR_ARG, "NULL options or workspace");
    if (!K && o->cg.matrix_free != 1) return fail(c, PD_ERR_ARG, "K is NULL (allowed with matrix_free = 1 only)");
    if (K && (s = check_bsr(c, p, K)) != PD_OK) return s;
    if ((s = check_state(c, st, false)) != PD_OK) return s;
    if (K && !K->assembled) return fail(c, PD_ERR_STATE, "K is not assembled");
    if (K && K->fp32) return fail(c, PD_ERR_UNSUPPORTED, "the implicit step needs K in double");
    if (nsteps < 0) return fail(c, PD_ERR_ARG, "nsteps < 0");
    if (!(o->dt > 0.0) || !std::isfinite(o->dt)) return fail(c, PD_ERR_ARG, "dt must be positive and finite");
    if (!(o->cg.tol > 0.0) || o->cg.max_iter <= 0 || o->cg.check_every <= 0 ||
        (o->cg.matrix_free != 0 && o->cg.matrix_free != 1))
        return fail(c, PD_ERR_ARG, "bad solver options");
    if (o->breaking != 0 && o->breaking != 1) return fail(c, PD_ERR_ARG, "breaking must be 0 or 1");
    if (reinterpret_cast<uintptr_t>(work) % 32 != 0) return fail(c, PD_ERR_ARG, "workspace must be 32-byte aligned");
    if (!p->aux || !p->fext) return fail(c, PD_ERR_ARG, "aux/fext are NULL (call pd_state_init first)");
    HIP_TRY(c, hipSetDevice(c->device));
    const double *scal = pdk::cg_scalars(work, p->n_pad);
    int total = 0;
    bool all_conv = true;
    double worst = 0.0;
    for (int n = 0; n < nsteps; n++) {
        pdk::StepArgs a = make_args(p, st);
        const int cur = st->cur;
        if (o->breaking) {
            // critical stretch at u_n, then K re-assembled around new breaks
            if (K) {
                HIP_TRY(c, pdk::launch_break_mark(a, p, K, cur, c->stream));
                HIP_TRY(c, pdk::launch_bsr_prep_assemble(a, p, K, false, cur, c->stream));
            } else {
                // no stored K: the double force pass 1 with its breaking test
                // (its dilatation and force outputs are scratch here)
                const bool tiled = pdk::tiled64_supported(a);
                HIP_TRY(c, tiled ? pdk::launch_tpass1_f64(a, cur, true, c->stream)
                                 : pdk::launch_pass1_f64(a, cur, true, 256, c->stream));
            }
        }
        HIP_TRY(c, pdk::launch_nm_start(a, K, work, o->dt, cur, o->cg.matrix_free != 0, c->stream));
        double h[8] = {0};
        int it = 0;
        HIP_TRY(c, hipMemcpyAsync(h, scal, sizeof(h), hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        bool conv = h[4] == 0.0;
        while (!conv && it < o->cg.max_iter) {
            const int chunk = std::min(o->cg.check_every, o->cg.max_iter - it);
            for (int k = 0; k < chunk; k++)
                HIP_TRY(c, pdk::launch_cg_iteration(a, K, work, o->dt, cur, o->cg.matrix_free != 0, c->stream));
            it += chunk;
            HIP_TRY(c, hipMemcpyAsync(h, scal, sizeof(h), hipMemcpyDeviceToHost, c->stream));
            HIP_TRY(c, hipStreamSynchronize(c->stream));
            if (!std::isfinite(h[5])) return fail(c, PD_ERR_UNSTABLE, "non-finite residual in the implicit step");
            conv = h[5] <= o->cg.tol;
        }
        HIP_TRY(c, pdk::launch_nm_finish(a, K, work, o->dt, cur, c->stream));
        HIP_TRY(c, pdk::launch_shadow_invalidate(reinterpret_cast<pd_ctl *>(st->ctl), c->stream));
        st->cur = cur ^ 1;
        total += (int)h[6];
        all_conv = all_conv && conv;
        worst = std::max(worst, conv && h[4] == 0.0 ? 0.0 : h[5]);
    }
    if (rep) {
        rep->iterations = total;
        rep->converged = all_conv ? 1 : 0;
        rep->rel_residual = worst;
    }
    return PD_OK;
}

pd_status pd_autotune(pd_ctx *c, const pd_problem_dev *p, pd_state_dev *st, int32_t precision, int32_t trial_steps,
                      pd_tune_result *out) {
    if (!c) return PD_ERR_ARG;
    pd_status s = check_problem(c, p);
    if (s != PD_OK) return s;
    if (precision != PD_FP64 && precision != PD_FP32_RECHECK) return fail(c, PD_ERR_ARG, "unknown precision");
    if ((s = check_state(c, st, precision == PD_FP32_RECHECK)) != PD_OK) return s;
    if (!out || trial_steps < 1 || trial_steps > 10000) return fail(c, PD_ERR_ARG, "bad tuning arguments");
    if (!p->aux || !p->fext) return fail(c, PD_ERR_ARG, "aux/fext are NULL (call pd_state_init first)");
    HIP_TRY(c, hipSetDevice(c->device));
    std::memset(out, 0, sizeof(*out));
    int nc = 0;
    int ck[8], cb[8];
    {
        pdk::StepArgs a = make_args(p, st);
        if (precision == PD_FP32_RECHECK ? pdk::tiled_supported(a) : pdk::tiled64_supported(a)) {
            ck[nc] = 2;
            cb[nc++] = 0;
        }
        if (precision == PD_FP32_RECHECK && pdk::supertiles_supported(a)) {
            ck[nc] = 3;
            cb[nc++] = 0;
        }
        // 2D: one tile per workgroup as well as one per wave
        pdk::StepArgs a1 = a;
        a1.one_tile_per_group = 1;
        if (p->dim == 2 && (precision == PD_FP32_RECHECK ? pdk::tiled_supported(a1) : pdk::tiled64_supported(a1))) {
            ck[nc] = 4;
            cb[nc++] = 0;
        }
    }
    for (int b : {64, 128, 256}) {
        ck[nc] = 1;
        cb[nc++] = b;
    }
    hipEvent_t e0, e1;
    HIP_TRY(c, hipEventCreate(&e0));
    HIP_TRY(c, hipEventCreate(&e1));
    double best = 1e300;
    for (int i = 0; i < nc; i++) {
        pd_step_opts o{};
        o.precision = precision;
        o.form = PD_MATRIX_FREE;
        o.kernel = ck[i];
        o.block = cb[i];
        s = pd_step(c, p, st, 2, &o, nullptr, nullptr);
        if (s == PD_OK && hipEventRecord(e0, c->stream) != hipSuccess) s = PD_ERR_HIP;
        if (s == PD_OK) s = pd_step(c, p, st, trial_steps, &o, nullptr, nullptr);
        if (s == PD_OK && hipEventRecord(e1, c->stream) != hipSuccess) s = PD_ERR_HIP;
        float ms = 0.0f;
        if (s == PD_OK && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
            s = PD_ERR_HIP;
        if (s != PD_OK) {
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            return s;
        }
        out->cand_kernel[i] = ck[i];
        out->cand_block[i] = cb[i];
        out->cand_ms[i] = (double)ms / trial_steps;
        if (out->cand_ms[i] < best) {
            best = out->cand_ms[i];
            out->kernel = ck[i];
            out->block = cb[i];
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    out->n_candidates = nc;
    out->ms_per_step = best;
    return PD_OK;
}

pd_status pd_damage(pd_ctx *c, const pd_problem_dev *p, const uint64_t *mask, double *phi) {
    if (!c) return PD_ERR_ARG;
    pd_status s = check_problem(c, p);
    if (s != PD_OK) return s;
    if (!mask || !phi) return fail(c, PD_ERR_ARG, "NULL mask/phi");
    HIP_TRY(c, hipSetDevice(c->device));
    pdk::DamageArgs a{};
    a.n_slices = p->n_slices;
    a.slice_ptr = p->slice_ptr;
    a.words = p->words;
    a.mask = mask;
    a.vol = p->vol;
    a.phi = phi;
    HIP_TRY(c, pdk::launch_damage(a, c->stream));
    return PD_OK;
}

pd_status pd_energy(pd_ctx *c, const pd_problem_dev *p, pd_state_dev *st, double *f_scratch, double *kinetic,
                    double *strain) {
    if (!c) return PD_ERR_ARG;
    pd_status s = check_problem(c, p);
    if (s != PD_OK) return s;
    if ((s = check_state(c, st, false)) != PD_OK) return s;
    if (!f_scratch || !kinetic || !strain) return fail(c, PD_ERR_ARG, "NULL output");
    if (reinterpret_cast<uintptr_t>(f_scratch) % 32 != 0) return fail(c, PD_ERR_ARG, "f_scratch must be 32-byte aligned");
    if (!p->aux) return fail(c, PD_ERR_ARG, "aux is NULL (call pd_state_init first)");
    HIP_TRY(c, hipSetDevice(c->device));
    const pdk::StepArgs a = make_args(p, st);
    // partials, then the four sums, inside the caller's n_pad*4 doubles
    double4 *part = reinterpret_cast<double4 *>(f_scratch);
    double *out = f_scratch + 4 * pdk::reduce_parts(p->n_pad);
    HIP_TRY(c, pdk::launch_energy(a, st->cur, false, part, out, 4, nullptr, c->stream));
    double h[4];
    HIP_TRY(c, hipMemcpyAsync(h, out, sizeof(h), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    *kinetic = h[0];
    *strain = h[1];
    return PD_OK;
}

pd_status pd_energy_noalloc(pd_ctx *c, const pd_problem_dev *p, const pd_state_dev *st, double *out) {
    if (!c) return PD_ERR_ARG;
    pd_status s = check_problem(c, p);
    if (s != PD_OK) return s;
    if ((s = check_state(c, st, false)) != PD_OK) return s;
    if (!out) return fail(c, PD_ERR_ARG, "out is NULL");
    if (reinterpret_cast<uintptr_t>(out) % 8 != 0) return fail(c, PD_ERR_ARG, "out must be 8-byte aligned");
    if (!p->aux) return fail(c, PD_ERR_ARG, "aux is NULL (call pd_state_init first)");
    if (pdk::reduce_parts(p->n_pad) > PD_NOALLOC_PARTS)
        return fail(c, PD_ERR_SIZE, "n_pad %lld exceeds the %lld rows of the fixed reduction array",
                    (long long)p->n_pad, (long long)PD_NOALLOC_MAX_ROWS);
    if (!c->scratch_dev) return fail(c, PD_ERR_STATE, "no scratch address for this device");
    HIP_TRY(c, hipSetDevice(c->device));
    pd_state_dev tmp = *st;
    const pdk::StepArgs a = make_args(p, &tmp);
    HIP_TRY(c, pdk::launch_energy(a, st->cur, false, c->scratch_dev, out, 2, nullptr, c->stream));
    return PD_OK;
}

pd_status pd_stable_dt(pd_ctx *c, const pd_problem_dev *p, pd_state_dev *st, double *f_scratch, int32_t iters,
                       uint64_t seed, double *dt_crit) {
    if (!c) return PD_ERR_ARG;
    pd_status s = check_problem(c, p);
    if (s != PD_OK) return s;
    if ((s = check_state(c, st, false)) != PD_OK) return s;
    if (!f_scratch || !dt_crit || iters < 1 || !p->aux) return fail(c, PD_ERR_ARG, "bad arguments");
    HIP_TRY(c, hipSetDevice(c->device));
    if ((s = need_parts(c, p->n_pad)) != PD_OK) return s;
    double4 *x = reinterpret_cast<double4 *>(st->uv[st->cur]);
    double4 *y = reinterpret_cast<double4 *>(st->uv[st->cur ^ 1]);
    pd_ctl *ctl = reinterpret_cast<pd_ctl *>(st->ctl);
    // u and v are overwritten: the FP32 shadow no longer describes them
    HIP_TRY(c, pdk::launch_shadow_invalidate(ctl, c->stream));
    HIP_TRY(c, pdk::launch_pi_init(p->n_pad, p->dim, p->aux, x, seed, c->stream));
    double lam = 0.0;
    for (int it = 0; it < iters; it++) {
        if ((s = pd_force(c, p, st, PD_FP64, f_scratch, nullptr)) != PD_OK) return s;
        HIP_TRY(c, pdk::launch_pi_step(p->n_pad, p->dim, p->aux, p->spec, x,
                                       reinterpret_cast<const double4 *>(f_scratch), y, ctl, c->part, c->stream));
        if (it == iters - 1) {
            HIP_TRY(c, hipMemcpyAsync(c->host_ctl, st->ctl, kCtlHead, hipMemcpyDeviceToHost, c->stream));
            HIP_TRY(c, hipStreamSynchronize(c->stream));
            lam = c->host_ctl->red[0] / c->host_ctl->red[1];
        }
    }
    if (!(lam > 0.0)) return fail(c, PD_ERR_UNSTABLE, "power iteration did not converge");
    *dt_crit = 2.0 / std::sqrt(lam);
    return PD_OK;
}

}  // extern "C"
