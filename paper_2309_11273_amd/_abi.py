"""ctypes declarations of the C ABI in include/pd.h (argument marshalling only)."""

from __future__ import annotations

import ctypes as C
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libpd.so")

P = C.c_void_p
i32, i64, u64, dbl = C.c_int32, C.c_int64, C.c_uint64, C.c_double

PD_OK = 0
STATUS = {0: "PD_OK", -1: "PD_ERR_ARG", -2: "PD_ERR_SIZE", -3: "PD_ERR_HIP", -4: "PD_ERR_UNSTABLE",
          -5: "PD_ERR_UNSUPPORTED", -6: "PD_ERR_STATE"}
PD_3D, PD_PLANE_STRESS, PD_PLANE_STRAIN = 0, 1, 2
PD_FP64, PD_FP32_RECHECK = 0, 1
PD_MATRIX_FREE, PD_BSR, PD_FACTORED = 0, 1, 2
PD_CTL_BYTES = 16640


class pd_body(C.Structure):
    _fields_ = [("n", i64), ("dim", i32), ("pad0", i32), ("lat", P), ("dx", dbl), ("origin", dbl * 3),
                ("delta", dbl), ("vol", P), ("specimen", P)]


class pd_cut(C.Structure):
    _fields_ = [("kind", i32), ("specimen", i32), ("p", dbl * 10)]


class pd_family_sizes(C.Structure):
    _fields_ = [("n", i64), ("n_pad", i64), ("n_slices", i64), ("n_words", i64), ("n_mask", i64),
                ("nnz", i64), ("n_bonds", i64), ("n_cut", i64), ("n_stencil", i32), ("max_row", i32),
                ("dim", i32), ("n_specimens", i32), ("n_tiles", i64), ("tile", i32 * 3),
                ("words_per_row", i32), ("reach", i32), ("n_halo", i32), ("n_box", i32),
                ("vol_uniform", C.c_float), ("pad_vu", i32)]


class pd_family_host(C.Structure):
    _fields_ = [("perm", P), ("row_of", P), ("slice_ptr", P), ("words", P), ("mask", P), ("stencil", P),
                ("stencil_off", P), ("vol", P), ("inv_m", P), ("spec", P), ("lat4", P), ("tile_org", P),
                ("tile_nbr", P), ("ktab", P), ("halo_map", P), ("halo_pos", P)]


class pd_spec(C.Structure):
    _fields_ = [("kp", dbl), ("G", dbl), ("A", dbl), ("rho", dbl), ("s0", dbl), ("dt", dbl),
                ("pad", dbl * 2)]


class pd_problem_dev(C.Structure):
    _fields_ = [("n_pad", i64), ("n_slices", i64), ("dim", i32), ("n_stencil", i32),
                ("n_specimens", i32), ("pad0", i32), ("slice_ptr", P), ("words", P), ("stencil", P),
                ("vol", P), ("inv_m", P), ("lat4", P), ("spec", P), ("aux", P), ("fext", P),
                ("ramp_steps", i64), ("stencil_off", P), ("tile_nbr", P), ("tile", i32 * 3), ("reach", i32),
                ("ktab", P), ("halo_map", P), ("halo_pos", P), ("n_pos", i32), ("vol_uniform", C.c_float),
                ("st_tiles", P), ("st_nbr", P), ("st_pos", P), ("st_ktab", P), ("n_st", i64),
                ("st_n_pos", i32), ("pad2", i32)]


class pd_st_sizes(C.Structure):
    _fields_ = [("n_st", i64), ("n_pos", i32), ("pad0", i32)]


class pd_state_dev(C.Structure):
    _fields_ = [("uv", P * 2), ("vel", P), ("qr", P), ("mask", P), ("ush", P * 2), ("qr32", P),
                ("dsum", P), ("fe32", P), ("fe64", P), ("qv32", P), ("ctl", P), ("cur", i32), ("pad0", i32)]


class pd_step_opts(C.Structure):
    _fields_ = [("precision", i32), ("form", i32), ("graph_chunk", i32), ("block", i32),
                ("check_every", i32), ("profile", i32), ("kernel", i32), ("extension", i32),
                ("energy_check", i32), ("pad0", i32), ("energy_growth", dbl)]


class pd_profile_stats(C.Structure):
    _fields_ = [("steps", i64), ("ms_pass1", dbl), ("ms_pass2", dbl), ("ms_extra", dbl)]


class pd_tune_result(C.Structure):
    _fields_ = [("kernel", i32), ("block", i32), ("n_candidates", i32), ("pad0", i32), ("ms_per_step", dbl),
                ("cand_kernel", i32 * 8), ("cand_block", i32 * 8), ("cand_ms", dbl * 8)]


class pd_step_report(C.Structure):
    _fields_ = [("step", i64), ("broken_total", i64), ("rechecks", i64), ("nonfinite", i32),
                ("pad0", i32), ("umax", dbl), ("min_margin", dbl), ("kinetic", dbl), ("strain", dbl),
                ("energy_step", i64)]


class pd_bsr_sizes(C.Structure):
    _fields_ = [("nnzb", i64), ("max_row_blocks", i32), ("reach", i32)]


class pd_bsr_dev(C.Structure):
    _fields_ = [("nnzb", i64), ("dim", i32), ("fp32", i32), ("max_row_blocks", i32), ("reach", i32),
                ("row_ptr", P), ("col", P), ("vals", P), ("bc", P), ("dirty", P), ("assembled", i32),
                ("pad0", i32)]


class pd_fac_sizes(C.Structure):
    _fields_ = [("nb", i64), ("n_words", i64)]


class pd_fac_dev(C.Structure):
    _fields_ = [("nb", i64), ("n_words", i64), ("dim", i32), ("assembled", i32),
                ("bond_ij", P), ("bond_pos", P), ("bid", P), ("ce", P), ("xi", P), ("cth", P),
                ("ke", P), ("kth", P), ("kth_diag", P), ("E", P), ("theta", P), ("dirty", P)]


class pd_adr_dev(C.Structure):
    _fields_ = [("dt", dbl), ("lambda_", P), ("f_prev", P), ("f_int", P), ("partial", P), ("stats", P)]


class pd_cg_opts(C.Structure):
    _fields_ = [("tol", dbl), ("max_iter", i32), ("check_every", i32), ("matrix_free", i32), ("reserved", i32)]


class pd_cg_report(C.Structure):
    _fields_ = [("iterations", i32), ("converged", i32), ("rel_residual", dbl)]


class pd_newmark_opts(C.Structure):
    _fields_ = [("dt", dbl), ("cg", pd_cg_opts), ("breaking", i32), ("reserved", i32)]


# name -> (restype, argtypes)
SIGNATURES = {
    "pd_version": (C.c_char_p, []),
    "pd_ctx_create": (i32, [C.POINTER(P), i32, P]),
    "pd_ctx_destroy": (i32, [P]),
    "pd_last_error": (C.c_char_p, [P]),
    "pd_profile_read": (i32, [P, C.POINTER(pd_profile_stats), i32]),
    "pd_autotune": (i32, [P, C.POINTER(pd_problem_dev), C.POINTER(pd_state_dev), i32, i32,
                          C.POINTER(pd_tune_result)]),
    "pd_critical_stretch": (i32, [i32, dbl, dbl, dbl, dbl, i32, C.POINTER(dbl)]),
    "pd_specimen_params": (i32, [i32, dbl, dbl, dbl, dbl, dbl, C.POINTER(pd_spec)]),
    "pd_build_family": (i32, [C.POINTER(pd_body), P, i32, C.POINTER(pd_family_sizes),
                              C.POINTER(pd_family_host)]),
    "pd_state_init": (i32, [P, C.POINTER(pd_problem_dev), P, i64, P, P, P, P, P, P, P,
                            C.POINTER(pd_state_dev), i64]),
    "pd_state_read": (i32, [P, C.POINTER(pd_problem_dev), P, i64, C.POINTER(pd_state_dev), P, P]),
    "pd_get_step": (i32, [P, C.POINTER(pd_state_dev), C.POINTER(i64)]),
    "pd_tile_kernels_apply": (i32, [C.POINTER(pd_problem_dev), C.POINTER(pd_state_dev), i32, C.POINTER(i32)]),
    "pd_force": (i32, [P, C.POINTER(pd_problem_dev), C.POINTER(pd_state_dev), i32, P, P]),
    "pd_energy_noalloc": (i32, [P, C.POINTER(pd_problem_dev), C.POINTER(pd_state_dev), P]),
    "pd_step": (i32, [P, C.POINTER(pd_problem_dev), C.POINTER(pd_state_dev), i64,
                      C.POINTER(pd_step_opts), C.POINTER(pd_bsr_dev), C.POINTER(pd_step_report)]),
    "pd_build_supertiles": (i32, [C.POINTER(pd_family_sizes), C.POINTER(pd_family_host), C.POINTER(pd_st_sizes),
                                  P, P, P, P]),
    "pd_bsr_pattern": (i32, [C.POINTER(pd_family_sizes), C.POINTER(pd_family_host),
                             C.POINTER(pd_bsr_sizes), P, P]),
    "pd_assemble_K": (i32, [P, C.POINTER(pd_problem_dev), P, C.POINTER(pd_bsr_dev)]),
    "pd_bsr_apply": (i32, [P, C.POINTER(pd_problem_dev), C.POINTER(pd_bsr_dev),
                           C.POINTER(pd_state_dev), P]),
    "pd_fac_pattern": (i32, [C.POINTER(pd_family_sizes), C.POINTER(pd_family_host),
                             C.POINTER(pd_fac_sizes), P, P, P]),
    "pd_fac_assemble": (i32, [P, C.POINTER(pd_problem_dev), P, C.POINTER(pd_fac_dev)]),
    "pd_fac_apply": (i32, [P, C.POINTER(pd_problem_dev), C.POINTER(pd_fac_dev), C.POINTER(pd_state_dev), P]),
    "pd_fac_step": (i32, [P, C.POINTER(pd_problem_dev), C.POINTER(pd_state_dev), i64,
                          C.POINTER(pd_step_opts), C.POINTER(pd_fac_dev), C.POINTER(pd_step_report)]),
    "pd_force_finite": (i32, [P, C.POINTER(pd_problem_dev), C.POINTER(pd_state_dev), P, P]),
    "pd_adr_density": (i32, [P, C.POINTER(pd_problem_dev), P, C.POINTER(pd_adr_dev)]),
    "pd_adr_step": (i32, [P, C.POINTER(pd_problem_dev), C.POINTER(pd_state_dev), i64,
                          C.POINTER(pd_step_opts), C.POINTER(pd_adr_dev), C.POINTER(pd_step_report)]),
    "pd_static_workspace": (i64, [i64]),
    "pd_newmark_workspace": (i64, [i64]),
    "pd_newmark_step": (i32, [P, C.POINTER(pd_problem_dev), C.POINTER(pd_bsr_dev), C.POINTER(pd_state_dev), i32,
                              C.POINTER(pd_newmark_opts), P, C.POINTER(pd_cg_report)]),
    "pd_static_solve": (i32, [P, C.POINTER(pd_problem_dev), C.POINTER(pd_bsr_dev), C.POINTER(pd_state_dev),
                              C.POINTER(pd_cg_opts), P, C.POINTER(pd_cg_report)]),
    "pd_damage": (i32, [P, C.POINTER(pd_problem_dev), P, P]),
    "pd_energy": (i32, [P, C.POINTER(pd_problem_dev), C.POINTER(pd_state_dev), P,
                        C.POINTER(dbl), C.POINTER(dbl)]),
    "pd_stable_dt": (i32, [P, C.POINTER(pd_problem_dev), C.POINTER(pd_state_dev), P, i32, u64,
                           C.POINTER(dbl)]),
}

_lib = None


def load():
    """Load the in-tree libpd.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libpd.so is not built (run python -m paper_2309_11273_amd.build)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class PDError(RuntimeError):
    def __init__(self, fn: str, status: int, msg: str = ""):
        super().__init__(f"{fn} returned {STATUS.get(status, status)}: {msg}")
        self.status = status


def check(fn: str, status: int, ctx=None):
    if status != PD_OK:
        msg = ""
        if ctx is not None:
            m = load().pd_last_error(ctx)
            msg = m.decode() if m else ""
        raise PDError(fn, status, msg)
