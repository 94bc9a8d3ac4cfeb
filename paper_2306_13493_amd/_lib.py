"""ctypes declarations of the C ABI in include/cesmlmc.h (marshalling only).

Loading fails loudly when libcesmlmc.so has not been built: there is no
fallback implementation.
"""

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libcesmlmc.so")

c_int32 = ctypes.c_int32
c_int64 = ctypes.c_int64
c_uint32 = ctypes.c_uint32
c_uint64 = ctypes.c_uint64
c_double = ctypes.c_double
c_size_t = ctypes.c_size_t
c_void_p = ctypes.c_void_p
c_dptr = ctypes.c_void_p  # device pointers are passed as integers

CES_OK = 0
ERRORS = {-1: "CES_ERR_ARG", -2: "CES_ERR_NOT_PSD", -3: "CES_ERR_NOMEM", -4: "CES_ERR_NOCONV",
          -5: "CES_ERR_DEVICE", -6: "CES_ERR_BUSY"}


class LevelDesc(ctypes.Structure):
    _fields_ = [
        ("struct_size", c_int32), ("cov_kind", c_int32), ("nu", c_double), ("lambda_", c_double),
        ("sigma2", c_double), ("m_fine", c_int32), ("level_kind", c_int32), ("tau_fine", c_int64),
        ("tau_coarse", c_int64), ("psd_policy", c_int32), ("periodization", c_int32),
        ("max_pad_factor", c_int32), ("field_mode", c_int32), ("precision", c_int32), ("bc", c_int32),
        ("qoi", c_int32), ("coupling", c_int32), ("qoi_x", c_double), ("qoi_y", c_double), ("f_value", c_double),
        ("cg_rtol", c_double), ("cg_max_iter", c_int32), ("stream", c_uint32), ("mg_cycle", c_int32),
        ("reserved", c_int32)]


class PlanInfo(ctypes.Structure):
    _fields_ = [
        ("n", c_int32), ("J", c_int32), ("lam_min", c_double), ("lam_max", c_double),
        ("n_clamped", c_int64), ("tau_fine", c_int64), ("tau_coarse", c_int64),
        ("boundary_gap", c_double), ("mg_levels", c_int32), ("n_coarse", c_int32),
        ("bytes_per_sample", c_size_t)]


class ProfileEntry(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("launches", c_int64), ("total_ms", c_double), ("bytes", c_double)]


class Request(ctypes.Structure):
    _fields_ = [("plan", c_void_p), ("seed", c_uint64), ("first_sample", c_uint64), ("count", c_int64),
                ("y", c_dptr), ("q_fine", c_dptr), ("q_coarse", c_dptr), ("iters", c_dptr), ("status", c_dptr)]


class Schedule(ctypes.Structure):
    _fields_ = [("depth", c_int32), ("max_lanes", c_int32), ("chunk_samples", c_int64), ("graphs", c_int32),
                ("reserved", c_int32)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", c_int64), ("completed", c_int64), ("failed", c_int64), ("queued", c_int64),
                ("admitted", c_int64), ("samples_done", c_int64), ("mem_in_use", c_size_t),
                ("mem_peak", c_size_t), ("plans_cached", c_int32), ("reserved", c_int32)]


MLMC_MAX_LEVELS = 16


class MlmcOpts(ctypes.Structure):
    _fields_ = [("struct_size", c_int32), ("eps", c_double), ("l_start", c_int32), ("reserved0", c_int32),
                ("n_pilot", c_int64), ("theta", c_double), ("alpha", c_double), ("cost_model", c_int32),
                ("max_rounds", c_int32), ("seed", c_uint64)]


class MlmcResult(ctypes.Structure):
    _fields_ = [("estimate", c_double), ("variance", c_double), ("bias", c_double), ("alpha", c_double),
                ("beta", c_double), ("gamma", c_double), ("levels", c_int32), ("converged", c_int32),
                ("rounds", c_int32), ("reserved", c_int32), ("n", c_int64 * MLMC_MAX_LEVELS),
                ("mean", c_double * MLMC_MAX_LEVELS), ("var", c_double * MLMC_MAX_LEVELS),
                ("cost", c_double * MLMC_MAX_LEVELS)]


class MlqmcOpts(ctypes.Structure):
    _fields_ = [("struct_size", c_int32), ("l_start", c_int32), ("eps", c_double), ("n_pilot", c_int64),
                ("theta", c_double), ("alpha", c_double), ("cost_model", c_int32), ("max_rounds", c_int32),
                ("seed", c_uint64)]


class SmoothingStats(ctypes.Structure):
    _fields_ = [("struct_size", c_int32), ("reserved", c_int32), ("n", c_int64), ("mean", c_double),
                ("mean_abs", c_double), ("var", c_double), ("mean_q", c_double), ("mean_q_smoothed", c_double)]


# name -> (restype, argtypes); every function declared in include/cesmlmc.h
SIGNATURES = {
    "ces_level_desc_default": (None, [ctypes.POINTER(LevelDesc)]),
    "ces_context_create": (c_int32, [c_int32, c_size_t, ctypes.POINTER(c_void_p)]),
    "ces_context_destroy": (c_int32, [c_void_p]),
    "ces_plan_create": (c_int32, [c_void_p, ctypes.POINTER(LevelDesc), ctypes.POINTER(c_void_p)]),
    "ces_plan_info_get": (c_int32, [c_void_p, ctypes.POINTER(PlanInfo)]),
    "ces_plan_destroy": (c_int32, [c_void_p]),
    "ces_sample": (c_int32, [c_void_p, c_uint64, c_uint64, c_int64, c_dptr, c_dptr, c_dptr, c_dptr,
                             c_dptr, c_void_p]),
    "ces_sample_noalloc": (c_int32, [c_void_p, c_uint64, c_uint64, c_int64, c_dptr, c_dptr, c_dptr, c_dptr,
                                     c_dptr, c_void_p]),
    "ces_sample_batch": (c_int32, [c_void_p, ctypes.POINTER(Request), c_int32, c_void_p]),
    "ces_schedule_get": (c_int32, [c_void_p, ctypes.POINTER(Schedule)]),
    "ces_schedule_set": (c_int32, [c_void_p, ctypes.POINTER(Schedule)]),
    "ces_autotune": (c_int32, [c_void_p, ctypes.POINTER(Request), c_int32, c_void_p, ctypes.POINTER(Schedule),
                               ctypes.POINTER(c_double)]),
    "ces_server_create": (c_int32, [c_void_p, c_size_t, c_int32, ctypes.POINTER(c_void_p)]),
    "ces_server_submit": (c_int32, [c_void_p, ctypes.POINTER(LevelDesc), c_uint64, c_uint64, c_int64, c_void_p,
                                    c_void_p, ctypes.POINTER(c_int64)]),
    "ces_server_poll": (c_int32, [c_void_p, c_int64, ctypes.POINTER(c_int32), ctypes.POINTER(c_double)]),
    "ces_server_drain": (c_int32, [c_void_p]),
    "ces_server_get_stats": (c_int32, [c_void_p, ctypes.POINTER(ServerStats)]),
    "ces_server_destroy": (c_int32, [c_void_p]),
    "ces_mlmc_opts_default": (None, [ctypes.POINTER(MlmcOpts)]),
    "ces_mlmc_run": (c_int32, [c_void_p, ctypes.POINTER(c_void_p), ctypes.POINTER(c_void_p), c_int32,
                               ctypes.POINTER(MlmcOpts), c_void_p, ctypes.POINTER(MlmcResult)]),
    "ces_mlmc_run_checkpointed": (c_int32, [c_void_p, ctypes.POINTER(c_void_p), ctypes.POINTER(c_void_p), c_int32,
                                            ctypes.POINTER(MlmcOpts), ctypes.c_char_p, c_int32, c_void_p,
                                            ctypes.POINTER(MlmcResult)]),
    "ces_mlmc_coarsest_mesh": (c_int32, [ctypes.POINTER(LevelDesc), ctypes.POINTER(c_int32)]),
    "ces_tau_rule": (c_int32, [c_int32, c_double, c_int32, c_int32, c_double, c_double, ctypes.POINTER(c_int64),
                               ctypes.POINTER(c_double)]),
    "ces_smoothing_error": (c_int32, [c_void_p, c_void_p, c_void_p, c_uint64, c_uint64, c_int64, c_void_p,
                                      ctypes.POINTER(SmoothingStats)]),
    "ces_lattice_cbc": (c_int32, [c_int32, c_int32, c_void_p, c_void_p]),
    "ces_plan_lattice_order": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p]),
    "ces_plan_set_lattice": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_int32]),
    "ces_plan_set_lattice_default": (c_int32, [c_void_p, c_int32, c_int32, c_int32]),
    "ces_mlqmc_opts_default": (None, [ctypes.POINTER(MlqmcOpts)]),
    "ces_mlqmc_run": (c_int32, [c_void_p, ctypes.POINTER(c_void_p), ctypes.POINTER(c_void_p), c_int32,
                                ctypes.POINTER(MlqmcOpts), c_void_p, ctypes.POINTER(MlmcResult)]),
    "ces_normals": (c_int32, [c_uint64, c_uint64, c_uint32, c_uint64, c_int64, c_dptr, c_void_p]),
    "ces_plan_eigenvalues": (c_int32, [c_void_p, c_void_p]),
    "ces_plan_mask": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "ces_field": (c_int32, [c_void_p, c_uint64, c_uint64, c_dptr, c_dptr, c_void_p]),
    "ces_solve": (c_int32, [c_void_p, c_int32, c_int64, c_dptr, c_dptr, c_dptr, c_void_p]),
    "ces_profile_enable": (c_int32, [c_int32]),
    "ces_profile_only": (c_int32, [ctypes.c_char_p]),
    "ces_profile_read": (c_int32, [ctypes.POINTER(ProfileEntry), c_int32, ctypes.POINTER(c_int32)]),
    "ces_last_error": (ctypes.c_char_p, []),
}

_lib = None


def load(path=LIB_PATH):
    """Load libcesmlmc.so and declare the ABI; raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libcesmlmc.so is not built (%s); run paper_2306_13493_amd.build.build()" % path)
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    d = LevelDesc()
    lib.ces_level_desc_default(ctypes.byref(d))
    if d.struct_size != ctypes.sizeof(LevelDesc):
        raise ImportError("ces_level_desc layout mismatch (%d vs %d)" % (d.struct_size, ctypes.sizeof(LevelDesc)))
    _lib = lib
    return lib


class CesError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (ERRORS.get(code, "?"), code, msg))
        self.code = code


def check(rc):
    if rc != CES_OK:
        raise CesError(rc, load().ces_last_error().decode(errors="replace"))
    return rc
