"""ctypes declarations of the celmi C ABI (include/celmi.h).  Argument marshalling only.

Importing this module loads paper_1803_00113_amd/libcelmi.so and raises ImportError if it
is missing: there is no fallback implementation.
"""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcelmi.so")

MAX_PSF = 4
MAX_PROFILE = 8
N_COLOUR_COMPONENTS = 8
N_THETA = 32
N_PARAM = 27
N_Z = 16

CEL_OK, CEL_EINVAL, CEL_ENOMEM, CEL_EHIP, CEL_EUNSUPPORTED, CEL_ESCRATCH = 0, -1, -2, -3, -4, -5
STATIC_SCRATCH_BYTES = 256 << 20
ST_SKIPPED, ST_ACCEPTED, ST_REJECTED, ST_CONVERGED, ST_NONFINITE = 0, 1, 2, 3, 4
DEVERR_NONFINITE_OBJECTIVE, DEVERR_NONFINITE_STEP, DEVERR_NONFINITE_HESSIAN, DEVERR_BAD_INDEX = 1, 2, 4, 8
MAX_EIGEN = 4
PSF_MAX_SIDE = 63


class CelImage(C.Structure):
    _fields_ = [("band", C.c_int32), ("H", C.c_int32), ("W", C.c_int32), ("n_psf", C.c_int32),
                ("psf", (C.c_double * 6) * MAX_PSF), ("A", (C.c_double * 2) * 2), ("b", C.c_double * 2),
                ("iota", C.c_double), ("sky_qh", C.c_int32), ("sky_qw", C.c_int32), ("sky_off", C.c_int64)]


class CelPatch(C.Structure):
    _fields_ = [("src", C.c_int32), ("img", C.c_int32), ("x0", C.c_int32), ("y0", C.c_int32),
                ("w", C.c_int32), ("h", C.c_int32), ("pix_off", C.c_int64)]


class CelPrior(C.Structure):
    _fields_ = [("star_prob", C.c_double), ("r", (C.c_double * 2) * 2),
                ("c_w", (C.c_double * N_COLOUR_COMPONENTS) * 2),
                ("c_mean", ((C.c_double * 4) * N_COLOUR_COMPONENTS) * 2),
                ("c_cov", (((C.c_double * 4) * 4) * N_COLOUR_COMPONENTS) * 2),
                ("radius", C.c_double * 2), ("profile", C.c_double * 2), ("axis", C.c_double * 2)]


class CelProfiles(C.Structure):
    _fields_ = [("n_exp", C.c_int32), ("n_dev", C.c_int32),
                ("exp_alpha", C.c_double * MAX_PROFILE), ("exp_tau", C.c_double * MAX_PROFILE),
                ("dev_alpha", C.c_double * MAX_PROFILE), ("dev_tau", C.c_double * MAX_PROFILE)]


class CelProblem(C.Structure):
    _fields_ = [("n_sources", C.c_int32), ("n_images", C.c_int32), ("n_patches", C.c_int32),
                ("images", C.POINTER(CelImage)), ("sky_knots", C.POINTER(C.c_double)),
                ("n_sky_knots", C.c_int64), ("patches", C.POINTER(CelPatch)), ("pixels", C.c_void_p),
                ("n_pixels", C.c_int64), ("prior", C.POINTER(CelPrior)), ("profiles", C.POINTER(CelProfiles)),
                ("patch_psf", C.POINTER(C.c_double))]


class CelPsfModel(C.Structure):
    _fields_ = [("n_images", C.c_int32), ("n_eigen", C.c_int32), ("side", C.c_int32), ("eigen", C.c_void_p),
                ("coef", C.c_void_p), ("size", C.c_void_p)]


class CelOptions(C.Structure):
    _fields_ = [("pixels_per_lane", C.c_int32), ("chunk_pixels", C.c_int32), ("pixel_fp64", C.c_int32),
                ("hessian_fp64", C.c_int32), ("hessian_fd", C.c_int32), ("fd_step", C.c_double), ("radius0", C.c_double),
                ("radius_max", C.c_double), ("eta", C.c_double), ("gtol", C.c_double), ("ftol", C.c_double),
                ("radius_min", C.c_double), ("timing", C.c_int32), ("map_pixels_per_lane", C.c_int32)]


class CelMcmcOpts(C.Structure):
    _fields_ = [("n_temps", C.c_int32), ("n_runs", C.c_int32), ("n_post", C.c_int32), ("max_step_out", C.c_int32),
                ("max_shrink", C.c_int32), ("gamma", C.POINTER(C.c_double)), ("width", C.c_double * N_Z),
                ("box", C.c_double), ("seed", C.c_uint64)]


class CelMcmcReport(C.Structure):
    _fields_ = [("rounds", C.c_int64), ("n_chains", C.c_int64), ("evaluations", C.c_int64),
                ("candidate_pixels", C.c_int64)]


class CelTuneSpace(C.Structure):
    _fields_ = [("n_chunk", C.c_int32), ("chunk_pixels", C.c_int32 * 8), ("n_pixels_per_lane", C.c_int32),
                ("pixels_per_lane", C.c_int32 * 4), ("n_map", C.c_int32), ("map_pixels_per_lane", C.c_int32 * 6)]


class CelTuning(C.Structure):
    _fields_ = [("chunk_pixels", C.c_int32), ("pixels_per_lane", C.c_int32), ("map_pixels_per_lane", C.c_int32),
                ("n_timed", C.c_int32), ("ms_per_eval", C.c_double)]


class CelSweepOpts(C.Structure):
    _fields_ = [("n_sweeps", C.c_int32), ("max_newton_iters", C.c_int32), ("use_graph", C.c_int32),
                ("start_colour", C.c_int32), ("max_classes", C.c_int32)]


class CelSweepReport(C.Structure):
    _fields_ = [("elbo_total", C.c_double), ("n_colours", C.c_int32), ("n_newton_steps", C.c_int64),
                ("seconds", C.c_double), ("sweeps_done", C.c_int32), ("next_colour", C.c_int32)]


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1803_00113_amd.build` "
                      "(there is no fallback implementation)")
lib = C.CDLL(LIB_PATH)

_vp = C.c_void_p
_sig = {
    "cel_strerror": (C.c_char_p, [C.c_int32]),
    "cel_create": (C.c_int32, [C.POINTER(_vp), C.c_int32, C.POINTER(CelOptions)]),
    "cel_destroy": (None, [_vp]),
    "cel_prepare": (C.c_int32, [_vp, C.POINTER(CelProblem), C.POINTER(_vp), _vp]),
    "cel_plan_free": (None, [_vp]),
    "cel_plan_append": (C.c_int32, [_vp, _vp, C.POINTER(CelProblem), _vp]),
    "cel_plan_info": (C.c_int32, [_vp, C.POINTER(C.c_int64), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                  C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "cel_elbo_eval": (C.c_int32, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "cel_elbo_grad": (C.c_int32, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "cel_elbo_grad_plain": (C.c_int32, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "cel_elbo_grad_static": (C.c_int32, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "cel_elbo_hessian": (C.c_int32, [_vp, _vp, _vp, C.POINTER(C.c_uint8), _vp, _vp, _vp, _vp]),
    "cel_newton_step": (C.c_int32, [_vp, _vp, _vp, _vp, C.POINTER(C.c_uint8), _vp, _vp, _vp]),
    "cel_phase_times": (C.c_int32, [_vp, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.c_int32]),
    "cel_tune": (C.c_int32, [_vp, _vp, _vp, C.POINTER(CelTuneSpace), C.POINTER(CelTuning), _vp]),
    "cel_loglik": (C.c_int32, [_vp, _vp, _vp, C.c_int32, _vp, C.POINTER(C.c_uint8), _vp, _vp]),
    "cel_log_prior": (C.c_int32, [_vp, _vp, C.c_int64, _vp, _vp, _vp]),
    "cel_sweep": (C.c_int32, [_vp, _vp, _vp, _vp, _vp, C.POINTER(CelSweepOpts), C.POINTER(CelSweepReport), _vp]),
    "cel_last_device_error": (C.c_int32, [_vp, C.POINTER(C.c_int32)]),
    "cel_mcmc_step": (C.c_int32, [_vp, _vp, _vp, C.POINTER(C.c_uint8), _vp, C.POINTER(CelMcmcOpts), C.c_uint64, _vp,
                                  _vp, _vp, _vp, _vp, C.POINTER(CelMcmcReport), _vp]),
    "cel_psf_fit": (C.c_int32, [_vp, C.POINTER(CelPsfModel), C.c_int32, _vp, _vp, C.c_int32, C.c_int32, _vp, _vp]),
}
EXPORTED = tuple(_sig)
for _name, (_res, _args) in _sig.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args


class CelError(RuntimeError):
    def __init__(self, fn, status):
        super().__init__(f"{fn} failed: {lib.cel_strerror(status).decode()} ({status})")
        self.status = status


def check(fn, status):
    if status < 0:
        raise CelError(fn, status)
    return status
