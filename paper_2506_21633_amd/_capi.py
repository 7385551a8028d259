"""ctypes mirror of include/sdgr.h and include/sdgr_train.h (argument
marshalling only).

Loading fails loudly when libsdgr.so has not been built: there is no
fallback implementation anywhere in the package.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsdgr.so")

SDGR_OK = 0
SDGR_EINVAL = -1
SDGR_EWORKSPACE = -2
SDGR_EHIP = -3
SDGR_EOVERFLOW = -4
SDGR_EUNSUPPORTED = -5

EXPORTED = ("sdgr_version", "sdgr_last_error", "sdgr_default_options",
            "sdgr_query_bytes", "sdgr_plan_query", "sdgr_forward",
            "sdgr_backward", "sdgr_status", "sdgr_read_intensity",
            "sdgr_read_optical_depth", "sdgr_profile_enable", "sdgr_profile_read",
            "sdgr_profile_stage", "sdgr_profile_count", "sdgr_read_work",
            "sdgr_plan_resize", "sdgr_forward_static", "sdgr_plan_host", "sdgr_status_accumulate",
            # reconstruction loop and metrics
            "sdgr_adam_step", "sdgr_densify_stats", "sdgr_densify_workspace_bytes",
            "sdgr_densify", "sdgr_nearest_sq", "sdgr_image_metrics")

STATIC_SCRATCH_BYTES = 64 << 20   # SDGR_STATIC_SCRATCH_BYTES


class Scene(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64),
                ("means", ctypes.c_void_p), ("scales", ctypes.c_void_p),
                ("quats", ctypes.c_void_p), ("amp", ctypes.c_void_p),
                ("ext", ctypes.c_void_p), ("ext_back", ctypes.c_void_p),
                ("sh", ctypes.c_void_p), ("sh_degree", ctypes.c_int32),
                ("sh_stride", ctypes.c_int32)]


class SceneGrad(ctypes.Structure):
    _fields_ = [("d_means", ctypes.c_void_p), ("d_scales", ctypes.c_void_p),
                ("d_quats", ctypes.c_void_p), ("d_amp", ctypes.c_void_p),
                ("d_ext", ctypes.c_void_p), ("d_ext_back", ctypes.c_void_p),
                ("d_sh", ctypes.c_void_p)]


class View(ctypes.Structure):
    _fields_ = [("azimuth", ctypes.c_double), ("grazing", ctypes.c_double),
                ("d_az", ctypes.c_double), ("d_rg", ctypes.c_double),
                ("comp_d_az", ctypes.c_double), ("comp_d_el", ctypes.c_double),
                ("img_offset", ctypes.c_int64),
                ("img_w", ctypes.c_int32), ("img_h", ctypes.c_int32),
                ("comp_w", ctypes.c_int32), ("comp_h", ctypes.c_int32),
                ("scene", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("radar_range", ctypes.c_double)]


class Options(ctypes.Structure):
    _fields_ = [("shadowing", ctypes.c_int32), ("recompute", ctypes.c_int32),
                ("q_max", ctypes.c_float), ("tau_max", ctypes.c_float),
                ("dilation", ctypes.c_float), ("deterministic", ctypes.c_int32),
                ("tile", ctypes.c_int32), ("cell_area", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class Plan(ctypes.Structure):
    _fields_ = [("state_bytes", ctypes.c_size_t),
                ("fwd_scratch_bytes", ctypes.c_size_t),
                ("bwd_scratch_bytes", ctypes.c_size_t),
                ("image_floats", ctypes.c_size_t),
                ("records", ctypes.c_int64), ("pairs_c", ctypes.c_int64),
                ("pairs_i", ctypes.c_int64), ("tiles_c", ctypes.c_int64),
                ("tiles_i", ctypes.c_int64), ("rays", ctypes.c_int64),
                ("gaussians", ctypes.c_int64), ("nviews", ctypes.c_int32), ("nscenes", ctypes.c_int32),
                ("tile", ctypes.c_int32), ("recompute", ctypes.c_int32),
                ("deterministic", ctypes.c_int32), ("sh_coeffs", ctypes.c_int32),
                ("hit_bytes", ctypes.c_int64)]


ADAM_MAX_GROUPS = 16   # SDGR_ADAM_MAX_GROUPS


class ParamGroup(ctypes.Structure):
    _fields_ = [("param", ctypes.c_void_p), ("grad", ctypes.c_void_p),
                ("m", ctypes.c_void_p), ("v", ctypes.c_void_p),
                ("count", ctypes.c_int64), ("lr", ctypes.c_float),
                ("log_space", ctypes.c_int32), ("lo", ctypes.c_float), ("hi", ctypes.c_float),
                ("reserved", ctypes.c_int32)]


class AdamConfig(ctypes.Structure):
    _fields_ = [("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float), ("reserved", ctypes.c_int32)]


class DensifyConfig(ctypes.Structure):
    _fields_ = [("grad_threshold", ctypes.c_float), ("split_scale", ctypes.c_float),
                ("max_radius", ctypes.c_float), ("kappa_min", ctypes.c_float),
                ("split_factor", ctypes.c_float), ("reserved", ctypes.c_int32)]


SET_GROUPS = ("means", "scales", "quats", "amp", "ext", "sh")


class GaussianSet(ctypes.Structure):
    _fields_ = [f for g in SET_GROUPS
                for f in ((g, ctypes.c_void_p), ("m_" + g, ctypes.c_void_p),
                          ("v_" + g, ctypes.c_void_p))] + \
               [("sh_coeffs", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class SDGRError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"sdgr error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load libsdgr.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} not found: build the HIP library first "
            "(python -m paper_2506_21633_amd.build)")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp = ctypes.c_void_p
    L.sdgr_version.restype = ctypes.c_int
    L.sdgr_last_error.restype = ctypes.c_char_p
    L.sdgr_default_options.argtypes = [P(Options)]
    L.sdgr_query_bytes.restype = ctypes.c_size_t
    L.sdgr_query_bytes.argtypes = [ctypes.c_int32, ctypes.c_int32]
    L.sdgr_plan_query.argtypes = [P(Scene), ctypes.c_int32, P(View), ctypes.c_int32,
                                  P(Options), vp, ctypes.c_size_t, vp, P(Plan)]
    L.sdgr_forward.argtypes = [P(Scene), ctypes.c_int32, P(View), ctypes.c_int32,
                               P(Options), P(Plan), vp, vp, vp, vp]
    L.sdgr_backward.argtypes = [P(Scene), ctypes.c_int32, P(View), ctypes.c_int32,
                                P(Options), P(Plan), vp, vp, vp, P(SceneGrad), vp]
    L.sdgr_forward_static.argtypes = [P(Scene), ctypes.c_int32, P(View), ctypes.c_int32,
                                      P(Options), vp, vp]
    L.sdgr_status.argtypes = [P(Plan), vp, vp]
    L.sdgr_status_accumulate.argtypes = [P(Plan), vp, vp, vp]
    L.sdgr_status_accumulate.restype = ctypes.c_int
    L.sdgr_read_intensity.argtypes = [P(Plan), vp, vp, vp]
    L.sdgr_read_optical_depth.argtypes = [P(Plan), vp, vp, vp]
    L.sdgr_profile_enable.argtypes = [ctypes.c_int32]
    L.sdgr_profile_read.argtypes = [P(ctypes.c_double), P(ctypes.c_int64), ctypes.c_int32]
    L.sdgr_profile_stage.argtypes = [ctypes.c_int32]
    L.sdgr_profile_stage.restype = ctypes.c_char_p
    L.sdgr_profile_count.argtypes = [ctypes.c_int32]
    L.sdgr_plan_resize.argtypes = [P(Plan), ctypes.c_int64, ctypes.c_int64]
    L.sdgr_plan_host.argtypes = [P(Scene), ctypes.c_int32, P(View), ctypes.c_int32, P(Options),
                                 ctypes.c_int64, ctypes.c_int64, P(Plan)]
    L.sdgr_plan_host.restype = ctypes.c_int
    L.sdgr_read_work.argtypes = [P(Plan), vp, P(ctypes.c_uint64), ctypes.c_int32, vp]
    L.sdgr_adam_step.argtypes = [P(ParamGroup), ctypes.c_int32, ctypes.c_int64, P(AdamConfig),
                                 vp]
    L.sdgr_densify_stats.argtypes = [vp, ctypes.c_int64, vp, vp, vp, vp]
    L.sdgr_densify_workspace_bytes.argtypes = [ctypes.c_int64]
    L.sdgr_densify_workspace_bytes.restype = ctypes.c_size_t
    L.sdgr_densify.argtypes = [P(GaussianSet), ctypes.c_int64, vp, vp, vp, P(DensifyConfig),
                               P(GaussianSet), ctypes.c_int64, vp, vp, ctypes.c_size_t, vp]
    L.sdgr_nearest_sq.argtypes = [vp, ctypes.c_int64, vp, ctypes.c_int64, vp, vp]
    L.sdgr_image_metrics.argtypes = [vp, vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_float, vp, vp, vp, vp]
    for name in ("sdgr_adam_step", "sdgr_densify_stats", "sdgr_densify", "sdgr_nearest_sq",
                 "sdgr_image_metrics"):
        getattr(L, name).restype = ctypes.c_int
    for name in ("sdgr_plan_resize", "sdgr_profile_count", "sdgr_read_work",
                 "sdgr_profile_enable", "sdgr_profile_read", "sdgr_plan_query", "sdgr_forward", "sdgr_backward", "sdgr_status",
                 "sdgr_read_intensity", "sdgr_read_optical_depth", "sdgr_forward_static"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def check(code):
    if code != SDGR_OK:
        raise SDGRError(code, lib().sdgr_last_error().decode(errors="replace"))


def profile_read():
    """{stage name: (total ms, timed calls)} since the last read."""
    L = lib()
    n = 32
    ms = (ctypes.c_double * n)()
    calls = (ctypes.c_int64 * n)()
    k = L.sdgr_profile_read(ms, calls, n)
    if k < 0:
        check(k)
    return {L.sdgr_profile_stage(i).decode(): (ms[i], calls[i]) for i in range(k)}
