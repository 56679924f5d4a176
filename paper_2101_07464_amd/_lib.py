"""ctypes binding of libhd.so (argument marshalling only).

The functions mirror include/hd.h one for one.  Every computation happens in
the HIP kernels behind the C ABI; this module never falls back to anything
else and raises when the library is missing.
"""
import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libhd.so")

HD_OK = 0
HD_ERR_INVALID = -1
HD_ERR_CAPACITY = -2
HD_ERR_NOMEM = -3
HD_ERR_HIP = -4
HD_ERR_NONFINITE = -5
HD_ERR_UNSUPPORTED = -6
HD_ERR_TOO_LARGE = -7
HD_NOALLOC_SCRATCH_BYTES = 64 << 20
HD_ISTA_GRAD = 1

HD_GINIBRE = 0
HD_HAAR = 1
HD_F32 = 0
HD_F64 = 1

HD_DYN_TANH = 1
HD_DYN_SOFT_HIST = 2
HD_DYN_NORMALIZE = 3
HD_PATTERN_Q = 0
HD_PATTERN_ALT = 1

EXPORTS = ["hd_init", "hd_free", "hd_step", "hd_apply_T", "hd_status",
           "hd_counts", "hd_reset", "hd_set_stream", "hd_pivots", "hd_run",
           "hd_profile", "hd_profile_read", "hd_strerror",
           "hd_batch_init", "hd_batch_run", "hd_batch_status",
           "hd_batch_set_stream", "hd_batch_free", "hd_lista_forward",
           "hd_lista_backward", "hd_autotune", "hd_shape_rule",
           "hd_autotune_clear", "hd_export", "hd_import", "hd_goe_step",
           "hd_usv_step", "hd_batch_set_graph", "hd_run_noalloc",
           "hd_batch_set_shape", "hd_batch_shape", "hd_batch_autotune",
           "hd_noalloc_scratch_bytes", "hd_spectral_power", "hd_ista_init",
           "hd_ista_run", "hd_ista_grad", "hd_ista_status",
           "hd_ista_set_stream", "hd_ista_free", "hd_cinit", "hd_cstep", "hd_crun",
           "hd_cgue_step", "hd_creset", "hd_ccounts", "hd_cstatus",
           "hd_cset_stream", "hd_cfree", "hd_cprofile", "hd_cprofile_read"]


class HDConfig(ctypes.Structure):
    _fields_ = [("ensemble", ctypes.c_int32), ("storage", ctypes.c_int32),
                ("m", ctypes.c_int64), ("n", ctypes.c_int64),
                ("t_max", ctypes.c_int32), ("seed", ctypes.c_uint32),
                ("trial", ctypes.c_uint32), ("sigma", ctypes.c_double),
                ("stream", ctypes.c_void_p)]


class HDDynamics(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("pattern", ctypes.c_int32),
                ("a", ctypes.c_double), ("b", ctypes.c_double)]


class HDBatchTrial(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("T", ctypes.c_int32),
                ("seed", ctypes.c_uint32), ("trial", ctypes.c_uint32)]


class HDError(RuntimeError):
    def __init__(self, code, what):
        self.code = code
        super().__init__("%s: %s (%d)" % (what, strerror(code), code))


class HDCapacityError(HDError):
    pass


_LIB = None


def load():
    """Load libhd.so; raises if it has not been built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libhd.so is not built (run __graft_entry__.build())")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                         ctypes.c_double)
    P = ctypes.POINTER
    sig = {
        "hd_init": (i32, [P(HDConfig), P(vp)]),
        "hd_free": (i32, [vp]),
        "hd_step": (i32, [vp, vp, vp]),
        "hd_apply_T": (i32, [vp, vp, vp]),
        "hd_status": (i32, [vp]),
        "hd_counts": (i32, [vp, P(i32), P(i32), P(i32)]),
        "hd_reset": (i32, [vp, ctypes.c_uint32, ctypes.c_uint32]),
        "hd_set_stream": (i32, [vp, vp]),
        "hd_pivots": (i32, [vp, i32, i32, vp, vp, vp]),
        "hd_run": (i32, [vp, P(HDDynamics), i32, vp, vp, vp, vp, vp]),
        "hd_profile": (i32, [vp, i32]),
        "hd_profile_read": (i32, [vp, i32, P(dbl), P(i64), P(dbl)]),
        "hd_strerror": (ctypes.c_char_p, [i32]),
        "hd_batch_init": (i32, [i32, P(HDBatchTrial), i32, vp, P(vp)]),
        "hd_batch_run": (i32, [vp, P(HDDynamics), P(vp), P(vp), P(vp),
                               P(vp)]),
        "hd_batch_status": (i32, [vp]),
        "hd_batch_set_stream": (i32, [vp, vp]),
        "hd_batch_free": (i32, [vp]),
        "hd_lista_forward": (i32, [vp, i32, P(ctypes.c_float),
                                   P(ctypes.c_float), vp, vp, vp, vp]),
        "hd_lista_backward": (i32, [vp, i32, P(ctypes.c_float),
                                    P(ctypes.c_float), vp, vp, vp, vp, vp,
                                    vp]),
        "hd_autotune": (i32, [i32, i32, P(i64), i32, i32, vp, P(dbl)]),
        "hd_shape_rule": (i32, [i32, i32, i64, P(i32)]),
        "hd_autotune_clear": (i32, []),
        "hd_export": (i32, [vp, vp, P(ctypes.c_size_t)]),
        "hd_goe_step": (i32, [vp, vp, vp]),
        "hd_usv_step": (i32, [vp, vp, vp, i32, vp, vp]),
        "hd_batch_set_graph": (i32, [vp, i32]),
        "hd_batch_set_shape": (i32, [vp, i32]),
        "hd_batch_shape": (i32, [vp]),
        "hd_batch_autotune": (i32, [vp, P(HDDynamics), P(vp), i32,
                                    P(ctypes.c_double), P(i32)]),
        "hd_import": (i32, [P(HDConfig), vp, ctypes.c_size_t, P(vp)]),
        "hd_run_noalloc": (i32, [P(HDConfig), P(HDDynamics), i32, vp, vp,
                                 vp, vp, vp]),
        "hd_noalloc_scratch_bytes": (i32, [P(HDConfig),
                                           P(ctypes.c_size_t)]),
        "hd_spectral_power": (i32, [vp, i64, vp, vp, i32, dbl, vp, vp]),
        "hd_ista_init": (i32, [i32, i64, i64, i32, i32, ctypes.c_uint32,
                               ctypes.c_uint32, dbl, i32, vp, P(vp)]),
        "hd_ista_grad": (i32, [vp, P(ctypes.c_float), P(ctypes.c_float), vp,
                               vp, vp]),
        "hd_ista_run": (i32, [vp, P(ctypes.c_float), P(ctypes.c_float), vp,
                              vp, vp]),
        "hd_ista_status": (i32, [vp]),
        "hd_ista_set_stream": (i32, [vp, vp]),
        "hd_ista_free": (i32, [vp]),
        "hd_cinit": (i32, [i32, i32, i64, i64, i32, ctypes.c_uint32,
                           ctypes.c_uint32, ctypes.c_double, vp,
                           P(vp)]),
        "hd_cstep": (i32, [vp, i32, vp, vp]),
        "hd_crun": (i32, [vp, i32, ctypes.c_double, ctypes.c_double, vp, vp]),
        "hd_cgue_step": (i32, [vp, vp, vp]),
        "hd_creset": (i32, [vp, ctypes.c_uint32, ctypes.c_uint32]),
        "hd_ccounts": (i32, [vp, P(i32), P(i32), P(i32)]),
        "hd_cstatus": (i32, [vp]),
        "hd_cset_stream": (i32, [vp, vp]),
        "hd_cfree": (i32, [vp]),
        "hd_cprofile": (i32, [vp, i32]),
        "hd_cprofile_read": (i32, [vp, i32, P(dbl), P(i64), P(dbl)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _LIB = L
    return L


def strerror(code):
    return load().hd_strerror(code).decode()


def check(code, what):
    if code == HD_OK:
        return
    if code == HD_ERR_CAPACITY:
        raise HDCapacityError(code, what)
    raise HDError(code, what)
