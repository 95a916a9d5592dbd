"""ctypes declarations of the C ABI in include/scw.h.

Loading fails loudly (ImportError) when libscw.so has not been built: there is
no fallback implementation.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libscw.so")

SCW_OK = 0
STATUS = {0: "SCW_OK", -1: "SCW_EINVAL", -2: "SCW_ENOMEM", -3: "SCW_EHIP",
          -4: "SCW_ELAPACK", -5: "SCW_EGRAZING", -6: "SCW_EDEFECTIVE",
          -7: "SCW_EILLCOND"}
PRECISION = {"fp64": 0, "fp32": 1, "bf16x3": 2, "fp16x3": 3}
ROUTE = {"stable": 0, "connection": 1, "stable_device": 2, "connection_device": 3}
EIG = {"host": 0, "device": 1}
STAGE = {"modal": 1, "exterior": 2, "transform": 4, "all": 7}
EIG_MAX_N = 2048

c_dp = ctypes.POINTER(ctypes.c_double)


class ScwProblem(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("px", ctypes.c_double), ("py", ctypes.c_double), ("pz", ctypes.c_double),
        ("n", c_dp),
        ("lam", ctypes.c_double),
        ("n_top", ctypes.c_double),
        ("n_bot_re", ctypes.c_double), ("n_bot_im", ctypes.c_double),
        ("U", ctypes.c_int), ("V", ctypes.c_int),
        ("inc_ex", c_dp), ("inc_ey", c_dp),
        ("inc_nx", ctypes.c_int), ("inc_ny", ctypes.c_int),
        ("pw_u", ctypes.c_int), ("pw_v", ctypes.c_int),
        ("pw_ex", ctypes.c_double * 2), ("pw_ey", ctypes.c_double * 2),
        ("route", ctypes.c_int),
        ("eig", ctypes.c_int),
    ]


class ScwGrid(ctypes.Structure):
    _fields_ = [("fx", ctypes.c_int), ("fy", ctypes.c_int), ("fz", ctypes.c_int),
                ("z_begin", ctypes.c_double), ("z_end", ctypes.c_double)]


class ScwSlice(ctypes.Structure):
    _fields_ = [("axis", ctypes.c_int), ("position", ctypes.c_double), ("n", ctypes.c_int),
                ("fz", ctypes.c_int), ("z_begin", ctypes.c_double), ("z_end", ctypes.c_double)]


SLICE_AXIS = {"xz": 0, "yz": 1}


class ScwPlaneWave(ctypes.Structure):
    _fields_ = [("u", ctypes.c_int), ("v", ctypes.c_int), ("ex", ctypes.c_double * 2),
                ("ey", ctypes.c_double * 2)]


class ScwSolutionInfo(ctypes.Structure):
    _fields_ = [
        ("M", ctypes.c_int), ("L", ctypes.c_int),
        ("min_abs_sz", ctypes.c_double),
        ("min_abs_gamma_rel", ctypes.c_double),
        ("growth_exponent", ctypes.c_double),
        ("connection_rcond", ctypes.c_double),
        ("setup_seconds", ctypes.c_double),
        ("eig_seconds", ctypes.c_double),
        ("assembly_device_ms", ctypes.c_double),
        ("boundary_seconds", ctypes.c_double),
    ]


TRANSFORM = {"auto": 0, "fft": 1, "mfma": 2, "direct": 3}
TRANSFORM_NAME = {v: k for k, v in TRANSFORM.items()}


class ScwSynthConfig(ctypes.Structure):
    _fields_ = [("modal_rows", ctypes.c_int), ("transform", ctypes.c_int),
                ("fft_radix", ctypes.c_int), ("tiles", ctypes.c_int)]


class ScwTuneReport(ctypes.Structure):
    _fields_ = [("n_candidates", ctypes.c_int),
                ("default_ms", ctypes.c_double),
                ("best_ms", ctypes.c_double),
                ("config", ScwSynthConfig),
                ("batch_radix", ctypes.c_int),
                ("batch_blocks_per_cu", ctypes.c_int),
                ("batch_chunk", ctypes.c_int)]


# name -> (restype, argtypes); every entry point of include/scw.h
SIGNATURES = {
    "scw_last_error": (ctypes.c_char_p, []),
    "scw_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.c_int]),
    "scw_destroy": (None, [ctypes.c_void_p]),
    "scw_solve": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ScwProblem),
                                 ctypes.POINTER(ctypes.c_void_p)]),
    "scw_solve_illuminations": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ScwProblem),
                                               ctypes.c_int, ctypes.POINTER(ScwPlaneWave),
                                               ctypes.POINTER(ctypes.c_void_p)]),
    "scw_synthesize_illuminations": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p,
                                                    ctypes.POINTER(ScwGrid), ctypes.c_int,
                                                    ctypes.c_void_p, ctypes.c_void_p]),
    "scw_solution_free": (None, [ctypes.c_void_p]),
    "scw_solution_info_get": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ScwSolutionInfo)]),
    "scw_solution_exterior": (ctypes.c_int, [ctypes.c_void_p, c_dp, c_dp, c_dp]),
    "scw_synthesize_filtered": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p,
                                               ctypes.POINTER(ScwGrid), ctypes.c_int,
                                               ctypes.c_void_p, ctypes.c_void_p,
                                               ctypes.c_void_p, ctypes.c_void_p]),
    "scw_synthesize_image": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.POINTER(ScwGrid), ctypes.c_int,
                                            ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.c_void_p]),
    "scw_synthesize_slice": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.POINTER(ScwSlice), ctypes.c_int,
                                            ctypes.c_void_p, ctypes.c_void_p]),
    "scw_solve_batch": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ScwProblem),
                                       ctypes.c_int, ctypes.POINTER(ctypes.c_void_p)]),
    "scw_eig_batched": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p]),
    "scw_synthesize_tiled": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.POINTER(ScwGrid), ctypes.c_int, ctypes.c_int,
                                            ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]),
    "scw_synthesize_composed": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p),
                                               ctypes.c_int, ctypes.c_int,
                                               ctypes.POINTER(ScwGrid), ctypes.c_int,
                                               ctypes.c_void_p, ctypes.c_void_p]),
    "scw_synthesize": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ScwGrid),
                                      ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]),
    "scw_synthesize_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p,
                                              ctypes.POINTER(ScwGrid), ctypes.c_int,
                                              ctypes.c_void_p, ctypes.c_void_p]),
    "scw_synthesize_stages": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.POINTER(ScwGrid), ctypes.c_int, ctypes.c_int,
                                             ctypes.c_void_p, ctypes.c_void_p]),
    "scw_field": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ScwProblem),
                                 ctypes.POINTER(ScwGrid), ctypes.c_int, ctypes.c_void_p,
                                 ctypes.c_void_p]),
    "scw_synthesis_bytes": (ctypes.c_double, [ctypes.c_void_p, ctypes.POINTER(ScwGrid),
                                              ctypes.c_int]),
    "scw_profile_begin": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "scw_profile_end": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                       ctypes.c_int, ctypes.POINTER(ctypes.c_int)]),
    "scw_stage_name": (ctypes.c_char_p, [ctypes.c_int]),
    "scw_batch_plan": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p),
                                      ctypes.c_int, ctypes.POINTER(ScwGrid), ctypes.c_int,
                                      ctypes.POINTER(ctypes.c_void_p)]),
    "scw_batch_launch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "scw_batch_free": (None, [ctypes.c_void_p]),
    "scw_batch_tune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_int, ctypes.POINTER(ScwTuneReport)]),
    "scw_batch_configure": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                           ctypes.c_int]),
    "scw_synthesis_configure": (ctypes.c_int, [ctypes.c_void_p,
                                               ctypes.POINTER(ScwSynthConfig)]),
    "scw_tune_synthesis": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.POINTER(ScwGrid), ctypes.c_int,
                                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                          ctypes.POINTER(ScwTuneReport)]),
    "scw_sur_param_count": (ctypes.c_longlong, []),
    "scw_sur_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_ulonglong,
                                      ctypes.POINTER(ctypes.c_void_p)]),
    "scw_sur_free": (None, [ctypes.c_void_p]),
    "scw_sur_get_params": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "scw_sur_set_params": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "scw_sur_set_compute": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "scw_sur_encode": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                      ctypes.c_void_p, ctypes.c_void_p]),
    "scw_sur_forward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                       ctypes.c_void_p, ctypes.c_void_p]),
    "scw_sur_loss_grad": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                         ctypes.c_void_p, ctypes.c_void_p]),
    "scw_sur_train_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_int, ctypes.c_float,
                                          ctypes.POINTER(ctypes.c_double), ctypes.c_void_p]),
    "scw_sur_infer_checked": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, c_dp,
                                             ctypes.c_int, ctypes.c_int, ctypes.c_ulonglong,
                                             ctypes.c_double, c_dp,
                                             ctypes.POINTER(ctypes.c_int),
                                             ctypes.POINTER(ctypes.c_double)]),
}

_lib = None


def load(path=LIB_PATH):
    """Load libscw.so and declare its signatures (cached)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libscw.so is not built (%s); run python -m "
                          "paper_2404_07293_amd.build" % path)
    # PyTorch ships its own HIP runtime under the same soname as the system
    # one. Loading torch first makes the library bind to torch's runtime, so
    # that both share one runtime (device pointers and streams); loading the
    # library first would hand torch a runtime it was not built against.
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class ScwError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (STATUS.get(code, "?"), code, msg))
        self.code = code


def check(rc):
    if rc != SCW_OK:
        msg = _lib.scw_last_error()
        raise ScwError(rc, msg.decode() if msg else "")
    return rc
