"""ctypes binding of libhipfit.so (argument marshalling only).

Every computation happens in the library's HIP kernels and C++ runtime; this
module only converts Python/numpy arguments.  It raises at import of the
first call if the library has not been built -- there is no fallback path.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhipfit.so")

HF_OK = 0
HF_E_INVALID = -1
HF_E_GRAPH = -2
HF_E_SHAPE = -3
HF_E_OOM = -4
HF_E_HIP = -5
HF_E_DOMAIN = -6
HF_E_NOT_CONVERGED = -7
HF_E_BUDGET = -8
HF_E_FULL = -9

HF_FP64 = 0
HF_FP32_EVAL = 1
HF_METRIC_BNLL = 1
HF_METRIC_CHI2 = 2

OP = {"exp": 1, "gauss": 2, "poly": 3, "add": 4, "prod": 5, "dalitz": 6, "tddp": 7, "map": 8, "dpmap": 9, "conv": 10, "comp": 11}

STATUS_NAMES = {0: "OK", -1: "E_INVALID", -2: "E_GRAPH", -3: "E_SHAPE", -4: "E_OOM", -5: "E_HIP",
                -6: "E_DOMAIN", -7: "E_NOT_CONVERGED", -8: "E_BUDGET", -9: "E_FULL"}


class HipfitError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (STATUS_NAMES.get(code, "?"), code, msg))
        self.code = code


class hf_obs(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char_p), ("lo", ctypes.c_double), ("hi", ctypes.c_double)]


class hf_param(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char_p), ("init", ctypes.c_double), ("step", ctypes.c_double),
                ("lo", ctypes.c_double), ("hi", ctypes.c_double), ("fixed", ctypes.c_int32)]


_I32P = ctypes.POINTER(ctypes.c_int32)
_DP = ctypes.POINTER(ctypes.c_double)


class hf_node(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int32),
                ("n_child", ctypes.c_int32), ("child", _I32P),
                ("n_par", ctypes.c_int32), ("par", _I32P),
                ("n_obs", ctypes.c_int32), ("obs", _I32P),
                ("n_const", ctypes.c_int32), ("consts", _DP)]


class hf_fit_opts(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int32), ("edm_tol", ctypes.c_double), ("grad_mode", ctypes.c_int32),
                ("want_errors", ctypes.c_int32), ("param_eps", ctypes.c_double)]


class hf_fit_summary(ctypes.Structure):
    _fields_ = [("nll", ctypes.c_double), ("edm", ctypes.c_double), ("n_iter", ctypes.c_int32),
                ("n_eval", ctypes.c_int32), ("status", ctypes.c_int32)]


# name -> (restype, argtypes); the exported C ABI of include/hipfit.h
_VP = ctypes.c_void_p
FG_FN = ctypes.CFUNCTYPE(ctypes.c_int, _DP, _DP, _DP, _VP)
SIGNATURES = {
    "pdf_graph_create": (ctypes.c_int, [ctypes.POINTER(hf_obs), ctypes.c_int32, ctypes.POINTER(hf_param),
                                        ctypes.c_int32, ctypes.POINTER(hf_node), ctypes.c_int32, ctypes.c_int32,
                                        ctypes.POINTER(_VP)]),
    "pdf_graph_destroy": (None, [_VP]),
    "pdf_graph_shape": (ctypes.c_int, [_VP, _I32P, _I32P]),
    "dataset_upload": (ctypes.c_int, [_VP, ctypes.POINTER(_DP), ctypes.c_int64, ctypes.c_int, _VP,
                                      ctypes.POINTER(_VP)]),
    "dataset_wrap_device": (ctypes.c_int, [_VP, ctypes.POINTER(_VP), ctypes.c_int64, ctypes.c_int,
                                           ctypes.POINTER(_VP)]),
    "hf_column_ref": (ctypes.c_int, [_VP, ctypes.c_int32, ctypes.c_int, _DP]),
    "dataset_upload_binned": (ctypes.c_int, [_VP, ctypes.POINTER(_DP), _DP, ctypes.c_int64, ctypes.c_double,
                                             ctypes.c_int32, ctypes.c_int, _VP, ctypes.POINTER(_VP)]),
    "dataset_generate": (ctypes.c_int, [_VP, _DP, ctypes.c_int64, ctypes.c_uint64, ctypes.c_int, _VP,
                                        ctypes.POINTER(_VP)]),
    "dataset_read_column": (ctypes.c_int, [_VP, ctypes.c_int32, _VP, _DP]),
    "dataset_generate_ar": (ctypes.c_int, [_VP, _DP, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double,
                                           ctypes.c_int32, ctypes.c_int, _VP, ctypes.POINTER(_VP)]),
    "dataset_free": (None, [_VP]),
    "dataset_device_bytes": (ctypes.c_int64, [_VP]),
    "dataset_bytes_needed": (ctypes.c_int, [_VP, ctypes.c_int64, ctypes.c_int, ctypes.POINTER(ctypes.c_int64)]),
    # theta and grad are passed as raw addresses (numpy .ctypes.data)
    "nll_eval": (ctypes.c_int, [_VP, _VP, _VP, _VP, _DP]),
    "nll_grad": (ctypes.c_int, [_VP, _VP, _VP, _VP, _DP, _VP]),
    "nll_terms": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, _VP]),
    "nll_grad_noalloc": (ctypes.c_int, [_VP, _VP, ctypes.c_int64, ctypes.c_int, _VP, _VP, _DP, _VP]),
    "nll_grad_batched": (ctypes.c_int, [_VP, ctypes.POINTER(_VP), ctypes.c_int32, _DP, _VP, _DP, _DP]),
    "fit": (ctypes.c_int, [_VP, _VP, ctypes.POINTER(hf_fit_opts), _VP, _DP, _DP, _DP,
                           ctypes.POINTER(hf_fit_summary)]),
    "hf_minimize": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(hf_param), _DP, ctypes.POINTER(hf_fit_opts),
                                   ctypes.c_double, FG_FN, _VP, _DP, _DP, _DP, ctypes.POINTER(hf_fit_summary)]),
    "batch_create": (ctypes.c_int, [_VP, ctypes.c_int32, ctypes.c_int64, _VP, ctypes.POINTER(_VP)]),
    "batch_destroy": (None, [_VP]),
    "batch_admit": (ctypes.c_int, [_VP, _VP, _DP, ctypes.POINTER(hf_fit_opts), ctypes.c_int64, _I32P]),
    "batch_step": (ctypes.c_int, [_VP, _I32P, _I32P]),
    "batch_poll": (ctypes.c_int, [_VP, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64), _I32P, _DP, _DP, _DP,
                                  _I32P]),
    "batch_cancel": (ctypes.c_int, [_VP, ctypes.c_int64]),
    "hf_dalitz_inside": (ctypes.c_int, [_VP, ctypes.c_int32, ctypes.c_int64, _DP, _DP,
                                        ctypes.POINTER(ctypes.c_uint8)]),
    "hf_profile": (ctypes.c_int, [ctypes.c_int32, _DP, _DP, ctypes.POINTER(ctypes.c_int64)]),
    "hf_last_error": (ctypes.c_char_p, []),
    "last_error_message": (ctypes.c_char_p, []),
    "hf_version": (ctypes.c_char_p, []),
}

_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libhipfit.so is not built (run paper_1311_1753_amd.build.build()); "
                              "there is no CPU fallback")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(rc, allow=()):
    if rc < 0 and rc not in allow:
        msg = lib().hf_last_error()
        raise HipfitError(rc, msg.decode() if msg else "")
    return rc
