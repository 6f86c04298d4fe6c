"""ctypes binding of the plprof C ABI (include/plprof.h).  Argument
marshalling only; every step runs in the HIP library."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libplprof.so")

PL_FP64, PL_MIXED = 0, 1
PL_F64, PL_F32 = 0, 1
PL_INFO_RANK, PL_INFO_BAD_Y, PL_INFO_FALLBACK = -1, -2, 1 << 30
PL_MAX_P, PL_MAX_M = 32, 64

# every symbol the header declares
EXPORTS = ("pl_version", "pl_error_string", "pl_workspace_size", "pl_matern_workspace_size",
           "pl_matern_cov", "pl_chol_workspace_size", "pl_chol_batched", "pl_profile_loglik",
           "pl_profiling_enable", "pl_profiling_read", "pl_curves_workspace_size",
           "pl_profile_curves", "pl_profile_param", "pl_autotune_workspace_size",
           "pl_autotune", "pl_to_internal", "pl_from_internal", "pl_mle_workspace_size",
           "pl_mle", "pl_hessian_workspace_size", "pl_hessian", "pl_config_points",
           "pl_sphere_points", "pl_lambda_grid", "pl_chisq_quantile", "pl_batch_create",
           "pl_batch_workspace_size", "pl_batch_stats", "pl_batch_run", "pl_batch_error",
           "pl_batch_destroy", "pl_profile_loglik_noalloc", "pl_batch_autotune_workspace_size",
           "pl_batch_autotune", "pl_tune_cache_set", "pl_tune_store", "pl_tune_lookup",
           "pl_tune_cache_stats")
PL_TUNE_MISS = 5
KERNEL_CLASSES = ("tables", "matern", "gemm", "potrf", "trsm", "other")


class PlResult(ctypes.Structure):
    _fields_ = [("loglik", ctypes.c_double), ("logdet_v", ctypes.c_double),
                ("logdet_xvx", ctypes.c_double), ("ssq_y", ctypes.c_double),
                ("ssq_betahat", ctypes.c_double), ("ssq_resid", ctypes.c_double),
                ("sigma2_hat", ctypes.c_double), ("jacobian", ctypes.c_double),
                ("loglik_reml", ctypes.c_double), ("info", ctypes.c_int32),
                ("pad", ctypes.c_int32)]


class PlOpts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("refine", ctypes.c_int32),
                ("chunk", ctypes.c_int64), ("flags", ctypes.c_int32),
                ("flush", ctypes.c_int32), ("wait_us", ctypes.c_int32),
                ("lanes", ctypes.c_int32)]


PL_OPT_NO_FALLBACK = 1
PL_OPT_BATCH_PERSISTENT = 2


class PlDataset(ctypes.Structure):
    _fields_ = [("locs", ctypes.c_void_p), ("y", ctypes.c_void_p), ("X", ctypes.c_void_p),
                ("n", ctypes.c_int64), ("omega", ctypes.c_void_p), ("K", ctypes.c_int64)]


class PlError(RuntimeError):
    pass


_lib = None

_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_SZ = ctypes.c_size_t


def load(path: str = None):
    """Load the shared library; raises if it has not been built."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise PlError(f"plprof HIP library not found at {p}; run __graft_entry__.build()")
    # PyTorch ships its own HIP runtime.  Importing it first makes the
    # library bind to that runtime, the one that owns torch's device memory
    # and streams; loaded the other way round, the library's kernel launches
    # fail in a process that then imports torch.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(p)
    lib.pl_version.restype = ctypes.c_char_p
    lib.pl_version.argtypes = []
    lib.pl_error_string.restype = ctypes.c_char_p
    lib.pl_error_string.argtypes = [ctypes.c_int]
    lib.pl_workspace_size.restype = ctypes.c_int
    lib.pl_workspace_size.argtypes = [_I64, _I64, _I64, _I64, ctypes.POINTER(PlOpts),
                                      ctypes.POINTER(_SZ)]
    lib.pl_matern_workspace_size.restype = ctypes.c_int
    lib.pl_matern_workspace_size.argtypes = [_I64, ctypes.POINTER(_SZ)]
    lib.pl_matern_cov.restype = ctypes.c_int
    lib.pl_matern_cov.argtypes = [_P, _I64, _P, _I64, ctypes.c_int, _P, _I64, _P, _SZ, _P]
    lib.pl_chol_workspace_size.restype = ctypes.c_int
    lib.pl_chol_workspace_size.argtypes = [_I64, ctypes.c_int, ctypes.POINTER(_SZ)]
    lib.pl_chol_batched.restype = ctypes.c_int
    lib.pl_chol_batched.argtypes = [_P, _I64, _I64, _I64, ctypes.c_int, _P, _P, _P, _SZ, _P]
    lib.pl_profile_loglik.restype = ctypes.c_int
    lib.pl_profile_loglik.argtypes = [_P, _P, _P, _I64, _I64, _P, _I64, _P, _I64, _P, _P, _P,
                                      ctypes.POINTER(PlOpts), _P, _SZ, _P]
    lib.pl_profile_loglik_noalloc.restype = ctypes.c_int
    lib.pl_profile_loglik_noalloc.argtypes = [_P, _P, _P, _I64, _I64, _P, _I64, _P, _I64, _P, _P,
                                              _P, ctypes.POINTER(PlOpts), _P]
    lib.pl_curves_workspace_size.restype = ctypes.c_int
    lib.pl_curves_workspace_size.argtypes = [_I64, _I64, _I64, _I64, ctypes.POINTER(_SZ)]
    lib.pl_profile_curves.restype = ctypes.c_int
    lib.pl_profile_curves.argtypes = [_P, _P, _P, _I64, _I64, _I64, _P, _I64, _P, _I64, _P, _I64,
                                      _P, _P, _P, _P, _P, _SZ, _P]
    lib.pl_profiling_enable.restype = ctypes.c_int
    lib.pl_profiling_enable.argtypes = [ctypes.c_int]
    lib.pl_profiling_read.restype = ctypes.c_int
    lib.pl_profiling_read.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_int64), ctypes.c_int]
    lib.pl_profile_param.restype = ctypes.c_int
    lib.pl_profile_param.argtypes = [_P, _I64, _I64, _P, _P, ctypes.c_int, ctypes.c_double, _P, _P,
                                     ctypes.POINTER(_I64), _P, ctypes.POINTER(ctypes.c_int32)]
    lib.pl_autotune_workspace_size.restype = ctypes.c_int
    lib.pl_autotune_workspace_size.argtypes = [_I64, _I64, _I64, _I64, _I64, ctypes.POINTER(_SZ)]
    lib.pl_autotune.restype = ctypes.c_int
    lib.pl_autotune.argtypes = [_P, _P, _P, _I64, _I64, _P, _I64, _P, _I64, _I64, ctypes.c_double,
                                ctypes.POINTER(PlOpts), ctypes.POINTER(ctypes.c_double), _P, _SZ,
                                _P]
    lib.pl_to_internal.restype = ctypes.c_int
    lib.pl_to_internal.argtypes = [_P, _I64, ctypes.c_int, _P]
    lib.pl_from_internal.restype = ctypes.c_int
    lib.pl_from_internal.argtypes = [_P, _I64, ctypes.c_int, _P]
    lib.pl_mle_workspace_size.restype = ctypes.c_int
    lib.pl_mle_workspace_size.argtypes = [_I64, _I64, _I64, _I64, ctypes.POINTER(PlOpts),
                                          ctypes.POINTER(_SZ)]
    lib.pl_mle.restype = ctypes.c_int
    lib.pl_mle.argtypes = [_P, _P, _P, _I64, _I64, _P, _I64, _P, _I64, ctypes.c_int32,
                           ctypes.c_int32, ctypes.c_double, ctypes.c_int32, _P, _P, _P,
                           ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(PlOpts), _P, _SZ, _P]
    lib.pl_hessian_workspace_size.restype = ctypes.c_int
    lib.pl_hessian_workspace_size.argtypes = [_I64, _I64, ctypes.POINTER(PlOpts),
                                              ctypes.POINTER(_SZ)]
    lib.pl_hessian.restype = ctypes.c_int
    lib.pl_hessian.argtypes = [_P, _P, _P, _I64, _I64, _P, ctypes.c_double, ctypes.c_int,
                               ctypes.c_int, ctypes.c_double, _P, _P, _P, ctypes.POINTER(PlOpts),
                               _P, _SZ, _P]
    lib.pl_config_points.restype = ctypes.c_int
    lib.pl_config_points.argtypes = [_P, ctypes.c_int, ctypes.c_int, _P, _P, _I64, _P, _I64, _P,
                                     _P, _P, ctypes.POINTER(_I64)]
    lib.pl_sphere_points.restype = ctypes.c_int
    lib.pl_sphere_points.argtypes = [ctypes.c_int, _I64, _P, ctypes.c_int, _P,
                                     ctypes.POINTER(ctypes.c_double)]
    lib.pl_lambda_grid.restype = ctypes.c_int
    lib.pl_lambda_grid.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, _I64, _P]
    lib.pl_chisq_quantile.restype = ctypes.c_int
    lib.pl_chisq_quantile.argtypes = [ctypes.c_int, ctypes.c_double,
                                      ctypes.POINTER(ctypes.c_double)]
    lib.pl_batch_create.restype = ctypes.c_int
    lib.pl_batch_create.argtypes = [ctypes.POINTER(PlDataset), _I64, _I64, _P, _I64,
                                    ctypes.POINTER(PlOpts), ctypes.POINTER(ctypes.c_void_p)]
    lib.pl_batch_workspace_size.restype = ctypes.c_int
    lib.pl_batch_workspace_size.argtypes = [_P, ctypes.POINTER(_SZ)]
    lib.pl_batch_stats.restype = ctypes.c_int
    lib.pl_batch_stats.argtypes = [_P, ctypes.POINTER(_I64), ctypes.POINTER(_I64),
                                   ctypes.POINTER(_I64)]
    lib.pl_batch_run.restype = ctypes.c_int
    lib.pl_batch_run.argtypes = [_P, _P, _P, _P, _SZ, _P]
    lib.pl_batch_error.restype = ctypes.c_int
    lib.pl_batch_error.argtypes = [_P, _P, ctypes.POINTER(ctypes.c_int32)]
    lib.pl_batch_destroy.restype = None
    lib.pl_batch_destroy.argtypes = [_P]
    lib.pl_batch_autotune_workspace_size.restype = ctypes.c_int
    lib.pl_batch_autotune_workspace_size.argtypes = [ctypes.POINTER(PlDataset), _I64, _I64, _P,
                                                     _I64, ctypes.POINTER(_SZ)]
    lib.pl_batch_autotune.restype = ctypes.c_int
    lib.pl_batch_autotune.argtypes = [ctypes.POINTER(PlDataset), _I64, _I64, _P, _I64,
                                      ctypes.c_double, ctypes.POINTER(PlOpts), _P, _P, _SZ, _P]
    lib.pl_tune_cache_set.restype = ctypes.c_int
    lib.pl_tune_cache_set.argtypes = [ctypes.c_char_p]
    lib.pl_tune_store.restype = ctypes.c_int
    lib.pl_tune_store.argtypes = [ctypes.c_char_p, ctypes.c_int, _I64, _I64, _I64, ctypes.c_double,
                                  ctypes.POINTER(PlOpts), ctypes.c_double]
    lib.pl_tune_lookup.restype = ctypes.c_int
    lib.pl_tune_lookup.argtypes = [ctypes.c_char_p, ctypes.c_int, _I64, _I64, _I64,
                                   ctypes.c_double, ctypes.POINTER(PlOpts)]
    lib.pl_tune_cache_stats.restype = ctypes.c_int
    lib.pl_tune_cache_stats.argtypes = [ctypes.POINTER(_I64), ctypes.POINTER(_I64),
                                        ctypes.POINTER(_I64)]
    if path is None:
        _lib = lib
    return lib


def check(rc: int, what: str):
    if rc != 0:
        msg = load().pl_error_string(rc).decode()
        raise PlError(f"{what} returned {rc} ({msg})")
