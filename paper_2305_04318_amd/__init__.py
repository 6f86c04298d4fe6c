"""MI355X-native profile log-likelihoods for Box-Cox transformed Gaussian
geostatistical models with anisotropic Matern correlation.

The computation lives in the HIP library libplprof.so (C ABI in
include/plprof.h); this package marshals arguments and provides device
memory and streams through PyTorch.  There is no CPU fallback: if the
library is missing every entry point raises.
"""
from ._lib import (PL_FP64, PL_MIXED, PL_INFO_BAD_Y, PL_INFO_FALLBACK, PL_INFO_RANK, PlError,
                   load)


_SUBMODULES = {"api", "build", "_lib", "batch", "serve", "profiles"}


def __getattr__(name):
    # torch-facing entry points are imported lazily so that loading the
    # library (and the CPU tests of the ABI) need not import torch
    import importlib
    if name.startswith("__"):
        raise AttributeError(name)
    if name in _SUBMODULES:
        return importlib.import_module(f"{__name__}.{name}")
    api = importlib.import_module(f"{__name__}.api")
    if hasattr(api, name):
        return getattr(api, name)
    raise AttributeError(name)


__all__ = ["load", "PlError", "PL_FP64", "PL_MIXED", "PL_INFO_RANK", "PL_INFO_BAD_Y",
           "PL_INFO_FALLBACK", "profile_loglik", "matern_cov", "chol_batched",
           "workspace_size", "Inputs", "version"]
