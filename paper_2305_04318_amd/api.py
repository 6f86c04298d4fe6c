"""Python entry points with the C ABI's names.  PyTorch provides device
memory and the stream; all arithmetic happens in the HIP library."""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import PlOpts, check, load

RESULT_FIELDS = ("loglik", "logdet_v", "logdet_xvx", "ssq_y", "ssq_betahat",
                 "ssq_resid", "sigma2_hat", "jacobian", "loglik_reml")
_PREC = {"fp64": _lib.PL_FP64, "mixed": _lib.PL_MIXED}


def _stream_ptr(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev_f64(t, device, shape=None):
    t = torch.as_tensor(t, dtype=torch.float64, device=device)
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"expected shape {shape}, got {tuple(t.shape)}")
    return t.contiguous()


def _host_f64(a, ncol=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if ncol is not None:
        a = a.reshape(-1, ncol)
    return a


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _opts(precision="fp64", chunk=0, refine=1, fallback=True, flush=0):
    o = PlOpts()
    o.precision = _PREC[precision]
    o.refine = int(refine)
    o.chunk = int(chunk or 0)
    o.flags = 0 if fallback else _lib.PL_OPT_NO_FALLBACK
    o.flush = int(flush or 0)
    return o


def version() -> str:
    return load().pl_version().decode()


def workspace_size(n, p, K, M, precision="fp64", chunk=0) -> int:
    lib = load()
    out = ctypes.c_size_t(0)
    o = _opts(precision, chunk)
    check(lib.pl_workspace_size(n, p, K, M, ctypes.byref(o), ctypes.byref(out)), "pl_workspace_size")
    return int(out.value)


def matern_cov(locs, omega, device="cuda", ld=None, stream=None, dtype="f64"):
    """V_k = R(omega_k) + nu_k^2 I, lower triangle, as a (K, n, ld) tensor whose
    row k*... is column-major per matrix (V[k].T[:n, :n] is the matrix).
    dtype "f64" or "f32" (elements computed in FP64, rounded once)."""
    lib = load()
    locs_d = _dev_f64(locs, device)
    n = locs_d.shape[0]
    om = _host_f64(omega, 5)
    K = om.shape[0]
    ld = ld or n
    tdt = {"f64": torch.float64, "f32": torch.float32}[dtype]
    V = torch.zeros((K, n, ld), dtype=tdt, device=device)
    wb = ctypes.c_size_t(0)
    check(lib.pl_matern_workspace_size(K, ctypes.byref(wb)), "pl_matern_workspace_size")
    work = torch.empty(max(1, wb.value), dtype=torch.uint8, device=device)
    rc = lib.pl_matern_cov(_ptr(locs_d), n, om.ctypes.data_as(ctypes.c_void_p), K,
                           _lib.PL_F64 if dtype == "f64" else _lib.PL_F32, _ptr(V), ld,
                           _ptr(work), wb.value, _stream_ptr(stream))
    check(rc, "pl_matern_cov")
    return V


def chol_batched(V, n=None, stream=None):
    """In-place Cholesky of V (K, n, ld) column-major matrices; returns
    (logdet, info).  A float64 V is factored in FP64, a float32 V in the mixed
    form (FP32 factor, FP64 diagonal tiles and log-determinant)."""
    lib = load()
    K, n_, ld = V.shape
    n = n or n_
    prec = {torch.float64: _lib.PL_FP64, torch.float32: _lib.PL_MIXED}[V.dtype]
    logdet = torch.empty(K, dtype=torch.float64, device=V.device)
    info = torch.empty(K, dtype=torch.int32, device=V.device)
    wb = ctypes.c_size_t(0)
    check(lib.pl_chol_workspace_size(K, prec, ctypes.byref(wb)), "pl_chol_workspace_size")
    work = torch.empty(max(1, wb.value), dtype=torch.uint8, device=V.device)
    rc = lib.pl_chol_batched(_ptr(V), n, K, ld, prec, _ptr(logdet), _ptr(info), _ptr(work),
                             wb.value, _stream_ptr(stream))
    check(rc, "pl_chol_batched")
    return logdet, info


def unpack_records(rec: torch.Tensor) -> dict:
    """(K, M, 10) float64 record tensor -> dict of (K, M) tensors."""
    out = {f: rec[..., i] for i, f in enumerate(RESULT_FIELDS)}
    out["info"] = rec.view(torch.int32)[..., 18]
    return out


class Inputs:
    """Device-resident copy of one dataset (locs, y, X in column-major)."""

    def __init__(self, locs, y, X, device="cuda"):
        self.locs = _dev_f64(locs, device)
        self.n = self.locs.shape[0]
        self.y = _dev_f64(y, device, (self.n,))
        Xt = torch.as_tensor(X, dtype=torch.float64)
        if Xt.dim() == 1:
            Xt = Xt[:, None]
        self.p = Xt.shape[1]
        # column-major n x p: columns contiguous
        self.Xc = Xt.to(device).t().contiguous()
        self.device = device


def profile_loglik(locs, y, X, omega, lam, precision="fp64", chunk=0, return_beta=False,
                   out=None, beta=None, work=None, stream=None, device="cuda", inputs=None,
                   refine=1, fallback=True, flush=0, return_xvx_inv=False, xvx_inv=None):
    """Records for every (omega_k, lambda_m): dict of (K, M) tensors on the
    device, plus "beta" (K, M, p) when return_beta and "xvx_inv" (K, p, p),
    (X^T V_k^-1 X)^-1, when return_xvx_inv."""
    lib = load()
    inp = inputs if inputs is not None else Inputs(locs, y, X, device)
    om = _host_f64(omega, 5)
    lm = _host_f64(lam).reshape(-1)
    K, M = om.shape[0], lm.shape[0]
    dev = inp.device
    if out is None:
        out = torch.empty((K, M, 10), dtype=torch.float64, device=dev)
    if return_beta and beta is None:
        beta = torch.empty((K, M, inp.p), dtype=torch.float64, device=dev)
    if return_xvx_inv and xvx_inv is None:
        xvx_inv = torch.empty((K, inp.p, inp.p), dtype=torch.float64, device=dev)
    o = _opts(precision, chunk, refine, fallback, flush)
    if work is None:
        work = torch.empty(workspace_size(inp.n, inp.p, K, M, precision, chunk),
                           dtype=torch.uint8, device=dev)
    rc = lib.pl_profile_loglik(_ptr(inp.locs), _ptr(inp.y), _ptr(inp.Xc), inp.n, inp.p,
                               om.ctypes.data_as(ctypes.c_void_p), K,
                               lm.ctypes.data_as(ctypes.c_void_p), M, _ptr(out),
                               _ptr(beta) if return_beta else None,
                               _ptr(xvx_inv) if return_xvx_inv else None, ctypes.byref(o),
                               _ptr(work), work.numel(), _stream_ptr(stream))
    check(rc, "pl_profile_loglik")
    res = unpack_records(out)
    res["records"] = out
    if return_beta:
        res["beta"] = beta
    if return_xvx_inv:
        res["xvx_inv"] = xvx_inv
    return res


def profile_loglik_noalloc(locs, y, X, omega, lam, precision="fp64", chunk=0,
                           return_beta=False, out=None, beta=None, stream=None, device="cuda",
                           inputs=None, refine=1, fallback=True, flush=0):
    """profile_loglik with the library's fixed per-GPU scratch array as its
    workspace (pl_profile_loglik_noalloc): the library allocates nothing.
    Output tensors are allocated here unless `out` (and `beta`) are given."""
    lib = load()
    inp = inputs if inputs is not None else Inputs(locs, y, X, device)
    om = _host_f64(omega, 5)
    lm = _host_f64(lam).reshape(-1)
    K, M = om.shape[0], lm.shape[0]
    dev = inp.device
    if out is None:
        out = torch.empty((K, M, 10), dtype=torch.float64, device=dev)
    if return_beta and beta is None:
        beta = torch.empty((K, M, inp.p), dtype=torch.float64, device=dev)
    o = _opts(precision, chunk, refine, fallback, flush)
    rc = lib.pl_profile_loglik_noalloc(_ptr(inp.locs), _ptr(inp.y), _ptr(inp.Xc), inp.n, inp.p,
                                       om.ctypes.data_as(ctypes.c_void_p), K,
                                       lm.ctypes.data_as(ctypes.c_void_p), M, _ptr(out),
                                       _ptr(beta) if return_beta else None, None,
                                       ctypes.byref(o), _stream_ptr(stream))
    check(rc, "pl_profile_loglik_noalloc")
    res = unpack_records(out)
    res["records"] = out
    if return_beta:
        res["beta"] = beta
    return res


def profile_curves(res, lam, n, sigma_grid=None, beta_grid=None, stream=None):
    """pl_profile_curves over the output `res` of one profile_loglik call
    (made with return_beta and return_xvx_inv when beta_grid is given).
    sigma_grid: (Gs,) values > 0; beta_grid: (p, Gb), row j the values of
    coefficient j.  Returns a dict with "sigma" (Gs,), "sigma_arg" (Gs,),
    "beta" (p, Gb), "beta_arg" (p, Gb) device tensors (arg = record index
    k*M + m of the maximum)."""
    lib = load()
    rec = res["records"]
    K, M = rec.shape[0], rec.shape[1]
    lm = _host_f64(lam).reshape(-1)
    if lm.shape[0] != M:
        raise ValueError("lam must be the lambda values of that call")
    dev = rec.device
    sg = _host_f64(sigma_grid).reshape(-1) if sigma_grid is not None else np.zeros(0)
    Gs = sg.shape[0]
    beta = res.get("beta")
    xvi = res.get("xvx_inv")
    p = beta.shape[2] if beta is not None else (xvi.shape[1] if xvi is not None else 1)
    if beta_grid is not None:
        if beta is None or xvi is None:
            raise ValueError("beta curves need return_beta and return_xvx_inv")
        bg = _host_f64(beta_grid)
        if bg.ndim != 2 or bg.shape[0] != p:
            raise ValueError(f"beta_grid must be (p={p}, Gb)")
        bg = np.ascontiguousarray(bg)
    else:
        bg = np.zeros((p, 0))
    Gb = bg.shape[1]
    prof_s = torch.empty(max(Gs, 1), dtype=torch.float64, device=dev)
    arg_s = torch.empty(max(Gs, 1), dtype=torch.int64, device=dev)
    prof_b = torch.empty((p, max(Gb, 1)), dtype=torch.float64, device=dev)
    arg_b = torch.empty((p, max(Gb, 1)), dtype=torch.int64, device=dev)
    sz = ctypes.c_size_t(0)
    check(lib.pl_curves_workspace_size(p, M, Gs, Gb, ctypes.byref(sz)), "pl_curves_workspace_size")
    work = torch.empty(max(1, sz.value), dtype=torch.uint8, device=dev)
    rc = lib.pl_profile_curves(_ptr(rec), _ptr(beta) if beta is not None else None,
                               _ptr(xvi) if xvi is not None else None, int(n), p, K,
                               lm.ctypes.data_as(ctypes.c_void_p), M,
                               sg.ctypes.data_as(ctypes.c_void_p), Gs,
                               bg.ctypes.data_as(ctypes.c_void_p), Gb, _ptr(prof_s), _ptr(arg_s),
                               _ptr(prof_b), _ptr(arg_b), _ptr(work), work.numel(),
                               _stream_ptr(stream))
    check(rc, "pl_profile_curves")
    return {"sigma": prof_s[:Gs], "sigma_arg": arg_s[:Gs], "beta": prof_b[:, :Gb],
            "beta_arg": arg_b[:, :Gb]}


PARAMS = ("range", "shape", "nugget", "ratio", "angle", "lambda")


def profile_param(res, omega, lam, which, drop=1.92):
    """pl_profile_param on the records of one profile_loglik call: the
    profile curve of parameter `which` (an index or a name from PARAMS) and
    its likelihood interval at level drop (1.92: 95%).  Returns a dict with
    "x", "y" (curve vertices), "argmax", "lower", "upper" and "open"
    (open_ends bits)."""
    lib = load()
    if isinstance(which, str):
        which = PARAMS.index(which)
    rec = res["records"] if isinstance(res, dict) else res
    K, M = rec.shape[0], rec.shape[1]
    host = np.ascontiguousarray(rec.detach().to("cpu").numpy())
    om = _host_f64(omega, 5)
    lm = _host_f64(lam).reshape(-1)
    if om.shape[0] != K or lm.shape[0] != M:
        raise ValueError("omega and lam must be those of the call")
    cap = max(K, M)
    cx = np.empty(cap)
    cy = np.empty(cap)
    npts = ctypes.c_int64(0)
    iv = np.empty(3)
    op = ctypes.c_int32(0)
    rc = lib.pl_profile_param(host.ctypes.data_as(ctypes.c_void_p), K, M,
                              om.ctypes.data_as(ctypes.c_void_p),
                              lm.ctypes.data_as(ctypes.c_void_p), int(which), float(drop),
                              cx.ctypes.data_as(ctypes.c_void_p),
                              cy.ctypes.data_as(ctypes.c_void_p), ctypes.byref(npts),
                              iv.ctypes.data_as(ctypes.c_void_p), ctypes.byref(op))
    check(rc, "pl_profile_param")
    k = npts.value
    return {"x": cx[:k].copy(), "y": cy[:k].copy(), "argmax": iv[0], "lower": iv[1],
            "upper": iv[2], "open": op.value}


AUTOTUNE_CANDIDATES = (("fp64", 0), ("mixed", 4), ("mixed", 2), ("mixed", 1))


class TuneReport(dict):
    """Per-candidate measurements of an autotuner; `cached` is True when the
    choice came from the tuning cache (nothing was timed)."""
    cached = False


def autotune(locs, y, X, omega, lam, tol=1e-3, sample=0, device="cuda", stream=None,
             inputs=None):
    """pl_autotune: the fastest form whose |delta loglik| against FP64 on the
    first `sample` omega points (0: 64) is <= tol.  Returns (choice, report) with
    choice = {"precision", "flush"} (keyword arguments of profile_loglik) and
    report = per candidate {"ms_per_omega", "max_abs_dl"}."""
    lib = load()
    inp = inputs if inputs is not None else Inputs(locs, y, X, device)
    om = _host_f64(omega, 5)
    lm = _host_f64(lam).reshape(-1)
    K, M = om.shape[0], lm.shape[0]
    sz = ctypes.c_size_t(0)
    check(lib.pl_autotune_workspace_size(inp.n, inp.p, K, M, int(sample), ctypes.byref(sz)),
          "pl_autotune_workspace_size")
    work = torch.empty(sz.value, dtype=torch.uint8, device=inp.device)
    o = _opts()
    rep = (ctypes.c_double * 8)()
    rc = lib.pl_autotune(_ptr(inp.locs), _ptr(inp.y), _ptr(inp.Xc), inp.n, inp.p,
                         om.ctypes.data_as(ctypes.c_void_p), K,
                         lm.ctypes.data_as(ctypes.c_void_p), M, int(sample), float(tol),
                         ctypes.byref(o), rep,
                         _ptr(work), work.numel(), _stream_ptr(stream))
    check(rc, "pl_autotune")
    choice = {"precision": "mixed" if o.precision == _lib.PL_MIXED else "fp64", "flush": o.flush}
    report = TuneReport({f"{pr}" + (f"/flush{f}" if f else ""):
                         {"ms_per_omega": rep[i], "max_abs_dl": rep[4 + i]}
                         for i, (pr, f) in enumerate(AUTOTUNE_CANDIDATES)})
    report.cached = bool(rep[0] == -2.0)
    return choice, report


def tune_cache_set(path=None):
    """pl_tune_cache_set: the autotuners reuse and persist their choices in the
    file `path` ("" : in memory only; None: no cache, every call measures)."""
    check(load().pl_tune_cache_set(None if path is None else path.encode()), "pl_tune_cache_set")


def _choice(o):
    return {"precision": "mixed" if o.precision == _lib.PL_MIXED else "fp64", "flush": o.flush,
            "chunk": int(o.chunk), "lanes": int(o.lanes),
            "schedule": "persistent" if o.flags & _lib.PL_OPT_BATCH_PERSISTENT else "bucketed"}


def tune_lookup(n, q, tol, kind=0, units=0, arch=None):
    """pl_tune_lookup: the stored choice for this key as a dict, or None."""
    o = _opts()
    rc = load().pl_tune_lookup(arch.encode() if arch else None, int(kind), int(n), int(units),
                               int(q), float(tol), ctypes.byref(o))
    if rc == _lib.PL_TUNE_MISS:
        return None
    check(rc, "pl_tune_lookup")
    return _choice(o)


def tune_store(choice, n, q, tol, kind=0, units=0, arch=None, ms=0.0):
    """pl_tune_store: store `choice` (a dict as tune_lookup returns) for this key."""
    o = _opts(choice.get("precision", "fp64"), choice.get("chunk", 0), 1, True,
              choice.get("flush", 0))
    o.lanes = int(choice.get("lanes", 0))
    if choice.get("schedule") == "persistent":
        o.flags |= _lib.PL_OPT_BATCH_PERSISTENT
    check(load().pl_tune_store(arch.encode() if arch else None, int(kind), int(n), int(units),
                               int(q), float(tol), ctypes.byref(o), float(ms)), "pl_tune_store")


def tune_stats():
    e, h, m = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    check(load().pl_tune_cache_stats(ctypes.byref(e), ctypes.byref(h), ctypes.byref(m)),
          "pl_tune_cache_stats")
    return {"entries": e.value, "hits": h.value, "misses": m.value}


PARAM_NAMES_INTERNAL = ("gamma1", "shape~", "nu", "gamma2", "gamma3")


def to_internal(omega, shape_transform=0):
    """pl_to_internal: natural omega (K x 5) -> internal (gamma1, kappa~, nu,
    gamma2, gamma3); shape_transform 0: log kappa, 1: 1/sqrt(kappa)."""
    om = _host_f64(omega, 5)
    out = np.empty_like(om)
    check(load().pl_to_internal(om.ctypes.data_as(ctypes.c_void_p), om.shape[0],
                                int(shape_transform), out.ctypes.data_as(ctypes.c_void_p)),
          "pl_to_internal")
    return out


def from_internal(internal, shape_transform=0):
    """pl_from_internal: the inverse of to_internal (a negative nu gives a
    negative nugget -nu^2)."""
    w = _host_f64(internal, 5)
    out = np.empty_like(w)
    check(load().pl_from_internal(w.ctypes.data_as(ctypes.c_void_p), w.shape[0],
                                  int(shape_transform), out.ctypes.data_as(ctypes.c_void_p)),
          "pl_from_internal")
    return out


def default_starts(locs, fractions=(0.05, 0.2, 0.5), shapes=(0.5, 2.0), nuggets=(0.1, 0.5)):
    """Isotropic starting points for mle: ranges at `fractions` of the
    diagonal of the locations' bounding box, every combination with `shapes`
    and `nuggets` (ratio 1, angle 0)."""
    xy = np.asarray(locs.cpu() if isinstance(locs, torch.Tensor) else locs, dtype=np.float64)
    diag = float(np.hypot(*(xy.max(axis=0) - xy.min(axis=0))))
    return np.array([[f * diag, k, nu, 1.0, 0.0] for f in fractions for k in shapes
                     for nu in nuggets])


def mle(locs, y, X, lam, omega0=None, fixed=(), reml=False, tol=1e-4, max_iter=200,
        precision="fp64", flush=0, device="cuda", stream=None, inputs=None):
    """pl_mle: maximum-likelihood (reml: restricted) estimates of omega and
    lambda from the starts omega0 (default: default_starts(locs)), searching
    lambda over the values `lam` and then a fine set around the best one.
    `fixed` names search coordinates held at their start values: any of
    "range" (gamma1), "shape", "nugget", "aniso" (gamma2 and gamma3).
    Returns {"omega", "lambda", "loglik", "iterations"}."""
    lib = load()
    inp = inputs if inputs is not None else Inputs(locs, y, X, device)
    om = _host_f64(default_starts(locs) if omega0 is None else omega0, 5)
    lm = _host_f64(lam).reshape(-1)
    bits = {"range": 1, "shape": 2, "nugget": 4, "aniso": 8 | 16}
    mask = 0
    for name in fixed:
        mask |= bits[name]
    o = _opts(precision, flush=flush)
    sz = ctypes.c_size_t(0)
    check(lib.pl_mle_workspace_size(inp.n, inp.p, om.shape[0], lm.shape[0], ctypes.byref(o),
                                    ctypes.byref(sz)), "pl_mle_workspace_size")
    work = torch.empty(sz.value, dtype=torch.uint8, device=inp.device)
    oh = np.empty(5)
    lh, llh = ctypes.c_double(0.0), ctypes.c_double(0.0)
    its = ctypes.c_int32(0)
    rc = lib.pl_mle(_ptr(inp.locs), _ptr(inp.y), _ptr(inp.Xc), inp.n, inp.p,
                    om.ctypes.data_as(ctypes.c_void_p), om.shape[0],
                    lm.ctypes.data_as(ctypes.c_void_p), lm.shape[0], mask, 1 if reml else 0,
                    float(tol), int(max_iter), oh.ctypes.data_as(ctypes.c_void_p),
                    ctypes.byref(lh), ctypes.byref(llh), ctypes.byref(its), ctypes.byref(o),
                    _ptr(work), work.numel(), _stream_ptr(stream))
    check(rc, "pl_mle")
    return {"omega": oh, "lambda": lh.value, "loglik": llh.value, "iterations": its.value}


# contour levels (upper-tail probabilities) of the paper's two data examples
PAPER_ALPHA = (1e-5, 0.01, 0.1, 0.2, 0.25, 0.3, 0.5, 0.8, 0.9, 0.95, 0.99, 0.999)


def chisq_quantile(dof, upper):
    """pl_chisq_quantile: q with Pr(chi^2_dof > q) = upper."""
    q = ctypes.c_double(0.0)
    check(load().pl_chisq_quantile(int(dof), float(upper), ctypes.byref(q)), "pl_chisq_quantile")
    return q.value


def sphere_points(d, npts, seed=0, iters=300, init=None):
    """pl_sphere_points from `init` (npts x d) or from standard normal draws
    of a PCG64 generator seeded with `seed`.  Returns (points, closest
    distance)."""
    if init is None:
        init = np.random.Generator(np.random.PCG64(seed)).standard_normal((npts, d))
    x0 = _host_f64(init, d)
    out = np.empty_like(x0)
    md = ctypes.c_double(0.0)
    check(load().pl_sphere_points(int(d), x0.shape[0], x0.ctypes.data_as(ctypes.c_void_p),
                                  int(iters), out.ctypes.data_as(ctypes.c_void_p),
                                  ctypes.byref(md)), "pl_sphere_points")
    return out, md.value


def shape_transform_for(kappa_hat):
    """The paper's choice of shape transform: log below 4, 1/sqrt from 4 on."""
    return 0 if kappa_hat < 4.0 else 1


def hessian(locs, y, X, omega_hat, lambda_hat, shape_transform=None, fix_shape=False,
            delta=0.05, precision="fp64", device="cuda", stream=None, inputs=None):
    """pl_hessian: {"H" (d x d), "lambda_curv", "loglik", "shape_transform"}."""
    lib = load()
    inp = inputs if inputs is not None else Inputs(locs, y, X, device)
    om = _host_f64(omega_hat, 5)
    st = shape_transform_for(om[0, 1]) if shape_transform is None else int(shape_transform)
    o = _opts(precision)
    sz = ctypes.c_size_t(0)
    check(lib.pl_hessian_workspace_size(inp.n, inp.p, ctypes.byref(o), ctypes.byref(sz)),
          "pl_hessian_workspace_size")
    work = torch.empty(sz.value, dtype=torch.uint8, device=inp.device)
    d = 4 if fix_shape else 5
    H = np.empty((d, d))
    curv, ll = ctypes.c_double(0.0), ctypes.c_double(0.0)
    rc = lib.pl_hessian(_ptr(inp.locs), _ptr(inp.y), _ptr(inp.Xc), inp.n, inp.p,
                        om.ctypes.data_as(ctypes.c_void_p), float(lambda_hat), st,
                        1 if fix_shape else 0, float(delta), H.ctypes.data_as(ctypes.c_void_p),
                        ctypes.byref(curv), ctypes.byref(ll), ctypes.byref(o), _ptr(work),
                        work.numel(), _stream_ptr(stream))
    check(rc, "pl_hessian")
    return {"H": H, "lambda_curv": curv.value, "loglik": ll.value, "shape_transform": st}


def config_points(omega_hat, H, alpha, sphere, uniforms, shape_transform=0, fix_shape=False):
    """pl_config_points: (omega rows, level-major; repaired eigenvalues;
    number of repaired nuggets)."""
    om = _host_f64(omega_hat, 5)
    Hh = _host_f64(H)
    al = _host_f64(alpha).reshape(-1)
    d = 4 if fix_shape else 5
    sp = _host_f64(sphere, d)
    un = _host_f64(uniforms).reshape(-1)
    if un.shape[0] < al.shape[0] * sp.shape[0]:
        raise ValueError("need one uniform per output point")
    out = np.empty((al.shape[0] * sp.shape[0], 5))
    eig = np.empty(d)
    nrep = ctypes.c_int64(0)
    P = ctypes.c_void_p
    check(load().pl_config_points(om.ctypes.data_as(P), int(shape_transform),
                                  1 if fix_shape else 0, Hh.ctypes.data_as(P),
                                  al.ctypes.data_as(P), al.shape[0], sp.ctypes.data_as(P),
                                  sp.shape[0], un.ctypes.data_as(P), out.ctypes.data_as(P),
                                  eig.ctypes.data_as(P), ctypes.byref(nrep)), "pl_config_points")
    return out, eig, nrep.value


def lambda_grid(lambda_hat, lambda_curv, m=30, tail=0.01):
    """pl_lambda_grid: m values between the tail and 1 - tail quantiles of
    the normal approximation in lambda."""
    out = np.empty(int(m))
    check(load().pl_lambda_grid(float(lambda_hat), float(lambda_curv), float(tail), int(m),
                                out.ctypes.data_as(ctypes.c_void_p)), "pl_lambda_grid")
    return out


def configure(locs, y, X, fits, alpha=PAPER_ALPHA, npts=None, n_lambda=30, delta=0.05,
              seed=0, sphere_iters=300, device="cuda", stream=None, inputs=None):
    """Step 2 end to end: for every fit (a dict from mle, with "fixed_shape"
    True for the fits with the shape held), the Hessian, its repair and the
    points on every level (726 unit-sphere points in 5-D, 120 in 4-D unless
    npts is given); the Box-Cox grid from the first fit.  Returns {"omega"
    (all points), "lambda", "fits" (per fit: H, shape transform, eigenvalues,
    number of points, repaired nuggets)}."""
    inp = inputs if inputs is not None else Inputs(locs, y, X, device)
    rng = np.random.Generator(np.random.PCG64(seed))
    spheres = {}
    omegas, info = [], []
    lam_grid = None
    for f in fits:
        fix = bool(f.get("fixed_shape", False))
        d = 4 if fix else 5
        npd = npts if npts is not None else (120 if fix else 726)
        if d not in spheres:
            spheres[d] = sphere_points(d, npd, init=rng.standard_normal((npd, d)),
                                       iters=sphere_iters)[0]
        h = hessian(None, None, None, f["omega"], f["lambda"], fix_shape=fix, delta=delta,
                    stream=stream, inputs=inp)
        u = rng.uniform(size=len(alpha) * spheres[d].shape[0])
        pts, eig, nrep = config_points(f["omega"], h["H"], alpha, spheres[d], u,
                                       h["shape_transform"], fix)
        omegas.append(pts)
        info.append({"H": h["H"], "shape_transform": h["shape_transform"], "eigvals": eig,
                     "points": pts.shape[0], "nugget_repaired": nrep,
                     "lambda_curv": h["lambda_curv"]})
        if lam_grid is None:
            lam_grid = lambda_grid(f["lambda"], h["lambda_curv"], n_lambda)
    return {"omega": np.concatenate(omegas), "lambda": lam_grid, "fits": info}


def profiling_enable(on: bool = True):
    """Start (clearing counters) or stop HIP-event timing of the library's kernels."""
    check(load().pl_profiling_enable(1 if on else 0), "pl_profiling_enable")


def profiling_read() -> dict:
    """Per kernel class: total ms, algorithmic flops and launch count of the
    launches recorded since profiling_enable(True)."""
    n = len(_lib.KERNEL_CLASSES)
    ms = (ctypes.c_double * n)()
    fl = (ctypes.c_double * n)()
    ln = (ctypes.c_int64 * n)()
    check(load().pl_profiling_read(ms, fl, ln, n), "pl_profiling_read")
    return {c: {"ms": ms[i], "flops": fl[i], "launches": ln[i]}
            for i, c in enumerate(_lib.KERNEL_CLASSES)}
