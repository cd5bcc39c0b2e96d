"""ctypes binding of libglam.so (the C ABI of include/glam.h).

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  torch tensors supply device memory and the HIP stream.  Importing this
module raises if the built library is missing (build it with
``python -m paper_1510_03298_amd.build``).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libglam.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1510_03298_amd.build`")

_lib = ctypes.CDLL(LIB_PATH)

GLAM_OK, GLAM_EINVAL, GLAM_ENOMEM, GLAM_EDEVICE, GLAM_ENOCONV, GLAM_ENONFINITE = range(6)
GAUSSIAN, POISSON, BINOMIAL, GAMMA = 0, 1, 2, 3
F64, F32, BF16 = 0, 1, 2
MAX_INNER_P = 32
MAX_INNER_N = 256
DTYPES = {"f64": F64, "f32": F32, "bf16": BF16}
FAMILIES = {"gaussian": GAUSSIAN, "poisson": POISSON, "binomial": BINOMIAL, "gamma": GAMMA}
PENALTIES = {"lasso": 0, "scad": 1, "ridge": 2}

_i64p = ctypes.POINTER(ctypes.c_int64)
_vp = ctypes.c_void_p


class GlamProblem(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int), ("n", ctypes.c_int64 * 3), ("p", ctypes.c_int64 * 3),
                ("X", _vp * 3), ("Y", _vp), ("obs_w", _vp), ("family", ctypes.c_int), ("pen_w", _vp)]


class GlamOptions(ctypes.Structure):
    _fields_ = [("lambda_", ctypes.POINTER(ctypes.c_double)), ("nlambda", ctypes.c_int),
                ("lambda_min_ratio", ctypes.c_double), ("dtype", ctypes.c_int), ("kkt_tol", ctypes.c_double),
                ("nu", ctypes.c_double), ("max_outer", ctypes.c_int), ("max_inner", ctypes.c_int),
                ("check_every", ctypes.c_int), ("theta0", _vp), ("stream", _vp), ("profile_every", ctypes.c_int),
                ("graph_mode", ctypes.c_int), ("inner_mode", ctypes.c_int), ("alpha", ctypes.c_double),
                ("penalty", ctypes.c_int), ("scad_a", ctypes.c_double), ("msa_steps", ctypes.c_int),
                ("extrapolation", ctypes.c_int), ("kron_step", ctypes.c_int)]


class GlamMultiProblem(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int), ("n", ctypes.c_int64 * 3), ("c", ctypes.c_int), ("p", _i64p),
                ("X", ctypes.POINTER(_vp)), ("Y", _vp), ("obs_w", _vp), ("family", ctypes.c_int), ("pen_w", _vp)]


class GlamResult(ctypes.Structure):
    _fields_ = [("theta", _vp), ("lambda_out", ctypes.POINTER(ctypes.c_double)),
                ("kkt", ctypes.POINTER(ctypes.c_double)), ("objective", ctypes.POINTER(ctypes.c_double)),
                ("iters_outer", ctypes.POINTER(ctypes.c_int)), ("iters_inner", ctypes.POINTER(ctypes.c_int)),
                ("status", ctypes.POINTER(ctypes.c_int)), ("n_done", ctypes.c_int), ("lambda_max", ctypes.c_double),
                ("seconds", ctypes.c_double), ("chain_ms", ctypes.c_double), ("chain_samples", ctypes.c_int),
                ("iter_ms", ctypes.c_double), ("inner_total", ctypes.c_longlong), ("escalated_at", ctypes.c_int),
                ("adj_ms", ctypes.c_double), ("fwd_ms", ctypes.c_double)]


class GlamBatchOptions(ctypes.Structure):
    _fields_ = [("lambda_", ctypes.POINTER(ctypes.c_double)), ("lambda_ratio", ctypes.c_double),
                ("dtype", ctypes.c_int), ("kkt_tol", ctypes.c_double), ("max_outer", ctypes.c_int),
                ("max_inner", ctypes.c_int), ("check_every", ctypes.c_int), ("stream", _vp),
                ("alpha", ctypes.c_double), ("tuning", ctypes.c_int), ("graph_mode", ctypes.c_int)]


class GlamBatchResult(ctypes.Structure):
    _fields_ = [("theta", ctypes.POINTER(_vp)), ("lambda_out", ctypes.POINTER(ctypes.c_double)),
                ("lambda_max", ctypes.POINTER(ctypes.c_double)), ("kkt", ctypes.POINTER(ctypes.c_double)),
                ("objective", ctypes.POINTER(ctypes.c_double)), ("iters_outer", ctypes.POINTER(ctypes.c_int)),
                ("status", ctypes.POINTER(ctypes.c_int)), ("steps", ctypes.c_longlong),
                ("problem_steps", ctypes.c_longlong), ("seconds", ctypes.c_double),
                ("graph_replays", ctypes.c_longlong), ("tune_seconds", ctypes.c_double)]


def _sig(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args
    return f


glam_status_string = _sig("glam_status_string", ctypes.c_char_p, [ctypes.c_int])
glam_last_error = _sig("glam_last_error", ctypes.c_char_p, [])
glam_version = _sig("glam_version", ctypes.c_char_p, [])
glam_rho_workspace_size = _sig("glam_rho_workspace_size", ctypes.c_size_t, [ctypes.c_int, _i64p, _i64p, ctypes.c_int])
glam_rho_forward = _sig("glam_rho_forward", ctypes.c_int,
                        [ctypes.c_int, _i64p, _i64p, ctypes.POINTER(_vp), _vp, _vp, ctypes.c_int, _vp,
                         ctypes.c_size_t, _vp])
glam_rho_forward_static = _sig("glam_rho_forward_static", ctypes.c_int,
                               [ctypes.c_int, _i64p, _i64p, ctypes.POINTER(_vp), _vp, _vp, ctypes.c_int, _vp])
glam_rho_adjoint = _sig("glam_rho_adjoint", ctypes.c_int,
                        [ctypes.c_int, _i64p, _i64p, ctypes.POINTER(_vp), _vp, _vp, ctypes.c_int, _vp,
                         ctypes.c_size_t, _vp])
glam_fit_path = _sig("glam_fit_path", ctypes.c_int,
                     [ctypes.POINTER(GlamProblem), ctypes.POINTER(GlamOptions), ctypes.POINTER(GlamResult)])
glam_fit_path_multi = _sig("glam_fit_path_multi", ctypes.c_int,
                           [ctypes.POINTER(GlamMultiProblem), ctypes.POINTER(GlamOptions), ctypes.POINTER(GlamResult)])
glam_fit_batched = _sig("glam_fit_batched", ctypes.c_int,
                        [ctypes.POINTER(GlamProblem), ctypes.c_int, ctypes.POINTER(GlamBatchOptions),
                         ctypes.POINTER(GlamBatchResult)])
glam_nll_workspace_size = _sig("glam_nll_workspace_size", ctypes.c_size_t, [_i64p, _i64p, ctypes.c_int])
glam_poisson_nll_forward = _sig("glam_poisson_nll_forward", ctypes.c_int,
                                [_i64p, _i64p, ctypes.POINTER(_vp), _vp, _vp, _vp, ctypes.c_int, _vp,
                                 ctypes.c_size_t, _vp])
glam_poisson_nll_backward = _sig("glam_poisson_nll_backward", ctypes.c_int,
                                 [_i64p, _i64p, ctypes.POINTER(_vp), _vp, _vp, _vp, _vp, ctypes.c_int, _vp,
                                  ctypes.c_size_t, _vp])

glam_nll_packed_workspace_size = _sig("glam_nll_packed_workspace_size", ctypes.c_size_t, [_i64p, _i64p, ctypes.c_int])
glam_poisson_nll_pack = _sig("glam_poisson_nll_pack", ctypes.c_int,
                             [_i64p, _i64p, ctypes.POINTER(_vp), _vp, ctypes.c_int, _vp, ctypes.c_size_t, _vp])
glam_poisson_nll_forward_packed = _sig("glam_poisson_nll_forward_packed", ctypes.c_int,
                                       [_i64p, _i64p, _vp, _vp, ctypes.c_int, _vp, ctypes.c_size_t, _vp])
glam_poisson_nll_backward_packed = _sig("glam_poisson_nll_backward_packed", ctypes.c_int,
                                        [_i64p, _i64p, _vp, _vp, _vp, ctypes.c_int, _vp, ctypes.c_size_t, _vp])

EXPORTED = ["glam_status_string", "glam_last_error", "glam_version", "glam_rho_workspace_size",
            "glam_rho_forward", "glam_rho_forward_static", "glam_rho_adjoint", "glam_fit_path", "glam_fit_path_multi", "glam_fit_batched", "glam_nll_workspace_size",
            "glam_poisson_nll_forward", "glam_poisson_nll_backward", "glam_nll_packed_workspace_size",
            "glam_poisson_nll_pack", "glam_poisson_nll_forward_packed", "glam_poisson_nll_backward_packed"]


class GlamError(RuntimeError):
    def __init__(self, code, where=""):
        self.code = code
        msg = glam_status_string(code).decode()
        detail = glam_last_error().decode()
        super().__init__(f"{where}: {msg} ({detail})" if where else f"{msg} ({detail})")


def _check(code, where):
    if code != GLAM_OK:
        raise GlamError(code, where)


# ----------------------------------------------------------------------------- torch helpers
def _torch():
    import torch
    return torch


def torch_dtype(dt):
    torch = _torch()
    return {F64: torch.float64, F32: torch.float32, BF16: torch.bfloat16}[dt]


def out_dtype(dt):
    torch = _torch()
    return torch.float64 if dt == F64 else torch.float32


def _stream_ptr(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _sizes(n, p):
    """Host size arrays (d = len(n) entries, padded to 3)."""
    pad = [0] * (3 - len(n))
    return (ctypes.c_int64 * 3)(*([int(v) for v in n] + pad)), (ctypes.c_int64 * 3)(*([int(v) for v in p] + pad))


def _ptrs(Xs):
    return (_vp * 3)(*([x.data_ptr() for x in Xs] + [None] * (3 - len(Xs))))


def _fortran_flat(t):
    """Column-major (vec) flattening of a 3-D torch tensor."""
    return t.permute(*reversed(range(t.dim()))).contiguous().reshape(-1)


def to_device_colmajor(a, dtype, device="cuda"):
    """numpy array (any order) -> 1-D device tensor holding its column-major vec."""
    torch = _torch()
    flat = np.asarray(a, dtype=np.float64).reshape(-1, order="F")
    tdt = torch_dtype(dtype) if isinstance(dtype, int) else dtype
    return torch.from_numpy(np.ascontiguousarray(flat)).to(tdt).to(device=device)


def from_colmajor(t, dims):
    return t.detach().to("cpu", dtype=_torch().float64).numpy().reshape(tuple(dims), order="F")


# ----------------------------------------------------------------------------- rho transforms
def rho_workspace_size(n, p, dtype):
    nn, pp = _sizes(n, p)
    return int(glam_rho_workspace_size(len(n), nn, pp, int(dtype)))


def rho_forward(Xs, theta, n, p, dtype, eta=None, workspace=None, stream=None):
    """eta = H(<X_j>, theta) on the device (all tensors 1-D column-major device tensors)."""
    torch = _torch()
    nn, pp = _sizes(n, p)
    ws_bytes = rho_workspace_size(n, p, dtype)
    if ws_bytes == 0:
        raise GlamError(GLAM_EINVAL, "rho_forward")
    if workspace is None:
        workspace = torch.empty(ws_bytes, dtype=torch.uint8, device=theta.device)
    if eta is None:
        eta = torch.empty(int(np.prod(n)), dtype=out_dtype(dtype), device=theta.device)
    xp = _ptrs(Xs)
    _check(glam_rho_forward(len(n), nn, pp, xp, theta.data_ptr(), eta.data_ptr(), int(dtype), workspace.data_ptr(),
                            ws_bytes, _stream_ptr(stream)), "glam_rho_forward")
    return eta


STATIC_SCRATCH_BYTES = 32 << 20


def rho_forward_static(Xs, theta, n, p, dtype, eta, stream=None):
    """eta = H(<X_j>, theta) into the caller's eta, with the library's static device scratch as the
    workspace (no allocation in the call; calls on one GPU must not overlap)."""
    nn, pp = _sizes(n, p)
    xp = _ptrs(Xs)
    _check(glam_rho_forward_static(len(n), nn, pp, xp, theta.data_ptr(), eta.data_ptr(), int(dtype),
                                   _stream_ptr(stream)), "glam_rho_forward_static")
    return eta


def rho_adjoint(Xs, U, n, p, dtype, out=None, workspace=None, stream=None):
    """out = G(<X_j>, U) on the device."""
    torch = _torch()
    nn, pp = _sizes(n, p)
    ws_bytes = rho_workspace_size(n, p, dtype)
    if ws_bytes == 0:
        raise GlamError(GLAM_EINVAL, "rho_adjoint")
    if workspace is None:
        workspace = torch.empty(ws_bytes, dtype=torch.uint8, device=U.device)
    if out is None:
        out = torch.empty(int(np.prod(p)), dtype=out_dtype(dtype), device=U.device)
    xp = _ptrs(Xs)
    _check(glam_rho_adjoint(len(n), nn, pp, xp, U.data_ptr(), out.data_ptr(), int(dtype), workspace.data_ptr(),
                            ws_bytes, _stream_ptr(stream)), "glam_rho_adjoint")
    return out


# ----------------------------------------------------------------------------- Poisson NLL
def nll_workspace_size(n, p, dtype):
    nn, pp = _sizes(n, p)
    return int(glam_nll_workspace_size(nn, pp, int(dtype)))


def poisson_nll_forward(Xs, beta, Y, n, p, dtype, workspace=None, stream=None, out=None):
    torch = _torch()
    nn, pp = _sizes(n, p)
    wsb = nll_workspace_size(n, p, dtype)
    if workspace is None:
        workspace = torch.empty(wsb, dtype=torch.uint8, device=beta.device)
    loss = out if out is not None else torch.empty(1, dtype=torch.float64, device=beta.device)
    xp = (_vp * 3)(*[x.data_ptr() for x in Xs])
    _check(glam_poisson_nll_forward(nn, pp, xp, beta.data_ptr(), Y.data_ptr(), loss.data_ptr(), int(dtype),
                                    workspace.data_ptr(), wsb, _stream_ptr(stream)), "glam_poisson_nll_forward")
    return loss


def poisson_nll_backward(Xs, beta, Y, gscale, n, p, dtype, workspace=None, stream=None, out=None):
    torch = _torch()
    nn, pp = _sizes(n, p)
    wsb = nll_workspace_size(n, p, dtype)
    if workspace is None:
        workspace = torch.empty(wsb, dtype=torch.uint8, device=beta.device)
    grad = out if out is not None else torch.empty(int(np.prod(p)), dtype=out_dtype(dtype), device=beta.device)
    gs = gscale if (gscale.dtype == torch.float64 and gscale.is_contiguous()) else \
        gscale.to(torch.float64).reshape(1).contiguous()
    xp = (_vp * 3)(*[x.data_ptr() for x in Xs])
    _check(glam_poisson_nll_backward(nn, pp, xp, beta.data_ptr(), Y.data_ptr(), gs.data_ptr(), grad.data_ptr(),
                                     int(dtype), workspace.data_ptr(), wsb, _stream_ptr(stream)),
           "glam_poisson_nll_backward")
    return grad


class PackedPoissonNLL:
    """Poisson NLL with X and Y packed once into a workspace of its own: forward(beta) and
    backward(beta, gscale) then run only the beta-dependent work."""

    def __init__(self, Xs, Y, n, p, dtype, stream=None):
        torch = _torch()
        self.n, self.p, self.dtype, self.stream = tuple(n), tuple(p), int(dtype), stream
        nn, pp = _sizes(n, p)
        self.wsb = int(glam_nll_packed_workspace_size(nn, pp, self.dtype))
        if self.wsb == 0:
            raise GlamError(GLAM_EINVAL, "glam_nll_packed_workspace_size")
        self.ws = torch.empty(self.wsb, dtype=torch.uint8, device=Y.device)
        xp = (_vp * 3)(*[x.data_ptr() for x in Xs])
        _check(glam_poisson_nll_pack(nn, pp, xp, Y.data_ptr(), self.dtype, self.ws.data_ptr(), self.wsb,
                                     _stream_ptr(stream)), "glam_poisson_nll_pack")

    def forward(self, beta, out=None):
        """loss (device FP64 1-tensor, written into out when given)."""
        torch = _torch()
        nn, pp = _sizes(self.n, self.p)
        loss = out if out is not None else torch.empty(1, dtype=torch.float64, device=beta.device)
        _check(glam_poisson_nll_forward_packed(nn, pp, beta.data_ptr(), loss.data_ptr(), self.dtype,
                                               self.ws.data_ptr(), self.wsb, _stream_ptr(self.stream)),
               "glam_poisson_nll_forward_packed")
        return loss

    def backward(self, beta, gscale, out=None):
        """gscale * grad L(beta) (written into out when given: FP32 for F32/BF16, FP64 for F64)."""
        torch = _torch()
        nn, pp = _sizes(self.n, self.p)
        grad = out if out is not None else torch.empty(int(np.prod(self.p)), dtype=out_dtype(self.dtype),
                                                        device=beta.device)
        gs = gscale if (gscale.dtype == torch.float64 and gscale.is_contiguous()) else \
            gscale.to(torch.float64).reshape(1).contiguous()
        _check(glam_poisson_nll_backward_packed(nn, pp, beta.data_ptr(), gs.data_ptr(), grad.data_ptr(), self.dtype,
                                                self.ws.data_ptr(), self.wsb, _stream_ptr(self.stream)),
               "glam_poisson_nll_backward_packed")
        return grad


class PoissonNLL:
    """torch.autograd.Function for L(beta) = (1/n) sum(exp(eta) - y eta), eta = H(beta).

    Usage: ``loss = PoissonNLL.apply(beta, Xs, Y, n, p, dtype)``; beta is a 1-D
    column-major device tensor of the chain dtype (its gradient is returned as
    FP32 for F32/BF16 and FP64 for F64, cast to beta's dtype)."""

    _fn = None

    @classmethod
    def apply(cls, beta, Xs, Y, n, p, dtype):
        if cls._fn is None:
            torch = _torch()

            class _F(torch.autograd.Function):
                @staticmethod
                def forward(ctx, b, Xs_, Y_, n_, p_, dt_):
                    ctx.save_for_backward(b)
                    ctx.extra = (Xs_, Y_, n_, p_, dt_)
                    return poisson_nll_forward(Xs_, b.detach().contiguous(), Y_, n_, p_, dt_).reshape(())

                @staticmethod
                def backward(ctx, gout):
                    (b,) = ctx.saved_tensors
                    Xs_, Y_, n_, p_, dt_ = ctx.extra
                    g = poisson_nll_backward(Xs_, b.detach().contiguous(), Y_, gout.reshape(1), n_, p_, dt_)
                    return g.to(b.dtype), None, None, None, None, None

            cls._fn = _F
        return cls._fn.apply(beta, Xs, Y, n, p, dtype)


# ----------------------------------------------------------------------------- lambda path
@dataclass
class PathResult:
    lambdas: np.ndarray
    theta: "object"          # device tensor (nlambda, p) FP64, column-major p-arrays
    kkt: np.ndarray
    objective: np.ndarray
    iters_outer: np.ndarray
    iters_inner: np.ndarray
    status: np.ndarray
    n_done: int
    lambda_max: float
    seconds: float
    code: int
    chain_ms: float = 0.0
    chain_samples: int = 0
    iter_ms: float = 0.0
    inner_total: int = 0
    escalated_at: int = -1   # first model fitted on with the FP64 inner chain, or -1
    adj_ms: float = 0.0      # summed sampled launch durations of the adjoint + step kernel
    fwd_ms: float = 0.0      # ... and of the mode-3 forward kernel


def _path_options(lambdas, nlambda, lambda_min_ratio, dtype, kkt_tol, nu, max_outer, max_inner, check_every,
                  theta0, stream, profile_every, graph, inner, alpha, penalty, scad_a, msa_steps, extrapolation,
                  kron_step):
    L = int(nlambda if lambdas is None else len(lambdas))
    opt = GlamOptions()
    lam_arr = None
    if lambdas is not None:
        lam_arr = (ctypes.c_double * L)(*[float(v) for v in lambdas])
        opt.lambda_ = lam_arr
    opt.nlambda = L
    opt.lambda_min_ratio = float(lambda_min_ratio)
    opt.dtype = int(dtype)
    opt.kkt_tol = float(kkt_tol)
    opt.nu = float(nu)
    opt.max_outer = int(max_outer)
    opt.max_inner = int(max_inner)
    opt.check_every = int(check_every)
    opt.theta0 = theta0.data_ptr() if theta0 is not None else None
    opt.stream = _stream_ptr(stream)
    opt.profile_every = int(profile_every)
    opt.graph_mode = 0 if graph else 1
    opt.inner_mode = {"chain": 0, "gram": 1, "kron": 2, "one": 3}[inner]
    opt.alpha = float(alpha)
    opt.penalty = PENALTIES[penalty] if isinstance(penalty, str) else int(penalty)
    opt.scad_a = float(scad_a)
    opt.msa_steps = int(msa_steps)
    opt.extrapolation = {"restarted": 0, "plain": 1}[extrapolation]
    opt.kron_step = {"prop1": 0, "exact": 1}[kron_step]
    return opt, lam_arr, L


def _run_path(fn, where, prob, opt, L, P, device, raise_on_error):
    torch = _torch()
    theta = torch.zeros((L, P), dtype=torch.float64, device=device)
    lam_out = (ctypes.c_double * L)()
    kkt = (ctypes.c_double * L)()
    obj = (ctypes.c_double * L)()
    io = (ctypes.c_int * L)()
    ii = (ctypes.c_int * L)()
    stt = (ctypes.c_int * L)(*([-1] * L))
    res = GlamResult()
    res.theta = theta.data_ptr()
    res.lambda_out, res.kkt, res.objective = lam_out, kkt, obj
    res.iters_outer, res.iters_inner, res.status = io, ii, stt
    code = fn(ctypes.byref(prob), ctypes.byref(opt), ctypes.byref(res))
    if code == GLAM_EINVAL or code == GLAM_ENOMEM or code == GLAM_EDEVICE:
        raise GlamError(code, where)
    out = PathResult(np.array(lam_out[:]), theta, np.array(kkt[:]), np.array(obj[:]), np.array(io[:]),
                     np.array(ii[:]), np.array(stt[:]), int(res.n_done), float(res.lambda_max),
                     float(res.seconds), int(code), float(res.chain_ms), int(res.chain_samples),
                     float(res.iter_ms), int(res.inner_total), int(res.escalated_at), float(res.adj_ms),
                     float(res.fwd_ms))
    if raise_on_error and code != GLAM_OK:
        raise GlamError(code, where)
    return out


def fit_path(Xs, Y, n, p, family="gaussian", obs_w=None, pen_w=None, lambdas=None, nlambda=100,
             lambda_min_ratio=1e-4, dtype=F64, kkt_tol=1e-6, nu=1.0, max_outer=100, max_inner=100000,
             check_every=8, theta0=None, stream=None, raise_on_error=True, profile_every=0,
             graph=True, inner="chain", alpha=0.0, penalty="lasso", scad_a=3.7, msa_steps=3,
             extrapolation="restarted", kron_step="prop1") -> PathResult:
    """GD-PG lambda path on the device.  Xs: FP64 device factors (column-major,
    1-D); Y, obs_w: FP64 device n-arrays; pen_w, theta0: FP64 device p-arrays;
    alpha: elastic-net weight (0 = lasso); penalty="scad": SCAD by msa_steps steps of
    the multi-step adaptive lasso per lambda.  extrapolation: "restarted" (omega_l counted from
    the last gradient restart at a check) or "plain" (omega_l = (l-1)/(l+2) through each inner loop).
    check_every: inner iterations between convergence checks; each check also runs the restart
    test of the extrapolation.  The stall window is 10 or 20 times max(check_every, 10)
    iterations.  (8: the n = (100, 100, 1000) Gaussian BF16 path took 0.938 s against 0.951 s
    at 10, the Poisson n = (64, 64, 365) path 0.994 against 1.004 s.)"""
    fam = FAMILIES[family] if isinstance(family, str) else int(family)
    prob = GlamProblem()
    prob.d = len(n)
    for j in range(len(n)):
        prob.n[j] = int(n[j])
        prob.p[j] = int(p[j])
        prob.X[j] = Xs[j].data_ptr()
    prob.Y = Y.data_ptr()
    prob.obs_w = obs_w.data_ptr() if obs_w is not None else None
    prob.family = fam
    prob.pen_w = pen_w.data_ptr() if pen_w is not None else None
    opt, lam_arr, L = _path_options(lambdas, nlambda, lambda_min_ratio, dtype, kkt_tol, nu, max_outer, max_inner,
                                    check_every, theta0, stream, profile_every, graph, inner, alpha, penalty, scad_a,
                                    msa_steps, extrapolation, kron_step)
    return _run_path(glam_fit_path, "glam_fit_path", prob, opt, L, int(np.prod(p)), Y.device, raise_on_error)


def fit_path_multi(components, Y, n, family="gaussian", obs_w=None, pen_w=None, lambdas=None, nlambda=100,
                   lambda_min_ratio=1e-4, dtype=F64, kkt_tol=1e-6, nu=1.0, max_outer=100, max_inner=100000,
                   check_every=8, theta0=None, stream=None, raise_on_error=True, inner="chain", alpha=0.0,
                   penalty="lasso", scad_a=3.7, msa_steps=3, extrapolation="restarted") -> PathResult:
    """GD-PG lambda path of a c-component model X = [X_1 | ... | X_c] (Sec. 2): components is a
    list of (Xs_r, p_r), Xs_r the d FP64 device factors of component r and p_r its d sizes;
    theta rows hold (vec(Theta_1), ..., vec(Theta_c)).  Other arguments as fit_path."""
    fam = FAMILIES[family] if isinstance(family, str) else int(family)
    d = len(n)
    c = len(components)
    prob = GlamMultiProblem()
    prob.d = d
    for j in range(d):
        prob.n[j] = int(n[j])
    prob.c = c
    p_arr = (ctypes.c_int64 * (3 * c))()
    x_arr = (_vp * (3 * c))()
    P = 0
    for r, (Xs_r, p_r) in enumerate(components):
        if len(Xs_r) != d or len(p_r) != d:
            raise ValueError("every component needs d factors and d sizes")
        for j in range(d):
            p_arr[3 * r + j] = int(p_r[j])
            x_arr[3 * r + j] = Xs_r[j].data_ptr()
        P += int(np.prod(p_r))
    prob.p = p_arr
    prob.X = x_arr
    prob.Y = Y.data_ptr()
    prob.obs_w = obs_w.data_ptr() if obs_w is not None else None
    prob.family = fam
    prob.pen_w = pen_w.data_ptr() if pen_w is not None else None
    opt, lam_arr, L = _path_options(lambdas, nlambda, lambda_min_ratio, dtype, kkt_tol, nu, max_outer, max_inner,
                                    check_every, theta0, stream, 0, True, inner, alpha, penalty, scad_a, msa_steps,
                                    extrapolation, "prop1")
    return _run_path(glam_fit_path_multi, "glam_fit_path_multi", prob, opt, L, P, Y.device, raise_on_error)


# ----------------------------------------------------------------------------- batched fits
@dataclass
class BatchResult:
    theta: list              # device FP64 tensors, one p_i-array per problem
    lambdas: np.ndarray
    lambda_max: np.ndarray
    kkt: np.ndarray
    objective: np.ndarray
    iters_outer: np.ndarray
    status: np.ndarray
    steps: int
    problem_steps: int
    seconds: float
    code: int
    graph_replays: int = 0
    tune_seconds: float = 0.0


def fit_batched(problems, lambdas=None, lambda_ratio=0.1, dtype=F32, kkt_tol=1e-6, max_outer=100,
                max_inner=100000, check_every=10, stream=None, raise_on_error=True, alpha=0.0, tuning="auto",
                graph=True) -> BatchResult:
    """Fit many independent problems (one lambda each) with three batched launches per
    batched proximal step.  problems: list of dicts with keys X (3 FP64 device
    factors), Y (FP64 device n-array), n, p, family, and optional obs_w, pen_w.  tuning: "auto"
    (the slab-phase variants timed once per shape class) or "fixed"; graph: replay each block of
    check_every steps as a captured HIP graph."""
    torch = _torch()
    nprob = len(problems)
    arr = (GlamProblem * nprob)()
    for i, pr in enumerate(problems):
        P = arr[i]
        P.d = len(pr["n"])
        for j in range(len(pr["n"])):
            P.n[j] = int(pr["n"][j])
            P.p[j] = int(pr["p"][j])
            P.X[j] = pr["X"][j].data_ptr()
        P.Y = pr["Y"].data_ptr()
        P.obs_w = pr["obs_w"].data_ptr() if pr.get("obs_w") is not None else None
        fam = pr.get("family", "gaussian")
        P.family = FAMILIES[fam] if isinstance(fam, str) else int(fam)
        P.pen_w = pr["pen_w"].data_ptr() if pr.get("pen_w") is not None else None
    opt = GlamBatchOptions()
    lam_arr = None
    if lambdas is not None:
        lam_arr = (ctypes.c_double * nprob)(*[float(v) for v in lambdas])
        opt.lambda_ = lam_arr
    opt.lambda_ratio = float(lambda_ratio)
    opt.dtype = int(dtype)
    opt.kkt_tol = float(kkt_tol)
    opt.max_outer, opt.max_inner, opt.check_every = int(max_outer), int(max_inner), int(check_every)
    opt.stream = _stream_ptr(stream)
    opt.alpha = float(alpha)
    opt.tuning = {"auto": 0, "fixed": 1}[tuning]
    opt.graph_mode = 0 if graph else 1
    dev = problems[0]["Y"].device
    thetas = [torch.zeros(int(np.prod(pr["p"])), dtype=torch.float64, device=dev) for pr in problems]
    tp = (_vp * nprob)(*[t.data_ptr() for t in thetas])
    outs = [(ctypes.c_double * nprob)() for _ in range(5)]
    io = (ctypes.c_int * nprob)()
    st = (ctypes.c_int * nprob)(*([-1] * nprob))
    res = GlamBatchResult()
    res.theta = tp
    res.lambda_out, res.lambda_max, res.kkt, res.objective = outs[0], outs[1], outs[2], outs[3]
    res.iters_outer, res.status = io, st
    code = glam_fit_batched(arr, nprob, ctypes.byref(opt), ctypes.byref(res))
    if code in (GLAM_EINVAL, GLAM_ENOMEM, GLAM_EDEVICE):
        raise GlamError(code, "glam_fit_batched")
    out = BatchResult(thetas, np.array(outs[0][:]), np.array(outs[1][:]), np.array(outs[2][:]),
                      np.array(outs[3][:]), np.array(io[:]), np.array(st[:]), int(res.steps),
                      int(res.problem_steps), float(res.seconds), int(code), int(res.graph_replays),
                      float(res.tune_seconds))
    if raise_on_error and code != GLAM_OK:
        raise GlamError(code, "glam_fit_batched")
    return out
