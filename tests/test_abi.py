"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and rejects invalid arguments before touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "glam.h")
LIB = os.path.join(ROOT, "paper_1510_03298_amd", "libglam.so")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"\b(glam_[a-z0-9_]+)\s*\(", txt)
    return sorted(set(names))


def lib():
    if not os.path.exists(LIB):
        pytest.fail("libglam.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["glam_fit_path", "glam_rho_forward", "glam_rho_adjoint", "glam_rho_workspace_size",
                     "glam_poisson_nll_forward", "glam_poisson_nll_backward", "glam_status_string",
                     "glam_last_error"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    L = lib()
    for name in declared_functions():
        assert hasattr(L, name), f"{name} declared in glam.h but not exported"


def test_binding_exports_match_header():
    from paper_1510_03298_amd import glam
    assert sorted(glam.EXPORTED) == declared_functions()


def test_status_strings_and_version():
    from paper_1510_03298_amd import glam
    assert glam.glam_status_string(0) == b"ok"
    assert b"invalid" in glam.glam_status_string(1)
    assert b"gfx950" in glam.glam_version()


def _sizes(n, p):
    return (ctypes.c_int64 * 3)(*n), (ctypes.c_int64 * 3)(*p)


def test_workspace_size_and_limits():
    from paper_1510_03298_amd import glam
    n, p = _sizes((100, 100, 1000), (30, 30, 200))
    w32 = glam.glam_rho_workspace_size(3, n, p, glam.F32)
    w64 = glam.glam_rho_workspace_size(3, n, p, glam.F64)
    assert w32 >= 1000 * 900 * 4 * 2 and w64 > w32
    assert glam.glam_rho_workspace_size(4, n, p, glam.F64) == 0          # d must be 2 or 3
    assert glam.glam_rho_workspace_size(1, n, p, glam.F64) == 0
    # d = 2: (n1, n2) = (100, 1000) runs as (100, 1, 1000); mode 2 is the unrestricted slab mode
    assert glam.glam_rho_workspace_size(2, n, p, glam.F64) > 0
    n2, p2 = _sizes((100, 5000, 0), (30, 400, 0))
    assert glam.glam_rho_workspace_size(2, n2, p2, glam.F32) > 0
    # n_1 beyond the inner-mode limit: the transform runs in another mode order (mode 1 last),
    # with room for the permuted input and output in the workspace
    n2, p2 = _sizes((300, 50, 0), (30, 20, 0))
    w_re = glam.glam_rho_workspace_size(2, n2, p2, glam.F32)
    assert w_re >= 300 * 50 * 8
    # only one mode with p <= 32: no order fits the slab kernels, the generic GEMM chain runs;
    # its workspace holds X_j^T and two intermediates of the largest partial product
    n, p = _sizes((100, 100, 1000), (33, 30, 200))
    tmp = max(30 * 200 * 100, 200 * 100 * 100, 100 * 1000 * 33, 1000 * 33 * 30)
    w_gen = glam.glam_rho_workspace_size(3, n, p, glam.F32)
    assert w_gen >= 2 * tmp * 4 + (100 * 33 + 100 * 30 + 1000 * 200) * 4
    n, p = _sizes((0, 100, 1000), (3, 3, 3))
    assert glam.glam_rho_workspace_size(3, n, p, glam.F32) == 0          # empty mode
    n, p = _sizes((256, 256, 10), (32, 32, 3))
    assert glam.glam_rho_workspace_size(3, n, p, glam.F32) > 0
    # FP64 copies of X1, X2 exceed the LDS budget in this order; (256, 10, 256) fits
    assert glam.glam_rho_workspace_size(3, n, p, glam.F64) > glam.glam_rho_workspace_size(3, n, p, glam.F32)
    n, p = _sizes((256, 256, 256), (32, 32, 32))
    # no order fits the FP64 LDS budget: the generic chain (FP32 still takes the slab kernels)
    w_gen = glam.glam_rho_workspace_size(3, n, p, glam.F64)
    assert w_gen >= 2 * (256 * 256 * 32) * 8


def test_invalid_arguments_rejected_without_device_work():
    from paper_1510_03298_amd import glam
    n, p = _sizes((10, 10, 10), (4, 4, 4))
    X = (ctypes.c_void_p * 3)(None, None, None)
    rc = glam.glam_rho_forward(3, n, p, X, None, None, glam.F64, None, 0, None)
    assert rc == glam.GLAM_EINVAL and b"NULL" in glam.glam_last_error()
    rc = glam.glam_rho_adjoint(4, n, p, X, None, None, glam.F64, None, 0, None)
    assert rc == glam.GLAM_EINVAL
    rc = glam.glam_rho_forward(3, n, p, X, None, None, 7, None, 0, None)
    assert rc == glam.GLAM_EINVAL
    assert glam.glam_fit_path(None, None, None) == glam.GLAM_EINVAL
    prob = glam.GlamProblem()
    prob.d = 3
    for j in range(3):
        prob.n[j], prob.p[j] = 10, 4
    opt = glam.GlamOptions()
    res = glam.GlamResult()
    rc = glam.glam_fit_path(ctypes.byref(prob), ctypes.byref(opt), ctypes.byref(res))
    assert rc == glam.GLAM_EINVAL       # NULL factors
    # a non-decreasing lambda sequence is rejected before any device work
    dummy = ctypes.c_double(0.0)
    for j in range(3):
        prob.X[j] = ctypes.addressof(dummy)
    prob.Y = ctypes.addressof(dummy)
    lam = (ctypes.c_double * 3)(1.0, 2.0, 0.5)
    opt.lambda_ = lam
    opt.nlambda = 3
    opt.kkt_tol, opt.nu, opt.max_outer, opt.max_inner, opt.check_every = 1e-6, 1.0, 10, 10, 1
    out = (ctypes.c_double * 3)()
    io = (ctypes.c_int * 3)()
    res.theta = ctypes.addressof(dummy)
    res.lambda_out = res.kkt = res.objective = out
    res.iters_outer = res.iters_inner = res.status = io
    rc = glam.glam_fit_path(ctypes.byref(prob), ctypes.byref(opt), ctypes.byref(res))
    assert rc == glam.GLAM_EINVAL and b"decreasing" in glam.glam_last_error()
    lam2 = (ctypes.c_double * 3)(3.0, 2.0, 1.0)
    opt.lambda_ = lam2
    for bad_nu in (-0.5, 1.5, float("nan")):   # nu in [0, 1] (Sec. 6.4; 0: delta = 1 with backtracking)
        opt.nu = bad_nu
        assert glam.glam_fit_path(ctypes.byref(prob), ctypes.byref(opt), ctypes.byref(res)) == glam.GLAM_EINVAL
        assert b"nu" in glam.glam_last_error()
    opt.nu = 1.0
    for field, value in (("extrapolation", 2), ("kron_step", 2)):
        setattr(opt, field, value)
        assert glam.glam_fit_path(ctypes.byref(prob), ctypes.byref(opt), ctypes.byref(res)) == glam.GLAM_EINVAL
        setattr(opt, field, 0)
    opt.penalty, opt.alpha = 2, 0.5   # ridge takes no elastic-net weight
    assert glam.glam_fit_path(ctypes.byref(prob), ctypes.byref(opt), ctypes.byref(res)) == glam.GLAM_EINVAL
    assert b"ridge" in glam.glam_last_error()
    opt.penalty, opt.alpha = 0, 0.0
    prob.family = 4   # families are 0..3
    rc = glam.glam_fit_path(ctypes.byref(prob), ctypes.byref(opt), ctypes.byref(res))
    assert rc == glam.GLAM_EINVAL and b"family" in glam.glam_last_error()
    prob.family = glam.GAMMA
    for field, value in (("penalty", 3), ("msa_steps", 0), ("scad_a", 1.5)):   # SCAD options checked on the host
        opt.penalty, opt.msa_steps, opt.scad_a = 1, 3, 0.0
        setattr(opt, field, value)
        assert glam.glam_fit_path(ctypes.byref(prob), ctypes.byref(opt), ctypes.byref(res)) == glam.GLAM_EINVAL
    opt.penalty, opt.scad_a, opt.alpha = 1, 0.0, 0.5
    assert glam.glam_fit_path(ctypes.byref(prob), ctypes.byref(opt), ctypes.byref(res)) == glam.GLAM_EINVAL
    assert b"SCAD" in glam.glam_last_error()
    opt.penalty = 0
    for bad in (-0.5, float("nan"), float("inf")):   # elastic-net weight must be finite and >= 0
        opt.alpha = bad
        rc = glam.glam_fit_path(ctypes.byref(prob), ctypes.byref(opt), ctypes.byref(res))
        assert rc == glam.GLAM_EINVAL and b"alpha" in glam.glam_last_error()


def test_no_mode_order_fits_refuses_the_gram_forms_on_the_host():
    """When no order of the three modes puts two of them within the slab kernels' limits
    (p <= 32), the fit runs on the generic GEMM solver, which has no Gram inner forms: those
    are refused before any device work."""
    from paper_1510_03298_amd import glam
    prob = glam.GlamProblem()
    prob.d = 3
    dummy = ctypes.c_double(0.0)
    for j in range(3):
        prob.n[j], prob.p[j] = 50, 40
        prob.X[j] = ctypes.addressof(dummy)
    prob.Y = ctypes.addressof(dummy)
    opt = glam.GlamOptions()
    opt.nlambda, opt.lambda_min_ratio, opt.dtype = 2, 0.1, glam.F64
    opt.kkt_tol, opt.nu, opt.max_outer, opt.max_inner, opt.check_every = 1e-6, 1.0, 10, 10, 1
    res = glam.GlamResult()
    out = (ctypes.c_double * 2)()
    io = (ctypes.c_int * 2)()
    res.theta = ctypes.addressof(dummy)
    res.lambda_out = res.kkt = res.objective = out
    res.iters_outer = res.iters_inner = res.status = io
    opt.inner_mode = 1   # Gram form
    rc = glam.glam_fit_path(ctypes.byref(prob), ctypes.byref(opt), ctypes.byref(res))
    assert rc == glam.GLAM_EINVAL and b"order of the modes" in glam.glam_last_error()


def test_multi_component_entry_point_refuses_bad_arguments_on_the_host():
    """glam_fit_path_multi: sizes, pointers and options are checked before any device work."""
    from paper_1510_03298_amd import glam
    dummy = ctypes.c_double(0.0)
    ptr = ctypes.addressof(dummy)
    opt = glam.GlamOptions()
    opt.nlambda, opt.lambda_min_ratio, opt.dtype = 2, 0.1, glam.F64
    opt.kkt_tol, opt.nu, opt.max_outer, opt.max_inner, opt.check_every = 1e-6, 1.0, 10, 10, 1
    res = glam.GlamResult()
    out = (ctypes.c_double * 2)()
    io = (ctypes.c_int * 2)()
    res.theta = ptr
    res.lambda_out = res.kkt = res.objective = out
    res.iters_outer = res.iters_inner = res.status = io
    pa = (ctypes.c_int64 * 6)(3, 4, 2, 2, 2, 5)
    xa = (ctypes.c_void_p * 6)(*([ptr] * 6))

    def prob(c=2, d=3, p=pa, X=xa, family=0, Y=ptr):
        pr = glam.GlamMultiProblem()
        pr.d, pr.c, pr.family, pr.Y = d, c, family, Y
        for j in range(3):
            pr.n[j] = 10
        pr.p, pr.X = p, X
        return pr

    def call(pr, o=opt):
        return glam.glam_fit_path_multi(ctypes.byref(pr), ctypes.byref(o), ctypes.byref(res))

    assert glam.glam_fit_path_multi(None, None, None) == glam.GLAM_EINVAL
    assert call(prob(c=0)) == glam.GLAM_EINVAL and b"c must be" in glam.glam_last_error()
    assert call(prob(d=4)) == glam.GLAM_EINVAL
    assert call(prob(p=None)) == glam.GLAM_EINVAL and b"NULL" in glam.glam_last_error()
    assert call(prob(Y=None)) == glam.GLAM_EINVAL
    assert call(prob(family=9)) == glam.GLAM_EINVAL and b"family" in glam.glam_last_error()
    bad_p = (ctypes.c_int64 * 6)(3, 0, 2, 2, 2, 5)
    assert call(prob(p=bad_p)) == glam.GLAM_EINVAL and b"sizes" in glam.glam_last_error()
    bad_x = (ctypes.c_void_p * 6)(ptr, ptr, ptr, ptr, None, ptr)
    assert call(prob(X=bad_x)) == glam.GLAM_EINVAL and b"NULL factor" in glam.glam_last_error()
    gram = glam.GlamOptions.from_buffer_copy(opt)
    gram.inner_mode = 1
    assert call(prob(), gram) == glam.GLAM_EINVAL and b"rho-chain" in glam.glam_last_error()
    neg = glam.GlamOptions.from_buffer_copy(opt)
    neg.nu = 1.5
    assert call(prob(), neg) == glam.GLAM_EINVAL and b"nu" in glam.glam_last_error()


def test_packed_nll_workspace_and_argument_checks():
    """The packed NLL entry points: workspace size (the rho workspace plus the counts) and the
    host-side refusals that come before any device work."""
    from paper_1510_03298_amd import glam
    n, p = _sizes((128, 128, 256), (32, 32, 64))
    w = glam.glam_nll_workspace_size(n, p, glam.BF16)
    wp = glam.glam_nll_packed_workspace_size(n, p, glam.BF16)
    assert wp >= w + 128 * 128 * 256 * 4          # tiled FP32 counts
    wp64 = glam.glam_nll_packed_workspace_size(n, p, glam.F64)
    assert wp64 >= glam.glam_nll_workspace_size(n, p, glam.F64) + 128 * 128 * 256 * 8   # FP64 copy
    re_n, re_p = _sizes((128, 128, 256), (40, 32, 16))   # p_1 > 32: another mode order, plus the permuted arrays
    assert glam.glam_nll_packed_workspace_size(re_n, re_p, glam.BF16) > glam.glam_nll_workspace_size(re_n, re_p, glam.BF16) > 0
    bad_n, bad_p = _sizes((128, 128, 256), (40, 40, 64))  # no order fits
    assert glam.glam_nll_packed_workspace_size(bad_n, bad_p, glam.BF16) == 0
    assert glam.glam_nll_workspace_size(bad_n, bad_p, glam.BF16) == 0
    X = (ctypes.c_void_p * 3)(None, None, None)
    assert glam.glam_poisson_nll_pack(n, p, X, None, glam.BF16, None, 0, None) == glam.GLAM_EINVAL
    assert b"NULL" in glam.glam_last_error()
    dummy = ctypes.c_double(0.0)
    ptr = ctypes.addressof(dummy)
    rc = glam.glam_poisson_nll_forward_packed(n, p, ptr, ptr, glam.BF16, ptr, wp - 1, None)
    assert rc == glam.GLAM_EINVAL and b"workspace" in glam.glam_last_error()
    rc = glam.glam_poisson_nll_backward_packed(n, p, ptr, ptr, None, glam.BF16, ptr, wp, None)
    assert rc == glam.GLAM_EINVAL and b"NULL" in glam.glam_last_error()


def test_static_forward_refuses_oversize_and_bad_arguments_on_the_host():
    """glam_rho_forward_static checks sizes against its static scratch before any device call."""
    from paper_1510_03298_amd import glam
    n, p = _sizes((600, 100, 100), (40, 30, 30))     # reordered (mode 1 last): a 48 MB region for eta
    assert glam.glam_rho_workspace_size(3, n, p, glam.F64) > glam.STATIC_SCRATCH_BYTES
    X = (ctypes.c_void_p * 3)(None, None, None)
    rc = glam.glam_rho_forward_static(3, n, p, X, None, None, glam.F64, None)
    assert rc == glam.GLAM_EINVAL and b"static scratch" in glam.glam_last_error()
    ok_n, ok_p = _sizes((100, 100, 1000), (30, 30, 200))
    for dt in (glam.F64, glam.F32, glam.BF16):   # the headline sizes fit in every dtype
        assert 0 < glam.glam_rho_workspace_size(3, ok_n, ok_p, dt) <= glam.STATIC_SCRATCH_BYTES
    assert glam.glam_rho_forward_static(3, ok_n, ok_p, X, None, None, 7, None) == glam.GLAM_EINVAL
    assert glam.glam_rho_forward_static(4, ok_n, ok_p, X, None, None, glam.F32, None) == glam.GLAM_EINVAL
