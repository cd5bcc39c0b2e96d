"""Poisson NLL forward/backward (torch.autograd.Function over the fused adjoint
kernel) against the oracle and central finite differences."""
import numpy as np
import pytest

import oracle.glam_oracle as O
from paper_1510_03298_amd import inputs
from tests.gpu_util import need_gpu, rel_inf

pytestmark = pytest.mark.gpu

TOL = {0: 1e-10, 1: 1e-5, 2: 3e-2}


def _check(glam, d, beta, loss, grad, dt):
    """Value: relative to sum |exp(eta) - y eta| / n.  Gradient: entrywise, relative
    to G(|X|, |exp(eta) - y|) / n, the sum of magnitudes of the terms (the
    gradient itself cancels, so the rounding bound scales with these sums)."""
    eta = O.H(d.X, beta)
    Lref = O.poisson_nll(d.X, beta, d.Y)
    Lscale = float(np.sum(np.abs(np.exp(eta) - d.Y * eta))) / d.Y.size
    assert abs(loss - Lref) <= TOL[dt] * Lscale, (loss, Lref)
    gref = O.poisson_nll_grad(d.X, beta, d.Y)
    gabs = O.G([np.abs(X) for X in d.X], np.abs(np.exp(eta) - d.Y)) / d.Y.size
    g = glam.from_colmajor(grad.float() if dt else grad, d.p)
    err = float(np.max(np.abs(g - gref) / gabs))
    assert err <= TOL[dt], err


@pytest.mark.parametrize("dt", [0, 1, 2])
@pytest.mark.parametrize("n,p", [((21, 18, 30), (7, 6, 9)), ((40, 33, 17), (20, 17, 5)),
                                 ((60, 18, 30), (40, 6, 9)),      # p_1 > 32: runs in another mode order
                                 ((150, 20, 30), (10, 40, 6))])   # p_2 > 32: reordered, LDS slab kernel
def test_nll_value_and_gradient(n, p, dt):
    torch, glam = need_gpu()
    print(f"nll n={n} p={p} dt={dt}", flush=True)
    d = inputs.random_problem(n, p, family="poisson", seed=31, scale=0.3)
    beta = np.random.default_rng(5).normal(0.0, 0.2, p)
    Xd = [glam.to_device_colmajor(X, dt) for X in d.X]
    Yd = glam.to_device_colmajor(d.Y, 0)
    b = glam.to_device_colmajor(beta, dt).requires_grad_(True)
    loss = glam.PoissonNLL.apply(b, Xd, Yd, n, p, dt)
    loss.backward()
    torch.cuda.synchronize()
    Lref = O.poisson_nll(d.X, beta, d.Y)
    _check(glam, d, beta, float(loss.detach()), b.grad, dt)


def test_nll_gradient_central_differences_f64():
    """Gradient of the device loss vs central differences of the device loss (h = 1e-6)."""
    torch, glam = need_gpu()
    n, p = (16, 12, 10), (5, 4, 3)
    d = inputs.random_problem(n, p, family="poisson", seed=32, scale=0.3, basis="gauss")
    beta = np.random.default_rng(6).normal(0.0, 0.2, p)
    Xd = [glam.to_device_colmajor(X, 0) for X in d.X]
    Yd = glam.to_device_colmajor(d.Y, 0)
    b = glam.to_device_colmajor(beta, 0).requires_grad_(True)
    glam.PoissonNLL.apply(b, Xd, Yd, n, p, 0).backward()
    g = b.grad.cpu().numpy()
    rng = np.random.default_rng(7)
    h = 1e-6
    for _ in range(16):
        v = rng.standard_normal(b.numel())
        v /= np.linalg.norm(v)
        vd = torch.from_numpy(v).cuda()
        with torch.no_grad():
            lp = float(glam.poisson_nll_forward(Xd, b + h * vd, Yd, n, p, 0))
            lm = float(glam.poisson_nll_forward(Xd, b - h * vd, Yd, n, p, 0))
        fd = (lp - lm) / (2 * h)
        assert abs(fd - float(g @ v)) <= 1e-7 * max(1.0, abs(fd))


@pytest.mark.parametrize("dt", [1, 2])
def test_nll_full_size_workload(dt):
    """n=(128,128,256), p=(32,32,64): value and gradient vs the FP64 oracle, the gradient both
    entrywise on the scale of its terms and as the relative sup norm ||g - g_ref|| / ||g_ref||
    (BF16 3e-2, FP32 1e-5), with an upstream gradient other than 1 (loss scaled by -1.75)."""
    torch, glam = need_gpu()
    d = inputs.config_c5()
    n, p = d.n, d.p
    beta = d.extra["beta"]
    Xd = [glam.to_device_colmajor(X, dt) for X in d.X]
    Yd = glam.to_device_colmajor(d.Y, 0)
    b = glam.to_device_colmajor(beta, dt).requires_grad_(True)
    c = -1.75
    loss = glam.PoissonNLL.apply(b, Xd, Yd, n, p, dt)
    (c * loss).backward()
    torch.cuda.synchronize()
    g = glam.from_colmajor(b.grad.double(), p) / c
    _check(glam, d, beta, float(loss.detach()), torch.from_numpy(O.vec(g)).to(b.grad.device), dt)
    gref = O.poisson_nll_grad(d.X, beta, d.Y)
    err = rel_inf(g, gref)
    print(f"NLL gradient dt={dt}: relative sup-norm error {err:.3e} against the exact inputs", flush=True)
    if dt == 1:
        assert err <= TOL[dt], err
    else:
        # BF16 (R10): the inputs themselves carry 8-bit mantissas.  At this evaluation point, 0.05 from
        # the optimum, the gradient is small next to its terms, and rounding beta and X to BF16 alone
        # moves the exact FP64 gradient by 6% in this norm.  The bar is therefore taken against the
        # oracle fed the same RNE-rounded inputs (the tight BF16 form), and the distance to the
        # unrounded inputs' gradient is only bounded by that input effect plus the bar.
        Xr = [O.round_to_bf16(X) for X in d.X]
        br = O.round_to_bf16(beta)
        g_in = O.poisson_nll_grad(Xr, br, d.Y)
        err_r = rel_inf(g, g_in)
        in_eff = rel_inf(g_in, gref)
        print(f"NLL gradient BF16: {err_r:.3e} against the oracle on the rounded inputs (bar {TOL[dt]:.0e}); "
              f"input rounding alone moves the gradient by {in_eff:.3e}", flush=True)
        assert err_r <= TOL[dt], err_r
        assert err <= in_eff + TOL[dt], (err, in_eff)


_FD = {}


def _oracle_fd_probes(rounded_inputs=False):
    """Central differences (h = 1e-6) of the oracle's FP64 loss at the n=(128,128,256) evaluation point,
    along 16 random unit directions and 16 random coordinates; and the same probes of the oracle's
    analytic gradient (whose difference to the FD values is the FD's own error at this size).
    rounded_inputs: the loss of the BF16-rounded (RNE) factors and beta, the values a BF16 chain
    is given (R10)."""
    key = bool(rounded_inputs)
    if key not in _FD:
        d = inputs.config_c5()
        beta = d.extra["beta"]
        if rounded_inputs:
            d.X = [O.round_to_bf16(X) for X in d.X]
            beta = O.round_to_bf16(beta)
        rng = np.random.default_rng(11)
        P = int(np.prod(d.p))
        dirs = [v / np.linalg.norm(v) for v in (rng.standard_normal(P) for _ in range(16))]
        for m in rng.choice(P, size=16, replace=False):
            e = np.zeros(P)
            e[m] = 1.0
            dirs.append(e)
        h = 1e-6
        fd = []
        for v in dirs:
            V = O.unvec(v, d.p)
            fd.append((O.poisson_nll(d.X, beta + h * V, d.Y) - O.poisson_nll(d.X, beta - h * V, d.Y)) / (2 * h))
        ga = O.vec(O.poisson_nll_grad(d.X, beta, d.Y))
        _FD[key] = dict(d=d, dirs=np.array(dirs), fd=np.array(fd), analytic=np.array([ga @ v for v in dirs]))
    return _FD[key]


@pytest.mark.parametrize("dt", [2, 1])
def test_nll_gradient_vs_central_differences_full_size(dt):
    """The device gradient (BF16 or FP32 chain) against central differences of the oracle's FP64 loss
    (h = 1e-6) along 16 random unit directions and 16 random coordinates, at the full size.  The
    error is taken relative to the largest probe (sup norm over the 32 probes).  At this size the
    loss (about 3) moves by about 1e-12 over +-h, a few thousand ulps, so the differences themselves
    resolve the derivative to about 1e-3 of that scale: the bar is the dtype's tolerance (BF16 3e-2)
    or four times the differences' own measured error (the FP32 1e-5 bar is then the oracle-gradient
    comparison of test_nll_full_size_workload).  The BF16 chain is compared with the differences of
    the loss at its own BF16-rounded inputs (R10; rounding the inputs alone moves this gradient by
    6% in this norm, see test_nll_full_size_workload)."""
    torch, glam = need_gpu()
    F = _oracle_fd_probes(rounded_inputs=(dt == 2))
    d = F["d"]
    Xd = [glam.to_device_colmajor(X, dt) for X in d.X]
    Yd = glam.to_device_colmajor(d.Y, 0)
    b = glam.to_device_colmajor(d.extra["beta"], dt).requires_grad_(True)
    glam.PoissonNLL.apply(b, Xd, Yd, d.n, d.p, dt).backward()
    torch.cuda.synchronize()
    g = b.grad.double().cpu().numpy()
    probes = F["dirs"] @ g
    scale = float(np.max(np.abs(F["fd"])))
    fd_err = float(np.max(np.abs(F["analytic"] - F["fd"]))) / scale
    err = float(np.max(np.abs(probes - F["fd"]))) / scale
    bar = max(TOL[dt], 4.0 * fd_err)
    print(f"NLL central differences dt={dt}: error {err:.3e}, the differences' own error {fd_err:.3e}, "
          f"bar {bar:.3e}", flush=True)
    assert fd_err <= 1e-2   # the probes resolve the derivative (BF16's bar is 3x above this)
    assert err <= bar, (err, bar)


@pytest.mark.parametrize("dt", [0, 1, 2])
@pytest.mark.parametrize("n,p", [((21, 18, 30), (7, 6, 9)), ((40, 33, 17), (20, 17, 5)),
                                 ((150, 20, 12), (10, 8, 5)),    # n_1 > 128: the LDS kernel, FP64 counts
                                 ((60, 18, 30), (40, 6, 9))])    # reordered: beta, Y and the gradient permuted
def test_nll_packed_matches_unpacked(n, p, dt):
    """X and Y packed once: loss and gradient at two successive betas bit for bit those of the
    one-shot entry points (integer counts), and within the oracle's bound."""
    torch, glam = need_gpu()
    print(f"nll packed n={n} p={p} dt={dt}", flush=True)
    d = inputs.random_problem(n, p, family="poisson", seed=33, scale=0.3)
    Xd = [glam.to_device_colmajor(X, dt) for X in d.X]
    Yd = glam.to_device_colmajor(d.Y, 0)
    one = torch.ones(1, dtype=torch.float64, device=Yd.device)
    packed = glam.PackedPoissonNLL(Xd, Yd, n, p, dt)
    for k in range(2):
        beta = np.random.default_rng(50 + k).normal(0.0, 0.2, p)
        b = glam.to_device_colmajor(beta, dt)
        l1 = packed.forward(b)
        g1 = packed.backward(b, one)
        l0 = glam.poisson_nll_forward(Xd, b, Yd, n, p, dt)
        g0 = glam.poisson_nll_backward(Xd, b, Yd, one, n, p, dt)
        torch.cuda.synchronize()
        assert float(l1) == float(l0)
        assert torch.equal(g1, g0)
        _check(glam, d, beta, float(l1), g1, dt)


def test_nll_packed_full_size_workload():
    """n=(128,128,256), p=(32,32,64), BF16: the packed calls bit for bit the one-shot calls."""
    torch, glam = need_gpu()
    d = inputs.config_c5()
    dt = 2
    Xd = [glam.to_device_colmajor(X, dt) for X in d.X]
    Yd = glam.to_device_colmajor(d.Y, 0)
    b = glam.to_device_colmajor(d.extra["beta"], dt)
    one = torch.ones(1, dtype=torch.float64, device=Yd.device)
    packed = glam.PackedPoissonNLL(Xd, Yd, d.n, d.p, dt)
    l1, g1 = packed.forward(b), packed.backward(b, one)
    l0 = glam.poisson_nll_forward(Xd, b, Yd, d.n, d.p, dt)
    g0 = glam.poisson_nll_backward(Xd, b, Yd, one, d.n, d.p, dt)
    torch.cuda.synchronize()
    assert float(l1) == float(l0)
    assert torch.equal(g1, g0)
