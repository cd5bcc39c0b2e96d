"""Parity of the HIP rho chain (glam_rho_forward / glam_rho_adjoint) with the oracle.

Tolerances (relative sup norm): FP64 1e-10, FP32 1e-5, BF16 3e-2 against the
exact FP64 transform of the unrounded inputs, and 1e-2 against the exact
transform of the BF16-rounded inputs (intermediates are rounded to BF16 on the
way, so only the first comparison is the stated bar).
"""
import numpy as np
import pytest

import oracle.glam_oracle as O
from tests.gpu_util import need_gpu, rel_inf, rounded

pytestmark = pytest.mark.gpu

TOL = {0: 1e-10, 1: 1e-5, 2: 3e-2}

SHAPES = [
    ((20, 20, 20), (8, 8, 8)),          # small config: one tile per mode
    ((37, 21, 45), (13, 7, 19)),        # ragged tails everywhere
    ((100, 77, 33), (30, 29, 5)),       # two p-tiles, N1T > 4 (chunk loop)
    ((70, 20, 30), (20, 10, 9)),        # N1T = 5: a group of 4 tiles, then one left over
    ((90, 33, 25), (17, 30, 6)),        # N1T = 6: a group of 4 tiles, then two left over
    ((100, 90, 1000), (30, 28, 7)),     # FP64: one slab per wave (1000 slabs of 6 column blocks)
    ((16, 16, 16), (16, 16, 16)),       # exact tiles
    ((1, 1, 1), (1, 1, 1)),             # degenerate
    ((5, 3, 200), (1, 2, 70)),          # tiny inner modes, long slab mode
    ((128, 128, 8), (32, 32, 4)),       # largest inner p
    ((64, 64, 37), (24, 24, 12)),       # Poisson workload's inner modes
    ((40, 30, 700), (25, 30, 50)),      # FP64 forward with 64 x 64 tiles (132 of them), ragged
]


# modes 1-2 of the caller's order beyond the slab kernels: run in another order, permuted in and out
SHAPES_REORDERED = [
    ((300, 20, 24), (10, 8, 6)),        # n_1 > 256
    ((120, 40, 20), (60, 20, 10)),      # p_1 > 32 (Sec. 6.5's design in the paper's mode order)
    ((17, 200, 250), (5, 40, 7)),       # p_2 > 32, ragged: mode 2 runs last
]


# d = 2 models (run as X_2 (x) [1] (x) X_1)
SHAPES_2D = [
    ((37, 53), (9, 13)),
    ((100, 700), (30, 150)),            # long second mode (the slab mode)
    ((256, 40), (32, 7)),               # largest first mode
    ((1, 1), (1, 1)),
    ((300, 50), (30, 20)),              # n_1 > 256: mode 1 runs last
]


def _factors(n, p, seed):
    rng = np.random.default_rng(seed)
    return [rng.standard_normal((nj, pj)) for nj, pj in zip(n, p)]


@pytest.mark.parametrize("dt", [0, 1, 2])
@pytest.mark.parametrize("n,p", SHAPES + SHAPES_2D + SHAPES_REORDERED)
def test_forward_parity(n, p, dt):
    torch, glam = need_gpu()
    print(f"forward n={n} p={p} dt={dt}", flush=True)
    Xs = _factors(n, p, 1)
    Th = np.random.default_rng(2).standard_normal(p)
    Xd = [glam.to_device_colmajor(X, dt) for X in Xs]
    th = glam.to_device_colmajor(Th, dt)
    eta = glam.rho_forward(Xd, th, n, p, dt)
    torch.cuda.synchronize()
    got = glam.from_colmajor(eta, n)
    ref = O.H(Xs, Th)
    assert rel_inf(got, ref) <= TOL[dt], rel_inf(got, ref)
    if dt == 2:
        ref_r = O.H([rounded(glam, torch, X, dt) for X in Xs], rounded(glam, torch, Th, dt))
        assert rel_inf(got, ref_r) <= 1e-2


@pytest.mark.parametrize("dt", [0, 1, 2])
@pytest.mark.parametrize("n,p", SHAPES + SHAPES_2D + SHAPES_REORDERED)
def test_adjoint_parity(n, p, dt):
    torch, glam = need_gpu()
    print(f"adjoint n={n} p={p} dt={dt}", flush=True)
    Xs = _factors(n, p, 3)
    U = np.random.default_rng(4).standard_normal(n)
    Xd = [glam.to_device_colmajor(X, dt) for X in Xs]
    u = glam.to_device_colmajor(U, dt)
    out = glam.rho_adjoint(Xd, u, n, p, dt)
    torch.cuda.synchronize()
    got = glam.from_colmajor(out, p)
    ref = O.G(Xs, U)
    assert rel_inf(got, ref) <= TOL[dt], rel_inf(got, ref)
    if dt == 2:
        ref_r = O.G([rounded(glam, torch, X, dt) for X in Xs], rounded(glam, torch, U, dt))
        assert rel_inf(got, ref_r) <= 1e-2


@pytest.mark.parametrize("dt", [1, 2, 0])
def test_largest_inner_n_and_p(dt):
    """n_1 = n_2 = 256 with p_1, p_2 near 32: BF16 and FP32 chains take it as given; the FP64 slab
    kernel's LDS image (both orientations of X_1, X_2 in FP64) does not, so FP64 runs it in
    another mode order (X_3 inner, permuted in and out through the workspace)."""
    torch, glam = need_gpu()
    n, p = (256, 256, 3), (32, 31, 2)
    print(f"largest inner modes dt={dt}", flush=True)
    Xs = _factors(n, p, 5)
    Th = np.random.default_rng(6).standard_normal(p)
    Xd = [glam.to_device_colmajor(X, dt) for X in Xs]
    th = glam.to_device_colmajor(Th, dt)
    got = glam.from_colmajor(glam.rho_forward(Xd, th, n, p, dt), n)
    assert rel_inf(got, O.H(Xs, Th)) <= TOL[dt]
    U = np.random.default_rng(7).standard_normal(n)
    got = glam.from_colmajor(glam.rho_adjoint(Xd, glam.to_device_colmajor(U, dt), n, p, dt), p)
    assert rel_inf(got, O.G(Xs, U)) <= TOL[dt]


@pytest.mark.parametrize("dt", [0, 1])
def test_kronecker_explicit_small(dt):
    """Device H against the explicit Kronecker design (App. A identity)."""
    torch, glam = need_gpu()
    n, p = (9, 7, 5), (4, 3, 2)
    Xs = _factors(n, p, 5)
    Th = np.random.default_rng(6).standard_normal(p)
    eta = glam.rho_forward([glam.to_device_colmajor(X, dt) for X in Xs], glam.to_device_colmajor(Th, dt), n, p, dt)
    torch.cuda.synchronize()
    ref = O.kron_design(Xs) @ O.vec(Th)
    assert rel_inf(eta.cpu().numpy(), ref) <= TOL[dt]


@pytest.mark.parametrize("dt", [0, 1, 2])
def test_full_size_gaussian_workload_sampled(dt):
    """At n=(100,100,1000), p=(30,30,200) (B-spline factors): sampled entries of H computed one by
    one from the defining sum, then every entry of H and of the adjoint G against the oracle."""
    torch, glam = need_gpu()
    from paper_1510_03298_amd import inputs
    n, p = (100, 100, 1000), (30, 30, 200)
    Xs = [inputs.bspline_basis(inputs.grid(nj), pj) for nj, pj in zip(n, p)]
    rng = np.random.default_rng(7)
    Th = rng.standard_normal(p)
    Xd = [glam.to_device_colmajor(X, dt) for X in Xs]
    eta = glam.from_colmajor(glam.rho_forward(Xd, glam.to_device_colmajor(Th, dt), n, p, dt), n)
    idx = [tuple(int(rng.integers(0, nj)) for nj in n) for _ in range(200)]
    ref = np.array([np.einsum("a,b,c,abc->", Xs[0][i], Xs[1][j], Xs[2][k], Th) for i, j, k in idx])
    got = np.array([eta[i] for i in idx])
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(got - ref)) / scale <= TOL[dt]
    # every entry of H against the oracle's FP64 transform
    err = rel_inf(eta, O.H(Xs, Th))
    print(f"full-size forward dt={dt}: relative sup-norm error {err:.3e}", flush=True)
    assert err <= TOL[dt]
    # every entry of the adjoint G(U) against the oracle, U random
    U = rng.standard_normal(n)
    g = glam.from_colmajor(glam.rho_adjoint(Xd, glam.to_device_colmajor(U, dt), n, p, dt), p)
    err = rel_inf(g, O.G(Xs, U))
    print(f"full-size adjoint dt={dt}: relative sup-norm error {err:.3e}", flush=True)
    assert err <= TOL[dt]


def test_invalid_sizes_raise():
    """Sizes refused on the host (an empty mode, a mode beyond 2^30 entries), before any device
    work: the workspace query returns 0 and the binding raises (the dummy operands are never read).
    Designs that fit no mode order of the slab kernels are valid: they run on the generic chain."""
    torch, glam = need_gpu()
    for n, p in [((0, 5, 5), (1, 2, 3)), ((5, 5, 5), (2, 0, 3)), ((2 ** 31, 1, 1), (1, 1, 1))]:
        assert glam.rho_workspace_size(n, p, 0) == 0
        with pytest.raises(glam.GlamError):
            glam.rho_forward([torch.zeros(1, device="cuda", dtype=torch.float64)] * 3,
                             torch.zeros(64, device="cuda", dtype=torch.float64), n, p, 0)