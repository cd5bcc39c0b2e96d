"""The allocation-free forward transform (glam_rho_forward_static): the same values, bit for bit,
as glam_rho_forward with a caller workspace, on two calls in a row (the second smaller, so it
runs on what the first left in the static scratch), and the oracle's bar on both."""
import numpy as np
import pytest

import oracle.glam_oracle as O
from tests.gpu_util import need_gpu, rel_inf

pytestmark = pytest.mark.gpu

TOL = {0: 1e-10, 1: 1e-5, 2: 3e-2}

CALLS = [((64, 64, 365), (24, 24, 120)),    # the Poisson workload's sizes
         ((37, 21, 45), (13, 7, 19))]       # smaller, ragged tiles in every mode


@pytest.mark.parametrize("dt", [2, 1, 0])
def test_static_forward_matches_workspace_forward(dt):
    torch, glam = need_gpu()
    for k, (n, p) in enumerate(CALLS):
        print(f"static forward call {k} n={n} p={p} dt={dt}", flush=True)
        assert glam.rho_workspace_size(n, p, dt) <= glam.STATIC_SCRATCH_BYTES
        rng = np.random.default_rng(100 + k)
        Xs = [rng.standard_normal((nj, pj)) for nj, pj in zip(n, p)]
        Th = rng.standard_normal(p)
        Xd = [glam.to_device_colmajor(X, dt) for X in Xs]
        th = glam.to_device_colmajor(Th, dt)
        eta_s = torch.full((int(np.prod(n)),), float("nan"), dtype=glam.out_dtype(dt), device=th.device)
        glam.rho_forward_static(Xd, th, n, p, dt, eta_s)
        eta_w = glam.rho_forward(Xd, th, n, p, dt)
        torch.cuda.synchronize()
        assert torch.equal(eta_s, eta_w)
        err = rel_inf(glam.from_colmajor(eta_s, n), O.H(Xs, Th))
        assert err <= TOL[dt], err


def test_static_forward_reordered_and_refused_sizes():
    """A problem run in another mode order (its permuted input and output also live in the static
    scratch), one that no order fits (the generic chain's transposed factors and intermediates live
    there), and sizes whose workspace exceeds the static scratch: refused on the host before any
    device work."""
    torch, glam = need_gpu()
    n, p = (120, 40, 20), (60, 20, 10)        # p_1 > 32: reordered
    rng = np.random.default_rng(7)
    Xs = [rng.standard_normal((nj, pj)) for nj, pj in zip(n, p)]
    Th = rng.standard_normal(p)
    Xd = [glam.to_device_colmajor(X, 1) for X in Xs]
    th = glam.to_device_colmajor(Th, 1)
    eta_s = torch.empty(int(np.prod(n)), dtype=torch.float32, device=th.device)
    glam.rho_forward_static(Xd, th, n, p, 1, eta_s)
    eta_w = glam.rho_forward(Xd, th, n, p, 1)
    torch.cuda.synchronize()
    assert torch.equal(eta_s, eta_w)
    n, p = (20, 10, 60), (60, 30, 180)        # no mode order fits the slab kernels: the generic GEMM chain
    Xs = [rng.standard_normal((nj, pj)) for nj, pj in zip(n, p)]
    Th = rng.standard_normal(p)
    Xg = [glam.to_device_colmajor(X, 1) for X in Xs]
    thg = glam.to_device_colmajor(Th, 1)
    eta_g = torch.empty(int(np.prod(n)), dtype=torch.float32, device=th.device)
    glam.rho_forward_static(Xg, thg, n, p, 1, eta_g)
    eta_w = glam.rho_forward(Xg, thg, n, p, 1)
    torch.cuda.synchronize()
    assert torch.equal(eta_g, eta_w)
    assert rel_inf(glam.from_colmajor(eta_g, n), O.H(Xs, Th)) <= TOL[1]
    big_n, big_p = (600, 100, 100), (40, 30, 30)   # reordered (mode 1 last): needs n * 8 = 48 MB of workspace
    assert glam.rho_workspace_size(big_n, big_p, 0) > glam.STATIC_SCRATCH_BYTES
    with pytest.raises(glam.GlamError, match="static scratch"):
        glam.rho_forward_static(Xd, th, big_n, big_p, 0, eta_s)
