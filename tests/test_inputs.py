"""Checks of the seeded input generators (basis matrices and workload recipes)."""
import math

import numpy as np
import pytest

from paper_1510_03298_amd import inputs


def test_bspline_basis_matches_scipy():
    si = pytest.importorskip("scipy.interpolate")
    for n, p in [(20, 8), (100, 30), (33, 9), (1000, 200)]:
        x = inputs.grid(n)
        B = inputs.bspline_basis(x, p)
        t = inputs.clamped_knots(p)
        ref = si.BSpline.design_matrix(x, t, 3).toarray()
        np.testing.assert_allclose(B, ref, atol=1e-13)
        np.testing.assert_allclose(B.sum(axis=1), 1.0, atol=1e-13)  # partition of unity
        assert B.min() >= 0.0


def test_basis_count_rule_reproduces_paper_sizes():
    """Sec. 4.2: p_j = max{[n_j/k], 5}; printed sizes fix the rounding as the ceiling."""
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "paper_sizes.json")) as f:
        g = json.load(f)
    for case in g["cases"]:
        p = [inputs.basis_count(nj, case["k"]) for nj in case["n"]]
        assert p == case["p"], case
        P = int(np.prod(p))
        N = int(np.prod(case["n"]))
        assert N == case["n_total"] and P == case["p_total"]
        gib = N * P * 8 / 2 ** 30
        assert abs(gib - case["dense_design_gb"]) < 0.6


def test_configs_shapes_and_seeds():
    c1 = inputs.config_c1()
    assert c1.n == (20, 20, 20) and c1.p == (8, 8, 8)
    assert np.count_nonzero(c1.theta_true) == 51
    c1b = inputs.config_c1()
    np.testing.assert_array_equal(c1.Y, c1b.Y)
    c3 = inputs.config_c3(n=(16, 16, 30), p=(6, 6, 10))
    assert c3.family == "poisson" and np.all(c3.Y >= 0) and np.all(c3.Y == np.round(c3.Y))
    assert abs(np.mean(c3.Y) - 5.0) < 0.5


def test_sec65_rows_have_the_stated_covariance_and_do_not_depend_on_blas_threads():
    """Sec. 6.5's factor rows are N(0, Sigma), Sigma = (sigma - kappa) I + kappa 1 1^T: the sample
    covariance of many rows matches (diagonal sigma, off-diagonal kappa), and the draw is the same
    bytes whatever the BLAS thread count (no factorisation of Sigma is involved)."""
    threadpoolctl = pytest.importorskip("threadpoolctl")
    for fam, sigma in (("gaussian", 1.0), ("poisson", 0.71)):
        d = inputs.config_sim(r=9, q=0.1, family=fam, kappa=0.25)   # n = (180, 90, 540), p = (18, 9, 54)
        Xj = d.X[2]
        C = np.cov(Xj.T, bias=True)
        off = C[~np.eye(C.shape[0], dtype=bool)]
        assert abs(np.mean(np.diag(C)) - sigma) < 0.05, np.mean(np.diag(C))
        assert abs(np.mean(off) - 0.25) < 0.05, np.mean(off)
    with threadpoolctl.threadpool_limits(1):
        a = inputs.config_sim(r=3, family="poisson")
    with threadpoolctl.threadpool_limits(8):
        b = inputs.config_sim(r=3, family="poisson")
    for Xa, Xb in zip(a.X, b.X):
        assert Xa.tobytes() == Xb.tobytes()
    assert a.Y.tobytes() == b.Y.tobytes()
