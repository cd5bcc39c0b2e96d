"""Pins of the CPU oracle against facts the paper and the mathematics fix.

Each test compares the oracle with something other than itself: the defining
sum of rho written as loops, the explicit Kronecker design, closed forms,
a textbook coordinate-descent / Newton solver on the explicit design,
brute-force scalar minimisation, or a theorem's inequality.  A plausible
mistake in the oracle (dropped term, wrong sign, wrong index, transposed
operand, wrong 1/n scale) fails at least one of them.
"""
import math

import numpy as np
import pytest

import oracle.glam_oracle as O
from paper_1510_03298_amd import inputs


def rnd(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


# ---------------------------------------------------------------- App. A ----
@pytest.mark.parametrize("dims,r", [((3,), 2), ((3, 4), 5), ((2, 3, 4), 3), ((4, 2, 3, 2), 3)])
def test_rho_matches_defining_sum(dims, r):
    """App. A: rho(X, A)[i1..id] = sum_j X[id, j] A[j, i1..i_{d-1}]."""
    X = rnd((r, dims[0]), 1)
    A = rnd(dims, 2)
    np.testing.assert_allclose(O.rho(X, A), O.rho_loops(X, A), rtol=1e-13, atol=1e-13)
    assert O.rho(X, A).shape == tuple(dims[1:]) + (r,)


def test_rho_identity_factor_is_cyclic_rotation():
    """With X = I, rho only moves mode 1 to the end (layout pin)."""
    A = rnd((3, 4, 5), 3)
    R = O.rho(np.eye(3), A)
    np.testing.assert_array_equal(R, np.moveaxis(A, 0, -1))
    R3 = O.rho(np.eye(5), O.rho(np.eye(4), R))
    np.testing.assert_array_equal(R3, A)


def test_linear_index_is_column_major():
    """eq. (index): [i1..id] with 1-based indices equals Fortran-order flattening."""
    dims = (3, 4, 5)
    A = rnd(dims, 4)
    v = O.vec(A)
    for idx in [(1, 1, 1), (3, 1, 1), (1, 2, 1), (2, 3, 4), (3, 4, 5)]:
        assert v[O.linear_index(idx, dims) - 1] == A[tuple(i - 1 for i in idx)]


@pytest.mark.parametrize("n,p", [((5,), (3,)), ((4, 6), (3, 2)), ((5, 4, 3), (2, 3, 4)),
                                 ((3, 2, 4), (5, 4, 6)), ((6, 5, 4), (6, 5, 4))])
def test_kronecker_rho_identity(n, p):
    """App. A / eq. (seventeen): (X_d x ... x X_1) vec(A) = vec rho(X_d, ... rho(X_1, A))."""
    Xs = [rnd((nj, pj), 10 + j) for j, (nj, pj) in enumerate(zip(n, p))]
    Th = rnd(p, 20)
    lhs = O.kron_design(Xs) @ O.vec(Th)
    rhs = O.vec(O.H(Xs, Th))
    np.testing.assert_allclose(rhs, lhs, rtol=1e-12, atol=1e-12)
    # G is the transpose of H: X^T vec(U)
    U = rnd(n, 21)
    np.testing.assert_allclose(O.vec(O.G(Xs, U)), O.kron_design(Xs).T @ O.vec(U), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("n,p", [((5, 4, 3), (2, 3, 4)), ((6, 5, 7), (6, 5, 4)), ((3, 8, 5), (3, 2, 5))])
def test_gram_apply_is_the_explicit_normal_matrix(n, p):
    """Sec. 6.2 with identity weights: X^T X vec(D) by three p-sized Gram mode products equals the
    explicit (X_3 x X_2 x X_1)^T (X_3 x X_2 x X_1) vec(D), and G(H(D))."""
    Xs = [rnd((nj, pj), 60 + j) for j, (nj, pj) in enumerate(zip(n, p))]
    D = rnd(p, 70)
    Xd = O.kron_design(Xs)
    np.testing.assert_allclose(O.vec(O.gram_apply(Xs, D)), Xd.T @ (Xd @ O.vec(D)), rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(O.gram_apply(Xs, D), O.G(Xs, O.H(Xs, D)), rtol=1e-11, atol=1e-11)


def test_adjoint_dot_product():
    """<H(Theta), U> = <Theta, G(U)> (G uses the transposed factors, eq. nineteen)."""
    n, p = (7, 6, 9), (3, 5, 4)
    Xs = [rnd((nj, pj), 30 + j) for j, (nj, pj) in enumerate(zip(n, p))]
    Th, U = rnd(p, 40), rnd(n, 41)
    lhs = float(np.sum(O.H(Xs, Th) * U))
    rhs = float(np.sum(Th * O.G(Xs, U)))
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))


def test_flop_model_square_factors():
    """Sec. 2: the array product costs O(d n^{d+1}) for square n x n factors:
    each of the d mode products is 2 n^{d+1} flops."""
    for d, nr in [(2, 7), (3, 5), (4, 3)]:
        assert O.rho_chain_flops([nr] * d, [nr] * d, range(d)) == d * 2 * nr ** (d + 1)


# ---------------------------------------------------------------- App. B ----
def _responses(fam, rng, size):
    """Valid responses of each family: reals, counts, proportions, positive reals."""
    if fam == "poisson":
        return rng.poisson(3.0, size=size).astype(float)
    if fam == "binomial":
        return rng.uniform(0.0, 1.0, size=size)
    if fam == "gamma":
        return rng.gamma(2.0, 1.0, size=size)
    return rng.standard_normal(size)


FAMS = ["gaussian", "poisson", "binomial", "gamma"]


@pytest.mark.parametrize("fam", FAMS)
def test_working_response_forms_agree(fam):
    """eq. (ten) z = W^{-1}u + eta equals eq. (tennew) with the weights of eq. (nine)."""
    rng = np.random.default_rng(5)
    eta = rng.uniform(-2, 2, size=50)
    y = _responses(fam, rng, 50)
    a = rng.uniform(0, 2, size=50)
    u = O.score(fam, eta, y, a)
    w = O.irls_weights(fam, eta)
    np.testing.assert_allclose(O.working_response_eq10(u, w, eta), O.working_response(fam, eta, y, a),
                               rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("fam", FAMS)
def test_score_is_derivative_of_loglik(fam):
    """u = grad_eta l (eq. four) checked by central differences of eq. (two)."""
    rng = np.random.default_rng(6)
    eta = rng.uniform(-1, 1, size=8)
    y = _responses(fam, rng, 8)
    a = rng.uniform(0.5, 1.5, size=8)
    u = O.score(fam, eta, y, a)
    h = 1e-6
    for i in range(8):
        e1, e2 = eta.copy(), eta.copy()
        e1[i] += h
        e2[i] -= h
        fd = (O.loglik(fam, e1, y, a) - O.loglik(fam, e2, y, a)) / (2 * h)
        assert abs(fd - u[i]) < 1e-7 * max(1, abs(u[i]))
    # eq. (nine): the weight is the expected information, -d^2 l / d eta^2 at y = mu
    # (for canonical links this is the derivative of the mean whatever y is)
    w = O.irls_weights(fam, eta)
    mu = O.family(fam).ginv(eta)
    h2 = 1e-4
    for i in range(8):
        f = [O.loglik(fam, np.array([eta[i] + k * h2]), np.array([mu[i]])) for k in (-1, 0, 1)]
        info = -(f[0] - 2 * f[1] + f[2]) / (h2 * h2)
        assert abs(info - w[i]) < 1e-5 * max(1.0, w[i]), (i, info, w[i])
    if fam != "gamma":
        mu_d = (O.family(fam).ginv(eta + h) - O.family(fam).ginv(eta - h)) / (2 * h)
        np.testing.assert_allclose(w, mu_d, rtol=1e-8)


@pytest.mark.parametrize("fam", FAMS)
def test_objective_change_is_the_difference_of_objectives(fam):
    """R5: the entrywise change along t xd equals the difference of the two totals
    (at sizes where subtracting the totals loses nothing), for steps of both signs."""
    rng = np.random.default_rng(8)
    eta = rng.uniform(-3, 3, size=40)
    xd = rng.uniform(-2, 2, size=40)
    y = _responses(fam, rng, 40)
    a = rng.uniform(0.5, 1.5, size=40)
    for t in (1.0, 0.25, -0.5, 1e-3):
        direct = O.neg_loglik_scaled(fam, eta + t * xd, y, a) - O.neg_loglik_scaled(fam, eta, y, a)
        assert abs(O.objective_change(fam, eta, xd, t, y, a) - direct) <= 1e-12 * max(1.0, abs(direct))


def test_gaussian_objective_is_half_rss():
    """R13: for the Gaussian family -l/n is (1/2n) sum a (y - eta)^2."""
    rng = np.random.default_rng(7)
    eta, y, a = rng.standard_normal(30), rng.standard_normal(30), rng.uniform(0, 1, 30)
    assert abs(O.neg_loglik_scaled("gaussian", eta, y, a) - 0.5 * np.sum(a * (y - eta) ** 2) / 30) < 1e-14


# ---------------------------------------------------------------- Sec. 6.3 --
def test_soft_threshold_is_the_l1_prox():
    """prox_gamma(z) = argmin_x 0.5 (x - z)^2 + gamma |x|, brute-forced on a fine grid."""
    xs = np.linspace(-5, 5, 2000001)
    for z, g in [(2.3, 0.7), (-1.1, 0.4), (0.3, 0.5), (-0.5, 0.5), (0.0, 1.0), (4.0, 0.0)]:
        f = 0.5 * (xs - z) ** 2 + g * np.abs(xs)
        assert abs(O.soft_threshold(z, g) - xs[np.argmin(f)]) <= 1e-5
    assert O.soft_threshold(0.5, 0.5) == 0.0 and O.soft_threshold(-0.5, 0.5) == 0.0


def test_ridge_and_elastic_net_prox():
    xs = np.linspace(-5, 5, 2000001)
    for z, g, al in [(2.3, 0.7, 0.5), (-1.7, 0.2, 2.0)]:
        f = 0.5 * (xs - z) ** 2 + g * xs ** 2
        assert abs(O.prox_ridge(z, g) - xs[np.argmin(f)]) <= 1e-5
        f = 0.5 * (xs - z) ** 2 + g * (np.abs(xs) + al * xs ** 2)
        assert abs(O.prox_elastic_net(z, g, al) - xs[np.argmin(f)]) <= 1e-5


# ---------------------------------------------------------------- Sec. 5 ----
def test_lipschitz_bound_prop1():
    """Proposition 1: ||X^T W X||_2 / n <= Lhat, with equality when W = I."""
    n, p = (6, 5, 4), (3, 4, 2)
    Xs = [rnd((nj, pj), 50 + j) for j, (nj, pj) in enumerate(zip(n, p))]
    Xd = O.kron_design(Xs)
    N = Xd.shape[0]
    L_exact = np.max(np.linalg.eigvalsh(Xd.T @ Xd)) / N
    assert abs(O.lipschitz_bound(Xs, np.ones(N), N) - L_exact) <= 1e-12 * L_exact
    w = np.random.default_rng(3).uniform(0.1, 3.0, N)
    L_w = np.max(np.linalg.eigvalsh(Xd.T @ (Xd * w[:, None]))) / N
    assert L_w <= O.lipschitz_bound(Xs, w, N) * (1 + 1e-12)


def test_exact_lipschitz_for_tensor_product_weights():
    """Sec. 5: for W = W_d x ... x W_1, L = prod_j rho(X_j^T W_j X_j) / n."""
    n, p = (5, 4, 3), (3, 2, 2)
    Xs = [rnd((nj, pj), 60 + j) for j, (nj, pj) in enumerate(zip(n, p))]
    ws = [np.random.default_rng(70 + j).uniform(0.2, 2.0, nj) for j, nj in enumerate(n)]
    Wd = np.ones(1)
    for w in ws:
        Wd = np.kron(w, Wd)
    Xd = O.kron_design(Xs)
    N = Xd.shape[0]
    L = np.max(np.linalg.eigvalsh(Xd.T @ (Xd * Wd[:, None]))) / N
    prod = np.prod([np.max(np.linalg.eigvalsh(X.T @ (X * w[:, None]))) for X, w in zip(Xs, ws)])
    assert abs(L - prod / N) <= 1e-12 * L


# ------------------------------------------------------- lambda_max, KKT ----
@pytest.mark.parametrize("fam", FAMS)
def test_lambda_max_gives_zero_solution(fam):
    """Sec. 6.4: lambda_max is the infimum of lambdas with the zero solution."""
    d = inputs.random_problem((5, 4, 4), (3, 3, 2), family=fam, seed=1, scale=0.5, basis="gauss")
    lm = O.lambda_max(fam, d.X, d.Y)
    th, info = O.gdpg(fam, d.X, d.Y, lm, lm, tol=1e-12)
    assert info.converged and np.all(th == 0)
    th2, info2 = O.gdpg(fam, d.X, d.Y, (1 - 1e-3) * lm, lm, tol=1e-12)
    assert info2.converged and np.count_nonzero(th2) >= 1
    # explicit-design certificate: X^T u(0) / n has sup-norm lambda_max
    Xd = O.kron_design(d.X)
    u0 = O.score(fam, np.zeros(Xd.shape[0]), O.vec(d.Y))
    assert abs(np.max(np.abs(Xd.T @ u0)) / Xd.shape[0] - lm) <= 1e-13 * lm


@pytest.mark.parametrize("fam", ["binomial", "gamma"])
def test_identity_factors_closed_form(fam):
    """X_j = I makes every cell its own one-parameter problem,
    (1/n)(b(theta(t)) - y theta(t)) + lambda w |t|, whose minimiser is closed form:
    Binomial-logit  t = logit(y - n lambda w s),     zero iff |y - 1/2| <= n lambda w;
    Gamma-log       t = log(y / (1 + n lambda w s)), zero iff |y - 1| <= n lambda w;
    with s = sign(t).  GD-PG (outer Armijo steps included) must land on it."""
    n = (3, 2, 2)
    N = 12
    rng = np.random.default_rng(11)
    Xs = [np.eye(k) for k in n]
    if fam == "binomial":
        Y = rng.uniform(0.08, 0.92, size=n)
        gap = np.abs(O.vec(Y) - 0.5)
    else:
        Y = rng.uniform(0.25, 4.0, size=n)
        gap = np.abs(O.vec(Y) - 1.0)
    pen = rng.uniform(0.5, 1.5, size=n)
    w = O.vec(pen)
    lam = float(np.median(gap / w)) / N     # about half of the cells stay at zero
    lm = O.lambda_max(fam, Xs, Y, pen_w=pen)
    assert abs(lm - np.max(gap / w) / N) <= 1e-14 * lm
    th, info = O.gdpg(fam, Xs, Y, lam, lm, pen_w=pen, tol=1e-12, max_outer=200)
    assert info.converged
    y = O.vec(Y)
    with np.errstate(invalid="ignore", divide="ignore"):   # the log branch is discarded where zero
        if fam == "binomial":
            s = np.sign(y - 0.5)
            q = y - N * lam * w * s
            expect = np.where(gap <= N * lam * w, 0.0, np.log(q / (1 - q)))
        else:
            s = np.sign(y - 1.0)
            expect = np.where(gap <= N * lam * w, 0.0, np.log(y / (1 + N * lam * w * s)))
    assert np.count_nonzero(expect) not in (0, N)
    np.testing.assert_allclose(O.vec(th), expect, rtol=1e-9, atol=1e-10)


@pytest.mark.parametrize("fam", ["binomial", "gamma"])
def test_new_families_stationary_on_explicit_design(fam):
    """Binomial and Gamma lasso fits on a dense Gaussian design: no coordinate move,
    of either sign, lowers the objective evaluated on the explicit Kronecker design."""
    d = inputs.random_problem((6, 5, 4), (3, 3, 2), family=fam, seed=12, basis="gauss", scale=0.3)
    lm = O.lambda_max(fam, d.X, d.Y)
    lam = 0.1 * lm
    th, info = O.gdpg(fam, d.X, d.Y, lam, lm, tol=1e-12, max_outer=200, max_inner=20000)
    assert info.converged and np.count_nonzero(th) >= 2
    Xd = O.kron_design(d.X)
    y = O.vec(d.Y)

    def F(v):
        eta = Xd @ v
        if fam == "binomial":
            nll = np.logaddexp(0.0, eta) - y * eta
        else:
            nll = y * np.exp(-eta) + eta
        return float(np.mean(nll)) + lam * float(np.sum(np.abs(v)))
    v = O.vec(th)
    F0 = F(v)
    assert abs(F0 - O.objective(fam, d.X, th, d.Y, lam)) <= 1e-12 * abs(F0)
    for m in range(v.size):
        for h in (1e-4, -1e-4):
            t = v.copy()
            t[m] += h
            assert F(t) >= F0 - 1e-13


def test_scad_penalty_and_slope():
    """Fan-Li SCAD: p'(t) = lambda up to lambda, (a lambda - t)_+ / (a - 1) beyond; the
    penalty is continuous with p(lambda) = lambda^2 and the constant (a + 1) lambda^2 / 2
    from a lambda on; the slope is the penalty's central difference everywhere."""
    lam, a = 0.7, O.SCAD_A
    t = np.concatenate([np.linspace(0.0, 4.0 * lam * a, 401), [lam, a * lam, 2 * lam]])
    h = 1e-6
    fd = (O.scad_penalty(t + h, lam) - O.scad_penalty(np.maximum(t - h, 0.0), lam)) / (t + h - np.maximum(t - h, 0.0))
    d = O.scad_derivative(t, lam)
    ok = (np.abs(t - lam) > 2 * h) & (np.abs(t - a * lam) > 2 * h)   # the slope itself has kinks there
    np.testing.assert_allclose(fd[ok], d[ok], rtol=1e-6, atol=1e-8)
    assert abs(float(O.scad_penalty(lam, lam)) - lam * lam) < 1e-15
    for e in (1e-12, -1e-12):
        assert abs(float(O.scad_penalty(a * lam + e, lam)) - 0.5 * (a + 1) * lam * lam) < 1e-11
    assert float(O.scad_derivative(lam, lam)) == lam and float(O.scad_derivative(a * lam, lam)) == 0.0
    assert float(O.scad_derivative(0.5 * (lam + a * lam), lam)) == pytest.approx(0.5 * lam * (a - 1) / (a - 1))


def test_msa_orthogonal_design_reaches_scad_thresholding():
    """With X^T X = n I the SCAD problem separates, and the MSA-lasso iteration converges
    to Fan and Li's thresholding rule for z = X^T y / n:
    sign(z)(|z| - lambda)_+ for |z| <= 2 lambda, ((a-1) z - sign(z) a lambda)/(a-2) up to
    a lambda, and z itself beyond."""
    d = inputs.random_problem((8, 7, 6), (4, 3, 5), seed=13, basis="orth")
    Xd = O.kron_design(d.X)
    N = Xd.shape[0]
    z = Xd.T @ O.vec(d.Y) / N
    a = O.SCAD_A
    lam = float(np.median(np.abs(z))) / 1.5
    az = np.abs(z)
    regimes = [np.sum(az <= lam), np.sum((az > lam) & (az <= 2 * lam)), np.sum((az > 2 * lam) & (az <= a * lam)),
               np.sum(az > a * lam)]
    assert min(regimes) >= 2, regimes
    lm = O.lambda_max("gaussian", d.X, d.Y)
    th, info, w = O.msa_scad("gaussian", d.X, d.Y, lam, lm, steps=60, tol=1e-13, max_outer=3, max_inner=5000)
    assert info.converged
    expect = np.where(az <= 2 * lam, np.sign(z) * np.maximum(az - lam, 0.0),
                      np.where(az <= a * lam, ((a - 1) * z - np.sign(z) * a * lam) / (a - 2), z))
    np.testing.assert_allclose(O.vec(th), expect, rtol=1e-10, atol=1e-11)
    # one step is the lasso
    th1, _, _ = O.msa_scad("gaussian", d.X, d.Y, lam, lm, steps=1, tol=1e-13, max_outer=3, max_inner=5000)
    np.testing.assert_allclose(O.vec(th1), O.soft_threshold(z, lam), rtol=1e-10, atol=1e-11)


def test_kron_weights_exact_for_tensor_products():
    """Sec. 6.2 (R18): a weight array that is already a tensor product is reproduced; for
    any positive V, log V-hat is additively separable and has the marginal means of log V."""
    rng = np.random.default_rng(14)
    u = [rng.uniform(0.2, 3.0, size=k) for k in (5, 4, 6)]
    V = u[0][:, None, None] * u[1][None, :, None] * u[2][None, None, :]
    Vh, vs, vbar = O.kron_weights(V)
    np.testing.assert_allclose(Vh, V, rtol=1e-13)
    W = rng.uniform(0.1, 5.0, size=(5, 4, 6))
    Wh, _, _ = O.kron_weights(W)
    L, Lh = np.log(W), np.log(Wh)
    for axes in ((1, 2), (0, 2), (0, 1)):
        np.testing.assert_allclose(Lh.mean(axis=axes), L.mean(axis=axes), atol=1e-13)
    # separability: every mixed second difference of log V-hat vanishes
    mixed = Lh[1:, 1:, :] - Lh[1:, :-1, :] - Lh[:-1, 1:, :] + Lh[:-1, :-1, :]
    assert np.max(np.abs(mixed)) < 1e-13
    mixed = Lh[:, 1:, 1:] - Lh[:, 1:, :-1] - Lh[:, :-1, 1:] + Lh[:, :-1, :-1]
    assert np.max(np.abs(mixed)) < 1e-13


def test_kron_weights_reach_the_same_pmle():
    """GD-PG with the tensor-product weights of Sec. 6.2 converges to the Poisson PMLE that
    proximal Newton finds on the explicit design (the weights only shape the steps, and a
    poor approximation makes them short: this problem's counts reach 177)."""
    d = inputs.random_problem((6, 5, 4), (3, 3, 2), family="poisson", seed=15, basis="gauss", scale=0.4)
    lm = O.lambda_max("poisson", d.X, d.Y)
    lam = 0.1 * lm
    th, info = O.gdpg("poisson", d.X, d.Y, lam, lm, tol=1e-9, weights="kron", max_outer=400, max_inner=20000)
    assert info.converged
    ref = O.poisson_lasso_explicit(d.X, d.Y, lam)
    np.testing.assert_allclose(O.vec(th), ref, rtol=1e-6, atol=1e-8)


def test_kkt_residual_definition():
    """R6 on a hand-made case: zero and nonzero coordinates."""
    th = np.array([0.0, 1.0, -2.0, 0.0])
    g = np.array([0.5, -0.3, 0.1, -1.4])
    lam, lm = 1.0, 2.0
    # r = [max(.5-1,0), |-.3+1|, |.1-1|, max(1.4-1,0)] = [0, .7, .9, .4]
    assert abs(O.kkt_residual(th, g, lam, lm) - 0.45) < 1e-15
    assert O.kkt_residual(np.zeros(3), np.array([0.2, -0.9, 1.0]), 1.0, 1.0) == 0.0


# ----------------------------------------------------- Gaussian solutions ----
def test_gaussian_closed_form_orthogonal_design():
    """X_j = sqrt(n_j) Q_j gives X^T X = n I, so theta* = S_{lambda w}(X^T y / n)."""
    d = inputs.random_problem((8, 7, 6), (4, 3, 5), seed=2, basis="orth")
    Xd = O.kron_design(d.X)
    N = Xd.shape[0]
    np.testing.assert_allclose(Xd.T @ Xd / N, np.eye(Xd.shape[1]), atol=1e-12)
    lm = O.lambda_max("gaussian", d.X, d.Y)
    pen = np.random.default_rng(9).uniform(0.5, 2.0, d.p)
    lmw = O.lambda_max("gaussian", d.X, d.Y, pen_w=pen)
    lam = 0.3 * lmw
    th, info = O.gdpg("gaussian", d.X, d.Y, lam, lmw, pen_w=pen, tol=1e-13)
    expect = O.soft_threshold(Xd.T @ O.vec(d.Y) / N, lam * O.vec(pen))
    np.testing.assert_allclose(O.vec(th), expect, rtol=1e-11, atol=1e-12 * lm)
    assert info.outer == 1  # Gaussian: a single outer pass


def test_elastic_net_kkt_residual_definition():
    """R15: the smooth term's derivative 2 alpha lambda w theta joins the gradient."""
    th = np.array([0.0, 1.0, -2.0])
    g = np.array([0.5, -0.3, 0.1])
    lam, lm, al = 1.0, 2.0, 0.25
    # gs = g + 2 al lam th = [.5, .2, -.9]; r = [max(.5-1, 0), |.2+1|, |-.9-1|] = [0, 1.2, 1.9]
    assert abs(O.kkt_residual(th, g, lam, lm, alpha=al) - 0.95) < 1e-15
    assert abs(O.penalty(th, alpha=al) - (3.0 + 0.25 * 5.0)) < 1e-15


def test_elastic_net_closed_form_orthogonal_design():
    """Sec. 6.3 elastic net with X^T X = n I: the minimiser of
    (1/2n)||y - X theta||^2 + lambda sum w (|theta| + alpha theta^2) is
    S_{lambda w}(X^T y / n) / (1 + 2 alpha lambda w), coordinate by coordinate."""
    d = inputs.random_problem((8, 7, 6), (4, 3, 5), seed=3, basis="orth")
    Xd = O.kron_design(d.X)
    N = Xd.shape[0]
    pen = np.random.default_rng(10).uniform(0.5, 2.0, d.p)
    lmw = O.lambda_max("gaussian", d.X, d.Y, pen_w=pen)
    lam, al = 0.3 * lmw, 0.7
    th, info = O.gdpg("gaussian", d.X, d.Y, lam, lmw, pen_w=pen, tol=1e-13, alpha=al, max_outer=3, max_inner=3000)
    assert info.converged
    w = O.vec(pen)
    expect = O.soft_threshold(Xd.T @ O.vec(d.Y) / N, lam * w) / (1.0 + 2.0 * al * lam * w)
    np.testing.assert_allclose(O.vec(th), expect, rtol=1e-11, atol=1e-12 * lmw)


def test_elastic_net_poisson_is_stationary_on_explicit_design():
    """Poisson elastic net: the GD-PG solution is a stationary point of the objective
    on the explicit design (scalar brute force along every coordinate direction)."""
    d = inputs.random_problem((6, 5, 4), (3, 3, 2), family="poisson", seed=5, basis="gauss", scale=0.3)
    lm = O.lambda_max("poisson", d.X, d.Y)
    lam, al = 0.2 * lm, 0.5
    th, info = O.gdpg("poisson", d.X, d.Y, lam, lm, tol=1e-12, alpha=al, max_outer=60, max_inner=5000)
    assert info.converged
    F0 = O.objective("poisson", d.X, th, d.Y, lam, alpha=al)
    v = O.vec(th)
    for m in range(v.size):
        for h in (1e-4, -1e-4):
            t = v.copy()
            t[m] += h
            assert O.objective("poisson", d.X, O.unvec(t, d.p), d.Y, lam, alpha=al) >= F0 - 1e-13


@pytest.mark.parametrize("basis", ["bspline", "gauss"])
def test_gaussian_matches_coordinate_descent(basis):
    """GD-PG (design-free) vs textbook CD on the explicit design (independent algorithm)."""
    d = inputs.random_problem((9, 8, 7), (5, 4, 4), seed=3, basis=basis)
    lm = O.lambda_max("gaussian", d.X, d.Y)
    for frac in [0.5, 0.1, 0.01]:
        lam = frac * lm
        th, info = O.gdpg("gaussian", d.X, d.Y, lam, lm, tol=1e-12)
        assert info.converged
        cd = O.gaussian_lasso_explicit(d.X, d.Y, lam)
        scale = np.max(np.abs(cd))
        np.testing.assert_allclose(O.vec(th), cd, atol=1e-8 * scale)
        # objective relative deviation (eq. thirtythree) ~ 0
        F1 = O.objective("gaussian", d.X, th, d.Y, lam)
        F2 = O.objective("gaussian", d.X, O.unvec(cd, d.p), d.Y, lam)
        assert abs(F1 - F2) / abs(F2) < 1e-12


def test_gaussian_with_observation_weights_matches_cd():
    """Observation weights a_i (some zero = missing cells): Alg. 1 with z of eq. (tennew)."""
    d = inputs.random_problem((7, 6, 6), (4, 4, 3), seed=4, obs_weights=True, basis="gauss")
    lm = O.lambda_max("gaussian", d.X, d.Y, a=d.a)
    lam = 0.05 * lm
    th, info = O.gdpg("gaussian", d.X, d.Y, lam, lm, a=d.a, tol=1e-11)
    assert info.converged and info.outer > 1  # a != 1: z depends on eta, several outer passes
    cd = O.gaussian_lasso_explicit(d.X, d.Y, lam, a=d.a)
    np.testing.assert_allclose(O.vec(th), cd, atol=1e-7 * np.max(np.abs(cd)))


def test_gaussian_lambda_zero_is_least_squares():
    d = inputs.random_problem((6, 5, 5), (3, 3, 2), seed=5, basis="gauss")
    Xd = O.kron_design(d.X)
    ls, *_ = np.linalg.lstsq(Xd, O.vec(d.Y), rcond=None)
    lm = O.lambda_max("gaussian", d.X, d.Y)
    th, info = O.gdpg("gaussian", d.X, d.Y, 0.0, lm, tol=1e-13)
    np.testing.assert_allclose(O.vec(th), ls, rtol=1e-8, atol=1e-9 * np.max(np.abs(ls)))


# ------------------------------------------------------ Poisson solutions ----
def test_poisson_lambda_zero_is_mle():
    """lambda = 0: the PMLE is the MLE, computed by textbook Newton on the explicit design."""
    d = inputs.random_problem((6, 5, 5), (3, 3, 2), family="poisson", seed=6, scale=0.3, basis="gauss")
    mle = O.poisson_mle_newton(d.X, d.Y)
    lm = O.lambda_max("poisson", d.X, d.Y)
    th, info = O.gdpg("poisson", d.X, d.Y, 0.0, lm, tol=1e-12, max_outer=200)
    assert info.converged
    np.testing.assert_allclose(O.vec(th), mle, atol=1e-8 * np.max(np.abs(mle)))


@pytest.mark.parametrize("frac", [0.3, 0.05])
def test_poisson_matches_prox_newton(frac):
    d = inputs.random_problem((7, 6, 5), (4, 3, 3), family="poisson", seed=7, scale=0.5, basis="gauss")
    lm = O.lambda_max("poisson", d.X, d.Y)
    lam = frac * lm
    th, info = O.gdpg("poisson", d.X, d.Y, lam, lm, tol=1e-11, max_outer=200)
    assert info.converged
    ref = O.poisson_lasso_explicit(d.X, d.Y, lam)
    np.testing.assert_allclose(O.vec(th), ref, atol=1e-7 * max(1e-3, np.max(np.abs(ref))))
    # Theorem 2: F(theta^k) is nonincreasing over the outer iterations
    hist = np.array(info.objective_history)
    assert np.all(np.diff(hist) <= 1e-14 * np.abs(hist[:-1]))


def test_poisson_with_observation_weights():
    d = inputs.random_problem((6, 6, 5), (3, 3, 3), family="poisson", seed=8, scale=0.4, obs_weights=True, basis="gauss")
    lm = O.lambda_max("poisson", d.X, d.Y, a=d.a)
    lam = 0.1 * lm
    th, info = O.gdpg("poisson", d.X, d.Y, lam, lm, a=d.a, tol=1e-11, max_outer=200)
    assert info.converged
    ref = O.poisson_lasso_explicit(d.X, d.Y, lam, a=d.a)
    np.testing.assert_allclose(O.vec(th), ref, atol=1e-7 * max(1e-3, np.max(np.abs(ref))))


# ------------------------------------------------------------ Theorem 1 ----
def test_fista_rate_theorem1():
    """Thm. 1: with delta = 1/L, G(x^(l+1)) - G(x*) <= 2 L ||x^(0) - x*||^2 / (l+1)^2
    for the iterate produced at inner step l (R4 off: fixed number of steps)."""
    d = inputs.random_problem((7, 6, 5), (4, 4, 3), seed=9, basis="gauss")
    Xs, Y = d.X, d.Y
    N = Y.size
    Xd = O.kron_design(Xs)
    L = np.max(np.linalg.eigvalsh(Xd.T @ Xd)) / N
    lm = O.lambda_max("gaussian", Xs, Y)
    lam = 0.05 * lm
    xstar = O.unvec(O.gaussian_lasso_explicit(Xs, Y, lam), d.p)
    V = np.ones_like(Y)
    cz = O.G(Xs, Y) / N
    x0 = np.zeros(d.p)
    _, _, trace = O.inner_pg(Xs, V, cz, x0, lam, 1.0 / L, None, -1.0, lm, 60, record=True)

    def Gobj(x):
        return 0.5 * np.sum((O.H(Xs, x) - Y) ** 2) / N + lam * O.penalty(x)
    Gs = Gobj(xstar)
    R2 = np.sum((x0 - xstar) ** 2)
    for l, x in enumerate(trace, start=1):
        assert Gobj(x) - Gs <= 2 * L * R2 / (l + 1) ** 2 * (1 + 1e-9) + 1e-14


def test_exact_lipschitz_for_tensor_product_weights():
    """Sec. 5: for W = W_3 (x) W_2 (x) W_1 the Lipschitz constant of grad h, rho(X^T W X)/n on the
    explicit design, equals (1/n) prod_j rho(X_j^T W_j X_j); for other positive W Proposition 1's
    max(w) prod_j rho(X_j^T X_j)/n only bounds it."""
    rng = np.random.default_rng(17)
    Xs = [rng.standard_normal((nj, pj)) for nj, pj in ((6, 3), (5, 4), (7, 2))]
    vs = [rng.uniform(0.2, 3.0, X.shape[0]) for X in Xs]
    Xd = O.kron_design(Xs)
    w = np.kron(vs[2], np.kron(vs[1], vs[0]))   # vec order: mode 1 fastest
    n = Xd.shape[0]
    L = float(np.linalg.eigvalsh(Xd.T @ (w[:, None] * Xd))[-1]) / n
    assert abs(O.lipschitz_tensor_weights(Xs, vs, n) - L) <= 1e-12 * L
    assert O.lipschitz_bound(Xs, w, n) >= L * (1 - 1e-12)


def test_ridge_closed_form_orthogonal_design():
    """Sec. 6.3 ridge penalty (R21): with X^T X = n I the Gaussian ridge estimate is the
    multiplicative shrinkage z / (1 + 2 lambda w) of z = X^T y / n, coordinate by coordinate."""
    d = inputs.random_problem((8, 7, 6), (4, 3, 5), seed=20, basis="orth")
    pen = np.random.default_rng(21).uniform(0.5, 2.0, d.p)
    Xd = O.kron_design(d.X)
    z = Xd.T @ O.vec(d.Y) / Xd.shape[0]
    lm = O.lambda_max("gaussian", d.X, d.Y)
    lam = 0.3 * lm
    th, info = O.gdpg("gaussian", d.X, d.Y, lam, lm, pen_w=pen, tol=1e-12, alpha=1.0, l1=0.0, max_outer=3,
                      max_inner=5000)
    assert info.converged
    np.testing.assert_allclose(O.vec(th), z / (1.0 + 2.0 * lam * O.vec(pen)), rtol=1e-9, atol=1e-12)


def test_ridge_matches_normal_equations():
    """Gaussian ridge on a general (correlated) design: (X^T X / n + 2 lambda I) theta = X^T y / n."""
    d = inputs.random_problem((7, 6, 5), (3, 4, 3), seed=22, basis="gauss")
    Xd = O.kron_design(d.X)
    n = Xd.shape[0]
    lm = O.lambda_max("gaussian", d.X, d.Y)
    lam = 0.05 * lm
    ref = np.linalg.solve(Xd.T @ Xd / n + 2 * lam * np.eye(Xd.shape[1]), Xd.T @ O.vec(d.Y) / n)
    th, info = O.gdpg("gaussian", d.X, d.Y, lam, lm, tol=1e-12, alpha=1.0, l1=0.0, max_inner=20000)
    assert info.converged
    np.testing.assert_allclose(O.vec(th), ref, rtol=1e-8, atol=1e-10 * np.max(np.abs(ref)))
    g = O.smooth_gradient("gaussian", d.X, th, d.Y)
    assert O.kkt_residual(th, g, lam, lm, alpha=1.0, l1=0.0) <= 1e-12


def test_poisson_ridge_matches_newton():
    """Poisson ridge: Newton's method on the explicit design for (1/n) sum (e^eta - y eta) +
    lambda ||theta||^2 (smooth and strictly convex) gives the same estimate."""
    d = inputs.random_problem((7, 6, 5), (3, 3, 2), family="poisson", seed=23, scale=0.3, basis="gauss")
    Xd = O.kron_design(d.X)
    y = O.vec(d.Y)
    n, P = Xd.shape
    lm = O.lambda_max("poisson", d.X, d.Y)
    lam = 0.2 * lm
    b = np.zeros(P)
    for _ in range(100):
        mu = np.exp(Xd @ b)
        gr = Xd.T @ (mu - y) / n + 2 * lam * b
        Hs = Xd.T @ (mu[:, None] * Xd) / n + 2 * lam * np.eye(P)
        b = b - np.linalg.solve(Hs, gr)
        if np.max(np.abs(gr)) < 1e-15:
            break
    th, info = O.gdpg("poisson", d.X, d.Y, lam, lm, tol=1e-12, alpha=1.0, l1=0.0, max_outer=300)
    assert info.converged
    np.testing.assert_allclose(O.vec(th), b, rtol=1e-7, atol=1e-9)


@pytest.mark.parametrize("fam", ["gaussian", "poisson"])
def test_nu_zero_reaches_same_solution(fam):
    """Sec. 6.4, nu = 0 (R22): the inner step starts at 1 with Beck-Teboulle backtracking at every
    iteration; the fit reaches the same PMLE as nu = 1."""
    d = inputs.random_problem((7, 6, 5), (4, 3, 3), family=fam, seed=24, scale=0.4, basis="gauss")
    lm = O.lambda_max(fam, d.X, d.Y)
    th1, i1 = O.gdpg(fam, d.X, d.Y, 0.1 * lm, lm, tol=1e-11, max_outer=200)
    th0, i0 = O.gdpg(fam, d.X, d.Y, 0.1 * lm, lm, tol=1e-11, max_outer=200, nu=0.0)
    assert i1.converged and i0.converged
    np.testing.assert_allclose(O.vec(th0), O.vec(th1), atol=1e-8 * np.max(np.abs(th1)))


def test_nu_backtracking_reaches_same_solution():
    """nu in (0,1): larger initial step with backtracking (R7) gives the same PMLE."""
    d = inputs.random_problem((7, 6, 5), (4, 3, 3), family="poisson", seed=10, scale=0.4, basis="gauss")
    lm = O.lambda_max("poisson", d.X, d.Y)
    lam = 0.1 * lm
    th1, i1 = O.gdpg("poisson", d.X, d.Y, lam, lm, tol=1e-11, max_outer=200)
    th2, i2 = O.gdpg("poisson", d.X, d.Y, lam, lm, tol=1e-11, max_outer=200, nu=0.5)
    assert i1.converged and i2.converged
    np.testing.assert_allclose(O.vec(th2), O.vec(th1), atol=1e-8 * np.max(np.abs(th1)))


def test_armijo_takes_no_step_along_a_non_descent_direction(monkeypatch):
    """Sec. 5: the Armijo rule presumes a descent direction (Delta_k < 0) and Theorem 2 then gives a
    nonincreasing F.  An inexact inner solve that returns the reflection 2 theta^k - x of the model's
    minimiser x gives Delta_k > 0 (J is convex); no step may be taken along it, so F stays put."""
    d = inputs.random_problem((7, 6, 5), (4, 3, 3), family="poisson", seed=16, scale=0.4, basis="gauss")
    lm = O.lambda_max("poisson", d.X, d.Y)
    orig = O.inner_pg

    def reflected(Xs, V, cz, x0, *args, **kw):
        x, nin, trace = orig(Xs, V, cz, x0, *args, **kw)
        return 2.0 * x0 - x, nin, trace

    th_ok, info_ok = O.gdpg("poisson", d.X, d.Y, 0.1 * lm, lm, tol=1e-10, max_outer=3)
    assert info_ok.alphas[0] > 0.0   # the unplanted first step moves
    monkeypatch.setattr(O, "inner_pg", reflected)
    th0 = np.full(d.p, 0.05)
    th, info = O.gdpg("poisson", d.X, d.Y, 0.1 * lm, lm, theta0=th0, tol=1e-10, max_outer=3)
    assert info.alphas == [0.0, 0.0, 0.0]
    assert np.array_equal(th, th0)
    hist = info.objective_history
    assert all(b <= a for a, b in zip(hist, hist[1:]))


# ---------------------------------------------------------------- path -----
def test_path_warm_start_and_kkt():
    d = inputs.random_problem((6, 6, 6), (4, 4, 4), seed=11)
    lams, thetas, infos, lm = O.fit_path("gaussian", d.X, d.Y, nlambda=8, ratio=1e-2, tol=1e-10)
    assert len(thetas) == 8 and abs(lams[0] - lm) < 1e-15 * lm
    assert np.all(np.diff(lams) < 0)
    assert np.all(thetas[0] == 0)
    for lam, th, info in zip(lams, thetas, infos):
        g = O.smooth_gradient("gaussian", d.X, th, d.Y)
        assert O.kkt_residual(th, g, lam, lm) <= 1e-10
    nnz = [np.count_nonzero(t) for t in thetas]
    assert nnz[-1] > nnz[1]


@pytest.mark.parametrize("nlambda,ratio", [(100, 1e-4), (50, 1e-4), (12, 1e-3), (2, 0.5)])
def test_lambda_grid_end_point_and_log_spacing(nlambda, ratio):
    """Sec. 6.4 (R3): the path starts at lambda_max, ends at lambda_min = ratio * lambda_max and its
    points are equally spaced in log lambda.  The reference is built by repeated multiplication with
    the common ratio q, q^(nlambda - 1) = ratio, not by the oracle's closed form."""
    lm = 0.7311
    grid = O.lambda_grid(lm, nlambda, ratio)
    assert grid.shape == (nlambda,)
    assert grid[0] == lm
    assert abs(grid[-1] - ratio * lm) <= 1e-13 * lm
    q = math.exp(math.log(ratio) / (nlambda - 1))
    ref = [lm]
    for _ in range(nlambda - 1):
        ref.append(ref[-1] * q)
    np.testing.assert_allclose(grid, ref, rtol=1e-12)
    steps = np.diff(np.log(grid))
    np.testing.assert_allclose(steps, math.log(ratio) / (nlambda - 1), rtol=1e-9)


def test_lambda_grid_single_value():
    """A one-model path is lambda_max alone (the zero solution)."""
    assert list(O.lambda_grid(2.5, 1, 1e-4)) == [2.5]


def test_path_early_exit_returns_preceding_models():
    """Sec. 6.5: on non-convergence the path stops and returns only the preceding models."""
    d = inputs.random_problem((6, 6, 6), (4, 4, 4), seed=12)
    lams, thetas, infos, lm = O.fit_path("gaussian", d.X, d.Y, nlambda=6, ratio=1e-3, tol=1e-12,
                                         max_inner=3)
    assert not infos[-1].converged and len(thetas) < 6


# ---------------------------------------------------------- Poisson NLL ---
def test_poisson_nll_gradient_central_differences():
    d = inputs.random_problem((6, 5, 4), (3, 3, 2), family="poisson", seed=13, scale=0.3, basis="gauss")
    beta = np.random.default_rng(1).normal(0, 0.3, d.p)
    g = O.poisson_nll_grad(d.X, beta, d.Y)
    h = 1e-6
    for m in range(beta.size):
        e = np.zeros(beta.size)
        e[m] = h
        e = O.unvec(e, d.p)
        fd = (O.poisson_nll(d.X, beta + e, d.Y) - O.poisson_nll(d.X, beta - e, d.Y)) / (2 * h)
        assert abs(fd - O.vec(g)[m]) <= 1e-7 * max(1.0, abs(fd))
    # and against the explicit-design gradient X^T (e^eta - y) / n
    Xd = O.kron_design(d.X)
    eta = Xd @ O.vec(beta)
    np.testing.assert_allclose(O.vec(g), Xd.T @ (np.exp(eta) - O.vec(d.Y)) / Xd.shape[0], rtol=1e-12, atol=1e-14)


def test_poisson_nll_value_on_the_explicit_design():
    """Sec. 2, eqs. (two)-(four) with a = 1 and log y! dropped: L(beta) = (1/n) sum_i (e^{eta_i} -
    y_i eta_i) with eta = X beta on the explicit Kronecker design (App. A)."""
    d = inputs.random_problem((6, 5, 4), (3, 3, 2), family="poisson", seed=14, scale=0.3, basis="gauss")
    beta = np.random.default_rng(4).normal(0, 0.3, d.p)
    Xd = O.kron_design(d.X)
    eta = Xd @ O.vec(beta)
    y = O.vec(d.Y)
    ref = sum(math.exp(e) - yi * e for e, yi in zip(eta, y)) / len(y)
    assert abs(O.poisson_nll(d.X, beta, d.Y) - ref) <= 1e-13 * max(1.0, abs(ref))


def test_poisson_nll_constant_predictor_closed_form():
    """Clamped B-spline factors are a partition of unity, so beta = c 1 gives eta = c everywhere and
    L = e^c - c mean(y) in closed form."""
    d = inputs.random_problem((9, 7, 8), (5, 4, 6), family="poisson", seed=15, scale=0.3)
    for c in (-0.4, 0.0, 1.3):
        beta = np.full(d.p, c)
        ref = math.exp(c) - c * float(np.mean(d.Y))
        assert abs(O.poisson_nll(d.X, beta, d.Y) - ref) <= 1e-12 * max(1.0, abs(ref))


# ---------------------------------------------------------- rounding -------
def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    x = np.random.default_rng(2).standard_normal(10000) * 10.0 ** np.random.default_rng(3).integers(-5, 5, 10000)
    ref = torch.from_numpy(x).to(torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(O.round_to_bf16(x), ref)


def test_unit_weights_gaussian_is_the_exact_form():
    """Sec. 5, after the corollary to Theorem 2 (constant weights): the Gaussian IRLS weights are already 1, so weights="one" takes
    the very same steps as the exact weights."""
    d = inputs.random_problem((7, 6, 5), (4, 4, 3), family="gaussian", seed=18, basis="gauss")
    lm = O.lambda_max("gaussian", d.X, d.Y)
    a, ia = O.gdpg("gaussian", d.X, d.Y, 0.2 * lm, lm, tol=1e-10)
    b, ib = O.gdpg("gaussian", d.X, d.Y, 0.2 * lm, lm, tol=1e-10, weights="one")
    assert np.array_equal(a, b) and ia.inner == ib.inner


@pytest.mark.parametrize("fam", ["poisson", "binomial"])
def test_unit_weights_reach_the_same_pmle(fam):
    """Sec. 5, after the corollary to Theorem 2: any strictly positive continuous weights give a convergent GD-PG; with w_i = 1 the
    quadratic models differ from the IRLS ones but the minimiser reached is the same."""
    d = inputs.random_problem((7, 6, 5), (4, 4, 3), family=fam, seed=19, scale=0.5, basis="gauss")
    lm = O.lambda_max(fam, d.X, d.Y)
    exact, ie = O.gdpg(fam, d.X, d.Y, 0.2 * lm, lm, tol=1e-10, max_outer=400)
    one, io = O.gdpg(fam, d.X, d.Y, 0.2 * lm, lm, tol=1e-10, max_outer=400, weights="one")
    assert ie.converged and io.converged
    assert np.max(np.abs(one - exact)) <= 1e-6 * max(1.0, np.max(np.abs(exact)))
    g = O.smooth_gradient(fam, d.X, one, d.Y)
    assert O.kkt_residual(one, g, 0.2 * lm, lm) <= 1e-10


# =============================================================================
# c > 1 tensor components (Sec. 2 eq. fivenew; Sec. 6.1 eqs. eighteen, nineteen; Proposition 1)
# =============================================================================
def _concatenated_design(comps):
    """[X_1 | ... | X_c] with X_r = X_{r,d} (x) ... (x) X_{r,1}, built here with numpy's kron."""
    blocks = []
    for Xs in comps:
        D = np.ones((1, 1))
        for X in Xs:
            D = np.kron(X, D)
        blocks.append(D)
    return np.hstack(blocks)


@pytest.mark.parametrize("n,ps", [((6, 5, 4), [(3, 2, 2), (2, 3, 3)]),
                                  ((7, 6), [(3, 2), (2, 4), (4, 3)]),
                                  ((5, 4, 3), [(2, 2, 2)])])
def test_components_H_and_G_are_the_concatenated_design(n, ps):
    """vec(H(<X_rj>, <Theta_r>)) = X theta and G(<X_rj>, U) = X^T vec(U), stacked as theta is."""
    d = inputs.random_components_problem(n, ps, seed=11)
    C = O.Components(d.comps)
    D = _concatenated_design(d.comps)
    np.testing.assert_array_equal(O.kron_design(C), D)
    rng = np.random.default_rng(5)
    th = rng.standard_normal(D.shape[1])
    np.testing.assert_allclose(O.vec(O.H(C, th)), D @ th, rtol=1e-12, atol=1e-12)
    U = rng.standard_normal(tuple(n))
    np.testing.assert_allclose(O.G(C, U), D.T @ O.vec(U), rtol=1e-12, atol=1e-12)
    assert O.param_shape(C) == (D.shape[1],)


def test_prop1_bound_sums_over_components():
    """Proposition 1: L = rho(X^T W X)/n <= max(w) sum_r prod_j rho(X_rj^T X_rj) / n; with two
    copies of one component and W = I, X^T X has the spectrum of 2 X_1^T X_1, so the bound is
    attained."""
    d = inputs.random_components_problem((6, 5, 4), [(3, 2, 2), (2, 3, 3)], seed=12)
    C = O.Components(d.comps)
    D = _concatenated_design(d.comps)
    n = D.shape[0]
    w = np.random.default_rng(6).uniform(0.2, 2.0, n)
    L = float(np.linalg.eigvalsh(D.T @ (w[:, None] * D))[-1]) / n
    assert L <= O.lipschitz_bound(C, w, n) * (1 + 1e-12)
    dup = O.Components([d.comps[0], d.comps[0]])
    Dd = _concatenated_design(dup.__iter__())
    Ld = float(np.linalg.eigvalsh(Dd.T @ Dd)[-1]) / n
    np.testing.assert_allclose(O.lipschitz_bound(dup, np.ones(n), n), Ld, rtol=1e-10)


def test_components_gaussian_matches_coordinate_descent():
    """GD-PG on a c = 2 model vs textbook CD on the concatenated explicit design."""
    d = inputs.random_components_problem((8, 7, 6), [(3, 3, 2), (2, 2, 3)], seed=13)
    C = O.Components(d.comps)
    D = _concatenated_design(d.comps)
    y = O.vec(d.Y)
    lm = O.lambda_max("gaussian", C, d.Y)
    np.testing.assert_allclose(lm, np.max(np.abs(D.T @ y)) / y.size, rtol=1e-12)
    for frac in [0.3, 0.02]:
        lam = frac * lm
        th, info = O.gdpg("gaussian", C, d.Y, lam, lm, tol=1e-12)
        assert info.converged
        cd = O.cd_weighted_lasso(D, y, np.ones_like(y), lam, tol=1e-15)
        np.testing.assert_allclose(th, cd, atol=1e-8 * np.max(np.abs(cd)))


def test_components_poisson_matches_prox_newton():
    """Poisson c = 2 with prior weights: GD-PG vs proximal Newton on the explicit design."""
    d = inputs.random_components_problem((7, 6, 5), [(2, 3, 2), (3, 2, 2)], family="poisson", seed=14,
                                         obs_weights=True)
    C = O.Components(d.comps)
    lm = O.lambda_max("poisson", C, d.Y, a=d.a)
    lam = 0.1 * lm
    th, info = O.gdpg("poisson", C, d.Y, lam, lm, a=d.a, tol=1e-10)
    assert info.converged
    ref = O.poisson_lasso_explicit(C, d.Y, lam, a=d.a)
    np.testing.assert_allclose(th, ref, atol=1e-7 * max(1.0, np.max(np.abs(ref))))


def test_duplicated_component_ridge_splits_evenly():
    """Two copies of one component under the ridge penalty: for a fixed sum s = theta_1 + theta_2
    the penalty lambda (|theta_1|^2 + |theta_2|^2) is least at theta_1 = theta_2 = s/2, where it is
    (lambda/2) |s|^2, so each half is half the single-component ridge fit at lambda/2."""
    d = inputs.random_components_problem((7, 6, 5), [(3, 2, 2)], family="poisson", seed=15)
    one = d.comps
    dup = O.Components([one[0], one[0]])
    lm = O.lambda_max("poisson", one[0], d.Y)
    lam = 0.05 * lm
    th2, info2 = O.gdpg("poisson", dup, d.Y, lam, lm, tol=1e-11, alpha=1.0, l1=0.0)
    th1, info1 = O.gdpg("poisson", one[0], d.Y, lam / 2, lm, tol=1e-11, alpha=1.0, l1=0.0)
    assert info1.converged and info2.converged
    half = O.vec(th1) / 2
    k = half.size
    np.testing.assert_allclose(th2[:k], half, atol=1e-8 * np.max(np.abs(half)))
    np.testing.assert_allclose(th2[k:], half, atol=1e-8 * np.max(np.abs(half)))
