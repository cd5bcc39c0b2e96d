"""Seeded synthetic inputs for the GLAM lasso path (shared by tests, bench and smoke).

This module only *generates data*: marginal B-spline design matrices, response
arrays and observation weights.  It holds none of the solver's arithmetic (no
rho/H/G map, no family update, no prox, no line search), so the oracle and the
HIP path can both read from it without sharing any of the method.

Conventions
-----------
* Arrays are column-major ("vec" of App. A, eq. (index)): the first index runs
  fastest.  Every array returned here is a C-contiguous NumPy array whose
  *Fortran-order* flattening is the paper's vec, i.e. ``A.reshape(-1, order="F")``.
  We therefore store response arrays with ``np.asfortranarray``.
* Grids are equispaced on [0, 1] (Section 4.1, the smoothing model).
* Marginal factors are clamped (open-uniform) cubic B-spline bases with
  ``p - 3`` equal knot intervals on [0, 1] (Section 4.1; the paper leaves the
  knot placement to the cited literature).
* Seeds: configuration c uses ``numpy.random.default_rng(1510032980 + c)``.

The synthetic signal of the Gaussian configurations is evaluated directly on the
grid from the basis functions (a data-generating process, never used as an
expected value by any test).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

SEED_BASE = 1510032980


# ----------------------------------------------------------------------------
# B-spline bases (Section 4.1: tensor-product B-spline smoothing model)
# ----------------------------------------------------------------------------
def clamped_knots(p: int, degree: int = 3) -> np.ndarray:
    """Open-uniform knot vector on [0, 1] giving ``p`` basis functions."""
    if p < degree + 1:
        raise ValueError(f"need p >= {degree + 1} basis functions, got {p}")
    n_int = p - degree
    inner = np.linspace(0.0, 1.0, n_int + 1)
    return np.concatenate([np.zeros(degree), inner, np.ones(degree)])


def bspline_basis(x: np.ndarray, p: int, degree: int = 3) -> np.ndarray:
    """Evaluate the ``p`` clamped B-splines of the given degree at ``x``.

    Cox-de Boor recursion on half-open knot spans; the right end point x = 1
    is assigned to the last non-degenerate span so that rows still sum to one.
    Returns a ``len(x) x p`` float64 matrix.
    """
    x = np.asarray(x, dtype=np.float64)
    t = clamped_knots(p, degree)
    m = len(t) - 1  # number of knot spans
    # degree-0 indicator functions
    B = np.zeros((x.size, m))
    for i in range(m):
        lo, hi = t[i], t[i + 1]
        if hi > lo:
            B[:, i] = (x >= lo) & (x < hi)
    last = np.max(np.nonzero(t[1:] > t[:-1])[0])
    B[x >= t[-1], :] = 0.0
    B[x >= t[-1], last] = 1.0
    for k in range(1, degree + 1):
        Bn = np.zeros((x.size, m - k))
        for i in range(m - k):
            d1 = t[i + k] - t[i]
            d2 = t[i + k + 1] - t[i + 1]
            term = np.zeros(x.size)
            if d1 > 0:
                term += (x - t[i]) / d1 * B[:, i]
            if d2 > 0:
                term += (t[i + k + 1] - x) / d2 * B[:, i + 1]
            Bn[:, i] = term
        B = Bn
    assert B.shape[1] == p
    return B


def grid(n: int) -> np.ndarray:
    return np.linspace(0.0, 1.0, n)


def basis_count(n_j: int, k: int) -> int:
    """Basis-count rule p_j = max{ceil(n_j / k), 5} of Section 4.2.

    The bracket in the paper is read as the ceiling: it is the only rounding
    that reproduces the printed parameter-array sizes (977/5 -> 196,
    33/4 -> 9, 81/4 -> 21, 168/4 -> 42).
    """
    return max(int(math.ceil(n_j / k)), 5)


# ----------------------------------------------------------------------------
# Problem container
# ----------------------------------------------------------------------------
@dataclass
class GlamData:
    name: str
    family: str                    # "gaussian" | "poisson" | "binomial" | "gamma"
    X: List[np.ndarray]            # X[j] is n_j x p_j, float64, C-contiguous
    Y: np.ndarray                  # n1 x n2 x n3 float64 (Fortran order)
    a: Optional[np.ndarray] = None  # observation weights (None: all ones)
    pen_w: Optional[np.ndarray] = None  # p1 x p2 x p3 penalty weights (None: ones)
    nlambda: int = 1
    lambda_min_ratio: float = 0.1
    single_lambda_ratio: Optional[float] = None  # one lambda = ratio * lambda_max
    theta_true: Optional[np.ndarray] = None
    extra: dict = field(default_factory=dict)

    @property
    def n(self):
        return tuple(int(x.shape[0]) for x in self.X)

    @property
    def p(self):
        return tuple(int(x.shape[1]) for x in self.X)


def _bases(n, p):
    return [np.ascontiguousarray(bspline_basis(grid(nj), pj)) for nj, pj in zip(n, p)]


def _signal_from_coefficients(X, theta):
    """Evaluate sum_m theta_m phi_m on the grid (data generation only)."""
    f = np.einsum("ia,jb,kc,abc->ijk", X[0], X[1], X[2], theta, optimize=True)
    return np.asfortranarray(f)


# ----------------------------------------------------------------------------
# Workloads (shapes and distributions of the paper's smoothing examples)
# ----------------------------------------------------------------------------
def config_c1() -> GlamData:
    """Gaussian, n=(20,20,20), p=(8,8,8), 10 % nonzero N(0,1) coefficients,
    noise N(0, 0.5^2), one lambda = 0.1 lambda_max."""
    rng = np.random.default_rng(SEED_BASE + 1)
    n, p = (20, 20, 20), (8, 8, 8)
    X = _bases(n, p)
    P = int(np.prod(p))
    k = int(round(0.1 * P))
    theta = np.zeros(P)
    idx = rng.choice(P, size=k, replace=False)
    theta[idx] = rng.standard_normal(k)
    theta = theta.reshape(p, order="F")
    Y = _signal_from_coefficients(X, theta) + 0.5 * rng.standard_normal(n)
    return GlamData("c1_gauss_20x20x20", "gaussian", X, np.asfortranarray(Y),
                    nlambda=1, single_lambda_ratio=0.1, theta_true=theta)


def _bumps(rng, K=5):
    c = rng.uniform(0.15, 0.85, size=(K, 2))
    s = rng.uniform(0.05, 0.15, size=K)
    return c, s


def config_c2(n=(100, 100, 1000), p=(30, 30, 200), nlambda=100, ratio=1e-4) -> GlamData:
    """Gaussian spatio-temporal smoothing: 5 Gaussian bumps in space times a
    sinusoid in time, N(0,1) noise; 100-value log grid to 1e-4 lambda_max."""
    rng = np.random.default_rng(SEED_BASE + 2)
    X = _bases(n, p)
    c, s = _bumps(rng)
    A = rng.uniform(1.0, 3.0, size=5)
    nu = rng.integers(1, 6, size=5)
    phi = rng.uniform(0.0, 2 * np.pi, size=5)
    x1, x2, t = grid(n[0]), grid(n[1]), grid(n[2])
    f = np.zeros(n)
    for k in range(5):
        sp = np.exp(-((x1[:, None] - c[k, 0]) ** 2 + (x2[None, :] - c[k, 1]) ** 2) / (2 * s[k] ** 2))
        tm = np.sin(2 * np.pi * nu[k] * t + phi[k])
        f += A[k] * sp[:, :, None] * tm[None, None, :]
    Y = f + rng.standard_normal(n)
    return GlamData("c2_gauss_100x100x1000", "gaussian", X, np.asfortranarray(Y),
                    nlambda=nlambda, lambda_min_ratio=ratio)


def config_c3(n=(64, 64, 365), p=(24, 24, 120), nlambda=50, ratio=1e-4, mean_count=5.0) -> GlamData:
    """Poisson counts: log-intensity = offset + 5 spatial bumps + weekly term,
    scaled to mean count 5; 50-value log grid to 1e-4 lambda_max."""
    rng = np.random.default_rng(SEED_BASE + 3)
    X = _bases(n, p)
    c, s = _bumps(rng)
    A = rng.uniform(0.5, 1.5, size=5)
    x1, x2 = grid(n[0]), grid(n[1])
    day = np.arange(n[2], dtype=np.float64)
    g = np.zeros(n)
    for k in range(5):
        sp = np.exp(-((x1[:, None] - c[k, 0]) ** 2 + (x2[None, :] - c[k, 1]) ** 2) / (2 * s[k] ** 2))
        g += A[k] * sp[:, :, None]
    g = g + 0.3 * np.sin(2 * np.pi * day / 7.0)[None, None, :]
    b0 = math.log(mean_count) - math.log(np.mean(np.exp(g)))
    mu = np.exp(b0 + g)
    Y = rng.poisson(mu).astype(np.float64)
    return GlamData("c3_poisson_64x64x365", "poisson", X, np.asfortranarray(Y),
                    nlambda=nlambda, lambda_min_ratio=ratio)


def config_c4(nprob=256, lo=16, hi=96, seed_offset=4) -> List[GlamData]:
    """256 independent GLAMs of uneven size: n_ij ~ U{16..96}, p_ij = round(n_ij/4),
    even index Gaussian, odd Poisson, 5-20 % nonzero coefficients, lambda = 0.1 lambda_max."""
    rng = np.random.default_rng(SEED_BASE + seed_offset)
    probs = []
    for i in range(nprob):
        n = tuple(int(v) for v in rng.integers(lo, hi + 1, size=3))
        p = tuple(max(4, int(math.floor(v / 4 + 0.5))) for v in n)
        X = _bases(n, p)
        P = int(np.prod(p))
        sfrac = rng.uniform(0.05, 0.20)
        k = max(1, int(round(sfrac * P)))
        theta = np.zeros(P)
        idx = rng.choice(P, size=k, replace=False)
        gauss = (i % 2 == 0)
        theta[idx] = rng.standard_normal(k) * (1.0 if gauss else 0.5)
        theta = theta.reshape(p, order="F")
        eta = _signal_from_coefficients(X, theta)
        if gauss:
            Y = eta + rng.standard_normal(n)
            fam = "gaussian"
        else:
            Y = rng.poisson(np.exp(eta)).astype(np.float64)
            fam = "poisson"
        probs.append(GlamData(f"c4_{i}", fam, X, np.asfortranarray(Y), nlambda=1,
                              single_lambda_ratio=0.1, theta_true=theta))
    return probs


def config_c5(n=(128, 128, 256), p=(32, 32, 64)) -> GlamData:
    """Poisson NLL evaluation point: beta_true = log 5 + N(0, 0.3^2),
    Y ~ Poisson(exp(X beta_true)), evaluated at beta_true + N(0, 0.05^2)."""
    rng = np.random.default_rng(SEED_BASE + 5)
    X = _bases(n, p)
    beta_true = math.log(5.0) + 0.3 * rng.standard_normal(p)
    eta = _signal_from_coefficients(X, beta_true)
    Y = rng.poisson(np.exp(eta)).astype(np.float64)
    beta = beta_true + 0.05 * rng.standard_normal(p)
    return GlamData("c5_poisson_nll_128x128x256", "poisson", X, np.asfortranarray(Y),
                    theta_true=beta_true, extra={"beta": np.asfortranarray(beta)})


def config_sim(r=3, q=0.5, family="gaussian", kappa=0.25, seed=6, nlambda=100, ratio=1e-4) -> GlamData:
    """The simulated design of Section 6.5: n = (60r, 20r, 10r), p_j = max(3, n_j q), rows
    of X_j i.i.d. N(0, Sigma) with Sigma = (sigma - kappa) I + kappa 1 1^T,
    theta_m = (-1)^m exp(-(m - 1)/10) B_m with B_m ~ Bernoulli(s).  Gaussian: sigma = 1,
    s = 1, unit noise; Poisson: sigma = 0.71, s = 0.01.

    The modes are listed with the largest last: (20r, 10r, 60r).  A GLAM is unchanged by a
    joint permutation of its modes, Y's axes and Theta's axes, and the solver's slab
    kernel takes the two smaller modes (p_j <= 32 there, hence r <= 3 at q = 0.5; the
    p > n designs, q = 3, run on the generic GEMM chain).  The coefficient index m runs over
    the permuted array in vec order."""
    rng = np.random.default_rng(SEED_BASE + seed)
    n_paper = (60 * r, 20 * r, 10 * r)
    order = (1, 2, 0)
    n = tuple(n_paper[j] for j in order)
    p = tuple(max(3, int(round(nj * q))) for nj in n)
    gaussian = family == "gaussian"
    sigma, s = (1.0, 1.0) if gaussian else (0.71, 0.01)
    X = []
    for nj, pj in zip(n, p):
        # a row of N(0, Sigma) drawn exactly as sqrt(sigma - kappa) z + sqrt(kappa) w 1 (z ~ N(0, I),
        # w ~ N(0, 1)): no matrix factorisation, whose eigenbasis for the repeated eigenvalue
        # sigma - kappa would depend on the BLAS threading
        z = rng.standard_normal((nj, pj))
        w = rng.standard_normal((nj, 1))
        X.append(np.ascontiguousarray(np.sqrt(sigma - kappa) * z + np.sqrt(kappa) * w))
    P = int(np.prod(p))
    m = np.arange(1, P + 1)
    B = rng.uniform(size=P) < s
    theta = np.asfortranarray(((-1.0) ** m * np.exp(-(m - 1) / 10.0) * B).reshape(p, order="F"))
    eta = _signal_from_coefficients(X, theta)
    if gaussian:
        Y = eta + rng.standard_normal(n)
    else:
        Y = rng.poisson(np.exp(np.clip(eta, -30, 30))).astype(np.float64)
    return GlamData(f"sim65_{family}_r{r}_q{q}_k{kappa}", family, X, np.asfortranarray(Y), nlambda=nlambda,
                    lambda_min_ratio=ratio, theta_true=theta)


def random_problem(n, p, family="gaussian", seed=0, sparsity=0.2, noise=0.5, basis="bspline",
                   obs_weights=False, scale=1.0) -> GlamData:
    """Small seeded problem for parity tests.

    basis="bspline": clamped cubic B-splines (needs p_j >= 4);
    basis="gauss": i.i.d. N(0,1) entries (the simulated design of Section 6.5);
    basis="orth": sqrt(n_j) * Q_j with orthonormal columns Q_j (needs p_j <= n_j).
    """
    rng = np.random.default_rng(SEED_BASE + 1000 + seed)
    X = []
    for nj, pj in zip(n, p):
        if basis == "bspline":
            X.append(np.ascontiguousarray(bspline_basis(grid(nj), pj)))
        elif basis == "gauss":
            X.append(np.ascontiguousarray(rng.standard_normal((nj, pj))))
        elif basis == "orth":
            q, _ = np.linalg.qr(rng.standard_normal((nj, pj)))
            X.append(np.ascontiguousarray(math.sqrt(nj) * q))
        else:
            raise ValueError(basis)
    P = int(np.prod(p))
    theta = np.zeros(P)
    k = max(1, int(round(sparsity * P)))
    idx = rng.choice(P, size=k, replace=False)
    theta[idx] = scale * rng.standard_normal(k)
    theta = theta.reshape(p, order="F")
    eta = _signal_from_coefficients(X, theta)
    if family == "gaussian":
        Y = eta + noise * rng.standard_normal(n)
    elif family == "poisson":
        Y = rng.poisson(np.exp(np.clip(eta, -20, 5))).astype(np.float64)
    elif family == "binomial":   # Bernoulli responses with success probability 1 / (1 + e^-eta)
        Y = (rng.uniform(size=n) < 1.0 / (1.0 + np.exp(-np.clip(eta, -30, 30)))).astype(np.float64)
    elif family == "gamma":      # Gamma responses of shape 2 and mean e^eta
        Y = rng.gamma(2.0, 0.5 * np.exp(np.clip(eta, -5, 5)))
    else:
        raise ValueError(family)
    a = None
    if obs_weights:
        a = rng.uniform(0.5, 1.5, size=n)
        a[rng.uniform(size=n) < 0.1] = 0.0
        a = np.asfortranarray(a)
    return GlamData(f"rand_{family}_{n}_{p}_{seed}", family, X, np.asfortranarray(Y), a=a,
                    theta_true=theta)


@dataclass
class GlamMultiData:
    """A model of c tensor components (Sec. 2): comps[r] = [X_{r,1}, ..., X_{r,d}]."""
    name: str
    family: str
    comps: List[List[np.ndarray]]
    Y: np.ndarray
    a: Optional[np.ndarray] = None
    theta_true: Optional[np.ndarray] = None   # flat: (vec(Theta_1), ..., vec(Theta_c))

    @property
    def n(self):
        return tuple(int(x.shape[0]) for x in self.comps[0])

    @property
    def ps(self):
        return [tuple(int(x.shape[1]) for x in Xs) for Xs in self.comps]


def random_components_problem(n, ps, family="gaussian", seed=0, sparsity=0.3, noise=0.5, obs_weights=False,
                              scale=0.5) -> GlamMultiData:
    """Small seeded c-component problem: component r has i.i.d. N(0, 1) factors of sizes
    n_j x ps[r][j] (d = len(n)) and a sparse coefficient array; Y is drawn around the sum of the
    components' signals (evaluated on the grid, data generation only)."""
    rng = np.random.default_rng(SEED_BASE + 3000 + seed)
    d = len(n)
    comps, thetas = [], []
    signal = np.zeros(tuple(n))
    letters = "abc"[:d]
    for p in ps:
        Xs = [np.ascontiguousarray(rng.standard_normal((nj, pj))) for nj, pj in zip(n, p)]
        P = int(np.prod(p))
        th = np.zeros(P)
        k = max(1, int(round(sparsity * P)))
        th[rng.choice(P, size=k, replace=False)] = scale * rng.standard_normal(k)
        T = th.reshape(p, order="F")
        spec = ",".join(f"{'ijk'[j]}{letters[j]}" for j in range(d)) + "," + letters + "->" + "ijk"[:d]
        signal = signal + np.einsum(spec, *Xs, T, optimize=True)
        comps.append(Xs)
        thetas.append(th)
    eta = signal
    if family == "gaussian":
        Y = eta + noise * rng.standard_normal(tuple(n))
    elif family == "poisson":
        Y = rng.poisson(np.exp(np.clip(eta, -20, 4))).astype(np.float64)
    elif family == "binomial":
        Y = (rng.uniform(size=tuple(n)) < 1.0 / (1.0 + np.exp(-np.clip(eta, -30, 30)))).astype(np.float64)
    elif family == "gamma":
        Y = rng.gamma(2.0, 0.5 * np.exp(np.clip(eta, -5, 5)))
    else:
        raise ValueError(family)
    a = None
    if obs_weights:
        a = rng.uniform(0.5, 1.5, size=tuple(n))
        a[rng.uniform(size=tuple(n)) < 0.1] = 0.0
        a = np.asfortranarray(a)
    return GlamMultiData(f"comp_{family}_{tuple(n)}_{len(ps)}_{seed}", family, comps, np.asfortranarray(Y), a=a,
                         theta_true=np.concatenate(thetas))
