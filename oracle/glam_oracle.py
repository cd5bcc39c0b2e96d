"""CPU FP64 oracle for l1-penalised generalized linear array models (GLAMs).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or call anything in ``oracle/``.
The product path (the HIP library and its Python binding) never touches it.

It is a plain, slow, obviously-correct NumPy implementation of what the paper
(Lund, Vincent & Hansen, "Penalized estimation in large-scale generalized
linear array models", arXiv:1510.03298) computes, written from the paper's
definitions in the paper's notation:

* vec / rho / Kronecker identity ............ App. A (eq. "index", the rho map)
* H and G maps .............................. Sec. 6.1, eqs. (eighteen), (nineteen)
* c > 1 tensor components ................... Sec. 2, eq. (fivenew): H sums the components'
                                              chains, G stacks their adjoints as theta is
                                              stacked, Proposition 1 sums over components
* exponential families, score, weights ...... App. B, eqs. (four), (weights), (tennew)
* log-likelihood and gradient ............... Sec. 2, eqs. (two), (three)
* PMLE objective ............................ Sec. 2, eq. (five)
* outer GD loop ............................. Sec. 3.1, eqs. (ten), (eleven)
* inner PG loop (FISTA extrapolation) ....... Sec. 3.2, eqs. (twentyfour), (twentyfive)
* GD-PG ..................................... Sec. 3.3, Algorithm 1 (GD-PG)
* Lipschitz bound ........................... Sec. 5, Proposition 1
* Armijo rule ............................... Sec. 5 (Tseng-Yun step size, before Thm. 2)
* proximal operators ........................ Sec. 6.3
* lambda path with warm starts .............. Sec. 6.4 (glamlasso package description)
* SCAD via the multi-step adaptive lasso .... Sec. 6.4 (penalty, steps); SCAD is Fan and Li's

Readings of places where the paper is silent or ambiguous (listed again in the
design notes):

R1  objective scale: F = -l/n + lambda J (the 1/n of eqs. (eleven), (twentyfour)
    carried to the objective; lambda_max, Delta_k, Armijo F and KKT all use it).
R2  prior weights a_i enter the score (eq. four) and the working response
    (eq. tennew) but not the IRLS weights (eq. nine), exactly as printed.
R3  lambda grid: log-spaced from lambda_max down to ratio * lambda_max.
R4  inner stopping rule: inner KKT residual of h + lambda J at x^{l+1}
    <= max(0.1 tol, 0.1 KKT(theta^k)); for the Gaussian family with a = 1 the
    model is exact and there is no outer loop (Sec. 6.5), so the inner loop
    runs to 0.5 tol and one outer pass suffices.
R5  Armijo constants alpha_0 = 1, b = 0.5, v = 0.1; a non-finite F fails a trial.
    The test is evaluated on the change F(theta + t d) - F(theta), summed
    entrywise, instead of on two totals (same inequality, no cancellation).
R6  KKT residual (convergence criterion of Alg. 1): with g the gradient of -l/n,
    r_m = |g_m + lambda w_m sign(theta_m)| for theta_m != 0, else
    max(|g_m| - lambda w_m, 0); KKT = max_m r_m / lambda_max.
R7  nu in (0,1): delta = 1/(nu Lhat) with Beck-Teboulle sufficient-decrease
    backtracking (halve delta, never below 1/Lhat) when the test fails.
R9  soft threshold gives exactly 0 at |z| = t; sign(0) = 0.
R12 no intercept (the paper's model has none).
R13 the Gaussian objective keeps the y^2/2 term of the log-density, i.e.
    -l/n = (1/2n) sum a (y - eta)^2 (does not move the minimiser).
R16 families beyond Gaussian and Poisson (Sec. 6.4 lists Binomial-logit and Gamma-log):
    Binomial responses are proportions in [0, 1]; Gamma has dispersion 1 and
    y > 0.  The IRLS weight is eq. (nine) as printed, vartheta'(eta) (g^{-1})'(eta):
    mu (1 - mu) for the logit, and exactly 1 for the Gamma-log model (Fisher
    scoring, a non-canonical link), so Gamma shares the Gaussian's unit weights
    but not its exact quadratic model.
R18 tensor-product weights (Sec. 6.2): V-hat = Vbar * prod_j v_j with the paper's
    geometric-mean factors v_j; the displayed product omits Vbar, without which V-hat
    would not reproduce a V that is already a tensor product.  W = V-hat enters the outer
    loop through eq. (ten) (z = W^{-1} u + eta), so the model's gradient at theta^k is
    exact and only its curvature is approximated; Lhat is Proposition 1 with max V-hat.
R17 SCAD (Sec. 6.4): Fan and Li's penalty with a = 3.7; MSA-lasso step 1 is the lasso
    (with the caller's penalty weights), each further step the weighted lasso with
    w_m = pen_w_m p'_lambda(|theta_m|) / lambda at the previous step's estimate.  The
    lambda grid and the KKT scale are the lasso's (lambda_max of step 1); the reported
    KKT residual and objective are those of the last step's weighted lasso.
R21 ridge penalty (Sec. 6.3): J(theta) = sum_m w_m theta_m^2, prox z / (1 + 2 gamma w_m); it has
    no zero solution, so the lambda grid and the KKT scale are the lasso's lambda_max.
R22 nu = 0 (Sec. 6.4): the inner step starts at delta = 1 (not relative to Lhat) and the
    Beck-Teboulle test runs every iteration, halving delta on failure (never below 1/Lhat).
R15 elastic net (Sec. 6.3): J(theta) = sum_m w_m (|theta_m| + alpha theta_m^2), the
    penalty weights scaling both terms; its prox is the soft threshold divided by
    1 + 2 alpha gamma w_m, lambda_max is the lasso's (the quadratic term has zero
    slope at 0), and the KKT residual adds 2 alpha lambda w_m theta_m to the gradient.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np


# =============================================================================
# App. A: vec and rho
# =============================================================================
def vec(A: np.ndarray) -> np.ndarray:
    """vec of App. A: column-major flattening (first index fastest)."""
    return np.asarray(A).reshape(-1, order="F")


def unvec(v: np.ndarray, dims: Sequence[int]) -> np.ndarray:
    return np.asarray(v).reshape(tuple(dims), order="F")


def linear_index(idx: Sequence[int], dims: Sequence[int]) -> int:
    """eq. (index) with 1-based i_j: [i_1..i_d] = i_1 + n_1((i_2-1) + n_2(...))."""
    out = 0
    for j in reversed(range(len(dims))):
        out = out * dims[j] + (idx[j] - 1)
    return out + 1


def rho(X: np.ndarray, A: np.ndarray) -> np.ndarray:
    """The rho map of App. A.

    X is r x n_1, A is n_1 x ... x n_d; the result is n_2 x ... x n_d x r with
    rho(X, A)[i_1, ..., i_d] = sum_j X[i_d, j] A[j, i_1, ..., i_{d-1}]
    (mode 1 of A is contracted and the new mode is appended last).
    """
    X = np.asarray(X, dtype=np.float64)
    A = np.asarray(A, dtype=np.float64)
    if X.shape[1] != A.shape[0]:
        raise ValueError("rho: X has %d columns, A has %d rows" % (X.shape[1], A.shape[0]))
    return np.tensordot(A, X, axes=([0], [1]))


def rho_loops(X: np.ndarray, A: np.ndarray) -> np.ndarray:
    """rho written as the defining sum with explicit loops (tiny inputs only)."""
    X = np.asarray(X, dtype=np.float64)
    A = np.asarray(A, dtype=np.float64)
    r, n1 = X.shape
    rest = A.shape[1:]
    out = np.zeros(tuple(rest) + (r,))
    for idx in np.ndindex(*(tuple(rest) + (r,))):
        i_d = idx[-1]
        lead = idx[:-1]
        s = 0.0
        for j in range(n1):
            s += X[i_d, j] * A[(j,) + lead]
        out[idx] = s
    return out


class Components(list):
    """A design of c tensor components, X = [X_1 | ... | X_c] with X_r = X_{r,d} (x) ... (x) X_{r,1}
    (Sec. 2, eq. fivenew): Components([Xs_1, ..., Xs_c]), Xs_r the list of component r's marginal
    matrices.  Its parameter is the flat p-vector theta = (vec(Theta_1), ..., vec(Theta_c)),
    p = sum_r prod_j p_{r,j}.  A plain list of matrices is the single-component design (c = 1)."""

    def dims(self):
        return [tuple(np.asarray(X).shape[1] for X in Xs) for Xs in self]

    def split(self, theta):
        """The arrays Theta_r of a flat theta."""
        th = vec(theta)
        out, off = [], 0
        for dims in self.dims():
            k = int(np.prod(dims))
            out.append(unvec(th[off:off + k], dims))
            off += k
        if off != th.size:
            raise ValueError("theta has %d entries, the components %d" % (th.size, off))
        return out


def param_shape(Xs) -> tuple:
    """Shape of the parameter: (p_1, ..., p_d) for one component, (p,) for Components."""
    if isinstance(Xs, Components):
        return (sum(int(np.prod(d)) for d in Xs.dims()),)
    return tuple(np.asarray(X).shape[1] for X in Xs)


def H(Xs: Sequence[np.ndarray], Theta: np.ndarray) -> np.ndarray:
    """H map, eq. (eighteen): rho(X_d, ..., rho(X_1, Theta)), summed over the components of a
    Components design."""
    if isinstance(Xs, Components):
        return sum(H(Xr, Tr) for Xr, Tr in zip(Xs, Xs.split(Theta)))
    out = np.asarray(Theta, dtype=np.float64)
    for X in Xs:
        out = rho(X, out)
    return out


def G(Xs: Sequence[np.ndarray], U: np.ndarray) -> np.ndarray:
    """G map, eq. (nineteen): rho(X_d^T, ..., rho(X_1^T, U)); for a Components design the tuple
    of the components' arrays, stacked as theta is (vec of each, in component order)."""
    if isinstance(Xs, Components):
        return np.concatenate([vec(G(Xr, U)) for Xr in Xs])
    out = np.asarray(U, dtype=np.float64)
    for X in Xs:
        out = rho(np.asarray(X).T, out)
    return out


def kron_design(Xs: Sequence[np.ndarray]) -> np.ndarray:
    """Explicit design X = X_d (x) ... (x) X_1, eq. (fivenew), and [X_1 | ... | X_c] for a
    Components design (tiny inputs only)."""
    if isinstance(Xs, Components):
        return np.hstack([kron_design(Xr) for Xr in Xs])
    D = np.ones((1, 1))
    for X in Xs:
        D = np.kron(np.asarray(X, dtype=np.float64), D)
    return D


def gram_apply(Xs: Sequence[np.ndarray], D: np.ndarray) -> np.ndarray:
    """X^T X vec(D) for a tensor-product design, taken as the three p-sized mode
    products with the Gram factors X_j^T X_j (Sec. 6.2: with identity weights the
    weighted Gram matrix of the array design is the Kronecker product of the
    factors' Gram matrices, by the mixed-product property of App. A)."""
    out = np.asarray(D, dtype=np.float64)
    for X in Xs:
        S = np.asarray(X, dtype=np.float64).T @ np.asarray(X, dtype=np.float64)
        out = rho(S, out)
    return out


def rho_chain_flops(n: Sequence[int], p: Sequence[int], order: Sequence[int]) -> int:
    """Multiply-add count (x2) of applying the factors one mode at a time in
    ``order`` (0-based modes) to a p-array, i.e. the cost of the H map when the
    mode products are taken in that order (Sec. 2, cost of the array product)."""
    dims = list(p)
    total = 0
    for j in order:
        others = int(np.prod([dims[k] for k in range(len(dims)) if k != j]))
        total += 2 * others * n[j] * p[j]
        dims[j] = n[j]
    return total


# =============================================================================
# App. B: exponential families.  Gaussian-identity, Poisson-log and Binomial-logit
# are canonical (vartheta = eta); Gamma-log is not (vartheta = -1/mu).  These four
# are the models the paper's package supports (Sec. 6.4).
# =============================================================================
class Family:
    name = ""

    def ginv(self, eta):            # mean g^{-1}(eta)
        raise NotImplementedError

    def dginv(self, eta):           # (g^{-1})'(eta)
        raise NotImplementedError

    def dtheta(self, eta):          # vartheta'(eta)
        raise NotImplementedError

    def gprime(self, mu):           # g'(mu)
        raise NotImplementedError

    def theta(self, eta):           # vartheta(eta)
        raise NotImplementedError

    def b(self, th):                # log-normaliser b(vartheta)
        raise NotImplementedError

    def c(self, y):                 # y-only part kept in -l (R13)
        return np.zeros_like(y)


class Gaussian(Family):
    """Identity link: vartheta(eta) = eta, b(t) = t^2/2, g^{-1}(eta) = eta."""
    name = "gaussian"

    def ginv(self, eta):
        return eta

    def dginv(self, eta):
        return np.ones_like(eta)

    def dtheta(self, eta):
        return np.ones_like(eta)

    def gprime(self, mu):
        return np.ones_like(mu)

    def theta(self, eta):
        return eta

    def b(self, th):
        return 0.5 * th * th

    def c(self, y):
        return 0.5 * y * y


class Poisson(Family):
    """Log link (canonical): vartheta(eta) = eta, b(t) = e^t, g^{-1}(eta) = e^eta."""
    name = "poisson"

    def ginv(self, eta):
        return np.exp(eta)

    def dginv(self, eta):
        return np.exp(eta)

    def dtheta(self, eta):
        return np.ones_like(eta)

    def gprime(self, mu):
        return 1.0 / mu

    def theta(self, eta):
        return eta

    def b(self, th):
        return np.exp(th)


def _softplus(t):
    """log(1 + e^t) without overflow."""
    return np.logaddexp(0.0, t)


class Binomial(Family):
    """Logit link (canonical): vartheta(eta) = eta, b(t) = log(1 + e^t),
    g^{-1}(eta) = 1 / (1 + e^-eta); responses are proportions y in [0, 1]
    (a binomial count out of m trials enters as y = count / m with a = m)."""
    name = "binomial"

    def ginv(self, eta):
        return 0.5 * (1.0 + np.tanh(0.5 * eta))

    def dginv(self, eta):
        mu = self.ginv(eta)
        return mu * (1.0 - mu)

    def dtheta(self, eta):
        return np.ones_like(eta)

    def gprime(self, mu):
        return 1.0 / (mu * (1.0 - mu))

    def theta(self, eta):
        return eta

    def b(self, th):
        return _softplus(th)


class Gamma(Family):
    """Log link (not canonical): mu = e^eta, vartheta(eta) = -1/mu = -e^-eta,
    b(t) = -log(-t) (dispersion 1; its scale does not move the PMLE's support
    pattern along a lambda path, it rescales lambda).  Responses y > 0."""
    name = "gamma"

    def ginv(self, eta):
        return np.exp(eta)

    def dginv(self, eta):
        return np.exp(eta)

    def dtheta(self, eta):
        return np.exp(-eta)

    def gprime(self, mu):
        return 1.0 / mu

    def theta(self, eta):
        return -np.exp(-eta)

    def b(self, th):
        return -np.log(-th)


FAMILIES = {"gaussian": Gaussian(), "poisson": Poisson(), "binomial": Binomial(), "gamma": Gamma()}


def family(name) -> Family:
    return FAMILIES[name] if isinstance(name, str) else name


def loglik(fam, eta, y, a=None):
    """eq. (two): l(eta) = sum_i a_i (y_i vartheta(eta_i) - b(vartheta(eta_i)))."""
    fam = family(fam)
    a = np.ones_like(y) if a is None else a
    th = fam.theta(eta)
    return float(np.sum(a * (y * th - fam.b(th))))


def neg_loglik_scaled(fam, eta, y, a=None):
    """-l/n (R1), with the Gaussian y^2/2 term kept (R13)."""
    fam = family(fam)
    a = np.ones_like(y) if a is None else a
    n = y.size
    th = fam.theta(eta)
    return float(np.sum(a * (fam.b(th) - y * th + fam.c(y)))) / n


def score(fam, eta, y, a=None):
    """eq. (four): u_i = a_i vartheta'(eta_i) (y_i - g^{-1}(eta_i))."""
    fam = family(fam)
    a = np.ones_like(y) if a is None else a
    return a * fam.dtheta(eta) * (y - fam.ginv(eta))


def irls_weights(fam, eta):
    """eq. (nine) / (weights): w_i = vartheta'(eta_i) (g^{-1})'(eta_i) (no a_i, R2)."""
    fam = family(fam)
    return fam.dtheta(eta) * fam.dginv(eta)


def working_response(fam, eta, y, a=None):
    """eq. (tennew): z_i = a_i (y_i - g^{-1}(eta_i)) g'(g^{-1}(eta_i)) + eta_i."""
    fam = family(fam)
    a = np.ones_like(y) if a is None else a
    mu = fam.ginv(eta)
    return a * (y - mu) * fam.gprime(mu) + eta


def working_response_eq10(u, w, eta):
    """eq. (ten): z = W^{-1} u + eta."""
    return u / w + eta


def kron_weights(V):
    """Sec. 6.2: the tensor-product approximation of a positive weight array V.
    v_j[i] = exp(mean of log V over the other indices at i_j = i, minus log Vbar), with
    Vbar the geometric mean of V; V-hat = Vbar * prod_j v_j[i_j] (R18: the factor Vbar
    makes V-hat = V whenever V is itself a tensor product).  Returns (V-hat, [v_j], Vbar)."""
    L = np.log(V)
    d = V.ndim
    logbar = float(L.mean())
    Vh = np.full(V.shape, math.exp(logbar))
    factors = []
    for j in range(d):
        axes = tuple(k for k in range(d) if k != j)
        vj = np.exp(L.mean(axis=axes) - logbar)
        factors.append(vj)
        shape = [1] * d
        shape[j] = V.shape[j]
        Vh = Vh * vj.reshape(shape)
    return Vh, factors, math.exp(logbar)


# =============================================================================
# Penalty, prox, objective, KKT
# =============================================================================
def penalty(theta, pen_w=None, alpha=0.0, l1=1.0):
    """Weighted penalty J(theta) = sum_m w_m (l1 |theta_m| + alpha theta_m^2): the l1 penalty
    (alpha = 0), the elastic net of Sec. 6.3 (R15: the weights scale both terms), or the ridge
    penalty of Sec. 6.3 (l1 = 0, alpha = 1)."""
    th = vec(theta)
    t = l1 * np.abs(th) + alpha * th * th
    return float(np.sum(t if pen_w is None else vec(pen_w) * t))


def penalty_change(theta_old, theta_new, pen_w=None, alpha=0.0, l1=1.0):
    """J(theta_new) - J(theta_old) summed entrywise (no subtraction of totals)."""
    a, b = vec(theta_old), vec(theta_new)
    dj = l1 * (np.abs(b) - np.abs(a)) + alpha * (b - a) * (b + a)
    return float(np.sum(dj if pen_w is None else vec(pen_w) * dj))


def soft_threshold(z, t):
    """Sec. 6.3: prox of gamma ||.||_1 is (|z| - gamma)_+ sign(z) (R9 at ties)."""
    return np.sign(z) * np.maximum(np.abs(z) - t, 0.0)


def prox_ridge(z, gamma):
    """Sec. 6.3: prox of gamma ||.||_2^2 is z / (1 + 2 gamma)."""
    return z / (1.0 + 2.0 * gamma)


def prox_elastic_net(z, gamma, alpha, l1=1.0):
    """Sec. 6.3: prox of gamma (l1 ||.||_1 + alpha ||.||_2^2): the soft threshold at l1 gamma, then
    the multiplicative shrinkage 1 / (1 + 2 alpha gamma) (l1 = 0: the ridge prox alone)."""
    return soft_threshold(z, l1 * gamma) / (1.0 + 2.0 * alpha * gamma)


def objective(fam, Xs, Theta, Y, lam, a=None, pen_w=None, alpha=0.0, l1=1.0):
    """F = -l/n + lambda J (eq. five under R1)."""
    eta = H(Xs, Theta)
    return neg_loglik_scaled(fam, eta, Y, a) + lam * penalty(Theta, pen_w, alpha, l1)


def objective_change(fam, eta, xd, t, Y, a=None):
    """(-l(eta + t xd) + l(eta)) / n, the change of the smooth part of F along a
    line, written so that no two large totals are subtracted (R5): the Armijo
    test F(theta + t d) <= F(theta) + t v Delta is evaluated as
    [F(theta + t d) - F(theta)] <= t v Delta."""
    fam = family(fam)
    a = np.ones_like(Y) if a is None else a
    s = t * xd
    with np.errstate(over="ignore", invalid="ignore"):
        if fam.name == "gaussian":
            dl = s * (eta + 0.5 * s) - Y * s
        elif fam.name == "poisson":
            dl = np.exp(eta) * np.expm1(s) - Y * s
        elif fam.name == "binomial":
            # b(eta + s) - b(eta) = log(1 + mu (e^s - 1)), mu = g^{-1}(eta); for s < 0 the same
            # identity taken from eta + s back to eta (both arguments of log1p stay >= 0)
            up = np.log1p(fam.ginv(eta) * np.expm1(np.abs(s)))
            dn = -np.log1p(fam.ginv(eta + s) * np.expm1(np.abs(s)))
            dl = np.where(s >= 0, up, dn) - Y * s
        elif fam.name == "gamma":
            # b(vartheta) = eta and -y vartheta = y e^-eta:  s + y e^-eta (e^-s - 1)
            dl = s + Y * np.exp(-eta) * np.expm1(-s)
        else:
            th0, th1 = fam.theta(eta), fam.theta(eta + s)
            dl = (fam.b(th1) - fam.b(th0)) - Y * (th1 - th0)
        return float(np.sum(a * dl)) / Y.size


def smooth_gradient(fam, Xs, Theta, Y, a=None):
    """Gradient of -l/n: -X^T u / n = -G(U)/n (eq. three, eq. nineteen)."""
    eta = H(Xs, Theta)
    return -G(Xs, score(fam, eta, Y, a)) / Y.size


def kkt_residual(Theta, grad, lam, lam_max, pen_w=None, alpha=0.0, l1=1.0):
    """R6: max_m r_m / lambda_max with the subgradient residual r_m of the penalty
    (elastic net: the smooth term's derivative 2 alpha w theta joins the gradient; ridge, l1 = 0:
    r_m = |g_m + 2 lambda w_m theta_m|, the gradient of the smooth objective)."""
    th = vec(Theta)
    g = vec(grad)
    w = np.ones_like(th) if pen_w is None else vec(pen_w)
    nz = th != 0
    gs = g + 2.0 * alpha * lam * w * th
    r = np.where(nz, np.abs(gs + l1 * lam * w * np.sign(th)), np.maximum(np.abs(gs) - l1 * lam * w, 0.0))
    return float(np.max(r)) / lam_max if r.size else 0.0


# =============================================================================
# Step size (Sec. 5, Proposition 1) and lambda path (Sec. 6.4)
# =============================================================================
def spectral_radii(Xs):
    return [float(np.max(np.linalg.eigvalsh(np.asarray(X).T @ np.asarray(X)))) for X in Xs]


def spectral_bound(Xs):
    """Proposition 1's factor sum_r prod_j rho(X_{r,j}^T X_{r,j}) (one term for c = 1)."""
    if isinstance(Xs, Components):
        return float(sum(np.prod(spectral_radii(Xr)) for Xr in Xs))
    return float(np.prod(spectral_radii(Xs)))


def lipschitz_bound(Xs, w, n):
    """Proposition 1: Lhat = max(w) sum_r prod_j rho(X_{r,j}^T X_{r,j}) / n."""
    return float(np.max(w)) * spectral_bound(Xs) / n


def lipschitz_tensor_weights(Xs, factors, n):
    """Sec. 5, after Proposition 1: when the weights form a tensor product W = W_d (x) ... (x) W_1
    (W_j = diag(factors[j])), X^T W X is the tensor product of the X_j^T W_j X_j, so the Lipschitz
    constant of grad h is exactly (1/n) prod_j rho(X_j^T W_j X_j)."""
    return float(np.prod([np.linalg.eigvalsh(np.asarray(X).T @ (np.asarray(v)[:, None] * np.asarray(X)))[-1]
                          for X, v in zip(Xs, factors)])) / n


def lambda_max(fam, Xs, Y, a=None, pen_w=None):
    """Smallest lambda with the zero solution (Sec. 6.4): at theta = 0 the KKT
    conditions read |g_m| <= lambda w_m with g = -G(U(0))/n."""
    fam = family(fam)
    eta0 = np.zeros_like(Y)
    g0 = -G(Xs, score(fam, eta0, Y, a)) / Y.size
    w = np.ones_like(vec(g0)) if pen_w is None else vec(pen_w)
    return float(np.max(np.abs(vec(g0)) / w))


def lambda_grid(lam_max, nlambda, ratio):
    """R3: log-spaced lambda_max > ... > ratio * lambda_max."""
    if nlambda == 1:
        return np.array([lam_max])
    l = np.arange(nlambda)
    return lam_max * ratio ** (l / (nlambda - 1))


# =============================================================================
# Sec. 3.2: inner PG loop; Sec. 3.1 / Alg. 1: outer GD loop with Armijo
# =============================================================================
@dataclass
class FitInfo:
    converged: bool
    kkt: float
    objective: float
    outer: int
    inner: List[int] = field(default_factory=list)
    objective_history: List[float] = field(default_factory=list)
    alphas: List[float] = field(default_factory=list)
    inner_traces: List[list] = field(default_factory=list)


def inner_pg(Xs, V, cz, x0, lam, delta, pen_w, tol_inner, lam_max, max_inner,
             nu=1.0, Lhat=None, Z=None, record=False, alpha=0.0, l1=1.0):
    """Inner PG loop of Sec. 3.2 on h(x) = (1/2n)||sqrt(W)(Xx - z)||^2.

    grad h(x) = G(V * H(x))/n - c_z  with c_z = G(V * Z)/n  (eqs. twentyfive,
    twentyeight, twentysixnew).  Extrapolation omega_l = (l-1)/(l+2), initial
    values x^(0) = x^(1) = x0.  Stops by R4.  With nu < 1 the step starts at
    1/(nu Lhat) and is halved while the Beck-Teboulle sufficient-decrease test
    fails (R7); that test needs h itself, hence the optional Z.
    """
    n = V.size
    w = None if pen_w is None else pen_w

    def grad_h(x):
        return G(Xs, V * H(Xs, x)) / n - cz

    def h_val(x):
        r = H(Xs, x) - Z
        return 0.5 * float(np.sum(V * r * r)) / n

    x_prev = x0.copy()
    x = x0.copy()
    trace = []
    thr_w = 1.0 if w is None else w
    for l in range(1, max_inner + 1):
        om = (l - 1.0) / (l + 2.0)
        y = x + om * (x - x_prev)
        gy = grad_h(y)
        while True:
            x_new = prox_elastic_net(y - delta * gy, delta * lam * thr_w, alpha, l1)
            if nu >= 1.0 or Z is None:
                break
            dlt = x_new - y
            lhs = h_val(x_new)
            rhs = h_val(y) + float(np.sum(gy * dlt)) + float(np.sum(dlt * dlt)) / (2 * delta)
            if lhs <= rhs * (1 + 1e-15) + 1e-300 or delta <= 1.0 / Lhat:
                break
            delta = max(delta / 2.0, 1.0 / Lhat)
        x_prev, x = x, x_new
        gx = grad_h(x)
        r = kkt_residual(x, gx, lam, lam_max, pen_w, alpha, l1)
        if record:
            trace.append(x.copy())
        if r <= tol_inner:
            return x, l, trace
    return x, max_inner, trace


def gdpg(fam, Xs, Y, lam, lam_max, a=None, pen_w=None, theta0=None, tol=1e-10,
         max_outer=100, max_inner=100000, nu=1.0, alpha0=1.0, b=0.5, v=0.1,
         max_ls=60, record_inner=False, alpha=0.0, weights="exact", l1=1.0) -> tuple:
    """GD-PG, Algorithm 1, for one lambda.

    Step 2: eta = H(theta^k); U, V (eq. nine), Z (eq. tennew).  weights="kron": W^(k)
    is the tensor-product approximation V-hat of Sec. 6.2 and Z follows eq. (ten) with
    that W (the outer loop of Sec. 3.1 admits any positive diagonal W^(k); the model's
    gradient at theta^k stays -X^T u / n).  weights="one": W^(k) = I, the special case of
    constant weights named in Sec. 5 after the corollary to Theorem 2 (Z again from eq. (ten)).
    Step 3: delta = 1/(nu Lhat) with Lhat from Proposition 1.
    Step 4: inner PG loop from x^(0) = x^(1) = theta^k.
    Step 5: Armijo rule (alpha_0 b^j, v), Delta_k = -u^T X d / n + lambda (J(theta~) - J(theta)).
    Convergence criterion: R6 KKT residual <= tol at theta^k.
    """
    fam = family(fam)
    n = Y.size
    p = param_shape(Xs)
    theta = np.zeros(p) if theta0 is None else np.array(theta0, dtype=np.float64).reshape(p, order="F")
    s_prod = spectral_bound(Xs)
    info = FitInfo(False, float("inf"), float("nan"), 0)
    for k in range(max_outer + 1):
        eta = H(Xs, theta)
        u = score(fam, eta, Y, a)
        g = -G(Xs, u) / n
        kkt_k = kkt_residual(theta, g, lam, lam_max, pen_w, alpha, l1)
        F_k = neg_loglik_scaled(fam, eta, Y, a) + lam * penalty(theta, pen_w, alpha, l1)
        info.objective_history.append(F_k)
        info.kkt, info.objective, info.outer = kkt_k, F_k, k
        if kkt_k <= tol:
            info.converged = True
            return theta, info
        if k == max_outer:
            break
        V = irls_weights(fam, eta)
        Z = working_response(fam, eta, Y, a)
        if weights == "kron":
            V = kron_weights(V)[0]
            Z = working_response_eq10(u, V, eta)
        elif weights == "one":
            V = np.ones_like(V)
            Z = working_response_eq10(u, V, eta)
        Lhat = float(np.max(V)) * s_prod / n
        delta = 1.0 / (nu * Lhat) if nu > 0 else 1.0
        cz = G(Xs, V * Z) / n
        # R4.  For the Gaussian family with a = 1 the quadratic model h is the
        # smooth part of F itself (w = 1, z = y), so there is no outer loop
        # (Sec. 6.5): the inner loop runs to the final tolerance.
        exact_model = fam.name == "gaussian" and (a is None or bool(np.all(a == 1.0)))
        tol_in = 0.5 * tol if exact_model else max(0.1 * tol, 0.1 * kkt_k)
        x, nin, trace = inner_pg(Xs, V, cz, theta, lam, delta, pen_w, tol_in, lam_max,
                                 max_inner, nu=nu, Lhat=Lhat, Z=Z, record=record_inner, alpha=alpha, l1=l1)
        info.inner.append(nin)
        if record_inner:
            info.inner_traces.append(trace)
        d = x - theta
        xd = H(Xs, d)
        Delta = -float(np.sum(u * xd)) / n + lam * penalty_change(theta, x, pen_w, alpha, l1)
        step = alpha0
        # the rule needs a descent direction (Delta < 0, Sec. 5, Theorem 2's search direction);
        # an inexact inner solve that returns one with Delta >= 0 gives no step
        if not Delta < 0.0:
            step, max_ls = 0.0, 0
        for _ in range(max_ls):
            dF = objective_change(fam, eta, xd, step, Y, a) + lam * penalty_change(
                theta, theta + step * d, pen_w, alpha, l1)
            if np.isfinite(dF) and dF <= step * v * Delta:
                break
            step *= b
        info.alphas.append(step)
        theta = theta + step * d
    return theta, info


def fit_path(fam, Xs, Y, a=None, pen_w=None, lambdas=None, nlambda=100, ratio=1e-4,
             tol=1e-10, max_outer=100, max_inner=100000, nu=1.0, theta0=None,
             max_lambdas=None, alpha=0.0, weights="exact", l1=1.0):
    """lambda path with warm starts (Sec. 6.4).  Returns (lambdas, thetas, infos,
    lam_max).  Stops early, returning the preceding models, when a fit does not
    converge (the packages' early-exit convention, Sec. 6.5).  The ridge penalty (l1 = 0,
    alpha = 1) has no zero solution; its grid and KKT scale are the lasso's lambda_max (R21)."""
    lam_max = lambda_max(fam, Xs, Y, a, pen_w)
    if lambdas is None:
        lambdas = lambda_grid(lam_max, nlambda, ratio)
    lambdas = np.asarray(lambdas, dtype=np.float64)
    if max_lambdas is not None:
        lambdas = lambdas[:max_lambdas]
    p = param_shape(Xs)
    theta = np.zeros(p) if theta0 is None else np.array(theta0, dtype=np.float64).reshape(p, order="F")
    thetas, infos = [], []
    for lam in lambdas:
        theta, info = gdpg(fam, Xs, Y, lam, lam_max, a, pen_w, theta, tol, max_outer, max_inner, nu, alpha=alpha,
                           weights=weights, l1=l1)
        thetas.append(theta.copy())
        infos.append(info)
        if not info.converged:
            break
    return lambdas, thetas, infos, lam_max


# =============================================================================
# Sec. 6.4: the SCAD penalty through the multi-step adaptive lasso (MSA-lasso).
# The SCAD penalty itself is Fan and Li's (the paper cites it, not defines it);
# each step replaces it by its local linear approximation at the previous
# estimate, a weighted l1 problem that Algorithm 1 solves.
# =============================================================================
SCAD_A = 3.7


def scad_penalty(t, lam, a=SCAD_A):
    """Fan-Li SCAD penalty p_lambda(t) for t >= 0: lambda t up to lambda, a quadratic
    joining piece up to a lambda, the constant (a + 1) lambda^2 / 2 beyond."""
    t = np.abs(np.asarray(t, dtype=np.float64))
    mid = (2.0 * a * lam * t - t * t - lam * lam) / (2.0 * (a - 1.0))
    return np.where(t <= lam, lam * t, np.where(t <= a * lam, mid, 0.5 * (a + 1.0) * lam * lam))


def scad_derivative(t, lam, a=SCAD_A):
    """p'_lambda(t) for t >= 0: lambda for t <= lambda, then (a lambda - t)_+ / (a - 1)."""
    t = np.abs(np.asarray(t, dtype=np.float64))
    return np.where(t <= lam, lam, np.maximum(a * lam - t, 0.0) / (a - 1.0))


def msa_weights(theta, lam, pen_w=None, a=SCAD_A):
    """Weights of the next MSA step: w_m = pen_w_m p'_lambda(|theta_m|) / lambda, in [0, 1]
    times pen_w (zero where |theta_m| >= a lambda: those coordinates go unpenalised)."""
    w = scad_derivative(vec(theta), lam, a) / lam
    return w if pen_w is None else vec(pen_w) * w


def msa_scad(fam, Xs, Y, lam, lam_max, steps, a=None, pen_w=None, theta0=None, tol=1e-10, max_outer=100,
             max_inner=100000, nu=1.0, scad_a=SCAD_A):
    """MSA-lasso for one lambda: step 1 is the (pen_w-weighted) lasso, warm-started at
    theta0; each of the steps - 1 further steps solves the weighted lasso with the
    msa_weights of the previous step's estimate, warm-started there.  Returns
    (theta, info of the last step, weights of the last step)."""
    p = param_shape(Xs)
    theta = np.zeros(p) if theta0 is None else np.array(theta0, dtype=np.float64).reshape(p, order="F")
    w = np.ones(int(np.prod(p))) if pen_w is None else vec(pen_w).copy()
    info = None
    for s in range(steps):
        if s > 0:
            w = msa_weights(theta, lam, pen_w, scad_a)
        theta, info = gdpg(fam, Xs, Y, lam, lam_max, a, unvec(w, p), theta, tol, max_outer, max_inner, nu)
        if not info.converged:
            break
    return theta, info, w


def msa_scad_path(fam, Xs, Y, steps, a=None, pen_w=None, lambdas=None, nlambda=100, ratio=1e-4, tol=1e-10,
                  max_outer=100, max_inner=100000, nu=1.0, scad_a=SCAD_A):
    """SCAD lambda path (Sec. 6.4): the lasso's lambda_max and grid, MSA-lasso at each
    lambda warm-started at the previous lambda's estimate."""
    lam_max = lambda_max(fam, Xs, Y, a, pen_w)
    if lambdas is None:
        lambdas = lambda_grid(lam_max, nlambda, ratio)
    p = param_shape(Xs)
    theta = np.zeros(p)
    thetas, infos, weights = [], [], []
    for lam in np.asarray(lambdas, dtype=np.float64):
        theta, info, w = msa_scad(fam, Xs, Y, lam, lam_max, steps, a, pen_w, theta, tol, max_outer, max_inner, nu,
                                  scad_a)
        thetas.append(theta.copy())
        infos.append(info)
        weights.append(w)
        if not info.converged:
            break
    return np.asarray(lambdas, dtype=np.float64), thetas, infos, weights, lam_max


# =============================================================================
# Independent certificates on the explicit design (tiny problems only)
# =============================================================================
def cd_weighted_lasso(Xd, z, wts, lam, pen_w=None, theta0=None, tol=1e-15, max_sweeps=200000):
    """Textbook cyclic coordinate descent for
    min_theta (1/2n) sum_i wts_i (z_i - x_i^T theta)^2 + lambda sum_m pen_m |theta_m|
    on an explicit design matrix (n = number of rows).  Not the paper's
    algorithm: an independent route to the same unique minimiser."""
    n, p = Xd.shape
    pen = np.ones(p) if pen_w is None else vec(pen_w)
    th = np.zeros(p) if theta0 is None else vec(theta0).copy()
    r = z - Xd @ th
    col = (wts[:, None] * Xd * Xd).sum(axis=0) / n
    for _ in range(max_sweeps):
        big = 0.0
        for m in range(p):
            if col[m] == 0.0:
                continue
            xm = Xd[:, m]
            rho_m = float(np.dot(wts * xm, r)) / n + col[m] * th[m]
            new = soft_threshold(rho_m, lam * pen[m]) / col[m]
            dlt = new - th[m]
            if dlt != 0.0:
                r -= dlt * xm
                th[m] = new
                big = max(big, abs(dlt))
        if big <= tol * max(1.0, float(np.max(np.abs(th)))):
            break
    return th


def gaussian_lasso_explicit(Xs, Y, lam, a=None, pen_w=None, tol=1e-15):
    Xd = kron_design(Xs)
    y = vec(Y)
    wts = np.ones_like(y) if a is None else vec(a)
    return cd_weighted_lasso(Xd, y, wts, lam, pen_w, tol=tol)


def poisson_lasso_explicit(Xs, Y, lam, a=None, pen_w=None, tol=1e-13, max_newton=200):
    """Proximal Newton on the explicit design: exact Hessian X^T diag(a e^eta) X / n,
    coordinate descent on each quadratic model, backtracking on F."""
    Xd = kron_design(Xs)
    y = vec(Y)
    av = np.ones_like(y) if a is None else vec(a)
    n, p = Xd.shape
    pen = np.ones(p) if pen_w is None else vec(pen_w)

    def F(th):
        eta = Xd @ th
        return float(np.sum(av * (np.exp(eta) - y * eta))) / n + lam * float(np.sum(pen * np.abs(th)))

    th = np.zeros(p)
    for _ in range(max_newton):
        eta = Xd @ th
        mu = np.exp(eta)
        wts = av * mu
        z = eta + (y - mu) / mu          # Newton working response for the a-weighted loss
        th_new = cd_weighted_lasso(Xd, z, wts, lam, pen, theta0=th, tol=1e-15)
        d = th_new - th
        t = 1.0
        F0 = F(th)
        while t > 1e-12 and not (F(th + t * d) <= F0 + 1e-14 * abs(F0)):
            t *= 0.5
        th = th + t * d
        if np.max(np.abs(t * d)) <= tol * max(1.0, np.max(np.abs(th))):
            break
    return th


def poisson_mle_newton(Xs, Y, a=None, iters=100):
    """Unpenalised Poisson MLE by textbook Newton-Raphson on the explicit design."""
    Xd = kron_design(Xs)
    y = vec(Y)
    av = np.ones_like(y) if a is None else vec(a)
    th = np.zeros(Xd.shape[1])
    for _ in range(iters):
        eta = Xd @ th
        mu = np.exp(eta)
        grad = Xd.T @ (av * (y - mu))
        Hm = Xd.T @ (Xd * (av * mu)[:, None])
        step = np.linalg.solve(Hm, grad)
        t = 1.0

        def ll(v):
            e = Xd @ v
            return float(np.sum(av * (y * e - np.exp(e))))
        l0 = ll(th)
        while ll(th + t * step) < l0 and t > 1e-10:
            t *= 0.5
        th = th + t * step
        if np.max(np.abs(t * step)) < 1e-14 * max(1.0, np.max(np.abs(th))):
            break
    return th


# =============================================================================
# Poisson negative log-likelihood as a function of beta (its gradient is the
# transposed rho chain applied to the score, eqs. three and four)
# =============================================================================
def poisson_nll(Xs, beta, Y):
    """L(beta) = (1/n) sum_i (exp(eta_i) - y_i eta_i), eta = H(beta) (log y! dropped)."""
    eta = H(Xs, beta)
    return float(np.sum(np.exp(eta) - Y * eta)) / Y.size


def poisson_nll_grad(Xs, beta, Y):
    """grad L = -G(U)/n = G(exp(eta) - y)/n."""
    eta = H(Xs, beta)
    return G(Xs, np.exp(eta) - Y) / Y.size


# =============================================================================
# Rounding helpers used when a test feeds reduced-precision inputs
# =============================================================================
def round_to_bf16(x):
    """Round float64 -> float32 (nearest-even) -> bfloat16 (nearest-even on the
    top 16 bits), returned as float64."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)
