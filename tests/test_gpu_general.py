"""Parity of the generic-GEMM path with the oracle: the rho transforms of designs that fit no
mode order of the slab kernels, the lambda path of models of c > 1 tensor components
(glam_fit_path_multi; Sec. 2 eq. fivenew, Sec. 6.1 eqs. eighteen and nineteen, Proposition 1's
sum over components) and the p > n designs of Sec. 6.5 (q = 3), which glam_fit_path routes to it.

Tolerances as the slab-kernel tests: rho transforms relative sup norm FP64 1e-10, FP32 1e-5,
BF16 3e-2 (intermediates rounded to BF16); fits: the oracle's FP64 KKT residual on the GPU's
theta <= kkt_tol, the objective's relative deviation from the oracle's fit, and theta itself where
the PMLE is unique (full-column-rank concatenated designs).  For p > n the lasso solution need
not be unique: there the certificate is the oracle's KKT residual and the objective.
"""
import numpy as np
import pytest

import oracle.glam_oracle as O
from paper_1510_03298_amd import inputs
from tests.gpu_util import need_gpu, rel_inf, rounded

pytestmark = pytest.mark.gpu

TOL = {0: 1e-10, 1: 1e-5, 2: 3e-2}

# no order of the modes puts two of them within the slab kernels' limits (p <= 32, n <= 256)
SHAPES_GENERIC = [
    ((20, 10, 60), (60, 30, 180)),     # Sec. 6.5, q = 3, r = 1 (largest mode last)
    ((37, 45, 21), (40, 50, 7)),       # ragged tiles in every GEMM
    ((5, 6, 7), (40, 33, 35)),         # p_j > n_j in every mode
    ((300, 280, 3), (33, 2, 1)),       # n_1, n_2 > 256
    ((50, 60), (40, 70)),              # d = 2
    ((1, 1, 1), (1, 1, 1)),            # (fits the slab kernels; here for the degenerate sizes)
]


def _factors(n, p, seed):
    rng = np.random.default_rng(seed)
    return [rng.standard_normal((nj, pj)) for nj, pj in zip(n, p)]


@pytest.mark.parametrize("dt", [0, 1, 2])
@pytest.mark.parametrize("n,p", SHAPES_GENERIC)
def test_generic_rho_forward_and_adjoint(n, p, dt):
    torch, glam = need_gpu()
    print(f"generic rho n={n} p={p} dt={dt}", flush=True)
    Xs = _factors(n, p, 31)
    Th = np.random.default_rng(32).standard_normal(p)
    U = np.random.default_rng(33).standard_normal(n)
    Xd = [glam.to_device_colmajor(X, dt) for X in Xs]
    eta = glam.rho_forward(Xd, glam.to_device_colmajor(Th, dt), n, p, dt)
    out = glam.rho_adjoint(Xd, glam.to_device_colmajor(U, dt), n, p, dt)
    torch.cuda.synchronize()
    got_f = glam.from_colmajor(eta, n)
    got_a = glam.from_colmajor(out, p)
    assert rel_inf(got_f, O.H(Xs, Th)) <= TOL[dt], rel_inf(got_f, O.H(Xs, Th))
    assert rel_inf(got_a, O.G(Xs, U)) <= TOL[dt], rel_inf(got_a, O.G(Xs, U))
    if dt == 2:
        Xr = [rounded(glam, torch, X, dt) for X in Xs]
        assert rel_inf(got_f, O.H(Xr, rounded(glam, torch, Th, dt))) <= 1e-2


@pytest.mark.parametrize("dt", [1, 2])
def test_generic_rho_sec65_r2_sampled(dt):
    """Sec. 6.5's q = 3 design at r = 2 (p = 2.59 million coefficients, n = 96,000): the whole
    forward transform and sampled adjoint entries, each an explicit sum on the CPU."""
    torch, glam = need_gpu()
    n, p = (40, 20, 120), (120, 60, 360)
    print(f"generic rho r=2 q=3 dt={dt}", flush=True)
    Xs = _factors(n, p, 34)
    Th = np.random.default_rng(35).standard_normal(p)
    U = np.random.default_rng(36).standard_normal(n)
    Xd = [glam.to_device_colmajor(X, dt) for X in Xs]
    got_f = glam.from_colmajor(glam.rho_forward(Xd, glam.to_device_colmajor(Th, dt), n, p, dt), n)
    got_a = glam.from_colmajor(glam.rho_adjoint(Xd, glam.to_device_colmajor(U, dt), n, p, dt), p)
    torch.cuda.synchronize()
    assert rel_inf(got_f, O.H(Xs, Th)) <= TOL[dt]
    rng = np.random.default_rng(37)
    ref_a = O.G(Xs, U)
    scale = np.max(np.abs(ref_a))
    for _ in range(64):
        i, j, k = (int(rng.integers(0, pj)) for pj in p)
        # entry (i, j, k) of G = sum over the response grid of X1[a, i] X2[b, j] X3[c, k] U[a, b, c]
        v = float(np.einsum("a,b,c,abc->", Xs[0][:, i], Xs[1][:, j], Xs[2][:, k], U))
        assert abs(got_a[i, j, k] - v) <= TOL[dt] * scale


# ----------------------------------------------------------------------------- c-component fits
def _dev_multi(glam, d):
    comps = [([glam.to_device_colmajor(X, 0) for X in Xs], tuple(X.shape[1] for X in Xs)) for Xs in d.comps]
    Yd = glam.to_device_colmajor(d.Y, 0)
    ad = glam.to_device_colmajor(d.a, 0) if d.a is not None else None
    return comps, Yd, ad


_ORACLE = {}


def _oracle_path(key, fam, C, Y, **kw):
    if key not in _ORACLE:
        lams, ths, infos, lm = O.fit_path(fam, C, Y, **kw)
        assert all(i.converged for i in infos), key
        _ORACLE[key] = (np.asarray(lams), [O.vec(t) for t in ths], lm)
    return _ORACLE[key]


def _check(fam, C, Y, th, lam, lm, tol, a=None, ref=None, theta_tol=None, alpha=0.0, l1=1.0, obj=None):
    g = O.smooth_gradient(fam, C, th, Y, a)
    kkt = O.kkt_residual(th, g, lam, lm, alpha=alpha, l1=l1)
    assert kkt <= tol, f"oracle KKT {kkt:.3e} > {tol}"
    F1 = O.objective(fam, C, th, Y, lam, a, alpha=alpha, l1=l1)
    if obj is not None:
        assert abs(obj - F1) <= 1e-9 * abs(F1)
    if ref is not None:
        F2 = O.objective(fam, C, ref, Y, lam, a, alpha=alpha, l1=l1)
        assert (F1 - F2) / abs(F2) <= 1e-7
        if theta_tol is not None:
            assert rel_inf(th, ref) <= theta_tol, rel_inf(th, ref)


CASES_C = [
    # (family, n, component sizes, dtype, obs_w)
    ("gaussian", (13, 11, 17), [(5, 4, 6), (3, 6, 4)], 0, False),
    ("gaussian", (13, 11, 17), [(5, 4, 6), (3, 6, 4)], 2, False),
    ("poisson", (12, 10, 14), [(4, 3, 5), (3, 4, 3)], 0, True),
    ("poisson", (12, 10, 14), [(4, 3, 5), (3, 4, 3)], 1, True),
    ("binomial", (12, 10, 14), [(3, 3, 4), (4, 3, 2), (2, 2, 2)], 1, False),
    ("gamma", (12, 10, 14), [(3, 3, 4), (4, 3, 2)], 0, False),
    ("gaussian", (41, 37), [(9, 7), (6, 11), (5, 5)], 1, False),   # d = 2, c = 3
    ("poisson", (41, 37), [(6, 5), (4, 7)], 2, False),              # d = 2, c = 2
]


@pytest.mark.parametrize("fam,n,ps,dt,obs", CASES_C)
def test_components_path_matches_oracle(fam, n, ps, dt, obs):
    torch, glam = need_gpu()
    print(f"components {fam} n={n} ps={ps} dt={dt} obs={obs}", flush=True)
    d = inputs.random_components_problem(n, ps, family=fam, seed=40 + len(ps), obs_weights=obs,
                                         scale=0.2 if fam == "poisson" else 0.5)
    C = O.Components(d.comps)
    comps, Yd, ad = _dev_multi(glam, d)
    tol = 1e-7
    res = glam.fit_path_multi(comps, Yd, n, fam, obs_w=ad, nlambda=5, lambda_min_ratio=0.02, dtype=dt, kkt_tol=tol)
    assert res.code == 0, (res.code, res.status)
    olams, oths, lm = _oracle_path(f"{fam}{n}{ps}{obs}", fam, C, d.Y, a=d.a, nlambda=5, ratio=0.02, tol=1e-10,
                                   max_outer=300)
    assert abs(res.lambda_max - lm) <= 1e-12 * lm
    np.testing.assert_allclose(res.lambdas, olams, rtol=1e-12)
    for l in range(5):
        th = res.theta[l].cpu().numpy()
        _check(fam, C, d.Y, th, res.lambdas[l], lm, tol, a=d.a, ref=oths[l], theta_tol=1e-4, obj=res.objective[l])


def test_single_component_on_the_generic_path_matches_the_slab_path():
    """c = 1 through glam_fit_path_multi (generic GEMMs) and glam_fit_path (slab kernels): both
    reach the oracle's PMLE on a Poisson path."""
    torch, glam = need_gpu()
    print("c=1 generic vs slab", flush=True)
    d = inputs.random_problem((21, 17, 29), (8, 7, 9), family="poisson", seed=50, basis="gauss", scale=0.3)
    Xd = [glam.to_device_colmajor(X, 0) for X in d.X]
    Yd = glam.to_device_colmajor(d.Y, 0)
    r1 = glam.fit_path(Xd, Yd, d.n, d.p, "poisson", nlambda=4, lambda_min_ratio=0.05, dtype=1, kkt_tol=1e-7)
    r2 = glam.fit_path_multi([(Xd, d.p)], Yd, d.n, "poisson", nlambda=4, lambda_min_ratio=0.05, dtype=1, kkt_tol=1e-7)
    assert r1.code == 0 and r2.code == 0
    np.testing.assert_allclose(r2.lambdas, r1.lambdas, rtol=0)
    lm = O.lambda_max("poisson", d.X, d.Y)
    for l in range(4):
        t1 = r1.theta[l].cpu().numpy()
        t2 = r2.theta[l].cpu().numpy()
        _check("poisson", d.X, d.Y, O.unvec(t2, d.p), r2.lambdas[l], lm, 1e-7, obj=r2.objective[l])
        assert rel_inf(t2, t1) <= 1e-4


PEN_CASES = [
    # (penalty, alpha, nu, inner, extrapolation, dtype, pen_w)
    ("lasso", 0.5, 1.0, "chain", "restarted", 1, False),   # elastic net
    ("ridge", 0.0, 1.0, "chain", "plain", 0, False),
    ("lasso", 0.0, 0.5, "chain", "plain", 0, True),        # backtracking, penalty weights
    ("lasso", 0.0, 0.0, "chain", "plain", 1, False),       # nu = 0
    ("lasso", 0.0, 1.0, "one", "restarted", 0, False),     # unit IRLS weights
    ("scad", 0.0, 1.0, "chain", "restarted", 0, False),
]


@pytest.mark.parametrize("pen,alpha,nu,inner,extrap,dt,pw", PEN_CASES)
def test_components_penalties_and_step_control(pen, alpha, nu, inner, extrap, dt, pw):
    """Poisson c = 2: the elastic net, ridge (R21), SCAD by MSA (R17), penalty weights, nu < 1
    backtracking (R7), nu = 0 (R22), unit weights and both extrapolation sequences, against the
    oracle's fit of the same model."""
    torch, glam = need_gpu()
    print(f"components pen={pen} alpha={alpha} nu={nu} inner={inner} {extrap} dt={dt} pw={pw}", flush=True)
    # counts up to about 40: unit IRLS weights (Sec. 5) then need some 25 outer steps, not 150
    d = inputs.random_components_problem((12, 10, 14), [(4, 3, 5), (3, 4, 3)], family="poisson", seed=60, scale=0.2)
    C = O.Components(d.comps)
    comps, Yd, _ = _dev_multi(glam, d)
    P = sum(int(np.prod(p)) for p in d.ps)
    pen_w = np.random.default_rng(61).uniform(0.5, 2.0, P) if pw else None
    pwd = torch.from_numpy(pen_w).cuda() if pw else None
    lm = O.lambda_max("poisson", C, d.Y, pen_w=pen_w)
    lams = [0.5 * lm, 0.1 * lm]
    tol = 1e-7
    res = glam.fit_path_multi(comps, Yd, d.n, "poisson", pen_w=pwd, lambdas=lams, dtype=dt, kkt_tol=tol, nu=nu,
                              inner=inner, alpha=alpha, penalty=pen, msa_steps=3, extrapolation=extrap)
    assert res.code == 0, (res.code, res.status)
    l1 = 0.0 if pen == "ridge" else 1.0
    a_en = 1.0 if pen == "ridge" else alpha
    if pen == "scad":
        _, oths, oinfos, ows, _ = O.msa_scad_path("poisson", C, d.Y, 3, lambdas=lams, tol=1e-10, max_outer=300)
        for l in range(2):
            th = res.theta[l].cpu().numpy()
            g = O.smooth_gradient("poisson", C, th, d.Y)
            # the last MSA step's weighted lasso (its weights from the GPU's own previous step agree
            # with the oracle's to the fit's accuracy; theta is compared directly)
            assert rel_inf(th, O.vec(oths[l])) <= 1e-4
            assert O.kkt_residual(th, g, lams[l], lm, pen_w=ows[l]) <= 1e-5
        return
    ref_path = O.fit_path("poisson", C, d.Y, pen_w=pen_w, lambdas=lams, tol=1e-10, max_outer=300, alpha=a_en, l1=l1)
    for l in range(2):
        th = res.theta[l].cpu().numpy()
        g = O.smooth_gradient("poisson", C, th, d.Y)
        assert O.kkt_residual(th, g, lams[l], lm, pen_w=pen_w, alpha=a_en, l1=l1) <= tol
        ref = O.vec(ref_path[1][l])
        F1 = O.objective("poisson", C, th, d.Y, lams[l], pen_w=pen_w, alpha=a_en, l1=l1)
        F2 = O.objective("poisson", C, ref, d.Y, lams[l], pen_w=pen_w, alpha=a_en, l1=l1)
        assert (F1 - F2) / abs(F2) <= 1e-7
        assert rel_inf(th, ref) <= 1e-4


# ----------------------------------------------------------------------------- Sec. 6.5, q = 3
@pytest.mark.parametrize("fam,dt,r", [("gaussian", 1, 1), ("gaussian", 2, 1), ("poisson", 0, 1), ("gaussian", 2, 2)])
def test_sec65_p_greater_than_n_path(fam, dt, r):
    """Sec. 6.5's simulated design with q = 3 (p = 324,000 > n = 12,000 at r = 1, kappa = 0):
    glam_fit_path runs it on the generic path.  The lasso solution need not be unique, so each
    model is certified by the oracle's FP64 KKT residual on the GPU's theta and its objective;
    for the Gaussian family also by the lasso's duality gap, which bounds the distance of the
    objective from its minimum without a reference fit.  At r = 2 (p = 2.59 million; the last
    adjoint product, 7,200 x 360, has 678 workgroups, ragged in both directions) the increment
    step runs fused into that product; at r = 1 (87 workgroups) as a kernel of its own."""
    torch, glam = need_gpu()
    print(f"sec 6.5 q=3 {fam} dt={dt} r={r}", flush=True)
    d = inputs.config_sim(r=r, q=3, family=fam, kappa=0.0)
    assert int(np.prod(d.p)) > int(np.prod(d.n))
    Xd = [glam.to_device_colmajor(X, 0) for X in d.X]
    Yd = glam.to_device_colmajor(d.Y, 0)
    tol = 1e-6
    L = 4
    res = glam.fit_path(Xd, Yd, d.n, d.p, fam, nlambda=L, lambda_min_ratio=0.3, dtype=dt, kkt_tol=tol)
    assert res.code == 0, (res.code, res.status)
    lm = O.lambda_max(fam, d.X, d.Y)
    assert abs(res.lambda_max - lm) <= 1e-12 * lm
    y = O.vec(d.Y)
    n = y.size
    for l in range(L):
        th = glam.from_colmajor(res.theta[l], d.p)
        lam = res.lambdas[l]
        g = O.smooth_gradient(fam, d.X, th, d.Y)
        assert O.kkt_residual(th, g, lam, lm) <= tol
        F1 = O.objective(fam, d.X, th, d.Y, lam)
        assert abs(res.objective[l] - F1) <= 1e-9 * abs(F1)
        if fam == "gaussian":
            # weak duality of n F = |y - X theta|^2 / 2 + n lambda |theta|_1: u = s r with
            # s = min(1, n lambda / |X^T r|_inf) is dual feasible, |y|^2/2 - |y - u|^2/2 <= n F*
            r = y - O.vec(O.H(d.X, th))
            c = float(np.max(np.abs(O.G(d.X, O.unvec(r, d.n)))))
            s = min(1.0, n * lam / c) if c > 0 else 1.0
            u = s * r
            dual = (0.5 * float(y @ y) - 0.5 * float((y - u) @ (y - u))) / n
            assert 0.0 <= F1 - dual <= 1e-6 * abs(F1), (F1, dual)


def test_precision_escalation_on_the_generic_path():
    """Section 6.5's Poisson design at r = 3 (correlated Gaussian factors, X^T X condition number in
    the tens of millions) through the generic solver: the BF16 chain cannot refine it, the fit
    continues one rung up (FP32, then FP64), and every model still meets the oracle's KKT bar."""
    torch, glam = need_gpu()
    d = inputs.config_sim(r=3, family="poisson")
    print(f"generic escalation n={d.n} p={d.p}", flush=True)
    Xd = [glam.to_device_colmajor(X, 0) for X in d.X]
    Yd = glam.to_device_colmajor(d.Y, 0)
    res = glam.fit_path_multi([(Xd, d.p)], Yd, d.n, "poisson", nlambda=40, lambda_min_ratio=0.02, dtype=2,
                              kkt_tol=1e-6)
    assert res.code == 0 and res.n_done == 40
    assert 0 <= res.escalated_at < 40
    lm = O.lambda_max("poisson", d.X, d.Y)
    for l in (res.escalated_at, 39):
        th = glam.from_colmajor(res.theta[l], d.p)
        g = O.smooth_gradient("poisson", d.X, th, d.Y)
        assert O.kkt_residual(th, g, res.lambdas[l], lm) <= 1e-6
