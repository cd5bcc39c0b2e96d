"""The oracle's pins must catch plausible mistakes.

Each case plants one mistake in the oracle (on the CPU, through monkeypatch) and
checks that at least one of the pins in test_oracle_pins fails with it.
"""
import numpy as np
import pytest

import oracle.glam_oracle as O
from tests import test_oracle_pins as P


def _fails(fns):
    for fn in fns:
        try:
            fn()
        except Exception:
            return True
    return False


def _gauss_pins():
    return [lambda: P.test_gaussian_closed_form_orthogonal_design(),
            lambda: P.test_gaussian_matches_coordinate_descent("gauss")]


def _poisson_pins():
    return [lambda: P.test_poisson_matches_prox_newton(0.3), lambda: P.test_poisson_lambda_zero_is_mle()]


MUTANTS = {
    # wrong sign of the score (eq. four)
    "score_sign": ("score", lambda orig: (lambda fam, eta, y, a=None: -orig(fam, eta, y, a)),
                   lambda: _gauss_pins() + [lambda: P.test_score_is_derivative_of_loglik("poisson")]),
    # prior weights dropped from the score
    "score_drops_a": ("score", lambda orig: (lambda fam, eta, y, a=None: orig(fam, eta, y, None)),
                      lambda: [lambda: P.test_score_is_derivative_of_loglik("gaussian"),
                               lambda: P.test_gaussian_with_observation_weights_matches_cd()]),
    # working response without the + eta term (eq. tennew)
    "z_drops_eta": ("working_response",
                    lambda orig: (lambda fam, eta, y, a=None: orig(fam, eta, y, a) - eta),
                    lambda: [lambda: P.test_working_response_forms_agree("poisson")] + _poisson_pins()),
    # soft threshold at half the level
    "prox_half": ("soft_threshold", lambda orig: (lambda z, t: orig(z, 0.5 * t)),
                  lambda: [P.test_soft_threshold_is_the_l1_prox] + _gauss_pins()),
    # KKT residual with the wrong subgradient sign
    "kkt_sign": ("kkt_residual",
                 lambda orig: (lambda th, g, lam, lm, pen_w=None, alpha=0.0, l1=1.0: orig(th, -np.asarray(g), lam, lm,
                                                                                       pen_w, alpha, l1)),
                 lambda: [P.test_kkt_residual_definition] + _gauss_pins()),
    # elastic-net prox with 1 + alpha gamma instead of 1 + 2 alpha gamma (Sec. 6.3)
    "enet_prox_factor": ("prox_elastic_net",
                         lambda orig: (lambda z, gamma, alpha, l1=1.0: orig(z, gamma, 0.5 * alpha, l1)),
                         lambda: [P.test_elastic_net_closed_form_orthogonal_design]),
    # ridge prox with 1 + gamma instead of 1 + 2 gamma (Sec. 6.3)
    "ridge_prox_factor": ("prox_elastic_net",
                          lambda orig: (lambda z, gamma, alpha, l1=1.0: orig(z, gamma, 0.5 * alpha, l1) if l1 == 0.0
                                        else orig(z, gamma, alpha, l1)),
                          lambda: [P.test_ridge_closed_form_orthogonal_design, P.test_ridge_matches_normal_equations]),
    # KKT residual without the elastic net's smooth term
    "kkt_drops_enet": ("kkt_residual",
                       lambda orig: (lambda th, g, lam, lm, pen_w=None, alpha=0.0, l1=1.0: orig(th, g, lam, lm, pen_w, 0.0,
                                                                                               l1)),
                       lambda: [P.test_elastic_net_kkt_residual_definition,
                                P.test_elastic_net_closed_form_orthogonal_design]),
    # Gamma-log score taken as if the link were canonical (vartheta' = 1 dropped)
    "gamma_score_canonical": ("score",
                              lambda orig: (lambda fam, eta, y, a=None: (
                                  (np.ones_like(y) if a is None else a) * (y - np.exp(eta))
                                  if O.family(fam).name == "gamma" else orig(fam, eta, y, a))),
                              lambda: [lambda: P.test_identity_factors_closed_form("gamma"),
                                       lambda: P.test_score_is_derivative_of_loglik("gamma")]),
    # Binomial IRLS weight mu instead of mu (1 - mu) (eq. nine)
    "binomial_weight_mu": ("irls_weights",
                           lambda orig: (lambda fam, eta: O.family(fam).ginv(eta)
                                         if O.family(fam).name == "binomial" else orig(fam, eta)),
                           lambda: [lambda: P.test_score_is_derivative_of_loglik("binomial"),
                                    lambda: P.test_working_response_forms_agree("binomial")]),
    # Binomial Armijo change without the -y s term
    "binomial_change_drops_ys": ("objective_change",
                                 lambda orig: (lambda fam, eta, xd, t, Y, a=None: orig(fam, eta, xd, t, Y, a) + (
                                     float(np.sum((np.ones_like(Y) if a is None else a) * Y * t * xd)) / Y.size
                                     if O.family(fam).name == "binomial" else 0.0)),
                                 lambda: [lambda: P.test_objective_change_is_the_difference_of_objectives("binomial")]),
    # SCAD slope divided by a instead of a - 1 beyond lambda
    "scad_slope": ("scad_derivative",
                   lambda orig: (lambda t, lam, a=O.SCAD_A: np.where(np.abs(t) <= lam, lam,
                                                                     np.maximum(a * lam - np.abs(t), 0.0) / a)),
                   lambda: [P.test_scad_penalty_and_slope, P.test_msa_orthogonal_design_reaches_scad_thresholding]),
    # tensor-product weights without the geometric-mean factor Vbar (the displayed product alone)
    "kron_no_vbar": ("kron_weights",
                     lambda orig: (lambda V: (lambda r: (r[0] / r[2], r[1], r[2]))(orig(V))),
                     lambda: [P.test_kron_weights_exact_for_tensor_products]),
    # H applies the factors in reverse order (wrong mode index)
    "H_reversed": ("H", lambda orig: (lambda Xs, Th: orig(list(Xs)[::-1], Th)),
                   lambda: [lambda: P.test_kronecker_rho_identity((6, 5, 4), (6, 5, 4)), P.test_adjoint_dot_product]),
    # G forgets the transpose on the factors (transposed operand)
    "G_no_transpose": ("G", lambda orig: (lambda Xs, U: orig([np.asarray(X).T for X in Xs], U)),
                       lambda: [lambda: P.test_kronecker_rho_identity((6, 5, 4), (6, 5, 4)), P.test_adjoint_dot_product]),
    # rho appends the new mode first instead of last
    "rho_mode_first": ("rho", lambda orig: (lambda X, A: np.moveaxis(orig(X, A), -1, 0)),
                       lambda: [lambda: P.test_rho_matches_defining_sum((2, 3, 4), 3),
                                P.test_rho_identity_factor_is_cyclic_rotation]),
    # lambda_max without the 1/n scale
    "lmax_no_n": ("lambda_max",
                  lambda orig: (lambda fam, Xs, Y, a=None, pen_w=None: orig(fam, Xs, Y, a, pen_w) * Y.size),
                  lambda: [lambda: P.test_lambda_max_gives_zero_solution("gaussian")]),
    # lambda grid with the exponent l / nlambda (one step short of lambda_min)
    "grid_off_by_one": ("lambda_grid",
                        lambda orig: (lambda lm, nl, ratio: lm * ratio ** (np.arange(nl) / nl) if nl > 1
                                      else orig(lm, nl, ratio)),
                        lambda: [lambda: P.test_lambda_grid_end_point_and_log_spacing(100, 1e-4)]),
    # Poisson NLL without the 1/n scale, or with +y eta
    "nll_no_n": ("poisson_nll", lambda orig: (lambda Xs, beta, Y: orig(Xs, beta, Y) * Y.size),
                 lambda: [P.test_poisson_nll_value_on_the_explicit_design]),
    "nll_sign_y": ("poisson_nll",
                   lambda orig: (lambda Xs, beta, Y: float(np.sum(np.exp(O.H(Xs, beta)) + Y * O.H(Xs, beta))) / Y.size),
                   lambda: [P.test_poisson_nll_constant_predictor_closed_form]),
    # exact tensor-weight Lipschitz constant with the weights dropped from the Gram factors
    "lexact_no_weights": ("lipschitz_tensor_weights",
                          lambda orig: (lambda Xs, factors, n: orig(Xs, [np.ones_like(v) for v in factors], n)),
                          lambda: [P.test_exact_lipschitz_for_tensor_product_weights]),
    # c > 1: H without the last component's chain (the sum of eq. eighteen cut short)
    "components_H_drops_last": ("H",
                                lambda orig: (lambda Xs, Theta: sum(orig(Xr, Tr) for Xr, Tr in
                                                                    list(zip(Xs, Xs.split(Theta)))[:-1])
                                              if isinstance(Xs, O.Components) and len(Xs) > 1 else orig(Xs, Theta)),
                                lambda: [lambda: P.test_components_H_and_G_are_the_concatenated_design(
                                    (6, 5, 4), [(3, 2, 2), (2, 3, 3)]),
                                         P.test_components_gaussian_matches_coordinate_descent]),
    # c > 1: the tuple of eq. nineteen stacked in reverse component order
    "components_G_reversed": ("G",
                              lambda orig: (lambda Xs, U: np.concatenate([O.vec(orig(Xr, U)) for Xr in reversed(Xs)])
                                            if isinstance(Xs, O.Components) else orig(Xs, U)),
                              lambda: [lambda: P.test_components_H_and_G_are_the_concatenated_design(
                                  (6, 5, 4), [(3, 2, 2), (2, 3, 3)])]),
    # Proposition 1 with the largest component's product instead of the sum over components
    "prop1_max_over_components": ("spectral_bound",
                                  lambda orig: (lambda Xs: max(float(np.prod(O.spectral_radii(Xr))) for Xr in Xs)
                                                if isinstance(Xs, O.Components) else orig(Xs)),
                                  lambda: [P.test_prop1_bound_sums_over_components]),
    # Lipschitz bound with a sum of spectral radii instead of the product
    "lhat_sum": ("lipschitz_bound",
                 lambda orig: (lambda Xs, w, n: float(np.max(w)) * float(np.sum(O.spectral_radii(Xs))) / n),
                 lambda: [P.test_lipschitz_bound_prop1]),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name, monkeypatch):
    attr, make, pins = MUTANTS[name]
    orig = getattr(O, attr)
    monkeypatch.setattr(O, attr, make(orig))
    assert _fails(pins()), f"no pin caught mutant {name}"


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_pass_without_mutation(name):
    """Control: the same pin lists pass on the unmodified oracle."""
    _, _, pins = MUTANTS[name]
    for fn in pins():
        fn()
