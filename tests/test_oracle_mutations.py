"""Plant plausible mistakes in the oracle (on the CPU, in a copy of one function) and
check that at least one pin catches each.  This shows the pins are strong enough
to detect a dropped term, a wrong sign, a wrong index or a transposed operand."""
import inspect
import textwrap

import pytest

from oracle import tmc_oracle as O
from tests import test_oracle_pins as P


def _mutant(func_name, old, new):
    src = textwrap.dedent(inspect.getsource(getattr(O, func_name)))
    assert old in src, (func_name, old)
    ns = dict(O.__dict__)
    exec(compile(src.replace(old, new, 1), f"<mutant {func_name}>", "exec"), ns)
    return ns[func_name]


MUTATIONS = [
    ("logmmexp", "Y[..., None, :, :], axis=-2)", "Y[..., None, :, :], axis=-1)",
     P.test_logmmexp_equals_scipy_and_matrix_product),
    ("logmmexp", "X[..., :, :, None] + Y[..., None, :, :]", "X[..., :, :, None] + np.swapaxes(Y, -1, -2)[..., None, :, :]",
     P.test_logmmexp_chain_is_the_discrete_tmc_estimator),
    ("gauss_pair_logfactor_pp", "-np.sum(sp, axis=1)", "-np.sum(sp, axis=0).sum() / sp.shape[0]",
     P.test_pp_factor_equals_scipy_normal_logpdf),
    ("gauss_pair_logfactor_pp", "lam[None, :, :] * diff * diff", "lam[None, :, :].mean(axis=1, keepdims=True) * diff * diff",
     P.test_pp_factor_equals_scipy_normal_logpdf),
    ("gauss_chain_grads_pp", "g * (lam[None] * diff * diff - 1.0), axis=0", "g * (lam[None] * diff * diff), axis=0",
     P.test_pp_gradients_against_finite_differences),
    ("gauss_chain_grads_pp", "np.sum(g * (-lam[None] * diff), axis=1)", "np.sum(g * (-lam.mean(axis=0) * diff), axis=1)",
     P.test_pp_gradients_against_finite_differences),
    # (function, original text, planted mistake, pin that must fail)
    ("logsumexp", ") + m_safe", ")", P.test_logsumexp_matches_scipy_and_handles_inf),
    ("gauss_pair_logfactor", "-np.sum(s)", "np.sum(s)", P.test_gauss_factor_equals_scipy_normal_logpdf),
    ("gauss_pair_logfactor", "lam * diff * diff", "lam * diff", P.test_gauss_factor_equals_scipy_normal_logpdf),
    ("gauss_pair_logfactor", "- z.shape[1] * HALF_LOG_2PI", "", P.test_zero_variance_gives_exact_evidence),
    ("chain_messages", "f[l] + alpha[l + 1][None, :]", "f[l].T + alpha[l + 1][None, :]",
     lambda: P.test_chain_recursion_equals_brute_force((8, 8, 8, 8))),
    ("chain_messages", "- log_k(K_up)", "", lambda: P.test_tmc_on_discrete_chain_is_exact_marginal((3, 4, 2))),
    ("chain_messages", "alpha[L - 1] = np.asarray(u[L - 1], np.float64)",
     "alpha[L - 1] = np.zeros(len(u[L - 1]))", P.test_single_layer_is_iwae),
    ("chain_marginals", "beta[0] = np.full(len(u[0]), -log_k(len(u[0])))",
     "beta[0] = np.zeros(len(u[0]))", P.test_marginals_are_factor_derivatives),
    ("chain_marginals", "- log_k(len(u[l + 1])) - logp)", "- logp)", P.test_marginals_are_factor_derivatives),
    ("gauss_chain_grads", "lam * diff * diff - 1.0", "lam * diff * diff",
     P.test_gauss_gradients_against_finite_differences),
    ("gauss_chain_grads", "np.sum(g * (-lam * diff), axis=1)", "np.sum(g * (lam * diff), axis=1)",
     P.test_gauss_gradients_against_finite_differences),
    ("gauss_chain_grads", "gmu += np.sum(g * (lam * diff), axis=0)", "gmu += np.sum(g * (lam * diff), axis=1).sum(0)",
     P.test_gauss_gradients_against_finite_differences),
    ("linear_gauss_log_evidence", "sigma_x ** 2", "sigma_x", P.test_linear_gauss_evidence_against_quadrature),
    ("hmm_log_evidence", "v = T @ v", "v = T.T @ v", P.test_hmm_evidence_by_enumeration),
    ("gauss_layer0_row_grads", "- log_k(K1) - logp)", "- logp)",
     P.test_layer0_row_grads_agree_with_full_marginals),
    ("gauss_pair_logfactor_expanded", "- 2.0 * cross", "- cross",
     P.test_expanded_factor_equals_direct_difference),
    ("gauss_pair_logfactor_expanded", "mm = np.sum(lam * mu * mu, axis=1)", "mm = np.sum(mu * mu, axis=1)",
     P.test_expanded_factor_equals_direct_difference),
    ("gauss_chain_grads_expanded", "rG[:, None] * zl - gmu", "cG[:, None] * zl - gmu",
     P.test_expanded_gradients_equal_direct_difference),
    ("gauss_chain_grads_expanded", "gtz = g.T @ zl", "gtz = g @ zl",
     P.test_expanded_gradients_equal_direct_difference),
    ("gauss_chain_grads_expanded", "\n                  - g.sum())", ")",
     P.test_expanded_gradients_equal_direct_difference),
    ("tempered_chain_logp", "[kappa * np.asarray(a, np.float64) for a in u]",
     "[np.asarray(a, np.float64) for a in u]",
     P.test_tempered_estimator_equals_enumeration_of_powered_weights),
    ("gauss_chain_grads_tempered", "dz[l] = kappa * np.sum", "dz[l] = np.sum",
     P.test_tempered_gradients_against_enumeration_and_differences),
    ("gauss_chain_grads_tempered", "(lam * diff * diff - 1.0)", "(lam * diff * diff)",
     P.test_tempered_gradients_against_enumeration_and_differences),
    ("dregs_gradients", "h = 0.5 * c", "h = c",
     P.test_dregs_surrogate_gradient_is_the_dregs_estimator),
    ("dregs_gradients", "- 2.0 * lp1 - sum(log_k(len(a)) for a in u))", "- 2.0 * lp1)",
     P.test_dregs_surrogate_gradient_is_the_dregs_estimator),
    ("star_logp", "\\\n            - log_k(len(ui))", "",
     P.test_star_equals_enumeration_and_one_point_chain),
    ("star_logp", "axis=1)", "axis=0)", P.test_star_equals_enumeration_and_one_point_chain),
    ("star_marginals", "- (mi + log_k(len(ui)))[:, None]", "- mi[:, None]",
     P.test_star_marginals_and_gradients_against_differences),
    ("gauss_star_grads", "dz.append(np.sum(g * (-lam * diff), axis=0))", "dz.append(np.sum(g * (lam * diff), axis=0))",
     P.test_star_marginals_and_gradients_against_differences),
    ("gauss_star_log_evidence", "+ 2.0 * np.eye(n)", "+ np.eye(n)",
     P.test_star_evidence_closed_form_against_quadrature),
]


@pytest.mark.parametrize("func,old,new,pin", MUTATIONS,
                         ids=[f"{m[0]}:{i}" for i, m in enumerate(MUTATIONS)])
def test_planted_mistake_is_caught(monkeypatch, func, old, new, pin):
    pin()                                        # the pin passes on the true oracle
    monkeypatch.setattr(O, func, _mutant(func, old, new))
    with pytest.raises((AssertionError, ValueError, IndexError)):
        pin()
