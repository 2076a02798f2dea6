"""Pins for the FP64 oracle: each check ties an oracle function to something other
than itself (a library routine, enumeration of the paper's eq. (is), a special case
with a textbook answer, a closed form, finite differences or an exact invariant)."""
import itertools
import math

import numpy as np
import pytest
from scipy import integrate, special, stats

from oracle import tmc_oracle as O
from workloads import make, linear_gauss


def _rand_chain(rng, K, D, scale=1.0):
    L = len(K)
    z = [rng.normal(size=(K[l], D[l])) for l in range(L)]
    mu = [rng.normal(size=(K[l + 1], D[l])) * scale for l in range(L - 1)]
    s = [rng.uniform(-1.0, 0.0, size=D[l]) for l in range(L - 1)]
    u = [rng.normal(size=K[l]) * 3.0 for l in range(L)]
    return z, mu, s, u


# --- logsumexp ----------------------------------------------------------------

def test_logsumexp_matches_scipy_and_handles_inf():
    rng = np.random.default_rng(0)
    a = rng.normal(size=(7, 13)) * 300.0
    for ax in (0, 1):
        np.testing.assert_allclose(O.logsumexp(a, ax), special.logsumexp(a, axis=ax), rtol=1e-14)
    b = np.array([[-np.inf, -np.inf], [0.0, -np.inf], [np.nan, 1.0]])
    out = O.logsumexp(b, 1)
    assert out[0] == -np.inf and out[1] == 0.0 and np.isnan(out[2])


# --- factor (T10) ----------------------------------------------------------------

def test_gauss_factor_equals_scipy_normal_logpdf():
    rng = np.random.default_rng(1)
    z = rng.normal(size=(5, 7))
    mu = rng.normal(size=(6, 7))
    s = rng.uniform(-1.5, 0.5, size=7)
    f = O.gauss_pair_logfactor(z, mu, s, chunk=2)
    ref = np.array([[stats.norm.logpdf(z[i], loc=mu[j], scale=np.exp(s)).sum()
                     for j in range(6)] for i in range(5)])
    np.testing.assert_allclose(f, ref, rtol=1e-13, atol=1e-12)


# --- chain recursion vs enumeration of eq. (is) (T1) ------------------------------

@pytest.mark.parametrize("K", [(8, 8, 8, 8), (3, 5, 2, 4), (1, 6, 3), (4, 1, 5, 2, 3)])
def test_chain_recursion_equals_brute_force(K):
    rng = np.random.default_rng(sum(K))
    D = [3] * len(K)
    z, mu, s, u = _rand_chain(rng, K, D)
    f = O.gauss_chain_factors(z, mu, s)
    assert abs(O.chain_logp(f, u) - O.brute_force_logp(f, u)) < 1e-10


def test_c1_recursion_equals_brute_force():
    w = make("c1", B=4)
    for c in w.chains:
        f = O.gauss_chain_factors(c.z, c.mu, c.s)
        a, b = O.chain_logp(f, c.u), O.brute_force_logp(f, c.u)
        assert abs(a - b) <= 1e-12 * max(1.0, abs(b))


def test_brute_force_small_probability_space():
    """Enumeration checked in probability space with plain Python products."""
    rng = np.random.default_rng(3)
    K = (2, 3, 2)
    u = [rng.normal(size=k) for k in K]
    f = [rng.normal(size=(K[0], K[1])), rng.normal(size=(K[1], K[2]))]
    tot = 0.0
    for a in range(2):
        for b in range(3):
            for c in range(2):
                tot += (math.exp(u[0][a]) * math.exp(u[1][b]) * math.exp(u[2][c])
                        * math.exp(f[0][a, b]) * math.exp(f[1][b, c]))
    assert abs(O.brute_force_logp(f, u) - math.log(tot / 12.0)) < 1e-13


# --- special cases (T3, T4) ------------------------------------------------------

def test_single_layer_is_iwae():
    rng = np.random.default_rng(4)
    u0 = rng.normal(size=37) * 50.0
    ref = special.logsumexp(u0) - math.log(37)
    assert abs(O.chain_logp([], [u0]) - ref) < 1e-12
    assert abs(O.iwae_logp(u0) - ref) < 1e-12


def test_one_sample_per_layer_is_vae():
    rng = np.random.default_rng(5)
    K = (1, 1, 1, 1)
    z, mu, s, u = _rand_chain(rng, K, (4, 4, 4, 4))
    f = O.gauss_chain_factors(z, mu, s)
    ref = sum(a[0] for a in u) + sum(a[0, 0] for a in f)
    assert abs(O.chain_logp(f, u) - ref) < 1e-12


# --- exact discrete marginalisation (T2) -----------------------------------------

def _random_hmm(rng, S):
    L = len(S)
    prior = rng.dirichlet(np.ones(S[-1]))
    trans = []
    for l in range(L - 1):
        T = rng.dirichlet(np.ones(S[l]), size=S[l + 1]).T      # columns sum to 1
        trans.append(T)
    emit = np.log(rng.dirichlet(np.ones(5), size=S[0])[:, 2])  # P(x = 2 | state)
    return prior, trans, emit


def test_hmm_evidence_by_enumeration():
    rng = np.random.default_rng(6)
    S = (3, 4, 2)
    prior, trans, emit = _random_hmm(rng, S)
    tot = 0.0
    for a, b, c in itertools.product(range(3), range(4), range(2)):
        tot += prior[c] * trans[1][b, c] * trans[0][a, b] * math.exp(emit[a])
    assert abs(O.hmm_log_evidence(prior, trans, emit) - math.log(tot)) < 1e-13


@pytest.mark.parametrize("S", [(3, 4, 2), (5, 5, 5, 5, 5), (2, 7, 3, 6)])
def test_tmc_on_discrete_chain_is_exact_marginal(S):
    """Appendix, exact marginalisation: K_l = number of states, z_l^k = k, uniform
    proposal Q = 1/K_l  =>  the TMC estimate is exactly log P(x)."""
    rng = np.random.default_rng(len(S) * 10 + S[0])
    prior, trans, emit = _random_hmm(rng, S)
    L = len(S)
    f = [np.log(trans[l]) for l in range(L - 1)]
    u = [np.full(S[l], math.log(S[l])) for l in range(L)]   # -log Q = log K_l
    u[0] = u[0] + emit
    u[L - 1] = u[L - 1] + np.log(prior)
    assert abs(O.chain_logp(f, u) - O.hmm_log_evidence(prior, trans, emit)) < 1e-12


# --- closed forms (pins for the linear-Gaussian helpers) -------------------------

def test_linear_gauss_evidence_against_quadrature():
    # one latent: z ~ N(0,1), x | z ~ N(w z, sx^2)
    w, sx, x = 1.7, 0.6, 0.9
    ref = integrate.quad(lambda z: stats.norm.pdf(x, w * z, sx) * stats.norm.pdf(z), -12, 12,
                         epsabs=1e-14)[0]
    got = O.linear_gauss_log_evidence([], np.array([[w]]), np.array([x]), 0.5, sx)
    assert abs(got - math.log(ref)) < 1e-10
    # two latents: z1 ~ N(0,1), z0 | z1 ~ N(a z1, sz^2), x | z0 ~ N(w z0, sx^2)
    a, sz = -0.8, 0.5
    ref2 = integrate.dblquad(
        lambda z0, z1: stats.norm.pdf(x, w * z0, sx) * stats.norm.pdf(z0, a * z1, sz)
        * stats.norm.pdf(z1), -10, 10, -10, 10, epsabs=1e-13)[0]
    got2 = O.linear_gauss_log_evidence([np.array([[a]])], np.array([[w]]), np.array([x]), sz, sx)
    assert abs(got2 - math.log(ref2)) < 1e-8


def test_linear_gauss_posterior_bayes_identity():
    """log P(x) = log P(x|z) + log P(z) - log P(z|x) at any z, with the joint prior of
    all layers and the oracle's exact posterior."""
    w = linear_gauss(B=1, L=3, K=2, D=3, x_dim=4)
    W, Wx, x = w.extra["W"], w.extra["Wx"], w.extra["x"][0]
    sz, sx = 0.5, 0.3
    post = O.linear_gauss_posterior_marginals(W, Wx, x, sz, sx)
    C, D = O.linear_gauss_joint_cov(W, Wx, sz, sx)
    nz = sum(D)
    Czz, Czx, Cxx = C[:nz, :nz], C[:nz, nz:], C[nz:, nz:]
    mpost = np.concatenate([m for m, _ in post])
    Ppost = Czz - Czx @ np.linalg.solve(Cxx, Czx.T)
    rng = np.random.default_rng(7)
    zz = rng.normal(size=nz)
    z0 = zz[:D[0]]
    lx = stats.multivariate_normal(Wx @ z0, sx ** 2 * np.eye(len(x))).logpdf(x)
    lz = stats.multivariate_normal(np.zeros(nz), Czz).logpdf(zz)
    lpost = stats.multivariate_normal(mpost, Ppost).logpdf(zz)
    ev = O.linear_gauss_log_evidence(W, Wx, x, sz, sx)
    assert abs(ev - (lx + lz - lpost)) < 1e-9
    # marginal blocks are the diagonal blocks of the full posterior
    o = 0
    for (m, P), d in zip(post, D):
        np.testing.assert_allclose(P, Ppost[o:o + d, o:o + d], atol=1e-12)
        o += d


# --- whole-estimator pins (T6, T5, T7) -------------------------------------------

def test_zero_variance_gives_exact_evidence():
    """W_l = 0 above layer 0 and Q(z_0) = P(z_0 | x), Q(z_l) = P(z_l): every
    importance ratio equals P(x), so log P_TMC = log P(x) whatever the samples."""
    rng = np.random.default_rng(8)
    L, D, K, dx, sz, sx = 4, 3, 6, 5, 0.5, 0.3
    W = [np.zeros((D, D)) for _ in range(L - 1)]
    Wx = rng.normal(size=(dx, D)) / math.sqrt(D)
    x = rng.normal(size=dx)
    post = O.linear_gauss_posterior_marginals(W, Wx, x, sz, sx)
    m0, P0 = post[0]
    z = [rng.multivariate_normal(m0, P0, size=K)]
    z += [rng.normal(size=(K, D)) * sz for _ in range(L - 2)] + [rng.normal(size=(K, D))]
    mu = [z[l + 1] @ W[l].T for l in range(L - 1)]
    s = [np.full(D, math.log(sz)) for _ in range(L - 1)]
    u = [None] * L
    u[0] = (stats.multivariate_normal(np.zeros(dx), sx ** 2 * np.eye(dx)).logpdf(x - z[0] @ Wx.T)
            - stats.multivariate_normal(m0, P0).logpdf(z[0]))
    for l in range(1, L - 1):
        u[l] = -stats.norm.logpdf(z[l], 0.0, sz).sum(-1)
    u[L - 1] = np.zeros(K)       # Q(z_top) = P(z_top): prior and proposal cancel
    got = O.gauss_chain_logp(z, mu, s, u)
    assert abs(got - O.linear_gauss_log_evidence(W, Wx, x, sz, sx)) < 1e-10


def _posterior_marginal_proposal(W, Wx, sz, sx, widen=1.0):
    def prop(b, x):
        post = O.linear_gauss_posterior_marginals(W, Wx, x, sz, sx)
        qm = np.stack([m for m, _ in post])
        qs = np.stack([np.sqrt(np.diag(P)) * widen for _, P in post])
        return qm, qs
    return prop


def _tmc_ratio_samples(n, K, seed=11):
    base = linear_gauss(B=1, L=4, K=K, D=8, x_dim=32, seed=seed)
    W, Wx = base.extra["W"], base.extra["Wx"]
    w = linear_gauss(B=n, L=4, K=K, D=8, x_dim=32, seed=seed,
                     proposal=_posterior_marginal_proposal(W, Wx, 0.5, 0.3))
    out = []
    for b, c in enumerate(w.chains):
        ev = O.linear_gauss_log_evidence(W, Wx, w.extra["x"][b], 0.5, 0.3)
        out.append(O.gauss_chain_logp(c.z, c.mu, c.s, c.u) - ev)
    return np.array(out)


@pytest.mark.slow
def test_unbiased_against_closed_form_evidence():
    """E_Q[exp(log P_TMC)] = P(x) (eq. (is) averages unbiased single-tuple estimates).
    Checked on the linear-Gaussian chain with posterior-marginal proposals, K=64,
    4000 replicates: the mean ratio exp(log P_TMC - log P(x)) must lie within 4
    bootstrap standard errors of 1."""
    d = _tmc_ratio_samples(4000, 64)
    r = np.exp(d)
    rng = np.random.default_rng(12)
    boots = np.array([r[rng.integers(0, len(r), len(r))].mean() for _ in range(400)])
    se = boots.std()
    assert abs(r.mean() - 1.0) < 4.0 * se, (r.mean(), se)
    assert se < 0.1


def test_jensen_bound_and_tightening_with_K():
    """log P(x) >= E[log P_TMC] (Sec. "Background"); the gap shrinks as K grows."""
    gaps = [np.mean(_tmc_ratio_samples(300, K, seed=13)) for K in (1, 4, 16)]
    assert all(g < 0 for g in gaps)
    assert gaps[0] < gaps[1] < gaps[2]


# --- gradients (T8, T9) ----------------------------------------------------------

def test_marginals_are_factor_derivatives():
    rng = np.random.default_rng(14)
    K = (3, 4, 2)
    f = [rng.normal(size=(3, 4)) * 2, rng.normal(size=(4, 2)) * 2]
    u = [rng.normal(size=k) for k in K]
    logp, G, p = O.chain_marginals(f, u)
    for l in range(2):
        fd = O.finite_difference(lambda a: O.chain_logp([a if m == l else f[m] for m in range(2)], u),
                                 f[l], h=1e-6)
        np.testing.assert_allclose(G[l].reshape(-1), fd, atol=1e-8)
    for l in range(3):
        fd = O.finite_difference(lambda a: O.chain_logp(f, [a if m == l else u[m] for m in range(3)]),
                                 u[l], h=1e-6)
        np.testing.assert_allclose(p[l], fd, atol=1e-8)


def test_marginal_invariants():
    rng = np.random.default_rng(15)
    K = (5, 7, 4, 6)
    z, mu, s, u = _rand_chain(rng, K, (3, 3, 3, 3))
    f = O.gauss_chain_factors(z, mu, s)
    logp, G, p = O.chain_marginals(f, u)
    for l in range(3):
        assert abs(G[l].sum() - 1.0) < 1e-12
        np.testing.assert_allclose(G[l].sum(1), p[l], atol=1e-13)
        np.testing.assert_allclose(G[l].sum(0), p[l + 1], atol=1e-13)
    # permutation of one layer's samples leaves log P unchanged
    perm = rng.permutation(K[1])
    z2 = list(z); mu2 = list(mu); u2 = list(u)
    z2[1] = z[1][perm]; u2[1] = u[1][perm]; mu2[0] = mu[0][perm]
    mu2[1] = mu[1]
    assert abs(O.gauss_chain_logp(z2, mu2, s, u2) - logp) < 1e-11
    # adding c to one factor adds c to log P
    f2 = [a.copy() for a in f]; f2[2] += 3.25
    assert abs(O.chain_logp(f2, u) - logp - 3.25) < 1e-11


def test_gauss_gradients_against_finite_differences():
    rng = np.random.default_rng(16)
    K, D = (4, 5, 3, 4), (3, 2, 4, 2)
    z, mu, s, u = _rand_chain(rng, K, D, scale=0.7)
    logp, dz, dmu, ds, du = O.gauss_chain_grads(z, mu, s, u, chunk=2)
    L = len(K)

    def with_(lst, l, a):
        return [a if m == l else lst[m] for m in range(len(lst))]

    for l in range(L):
        fd = O.finite_difference(lambda a: O.gauss_chain_logp(with_(z, l, a), mu, s, u), z[l])
        np.testing.assert_allclose(dz[l].reshape(-1), fd, atol=2e-7)
        fd = O.finite_difference(lambda a: O.gauss_chain_logp(z, mu, s, with_(u, l, a)), u[l])
        np.testing.assert_allclose(du[l], fd, atol=2e-7)
    for l in range(L - 1):
        fd = O.finite_difference(lambda a: O.gauss_chain_logp(z, with_(mu, l, a), s, u), mu[l])
        np.testing.assert_allclose(dmu[l].reshape(-1), fd, atol=2e-7)
        fd = O.finite_difference(lambda a: O.gauss_chain_logp(z, mu, with_(s, l, a), u), s[l])
        np.testing.assert_allclose(ds[l], fd, atol=2e-7)
    assert np.all(dz[L - 1] == 0)


def test_layer0_row_grads_agree_with_full_marginals():
    """The spot-check routine for large chains gives the same dz_0 and du_0 rows as the
    full forward-backward gradients (and the same log P)."""
    rng = np.random.default_rng(11)
    Ks, Ds = (9, 7, 5), (4, 3, 2)
    z = [rng.normal(size=(Ks[l], Ds[l])) for l in range(3)]
    mu = [rng.normal(size=(Ks[l + 1], Ds[l])) for l in range(2)]
    s = [rng.uniform(-1, 0, size=Ds[l]) for l in range(2)]
    u = [rng.normal(size=Ks[l]) for l in range(3)]
    lp, dz, dmu, ds, du = O.gauss_chain_grads(z, mu, s, u)
    rows = [0, 3, 8]
    lp2, dz_r, du_r = O.gauss_layer0_row_grads(z, mu, s, u, rows)
    assert abs(lp - lp2) < 1e-12
    assert np.allclose(dz_r, dz[0][rows], rtol=1e-12, atol=1e-14)
    assert np.allclose(du_r, du[0][rows], rtol=1e-12, atol=1e-14)


def test_expanded_factor_equals_direct_difference():
    """The matrix-product form of the factor (large configurations) against the direct
    difference and scipy's normal log-density, at the scale of the 128-wide layers
    (|f| in the hundreds, cancelling terms in the thousands)."""
    rng = np.random.default_rng(21)
    z = rng.normal(0.0, 1.0, size=(48, 128)) + rng.normal(0.0, 1.0, size=128)
    mu = np.tanh(rng.normal(size=(40, 128)))
    s = rng.uniform(-1.0, 0.0, size=128)
    f_dir = O.gauss_pair_logfactor(z, mu, s, chunk=7)
    f_exp = O.gauss_pair_logfactor_expanded(z, mu, s)
    assert np.abs(f_dir).max() > 100.0
    np.testing.assert_allclose(f_exp, f_dir, rtol=0, atol=1e-10 * np.abs(f_dir).max())
    zs, ms, ss = z[:3, :5], mu[:4, :5], s[:5]
    ref = np.array([[stats.norm.logpdf(zs[i], loc=ms[j], scale=np.exp(ss)).sum()
                     for j in range(4)] for i in range(3)])
    np.testing.assert_allclose(O.gauss_pair_logfactor_expanded(zs, ms, ss), ref, rtol=1e-13, atol=1e-12)


def test_expanded_gradients_equal_direct_difference():
    """The matrix-product gradients (large configurations) equal the G-weighted
    direct-difference sums element by element, on a chain with equal K in every layer
    (so that a transposed marginal still has the right shape and must fail on values)."""
    rng = np.random.default_rng(22)
    K, D = (6, 6, 6, 6), (5, 3, 4, 2)
    z, mu, s, u = _rand_chain(rng, K, D, scale=0.8)
    a = O.gauss_chain_grads(z, mu, s, u, chunk=4)
    b = O.gauss_chain_grads_expanded(z, mu, s, u)
    assert abs(a[0] - b[0]) < 1e-12
    for k in range(1, 5):
        for x, y in zip(a[k], b[k]):
            np.testing.assert_allclose(y, x, rtol=1e-10, atol=1e-12 * max(1.0, np.abs(x).max()))


# --- tempered weights and the DReGs surrogate (Appendix "Combining DReGs and TMC") ---

def test_tempered_estimator_equals_enumeration_of_powered_weights():
    rng = np.random.default_rng(31)
    K, D = (3, 4, 2), (2, 3, 2)
    z, mu, s, u = _rand_chain(rng, K, D, scale=0.6)
    f = O.gauss_chain_factors(z, mu, s)
    logw = [sum(u[l][t[l]] for l in range(3)) + sum(f[l][t[l], t[l + 1]] for l in range(2))
            for t in itertools.product(*[range(k) for k in K])]
    for kappa in (1.0, 2.0, 0.5):
        ref = special.logsumexp(kappa * np.array(logw)) - sum(math.log(k) for k in K)
        assert abs(O.tempered_chain_logp(f, u, kappa) - ref) < 1e-11
    assert abs(O.tempered_chain_logp(f, u, 1.0) - O.chain_logp(f, u)) < 1e-12


def test_tempered_gradients_against_enumeration_and_differences():
    """Tempered gradients: the enumeration of kappa * softmax(kappa log w)_t * d log w_t over
    tuples, and central finite differences of the tempered log P."""
    rng = np.random.default_rng(32)
    K, D = (3, 2, 3), (2, 2, 3)
    z, mu, s, u = _rand_chain(rng, K, D, scale=0.6)
    kappa = 2.0
    lp, dz, dmu, ds, du = O.gauss_chain_grads_tempered(z, mu, s, u, kappa)
    bz, bmu, bs, bu = O.brute_force_weighted_grads(
        z, mu, s, u, lambda lw: kappa * np.exp(kappa * lw - special.logsumexp(kappa * lw)))
    for a, b in zip(dz + dmu + ds + du, bz + bmu + bs + bu):
        np.testing.assert_allclose(a, b, rtol=1e-9, atol=1e-12)
    tl = lambda zz, mm, ss, uu: O.tempered_chain_logp(O.gauss_chain_factors(zz, mm, ss), uu, kappa)
    fd = O.finite_difference(lambda a: tl([a, z[1], z[2]], mu, s, u), z[0])
    np.testing.assert_allclose(dz[0].reshape(-1), fd, atol=2e-7)
    fd = O.finite_difference(lambda a: tl(z, [mu[0], a], s, u), mu[1])
    np.testing.assert_allclose(dmu[1].reshape(-1), fd, atol=2e-7)
    fd = O.finite_difference(lambda a: tl(z, mu, [a, s[1]], u), s[0])
    np.testing.assert_allclose(ds[0], fd, atol=2e-7)


def test_dregs_surrogate_gradient_is_the_dregs_estimator():
    """The surrogate's gradient, from two tempered passes, equals the DReGs recognition
    update sum_t w_t^2 / (sum_t w_t)^2 * d log w_t summed over every tuple."""
    rng = np.random.default_rng(33)
    K, D = (2, 3, 2), (2, 2, 2)
    z, mu, s, u = _rand_chain(rng, K, D, scale=0.6)
    c, dz, dmu, ds, du = O.dregs_gradients(z, mu, s, u)
    bz, bmu, bs, bu = O.brute_force_weighted_grads(
        z, mu, s, u, lambda lw: np.exp(2.0 * lw - 2.0 * special.logsumexp(lw)))
    for a, b in zip(dz + dmu + ds + du, bz + bmu + bs + bu):
        np.testing.assert_allclose(a, b, rtol=1e-9, atol=1e-13)
    # coefficient = sum w^2 / (sum w)^2, in (0, 1]
    f = O.gauss_chain_factors(z, mu, s)
    lw = np.array([sum(u[l][t[l]] for l in range(3)) + sum(f[l][t[l], t[l + 1]] for l in range(2))
                   for t in itertools.product(*[range(k) for k in K])])
    assert abs(c - np.exp(special.logsumexp(2 * lw) - 2 * special.logsumexp(lw))) < 1e-12


# --- star model: one global latent, N local latents (Sec. "Efficient averaging") ---

def _rand_star(rng, N, Kt, K, D):
    mth = rng.normal(size=(Kt, D))
    s = rng.uniform(-1.0, 0.0, size=D)
    z = [rng.normal(size=(K, D)) for _ in range(N)]
    u = [rng.normal(size=K) * 2.0 for _ in range(N)]
    uth = rng.normal(size=Kt)
    return mth, s, z, u, uth


def test_star_equals_enumeration_and_one_point_chain():
    rng = np.random.default_rng(41)
    mth, s, z, u, uth = _rand_star(rng, 3, 3, 2, 2)
    f = [O.gauss_pair_logfactor(mth, zi, s) for zi in z]
    assert abs(O.star_logp(uth, f, u) - O.star_brute_force(uth, f, u)) < 1e-11
    # one data point: a chain of two layers (local latent next to the data, theta on top)
    assert abs(O.star_logp(uth, f[:1], u[:1]) - O.chain_logp([f[0].T], [u[0], uth])) < 1e-11
    # permuting the data points leaves the estimate unchanged
    assert abs(O.star_logp(uth, f[::-1], u[::-1]) - O.star_logp(uth, f, u)) < 1e-11


def test_star_marginals_and_gradients_against_differences():
    rng = np.random.default_rng(42)
    mth, s, z, u, uth = _rand_star(rng, 3, 4, 3, 2)
    lp, dm, ds, dz, du, w = O.gauss_star_grads(mth, s, z, u, uth)
    fl = lambda mm, ss, zz, uu, tt: O.star_logp(tt, [O.gauss_pair_logfactor(mm, zi, ss) for zi in zz], uu)
    np.testing.assert_allclose(dm.reshape(-1), O.finite_difference(lambda a: fl(a, s, z, u, uth), mth), atol=2e-7)
    np.testing.assert_allclose(ds, O.finite_difference(lambda a: fl(mth, a, z, u, uth), s), atol=2e-7)
    np.testing.assert_allclose(dz[1].reshape(-1),
                               O.finite_difference(lambda a: fl(mth, s, [z[0], a, z[2]], u, uth), z[1]), atol=2e-7)
    np.testing.assert_allclose(du[2], O.finite_difference(lambda a: fl(mth, s, z, [u[0], u[1], a], uth), u[2]), atol=2e-7)
    np.testing.assert_allclose(w, O.finite_difference(lambda a: fl(mth, s, z, u, a), uth), atol=2e-7)
    assert abs(w.sum() - 1.0) < 1e-12 and all(abs(d.sum() - 1.0) < 1e-12 for d in du)


@pytest.mark.slow
def test_star_estimate_unbiased_for_the_gaussian_model():
    """The paper's Gaussian star model (theta ~ N(0,1), z_i | theta ~ N(theta, 1),
    x_i | z_i ~ N(z_i, 1); proposals N(0, 1) for theta and N(0, 2) for z_i): the mean of
    exp(log P_TMC - log P(x)) over independent replicates is 1 within 4 standard errors."""
    rng = np.random.default_rng(43)
    N, K, Kt, R = 4, 16, 16, 3000
    x = rng.normal(size=N) * np.sqrt(3.0)
    lpx = O.gauss_star_log_evidence(x)
    ratios = []
    for _ in range(R):
        th = rng.normal(size=Kt)
        zs = [rng.normal(size=K) * np.sqrt(2.0) for _ in range(N)]
        uth = stats.norm.logpdf(th) - stats.norm.logpdf(th)                  # P(theta)/Q(theta)
        u = [stats.norm.logpdf(x[i], loc=zs[i]) - stats.norm.logpdf(zs[i], scale=np.sqrt(2.0))
             for i in range(N)]
        f = [O.gauss_pair_logfactor(th[:, None], zs[i][:, None], np.zeros(1)) for i in range(N)]
        ratios.append(np.exp(O.star_logp(uth, f, u) - lpx))
    ratios = np.array(ratios)
    assert abs(ratios.mean() - 1.0) < 4.0 * ratios.std() / np.sqrt(R), (ratios.mean(), ratios.std())


def test_star_evidence_closed_form_against_quadrature():
    x = np.array([0.3, -1.2, 0.8])
    # integrate theta out numerically: x_i | theta ~ N(theta, 2) independently
    val, _ = integrate.quad(lambda t: stats.norm.pdf(t) * np.prod(stats.norm.pdf(x, loc=t, scale=np.sqrt(2.0))),
                            -12, 12)
    assert abs(O.gauss_star_log_evidence(x) - np.log(val)) < 1e-9


# --- parent-dependent scale (sigma produced from the parent sample) ------------------

def _rand_chain_pp(rng, K, D, scale=1.0):
    z, mu, s, u = _rand_chain(rng, K, D, scale=scale)
    sp = [rng.uniform(-1.0, 0.3, size=(K[l + 1], D[l])) for l in range(len(K) - 1)]
    return z, mu, sp, u


def test_pp_factor_equals_scipy_normal_logpdf():
    """Each parent sample j brings its own scale exp(sp[j])."""
    rng = np.random.default_rng(41)
    z = rng.normal(size=(5, 4))
    mu = rng.normal(size=(6, 4))
    sp = rng.uniform(-1.5, 0.5, size=(6, 4))
    f = O.gauss_pair_logfactor_pp(z, mu, sp, chunk=2)
    ref = np.array([[stats.norm.logpdf(z[i], loc=mu[j], scale=np.exp(sp[j])).sum()
                     for j in range(6)] for i in range(5)])
    np.testing.assert_allclose(f, ref, rtol=1e-13, atol=1e-12)


def test_pp_with_equal_rows_reduces_to_shared_scale():
    """When every parent produces the same scale, the factor, log P and every gradient
    equal those of the shared-scale chain, with ds = the sum over parents of dsp."""
    rng = np.random.default_rng(42)
    K, D = (5, 4, 6), (3, 2, 4)
    z, mu, s, u = _rand_chain(rng, K, D)
    sp = [np.tile(s[l], (K[l + 1], 1)) for l in range(len(K) - 1)]
    a = O.gauss_chain_grads(z, mu, s, u)
    b = O.gauss_chain_grads_pp(z, mu, sp, u)
    assert abs(a[0] - b[0]) < 1e-12
    for l in range(len(K)):
        np.testing.assert_allclose(b[1][l], a[1][l], atol=1e-12)
        np.testing.assert_allclose(b[4][l], a[4][l], atol=1e-12)
    for l in range(len(K) - 1):
        np.testing.assert_allclose(b[2][l], a[2][l], atol=1e-12)
        np.testing.assert_allclose(b[3][l].sum(axis=0), a[3][l], atol=1e-11)


def test_pp_chain_equals_brute_force():
    rng = np.random.default_rng(43)
    K, D = (3, 4, 2, 3), (2, 3, 1, 2)
    z, mu, sp, u = _rand_chain_pp(rng, K, D)
    f = [O.gauss_pair_logfactor_pp(z[l], mu[l], sp[l]) for l in range(len(K) - 1)]
    assert abs(O.gauss_chain_logp_pp(z, mu, sp, u) - O.brute_force_logp(f, u)) < 1e-10


def test_pp_gradients_against_finite_differences():
    rng = np.random.default_rng(44)
    K, D = (4, 5, 3), (3, 2, 2)
    z, mu, sp, u = _rand_chain_pp(rng, K, D, scale=0.7)
    logp, dz, dmu, dsp, du = O.gauss_chain_grads_pp(z, mu, sp, u, chunk=2)
    L = len(K)

    def with_(lst, l, a):
        return [a if m == l else lst[m] for m in range(len(lst))]

    for l in range(L):
        fd = O.finite_difference(lambda a: O.gauss_chain_logp_pp(with_(z, l, a), mu, sp, u), z[l])
        np.testing.assert_allclose(dz[l].reshape(-1), fd, atol=2e-7)
        fd = O.finite_difference(lambda a: O.gauss_chain_logp_pp(z, mu, sp, with_(u, l, a)), u[l])
        np.testing.assert_allclose(du[l], fd, atol=2e-7)
    for l in range(L - 1):
        fd = O.finite_difference(lambda a: O.gauss_chain_logp_pp(z, with_(mu, l, a), sp, u), mu[l])
        np.testing.assert_allclose(dmu[l].reshape(-1), fd, atol=2e-7)
        fd = O.finite_difference(lambda a: O.gauss_chain_logp_pp(z, mu, with_(sp, l, a), u), sp[l])
        np.testing.assert_allclose(dsp[l].reshape(-1), fd, atol=2e-7)
    assert np.all(dz[L - 1] == 0)


# --- log-domain matrix product (matrix-matrix form) ------------------------------

def test_logmmexp_equals_scipy_and_matrix_product():
    """Against scipy's logsumexp written per entry, and against log(exp(X) @ exp(Y)) where
    the plain product cannot under- or overflow."""
    rng = np.random.default_rng(51)
    X = rng.normal(size=(2, 5, 7)) * 3
    Y = rng.normal(size=(2, 7, 4)) * 3
    Z = O.logmmexp(X, Y)
    for b in range(2):
        for i in range(5):
            for k in range(4):
                assert abs(Z[b, i, k] - special.logsumexp(X[b, i, :] + Y[b, :, k])) < 1e-12
    np.testing.assert_allclose(Z, np.log(np.exp(X) @ np.exp(Y)), rtol=1e-12, atol=1e-12)


def test_logmmexp_chain_is_the_discrete_tmc_estimator():
    """Summing a discrete chain's indices with matrix-matrix log-products (several chains
    at once, their messages as columns) gives the chain estimator of eq. (is) of each."""
    rng = np.random.default_rng(52)
    K = (4, 5, 3)
    chains = []
    for c in range(3):
        f = [rng.normal(size=(K[l], K[l + 1])) for l in range(2)]
        u = [rng.normal(size=k) for k in K]
        chains.append((f, u))
    # M[l][i, j] = u_l[i] + f_l[i, j] - ln K_{l+1}: one chain per batch entry
    prod = None
    for l in range(2):
        M = np.stack([ch[1][l][:, None] + ch[0][l] - O.log_k(K[l + 1]) for ch in chains])
        prod = M if prod is None else O.logmmexp(prod, M)
    top = np.stack([ch[1][2] for ch in chains])[:, :, None]            # [c, K_top, 1]
    col = O.logmmexp(prod, top)[:, :, 0]                               # [c, K_0]
    got = O.logsumexp(col, axis=1) - O.log_k(K[0])
    for c, (f, u) in enumerate(chains):
        assert abs(got[c] - O.brute_force_logp(f, u)) < 1e-11


def test_logmmexp_where_the_operand_shift_underflows():
    """X_i peaks at j = 0 and Y_k at j = 1: every product of the per-operand shifted
    exponentials underflows (the Appendix's form gives -inf), while the exact value is
    finite: max_j (X_ij + Y_jk) = -800."""
    X = np.array([[0.0, -900.0]])
    Y = np.array([[-800.0], [0.0]])
    with np.errstate(over="ignore", under="ignore"):
        assert O.logmmexp_shifted(X, Y)[0, 0] == -np.inf
    z = O.logmmexp(X, Y)[0, 0]
    assert abs(z - (-800.0 + np.log1p(np.exp(-100.0)))) < 1e-12
    # all -inf rows and columns give -inf, never NaN
    X2 = np.array([[-np.inf, -np.inf], [0.0, 1.0]])
    Z2 = O.logmmexp(X2, np.zeros((2, 3)))
    assert np.all(Z2[0] == -np.inf) and np.all(np.isfinite(Z2[1]))
