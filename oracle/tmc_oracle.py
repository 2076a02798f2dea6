"""FP64 CPU oracle for the Tensor Monte Carlo (TMC) chain estimator.

TEST INFRASTRUCTURE ONLY.  The library never imports, calls, links or executes
anything here; only the test-suite, the smoke check and the benchmark's
CPU-baseline leg do.  It shares no code, constants or helpers with the HIP path.

Paper: L. Aitchison, "Tensor Monte Carlo: Particle Methods for the GPU Era",
arXiv 1806.08593.  Every function names the passage it follows.

Conventions (0-based layers, layer 0 is adjacent to the data x, layer L-1 is the
top of the chain):
    z[l]  [K_l, D_l]      samples of layer l
    mu[l] [K_{l+1}, D_l]  mean of z_l given sample j of its parent z_{l+1}
    s[l]  [D_l]           log std of P(z_l | z_{l+1}), shared by all parent samples
    sp[l] [K_{l+1}, D_l]  (the *_pp functions) log std given parent sample j
    u[l]  [K_l]           unary log-terms (-log Q(z_l), log-likelihood on layer 0,
                          log-prior on the top layer)
    f[l]  [K_l, K_{l+1}]  pairwise log-factor log P(z_l^i | z_{l+1}^j)

Parity pins (tests/test_oracle_*.py) tie each function to something outside
itself: brute-force enumeration of eq. (is), the IWAE and VAE special cases, the
exact discrete marginalisation of the Appendix (an HMM evaluated in probability
space), closed-form linear-Gaussian evidence, scipy's normal log-density,
finite differences and exact invariants.
"""
from __future__ import annotations

import itertools
import math
from typing import List, Sequence

import numpy as np

# ---------------------------------------------------------------------------
# small helpers (kept separate so tests can plant mistakes in them)
# ---------------------------------------------------------------------------

HALF_LOG_2PI = 0.5 * math.log(2.0 * math.pi)


def log_k(K: int) -> float:
    """ln K_l: the 1/K_l of eq. (is), paid once per latent layer."""
    return math.log(K)


def logsumexp(a: np.ndarray, axis: int) -> np.ndarray:
    """log sum exp along `axis`, shifted by the exact maximum (the Appendix's
    numerically stable log-domain product, with x_i = max_j X_ij).  A slice that is
    all -inf gives -inf (never NaN); NaN propagates."""
    a = np.asarray(a, dtype=np.float64)
    m = np.max(a, axis=axis, keepdims=True)
    m_safe = np.where(np.isfinite(m), m, 0.0)
    with np.errstate(divide="ignore"):
        out = np.log(np.sum(np.exp(a - m_safe), axis=axis, keepdims=True)) + m_safe
    return np.squeeze(out, axis=axis)


# ---------------------------------------------------------------------------
# factors (eq. (fac), Appendix "typical choice of factors", Gaussian conditional
# of Sec. "Computational costs for TMC and IWAE")
# ---------------------------------------------------------------------------

def gauss_pair_logfactor(z: np.ndarray, mu: np.ndarray, s: np.ndarray,
                         chunk: int = 256) -> np.ndarray:
    """f[i, j] = log N(z^i ; mu^j, diag exp(2 s)), written out by direct difference:
        sum_d [ -1/2 exp(-2 s_d) (z_id - mu_jd)^2 - s_d - 1/2 log 2 pi ].
    This is the latent factor P(z_l | z_{l+1}) of the chain model; the 1/Q(z_l) part
    of the Appendix's factor is a row term and is carried in u[l]."""
    z = np.asarray(z, np.float64)
    mu = np.asarray(mu, np.float64)
    s = np.asarray(s, np.float64)
    lam = np.exp(-2.0 * s)
    const = -np.sum(s) - z.shape[1] * HALF_LOG_2PI
    out = np.empty((z.shape[0], mu.shape[0]))
    for i0 in range(0, z.shape[0], chunk):
        diff = z[i0:i0 + chunk, None, :] - mu[None, :, :]
        out[i0:i0 + chunk] = -0.5 * np.sum(lam * diff * diff, axis=-1) + const
    return out


def gauss_chain_factors(z: Sequence[np.ndarray], mu: Sequence[np.ndarray],
                        s: Sequence[np.ndarray]) -> List[np.ndarray]:
    return [gauss_pair_logfactor(z[l], mu[l], s[l]) for l in range(len(mu))]


# ---------------------------------------------------------------------------
# the estimator (eq. (is)) and its chain evaluation (Sec. "Efficient averaging")
# ---------------------------------------------------------------------------

def brute_force_logp(f: Sequence[np.ndarray], u: Sequence[np.ndarray]) -> float:
    """eq. (is) written out: log of the average, over every tuple (k_0..k_{L-1}), of
    exp(sum_l u_l[k_l] + sum_l f_l[k_l, k_{l+1}]).  Exponential in L: tiny chains only."""
    L = len(u)
    K = [len(a) for a in u]
    terms = []
    for ks in itertools.product(*[range(k) for k in K]):
        t = sum(u[l][ks[l]] for l in range(L))
        t += sum(f[l][ks[l], ks[l + 1]] for l in range(L - 1))
        terms.append(t)
    return float(logsumexp(np.array(terms), axis=0) - sum(log_k(k) for k in K))


def chain_messages(f: Sequence[np.ndarray], u: Sequence[np.ndarray]):
    """Sum the indices out one at a time, from the top of the chain down (the
    sum/product swap of Sec. "Efficient averaging", each step a log-domain
    matrix-vector product as in the Appendix):
        alpha_{L-1} = u_{L-1}
        alpha_l[i]  = u_l[i] + logsumexp_j(f_l[i, j] + alpha_{l+1}[j]) - ln K_{l+1}
        log P_TMC   = logsumexp_i(alpha_0[i]) - ln K_0
    Returns (log P_TMC, [alpha_0 .. alpha_{L-1}])."""
    L = len(u)
    alpha = [None] * L
    alpha[L - 1] = np.asarray(u[L - 1], np.float64)
    for l in range(L - 2, -1, -1):
        K_up = len(u[l + 1])
        alpha[l] = u[l] + logsumexp(f[l] + alpha[l + 1][None, :], axis=1) - log_k(K_up)
    logp = float(logsumexp(alpha[0], axis=0) - log_k(len(u[0])))
    return logp, alpha


def chain_logp(f: Sequence[np.ndarray], u: Sequence[np.ndarray]) -> float:
    return chain_messages(f, u)[0]


def chain_marginals(f: Sequence[np.ndarray], u: Sequence[np.ndarray]):
    """Derivatives of log P_TMC with respect to the log-factors and unaries.

    log P_TMC is a log-sum-exp over index tuples, so d log P / d f_l[i, j] is the
    weight of all tuples with k_l = i, k_{l+1} = j (a pairwise marginal over sample
    indices), and d log P / d u_l[k] the weight of tuples with k_l = k.  These follow
    from bottom-up messages
        beta_0 = -ln K_0
        beta_{l+1}[j] = logsumexp_i(beta_l[i] + u_l[i] + f_l[i, j]) - ln K_{l+1}
    combined with the top-down alpha:
        G_l[i, j] = exp(beta_l[i] + u_l[i] + f_l[i, j] + alpha_{l+1}[j] - ln K_{l+1} - log P)
        p_l[k]    = exp(beta_l[k] + alpha_l[k] - log P).
    Returns (log P, G list, p list)."""
    L = len(u)
    logp, alpha = chain_messages(f, u)
    beta = [None] * L
    beta[0] = np.full(len(u[0]), -log_k(len(u[0])))
    for l in range(L - 1):
        beta[l + 1] = (logsumexp((beta[l] + u[l])[:, None] + f[l], axis=0)
                       - log_k(len(u[l + 1])))
    G = []
    for l in range(L - 1):
        e = ((beta[l] + u[l])[:, None] + f[l] + alpha[l + 1][None, :]
             - log_k(len(u[l + 1])) - logp)
        G.append(np.exp(e))
    p = [np.exp(beta[l] + alpha[l] - logp) for l in range(L)]
    return logp, G, p


# ---------------------------------------------------------------------------
# Gaussian chain: value and gradients
# ---------------------------------------------------------------------------

def gauss_chain_logp(z, mu, s, u) -> float:
    return chain_logp(gauss_chain_factors(z, mu, s), u)


def gauss_chain_grads(z, mu, s, u, chunk: int = 128):
    """log P_TMC and its gradients with respect to z, mu, s and u for the Gaussian
    chain (the reparameterised-gradient objective of Sec. "Efficient averaging",
    obtained there by automatic differentiation).  By the chain rule through the
    factors, with G the pairwise marginals of `chain_marginals` and lam = exp(-2 s):
        dz_l[i]  = sum_j G_l[i,j] * (-lam * (z_l[i] - mu_l[j]))
        dmu_l[j] = sum_i G_l[i,j] * ( lam * (z_l[i] - mu_l[j]))
        ds_l     = sum_ij G_l[i,j] * ( lam * (z_l[i] - mu_l[j])^2 - 1 )
        du_l     = p_l
    The top layer's samples enter only through mu and u, so dz of layer L-1 is 0.
    Returns (log P, dz list, dmu list, ds list, du list)."""
    f = gauss_chain_factors(z, mu, s)
    logp, G, p = chain_marginals(f, u)
    L = len(u)
    dz = [np.zeros_like(np.asarray(a, np.float64)) for a in z]
    dmu, ds = [], []
    for l in range(L - 1):
        lam = np.exp(-2.0 * np.asarray(s[l], np.float64))
        zl = np.asarray(z[l], np.float64)
        ml = np.asarray(mu[l], np.float64)
        gmu = np.zeros_like(ml)
        gs = np.zeros_like(lam)
        for i0 in range(0, zl.shape[0], chunk):
            diff = zl[i0:i0 + chunk, None, :] - ml[None, :, :]       # [i, j, d]
            g = G[l][i0:i0 + chunk, :, None]
            dz[l][i0:i0 + chunk] = np.sum(g * (-lam * diff), axis=1)
            gmu += np.sum(g * (lam * diff), axis=0)
            gs += np.sum(g * (lam * diff * diff - 1.0), axis=(0, 1))
        dmu.append(gmu)
        ds.append(gs)
    return logp, dz, dmu, ds, [np.asarray(a) for a in p]


def gauss_layer0_row_grads(z, mu, s, u, rows):
    """log P_TMC and, for the listed sample indices i of layer 0 (the layer next to the
    data), dlogP/dz_0[i] and dlogP/du_0[i], without forming every pairwise marginal:
    layer 0 is where the bottom-up message starts, beta_0 = -ln K_0, so its marginals
    need only the top-down messages (see `chain_marginals`):
        G_0[i, j] = exp(beta_0 + u_0[i] + f_0[i, j] + alpha_1[j] - ln K_1 - log P)
        dz_0[i]   = sum_j G_0[i, j] * (-lam * (z_0[i] - mu_0[j]))
        du_0[i]   = exp(beta_0 + alpha_0[i] - log P)
    For spot checks of large chains.  Returns (log P, dz rows [n, D_0], du rows [n])."""
    f = gauss_chain_factors(z, mu, s)
    logp, alpha = chain_messages(f, u)
    rows = np.asarray(rows, dtype=np.int64)
    K0, K1 = len(u[0]), len(u[1])
    beta0 = -log_k(K0)
    lam = np.exp(-2.0 * np.asarray(s[0], np.float64))
    z0 = np.asarray(z[0], np.float64)
    m0 = np.asarray(mu[0], np.float64)
    e = (beta0 + np.asarray(u[0], np.float64)[rows][:, None] + f[0][rows]
         + alpha[1][None, :] - log_k(K1) - logp)
    G = np.exp(e)                                             # [n, K1]
    diff = z0[rows][:, None, :] - m0[None, :, :]              # [n, K1, D]
    dz = np.sum(G[:, :, None] * (-lam * diff), axis=1)
    du = np.exp(beta0 + alpha[0][rows] - logp)
    return logp, dz, du


def gauss_pair_logfactor_expanded(z: np.ndarray, mu: np.ndarray, s: np.ndarray) -> np.ndarray:
    """The same f[i, j] as `gauss_pair_logfactor`, with the square written out,
        sum_d lam_d (z_id - mu_jd)^2 = sum_d lam_d z_id^2 - 2 sum_d lam_d z_id mu_jd
                                       + sum_d lam_d mu_jd^2,
    so that the cross term is one matrix product.  For the large configurations only
    (K in the thousands), where the direct difference would take minutes; FP64 keeps
    the cancellation of the three terms (each at most a few thousand) near 1e-12."""
    z = np.asarray(z, np.float64)
    mu = np.asarray(mu, np.float64)
    s = np.asarray(s, np.float64)
    lam = np.exp(-2.0 * s)
    const = -np.sum(s) - z.shape[1] * HALF_LOG_2PI
    zz = np.sum(lam * z * z, axis=1)
    mm = np.sum(lam * mu * mu, axis=1)
    cross = (z * lam) @ mu.T
    return -0.5 * (zz[:, None] - 2.0 * cross + mm[None, :]) + const


def gauss_chain_grads_expanded(z, mu, s, u):
    """`gauss_chain_grads` with the factors of `gauss_pair_logfactor_expanded` and the
    G-weighted sums over (z_i - mu_j) written as matrix products (same quantities,
    the differences expanded):
        dz_l[i]  = -lam * (rG_i z_l[i] - (G mu_l)_i),          rG = G 1 (row sums)
        dmu_l[j] =  lam * ((G^T z_l)_j - cG_j mu_l[j]),         cG = G^T 1 (column sums)
        ds_l     =  lam * (sum_i rG_i z_i^2 - 2 sum_j (G^T z_l)_j mu_j + sum_j cG_j mu_j^2)
                    - sum_ij G_ij
    For the large configurations.  Returns (log P, dz, dmu, ds, du) like
    `gauss_chain_grads`."""
    f = [gauss_pair_logfactor_expanded(z[l], mu[l], s[l]) for l in range(len(mu))]
    logp, G, p = chain_marginals(f, u)
    L = len(u)
    dz = [np.zeros_like(np.asarray(a, np.float64)) for a in z]
    dmu, ds = [], []
    for l in range(L - 1):
        lam = np.exp(-2.0 * np.asarray(s[l], np.float64))
        zl = np.asarray(z[l], np.float64)
        ml = np.asarray(mu[l], np.float64)
        g = G[l]
        rG = g.sum(axis=1)
        cG = g.sum(axis=0)
        gmu = g @ ml
        gtz = g.T @ zl
        dz[l] = -lam * (rG[:, None] * zl - gmu)
        dmu.append(lam * (gtz - cG[:, None] * ml))
        ds.append(lam * (rG @ (zl * zl) - 2.0 * np.sum(gtz * ml, axis=0) + cG @ (ml * ml))
                  - g.sum())
    return logp, dz, dmu, ds, [np.asarray(a) for a in p]


def tempered_chain_logp(f: Sequence[np.ndarray], u: Sequence[np.ndarray], kappa: float) -> float:
    """log of the average over all index tuples of w_t**kappa, w_t the importance weight of
    tuple t (eq. (is) with every weight raised to the power kappa): the chain evaluation
    with every log-factor and unary multiplied by kappa.  kappa = 2 gives the sum of
    squared weights that Appendix "Combining DReGs and TMC" obtains by running TMC again
    with squared weights."""
    return chain_logp([kappa * np.asarray(a, np.float64) for a in f],
                      [kappa * np.asarray(a, np.float64) for a in u])


def gauss_chain_grads_tempered(z, mu, s, u, kappa: float):
    """log of the kappa-tempered estimator (`tempered_chain_logp` of the Gaussian chain) and
    its gradients.  Each tuple's weight enters as exp(kappa log w_t), so with G the
    pairwise marginals of the tempered chain and lam = exp(-2 s):
        dz_l[i]  = kappa sum_j G_l[i,j] (-lam (z_l[i] - mu_l[j]))
        dmu_l[j] = kappa sum_i G_l[i,j] ( lam (z_l[i] - mu_l[j]))
        ds_l     = kappa sum_ij G_l[i,j] (lam (z_l[i] - mu_l[j])^2 - 1)
        du_l     = kappa p_l
    Returns (log P_kappa, dz, dmu, ds, du)."""
    f = gauss_chain_factors(z, mu, s)
    logp, G, p = chain_marginals([kappa * a for a in f], [kappa * np.asarray(a, np.float64) for a in u])
    L = len(u)
    dz = [np.zeros_like(np.asarray(a, np.float64)) for a in z]
    dmu, ds = [], []
    for l in range(L - 1):
        lam = np.exp(-2.0 * np.asarray(s[l], np.float64))
        diff = np.asarray(z[l], np.float64)[:, None, :] - np.asarray(mu[l], np.float64)[None, :, :]
        g = G[l][:, :, None]
        dz[l] = kappa * np.sum(g * (-lam * diff), axis=1)
        dmu.append(kappa * np.sum(g * (lam * diff), axis=0))
        ds.append(kappa * np.sum(g * (lam * diff * diff - 1.0), axis=(0, 1)))
    return logp, dz, dmu, ds, [kappa * np.asarray(a) for a in p]


def dregs_gradients(z, mu, s, u):
    """Gradients of the DReGs surrogate of Appendix "Combining DReGs and TMC",
        1/2 * stopgrad(sum_t w_t^2 / (sum_t w_t)^2) * log sum_t w_t^2,
    with respect to the inputs through which the weights' gradients flow (the caller
    stops the direct dependence on the proposal parameters in u): the coefficient is
    exp(logP_2 - 2 logP_1 - sum_l ln K_l) with logP_kappa the kappa-tempered estimator,
    and d log sum_t w_t^2 = d logP_2.  By the paper's derivation this equals
    sum_t w_t^2 / (sum_t w_t)^2 * d log w_t.  Returns (coefficient, dz, dmu, ds, du)."""
    lp1 = gauss_chain_logp(z, mu, s, u)
    lp2, dz, dmu, ds, du = gauss_chain_grads_tempered(z, mu, s, u, 2.0)
    c = math.exp(lp2 - 2.0 * lp1 - sum(log_k(len(a)) for a in u))
    h = 0.5 * c
    return c, [h * a for a in dz], [h * a for a in dmu], [h * a for a in ds], [h * a for a in du]


def brute_force_weighted_grads(z, mu, s, u, weight):
    """sum over every index tuple t of weight(log w) [t] * d log w_t, with d log w_t written
    out per tuple (the factors' and unaries' own derivatives); `weight` maps the vector of
    log weights of all tuples to per-tuple coefficients.  Exponential in L: tiny chains.
    Returns (dz, dmu, ds, du)."""
    L = len(u)
    K = [len(a) for a in u]
    f = gauss_chain_factors(z, mu, s)
    tuples = list(itertools.product(*[range(k) for k in K]))
    logw = np.array([sum(u[l][t[l]] for l in range(L)) + sum(f[l][t[l], t[l + 1]] for l in range(L - 1))
                     for t in tuples])
    wt = weight(logw)
    dz = [np.zeros_like(np.asarray(a, np.float64)) for a in z]
    dmu = [np.zeros_like(np.asarray(a, np.float64)) for a in mu]
    ds = [np.zeros_like(np.asarray(a, np.float64)) for a in s]
    du = [np.zeros(k) for k in K]
    for c, t in zip(wt, tuples):
        for l in range(L):
            du[l][t[l]] += c
        for l in range(L - 1):
            lam = np.exp(-2.0 * np.asarray(s[l], np.float64))
            d = np.asarray(z[l][t[l]], np.float64) - np.asarray(mu[l][t[l + 1]], np.float64)
            dz[l][t[l]] += c * (-lam * d)
            dmu[l][t[l + 1]] += c * (lam * d)
            ds[l] += c * (lam * d * d - 1.0)
    return dz, dmu, ds, du


# ---------------------------------------------------------------------------
# star-shaped model: one global latent, N local latents (Sec. "Efficient averaging",
# the latent-variable model with unknown parameters theta)
# ---------------------------------------------------------------------------

def star_logp(uth: np.ndarray, f: Sequence[np.ndarray], u: Sequence[np.ndarray]) -> float:
    """TMC estimate of the star model: K_theta samples of the global latent theta (unary
    log-terms uth[kt]) and, for each data point i, K_i samples of its local latent
    (unaries u[i][k]) joined to theta by the log-factor f[i][kt, k].  Summing the local
    indices out first, then theta:
        log P = logsumexp_kt( uth[kt] + sum_i [logsumexp_k(f[i][kt, k] + u[i][k]) - ln K_i] )
                - ln K_theta."""
    uth = np.asarray(uth, np.float64)
    a = uth.copy()
    for fi, ui in zip(f, u):
        a = a + logsumexp(np.asarray(fi, np.float64) + np.asarray(ui, np.float64)[None, :], axis=1) \
            - log_k(len(ui))
    return float(logsumexp(a, axis=0) - log_k(len(uth)))


def star_brute_force(uth, f, u) -> float:
    """eq. (is) for the star model written out: log of the average over every tuple
    (kt, k_1 .. k_N) of exp(uth[kt] + sum_i (f[i][kt, k_i] + u[i][k_i])).  Tiny cases only."""
    Ks = [len(a) for a in u]
    terms = []
    for kt in range(len(uth)):
        for ks in itertools.product(*[range(k) for k in Ks]):
            terms.append(uth[kt] + sum(f[i][kt, ks[i]] + u[i][ks[i]] for i in range(len(u))))
    return float(logsumexp(np.array(terms), axis=0) - log_k(len(uth)) - sum(log_k(k) for k in Ks))


def star_marginals(uth, f, u):
    """d log P / d uth[kt] = w[kt] (the weight of global sample kt) and
    d log P / d f[i][kt, k] = G_i[kt, k] = w[kt] * softmax_k(f[i][kt, k] + u[i][k]) (= d / d u[i][k]
    summed over kt).  Returns (log P, w, [G_i])."""
    uth = np.asarray(uth, np.float64)
    msg = [logsumexp(np.asarray(fi, np.float64) + np.asarray(ui, np.float64)[None, :], axis=1)
           - log_k(len(ui)) for fi, ui in zip(f, u)]
    a = uth + sum(msg) if msg else uth.copy()
    logp = float(logsumexp(a, axis=0) - log_k(len(uth)))
    w = np.exp(a - log_k(len(uth)) - logp)
    G = []
    for fi, ui, mi in zip(f, u, msg):
        G.append(w[:, None] * np.exp(np.asarray(fi, np.float64) + np.asarray(ui, np.float64)[None, :]
                                     - (mi + log_k(len(ui)))[:, None]))
    return logp, w, G


def gauss_star_grads(mth, s, z, u, uth):
    """Star model with Gaussian local conditionals z_i | theta^kt ~ N(mth[kt], diag exp(2 s))
    (mth[kt] the mean produced from global sample kt): f[i][kt, k] = log N(z[i][k]; mth[kt], .)
    by direct difference.  Returns (log P, d mth [Kt, D], d s [D], d z [N][K, D], d u [N][K],
    d uth [Kt]); with G_i the marginals of `star_marginals` and lam = exp(-2 s):
        d mth[kt] = sum_i sum_k G_i[kt, k] lam (z_ik - mth[kt])
        d z_ik    = sum_kt G_i[kt, k] (-lam (z_ik - mth[kt]))
        d s       = sum_i sum_{kt, k} G_i[kt, k] (lam (z_ik - mth[kt])^2 - 1)."""
    mth = np.asarray(mth, np.float64)
    lam = np.exp(-2.0 * np.asarray(s, np.float64))
    f = [gauss_pair_logfactor(mth, zi, s) for zi in z]   # [Kt, K] (the density is symmetric)
    logp, w, G = star_marginals(uth, f, u)
    dm = np.zeros_like(mth)
    ds = np.zeros_like(lam)
    dz, du = [], []
    for zi, gi in zip(z, G):
        diff = np.asarray(zi, np.float64)[None, :, :] - mth[:, None, :]      # [Kt, K, D]
        g = gi[:, :, None]
        dm += np.sum(g * (lam * diff), axis=1)
        dz.append(np.sum(g * (-lam * diff), axis=0))
        ds += np.sum(g * (lam * diff * diff - 1.0), axis=(0, 1))
        du.append(gi.sum(axis=0))
    return logp, dm, ds, dz, du, w


def gauss_star_log_evidence(x: np.ndarray) -> float:
    """Exact log P(x) of the Gaussian model of Sec. "Comparing TMC, SMC and IWAE":
    theta ~ N(0, 1), z_i | theta ~ N(theta, 1), x_i | z_i ~ N(z_i, 1), so x is Gaussian
    with mean 0 and covariance 1 1^T + 2 I."""
    from scipy.stats import multivariate_normal
    n = len(x)
    return float(multivariate_normal(mean=np.zeros(n), cov=np.ones((n, n)) + 2.0 * np.eye(n)).logpdf(x))


# ---------------------------------------------------------------------------
# parent-dependent scale: the general conditional N(z_l; mu(z_{l+1}), diag sigma(z_{l+1})^2)
# of Sec. "Computational costs for TMC and IWAE" (the generative networks of Sec.
# "Experiments" produce a standard deviation from the parent as well as a mean)
# ---------------------------------------------------------------------------

def gauss_pair_logfactor_pp(z: np.ndarray, mu: np.ndarray, sp: np.ndarray,
                            chunk: int = 256) -> np.ndarray:
    """f[i, j] = log N(z^i ; mu^j, diag exp(2 sp[j])), where sp [K_{l+1}, D] holds the log
    standard deviation produced from parent sample j (as mu[j] holds its mean).  Direct
    difference:  sum_d [ -1/2 exp(-2 sp_jd) (z_id - mu_jd)^2 - sp_jd - 1/2 log 2 pi ]."""
    z = np.asarray(z, np.float64)
    mu = np.asarray(mu, np.float64)
    sp = np.asarray(sp, np.float64)
    lam = np.exp(-2.0 * sp)                                  # [J, D]
    const = -np.sum(sp, axis=1) - z.shape[1] * HALF_LOG_2PI   # [J]
    out = np.empty((z.shape[0], mu.shape[0]))
    for i0 in range(0, z.shape[0], chunk):
        diff = z[i0:i0 + chunk, None, :] - mu[None, :, :]
        out[i0:i0 + chunk] = -0.5 * np.sum(lam[None, :, :] * diff * diff, axis=-1) + const[None, :]
    return out


def gauss_chain_logp_pp(z, mu, sp, u) -> float:
    """log P_TMC of a Gaussian chain whose scales depend on the parent sample."""
    L = len(u)
    f = [gauss_pair_logfactor_pp(z[l], mu[l], sp[l]) for l in range(L - 1)]
    return chain_logp(f, u)


def gauss_chain_grads_pp(z, mu, sp, u, chunk: int = 128):
    """log P_TMC and its gradients for parent-dependent scales, by the chain rule through
    the factors with G the pairwise marginals of `chain_marginals` and
    lam_j = exp(-2 sp[j]) (the scale of parent sample j):
        dz_l[i]   = sum_j G_l[i,j] * (-lam_j * (z_l[i] - mu_l[j]))
        dmu_l[j]  = sum_i G_l[i,j] * ( lam_j * (z_l[i] - mu_l[j]))
        dsp_l[j]  = sum_i G_l[i,j] * ( lam_j * (z_l[i] - mu_l[j])^2 - 1 )
        du_l      = p_l
    Returns (log P, dz list, dmu list, dsp list, du list)."""
    L = len(u)
    f = [gauss_pair_logfactor_pp(z[l], mu[l], sp[l]) for l in range(L - 1)]
    logp, G, p = chain_marginals(f, u)
    dz = [np.zeros_like(np.asarray(a, np.float64)) for a in z]
    dmu, dsp = [], []
    for l in range(L - 1):
        lam = np.exp(-2.0 * np.asarray(sp[l], np.float64))    # [J, D]
        zl = np.asarray(z[l], np.float64)
        ml = np.asarray(mu[l], np.float64)
        gmu = np.zeros_like(ml)
        gs = np.zeros_like(lam)
        for i0 in range(0, zl.shape[0], chunk):
            diff = zl[i0:i0 + chunk, None, :] - ml[None, :, :]       # [i, j, d]
            g = G[l][i0:i0 + chunk, :, None]
            dz[l][i0:i0 + chunk] = np.sum(g * (-lam[None] * diff), axis=1)
            gmu += np.sum(g * (lam[None] * diff), axis=0)
            gs += np.sum(g * (lam[None] * diff * diff - 1.0), axis=0)
        dmu.append(gmu)
        dsp.append(gs)
    return logp, dz, dmu, dsp, [np.asarray(a) for a in p]


# ---------------------------------------------------------------------------
# log-domain matrix product (Appendix "Numerically stable matrix (tensor) products in
# the log-domain"): the matrix-matrix form that loopy graphs and the discrete
# marginalisation of several chains at once need (Sec. "Efficient averaging")
# ---------------------------------------------------------------------------

def logmmexp(X: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """Z[..., i, k] = log sum_j exp(X[..., i, j] + Y[..., j, k]), by definition: every
    sum X_ij + Y_jk is formed and reduced with the exact-max `logsumexp` (so no shift can
    underflow).  Leading axes are batch axes."""
    X = np.asarray(X, np.float64)
    Y = np.asarray(Y, np.float64)
    return logsumexp(X[..., :, :, None] + Y[..., None, :, :], axis=-2)


def logmmexp_shifted(X: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """The Appendix's form: shift each row of X by its max x_i and each column of Y by
    its max y_k, multiply the exponentials as ordinary matrices and add the shifts back,
        Z_ik = log sum_j exp(X_ij - x_i) exp(Y_jk - y_k) + x_i + y_k.
    Equal to `logmmexp` while no product underflows; used by the pins to show where the
    per-operand shift loses the result."""
    X = np.asarray(X, np.float64)
    Y = np.asarray(Y, np.float64)
    x = np.max(X, axis=-1, keepdims=True)
    y = np.max(Y, axis=-2, keepdims=True)
    xs = np.where(np.isfinite(x), x, 0.0)
    ys = np.where(np.isfinite(y), y, 0.0)
    with np.errstate(divide="ignore"):
        return np.log(np.exp(X - xs) @ np.exp(Y - ys)) + xs + ys


def finite_difference(fun, x: np.ndarray, h: float = 1e-5, idx=None) -> np.ndarray:
    """Central differences (fun(x + h e) - fun(x - h e)) / 2h at the flat indices
    `idx` (all entries when None)."""
    x = np.array(x, dtype=np.float64, copy=True)
    flat = x.reshape(-1)
    idx = range(flat.size) if idx is None else idx
    out = []
    for k in idx:
        old = flat[k]
        flat[k] = old + h
        fp = fun(x)
        flat[k] = old - h
        fm = fun(x)
        flat[k] = old
        out.append((fp - fm) / (2.0 * h))
    return np.array(out)


# ---------------------------------------------------------------------------
# special cases and closed forms used as pins
# ---------------------------------------------------------------------------

def iwae_logp(u0: np.ndarray) -> float:
    """The IWAE estimator of Sec. "Background" in log form: log (1/K) sum_k w_k with
    log w_k = u0[k]; equal to TMC with a single latent."""
    return float(logsumexp(np.asarray(u0, np.float64), axis=0) - log_k(len(u0)))


def linear_gauss_marginal_covs(W: Sequence[np.ndarray], sigma_z: float,
                               top_dim: int) -> List[np.ndarray]:
    """Prior marginal covariances of the linear-Gaussian chain
    z_{L-1} ~ N(0, I), z_l = W_l z_{l+1} + N(0, sigma_z^2 I)."""
    L = len(W) + 1
    cov = [None] * L
    cov[L - 1] = np.eye(top_dim)
    for l in range(L - 2, -1, -1):
        cov[l] = W[l] @ cov[l + 1] @ W[l].T + sigma_z ** 2 * np.eye(W[l].shape[0])
    return cov


def linear_gauss_log_evidence(W, Wx, x, sigma_z: float, sigma_x: float) -> float:
    """Closed-form log P(x) for the linear-Gaussian chain: x is Gaussian with mean 0
    and covariance Wx Sigma_0 Wx^T + sigma_x^2 I (all variables jointly Gaussian, as in
    the paper's toy experiments)."""
    from scipy.stats import multivariate_normal
    top = W[-1].shape[1] if len(W) else Wx.shape[1]
    S0 = linear_gauss_marginal_covs(W, sigma_z, top)[0]
    C = Wx @ S0 @ Wx.T + sigma_x ** 2 * np.eye(Wx.shape[0])
    return float(multivariate_normal(mean=np.zeros(len(x)), cov=C).logpdf(x))


def linear_gauss_joint_cov(W, Wx, sigma_z, sigma_x):
    """Joint covariance of (z_0, ..., z_{L-1}, x) for the linear-Gaussian chain; each
    variable is a linear map of independent standard normals."""
    L = len(W) + 1
    D = [W[l].shape[0] for l in range(L - 1)] + [W[-1].shape[1]]
    dx = Wx.shape[0]
    # noise blocks: eps_top (D_{L-1}), eps_l (D_l) for l < L-1, eps_x (dx)
    n_noise = sum(D) + dx
    A = [None] * L
    off = {}
    o = 0
    for l in range(L):
        off[l] = o
        o += D[l]
    A[L - 1] = np.zeros((D[L - 1], n_noise))
    A[L - 1][:, off[L - 1]:off[L - 1] + D[L - 1]] = np.eye(D[L - 1])
    for l in range(L - 2, -1, -1):
        A[l] = W[l] @ A[l + 1]
        A[l][:, off[l]:off[l] + D[l]] += sigma_z * np.eye(D[l])
    Ax = Wx @ A[0]
    Ax[:, o:o + dx] += sigma_x * np.eye(dx)
    M = np.vstack(A + [Ax])
    return M @ M.T, D


def linear_gauss_posterior_marginals(W, Wx, x, sigma_z, sigma_x):
    """Exact posterior P(z_l | x) of every layer (Gaussian conditioning on the joint);
    returns per-layer (mean, full covariance)."""
    C, D = linear_gauss_joint_cov(W, Wx, sigma_z, sigma_x)
    nz = sum(D)
    Czz, Czx, Cxx = C[:nz, :nz], C[:nz, nz:], C[nz:, nz:]
    K = np.linalg.solve(Cxx, Czx.T).T
    m = K @ x
    P = Czz - K @ Czx.T
    out, o = [], 0
    for d in D:
        out.append((m[o:o + d], P[o:o + d, o:o + d]))
        o += d
    return out


def hmm_log_evidence(prior_top: np.ndarray, trans: Sequence[np.ndarray],
                     emit_logp0: np.ndarray) -> float:
    """Exact log P(x) of a discrete chain by products of probability matrices (no
    logs inside): v_{L-1} = prior; v_l = T_l v_{l+1}; P(x) = sum_k P(x | state k of
    layer 0) v_0[k].  trans[l][i, j] = P(z_l = i | z_{l+1} = j)."""
    v = np.asarray(prior_top, np.float64)
    for T in reversed(list(trans)):
        v = T @ v
    return float(np.log(np.dot(np.exp(emit_logp0), v)))
