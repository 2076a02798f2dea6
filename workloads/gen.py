"""Seeded synthetic inputs for the TMC chain estimator.

This module only draws samples and evaluates the *caller-side* model pieces that
the estimator takes as inputs (proposal samples, the conditional means produced by
the generative network, per-sample unary log-terms).  It contains none of the
estimator's own arithmetic: no pairwise factor, no log-sum-exp message, no
normaliser.  Log-densities of the proposal, the prior of the top layer and the
likelihood are taken from scipy library routines.

Both the FP64 oracle tests and the GPU tests draw their inputs from here, so the
two sides see identical samples.  Every instance b has its own PCG64 stream keyed
by (seed, 1, b), so an instance does not depend on the batch size; shared model
parameters come from the stream keyed by (seed, 0) (or (seed, 0, c) for the
per-chain parameters of a ragged batch).

Layer indexing is 0-based: layer 0 is adjacent to the data x, layer L-1 is the
top of the chain (the paper's z_1 ... z_n).  For a chain of L layers the
estimator needs, per instance:
    z[l]   [K_l, D_l]        samples of layer l        (l = 0 .. L-1)
    mu[l]  [K_{l+1}, D_l]    mean of z_l given sample j of z_{l+1} (l = 0 .. L-2)
    s[l]   [D_l]             log standard deviation of P(z_l | z_{l+1}) (l = 0 .. L-2)
    u[l]   [K_l]             unary log-terms: -log Q(z_l^k), plus log P(x | z_0^k)
                             on layer 0 and log P(z_{L-1}^k) on the top layer.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np
from scipy import special, stats

SEED_BASE = 1806085930

# Workloads of the benchmark suite.  Sizes follow the five configurations the
# estimator is evaluated on; 'index' offsets the seed.
CONFIGS = {
    "c1": dict(index=0, kind="linear_gauss", B=16, L=4, K=8, D=8, x_dim=32,
               sigma_z=0.5, sigma_x=0.3),
    "c2": dict(index=1, kind="tanh_bernoulli", B=128, L=4, K=64, D=50, x_dim=784, p=0.13),
    "c3": dict(index=2, kind="tanh_bernoulli", B=256, L=6, K=256, D=100, x_dim=784, p=0.13),
    "c4": dict(index=3, kind="ragged", n_chains=512, L_range=(2, 12), D_set=(16, 32, 64),
               K_set=(32, 64, 128, 256, 512), x_dim=784, p=0.13),
    "c5": dict(index=4, kind="tanh_bernoulli", B=32, L=8, K=2048, D=128, x_dim=784, p=0.13),
}


@dataclass
class Chain:
    """One independent chain instance (lists indexed by layer, 0 = next to x)."""
    z: List[np.ndarray]
    mu: List[np.ndarray]
    s: List[np.ndarray]
    u: List[np.ndarray]

    @property
    def L(self) -> int:
        return len(self.z)

    @property
    def K(self) -> List[int]:
        return [int(a.shape[0]) for a in self.z]

    @property
    def D(self) -> List[int]:
        return [int(a.shape[1]) for a in self.z]

    def entries(self) -> int:
        k = self.K
        return int(sum(k[l] * k[l + 1] for l in range(self.L - 1)))


@dataclass
class Workload:
    name: str
    chains: List[Chain]
    # Homogeneous batches also expose stacked arrays (views share memory with chains):
    z: Optional[np.ndarray] = None    # [B, L, K, D]
    mu: Optional[np.ndarray] = None   # [B, L-1, K, D]
    s: Optional[np.ndarray] = None    # [L-1, D]   (shared by all instances)
    u: Optional[np.ndarray] = None    # [B, L, K]
    extra: dict = field(default_factory=dict)

    def entries(self) -> int:
        return int(sum(c.entries() for c in self.chains))


def _rng(*key: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence(list(key)))


def _normal_logpdf_rows(z: np.ndarray, mean, std) -> np.ndarray:
    return stats.norm.logpdf(z, loc=mean, scale=std).sum(axis=-1)


def _bernoulli_logit_loglik(x: np.ndarray, logits: np.ndarray) -> np.ndarray:
    # log Bernoulli(x; sigmoid(a)) = x*log sigmoid(a) + (1-x)*log sigmoid(-a)
    return (x * special.log_expit(logits) + (1.0 - x) * special.log_expit(-logits)).sum(-1)


def _tanh_chain_params(rng: np.random.Generator, L: int, D: int, x_dim: int, p: float):
    W = [rng.normal(0.0, 1.0 / np.sqrt(D), size=(D, D)) for _ in range(L - 1)]
    bias = [rng.normal(0.0, 0.1, size=D) for _ in range(L - 1)]
    s = [rng.uniform(-1.0, 0.0, size=D) for _ in range(L - 1)]
    W0 = rng.normal(0.0, 1.0 / np.sqrt(D), size=(x_dim, D))
    b0 = np.full(x_dim, special.logit(p))
    return W, bias, s, W0, b0


def _tanh_chain_instance(rng, L, K, D, x_dim, p, W, bias, s, W0, b0) -> Chain:
    x = (rng.random(x_dim) < p).astype(np.float64)
    qm = rng.normal(0.0, 1.0, size=(L, D))
    qls = rng.uniform(-1.0, 0.0, size=(L, D))
    z = [qm[l] + np.exp(qls[l]) * rng.normal(size=(K, D)) for l in range(L)]
    mu = [np.tanh(z[l + 1] @ W[l].T + bias[l]) for l in range(L - 1)]
    u = [-_normal_logpdf_rows(z[l], qm[l], np.exp(qls[l])) for l in range(L)]
    u[0] = u[0] + _bernoulli_logit_loglik(x, z[0] @ W0.T + b0)
    u[L - 1] = u[L - 1] + _normal_logpdf_rows(z[L - 1], 0.0, 1.0)
    return Chain(z=z, mu=mu, s=[a.copy() for a in s], u=u)


def linear_gauss(B=16, L=4, K=8, D=8, x_dim=32, sigma_z=0.5, sigma_x=0.3,
                 seed=SEED_BASE, instances: Optional[Sequence[int]] = None,
                 proposal=None) -> Workload:
    """Linear-Gaussian chain: z_{L-1} ~ N(0, I); z_l | z_{l+1} ~ N(W_l z_{l+1}, sigma_z^2 I);
    x | z_0 ~ N(W_x z_0, sigma_x^2 I).  W entries ~ N(0, 1/D).  x is an ancestral sample
    per instance.  Proposals are factorised Gaussians, means N(0,1), log-std U(-1,0),
    unless `proposal(b) -> (means [L,D], stds [L,D])` is supplied."""
    mrng = _rng(seed, 0)
    W = [mrng.normal(0.0, 1.0 / np.sqrt(D), size=(D, D)) for _ in range(L - 1)]
    Wx = mrng.normal(0.0, 1.0 / np.sqrt(D), size=(x_dim, D))
    s = [np.full(D, np.log(sigma_z)) for _ in range(L - 1)]
    ids = list(range(B)) if instances is None else list(instances)
    chains, xs = [], []
    for b in ids:
        rng = _rng(seed, 1, b)
        # ancestral sample of x
        zt = rng.normal(size=D)
        for l in range(L - 2, -1, -1):
            zt = W[l] @ zt + sigma_z * rng.normal(size=D)
        x = Wx @ zt + sigma_x * rng.normal(size=x_dim)
        if proposal is None:
            qm = rng.normal(0.0, 1.0, size=(L, D))
            qs = np.exp(rng.uniform(-1.0, 0.0, size=(L, D)))
        else:
            qm, qs = proposal(b, x)
        z = [qm[l] + qs[l] * rng.normal(size=(K, D)) for l in range(L)]
        mu = [z[l + 1] @ W[l].T for l in range(L - 1)]
        u = [-_normal_logpdf_rows(z[l], qm[l], qs[l]) for l in range(L)]
        u[0] = u[0] + stats.norm.logpdf(x[None, :], loc=z[0] @ Wx.T, scale=sigma_x).sum(-1)
        u[L - 1] = u[L - 1] + _normal_logpdf_rows(z[L - 1], 0.0, 1.0)
        chains.append(Chain(z=z, mu=mu, s=[a.copy() for a in s], u=u))
        xs.append(x)
    wl = _stack("linear_gauss", chains, s)
    wl.extra.update(W=W, Wx=Wx, x=np.array(xs), sigma_z=sigma_z, sigma_x=sigma_x)
    return wl


def tanh_bernoulli(B, L, K, D, x_dim=784, p=0.13, seed=SEED_BASE,
                   instances: Optional[Sequence[int]] = None, name="tanh_bernoulli") -> Workload:
    """Nonlinear chain: z_l | z_{l+1} ~ N(tanh(W_l z_{l+1} + b_l), diag exp(2 s_l)),
    Bernoulli(sigmoid(W_x z_0 + b_x)) likelihood over x_dim synthetic binary pixels
    with P(pixel=1) = p, top layer prior N(0, I)."""
    W, bias, s, W0, b0 = _tanh_chain_params(_rng(seed, 0), L, D, x_dim, p)
    ids = list(range(B)) if instances is None else list(instances)
    chains = [_tanh_chain_instance(_rng(seed, 1, b), L, K, D, x_dim, p, W, bias, s, W0, b0)
              for b in ids]
    return _stack(name, chains, s)


def ragged(n_chains=512, L_range=(2, 12), D_set=(16, 32, 64), K_set=(32, 64, 128, 256, 512),
           x_dim=784, p=0.13, seed=SEED_BASE, instances: Optional[Sequence[int]] = None,
           shapes_only=False):
    """Independent chains of uneven depth L, width D and sample count K (one L, D, K per
    chain, drawn uniformly); each chain has its own tanh-Gaussian model as `tanh_bernoulli`.
    With shapes_only=True returns the list of (L, K, D) without drawing samples."""
    ids = list(range(n_chains)) if instances is None else list(instances)
    shapes = []
    for c in ids:
        r = _rng(seed, 2, c)
        Lc = int(r.integers(L_range[0], L_range[1] + 1))
        Dc = int(r.choice(D_set))
        Kc = int(r.choice(K_set))
        shapes.append((Lc, Kc, Dc))
    if shapes_only:
        return shapes
    chains = []
    for c, (Lc, Kc, Dc) in zip(ids, shapes):
        W, bias, s, W0, b0 = _tanh_chain_params(_rng(seed, 0, c), Lc, Dc, x_dim, p)
        chains.append(_tanh_chain_instance(_rng(seed, 1, c), Lc, Kc, Dc, x_dim, p,
                                           W, bias, s, W0, b0))
    return Workload(name="ragged", chains=chains, extra=dict(shapes=shapes))


def _stack(name, chains: List[Chain], s) -> Workload:
    """Stack a homogeneous list of chains into [B, L, K, D] arrays and re-point the
    per-chain lists at views of them (so both forms share memory)."""
    B, L = len(chains), chains[0].L
    z = np.stack([np.stack(c.z) for c in chains])
    mu = np.stack([np.stack(c.mu) for c in chains]) if L > 1 else np.zeros((B, 0) + z.shape[2:])
    u = np.stack([np.stack(c.u) for c in chains])
    s_arr = np.stack(s) if L > 1 else np.zeros((0, z.shape[-1]))
    for b, c in enumerate(chains):
        c.z = [z[b, l] for l in range(L)]
        c.mu = [mu[b, l] for l in range(L - 1)]
        c.u = [u[b, l] for l in range(L)]
        c.s = [s_arr[l] for l in range(L - 1)]
    return Workload(name=name, chains=chains, z=z, mu=mu, s=s_arr, u=u)


def make(config: str, B: Optional[int] = None, instances: Optional[Sequence[int]] = None,
         **over):
    """Build a named workload ('c1'..'c5').  B (or an explicit instance list) selects a
    subset of instances; instance b is identical whatever B is."""
    cfg = dict(CONFIGS[config])
    cfg.update(over)
    seed = SEED_BASE + cfg.pop("index")
    kind = cfg.pop("kind")
    if kind == "linear_gauss":
        if B is not None:
            cfg["B"] = B
        return linear_gauss(seed=seed, instances=instances, **cfg)
    if kind == "tanh_bernoulli":
        if B is not None:
            cfg["B"] = B
        return tanh_bernoulli(seed=seed, instances=instances, name=config, **cfg)
    if kind == "ragged":
        if B is not None:
            cfg["n_chains"] = B
        return ragged(seed=seed, instances=instances, **cfg)
    raise ValueError(kind)


def cast_chain(c: Chain, dtype) -> Chain:
    """Round every input to `dtype` and return it as float64 again (the exact values a
    reduced-precision GPU run sees)."""
    f = lambda a: np.asarray(a, dtype=dtype).astype(np.float64)
    return Chain(z=[f(a) for a in c.z], mu=[f(a) for a in c.mu], s=[f(a) for a in c.s],
                 u=[f(a) for a in c.u])


def pack(chains: List[Chain], dtype=np.float32):
    """Flatten chains back to back (the layout of the library's ragged problem
    descriptor): returns (shapes, dict of flat z, mu, s, u arrays) where shapes is a
    list of (K_list, D_list) per chain."""
    shapes = [([int(a.shape[0]) for a in c.z], [int(a.shape[1]) for a in c.z]) for c in chains]
    cat = lambda arrs: (np.concatenate([a.reshape(-1) for a in arrs]) if arrs
                        else np.zeros(1)).astype(dtype)
    return shapes, dict(z=cat([a for c in chains for a in c.z]),
                        mu=cat([a for c in chains for a in c.mu]),
                        s=cat([a for c in chains for a in c.s]),
                        u=cat([a for c in chains for a in c.u]))


# ---------------------------------------------------------------------------
# star model: one global latent theta shared by N local latents
# ---------------------------------------------------------------------------

# The Gaussian example of Sec. "Comparing TMC, SMC and IWAE" toward the large ends of its
# two sweeps: N = 4096 data points with K = 128 samples (the sweep over N at K = 128), and
# N = 128 with K = 2048 (the sweep over K at N = 128); K_theta = K.
STAR_CONFIGS = {
    "s1": dict(index=10, S=1, N=4096, Kt=128, K=128, D=1, kind="toy"),
    "s2": dict(index=11, S=1, N=128, Kt=2048, K=2048, D=1, kind="toy"),
}


@dataclass
class StarWorkload:
    """S independent instances of the star model, as the estimator takes them:
        mth [S, Kt, D]  mean of every local latent given global sample kt
        s   [S, D]      log standard deviation of the local latents given theta
        z   [S, N, K, D] samples of the local latents
        u   [S, N, K]   log P(x_i | z_i^k) - log Q(z_i^k)
        uth [S, Kt]     log P(theta^kt) - log Q(theta^kt)
    plus the data x [S, N, D] and the global samples theta [S, Kt, D]."""
    name: str
    mth: np.ndarray
    s: np.ndarray
    z: np.ndarray
    u: np.ndarray
    uth: np.ndarray
    x: np.ndarray
    theta: np.ndarray

    @property
    def shape(self):
        S, N, K, D = self.z.shape
        return dict(S=S, N=N, Kt=self.mth.shape[1], K=K, D=D)

    def entries(self) -> int:
        sh = self.shape
        return int(sh["S"] * sh["N"] * sh["Kt"] * sh["K"])


def gauss_star(S=1, N=128, Kt=128, K=128, D=1, kind="toy", seed=SEED_BASE + 10,
               name="star") -> StarWorkload:
    """kind 'toy': the model of Sec. "Comparing TMC, SMC and IWAE" in each of D dimensions,
    theta ~ N(0, 1), z_i | theta ~ N(theta, 1), x_i | z_i ~ N(z_i, 1), with the generative
    marginals as proposals, Q(theta) = N(0, 1) and Q(z_i) = N(0, 2); so mth = theta, s = 0
    and uth = 0.  kind 'general': the mean of the local latents is a nonlinear function of
    theta, mth = tanh(A theta + b) (A entries N(0, 1/D), b ~ N(0, 0.1)), s ~ U(-1, 0) per
    dimension, and Q(theta) = N(0, 1.5^2) so uth is not constant.  Instance i draws
    from the stream keyed (seed, 1, i); shared parameters from (seed, 0)."""
    mrng = _rng(seed, 0)
    if kind == "general":
        A = mrng.normal(0.0, 1.0 / np.sqrt(D), size=(D, D))
        b = mrng.normal(0.0, 0.1, size=D)
        s = np.tile(mrng.uniform(-1.0, 0.0, size=D), (S, 1))
        qth = 1.5
    elif kind == "toy":
        s = np.zeros((S, D))
        qth = 1.0
    else:
        raise ValueError(kind)
    mth = np.empty((S, Kt, D))
    theta = np.empty((S, Kt, D))
    z = np.empty((S, N, K, D))
    u = np.empty((S, N, K))
    uth = np.empty((S, Kt))
    x = np.empty((S, N, D))
    for i in range(S):
        rng = _rng(seed, 1, i)
        th_true = rng.normal(size=D)
        if kind == "general":
            zt = np.tanh(A @ th_true + b) + np.exp(s[i]) * rng.normal(size=(N, D))
        else:
            zt = th_true + rng.normal(size=(N, D))
        x[i] = zt + rng.normal(size=(N, D))
        theta[i] = qth * rng.normal(size=(Kt, D))
        mth[i] = np.tanh(theta[i] @ A.T + b) if kind == "general" else theta[i]
        uth[i] = _normal_logpdf_rows(theta[i], 0.0, 1.0) - _normal_logpdf_rows(theta[i], 0.0, qth)
        z[i] = np.sqrt(2.0) * rng.normal(size=(N, K, D))
        u[i] = (_normal_logpdf_rows(x[i][:, None, :], z[i], 1.0)
                - _normal_logpdf_rows(z[i], 0.0, np.sqrt(2.0)))
    return StarWorkload(name=name, mth=mth, s=s, z=z, u=u, uth=uth, x=x, theta=theta)


def make_star(config: str, **over) -> StarWorkload:
    """A named star workload ('s1', 's2'); keyword arguments override its sizes."""
    cfg = dict(STAR_CONFIGS[config])
    cfg.update(over)
    seed = SEED_BASE + cfg.pop("index")
    return gauss_star(seed=seed, name=config, **cfg)
