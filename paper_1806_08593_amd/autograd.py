"""torch.autograd wrappers of the Gaussian-chain TMC estimator, of the DReGs surrogate and of
the star model.

Only marshalling: the forward and backward passes are the library's tmc_gauss_fwd /
tmc_gauss_bwd (tmc_star_gauss_fwd / _bwd) kernels.  torch provides device memory, the stream, and carries the
returned gradients on into the caller's networks (mu and u are functions of the
caller's parameters and of the reparameterised samples z).
"""
from __future__ import annotations

import numpy as np
import torch

from . import tmc as T

_DT = {T.TMC_FP64: torch.float64, T.TMC_FP32: torch.float32, T.TMC_BF16X3: torch.float32}


class GaussChainTMC:
    """Batch of B chains with L layers of K samples and width D:
        z [B, L, K, D], mu [B, L-1, K, D], s [L-1, D] (shared by the batch), u [B, L, K]
    -> log P_TMC [B] (float64), differentiable in z, mu, s and u.
    precision: 'fp64' | 'fp32' | 'bf16x3'; engine: 'auto' | 'fused' | 'plain'."""

    def __init__(self, B, L, K, D, precision="fp32", engine="auto", device=0, flags=0):
        self.shape = (B, L, K, D)
        self.problem = T.homogeneous_problem(B, L, K, D, precision, engine, flags)
        self.plan = T.Plan(self.problem, device)
        self.dtype = _DT[self.problem.c.precision]
        self.device = torch.device(f"cuda:{device}")

    def _check(self, z, mu, s, u):
        B, L, K, D = self.shape
        want = {"z": (z, (B, L, K, D)), "mu": (mu, (B, L - 1, K, D)), "s": (s, (L - 1, D)),
                "u": (u, (B, L, K))}
        for name, (t, shp) in want.items():
            if tuple(t.shape) != shp:
                raise ValueError(f"{name}: shape {tuple(t.shape)}, expected {shp}")
            if t.dtype != self.dtype or t.device != self.device or not t.is_contiguous():
                raise ValueError(f"{name}: needs a contiguous {self.dtype} tensor on {self.device}")

    def __call__(self, z, mu, s, u):
        self._check(z, mu, s, u)
        return _GaussChainFn.apply(z, mu, s, u, self)


class RaggedGaussChainTMC:
    """Chains of uneven depth, sample counts and widths, given as a list of
    (K_list, D_list) per chain, with z, mu, s, u packed back to back in flat tensors (the
    layout of tmc.ragged_problem: each chain's layers in order, each layer's block
    row-major) -> log P_TMC [n_chains] (float64), differentiable in the four flat
    tensors.  Every chain has its own s blocks."""

    def __init__(self, shapes, precision="fp32", engine="auto", device=0, flags=0):
        self.problem, self.sizes = T.ragged_problem(shapes, precision, engine, flags)
        self.plan = T.Plan(self.problem, device)
        self.shape = (len(shapes),)
        self.dtype = _DT[self.problem.c.precision]
        self.device = torch.device(f"cuda:{device}")

    def __call__(self, z, mu, s, u):
        for name, t in (("z", z), ("mu", mu), ("s", s), ("u", u)):
            if t.dim() != 1 or t.numel() < max(self.sizes[name], 1):
                raise ValueError(f"{name}: needs a flat tensor of {self.sizes[name]} elements")
            if t.dtype != self.dtype or t.device != self.device or not t.is_contiguous():
                raise ValueError(f"{name}: needs a contiguous {self.dtype} tensor on {self.device}")
        return _GaussChainFn.apply(z, mu, s, u, self)


class GaussChainDReGs:
    """The DReGs surrogate of the Appendix "Combining DReGs and TMC" for a homogeneous batch:
        S = 1/2 stopgrad(sum_t w_t^2 / (sum_t w_t)^2) log sum_t w_t^2     (per chain)
    over the importance weights w_t of every index tuple t, whose gradient is the DReGs
    estimator (the caller stops the direct dependence of u on the proposal parameters).
    A forward with kappa = 1 gives log P_1 and a forward with kappa = 2 (the squared
    weights) log P_2 = log sum_t w_t^2 - sum_l ln K_l; the coefficient is
    c = exp(log P_2 - 2 log P_1 - sum_l ln K_l), S = c (log P_2 + sum_l ln K_l) / 2, and the
    backward is the kappa = 2 backward with upstream gradient c g / 2.  Same shapes as
    GaussChainTMC; returns S [B] (float64)."""

    def __init__(self, B, L, K, D, precision="fp32", engine="auto", device=0):
        self.shape = (B, L, K, D)
        self.plan1 = T.Plan(T.homogeneous_problem(B, L, K, D, precision, engine,
                                                  T.TMC_FLAG_FORWARD_ONLY, exponent=1.0), device)
        self.plan2 = T.Plan(T.homogeneous_problem(B, L, K, D, precision, engine, 0, exponent=2.0),
                            device)
        self.dtype = _DT[self.plan2.problem.c.precision]
        self.device = torch.device(f"cuda:{device}")
        self.sum_log_k = L * float(np.log(K))

    def __call__(self, z, mu, s, u):
        GaussChainTMC._check(self, z, mu, s, u)
        return _DReGsFn.apply(z, mu, s, u, self)


class _DReGsFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, z, mu, s, u, runner: GaussChainDReGs):
        B = runner.shape[0]
        lp1 = torch.empty(B, dtype=torch.float64, device=z.device)
        lp2 = torch.empty(B, dtype=torch.float64, device=z.device)
        ws1 = runner.plan1.new_workspace()
        T.tmc_gauss_fwd(runner.plan1.handle, z, mu, s, u, lp1, ws1)
        ws2 = runner.plan2.new_workspace()
        T.tmc_gauss_fwd(runner.plan2.handle, z, mu, s, u, lp2, ws2)
        c = torch.exp(lp2 - 2.0 * lp1 - runner.sum_log_k)
        ctx.save_for_backward(z, mu, s, u, c)
        ctx.ws2 = ws2
        ctx.runner = runner
        return 0.5 * c * (lp2 + runner.sum_log_k)

    @staticmethod
    def backward(ctx, g):
        z, mu, s, u, c = ctx.saved_tensors
        dlogp = (0.5 * c * g.to(torch.float64)).contiguous()
        need = ctx.needs_input_grad
        dz = torch.empty_like(z) if need[0] else None
        dmu = torch.empty_like(mu) if need[1] else None
        ds = torch.empty_like(s) if need[2] else None
        du = torch.empty_like(u) if need[3] else None
        T.tmc_gauss_bwd(ctx.runner.plan2.handle, z, mu, s, u, dlogp, ctx.ws2, dz, dmu, ds, du)
        return dz, dmu, ds, du, None


class _GaussChainFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, z, mu, s, u, runner: GaussChainTMC):
        ws = runner.plan.new_workspace()
        logp = torch.empty(runner.shape[0], dtype=torch.float64, device=z.device)
        T.tmc_gauss_fwd(runner.plan.handle, z, mu, s, u, logp, ws)
        ctx.save_for_backward(z, mu, s, u)
        ctx.ws = ws
        ctx.runner = runner
        return logp

    @staticmethod
    def backward(ctx, dlogp):
        z, mu, s, u = ctx.saved_tensors
        dlogp = dlogp.to(torch.float64).contiguous()
        need = ctx.needs_input_grad
        dz = torch.empty_like(z) if need[0] else None
        dmu = torch.empty_like(mu) if need[1] else None
        ds = torch.empty_like(s) if need[2] else None
        du = torch.empty_like(u) if need[3] else None
        T.tmc_gauss_bwd(ctx.runner.plan.handle, z, mu, s, u, dlogp, ctx.ws, dz, dmu, ds, du)
        return dz, dmu, ds, du, None


class StarGaussTMC:
    """S instances of the star model -- one global latent with K_theta samples shared by N
    local latents with K samples of width D each:
        mth [S, Kt, D] (mean of every local latent given global sample kt), s [S, D],
        z [S, N, K, D], u [S, N, K], uth [S, Kt]
    -> log P_TMC [S] (float64), differentiable in all five.
    precision: 'fp64' | 'fp32'."""

    def __init__(self, S, N, Kt, K, D, precision="fp32", device=0):
        self.problem = T.StarProblem(S, N, Kt, K, D, precision)
        self.plan = T.Plan(self.problem, device)
        self.shape = (S, N, Kt, K, D)
        self.dtype = _DT[self.problem.c.precision]
        self.device = torch.device(f"cuda:{device}")

    def __call__(self, mth, s, z, u, uth):
        S, N, Kt, K, D = self.shape
        want = {"mth": (mth, (S, Kt, D)), "s": (s, (S, D)), "z": (z, (S, N, K, D)),
                "u": (u, (S, N, K)), "uth": (uth, (S, Kt))}
        for name, (t, shp) in want.items():
            if tuple(t.shape) != shp:
                raise ValueError(f"{name}: shape {tuple(t.shape)}, expected {shp}")
            if t.dtype != self.dtype or t.device != self.device or not t.is_contiguous():
                raise ValueError(f"{name}: needs a contiguous {self.dtype} tensor on {self.device}")
        return _StarFn.apply(mth, s, z, u, uth, self)


class _StarFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, mth, s, z, u, uth, runner: StarGaussTMC):
        ws = runner.plan.new_workspace()
        logp = torch.empty(runner.shape[0], dtype=torch.float64, device=z.device)
        T.tmc_star_gauss_fwd(runner.plan.handle, mth, s, z, u, uth, logp, ws)
        ctx.save_for_backward(mth, s, z, u)
        ctx.ws = ws
        ctx.runner = runner
        ctx.uth_like = uth
        return logp

    @staticmethod
    def backward(ctx, dlogp):
        mth, s, z, u = ctx.saved_tensors
        dlogp = dlogp.to(torch.float64).contiguous()
        need = ctx.needs_input_grad
        dmth = torch.empty_like(mth) if need[0] else None
        ds = torch.empty_like(s) if need[1] else None
        dz = torch.empty_like(z) if need[2] else None
        du = torch.empty_like(u) if need[3] else None
        duth = torch.empty_like(ctx.uth_like) if need[4] else None
        T.tmc_star_gauss_bwd(ctx.runner.plan.handle, mth, s, z, u, dlogp, ctx.ws, dmth, ds, dz,
                             du, duth)
        return dmth, ds, dz, du, duth, None
