"""Seeded synthetic workloads for the TMC chain estimator (inputs only)."""
from .gen import CONFIGS, SEED_BASE, Chain, Workload, make, cast_chain, linear_gauss, tanh_bernoulli, ragged, pack

__all__ = ["CONFIGS", "SEED_BASE", "Chain", "Workload", "make", "cast_chain",
           "linear_gauss", "tanh_bernoulli", "ragged", "pack"]
