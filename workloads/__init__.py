"""Seeded synthetic workloads for the TMC estimators (inputs only)."""
from .gen import (CONFIGS, SEED_BASE, STAR_CONFIGS, Chain, StarWorkload, Workload, cast_chain,
                  gauss_star, linear_gauss, make, make_star, pack, ragged, tanh_bernoulli)

__all__ = ["CONFIGS", "SEED_BASE", "STAR_CONFIGS", "Chain", "StarWorkload", "Workload", "make",
           "make_star", "cast_chain", "gauss_star", "linear_gauss", "tanh_bernoulli", "ragged",
           "pack"]
