"""FP64 CPU oracle for the TMC chain estimator.

Test infrastructure only: tests, the smoke check and the benchmark's CPU-baseline
leg use it.  The library (paper_1806_08593_amd) never imports it.
"""
from . import tmc_oracle
from .tmc_oracle import *  # noqa: F401,F403
