"""Writes the stored expected values under tests/golden/ from the FP64 oracle only.

    python tests/golden/make_golden.py

c1_logp.txt: per instance of the 16-instance linear-Gaussian workload (4 layers of
D=8, K=8), log P_TMC by enumeration of all 8^4 index tuples (eq. (is)) and by the
chain recursion; the closed-form log P(x) is listed beside them for context.
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import tmc_oracle as O  # noqa: E402
from workloads import make  # noqa: E402


def main():
    w = make("c1")
    lines = ["# instance  brute_force_logp  chain_logp  closed_form_log_evidence"]
    for b, c in enumerate(w.chains):
        f = O.gauss_chain_factors(c.z, c.mu, c.s)
        ev = O.linear_gauss_log_evidence(w.extra["W"], w.extra["Wx"], w.extra["x"][b],
                                         w.extra["sigma_z"], w.extra["sigma_x"])
        lines.append(f"{b} {O.brute_force_logp(f, c.u):.17g} {O.chain_logp(f, c.u):.17g} {ev:.17g}")
    with open(os.path.join(HERE, "c1_logp.txt"), "w") as fh:
        fh.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
