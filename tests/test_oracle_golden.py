"""The oracle still reproduces its stored C1 values (written by
tests/golden/make_golden.py, which calls only the oracle)."""
import os

import numpy as np

from oracle import tmc_oracle as O
from workloads import make

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "c1_logp.txt")


def test_c1_golden_values():
    rows = np.loadtxt(GOLDEN)
    w = make("c1")
    assert rows.shape[0] == len(w.chains)
    for (b, bf, ch, ev), c in zip(rows, w.chains):
        f = O.gauss_chain_factors(c.z, c.mu, c.s)
        got = O.chain_logp(f, c.u)
        assert abs(got - bf) <= 1e-12 * abs(bf)
        assert abs(got - ch) <= 1e-13 * abs(ch)
        assert got <= ev + 50.0   # bound holds loosely for random proposals (Jensen in expectation)
