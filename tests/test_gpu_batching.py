"""Ragged batching through the C ABI: persistent launches over a queue of whole chains
(most expensive first), their graph capture and the launch-shape tuner.  The persistent launch runs the same per-item arithmetic as the per-depth
launches, so its outputs must be bit-identical to them; both are also checked against
the FP64 oracle on the same FP32-cast inputs."""
import os

import numpy as np
import pytest

from oracle import tmc_oracle as O
from workloads import make

from .gpu_helpers import cast_chains, oracle_grads, pack_chains, rel_l2, to_dev, torch, unpack

pytestmark = pytest.mark.gpu

LOGP_TOL = {"fp32": 1e-4, "bf16x3": 2e-3}


def _setup(chains, prec, flags):
    from paper_1806_08593_amd import tmc as T
    shapes, flat = pack_chains(chains, "fp32")
    prob, _ = T.ragged_problem(shapes, prec, "fused", flags)
    plan = T.Plan(prob)
    ws = plan.new_workspace()
    d = {k: to_dev(v) for k, v in flat.items()}
    return plan, ws, d


def _run(plan, ws, d, n, bwd=True, stream=None):
    from paper_1806_08593_amd import tmc as T
    lp = torch.empty(n, dtype=torch.float64, device="cuda:0")
    dl = torch.ones(n, dtype=torch.float64, device="cuda:0")
    g = {k: torch.empty_like(v) for k, v in d.items()}
    T.tmc_gauss_fwd(plan.handle, d["z"], d["mu"], d["s"], d["u"], lp, ws, stream)
    if bwd:
        T.tmc_gauss_bwd(plan.handle, d["z"], d["mu"], d["s"], d["u"], dl, ws, g["z"], g["mu"],
                        g["s"], g["u"], stream)
    torch.cuda.synchronize()
    return lp, g


def _c4_subset(n=40):
    # the first n chains of the ragged workload (uneven depth 2..12, K 32..512, D 16..64)
    return cast_chains(make("c4", instances=list(range(n))).chains, "fp32")


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_persistent_equals_per_depth_and_oracle(prec):
    """The C4 subset mixes d = 16, 32, 64 at every depth: the per-depth plan runs those
    buckets of a step in one mixed launch, the persistent plan in one kernel per bucket;
    log P and every gradient bitwise equal, and within tolerance of the oracle."""
    from paper_1806_08593_amd import tmc as T
    chains = _c4_subset()
    n = len(chains)
    plan_l, ws_l, d = _setup(chains, prec, 0)
    plan_p, ws_p, _ = _setup(chains, prec, T.TMC_FLAG_PERSISTENT)
    assert plan_l.info["persistent"] == 0 and plan_p.info["persistent"] == 1
    lp_l, g_l = _run(plan_l, ws_l, d, n)
    lp_p, g_p = _run(plan_p, ws_p, d, n)
    T.tmc_plan_check(plan_p.handle)
    assert torch.equal(lp_l, lp_p)
    for k in g_l:
        assert torch.equal(g_l[k], g_p[k]), k
    lp = lp_p.cpu().numpy()
    errs = [abs(lp[b] - O.gauss_chain_logp(c.z, c.mu, c.s, c.u)) for b, c in enumerate(chains)]
    assert max(errs) <= LOGP_TOL[prec], max(errs)
    ref = oracle_grads(chains[:8])
    gz = unpack(g_p["z"].cpu().numpy(), chains, "z")
    gmu = unpack(g_p["mu"].cpu().numpy(), chains, "mu")
    for c, r in enumerate(ref):
        for l in range(len(r[2])):
            assert rel_l2(gz[c][l], r[1][l]) < 1e-2
            assert rel_l2(gmu[c][l], r[2][l]) < 1e-2


def _c3_like(n):
    # n chains of the homogeneous benchmark shape (L = 6 layers of K = 256, D = 100)
    return cast_chains(make("c3", B=n).chains, "fp32")


@pytest.mark.parametrize("case", ["persistent_fp32_c4", "per_depth_bf16x3_c3"])
def test_graph_replay(case):
    """Replays of the captured forward and backward graphs equal the eager launches
    bitwise, three times over, with eager work and synchronisation between replays."""
    from paper_1806_08593_amd import tmc as T
    if case == "persistent_fp32_c4":
        chains, prec, flags = _c4_subset(24), "fp32", T.TMC_FLAG_PERSISTENT
    else:
        chains, prec, flags = _c3_like(64), "bf16x3", 0
    n = len(chains)
    plan, ws, d = _setup(chains, prec, flags)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        lp0, g0 = _run(plan, ws, d, n, stream=st)
        lp = torch.empty(n, dtype=torch.float64, device="cuda:0")
        dl = torch.ones(n, dtype=torch.float64, device="cuda:0")
        g = {k: torch.empty_like(v) for k, v in d.items()}
        T.tmc_plan_graph_capture_gauss(plan.handle, 0, d["z"], d["mu"], d["s"], d["u"], lp, None,
                                       ws, None, None, None, None, st)
        T.tmc_plan_graph_capture_gauss(plan.handle, 1, d["z"], d["mu"], d["s"], d["u"], None, dl,
                                       ws, g["z"], g["mu"], g["s"], g["u"], st)
        for rep in range(3):
            lp.zero_()
            for v in g.values():
                v.zero_()
            st.synchronize()
            T.tmc_plan_graph_launch(plan.handle, 0, st)
            T.tmc_plan_graph_launch(plan.handle, 1, st)
            st.synchronize()
            assert torch.equal(lp, lp0), rep
            for k in g:
                assert torch.equal(g[k], g0[k]), (rep, k)
    T.tmc_plan_check(plan.handle)


def test_persistent_longest_chains_first_one_workgroup_per_chain():
    """Chains of very different cost in one persistent launch, with fewer workgroups
    than chains when the queue is longer than the resident capacity: results equal the
    per-depth launches and the oracle."""
    from paper_1806_08593_amd import tmc as T
    rng = np.random.default_rng(77)
    from workloads import Chain
    chains = []
    for c in range(20):
        L = int(rng.integers(2, 9))
        K = int(rng.choice([1, 5, 33, 128, 129, 300]))
        D = int(rng.choice([3, 16, 40]))
        z = [rng.normal(size=(K, D)) for _ in range(L)]
        mu = [np.tanh(rng.normal(size=(K, D))) for _ in range(L - 1)]
        s = [rng.uniform(-1.0, 0.0, size=D) for _ in range(L - 1)]
        u = [rng.normal(size=K) * 3.0 for _ in range(L)]
        chains.append(Chain(z=z, mu=mu, s=s, u=u))
    chains = cast_chains(chains, "fp32")
    n = len(chains)
    plan_l, ws_l, d = _setup(chains, "fp32", 0)
    plan_p, ws_p, _ = _setup(chains, "fp32", T.TMC_FLAG_PERSISTENT)
    lp_l, g_l = _run(plan_l, ws_l, d, n)
    lp_p, g_p = _run(plan_p, ws_p, d, n)
    assert torch.equal(lp_l, lp_p)
    for k in g_l:
        assert torch.equal(g_l[k], g_p[k]), k
    lp = lp_p.cpu().numpy()
    for b, c in enumerate(chains):
        assert abs(lp[b] - O.gauss_chain_logp(c.z, c.mu, c.s, c.u)) <= 1e-4, b


def test_autotune_picks_a_shape_and_caches_it(tmp_path, monkeypatch):
    from paper_1806_08593_amd import tmc as T
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("TMC_TUNE_CACHE", str(cache))
    chains = _c4_subset(32)
    n = len(chains)
    plan, ws, d = _setup(chains, "fp32", 0)
    assert plan.info["tuned"] == 0
    lp = torch.empty(n, dtype=torch.float64, device="cuda:0")
    dl = torch.ones(n, dtype=torch.float64, device="cuda:0")
    g = {k: torch.empty_like(v) for k, v in d.items()}
    T.tmc_plan_autotune(plan.handle, d["z"], d["mu"], d["s"], d["u"], dl, ws, g["z"], g["mu"],
                        g["s"], g["u"], reps=2)
    info = T.tmc_plan_info_get(plan.handle)
    assert info["tuned"] == 1
    line = cache.read_text().strip().splitlines()[-1].split()
    assert len(line) == 6 and int(line[1]) == info["persistent"]
    # results after tuning are those of the chosen shape, and correct
    lp2, _ = _run(plan, ws, d, n)
    c = chains[5]
    assert abs(lp2.cpu().numpy()[5] - O.gauss_chain_logp(c.z, c.mu, c.s, c.u)) < 1e-4
    # a new plan with the same shapes starts from the cached choice
    plan2, _, _ = _setup(chains, "fp32", 0)
    assert plan2.info["tuned"] == 1 and plan2.info["persistent"] == info["persistent"]
