"""The allocation-free forward (tmc_gauss_fwd_noalloc, workspace in the library's static
device array) against tmc_gauss_fwd with a caller workspace, through the C ABI: the same
kernels, so log P must be bitwise equal.  Two calls in a row, the second with a smaller
problem (the array keeps the first call's contents), then a plain-engine FP64 plan, and
the size limit."""
import numpy as np
import pytest

from workloads import make

from .gpu_helpers import cast_chains, pack_chains, to_dev, torch

pytestmark = pytest.mark.gpu


def _both(chains, prec, engine, flags):
    from paper_1806_08593_amd import tmc as T
    shapes, flat = pack_chains(chains, prec)
    prob, _ = T.ragged_problem(shapes, prec, engine, flags)
    plan = T.Plan(prob)
    assert plan.workspace_bytes <= T.TMC_NOALLOC_WORKSPACE_MAX
    d = {k: to_dev(v) for k, v in flat.items()}
    n = len(chains)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        ref = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda:0")
        got = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda:0")
        ws = plan.new_workspace()
        T.tmc_gauss_fwd(plan.handle, d["z"], d["mu"], d["s"], d["u"], ref, ws, st)
        T.tmc_gauss_fwd_noalloc(plan.handle, d["z"], d["mu"], d["s"], d["u"], got, st)
        st.synchronize()
    T.tmc_plan_check(plan.handle, st)
    out = ref.cpu().numpy(), got.cpu().numpy()
    plan.close()
    return out


def test_noalloc_forward_equals_workspace_forward():
    from paper_1806_08593_amd import tmc as T
    rng = np.random.default_rng(3)
    big = cast_chains(make("c2", B=16).chains, "fp32")
    small = cast_chains(make("c2", instances=[3, 9]).chains, "fp32")
    # ragged, smaller than the first problem: K and D off the tile boundaries
    for c in small:
        c.z = [a[:37, :45] for a in c.z]
        c.mu = [a[:37, :45] for a in c.mu]
        c.s = [a[:45] for a in c.s]
        c.u = [a[:37] for a in c.u]
    for chains, prec, engine, flags in ((big, "bf16x3", "fused", T.TMC_FLAG_FORWARD_ONLY),
                                        (small, "bf16x3", "fused", T.TMC_FLAG_FORWARD_ONLY),
                                        (small, "fp32", "fused", 0),
                                        (cast_chains(small, "fp64"), "fp64", "plain", 0)):
        ref, got = _both(chains, prec, engine, flags)
        assert np.all(np.isfinite(ref)), (prec, engine)
        assert np.array_equal(ref, got), (prec, engine, ref, got)


def test_noalloc_rejects_a_plan_larger_than_the_array():
    from paper_1806_08593_amd import tmc as T
    B, L, K, D = 256, 6, 256, 100         # gradient plan: the softmax means alone take 131 MB
    plan = T.Plan(T.homogeneous_problem(B, L, K, D, "bf16x3", "fused"))
    assert plan.workspace_bytes > T.TMC_NOALLOC_WORKSPACE_MAX
    with pytest.raises(T.TMCError) as ei:
        T.tmc_gauss_fwd_noalloc(plan.handle, 1, 1, 1, 1, 1)   # rejected before any launch
    assert ei.value.status == T.TMC_ERR_WORKSPACE
    plan.close()
