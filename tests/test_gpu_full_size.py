"""Parity at the full sizes of the benchmark workloads, in the launch configurations the
benchmark times (the library's tuner picks the launch shape, as in bench.py) and in
each forced workgroup width, against the FP64 oracle.  At these sizes the oracle uses
its matrix-product forms (`gauss_chain_grads_expanded`, pinned against the
direct-difference forms on the CPU), so every instance's log P, every gradient element
of sampled instances and the batch-summed ds of a shared s are checked."""
import concurrent.futures as cf
import os

import numpy as np
import pytest

from oracle import tmc_oracle as O
from workloads import cast_chain, make, pack

from .gpu_helpers import GRAD_ELEM_TOL, assert_elem, torch

pytestmark = pytest.mark.gpu

LOGP_TOL = {"fp32": 1e-4, "bf16x3": 2e-3}


def _oracle_all(chains):
    """Expanded-form oracle gradients of every chain (threads: numpy releases the GIL)."""
    n = max(1, min(8, len(os.sched_getaffinity(0))))
    with cf.ThreadPoolExecutor(n) as ex:
        return list(ex.map(lambda c: O.gauss_chain_grads_expanded(c.z, c.mu, c.s, c.u), chains))


def _force_widths(monkeypatch, tmp_path, sig, wf, wb):
    cache = tmp_path / f"tune_{wf}{wb}.txt"
    cache.write_text(f"{sig} 0 1 2 {wf} {wb}\n")
    monkeypatch.setenv("TMC_TUNE_CACHE", str(cache))


def _homog_signature(prec, B, L, K, D):
    buckets = [1, 2, 3, 4, 5, 6, 7, 8, 12, 16]
    nk = next(b for b in buckets if b >= (D + 15) // 16)
    code = {"fp32": 1, "bf16x3": 2}[prec]
    return f"p{code}f0c{B}_{K}x{K}x{nk}:{B * (L - 1)}"


def _run_homog(w, prec, tune):
    """Forward + backward of a stacked workload (s shared by the batch), with the
    library's launch-shape tuner first when `tune` (the benchmark's configuration)."""
    from paper_1806_08593_amd import tmc as T
    B, L, K, D = w.z.shape
    plan = T.Plan(T.homogeneous_problem(B, L, K, D, prec, "fused"))
    ws = plan.new_workspace()
    d = {k: torch.tensor(np.ascontiguousarray(getattr(w, k)), dtype=torch.float32, device="cuda:0")
         for k in ("z", "mu", "s", "u")}
    lp = torch.empty(B, dtype=torch.float64, device="cuda:0")
    dl = torch.ones(B, dtype=torch.float64, device="cuda:0")
    g = {k: torch.empty_like(v) for k, v in d.items()}
    if tune:
        T.tmc_plan_autotune(plan.handle, d["z"], d["mu"], d["s"], d["u"], dl, ws, g["z"], g["mu"],
                            g["s"], g["u"], reps=2)
    for k in g:
        g[k].fill_(float("nan"))
    T.tmc_gauss_fwd(plan.handle, d["z"], d["mu"], d["s"], d["u"], lp, ws)
    T.tmc_gauss_bwd(plan.handle, d["z"], d["mu"], d["s"], d["u"], dl, ws, g["z"], g["mu"], g["s"],
                    g["u"])
    T.tmc_plan_check(plan.handle)
    info = plan.info
    out = lp.cpu().numpy(), {k: v.cpu().numpy().astype(np.float64) for k, v in g.items()}, info
    plan.close()
    return out


def _check_homog(lp, g, refs, prec, label, grad_instances):
    """log P of every instance, every gradient element of the sampled instances, and the
    batch-summed ds against the sum of the oracle's per-instance ds."""
    errs = np.array([abs(lp[b] - refs[b][0]) for b in range(len(refs))])
    print(f"ERRREC {label}/logp {errs.max():.3e}")
    assert errs.max() <= LOGP_TOL[prec], (label, int(errs.argmax()), errs.max())
    ea, er = GRAD_ELEM_TOL[prec]
    for b in grad_instances:
        _, dz, dmu, ds, du = refs[b]
        for l in range(len(dmu)):
            assert_elem(g["z"][b, l], dz[l], ea, er, f"{label}/dz/b{b}/l{l}")
            assert_elem(g["mu"][b, l], dmu[l], ea, er, f"{label}/dmu/b{b}/l{l}")
        assert np.all(g["z"][b, -1] == 0.0)
        for l in range(len(du)):
            assert_elem(g["u"][b, l], du[l], ea, er, f"{label}/du/b{b}/l{l}")
    ds_ref = sum(np.stack(r[3]) for r in refs)
    for l in range(ds_ref.shape[0]):
        assert_elem(g["s"][l], ds_ref[l], ea, er, f"{label}/ds-batch-sum/l{l}")


@pytest.mark.timeout(300)
@pytest.mark.parametrize("prec", ["bf16x3", "fp32"])
def test_c3_full_batch_tuned(prec):
    """B=256, L=6, K=256, D=100 with s shared by the batch, tuned launch shape (the
    benchmark's step in BF16X3 and its FP32 fused comparator): all 256 log P, every
    gradient element of four instances, the batch-summed ds."""
    w = make("c3")
    lp, g, info = _run_homog(w, prec, tune=True)
    print("launch", {k: info[k] for k in ("wide_fwd", "wide_bwd", "persistent")})
    refs = _oracle_all([cast_chain(c, np.float32) for c in w.chains])
    _check_homog(lp, g, refs, prec, f"c3-{prec}-tuned", (0, 77, 160, 255))
    assert np.allclose(g["u"].sum(axis=2), 1.0, atol=1e-3)


@pytest.mark.timeout(300)
@pytest.mark.parametrize("prec", ["bf16x3", "fp32"])
def test_c3_shared_s_each_width(prec, tmp_path, monkeypatch):
    """Sixteen C3 instances, s shared, with the workgroup width forced in both directions
    (4 waves: backward + row-term launch; 8 waves: the backward writes dz and the ds row
    part of these aligned pairs itself): each against the oracle element by element,
    ds against the batch sum, and the two widths against each other."""
    w = make("c3", B=16)
    B, L, K, D = w.z.shape
    refs = _oracle_all([cast_chain(c, np.float32) for c in w.chains])
    sig = _homog_signature(prec, B, L, K, D)
    res = {}
    for wf, wb in ((0, 0), (1, 1)):
        _force_widths(monkeypatch, tmp_path, sig, wf, wb)
        lp, g, info = _run_homog(w, prec, tune=False)
        assert info["tuned"] == 1 and info["wide_bwd"] == wb and info["wide_fwd"] == wf
        _check_homog(lp, g, refs, prec, f"c3x16-{prec}-w{wf}{wb}", range(B))
        res[(wf, wb)] = (lp, g)
    (lp0, g0), (lp1, g1) = res[(0, 0)], res[(1, 1)]
    assert np.array_equal(lp0, lp1)
    for k in ("z", "mu", "u"):
        assert np.array_equal(g0[k], g1[k]), k
    # ds: the 8-wave backward sums its row terms over all rows of a workgroup
    assert np.allclose(g1["s"], g0["s"], rtol=1e-5, atol=1e-6 * np.abs(g0["s"]).max())


@pytest.mark.timeout(400)
def test_c5_large_k_bf16x3_tuned():
    """B=32, L=8, K=2048, D=128, BF16X3 with the tuned launch shape (the benchmark's
    headline step): every instance's log P, every gradient element of instances 0 and
    31, and the batch-summed ds, against the oracle."""
    w = make("c5")
    lp, g, info = _run_homog(w, "bf16x3", tune=True)
    print("launch", {k: info[k] for k in ("wide_fwd", "wide_bwd", "persistent")})
    refs = _oracle_all([cast_chain(c, np.float32) for c in w.chains])
    _check_homog(lp, g, refs, "bf16x3", "c5-bf16x3-tuned", (0, 31))
    assert np.allclose(g["u"].sum(axis=2), 1.0, atol=2e-3)


@pytest.mark.timeout(300)
@pytest.mark.parametrize("persistent", [False, True])
def test_c4_full_ragged_fp32(persistent):
    """All 512 ragged chains in FP32 (the configuration's precision), per-depth launches
    with the tuned shape or persistent launches: every chain's log P within 1e-4, every
    gradient element of sixteen chains of all shapes, marginal sums of every layer."""
    from paper_1806_08593_amd import tmc as T
    w = make("c4")
    chains = [cast_chain(c, np.float32) for c in w.chains]
    shapes, flat = pack(chains, np.float32)
    flags = T.TMC_FLAG_PERSISTENT if persistent else 0
    prob, _ = T.ragged_problem(shapes, "fp32", "fused", flags)
    plan = T.Plan(prob)
    ws = plan.new_workspace()
    d = {k: torch.tensor(v, device="cuda:0") for k, v in flat.items()}
    n = len(chains)
    lp = torch.empty(n, dtype=torch.float64, device="cuda:0")
    dl = torch.ones(n, dtype=torch.float64, device="cuda:0")
    g = {k: torch.full_like(v, float("nan")) for k, v in d.items()}
    if not persistent:
        T.tmc_plan_autotune(plan.handle, d["z"], d["mu"], d["s"], d["u"], dl, ws, g["z"], g["mu"],
                            g["s"], g["u"], reps=2)
        for v in g.values():
            v.fill_(float("nan"))
    assert plan.info["persistent"] == (1 if persistent else 0)
    T.tmc_gauss_fwd(plan.handle, d["z"], d["mu"], d["s"], d["u"], lp, ws)
    T.tmc_gauss_bwd(plan.handle, d["z"], d["mu"], d["s"], d["u"], dl, ws, g["z"], g["mu"], g["s"],
                    g["u"])
    T.tmc_plan_check(plan.handle)
    lp = lp.cpu().numpy()
    g = {k: v.cpu().numpy().astype(np.float64) for k, v in g.items()}
    plan.close()
    refs = _oracle_all(chains)
    errs = np.array([abs(lp[b] - refs[b][0]) for b in range(n)])
    label = f"c4-fp32-{'persistent' if persistent else 'tuned'}"
    print(f"ERRREC {label}/logp {errs.max():.3e}")
    assert errs.max() <= 1e-4, (int(errs.argmax()), errs.max())
    # sixteen chains spread over the shapes: every (K, D) combination present, short and long
    order = sorted(range(n), key=lambda b: (chains[b].K[0], chains[b].D[0], chains[b].L))
    sample = sorted(set(order[:: max(1, n // 16)][:16]))
    ea, er = GRAD_ELEM_TOL["fp32"]
    offs = {k: 0 for k in ("z", "mu", "s", "u")}
    for b, c in enumerate(chains):
        for k, arrs, idx in (("z", c.z, 1), ("mu", c.mu, 2), ("s", c.s, 3), ("u", c.u, 4)):
            for l, a in enumerate(arrs):
                got = g[k][offs[k]:offs[k] + a.size].reshape(a.shape)
                offs[k] += a.size
                if k == "u":
                    assert abs(got.sum() - 1.0) < 1e-3, (b, l)
                if b in sample:
                    ref = refs[b][idx][l]
                    if np.abs(ref).max() == 0:
                        assert np.abs(got).max() == 0, (k, b, l)
                    else:
                        assert_elem(got, ref, ea, er, f"{label}/d{k}/c{b}/l{l}")
