"""GPU parity of the fused engine (factors recomputed on MFMA, never stored) against
the FP64 oracle on the same cast inputs, through the C ABI.

Tolerances on log P per instance: FP32 1e-4 absolute, BF16X3 2e-3 absolute.
Gradients against the oracle's closed-form gradients, per layer block: relative L2
(FP32 1e-4, BF16X3 1e-2) and element by element (GRAD_ELEM_TOL: every element within
a fraction of the block's largest reference value plus a relative term)."""
import numpy as np
import pytest

from oracle import tmc_oracle as O
from workloads import Chain, make

from .gpu_helpers import (GRAD_ELEM_TOL, assert_elem, cast_chains, oracle_grads, pack_chains, rel_l2,
                          run_gauss, to_dev, torch, unpack)

pytestmark = pytest.mark.gpu

LOGP_TOL = {"fp32": 1e-4, "bf16x3": 2e-3}
GRAD_TOL = {"fp32": 1e-4, "bf16x3": 1e-2}   # relative L2 per layer block (and GRAD_ELEM_TOL per element)


def _rand_chain(rng, Ks, Ds):
    L = len(Ks)
    z = [rng.normal(size=(Ks[l], Ds[l])) for l in range(L)]
    mu = [np.tanh(rng.normal(size=(Ks[l + 1], Ds[l]))) for l in range(L - 1)]
    s = [rng.uniform(-1.0, 0.0, size=Ds[l]) for l in range(L - 1)]
    u = [rng.normal(size=Ks[l]) * 5.0 for l in range(L)]
    return Chain(z=z, mu=mu, s=s, u=u)


def _check(out, chains, prec, grads=True):
    errs = []
    for b, c in enumerate(chains):
        ref = O.gauss_chain_logp(c.z, c.mu, c.s, c.u)
        errs.append(abs(out["logp"][b] - ref))
    assert max(errs) <= LOGP_TOL[prec], errs
    if not grads:
        return errs
    ref = oracle_grads(chains)
    tol = GRAD_TOL[prec]
    ea, er = GRAD_ELEM_TOL[prec]
    for name, key, idx in (("dz", "z", 1), ("dmu", "mu", 2), ("ds", "s", 3), ("du", "u", 4)):
        got = unpack(out[name], chains, key)
        for c, r in enumerate(ref):
            for l, rb in enumerate(r[idx]):
                if np.linalg.norm(rb) == 0:
                    assert np.abs(got[c][l]).max() == 0, (name, c, l)
                    continue
                e = rel_l2(got[c][l], rb)
                assert e < tol, (name, c, l, e)
                assert_elem(got[c][l], rb, ea, er, f"{prec}/{name}/chain{c}/layer{l}")
    return errs


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_fused_ragged_tails(prec):
    """K and D off every tile boundary (K 1..300, D 1..256), chains of 1-5 layers."""
    rng = np.random.default_rng(321)
    shapes = [((3,), (2,)), ((17, 3), (5, 1)), ((63, 65, 130), (33, 3, 65)),
              ((1, 1, 1), (4, 4, 4)), ((257, 17, 64, 5, 9), (100, 7, 2, 1, 3)),
              ((130, 257), (200, 16)), ((40, 300, 33), (256, 129, 64)), ((31, 32, 33), (16, 17, 15))]
    chains = cast_chains([_rand_chain(rng, Ks, Ds) for Ks, Ds in shapes], "fp32")
    out = run_gauss(chains, prec, engine="fused")
    assert out["info"]["engine"] == 1
    _check(out, chains, prec)


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_fused_c2_subset(prec):
    w = make("c2", B=8)
    chains = cast_chains(w.chains, "fp32")
    out = run_gauss(chains, prec, engine="fused")
    _check(out, chains, prec)


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_fused_c3_instances(prec):
    """Full C3 shape (L=6, K=256, D=100) on 3 instances."""
    w = make("c3", instances=[0, 101, 255])
    chains = cast_chains(w.chains, "fp32")
    out = run_gauss(chains, prec, engine="fused")
    errs = _check(out, chains, prec)
    print(prec, "c3 |dlogP|", errs)


def test_fused_deterministic_and_graph_replay():
    from paper_1806_08593_amd import tmc as T
    w = make("c2", B=6)
    chains = cast_chains(w.chains, "fp32")
    shapes, flat = pack_chains(chains, "fp32")
    prob, _ = T.ragged_problem(shapes, "bf16x3", "fused")
    plan = T.Plan(prob)
    ws = plan.new_workspace()
    d = {k: to_dev(v) for k, v in flat.items()}
    n = len(chains)
    dl = torch.ones(n, dtype=torch.float64, device="cuda:0")
    st = torch.cuda.Stream()
    res = []
    with torch.cuda.stream(st):
        for rep in range(2):
            lp = torch.empty(n, dtype=torch.float64, device="cuda:0")
            g = {k: torch.empty_like(v) for k, v in d.items()}
            T.tmc_gauss_fwd(plan.handle, d["z"], d["mu"], d["s"], d["u"], lp, ws, st)
            T.tmc_gauss_bwd(plan.handle, d["z"], d["mu"], d["s"], d["u"], dl, ws, g["z"], g["mu"],
                            g["s"], g["u"], st)
            st.synchronize()
            res.append((lp.clone(), {k: v.clone() for k, v in g.items()}))
        assert torch.equal(res[0][0], res[1][0])
        for k in res[0][1]:
            assert torch.equal(res[0][1][k], res[1][1][k]), k
        lpg = torch.empty(n, dtype=torch.float64, device="cuda:0")
        gg = {k: torch.empty_like(v) for k, v in d.items()}
        T.tmc_plan_graph_capture_gauss(plan.handle, 0, d["z"], d["mu"], d["s"], d["u"], lpg, None, ws,
                                       None, None, None, None, st)
        T.tmc_plan_graph_capture_gauss(plan.handle, 1, d["z"], d["mu"], d["s"], d["u"], None, dl, ws,
                                       gg["z"], gg["mu"], gg["s"], gg["u"], st)
        for rep in range(3):
            lpg.zero_()
            for v in gg.values():
                v.zero_()
            T.tmc_plan_graph_launch(plan.handle, 0, st)
            T.tmc_plan_graph_launch(plan.handle, 1, st)
            st.synchronize()
            assert torch.equal(lpg, res[0][0]), rep
            for k in gg:
                assert torch.equal(gg[k], res[0][1][k]), (rep, k)


def test_fused_minus_inf_and_forward_only():
    from paper_1806_08593_amd import tmc as T
    rng = np.random.default_rng(5)
    good = _rand_chain(rng, (40, 33, 20), (10, 10, 10))
    dead = _rand_chain(rng, (40, 33, 20), (10, 10, 10))
    dead.u[2][:] = -np.inf
    chains = cast_chains([good, dead], "fp32")
    out = run_gauss(chains, "fp32", engine="fused")
    ref = O.gauss_chain_logp(chains[0].z, chains[0].mu, chains[0].s, chains[0].u)
    assert abs(out["logp"][0] - ref) < 1e-4
    assert out["logp"][1] == -np.inf
    n0 = sum(a.size for a in chains[0].z)
    assert np.all(out["dz"][n0:] == 0.0)
    out2 = run_gauss(chains, "bf16x3", engine="fused", flags=T.TMC_FLAG_FORWARD_ONLY, bwd=False)
    assert abs(out2["logp"][0] - ref) < 2e-3
    with pytest.raises(T.TMCError) as ei:
        run_gauss(chains, "bf16x3", engine="fused", flags=T.TMC_FLAG_FORWARD_ONLY, bwd=True)
    assert ei.value.status == T.TMC_ERR_STATE


def test_fused_shared_s_autograd():
    """Homogeneous batch with s shared: autograd wrapper returns the batch-summed ds."""
    from paper_1806_08593_amd import autograd as A
    w = make("c2", B=4)
    B, L, K, D = w.z.shape
    run = A.GaussChainTMC(B, L, K, D, precision="fp32", engine="fused")
    t = {k: torch.tensor(getattr(w, k), dtype=torch.float32, device="cuda:0", requires_grad=True)
         for k in ("z", "mu", "s", "u")}
    logp = run(t["z"], t["mu"], t["s"], t["u"])
    logp.sum().backward()
    chains = cast_chains(w.chains, "fp32")
    ref = oracle_grads(chains)
    ds_ref = sum(np.stack(r[3]) for r in ref)
    assert rel_l2(t["s"].grad.cpu().numpy(), ds_ref) < 1e-4
    for b in range(B):
        assert abs(logp[b].item() - ref[b][0]) < 1e-4


def _shape_signature(shapes, prec, flags=0):
    """The launch-shape signature the library keys its tuning cache on: precision,
    flags, chain count and the multiset of (K_l, K_{l+1}, chunk bucket of D_l)."""
    buckets = [1, 2, 3, 4, 5, 6, 7, 8, 12, 16]
    hist = {}
    for Ks, Ds in shapes:
        for l in range(len(Ks) - 1):
            need = (Ds[l] + 15) // 16
            key = (Ks[l], Ks[l + 1], next(b for b in buckets if b >= need))
            hist[key] = hist.get(key, 0) + 1
    code = {"fp32": 1, "bf16x3": 2}[prec]
    return f"p{code}f{flags}c{len(shapes)}" + "".join(
        f"_{k[0]}x{k[1]}x{k[2]}:{v}" for k, v in sorted(hist.items()))


@pytest.mark.parametrize("prec", ["bf16x3", "fp32"])
def test_wide_workgroups_bitwise_equal_narrow(prec, tmp_path, monkeypatch):
    """8-wave workgroups (256 rows in the forward, 256 columns in the backward), forced in
    each direction through the tuning cache, on widths d = 97..128 with row counts on and
    off the 256 boundary: outputs bitwise equal to the 4-wave kernels (the same summation
    orders), and within tolerance of the oracle.  The one exception is ds with the
    8-wave backward: it also sums the row terms of its pairs (over all rows in one
    workgroup instead of per 64 rows), so ds matches to rounding.  The last two chains
    keep the row-term launch under 8-wave backwards: d = 99 (rows not 16-byte aligned)
    and 3 column workgroups for a single 64-row partial."""
    rng = np.random.default_rng(97)
    shapes = [((300, 256, 257), (100, 112, 128)), ((257, 300), (128, 97)),
              ((256, 64, 256), (104, 100, 120)), ((129, 520), (128, 100)),
              ((300, 256), (99, 64)), ((64, 600), (128, 64))]
    chains = cast_chains([_rand_chain(rng, Ks, Ds) for Ks, Ds in shapes], "fp32")
    sig = _shape_signature(shapes, prec)
    outs = {}
    for wf in (0, 1):
        for wb in (0, 1):
            cache = tmp_path / f"tune_{wf}{wb}.txt"
            cache.write_text(f"{sig} 0 1 2 {wf} {wb}\n")
            monkeypatch.setenv("TMC_TUNE_CACHE", str(cache))
            out = run_gauss(chains, prec, engine="fused")
            assert out["info"]["tuned"] == 1, "cache line not matched"
            assert out["info"]["waves_per_group"] == (8 if (wf or wb) else 4)
            outs[(wf, wb)] = out
    ref = outs[(0, 0)]
    for key, out in outs.items():
        assert np.array_equal(out["logp"], ref["logp"]), key
        for g in ("dz", "dmu", "ds", "du"):
            if g == "ds" and key[1] == 1:
                scale = float(np.abs(ref[g]).max())
                assert np.allclose(out[g], ref[g], rtol=1e-5, atol=1e-6 * scale), (key, g)
            else:
                assert np.array_equal(out[g], ref[g]), (key, g)
    _check(outs[(1, 1)], chains, prec)


def test_forward_only_launch_shapes_bitwise_equal(tmp_path, monkeypatch):
    """Forward without gradients (TMC_FLAG_FORWARD_ONLY) in BF16X3, every launch shape forced
    through the tuning cache -- 4 or 8 waves, one or two staged subtiles -- on widths
    d = 97..128 with row counts on and off the 256 boundary: log P bitwise equal between 4
    and 8 waves with one subtile per stage (one summation order), and every shape within
    the BF16X3 bound of the oracle (two subtiles per stage merge the online log-sum-exp in
    another order)."""
    from paper_1806_08593_amd import tmc as T
    rng = np.random.default_rng(131)
    shapes = [((300, 256, 257), (100, 112, 128)), ((257, 300), (128, 97)),
              ((256, 64, 256), (104, 100, 120)), ((129, 520), (128, 100)),
              ((64, 600), (128, 64))]
    chains = cast_chains([_rand_chain(rng, Ks, Ds) for Ks, Ds in shapes], "fp32")
    sig = _shape_signature(shapes, "bf16x3", flags=T.TMC_FLAG_FORWARD_ONLY)
    outs = {}
    for wf in (0, 1):
        for ns in (1, 2):
            cache = tmp_path / f"tune_fo_{wf}{ns}.txt"
            cache.write_text(f"{sig} 0 1 {ns} {wf} 0\n")
            monkeypatch.setenv("TMC_TUNE_CACHE", str(cache))
            out = run_gauss(chains, "bf16x3", engine="fused", flags=T.TMC_FLAG_FORWARD_ONLY, bwd=False)
            assert out["info"]["tuned"] == 1, "cache line not matched"
            outs[(wf, ns)] = out["logp"]
    assert np.array_equal(outs[(1, 1)], outs[(0, 1)])
    refs = [O.gauss_chain_logp(c.z, c.mu, c.s, c.u) for c in chains]
    for key, lps in outs.items():
        for lp, ref in zip(lps, refs):
            assert abs(lp - ref) < 2e-3, (key, lp, ref)


def test_ragged_autograd_wrapper():
    """torch.autograd over a ragged batch: the weighted sum of log P differentiates to the
    weighted oracle gradients of every chain (weights 1..n through dlogp)."""
    from paper_1806_08593_amd import autograd as A
    rng = np.random.default_rng(44)
    shapes = [((37, 64, 9), (16, 33, 5)), ((130, 70), (64, 7)), ((12,), (3,))]
    chains = cast_chains([_rand_chain(rng, Ks, Ds) for Ks, Ds in shapes], "fp32")
    shp, flat = pack_chains(chains, "fp32")
    run = A.RaggedGaussChainTMC(shp, precision="fp32", engine="fused")
    t = {k: torch.tensor(v, device="cuda:0", requires_grad=True) for k, v in flat.items()}
    logp = run(t["z"], t["mu"], t["s"], t["u"])
    wts = torch.arange(1, len(chains) + 1, dtype=torch.float64, device="cuda:0")
    (logp * wts).sum().backward()
    ref = oracle_grads(chains)
    ea, er = GRAD_ELEM_TOL["fp32"]
    for k, idx in (("z", 1), ("mu", 2), ("s", 3), ("u", 4)):
        got = unpack(t[k].grad.cpu().numpy().astype(np.float64), chains, k)
        for c, r in enumerate(ref):
            assert abs(logp[c].item() - r[0]) <= 1e-4
            for l, rb in enumerate(r[idx]):
                want = (c + 1) * np.asarray(rb)
                if np.abs(want).max() == 0:
                    assert np.abs(got[c][l]).max() == 0
                else:
                    assert_elem(got[c][l], want, ea, er, f"ragged-autograd/d{k}/chain{c}/layer{l}")
