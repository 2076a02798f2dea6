"""Parent-dependent scales (TMC_FLAG_PARENT_SCALE: the conditional's standard deviation,
like its mean, produced from each parent sample) on the GPU against the FP64 oracle,
element-wise: log P and dz, dmu, ds (one row per parent sample) and du, plus the
materialised factors, on ragged chains with tile tails in K and D; and the reduction to
the shared-scale plan when every parent produces the same scale."""
import numpy as np
import pytest

from oracle import tmc_oracle as O
from tests.gpu_helpers import GRAD_ELEM_TOL, assert_elem, np_dtype, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

LOGP_TOL = {"fp64": 1e-9, "fp32": 1e-4}


def _chains(seed, shapes):
    rng = np.random.default_rng(seed)
    out = []
    for Ks, Ds in shapes:
        L = len(Ks)
        z = [rng.normal(size=(Ks[l], Ds[l])) for l in range(L)]
        mu = [np.tanh(rng.normal(size=(Ks[l + 1], Ds[l]))) for l in range(L - 1)]
        sp = [rng.uniform(-1.0, 0.2, size=(Ks[l + 1], Ds[l])) for l in range(L - 1)]
        u = [rng.normal(size=Ks[l]) * 2.0 for l in range(L)]
        out.append((z, mu, sp, u))
    return out


def _flat(chains, k, dt):
    idx = {"z": 0, "mu": 1, "s": 2, "u": 3}[k]
    parts = [np.asarray(a).reshape(-1) for c in chains for a in c[idx]]
    return (np.concatenate(parts) if parts else np.zeros(1)).astype(dt)


def _split(flat, chains, k):
    idx = {"z": 0, "mu": 1, "s": 2, "u": 3}[k]
    out, o = [], 0
    for c in chains:
        lst = []
        for a in c[idx]:
            lst.append(flat[o:o + a.size].reshape(a.shape))
            o += a.size
        out.append(lst)
    return out


def _run(chains, prec, flags=0, factors=False):
    from paper_1806_08593_amd import tmc as T
    shapes = [([a.shape[0] for a in c[0]], [a.shape[1] for a in c[0]]) for c in chains]
    prob, sizes = T.ragged_problem(shapes, prec, "auto", flags | T.TMC_FLAG_PARENT_SCALE)
    plan = T.Plan(prob)
    assert plan.info["engine"] == T.TMC_ENGINE_PLAIN
    ws = plan.new_workspace()
    dt = np_dtype(prec)
    d = {k: to_dev(_flat(chains, k, dt)) for k in ("z", "mu", "s", "u")}
    n = len(chains)
    logp = torch.empty(n, dtype=torch.float64, device="cuda:0")
    T.tmc_gauss_fwd(plan.handle, d["z"], d["mu"], d["s"], d["u"], logp, ws)
    dl = to_dev(np.linspace(0.5, 1.5, n))
    g = {k: torch.full_like(v, float("nan")) for k, v in d.items()}
    T.tmc_gauss_bwd(plan.handle, d["z"], d["mu"], d["s"], d["u"], dl, ws, g["z"], g["mu"], g["s"], g["u"])
    out = {k: v.cpu().numpy().astype(np.float64) for k, v in g.items()}
    if factors:
        f = torch.empty(max(sizes["f"], 1), dtype=d["z"].dtype, device="cuda:0")
        T.tmc_gauss_factors(plan.handle, d["z"], d["mu"], d["s"], f)
        out["f"] = f.cpu().numpy().astype(np.float64)
    torch.cuda.synchronize()
    T.tmc_plan_check(plan.handle)
    out["logp"] = logp.cpu().numpy()
    out["dlogp"] = dl.cpu().numpy()
    return out


SHAPES = [((33, 70, 65), (5, 3, 4)), ((64, 64), (1, 2)), ((1, 3, 2), (7, 1, 3)),
          ((100, 37, 129, 8), (33, 64, 2, 5))]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_parent_scale_matches_oracle(prec):
    chains = _chains(5, SHAPES)
    dt = np_dtype(prec)
    cast = [tuple([np.asarray(a, dt).astype(np.float64) for a in part] for part in c) for c in chains]
    got = _run(chains, prec, factors=True)
    ga, gr = GRAD_ELEM_TOL[prec]
    fo = 0
    for c, (z, mu, sp, u) in enumerate(cast):
        lp, dz, dmu, dsp, du = O.gauss_chain_grads_pp(z, mu, sp, u)
        err = abs(got["logp"][c] - lp)
        print(f"ERRREC pp-{prec} logp[{c}] {err:.3e}")
        assert err <= LOGP_TOL[prec] * max(1.0, abs(lp)), (c, got["logp"][c], lp)
        g = got["dlogp"][c]
        for k, ref in (("z", dz), ("mu", dmu), ("s", dsp), ("u", du)):
            blocks = _split(got[k], chains, k)[c]
            for l, rb in enumerate(ref):
                if l == len(ref) - 1 and k == "z":
                    assert np.all(blocks[l] == 0.0)
                    continue
                assert_elem(blocks[l], g * rb, ga, gr, f"pp-{prec}/d{k}/chain{c}/layer{l}")
        for l in range(len(u) - 1):
            fl = O.gauss_pair_logfactor_pp(z[l], mu[l], sp[l])
            n = fl.size
            gf = got["f"][fo:fo + n].reshape(fl.shape)
            fo += n
            tol = 1e-12 if prec == "fp64" else 2e-6
            assert np.max(np.abs(gf - fl)) <= tol * max(1.0, np.max(np.abs(fl))), (c, l)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_equal_scales_reduce_to_shared_scale(prec):
    """Every parent producing the same scale gives the shared-scale plan's log P and
    gradients, with its ds equal to the sum over parents of the per-parent ds."""
    from paper_1806_08593_amd import tmc as T
    chains = _chains(6, [((40, 50, 30), (6, 4, 3)), ((20, 90), (8, 2))])
    shared = []
    for z, mu, sp, u in chains:
        s_row = [a[0] for a in sp]
        shared.append((z, mu, [np.tile(r, (a.shape[0], 1)) for r, a in zip(s_row, sp)], u, s_row))
    pp_chains = [(z, mu, sp, u) for z, mu, sp, u, _ in shared]
    got = _run(pp_chains, prec)
    # the shared-scale plan on the same inputs, plain engine
    shapes = [([a.shape[0] for a in c[0]], [a.shape[1] for a in c[0]]) for c in pp_chains]
    prob, _ = T.ragged_problem(shapes, prec, "plain")
    plan = T.Plan(prob)
    ws = plan.new_workspace()
    dt = np_dtype(prec)
    s_flat = np.concatenate([np.asarray(r).reshape(-1) for c in shared for r in c[4]]).astype(dt)
    d = {k: to_dev(_flat(pp_chains, k, dt)) for k in ("z", "mu", "u")}
    d["s"] = to_dev(s_flat)
    logp = torch.empty(len(pp_chains), dtype=torch.float64, device="cuda:0")
    T.tmc_gauss_fwd(plan.handle, d["z"], d["mu"], d["s"], d["u"], logp, ws)
    dl = to_dev(np.linspace(0.5, 1.5, len(pp_chains)))
    g = {k: torch.empty_like(v) for k, v in d.items()}
    T.tmc_gauss_bwd(plan.handle, d["z"], d["mu"], d["s"], d["u"], dl, ws, g["z"], g["mu"], g["s"], g["u"])
    torch.cuda.synchronize()
    ref = {k: v.cpu().numpy().astype(np.float64) for k, v in g.items()}
    rt = 1e-12 if prec == "fp64" else 2e-5
    np.testing.assert_allclose(got["logp"], logp.cpu().numpy(), rtol=rt, atol=rt)
    for k in ("z", "mu", "u"):
        scale = np.abs(ref[k]).max()
        assert np.max(np.abs(got[k] - ref[k])) <= 10 * rt * scale, k
    o = so = 0
    for c in shared:
        for l, r in enumerate(c[4]):
            K1, D = c[2][l].shape
            blk = got["s"][so:so + K1 * D].reshape(K1, D).sum(axis=0)
            so += K1 * D
            want = ref["s"][o:o + D]
            o += D
            assert np.max(np.abs(blk - want)) <= 10 * rt * max(1.0, np.abs(want).max()), (l,)


def test_parent_scale_rejects_fused_and_shared_blocks():
    from paper_1806_08593_amd import tmc as T
    with pytest.raises(T.TMCError) as ei:
        T.Plan(T.homogeneous_problem(2, 3, 16, 8, "fp32", "fused", T.TMC_FLAG_PARENT_SCALE))
    assert ei.value.status == T.TMC_ERR_UNSUPPORTED
    # shared [D] blocks under the flag overlap as [K][D] blocks: the Gaussian calls refuse
    prob = T.homogeneous_problem(2, 3, 16, 8, "fp32", "plain")
    prob.c.flags = T.TMC_FLAG_PARENT_SCALE
    plan = T.Plan(prob)
    d = to_dev(np.zeros(2 * 3 * 16 * 8, np.float32))
    lp = torch.empty(2, dtype=torch.float64, device="cuda:0")
    with pytest.raises(T.TMCError) as ei:
        T.tmc_gauss_fwd(plan.handle, d, d, d, d, lp, plan.new_workspace())
    assert "overlap" in str(ei.value)
