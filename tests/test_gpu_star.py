"""GPU parity of the star-model entry points (tmc_star_gauss_fwd / _bwd) against the FP64
oracle: log P of every instance and every gradient element, on seeded inputs rounded to
the precision the kernels see.  Shapes span several 64-sample blocks of both indices with
ragged tails, point groups of one and of several points, every width bucket (D = 1, 4,
16, 32), and the degenerate cases (one sample, one point, -inf and NaN terms).  The
full-size cases are the two ends of the Gaussian example's sweeps: N = 4096 points with
K = K_theta = 128, and N = 128 with K = K_theta = 2048."""
import functools

import numpy as np
import pytest

from oracle import tmc_oracle as O
from tests.gpu_helpers import GRAD_ELEM_TOL, assert_elem, np_dtype, to_dev
from workloads import gauss_star, make_star

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

# |log P - oracle| <= rtol |log P| + atol: FP32 rounds every entry of the N sums that make
# up log P (|log P| ~ N nats here), FP64 only at 1e-16 per operation.
LOGP_TOL = {"fp64": (1e-12, 1e-10), "fp32": (2e-6, 1e-5)}
# Element-wise gradient bounds (atol as a fraction of the block's max |ref|, rtol).  The
# weights are exp(uth + sum_i m_i - log P) with |sum_i m_i| ~ |log P| (~1e4 nats at
# N = 4096), so an FP64 rounding of 1e-16 |log P| in that sum is a relative error of
# ~1e-12 in every weight and gradient (measured 6.7e-12 at N = 4096); FP32 as for chains
# (measured 1.2e-5).
STAR_GRAD_TOL = {"fp64": (1e-10, 1e-10), "fp32": GRAD_ELEM_TOL["fp32"]}


def run_star(w, prec, bwd=True, flags=0, dlogp=None):
    from paper_1806_08593_amd import tmc as T
    sh = w.shape
    plan = T.Plan(T.StarProblem(sh["S"], sh["N"], sh["Kt"], sh["K"], sh["D"], prec, flags))
    ws = plan.new_workspace()
    dt = np_dtype(prec)
    dev = {k: to_dev(getattr(w, k).astype(dt)) for k in ("mth", "s", "z", "u", "uth")}
    logp = torch.full((sh["S"],), float("nan"), dtype=torch.float64, device="cuda:0")
    T.tmc_star_gauss_fwd(plan.handle, dev["mth"], dev["s"], dev["z"], dev["u"], dev["uth"], logp, ws)
    out = {"plan": plan}
    if bwd:
        g = np.linspace(0.5, 1.5, sh["S"]) if dlogp is None else np.asarray(dlogp, np.float64)
        dl = to_dev(g)
        grads = {k: torch.full_like(dev[k], float("nan")) for k in ("mth", "s", "z", "u", "uth")}
        T.tmc_star_gauss_bwd(plan.handle, dev["mth"], dev["s"], dev["z"], dev["u"], dl, ws,
                             grads["mth"], grads["s"], grads["z"], grads["u"], grads["uth"])
        out.update({"d" + k: v.cpu().numpy().astype(np.float64) for k, v in grads.items()})
        out["dlogp"] = g
    torch.cuda.synchronize()
    out["logp"] = logp.cpu().numpy()
    return out


def oracle_star(w, prec):
    """Per instance: (log P, d mth, d s, d z [N, K, D], d u [N, K], weights) of the oracle on
    the inputs rounded to `prec`."""
    c = lambda a: np.asarray(a, np_dtype(prec)).astype(np.float64)
    sh = w.shape
    res = []
    for i in range(sh["S"]):
        lp, dm, ds, dz, du, wt = O.gauss_star_grads(c(w.mth[i]), c(w.s[i]),
                                                    [c(w.z[i, n]) for n in range(sh["N"])],
                                                    [c(w.u[i, n]) for n in range(sh["N"])],
                                                    c(w.uth[i]))
        res.append(dict(logp=lp, dmth=dm, ds=ds, dz=np.stack(dz), du=np.stack(du), duth=wt))
    return res


def check(w, prec, got, ref, label):
    rt, at = LOGP_TOL[prec]
    ga, gr = STAR_GRAD_TOL[prec]
    for i, r in enumerate(ref):
        err = abs(got["logp"][i] - r["logp"])
        print(f"ERRREC {label} logp[{i}] {err:.3e} (|logp| {abs(r['logp']):.3e})")
        assert err <= rt * abs(r["logp"]) + at, (label, i, got["logp"][i], r["logp"])
        if "dmth" not in got:
            continue
        g = got["dlogp"][i]
        for k in ("dmth", "ds", "dz", "du", "duth"):
            assert_elem(got[k][i], g * r[k], ga, gr, f"{label} {k}[{i}]")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("D", [1, 3, 16, 32])
def test_star_parity_small(prec, D):
    """Three global-sample blocks (150 = 64 + 64 + 22), two local blocks (100 = 64 + 36),
    two instances with different upstream gradients, one point per group."""
    w = gauss_star(S=2, N=37, Kt=150, K=100, D=D, kind="general")
    check(w, prec, run_star(w, prec), oracle_star(w, prec), f"star-small-{prec}-D{D}")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_star_parity_groups(prec):
    """Many points: groups of four (one per wave), the last group with one point."""
    w = gauss_star(S=1, N=3001, Kt=100, K=20, D=2, kind="general")
    out = run_star(w, prec)
    assert out["plan"].workspace_bytes > 0
    check(w, prec, out, oracle_star(w, prec), f"star-groups-{prec}")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("shape", [(1, 1, 1, 1), (3, 1, 1, 5), (2, 5, 1, 64), (1, 2, 64, 1),
                                   (1, 4, 65, 129)])
def test_star_degenerate_shapes(prec, shape):
    """One point, one sample of either latent, exact block multiples and one past them."""
    S, N, Kt, K = shape
    w = gauss_star(S=S, N=N, Kt=Kt, K=K, D=2, kind="general")
    check(w, prec, run_star(w, prec), oracle_star(w, prec), f"star-edge-{prec}-{shape}")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_star_infinite_terms(prec):
    """-inf unary terms: instance 0 has some local samples and some global samples
    removed (finite log P; their gradients are 0); instance 1 has a point whose every
    local sample is removed (log P = -inf, every gradient 0, no NaN, no numeric flag)."""
    from paper_1806_08593_amd import tmc as T
    w = gauss_star(S=2, N=9, Kt=70, K=66, D=2, kind="general")
    w.u[0, 3, ::3] = -np.inf
    w.uth[0, 5:40] = -np.inf
    w.u[1, 4, :] = -np.inf
    out = run_star(w, prec)
    ref = oracle_star(w, prec)
    assert out["logp"][1] == -np.inf and ref[1]["logp"] == -np.inf
    for k in ("dmth", "ds", "dz", "du", "duth"):
        assert np.all(out[k][1] == 0.0), k
    check(w, prec, {k: (v[:1] if isinstance(v, np.ndarray) else v) for k, v in out.items()},
          ref[:1], f"star-inf-{prec}")
    T.tmc_plan_check(out["plan"].handle)


def test_star_nan_flags():
    """A NaN unary term makes its instance's log P NaN and raises the numeric flag; the
    other instance is unaffected."""
    from paper_1806_08593_amd import tmc as T
    w = gauss_star(S=2, N=5, Kt=10, K=12, D=1, kind="toy")
    w.u[1, 2, 7] = np.nan
    out = run_star(w, "fp32", bwd=False)
    assert np.isnan(out["logp"][1])
    ref = oracle_star(w, "fp32")
    assert abs(out["logp"][0] - ref[0]["logp"]) < 1e-4
    with pytest.raises(T.TMCError) as ei:
        T.tmc_plan_check(out["plan"].handle)
    assert ei.value.status == T.TMC_ERR_NUMERIC


def test_star_forward_only_and_kind_checks():
    """A forward-only plan has a smaller workspace and refuses the backward; chain and star
    plans refuse each other's entry points."""
    from paper_1806_08593_amd import tmc as T
    w = gauss_star(S=1, N=20, Kt=30, K=40, D=2, kind="general")
    full = run_star(w, "fp32", bwd=False)
    fo = run_star(w, "fp32", bwd=False, flags=T.TMC_FLAG_FORWARD_ONLY)
    assert fo["plan"].workspace_bytes < full["plan"].workspace_bytes
    assert fo["logp"][0] == full["logp"][0]
    d = to_dev(np.ones(1))
    ws = fo["plan"].new_workspace()
    with pytest.raises(T.TMCError) as ei:
        T.tmc_star_gauss_bwd(fo["plan"].handle, d, d, d, d, d, ws, None, None, None, None, None)
    assert ei.value.status == T.TMC_ERR_STATE
    with pytest.raises(T.TMCError) as ei:
        T.tmc_gauss_fwd(fo["plan"].handle, d, d, d, d, d, ws)
    assert ei.value.status == T.TMC_ERR_INVALID_ARG and "star" in str(ei.value)
    chain = T.Plan(T.homogeneous_problem(1, 2, 8, 4))
    with pytest.raises(T.TMCError) as ei:
        T.tmc_star_gauss_fwd(chain.handle, d, d, d, d, d, d, chain.new_workspace())
    assert ei.value.status == T.TMC_ERR_INVALID_ARG


def test_star_partial_gradients():
    """NULL gradient pointers skip their outputs; the others are unchanged."""
    from paper_1806_08593_amd import tmc as T
    w = gauss_star(S=1, N=11, Kt=20, K=30, D=3, kind="general")
    full = run_star(w, "fp64")
    sh = w.shape
    plan = T.Plan(T.StarProblem(sh["S"], sh["N"], sh["Kt"], sh["K"], sh["D"], "fp64"))
    ws = plan.new_workspace()
    dev = {k: to_dev(getattr(w, k)) for k in ("mth", "s", "z", "u", "uth")}
    logp = torch.empty(1, dtype=torch.float64, device="cuda:0")
    T.tmc_star_gauss_fwd(plan.handle, dev["mth"], dev["s"], dev["z"], dev["u"], dev["uth"], logp, ws)
    dl = to_dev(np.array([0.5]))
    dmth = torch.full_like(dev["mth"], float("nan"))
    ds = torch.full_like(dev["s"], float("nan"))
    T.tmc_star_gauss_bwd(plan.handle, dev["mth"], dev["s"], dev["z"], dev["u"], dl, ws, dmth, ds,
                         None, None, None)
    torch.cuda.synchronize()
    assert np.array_equal(dmth.cpu().numpy(), full["dmth"])
    assert np.array_equal(ds.cpu().numpy(), full["ds"])


def test_star_deterministic():
    """Two runs give bit-identical results (fixed-order sums everywhere)."""
    w = gauss_star(S=2, N=300, Kt=90, K=70, D=4, kind="general")
    a = run_star(w, "fp32")
    b = run_star(w, "fp32")
    for k in ("logp", "dmth", "ds", "dz", "du", "duth"):
        assert np.array_equal(a[k], b[k]), k


@functools.lru_cache(maxsize=None)
def _exact_evidence(config):
    return O.gauss_star_log_evidence(make_star(config).x[0, :, 0])


@pytest.mark.parametrize("config", ["s1", "s2"])
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_star_full_size(config, prec):
    """The Gaussian example's full-size workloads, every output against the oracle, and
    log P against the exact log-evidence of the model (a lower bound in expectation that
    tightens with K: within 0.1 nats per data point at these sizes)."""
    w = make_star(config)
    out = run_star(w, prec, dlogp=[1.0])
    ref = oracle_star(w, prec)
    check(w, prec, out, ref, f"star-{config}-{prec}")
    exact = _exact_evidence(config)
    N = w.shape["N"]
    assert exact - 0.1 * N < out["logp"][0] < exact + 0.01 * N, (out["logp"][0], exact)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_star_autograd_wrapper(prec):
    """torch.autograd over the star model: a weighted sum of the instances' log P
    differentiates to the weighted oracle gradients of all five inputs."""
    from paper_1806_08593_amd import autograd as A
    w = gauss_star(S=3, N=9, Kt=70, K=65, D=3, kind="general")
    sh = w.shape
    run = A.StarGaussTMC(sh["S"], sh["N"], sh["Kt"], sh["K"], sh["D"], precision=prec)
    dt = np_dtype(prec)
    t = {k: to_dev(getattr(w, k).astype(dt)).requires_grad_(True) for k in ("mth", "s", "z", "u", "uth")}
    logp = run(t["mth"], t["s"], t["z"], t["u"], t["uth"])
    wts = torch.tensor([1.0, -0.5, 2.0], dtype=torch.float64, device="cuda:0")
    (logp * wts).sum().backward()
    got = {"logp": logp.detach().cpu().numpy(), "dlogp": wts.cpu().numpy()}
    got.update({"d" + k: v.grad.cpu().numpy().astype(np.float64) for k, v in t.items()})
    check(w, prec, got, oracle_star(w, prec), f"star-autograd-{prec}")
