"""Helpers for the GPU parity tests: upload seeded workloads, run the library through
its C ABI (ctypes binding), run the oracle on the same (cast) inputs."""
import numpy as np
import pytest

from oracle import tmc_oracle as O
from workloads import Chain, cast_chain

torch = pytest.importorskip("torch")


def np_dtype(prec):
    return np.float64 if prec == "fp64" else np.float32


def torch_dtype(prec):
    return torch.float64 if prec == "fp64" else torch.float32


def pack_chains(chains, prec, with_f=False):
    """Flatten chains into the ragged layout of tmc.ragged_problem; returns
    (shapes, dict of numpy flat arrays)."""
    dt = np_dtype(prec)
    shapes = [([int(a.shape[0]) for a in c.z], [int(a.shape[1]) for a in c.z]) for c in chains]
    z = np.concatenate([a.reshape(-1) for c in chains for a in c.z]).astype(dt)
    u = np.concatenate([a.reshape(-1) for c in chains for a in c.u]).astype(dt)
    mus = [a.reshape(-1) for c in chains for a in c.mu]
    mu = (np.concatenate(mus) if mus else np.zeros(1)).astype(dt)
    ss = [a.reshape(-1) for c in chains for a in c.s]
    s = (np.concatenate(ss) if ss else np.zeros(1)).astype(dt)
    out = dict(z=z, u=u, mu=mu, s=s)
    return shapes, out


def unpack(flat, chains, what):
    """Split a flat gradient array back into per-chain per-layer arrays."""
    out, o = [], 0
    for c in chains:
        lst = []
        arrs = getattr(c, what)
        for a in arrs:
            n = a.size
            lst.append(flat[o:o + n].reshape(a.shape))
            o += n
        out.append(lst)
    return out


def to_dev(a, prec=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    return t.to("cuda:0")


def oracle_grads(chains):
    res = []
    for c in chains:
        res.append(O.gauss_chain_grads(c.z, c.mu, c.s, c.u))
    return res


def elem_err(got, ref):
    """max_k |got_k - ref_k| / max_k |ref_k| over one block (0 for an all-zero block that
    is matched exactly)."""
    got = np.asarray(got, np.float64).reshape(-1)
    ref = np.asarray(ref, np.float64).reshape(-1)
    d = np.abs(got - ref).max() if ref.size else 0.0
    scale = np.abs(ref).max() if ref.size else 0.0
    return float(d / scale) if scale > 0 else float(d)


def assert_elem(got, ref, atol_frac, rtol, label):
    """Element-wise parity of one block: |got - ref| <= atol_frac * max|ref| + rtol * |ref|
    for every element (NaN fails).  Prints the block-scaled maximum error on a line
    starting with ERRREC, so a run with -s records the measured errors."""
    got = np.asarray(got, np.float64).reshape(-1)
    ref = np.asarray(ref, np.float64).reshape(-1)
    assert got.shape == ref.shape, (label, got.shape, ref.shape)
    scale = np.abs(ref).max() if ref.size else 0.0
    bound = atol_frac * scale + rtol * np.abs(ref)
    err = np.abs(got - ref)
    e = elem_err(got, ref)
    print(f"ERRREC {label} {e:.3e}")
    bad = ~(err <= bound)
    if bad.any():
        k = int(np.argmax(np.where(bad, err - bound, -np.inf)))
        raise AssertionError(f"{label}: element {k} got {got[k]!r} ref {ref[k]!r} "
                             f"(|d| {err[k]:.3e} > bound {bound[k]:.3e}; block max|ref| {scale:.3e}; "
                             f"{int(bad.sum())} of {bad.size} outside)")
    return e


# Element-wise gradient tolerances (atol as a fraction of the block's max |ref|, rtol),
# per arithmetic mode: about five times the largest block-scaled error measured over
# every gradient block of the GPU parity tests (FP64 2.5e-13, FP32 fused 8.0e-6, FP32
# plain 3.5e-6, BF16X3 9.5e-5), rounded up.
GRAD_ELEM_TOL = {"fp64": (1e-11, 1e-10), "fp32": (5e-5, 1e-4), "bf16x3": (5e-4, 5e-3)}


def rel_l2(a, b):
    a = np.asarray(a, np.float64).reshape(-1)
    b = np.asarray(b, np.float64).reshape(-1)
    den = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (den if den > 0 else 1.0)


def run_gauss(chains, prec, engine="auto", flags=0, bwd=True, graph=False):
    """Run fwd (and bwd with dlogp = 1) of the Gaussian chain entry points on the
    ragged packing of `chains`.  Returns dict with logp and flat gradients."""
    from paper_1806_08593_amd import tmc as T
    shapes, flat = pack_chains(chains, prec)
    prob, sizes = T.ragged_problem(shapes, prec, engine, flags)
    plan = T.Plan(prob)
    ws = plan.new_workspace()
    dev = {k: to_dev(v) for k, v in flat.items()}
    n = len(chains)
    logp = torch.empty(n, dtype=torch.float64, device="cuda:0")
    T.tmc_gauss_fwd(plan.handle, dev["z"], dev["mu"], dev["s"], dev["u"], logp, ws)
    out = dict(plan=plan, info=plan.info)
    if bwd:
        dlogp = torch.ones(n, dtype=torch.float64, device="cuda:0")
        g = {k: torch.full_like(dev[k], float("nan")) for k in ("z", "mu", "s", "u")}
        T.tmc_gauss_bwd(plan.handle, dev["z"], dev["mu"], dev["s"], dev["u"], dlogp, ws,
                        g["z"], g["mu"], g["s"], g["u"])
        out.update({"d" + k: v.cpu().numpy().astype(np.float64) for k, v in g.items()})
    torch.cuda.synchronize()
    out["logp"] = logp.cpu().numpy()
    T.tmc_plan_check(plan.handle)
    return out


def cast_chains(chains, prec):
    return [cast_chain(c, np_dtype(prec)) for c in chains]
