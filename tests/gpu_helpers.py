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
