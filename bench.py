#!/usr/bin/env python
"""Throughput of the TMC chain estimator on one MI355X.

One step = one forward + backward pass of the Gaussian-chain estimator (factor
construction, top-down log-sum-exp messages, FP64 log-normaliser, marginals and the
gradients with respect to z, mu, s and u) over one batch of synthetic inputs that
are already resident in device memory.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c3]
                    [--precision bf16x3|fp32|fp64] [--engine auto|fused|plain]

Prints one JSON line.  `value` is factor entries per second, where a step processes
sum over chains and adjacent layer pairs of K_l * K_{l+1} entries.  The roofline
object describes the kernel class with the largest device time, timed with HIP
events recorded by the library around each of its launches in the timed region.
The cpu_baseline object times the FP64 NumPy oracle on a bounded sample of the same
workload on the host.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# dense peaks (TFLOP/s) of MI355X: matrix cores by dtype, vector ALU without packed FP32
MFMA_PEAK = {"bf16x3": 2500.0, "fp32": 157.3, "fp64": 78.6}
VALU_PEAK = {"fp32": 78.6, "fp64": 78.6, "bf16x3": 78.6}


def _algorithmic(kc_name, entries, D, prec, pairs_bytes):
    """(amount per step, unit, bound, peak) of one kernel class.
    Fused kernels: the factor GEMM counts 2*D flops per entry; the forward also
    forms the softmax-weighted mean of mu (2*D), the backward recomputes the
    factors (2*D) and forms G^T z (2*D).  Plain log-sum-exp passes are HBM-bound:
    the forward reads f once (esz bytes per entry), the backward reads f and
    writes G (2*esz)."""
    esz = 8 if prec == "fp64" else 4
    if kc_name == "fused_fwd":
        return 4.0 * D * entries, "TFLOP/s", "mfma", MFMA_PEAK[prec]
    if kc_name == "fused_bwd":
        return 4.0 * D * entries, "TFLOP/s", "mfma", MFMA_PEAK[prec]
    if kc_name == "plain_lse_fwd":
        return float(esz * entries), "GB/s", "hbm", HBM_PEAK_GBS
    if kc_name == "plain_lse_bwd":
        return float(2 * esz * entries), "GB/s", "hbm", HBM_PEAK_GBS
    if kc_name == "plain_factor":
        # direct difference: 3 flops per (entry, d)
        return 3.0 * D * entries, "TFLOP/s", "alu", VALU_PEAK[prec]
    if kc_name == "plain_grad":
        # G mu and G^T z: 2 * 2*D flops per entry
        return 4.0 * D * entries, "TFLOP/s", "alu", VALU_PEAK[prec]
    if kc_name == "fused_prep":
        return float(pairs_bytes), "GB/s", "hbm", HBM_PEAK_GBS
    return None


def cpu_baseline(chains, budget_s=15.0):
    """Time the FP64 oracle (forward + backward) on as many instances as fit in
    about budget_s seconds of host time; returns (entries/s, sample description,
    per-instance oracle log P)."""
    from oracle import tmc_oracle as O
    t0 = time.perf_counter()
    done, ent, refs = 0, 0, []
    for c in chains:
        refs.append(O.gauss_chain_grads(c.z, c.mu, c.s, c.u)[0])
        done += 1
        ent += c.entries()
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return ent / dt, done, dt, refs


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c3")
    ap.add_argument("--precision", default=None)
    ap.add_argument("--engine", default="auto")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1806_08593_amd import tmc as T
    from workloads import CONFIGS, cast_chain, make

    cfg = CONFIGS[args.workload]
    prec = args.precision or ("fp64" if args.workload == "c1" else "bf16x3")
    print(f"[bench] generating workload {args.workload} ...", file=sys.stderr, flush=True)
    w = make(args.workload)
    B, L, K, D = w.z.shape
    tdt = torch.float64 if prec == "fp64" else torch.float32
    dev = "cuda:0"
    z = torch.tensor(w.z, dtype=tdt, device=dev)
    mu = torch.tensor(w.mu, dtype=tdt, device=dev)
    s = torch.tensor(w.s, dtype=tdt, device=dev)
    u = torch.tensor(w.u, dtype=tdt, device=dev)
    prob = T.homogeneous_problem(B, L, K, D, prec, args.engine)
    plan = T.Plan(prob)
    ws = plan.new_workspace()
    logp = torch.empty(B, dtype=torch.float64, device=dev)
    dlogp = torch.ones(B, dtype=torch.float64, device=dev)
    dz, dmu, ds, du = (torch.empty_like(t) for t in (z, mu, s, u))
    entries = plan.info["factor_entries"]
    h = plan.handle

    def step():
        T.tmc_gauss_fwd(h, z, mu, s, u, logp, ws)
        T.tmc_gauss_bwd(h, z, mu, s, u, dlogp, ws, dz, dmu, ds, du)

    print(f"[bench] warmup {args.warmup} steps ...", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    T.tmc_plan_check(h)

    T.tmc_plan_set_timing(h, True)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall_ms = (t1 - t0) * 1e3 / args.steps
    ev_ms = e0.elapsed_time(e1) / args.steps
    kc = {}
    for i, name in enumerate(T.KERNEL_CLASSES):
        ms, n = T.tmc_plan_timing(h, i)
        if n:
            kc[name] = dict(ms_per_step=ms / args.steps, launches_per_step=n / args.steps,
                            avg_launch_us=1e3 * ms / n)
    T.tmc_plan_set_timing(h, False)
    T.tmc_plan_check(h)
    ms_per_step = wall_ms
    value = entries / (ms_per_step / 1e3)

    dom = max((k for k in kc if k != "other"), key=lambda k: kc[k]["ms_per_step"])
    alg = _algorithmic(dom, entries, D, prec, 0)
    roofline = None
    if alg is not None:
        amount, unit, bound, peak = alg
        per_launch = amount / kc[dom]["launches_per_step"]
        secs = kc[dom]["avg_launch_us"] * 1e-6
        achieved = per_launch / secs / (1e12 if unit == "TFLOP/s" else 1e9)
        roofline = dict(kernel=dom, bound=bound, achieved=round(achieved, 3), peak=peak, unit=unit,
                        frac=round(achieved / peak, 4), traffic=None,
                        algorithmic_per_launch=per_launch,
                        avg_launch_us=round(kc[dom]["avg_launch_us"], 3))

    # accuracy and CPU baseline on the same instances
    out_logp = logp.cpu().numpy()
    cpu = None
    err = None
    if not args.no_cpu_baseline:
        npdt = np.float64 if prec == "fp64" else np.float32
        sample = [cast_chain(c, npdt) for c in w.chains]
        print(f"[bench] CPU oracle baseline (~{args.cpu_budget:.0f} s) ...", file=sys.stderr, flush=True)
        rate, done, dt, refs = cpu_baseline(sample, args.cpu_budget)
        err = float(max(abs(out_logp[b] - refs[b]) for b in range(done)))
        cpu = dict(value=rate, unit="factor entries/s", cores=1, kind="oracle",
                   sample=f"forward+backward of {done} of {B} instances "
                          f"({done * entries // B} entries) in {dt:.1f} s, FP64 NumPy, one thread")

    line = {
        "metric": "factor entries/s (fwd+bwd)",
        "value": value,
        "unit": "factor entries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"bf16x3": "bf16", "fp32": "f32", "fp64": "f64"}[prec],
        "data": "synthetic",
        "config": {"workload": args.workload, "B": B, "L": L, "K": K, "D": D,
                   "precision": prec, "engine": ["auto", "fused", "plain"][plan.info["engine"]],
                   "factor_entries": entries, "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "max_abs_err_logp_vs_oracle": err,
        "event_ms_per_step": ev_ms,
        "kernels": kc,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
