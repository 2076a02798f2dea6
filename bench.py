#!/usr/bin/env python
"""Throughput of the TMC chain estimator on one MI355X.

One step = one forward + backward pass of the Gaussian-chain estimator over one batch
of synthetic inputs already resident in device memory: the pairwise factors on
MFMA, the top-down log-sum-exp messages, the FP64 log-normaliser, the pairwise
marginals and the gradients with respect to z, mu, s and u.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c3]
                    [--precision bf16x3|fp32|fp64] [--engine auto|fused|plain]
                    [--no-compare] [--no-cpu-baseline] [--calibrate-copy MB]

Prints one JSON line.  `value` is factor entries per second (a step processes the
sum over chains and adjacent layer pairs of K_l * K_{l+1} entries); the timed steps
replay the forward and backward graphs captured from the library's launches
(--no-graph: eager launches).  `roofline` describes the kernel class with the largest
device time in a second region of eager steps, timed with HIP events that the
library records around each of its launches on the stream it launches on.  `compare` times the same step in the other precisions / engines
and gives each one's error against the FP64 oracle; `cpu_baseline` times the FP64
oracle on a bounded sample of the workload on the host.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# dense peaks of MI355X (TFLOP/s): matrix cores by operand type; vector ALU without
# packed FP32 (256 CUs x 4 SIMD x 16 lanes x 2 flops x 2.4 GHz)
MFMA_PEAK = {"bf16x3": 2500.0, "fp32": 157.3, "fp64": 78.6}
VALU_PEAK = 78.6


def algorithmic(kc_name, entries, d_weighted, prec):
    """(amount per step, unit, bound, peak) of one kernel class; d_weighted is
    sum over pairs of K_l K_{l+1} D_l.  Fused forward: the factor GEMM (2 D flops per
    entry) and the softmax-weighted mean of mu (2 D); fused backward: the recomputed
    factor GEMM (2 D) and G^T z (2 D).  Plain log-sum-exp passes stream the stored
    factors: the forward reads esz bytes per entry, the backward reads f and writes G."""
    esz = 8 if prec == "fp64" else 4
    if kc_name in ("fused_fwd", "fused_bwd"):
        return 4.0 * d_weighted, "TFLOP/s", "mfma", MFMA_PEAK[prec]
    if kc_name == "plain_lse_fwd":
        return float(esz * entries), "GB/s", "hbm", HBM_PEAK_GBS
    if kc_name == "plain_lse_bwd":
        return float(2 * esz * entries), "GB/s", "hbm", HBM_PEAK_GBS
    if kc_name == "plain_factor":
        return 3.0 * d_weighted, "TFLOP/s", "alu", VALU_PEAK
    if kc_name == "plain_grad":
        return 4.0 * d_weighted, "TFLOP/s", "alu", VALU_PEAK
    return None


# Sources whose compiled code the fused kernels are (their hash dates a counter record).
KERNEL_SOURCES = ["fused_kernels.h", "k_fused_inst.inc", "k_fused_bf16.hip", "k_fused_f32.hip",
                  "dev_util.h", "tmc_internal.h"]
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "fused_c3_bf16x3_pmc.md")


def kernel_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1806_08593_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic(kernel, workload, prec, waves=4):
    """(read bytes, written bytes) per launch of `kernel` in its `waves`-wave form from the
    committed counter record, or None when there is none for this workload, precision
    and form or the kernel sources changed since it was taken.  The record is a block of
    lines
        traffic-record sources-sha256 <hex> workload <w> precision <p>
        traffic-record <kernel class> waves <n> read-bytes <r> written-bytes <w>
    in the profile summary (FETCH_SIZE and WRITE_SIZE scaled by the copy calibration)."""
    try:
        lines = open(TRAFFIC_RECORD).read().splitlines()
    except OSError:
        return None
    head, rows = None, {}
    for ln in lines:
        t = ln.split()
        if len(t) >= 7 and t[0] == "traffic-record" and t[1] == "sources-sha256":
            head = dict(sha=t[2], workload=t[4], precision=t[6])
        elif len(t) == 8 and t[0] == "traffic-record" and t[2] == "waves":
            rows[(t[1], int(t[3]))] = (float(t[5]), float(t[7]))
    if head is None or head["workload"] != workload or head["precision"] != prec:
        return None
    if head["sha"] != kernel_sources_sha256():
        return None
    return rows.get((kernel, waves))


def upload(w, prec, engine, flags=0):
    """Device buffers and the problem for workload w (homogeneous layout with s shared
    by the batch when w is a stacked batch, packed ragged layout otherwise)."""
    import numpy as np
    import torch
    from paper_1806_08593_amd import tmc as T
    from workloads import pack
    tdt = torch.float64 if prec == "fp64" else torch.float32
    npdt = np.float64 if prec == "fp64" else np.float32
    if w.z is not None:
        B, L, K, D = w.z.shape
        prob = T.homogeneous_problem(B, L, K, D, prec, engine, flags)
        arrs = {k: getattr(w, k) for k in ("z", "mu", "s", "u")}
    else:
        shapes, arrs = pack(w.chains, npdt)
        prob, _ = T.ragged_problem(shapes, prec, engine, flags)
    dev = {k: torch.tensor(np.ascontiguousarray(v), dtype=tdt, device="cuda:0") for k, v in arrs.items()}
    return prob, dev


def run_mode(w, prec, engine, steps, warmup, timing, tune=False, flags=0, graph=True):
    """Times `steps` steps of workload w after `warmup` eager steps, all on one stream.
    graph: the step is a replay of the forward and backward graphs captured from the
    library's own launches (the same kernels; no host launch gaps).  timing: afterwards,
    a second region of eager steps with the library's per-kernel HIP events, for the
    kernel breakdown."""
    import torch
    from paper_1806_08593_amd import tmc as T
    prob, d = upload(w, prec, engine, flags)
    plan = T.Plan(prob)
    ws = plan.new_workspace()
    n = prob.n_chains
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        logp = torch.empty(n, dtype=torch.float64, device="cuda:0")
        dlogp = torch.ones(n, dtype=torch.float64, device="cuda:0")
        g = {k: torch.empty_like(v) for k, v in d.items()}
        st.synchronize()
        h = plan.handle
        if tune and plan.info["engine"] == T.TMC_ENGINE_FUSED:
            # the library's launch-shape tuner, outside the timed region
            T.tmc_plan_autotune(h, d["z"], d["mu"], d["s"], d["u"], dlogp, ws, g["z"], g["mu"],
                                g["s"], g["u"], reps=3, stream=st)

        def eager():
            T.tmc_gauss_fwd(h, d["z"], d["mu"], d["s"], d["u"], logp, ws, st)
            T.tmc_gauss_bwd(h, d["z"], d["mu"], d["s"], d["u"], dlogp, ws, g["z"], g["mu"], g["s"],
                            g["u"], st)

        for _ in range(warmup):
            eager()
        st.synchronize()
        T.tmc_plan_check(h)
        step = eager
        if graph:
            T.tmc_plan_graph_capture_gauss(h, 0, d["z"], d["mu"], d["s"], d["u"], logp, None, ws,
                                           None, None, None, None, st)
            T.tmc_plan_graph_capture_gauss(h, 1, d["z"], d["mu"], d["s"], d["u"], None, dlogp, ws,
                                           g["z"], g["mu"], g["s"], g["u"], st)

            def step():
                T.tmc_plan_graph_launch(h, 0, st)
                T.tmc_plan_graph_launch(h, 1, st)

            step()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()                     # (one GPU: the barrier is this sync)
        t0 = time.perf_counter()
        e0.record(st)
        for _ in range(steps):
            step()
        e1.record(st)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        T.tmc_plan_check(h)
        lp = logp.cpu().numpy()
        kc, eager_ms = {}, None
        if timing:
            ksteps = max(3, steps // 2)
            T.tmc_plan_set_timing(h, True)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            for _ in range(ksteps):
                eager()
            torch.cuda.synchronize()
            eager_ms = (time.perf_counter() - t2) * 1e3 / ksteps
            for i, name in enumerate(T.KERNEL_CLASSES):
                ms, cnt = T.tmc_plan_timing(h, i)
                if cnt:
                    kc[name] = dict(ms_per_step=ms / ksteps, launches_per_step=cnt / ksteps,
                                    avg_launch_us=1e3 * ms / cnt)
            T.tmc_plan_set_timing(h, False)
            T.tmc_plan_check(h)
        out = dict(ms_per_step=(t1 - t0) * 1e3 / steps, event_ms_per_step=e0.elapsed_time(e1) / steps,
                   eager_ms_per_step=eager_ms, kernels=kc, logp=lp, info=T.tmc_plan_info_get(h))
    plan.close()
    del d, g, ws
    torch.cuda.empty_cache()
    return out


def cpu_baseline(chains, budget_s):
    """FP64 oracle (forward + backward) on as many instances as fit in about budget_s
    seconds of host time.  Returns (entries/s, instances done, seconds, log P list)."""
    from oracle import tmc_oracle as O
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):        # one host thread, so that `cores` is exact
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
    ap.add_argument("--no-compare", action="store_true")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the launch-shape tuner (per-depth launches unless --persistent)")
    ap.add_argument("--persistent", action="store_true", help="persistent launches (with --no-tune)")
    ap.add_argument("--no-graph", action="store_true",
                    help="time eager launches instead of replays of the captured step graphs")
    ap.add_argument("--calibrate-copy", type=float, default=0.0,
                    help="first copy this many MiB with a plain device copy (a known-size "
                         "kernel for scaling memory counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    from workloads import cast_chain, make

    if args.calibrate_copy > 0:
        n = int(args.calibrate_copy * 2 ** 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    prec = args.precision or ("fp64" if args.workload == "c1" else "bf16x3")
    print(f"[bench] generating workload {args.workload} ...", file=sys.stderr, flush=True)
    w = make(args.workload)
    entries = w.entries()
    d_weighted = float(sum(c.K[l] * c.K[l + 1] * c.D[l] for c in w.chains for l in range(c.L - 1)))

    print(f"[bench] {prec}/{args.engine}: warmup {args.warmup}, timed {args.steps} steps",
          file=sys.stderr, flush=True)
    from paper_1806_08593_amd import tmc as T
    main_run = run_mode(w, prec, args.engine, args.steps, args.warmup, timing=True,
                        tune=not args.no_tune,
                        flags=T.TMC_FLAG_PERSISTENT if args.persistent else 0,
                        graph=not args.no_graph)
    ms_per_step = main_run["ms_per_step"]
    value = entries / (ms_per_step / 1e3)
    kc = main_run["kernels"]
    dom = max((k for k in kc if k != "other"), key=lambda k: kc[k]["ms_per_step"])
    alg = algorithmic(dom, entries, d_weighted, prec)
    roofline = None
    if alg is not None:
        amount, unit, bound, peak = alg
        per_launch = amount / kc[dom]["launches_per_step"]
        achieved = per_launch / (kc[dom]["avg_launch_us"] * 1e-6) / (1e12 if unit == "TFLOP/s" else 1e9)
        roofline = dict(kernel=dom, bound=bound, achieved=round(achieved, 3), peak=peak, unit=unit,
                        frac=round(achieved / peak, 4), traffic=None,
                        algorithmic_per_launch=per_launch,
                        avg_launch_us=round(kc[dom]["avg_launch_us"], 3))
        # the form (workgroup width) the plan used for that kernel class (every layer of
        # the homogeneous workloads the record covers is eligible for the wide form)
        info = main_run["info"]
        waves = 8 if info.get("wide_fwd" if dom == "fused_fwd" else "wide_bwd") else 4
        rec = recorded_traffic(dom, args.workload, prec, waves)
        if rec is not None:
            # HBM bytes per launch (read + written), from the committed counter record
            roofline["traffic"] = rec[0] + rec[1]
            roofline["traffic_read"], roofline["traffic_written"] = rec
            roofline["traffic_unit"] = "bytes per launch"
            roofline["traffic_source"] = os.path.relpath(TRAFFIC_RECORD, ROOT)
            roofline["waves"] = waves

    # comparators: the other arithmetic modes of the same step
    compare = {}
    if not args.no_compare and prec != "fp64":
        for cp, ce in (("fp32", "fused"), ("fp32", "plain")):
            if (cp, ce) == (prec, args.engine):
                continue
            try:
                print(f"[bench] comparator {cp}/{ce}", file=sys.stderr, flush=True)
                r = run_mode(w, cp, ce, max(3, args.steps // 3), 2, timing=False,
                             tune=not args.no_tune and ce == "fused", graph=not args.no_graph)
                compare[f"{cp}_{ce}"] = dict(ms_per_step=r["ms_per_step"],
                                             value=entries / (r["ms_per_step"] / 1e3), logp=r["logp"])
            except Exception as e:   # e.g. a plain-engine workspace that does not fit
                compare[f"{cp}_{ce}"] = dict(error=str(e)[:200])

    # errors against the FP64 oracle on the CPU-baseline sample, and the baseline itself
    cpu = None
    errs = {}
    if not args.no_cpu_baseline:
        npdt = np.float64 if prec == "fp64" else np.float32
        sample = [cast_chain(c, npdt) for c in w.chains]
        print(f"[bench] CPU oracle baseline (~{args.cpu_budget:.0f} s) ...", file=sys.stderr, flush=True)
        rate, done, dt, refs = cpu_baseline(sample, args.cpu_budget)
        errs[prec] = float(max(abs(main_run["logp"][b] - refs[b]) for b in range(done)))
        for k, v in compare.items():
            if "logp" in v:
                errs[k] = float(max(abs(v["logp"][b] - refs[b]) for b in range(done)))
        cpu = dict(value=rate, unit="factor entries/s", cores=1, kind="oracle",
                   sample=f"forward+backward of the first {done} of {len(w.chains)} instances "
                          f"({sum(c.entries() for c in w.chains[:done])} entries) in {dt:.1f} s, "
                          f"FP64 NumPy, one thread")
    for v in compare.values():
        v.pop("logp", None)
    if compare:
        base = compare.get("fp32_plain", {}).get("ms_per_step")
        if base:
            compare["speedup_over_fp32_plain"] = base / ms_per_step

    info = main_run["info"]
    cfg = {"workload": args.workload, "chains": len(w.chains), "factor_entries": entries,
           "precision": prec, "engine": ["auto", "fused", "plain"][info["engine"]],
           "launch": ("persistent" if info["persistent"] else "per-depth") +
                     (" (tuned)" if info["tuned"] else "") +
                     ("" if info["persistent"] else
                      f", forward {8 if info['wide_fwd'] else 4} / backward "
                      f"{8 if info['wide_bwd'] else 4} waves where eligible") +
                     (", eager" if args.no_graph else ", graph replay"),
           "parallelism": "single GPU"}
    if w.z is not None:
        B, L, K, D = w.z.shape
        cfg.update(B=B, L=L, K=K, D=D)
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
        "config": cfg,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "max_abs_err_logp_vs_oracle": errs,
        "event_ms_per_step": main_run["event_ms_per_step"],
        "eager_ms_per_step": main_run["eager_ms_per_step"],
        "kernels": kc,
        "compare": compare,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
