#!/usr/bin/env python
"""Throughput of the TMC chain estimator on one MI355X.

One step = one forward + backward pass of the Gaussian-chain estimator over one batch
of synthetic inputs already resident in device memory: the pairwise factors on
MFMA, the top-down log-sum-exp messages, the FP64 log-normaliser, the pairwise
marginals and the gradients with respect to z, mu, s and u.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c5]
                    [--precision bf16x3|fp32|fp64] [--engine auto|fused|plain]
                    [--no-compare] [--no-cpu-baseline] [--calibrate-copy MB]

Prints one JSON line.  The default workload is the large-K chain (B=32, L=8, K=2048,
D=128, BF16X3 factor products): the largest configuration, on one GPU.  `value` is
factor entries per second (a step processes the sum over chains and adjacent layer
pairs of K_l * K_{l+1} entries); the timed steps replay the forward and backward graphs
captured from the library's launches (--no-graph: eager launches).  `roofline`
describes the kernel class with the largest device time in a second region of eager
steps, timed with HIP events that the library records around each of its launches on
the stream it launches on.  `compare` times the same step in the FP32 forms (fused, and
plain with stored factors, whose log-sum-exp passes stream more than a gigabyte of
factors: their HBM rates are reported), and the mixed-precision configuration
(B=256, L=6, K=256, D=100); every form's log P is compared with the FP64 oracle on
every instance.  `cpu_baseline` times the FP64 oracle, as it is, on a bounded sample of
the workload across the host's cores.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
LOGP_TOL = {"fp64": None, "fp32": 1e-4, "bf16x3": 2e-3}   # absolute, per instance
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
def traffic_record_path(workload, prec):
    return os.path.join(ROOT, "profiles", f"fused_{workload}_{prec}_pmc.md")


def kernel_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1806_08593_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_counters(kernel, workload, prec, waves=4):
    """Counter record of `kernel` in its `waves`-wave form from the committed profile
    summary of this workload and precision: dict with read/written bytes per launch (and
    the BF16 MFMA ops per launch when recorded), or None when there is none or the
    kernel sources changed since it was taken.  The record is a block of lines
        traffic-record sources-sha256 <hex> workload <w> precision <p>
        traffic-record <kernel class> waves <n> read-bytes <r> written-bytes <w>
        mfma-record <kernel class> waves <n> mops-bf16 <m>
    (FETCH_SIZE and WRITE_SIZE scaled by the copy calibration; SQ_INSTS_VALU_MFMA_MOPS_BF16,
    units of 512 flops)."""
    path = traffic_record_path(workload, prec)
    try:
        lines = open(path).read().splitlines()
    except OSError:
        return None
    head, rows, mops = None, {}, {}
    for ln in lines:
        t = ln.split()
        if len(t) >= 7 and t[0] == "traffic-record" and t[1] == "sources-sha256":
            head = dict(sha=t[2], workload=t[4], precision=t[6])
        elif len(t) == 8 and t[0] == "traffic-record" and t[2] == "waves":
            rows[(t[1], int(t[3]))] = (float(t[5]), float(t[7]))
        elif len(t) == 6 and t[0] == "mfma-record" and t[2] == "waves":
            mops[(t[1], int(t[3]))] = float(t[5])
    if head is None or head["workload"] != workload or head["precision"] != prec:
        return None
    if head["sha"] != kernel_sources_sha256():
        return None
    if (kernel, waves) not in rows:
        return None
    r, wr = rows[(kernel, waves)]
    out = dict(read=r, written=wr, source=os.path.relpath(path, ROOT))
    if (kernel, waves) in mops:
        out["mops_bf16"] = mops[(kernel, waves)]
    return out


def upload(w, prec, engine, flags=0, exponent=1.0, s_override=None):
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
        prob = T.homogeneous_problem(B, L, K, D, prec, engine, flags, exponent=exponent)
        arrs = {k: getattr(w, k) for k in ("z", "mu", "s", "u")}
        if s_override is not None:
            arrs["s"] = s_override
    else:
        shapes, arrs = pack(w.chains, npdt)
        prob, _ = T.ragged_problem(shapes, prec, engine, flags)
    dev = {k: torch.tensor(np.ascontiguousarray(v), dtype=tdt, device="cuda:0") for k, v in arrs.items()}
    return prob, dev


def run_mode(w, prec, engine, steps, warmup, timing, tune=False, flags=0, graph=True, exponent=1.0,
             s_override=None):
    """Times `steps` steps of workload w after `warmup` eager steps, all on one stream.
    graph: the step is a replay of the forward and backward graphs captured from the
    library's own launches (the same kernels; no host launch gaps).  timing: afterwards,
    a second region of eager steps with the library's per-kernel HIP events, for the
    kernel breakdown.  Also returns the device-memory high-water mark of the run (inputs,
    gradients, log P and the workspace; torch's allocator statistics, reset first)."""
    import torch
    from paper_1806_08593_amd import tmc as T
    torch.cuda.empty_cache()
    torch.cuda.reset_peak_memory_stats()
    prob, d = upload(w, prec, engine, flags, exponent, s_override)
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

        fwd_only = bool(flags & T.TMC_FLAG_FORWARD_ONLY)

        def eager():
            T.tmc_gauss_fwd(h, d["z"], d["mu"], d["s"], d["u"], logp, ws, st)
            if not fwd_only:
                T.tmc_gauss_bwd(h, d["z"], d["mu"], d["s"], d["u"], dlogp, ws, g["z"], g["mu"],
                                g["s"], g["u"], st)

        for _ in range(warmup):
            eager()
        st.synchronize()
        T.tmc_plan_check(h)
        step = eager
        if graph:
            T.tmc_plan_graph_capture_gauss(h, 0, d["z"], d["mu"], d["s"], d["u"], logp, None, ws,
                                           None, None, None, None, st)
            if not fwd_only:
                T.tmc_plan_graph_capture_gauss(h, 1, d["z"], d["mu"], d["s"], d["u"], None, dlogp,
                                               ws, g["z"], g["mu"], g["s"], g["u"], st)

            def step():
                T.tmc_plan_graph_launch(h, 0, st)
                if not fwd_only:
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
                   eager_ms_per_step=eager_ms, kernels=kc, logp=lp, info=T.tmc_plan_info_get(h),
                   mem_high_water_bytes=int(torch.cuda.max_memory_allocated()),
                   workspace_bytes=int(plan.workspace_bytes),
                   input_bytes=int(sum(v.numel() * v.element_size() for v in d.values())))
    plan.close()
    del d, g, ws
    torch.cuda.empty_cache()
    return out


# Star model: vector-ALU instructions per factor entry of the message pass: per
# dimension a difference, a product and a fused multiply-add (3 D), then the running max,
# the exponent's argument (one FMA), the exponential and the accumulation -> 3 D + 4 (the
# count of the compiled inner loop at D = 1: 56 instructions per 8 entries).  Peak: one
# wave64 instruction per SIMD every 4 cycles (16 lanes per cycle; the kernels are built
# without packed FP32), 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3 T lane-instructions/s;
# the exponential is counted as one issue (a quarter-rate exponential would put the
# measured N = 128, K = 2048 message kernel above this peak).
VALU_LANE_OPS_PEAK = 256 * 4 * 16 * 2.4e9 / 1e12   # T lane-instructions/s


def star_ops_per_entry(D):
    return 3 * D + 4


def run_star(w, prec, steps, warmup):
    """Times `steps` forward + backward steps of star workload w (inputs resident), then
    a region of steps with the library's per-kernel HIP events."""
    import numpy as np
    import torch
    from paper_1806_08593_amd import tmc as T
    sh = w.shape
    tdt = torch.float64 if prec == "fp64" else torch.float32
    plan = T.Plan(T.StarProblem(sh["S"], sh["N"], sh["Kt"], sh["K"], sh["D"], prec))
    ws = plan.new_workspace()
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        d = {k: torch.tensor(np.ascontiguousarray(getattr(w, k)), dtype=tdt, device="cuda:0")
             for k in ("mth", "s", "z", "u", "uth")}
        g = {k: torch.empty_like(v) for k, v in d.items()}
        logp = torch.empty(sh["S"], dtype=torch.float64, device="cuda:0")
        dlogp = torch.ones(sh["S"], dtype=torch.float64, device="cuda:0")
        h = plan.handle

        def step():
            T.tmc_star_gauss_fwd(h, d["mth"], d["s"], d["z"], d["u"], d["uth"], logp, ws, st)
            T.tmc_star_gauss_bwd(h, d["mth"], d["s"], d["z"], d["u"], dlogp, ws, g["mth"], g["s"],
                                 g["z"], g["u"], g["uth"], st)

        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        T.tmc_plan_check(h)
        T.tmc_plan_set_timing(h, True)
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        kc = {}
        for i, name in enumerate(T.KERNEL_CLASSES):
            tms, cnt = T.tmc_plan_timing(h, i)
            if cnt:
                kc[name] = dict(ms_per_step=tms / steps, launches_per_step=cnt / steps,
                                avg_launch_us=1e3 * tms / cnt)
        T.tmc_plan_set_timing(h, False)
        lp = logp.cpu().numpy()
    plan.close()
    ent = w.entries()
    out = dict(workload=w.name, shape=sh, precision=prec, ms_per_step=ms,
               value=ent / (ms / 1e3), unit="factor entries/s (fwd+bwd)", kernels=kc, logp=lp)
    if "star_msg" in kc:
        per_launch = ent * star_ops_per_entry(sh["D"]) / kc["star_msg"]["launches_per_step"]
        ach = per_launch / (kc["star_msg"]["avg_launch_us"] * 1e-6) / 1e12
        out["roofline"] = dict(kernel="star_msg", bound="alu", achieved=round(ach, 3),
                               peak=round(VALU_LANE_OPS_PEAK, 2), unit="T lane-instructions/s",
                               frac=round(ach / VALU_LANE_OPS_PEAK, 4),
                               ops_per_entry=star_ops_per_entry(sh["D"]),
                               avg_launch_us=round(kc["star_msg"]["avg_launch_us"], 3))
    return out


def host_cores():
    """Host threads the CPU legs use: the process's CPU affinity, at most 16 (the host
    share of one GPU on the benchmark machines)."""
    return max(1, min(16, len(os.sched_getaffinity(0))))


def oracle_logps(chains):
    """FP64 oracle log P of every chain (matrix-product factor form, pinned against the
    direct difference in the oracle's tests), threaded over chains."""
    import concurrent.futures as cf
    from oracle import tmc_oracle as O

    def one(c):
        f = [O.gauss_pair_logfactor_expanded(c.z[l], c.mu[l], c.s[l]) for l in range(len(c.mu))]
        return O.chain_logp(f, c.u)

    with cf.ThreadPoolExecutor(host_cores()) as ex:
        return list(ex.map(one, chains))


def cpu_baseline(chains, budget_s):
    """The FP64 oracle as it stands (direct-difference factors, forward + backward:
    gauss_chain_grads) on a bounded sample of the workload, spread over the host's
    cores (one chain per thread at a time, BLAS pinned to one thread per caller).  A
    sample unit is a whole chain, or, for chains of more than 8M factor entries (one such
    chain alone takes minutes), its first layer pair as a two-layer chain (the same
    per-entry work).  Units are started until budget_s has passed (at least one).
    Returns (entries/s, threads, description)."""
    import threading
    import concurrent.futures as cf
    from oracle import tmc_oracle as O
    from threadpoolctl import threadpool_limits
    from workloads import Chain

    big = max(c.entries() for c in chains) > 8_000_000
    units = [Chain(z=c.z[:2], mu=c.mu[:1], s=c.s[:1], u=c.u[:2]) if big else c for c in chains]
    n_thr = host_cores()
    lock = threading.Lock()
    state = dict(next=0, done=0, entries=0)
    t0 = time.perf_counter()

    def worker():
        while True:
            with lock:
                k = state["next"]
                if k >= len(units) or (k > 0 and time.perf_counter() - t0 > budget_s):
                    return
                state["next"] += 1
            c = units[k]
            O.gauss_chain_grads(c.z, c.mu, c.s, c.u)
            with lock:
                state["done"] += 1
                state["entries"] += c.entries()

    with threadpool_limits(limits=1):
        with cf.ThreadPoolExecutor(n_thr) as ex:
            for f in [ex.submit(worker) for _ in range(n_thr)]:
                f.result()
    dt = time.perf_counter() - t0
    what = ("the first layer pair (as a two-layer chain) of each of" if big else "whole chains:")
    desc = (f"FP64 oracle forward+backward (direct-difference factors) of {what} "
            f"{state['done']} instances ({state['entries']} factor entries) in {dt:.1f} s "
            f"on {n_thr} threads, one chain per thread")
    return state["entries"] / dt, n_thr, desc


def widen_section(args, log, w5):
    """The widened estimators at benchmark shapes: parent-dependent scales (the C3 shapes,
    one log standard deviation per parent sample, plain engine) and the DReGs surrogate at C5
    (a kappa = 1 forward-only pass plus a kappa = 2 forward and backward)."""
    import numpy as np
    from paper_1806_08593_amd import tmc as T
    from workloads import make
    out = {}
    try:
        log("parent-dependent scales, C3 shapes, FP32 plain")
        w3 = make("c3")
        B, L, K, D = w3.z.shape
        rng = np.random.default_rng(1806)
        sp = (np.asarray(w3.s)[None, :, None, :] + 0.2 * rng.normal(size=(B, L - 1, K, D))).astype(np.float32)
        r = run_mode(w3, "fp32", "plain", max(3, args.steps // 3), 2, timing=True,
                     flags=T.TMC_FLAG_PARENT_SCALE, s_override=sp)
        e = dict(workload="c3 shapes, s per parent sample", precision="fp32", engine="plain",
                 ms_per_step=r["ms_per_step"], value=w3.entries() / (r["ms_per_step"] / 1e3),
                 kernels={k: round(v["avg_launch_us"], 2) for k, v in r["kernels"].items()})
        for kk, nbytes in (("plain_lse_fwd", 4), ("plain_lse_bwd", 8)):
            if kk in r["kernels"]:
                per = nbytes * w3.entries() / r["kernels"][kk]["launches_per_step"]
                e[kk + "_gbs"] = round(per / (r["kernels"][kk]["avg_launch_us"] * 1e-6) / 1e9, 1)
        out["parent_scale"] = e
    except Exception as ex:
        out["parent_scale"] = dict(error=str(ex)[:200])
    try:
        log("DReGs surrogate passes at C5, BF16X3")
        steps = max(3, args.steps // 3)
        r1 = run_mode(w5, "bf16x3", "fused", steps, 2, timing=False, tune=not args.no_tune,
                      flags=T.TMC_FLAG_FORWARD_ONLY, graph=not args.no_graph)
        r2 = run_mode(w5, "bf16x3", "fused", steps, 2, timing=False, tune=not args.no_tune,
                      exponent=2.0, graph=not args.no_graph)
        # (the forward-only run times a forward; a step of the surrogate is that forward plus a
        # squared-weight forward and backward)
        ms = r1["ms_per_step"] + r2["ms_per_step"]
        out["dregs"] = dict(workload="c5", precision="bf16x3", ms_forward_kappa1=r1["ms_per_step"],
                            ms_fwd_bwd_kappa2=r2["ms_per_step"], ms_per_step=ms,
                            value=w5.entries() / (ms / 1e3))
    except Exception as ex:
        out["dregs"] = dict(error=str(ex)[:200])
    return out


def logmm_section(args, log):
    """The log-domain matrix product on a batch of square matrices, every precision;
    achieved = 2 M N K flops per product / call time (BF16X3 issues 3x that on the
    matrix cores), against the dense matrix-core peak of the operand type."""
    import numpy as np
    import torch
    from paper_1806_08593_amd import tmc as T
    from oracle import tmc_oracle as O
    out = {}
    B, M, K, N = 8, 1024, 1024, 1024
    rng = np.random.default_rng(1806)
    Xh = (rng.normal(size=(B, M, K)) * 3).astype(np.float32)
    Yh = (rng.normal(size=(B, K, N)) * 3).astype(np.float32)
    for prec, peak in (("bf16x3", MFMA_PEAK["bf16x3"]), ("fp32", MFMA_PEAK["fp32"]), ("fp64", MFMA_PEAK["fp64"])):
        try:
            log(f"log-domain product {prec}")
            dt = torch.float64 if prec == "fp64" else torch.float32
            X = torch.tensor(Xh, dtype=dt, device="cuda:0")
            Y = torch.tensor(Yh, dtype=dt, device="cuda:0")
            Z = torch.empty((B, M, N), dtype=dt, device="cuda:0")
            nb = T.tmc_logmmexp_workspace_size(B, M, K, N, prec)
            ws = torch.empty(max(nb, 256) + 256, dtype=torch.uint8, device="cuda:0")
            wp = ws.data_ptr() + (-ws.data_ptr()) % 256
            reps = 3 if prec == "fp64" else 10
            T.tmc_logmmexp(B, M, K, N, prec, X, Y, Z, wp)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                T.tmc_logmmexp(B, M, K, N, prec, X, Y, Z, wp)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            tf = 2.0 * B * M * N * K / (ms * 1e-3) / 1e12
            r = dict(batch=B, M=M, K=K, N=N, ms=ms, tflops=round(tf, 3), peak=peak,
                     frac=round(tf / peak, 4))
            if not args.no_oracle:
                z = Z[0, :64, :64].cpu().numpy().astype(np.float64)
                ref = O.logmmexp(Xh[0, :64].astype(np.float64), Yh[0, :, :64].astype(np.float64))
                r["max_abs_err_first_64x64"] = float(np.max(np.abs(z - ref)))
            out[prec] = r
            del X, Y, Z, ws
        except Exception as ex:
            out[prec] = dict(error=str(ex)[:200])
    return out


def star_section(args, log):
    import numpy as np
    from workloads import make_star
    star = {}
    for name in ("s1", "s2"):
        try:
            log(f"star workload {name}")
            w = make_star(name)
            r = run_star(w, "fp32", max(5, args.steps // 2), 3)
            if name == "s1" and not args.no_oracle:
                from oracle import tmc_oracle as O
                c = lambda a: np.asarray(a, np.float32).astype(np.float64)
                N = w.shape["N"]
                f = [O.gauss_pair_logfactor(c(w.mth[0]), c(w.z[0, n]), c(w.s[0])) for n in range(N)]
                ref = O.star_logp(c(w.uth[0]), f, [c(w.u[0, n]) for n in range(N)])
                r["max_abs_err_logp"] = float(abs(r["logp"][0] - ref))
                r["abs_logp"] = float(abs(ref))
            r.pop("logp")
            star[name] = r
        except Exception as ex:
            star[name] = dict(error=str(ex)[:200])
    return star


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c5")
    ap.add_argument("--precision", default=None)
    ap.add_argument("--engine", default="auto")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true")
    ap.add_argument("--no-oracle", action="store_true", help="skip the log P errors against the oracle")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the launch-shape tuner (per-depth launches unless --persistent)")
    ap.add_argument("--persistent", action="store_true", help="persistent launches (with --no-tune)")
    ap.add_argument("--no-graph", action="store_true",
                    help="time eager launches instead of replays of the captured step graphs")
    ap.add_argument("--no-star", action="store_true",
                    help="skip the star-model measurement (Gaussian example, FP32)")
    ap.add_argument("--no-peaks", action="store_true",
                    help="skip the measured machine peaks (HBM, MFMA, vector ALU, LDS probes)")
    ap.add_argument("--no-widen", action="store_true",
                    help="skip the parent-scale and DReGs-surrogate measurements")
    ap.add_argument("--no-logmm", action="store_true",
                    help="skip the log-domain matrix product measurement")
    ap.add_argument("--star-only", action="store_true",
                    help="only the star-model and log-domain product measurements (one JSON line)")
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

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    if args.star_only:
        print(json.dumps({"star": {} if args.no_star else star_section(args, log),
                          "logmm": {} if args.no_logmm else logmm_section(args, log)}))
        return

    prec = args.precision or ("fp64" if args.workload == "c1" else "bf16x3")
    log(f"generating workload {args.workload} ...")
    w = make(args.workload)

    def d_weighted(wl):
        return float(sum(c.K[l] * c.K[l + 1] * c.D[l] for c in wl.chains for l in range(c.L - 1)))

    entries = w.entries()
    log(f"{prec}/{args.engine}: warmup {args.warmup}, timed {args.steps} steps")
    from paper_1806_08593_amd import tmc as T
    main_run = run_mode(w, prec, args.engine, args.steps, args.warmup, timing=True,
                        tune=not args.no_tune,
                        flags=T.TMC_FLAG_PERSISTENT if args.persistent else 0,
                        graph=not args.no_graph)
    ms_per_step = main_run["ms_per_step"]
    value = entries / (ms_per_step / 1e3)
    kc = main_run["kernels"]
    info = main_run["info"]

    def roofline_of(kcs, wl, pr, inf, dom):
        alg = algorithmic(dom, wl.entries(), d_weighted(wl), pr)
        if alg is None:
            return None
        amount, unit, bound, peak = alg
        per_launch = amount / kcs[dom]["launches_per_step"]
        achieved = per_launch / (kcs[dom]["avg_launch_us"] * 1e-6) / (1e12 if unit == "TFLOP/s" else 1e9)
        r = dict(kernel=dom, bound=bound, achieved=round(achieved, 3), peak=peak, unit=unit,
                 frac=round(achieved / peak, 4), traffic=None, algorithmic_per_launch=per_launch,
                 avg_launch_us=round(kcs[dom]["avg_launch_us"], 3))
        if dom in ("fused_fwd", "fused_bwd"):
            # the form (workgroup width) the plan used for that kernel class (every layer of
            # the homogeneous workloads the record covers is eligible for the wide form)
            waves = 8 if inf.get("wide_fwd" if dom == "fused_fwd" else "wide_bwd") else 4
            rec = recorded_counters(dom, wl.name, pr, waves)
            if rec is not None:
                # HBM bytes per launch (read + written) from the committed counter record
                r["traffic"] = rec["read"] + rec["written"]
                r["traffic_read"], r["traffic_written"] = rec["read"], rec["written"]
                r["traffic_unit"] = "bytes per launch"
                r["traffic_source"] = rec["source"]
                r["waves"] = waves
                if "mops_bf16" in rec and pr == "bf16x3":
                    # issued matrix-core work (hi/lo products, padding included) per launch
                    issued = rec["mops_bf16"] * 512.0 / (kcs[dom]["avg_launch_us"] * 1e-6) / 1e12
                    r["issued_tflops"] = round(issued, 3)
                    r["issued_frac"] = round(issued / peak, 4)
        return r

    dom = max((k for k in kc if k != "other"), key=lambda k: kc[k]["ms_per_step"])
    roofline = roofline_of(kc, w, prec, info, dom)
    # the other kernel classes of the step, same measure
    kernel_roofline = {k: roofline_of(kc, w, prec, info, k) for k in kc if k not in ("other", dom)}

    # comparators: the FP32 forms of the same step, and the mixed-precision configuration
    compare = {}
    runs = {}
    if not args.no_compare and prec != "fp64":
        cands = [("fp32_fused", w, "fp32", "fused", 0), ("fp32_plain", w, "fp32", "plain", 0)]
        if args.workload != "c3":
            wc3 = make("c3")
            cands += [("c3_bf16x3", wc3, "bf16x3", "auto", 0), ("c3_fp32_fused", wc3, "fp32", "fused", 0),
                      ("c3_fp32_plain", wc3, "fp32", "plain", 0)]
        if args.workload != "c4":
            # the ragged batch in its configuration's precision: tuned per-depth launches and
            # persistent launches over the chain queue
            wc4 = make("c4")
            cands += [("c4_fp32_fused", wc4, "fp32", "fused", 0),
                      ("c4_fp32_persistent", wc4, "fp32", "fused", T.TMC_FLAG_PERSISTENT)]
        for name, wl, cp, ce, fl in cands:
            if (wl is w) and (cp, ce) == (prec, args.engine):
                continue
            try:
                log(f"comparator {name}")
                r = run_mode(wl, cp, ce, max(3, args.steps // 3), 2, timing=True,
                             tune=not args.no_tune and ce != "plain" and not fl, flags=fl,
                             graph=not args.no_graph)
                ent = wl.entries()
                e = dict(workload=wl.name, precision=cp, engine=ce, ms_per_step=r["ms_per_step"],
                         value=ent / (r["ms_per_step"] / 1e3),
                         mem_high_water_bytes=r["mem_high_water_bytes"],
                         launch="persistent" if r["info"]["persistent"] else "per-depth")
                # HBM rate of the plain engine's log-sum-exp passes over the stored factors
                for kk in ("plain_lse_fwd", "plain_lse_bwd"):
                    if kk in r["kernels"]:
                        rf = roofline_of(r["kernels"], wl, cp, r["info"], kk)
                        e[kk] = dict(achieved_gbs=rf["achieved"], frac=rf["frac"],
                                     avg_launch_us=rf["avg_launch_us"],
                                     bytes_per_launch=rf["algorithmic_per_launch"])
                compare[name] = e
                runs[name] = (wl, r["logp"])
            except Exception as ex:   # e.g. a plain-engine workspace that does not fit
                compare[name] = dict(error=str(ex)[:200])

    # log P errors against the FP64 oracle on every instance
    errs = {}
    if not args.no_oracle:
        npdt = np.float64 if prec == "fp64" else np.float32
        refs_by = {}

        def refs_for(wl):
            if wl.name not in refs_by:
                log(f"oracle log P of every {wl.name} instance ...")
                refs_by[wl.name] = np.array(oracle_logps([cast_chain(c, npdt) for c in wl.chains]))
            return refs_by[wl.name]

        errs[prec] = float(np.max(np.abs(main_run["logp"] - refs_for(w))))
        for name, (wl, lp) in runs.items():
            errs[name] = float(np.max(np.abs(lp - refs_for(wl))))
            compare[name]["max_abs_err_logp"] = errs[name]
            tol = LOGP_TOL[compare[name]["precision"]]
            compare[name]["within_tolerance"] = tol is not None and errs[name] <= tol

    # the star model (global latent shared by N local latents): both Gaussian-example
    # workloads in FP32; log P of the first against the oracle
    star = {} if args.no_star else star_section(args, log)
    logmm = {} if args.no_logmm else logmm_section(args, log)
    widen = {} if (args.no_widen or args.workload != "c5") else widen_section(args, log, w)

    # the machine's measured peaks next to the datasheet ones the roofline uses
    peaks = {}
    if not args.no_peaks:
        log("measured machine peaks")
        from paper_1806_08593_amd import peaks as PK
        try:
            peaks = PK.measure()
        except Exception as ex:
            peaks = dict(error=str(ex)[:200])

        def attach(rf, pr):
            # measured counterpart of the roofline's peak: MFMA of the kernel's precision,
            # HBM copy, or (vector-ALU bound) the FMA rate in lane instructions per second
            if not rf or "error" in peaks:
                return
            k = {"mfma": "mfma_bf16" if pr == "bf16x3" else "mfma_fp32", "hbm": "hbm_copy",
                 "alu": "valu_fma_fp32"}.get(rf.get("bound"))
            if k is None or k not in peaks:
                return
            pm = peaks[k]["value"] / (2.0 if rf["bound"] == "alu" else 1.0)
            rf["peak_measured"] = round(pm, 2)
            rf["frac_of_measured"] = round(rf["achieved"] / pm, 4)
            if "issued_tflops" in rf:
                rf["issued_frac_of_measured"] = round(rf["issued_tflops"] / pm, 4)

        for rf in [roofline] + list(kernel_roofline.values()):
            attach(rf, prec)
        for v in star.values():
            if isinstance(v, dict):
                attach(v.get("roofline"), v.get("precision", "fp32"))
        for pr, v in logmm.items():
            k = {"bf16x3": "mfma_bf16", "fp32": "mfma_fp32", "fp64": "mfma_fp64"}.get(pr)
            if isinstance(v, dict) and "tflops" in v and k in peaks:
                v["peak_measured"] = peaks[k]["value"]
                v["frac_of_measured"] = round(v["tflops"] / peaks[k]["value"], 4)

    cpu = None
    if not args.no_cpu_baseline:
        npdt = np.float64 if prec == "fp64" else np.float32
        log(f"CPU oracle baseline (~{args.cpu_budget:.0f} s) ...")
        rate, n_thr, desc = cpu_baseline([cast_chain(c, npdt) for c in w.chains], args.cpu_budget)
        cpu = dict(value=rate, unit="factor entries/s", cores=n_thr, kind="oracle", sample=desc,
                   host_cpus_visible=os.cpu_count())

    # speedups, each with both sides' errors and the tolerance band both meet
    if compare and prec in LOGP_TOL and LOGP_TOL[prec]:
        def band(e1, p1, e2, p2):
            b = [t for t in sorted({LOGP_TOL[p1], LOGP_TOL[p2]}) if e1 <= t and e2 <= t]
            return b[0] if b else None

        sp = {}
        for name in ("fp32_plain", "fp32_fused"):
            c = compare.get(name, {})
            if "ms_per_step" in c:
                ent = dict(speedup=c["ms_per_step"] / ms_per_step,
                           err=errs.get(prec), other_err=c.get("max_abs_err_logp"))
                if ent["err"] is not None and ent["other_err"] is not None:
                    ent["band_both_meet"] = band(ent["err"], prec, ent["other_err"], "fp32")
                sp[f"{prec}_over_{name}"] = ent
        a, b = compare.get("fp32_fused", {}), compare.get("fp32_plain", {})
        if "ms_per_step" in a and "ms_per_step" in b:
            ent = dict(speedup=b["ms_per_step"] / a["ms_per_step"], err=a.get("max_abs_err_logp"),
                       other_err=b.get("max_abs_err_logp"))
            if ent["err"] is not None and ent["other_err"] is not None:
                ent["band_both_meet"] = band(ent["err"], "fp32", ent["other_err"], "fp32")
            sp["fp32_fused_over_fp32_plain"] = ent
        compare["speedups"] = sp

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
        "memory": dict(high_water_bytes=main_run["mem_high_water_bytes"],
                       workspace_bytes=main_run["workspace_bytes"],
                       input_bytes=main_run["input_bytes"],
                       stored_factor_bytes_avoided=4 * entries),
        "event_ms_per_step": main_run["event_ms_per_step"],
        "eager_ms_per_step": main_run["eager_ms_per_step"],
        "kernels": kc,
        "kernel_roofline": kernel_roofline,
        "compare": compare,
        "star": star,
        "logmm": logmm,
        "widen": widen,
        "measured_peaks": peaks,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
