#!/usr/bin/env python3
"""Throughput of the ptychographic forward + adjoint on one MI355X.

Workload (config 1 of the synthetic suite): a 1024 x 1024 complex object, four
orthogonal Hermite-Gauss probe modes of 128 x 128, 2000 positions on a Fermat spiral
with sub-pixel offsets, Poisson loss, gradients of the object, the probe and the
positions. One step = one forward + adjoint pass over all 2000 patterns with inputs
resident in HBM. The fused kernel is timed; the per-step form is timed beside it.

Prints one JSON line. `value` is patterns/s of the fused form.

`--workload` measures one of the other synthetic workloads the same way (one JSON line
each): c1m0 (config 1 with mode 0 only), c0, c2, c3, c5 (30 probe modes, the paper's
benchmark shape) and c4 (32 uneven datasets in one batched, graph-captured launch).
The default (config 1) is the headline measurement.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0           # MI355X HBM3E, GB/s
FP32_VECTOR_PEAK_TFLOPS = 157.3  # MI355X FP32 vector (published)

KERNEL_SOURCES = [
    "paper_2510_20929_amd/csrc/kernels/fused_small.hip",
    "paper_2510_20929_amd/csrc/kernels/small_body.hpp",
    "paper_2510_20929_amd/csrc/kernels/lds_body.hpp",
    "paper_2510_20929_amd/csrc/kernels/lds_ms.hpp",
    "paper_2510_20929_amd/csrc/device/fft.hpp",
    "paper_2510_20929_amd/csrc/device/model.hpp",
    "paper_2510_20929_amd/csrc/device/common.hpp",
]


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def fft_flops(N: int) -> float:
    """Conventional flop count of one N x N complex FFT: 5 N^2 log2(N^2)."""
    return 5.0 * N * N * math.log2(N * N)


def algorithmic(prob):
    """Per-pattern algorithmic FFT flops and HBM bytes of one forward + adjoint pass:
    2 FFTs per mode (and 2 per propagation and slice); bytes = measured pattern (4 N^2)
    + position in/out (16) + one read and one write of object and probe amortised."""
    N, M, S, K = prob.N, prob.M, prob.S, prob.K
    ffts = M * (2 + 4 * (S - 1))
    flops = ffts * fft_flops(N)
    obj_bytes = 2 * prob.S * prob.H * prob.W * 8
    probe_bytes = 2 * prob.E * M * N * N * 8
    byts = 4 * N * N + 16 + (obj_bytes + probe_bytes) / K
    return flops, byts


def read_traffic(khash: str, kernel: str):
    """HBM bytes per launch of the fused kernel from the committed PMC summary, if it
    was taken on the current kernel sources and the same kernel instance."""
    path = os.path.join(ROOT, "profiles", "fused_c1_traffic.json")
    try:
        with open(path) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != khash or t.get("kernel") != kernel:
        return None
    return t.get("bytes_per_launch")


def copy_bandwidth(torch, dev, nbytes: int = 1 << 30, reps: int = 5) -> float:
    """Achievable HBM bandwidth on this GPU: a device-to-device copy of `nbytes`, timed with
    events on the current stream (median of `reps`); read + written bytes per second, GB/s."""
    x = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    y = torch.empty_like(x)
    y.copy_(x)
    times = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        y.copy_(x)
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    del x, y
    times.sort()
    return 2.0 * nbytes / (times[len(times) // 2] * 1e-3) / 1e9


def cpu_baseline(truth, start, budget_s: float = 10.0, pool_s: float = 8.0):
    """The FP64 oracle (as it stands) on the same workload on the host: forward + adjoint
    over the positions in chunks of 25, cycling through all positions until the time
    budget is spent (whole chunks only). Two legs: one thread in this process, then one
    single-threaded worker process per available core (at most 16), each on its own shard
    of the positions. ``value`` is the all-core rate. The measured intensities come from
    the oracle's own forward model of the truth plus Poisson noise."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import oracle
    from oracle import timing
    from synth import workloads as W

    n = truth.K
    kw = dict(loss=start.loss, eps=start.eps, norm_count=truth.K, grads=("obj", "probe", "pos"))
    with threadpool_limits(limits=1):
        _, I_clean = oracle.forward(truth.obj, truth.probe, truth.positions, np.zeros((n, truth.N, truth.N)),
                                    loss=truth.loss)
        I_meas = W.poisson_counts(I_clean, 4242)
        done, chunk, k0 = 0, 25, 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < budget_s:
            k1 = min(k0 + chunk, n)
            oracle.forward_adjoint(start.obj, start.probe, start.positions[k0:k1], I_meas[k0:k1], **kw)
            done += k1 - k0
            k0 = 0 if k1 == n else k1
        dt = time.perf_counter() - t0
    one = {"value": done / dt, "cores": 1,
           "sample": f"{done} patterns ({done / n:.2f} passes over the {n} positions, chunks of 25), {dt:.1f} s"}
    workers = timing.host_workers()
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = os.cpu_count() or 1
    rate, pdone, wall = timing.pool_rate(start.obj, start.probe, start.positions, I_meas, workers=workers,
                                         budget_s=pool_s, chunk=chunk, **kw)
    print(f"# cpu baseline: {one['value']:.1f} patterns/s on one thread, {rate:.1f} on {workers} processes",
          file=sys.stderr, flush=True)
    return {"value": rate, "unit": "patterns/s", "cores": workers, "kind": "oracle",
            "sample": f"{pdone} patterns of the same workload ({n} positions split into {workers} shards, one "
                      f"single-threaded process each, chunks of 25), FP64 NumPy oracle, {wall:.1f} s wall",
            "single_thread": one,
            "host_cpu": _host_cpu(),
            "affinity_cpus": affinity,
            "pool_cap": f"one worker per CPU this process may run on, at most {timing.HOST_SHARE} (the host CPUs "
                        f"allotted to one GPU on the measuring machine)"}


def _host_cpu() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


WORKLOADS = {
    "c1": "config 1: 1024x1024 complex object, 4 Hermite-Gauss probe modes of 128x128, 2000 Fermat-spiral "
          "positions with sub-pixel offsets, Poisson loss, gradients of object, probe and positions",
    "c1m0": "config 1 with probe mode 0 only (M = 1): 1024x1024 object, 128x128 frames, 2000 positions, "
            "Poisson loss, gradients of object, probe and positions",
    "c0": "config 0: 256x256 object, one 64x64 disk probe, 625 integer raster positions, amplitude loss, "
          "gradients of object and probe",
    "c2": "config 2: 2048x2048 object, 8 orthogonal eigenprobes of 256x256 with per-position weights, "
          "10000 jittered raster positions, amplitude loss, gradients of object, eigenprobes and weights",
    "c3": "config 3: 8 slices of 2048x2048, 2 probe modes of 128x128, 5000 Fermat-spiral positions, "
          "lambda z = 81.92 px^2, amplitude loss, gradients of all slices, probe and positions",
    "c5": "config 5 (mode-heavy): 413x535 object, 30 probe modes of 128x128, 6732 raster positions with "
          "sub-pixel offsets, amplitude loss, gradients of object, probe and positions",
    "c6": "config 6 (the supplement's speed-benchmark shape): 961 positions of 128^2, 15 probe modes, 3 OPR "
          "eigenprobes with per-position weights, 372x372 object, amplitude loss, gradients of object, "
          "eigenprobes and weights",
    "c6n512": "config 6 at 512^2 frames: 961 positions, 15 probe modes, 3 OPR eigenprobes, 1476x1476 object, "
              "amplitude loss, gradients of object, eigenprobes and weights",
    "c4": "config 4: 32 independent datasets (64^2-512^2 frames, 1-4 modes, 200-5000 positions each, "
          "per-position probe amplitudes), one batched persistent launch captured in a hipGraph, amplitude loss, "
          "gradients of objects, probes, positions and weights",
}


def build_workload(name):
    import dataclasses

    from synth import workloads as W
    if name == "c1m0":
        truth = W.make_config(1)
        truth = dataclasses.replace(truth, probe=truth.probe[:, :1].copy())
    elif name == "c6n512":
        truth = W.make_config(6, N=512)
    else:
        truth = W.make_config(int(name[1:]))
    return truth, W.perturb(truth, 21)


def kernel_name(plan, prob, tune):
    info = plan.info()
    loss = 1 if prob.loss == "poisson" else 0
    groups = int((tune or {}).get("mode_groups", 0) or 0)
    if groups > 1 and prob.M > 1:
        # mode-split form: three passes per chunk, timed together
        if prob.N >= 256:
            return "split_big_kernel<%d, %d, 1/2> + split_loss_nat_kernel<%d> (mode groups %d)" % (
                prob.N, info["threads"], loss, groups)
        lds = "_lds" if prob.N == 128 and (tune or {}).get("variant", 0) >= 5 else ""
        return "split_forward/loss/adjoint%s_kernel<%d, %d> (mode groups %d)" % (lds, prob.N, info["threads"], groups)
    if prob.N >= 256:
        return "fused_big_kernel<%d, %d, %d>" % (prob.N, info["threads"], loss)
    if prob.S > 1:
        if prob.N == 128 and (tune or {}).get("variant", 0) >= 5:
            return "fused_small_lds_ms_kernel<%d, %d, %d>" % (prob.N, info["threads"], loss)
        return "fused_small_ms_kernel<%d, %d, %d>" % (prob.N, info["threads"], loss)
    v = (tune or {}).get("variant", 0) if prob.N >= 64 else 0
    if prob.N == 128 and v >= 5:
        # working frame resident in LDS; dl/dI in registers (6) or scratch (5)
        return "fused_small_lds_kernel<%d, %d, %d, %s>" % (prob.N, info["threads"], loss,
                                                            "true" if v == 6 else "false")
    rv = "true" if v in (2, 3, 4) else "false"      # patch in registers
    goreg = "true" if v in (2, 3) else "false"      # patch gradient in registers
    if getattr(prob, "det_lambda_z", None) is not None:
        return "fused_small_near_kernel<%d, %d, %d>" % (prob.N, info["threads"], loss)
    return "fused_small_kernel<%d, %d, %d, %s, %s>" % (prob.N, info["threads"], loss, rv, goreg)


def measured_intensities(truth, dev, torch, t, Plan):
    """The clean far field of the truth (computed by the library) plus Poisson noise."""
    base = Plan.for_problem(truth)
    I_clean = torch.empty((truth.K, truth.N, truth.N), dtype=torch.float32, device=dev)
    w = t(truth.weights) if truth.weights is not None else None
    base.forward(t(truth.obj), t(truth.probe), t(truth.positions), torch.zeros_like(I_clean), weights=w,
                 I_pred=I_clean)
    gen = torch.Generator(device=dev)
    gen.manual_seed(20931)
    I = torch.poisson(I_clean, generator=gen).contiguous()
    del base, I_clean
    return I


def packing_bound(problems, cus):
    """How much of the GPU one call per dataset leaves idle on uneven datasets: with one
    position per workgroup per round, a call of K positions takes ceil(K / cus) rounds.
    Position cost is modelled as modes x N^2 log2 N^2 (the transforms). Returns the
    work-weighted occupancy of the per-call form and the gain a perfect packing of every
    dataset's positions onto the workgroups would give over it (an upper bound for any
    batched schedule)."""
    cost = [p.M * p.N * p.N * math.log2(p.N * p.N) for p in problems]
    work = sum(p.K * c for p, c in zip(problems, cost))
    slots = sum(math.ceil(p.K / cus) * cus * c for p, c in zip(problems, cost))
    return {"per_call_occupancy": work / slots, "perfect_packing_gain": slots / work, "workgroups": cus,
            "cost_model": "positions x modes x N^2 log2 N^2, one position per workgroup per round"}


def run_batched(args, dev, torch, t):
    """Config 4: one batched launch over 32 uneven datasets."""
    from paper_2510_20929_amd import Batch, Plan
    from synth import workloads as W
    truths = W.make_batched_config()
    starts = [W.perturb(p, 3) for p in truths]
    grads = ("obj", "probe", "pos", "weights")
    tensors = []
    for tr, st in zip(truths, starts):
        I = measured_intensities(tr, dev, torch, t, Plan)
        tensors.append((t(st.obj), t(st.probe), t(st.positions), I, t(st.weights)))
    # schedule by the autotuner (parity-gated against one call per dataset, cached)
    from paper_2510_20929_amd import autotune
    if args.tune:
        choice, src = json.loads(args.tune), "fixed"
    else:
        cache = os.environ.get("PTYHIP_TUNE_CACHE") or autotune.DEFAULT_CACHE
        choice, rep = autotune.tune_batch(starts, tensors, grads=grads, cache_path=cache, use_cache=not args.retune)
        src = "cache" if rep.get("cached") else "autotuned"
    per_call_choice = bool(choice.get("per_call"))
    b = Batch(starts, tune=None if per_call_choice else choice)
    outs = [b.bind(i, *ts[:4], weights=ts[4]) for i, ts in enumerate(tensors)]
    for _ in range(args.warmup):
        b.launch(grads, per_call=per_call_choice)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b.launch(grads, per_call=per_call_choice)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    K = sum(p.K for p in truths)
    flops = sum(algorithmic(p)[0] * p.K for p in starts)
    byts = sum(algorithmic(p)[1] * p.K for p in starts)
    b.launch(grads, per_call=True)
    torch.cuda.synchronize()
    tp0 = time.perf_counter()
    for _ in range(max(1, args.plain_steps)):
        b.launch(grads, per_call=True)
    torch.cuda.synchronize()
    per_call_ms = (time.perf_counter() - tp0) * 1e3 / max(1, args.plain_steps)
    ach = flops / (ms * 1e-3) / 1e12
    return {"value": K / (ms * 1e-3), "ms_per_step": ms, "K": K,
            "roofline": {"bound": "alu", "achieved": ach, "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": ach / FP32_VECTOR_PEAK_TFLOPS, "traffic": None,
                         "kernel": "whole batched step (graph replay)", "kernel_ms": ms},
            "hbm": {"alg_GBs": byts / (ms * 1e-3) / 1e9, "frac_of_peak": byts / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS},
            "per_call": {"value": K / (per_call_ms * 1e-3), "ms_per_step": per_call_ms},
            "batched_vs_per_call": per_call_ms / ms, "error_flags": b.get_error(),
            "packing_bound": packing_bound(truths, torch.cuda.get_device_properties(0).multi_processor_count),
            "tune": choice, "tune_source": src,
            "config": {"datasets": len(truths), "positions": K,
                       "frames": sorted({p.N for p in truths}),
                       "form": ("one call per dataset (the autotuner's choice)" if per_call_choice else
                                "batched persistent launches per frame-size class, " +
                                ("concurrent graph branches" if choice.get("variant") == 1 else "one after the other")
                                + ", hipGraph replay")}}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--plain-steps", type=int, default=5)
    ap.add_argument("--workload", default="c1", choices=sorted(WORKLOADS),
                    help="synthetic workload (default: config 1, the headline measurement)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--no-plain", action="store_true", help="skip the per-step form")
    ap.add_argument("--no-autograd", action="store_true", help="skip the autograd form")
    ap.add_argument("--batch", type=int, default=0,
                    help="positions per call (minibatch call shape); 0 = the whole workload in one call")
    ap.add_argument("--graphs", action="store_true",
                    help="replay each distinct call from a captured hipGraph (plan graph cache)")
    ap.add_argument("--tune", default=None,
                    help="fixed implementation choice as JSON (skips the autotuner; used for profiling runs)")
    ap.add_argument("--retune", action="store_true", help="ignore the frozen tune cache and autotune again")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a 1 GiB device copy (counter calibration for the PMC runs)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (it would shard positions "
              "and all-reduce the object and probe gradients)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2510_20929_amd import Plan

    dev = torch.device("cuda:0")
    if args.copy_calibration:
        x = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": x.numel() * 4}))
        return

    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    common = {"metric": "diffraction patterns/s forward+adjoint at 128² frames (fused vs plain), % HBM peak",
              "unit": "patterns/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
              "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic"}

    if args.workload == "c4":
        r = run_batched(args, dev, torch, t)
        cfg = dict(r.pop("config"))
        cfg["workload"] = WORKLOADS["c4"]
        line = dict(common, value=r.pop("value"), ms_per_step=r.pop("ms_per_step"), config=cfg, **r)
        print(json.dumps(line), flush=True)
        return

    truth, start = build_workload(args.workload)
    obj, probe, pos = t(start.obj), t(start.probe), t(start.positions)
    wts = t(start.weights) if start.weights is not None else None
    I_meas = measured_intensities(truth, dev, torch, t, Plan)
    grads = start.grads
    # implementation choice by the autotuner (parity-gated, untimed here)
    from paper_2510_20929_amd import autotune
    shape = dict(N=start.N, M=start.M, E=start.E, S=start.S, H=start.H, W=start.W, loss=start.loss, eps=start.eps,
                 lambda_z=start.lambda_z)
    cache = os.environ.get("PTYHIP_TUNE_CACHE") or autotune.DEFAULT_CACHE
    if args.tune:
        tune, tune_src = json.loads(args.tune), "fixed"
    else:
        Bt = min(args.batch, truth.K) if args.batch > 0 else truth.K
        tune, rep = autotune.tune_plan(shape, obj, probe, pos[:Bt], I_meas[:Bt],
                                       weights=None if wts is None else wts[:Bt], grads=grads, cache_path=cache,
                                       use_cache=not args.retune)
        tune_src = "cache" if rep.get("cached") else "autotuned"
    # call shape: the whole workload in one call, or minibatches of B positions (each call
    # normalised by its own position count, as a minibatch reconstructor calls it); a step
    # is one pass over every position either way
    K_all = truth.K
    B = min(args.batch, K_all) if args.batch > 0 else K_all
    calls = []
    for a in range(0, K_all, B):
        b = min(a + B, K_all)
        calls.append((pos[a:b], I_meas[a:b], None if wts is None else wts[a:b]))
    plan = Plan.for_problem(start, max_positions=B, tune=tune)
    if args.graphs:
        plan.set_graphs(True)
    outs = {}
    for (p_, m_, w_) in calls:
        n = int(p_.shape[0])
        if n not in outs:
            outs[n] = plan.forward_adjoint(obj, probe, p_, m_, weights=w_, grads=grads)

    def step(plain=False):
        for (p_, m_, w_) in calls:
            plan.forward_adjoint(obj, probe, p_, m_, weights=w_, grads=grads, out=outs[int(p_.shape[0])],
                                 plain=plain)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    plan.set_timing(True)
    plan.kernel_time()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    k_ms, k_n = plan.kernel_time()
    plan.set_timing(False)
    flags = plan.get_error()
    ms_step = (t1 - t0) * 1e3 / args.steps
    K = truth.K
    value = K / (ms_step * 1e-3)
    k_avg_ms = k_ms / max(k_n, 1)          # one launch (a chunk of positions)
    launches = max(k_n, 1) / args.steps     # launches per step (positions are chunked when the
    k_step_ms = k_ms / args.steps           # window buffer would exceed its budget)

    flops_pp, bytes_pp = algorithmic(start)
    achieved_tflops = flops_pp * K / (k_step_ms * 1e-3) / 1e12
    hbm_alg_gbs = bytes_pp * K / (k_step_ms * 1e-3) / 1e9
    khash = kernel_hash()
    headline = args.workload == "c1"
    traffic = read_traffic(khash, kernel_name(plan, start, tune)) if headline else None
    copy_gbs = copy_bandwidth(torch, dev)  # achievable HBM bandwidth, outside the timed region

    plain = None
    if not args.no_plain:
        step(plain=True)
        torch.cuda.synchronize()
        plan.set_timing(True)
        plan.kernel_time()
        tp0 = time.perf_counter()
        for _ in range(args.plain_steps):
            step(plain=True)
        torch.cuda.synchronize()
        tp1 = time.perf_counter()
        p_ms, p_n = plan.kernel_time()
        plan.set_timing(False)
        p_step = (tp1 - tp0) * 1e3 / args.plain_steps
        plain = {"value": K / (p_step * 1e-3), "ms_per_step": p_step, "steps": args.plain_steps,
                 "kernel_chain_ms": p_ms / max(p_n, 1),
                 "hbm_alg_frac": bytes_pp * K / (p_step * 1e-3) / 1e9 / HBM_PEAK_GBS}

    # the autograd form (torch.autograd.Function over the same plan): forward + backward
    # of the loss with respect to the same leaves, timed the same way as the per-call form
    autograd = None
    if not args.no_autograd and len(calls) == 1:
        from paper_2510_20929_amd import ptycho_loss
        leaves = {"obj": obj.clone().requires_grad_("obj" in grads),
                  "probe": probe.clone().requires_grad_("probe" in grads),
                  "pos": pos.clone().requires_grad_("pos" in grads)}
        w_leaf = None if wts is None else wts.clone().requires_grad_("weights" in grads)

        def ag_step():
            for v in list(leaves.values()) + ([w_leaf] if w_leaf is not None else []):
                v.grad = None
            L = ptycho_loss(leaves["obj"], leaves["probe"], leaves["pos"], I_meas, plan, weights=w_leaf)
            L.backward()

        for _ in range(max(1, args.warmup)):
            ag_step()
        torch.cuda.synchronize()
        ta0 = time.perf_counter()
        for _ in range(args.steps):
            ag_step()
        torch.cuda.synchronize()
        a_ms = (time.perf_counter() - ta0) * 1e3 / args.steps
        autograd = {"value": K / (a_ms * 1e-3), "ms_per_step": a_ms, "vs_per_call": ms_step / a_ms,
                    "form": "PtychoLoss (torch.autograd.Function) forward + backward, same plan"}

    cpu = None
    if headline and not args.no_cpu:
        cpu = cpu_baseline(truth, start)

    line = dict(common)
    line.update({
        "value": value,
        "ms_per_step": ms_step,
        "config": {"workload": WORKLOADS[args.workload], "frame": start.N, "modes": start.M,
                   "eigenprobes": start.E, "slices": start.S, "positions": K, "object": [start.H, start.W],
                   "loss": start.loss, "form": "fused persistent kernel",
                   "positions_per_call": B, "calls_per_step": len(calls), "graph_replay": bool(args.graphs)},
        "roofline": {"bound": "alu", "achieved": achieved_tflops, "peak": FP32_VECTOR_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved_tflops / FP32_VECTOR_PEAK_TFLOPS,
                     "traffic": traffic, "kernel": kernel_name(plan, start, tune),
                     "kernel_ms": k_avg_ms, "launches_per_step": launches, "kernel_ms_per_step": k_step_ms,
                     "flops_per_pattern": flops_pp},
        "hbm": {"alg_bytes_per_pattern": bytes_pp, "alg_GBs": hbm_alg_gbs, "frac_of_peak": hbm_alg_gbs / HBM_PEAK_GBS,
                "copy_GBs": copy_gbs, "frac_of_copy": hbm_alg_gbs / copy_gbs,
                "counter_GBs": (traffic / (k_avg_ms * 1e-3) / 1e9) if traffic else None},
        "plain": plain,
        "fused_vs_plain": (value / plain["value"]) if plain else None,
        "autograd": autograd,
        "cpu_baseline": cpu,
        "tune": tune,
        "tune_source": tune_src,
        "plan_bytes": {k: plan.info()[k] for k in ("workspace_bytes", "scratch_bytes", "window_bytes", "plain_bytes")},
        "error_flags": flags,
        "kernel_hash": khash,
    })
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
