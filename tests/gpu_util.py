"""Shared helpers of the GPU tests: seeded cases, oracle runs, and the comparison
protocol (relative L2 over re/im pairs; forward <= 1e-5, gradients <= 1e-4)."""
from __future__ import annotations

import os
import sys
from dataclasses import replace

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from synth import workloads as W  # noqa: E402

FWD_TOL = 1e-5
GRAD_TOL = 1e-4


def torch_cuda():
    try:
        import torch
    except Exception:  # pragma: no cover
        pytest.skip("torch missing")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def dev(a):
    torch = torch_cuda()
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def rel_l2(got, ref) -> float:
    g = np.asarray(got, dtype=np.complex128).ravel()
    r = np.asarray(ref, dtype=np.complex128).ravel()
    return float(np.linalg.norm(g - r) / max(np.linalg.norm(r), 1e-300))


def measured(truth, seed: int):
    """Noisy measured intensities of a truth problem (clean intensities from the oracle)."""
    _, I_clean = oracle.forward(truth.obj, truth.probe, truth.positions, np.zeros((truth.K, truth.N, truth.N)),
                                weights=truth.weights, lambda_z=truth.lambda_z,
                                det_lambda_z=getattr(truth, "det_lambda_z", None),
                                subpixel=getattr(truth, "subpixel", "bilinear"))
    return W.poisson_counts(I_clean, seed)


def case(config: int, seed: int = 5, **kw):
    truth = W.make_config(config, **kw)
    start = W.perturb(truth, seed)
    return start, measured(truth, seed + 1)


def run_oracle(prob, I_meas, grads, norm_count=None):
    return oracle.forward_adjoint(prob.obj, prob.probe, prob.positions, I_meas, weights=prob.weights,
                                  loss=prob.loss, eps=prob.eps, lambda_z=prob.lambda_z, norm_count=norm_count,
                                  grads=grads, det_lambda_z=getattr(prob, "det_lambda_z", None),
                                  subpixel=getattr(prob, "subpixel", "bilinear"))


def run_gpu(plan, prob, I_meas, grads, plain=False, want_ipred=True):
    torch = torch_cuda()
    w = None if prob.weights is None else dev(prob.weights)
    ipred = torch.zeros((prob.K, prob.N, prob.N), dtype=torch.float32, device="cuda") if want_ipred else None
    out = plan.forward_adjoint(dev(prob.obj), dev(prob.probe), dev(prob.positions), dev(I_meas), weights=w,
                               grads=grads, plain=plain, I_pred=ipred)
    torch.cuda.synchronize()
    res = {k: v.cpu().numpy() for k, v in out.items()}
    res["loss"] = float(res["loss"][0])
    res["flags"] = plan.get_error()
    return res


def compare(got, ref, grads, tag=""):
    errs = {"loss": abs(got["loss"] - ref["loss"]) / max(abs(ref["loss"]), 1e-300)}
    if "I_pred" in got:
        errs["I_pred"] = rel_l2(got["I_pred"], ref["I_pred"])
    names = {"obj": "g_obj", "probe": "g_probe", "pos": "g_pos", "weights": "g_weights", "lambda_z": "g_lambda_z"}
    for g in grads:
        errs[names[g]] = rel_l2(got[names[g]], ref[names[g]])
    print(f"{tag} rel errors: " + ", ".join(f"{k}={v:.2e}" for k, v in errs.items()), flush=True)
    for k, v in errs.items():
        tol = FWD_TOL if k in ("loss", "I_pred") else GRAD_TOL
        assert v <= tol, f"{tag}: {k} rel err {v:.3e} > {tol}"
    return errs


def custom_problem(seed, N, M, E, S, H, K, loss="amplitude", lz=0.0, weights=None, det_lambda_z=None,
                   subpixel="bilinear"):
    """Small generic problem (random smooth object, random smooth probes, random
    sub-pixel positions) for shapes no config covers."""
    rng = np.random.default_rng(seed)
    obj = np.stack([W.random_object(rng, H, H) for _ in range(S)])
    probe = np.stack([[W.disk_probe(N, N / 4.0) * np.exp(1j * rng.uniform(0, 1)) * (0.6 ** m)
                       * (1.0 + 0.3 * W.smooth_field((N, N), 2.0, rng)) for m in range(M)] for _ in range(E)])
    probe = probe * np.sqrt(1e4 / np.sum(np.abs(probe[0]) ** 2))
    pos = rng.uniform(0.0, H - N - 1.01, size=(K, 2))
    w = None
    if weights == "opr" or (weights is None and E > 1):
        w = np.concatenate([rng.normal(1.0, 0.1, (K, 1)), rng.normal(0.0, 0.05, (K, E - 1))], axis=1)[:, :E]
    elif weights == "amp":
        w = rng.uniform(0.85, 1.15, size=(K, E))
    truth = W.Problem("custom", obj.astype(np.complex64), probe.astype(np.complex64), pos.astype(np.float32),
                      None if w is None else w.astype(np.float32), loss, lambda_z=lz, det_lambda_z=det_lambda_z,
                      subpixel=subpixel)
    start = W.perturb(truth, seed + 1)
    return start, measured(truth, seed + 2)


def _oracle_clean_chunk(args):
    """Worker: the oracle's clean intensities of one chunk of positions (runs in a spawned
    process that never touches the GPU)."""
    obj, probe, pos, weights, lambda_z, det_lambda_z = args[:6]
    subpixel = args[6] if len(args) > 6 else "bilinear"
    return oracle.forward(obj, probe, pos, np.zeros((pos.shape[0], probe.shape[-1], probe.shape[-1])),
                          weights=weights, lambda_z=lambda_z, det_lambda_z=det_lambda_z,
                          subpixel=subpixel)[1].astype(np.float32)


def measured_many(truths, seeds, workers: int = 16, noise: bool = True):
    """``measured`` for full-size workloads: the oracle's clean intensities computed in
    parallel over chunks of positions (spawned CPU processes that never touch the GPU),
    then Poisson noise with each problem's seed."""
    import concurrent.futures as cf
    import multiprocessing as mp
    n = max(1, min(workers, os.cpu_count() or 1))
    jobs, owner = [], []
    for t_i, truth in enumerate(truths):
        pieces = max(1, min(n, truth.K // 8))
        bounds = np.linspace(0, truth.K, pieces + 1).astype(int)
        for a, b in zip(bounds[:-1], bounds[1:]):
            w = None if truth.weights is None else truth.weights[a:b]
            jobs.append((truth.obj, truth.probe, truth.positions[a:b], w, truth.lambda_z,
                         getattr(truth, "det_lambda_z", None), getattr(truth, "subpixel", "bilinear")))
            owner.append(t_i)
    import time
    t0 = time.time()
    parts = [None] * len(jobs)
    with cf.ProcessPoolExecutor(max_workers=n, mp_context=mp.get_context("spawn")) as ex:
        futs = {ex.submit(_oracle_clean_chunk, j): i for i, j in enumerate(jobs)}
        for done, f in enumerate(cf.as_completed(futs), 1):
            parts[futs[f]] = f.result()
            if done % max(1, len(jobs) // 10) == 0 or done == len(jobs):
                print(f"oracle intensities: {done}/{len(jobs)} chunks, {time.time() - t0:.0f} s", flush=True)
    out = []
    for t_i, seed in enumerate(seeds):
        I = np.concatenate([p for p, o in zip(parts, owner) if o == t_i], axis=0)
        out.append(W.poisson_counts(I, seed) if noise else I)
    return out


def measured_parallel(truth, seed: int, workers: int = 16):
    return measured_many([truth], [seed], workers)[0]


def measured_sparse(truths, needs, seeds, workers: int = 16):
    """Measured intensities for full-size launches whose outputs are checked only at some
    positions: the oracle's clean intensities at the positions in ``needs[i]`` (every
    output that is compared depends only on those), re-used cyclically for the other
    positions, then Poisson noise. Every position thus gets a diffraction pattern of
    the workload's own statistics without running the oracle over all of them."""
    subs = [t.subset(np.asarray(n)) for t, n in zip(truths, needs)]
    clean = measured_many(subs, [0] * len(subs), workers=workers, noise=False)
    out = []
    for t, n, c, seed in zip(truths, needs, clean, seeds):
        n = np.asarray(n)
        full = np.empty((t.K, t.N, t.N), dtype=np.float32)
        full[np.arange(t.K)] = c[np.arange(t.K) % len(n)]
        full[n] = c
        out.append(W.poisson_counts(full, seed))
    return out


def covering(prob, ty: int, tx: int, size: int):
    """Indices of the positions whose (N+1)^2 window touches the tile [ty, ty+size) x [tx, tx+size)."""
    y0 = np.floor(prob.positions[:, 0]).astype(int)
    x0 = np.floor(prob.positions[:, 1]).astype(int)
    N = prob.N
    hit = (y0 <= ty + size - 1) & (y0 + N >= ty) & (x0 <= tx + size - 1) & (x0 + N >= tx)
    return np.nonzero(hit)[0]


def bench_tune(prob, I_meas, grads, key_K=None):
    """The implementation choice the benchmark runs for this workload shape, looked up
    exactly as bench.py does (the autotuner's cache for the current sources; a fresh,
    parity-gated tune when it holds none). ``key_K``: the full workload's position count
    when ``prob`` carries only some of its positions."""
    from paper_2510_20929_amd import autotune
    shape = dict(N=prob.N, M=prob.M, E=prob.E, S=prob.S, H=prob.H, W=prob.W, loss=prob.loss, eps=prob.eps,
                 lambda_z=prob.lambda_z)
    w = None if prob.weights is None else dev(prob.weights)
    tune, rep = autotune.tune_plan(shape, dev(prob.obj), dev(prob.probe), dev(prob.positions), dev(I_meas),
                                   weights=w, grads=grads, key_K=key_K)
    print(f"bench tune for {rep['key']}: {tune} ({'cached' if rep.get('cached') else 'tuned now'})", flush=True)
    return tune


def kernel_instance(prob, tune, threads):
    """Name of the fused kernel instance a plan runs (as the benchmark reports it)."""
    loss = 1 if prob.loss == "poisson" else 0
    if prob.N >= 256:
        return f"fused_big_kernel<{prob.N},{threads},{loss}>"
    if prob.S > 1:
        if prob.N == 128 and (tune or {}).get("variant", 0) >= 5:
            return f"fused_small_lds_ms_kernel<{prob.N},{threads},{loss}>"
        return f"fused_small_ms_kernel<{prob.N},{threads},{loss}>"
    v = (tune or {}).get("variant", 0) if prob.N >= 64 else 0
    if prob.N == 128 and v >= 5:
        return f"fused_small_lds_kernel<{prob.N},{threads},{loss},{'true' if v == 6 else 'false'}>"
    rv = "true" if v in (2, 3, 4) else "false"
    goreg = "true" if v in (2, 3) else "false"
    return f"fused_small_kernel<{prob.N},{threads},{loss},{rv},{goreg}>"


def _oracle_shard(args):
    """Worker: the oracle's forward + adjoint over one shard of positions (spawned CPU
    process that never touches the GPU). Returns the parameter-sized sums and the
    per-position outputs of the shard."""
    obj, probe, pos, weights, I, kw = args
    r = oracle.forward_adjoint(obj, probe, pos, I, weights=weights, **kw)
    return {k: v for k, v in r.items() if k != "I_pred"}


def run_oracle_sharded(prob, I_meas, grads, norm_count=None, workers: int = 16):
    """``run_oracle`` over all positions of a full-size workload, split into shards run in
    parallel CPU processes with the global normaliser: the loss, object and probe
    gradients are the sums over the shards (the data-parallel identity the oracle's
    shard-sum pin checks), position and weight gradients the concatenation."""
    import concurrent.futures as cf
    import multiprocessing as mp
    import time
    K = prob.K
    n = max(1, min(workers, os.cpu_count() or 1))
    pieces = max(1, min(4 * n, K // 4))
    bounds = np.linspace(0, K, pieces + 1).astype(int)
    kw = dict(loss=prob.loss, eps=prob.eps, lambda_z=prob.lambda_z, norm_count=norm_count or K, grads=grads)
    jobs = [(prob.obj, prob.probe, prob.positions[a:b], None if prob.weights is None else prob.weights[a:b],
             I_meas[a:b], kw) for a, b in zip(bounds[:-1], bounds[1:])]
    parts = [None] * len(jobs)
    t0 = time.time()
    with cf.ProcessPoolExecutor(max_workers=n, mp_context=mp.get_context("spawn")) as ex:
        futs = {ex.submit(_oracle_shard, j): i for i, j in enumerate(jobs)}
        for done, f in enumerate(cf.as_completed(futs), 1):
            parts[futs[f]] = f.result()
            if done % max(1, len(jobs) // 8) == 0 or done == len(jobs):
                print(f"sharded oracle: {done}/{len(jobs)} shards, {time.time() - t0:.0f} s", flush=True)
    out = {"loss": sum(p["loss"] for p in parts)}
    for key in ("g_obj", "g_probe"):
        if key in parts[0]:
            acc = parts[0][key].copy()
            for p in parts[1:]:
                acc += p[key]
            out[key] = acc
    for key in ("g_pos", "g_weights"):
        if key in parts[0]:
            out[key] = np.concatenate([p[key] for p in parts], axis=0)
    return out
