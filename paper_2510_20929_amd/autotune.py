"""Autotuner for the fused forward + adjoint and the batched launch.

For a problem shape it enumerates implementation choices (thread layout of the
on-chip kernel or of the four-step kernel, storing vs recomputing far fields /
incident waves, persistent grid size; for batches the workgroup count of each
frame-size class's launch, or one call per dataset), runs every
candidate once and keeps it only if its loss and gradients agree with the per-step
form on the same inputs (forward <= 1e-5, gradients <= 1e-4 relative L2), then times
the survivors with HIP events (median of several launches) and caches the fastest
in a JSON file keyed by GPU architecture, a hash of the library sources and the
problem shape: an entry timed on other kernel sources is never used.
"""
from __future__ import annotations

import hashlib
import json
import os
import time
from typing import Dict, List, Optional, Sequence

import torch

from .ptyhip import Batch, Plan

# the frozen cache shipped with the package; PTYHIP_TUNE_CACHE points every lookup and
# every new result at another file (for a retuning run)
DEFAULT_CACHE = (os.environ.get("PTYHIP_TUNE_CACHE")
                 or os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json"))
FWD_TOL = 1e-5
GRAD_TOL = 1e-4


_SRC_HASH: Optional[str] = None


def source_hash() -> str:
    """Hash of every kernel and host source of the library (csrc/**): a tuning result
    belongs to the code it was timed on."""
    global _SRC_HASH
    if _SRC_HASH is None:
        root = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
        h = hashlib.sha256()
        files = []
        for d, _, fs in os.walk(root):
            files += [os.path.join(d, f) for f in fs if f.endswith((".hip", ".hpp", ".cpp", ".h"))]
        for f in sorted(files, key=lambda x: os.path.relpath(x, root)):
            h.update(os.path.relpath(f, root).encode())
            with open(f, "rb") as fh:
                h.update(fh.read())
        _SRC_HASH = h.hexdigest()[:12]
    return _SRC_HASH


def _arch() -> str:
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def _cus() -> int:
    return torch.cuda.get_device_properties(0).multi_processor_count


def shape_key(N, M, E, S, loss, grads: Sequence[str], K: int) -> str:
    kb = 1 << max(0, int(K - 1).bit_length())  # bucket positions by power of two
    return f"{_arch()}|src{source_hash()}|N{N}|M{M}|E{E}|S{S}|{loss}|{'+'.join(sorted(grads))}|K{kb}"


def load_cache(path: str = DEFAULT_CACHE) -> Dict[str, dict]:
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def save_cache(cache: Dict[str, dict], path: str = DEFAULT_CACHE) -> None:
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def plan_candidates(N: int, M: int, S: int, K: int = 0, split_ok: bool = True, E: int = 1,
                    lds_ok: bool = True) -> List[dict]:
    """Thread layout x far-field store/recompute x persistent grid; with few positions per
    call and several modes (K below two workgroups per CU), also the mode-split form with
    enough groups to give every CU one or two (position, group) items. ``lds_ok``: the
    LDS-resident 128^2 layouts (5, 6; far field, bilinear patch) apply."""
    cus = _cus()
    out = []
    variants = [0, 1, 2, 3, 4] if N in (64, 128) else [0, 1]
    recomputes = [0, 1] if (M > 1 or S > 1) else [0]
    grids = [0, 2 * cus] if N <= 128 else [0]
    for v in variants:
        for r in recomputes:
            for g in grids:
                out.append({"variant": v, "recompute": r, "grid": g})
    if N == 128 and lds_ok:
        if S == 1:
            # far fields are always recomputed in these layouts
            for v in (5, 6):
                out.append({"variant": v, "recompute": 1, "grid": 0})
        else:
            # several slices: one LDS-resident kernel (incident waves stored or recomputed)
            for r in recomputes:
                out.append({"variant": 5, "recompute": r, "grid": 0})
    # single eigenprobe: the probe gradients staged per position instead of accumulated
    # in the workgroups' scratch (a streaming write and a separate reduction in place of
    # a read-modify-write per mode)
    if S == 1 and E == 1:
        for v in ([1, 4] if N in (64, 128) else [0]):
            for r in recomputes:
                out.append({"variant": v, "recompute": r, "grid": 0, "probe_stage": 1})
    if split_ok and S == 1 and M > 1 and 0 < K < 2 * cus:
        groups = sorted({min(M, -(-c * cus // K)) for c in (1, 2)})
        for G in groups:
            if G < 2:
                continue
            for v in ([0, 4] if N in (64, 128) else [0]) + ([5] if N == 128 and lds_ok else []):
                out.append({"variant": v, "recompute": 0, "grid": 0, "mode_groups": G})
    return out


def _rel(a: torch.Tensor, b: torch.Tensor) -> float:
    a = torch.view_as_real(a) if a.is_complex() else a
    b = torch.view_as_real(b) if b.is_complex() else b
    return float((a.double() - b.double()).norm() / b.double().norm().clamp_min(1e-300))


def _agrees(out: dict, ref: dict, grads: Sequence[str]) -> Optional[str]:
    e = abs(float(out["loss"][0]) - float(ref["loss"][0])) / max(abs(float(ref["loss"][0])), 1e-300)
    if not e <= FWD_TOL:
        return f"loss {e:.2e}"
    for g in grads:
        key = {"obj": "g_obj", "probe": "g_probe", "pos": "g_pos", "weights": "g_weights"}[g]
        r = _rel(out[key], ref[key])
        if not r <= GRAD_TOL:
            return f"{key} {r:.2e}"
    return None


def _time(fn, reps: int) -> float:
    st = torch.cuda.current_stream()
    ts = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(st)
        fn()
        b.record(st)
        b.synchronize()
        ts.append(a.elapsed_time(b))
    ts.sort()
    return ts[len(ts) // 2]


def tune_plan(shape: dict, obj, probe, positions, I_meas, weights=None, grads=("obj", "probe", "pos"),
              reps: int = 5, cache_path: Optional[str] = DEFAULT_CACHE, use_cache: bool = True, log=None,
              key_K: Optional[int] = None):
    """Pick the fastest parity-passing fused configuration for one plan shape.
    ``shape`` holds N, M, E, S, H, W, loss, eps, lambda_z. Returns (tune, report).
    ``key_K`` looks the choice up under another position count (the full workload's,
    when fewer of its positions are passed); a choice tuned here on fewer positions is
    then not stored under that key."""
    K = int(positions.shape[0])
    key = shape_key(shape["N"], shape["M"], shape["E"], shape["S"], shape["loss"], grads, key_K or K)
    if key_K is not None and key_K != K:
        cache_path = cache_path if use_cache else None
        store = False
    else:
        store = True
    cache = load_cache(cache_path) if (cache_path and use_cache) else {}
    if use_cache and key in cache:
        return cache[key]["tune"], {"key": key, "cached": True}

    def make(tune):
        return Plan(shape["N"], shape["M"], shape["E"], shape["S"], shape["H"], shape["W"], shape["loss"],
                    shape.get("eps", 1e-3), shape.get("lambda_z", 0.0), 0.0, K, tune)

    ref_plan = make(None)
    ref = ref_plan.forward_adjoint(obj, probe, positions, I_meas, weights=weights, grads=grads, plain=True)
    torch.cuda.synchronize()
    del ref_plan
    results = []
    best = None
    split_ok = shape.get("det_lambda_z") is None and shape.get("subpixel", "bilinear") == "bilinear"
    for cand in plan_candidates(shape["N"], shape["M"], shape["S"], K, split_ok, shape["E"], lds_ok=split_ok):
        plan = make(cand)
        out = plan.forward_adjoint(obj, probe, positions, I_meas, weights=weights, grads=grads)
        torch.cuda.synchronize()
        bad = _agrees(out, ref, grads)
        if bad:
            results.append({"tune": cand, "parity": bad})
            continue
        ms = _time(lambda: plan.forward_adjoint(obj, probe, positions, I_meas, weights=weights, grads=grads,
                                                out=out), reps)
        results.append({"tune": cand, "ms": ms})
        if log:
            log(f"tune {cand}: {ms:.3f} ms")
        if best is None or ms < best[1]:
            best = (cand, ms)
        del plan
    if best is None:
        raise RuntimeError(f"no autotuner candidate passed parity for {key}: {results}")
    if cache_path and store:
        cache = load_cache(cache_path)
        cache[key] = {"tune": best[0], "ms": best[1], "when": time.strftime("%Y-%m-%d %H:%M:%S"),
                      "candidates": results}
        save_cache(cache, cache_path)
    return best[0], {"key": key, "cached": False, "candidates": results}


def batch_key(problems, grads) -> str:
    """Cache key of a batch: architecture, sources, every dataset's shape and the gradients."""
    h = hashlib.sha256()
    for p in problems:
        h.update(f"{p.N},{p.M},{p.E},{p.S},{p.H},{p.W},{p.K},{p.loss};".encode())
    return f"{_arch()}|src{source_hash()}|batch{len(problems)}|{h.hexdigest()[:12]}|{'+'.join(sorted(grads))}"


def tune_batch(problems, tensors, grads=("obj", "probe", "pos"), reps: int = 3, log=None,
               cache_path: Optional[str] = DEFAULT_CACHE, use_cache: bool = True):
    """Pick the batched schedule: the workgroup total of a launch, the frame-size classes
    one after the other or concurrently (graph branches sharing the CUs by work), or one
    call per dataset. ``tensors[i]`` = (obj, probe, positions, I_meas, weights) on the
    device. Every candidate must reproduce the per-call results of each dataset. The
    choice is cached under ``batch_key``. Returns (choice, report)."""
    key = batch_key(problems, grads)
    if cache_path and use_cache:
        cache = load_cache(cache_path)
        if key in cache:
            return cache[key]["tune"], {"key": key, "cached": True}
    cus = _cus()
    ref_b = Batch(problems)
    refs = [ref_b.bind(i, *t[:4], weights=t[4]) for i, t in enumerate(tensors)]
    ref_b.launch(grads, per_call=True)
    torch.cuda.synchronize()
    ref = [{k: v.clone() for k, v in r.items()} for r in refs]
    results = []
    best = None
    for variant in (0, 1):
        for total in (cus, 2 * cus, 4 * cus):
            cand = {"variant": variant, "grid": total}
            b = Batch(problems, tune=cand)
            outs = [b.bind(i, *t[:4], weights=t[4]) for i, t in enumerate(tensors)]
            b.launch(grads)
            torch.cuda.synchronize()
            bad = None
            for i, o in enumerate(outs):
                bad = bad or _agrees(o, ref[i], grads)
            if bad:
                results.append({"tune": cand, "parity": bad})
                continue
            ms = _time(lambda: b.launch(grads), reps)
            results.append({"tune": cand, "ms": ms})
            if log:
                log(f"batch {cand}: {ms:.3f} ms")
            if best is None or ms < best[1]:
                best = (cand, ms)
            del b, outs
    ms = _time(lambda: ref_b.launch(grads, per_call=True), reps)
    results.append({"tune": {"per_call": True}, "ms": ms})
    if best is None or ms < best[1]:
        best = ({"per_call": True}, ms)
    if cache_path:
        cache = load_cache(cache_path)
        cache[key] = {"tune": best[0], "ms": best[1], "when": time.strftime("%Y-%m-%d %H:%M:%S"),
                      "candidates": results}
        save_cache(cache, cache_path)
    return best[0], {"key": key, "cached": False, "candidates": results}
