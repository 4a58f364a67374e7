"""Illumination map and scale-normalised gradients on the GPU against the FP64 oracle,
through the C ABI."""
import numpy as np
import pytest

import oracle
from gpu_util import FWD_TOL, GRAD_TOL, case, custom_problem, dev, rel_l2, run_oracle, torch_cuda

pytestmark = pytest.mark.gpu


def _plan(prob, **kw):
    torch_cuda()
    from paper_2510_20929_amd import Plan
    return Plan.for_problem(prob, **kw)


def _illum(prob, **kw):
    torch = torch_cuda()
    plan = _plan(prob)
    w = None if prob.weights is None else dev(prob.weights)
    out = plan.illumination(dev(prob.probe), dev(prob.positions), weights=w, **kw)
    torch.cuda.synchronize()
    return out.cpu().numpy(), plan.get_error()


@pytest.mark.parametrize("which", ["c1", "c1full", "c0", "opr", "amp", "N16", "N256"])
def test_illumination_matches_oracle(which):
    if which == "c1":
        p, _ = case(1, H=400, K=300)              # 4 modes, sub-pixel spiral
    elif which == "c1full":
        from synth import workloads as W
        p = W.perturb(W.make_config(1), 5)        # full size: 1024^2 object, 2000 positions
    elif which == "c0":
        p, _ = case(0)                            # integer raster, one mode
        p = p.subset(np.arange(0, 625, 3))
    elif which == "opr":
        p, _ = custom_problem(41, 64, 2, 3, 1, 200, 80, weights="opr")
    elif which == "amp":
        p, _ = custom_problem(42, 128, 3, 1, 1, 400, 90, weights="amp")
    elif which == "N16":
        p, _ = custom_problem(43, 16, 1, 1, 1, 60, 40)
    else:
        p, _ = custom_problem(44, 256, 2, 2, 1, 600, 30, weights="opr")
    got, flags = _illum(p)
    ref = oracle.illumination(p.probe, p.positions, p.H, p.W, weights=p.weights)
    err = rel_l2(got, ref)
    print(f"illumination {which}: rel err {err:.2e}", flush=True)
    assert err <= FWD_TOL and flags == 0


def test_illumination_accumulate_and_empty():
    torch = torch_cuda()
    p, _ = custom_problem(45, 32, 2, 1, 1, 120, 50)
    plan = _plan(p)
    pr, pos = dev(p.probe), dev(p.positions)
    out = torch.full((p.H, p.W), 3.0, dtype=torch.float32, device="cuda")
    plan.illumination(pr, pos, out=out, accumulate=True)
    torch.cuda.synchronize()
    ref = 3.0 + oracle.illumination(p.probe, p.positions, p.H, p.W)
    assert rel_l2(out.cpu().numpy(), ref) <= FWD_TOL
    empty = pos[:0]
    plan.illumination(pr, empty, out=out)           # K = 0 overwrites with zeros
    torch.cuda.synchronize()
    assert float(out.abs().max()) == 0.0


def test_illumination_skips_invalid_positions():
    torch = torch_cuda()
    p, _ = custom_problem(46, 32, 1, 1, 1, 100, 20)
    bad = p.positions.copy()
    bad[7] = [90.0, 10.5]                            # window leaves the object
    q = p.subset(np.arange(p.K))
    q.positions[:] = bad
    got, flags = _illum(q)
    keep = np.array([k for k in range(p.K) if k != 7])
    ref = oracle.illumination(p.probe, bad[keep], p.H, p.W)
    assert rel_l2(got, ref) <= FWD_TOL
    assert flags & 1  # bounds flag latched


@pytest.mark.parametrize("which", ["c1", "opr"])
def test_normalized_gradients_match_oracle(which):
    torch = torch_cuda()
    if which == "c1":
        p, I = case(1, H=400, K=200)
        grads = ("obj", "probe", "pos")
    else:
        p, I = custom_problem(47, 64, 2, 3, 1, 200, 60, weights="opr")
        grads = ("obj", "probe", "weights")
    plan = _plan(p)
    w = None if p.weights is None else dev(p.weights)
    obj, pr = dev(p.obj), dev(p.probe)
    out = plan.forward_adjoint(obj, pr, dev(p.positions), dev(I), weights=w, grads=grads)
    plan.normalize_gradients(p.K, probe=pr, obj=obj, weights=w, g_obj=out["g_obj"], g_probe=out["g_probe"])
    torch.cuda.synchronize()
    ref = run_oracle(p, I, grads)
    go, gp = oracle.normalized_gradients(ref["g_obj"], ref["g_probe"], p.obj, p.probe, p.K, weights=p.weights)
    eo = rel_l2(out["g_obj"].cpu().numpy(), go)
    ep = rel_l2(out["g_probe"].cpu().numpy(), gp)
    print(f"normalized {which}: g_obj {eo:.2e} g_probe {ep:.2e}", flush=True)
    assert eo <= GRAD_TOL and ep <= GRAD_TOL
