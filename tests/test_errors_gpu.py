"""Device-detected errors latch a flag and drop only the offending position; host-
detectable errors return a status and launch nothing."""
import ctypes

import numpy as np
import pytest

from gpu_util import compare, custom_problem, dev, rel_l2, run_gpu, run_oracle, torch_cuda

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _needs_gpu():
    torch_cuda()


@pytest.mark.parametrize("plain", [False, True], ids=["fused", "plain"])
@pytest.mark.parametrize("kind", ["bounds", "nan_position", "nan_data"])
@pytest.mark.parametrize("N", [64, 256])
def test_bad_position_is_dropped_and_latched(N, kind, plain):
    from paper_2510_20929_amd import FLAG_BOUNDS, FLAG_NONFINITE, Plan
    p, I = custom_problem(41, N, 2, 1, 1, 3 * N, 30 if N <= 128 else 12)
    bad = 7
    pos = p.positions.copy()
    I = I.copy()
    if kind == "bounds":
        pos[bad] = (3 * N - 1.5, 3.0)
        expect = FLAG_BOUNDS
    elif kind == "nan_position":
        pos[bad, 1] = np.nan
        expect = FLAG_NONFINITE
    else:
        I[bad, 3, 4] = np.nan
        expect = FLAG_NONFINITE
    from dataclasses import replace
    q = replace(p, positions=pos)
    grads = ("obj", "probe", "pos")
    keep = np.array([k for k in range(p.K) if k != bad])
    ref = run_oracle(q.subset(keep), I[keep], grads, norm_count=p.K)
    plan = Plan.for_problem(q)
    got = run_gpu(plan, q, I, grads, plain=plain, want_ipred=False)
    assert got["flags"] & expect
    assert np.all(got["g_pos"][bad] == 0)
    got["g_pos"] = got["g_pos"][keep]
    compare(got, ref, grads, tag=f"{kind} {'plain' if plain else 'fused'}")
    plan.clear_error()
    assert plan.get_error() == 0


@pytest.mark.parametrize("model", ["near", "fourier", "multislice"])
def test_per_step_models_of_large_frames_drop_bad_positions_and_shard(model):
    """256^2 near-field, Fourier-shift and multislice plans (per-step form): a position
    outside the object is latched and dropped with the rest exact, and two shards
    accumulated with the global normaliser equal the whole call."""
    torch = torch_cuda()
    from dataclasses import replace
    from paper_2510_20929_amd import FLAG_BOUNDS, Plan
    N = 256
    kw = {"near": dict(det_lambda_z=(N / 2.0) ** 2 / 50.0), "fourier": dict(subpixel="fourier"),
          "multislice": dict(lz=N / 8.0)}[model]
    S = 2 if model == "multislice" else 1
    p, I = custom_problem(47, N, 2, 1, S, N + 96, 8, **kw)
    bad = 3
    pos = p.positions.copy()
    pos[bad] = (N + 90.0, 3.0)
    q = replace(p, positions=pos)
    grads = ("obj", "probe", "pos")
    keep = np.array([k for k in range(p.K) if k != bad])
    ref = run_oracle(q.subset(keep), I[keep], grads, norm_count=p.K)
    plan = Plan.for_problem(q)
    got = run_gpu(plan, q, I, grads, want_ipred=False)
    assert got["flags"] & FLAG_BOUNDS
    assert np.all(got["g_pos"][bad] == 0)
    got["g_pos"] = got["g_pos"][keep]
    compare(got, ref, grads, tag=f"{model} 256 bad position")
    plan.clear_error()
    sp = Plan.for_problem(p, norm_count=p.K)
    o, u, r, m = dev(p.obj), dev(p.probe), dev(p.positions), dev(I)
    whole = sp.forward_adjoint(o, u, r, m, grads=("obj", "probe"))
    whole = {k: v.clone() for k, v in whole.items()}
    acc = None
    for a_, b_ in ((0, 3), (3, p.K)):
        acc = sp.forward_adjoint(o, u, r[a_:b_].contiguous(), m[a_:b_].contiguous(), grads=("obj", "probe"),
                                 accumulate=acc is not None, out=acc)
    torch.cuda.synchronize()
    for key in ("loss", "g_obj", "g_probe"):
        assert rel_l2(acc[key].cpu().numpy(), whole[key].cpu().numpy()) <= 1e-5, key


def test_host_errors_launch_nothing():
    torch = torch_cuda()
    from paper_2510_20929_amd import Plan, PtyhipError, lib
    p, I = custom_problem(42, 32, 1, 1, 1, 96, 10)
    plan = Plan.for_problem(p)
    o, u, r, m = dev(p.obj), dev(p.probe), dev(p.positions), dev(I)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    L = lib()
    st = L.ptyhip_forward(plan._h, None, 11, ctypes.c_void_p(o.data_ptr()), ctypes.c_void_p(u.data_ptr()), None,
                          ctypes.c_void_p(r.data_ptr()), ctypes.c_void_p(m.data_ptr()),
                          ctypes.c_void_p(loss.data_ptr()), None)
    assert st == 3  # K > max_positions
    st = L.ptyhip_forward(plan._h, None, 10, None, ctypes.c_void_p(u.data_ptr()), None,
                          ctypes.c_void_p(r.data_ptr()), ctypes.c_void_p(m.data_ptr()),
                          ctypes.c_void_p(loss.data_ptr()), None)
    assert st == 1  # NULL object
    st = L.ptyhip_forward_adjoint(plan._h, None, 10, 8, ctypes.c_void_p(o.data_ptr()), ctypes.c_void_p(u.data_ptr()),
                                  None, ctypes.c_void_p(r.data_ptr()), ctypes.c_void_p(m.data_ptr()),
                                  ctypes.c_void_p(loss.data_ptr()), None, None, None, None, None)
    assert st == 1  # weight gradient without weights
    out = plan.forward_adjoint(o, u, r[:0], m[:0], grads=("obj", "probe"))
    torch.cuda.synchronize()
    assert float(out["loss"][0]) == 0.0 and float(out["g_obj"].abs().max()) == 0.0
    with pytest.raises(PtyhipError):
        Plan(100, 1, 1, 1, 200, 200)
