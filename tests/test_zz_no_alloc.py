"""The allocation-free entry point (ptyhip_forward_adjoint_static, for callers that cannot
call hipMalloc) against the plan-based ptyhip_forward_adjoint, through the C ABI: two
calls in a row, the second on a smaller input (other frame size, fewer positions), both
to the parity tolerances (forward <= 1e-5, gradients <= 1e-4 relative L2); and the
host-side rejection of a problem whose buffers exceed the fixed device array."""
import ctypes

import numpy as np
import pytest

from gpu_util import FWD_TOL, GRAD_TOL, custom_problem, dev, rel_l2, torch_cuda

pytestmark = pytest.mark.gpu

NAMES = {"obj": "g_obj", "probe": "g_probe", "pos": "g_pos", "weights": "g_weights"}


def _both(prob, I, grads, tune=None):
    torch = torch_cuda()
    from paper_2510_20929_amd import Plan
    from paper_2510_20929_amd.ptyhip import forward_adjoint_static, make_desc
    w = None if prob.weights is None else dev(prob.weights)
    args = (dev(prob.obj), dev(prob.probe), dev(prob.positions), dev(I))
    ip_a = torch.zeros((prob.K, prob.N, prob.N), dtype=torch.float32, device="cuda")
    ip_b = torch.zeros_like(ip_a)
    plan = Plan.for_problem(prob, tune=tune)
    ref = plan.forward_adjoint(*args, weights=w, grads=grads, I_pred=ip_a)
    desc = make_desc(prob.N, prob.M, prob.E, prob.S, prob.H, prob.W, prob.loss, prob.eps)
    got = forward_adjoint_static(desc, *args, weights=w, grads=grads, tune=tune, I_pred=ip_b)
    torch.cuda.synchronize()
    assert plan.get_error() == 0
    assert int(got["flags"].cpu()[0]) == 0
    e = abs(float(got["loss"].cpu()[0]) - float(ref["loss"].cpu()[0])) / abs(float(ref["loss"].cpu()[0]))
    errs = {"loss": e, "I_pred": rel_l2(ip_b.cpu().numpy(), ip_a.cpu().numpy())}
    for g in grads:
        errs[NAMES[g]] = rel_l2(got[NAMES[g]].cpu().numpy(), ref[NAMES[g]].cpu().numpy())
    print(f"static vs plan N={prob.N} M={prob.M} E={prob.E} K={prob.K} tune={tune}: "
          + ", ".join(f"{k}={v:.2e}" for k, v in errs.items()), flush=True)
    for k, v in errs.items():
        assert v <= (FWD_TOL if k in ("loss", "I_pred") else GRAD_TOL), (k, v)


def test_static_entry_point_matches_plan_twice():
    # first call: the headline shape (128^2, four modes, Poisson), 300 positions (several
    # chunks of the fixed array, several positions per workgroup)
    a, Ia = custom_problem(801, 128, 4, 1, 1, 400, 300, loss="poisson")
    _both(a, Ia, ("obj", "probe", "pos"))
    # second call, smaller: 64^2 frames, two modes, OPR eigenprobes with weights, 120 positions
    b, Ib = custom_problem(802, 64, 2, 2, 1, 200, 120, weights="opr")
    _both(b, Ib, ("obj", "probe", "pos", "weights"))


def test_static_entry_point_tuned_layout():
    # the benchmark's 128^2 layout (1024 threads, patch in registers, far fields recomputed)
    a, Ia = custom_problem(803, 128, 4, 1, 1, 360, 200, loss="poisson")
    _both(a, Ia, ("obj", "probe", "pos"), tune={"variant": 4, "recompute": 1})


def test_static_entry_point_rejects_what_does_not_fit():
    torch = torch_cuda()
    from paper_2510_20929_amd.ptyhip import ENOMEM, Tune, lib, make_desc
    # 64 modes x 16 eigenprobes of 128^2: one workgroup's accumulators alone exceed the array
    desc = make_desc(128, 64, 16, 1, 256, 256, "amplitude")
    obj = torch.zeros((1, 256, 256), dtype=torch.complex64, device="cuda")
    probe = torch.zeros(4, dtype=torch.complex64, device="cuda")     # never read: rejected on the host
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    st = lib().ptyhip_forward_adjoint_static(ctypes.byref(desc), ctypes.POINTER(Tune)(), None, 0, 0,
                                             ctypes.c_void_p(obj.data_ptr()), ctypes.c_void_p(probe.data_ptr()),
                                             None, None, None, ctypes.c_void_p(loss.data_ptr()), None, None, None,
                                             None, None, None)
    assert st == ENOMEM
    torch.cuda.synchronize()
