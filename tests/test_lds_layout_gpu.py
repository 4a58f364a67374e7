"""The LDS-resident 128^2 layouts of the fused forward + adjoint (tune variants 5 and 6:
the working frame in LDS, the patch, the running patch gradient and, in variant 6, dl/dI
in registers), against the FP64 oracle: Eqs. (1)-(2) through the forward model of the
Software design / Overview section, at the tolerances of the other parity tests
(forward <= 1e-5, gradients <= 1e-4 relative L2).

Every case runs on a grid of 16 workgroups, so that each workgroup takes several
positions with a ragged tail and its probe-gradient accumulator carries over from one
position to the next."""
import numpy as np
import pytest

import oracle
from gpu_util import compare, custom_problem, dev, rel_l2, run_gpu, run_oracle, torch_cuda

pytestmark = pytest.mark.gpu


def _plan(prob, **kw):
    torch_cuda()
    from paper_2510_20929_amd import Plan
    return Plan.for_problem(prob, **kw)


@pytest.mark.parametrize("variant", [5, 6])
@pytest.mark.parametrize("M,E,loss,weights", [(4, 1, "poisson", None), (4, 2, "poisson", "opr"),
                                               (1, 1, "amplitude", None), (3, 3, "amplitude", "opr")])
def test_lds_layouts_match_oracle(variant, M, E, loss, weights):
    """Modes, OPR eigenprobes with weight gradients (several eigenprobes stage their
    probe-wave gradients), both losses, every gradient."""
    start, I = custom_problem(700 + 10 * variant + M + 3 * E, 128, M, E, 1, 400, 75, loss=loss, weights=weights)
    grads = ("obj", "probe", "pos") + (("weights",) if start.weights is not None else ())
    ref = run_oracle(start, I, grads)
    got = run_gpu(_plan(start, tune={"variant": variant, "recompute": 1, "grid": 16}), start, I, grads)
    compare(got, ref, grads, tag=f"LDS layout {variant} M={M} E={E} {loss} grid=16")
    assert got["flags"] == 0


@pytest.mark.parametrize("variant", [5, 6])
def test_lds_layouts_probe_stage_and_forward_only(variant):
    """Staged single-eigenprobe probe gradients, and the forward-only call (loss and the
    predicted intensities)."""
    torch = torch_cuda()
    start, I = custom_problem(760 + variant, 128, 4, 1, 1, 360, 50, loss="poisson")
    grads = ("obj", "probe", "pos")
    ref = run_oracle(start, I, grads)
    plan = _plan(start, tune={"variant": variant, "recompute": 1, "grid": 16, "probe_stage": 1})
    got = run_gpu(plan, start, I, grads)
    compare(got, ref, grads, tag=f"LDS layout {variant} probe_stage")
    ipred = torch.zeros((start.K, 128, 128), dtype=torch.float32, device="cuda")
    loss = plan.forward(dev(start.obj), dev(start.probe), dev(start.positions), dev(I), I_pred=ipred)
    torch.cuda.synchronize()
    assert abs(float(loss.cpu()[0]) - ref["loss"]) <= 1e-5 * abs(ref["loss"])
    assert rel_l2(ipred.cpu().numpy(), ref["I_pred"]) <= 1e-5
    assert plan.get_error() == 0


@pytest.mark.parametrize("variant", [5, 6])
def test_lds_layouts_apply_A_AH(variant):
    """The linear map of Eq. (4) before the modulus and its adjoint through the same
    kernel (exit-wave output, adjoint from given far fields)."""
    torch = torch_cuda()
    p, _ = custom_problem(780 + variant, 128, 2, 2, 1, 384, 40, weights="opr")
    plan = _plan(p, tune={"variant": variant, "recompute": 1, "grid": 16})
    w = dev(p.weights)
    Psi = plan.apply_A(dev(p.obj), dev(p.probe), dev(p.positions), weights=w)
    ref = oracle.apply_A(p.obj, p.probe, p.positions, weights=p.weights)
    rng = np.random.default_rng(5)
    Y = (rng.standard_normal(ref.shape) + 1j * rng.standard_normal(ref.shape)).astype(np.complex64)
    gO, gU = plan.apply_AH(dev(Y), dev(p.obj), dev(p.probe), dev(p.positions), weights=w)
    torch.cuda.synchronize()
    rO, rU = oracle.apply_AH(Y, p.obj, p.probe, p.positions, weights=p.weights)
    e = (rel_l2(Psi.cpu().numpy(), ref), rel_l2(gO.cpu().numpy(), rO), rel_l2(gU.cpu().numpy(), rU))
    print(f"LDS layout {variant} apply_A {e[0]:.2e} apply_AH obj {e[1]:.2e} probe {e[2]:.2e}", flush=True)
    assert e[0] <= 1e-5 and e[1] <= 1e-4 and e[2] <= 1e-4


@pytest.mark.parametrize("variant", [5, 6])
def test_lds_layouts_drop_bad_positions(variant):
    """A window leaving the object, a non-finite position and a non-finite pattern are
    dropped and latched; the remaining positions match the oracle on them alone."""
    from dataclasses import replace
    from paper_2510_20929_amd import FLAG_BOUNDS, FLAG_NONFINITE
    start, I = custom_problem(790 + variant, 128, 2, 1, 1, 330, 40, loss="amplitude")
    pos = start.positions.copy()
    I = I.copy()
    pos[7] = (330.0 - 1.5, 5.0)          # the window leaves the object
    pos[21, 1] = np.nan
    I[30, 3, 4] = np.nan
    q = replace(start, positions=pos)
    keep = np.array([k for k in range(start.K) if k not in (7, 21, 30)])
    grads = ("obj", "probe", "pos")
    ref = run_oracle(q.subset(keep), I[keep], grads, norm_count=start.K)
    got = run_gpu(_plan(q, tune={"variant": variant, "recompute": 1, "grid": 16}), q, I, grads, want_ipred=False)
    assert got["flags"] & FLAG_BOUNDS and got["flags"] & FLAG_NONFINITE
    assert np.all(got["g_pos"][[7, 21, 30]] == 0)
    got["g_pos"] = got["g_pos"][keep]
    compare(got, ref, grads, tag=f"LDS layout {variant} bad positions")


@pytest.mark.parametrize("recompute", [0, 1])
def test_lds_multislice_config3_structure(recompute):
    """The LDS-resident multislice kernel (variant 5 with several slices), incident waves
    stored or recomputed, with the slice-spacing gradient dL/d(lambda z): config 3
    structure (128^2, 2 modes, weak-phase slices, lambda z = 81.92 px^2) with 3 slices of
    300^2 and 90 positions on 16 workgroups."""
    from gpu_util import case
    start, I = case(3, H=300, K=90, S=3)
    grads = ("obj", "probe", "pos", "lambda_z")
    ref = run_oracle(start, I, grads)
    got = run_gpu(_plan(start, tune={"variant": 5, "recompute": recompute, "grid": 16}), start, I, grads)
    compare(got, ref, grads, tag=f"LDS multislice recompute={recompute}")
    assert got["flags"] == 0
    # without the slice-spacing gradient (the other instantiation)
    grads = ("obj", "probe", "pos")
    got = run_gpu(_plan(start, tune={"variant": 5, "recompute": recompute, "grid": 16}), start, I, grads)
    compare(got, {k: v for k, v in ref.items() if k != "g_lambda_z"}, grads, tag=f"LDS multislice no lz")


@pytest.mark.parametrize("S,M,E,loss", [(2, 1, 1, "poisson"), (4, 2, 2, "amplitude")])
def test_lds_multislice_shapes(S, M, E, loss):
    """Slice counts, modes, OPR eigenprobes with weight gradients and both losses."""
    start, I = custom_problem(840 + S + M, 128, M, E, S, 360, 48, lz=16.0, loss=loss,
                              weights="opr" if E > 1 else None)
    grads = ("obj", "probe", "pos", "lambda_z") + (("weights",) if E > 1 else ())
    ref = run_oracle(start, I, grads)
    got = run_gpu(_plan(start, tune={"variant": 6, "recompute": 0, "grid": 16}), start, I, grads)
    compare(got, ref, grads, tag=f"LDS multislice S={S} M={M} E={E} {loss}")
    assert got["flags"] == 0


def test_lds_multislice_apply_A_AH():
    """The multislice linear map and its adjoint through the LDS-resident kernel."""
    torch = torch_cuda()
    p, _ = custom_problem(860, 128, 2, 1, 3, 384, 30, lz=16.0)
    plan = _plan(p, tune={"variant": 5, "grid": 16})
    Psi = plan.apply_A(dev(p.obj), dev(p.probe), dev(p.positions))
    ref = oracle.apply_A(p.obj, p.probe, p.positions, lambda_z=p.lambda_z)
    rng = np.random.default_rng(7)
    Y = (rng.standard_normal(ref.shape) + 1j * rng.standard_normal(ref.shape)).astype(np.complex64)
    gO, gU = plan.apply_AH(dev(Y), dev(p.obj), dev(p.probe), dev(p.positions))
    torch.cuda.synchronize()
    rO, rU = oracle.apply_AH(Y, p.obj, p.probe, p.positions, lambda_z=p.lambda_z)
    e = (rel_l2(Psi.cpu().numpy(), ref), rel_l2(gO.cpu().numpy(), rO), rel_l2(gU.cpu().numpy(), rU))
    print(f"LDS multislice apply_A {e[0]:.2e} apply_AH obj {e[1]:.2e} probe {e[2]:.2e}", flush=True)
    assert e[0] <= 1e-5 and e[1] <= 1e-4 and e[2] <= 1e-4


@pytest.mark.parametrize("M,E,G,loss", [(4, 1, 2, "poisson"), (4, 1, 4, "amplitude"), (15, 3, 4, "amplitude"),
                                        (5, 2, 2, "poisson")])
def test_lds_mode_split_form(M, E, G, loss):
    """The mode-split form (each position's modes in G groups: forward, loss and adjoint
    launches) with the LDS-resident layout, against the oracle: eigenprobe weights or
    none, groups of unequal size, every gradient, on 8 workgroups (several items each)."""
    start, I = custom_problem(880 + M + E + G, 128, M, E, 1, 384, 20, loss=loss, weights="opr" if E > 1 else None)
    grads = ("obj", "probe", "pos") + (("weights",) if E > 1 else ())
    ref = run_oracle(start, I, grads)
    got = run_gpu(_plan(start, tune={"variant": 5, "mode_groups": G, "grid": 8}), start, I, grads)
    compare(got, ref, grads, tag=f"LDS split M={M} E={E} G={G}")
    assert got["flags"] == 0


def test_lds_mode_split_forward_and_bad_position():
    """Mode-split LDS form: the forward call alone (loss and predicted intensities in the
    column layout's detector mapping), and a position whose window leaves the object
    (latched and dropped, the rest exact)."""
    from dataclasses import replace
    from paper_2510_20929_amd import FLAG_BOUNDS
    torch = torch_cuda()
    start, I = custom_problem(890, 128, 6, 1, 1, 360, 24, loss="poisson")
    plan = _plan(start, tune={"variant": 5, "mode_groups": 3, "grid": 8})
    ipred = torch.zeros((start.K, 128, 128), dtype=torch.float32, device="cuda")
    loss = plan.forward(dev(start.obj), dev(start.probe), dev(start.positions), dev(I), I_pred=ipred)
    torch.cuda.synchronize()
    ref_l, ref_I = oracle.forward(start.obj, start.probe, start.positions, I, loss=start.loss, eps=start.eps)
    compare({"loss": float(loss.cpu()[0]), "I_pred": ipred.cpu().numpy()}, {"loss": ref_l, "I_pred": ref_I}, (),
            tag="LDS split forward")
    pos = start.positions.copy()
    pos[5] = (360.0 - 10.0, 3.0)
    q = replace(start, positions=pos)
    keep = np.array([k for k in range(start.K) if k != 5])
    grads = ("obj", "probe", "pos")
    ref = run_oracle(q.subset(keep), I[keep], grads, norm_count=start.K)
    got = run_gpu(_plan(q, tune={"variant": 5, "mode_groups": 3, "grid": 8}), q, I, grads, want_ipred=False)
    assert got["flags"] & FLAG_BOUNDS
    got["g_pos"] = got["g_pos"][keep]
    compare(got, ref, grads, tag="LDS split bad position")


@pytest.mark.parametrize("variant", [5, 6])
def test_lds_layouts_workgroup_without_finished_position(variant):
    """A workgroup starts its probe-gradient accumulator at its first position whose
    adjoint finishes (written, not added), and one whose positions all drop clears it after
    its last position. 40 positions on 16 workgroups: workgroup 3 (positions 3, 19, 35)
    drops every position (two windows leaving the object, a non-finite pattern), workgroup
    9 drops its first (a non-finite pattern). Two calls in a row on one plan, the second
    finding the first call's accumulators in the scratch, both match the oracle on the
    kept positions."""
    from dataclasses import replace
    from paper_2510_20929_amd import FLAG_BOUNDS, FLAG_NONFINITE
    start, I = custom_problem(795 + variant, 128, 2, 1, 1, 330, 40, loss="amplitude")
    pos = start.positions.copy()
    I = I.copy()
    pos[3] = (330.0 - 1.5, 5.0)
    pos[19] = (5.0, 330.0 - 1.5)
    I[35, 0, 0] = np.nan
    I[9, 2, 2] = np.nan
    q = replace(start, positions=pos)
    drop = [3, 9, 19, 35]
    keep = np.array([k for k in range(start.K) if k not in drop])
    grads = ("obj", "probe", "pos")
    ref = run_oracle(q.subset(keep), I[keep], grads, norm_count=start.K)
    plan = _plan(q, tune={"variant": variant, "recompute": 1, "grid": 16})
    for call in range(2):
        got = run_gpu(plan, q, I, grads, want_ipred=False)
        assert got["flags"] & FLAG_BOUNDS and got["flags"] & FLAG_NONFINITE
        assert np.all(got["g_pos"][drop] == 0)
        got["g_pos"] = got["g_pos"][keep]
        compare(got, ref, grads, tag=f"LDS layout {variant} workgroup without a finished position, call {call}")
