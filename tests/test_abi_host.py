"""Host-side checks that need no GPU: the library loads, exports every symbol the
header declares, and validates descriptions without touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ptyhip.h")


def _lib():
    from paper_2510_20929_amd import ptyhip
    if not os.path.exists(ptyhip.LIB_PATH):
        pytest.skip("library not built")
    return ptyhip


def test_exports_every_declared_symbol():
    mod = _lib()
    decl = set(re.findall(r"\b(ptyhip_[a-z_A-Z]+)\s*\(", open(HEADER).read()))
    decl = {d for d in decl if not d.endswith("_t")}
    L = ctypes.CDLL(mod.LIB_PATH)
    missing = [d for d in sorted(decl) if not hasattr(L, d)]
    assert not missing, missing
    assert set(mod.EXPORTED) == decl


@pytest.mark.parametrize("kw,status", [
    (dict(frame=128, n_modes=4, obj_h=1024, obj_w=1024), 0),
    (dict(frame=100, obj_h=200, obj_w=200), 7),
    (dict(frame=8, obj_h=200, obj_w=200), 7),
    (dict(frame=64, n_modes=0, obj_h=200, obj_w=200), 1),
    (dict(frame=64, n_eig=17, obj_h=200, obj_w=200), 1),
    (dict(frame=64, n_slices=0, obj_h=200, obj_w=200), 1),
    (dict(frame=64, obj_h=63, obj_w=200), 2),
    (dict(frame=64, obj_h=200, obj_w=200, loss=5), 7),
    (dict(frame=64, obj_h=200, obj_w=200, poisson_eps=float("nan")), 4),
    (dict(frame=64, obj_h=200, obj_w=200, poisson_eps=-1.0), 4),
    (dict(frame=256, n_slices=2, obj_h=600, obj_w=600), 0),                    # multislice 256^2: per-step form
    (dict(frame=128, obj_h=300, obj_w=300, det_lambda_z=40.0), 0),            # near field
    (dict(frame=128, obj_h=300, obj_w=300, det_lambda_z=0.0), 0),
    (dict(frame=256, obj_h=600, obj_w=600, det_lambda_z=40.0), 0),            # near field of 256^2: per-step form
    (dict(frame=64, n_slices=2, obj_h=200, obj_w=200, det_lambda_z=40.0), 7),  # and one slice
    (dict(frame=64, obj_h=200, obj_w=200, det_lambda_z=float("inf")), 4),
    (dict(frame=128, obj_h=300, obj_w=300, subpixel="fourier"), 0),
    (dict(frame=256, obj_h=600, obj_w=600, subpixel="fourier"), 0),            # Fourier shift of 256^2: per-step form
    (dict(frame=64, n_slices=3, obj_h=200, obj_w=200, subpixel="fourier"), 7), # Fourier shift needs one slice
    (dict(frame=64, obj_h=200, obj_w=200, det_lambda_z=5.0, subpixel="fourier"), 7),  # and the far field
    (dict(frame=64, obj_h=200, obj_w=200, subpixel=3), 1),
    (dict(frame=512, obj_h=600, obj_w=600000), 2),                           # window span over 2^31 bytes
    (dict(frame=128, obj_h=600, obj_w=600000), 0),
])
def test_desc_validate(kw, status):
    mod = _lib()
    assert mod.ptyhip_desc_validate(mod.make_desc(**kw)) == status


def test_desc_rejects_unknown_propagation():
    mod = _lib()
    d = mod.make_desc(frame=64, obj_h=200, obj_w=200)
    d.propagation = 2
    assert mod.ptyhip_desc_validate(d) == 1


def test_status_strings_and_version():
    mod = _lib()
    L = mod.lib()
    assert L.ptyhip_version().startswith(b"ptyhip")
    for s in range(8):
        assert len(L.ptyhip_status_str(s)) > 0


@pytest.mark.parametrize("frame,variant,status,kw", [
    (128, 7, 1, {}), (64, 5, 1, {}), (256, 2, 1, {}), (512, 4, 1, {}), (64, -1, 1, {}),
    (128, 5, 7, {"det_lambda_z": 100.0}), (128, 6, 7, {"subpixel": "fourier"})])
def test_plan_rejects_tune_outside_the_layouts(frame, variant, status, kw):
    """Implementation choices outside a frame size's layouts are refused before any
    device memory is touched (0-4 on chip, 5-6 only at 128^2 with the far field and the
    bilinear patch, 0-1 for the four-step frames)."""
    mod = _lib()
    L = mod.lib()
    d = mod.make_desc(frame=frame, obj_h=3 * frame, obj_w=3 * frame, **kw)
    t = mod.Tune(variant=variant)
    h = ctypes.c_void_p(1)
    assert L.ptyhip_plan_create_ex(ctypes.byref(d), 10, ctypes.byref(t), ctypes.byref(h)) == status
    assert h.value is None


@pytest.mark.parametrize("variant,status", [(5, 1), (6, 1), (-1, 1)])
def test_static_entry_point_refuses_layouts_it_does_not_run(variant, status):
    """The allocation-free entry point runs the register-resident on-chip layouts 0-4 only;
    other tune variants are refused before any device call (non-null dummy pointers: the
    call returns before it would read them)."""
    mod = _lib()
    L = mod.lib()
    d = mod.make_desc(frame=128, n_modes=2, obj_h=400, obj_w=400)
    t = mod.Tune(variant=variant)
    dummy = ctypes.c_void_p(16)
    st = L.ptyhip_forward_adjoint_static(ctypes.byref(d), ctypes.byref(t), None, 4, 3, dummy, dummy, None, dummy,
                                         dummy, dummy, None, None, None, None, None, None)
    assert st == status
