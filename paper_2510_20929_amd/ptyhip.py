"""ctypes binding of libptyhip (the C ABI in include/ptyhip.h).

Argument marshalling only: every step of the forward model and its adjoint runs in
the library's HIP kernels. torch supplies device memory and the current stream. If
the shared library has not been built this module raises; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libptyhip.so")

LOSS_AMPLITUDE = 0
LOSS_POISSON = 1
GRAD_OBJ = 1
GRAD_PROBE = 2
GRAD_POS = 4
GRAD_WEIGHTS = 8
ACCUMULATE = 16
PLAIN = 32
GRAD_LAMBDA_Z = 128
PROP_FAR, PROP_NEAR = 0, 1
FLAG_BOUNDS = 1
FLAG_NONFINITE = 2

OK, EINVAL, ESHAPE, EBOUNDS, ENONFINITE, EHIP, ENOMEM, EUNSUPPORTED = range(8)
STATUS = {0: "PTYHIP_OK", 1: "PTYHIP_EINVAL", 2: "PTYHIP_ESHAPE", 3: "PTYHIP_EBOUNDS", 4: "PTYHIP_ENONFINITE",
          5: "PTYHIP_EHIP", 6: "PTYHIP_ENOMEM", 7: "PTYHIP_EUNSUPPORTED"}

EXPORTED = [
    "ptyhip_status_str", "ptyhip_version", "ptyhip_desc_validate", "ptyhip_plan_create", "ptyhip_plan_create_ex",
    "ptyhip_plan_destroy", "ptyhip_plan_get_info", "ptyhip_forward", "ptyhip_forward_adjoint",
    "ptyhip_forward_adjoint_ex", "ptyhip_apply_A",
    "ptyhip_apply_AH", "ptyhip_illumination", "ptyhip_normalize_gradients",
    "ptyhip_orthogonalize_modes", "ptyhip_plan_set_graphs", "ptyhip_plan_set_timing", "ptyhip_plan_kernel_time", "ptyhip_get_error",
    "ptyhip_clear_error", "ptyhip_batch_create", "ptyhip_batch_bind",
    "ptyhip_batch_launch", "ptyhip_batch_get_error", "ptyhip_batch_destroy", "ptyhip_forward_adjoint_static",
]


class Desc(ctypes.Structure):
    _fields_ = [("frame", ctypes.c_int32), ("n_modes", ctypes.c_int32), ("n_eig", ctypes.c_int32),
                ("n_slices", ctypes.c_int32), ("obj_h", ctypes.c_int32), ("obj_w", ctypes.c_int32),
                ("loss", ctypes.c_int32), ("poisson_eps", ctypes.c_float), ("lambda_z", ctypes.c_float),
                ("norm_count", ctypes.c_double), ("propagation", ctypes.c_int32), ("det_lambda_z", ctypes.c_float),
                ("subpixel", ctypes.c_int32)]


class Tune(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("recompute", ctypes.c_int32), ("plain_chunk", ctypes.c_int32), ("mode_groups", ctypes.c_int32),
                ("probe_stage", ctypes.c_int32)]


def make_tune(tune: Optional[dict]) -> Optional["Tune"]:
    """A ``Tune`` from a dict (variant, grid, recompute, plain_chunk, mode_groups, probe_stage;
    missing = 0)."""
    if not tune:
        return None
    return Tune(*[int(tune.get(f, 0)) for f, _ in Tune._fields_])


class PlanInfo(ctypes.Structure):
    _fields_ = [("workspace_bytes", ctypes.c_size_t), ("scratch_bytes", ctypes.c_size_t),
                ("window_bytes", ctypes.c_size_t), ("plain_bytes", ctypes.c_size_t), ("grid", ctypes.c_int32), ("threads", ctypes.c_int32),
                ("fused_on_chip", ctypes.c_int32), ("plain_chunk", ctypes.c_int32)]


class PtyhipError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {STATUS.get(status, status)} ({_lib().ptyhip_status_str(status).decode()})")


_LIB = None
_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_u32 = ctypes.c_uint32


def _lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(there is no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        L.ptyhip_status_str.restype = ctypes.c_char_p
        L.ptyhip_status_str.argtypes = [ctypes.c_int]
        L.ptyhip_version.restype = ctypes.c_char_p
        L.ptyhip_desc_validate.argtypes = [ctypes.POINTER(Desc)]
        L.ptyhip_plan_create.argtypes = [ctypes.POINTER(Desc), _i32, ctypes.POINTER(_vp)]
        L.ptyhip_plan_create_ex.argtypes = [ctypes.POINTER(Desc), _i32, ctypes.POINTER(Tune), ctypes.POINTER(_vp)]
        L.ptyhip_plan_destroy.argtypes = [_vp]
        L.ptyhip_plan_destroy.restype = None
        L.ptyhip_plan_get_info.argtypes = [_vp, ctypes.POINTER(PlanInfo)]
        L.ptyhip_forward.argtypes = [_vp, _vp, _i32] + [_vp] * 7
        L.ptyhip_forward_adjoint.argtypes = [_vp, _vp, _i32, _u32] + [_vp] * 11
        L.ptyhip_apply_A.argtypes = [_vp, _vp, _i32] + [_vp] * 5
        L.ptyhip_apply_AH.argtypes = [_vp, _vp, _i32] + [_vp] * 7
        L.ptyhip_plan_set_graphs.argtypes = [_vp, _i32]
        L.ptyhip_plan_set_timing.argtypes = [_vp, _i32]
        L.ptyhip_plan_kernel_time.argtypes = [_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_i32)]
        L.ptyhip_get_error.argtypes = [_vp, _vp, ctypes.POINTER(_u32)]
        L.ptyhip_clear_error.argtypes = [_vp, _vp]
        L.ptyhip_batch_create.argtypes = [ctypes.POINTER(Desc), ctypes.POINTER(_i32), _i32, ctypes.POINTER(Tune),
                                          ctypes.POINTER(_vp)]
        L.ptyhip_batch_bind.argtypes = [_vp, _i32] + [_vp] * 10
        L.ptyhip_batch_launch.argtypes = [_vp, _vp, _u32]
        L.ptyhip_batch_get_error.argtypes = [_vp, _vp, ctypes.POINTER(_u32)]
        L.ptyhip_forward_adjoint_static.argtypes = [ctypes.POINTER(Desc), ctypes.POINTER(Tune), _vp, _i32, _u32] + \
            [_vp] * 12
        L.ptyhip_batch_destroy.argtypes = [_vp]
        L.ptyhip_batch_destroy.restype = None
        for name in EXPORTED:
            if name not in ("ptyhip_status_str", "ptyhip_version", "ptyhip_plan_destroy", "ptyhip_batch_destroy"):
                getattr(L, name).restype = ctypes.c_int
        _LIB = L
    return _LIB


def lib():
    """The loaded shared library (raises if it has not been built)."""
    return _lib()


def _check(status: int, what: str):
    if status != 0:
        raise PtyhipError(status, what)


def make_desc(frame, n_modes=1, n_eig=1, n_slices=1, obj_h=0, obj_w=0, loss="amplitude", poisson_eps=1e-3,
              lambda_z=0.0, norm_count=0.0, det_lambda_z=None, subpixel="bilinear") -> Desc:
    """det_lambda_z=None: far-field detector; a number: near-field (Fresnel) detector.
    subpixel: "bilinear" or "fourier" (shift theorem on the integer window)."""
    lc = {"amplitude": LOSS_AMPLITUDE, "poisson": LOSS_POISSON}.get(loss, loss)
    near = det_lambda_z is not None
    return Desc(int(frame), int(n_modes), int(n_eig), int(n_slices), int(obj_h), int(obj_w), int(lc),
                float(poisson_eps), float(lambda_z), float(norm_count), PROP_NEAR if near else PROP_FAR,
                float(det_lambda_z) if near else 0.0, {"bilinear": 0, "fourier": 1}.get(subpixel, subpixel))


def ptyhip_desc_validate(desc: Desc) -> int:
    """Pure host check of a description (returns the status code)."""
    return int(_lib().ptyhip_desc_validate(ctypes.byref(desc)))


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _need(t, name, dtype, shape=None):
    if t is None:
        raise ValueError(f"{name} is required")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t


class Plan:
    """A ptyhip plan for one problem shape (owns the library workspace)."""

    def __init__(self, frame, n_modes=1, n_eig=1, n_slices=1, obj_h=0, obj_w=0, loss="amplitude",
                 poisson_eps=1e-3, lambda_z=0.0, norm_count=0.0, max_positions=1, tune: Optional[dict] = None,
                 det_lambda_z=None, subpixel="bilinear"):
        self.desc = make_desc(frame, n_modes, n_eig, n_slices, obj_h, obj_w, loss, poisson_eps, lambda_z, norm_count,
                              det_lambda_z, subpixel)
        self.max_positions = int(max_positions)
        h = ctypes.c_void_p()
        if tune:
            tu = make_tune(tune)
            st = _lib().ptyhip_plan_create_ex(ctypes.byref(self.desc), self.max_positions, ctypes.byref(tu),
                                              ctypes.byref(h))
        else:
            st = _lib().ptyhip_plan_create(ctypes.byref(self.desc), self.max_positions, ctypes.byref(h))
        _check(st, "ptyhip_plan_create")
        self._h = h
        self.N, self.M, self.E, self.S = int(frame), int(n_modes), int(n_eig), int(n_slices)
        self.H, self.W = int(obj_h), int(obj_w)

    @classmethod
    def for_problem(cls, prob, max_positions=None, norm_count=0.0, tune=None):
        """Plan sized for a synthetic ``synth.Problem``-like object."""
        return cls(prob.N, prob.M, prob.E, prob.S, prob.H, prob.W, prob.loss, prob.eps, prob.lambda_z, norm_count,
                   max_positions or prob.K, tune, getattr(prob, "det_lambda_z", None),
                   getattr(prob, "subpixel", "bilinear"))

    def close(self):
        if getattr(self, "_h", None):
            _lib().ptyhip_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> Dict[str, int]:
        inf = PlanInfo()
        _check(_lib().ptyhip_plan_get_info(self._h, ctypes.byref(inf)), "ptyhip_plan_get_info")
        return {f: getattr(inf, f) for f, _ in PlanInfo._fields_}

    # -------------------------------------------------------------------------- checks
    def _inputs(self, obj, probe, positions, weights):
        K = int(positions.shape[0])
        _need(obj, "obj", torch.complex64, (self.S, self.H, self.W))
        _need(probe, "probe", torch.complex64, (self.E, self.M, self.N, self.N))
        _need(positions, "positions", torch.float32, (K, 2))
        if weights is not None:
            _need(weights, "weights", torch.float32, (K, self.E))
        return K

    # -------------------------------------------------------------------------- calls
    def forward(self, obj, probe, positions, I_meas, weights=None, I_pred=None, loss=None, stream=None):
        K = self._inputs(obj, probe, positions, weights)
        _need(I_meas, "I_meas", torch.float32, (K, self.N, self.N))
        if loss is None:
            loss = torch.zeros(1, dtype=torch.float64, device=obj.device)
        if I_pred is not None:
            _need(I_pred, "I_pred", torch.float32, (K, self.N, self.N))
        st = _lib().ptyhip_forward(self._h, _stream(stream), K, _ptr(obj), _ptr(probe), _ptr(weights),
                                   _ptr(positions), _ptr(I_meas), _ptr(loss), _ptr(I_pred))
        _check(st, "ptyhip_forward")
        return loss

    def forward_adjoint(self, obj, probe, positions, I_meas, weights=None, grads: Sequence[str] = ("obj", "probe"),
                        accumulate=False, plain=False, out: Optional[dict] = None, I_pred=None, stream=None):
        K = self._inputs(obj, probe, positions, weights)
        _need(I_meas, "I_meas", torch.float32, (K, self.N, self.N))
        dev = obj.device
        out = dict(out or {})
        if "loss" not in out:
            out["loss"] = torch.zeros(1, dtype=torch.float64, device=dev)
        flags = 0
        if "obj" in grads:
            flags |= GRAD_OBJ
            if "g_obj" not in out:
                out["g_obj"] = torch.zeros((self.S, self.H, self.W), dtype=torch.complex64, device=dev)
        if "probe" in grads:
            flags |= GRAD_PROBE
            if "g_probe" not in out:
                out["g_probe"] = torch.zeros((self.E, self.M, self.N, self.N), dtype=torch.complex64, device=dev)
        if "pos" in grads:
            flags |= GRAD_POS
            if "g_pos" not in out:
                out["g_pos"] = torch.zeros((K, 2), dtype=torch.float32, device=dev)
        if "weights" in grads:
            flags |= GRAD_WEIGHTS
            if "g_weights" not in out:
                out["g_weights"] = torch.zeros((K, self.E), dtype=torch.float32, device=dev)
        if "lambda_z" in grads:
            flags |= GRAD_LAMBDA_Z
            if "g_lambda_z" not in out:
                out["g_lambda_z"] = torch.zeros(1, dtype=torch.float64, device=dev)
        if accumulate:
            flags |= ACCUMULATE
        if plain:
            flags |= PLAIN
        if I_pred is not None:
            _need(I_pred, "I_pred", torch.float32, (K, self.N, self.N))
            out["I_pred"] = I_pred
        st = _lib().ptyhip_forward_adjoint_ex(
            self._h, _stream(stream), K, flags, _ptr(obj), _ptr(probe), _ptr(weights), _ptr(positions),
            _ptr(I_meas), _ptr(out["loss"]), _ptr(I_pred), _ptr(out.get("g_obj")), _ptr(out.get("g_probe")),
            _ptr(out.get("g_pos")), _ptr(out.get("g_weights")), _ptr(out.get("g_lambda_z")))
        _check(st, "ptyhip_forward_adjoint")
        return out

    def apply_A(self, obj, probe, positions, weights=None, Psi=None, stream=None):
        K = self._inputs(obj, probe, positions, weights)
        if Psi is None:
            Psi = torch.empty((K, self.M, self.N, self.N), dtype=torch.complex64, device=obj.device)
        _need(Psi, "Psi", torch.complex64, (K, self.M, self.N, self.N))
        st = _lib().ptyhip_apply_A(self._h, _stream(stream), K, _ptr(obj), _ptr(probe), _ptr(weights),
                                   _ptr(positions), _ptr(Psi))
        _check(st, "ptyhip_apply_A")
        return Psi

    def apply_AH(self, Y, obj, probe, positions, weights=None, want=("obj", "probe"), stream=None):
        K = self._inputs(obj, probe, positions, weights)
        _need(Y, "Y", torch.complex64, (K, self.M, self.N, self.N))
        dev = obj.device
        g_obj = torch.empty((self.S, self.H, self.W), dtype=torch.complex64, device=dev) if "obj" in want else None
        g_probe = (torch.empty((self.E, self.M, self.N, self.N), dtype=torch.complex64, device=dev)
                   if "probe" in want else None)
        st = _lib().ptyhip_apply_AH(self._h, _stream(stream), K, _ptr(Y), _ptr(obj), _ptr(probe), _ptr(weights),
                                    _ptr(positions), _ptr(g_obj), _ptr(g_probe))
        _check(st, "ptyhip_apply_AH")
        return g_obj, g_probe

    def illumination(self, probe, positions, weights=None, out=None, accumulate=False, stream=None):
        """Probe intensity superimposed in the object frame, [H][W] float32."""
        K = int(positions.shape[0])
        _need(probe, "probe", torch.complex64, (self.E, self.M, self.N, self.N))
        _need(positions, "positions", torch.float32, (K, 2))
        if weights is not None:
            _need(weights, "weights", torch.float32, (K, self.E))
        if out is None:
            out = torch.empty((self.H, self.W), dtype=torch.float32, device=probe.device)
        _need(out, "illum", torch.float32, (self.H, self.W))
        st = _lib().ptyhip_illumination(self._h, _stream(stream), K, ACCUMULATE if accumulate else 0, _ptr(probe),
                                        _ptr(weights), _ptr(positions), _ptr(out))
        _check(st, "ptyhip_illumination")
        return out

    def normalize_gradients(self, K, probe=None, obj=None, weights=None, g_obj=None, g_probe=None, stream=None):
        """In place: g_obj *= K_norm N^2 / max probe intensity, g_probe *= K_norm N^2 / max |O|^2."""
        if g_obj is not None:
            _need(g_obj, "g_obj", torch.complex64, (self.S, self.H, self.W))
            _need(probe, "probe", torch.complex64, (self.E, self.M, self.N, self.N))
        if g_probe is not None:
            _need(g_probe, "g_probe", torch.complex64, (self.E, self.M, self.N, self.N))
            _need(obj, "obj", torch.complex64, (self.S, self.H, self.W))
        if weights is not None:
            _need(weights, "weights", torch.float32, (int(K), self.E))
        st = _lib().ptyhip_normalize_gradients(self._h, _stream(stream), int(K), _ptr(probe), _ptr(weights),
                                               _ptr(obj), _ptr(g_obj), _ptr(g_probe))
        _check(st, "ptyhip_normalize_gradients")
        return g_obj, g_probe

    def orthogonalize_modes(self, probe, out=None, stream=None):
        """Orthogonalised probe modes (strongest first) and their powers (float64 [M])."""
        _need(probe, "probe", torch.complex64, (self.E, self.M, self.N, self.N))
        if out is None:
            out = torch.empty_like(probe)
        _need(out, "probe_out", torch.complex64, (self.E, self.M, self.N, self.N))
        powers = torch.empty(self.M, dtype=torch.float64, device=probe.device)
        st = _lib().ptyhip_orthogonalize_modes(self._h, _stream(stream), _ptr(probe), _ptr(out), _ptr(powers))
        _check(st, "ptyhip_orthogonalize_modes")
        return out, powers

    def set_graphs(self, enable: bool = True):
        """Replay repeated calls (same tensors, K and flags) from captured hipGraphs."""
        _check(_lib().ptyhip_plan_set_graphs(self._h, 1 if enable else 0), "ptyhip_plan_set_graphs")

    def set_timing(self, enable: bool = True):
        _check(_lib().ptyhip_plan_set_timing(self._h, 1 if enable else 0), "ptyhip_plan_set_timing")

    def kernel_time(self):
        """(summed milliseconds, launches) of the main kernel since the last read."""
        ms = ctypes.c_double(0.0)
        n = ctypes.c_int32(0)
        _check(_lib().ptyhip_plan_kernel_time(self._h, ctypes.byref(ms), ctypes.byref(n)), "ptyhip_plan_kernel_time")
        return float(ms.value), int(n.value)

    def get_error(self, stream=None) -> int:
        f = ctypes.c_uint32(0)
        _check(_lib().ptyhip_get_error(self._h, _stream(stream), ctypes.byref(f)), "ptyhip_get_error")
        return int(f.value)

    def clear_error(self, stream=None):
        _check(_lib().ptyhip_clear_error(self._h, _stream(stream)), "ptyhip_clear_error")


BATCH_PER_CALL = 64


class Batch:
    """Many independent datasets (uneven frame sizes) run together: one persistent
    launch captured in a hipGraph (default), or one call per dataset."""

    def __init__(self, problems, tune: Optional[dict] = None):
        descs = (Desc * len(problems))(*[make_desc(p.N, p.M, p.E, p.S, p.H, p.W, p.loss, p.eps, p.lambda_z)
                                        for p in problems])
        Ks = (_i32 * len(problems))(*[int(p.K) for p in problems])
        h = ctypes.c_void_p()
        tu = None
        if tune:
            tu = ctypes.byref(make_tune(tune))
        _check(_lib().ptyhip_batch_create(descs, Ks, len(problems), tu, ctypes.byref(h)), "ptyhip_batch_create")
        self._h = h
        self.n = len(problems)
        self.shapes = [(p.N, p.M, p.E, p.S, p.H, p.W, p.K) for p in problems]
        self._keep = [None] * self.n

    def bind(self, i, obj, probe, positions, I_meas, weights=None, out: Optional[dict] = None):
        """Bind dataset i's device tensors; returns the output dict (allocated if absent)."""
        N, M, E, S, H, W, K = self.shapes[i]
        dev = obj.device
        out = dict(out or {})
        out.setdefault("loss", torch.zeros(1, dtype=torch.float64, device=dev))
        out.setdefault("g_obj", torch.zeros((S, H, W), dtype=torch.complex64, device=dev))
        out.setdefault("g_probe", torch.zeros((E, M, N, N), dtype=torch.complex64, device=dev))
        out.setdefault("g_pos", torch.zeros((K, 2), dtype=torch.float32, device=dev))
        if weights is not None:
            out.setdefault("g_weights", torch.zeros((K, E), dtype=torch.float32, device=dev))
        st = _lib().ptyhip_batch_bind(self._h, i, _ptr(obj), _ptr(probe), _ptr(weights), _ptr(positions),
                                      _ptr(I_meas), _ptr(out["loss"]), _ptr(out["g_obj"]), _ptr(out["g_probe"]),
                                      _ptr(out["g_pos"]), _ptr(out.get("g_weights")))
        _check(st, "ptyhip_batch_bind")
        self._keep[i] = (obj, probe, positions, I_meas, weights, out)
        return out

    def launch(self, grads=("obj", "probe", "pos"), per_call=False, plain=False, stream=None):
        flags = 0
        for g, f in (("obj", GRAD_OBJ), ("probe", GRAD_PROBE), ("pos", GRAD_POS), ("weights", GRAD_WEIGHTS)):
            if g in grads:
                flags |= f
        if per_call:
            flags |= BATCH_PER_CALL
        if plain:
            flags |= PLAIN
        _check(_lib().ptyhip_batch_launch(self._h, _stream(stream), flags), "ptyhip_batch_launch")

    def get_error(self, stream=None) -> int:
        f = ctypes.c_uint32(0)
        _check(_lib().ptyhip_batch_get_error(self._h, _stream(stream), ctypes.byref(f)), "ptyhip_batch_get_error")
        return int(f.value)

    def close(self):
        if getattr(self, "_h", None):
            _lib().ptyhip_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def forward_adjoint_static(desc: Desc, obj, probe, positions, I_meas, weights=None,
                           grads: Sequence[str] = ("obj", "probe"), tune: Optional[dict] = None,
                           accumulate=False, out: Optional[dict] = None, I_pred=None, stream=None):
    """``Plan.forward_adjoint`` without a plan (``ptyhip_forward_adjoint_static``): the
    library allocates nothing; its buffers come from a fixed device array. ``desc`` is a
    ``make_desc`` description. The output dict also holds ``flags`` (device uint32, the
    call's error latch). Outputs missing from ``out`` are allocated here, by torch, before
    the call."""
    N, M, E = int(desc.frame), int(desc.n_modes), int(desc.n_eig)
    K = int(positions.shape[0])
    _need(obj, "obj", torch.complex64, (int(desc.n_slices), int(desc.obj_h), int(desc.obj_w)))
    _need(probe, "probe", torch.complex64, (E, M, N, N))
    _need(positions, "positions", torch.float32, (K, 2))
    _need(I_meas, "I_meas", torch.float32, (K, N, N))
    if weights is not None:
        _need(weights, "weights", torch.float32, (K, E))
    dev = obj.device
    out = dict(out or {})
    out.setdefault("loss", torch.zeros(1, dtype=torch.float64, device=dev))
    out.setdefault("flags", torch.zeros(1, dtype=torch.int32, device=dev))
    flags = 0
    shapes = {"obj": ("g_obj", GRAD_OBJ, (int(desc.n_slices), int(desc.obj_h), int(desc.obj_w)), torch.complex64),
              "probe": ("g_probe", GRAD_PROBE, (E, M, N, N), torch.complex64),
              "pos": ("g_pos", GRAD_POS, (K, 2), torch.float32),
              "weights": ("g_weights", GRAD_WEIGHTS, (K, E), torch.float32)}
    for g in grads:
        key, bit, shape, dt = shapes[g]
        flags |= bit
        if key not in out:
            out[key] = torch.zeros(shape, dtype=dt, device=dev)
    if accumulate:
        flags |= ACCUMULATE
    if I_pred is not None:
        _need(I_pred, "I_pred", torch.float32, (K, N, N))
        out["I_pred"] = I_pred
    tu = ctypes.byref(make_tune(tune)) if tune else None
    st = _lib().ptyhip_forward_adjoint_static(
        ctypes.byref(desc), tu, _stream(stream), K, flags, _ptr(obj), _ptr(probe), _ptr(weights), _ptr(positions),
        _ptr(I_meas), _ptr(out["loss"]), _ptr(I_pred), _ptr(out.get("g_obj")), _ptr(out.get("g_probe")),
        _ptr(out.get("g_pos")), _ptr(out.get("g_weights")), _ptr(out["flags"]))
    _check(st, "ptyhip_forward_adjoint_static")
    return out
