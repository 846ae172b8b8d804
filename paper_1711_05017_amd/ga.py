"""ctypes binding of libga.so (include/ga.h). Argument marshalling only.

Device memory comes from torch tensors (their data_ptr() is passed through)
and work is enqueued on torch's current HIP stream unless a stream is given.
Every numerical step runs in the library's HIP kernels; when the library is
missing, loading fails with an error instead of falling back to anything.
"""

from __future__ import annotations

import ctypes
import os
from typing import Optional

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libga.so")

GA_OK, GA_PENDING = 0, 1
GA_R2C, GA_C2R = -1, 1
GA_FIELDS, GA_SINGLE = 0, 1
GA_OP_FFT_C2R, GA_OP_CORRELATE, GA_OP_ENERGY, GA_OP_FORCE_FIELDS, GA_OP_FORCE_SINGLE = 1, 2, 3, 4, 5

# Every symbol the header declares (checked by the CPU test suite).
EXPORTS = [
    "ga_status_str", "ga_version", "ga_supported_n", "ga_plan_create", "ga_plan_destroy", "ga_plan_n",
    "ga_workspace_size", "ga_splat", "ga_fft3d", "ga_correlate", "ga_energy_fields", "ga_force_torque",
    "ga_profile_enable", "ga_profile_read",
]
GA_K_SPLAT, GA_K_PLANE_FWD, GA_K_STRIP, GA_K_PLANE_INV, GA_K_READOUT, GA_K_BIN = 0, 1, 2, 3, 4, 5
KERNEL_KINDS = {"splat": 0, "plane_fwd": 1, "strip": 2, "plane_inv": 3, "readout": 4, "bin": 5}

_vp = ctypes.c_void_p
_SIGS = {
    "ga_status_str": (ctypes.c_char_p, [ctypes.c_int32]),
    "ga_version": (ctypes.c_char_p, []),
    "ga_supported_n": (ctypes.c_int32, [ctypes.c_int32]),
    "ga_plan_create": (ctypes.c_int32, [ctypes.POINTER(_vp), ctypes.c_int32, ctypes.c_int32, ctypes.c_uint32]),
    "ga_plan_destroy": (ctypes.c_int32, [_vp]),
    "ga_plan_n": (ctypes.c_int32, [_vp]),
    "ga_workspace_size": (ctypes.c_size_t, [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64]),
    "ga_splat": (ctypes.c_int32, [_vp, _vp, _vp, ctypes.c_int64, _vp, _vp, ctypes.c_float, ctypes.c_int32, _vp, _vp]),
    "ga_fft3d": (ctypes.c_int32, [_vp, ctypes.c_int32, _vp, _vp, ctypes.c_int32, _vp, ctypes.c_size_t, _vp]),
    "ga_correlate": (ctypes.c_int32, [_vp, _vp, ctypes.c_int64, _vp, ctypes.c_int32, _vp, _vp, ctypes.c_size_t, _vp]),
    "ga_energy_fields": (ctypes.c_int32, [_vp, _vp, _vp, _vp, ctypes.c_int64, _vp, _vp, ctypes.c_float, ctypes.c_int32,
                                          _vp, _vp, ctypes.c_size_t, _vp]),
    "ga_force_torque": (ctypes.c_int32, [_vp, _vp, _vp, _vp, ctypes.c_int32, ctypes.c_uint32, _vp, _vp, ctypes.c_size_t,
                                         _vp]),
    "ga_profile_enable": (ctypes.c_int32, [_vp, ctypes.c_int32]),
    "ga_profile_read": (ctypes.c_int32, [_vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_int64)]),
}

_lib = None


class GaError(RuntimeError):
    def __init__(self, fn: str, status: int):
        msg = _lib.ga_status_str(status).decode() if _lib is not None else str(status)
        super().__init__(f"{fn} failed: {msg} ({status})")
        self.status = status


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libga.so and declare its signatures. Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libga.so not found at {path}: build it first (python -c 'import __graft_entry__ as g; g.build()')")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(fn: str, status: int):
    if status != GA_OK:
        raise GaError(fn, status)


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream) -> ctypes.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _host_f32(a, count):
    if a is None:
        return None
    flat = [float(v) for v in torch.as_tensor(a, dtype=torch.float32).reshape(-1).tolist()]
    if len(flat) != count:
        raise ValueError(f"expected {count} values")
    return (ctypes.c_float * count)(*flat)


def spectrum_shape(n: int):
    return (n, n, n // 2 + 1)


def _spec_elems(n: int) -> int:
    return n * n * (n // 2 + 1)


def _need(t: torch.Tensor, dtype, min_numel: int, name: str, exact: bool = False):
    """Host-side check that a device buffer holds what the kernels will touch."""
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise ValueError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if (t.numel() != min_numel) if exact else (t.numel() < min_numel):
        raise ValueError(f"{name} has {t.numel()} elements, needs {'exactly ' if exact else ''}{min_numel}")


def _samples(xyzr: torch.Tensor, w: torch.Tensor) -> int:
    if xyzr.dim() != 2 or xyzr.shape[1] != 4:
        raise ValueError("xyzr must be [n_pts, 4]")
    m = int(xyzr.shape[0])
    _need(xyzr, torch.float32, 4 * m, "xyzr", exact=True)
    _need(w, torch.float32, m, "w", exact=True)
    return m


class Plan:
    """A ga_plan for grid edge n on the current device."""

    def __init__(self, n: int, max_batch: int = 1):
        lib = load()
        h = ctypes.c_void_p()
        _check("ga_plan_create", lib.ga_plan_create(ctypes.byref(h), int(n), int(max_batch), 0))
        self._h = h
        self.n = int(n)
        self.max_batch = int(max_batch)

    @property
    def handle(self):
        return self._h

    def workspace(self, op: int, batch: int = 1, n_items: int = 0, device=None) -> torch.Tensor:
        nbytes = load().ga_workspace_size(self._h, op, batch, n_items)
        return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device or "cuda")

    def profile(self, enable: bool = True):
        """Start (and clear) or stop per-kernel event timing."""
        _check("ga_profile_enable", load().ga_profile_enable(self._h, 1 if enable else 0))

    def profile_read(self, kind: int):
        """(total milliseconds, launches) of one kernel kind since profile()."""
        ms = ctypes.c_double()
        cnt = ctypes.c_int64()
        _check("ga_profile_read", load().ga_profile_read(self._h, int(kind), ctypes.byref(ms), ctypes.byref(cnt)))
        return ms.value, cnt.value

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().ga_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ga_supported_n(n: int) -> bool:
    return bool(load().ga_supported_n(int(n)))


def ga_splat(plan: Plan, xyzr: torch.Tensor, w: torch.Tensor, R=None, c=None, sigma: float = 0.5, channels: int = 1,
             out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    n = plan.n
    m = _samples(xyzr, w)
    if out is None:
        out = torch.empty((channels, n, n, n), dtype=torch.float32, device=xyzr.device)
    _need(out, torch.float32, channels * n ** 3, "out")
    st = load().ga_splat(plan.handle, _ptr(xyzr), _ptr(w), m, _host_f32(R, 9), _host_f32(c, 3),
                         float(sigma), int(channels), _ptr(out), _stream(stream))
    _check("ga_splat", st)
    return out


def ga_fft3d(plan: Plan, direction: int, x: torch.Tensor, out: Optional[torch.Tensor] = None, work=None,
             stream=None) -> torch.Tensor:
    n = plan.n
    batch = x.shape[0] if x.dim() == 4 else 1
    if direction == GA_R2C:
        _need(x, torch.float32, batch * n ** 3, "x", exact=True)
        if out is None:
            out = torch.empty((batch, *spectrum_shape(n)), dtype=torch.complex64, device=x.device)
        _need(out, torch.complex64, batch * _spec_elems(n), "out")
    else:
        _need(x, torch.complex64, batch * _spec_elems(n), "x", exact=True)
        if out is None:
            out = torch.empty((batch, n, n, n), dtype=torch.float32, device=x.device)
        _need(out, torch.float32, batch * n ** 3, "out")
        if work is None:
            work = plan.workspace(GA_OP_FFT_C2R, batch, device=x.device)
    st = load().ga_fft3d(plan.handle, int(direction), _ptr(x), _ptr(out), int(batch), _ptr(work),
                         int(work.numel()) if work is not None else 0, _stream(stream))
    _check("ga_fft3d", st)
    return out


def ga_correlate(plan: Plan, Ahat: torch.Tensor, Bhat: torch.Tensor, a_stride: Optional[int] = None,
                 out: Optional[torch.Tensor] = None, work=None, stream=None) -> torch.Tensor:
    n = plan.n
    batch = Bhat.shape[0] if Bhat.dim() == 4 else 1
    if a_stride is None:
        a_stride = 0 if (Ahat.dim() == 3 or Ahat.shape[0] == 1) else _spec_elems(n)
    _need(Bhat, torch.complex64, batch * _spec_elems(n), "Bhat", exact=True)
    _need(Ahat, torch.complex64, a_stride * (batch - 1) + _spec_elems(n), "Ahat")
    if out is None:
        out = torch.empty((batch, n, n, n), dtype=torch.float32, device=Bhat.device)
    _need(out, torch.float32, batch * n ** 3, "out")
    if work is None:
        work = plan.workspace(GA_OP_CORRELATE, batch, device=Bhat.device)
    st = load().ga_correlate(plan.handle, _ptr(Ahat), int(a_stride), _ptr(Bhat), int(batch), _ptr(out), _ptr(work),
                             int(work.numel()), _stream(stream))
    _check("ga_correlate", st)
    return out


def ga_energy_fields(plan: Plan, Ahat: torch.Tensor, xyzr: torch.Tensor, w: torch.Tensor, R: torch.Tensor, c,
                     sigma: float = 0.5, out: Optional[torch.Tensor] = None, work=None, stream=None) -> torch.Tensor:
    n = plan.n
    batch = int(R.shape[0])
    m = _samples(xyzr, w)
    _need(R, torch.float32, 9 * batch, "R", exact=True)
    _need(Ahat, torch.complex64, _spec_elems(n), "Ahat")
    if out is None:
        out = torch.empty((batch, n, n, n), dtype=torch.float32, device=xyzr.device)
    _need(out, torch.float32, batch * n ** 3, "out")
    if work is None:
        work = plan.workspace(GA_OP_ENERGY, batch, m, device=xyzr.device)
    st = load().ga_energy_fields(plan.handle, _ptr(Ahat), _ptr(xyzr), _ptr(w), m, _ptr(R),
                                 _host_f32(c, 3), float(sigma), batch, _ptr(out), _ptr(work), int(work.numel()),
                                 _stream(stream))
    _check("ga_energy_fields", st)
    return out


def ga_force_torque(plan: Plan, Ahat: torch.Tensor, Bhat4: torch.Tensor, t: torch.Tensor, mode: int = GA_FIELDS,
                    out: Optional[torch.Tensor] = None, work=None, stream=None) -> torch.Tensor:
    n = plan.n
    n_poses = int(t.shape[0])
    _need(t, torch.float32, 3 * n_poses, "t", exact=True)
    _need(Ahat, torch.complex64, _spec_elems(n), "Ahat")
    _need(Bhat4, torch.complex64, 4 * _spec_elems(n), "Bhat4")
    if out is None:
        out = torch.empty((n_poses, 7), dtype=torch.float32, device=t.device)
    _need(out, torch.float32, 7 * n_poses, "out")
    if work is None:
        op = GA_OP_FORCE_FIELDS if mode == GA_FIELDS else GA_OP_FORCE_SINGLE
        work = plan.workspace(op, 1, n_poses, device=t.device)
    st = load().ga_force_torque(plan.handle, _ptr(Ahat), _ptr(Bhat4), _ptr(t), n_poses, int(mode), _ptr(out),
                                _ptr(work), int(work.numel()), _stream(stream))
    _check("ga_force_torque", st)
    return out
