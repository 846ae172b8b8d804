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
GA_OP_FIELD_GRAD, GA_OP_POSE_LOCAL, GA_OP_SCORE, GA_OP_POSE_SPECTRAL = 6, 7, 8, 9
GA_SCORE_RE, GA_SCORE_IM = 1, 2
GA_SERVE_LOCAL, GA_SERVE_SPECTRAL = 0, 1
GA_PLAN_AXIS_PASSES = 1
GA_LOWPASS_COARSE, GA_LOWPASS_ZEROPAD = 0, 1

# Every symbol the header declares (checked by the CPU test suite).
EXPORTS = [
    "ga_status_str", "ga_version", "ga_supported_n", "ga_plan_create", "ga_plan_destroy", "ga_plan_n",
    "ga_workspace_size", "ga_splat", "ga_fft3d", "ga_correlate", "ga_energy_fields", "ga_force_torque",
    "ga_field_grad", "ga_pose_local", "ga_profile_enable", "ga_profile_read",
    "ga_server_create", "ga_server_destroy", "ga_pair_register", "ga_pair_release", "ga_submit", "ga_poll",
    "ga_server_get_stats", "ga_batch_create", "ga_batch_launch", "ga_batch_destroy",
    "ga_plan_autotune", "ga_plan_set_tuning", "ga_plan_get_tuning", "ga_lowpass",
    "ga_spectral_rotate", "ga_field_table", "ga_field_table_query", "ga_score", "ga_plan_set_overlap",
    "ga_plan_get_overlap", "ga_force_torque_noalloc", "ga_pose_prepare", "ga_pose_spectral",
    "ga_spectral_pack4", "ga_spectral_rotate_packed", "ga_plan_tune", "ga_plan_set_radix", "ga_plan_get_radix",
    "ga_plan_has_alt_radix",
]
GA_K_SPLAT, GA_K_PLANE_FWD, GA_K_STRIP, GA_K_PLANE_INV, GA_K_READOUT, GA_K_BIN = 0, 1, 2, 3, 4, 5
KERNEL_KINDS = {"splat": 0, "plane_fwd": 1, "strip": 2, "plane_inv": 3, "readout": 4, "bin": 5}

_vp = ctypes.c_void_p


MockQueryFn = ctypes.CFUNCTYPE(ctypes.c_int32, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_int32,
                               ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_int32),
                               ctypes.POINTER(ctypes.c_float))


class ServerCfg(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("hbm_budget_bytes", ctypes.c_uint64), ("max_slots", ctypes.c_int32),
                ("queue_depth", ctypes.c_int32), ("mode", ctypes.c_uint32), ("mock_fn", MockQueryFn),
                ("mock_user", ctypes.c_void_p), ("mock_launch_us", ctypes.c_uint32)]


class PartDesc(ctypes.Structure):
    _fields_ = [("xyzr", ctypes.c_void_p), ("w", ctypes.c_void_p), ("n_pts", ctypes.c_int64)]


class Result(ctypes.Structure):
    _fields_ = [("E", ctypes.c_float), ("F", ctypes.c_float * 3), ("tau", ctypes.c_float * 3),
                ("t_submit_ns", ctypes.c_uint64), ("t_start_ns", ctypes.c_uint64), ("t_done_ns", ctypes.c_uint64)]

    def values(self):
        return [self.E, *self.F, *self.tau]


class BatchItem(ctypes.Structure):
    _fields_ = [("plan", ctypes.c_void_p), ("d_Ahat", ctypes.c_void_p), ("d_xyzr", ctypes.c_void_p),
                ("d_w", ctypes.c_void_p), ("n_pts", ctypes.c_int64), ("d_R", ctypes.c_void_p),
                ("c", ctypes.c_float * 3), ("sigma", ctypes.c_float), ("batch", ctypes.c_int32),
                ("d_E", ctypes.c_void_p), ("d_work", ctypes.c_void_p), ("work_bytes", ctypes.c_size_t)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("launches", ctypes.c_uint64),
                ("rejected_full", ctypes.c_uint64), ("bytes_in_use", ctypes.c_uint64), ("pairs", ctypes.c_int32)]


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
    "ga_plan_set_overlap": (ctypes.c_int32, [_vp, ctypes.c_int32]),
    "ga_plan_get_overlap": (ctypes.c_int32, [_vp]),
    "ga_score": (ctypes.c_int32, [_vp, _vp, ctypes.c_int64, _vp, ctypes.c_int32, ctypes.c_uint32, _vp, _vp,
                                  ctypes.c_size_t, _vp]),
    "ga_energy_fields": (ctypes.c_int32, [_vp, _vp, _vp, _vp, ctypes.c_int64, _vp, _vp, ctypes.c_float, ctypes.c_int32,
                                          _vp, _vp, ctypes.c_size_t, _vp]),
    "ga_force_torque": (ctypes.c_int32, [_vp, _vp, _vp, _vp, ctypes.c_int32, ctypes.c_uint32, _vp, _vp, ctypes.c_size_t,
                                         _vp]),
    "ga_force_torque_noalloc": (ctypes.c_int32, [_vp, _vp, _vp, _vp, ctypes.c_int32, _vp, _vp]),
    "ga_field_grad": (ctypes.c_int32, [_vp, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]),
    "ga_pose_prepare": (ctypes.c_int32, [_vp, _vp, _vp, _vp]),
    "ga_pose_spectral": (ctypes.c_int32, [_vp, _vp, _vp, _vp, ctypes.c_int64, _vp, _vp, ctypes.c_float, _vp,
                                          ctypes.c_int32, _vp, _vp, ctypes.c_size_t, _vp]),
    "ga_pose_local": (ctypes.c_int32, [_vp, _vp, _vp, _vp, ctypes.c_int64, _vp, _vp, ctypes.c_float, _vp,
                                       ctypes.c_int32, _vp, _vp, ctypes.c_size_t, _vp]),
    "ga_profile_enable": (ctypes.c_int32, [_vp, ctypes.c_int32]),
    "ga_server_create": (ctypes.c_int32, [ctypes.POINTER(_vp), ctypes.POINTER(ServerCfg)]),
    "ga_server_destroy": (ctypes.c_int32, [_vp]),
    "ga_pair_register": (ctypes.c_int32, [_vp, ctypes.POINTER(PartDesc), ctypes.POINTER(PartDesc),
                                          ctypes.POINTER(ctypes.c_float), ctypes.c_int32, ctypes.c_float,
                                          ctypes.POINTER(ctypes.c_uint32)]),
    "ga_pair_release": (ctypes.c_int32, [_vp, ctypes.c_uint32]),
    "ga_submit": (ctypes.c_int32, [_vp, ctypes.c_uint32, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float),
                                   ctypes.POINTER(ctypes.c_uint64)]),
    "ga_poll": (ctypes.c_int32, [_vp, ctypes.c_uint64, ctypes.POINTER(Result)]),
    "ga_server_get_stats": (ctypes.c_int32, [_vp, ctypes.POINTER(ServerStats)]),
    "ga_field_table": (ctypes.c_int32, [_vp, _vp, _vp, ctypes.c_int32, _vp, _vp, ctypes.c_size_t, _vp]),
    "ga_field_table_query": (ctypes.c_int32, [_vp, _vp, ctypes.c_int32, _vp, _vp, ctypes.c_int32, _vp, _vp]),
    "ga_spectral_rotate": (ctypes.c_int32, [_vp, _vp, ctypes.c_int32, _vp, ctypes.c_int32, _vp, _vp]),
    "ga_spectral_pack4": (ctypes.c_int32, [_vp, _vp, _vp, _vp]),
    "ga_plan_set_radix": (ctypes.c_int32, [_vp, ctypes.c_int32]),
    "ga_plan_get_radix": (ctypes.c_int32, [_vp]),
    "ga_plan_has_alt_radix": (ctypes.c_int32, [_vp]),
    "ga_plan_tune": (ctypes.c_int32, [_vp, _vp, _vp, _vp, ctypes.c_int64, _vp, _vp, ctypes.c_float, ctypes.c_int32,
                                      _vp, _vp, ctypes.c_size_t, ctypes.c_uint32, ctypes.c_char_p, _vp, _vp]),
    "ga_spectral_rotate_packed": (ctypes.c_int32, [_vp, _vp, _vp, ctypes.c_int32, _vp, _vp]),
    "ga_lowpass": (ctypes.c_int32, [_vp, ctypes.c_int32, ctypes.c_uint32, _vp, _vp, ctypes.c_int32, ctypes.c_float,
                                    _vp]),
    "ga_plan_autotune": (ctypes.c_int32, [_vp, _vp, ctypes.c_int32, _vp, ctypes.c_size_t, _vp,
                                          ctypes.POINTER(ctypes.c_float), ctypes.c_int32]),
    "ga_plan_set_tuning": (ctypes.c_int32, [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "ga_plan_get_tuning": (ctypes.c_int32, [_vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                            ctypes.POINTER(ctypes.c_int32)]),
    "ga_batch_create": (ctypes.c_int32, [ctypes.POINTER(_vp), ctypes.POINTER(BatchItem), ctypes.c_int32]),
    "ga_batch_launch": (ctypes.c_int32, [_vp, _vp]),
    "ga_batch_destroy": (ctypes.c_int32, [_vp]),
    "ga_profile_read": (ctypes.c_int32, [_vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_int64)]),
}

_lib = None


GA_TUNE_XCD, GA_TUNE_OVERLAP = 1, 2


class GaTuning(ctypes.Structure):
    _fields_ = [("groups", ctypes.c_int32), ("k", ctypes.c_int32), ("xcd", ctypes.c_int32), ("radix", ctypes.c_int32),
                ("overlap", ctypes.c_int32), ("us", ctypes.c_float), ("from_cache", ctypes.c_int32)]


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
        raise RuntimeError(f"libga.so not found at {path}: build it first (python -m paper_1711_05017_amd._build)")
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

    def __init__(self, n: int, max_batch: int = 1, flags: int = 0):
        lib = load()
        h = ctypes.c_void_p()
        _check("ga_plan_create", lib.ga_plan_create(ctypes.byref(h), int(n), int(max_batch), int(flags)))
        self._h = h
        self.n = int(n)
        self.max_batch = int(max_batch)

    @property
    def handle(self):
        return self._h

    def workspace(self, op: int, batch: int = 1, n_items: int = 0, device=None) -> torch.Tensor:
        nbytes = load().ga_workspace_size(self._h, op, batch, n_items)
        return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device or "cuda")

    # every settable choice of the fused x pass (groups, members per
    # workgroup, XCD-aware grid 1 / plain 2, radix schedule 0 / 1), and the
    # ones ga_plan_autotune times (radix 1 only where the edge has it)
    TUNE_CANDIDATES = [(g, k, x, r) for x in (1, 2) for r in (0, 1) for g in (4, 8) for k in (1, 2, 4, 8)]
    AUTOTUNE_CANDIDATES = [(g, k, 2, r) for r in (0, 1) for g in (4, 8) for k in (1, 2, 4, 8)]

    def has_alt_radix(self) -> bool:
        return bool(load().ga_plan_has_alt_radix(self._h))

    def autotune(self, Ahat: torch.Tensor, batch: int, work: Optional[torch.Tensor] = None, stream=None):
        """Time the plain-grid fused x-pass candidates and keep the fastest;
        returns ((groups, k, xcd, radix), {candidate: microseconds}) over the
        candidates that exist for this edge."""
        _need(Ahat, torch.complex64, _spec_elems(self.n), "Ahat")
        if work is None:
            work = torch.empty(int(batch) * _spec_elems(self.n) * 8, dtype=torch.uint8, device=Ahat.device)
        nc = len(self.AUTOTUNE_CANDIDATES)
        us = (ctypes.c_float * nc)()
        _check("ga_plan_autotune", load().ga_plan_autotune(self._h, _ptr(Ahat), int(batch), _ptr(work),
                                                           int(work.numel()), _stream(stream), us, nc))
        alt = self.has_alt_radix()
        times = {c: round(us[i], 2) for i, c in enumerate(self.AUTOTUNE_CANDIDATES) if alt or c[3] == 0}
        return self.tuning() + (self.radix(),), times

    def set_radix(self, radix: int):
        _check("ga_plan_set_radix", load().ga_plan_set_radix(self._h, int(radix)))

    def radix(self) -> int:
        return int(load().ga_plan_get_radix(self._h))

    def tune(self, Ahat: torch.Tensor, xyzr: torch.Tensor, w: torch.Tensor, R: torch.Tensor, c, sigma: float = 0.5,
             flags: int = 0, cache_path: Optional[str] = None, out: Optional[torch.Tensor] = None, work=None,
             stream=None) -> dict:
        """ga_plan_tune: tune a whole ga_energy_fields call of this shape (or
        apply the choice stored under its key in cache_path); returns the
        choice as a dict (groups, k, xcd, overlap, us, from_cache)."""
        n = self.n
        batch = int(R.shape[0])
        m = _samples(xyzr, w)
        _need(R, torch.float32, 9 * batch, "R", exact=True)
        _need(Ahat, torch.complex64, _spec_elems(n), "Ahat")
        if out is None:
            out = torch.empty((batch, n, n, n), dtype=torch.float32, device=xyzr.device)
        _need(out, torch.float32, batch * n ** 3, "out")
        if work is None:
            work = self.workspace(GA_OP_ENERGY, batch, m, device=xyzr.device)
        res = GaTuning()
        path = None if cache_path is None else os.fsencode(cache_path)
        _check("ga_plan_tune", load().ga_plan_tune(self._h, _ptr(Ahat), _ptr(xyzr), _ptr(w), m, _ptr(R), _host_f32(c, 3),
                                                   float(sigma), batch, _ptr(out), _ptr(work), int(work.numel()),
                                                   int(flags), path, _stream(stream), ctypes.byref(res)))
        return {"groups": res.groups, "k": res.k, "xcd": res.xcd, "radix": res.radix, "overlap": res.overlap,
                "us": round(res.us, 2), "from_cache": res.from_cache}

    def set_tuning(self, groups: int, k: int, xcd: int = 0):
        _check("ga_plan_set_tuning", load().ga_plan_set_tuning(self._h, int(groups), int(k), int(xcd)))

    def tuning(self):
        g, k, x = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check("ga_plan_get_tuning", load().ga_plan_get_tuning(self._h, ctypes.byref(g), ctypes.byref(k),
                                                               ctypes.byref(x)))
        return g.value, k.value, x.value

    def set_overlap(self, chunks: int):
        """ga_energy_fields in `chunks` parts (1, 2, 4) over two streams."""
        _check("ga_plan_set_overlap", load().ga_plan_set_overlap(self._h, int(chunks)))

    def overlap(self) -> int:
        return int(load().ga_plan_get_overlap(self._h))

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


def ga_score(plan: Plan, A2: torch.Tensor, B2: torch.Tensor, parts: int = GA_SCORE_RE | GA_SCORE_IM,
             a_stride: Optional[int] = None, out: Optional[torch.Tensor] = None, work=None,
             stream=None) -> torch.Tensor:
    """Score of complex affinities: A2 = the 2 half spectra (real channel,
    imaginary channel) of the stationary part, [2, n, n, n/2+1] (or one pair
    per member, [batch, 2, ...]); B2 = [batch, 2, n, n, n/2+1]. Returns
    [batch, nparts, n, n, n] (Re before Im)."""
    n = plan.n
    batch = B2.shape[0] if B2.dim() == 5 else 1
    nparts = 2 if parts == (GA_SCORE_RE | GA_SCORE_IM) else 1
    if a_stride is None:
        a_stride = 0 if (A2.dim() == 4 or A2.shape[0] == 1) else 2 * _spec_elems(n)
    _need(B2, torch.complex64, batch * 2 * _spec_elems(n), "B2", exact=True)
    _need(A2, torch.complex64, a_stride * (batch - 1) + 2 * _spec_elems(n), "A2")
    if out is None:
        out = torch.empty((batch, nparts, n, n, n), dtype=torch.float32, device=B2.device)
    _need(out, torch.float32, batch * nparts * n ** 3, "out")
    if work is None:
        work = plan.workspace(GA_OP_SCORE, batch, nparts, device=B2.device)
    st = load().ga_score(plan.handle, _ptr(A2), int(a_stride), _ptr(B2), int(batch), int(parts), _ptr(out),
                         _ptr(work), int(work.numel()), _stream(stream))
    _check("ga_score", st)
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


GA_NOALLOC_SCRATCH_BYTES = 16 << 20


def ga_force_torque_noalloc(plan: Plan, Ahat: torch.Tensor, Bhat4: torch.Tensor, t: torch.Tensor,
                            out: torch.Tensor, stream=None) -> torch.Tensor:
    """GA_SINGLE readout with the library's static scratch (no workspace); the
    caller passes the output buffer, so the call allocates nothing."""
    n = plan.n
    n_poses = int(t.shape[0])
    _need(t, torch.float32, 3 * n_poses, "t", exact=True)
    _need(Ahat, torch.complex64, _spec_elems(n), "Ahat")
    _need(Bhat4, torch.complex64, 4 * _spec_elems(n), "Bhat4")
    _need(out, torch.float32, 7 * n_poses, "out")
    st = load().ga_force_torque_noalloc(plan.handle, _ptr(Ahat), _ptr(Bhat4), _ptr(t), n_poses, _ptr(out),
                                        _stream(stream))
    _check("ga_force_torque_noalloc", st)
    return out


def ga_field_grad(plan: Plan, uA: torch.Tensor, Ahat: torch.Tensor, out: Optional[torch.Tensor] = None, work=None,
                  stream=None) -> torch.Tensor:
    """(u_A, grad u_A) per voxel as an [n, n, n, 4] float32 tensor."""
    n = plan.n
    _need(uA, torch.float32, n ** 3, "uA", exact=True)
    _need(Ahat, torch.complex64, _spec_elems(n), "Ahat", exact=True)
    if out is None:
        out = torch.empty((n, n, n, 4), dtype=torch.float32, device=uA.device)
    _need(out, torch.float32, 4 * n ** 3, "out")
    if work is None:
        work = plan.workspace(GA_OP_FIELD_GRAD, 1, device=uA.device)
    st = load().ga_field_grad(plan.handle, _ptr(uA), _ptr(Ahat), _ptr(out), _ptr(work), int(work.numel()),
                              _stream(stream))
    _check("ga_field_grad", st)
    return out


def ga_pose_local(plan: Plan, FA4: torch.Tensor, xyzr: torch.Tensor, w: torch.Tensor, R: torch.Tensor, c,
                  t: torch.Tensor, sigma: float = 0.5, out: Optional[torch.Tensor] = None, work=None,
                  stream=None) -> torch.Tensor:
    """(E, F, tau) at n_poses single poses by local sums over the moving part."""
    n = plan.n
    m = _samples(xyzr, w)
    n_poses = int(t.shape[0])
    _need(FA4, torch.float32, 4 * n ** 3, "FA4", exact=True)
    _need(R, torch.float32, 9 * n_poses, "R", exact=True)
    _need(t, torch.float32, 3 * n_poses, "t", exact=True)
    if out is None:
        out = torch.empty((n_poses, 7), dtype=torch.float32, device=t.device)
    _need(out, torch.float32, 7 * n_poses, "out")
    if work is None:
        work = plan.workspace(GA_OP_POSE_LOCAL, n_poses, m, device=t.device)
    st = load().ga_pose_local(plan.handle, _ptr(FA4), _ptr(xyzr), _ptr(w), m, _ptr(R), _host_f32(c, 3), float(sigma),
                              _ptr(t), n_poses, _ptr(out), _ptr(work), int(work.numel()), _stream(stream))
    _check("ga_pose_local", st)
    return out


def ga_pose_prepare(plan: Plan, Ahat: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Resident AX, DX of the stationary part (2 x half spectrum) for ga_pose_spectral."""
    n = plan.n
    _need(Ahat, torch.complex64, _spec_elems(n), "Ahat")
    if out is None:
        out = torch.empty((2,) + spectrum_shape(n), dtype=torch.complex64, device=Ahat.device)
    _need(out, torch.complex64, 2 * _spec_elems(n), "out")
    _check("ga_pose_prepare", load().ga_pose_prepare(plan.handle, _ptr(Ahat), _ptr(out), _stream(stream)))
    return out


def ga_pose_spectral(plan: Plan, AX2: torch.Tensor, xyzr: torch.Tensor, w: torch.Tensor, R: torch.Tensor, c,
                     t: torch.Tensor, sigma: float = 0.5, out: Optional[torch.Tensor] = None, work=None,
                     stream=None) -> torch.Tensor:
    """(E, F, tau) at n_poses single poses by re-correlation: splat and z/y
    transforms of the rotated part per pose, the x transform folded into AX2."""
    n = plan.n
    m = _samples(xyzr, w)
    n_poses = int(t.shape[0])
    _need(AX2, torch.complex64, 2 * _spec_elems(n), "AX2")
    _need(R, torch.float32, 9 * n_poses, "R", exact=True)
    _need(t, torch.float32, 3 * n_poses, "t", exact=True)
    if out is None:
        out = torch.empty((n_poses, 7), dtype=torch.float32, device=t.device)
    _need(out, torch.float32, 7 * n_poses, "out")
    if work is None:
        work = plan.workspace(GA_OP_POSE_SPECTRAL, n_poses, m, device=t.device)
    st = load().ga_pose_spectral(plan.handle, _ptr(AX2), _ptr(xyzr), _ptr(w), m, _ptr(R), _host_f32(c, 3),
                                 float(sigma), _ptr(t), n_poses, _ptr(out), _ptr(work), int(work.numel()),
                                 _stream(stream))
    _check("ga_pose_spectral", st)
    return out


def ga_field_table(plan: Plan, Ahat: torch.Tensor, Bhat4: torch.Tensor, out: Optional[torch.Tensor] = None,
                   work: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """The 7 fields per orientation: Bhat4 [n_orient, 4, n, n, n/2+1] (or
    [4, ...] for one) -> tables [n_orient, n, n, n, 8] (the 7 fields of a
    voxel in one 32-byte record, the last float 0)."""
    n = plan.n
    n_orient = Bhat4.shape[0] if Bhat4.dim() == 5 else 1
    _need(Ahat, torch.complex64, _spec_elems(n), "Ahat")
    _need(Bhat4, torch.complex64, n_orient * 4 * _spec_elems(n), "Bhat4", exact=True)
    if out is None:
        out = torch.empty((n_orient, n, n, n, 8), dtype=torch.float32, device=Bhat4.device)
    _need(out, torch.float32, n_orient * 8 * n ** 3, "out")
    if work is None:
        work = torch.empty(7 * _spec_elems(n) * 8 + 7 * n ** 3 * 4, dtype=torch.uint8, device=Bhat4.device)
    _check("ga_field_table", load().ga_field_table(plan.handle, _ptr(Ahat), _ptr(Bhat4), n_orient, _ptr(out),
                                                   _ptr(work), int(work.numel()), _stream(stream)))
    return out


def ga_field_table_query(plan: Plan, tables: torch.Tensor, orient: torch.Tensor, t: torch.Tensor,
                         out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    n = plan.n
    n_orient = int(tables.shape[0])
    _need(tables, torch.float32, n_orient * 8 * n ** 3, "tables", exact=True)
    n_q = int(t.shape[0])
    _need(t, torch.float32, 3 * n_q, "t", exact=True)
    _need(orient, torch.int32, n_q, "orient", exact=True)
    if out is None:
        out = torch.empty((n_q, 7), dtype=torch.float32, device=t.device)
    _need(out, torch.float32, 7 * n_q, "out")
    _check("ga_field_table_query", load().ga_field_table_query(plan.handle, _ptr(tables), n_orient, _ptr(orient),
                                                               _ptr(t), n_q, _ptr(out), _stream(stream)))
    return out


def ga_spectral_rotate(plan: Plan, X: torch.Tensor, R: torch.Tensor, out: Optional[torch.Tensor] = None,
                       stream=None) -> torch.Tensor:
    """Spectra of the part rotated by each R (trilinear interpolation at
    R^T omega). X: [channels, n, n, n/2+1] with channels 1 or 4; R: [batch, 9]
    (or [batch, 3, 3]); returns [batch, channels, n, n, n/2+1]."""
    n = plan.n
    ch = X.shape[0] if X.dim() == 4 else 1
    _need(X, torch.complex64, ch * _spec_elems(n), "X", exact=True)
    batch = int(R.shape[0])
    _need(R, torch.float32, 9 * batch, "R", exact=True)
    if out is None:
        out = torch.empty((batch, ch, n, n, n // 2 + 1), dtype=torch.complex64, device=X.device)
    _need(out, torch.complex64, batch * ch * _spec_elems(n), "out")
    _check("ga_spectral_rotate", load().ga_spectral_rotate(plan.handle, _ptr(X), ch, _ptr(R), batch, _ptr(out),
                                                           _stream(stream)))
    return out


def ga_spectral_pack4(plan: Plan, X4: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """The 4 half spectra X4 [4, n, n, n/2+1] as one 32-byte record per
    frequency: returns [n, n, n/2+1, 4] complex64 (the 4 channels of a
    frequency side by side), the source of ga_spectral_rotate_packed."""
    n = plan.n
    _need(X4, torch.complex64, 4 * _spec_elems(n), "X4", exact=True)
    if out is None:
        out = torch.empty((n, n, n // 2 + 1, 4), dtype=torch.complex64, device=X4.device)
    _need(out, torch.complex64, 4 * _spec_elems(n), "out")
    _check("ga_spectral_pack4", load().ga_spectral_pack4(plan.handle, _ptr(X4), _ptr(out), _stream(stream)))
    return out


def ga_spectral_rotate_packed(plan: Plan, P: torch.Tensor, R: torch.Tensor, out: Optional[torch.Tensor] = None,
                              stream=None) -> torch.Tensor:
    """ga_spectral_rotate of the 4 channels from packed spectra P
    (ga_spectral_pack4); returns [batch, 4, n, n, n/2+1]."""
    n = plan.n
    _need(P, torch.complex64, 4 * _spec_elems(n), "P", exact=True)
    batch = int(R.shape[0])
    _need(R, torch.float32, 9 * batch, "R", exact=True)
    if out is None:
        out = torch.empty((batch, 4, n, n, n // 2 + 1), dtype=torch.complex64, device=P.device)
    _need(out, torch.complex64, batch * 4 * _spec_elems(n), "out")
    _check("ga_spectral_rotate_packed", load().ga_spectral_rotate_packed(plan.handle, _ptr(P), _ptr(R), batch,
                                                                         _ptr(out), _stream(stream)))
    return out


def ga_lowpass(plan: Plan, X: torch.Tensor, L: int, mode: int = GA_LOWPASS_COARSE, scale: float = 1.0,
               out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Keep the low-frequency box |kappa| <= L/2 - 1 of n-grid half spectra X
    ([batch,] n, n, n/2+1): on an L grid (coarse) or zero-padded at n."""
    n = plan.n
    batch = X.shape[0] if X.dim() == 4 else 1
    _need(X, torch.complex64, batch * _spec_elems(n), "X", exact=True)
    m = int(L) if mode == GA_LOWPASS_COARSE else n
    if out is None:
        out = torch.empty((batch, m, m, m // 2 + 1), dtype=torch.complex64, device=X.device)
    _need(out, torch.complex64, batch * _spec_elems(m), "out")
    _check("ga_lowpass", load().ga_lowpass(plan.handle, int(L), int(mode), _ptr(X), _ptr(out), int(batch), float(scale),
                                           _stream(stream)))
    return out


class Batch:
    """Energy-field calls of several (plan, pair, rotations) items recorded
    into one HIP graph (ga_batch_*). Each item is a dict with keys plan,
    Ahat, xyzr, w, R, c, sigma; outputs and workspaces are allocated here and
    kept with the batch. launch() replays the graph; inputs are read from the
    same tensors at every replay, so update them in place."""

    def __init__(self, items):
        lib = load()
        self._keep = []
        arr = (BatchItem * len(items))()
        self.outputs = []
        for i, it in enumerate(items):
            plan = it["plan"]
            n = plan.n
            xyzr, w, R, Ahat = it["xyzr"], it["w"], it["R"], it["Ahat"]
            m = _samples(xyzr, w)
            batch = int(R.shape[0])
            _need(R, torch.float32, 9 * batch, "R", exact=True)
            _need(Ahat, torch.complex64, _spec_elems(n), "Ahat")
            E = torch.empty((batch, n, n, n), dtype=torch.float32, device=xyzr.device)
            work = plan.workspace(GA_OP_ENERGY, batch, m, device=xyzr.device)
            if plan.overlap() > 1:  # room for the parts' 256-byte aligned workspace slices
                work = torch.empty(work.numel() + 4 * 512, dtype=torch.uint8, device=xyzr.device)
            self._keep += [plan, xyzr, w, R, Ahat, E, work]
            self.outputs.append(E)
            c = [float(v) for v in torch.as_tensor(it["c"], dtype=torch.float64).reshape(-1).tolist()]
            arr[i] = BatchItem(plan.handle.value, Ahat.data_ptr(), xyzr.data_ptr(), w.data_ptr(), m, R.data_ptr(),
                               (ctypes.c_float * 3)(*c), float(it.get("sigma", 0.5)), batch, E.data_ptr(),
                               work.data_ptr(), int(work.numel()))
        h = ctypes.c_void_p()
        _check("ga_batch_create", lib.ga_batch_create(ctypes.byref(h), arr, len(items)))
        self._h = h

    def launch(self, stream=None):
        _check("ga_batch_launch", load().ga_batch_launch(self._h, _stream(stream)))
        return self.outputs

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().ga_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


GA_EAGAIN, GA_ENOTFOUND = -3, -5


class Server:
    """A ga_server: resident pair fields, queued pose queries, continuous
    batching. Host numpy arrays in; results as ga_result. mode selects how a
    query is evaluated (GA_SERVE_LOCAL or GA_SERVE_SPECTRAL, same values)."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 8 << 30, max_slots: int = 8, queue_depth: int = 4096,
                 mode: int = GA_SERVE_LOCAL, mock=None, mock_launch_us: int = 0):
        """mock: a test executor, called as mock(pair_id, n, R (9 floats),
        t (3 ints)) -> 7 floats on the server's scheduler thread (an
        exception acts as a device error); the server then uses no device."""
        lib = load()
        self._mock = None
        if mock is not None:
            def call(user, pair_id, n, R, t, out7):
                try:
                    vals = mock(int(pair_id), int(n), [R[i] for i in range(9)], [t[i] for i in range(3)])
                    for i in range(7):
                        out7[i] = float(vals[i])
                    return 0
                except Exception:
                    return 1
            self._mock = MockQueryFn(call)
        cfg = ServerCfg(device, hbm_budget_bytes, max_slots, queue_depth, mode,
                        self._mock if self._mock is not None else MockQueryFn(), None, int(mock_launch_us))
        h = ctypes.c_void_p()
        _check("ga_server_create", lib.ga_server_create(ctypes.byref(h), ctypes.byref(cfg)))
        self._h = h
        self._keep = []

    @staticmethod
    def _part(xyzr, w):
        import numpy as np

        x = np.ascontiguousarray(xyzr, dtype=np.float32).reshape(-1, 4)
        ww = np.ascontiguousarray(w, dtype=np.float32).reshape(-1)
        if ww.shape[0] != x.shape[0]:
            raise ValueError("xyzr and w lengths differ")
        return PartDesc(x.ctypes.data, ww.ctypes.data, x.shape[0]), (x, ww)

    def register_pair(self, A_xyzr, A_w, B_xyzr, B_w, cB, n: int, sigma: float = 0.5) -> int:
        pa, ka = self._part(A_xyzr, A_w)
        pb, kb = self._part(B_xyzr, B_w)
        c = (ctypes.c_float * 3)(*[float(v) for v in cB])
        pid = ctypes.c_uint32()
        _check("ga_pair_register", load().ga_pair_register(self._h, ctypes.byref(pa), ctypes.byref(pb), c, int(n),
                                                           float(sigma), ctypes.byref(pid)))
        del ka, kb
        return pid.value

    def release_pair(self, pair_id: int):
        _check("ga_pair_release", load().ga_pair_release(self._h, int(pair_id)))

    def submit(self, pair_id: int, R, t):
        """Ticket, or None when the queue is full."""
        r = (ctypes.c_float * 9)(*[float(v) for v in list(_flat(R))])
        tt = (ctypes.c_float * 3)(*[float(v) for v in list(_flat(t))])
        tk = ctypes.c_uint64()
        st = load().ga_submit(self._h, int(pair_id), r, tt, ctypes.byref(tk))
        if st == GA_EAGAIN:
            return None
        _check("ga_submit", st)
        return tk.value

    def poll(self, ticket: int):
        """Result when done, None while pending."""
        res = Result()
        st = load().ga_poll(self._h, int(ticket), ctypes.byref(res))
        if st == GA_PENDING:
            return None
        _check("ga_poll", st)
        return res

    def wait(self, ticket: int, timeout_s: float = 30.0):
        import time

        t0 = time.perf_counter()
        while True:
            r = self.poll(ticket)
            if r is not None:
                return r
            if time.perf_counter() - t0 > timeout_s:
                raise TimeoutError(f"ticket {ticket} not done after {timeout_s} s")

    def stats(self) -> ServerStats:
        st = ServerStats()
        _check("ga_server_get_stats", load().ga_server_get_stats(self._h, ctypes.byref(st)))
        return st

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().ga_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _flat(a):
    try:
        import numpy as np

        return np.asarray(a, dtype=np.float64).reshape(-1).tolist()
    except Exception:
        return list(a)
