"""Store of resident density spectra on disk.

A part's density spectrum depends on its geometry alone, not on the relative
pose, so it can be computed once, before the interactive session, and reused
for every pose (Sec. 3.2, the forward transforms of eq. 7a). This module keeps such spectra
between processes: one ``.npy`` file of complex64 values per spectrum, laid out
[channels][n][n][n/2+1] as ``ga_fft3d`` writes them, beside a JSON record of
the grid edge, the channel count, sigma, the skeleton key and a SHA-256 of the
array's bytes. Files are read with numpy's loader with pickling off, and every
field of the record is checked on load; a mismatch raises ``ValueError``.

The key (``skeleton_key``) hashes everything the spectrum depends on: the
skeleton samples and weights as float32 bytes, the grid edge, sigma, the
channel count, and the pose the samples were placed at (if any). It does not
hash the library version: the spectrum is a function of those inputs alone,
up to float32 rounding.
"""

from __future__ import annotations

import hashlib
import json
import os
import struct
from typing import Optional

import numpy as np
import torch

FORMAT = "ga-spectrum/1"


def _f32_bytes(a) -> bytes:
    if isinstance(a, torch.Tensor):
        a = a.detach().to("cpu", torch.float32).contiguous().numpy()
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32)).tobytes()


def skeleton_key(xyzr, w, n: int, sigma: float, channels: int = 1, R=None, c=None) -> str:
    """Hex SHA-256 naming the spectrum of skeleton (xyzr [m, 4], w [m]) splatted
    on an n^3 grid with this sigma and channel count, optionally placed by
    rotation R (3 x 3) about reference point c (3)."""
    xyzr_b, w_b = _f32_bytes(xyzr), _f32_bytes(w)
    if len(xyzr_b) != 4 * len(w_b):
        raise ValueError("xyzr must hold four floats per weight")
    h = hashlib.sha256()
    h.update(FORMAT.encode())
    h.update(struct.pack("<iif", int(n), int(channels), float(sigma)))
    h.update(struct.pack("<q", len(w_b) // 4))
    h.update(xyzr_b)
    h.update(w_b)
    for tag, v, count in ((b"R", R, 9), (b"c", c, 3)):
        if v is None:
            h.update(tag + b"-")
        else:
            b = _f32_bytes(v)
            if len(b) != 4 * count:
                raise ValueError(f"{tag.decode()} must hold {count} floats")
            h.update(tag + b)
    return h.hexdigest()


def _paths(directory: str, key: str):
    if not key or any(ch not in "0123456789abcdef" for ch in key):
        raise ValueError("key must be a lowercase hex string (skeleton_key)")
    return os.path.join(directory, key + ".npy"), os.path.join(directory, key + ".json")


def _shape(n: int, channels: int):
    return (channels, n, n, n // 2 + 1)


def save_spectrum(directory: str, key: str, X: torch.Tensor, n: int, sigma: float, channels: int = 1) -> str:
    """Write spectrum X (complex64, channels * n * n * (n/2+1) values, on any
    device; copied to the host synchronously) under `key`. The array and its
    record are each written to a temporary file and renamed into place, so a
    reader never sees a partial file. Returns the array's path."""
    shape = _shape(n, channels)
    if not isinstance(X, torch.Tensor) or X.dtype != torch.complex64:
        raise ValueError("X must be a complex64 tensor")
    if X.numel() != int(np.prod(shape)):
        raise ValueError(f"X has {X.numel()} values, a spectrum of {channels} channel(s) at n = {n} has "
                         f"{int(np.prod(shape))}")
    arr = np.ascontiguousarray(X.detach().to("cpu").contiguous().numpy().reshape(shape))
    npy, rec = _paths(directory, key)
    os.makedirs(directory, exist_ok=True)
    tmp = npy + f".{os.getpid()}.tmp"
    with open(tmp, "wb") as f:
        np.save(f, arr, allow_pickle=False)
    os.replace(tmp, npy)
    meta = {"format": FORMAT, "key": key, "n": int(n), "channels": int(channels), "sigma": float(np.float32(sigma)),
            "dtype": "complex64", "shape": list(shape), "sha256": hashlib.sha256(arr.tobytes()).hexdigest()}
    tmp = rec + f".{os.getpid()}.tmp"
    with open(tmp, "w") as f:
        json.dump(meta, f, indent=1)
    os.replace(tmp, rec)
    return npy


def load_spectrum(directory: str, key: str, n: int, channels: int = 1, sigma: Optional[float] = None,
                  device=None) -> Optional[torch.Tensor]:
    """The spectrum stored under `key`, as a complex64 tensor [channels, n, n,
    n/2+1] on `device` (the host if None), or None if none is stored. Raises
    ValueError if the record or the array does not match (format, key, n,
    channels, sigma when given, dtype, shape, content hash)."""
    npy, rec = _paths(directory, key)
    if not (os.path.exists(npy) and os.path.exists(rec)):
        return None
    with open(rec) as f:
        meta = json.load(f)
    shape = _shape(n, channels)
    want = {"format": FORMAT, "key": key, "n": int(n), "channels": int(channels), "dtype": "complex64",
            "shape": list(shape)}
    for k, v in want.items():
        if meta.get(k) != v:
            raise ValueError(f"stored spectrum {key}: {k} is {meta.get(k)!r}, expected {v!r}")
    if sigma is not None and meta.get("sigma") != float(np.float32(sigma)):
        raise ValueError(f"stored spectrum {key}: sigma is {meta.get('sigma')!r}, expected {float(np.float32(sigma))!r}")
    arr = np.load(npy, allow_pickle=False)
    if arr.dtype != np.complex64 or arr.shape != shape:
        raise ValueError(f"stored spectrum {key}: array is {arr.dtype} {arr.shape}, expected complex64 {shape}")
    if hashlib.sha256(np.ascontiguousarray(arr).tobytes()).hexdigest() != meta.get("sha256"):
        raise ValueError(f"stored spectrum {key}: content hash does not match its record")
    t = torch.from_numpy(arr)
    return t if device is None else t.to(device)
