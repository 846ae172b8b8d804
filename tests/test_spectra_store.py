"""Store of resident spectra (paper_1711_05017_amd/spectra.py): round trip,
key sensitivity, and refusal of records or arrays that do not match."""

import json
import os

import numpy as np
import pytest
import torch

from paper_1711_05017_amd.spectra import load_spectrum, save_spectrum, skeleton_key


def _skeleton(seed=7, m=50):
    rng = np.random.default_rng(seed)
    xyzr = np.concatenate([rng.uniform(-5, 5, (m, 3)), rng.uniform(0.5, 2, (m, 1))], 1).astype(np.float32)
    w = rng.uniform(0.1, 1.0, m).astype(np.float32)
    return xyzr, w


def _spectrum(n, channels, seed=3):
    rng = np.random.default_rng(seed)
    shape = (channels, n, n, n // 2 + 1)
    a = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(np.complex64)
    return torch.from_numpy(a)


@pytest.mark.parametrize("n,channels", [(16, 1), (24, 4)])
def test_round_trip_is_bit_exact(tmp_path, n, channels):
    xyzr, w = _skeleton()
    key = skeleton_key(xyzr, w, n, 0.5, channels)
    X = _spectrum(n, channels)
    assert load_spectrum(str(tmp_path), key, n, channels) is None
    save_spectrum(str(tmp_path), key, X, n, 0.5, channels)
    Y = load_spectrum(str(tmp_path), key, n, channels, sigma=0.5)
    assert Y.dtype == torch.complex64 and tuple(Y.shape) == (channels, n, n, n // 2 + 1)
    assert torch.equal(torch.view_as_real(Y), torch.view_as_real(X))
    assert not [f for f in os.listdir(tmp_path) if f.endswith(".tmp")]


def test_single_channel_spectrum_from_a_batch_view(tmp_path):
    n = 16
    X = _spectrum(n, 1)[0]  # [n, n, n/2+1], as ga_fft3d's out[0]
    xyzr, w = _skeleton()
    key = skeleton_key(xyzr, w, n, 0.5)
    save_spectrum(str(tmp_path), key, X, n, 0.5)
    assert torch.equal(torch.view_as_real(load_spectrum(str(tmp_path), key, n)[0]), torch.view_as_real(X))


def test_key_changes_with_every_input():
    xyzr, w = _skeleton()
    R = np.eye(3, dtype=np.float32)
    c = np.zeros(3, np.float32)
    base = skeleton_key(xyzr, w, 32, 0.5, 1, R, c)
    assert base == skeleton_key(torch.from_numpy(xyzr), torch.from_numpy(w), 32, 0.5, 1, R, c)
    x2 = xyzr.copy()
    x2[17, 1] = np.nextafter(x2[17, 1], np.float32(np.inf))
    w2 = w.copy()
    w2[3] *= 2
    R2 = R.copy()
    R2[0, 1] = 1e-7
    variants = [
        skeleton_key(x2, w, 32, 0.5, 1, R, c),
        skeleton_key(xyzr, w2, 32, 0.5, 1, R, c),
        skeleton_key(xyzr, w, 48, 0.5, 1, R, c),
        skeleton_key(xyzr, w, 32, 0.75, 1, R, c),
        skeleton_key(xyzr, w, 32, 0.5, 4, R, c),
        skeleton_key(xyzr, w, 32, 0.5, 1, R2, c),
        skeleton_key(xyzr, w, 32, 0.5, 1, R, c + 1),
        skeleton_key(xyzr, w, 32, 0.5, 1),
        skeleton_key(xyzr[:-1], w[:-1], 32, 0.5, 1, R, c),
    ]
    assert len(set(variants + [base])) == len(variants) + 1
    with pytest.raises(ValueError):
        skeleton_key(xyzr, w[:-1], 32, 0.5)


def test_mismatches_are_refused(tmp_path):
    n = 16
    xyzr, w = _skeleton()
    key = skeleton_key(xyzr, w, n, 0.5)
    d = str(tmp_path)
    save_spectrum(d, key, _spectrum(n, 1), n, 0.5)
    with pytest.raises(ValueError, match="n is"):
        load_spectrum(d, key, 32)
    with pytest.raises(ValueError, match="channels is"):
        load_spectrum(d, key, n, 4)
    with pytest.raises(ValueError, match="sigma is"):
        load_spectrum(d, key, n, sigma=0.75)
    with pytest.raises(ValueError):
        load_spectrum(d, "../" + key, n)
    with pytest.raises(ValueError):
        save_spectrum(d, key, _spectrum(n, 1).real.contiguous(), n, 0.5)
    with pytest.raises(ValueError):
        save_spectrum(d, key, _spectrum(n, 4), n, 0.5, 1)

    # one flipped bit in the stored array
    npy = os.path.join(d, key + ".npy")
    raw = bytearray(open(npy, "rb").read())
    raw[-5] ^= 0x10
    open(npy, "wb").write(bytes(raw))
    with pytest.raises(ValueError, match="content hash"):
        load_spectrum(d, key, n)


def test_record_for_another_key_is_refused(tmp_path):
    n = 16
    d = str(tmp_path)
    xyzr, w = _skeleton()
    k1 = skeleton_key(xyzr, w, n, 0.5)
    k2 = skeleton_key(xyzr, w, n, 0.25)
    save_spectrum(d, k1, _spectrum(n, 1), n, 0.5)
    for ext in (".npy", ".json"):
        os.replace(os.path.join(d, k1 + ext), os.path.join(d, k2 + ext))
    with pytest.raises(ValueError, match="key is"):
        load_spectrum(d, k2, n)
    meta = json.load(open(os.path.join(d, k2 + ".json")))
    assert meta["format"] == "ga-spectrum/1" and meta["sigma"] == 0.5
