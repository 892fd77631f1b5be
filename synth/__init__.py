"""Seeded synthetic inputs shared by the CPU oracle and the GPU library.

This package holds none of the method's arithmetic: no decoding and no
beamforming.  It provides
  * workload descriptions (plain dicts with the paper's inputs, Sec. VI-B:
    array pitch and 4x4 transform, transmit columns and Hadamard order,
    channel map, sampling rate, sound speed, t0, F#, output grid);
  * a Sylvester Hadamard matrix for encoding the simulated acquisition;
  * an acquisition simulator (``synth.c``) and the seeded recipe that turns
    scatterer scenes into int16 RF channel data: element responses, Hadamard
    encoding across transmits, Gaussian noise at 1 % of peak, scaling to a
    30000 peak and round-half-even quantisation to int16.

The paper measures on its own scanner data, which is not available; these
inputs stand in for it, with the shapes, sampling and array sizes of the five
benchmark workloads.  Seed of workload ``k``: ``numpy.random.default_rng(1000 + k)``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import configs  # noqa: F401  (re-export)
from .configs import centered_xdc, workload  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsynth.so")
_lib = None


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=gnu11", "-Wall",
           "-o", _LIB_PATH + ".tmp", os.path.join(_HERE, "synth.c"), "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        D = ctypes.POINTER(ctypes.c_double)
        L.synth_echoes.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                   D, D, ctypes.c_int, D, D, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_double, ctypes.c_double, ctypes.c_double, D,
                                   ctypes.c_double, ctypes.c_double, D]
        _lib = L
    return _lib


def hadamard_sylvester(n: int) -> np.ndarray:
    """Order-n Sylvester Hadamard matrix by repeated Kronecker doubling."""
    if n < 1 or n & (n - 1):
        raise ValueError(f"Sylvester order must be a power of two, got {n}")
    H = np.ones((1, 1), dtype=np.int64)
    while H.shape[0] < n:
        H = np.block([[H, H], [H, -H]])
    return H.astype(np.int8)


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def to_array_frame(desc: dict, pts_global: np.ndarray) -> np.ndarray:
    M = np.asarray(desc["xdc"], dtype=np.float64).reshape(4, 4)
    P = np.asarray(pts_global, dtype=np.float64).reshape(-1, 3)
    return P @ M[:3, :3].T + M[:3, 3]


def element_responses(desc: dict, pts_global: np.ndarray, amps: np.ndarray,
                      c: float | None = None) -> np.ndarray:
    """Simulated (unencoded) element responses, float64 (n_tx, n_ch, S)."""
    mode = {"forces": 0, "hercules": 1, "tpw": 2, "vls": 3}[desc["mode"]]
    n_tx, n_ch, S = int(desc["n_tx"]), int(desc["n_ch"]), int(desc["n_samples"])
    px, py = (float(v) for v in desc["pitch"])
    tx_x = np.ascontiguousarray(np.asarray(desc["tx_elements"], dtype=np.float64) * px)
    rx_c = np.ascontiguousarray(np.asarray(desc["channel_map"], dtype=np.float64) *
                                (px if mode == 0 else py))
    sp = np.ascontiguousarray(to_array_frame(desc, pts_global))
    amps = np.ascontiguousarray(amps, dtype=np.float64)
    e = np.empty((n_tx, n_ch, S), dtype=np.float64)
    ang = np.ascontiguousarray(desc.get("tx_angles", np.zeros(n_tx)), dtype=np.float64)
    xc = 0.5 * (desc["n_elem"][0] - 1) * px
    yc = 0.5 * (desc["n_elem"][1] - 1) * py
    _load().synth_echoes(mode, n_tx, n_ch, S, _dptr(tx_x), _dptr(rx_c), sp.shape[0], _dptr(sp),
                         _dptr(amps), float(desc["fs"]), float(desc["fc"]),
                         float(desc["c"] if c is None else c), float(desc["t0"]),
                         float(desc.get("focal_depth", np.inf)), _dptr(ang), xc, yc, _dptr(e))
    return e


def encode(H: np.ndarray, e: np.ndarray) -> np.ndarray:
    """Hadamard-encoded acquisition r[k] = sum_i H[k][i] e[i] (float64)."""
    n = H.shape[0]
    return (H.astype(np.float64) @ e.reshape(n, -1)).reshape(e.shape)


def quantise(r: np.ndarray, rng: np.random.Generator, noise: float = 0.01,
             peak: float = 30000.0) -> np.ndarray:
    """Add Gaussian noise (sigma = noise * max|r|), scale to `peak`, rint, clip."""
    r = np.asarray(r, dtype=np.float64)
    m = float(np.max(np.abs(r)))
    if noise > 0 and m > 0:
        r = r + rng.standard_normal(r.shape) * (noise * m)
    m = float(np.max(np.abs(r)))
    scale = peak / m if m > 0 else 1.0
    return np.clip(np.rint(r * scale), -32768, 32767).astype(np.int16)


def acquire(desc: dict, pts_global, amps, rng: np.random.Generator, H=None,
            noise: float = 0.01, c: float | None = None, encoded: bool = True) -> np.ndarray:
    """Scene -> int16 RF (n_tx, n_ch, S), Hadamard-encoded across transmits
    unless ``encoded`` is False (conventional TPW / VLS acquisitions)."""
    e = element_responses(desc, pts_global, amps, c=c)
    if not encoded:
        return quantise(e, rng, noise=noise)
    if H is None:
        H = hadamard_sylvester(int(desc["n_tx"]))
    return quantise(encode(H, e), rng, noise=noise)


def make_inputs(k: int, frame: int | None = None):
    """Seeded inputs of workload k: (desc or list of descs, H or list, rf or list, scene info).

    Workloads 0 and 1 (and 2, which reuses 1's data) return one frame; 3 and 4
    return lists of frames.  Everything derives from default_rng(1000 + k).
    """
    return configs.make_inputs(k, frame=frame)
