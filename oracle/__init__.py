"""FP64 CPU oracle for Hadamard decoding + delay-and-sum beamforming.

TEST INFRASTRUCTURE ONLY: the test suite, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` are the only callers.  The product path
(``paper_2512_11086_amd``) never imports this package, and this package never
imports the product path.  The arithmetic lives in ``oracle.c`` (plain loops,
double precision, OpenMP over output points); this module only marshals
arguments through ctypes.

A problem description is a plain dict (see ``synth.configs``) holding the
paper's inputs: array geometry (pitch, 4x4 transform), transmit sequence and
Hadamard order, sampling rate, sound speed and output grid (Sec. VI-B).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

MODES = {"forces": 0, "hercules": 1, "tpw": 2, "vls": 3}
INTERPS = {"nearest": 0, "linear": 1, "cubic": 2}


def build(verbose: bool = False) -> str:
    """Compile liboracle.so with gcc (plain -O2, no fast-math)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=gnu11", "-Wall",
           "-o", _LIB_PATH + ".tmp", os.path.join(_HERE, "oracle.c"), "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


class _Geom(ctypes.Structure):
    _fields_ = [
        ("mode", ctypes.c_int), ("n_tx", ctypes.c_int), ("n_ch", ctypes.c_int),
        ("n_samples", ctypes.c_int),
        ("tx_elements", ctypes.POINTER(ctypes.c_int32)),
        ("channel_map", ctypes.POINTER(ctypes.c_int32)),
        ("pitch", ctypes.c_double * 2), ("xdc", ctypes.c_double * 16),
        ("fs", ctypes.c_double), ("c", ctypes.c_double), ("t0", ctypes.c_double),
        ("f_number", ctypes.c_double), ("interp", ctypes.c_int),
        ("dims", ctypes.c_int * 3), ("gmin", ctypes.c_double * 3), ("gmax", ctypes.c_double * 3),
        ("n_elem", ctypes.c_int * 2), ("focal_depth", ctypes.c_double),
        ("tx_angles", ctypes.POINTER(ctypes.c_double)),
    ]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.POINTER
        L.oracle_threads.argtypes = [ctypes.c_int]
        L.oracle_threads.restype = ctypes.c_int
        L.oracle_sylvester.argtypes = [ctypes.c_int, P(ctypes.c_int8)]
        L.oracle_decode.argtypes = [P(ctypes.c_int8), ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                    P(ctypes.c_int16), P(ctypes.c_int64)]
        L.oracle_hann.argtypes = [ctypes.c_double]
        L.oracle_hann.restype = ctypes.c_double
        for f in (L.oracle_interp, L.oracle_interp_deriv):
            f.argtypes = [P(ctypes.c_double), ctypes.c_int, ctypes.c_double, ctypes.c_int]
            f.restype = ctypes.c_double
        L.oracle_das.argtypes = [P(_Geom), P(ctypes.c_double), P(ctypes.c_double)]
        L.oracle_das_points.argtypes = [P(_Geom), P(ctypes.c_double), P(ctypes.c_int64),
                                        ctypes.c_int64, P(ctypes.c_double)]
        L.oracle_das_adjoint_e.argtypes = [P(_Geom), P(ctypes.c_double), P(ctypes.c_double)]
        L.oracle_das_dc.argtypes = [P(_Geom), P(ctypes.c_double), P(ctypes.c_double)]
        L.oracle_sharpness.argtypes = [P(ctypes.c_double), ctypes.c_int64, P(ctypes.c_double)]
        L.oracle_sharpness.restype = ctypes.c_double
        D = P(ctypes.c_double)
        L.oracle_demod.argtypes = [P(ctypes.c_int16), ctypes.c_int, ctypes.c_int, D, D,
                                   ctypes.c_int, ctypes.c_double, ctypes.c_int, D]
        L.oracle_quantise_i16.argtypes = [D, ctypes.c_int64, P(ctypes.c_int16)]
        L.oracle_das_iq.argtypes = [P(_Geom), ctypes.c_double, D, D, D, D]
        L.oracle_das_iq_points.argtypes = [P(_Geom), ctypes.c_double, D, D, P(ctypes.c_int64),
                                           ctypes.c_int64, D, D]
        L.oracle_envelope.argtypes = [D, ctypes.c_int64, ctypes.c_int, D]
        L.oracle_compress.argtypes = [D, ctypes.c_int64, ctypes.c_int, ctypes.c_double,
                                      ctypes.c_double, D]
        _lib = L
    return _lib


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def threads(n: int = 0) -> int:
    """Set the oracle's OpenMP worker count (n >= 1) and return the count in
    effect (n = 0 only queries it)."""
    return int(lib().oracle_threads(int(n)))


def sylvester(n: int) -> np.ndarray:
    H = np.empty((n, n), dtype=np.int8)
    if lib().oracle_sylvester(n, _ptr(H, ctypes.c_int8)) != 0:
        raise ValueError(f"no Sylvester Hadamard matrix of order {n}")
    return H


def decode(H: np.ndarray, r: np.ndarray) -> np.ndarray:
    """e[i][j][t] = sum_k H[k][i] r[k][j][t], exact int64."""
    H = np.ascontiguousarray(H, dtype=np.int8)
    r = np.ascontiguousarray(r, dtype=np.int16)
    n_tx, n_ch, S = r.shape
    assert H.shape == (n_tx, n_tx)
    e = np.empty(r.shape, dtype=np.int64)
    lib().oracle_decode(_ptr(H, ctypes.c_int8), n_tx, n_ch, S, _ptr(r, ctypes.c_int16),
                        _ptr(e, ctypes.c_int64))
    return e


def hann(u: float) -> float:
    return lib().oracle_hann(float(u))


def interp(trace: np.ndarray, s: float, mode: str = "cubic", deriv: bool = False) -> float:
    trace = np.ascontiguousarray(trace, dtype=np.float64)
    f = lib().oracle_interp_deriv if deriv else lib().oracle_interp
    return f(_ptr(trace, ctypes.c_double), trace.shape[0], float(s), INTERPS[mode])


class Geometry:
    """ctypes view of a problem description; keeps its arrays alive."""

    def __init__(self, desc: dict, c: float | None = None):
        g = _Geom()
        g.mode = MODES[desc["mode"]]
        g.n_tx, g.n_ch, g.n_samples = int(desc["n_tx"]), int(desc["n_ch"]), int(desc["n_samples"])
        self._tx = np.ascontiguousarray(desc["tx_elements"], dtype=np.int32)
        self._ch = np.ascontiguousarray(desc["channel_map"], dtype=np.int32)
        assert self._tx.shape == (g.n_tx,) and self._ch.shape == (g.n_ch,)
        g.tx_elements = _ptr(self._tx, ctypes.c_int32)
        g.channel_map = _ptr(self._ch, ctypes.c_int32)
        g.pitch[:] = [float(v) for v in desc["pitch"]]
        g.xdc[:] = [float(v) for v in np.asarray(desc["xdc"], dtype=np.float64).reshape(16)]
        g.fs, g.t0 = float(desc["fs"]), float(desc["t0"])
        g.c = float(desc["c"] if c is None else c)
        g.f_number = float(desc["f_number"])
        g.interp = INTERPS[desc.get("interp", "cubic")]
        g.dims[:] = [int(v) for v in desc["dims"]]
        g.gmin[:] = [float(v) for v in desc["gmin"]]
        g.gmax[:] = [float(v) for v in desc["gmax"]]
        g.n_elem[:] = [int(v) for v in desc["n_elem"]]
        g.focal_depth = float(desc.get("focal_depth", np.inf))
        self._ang = np.ascontiguousarray(desc.get("tx_angles", np.zeros(g.n_tx)), dtype=np.float64)
        assert self._ang.shape == (g.n_tx,)
        g.tx_angles = _ptr(self._ang, ctypes.c_double)
        self.g = g
        self.n_vox = int(np.prod(desc["dims"]))
        self.shape = (int(desc["dims"][1]), int(desc["dims"][0]), int(desc["dims"][2]))


def _e64(desc, e):
    e = np.ascontiguousarray(e, dtype=np.float64)
    assert e.shape == (desc["n_tx"], desc["n_ch"], desc["n_samples"]), e.shape
    return e


def das(desc: dict, e: np.ndarray, c: float | None = None) -> np.ndarray:
    """Beamformed image, shape (Ny, Nx, Nz), float64 (Eq. 1)."""
    geo = Geometry(desc, c)
    e = _e64(desc, e)
    out = np.empty(geo.shape, dtype=np.float64)
    lib().oracle_das(ctypes.byref(geo.g), _ptr(e, ctypes.c_double), _ptr(out, ctypes.c_double))
    return out


def das_points(desc: dict, e: np.ndarray, vox: np.ndarray, c: float | None = None) -> np.ndarray:
    """Eq. 1 at the listed linear voxel indices only."""
    geo = Geometry(desc, c)
    e = _e64(desc, e)
    vox = np.ascontiguousarray(vox, dtype=np.int64)
    assert vox.size == 0 or (vox.min() >= 0 and vox.max() < geo.n_vox)
    out = np.empty(vox.shape, dtype=np.float64)
    lib().oracle_das_points(ctypes.byref(geo.g), _ptr(e, ctypes.c_double),
                            _ptr(vox, ctypes.c_int64), vox.size, _ptr(out, ctypes.c_double))
    return out


def das_adjoint_e(desc: dict, G: np.ndarray, c: float | None = None) -> np.ndarray:
    """Transpose of e -> image applied to an image-shaped G; shape (n_tx, n_ch, S)."""
    geo = Geometry(desc, c)
    G = np.ascontiguousarray(G, dtype=np.float64).reshape(geo.shape)
    out = np.empty((desc["n_tx"], desc["n_ch"], desc["n_samples"]), dtype=np.float64)
    lib().oracle_das_adjoint_e(ctypes.byref(geo.g), _ptr(G, ctypes.c_double),
                               _ptr(out, ctypes.c_double))
    return out


def das_dc(desc: dict, e: np.ndarray, c: float | None = None) -> np.ndarray:
    """Per-voxel d(image)/d(sound speed), shape (Ny, Nx, Nz)."""
    geo = Geometry(desc, c)
    e = _e64(desc, e)
    out = np.empty(geo.shape, dtype=np.float64)
    lib().oracle_das_dc(ctypes.byref(geo.g), _ptr(e, ctypes.c_double), _ptr(out, ctypes.c_double))
    return out


def sharpness(img: np.ndarray, grad: bool = False):
    """Negative normalised L4 norm of one image; optionally its gradient."""
    img = np.ascontiguousarray(img, dtype=np.float64)
    g = np.empty_like(img) if grad else None
    L = lib().oracle_sharpness(_ptr(img, ctypes.c_double), img.size,
                               _ptr(g, ctypes.c_double) if grad else None)
    return (L, g) if grad else L


# ---------------------------------------------------------------------------
# Demodulation (Eq. 4) and IQ beamforming
# ---------------------------------------------------------------------------
def demod(x: np.ndarray, taps, fd: float, fs: float, D: int = 1) -> np.ndarray:
    """Mix, filter, decimate (Eq. 4) every trace of int16 ``x`` (..., S).

    Returns complex128 (..., ceil(S / D)) before any rounding.  ``taps`` may be
    real or complex."""
    x = np.ascontiguousarray(x, dtype=np.int16)
    S = x.shape[-1]
    n_tr = int(np.prod(x.shape[:-1])) if x.ndim > 1 else 1
    h = np.asarray(taps)
    hr = np.ascontiguousarray(h.real, dtype=np.float64)
    hi = np.ascontiguousarray(h.imag, dtype=np.float64) if np.iscomplexobj(h) else None
    n_out = (S + D - 1) // D
    y = np.empty(x.shape[:-1] + (n_out, 2), dtype=np.float64)
    lib().oracle_demod(_ptr(x, ctypes.c_int16), n_tr, S, _ptr(hr, ctypes.c_double),
                       _ptr(hi, ctypes.c_double) if hi is not None else None, hr.size,
                       float(fd) / float(fs), int(D), _ptr(y, ctypes.c_double))
    return y[..., 0] + 1j * y[..., 1]


def quantise_iq(y: np.ndarray) -> np.ndarray:
    """Complex values -> int16 (..., 2) (re, im): round half to even, saturate."""
    y = np.asarray(y)
    v = np.ascontiguousarray(np.stack([y.real, y.imag], axis=-1), dtype=np.float64)
    q = np.empty(v.shape, dtype=np.int16)
    lib().oracle_quantise_i16(_ptr(v, ctypes.c_double), v.size, _ptr(q, ctypes.c_int16))
    return q


def _planes(desc, e):
    e = np.asarray(e)
    assert e.shape == (desc["n_tx"], desc["n_ch"], desc["n_samples"]), e.shape
    return (np.ascontiguousarray(e.real, dtype=np.float64),
            np.ascontiguousarray(e.imag, dtype=np.float64))


def das_iq(desc: dict, e: np.ndarray, c: float | None = None) -> np.ndarray:
    """Complex IQ image (Ny, Nx, Nz) of complex decoded data e (n_tx, n_ch, S).

    ``desc["fs"]`` is the IQ sampling rate and ``desc["fc"]`` the
    demodulation frequency of the phase rotation."""
    geo = Geometry(desc, c)
    er, ei = _planes(desc, e)
    o_r = np.empty(geo.shape, dtype=np.float64)
    o_i = np.empty(geo.shape, dtype=np.float64)
    lib().oracle_das_iq(ctypes.byref(geo.g), float(desc["fc"]), _ptr(er, ctypes.c_double),
                        _ptr(ei, ctypes.c_double), _ptr(o_r, ctypes.c_double),
                        _ptr(o_i, ctypes.c_double))
    return o_r + 1j * o_i


def das_iq_points(desc: dict, e: np.ndarray, vox: np.ndarray, c: float | None = None) -> np.ndarray:
    """das_iq at the listed linear voxel indices only."""
    geo = Geometry(desc, c)
    er, ei = _planes(desc, e)
    vox = np.ascontiguousarray(vox, dtype=np.int64)
    assert vox.size == 0 or (vox.min() >= 0 and vox.max() < geo.n_vox)
    o_r = np.empty(vox.shape, dtype=np.float64)
    o_i = np.empty(vox.shape, dtype=np.float64)
    lib().oracle_das_iq_points(ctypes.byref(geo.g), float(desc["fc"]), _ptr(er, ctypes.c_double),
                               _ptr(ei, ctypes.c_double), _ptr(vox, ctypes.c_int64), vox.size,
                               _ptr(o_r, ctypes.c_double), _ptr(o_i, ctypes.c_double))
    return o_r + 1j * o_i


# ---------------------------------------------------------------------------
# Envelope (analytic signal along depth) and display compression
# ---------------------------------------------------------------------------
COMPRESS = {"none": 0, "log": 1, "power": 2}


def envelope(img: np.ndarray) -> np.ndarray:
    """|analytic signal| of every depth column (last axis) of a real image."""
    x = np.ascontiguousarray(img, dtype=np.float64)
    N = x.shape[-1]
    out = np.empty_like(x)
    lib().oracle_envelope(_ptr(x, ctypes.c_double), x.size // N, N, _ptr(out, ctypes.c_double))
    return out


def compress(env: np.ndarray, mode: str = "log", ref: float = 0.0, param: float = 60.0):
    """Display compression of an envelope (see oracle_compress)."""
    e = np.ascontiguousarray(env, dtype=np.float64)
    out = np.empty_like(e)
    lib().oracle_compress(_ptr(e, ctypes.c_double), e.size, COMPRESS[mode], float(ref),
                          float(param), _ptr(out, ctypes.c_double))
    return out
