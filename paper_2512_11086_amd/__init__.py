"""MI355X-native Hadamard aperture decoding + delay-and-sum beamforming.

Python face of libbf (include/bf.h).  Every step of the path runs in the HIP
kernels of libbf; this module only converts a problem description into the
C structure, passes device pointers of torch tensors (torch is used for
device memory and streams) and raises ``BfError`` on a failed status.

A problem description is a dict with the paper's inputs (Sec. VI-B): mode,
n_tx, n_ch, n_samples, n_elem, pitch, xdc (4x4 global -> array frame),
tx_elements, channel_map, fs, fc, c, t0, f_number, interp, dims, gmin, gmax,
and optionally iq (complex baseband data; fs is then the IQ rate and fc the
demodulation frequency).
"""
from __future__ import annotations

import ctypes
import math

import numpy as np

from ._lib import (BATCH_PATHS, BatchFrameInfo, BfError, COMPRESS, DECODE_ALGOS, DemodParams,
                   ETYPES, INTERPS, IQ_TYPES, MODES, Params, PlanInfo, VARIANTS, check, lib)

__all__ = ["BfError", "Plan", "BatchPlan", "Demod", "Envelope", "params_from_desc", "sharpness",
           "validate"]


class _Marshalled:
    """A bf_params plus the numpy arrays its pointers refer to."""

    def __init__(self, desc: dict, hadamard, e_type="f32", decode_algo="mfma"):
        p = Params()
        p.mode = MODES[desc["mode"]]
        p.n_tx, p.n_ch, p.n_samples = int(desc["n_tx"]), int(desc["n_ch"]), int(desc["n_samples"])
        p.n_elem[:] = [int(v) for v in desc["n_elem"]]
        p.pitch[:] = [float(v) for v in desc["pitch"]]
        p.xdc_transform[:] = [float(v) for v in np.asarray(desc["xdc"], dtype=np.float64).reshape(16)]
        self.H = None if hadamard is None else np.ascontiguousarray(hadamard, dtype=np.int8)
        self.tx = None if desc.get("tx_elements") is None else np.ascontiguousarray(
            desc["tx_elements"], dtype=np.int32)
        self.ch = None if desc.get("channel_map") is None else np.ascontiguousarray(
            desc["channel_map"], dtype=np.int32)
        P = ctypes.POINTER
        p.hadamard = self.H.ctypes.data_as(P(ctypes.c_int8)) if self.H is not None else None
        p.tx_elements = self.tx.ctypes.data_as(P(ctypes.c_int32)) if self.tx is not None else None
        p.channel_map = self.ch.ctypes.data_as(P(ctypes.c_int32)) if self.ch is not None else None
        p.fs, p.fc, p.c, p.t0 = (float(desc[k]) for k in ("fs", "fc", "c", "t0"))
        p.focal_depth = float(desc.get("focal_depth", math.inf))
        p.f_number = float(desc["f_number"])
        p.interp = INTERPS[desc.get("interp", "cubic")]
        p.e_type = ETYPES[e_type]
        p.decode_algo = DECODE_ALGOS[decode_algo]
        p.out_dims[:] = [int(v) for v in desc["dims"]]
        p.out_min[:] = [float(v) for v in desc["gmin"]]
        p.out_max[:] = [float(v) for v in desc["gmax"]]
        p.iq = 1 if desc.get("iq", False) else 0
        self.ang = (None if desc.get("tx_angles") is None
                    else np.ascontiguousarray(desc["tx_angles"], dtype=np.float64))
        p.tx_angles = self.ang.ctypes.data_as(P(ctypes.c_double)) if self.ang is not None else None
        self.p = p


def params_from_desc(desc, hadamard, e_type="f32", decode_algo="mfma") -> _Marshalled:
    return _Marshalled(desc, hadamard, e_type, decode_algo)


def validate(desc, hadamard, **kw) -> None:
    """Validate a description on the host (raises BfError)."""
    m = _Marshalled(desc, hadamard, **kw)
    check(lib().bf_validate(ctypes.byref(m.p)))


def _torch():
    import torch
    return torch


def _stream(stream):
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _check_tensor(t, name, dtype, shape=None, device=None):
    """Reject, before any library call, a tensor the kernels cannot take: a
    host tensor (its pointer would reach a kernel as a device address), one
    on another device than the call's other tensors, or one of the wrong
    dtype, shape or layout."""
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (device) tensor")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, the call's other tensors on {device}")
    if t.dtype != dtype:
        raise ValueError(f"{name} must have dtype {dtype}, not {t.dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


_TORCH_ETYPE = {"f32": "float32", "bf16": "bfloat16", "i32": "int32"}


class Plan:
    """Single-frame plan: bf_decode, bf_das, bf_das_adjoint on torch tensors."""

    def __init__(self, desc: dict, hadamard, e_type: str = "f32", decode_algo: str = "mfma",
                 tile=None):
        self.desc = desc
        self.e_type = e_type
        self._m = _Marshalled(desc, hadamard, e_type, decode_algo)
        h = ctypes.c_void_p()
        check(lib().bf_plan_create(ctypes.byref(self._m.p), ctypes.byref(h)))
        self._h = h
        self.n_tx, self.n_ch, self.n_samples = (int(desc[k]) for k in ("n_tx", "n_ch", "n_samples"))
        nx, ny, nz = (int(v) for v in desc["dims"])
        self.out_shape = (ny, nx, nz)
        self.iq = bool(desc.get("iq", False))
        # IQ plans: rf int16 and e float32 carry a trailing (re, im) axis; the
        # image is complex64
        tail = (2,) if self.iq else ()
        self.rf_shape = (self.n_tx, self.n_ch, self.n_samples) + tail
        self.e_shape = self.rf_shape
        self.c = float(desc["c"])
        if tile is not None:
            self.set_tile(*tile)

    def close(self):
        if getattr(self, "_h", None):
            check(lib().bf_plan_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> dict:
        inf = PlanInfo()
        check(lib().bf_plan_get_info(self._h, ctypes.byref(inf)))
        return dict(n_frames=inf.n_frames, tile=tuple(inf.tile), variant=inf.variant,
                    block=tuple(inf.block), nb=inf.nb,
                    workspace_bytes=inf.workspace_bytes, e_elems=inf.e_elems,
                    out_elems=inf.out_elems, channel_groups=inf.channel_groups)

    def set_tile(self, lx: int, ly: int, lz: int):
        check(lib().bf_set_tile(self._h, lx, ly, lz))

    def set_das_config(self, variant: str = "lds", block=(4, 4, 1), nb: int = 16):
        """variant: "lds" (LDS-staged windows), "gather" (direct gather) or
        "lds2" (LDS windows, two adjacent depth points per lane; HERCULES
        plans with real data)."""
        v = VARIANTS[variant]
        check(lib().bf_set_das_config(self._h, v, *[int(b) for b in block], int(nb)))

    def autotune(self, cache_path: str | None = None):
        check(lib().bf_autotune(self._h, cache_path.encode() if cache_path else None))
        return self.info()

    def e_dtype(self):
        return getattr(_torch(), _TORCH_ETYPE[self.e_type])

    def _check_rf(self, rf):
        _check_tensor(rf, "rf", _torch().int16, self.rf_shape)

    def _check_e(self, e, name="e", device=None):
        """Number of stacked frames of e: None for one frame of the plan's
        shape, F for an (F, *e_shape) stack."""
        _check_tensor(e, name, self.e_dtype(), device=device)
        if tuple(e.shape) == self.e_shape:
            return None
        if e.dim() == len(self.e_shape) + 1 and tuple(e.shape[1:]) == self.e_shape:
            return int(e.shape[0])
        raise ValueError(f"{name} has the wrong shape")

    def decode(self, rf, out=None, stream=None):
        torch = _torch()
        self._check_rf(rf)
        if out is None:
            out = torch.empty(rf.shape, dtype=self.e_dtype(), device=rf.device)
        if self._check_e(out, "out", rf.device) is not None:
            raise ValueError("out must hold one frame")
        check(lib().bf_decode(self._h, _ptr(rf), _ptr(out), _stream(stream)))
        return out

    def das(self, e, c: float | None = None, out=None, stream=None):
        """Image of e at sound speed c (the plan's by default).  e may be a
        stack (F, n_tx, n_ch, S) of frames: one call beamforms all of them
        (bf_das_frames) into an (F, *image shape) output."""
        torch = _torch()
        nf = self._check_e(e)
        odt = torch.complex64 if self.iq else torch.float32
        shape = self.out_shape if nf is None else (nf,) + self.out_shape
        if out is None:
            out = torch.empty(shape, dtype=odt, device=e.device)
        _check_tensor(out, "out", odt, shape, e.device)
        cv = float(self.c if c is None else c)
        if nf is None:
            check(lib().bf_das(self._h, _ptr(e), _ptr(out), cv, _stream(stream)))
        else:
            check(lib().bf_das_frames(self._h, _ptr(e), nf, _ptr(out), cv, _stream(stream)))
        return out

    def das_fused(self, rf, c: float | None = None, out=None, stream=None):
        """Decode fused into DAS (bf_das_fused, FORCES planes): the image of
        the int16 RF ``rf`` (n_tx, n_ch, S) in one kernel, equal bit for bit to
        ``das(decode(rf))`` when the plan decodes to exact values (f32 or i32;
        a bf16 plan's decode rounds, the fused taps do not)."""
        torch = _torch()
        self._check_rf(rf)
        if out is None:
            out = torch.empty(self.out_shape, dtype=torch.float32, device=rf.device)
        _check_tensor(out, "out", torch.float32, self.out_shape, rf.device)
        cv = float(self.c if c is None else c)
        check(lib().bf_das_fused(self._h, _ptr(rf), _ptr(out), cv, _stream(stream)))
        return out

    def das_adjoint(self, e, grad_out, c: float | None = None, want_e: bool = True,
                    want_c: bool = True, stream=None, out_e=None):
        """Returns (grad_e or None, grad_c tensor of shape () or None).

        ``e`` may be None when only grad_e is wanted (it does not depend on
        the data); ``out_e`` is an optional float32 buffer for grad_e.  A
        stack of frames (grad_out of shape (F, *image shape), e of shape
        (F, n_tx, n_ch, S)) runs bf_das_adjoint_frames: grad_e has shape
        (F, n_tx, n_ch, S) and grad_c shape (F,), one dL/dc term per frame."""
        torch = _torch()
        if not isinstance(grad_out, torch.Tensor) or not grad_out.is_cuda:
            raise ValueError("grad_out must be a CUDA (device) tensor")
        nf_e = self._check_e(e, "e", grad_out.device) if e is not None else None
        g = grad_out.contiguous().to(torch.float32)
        if tuple(g.shape) == self.out_shape:
            nf = None
        elif g.dim() == len(self.out_shape) + 1 and tuple(g.shape[1:]) == self.out_shape:
            nf = int(g.shape[0])
        else:
            raise ValueError("grad_out has the wrong shape")
        if e is not None and nf_e != nf:
            raise ValueError("e and grad_out hold different numbers of frames")
        lead = () if nf is None else (nf,)
        shape_e = lead + (self.n_tx, self.n_ch, self.n_samples)
        if want_e and out_e is not None:
            _check_tensor(out_e, "out_e", torch.float32, shape_e, g.device)
            ge = out_e
        else:
            ge = (torch.empty(shape_e, dtype=torch.float32, device=g.device)
                  if want_e else None)
        gc = torch.empty(lead, dtype=torch.float32, device=g.device) if want_c else None
        args = (_ptr(ge) if ge is not None else None, _ptr(gc) if gc is not None else None,
                _stream(stream))
        ep = _ptr(e) if e is not None else None
        cv = float(self.c if c is None else c)
        if nf is None:
            check(lib().bf_das_adjoint(self._h, ep, _ptr(g), cv, *args))
        else:
            check(lib().bf_das_adjoint_frames(self._h, ep, _ptr(g), nf, cv, *args))
        return ge, gc


class Demod:
    """bf_demodulate: mix with exp(-j 2 pi fd n / fs), FIR-filter, decimate (Eq. 4).

    ``taps`` is a real or complex 1-D sequence; ``out`` "i16" gives the int16
    (re, im) layout an IQ plan decodes, "f32" float32 pairs."""

    def __init__(self, n_traces: int, n_samples: int, taps, fd: float, fs: float,
                 decimation: int = 1, out: str = "i16"):
        h = np.asarray(taps)
        self._re = np.ascontiguousarray(h.real, dtype=np.float64).reshape(-1)
        self._im = (np.ascontiguousarray(h.imag, dtype=np.float64).reshape(-1)
                    if np.iscomplexobj(h) else None)
        P = ctypes.POINTER(ctypes.c_double)
        p = DemodParams()
        p.n_traces, p.n_samples = int(n_traces), int(n_samples)
        p.decimation, p.n_taps = int(decimation), int(self._re.size)
        p.taps_re = self._re.ctypes.data_as(P)
        p.taps_im = self._im.ctypes.data_as(P) if self._im is not None else None
        p.fs, p.fd = float(fs), float(fd)
        p.out_type = IQ_TYPES[out]
        self.out = out
        h_ = ctypes.c_void_p()
        check(lib().bf_demod_create(ctypes.byref(p), ctypes.byref(h_)))
        self._h = h_
        n = ctypes.c_int32()
        check(lib().bf_demod_out_samples(self._h, ctypes.byref(n)))
        self.n_traces, self.n_samples, self.n_out = int(n_traces), int(n_samples), int(n.value)

    def close(self):
        if getattr(self, "_h", None):
            check(lib().bf_demod_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __call__(self, rf, out=None, stream=None):
        """rf: contiguous int16 CUDA tensor whose last axis is the n_samples and
        whose leading axes hold n_traces traces; returns (..., n_out, 2)."""
        torch = _torch()
        _check_tensor(rf, "rf", torch.int16)
        if rf.shape[-1] != self.n_samples or rf.numel() != self.n_traces * self.n_samples:
            raise ValueError("rf does not hold n_traces x n_samples samples")
        shape = tuple(rf.shape[:-1]) + (self.n_out, 2)
        dt = torch.int16 if self.out == "i16" else torch.float32
        if out is None:
            out = torch.empty(shape, dtype=dt, device=rf.device)
        _check_tensor(out, "out", dt, shape, rf.device)
        check(lib().bf_demodulate(self._h, _ptr(rf), _ptr(out), _stream(stream)))
        return out


class Envelope:
    """bf_envelope: |analytic signal| along depth (or |z| of an IQ image) with
    optional log / power compression, for images whose last axis is depth."""

    def __init__(self, shape, iq: bool = False):
        shape = tuple(int(v) for v in shape)
        self.shape, self.iq = shape, bool(iq)
        self.n = shape[-1]
        self.n_cols = int(np.prod(shape[:-1])) if len(shape) > 1 else 1
        h = ctypes.c_void_p()
        check(lib().bf_env_create(self.n_cols, self.n, 1 if iq else 0, ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            check(lib().bf_env_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __call__(self, img, compress: str = "none", ref: float = 0.0, param: float = 60.0,
                 out=None, stream=None):
        torch = _torch()
        dt = torch.complex64 if self.iq else torch.float32
        _check_tensor(img, "img", dt, self.shape)
        if out is None:
            out = torch.empty(self.shape, dtype=torch.float32, device=img.device)
        _check_tensor(out, "out", torch.float32, self.shape, img.device)
        check(lib().bf_envelope(self._h, _ptr(img), _ptr(out), COMPRESS[compress], float(ref),
                                float(param), _stream(stream)))
        return out


class BatchPlan:
    """Plan over many frames with their own descriptions (persistent batched path)."""

    def __init__(self, descs, hadamards, e_type: str = "f32"):
        self.descs = list(descs)
        self._ms = [_Marshalled(d, H, e_type) for d, H in zip(self.descs, hadamards)]
        arr = (Params * len(self._ms))(*[m.p for m in self._ms])
        self._arr = arr
        h = ctypes.c_void_p()
        check(lib().bf_plan_create_batch(arr, len(self._ms), ctypes.byref(h)))
        self._h = h
        self.out_shapes = [(int(d["dims"][1]), int(d["dims"][0]), int(d["dims"][2]))
                           for d in self.descs]

    def close(self):
        if getattr(self, "_h", None):
            check(lib().bf_plan_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _ptrs(self, tensors):
        return (ctypes.c_void_p * len(tensors))(*[t.data_ptr() for t in tensors])

    def _check_frames(self, rfs, outs):
        """One int16 RF tensor and one float32 output tensor per frame, of the
        frame's shapes, all on one device (the library reads n_frames
        pointers from each list)."""
        torch = _torch()
        rfs, outs = list(rfs), list(outs)
        n = len(self.descs)
        if len(rfs) != n or len(outs) != n:
            raise ValueError(f"need {n} rf and {n} out tensors, got {len(rfs)} and {len(outs)}")
        dev = rfs[0].device if n and isinstance(rfs[0], torch.Tensor) else None
        for f, (d, r, o) in enumerate(zip(self.descs, rfs, outs)):
            iq = bool(d.get("iq", False))     # (the library refuses IQ frames in a batch)
            shape_rf = (int(d["n_tx"]), int(d["n_ch"]), int(d["n_samples"])) + ((2,) if iq else ())
            _check_tensor(r, f"rfs[{f}]", torch.int16, shape_rf, dev)
            _check_tensor(o, f"outs[{f}]", torch.complex64 if iq else torch.float32,
                          self.out_shapes[f], dev)
        return rfs, outs

    def run(self, rfs, outs, stream=None):
        rfs, outs = self._check_frames(rfs, outs)
        check(lib().bf_batch_run(self._h, self._ptrs(rfs), self._ptrs(outs), _stream(stream)))

    def graph_launch(self, rfs, outs, stream=None):
        rfs, outs = self._check_frames(rfs, outs)
        check(lib().bf_graph_launch(self._h, self._ptrs(rfs), self._ptrs(outs), _stream(stream)))

    def autotune(self, cache_path: str | None = None):
        check(lib().bf_autotune(self._h, cache_path.encode() if cache_path else None))

    def frame_info(self, frame: int) -> dict:
        """How the batched path runs a frame (after the first run/graph_launch)."""
        inf = BatchFrameInfo()
        check(lib().bf_batch_get_frame_info(self._h, int(frame), ctypes.byref(inf)))
        return dict(das_path=BATCH_PATHS[inf.das_path], das_class=inf.das_class,
                    channel_groups=inf.channel_groups, decode_class=inf.decode_class,
                    das_items=inf.das_items)

    def set_das_config(self, variant: str = "lds", block=(4, 4, 1), nb: int = 16):
        """As Plan.set_das_config, for every frame (before the first launch)."""
        check(lib().bf_set_das_config(self._h, VARIANTS[variant], *[int(b) for b in block],
                                      int(nb)))


def sharpness(img, grad: bool = True, stream=None):
    """Negative normalised L4 norm per image of a (n_images, ...) float32 tensor."""
    torch = _torch()
    if not isinstance(img, torch.Tensor) or not img.is_cuda:
        raise ValueError("img must be a CUDA (device) tensor")
    x = img.contiguous()
    if x.dtype != torch.float32:
        raise ValueError("img must be float32")
    n_images = x.shape[0] if x.dim() > 1 else 1
    n = x.numel() // n_images
    loss = torch.empty(n_images, dtype=torch.float32, device=x.device)
    g = torch.empty_like(x) if grad else None
    check(lib().bf_sharpness(_ptr(x), n, n_images, _ptr(loss), _ptr(g) if g is not None else None,
                             _stream(stream)))
    return (loss, g) if grad else loss
