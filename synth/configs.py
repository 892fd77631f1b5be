"""Workload descriptions and seeded scenes for the five benchmark workloads.

A description is a dict of the paper's beamforming inputs (Sec. VI-B):
  mode              "forces" (2D B-scan), "hercules" (3D volume), "tpw" or "vls"
                    (row-column volumes: columns transmit tilted plane waves /
                    virtual line sources, rows receive)
  n_tx, n_ch, n_samples
  n_elem            (columns, rows) of the TOBE array
  pitch             (x, y) element pitch, metres
  xdc               4x4 row-major affine, global frame -> array frame (origin at
                    the centre of the corner element, z along the normal)
  tx_elements       element column of each decoded transmit index
  channel_map       element column (FORCES) or row (HERCULES) of each channel
  fs, fc, c, t0     sampling rate, centre frequency, sound speed, time of sample 0
  f_number          receive F# of the Hann apodization (0 = none)
  interp            "nearest" | "linear" | "cubic"
  dims, gmin, gmax  output grid: (Nx, Ny, Nz) points, inclusive bounds (global frame)
  focal_depth       optional: HERCULES diverging source depth (< 0; default +inf =
                    plane wave), VLS virtual line depth
  tx_angles         optional: TPW tilt angle of each transmit, radians
"""
from __future__ import annotations

import numpy as np

MM = 1e-3


def centered_xdc(n_elem, pitch):
    """Translation that puts the global origin at the array centre."""
    M = np.eye(4)
    M[0, 3] = (n_elem[0] - 1) / 2.0 * pitch[0]
    M[1, 3] = (n_elem[1] - 1) / 2.0 * pitch[1]
    return M


def describe(mode, n_elem, pitch, n_tx, n_ch, n_samples, fs, fc, dims, gmin, gmax,
             c=1540.0, t0=0.0, f_number=1.0, interp="cubic", tx_elements=None,
             channel_map=None, xdc=None, focal_depth=None, tx_angles=None):
    d = dict(mode=mode, n_tx=int(n_tx), n_ch=int(n_ch), n_samples=int(n_samples),
             n_elem=tuple(int(v) for v in n_elem), pitch=tuple(float(v) for v in pitch),
             fs=float(fs), fc=float(fc), c=float(c), t0=float(t0), f_number=float(f_number),
             interp=interp, dims=tuple(int(v) for v in dims),
             gmin=tuple(float(v) for v in gmin), gmax=tuple(float(v) for v in gmax))
    d["tx_elements"] = (np.arange(n_tx, dtype=np.int32) if tx_elements is None
                        else np.asarray(tx_elements, dtype=np.int32))
    d["channel_map"] = (np.arange(n_ch, dtype=np.int32) if channel_map is None
                        else np.asarray(channel_map, dtype=np.int32))
    d["xdc"] = centered_xdc(n_elem, pitch) if xdc is None else np.asarray(xdc, dtype=np.float64)
    if focal_depth is not None:
        d["focal_depth"] = float(focal_depth)
    if tx_angles is not None:
        d["tx_angles"] = np.asarray(tx_angles, dtype=np.float64)
    return d


def workload(k: int) -> dict:
    """Description of workload k in 0..3 and 5..7 (workload 4 varies per frame, see
    frame_4; workload 8 is the cross-plane pair, see cross_planes)."""
    if k == 0:   # FORCES 2D B-scan, 32x32 array
        return describe("forces", (32, 32), (0.2 * MM, 0.2 * MM), 32, 32, 1024, 20e6, 5e6,
                        (128, 1, 128), (-6.4 * MM, 0, 5 * MM), (6.4 * MM, 0, 40 * MM), t0=4e-6)
    if k in (1, 2):   # HERCULES volume, 128x128 array
        return describe("hercules", (128, 128), (0.1 * MM, 0.1 * MM), 128, 128, 2048, 30e6, 7.5e6,
                        (128, 128, 256), (-6.4 * MM, -6.4 * MM, 5 * MM),
                        (6.4 * MM, 6.4 * MM, 30 * MM))
    if k == 3:   # differentiable FORCES, 64x64 array, 256x256 image
        return describe("forces", (64, 64), (0.2 * MM, 0.2 * MM), 64, 64, 2048, 20e6, 5e6,
                        (256, 1, 256), (-6.4 * MM, 0, 5 * MM), (6.4 * MM, 0, 45 * MM))
    if k == 5:   # diverging-wave HERCULES: workload 1 with a source 20 mm behind the array
        return describe("hercules", (128, 128), (0.1 * MM, 0.1 * MM), 128, 128, 2048, 30e6, 7.5e6,
                        (128, 128, 256), (-6.4 * MM, -6.4 * MM, 5 * MM),
                        (6.4 * MM, 6.4 * MM, 30 * MM), focal_depth=-20 * MM)
    if k == 6:   # TPW row-column volume: 32 tilted plane waves over +-10 deg, 128 rows
        return describe("tpw", (128, 128), (0.1 * MM, 0.1 * MM), 32, 128, 2048, 30e6, 7.5e6,
                        (128, 128, 256), (-6.4 * MM, -6.4 * MM, 5 * MM),
                        (6.4 * MM, 6.4 * MM, 30 * MM),
                        tx_angles=np.deg2rad(np.linspace(-10.0, 10.0, 32)))
    if k == 7:   # VLS-128 row-column volume: a virtual line 10 mm behind every column
        return describe("vls", (128, 128), (0.1 * MM, 0.1 * MM), 128, 128, 2048, 30e6, 7.5e6,
                        (128, 128, 256), (-6.4 * MM, -6.4 * MM, 5 * MM),
                        (6.4 * MM, 6.4 * MM, 30 * MM), focal_depth=-10 * MM)
    raise ValueError(k)


def cross_planes():
    """Cross-plane FORCES pair (one parameter set per plane, Sec. VI-B): the
    x-z plane at y = 0 acquired with the columns, and the y-z plane at x = 0
    acquired with the rows, described as an array frame rotated by 90 degrees
    about z so that the rows play the columns' role (128x128 array, 0.1 mm,
    128 tx x 128 ch x 2048 at 30 MHz, 256 x 256 points each)."""
    n, pitch = 128, 0.1 * MM
    xz = describe("forces", (n, n), (pitch, pitch), n, n, 2048, 30e6, 7.5e6, (256, 1, 256),
                  (-6.4 * MM, 0, 5 * MM), (6.4 * MM, 0, 30 * MM))
    # global (x, y, z) -> rotated array frame (y + c, -x + c, z): rows become columns
    R = np.array([[0.0, 1.0, 0.0, (n - 1) / 2 * pitch],
                  [-1.0, 0.0, 0.0, (n - 1) / 2 * pitch],
                  [0.0, 0.0, 1.0, 0.0],
                  [0.0, 0.0, 0.0, 1.0]])
    yz = describe("forces", (n, n), (pitch, pitch), n, n, 2048, 30e6, 7.5e6, (1, 256, 256),
                  (0, -6.4 * MM, 5 * MM), (0, 6.4 * MM, 30 * MM), xdc=R)
    return [xz, yz]


def frame_4(kind: str, tx_cols) -> dict:
    """One frame of the batched uFORCES/uHERCULES stream (128x128 array, 0.1 mm)."""
    tx_cols = np.sort(np.asarray(tx_cols, dtype=np.int32))
    if kind == "2d":
        return describe("forces", (128, 128), (0.1 * MM, 0.1 * MM), len(tx_cols), 128, 2048,
                        30e6, 7.5e6, (256, 1, 256), (-6.4 * MM, 0, 5 * MM),
                        (6.4 * MM, 0, 40 * MM), tx_elements=tx_cols)
    return describe("hercules", (128, 128), (0.1 * MM, 0.1 * MM), len(tx_cols), 128, 2048,
                    30e6, 7.5e6, (96, 96, 192), (-6.4 * MM, -6.4 * MM, 5 * MM),
                    (6.4 * MM, 6.4 * MM, 30 * MM), tx_elements=tx_cols)


def _uniform_pts(rng, n, lo, hi):
    lo, hi = np.asarray(lo, dtype=np.float64), np.asarray(hi, dtype=np.float64)
    return lo + (hi - lo) * rng.random((n, 3))


def scene(k: int, rng: np.random.Generator, desc: dict | None = None):
    """Scatterer positions (global frame, metres) and amplitudes of workload k."""
    if k == 0:
        pts = _uniform_pts(rng, 8, (-3.2 * MM, 0, 5 * MM), (3.2 * MM, 0, 40 * MM))
        return pts, np.ones(8)
    if k in (1, 2):
        lo, hi = (-6.4 * MM, -6.4 * MM, 5 * MM), (6.4 * MM, 6.4 * MM, 30 * MM)
        pts = _uniform_pts(rng, 64, lo, hi)
        speckle = _uniform_pts(rng, 10000, lo, hi)
        amps = np.concatenate([np.ones(64), rng.normal(0.0, 0.1, 10000)])
        return np.concatenate([pts, speckle]), amps
    if k == 3:
        pts = _uniform_pts(rng, 8, (-5.12 * MM, 0, 5 * MM), (5.12 * MM, 0, 45 * MM))
        return pts, np.ones(8)
    if k == 4:
        g0, g1 = np.asarray(desc["gmin"]), np.asarray(desc["gmax"])
        return _uniform_pts(rng, 16, g0, g1), np.ones(16)
    raise ValueError(k)


def make_inputs(k: int, frame=None):
    """Seeded inputs; see synth.make_inputs."""
    from . import acquire, hadamard_sylvester
    rng = np.random.default_rng(1000 + k)
    if k in (0, 1, 2):
        desc = workload(k)
        pts, amps = scene(k, rng)
        H = hadamard_sylvester(desc["n_tx"])
        rf = acquire(desc, pts, amps, rng, H=H)
        return desc, H, rf, dict(points=pts, amps=amps)
    if k == 3:
        desc = workload(3)
        c_true = float(rng.uniform(1450.0, 1600.0))
        H = hadamard_sylvester(desc["n_tx"])
        frames = []
        for f in range(8):
            pts, amps = scene(3, rng)
            if frame is None or f == frame:
                frames.append((pts, amps, acquire(desc, pts, amps, rng, H=H, c=c_true)))
            else:   # keep the random stream aligned when only one frame is wanted
                rng.standard_normal((desc["n_tx"], desc["n_ch"], desc["n_samples"]))
        return desc, H, [f[2] for f in frames], dict(c_true=c_true,
                                                     points=[f[0] for f in frames])
    if k in (5, 6, 7):
        desc = workload(k)
        pts, amps = scene(1, rng)
        encoded = k == 5                      # TPW and VLS are not Hadamard-encoded
        H = hadamard_sylvester(desc["n_tx"]) if encoded else None
        rf = acquire(desc, pts, amps, rng, H=H, encoded=encoded)
        return desc, H, rf, dict(points=pts, amps=amps)
    if k == 8:
        out = []
        for desc in cross_planes():
            H = hadamard_sylvester(desc["n_tx"])
            lo, hi = np.asarray(desc["gmin"]), np.asarray(desc["gmax"])
            pts = _uniform_pts(rng, 12, lo, hi)
            out.append((desc, H, acquire(desc, pts, np.ones(12), rng, H=H)))
        return [o[0] for o in out], [o[1] for o in out], [o[2] for o in out], {}
    if k == 4:
        plan = frames_4_plan(rng)
        out = []
        for f, (kind, cols) in enumerate(plan):
            desc = frame_4(kind, cols)
            H = hadamard_sylvester(desc["n_tx"])
            pts, amps = scene(4, rng, desc)
            if frame is None or f == frame:
                out.append((desc, H, acquire(desc, pts, amps, rng, H=H)))
            else:
                rng.standard_normal((desc["n_tx"], desc["n_ch"], desc["n_samples"]))
        return ([o[0] for o in out], [o[1] for o in out], [o[2] for o in out],
                dict(plan=plan))
    raise ValueError(k)


def frames_4_plan(rng: np.random.Generator, n_frames: int = 64):
    """Per-frame (kind, transmit columns) of the batched stream."""
    plan = []
    for _ in range(n_frames):
        n_tx = int(rng.choice([16, 32, 64, 128]))
        cols = np.sort(rng.choice(128, size=n_tx, replace=False)).astype(np.int32)
        kind = "2d" if rng.random() < 0.5 else "3d"
        plan.append((kind, cols))
    return plan


def lowpass_taps(n_taps: int, cutoff: float) -> np.ndarray:
    """Hamming-windowed sinc low-pass, cutoff in cycles/sample, unit DC gain.

    Input generation only: the paper's filters (a 36-tap low-pass for volumes,
    a 166-tap matched chirp filter for B-scans) are inputs to the method; this
    stands in for the low-pass one."""
    n = np.arange(n_taps) - (n_taps - 1) / 2.0
    h = 2 * cutoff * np.sinc(2 * cutoff * n) * np.hamming(n_taps)
    return h / h.sum()


def iq_frontend(desc: dict, n_taps: int = 36, decimation: int = 2):
    """Demodulation setup for an RF workload: (taps, decimation, IQ description).

    The RF is demodulated at its centre frequency with a low-pass of cutoff
    fc / 2 (the echo band is about +-0.4 fc around the carrier), decimated by
    `decimation`, and beamformed as IQ data: fs becomes fs / D, n_samples
    ceil(S / D), and t0 moves back by the filter's group delay (N_f - 1) / 2
    input samples so that IQ sample q lines up with record time."""
    fs, fc = float(desc["fs"]), float(desc["fc"])
    taps = lowpass_taps(n_taps, 0.5 * fc / fs)
    d = dict(desc)
    d["iq"] = True
    d["fs"] = fs / decimation
    d["n_samples"] = (int(desc["n_samples"]) + decimation - 1) // decimation
    d["t0"] = float(desc["t0"]) - (n_taps - 1) / 2.0 / fs
    return taps, decimation, d
