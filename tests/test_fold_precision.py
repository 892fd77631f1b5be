"""FP32 rounding of the folded window position of the separable forward
kernels (CPU emulation of the kernel's arithmetic).

The plane kernel takes a term's quad index and fraction from one FP32 sum,
(fB + k E_rx + nB - B_j - hc) + (k E_tx - A_i), where the window start of
trace (i, j) is split into A_i = floor(k tx_lo_i - Zb) and
B_j = floor(k rx_lo_j + Zb - t0 fs) - 2 (Zb = k times the box's top depth)
and hc = lmax / 4 centres the sum.  The unsplit form rounds
fB + k E_rx + k E_tx (one FMA) and adds the integers exactly.  Both are
emulated here step by step in FP32 (numpy float32, each operation rounded
once; FMAs rounded once from FP64) for the active (point, row) pairs of
sampled boxes of the workload-3 plane (FORCES, 64 x 64 traces, 256 x 256
points, F# 1) and compared with the FP64 position: the folded form stays
within a small factor of the unsplit one, and far below the 1e-4 samples at
which the 1e-5 image bound would be at risk.
"""
import math

import numpy as np

import synth
from tests.test_window_bounds import _dist, _grid


def _r32(x):
    return np.asarray(x, np.float64).astype(np.float32)


def _position_errors(desc, tile, bw, boxes, lmax):
    nx, ny, nz = desc["dims"]
    org, ax, ay, az, centre = _grid(desc)
    n_tx = desc["n_tx"]
    tx_x = np.arange(n_tx) * desc["pitch"][0] - centre[0]
    rx_c = np.arange(desc["n_ch"]) * desc["pitch"][0] - centre[0]
    k, t0fs = desc["fs"] / desc["c"], desc["t0"] * desc["fs"]
    kf, t0f = np.float32(k), np.float32(t0fs)
    f2 = desc["f_number"] ** 2
    tx, tz = bw[0] << tile[0], bw[2] << tile[2]
    hc = lmax >> 2
    e_old, e_new = [], []

    def excess(r2, Lz, Lz2):       # rho2 * rcp(sqrt(rho2 + z2) + z), each step rounded
        d = _r32(np.sqrt(_r32(r2.astype(np.float64) + Lz2)))
        return _r32(r2.astype(np.float64) * _r32(1.0 / _r32(d.astype(np.float64) + Lz)))

    for bx, bz in boxes:
        i0x, i1x = bx * tx, min(bx * tx + tx - 1, nx - 1)
        i0z, i1z = bz * tz, min(bz * tz + tz - 1, nz - 1)
        xmin, xmax = _r32(org[0] + i0x * ax[0]), _r32(org[0] + i1x * ax[0])
        zlo = max(_r32(org[2] + i0z * az[2]), np.float32(0))
        IX, IZ = np.meshgrid(np.arange(i0x, i0x + tx).clip(0, nx - 1),
                             np.arange(i0z, i0z + tz).clip(0, nz - 1), indexing="ij")
        px = (org[0] + IX * ax[0]).ravel()
        pz = np.maximum((org[2] + IZ * az[2]).ravel(), 1e-7)
        B = 2 * pz * k - t0fs
        nB = np.floor(B).astype(np.int64)
        fB = _r32(B - np.floor(B))
        Lx, Lz = _r32(px), _r32(pz)
        Lz2 = _r32(Lz.astype(np.float64) * Lz)
        thr = _r32(Lz2 * np.float32(0.25) / np.float32(f2))
        zb = _r32(np.float64(kf) * zlo)
        for cj in rx_c.astype(np.float32):
            rr = _r32(_dist(float(cj), float(xmin), float(xmax)))
            rxlo = _r32(math.sqrt(float(rr) ** 2 + float(zlo) ** 2))
            dxr = _r32(Lx.astype(np.float64) - cj)
            r2 = _r32(dxr.astype(np.float64) * dxr)
            act = r2 < thr
            if not act.any():
                continue
            Rj = _r32(excess(r2, Lz, Lz2).astype(np.float64) * kf + fB)          # FMA
            Bj = math.floor(_r32(np.float64(kf) * rxlo + (np.float64(zb) - t0f))) - 2
            Rj2 = _r32(Rj.astype(np.float64) + _r32(nB - Bj - hc))
            rxp = np.sqrt((px - float(cj)) ** 2 + pz ** 2)
            for xi in tx_x.astype(np.float32):
                rt = _r32(_dist(float(xi), float(xmin), float(xmax)))
                txlo = _r32(math.sqrt(float(rt) ** 2 + float(zlo) ** 2))
                w0_old = math.floor(_r32(_r32(np.float64(txlo) + rxlo) * np.float64(kf) - t0f)) - 2
                Ai = math.floor(_r32(np.float64(kf) * txlo - zb))
                dxt = _r32(Lx.astype(np.float64) - xi)
                ext = excess(_r32(dxt.astype(np.float64) * dxt), Lz, Lz2)
                s_abs = k * (np.sqrt((px - float(xi)) ** 2 + pz ** 2) + rxp) - t0fs
                sq = _r32(ext.astype(np.float64) * kf + Rj)                         # FMA
                pos_old = np.floor(sq) + nB - w0_old + (sq - np.floor(sq))
                T2 = _r32(np.float64(kf) * ext - Ai)                                # FMA
                pos_new = _r32(Rj2.astype(np.float64) + T2).astype(np.float64) + hc
                e_old.append((pos_old - (s_abs - w0_old))[act])
                e_new.append((pos_new - (s_abs - (Ai + Bj)))[act])
    return np.concatenate(e_old), np.concatenate(e_new)


def test_folded_position_rounding_workload3_plane():
    desc = synth.configs.workload(3)
    # default plane box: 32 x 2 lane tiles, 2 x 1 x 8 wavefronts (64 x 16 points);
    # lmax of that box with the fold (as tests/test_window_bounds.py derives it:
    # 127), rounded up to even as real data is staged in pairs of quads
    e_old, e_new = _position_errors(desc, (5, 0, 1), (2, 1, 8), [(1, 3), (2, 10), (3, 15)], 128)
    rms_old, rms_new = np.sqrt((e_old ** 2).mean()), np.sqrt((e_new ** 2).mean())
    assert len(e_new) > 10 ** 6
    assert rms_new <= 2.0 * rms_old and rms_new < 5e-6, (rms_old, rms_new)
    assert np.abs(e_new).max() < 1e-4, np.abs(e_new).max()


def _hercules_position_errors(desc, tile, bw, zp, boxes):
    """Errors against FP64 of the HERCULES window position (in samples) in the
    unsplit form, floor(B) + FP32 fma(rho^2, 1/(d/k + z/k), frac(B)), and in
    the folded form, nR + FP32 fma(rho^2, 1/(d/k + z/k), B - nR), where nR =
    floor(k (txlo + zmax) - t0 fs) is the box's reference sample (plane
    transmit: txlo = the box's top depth), over every receive element of the
    active (point, element) pairs of the sampled boxes."""
    nx, ny, nz = desc["dims"]
    org, ax, ay, az, centre = _grid(desc)
    ne, pitch = desc["n_elem"], desc["pitch"]
    xs = (np.arange(ne[0]) * pitch[0] - centre[0]).astype(np.float32)
    ys = (np.arange(ne[1]) * pitch[1] - centre[1]).astype(np.float32)
    k, t0fs = desc["fs"] / desc["c"], desc["t0"] * desc["fs"]
    kf, t0f = np.float32(k), np.float32(t0fs)
    ik2 = np.float32(1.0 / (k * k))
    f2 = desc["f_number"] ** 2
    tx, ty, tz = bw[0] << tile[0], bw[1] << tile[1], (bw[2] << tile[2]) * zp
    e_old, e_new = [], []
    for bx, by, bz in boxes:
        i0 = [bx * tx, by * ty, bz * tz]
        i1 = [min(i0[0] + tx - 1, nx - 1), min(i0[1] + ty - 1, ny - 1), min(i0[2] + tz - 1, nz - 1)]
        zlo = max(_r32(org[2] + i0[2] * az[2]), np.float32(0))
        zmax = max(_r32(org[2] + i1[2] * az[2]), np.float32(0))
        nR = math.floor(_r32(np.float64(_r32(np.float64(zlo) + zmax)) * kf - t0f))    # FMA
        IX, IY, IZ = np.meshgrid(np.arange(i0[0], i0[0] + tx).clip(0, nx - 1),
                                 np.arange(i0[1], i0[1] + ty).clip(0, ny - 1),
                                 np.arange(i0[2], i0[2] + tz).clip(0, nz - 1), indexing="ij")
        px = (org[0] + IX * ax[0]).ravel()
        py = (org[1] + IY * ay[1]).ravel()
        pz = np.maximum((org[2] + IZ * az[2]).ravel(), 1e-7)
        B = 2 * pz * k - t0fs
        nB = np.floor(B)
        fB_old, fB_new = _r32(B - nB), _r32(B - nR)
        Lx, Ly = _r32(px), _r32(py)
        zk = _r32(pz / k)
        zk2 = _r32(zk.astype(np.float64) * zk)
        for yj in ys:
            dy = _r32(Ly.astype(np.float64) - yj)
            dy2 = _r32(dy.astype(np.float64) * dy)
            dx = _r32(Lx[:, None].astype(np.float64) - xs[None, :])
            rho2 = _r32(dx.astype(np.float64) * dx + dy2[:, None])                      # FMA
            dk = _r32(np.sqrt(_r32(rho2.astype(np.float64) * ik2 + zk2[:, None])))       # FMA, sqrt
            r = _r32(1.0 / _r32(dk.astype(np.float64) + zk[:, None]))
            s_old = _r32(rho2.astype(np.float64) * r + fB_old[:, None])                  # FMA
            s_new = _r32(rho2.astype(np.float64) * r + fB_new[:, None])                  # FMA
            r2 = (px[:, None] - xs[None, :]) ** 2 + (py[:, None] - float(yj)) ** 2
            exact = B[:, None] + k * (np.sqrt(r2 + pz[:, None] ** 2) - pz[:, None])
            act = r2 < pz[:, None] ** 2 * 0.25 / f2
            e_old.append((s_old + nB[:, None] - exact)[act])
            e_new.append((s_new.astype(np.float64) + nR - exact)[act])
    return np.concatenate(e_old), np.concatenate(e_new)


def test_folded_position_rounding_workload1_volume():
    desc = synth.configs.workload(1)
    # default HERCULES box: 8 x 8 lane tiles, 2 x 2 x 3 wavefronts, two depth
    # points per lane (16 x 16 x 6 points); shallow, middle and deep boxes
    e_old, e_new = _hercules_position_errors(desc, (3, 3, 0), (2, 2, 3), 2,
                                             [(3, 4, 2), (4, 3, 20), (2, 5, 40)])
    rms_old, rms_new = np.sqrt((e_old ** 2).mean()), np.sqrt((e_new ** 2).mean())
    assert len(e_new) > 10 ** 6
    assert rms_new <= 1.5 * rms_old and rms_new < 5e-6, (rms_old, rms_new)
    assert np.abs(e_new).max() < 1e-4, np.abs(e_new).max()
