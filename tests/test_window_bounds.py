"""The LDS DAS kernels read staged windows without clamping the index (CPU).

For every lane of a workgroup box (each lane takes the nearest grid point of
its box, depth at least 1e-7) and every trace the box stages, the window
index floor(s) - w0 must lie in [-1, lmax + guard): -1 reads finite LDS data
before the windows, indices past a window read the next window or the zeroed
guard.  This re-derives, in FP64, the kernels' window start (the box's lowest
path, floored 2 samples down), the staged length lmax (Frame::lds_config: the
delay spread of active points plus 5) and the guard ((1 - srx) times the
receive-lateral extent, plus 3; real data, staged in pairs of quads, rounds
lmax up to even, which only widens the windows, so the checks take the
unrounded length), and checks them on sampled boxes of the
workload geometries and of small grids (tilted, through the array plane,
diverging, VLS focal lines, several F#).  Active points (apodization > 0)
must also read inside their own window: index at most lmax - 1 (the quad
covers taps n-1 .. n+2).  Paths per Table I's methods: HERCULES
tx = z (plane) or |p - v| - f (diverging), rx = |p - (x_i, y_j, 0)|; FORCES
tx = |p - col_i|_xz, rx = |p - col_j|_xz; TPW tx = x sin a + z cos a; VLS
tx = z_f + sgn(z - z_f) |(x - x_i, z - z_f)|; row receivers |(y - y_j, z)|.

The separable forward kernels on real data (FORCES, TPW, VLS) split the
start into a transmit part and a row part, each floored:
floor(k tx_lo - Zb) + floor(k rx_lo + Zb - t0 fs) - 2 with Zb = k times the
box's top depth, one quad longer windows and a guard two entries longer
(`fold`).  Their terms take the index as the floor of an FP32 sum, which may
round across an integer: there the index must fit with one entry to spare
at either end (at least 1, below lmax - 1 for active points, below
lmax + guard - 1 for all).
"""
import math

import numpy as np
import pytest

import synth
from synth.configs import MM, describe


def _grid(desc):
    M = np.asarray(desc["xdc"], dtype=np.float64).reshape(4, 4)
    gmin, gmax = np.array(desc["gmin"]), np.array(desc["gmax"])
    dims = desc["dims"]
    step = [(gmax[a] - gmin[a]) / (dims[a] - 1) if dims[a] > 1 else 0.0 for a in range(3)]
    R, T = M[:3, :3], M[:3, 3]
    ne, pitch = desc["n_elem"], desc["pitch"]
    centre = np.array([(ne[0] - 1) / 2 * pitch[0], (ne[1] - 1) / 2 * pitch[1], 0.0])
    org = R @ gmin + T - centre
    return org, R[:, 0] * step[0], R[:, 1] * step[1], R[:, 2] * step[2], centre


def _dist(v, a, b):
    return max(0.0, a - v, v - b)


def _far(v, a, b):
    return max(abs(v - a), abs(v - b))


def window_range(desc, tile, bw, zp=1, nboxes=8, seed=0, fold=False):
    """(min, max) of the window index over sampled boxes, the max over
    active points, lmax and lmax + guard."""
    mode = desc["mode"]
    nx, ny, nz = desc["dims"]
    org, ax, ay, az, centre = _grid(desc)
    n_tx = desc["n_tx"]
    tx_el = np.asarray(desc["tx_elements"] if desc.get("tx_elements") is not None
                       else np.arange(n_tx), float)
    ch = np.asarray(desc["channel_map"] if desc.get("channel_map") is not None
                    else np.arange(desc["n_ch"]), float)
    px_, py_ = desc["pitch"]
    tx_x = tx_el * px_ - centre[0]
    rx_c = ch * px_ - centre[0] if mode == "forces" else ch * py_ - centre[1]
    k, t0fs = desc["fs"] / desc["c"], desc["t0"] * desc["fs"]
    f2 = desc["f_number"] ** 2
    fd = desc.get("focal_depth", math.inf)
    div_f = -fd if mode == "hercules" and math.isfinite(fd) else 0.0
    zf = fd if mode == "vls" else 0.0
    ang = np.asarray(desc.get("tx_angles", np.zeros(n_tx)), float)
    lx, ly, lz = tile
    tx, ty, tz = bw[0] << lx, bw[1] << ly, (bw[2] << lz) * zp
    z_off = 0
    if mode == "vls":
        below = [np.float32(org[2] + iz * az[2]) - np.float32(zf) < 0 for iz in range(nz)]
        for iz in range(1, nz):
            if below[iz] != below[iz - 1]:
                z_off = (tz - iz % tz) % tz
                break
    E = [abs(ax[r]) * (tx - 1) + abs(ay[r]) * (ty - 1) + abs(az[r]) * (tz - 1) for r in range(3)]
    lat = math.hypot(E[0], E[1])
    srx = 1 / math.sqrt(1 + 4 * f2) if f2 > 0 else 1.0
    if mode == "forces":
        spread, rx_lat = 2 * E[2] + (1 + srx) * E[0], E[0]
    elif mode == "tpw":
        spread, rx_lat = 2 * E[2] + srx * E[1] + np.abs(np.sin(ang)).max() * E[0], E[1]
    elif mode == "vls":
        spread, rx_lat = E[2] + srx * E[1] + math.hypot(E[0], E[2]), E[1]
    else:
        spread = (E[2] + srx * lat + math.hypot(lat, E[2])) if div_f > 0 else 2 * E[2] + srx * lat
        rx_lat = lat
    lmax = math.ceil(k * spread) + 5 + (1 if fold else 0)
    guard = math.ceil(k * (1 - srx) * rx_lat) + 3 + (2 if fold else 0)
    nbx, nby, nbz = -(-nx // tx), -(-ny // ty), -(-(nz + z_off) // tz)
    rng = np.random.default_rng(seed)
    boxes = [(0, 0, 0), (nbx - 1, nby - 1, nbz - 1), (nbx // 2, nby // 2, nbz // 2)]
    boxes += [tuple(int(v) for v in rng.integers([nbx, nby, nbz])) for _ in range(nboxes)]
    lo_all, hi_all, hi_act = math.inf, -math.inf, -math.inf
    for bx, by, bz in boxes:
        i0 = [bx * tx, by * ty, max(bz * tz - z_off, 0)]
        i1 = [min(bx * tx + tx - 1, nx - 1), min(by * ty + ty - 1, ny - 1),
              min(bz * tz + tz - 1 - z_off, nz - 1)]
        if i1[2] < i0[2]:
            continue
        corners = np.array([org + ix * ax + iy * ay + iz * az
                            for ix in (i0[0], i1[0]) for iy in (i0[1], i1[1]) for iz in (i0[2], i1[2])])
        lo, hi = corners.min(0), corners.max(0)
        zlo, zmax = max(lo[2], 0.0), hi[2]
        if zmax <= 0:
            continue
        IX, IY, IZ = np.meshgrid(np.clip(np.arange(bx * tx, bx * tx + tx), 0, nx - 1),
                                 np.clip(np.arange(by * ty, by * ty + ty), 0, ny - 1),
                                 np.clip(np.arange(bz * tz - z_off, bz * tz + tz - z_off), 0, nz - 1),
                                 indexing="ij")
        P = org + IX[..., None] * ax + IY[..., None] * ay + IZ[..., None] * az
        px, py = P[..., 0].ravel(), P[..., 1].ravel()
        pz_raw = P[..., 2].ravel()
        pz = np.maximum(pz_raw, 1e-7)
        thr = np.where(pz_raw > 0, pz * pz * 0.25 / f2 if f2 > 0 else np.inf, -1.0)
        zb = k * zlo
        txlo = zlo
        if div_f > 0:
            ddx, ddy = max(0.0, lo[0], -hi[0]), max(0.0, lo[1], -hi[1])
            txlo = math.sqrt(ddx * ddx + ddy * ddy + (zlo + div_f) ** 2) - div_f
        for cj in rx_c:
            if f2 > 0:     # rows outside every point's receive aperture are not staged
                d = _dist(cj, lo[0], hi[0]) if mode == "forces" else _dist(cj, lo[1], hi[1])
                if zmax * zmax * 0.25 / f2 - d * d <= 0:
                    continue
            for i in range(n_tx):
                xi = tx_x[i]
                if mode == "hercules":
                    txp = (np.sqrt(px ** 2 + py ** 2 + (pz + div_f) ** 2) - div_f) if div_f > 0 else pz
                    rho2 = (px - xi) ** 2 + (py - cj) ** 2
                    rxp = np.sqrt(rho2 + pz ** 2)
                    rx_, ry_ = _dist(xi, lo[0], hi[0]), _dist(cj, lo[1], hi[1])
                    path = txlo + math.sqrt(rx_ * rx_ + ry_ * ry_ + zlo * zlo)
                elif mode == "forces":
                    txp = np.sqrt((px - xi) ** 2 + pz ** 2)
                    rho2 = (px - cj) ** 2
                    rxp = np.sqrt(rho2 + pz ** 2)
                    rt, rr = _dist(xi, lo[0], hi[0]), _dist(cj, lo[0], hi[0])
                    txb, rxb = math.sqrt(rt * rt + zlo * zlo), math.sqrt(rr * rr + zlo * zlo)
                    path = txb + rxb
                else:
                    rho2 = (py - cj) ** 2
                    rxp = np.sqrt(rho2 + pz ** 2)
                    ry_ = _dist(cj, lo[1], hi[1])
                    if mode == "tpw":
                        sn, cs = math.sin(ang[i]), math.cos(ang[i])
                        txp = px * sn + pz * cs
                        txb = (lo[0] if sn >= 0 else hi[0]) * sn + zlo * cs
                    else:
                        txp = zf + np.sign(pz - zf) * np.sqrt((px - xi) ** 2 + (pz - zf) ** 2)
                        if zf <= zlo:
                            r_ = _dist(xi, lo[0], hi[0])
                            txb = zf + math.sqrt(r_ * r_ + (zlo - zf) ** 2)
                        else:
                            r_ = _far(xi, lo[0], hi[0])
                            txb = zf - math.sqrt(r_ * r_ + (zf - zlo) ** 2)
                    rxb = math.sqrt(ry_ * ry_ + zlo * zlo)
                    path = txb + rxb
                if fold:
                    w0 = math.floor(k * txb - zb) + math.floor(k * rxb + zb - t0fs) - 2
                else:
                    w0 = math.floor(path * k - t0fs) - 2
                li = np.floor((txp + rxp) * k - t0fs) - w0
                lo_all, hi_all = min(lo_all, li.min()), max(hi_all, li.max())
                act = rho2 < thr
                if act.any():
                    hi_act = max(hi_act, li[act].max())
    return lo_all, hi_all, hi_act, lmax, lmax + guard


def _small(mode, z0=1.0 * MM, f_number=1.0, **kw):
    n_ch = 12 if mode == "forces" else 10
    dims = (37, 1, 53) if mode == "forces" else (13, 9, 29)
    if mode == "tpw":
        kw.setdefault("tx_angles", np.deg2rad(np.linspace(-10, 10, 8)))
    return describe(mode, (12, 10), (0.25 * MM, 0.3 * MM), 8, n_ch, 600, 25e6, 6e6, dims,
                    (-2 * MM, -1.5 * MM, z0), (2.2 * MM, 1.2 * MM, 9 * MM), t0=0.3e-6,
                    f_number=f_number, tx_elements=[0, 3, 4, 6, 7, 8, 10, 11],
                    channel_map=np.random.default_rng(2).permutation(n_ch), **kw)


def _tilted(desc):
    a = 0.25
    M = synth.configs.centered_xdc((12, 10), (0.25 * MM, 0.3 * MM))
    M[:3, :3] = [[np.cos(a), 0, np.sin(a)], [0, 1, 0], [-np.sin(a), 0, np.cos(a)]]
    M[:3, 3] += [0.2 * MM, -0.1 * MM, 0.5 * MM]
    return dict(desc, xdc=M)


CASES = [
    # full-size workload geometries with their default tiles
    ("w1 hercules", lambda: synth.configs.workload(1), (3, 3, 0), (2, 2, 3), 2),
    ("w5 diverging", lambda: synth.configs.workload(5), (3, 3, 0), (2, 2, 3), 2),
    ("w3 forces", lambda: synth.configs.workload(3), (5, 0, 1), (2, 1, 8), 1),
    ("w3 forces 16x4", lambda: synth.configs.workload(3), (4, 0, 2), (4, 1, 4), 1),
    ("w3 forces two points", lambda: synth.configs.workload(3), (5, 0, 1), (2, 1, 4), 2),
    ("w0 forces two points", lambda: synth.configs.workload(0), (5, 0, 1), (2, 1, 4), 2),
    ("w4 plane two points", lambda: synth.configs.frame_4("2d", np.arange(0, 128, 4)),
     (5, 0, 1), (2, 1, 4), 2),
    ("w6 tpw", lambda: synth.configs.workload(6), (3, 3, 0), (2, 2, 3), 1),
    ("w7 vls", lambda: synth.configs.workload(7), (2, 3, 1), (2, 2, 3), 1),
    # small grids: tiles, tilt, array plane, F#, focal lines
    ("hercules tilted", lambda: _tilted(_small("hercules", f_number=0.8)), (2, 2, 2), (1, 1, 1), 1),
    ("hercules plane", lambda: _small("hercules", z0=-0.15 * MM), (3, 3, 0), (2, 2, 2), 2),
    ("hercules F#0", lambda: _small("hercules", f_number=0.0), (0, 0, 6), (1, 1, 2), 2),
    ("forces plane", lambda: _small("forces", z0=-0.6 * MM), (2, 0, 4), (2, 1, 2), 1),
    ("forces F#2", lambda: _small("forces", f_number=2.0), (0, 0, 6), (1, 1, 1), 1),
    ("forces plane two points", lambda: _small("forces", z0=-0.6 * MM), (3, 0, 3), (2, 1, 2), 2),
    ("forces F#0 two points", lambda: _small("forces", f_number=0.0), (5, 0, 1), (1, 1, 4), 2),
    ("tpw plane", lambda: _small("tpw", z0=-0.6 * MM), (1, 1, 4), (1, 1, 2), 1),
    ("tpw F#0.5", lambda: _small("tpw", f_number=0.5), (3, 3, 0), (2, 2, 3), 1),
    ("vls diverging", lambda: _small("vls", focal_depth=-4 * MM), (2, 3, 1), (2, 2, 3), 1),
    ("vls focused", lambda: _small("vls", focal_depth=5.1 * MM), (2, 2, 2), (2, 2, 2), 1),
    ("vls focused plane", lambda: _small("vls", z0=-0.6 * MM, focal_depth=2.6 * MM), (1, 1, 4), (1, 1, 2), 1),
]


@pytest.mark.parametrize("name, make, tile, bw, zp", CASES, ids=[c[0] for c in CASES])
def test_unclamped_window_index_stays_in_bounds(name, make, tile, bw, zp):
    lo, hi, hi_act, lmax, limit = window_range(make(), tile, bw, zp,
                                               nboxes=3 if name.startswith("w") else 12)
    # (the separable kernels, whose windows sit after integer tables, need
    # an index of at least 0 after FP32 rounding: at least 1 here)
    sep = "hercules" not in name and "diverging" not in name
    assert lo >= (1 if sep else -1), (name, lo)
    assert hi < limit and hi_act <= lmax - 1, (name, lo, hi, hi_act, lmax, limit)


FOLD_CASES = [c for c in CASES if "hercules" not in c[0] and "diverging" not in c[0]]


@pytest.mark.parametrize("name, make, tile, bw, zp", FOLD_CASES, ids=[c[0] for c in FOLD_CASES])
def test_folded_window_start_stays_in_bounds(name, make, tile, bw, zp):
    lo, hi, hi_act, lmax, limit = window_range(make(), tile, bw, zp,
                                               nboxes=3 if name.startswith("w") else 12, fold=True)
    assert lo >= 1 and hi_act < lmax - 1 and hi < limit - 1, (name, lo, hi, hi_act, lmax, limit)
