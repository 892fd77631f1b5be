"""Tiny-input brute force of the DAS definition in pure Python (test cross-check).

A second, independent transcription of Eq. 1 with Eqs. 2-3 and the readings
of the C oracle (geometry, time of flight, zero-padded cubic Hermite with
Catmull-Rom tangents written as a 4x4 basis-matrix product).  It is a
cross-check of the C code's indexing, not a pin: pins live in
tests/test_oracle_pins.py.  Only for grids of a few points and elements.
"""
import math

import numpy as np

# Catmull-Rom basis: v(t) = [1 t t^2 t^3] . B . [p_-1 p_0 p_1 p_2]^T
_B = 0.5 * np.array([[0, 2, 0, 0],
                     [-1, 0, 1, 0],
                     [2, -5, 4, -1],
                     [-1, 3, -3, 1]], dtype=np.float64)


def _sample(tr, n):
    return float(tr[n]) if 0 <= n < len(tr) else 0.0


def _read(tr, s, interp):
    if interp == "nearest":
        return _sample(tr, int(math.floor(s + 0.5)))
    n = int(math.floor(s))
    t = s - n
    if interp == "linear":
        return (1 - t) * _sample(tr, n) + t * _sample(tr, n + 1)
    p = np.array([_sample(tr, n + k) for k in (-1, 0, 1, 2)])
    return float(np.array([1.0, t, t * t, t ** 3]) @ _B @ p)


def das(desc, e):
    Nx, Ny, Nz = desc["dims"]
    M = np.asarray(desc["xdc"], dtype=np.float64).reshape(4, 4)
    px, py = desc["pitch"]
    out = np.zeros((Ny, Nx, Nz))
    axes = [np.linspace(desc["gmin"][a], desc["gmax"][a], desc["dims"][a]) if desc["dims"][a] > 1
            else np.array([desc["gmin"][a]]) for a in range(3)]
    for iy in range(Ny):
        for ix in range(Nx):
            for iz in range(Nz):
                g = np.array([axes[0][ix], axes[1][iy], axes[2][iz], 1.0])
                x, y, z, _ = M @ g
                acc = 0.0
                for i, col in enumerate(desc["tx_elements"]):
                    for j, ch in enumerate(desc["channel_map"]):
                        if desc["mode"] == "forces":
                            xt, xr = col * px, ch * px
                            tof = (math.hypot(x - xt, z) + math.hypot(x - xr, z)) / desc["c"]
                            rho = abs(x - xr)
                        else:
                            rho = math.hypot(x - col * px, y - ch * py)
                            tof = (z + math.hypot(rho, z)) / desc["c"]
                        if z <= 0:
                            continue
                        if desc["f_number"] == 0:
                            a = 1.0
                        else:
                            u = desc["f_number"] * rho / z
                            a = math.cos(math.pi * u) ** 2 if abs(u) < 0.5 else 0.0
                        if a == 0.0:
                            continue
                        s = (tof - desc["t0"]) * desc["fs"]
                        acc += a * _read(e[i, j], s, desc.get("interp", "cubic"))
                out[iy, ix, iz] = acc
    return out
