"""Pins of the oracle's additional time-of-flight models: tilted plane waves
(TPW) and virtual line sources (VLS) on row-column volumes, and the diverging
HERCULES transmit.

Delays are read back through a ramp trace (e[n] = n, which every interpolator
reproduces exactly inside the record), so one (transmit, receiver) pair with
F# = 0 returns s = (tof - t0) fs; 3-4-5 triangles make every path a closed
form.  Limits (zero angle, distant virtual sources) reduce to the pinned
plane-wave model, and an echo simulated by the independent acquisition code
peaks at its scatterer.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from synth.configs import MM, describe

C, FS = 1500.0, 40e6


def _one(mode, tx_col, row, point, pitch=(1 * MM, 1 * MM), **kw):
    d = describe(mode, (8, 8), pitch, 1, 1, 4096, FS, 5e6, (1, 1, 1), point, point, c=C,
                 f_number=kw.pop("f_number", 0.0), tx_elements=[tx_col], channel_map=[row],
                 xdc=np.eye(4), **kw)
    return d


def _ramp(d):
    S = d["n_samples"]
    return np.broadcast_to(np.arange(S, dtype=np.float64), (d["n_tx"], d["n_ch"], S)).copy()


def _delay(d):
    return oracle.das(d, _ramp(d))[0, 0, 0]


def _s(path_mm):
    return path_mm * MM / C * FS


# array centre of the 8 x 8 grid at 1 mm pitch: (3.5, 3.5) mm
XC = YC = 3.5


def test_tpw_345_delays():
    th = math.atan2(0.6, 0.8)                 # sin 0.6, cos 0.8
    # row 2 at y = 2 mm; point 3 mm right of the centre, 3 mm off the row, z = 4
    p = ((XC + 3) * MM, 5 * MM, 4 * MM)
    d = _one("tpw", 0, 2, p, tx_angles=[th])
    assert _delay(d) == pytest.approx(_s(3 * 0.6 + 4 * 0.8 + 5), rel=1e-13)
    d = _one("tpw", 0, 2, p, tx_angles=[-th])              # tilted the other way
    assert _delay(d) == pytest.approx(_s(-3 * 0.6 + 4 * 0.8 + 5), rel=1e-13)
    d = _one("tpw", 5, 2, p, tx_angles=[0.0])              # zero angle: plane wave z
    assert _delay(d) == pytest.approx(_s(4 + 5), rel=1e-13)
    # the transmit column index does not enter a TPW delay
    assert _delay(_one("tpw", 7, 2, p, tx_angles=[th])) == pytest.approx(
        _s(3 * 0.6 + 4 * 0.8 + 5), rel=1e-13)
    # receivers are rows: a row pitch of 2 mm puts row 2 at y = 4 mm
    d = _one("tpw", 0, 2, p, pitch=(1 * MM, 2 * MM), tx_angles=[0.0])
    assert _delay(d) == pytest.approx(_s(4 + math.sqrt(1 + 16)), rel=1e-13)


def test_vls_345_delays():
    # column 2 at x = 2 mm; receiver row 1 at y = 1 mm, points on y = 1 mm
    # diverging virtual line at z_f = -2 mm: point (5, 1, 2): |dz| 4, dx 3 -> 5
    d = _one("vls", 2, 1, (5 * MM, 1 * MM, 2 * MM), focal_depth=-2 * MM)
    assert _delay(d) == pytest.approx(_s(-2 + 5 + 2), rel=1e-13)
    # focused at z_f = 8 mm: before the focus (z = 4) the wave converges
    d = _one("vls", 2, 1, (5 * MM, 1 * MM, 4 * MM), focal_depth=8 * MM)
    assert _delay(d) == pytest.approx(_s(8 - 5 + 4), rel=1e-13)
    # beyond the focus (z = 12) it diverges again
    d = _one("vls", 2, 1, (5 * MM, 1 * MM, 12 * MM), focal_depth=8 * MM)
    assert _delay(d) == pytest.approx(_s(8 + 5 + 12), rel=1e-13)
    # zero transmit delay at the element itself (just below it)
    d = _one("vls", 2, 1, (2 * MM, 1 * MM, 1e-9), focal_depth=8 * MM)
    assert _delay(d) == pytest.approx(_s(0.0), abs=1e-3)
    # z_f = 0: the cylindrical wave of the column itself
    d = _one("vls", 2, 1, (5 * MM, 1 * MM, 4 * MM), focal_depth=0.0)
    assert _delay(d) == pytest.approx(_s(5 + 4), rel=1e-13)


def test_diverging_hercules_delay_and_plane_wave_limit():
    # virtual source at (3.5, 3.5, -3) mm; point (6.5, 3.5, 1): 3-4-5 -> 5 - 3 = 2 mm
    p = (6.5 * MM, 3.5 * MM, 1 * MM)
    d = _one("hercules", 6, 3, p, focal_depth=-3 * MM)
    rx = math.sqrt(0.5 ** 2 + 0.5 ** 2 + 1.0)
    assert _delay(d) == pytest.approx(_s(2 + rx), rel=1e-13)
    # a very distant source gives the plane wave (z) to first order
    far = _one("hercules", 6, 3, p, focal_depth=-1e5)
    plane = _one("hercules", 6, 3, p)
    assert _delay(far) == pytest.approx(_delay(plane), rel=1e-6)
    assert _delay(plane) == pytest.approx(_s(1 + rx), rel=1e-13)


def test_row_receive_apodization():
    # F# 1, z = 4 mm: |y - y_j| = 1 mm gives u = 1/4, W = 1/2; the x offset
    # from the transmit column does not enter the receive apodization
    for mode, kw in (("tpw", dict(tx_angles=[0.0])), ("vls", dict(focal_depth=-2 * MM))):
        d = _one(mode, 0, 1, (6 * MM, 2 * MM, 4 * MM), f_number=1.0, **kw)
        d0 = _one(mode, 0, 1, (6 * MM, 2 * MM, 4 * MM), f_number=0.0, **kw)
        assert _delay(d) == pytest.approx(0.5 * _delay(d0), rel=1e-13)


def test_unencoded_decode_is_the_identity():
    rng = np.random.default_rng(0)
    r = rng.integers(-32768, 32767, size=(5, 3, 17)).astype(np.int16)
    np.testing.assert_array_equal(oracle.decode(np.eye(5, dtype=np.int8), r), r)


@pytest.mark.parametrize("mode, kw", [
    ("tpw", dict(tx_angles=np.deg2rad(np.linspace(-12, 12, 16)))),
    ("vls", dict(focal_depth=-4 * MM)),
    ("vls", dict(focal_depth=6 * MM)),
    ("hercules", dict(focal_depth=-10 * MM)),
])
def test_simulated_echo_peaks_at_the_scatterer(mode, kw):
    # the acquisition simulator (its own ToF code) and the oracle agree: the
    # image of one scatterer peaks within one grid cell of it
    n = 16
    d = describe(mode, (n, n), (0.3 * MM, 0.3 * MM), n, n, 1500, 40e6, 5e6, (21, 21, 41),
                 (-1.5 * MM, -1.5 * MM, 6 * MM), (1.5 * MM, 1.5 * MM, 12 * MM), f_number=0.0,
                 **kw)
    pt = np.array([[0.45 * MM, -0.3 * MM, 9.0 * MM]])
    e = synth.element_responses(d, pt, np.ones(1))
    img = np.abs(oracle.das(d, e))
    iy, ix, iz = np.unravel_index(np.argmax(img), img.shape)
    x = -1.5 * MM + ix * 0.15 * MM
    y = -1.5 * MM + iy * 0.15 * MM
    z = 6 * MM + iz * 0.15 * MM
    assert abs(x - pt[0, 0]) <= 0.15 * MM and abs(y - pt[0, 1]) <= 0.15 * MM
    assert abs(z - pt[0, 2]) <= 0.15 * MM
