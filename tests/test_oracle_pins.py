"""Pins of the FP64 CPU oracle against what the paper and mathematics fix.

Every oracle function is checked here against something other than itself:
closed forms (H H^T = N I, Pythagorean triples, Hann values), invariants
(decode of an encoded set, interpolator reproduction of low-order
polynomials, linearity, the adjoint identity, scale invariance of the
sharpness loss), finite differences and physically fixed outcomes (a point
scatterer's image peak).  A plausible slip in the oracle (a transposed H, a
dropped tangent term, a wrong sign in the delay, a swapped grid axis) fails at
least one of these.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import brute
from synth.configs import MM, describe

pytestmark = pytest.mark.filterwarnings("ignore")


# --------------------------------------------------------------------------
# Hadamard matrices and decoding (Sec. IV-A, Sec. VII-E)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n", [1, 2, 4, 8, 16, 32, 64, 128, 256])
def test_sylvester_is_hadamard(n):
    H = oracle.sylvester(n).astype(np.int64)
    assert set(np.unique(H)) <= {-1, 1}
    assert np.array_equal(H @ H.T, n * np.eye(n, dtype=np.int64))


def test_sylvester_doubling_rule():
    # Sylvester's construction: H_2n = [[H_n, H_n], [H_n, -H_n]], H_1 = [1].
    for n in (1, 2, 4, 8, 16, 32, 64, 128):
        H, H2 = oracle.sylvester(n), oracle.sylvester(2 * n)
        assert np.array_equal(H2, np.block([[H, H], [H, -H]]))
    with pytest.raises(ValueError):
        oracle.sylvester(12)


def _asymmetric_hadamard(n, rng):
    """A non-symmetric Hadamard matrix: rows permuted and negated."""
    H0 = oracle.sylvester(n).astype(np.int64)
    H = H0
    while np.array_equal(H, H.T):
        H = H0[rng.permutation(n)] * rng.choice([-1, 1], size=(n, 1))
        H = H * rng.choice([-1, 1], size=(1, n))
    assert np.array_equal(H @ H.T, n * np.eye(n, dtype=np.int64))
    return H.astype(np.int8)


@pytest.mark.parametrize("n", [2, 4, 16, 64])
def test_decode_of_encoded_set_is_n_times_elements(n):
    # Acquisition r_k = sum_i H[k][i] e_i (row k = polarity pattern of transmit
    # k); decoding must give back N e_i for every element (FORCES resolves to
    # an STA dataset).  The matrix is deliberately non-symmetric so that using
    # H instead of H^T fails.
    rng = np.random.default_rng(n)
    H = _asymmetric_hadamard(n, rng)
    e = rng.integers(-32768 // n, 32768 // n, size=(n, 3, 37))
    r = np.einsum("ki,ijt->kjt", H.astype(np.int64), e)
    assert np.abs(r).max() <= 32767
    d = oracle.decode(H, r.astype(np.int16))
    assert np.array_equal(d, n * e)


def test_decode_single_transmit_recovers_element_responses():
    # Each element responds with an impulse at its own sample; after decoding
    # of the encoded sequence every element's response is recovered alone.
    n, S = 8, 32
    H = oracle.sylvester(n)
    e = np.zeros((n, 1, S), dtype=np.int64)
    for i in range(n):
        e[i, 0, 2 * i + 1] = 1000 + i
    r = np.einsum("ki,ijt->kjt", H.astype(np.int64), e).astype(np.int16)
    d = oracle.decode(H, r)
    for i in range(n):
        nz = np.flatnonzero(d[i, 0])
        assert list(nz) == [2 * i + 1] and d[i, 0, 2 * i + 1] == n * (1000 + i)


def test_decode_matches_library_matmul_full_int16_range():
    rng = np.random.default_rng(7)
    n = 32
    H = _asymmetric_hadamard(n, rng)
    r = rng.integers(-32768, 32768, size=(n, 5, 41)).astype(np.int16)
    r[0, 0, :4] = [-32768, 32767, -32768, 32767]
    want = np.tensordot(H.astype(np.int64).T, r.astype(np.int64), axes=1)
    assert np.array_equal(oracle.decode(H, r), want)


def test_decode_noise_gain_is_sqrt_n():
    # Sec. IV-A: encoding over N transmits improves SNR by sqrt(N).  Decoded
    # signal scales by N while independent noise scales by sqrt(N).
    n, sigma = 64, 300.0
    rng = np.random.default_rng(3)
    H = oracle.sylvester(n)
    noise = np.rint(rng.normal(0, sigma, size=(n, 16, 512))).astype(np.int16)
    d = oracle.decode(H, noise).astype(np.float64)
    assert abs(d.std() / (math.sqrt(n) * noise.std()) - 1.0) < 0.03


def test_hi_lo_int8_split_identity_exhaustive():
    # x = 256 * (x >> 8) + ((x & 0xFF) - 128) + 128 for every int16, with both
    # halves representable as int8 (the exact split used by the int8 decode).
    x = np.arange(-32768, 32768, dtype=np.int64)
    hi = x >> 8
    lo = (x & 0xFF) - 128
    assert hi.min() >= -128 and hi.max() <= 127 and lo.min() >= -128 and lo.max() <= 127
    assert np.array_equal(256 * hi + lo + 128, x)


# --------------------------------------------------------------------------
# Window and interpolation (Eq. 3, Sec. IV-B)
# --------------------------------------------------------------------------

def test_hann_closed_form_values():
    assert oracle.hann(0.0) == 1.0
    assert oracle.hann(0.25) == pytest.approx(0.5, abs=1e-15)
    assert oracle.hann(-0.25) == pytest.approx(0.5, abs=1e-15)
    assert oracle.hann(1.0 / 3.0) == pytest.approx(0.25, abs=1e-15)
    assert oracle.hann(0.5) == 0.0 and oracle.hann(-0.5) == 0.0 and oracle.hann(0.7) == 0.0
    assert oracle.hann(0.5 - 1e-9) == pytest.approx(0.0, abs=1e-16)


@pytest.mark.parametrize("mode", ["nearest", "linear", "cubic"])
def test_interp_reproduces_constants(mode):
    tr = np.full(20, 3.25)
    for s in np.linspace(1.0, 17.9, 41):
        assert oracle.interp(tr, s, mode) == pytest.approx(3.25, abs=1e-13)


@pytest.mark.parametrize("mode", ["linear", "cubic"])
def test_interp_reproduces_ramps(mode):
    n = np.arange(40, dtype=np.float64)
    tr = 0.75 * n - 4.0
    for s in np.linspace(1.0, 37.99, 97):
        assert oracle.interp(tr, s, mode) == pytest.approx(0.75 * s - 4.0, abs=1e-12)
        assert oracle.interp(tr, s, mode, deriv=True) == pytest.approx(0.75, abs=1e-12)


def test_cubic_reproduces_quadratics_and_is_c1():
    # Catmull-Rom tangents are exact for quadratics, so the cubic Hermite
    # reproduces them; the derivative is continuous across sample points.
    n = np.arange(40, dtype=np.float64)
    tr = 0.5 * n * n - 3.0 * n + 1.0
    for s in np.linspace(1.0, 37.99, 97):
        assert oracle.interp(tr, s, "cubic") == pytest.approx(0.5 * s * s - 3 * s + 1, abs=1e-10)
        assert oracle.interp(tr, s, "cubic", deriv=True) == pytest.approx(s - 3.0, abs=1e-10)
    rng = np.random.default_rng(0)
    tr = rng.normal(size=30)
    for m in range(2, 27):
        a = oracle.interp(tr, m - 1e-9, "cubic", deriv=True)
        b = oracle.interp(tr, m + 1e-9, "cubic", deriv=True)
        assert a == pytest.approx(b, abs=1e-6)
        # and the curve passes through the samples
        assert oracle.interp(tr, float(m), "cubic") == tr[m]
    # the cubic is not exact for cubics (guards against a different kernel)
    tr3 = n ** 3
    assert abs(oracle.interp(tr3, 10.3, "cubic") - 10.3 ** 3) > 1e-3


def test_interp_zero_outside_and_nearest_rounding():
    tr = np.arange(1, 11, dtype=np.float64)       # 1..10 at n = 0..9
    assert oracle.interp(tr, -3.0, "cubic") == 0.0
    assert oracle.interp(tr, 12.0, "cubic") == 0.0
    # at t = 1/2 the Catmull-Rom cubic is the 4-point midpoint rule
    # (-p_-1 + 9 p_0 + 9 p_1 - p_2) / 16; left of the trace the taps are zero:
    # s = -0.5 reads (0, 0, 1, 2) -> 7/16, s = 3.5 reads (3, 4, 5, 6) -> 4.5
    assert oracle.interp(tr, -0.5, "cubic") == pytest.approx(7.0 / 16.0, abs=1e-15)
    assert oracle.interp(tr, 3.5, "cubic") == pytest.approx(4.5, abs=1e-15)
    assert oracle.interp(tr, 9.5, "cubic") == pytest.approx((-9 + 90) / 16.0, abs=1e-15)
    assert oracle.interp(tr, 2.49, "nearest") == 3.0
    assert oracle.interp(tr, 2.5, "nearest") == 4.0
    assert oracle.interp(tr, 9.6, "nearest") == 0.0


# --------------------------------------------------------------------------
# DAS geometry (Eqs. 1-3, Sec. VI-B data description)
# --------------------------------------------------------------------------

def _single(mode, tx_cols, ch, pitch, point, fs=40e6, c=1500.0, t0=0.0, f_number=0.0, S=4096,
            interp="cubic", xdc=None, dims=(1, 1, 1), gmax=None):
    d = describe(mode, (8, 8), pitch, len(tx_cols), len(ch), S, fs, 5e6, dims, point,
                 point if gmax is None else gmax, c=c, t0=t0, f_number=f_number, interp=interp,
                 tx_elements=tx_cols, channel_map=ch, xdc=np.eye(4) if xdc is None else xdc)
    return d


def _ramp(desc):
    S = desc["n_samples"]
    return np.broadcast_to(np.arange(S, dtype=np.float64),
                           (desc["n_tx"], desc["n_ch"], S)).copy()


def test_forces_345_triangle_delay():
    # Transmit and receive column at x = 0, point at (3, 4) mm: both paths are
    # 5 mm, so the ramp trace reads back s = (10 mm / c - t0) fs exactly.
    c, fs, t0 = 1500.0, 40e6, 1e-6
    d = _single("forces", [0], [0], (1 * MM, 1 * MM), (3 * MM, 0.0, 4 * MM), fs=fs, c=c, t0=t0)
    got = oracle.das(d, _ramp(d))[0, 0, 0]
    assert got == pytest.approx((10 * MM / c - t0) * fs, rel=1e-13)


def test_forces_separate_tx_rx_paths():
    # Transmit column 0 at x = 0, receive column 2 at x = 3 mm (pitch 1.5 mm),
    # point at (0, 4) mm: 4 mm out, 5 mm back.
    c, fs = 1540.0, 30e6
    d = _single("forces", [0], [2], (1.5 * MM, 1 * MM), (0.0, 0.0, 4 * MM), fs=fs, c=c)
    assert oracle.das(d, _ramp(d))[0, 0, 0] == pytest.approx(9 * MM / c * fs, rel=1e-13)
    # swapping transmit and receive columns leaves the delay unchanged
    d2 = _single("forces", [2], [0], (1.5 * MM, 1 * MM), (0.0, 0.0, 4 * MM), fs=fs, c=c)
    assert oracle.das(d2, _ramp(d2))[0, 0, 0] == pytest.approx(9 * MM / c * fs, rel=1e-13)


def test_hercules_plane_wave_and_point_receiver_delay():
    # Receiver (column 1, row 2) at (1, 2, 0) mm with 1 mm pitch; point at
    # (2, 4, 2) mm: transmit path z = 2 mm, receive path sqrt(1+4+4) = 3 mm.
    c, fs = 1540.0, 30e6
    d = _single("hercules", [1], [2], (1 * MM, 1 * MM), (2 * MM, 4 * MM, 2 * MM), fs=fs, c=c)
    assert oracle.das(d, _ramp(d))[0, 0, 0] == pytest.approx(5 * MM / c * fs, rel=1e-13)
    # the receive row pitch is the y pitch, not the x pitch
    d2 = _single("hercules", [1], [2], (1 * MM, 2 * MM), (2 * MM, 4 * MM, 2 * MM), fs=fs, c=c)
    # receiver now at (1, 4, 0): receive path sqrt(1 + 0 + 4) = sqrt(5) mm
    assert oracle.das(d2, _ramp(d2))[0, 0, 0] == pytest.approx(
        (2 + math.sqrt(5)) * MM / c * fs, rel=1e-13)


def test_transform_maps_global_points_to_array_frame():
    # Global frame rotated by 90 degrees about z and shifted: array (x, y) =
    # (-y_g + 5 mm, x_g).  The global point (0, -3 mm, 4 mm) lands at array
    # (8, 0, 4) mm; a receive column at x = 5 mm gives a 3-4-5 receive path,
    # and a transmit column at x = 8 mm a 4 mm transmit path.
    M = np.array([[0, -1, 0, 5 * MM], [1, 0, 0, 0], [0, 0, 1, 0], [0, 0, 0, 1]], dtype=float)
    c, fs = 1500.0, 40e6
    d = _single("forces", [8], [5], (1 * MM, 1 * MM), (0.0, -3 * MM, 4 * MM), fs=fs, c=c, xdc=M)
    assert oracle.das(d, _ramp(d))[0, 0, 0] == pytest.approx(9 * MM / c * fs, rel=1e-13)


def test_grid_linspace_and_layout():
    # Grid x in {-3, 0, 3} mm, y in {0, 1} mm (3D), z in {4, 8} mm; element at
    # the origin; HERCULES receive path is sqrt(x^2 + y^2 + z^2).  Output layout
    # is [iy][ix][iz].
    c, fs = 1500.0, 40e6
    d = _single("hercules", [0], [0], (1 * MM, 1 * MM), (-3 * MM, 0.0, 4 * MM), fs=fs, c=c,
                dims=(3, 2, 2), gmax=(3 * MM, 1 * MM, 8 * MM))
    out = oracle.das(d, _ramp(d))
    assert out.shape == (2, 3, 2)
    for iy, y in enumerate([0.0, 1.0]):
        for ix, x in enumerate([-3.0, 0.0, 3.0]):
            for iz, z in enumerate([4.0, 8.0]):
                path = z + math.sqrt(x * x + y * y + z * z)
                assert out[iy, ix, iz] == pytest.approx(path * MM / c * fs, rel=1e-12)


def test_receive_apodization_values():
    # F# = 1, receive at x = 0: point (1, 4) mm -> u = 0.25 -> a = 1/2;
    # (4/3, 4) -> u = 1/3 -> a = 1/4; (2, 4) -> u = 1/2 -> a = 0; z <= 0 -> 0.
    def one(point, mode="forces"):
        d = _single(mode, [0], [0], (1 * MM, 1 * MM), point, f_number=1.0)
        return oracle.das(d, np.ones((1, 1, d["n_samples"])))[0, 0, 0]
    assert one((1 * MM, 0, 4 * MM)) == pytest.approx(0.5, abs=1e-14)
    assert one((4 * MM / 3, 0, 4 * MM)) == pytest.approx(0.25, abs=1e-14)
    assert one((2 * MM, 0, 4 * MM)) == 0.0
    assert one((0.0, 0, 0.0)) == 0.0
    assert one((0.0, 0, -1 * MM)) == 0.0
    # HERCULES apodization is radial: (0.6, 0.8, 4) mm has rho = 1 mm -> 1/2
    assert one((0.6 * MM, 0.8 * MM, 4 * MM), "hercules") == pytest.approx(0.5, abs=1e-14)
    # FORCES apodization ignores y
    assert one((1 * MM, 7 * MM, 4 * MM)) == pytest.approx(0.5, abs=1e-14)


@pytest.mark.parametrize("mode", ["forces", "hercules"])
@pytest.mark.parametrize("interp", ["nearest", "linear", "cubic"])
def test_constant_data_sums_unit_weights(mode, interp):
    # With F# = 0 every weight is 1 and every interpolator reproduces
    # constants, so the image equals N_tx * N_ch wherever all taps are inside.
    d = describe(mode, (6, 5), (0.3 * MM, 0.3 * MM), 6, 5, 512, 20e6, 5e6, (4, 3 if mode ==
                 "hercules" else 1, 5), (-1 * MM, -0.5 * MM, 3 * MM), (1 * MM, 0.5 * MM, 9 * MM),
                 f_number=0.0, interp=interp)
    out = oracle.das(d, np.ones((6, 5, 512)))
    assert np.allclose(out, 30.0, rtol=0, atol=1e-12)


def test_das_is_linear_in_data():
    rng = np.random.default_rng(5)
    d = describe("hercules", (4, 4), (0.3 * MM, 0.3 * MM), 4, 4, 256, 20e6, 5e6, (3, 2, 4),
                 (-1 * MM, -1 * MM, 2 * MM), (1 * MM, 1 * MM, 4 * MM))
    e1, e2 = rng.normal(size=(2, 4, 4, 256))
    a = oracle.das(d, 2.0 * e1 - 0.5 * e2)
    b = 2.0 * oracle.das(d, e1) - 0.5 * oracle.das(d, e2)
    assert np.allclose(a, b, rtol=1e-12, atol=1e-12)


def _argmax_cell(img):
    return np.unravel_index(np.argmax(img), img.shape)


def test_point_scatterer_peak_forces():
    # A single scatterer imaged with FORCES: the image maximum lies within one
    # grid cell of the true position (physics fixes where the peak must be).
    d = describe("forces", (32, 32), (0.2 * MM, 0.2 * MM), 32, 32, 1024, 20e6, 5e6,
                 (65, 1, 81), (-3.2 * MM, 0, 10 * MM), (3.2 * MM, 0, 18 * MM), t0=4e-6)
    pt = np.array([[0.7 * MM, 0.0, 13.3 * MM]])
    rf = synth.acquire(d, pt, np.ones(1), np.random.default_rng(1), noise=0.0)
    e = oracle.decode(synth.hadamard_sylvester(32), rf)
    img = oracle.das(d, e)
    iy, ix, iz = _argmax_cell(img)
    xs = np.linspace(-3.2, 3.2, 65)[ix]
    zs = np.linspace(10, 18, 81)[iz]
    assert abs(xs - 0.7) <= 0.1 + 1e-9 and abs(zs - 13.3) <= 0.1 + 1e-9


def test_point_scatterer_peak_hercules():
    d = describe("hercules", (16, 16), (0.2 * MM, 0.2 * MM), 16, 16, 1024, 20e6, 5e6,
                 (17, 17, 21), (-1.6 * MM, -1.6 * MM, 4 * MM), (1.6 * MM, 1.6 * MM, 6 * MM))
    pt = np.array([[0.4 * MM, -0.6 * MM, 5.0 * MM]])
    rf = synth.acquire(d, pt, np.ones(1), np.random.default_rng(2), noise=0.0)
    e = oracle.decode(synth.hadamard_sylvester(16), rf)
    img = oracle.das(d, e)
    iy, ix, iz = _argmax_cell(img)
    ax = np.linspace(-1.6, 1.6, 17)
    assert abs(ax[ix] - 0.4) <= 0.2 + 1e-9 and abs(ax[iy] + 0.6) <= 0.2 + 1e-9
    assert abs(np.linspace(4, 6, 21)[iz] - 5.0) <= 0.1 + 1e-9


@pytest.mark.parametrize("mode", ["forces", "hercules"])
@pytest.mark.parametrize("interp", ["nearest", "linear", "cubic"])
def test_c_oracle_matches_python_brute_force(mode, interp):
    rng = np.random.default_rng(11)
    d = describe(mode, (5, 4), (0.3 * MM, 0.25 * MM), 3, 4, 96, 20e6, 5e6,
                 (4, 2 if mode == "hercules" else 1, 3), (-0.6 * MM, -0.4 * MM, 1.5 * MM),
                 (0.6 * MM, 0.4 * MM, 2.5 * MM), t0=0.2e-6, f_number=0.7, interp=interp,
                 tx_elements=[4, 0, 2], channel_map=[3, 1, 0, 2])
    e = rng.normal(size=(3, 4, 96))
    assert np.allclose(oracle.das(d, e), brute.das(d, e), rtol=1e-12, atol=1e-12)


def test_das_points_matches_full_image():
    rng = np.random.default_rng(4)
    d = describe("hercules", (6, 6), (0.3 * MM, 0.3 * MM), 6, 6, 256, 20e6, 5e6, (4, 3, 5),
                 (-1 * MM, -1 * MM, 2 * MM), (1 * MM, 1 * MM, 4 * MM))
    e = rng.normal(size=(6, 6, 256))
    full = oracle.das(d, e).reshape(-1)
    vox = np.array([0, 7, 33, 59, 59])
    assert np.array_equal(oracle.das_points(d, e, vox), full[vox])


# --------------------------------------------------------------------------
# Adjoint and sound-speed derivative
# --------------------------------------------------------------------------

@pytest.mark.parametrize("mode", ["forces", "hercules"])
@pytest.mark.parametrize("interp", ["nearest", "linear", "cubic"])
def test_adjoint_dot_product_identity(mode, interp):
    rng = np.random.default_rng(9)
    d = describe(mode, (6, 6), (0.3 * MM, 0.3 * MM), 5, 6, 200, 20e6, 5e6,
                 (5, 3 if mode == "hercules" else 1, 7), (-1 * MM, -0.5 * MM, 1 * MM),
                 (1 * MM, 0.5 * MM, 4 * MM), interp=interp, f_number=0.8,
                 tx_elements=[0, 1, 3, 4, 5])
    e = rng.normal(size=(5, 6, 200))
    G = rng.normal(size=oracle.Geometry(d).shape)
    lhs = float(np.sum(oracle.das(d, e) * G))
    rhs = float(np.sum(e * oracle.das_adjoint_e(d, G)))
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))


@pytest.mark.parametrize("mode", ["forces", "hercules"])
def test_sound_speed_derivative_matches_central_differences(mode):
    rng = np.random.default_rng(12)
    d = describe(mode, (6, 6), (0.3 * MM, 0.3 * MM), 4, 5, 300, 20e6, 5e6,
                 (4, 2 if mode == "hercules" else 1, 6), (-1 * MM, -0.5 * MM, 2 * MM),
                 (1 * MM, 0.5 * MM, 5 * MM), f_number=0.8)
    t = np.arange(300) / 20e6
    e = np.cos(2 * np.pi * 5e6 * t)[None, None, :] * rng.normal(size=(4, 5, 1))
    c0 = 1540.0
    an = oracle.das_dc(d, e, c=c0)
    errs = []
    for h in (0.1, 1e-2, 1e-3):
        fd = (oracle.das(d, e, c=c0 + h) - oracle.das(d, e, c=c0 - h)) / (2 * h)
        errs.append(np.abs(an - fd).max() / np.abs(an).max())
    # central differences converge to the analytic derivative at O(h^2)
    assert errs[0] < 2e-3 and errs[2] < 1e-7
    assert errs[1] < errs[0] / 50 and errs[2] < errs[1] / 50
    dn = dict(d, interp="nearest")
    assert np.all(oracle.das_dc(dn, e, c=c0) == 0.0)


# --------------------------------------------------------------------------
# Sharpness loss
# --------------------------------------------------------------------------

def test_sharpness_closed_forms_and_gradient():
    one_hot = np.zeros(100); one_hot[17] = -3.0
    assert oracle.sharpness(one_hot) == pytest.approx(-1.0, abs=1e-15)
    assert oracle.sharpness(np.full(64, 2.5)) == pytest.approx(-1.0 / 64, abs=1e-15)
    two = np.zeros(10); two[[1, 7]] = [4.0, -4.0]
    assert oracle.sharpness(two) == pytest.approx(-0.5, abs=1e-15)
    assert oracle.sharpness(np.zeros(5)) == 0.0
    rng = np.random.default_rng(1)
    x = rng.normal(size=50)
    L, g = oracle.sharpness(x, grad=True)
    assert oracle.sharpness(7.0 * x) == pytest.approx(L, rel=1e-13)   # scale invariant
    assert abs(np.dot(g, x)) < 1e-12                                   # Euler: degree 0
    h = 1e-6
    for q in (0, 13, 49):
        xp, xm = x.copy(), x.copy()
        xp[q] += h; xm[q] -= h
        fd = (oracle.sharpness(xp) - oracle.sharpness(xm)) / (2 * h)
        assert g[q] == pytest.approx(fd, rel=1e-6, abs=1e-10)
