"""Pins of the oracle's demodulation (Eq. 4) and IQ beamforming.

Each test checks the oracle against something other than itself: closed
forms of the mix + filter for a tone and an impulse, an independent library
filter (scipy.signal.lfilter), exact rounding cases, the reduction of IQ
beamforming to the (pinned) RF beamformer when the demodulation frequency is
zero, a single-trace geometry whose output phase is known in closed form, and
the physical identity 2 Re(IQ image) = RF image for a narrowband echo.
"""
import math

import numpy as np
import pytest
import scipy.signal

import oracle
from synth.configs import MM, describe
from tests.helpers import rel_l2


# ---------------------------------------------------------------------------
# Demodulation
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("phi_q, expect", [(0, 1000.0), (1, 1000.0j), (2, -1000.0), (3, -1000.0j)])
def test_demod_quadrature_tone_closed_form(phi_q, expect):
    # fs = 4 fd (quadrature sampling, Sec. IV-B): x[n] = A cos(pi n / 2 + phi)
    # with phi = phi_q * pi / 2 is an exact integer sequence.  Mixing gives
    # A/2 e^{j phi} + A/2 e^{-j (pi n + phi)}; the two-tap average (zero at the
    # Nyquist frequency, unit DC gain) removes the second term exactly, so every
    # output after the first equals A/2 e^{j phi}.  A sign error in the mix
    # would conjugate the result.
    A = 2000
    n = np.arange(64)
    x = np.rint(A * np.cos(np.pi * n / 2 + phi_q * np.pi / 2)).astype(np.int16)
    y = oracle.demod(x, [0.5, 0.5], fd=5e6, fs=20e6, D=1)
    np.testing.assert_allclose(y[1:], expect, atol=1e-9)


@pytest.mark.parametrize("D", [1, 3])
def test_demod_impulse_closed_form(D):
    # x = A delta[n - n0]: the mixed signal is A e^{-j 2 pi r n0} at n0 only, so
    # y[n] = A h[n - n0] e^{-j 2 pi r n0} for n0 <= n < n0 + N_f, else 0, and
    # decimation keeps n = q D.  Catches a reversed or shifted filter index and
    # a mix evaluated at the output index instead of the input index.
    rng = np.random.default_rng(7)
    h = rng.normal(size=9) + 1j * rng.normal(size=9)
    S, n0, A, r = 61, 17, 1234, 0.1234
    x = np.zeros(S, dtype=np.int16)
    x[n0] = A
    y = oracle.demod(x, h, fd=r, fs=1.0, D=D)
    n = np.arange(0, S, D)
    assert y.shape == ((S + D - 1) // D,)
    expect = np.zeros(n.shape, dtype=np.complex128)
    inside = (n >= n0) & (n < n0 + h.size)
    expect[inside] = A * h[n[inside] - n0] * np.exp(-2j * np.pi * r * n0)
    np.testing.assert_allclose(y, expect, atol=1e-9)


@pytest.mark.parametrize("D, n_taps", [(1, 1), (2, 36), (4, 166), (3, 7)])
def test_demod_matches_library_filter(D, n_taps):
    # independent implementation: mix with numpy, filter with scipy's lfilter
    rng = np.random.default_rng(100 + D)
    x = rng.integers(-30000, 30000, size=(3, 301)).astype(np.int16)
    h = rng.normal(size=n_taps) + 1j * rng.normal(size=n_taps)
    fd, fs = 3.7e6, 20e6
    n = np.arange(x.shape[1])
    mixed = x * np.exp(-2j * np.pi * fd / fs * n)
    ref = scipy.signal.lfilter(h, [1.0], mixed, axis=-1)[:, ::D]
    y = oracle.demod(x, h, fd=fd, fs=fs, D=D)
    np.testing.assert_allclose(y, ref, rtol=1e-11, atol=1e-7 * np.abs(ref).max())


def test_demod_real_taps_equal_complex_taps_with_zero_imag():
    rng = np.random.default_rng(3)
    x = rng.integers(-3000, 3000, size=(2, 97)).astype(np.int16)
    h = rng.normal(size=11)
    a = oracle.demod(x, h, fd=1.1e6, fs=7e6, D=2)
    b = oracle.demod(x, h + 0j, fd=1.1e6, fs=7e6, D=2)
    np.testing.assert_array_equal(a, b)


def test_quantise_rounds_half_to_even_and_saturates():
    y = np.array([2.5 + 3.5j, -2.5 - 3.5j, 0.5 - 0.5j, 1.4999999 + 1.5000001j,
                  40000.0 - 40000.0j, 32767.5 - 32768.5j, -32768.4 + 32766.6j])
    q = oracle.quantise_iq(y)
    expect = np.array([[2, 4], [-2, -4], [0, 0], [1, 2], [32767, -32768], [32767, -32768],
                       [-32768, 32767]], dtype=np.int16)
    np.testing.assert_array_equal(q, expect)


def test_complex_int16_decodes_plane_by_plane():
    # decoding is a product across transmits, so interleaved (re, im) int16
    # samples decode as two independent planes (exact integers)
    rng = np.random.default_rng(11)
    H = oracle.sylvester(8)
    iq = rng.integers(-32768, 32767, size=(8, 3, 20, 2)).astype(np.int16)
    e = oracle.decode(H, iq.reshape(8, 3, 40)).reshape(8, 3, 20, 2)
    np.testing.assert_array_equal(e[..., 0], oracle.decode(H, np.ascontiguousarray(iq[..., 0])))
    np.testing.assert_array_equal(e[..., 1], oracle.decode(H, np.ascontiguousarray(iq[..., 1])))


# ---------------------------------------------------------------------------
# IQ beamforming
# ---------------------------------------------------------------------------
def _small(mode, fd, fs, S, **kw):
    if mode == "forces":
        d = describe("forces", (8, 8), (0.3 * MM, 0.3 * MM), 8, 8, S, fs, fd, (7, 1, 9),
                     (-1 * MM, 0, 3 * MM), (1 * MM, 0, 9 * MM), **kw)
    else:
        d = describe("hercules", (8, 8), (0.3 * MM, 0.3 * MM), 8, 8, S, fs, fd, (4, 3, 6),
                     (-1 * MM, -0.5 * MM, 3 * MM), (1 * MM, 0.5 * MM, 9 * MM), **kw)
    return d


@pytest.mark.parametrize("mode", ["forces", "hercules"])
def test_das_iq_with_zero_demodulation_frequency_is_rf_das_per_plane(mode):
    d = _small(mode, 0.0, 10e6, 160, t0=1e-6)
    rng = np.random.default_rng(5)
    er = rng.normal(size=(8, 8, 160))
    ei = rng.normal(size=(8, 8, 160))
    img = oracle.das_iq(d, er + 1j * ei)
    np.testing.assert_allclose(img.real, oracle.das(d, er), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(img.imag, oracle.das(d, ei), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("mode", ["forces", "hercules"])
@pytest.mark.parametrize("f_number", [0.0, 1.5])
def test_das_iq_single_trace_phase_closed_form(mode, f_number):
    # One element under the points: tof = 2 z / c, weight W(0) = 1, and a
    # constant trace reads 1 exactly inside the record (the cubic reproduces
    # constants), so the output is exp(j 2 pi fd (2 z / c - t0)).
    fd, fs, c, t0, S = 2.7e6, 10e6, 1540.0, 1.3e-6, 512
    d = describe(mode, (1, 1), (0.3 * MM, 0.3 * MM), 1, 1, S, fs, fd, (1, 1, 7),
                 (0, 0, 4 * MM), (0, 0, 16 * MM), c=c, t0=t0, f_number=f_number)
    e = np.ones((1, 1, S), dtype=np.complex128)
    img = oracle.das_iq(d, e).reshape(-1)
    z = np.linspace(4 * MM, 16 * MM, 7)
    assert np.all(((2 * z / c - t0) * fs > 2) & ((2 * z / c - t0) * fs < S - 3))
    np.testing.assert_allclose(img, np.exp(2j * np.pi * fd * (2 * z / c - t0)), atol=1e-12)


def test_das_iq_narrowband_echo_matches_rf_beamforming():
    # A point echo s(t) = g(t - tau) cos(2 pi fd (t - tau)) demodulated with the
    # mix of Eq. 4 (phase counted from sample 0 at t0) is, before decimation and
    # up to the low-pass, b(t) = g(t - tau) exp(-j 2 pi fd (tau - t0)) / 2.  A
    # rotated IQ term is then half the analytic RF term, so 2 Re(IQ image) is
    # the RF image up to the interpolators' errors (both well oversampled here).
    # A wrong rotation sign or reference time breaks the identity.
    fd, c, t0 = 5e6, 1540.0, 11.3e-6         # fd t0 = 56.5 cycles
    fs_rf, fs_iq = 32 * fd, 8 * fd
    sig = 2.0 / fd
    d_rf = describe("hercules", (8, 8), (0.3 * MM, 0.3 * MM), 8, 8, 1200, fs_rf, fd, (5, 3, 7),
                    (-0.6 * MM, -0.3 * MM, 9.4 * MM), (0.6 * MM, 0.3 * MM, 10.6 * MM), c=c,
                    t0=t0, f_number=0.0)
    d_iq = dict(d_rf, fs=fs_iq, n_samples=300)
    sc = np.array([0.1 * MM, -0.05 * MM, 10 * MM])
    xe = (np.arange(8) - 3.5) * 0.3 * MM       # element columns / rows, array centred
    tau = np.empty((8, 8))
    for i in range(8):
        for j in range(8):
            tau[i, j] = (sc[2] + math.dist(sc, (xe[i], xe[j], 0.0))) / c
    t_rf = t0 + np.arange(1200) / fs_rf
    t_iq = t0 + np.arange(300) / fs_iq
    g = lambda t: np.exp(-t * t / (2 * sig * sig))
    rf = g(t_rf - tau[..., None]) * np.cos(2 * np.pi * fd * (t_rf - tau[..., None]))
    iq = 0.5 * g(t_iq - tau[..., None]) * np.exp(-2j * np.pi * fd * (tau[..., None] - t0))
    img_rf = oracle.das(d_rf, rf)
    img_iq = oracle.das_iq(d_iq, iq)
    assert np.abs(img_rf).max() > 10.0          # the grid sits on the echo
    assert rel_l2(2 * img_iq.real, img_rf) < 2e-4
    # the conjugate rotation (a sign error) is far off
    img_bad = oracle.das_iq(d_iq, np.conj(iq))
    assert rel_l2(2 * img_bad.real, img_rf) > 0.3
    # so is a rotation referenced to tof instead of tof - t0 (fd t0 = 56.5
    # cycles flips the sign): same as rotating the data by exp(j 2 pi fd t0)
    img_t0 = oracle.das_iq(d_iq, iq * np.exp(2j * np.pi * fd * t0))
    assert rel_l2(2 * img_t0.real, img_rf) > 1.9


def test_das_iq_points_match_full_image():
    d = _small("hercules", 3e6, 12e6, 200, t0=0.5e-6)
    rng = np.random.default_rng(9)
    e = rng.normal(size=(8, 8, 200)) + 1j * rng.normal(size=(8, 8, 200))
    full = oracle.das_iq(d, e).reshape(-1)
    vox = np.array([0, 5, 17, 71], dtype=np.int64)
    np.testing.assert_array_equal(oracle.das_iq_points(d, e, vox), full[vox])
