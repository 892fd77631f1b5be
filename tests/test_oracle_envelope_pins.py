"""Pins of the oracle's envelope (analytic signal along depth) and display
compression: an independent library (scipy.signal.hilbert), closed forms of
the analytic signal (tones, constants, the Nyquist sequence, N = 1 and 2),
the bound env >= |x|, and exact compression values."""
import numpy as np
import pytest
import scipy.signal

import oracle


@pytest.mark.parametrize("N", [1, 2, 3, 16, 37, 64, 255, 256])
def test_envelope_matches_scipy_hilbert(N):
    x = np.random.default_rng(N).normal(size=(4, N))
    ref = np.abs(scipy.signal.hilbert(x, axis=-1))
    np.testing.assert_allclose(oracle.envelope(x), ref, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("N, m", [(64, 1), (64, 31), (37, 5), (256, 100)])
def test_envelope_of_a_tone_is_its_amplitude(N, m):
    # x = A cos(2 pi m n / N + phi), 0 < m < N/2: the analytic signal is
    # A exp(j (2 pi m n / N + phi)), so the envelope is A at every sample
    n = np.arange(N)
    for A, phi in ((1.0, 0.0), (3.5, 0.7), (0.25, -2.0)):
        env = oracle.envelope(A * np.cos(2 * np.pi * m * n / N + phi))
        np.testing.assert_allclose(env, A, rtol=1e-12)


def test_envelope_special_sequences():
    # constant: only the DC bin, weight 1 -> |c|
    np.testing.assert_allclose(oracle.envelope(np.full(10, -2.5)), 2.5, rtol=1e-12)
    # Nyquist sequence (even N): only the N/2 bin, weight 1 -> 1
    np.testing.assert_allclose(oracle.envelope((-1.0) ** np.arange(12)), 1.0, rtol=1e-12)
    # N = 1 and N = 2: the analytic signal is the signal itself
    x = np.array([[-3.0], [4.0]])
    np.testing.assert_allclose(oracle.envelope(x), np.abs(x), rtol=1e-15)
    x = np.array([[1.0, -7.0], [0.5, 2.0]])
    np.testing.assert_allclose(oracle.envelope(x), np.abs(x), rtol=1e-12)


def test_envelope_bounds_the_signal():
    # Re(analytic signal) = x, so |x_a| >= |x| everywhere
    x = np.random.default_rng(1).normal(size=(5, 50))
    assert np.all(oracle.envelope(x) >= np.abs(x) - 1e-12)


def test_log_compression_values():
    env = np.array([8.0, 0.8, 0.08, 8e-3, 8e-5, 0.0, 16.0])
    y = oracle.compress(env, "log", ref=8.0, param=60.0)
    np.testing.assert_allclose(y, [0.0, -20.0, -40.0, -60.0, -60.0, -60.0,
                                   20 * np.log10(2.0)], atol=1e-12)
    # ref <= 0: the maximum (16) is the reference
    y = oracle.compress(env, "log", ref=0.0, param=30.0)
    np.testing.assert_allclose(y[[6, 0, 1]], [0.0, -20 * np.log10(2.0), -20 * np.log10(20.0)],
                               atol=1e-12)
    assert y[3] == -30.0
    # all-zero envelope
    assert np.all(oracle.compress(np.zeros(4), "log", 0.0, 50.0) == -50.0)


def test_power_and_no_compression_values():
    env = np.array([0.0, 1.0, 2.0, 4.0, 9.0])
    np.testing.assert_allclose(oracle.compress(env, "power", ref=4.0, param=0.5),
                               [0.0, 0.5, np.sqrt(0.5), 1.0, 1.0], atol=1e-15)
    np.testing.assert_allclose(oracle.compress(env, "power", ref=0.0, param=1.0), env / 9.0)
    np.testing.assert_array_equal(oracle.compress(env, "none"), env)
