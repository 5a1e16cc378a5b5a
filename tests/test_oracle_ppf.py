"""Pins for the oracle's channeliser and requantiser (CPU only).

Each test pins the oracle to something other than itself: numpy's FFT, the
closed-form response of a single impulse or of an exactly representable
tone, linearity, the expected power of white noise, and the float32
rounding rules for the requantiser.
"""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.filterwarnings("ignore")


def _rand_x(rng, L, R, amp=1000):
    return rng.integers(-amp, amp + 1, size=(L, R, 2)).astype(np.int16)


@pytest.mark.parametrize("P", [4, 8, 64])
def test_single_tap_is_blockwise_fft(P):
    """T = 1 and h = 1: y[s] is numpy's FFT of samples s*P .. s*P+P-1."""
    rng = np.random.default_rng(P)
    S, R = 6, 3
    x = _rand_x(rng, S * P, R)
    taps = np.ones(P, np.float32)
    for i in range(R):
        y = oracle.ppf_stream(x, taps, i, P, 1, 0, S)
        xc = x[:, i, 0].astype(np.float64) + 1j * x[:, i, 1]
        ref = np.fft.fft(xc.reshape(S, P), axis=1)
        np.testing.assert_allclose(y, ref, rtol=0, atol=1e-9 * np.abs(ref).max())


def test_polyphase_equals_windowed_dft():
    rng = np.random.default_rng(7)
    P, T, S, R = 16, 4, 9, 2
    x = _rand_x(rng, (S + T - 1) * P + 5, R)
    taps = rng.standard_normal(P * T).astype(np.float32)
    for i in range(R):
        a = oracle.ppf_stream(x, taps, i, P, T, 2, S)
        b = oracle.ppf_stream(x, taps, i, P, T, 2, S, direct=True)
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-9 * np.abs(b).max())


@pytest.mark.parametrize("n0", [0, 5, 37, 63, 64, 200, 511])
def test_impulse_response_closed_form(n0):
    """x = A*delta[n - n0]: y[s][k] = A h[n0 - sP] exp(-2 pi i k (n0 - sP)/P).

    Random (non-symmetric) taps, so a reversed tap order, a flipped FFT sign
    or a swapped branch/channel index all fail.
    """
    rng = np.random.default_rng(n0 + 11)
    P, T = 8, 4
    S = 70
    L = (S + T - 1) * P
    x = np.zeros((L, 3, 2), np.int16)
    A = 3 - 2j
    x[n0, 1, 0], x[n0, 1, 1] = 3, -2
    taps = rng.standard_normal(P * T).astype(np.float32)
    y = oracle.ppf_stream(x, taps, 1, P, T, 0, S)
    ref = np.zeros((S, P), np.complex128)
    k = np.arange(P)
    for s in range(S):
        m = n0 - s * P
        if 0 <= m < P * T:
            ref[s] = A * float(taps[m]) * np.exp(-2j * np.pi * k * m / P)
    np.testing.assert_allclose(y, ref, rtol=0, atol=1e-12)
    # the other inputs see nothing
    assert np.all(oracle.ppf_stream(x, taps, 0, P, T, 0, S) == 0)


def _dtft(h, nu):
    m = np.arange(h.size)
    return np.sum(h.astype(np.float64) * np.exp(2j * np.pi * nu * m))


@pytest.mark.parametrize("k0", [0, 16, 32, 48])
def test_tone_at_channel_centre(k0):
    """x[n] = A exp(2 pi i k0 n / P) with integer samples (k0 in {0,P/4,P/2,3P/4}).

    y[s][k] = A * G((k0 - k)/P), G(nu) = sum_m h[m] exp(2 pi i nu m):
    the peak channel is k0 with value A * sum(h), constant over s.
    """
    P, T, S = 64, 16, 5
    taps = W.prototype_taps(P, T)
    L = (S + T - 1) * P
    n = np.arange(L)
    ph = np.exp(2j * np.pi * k0 * n / P)
    A = 100
    xc = np.round(A * ph)
    assert np.allclose(xc, A * ph)          # exactly representable
    x = np.zeros((L, 1, 2), np.int16)
    x[:, 0, 0] = xc.real
    x[:, 0, 1] = xc.imag
    y = oracle.ppf_stream(x, taps, 0, P, T, 0, S)
    for k in range(P):
        g = A * _dtft(taps, (k0 - k) / P)
        np.testing.assert_allclose(y[:, k], np.full(S, g), rtol=0, atol=1e-9 * A * taps.sum())
    assert np.all(np.argmax(np.abs(y), axis=1) == k0)
    np.testing.assert_allclose(y[:, k0].real, A * taps.astype(np.float64).sum(), rtol=1e-12)


def test_off_grid_tone_magnitude():
    """Non-integer frequency: |y[s][k]| = A|G(f - k/P)| within the int16 rounding bound."""
    P, T, S = 64, 16, 4
    taps = W.prototype_taps(P, T)
    f = 10.3 / P
    L = (S + T - 1) * P
    n = np.arange(L)
    A = 8000.0
    xc = A * np.exp(2j * np.pi * f * n)
    x = np.zeros((L, 1, 2), np.int16)
    x[:, 0, 0] = np.round(xc.real)
    x[:, 0, 1] = np.round(xc.imag)
    y = oracle.ppf_stream(x, taps, 0, P, T, 0, S)
    bound = np.sqrt(0.5) * np.abs(taps.astype(np.float64)).sum()     # |rounding| <= sqrt(2)/2
    for k in range(P):
        g = A * abs(_dtft(taps, f - k / P))
        assert np.all(np.abs(np.abs(y[:, k]) - g) <= bound + 1e-9)
    assert np.all(np.argmax(np.abs(y), axis=1) == 10)


def test_linearity():
    rng = np.random.default_rng(3)
    P, T, S = 64, 16, 3
    L = (S + T - 1) * P
    taps = W.prototype_taps(P, T)
    a = _rand_x(rng, L, 1, 5000)
    b = _rand_x(rng, L, 1, 5000)
    ya = oracle.ppf_stream(a, taps, 0, P, T, 0, S)
    yb = oracle.ppf_stream(b, taps, 0, P, T, 0, S)
    yab = oracle.ppf_stream((a + b).astype(np.int16), taps, 0, P, T, 0, S)
    np.testing.assert_allclose(yab, ya + yb, rtol=0, atol=1e-8 * np.abs(yab).max())


def test_white_noise_power():
    """E|y|^2 = 2 sigma^2 sum h^2 for independent real/imag noise of variance sigma^2."""
    rng = np.random.default_rng(9)
    P, T, S = 64, 16, 400
    taps = W.prototype_taps(P, T)
    sigma = 300.0
    L = (S + T - 1) * P
    x = np.round(rng.normal(0, sigma, (L, 1, 2))).astype(np.int16)
    var = float(np.var(x.astype(np.float64)))           # includes the rounding variance
    y = oracle.ppf_stream(x, taps, 0, P, T, 0, S)
    expect = 2.0 * var * float(np.sum(taps.astype(np.float64) ** 2))
    # spectra overlap by T-1 blocks, so count only every T-th spectrum as independent
    n_indep = (S // T) * P
    meas = float(np.mean(np.abs(y) ** 2))
    assert abs(meas / expect - 1.0) < 5.0 / np.sqrt(n_indep)


def test_range_check():
    x = np.zeros((64 * 10, 1, 2), np.int16)
    taps = np.ones(64 * 16, np.float32)
    with pytest.raises(ValueError):
        oracle.ppf_stream(x, taps, 0, 64, 16, 0, 1)


# --------------------------------------------------------------------------
# requantiser
# --------------------------------------------------------------------------
def test_requant_ties_and_clamp():
    y = np.array([2.5, 3.5, -2.5, -3.5, 0.5, -0.5, 1.5, 126.5, 127.49, 127.5, 128.0, 1e9,
                  -126.5, -127.5, -1e9, 0.49999997, -0.0], np.float32)
    q = oracle.requant(y, 1.0)
    assert q.tolist() == [2, 4, -2, -4, 0, 0, 2, 126, 127, 127, 127, 127,
                          -126, -127, -127, 0, 0]


def test_requant_rounds_the_exact_product_once():
    rng = np.random.default_rng(5)
    y = (rng.standard_normal(200000) * 300).astype(np.float32)
    gain = np.float32(0.1273)
    q = oracle.requant(y, float(gain))
    # a float32 x float32 product is exact in float64 (48 significant bits)
    ref = np.clip(np.rint(y.astype(np.float64) * np.float64(gain)), -127, 127).astype(np.int8)
    np.testing.assert_array_equal(q, ref)
    assert q.min() >= -127
    # a double-rounding case: 7.5 * fp32(1/3) = 2.50000007..., which float32
    # rounds to 2.5 (then to 2, ties to even); the exact product rounds to 3
    g3 = np.float32(1.0 / 3.0)
    assert np.rint(np.float32(7.5) * g3) == 2.0
    assert oracle.requant(np.array([7.5, -7.5], np.float32), float(g3)).tolist() == [3, -3]
