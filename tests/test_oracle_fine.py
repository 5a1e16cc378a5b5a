"""Pins for the oracle's fine channeliser: 256-channel filterbank, delay and
bandpass compensation, 4:1 channel integration (CPU only).

Pinned against numpy's FFT through a folding identity, against the phase a
delayed tone must carry, and against the channel map of the integration.
"""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.filterwarnings("ignore")

F_SB = 195312.5
PF, T, R = 256, 16, 4
DF = F_SB / PF


def _rand_x(rng, L, n_in, amp=1000):
    return rng.integers(-amp, amp + 1, size=(L, n_in, 2)).astype(np.int16)


def test_integration_is_a_folded_64_point_fft():
    """With no delay and unit weights, summing fine channels 4c..4c+3 of a
    256-point DFT equals the 64-point DFT of v[p] = sum_m u[p+64m] g[p+64m],
    g[p] = sum_{j<4} exp(-2 pi i j p / 256): exp(-2 pi i (4c+j) p / 256) =
    exp(-2 pi i c p / 64) exp(-2 pi i j p / 256), and exp(-2 pi i c p / 64)
    has period 64 in p."""
    rng = np.random.default_rng(11)
    S = 5
    x = _rand_x(rng, (S + T - 1) * PF, 2)
    taps = rng.standard_normal(PF * T).astype(np.float32)
    w = np.ones(PF, np.float32)
    for i in range(2):
        z = oracle.fine_channelise(x, taps, i, PF, T, 0, S, 0.0, 60e6, DF, w, R)
        xc = x[:, i, 0].astype(np.float64) + 1j * x[:, i, 1]
        h = taps.astype(np.float64).reshape(T, PF)
        p = np.arange(PF)
        g = np.exp(-2j * np.pi * np.outer(np.arange(R), p) / PF).sum(0)
        for s in range(S):
            u = (h * xc[s * PF:(s + T) * PF].reshape(T, PF)).sum(0)
            v = (u * g).reshape(R, PF // R).sum(0)
            ref = np.fft.fft(v)
            np.testing.assert_allclose(z[s], ref, rtol=1e-10, atol=1e-6 * np.abs(ref).max())


def test_unit_ratio_without_delay_is_the_plain_filterbank():
    rng = np.random.default_rng(12)
    S = 3
    x = _rand_x(rng, (S + T - 1) * PF, 1)
    taps = rng.standard_normal(PF * T).astype(np.float32)
    z = oracle.fine_channelise(x, taps, 0, PF, T, 0, S, 0.0, 50e6, DF, np.ones(PF, np.float32), 1)
    y = oracle.ppf_stream(x, taps, 0, PF, T, 0, S)
    np.testing.assert_array_equal(z, y)


@pytest.mark.parametrize("k0", [37, 200])
def test_delay_compensation_realigns_a_delayed_tone(k0):
    """Input 1 carries the tone of input 0 delayed by tau (complex baseband
    of a late RF signal: times exp(-2 pi i nu tau), nu = nu_c + f0).  After
    compensation fine channel k0 of both inputs agrees; with the delay of the
    wrong sign they differ by twice the phase."""
    nu_c, tau, A = 60e6 + 2 * F_SB, 3.3e-9, 12000.0
    f0 = (k0 if k0 < PF // 2 else k0 - PF) * DF
    S = 4
    n = np.arange((S + T - 1) * PF)
    tone = A * np.exp(2j * np.pi * f0 * n / F_SB)
    delayed = tone * np.exp(-2j * np.pi * (nu_c + f0) * tau)
    x = np.zeros((n.size, 2, 2), np.int16)
    for i, sig in enumerate((tone, delayed)):
        x[:, i, 0] = np.rint(sig.real).astype(np.int16)
        x[:, i, 1] = np.rint(sig.imag).astype(np.int16)
    taps = np.hanning(PF * T).astype(np.float32)
    w = np.ones(PF, np.float32)
    z0 = oracle.fine_channelise(x, taps, 0, PF, T, 0, S, 0.0, nu_c, DF, w, 1)[:, k0]
    z1 = oracle.fine_channelise(x, taps, 1, PF, T, 0, S, tau, nu_c, DF, w, 1)[:, k0]
    assert np.abs(z0).min() > 1e6
    np.testing.assert_allclose(np.angle(z1 / z0), 0.0, atol=1e-3)
    np.testing.assert_allclose(np.abs(z1 / z0), 1.0, atol=1e-3)
    wrong = oracle.fine_channelise(x, taps, 1, PF, T, 0, S, -tau, nu_c, DF, w, 1)[:, k0]
    expect = np.angle(np.exp(-4j * np.pi * (nu_c + f0) * tau))
    np.testing.assert_allclose(np.angle(wrong / z0), expect, atol=1e-3)


@pytest.mark.parametrize("k0", [0, 5, 127, 130, 255])
def test_weights_and_channel_map(k0):
    """A weight vector that keeps only fine channel k0 leaves only coarse
    channel k0 // 4, equal to fine channel k0, and a common weight scales."""
    rng = np.random.default_rng(k0)
    S = 2
    x = _rand_x(rng, (S + T - 1) * PF, 1)
    taps = rng.standard_normal(PF * T).astype(np.float32)
    nu_c, tau = 61e6, 2.0e-8
    fine = oracle.fine_channelise(x, taps, 0, PF, T, 0, S, tau, nu_c, DF, np.ones(PF, np.float32), 1)
    w = np.zeros(PF, np.float32)
    w[k0] = 1.0
    z = oracle.fine_channelise(x, taps, 0, PF, T, 0, S, tau, nu_c, DF, w, R)
    for c in range(PF // R):
        if c == k0 // R:
            np.testing.assert_allclose(z[:, c], fine[:, k0], rtol=1e-12)
        else:
            assert np.all(z[:, c] == 0)
    z1 = oracle.fine_channelise(x, taps, 0, PF, T, 0, S, tau, nu_c, DF, np.ones(PF, np.float32), R)
    z25 = oracle.fine_channelise(x, taps, 0, PF, T, 0, S, tau, nu_c, DF, np.full(PF, 2.5, np.float32), R)
    np.testing.assert_allclose(z25, 2.5 * z1, rtol=1e-12)
    np.testing.assert_allclose(z1, fine.reshape(S, PF // R, R).sum(-1), rtol=1e-9, atol=1e-9)
