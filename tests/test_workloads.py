"""Pins for the seeded inputs: prototype taps, shapes, and the paper's arithmetic."""
import json
import os

import numpy as np
import pytest

import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _G(h, nu):
    m = np.arange(h.size)
    return abs(np.sum(h.astype(np.float64) * np.exp(2j * np.pi * nu * m)))


def test_prototype_matches_scipy_window():
    ss = pytest.importorskip("scipy.signal")
    P, T = 64, 16
    M = P * T
    ref = ss.windows.hann(M, sym=True) * np.sinc((np.arange(M) - (M - 1) / 2) / P)
    np.testing.assert_array_equal(W.prototype_taps(P, T), ref.astype(np.float32))


def test_prototype_response():
    P = 64
    h = W.prototype_taps(P, 16)
    assert np.array_equal(h, h[::-1])                     # symmetric
    assert abs(h.astype(np.float64).sum() - 64.01262) < 1e-4
    assert abs((h.astype(np.float64) ** 2).sum() - 60.73603) < 1e-4
    g0 = _G(h, 0.0)
    assert abs(_G(h, 0.5 / P) / g0 - 0.49991) < 1e-4     # -6 dB at the channel edge
    assert abs(_G(h, 0.25 / P) / g0 - 1.00062) < 1e-4
    assert _G(h, 1.0 / P) / g0 < 1e-4                     # adjacent channel centre


def test_voltage_shape_and_range():
    cfg = W.SMALL
    x = W.make_voltages(cfg, n_rows=4096)
    assert tuple(x.shape) == (1, 4096, 48, 2, 2)
    xf = x.float()
    s = float(xf.std())
    eff = np.sqrt(cfg.sigma_n ** 2 + 16.0 ** 2)
    assert abs(s / eff - 1) < 0.03


def test_voltage_source_coherence():
    """The injected source makes inputs correlated with the geometric phase."""
    cfg = W.SMALL
    x = W.make_voltages(cfg, n_rows=65536).numpy().astype(np.float64)
    z = x[0, ..., 0] + 1j * x[0, ..., 1]                   # [L][Na][2]
    pos = W.antenna_positions(cfg)
    ph = W.geometric_phases(pos, W.source_directions(cfg), W.subband_frequency(0))[0]
    c = np.mean(z[:, 3, 0] * np.conj(z[:, 7, 0]))
    expect = 2 * 16.0 ** 2 * ph[3] * np.conj(ph[7])
    assert abs(c - expect) < 0.15 * abs(expect)


def test_channelised_blocks_padding():
    z = W.make_channelised(1, 2, 13, 6, "i8", seed=1)
    assert tuple(z.shape) == (1, 2, 2, 6, 8, 2)
    assert int(z[:, :, 1, :, 5:, :].abs().max()) == 0
    assert int(z.min()) >= -127
    zn = W.blocked_to_natural(z, 13)
    assert tuple(zn.shape) == (1, 2, 13, 6, 2)
    assert np.array_equal(zn[0, 1, 9, 4].numpy(), z[0, 1, 1, 4, 1].numpy())


def test_batch_params():
    bp = W.batch_params(W.A12_BATCHED)
    assert bp.n_spectra.min() >= 500 and bp.n_spectra.max() <= 3051
    assert bp.flags.shape == (32, 576)
    assert bp.flags.sum(axis=1).max() <= round(0.1 * 576)
    assert set(np.unique(bp.dtypes)) <= {1, 2}


def test_paper_arithmetic():
    """The workload shapes reproduce the paper's own figures."""
    pn = json.load(open(os.path.join(GOLDEN, "paper_numbers.json")))
    f = pn["subband_hz"]
    assert f == W.F_SUBBAND
    N = pn["dipoles_a12"]
    flops = 8 * N * (N + 1) / 2 * f                            # 8 flop per complex MAC
    assert abs(flops / 1e12 - pn["tflops_per_subband"]) < 0.05
    gbps = pn["station_dipoles"] * pn["subbands_processed"] * f * 16 / 1e9
    assert abs(gbps - pn["station_gbps"]) / pn["station_gbps"] < 0.02
    t2 = pn["table2"]
    fir = N * f * pn["fir_taps"] * 4 / (t2["fir_ms"]["a12"] * 1e-3) / 1e12
    assert abs(fir - t2["fir_tflops"]["a12"]) / t2["fir_tflops"]["a12"] < 0.01
    n = t2["fft_points"]
    fft = N * f * 5 * np.log2(n) / (t2["fft_ms"]["a12"] * 1e-3) / 1e12
    assert abs(fft - t2["fft_tflops"]["a12"]) / t2["fft_tflops"]["a12"] < 0.01
    # 3051 spectra of 64 channels fill just under one second (Table 1: 1 s)
    assert 0.999 < 3051 * 64 / f < 1.0
    assert abs(f / 64 - 3051.7578125) < 1e-9                  # ~3 kHz channels
