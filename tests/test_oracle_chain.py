"""Pins for the oracle's per-input wrappers, its pair correlator, and the
chain channeliser -> correlator on an injected point source (CPU only).

Independent references: exact Python integers, numpy's FFT applied to the
polyphase sums, the closed-form visibilities of a plane-wave tone (noise
free, Sec. "Correlation Kernel": the covariance of every receiver pair after
the filter bank of Sec. "Polyphase Filterbank"), and the expectation of the
visibilities of a noise-like point source in receiver noise, checked within
five standard deviations derived from the filter's overlap.
"""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.filterwarnings("ignore")

P, T = 64, 16


def _bl(a, b):
    return a * (a + 1) // 2 + b


def _G(h, nu):
    """Frequency response sum_m h[m] exp(2 pi i nu m), by direct summation."""
    m = np.arange(h.size)
    return np.sum(h.astype(np.float64) * np.exp(2j * np.pi * nu * m))


# --------------------------------------------------------------------------
# pair correlator
# --------------------------------------------------------------------------
def _py_pair(z, i, j):
    """sum_s z_i(s) conj(z_j(s)) with Python integers."""
    re = sum(int(z[s, i, 0]) * int(z[s, j, 0]) + int(z[s, i, 1]) * int(z[s, j, 1]) for s in range(z.shape[0]))
    im = sum(int(z[s, i, 1]) * int(z[s, j, 0]) - int(z[s, i, 0]) * int(z[s, j, 1]) for s in range(z.shape[0]))
    return re, im


def test_pairs_int_every_pair_both_orders_exact():
    """Every ordered pair (i, j), including j > i and i == j, against Python
    integers; (j, i) is the conjugate of (i, j)."""
    rng = np.random.default_rng(21)
    S, R = 23, 6
    z = rng.integers(-127, 128, size=(S, R, 2)).astype(np.int8)
    pairs = np.array([(i, j) for i in range(R) for j in range(R)], np.int32)
    out = oracle.xcorr_pairs_int(z, pairs)
    for e, (i, j) in enumerate(pairs):
        assert tuple(out[e]) == _py_pair(z, i, j), (i, j)
    for e, (i, j) in enumerate(pairs):
        f = i * R + j
        r = j * R + i
        assert out[f, 0] == out[r, 0] and out[f, 1] == -out[r, 1]
    assert np.any(out[:, 1] != 0)          # the order matters for this data


def test_pairs_int_match_the_triangle_layout():
    """The pair form and the whole-triangle form give the same integers at
    (bl(a,b), p, q) for i = 2a+p, j = 2b+q, and the conjugate for (j, i)."""
    rng = np.random.default_rng(22)
    S, Na = 17, 5
    z = rng.integers(-127, 128, size=(S, 2 * Na, 2)).astype(np.int8)
    V, _ = oracle.xcorr_int(z)
    a, b = np.tril_indices(Na)
    for p in range(2):
        for q in range(2):
            i, j = 2 * a + p, 2 * b + q
            fwd = oracle.xcorr_pairs_int(z, np.stack([i, j], 1))
            rev = oracle.xcorr_pairs_int(z, np.stack([j, i], 1))
            np.testing.assert_array_equal(fwd, V[:, p, q, :])
            np.testing.assert_array_equal(rev[:, 0], V[:, p, q, 0])
            np.testing.assert_array_equal(rev[:, 1], -V[:, p, q, 1])


def test_pairs_float_every_pair_against_numpy():
    rng = np.random.default_rng(23)
    S, R = 31, 5
    z = rng.standard_normal((S, R)) + 1j * rng.standard_normal((S, R))
    pairs = np.array([(i, j) for i in range(R) for j in range(R)], np.int32)
    out = oracle.xcorr_pairs(z, pairs)
    C = z.T @ np.conj(z)
    np.testing.assert_allclose(out, C[pairs[:, 0], pairs[:, 1]], rtol=1e-12, atol=1e-12)


# --------------------------------------------------------------------------
# per-input channeliser wrappers
# --------------------------------------------------------------------------
def _numpy_polyphase(x, taps, S):
    """[P][S][R] spectra: FIR sums per branch with numpy, then numpy's FFT."""
    xc = x[..., 0].astype(np.float64) + 1j * x[..., 1]          # [L][R]
    R = xc.shape[1]
    xb = xc[: (S + T - 1) * P].reshape(S + T - 1, P, R)
    h = taps.astype(np.float64).reshape(T, P)
    u = np.zeros((S, P, R), np.complex128)
    for t in range(T):
        u += h[t][None, :, None] * xb[t:t + S]
    return np.fft.fft(u, axis=1).transpose(1, 0, 2)


@pytest.mark.parametrize("inputs", [None, [5, 0, 3], [2]])
def test_ppf_subband_against_numpy_fft(inputs):
    rng = np.random.default_rng(24)
    S, R = 7, 6
    x = rng.integers(-3000, 3001, size=((S + T - 1) * P + 9, R, 2)).astype(np.int16)
    taps = rng.standard_normal(P * T).astype(np.float32)     # not symmetric
    y = oracle.ppf_subband(x, taps, P, T, S, inputs=inputs)
    ref = _numpy_polyphase(x, taps, S)
    sel = list(range(R)) if inputs is None else inputs
    assert y.shape == (P, S, len(sel))
    np.testing.assert_allclose(y, ref[:, :, sel], rtol=0, atol=1e-9 * np.abs(ref).max())


def test_ppf_subband_accepts_antenna_pol_layout():
    rng = np.random.default_rng(25)
    S, Na = 4, 3
    x = rng.integers(-100, 101, size=((S + T - 1) * P, Na, 2, 2)).astype(np.int16)
    taps = W.prototype_taps(P, T)
    a = oracle.ppf_subband(x, taps, P, T, S, inputs=[3, 4])
    b = oracle.ppf_subband(x.reshape(x.shape[0], 2 * Na, 2), taps, P, T, S)
    np.testing.assert_array_equal(a, b[:, :, [3, 4]])


@pytest.mark.parametrize("inputs", [None, [3, 1]])
def test_fine_subband_against_per_input_calls(inputs):
    rng = np.random.default_rng(26)
    Pf, R4, S, R = 256, 4, 3, 4
    x = rng.integers(-2000, 2001, size=((S + T - 1) * Pf, R, 2)).astype(np.int16)
    taps = rng.standard_normal(Pf * T).astype(np.float32)
    tau = rng.uniform(0, 6e-7, R)
    w = rng.uniform(0.5, 1.5, Pf).astype(np.float32)
    nu_c, df = 60.2e6, 195312.5 / Pf
    z = oracle.fine_subband(x, taps, Pf, T, S, tau, nu_c, df, w, R4, inputs=inputs)
    sel = list(range(R)) if inputs is None else inputs
    assert z.shape == (Pf // R4, S, len(sel))
    for n, i in enumerate(sel):
        ref = oracle.fine_channelise(x, taps, i, Pf, T, 0, S, tau[i], nu_c, df, w, R4)
        np.testing.assert_array_equal(z[:, :, n], ref.T)
    # each receiver carries its own delay: swapping the delays changes the result
    if inputs is None:
        z2 = oracle.fine_subband(x, taps, Pf, T, S, tau[::-1].copy(), nu_c, df, w, R4)
        assert not np.allclose(z2, z)


# --------------------------------------------------------------------------
# point source through the oracle's channeliser and correlator
# --------------------------------------------------------------------------
def _chain(x, taps, S):
    """Oracle chain: channelise every receiver, then correlate each channel."""
    y = oracle.ppf_subband(x, taps, P, T, S)                    # [P][S][R]
    return np.stack([oracle.xcorr(y[k])[0] for k in range(P)])   # [P][Nbl][2][2]


@pytest.mark.parametrize("k0", [0, 16, 32, 48])
def test_tone_at_channel_centre_exact(k0):
    """Noise-free plane wave on the grid of quarter turns (samples are exact
    integers): x_i[n] = A i^{q_i} exp(2 pi i k0 n / P).  Then in every
    channel k,
        V_ij[k] = S A^2 |G((k0 - k)/P)|^2 i^{q_i - q_j},
    so V_ij[k0] = S A^2 (sum h)^2 i^{q_i - q_j}, and the other channels fall
    off as the prototype's response."""
    rng = np.random.default_rng(30 + k0)
    Na, S, A = 4, 24, 1500
    R = 2 * Na
    q = rng.integers(0, 4, R)
    n = np.arange((S + T - 1) * P)
    quarter = np.array([1, 1j, -1, -1j])                       # i^0 .. i^3, exact
    xc = A * quarter[(q[None, :] + (k0 * n[:, None]) // (P // 4)) % 4]
    assert np.allclose(xc, A * np.exp(1j * (np.pi / 2 * q[None, :] + 2 * np.pi * k0 * n[:, None] / P)))
    xr = np.round(xc)
    assert np.array_equal(xr, xc)                              # exactly representable
    x = np.stack([xr.real, xr.imag], -1).astype(np.int16)       # [L][R][2]
    taps = W.prototype_taps(P, T)
    V = _chain(x, taps, S)
    g2 = np.array([abs(_G(taps, (k0 - k) / P)) ** 2 for k in range(P)])
    peak = S * A * A * g2[k0]
    assert abs(g2[k0] - float(taps.astype(np.float64).sum()) ** 2) < 1e-9 * g2[k0]
    a, b = np.tril_indices(Na)
    for p in range(2):
        for qq in range(2):
            i, j = 2 * a + p, 2 * b + qq
            ph = quarter[(q[i] - q[j]) % 4]
            ref = S * A * A * g2[:, None] * ph[None, :]          # [P][Nbl]
            np.testing.assert_allclose(V[:, :, p, qq], ref, rtol=1e-6, atol=1e-12 * peak)
    assert np.all(np.argmax(np.abs(V[:, 0, 0, 0])) == k0)


@pytest.mark.parametrize("k0,frac", [(5, 0.0), (40, 0.3), (61, 0.5)])
def test_geometric_plane_wave_within_rounding_bound(k0, frac):
    """A point source at direction (l, m) seen by antennas in a 30 m disc at
    60 MHz: phase phi_a = 2 pi nu (l x_a + m y_a) / c on both polarisations,
    frequency f = (k0 + frac)/P, amplitude A, int16-rounded.  Closed form
    V_ab[k] = S A^2 |G(f - k/P)|^2 exp(i (phi_a - phi_b)); each sample is off
    by at most sqrt(2)/2, so each spectrum by D = sqrt(2)/2 sum|h| and each
    visibility by S (|y_a| D + |y_b| D + D^2)."""
    cfg = W.Config("pin", 6, 1, n_spectra=16, layout="disc", seed=7)
    pos = W.antenna_positions(cfg)
    lm = np.array([[0.31, -0.52]])
    phi = np.angle(W.geometric_phases(pos, lm, 60e6)[0])          # [Na]
    Na, S, A = pos.shape[0], 16, 8000.0
    f = (k0 + frac) / P
    n = np.arange((S + T - 1) * P)
    xc = A * np.exp(1j * (2 * np.pi * f * n[:, None] + np.repeat(phi, 2)[None, :]))   # [L][2Na]
    x = np.stack([np.round(xc.real), np.round(xc.imag)], -1).astype(np.int16)
    taps = W.prototype_taps(P, T)
    V = _chain(x, taps, S)
    D = np.sqrt(0.5) * np.abs(taps.astype(np.float64)).sum()
    a, b = np.tril_indices(Na)
    ph = np.exp(1j * (phi[a] - phi[b]))
    for k in range(P):
        g = abs(_G(taps, f - k / P))
        ref = S * A * A * g * g * ph
        tol = S * (2 * A * g * D + D * D)
        for p in range(2):
            for qq in range(2):
                assert np.all(np.abs(V[k, :, p, qq] - ref) <= tol * (1 + 1e-9)), (k, p, qq)
    # the strongest channel is the nearest channel centre (ties to the lower one)
    assert int(np.argmax(np.abs(V[:, 0, 0, 0]))) == k0 + (1 if frac > 0.5 else 0)


def test_noise_and_source_expectation():
    """Receiver noise (sigma_n per component) plus an unpolarised noise-like
    point source (sigma_s per component, independent in X and Y) with
    geometric phases.  With rounding variance 1/12 per component:
        E V_ab^{pp} = S 2 sigma_s^2 sum h^2 e^{i(phi_a - phi_b)}
                      + [a = b] S 2 (sigma_n^2 + 1/12) sum h^2,
        E V_ab^{XY} = 0.
    Each visibility must lie within 5 standard deviations, from the complex
    Gaussian fourth moment: Var V_ij = S R_ii R_jj sum_d rho_d^2, where
    R = 2 (sigma_n^2 + sigma_s^2 + 1/12) sum h^2 and rho_d = sum_m h[m]
    h[m + dP] / sum h^2 is the correlation of spectra d apart (the windows
    overlap).  The mean over all baselines of the de-rotated cross power
    must also be within 5 standard errors of its expectation."""
    rng = np.random.default_rng(40)
    cfg = W.Config("pin", 8, 1, n_spectra=16, layout="disc", seed=9)
    pos = W.antenna_positions(cfg)
    Na, S = pos.shape[0], 6000
    sn, ss = 24.0, 24.0
    phi = np.angle(W.geometric_phases(pos, np.array([[-0.2, 0.45]]), 60e6)[0])
    L = (S + T - 1) * P
    src = (rng.standard_normal((L, 2)) + 1j * rng.standard_normal((L, 2))) * ss          # [L][pol]
    noise = (rng.standard_normal((L, Na, 2)) + 1j * rng.standard_normal((L, Na, 2))) * sn
    v = noise + src[:, None, :] * np.exp(1j * phi)[None, :, None]
    x = np.stack([np.round(v.real), np.round(v.imag)], -1).astype(np.int16).reshape(L, 2 * Na, 2)
    taps = W.prototype_taps(P, T)
    h = taps.astype(np.float64)
    sh2 = float(np.sum(h * h))
    rho = np.array([np.sum(h[: h.size - d * P] * h[d * P:]) / sh2 for d in range(T)])
    infl = rho[0] ** 2 + 2 * np.sum(rho[1:] ** 2)
    Y = oracle.ppf_subband(x, taps, P, T, S)                    # [P][S][R]
    for k in (0, 9, 40):
        V, _ = oracle.xcorr(Y[k])
        R = 2 * (sn * sn + ss * ss + 1 / 12) * sh2
        sd = np.sqrt(S * R * R * infl)
        a, b = np.tril_indices(Na)
        for p in range(2):
            for q in range(2):
                e = np.zeros(a.size, np.complex128)
                if p == q:
                    e += S * 2 * ss * ss * sh2 * np.exp(1j * (phi[a] - phi[b]))
                    e += np.where(a == b, S * 2 * (sn * sn + 1 / 12) * sh2, 0.0)
                dev = np.abs(V[:, p, q] - e)
                assert np.all(dev <= 5 * sd), (k, p, q, float(dev.max() / sd))
        # de-rotated mean cross power over the distinct baselines (XX and YY)
        cross = a != b
        der = np.concatenate([V[cross, p, p] * np.exp(-1j * (phi[a] - phi[b]))[cross] for p in range(2)])
        m = np.mean(der.real) / (S * 2 * ss * ss * sh2)
        # the source's own power fluctuation is common to all baselines of a
        # polarisation: its relative sd is sqrt(infl / S) per polarisation
        se = np.sqrt(infl / S) * np.sqrt(0.5) + sd / (S * 2 * ss * ss * sh2) / np.sqrt(cross.sum())
        assert abs(m - 1.0) <= 5 * se, (k, m, se)
