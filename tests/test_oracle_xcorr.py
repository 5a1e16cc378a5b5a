"""Pins for the oracle's correlator (CPU only).

Independent references: numpy's matrix product Z^T conj(Z), exact Python
integers, the closed-form visibilities of a plane wave, Hermitian symmetry
checked through an antenna permutation, additivity over time, and the
flag/weight rules.
"""
import numpy as np
import pytest

import oracle


def _tri(Na):
    a, b = np.tril_indices(Na)
    return a, b


def _full_from_numpy(z):
    """numpy reference: C[i][j] = sum_s z[s][i] conj(z[s][j])."""
    return z.T @ np.conj(z)


def _lower_layout(C, Na):
    a, b = _tri(Na)
    out = np.empty((a.size, 2, 2), np.complex128)
    for p in range(2):
        for q in range(2):
            out[:, p, q] = C[2 * a + p, 2 * b + q]
    return out


@pytest.mark.parametrize("Na,S", [(1, 5), (3, 17), (7, 40)])
def test_matches_numpy_matmul(Na, S):
    rng = np.random.default_rng(Na * 100 + S)
    z = rng.standard_normal((S, 2 * Na)) + 1j * rng.standard_normal((S, 2 * Na))
    V, W = oracle.xcorr(z)
    ref = _lower_layout(_full_from_numpy(z), Na)
    np.testing.assert_allclose(V, ref, rtol=1e-12, atol=1e-12)
    assert np.all(W == S)


def test_int_exact_against_python_ints():
    rng = np.random.default_rng(1)
    S, Na = 33, 4
    z = rng.integers(-127, 128, size=(S, 2 * Na, 2)).astype(np.int8)
    V, W = oracle.xcorr_int(z)
    zc = z[..., 0].astype(object) + 1j * z[..., 1].astype(object)   # not used for ints
    a, b = _tri(Na)
    for e in range(a.size):
        for p in range(2):
            for q in range(2):
                i, j = 2 * a[e] + p, 2 * b[e] + q
                re = sum(int(z[s, i, 0]) * int(z[s, j, 0]) + int(z[s, i, 1]) * int(z[s, j, 1]) for s in range(S))
                im = sum(int(z[s, i, 1]) * int(z[s, j, 0]) - int(z[s, i, 0]) * int(z[s, j, 1]) for s in range(S))
                assert V[e, p, q, 0] == re and V[e, p, q, 1] == im
    del zc


def test_int_overflow_detected():
    S = 66600                     # 2 * 127^2 * S > 2^31
    z = np.full((S, 2, 2), 127, np.int8)
    with pytest.raises(OverflowError):
        oracle.xcorr_int(z)


def test_plane_wave_closed_form():
    """z_i(s) = A exp(i phi_i) exp(i theta_s): V_ij = S A^2 exp(i (phi_i - phi_j))."""
    rng = np.random.default_rng(4)
    Na, S, A = 5, 64, 2.5
    phi = rng.uniform(0, 2 * np.pi, 2 * Na)
    theta = rng.uniform(0, 2 * np.pi, S)
    z = A * np.exp(1j * (phi[None, :] + theta[:, None]))
    V, _ = oracle.xcorr(z)
    a, b = _tri(Na)
    for p in range(2):
        for q in range(2):
            ref = S * A * A * np.exp(1j * (phi[2 * a + p] - phi[2 * b + q]))
            np.testing.assert_allclose(V[:, p, q], ref, rtol=1e-12, atol=1e-10)


def test_hermitian_through_antenna_reversal():
    """Reversing antennas maps (a, b, p, q) to (Na-1-b, Na-1-a, q, p) conjugated."""
    rng = np.random.default_rng(8)
    Na, S = 6, 21
    z = rng.standard_normal((S, 2 * Na)) + 1j * rng.standard_normal((S, 2 * Na))
    zr = z.reshape(S, Na, 2)[:, ::-1, :].reshape(S, 2 * Na)
    V, _ = oracle.xcorr(z)
    Vr, _ = oracle.xcorr(zr)
    bl = lambda a, b: a * (a + 1) // 2 + b
    for a in range(Na):
        for b in range(a + 1):
            for p in range(2):
                for q in range(2):
                    a2, b2 = Na - 1 - b, Na - 1 - a
                    assert np.isclose(Vr[bl(a2, b2), q, p], np.conj(V[bl(a, b), p, q]), rtol=1e-12, atol=1e-12)


def test_autocorrelations_real_nonnegative():
    rng = np.random.default_rng(2)
    Na, S = 4, 50
    z = rng.integers(-127, 128, size=(S, 2 * Na, 2)).astype(np.int8)
    V, _ = oracle.xcorr_int(z)
    Vf, _ = oracle.xcorr(z.astype(np.float64))
    for a in range(Na):
        e = a * (a + 1) // 2 + a
        for p in range(2):
            assert V[e, p, p, 1] == 0 and V[e, p, p, 0] >= 0
            assert Vf[e, p, p].imag == 0.0 and Vf[e, p, p].real >= 0


def test_additive_over_time():
    rng = np.random.default_rng(6)
    Na, S1, S2 = 3, 13, 29
    z = rng.integers(-127, 128, size=(S1 + S2, 2 * Na, 2)).astype(np.int8)
    V, W = oracle.xcorr_int(z)
    V1, _ = oracle.xcorr_int(z[:S1])
    V2, _ = oracle.xcorr_int(z[S1:])
    np.testing.assert_array_equal(V, V1 + V2)
    assert np.all(W == S1 + S2)


def test_flags_zero_baselines():
    rng = np.random.default_rng(12)
    Na, S = 5, 9
    z = rng.standard_normal((S, 2 * Na)) + 1j * rng.standard_normal((S, 2 * Na))
    flags = np.array([0, 1, 0, 0, 1], np.uint8)
    V, W = oracle.xcorr(z, flags)
    V0, _ = oracle.xcorr(z)
    a, b = _tri(Na)
    hit = (flags[a] == 1) | (flags[b] == 1)
    assert np.all(V[hit] == 0) and np.all(W[hit] == 0)
    np.testing.assert_array_equal(V[~hit], V0[~hit])
    assert np.all(W[~hit] == S)


def test_pairs_match_triangle():
    rng = np.random.default_rng(13)
    Na, S = 4, 11
    z = rng.standard_normal((S, 2 * Na)) + 1j * rng.standard_normal((S, 2 * Na))
    V, _ = oracle.xcorr(z)
    pairs = np.array([[7, 0], [5, 5], [3, 2]])
    out = oracle.xcorr_pairs(z, pairs)
    bl = lambda a, b: a * (a + 1) // 2 + b
    assert np.allclose(out[0], V[bl(3, 0), 1, 0])
    assert np.allclose(out[1], V[bl(2, 2), 1, 1])
    assert np.allclose(out[2], V[bl(1, 1), 1, 0])


def test_int_flags_zero_baselines_and_weights():
    """Integer form: a baseline touching a flagged antenna is exactly 0 with
    weight 0; the others keep their exact sums and weight S."""
    rng = np.random.default_rng(14)
    Na, S = 5, 12
    z = rng.integers(-127, 128, size=(S, 2 * Na, 2)).astype(np.int8)
    flags = np.array([1, 0, 0, 1, 0], np.uint8)
    V, W = oracle.xcorr_int(z, flags)
    V0, W0 = oracle.xcorr_int(z)
    a, b = _tri(Na)
    hit = (flags[a] == 1) | (flags[b] == 1)
    assert np.all(V[hit] == 0) and np.all(W[hit] == 0)
    np.testing.assert_array_equal(V[~hit], V0[~hit])
    assert np.all(W[~hit] == S) and np.all(W0 == S)
