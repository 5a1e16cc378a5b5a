"""Pins for the oracle's lost-packet handling: spectrum validity and the
weighting matrix (CPU only).

Pinned against the closed form of the spectra one lost packet touches, a
brute-force sample-level sliding-window formulation in numpy, and the
correlation of a contiguous run of spectra when every antenna loses the
same packets.
"""
import numpy as np
import pytest

import oracle

Q, P, T = 16, 64, 16


def _sliding(pkt, Q, P, T, S):
    """Independent formulation: expand packets to samples, count lost samples
    in each window with a cumulative sum."""
    n_pk, Na = pkt.shape
    samp = np.repeat(pkt.astype(bool), Q, axis=0)                     # [n_samples][Na]
    need = (S + T - 1) * P
    if samp.shape[0] < need:
        samp = np.vstack([samp, np.zeros((need - samp.shape[0], Na), bool)])
    lost = np.concatenate([np.zeros((1, Na), np.int64), np.cumsum(~samp, axis=0)])
    s = np.arange(S)
    cnt = lost[(s + T) * P] - lost[s * P]                             # [S][Na]
    return (cnt == 0).T.astype(np.uint8)


@pytest.mark.parametrize("k", [0, 3, 63, 64, 200, 299])
def test_one_lost_packet_closed_form(k):
    """Spectrum s reads samples [sP, (s+T)P); packet k holds [kQ, (k+1)Q):
    s is invalid iff sP <= (k+1)Q - 1 and (s+T)P - 1 >= kQ."""
    S = 60
    n_pk = (S + T - 1) * P // Q
    pkt = np.ones((n_pk, 2), np.uint8)
    pkt[k, 1] = 0
    v = oracle.spectrum_validity(pkt, Q, P, T, S)
    lo = max(0, -(-(k * Q - T * P + 1) // P))
    hi = min(S - 1, ((k + 1) * Q - 1) // P)
    expect = np.ones(S, np.uint8)
    expect[lo:hi + 1] = 0
    np.testing.assert_array_equal(v[1], expect)
    assert np.all(v[0] == 1)
    assert (expect == 0).sum() in (16, 17) or lo == 0 or hi == S - 1


@pytest.mark.parametrize("P_,Q_,seed", [(64, 16, 1), (256, 16, 2), (64, 7, 3), (256, 100, 4)])
def test_random_loss_matches_sliding_window(P_, Q_, seed):
    rng = np.random.default_rng(seed)
    S, Na = 23, 5
    n_pk = -(-((S + T - 1) * P_) // Q_) - (seed % 2)                # sometimes one packet short
    pkt = (rng.random((n_pk, Na)) > 0.01).astype(np.uint8)
    v = oracle.spectrum_validity(pkt, Q_, P_, T, S)
    np.testing.assert_array_equal(v, _sliding(pkt, Q_, P_, T, S))
    sub = oracle.spectrum_validity(pkt, Q_, P_, T, S, antennas=(2, 4))
    np.testing.assert_array_equal(sub, v[2:4])


def test_weights_brute_force_and_flags():
    rng = np.random.default_rng(7)
    Na, S = 6, 40
    v = (rng.random((Na, S + 3)) > 0.3).astype(np.uint8)
    flags = np.zeros(Na, np.uint8)
    flags[4] = 1
    W = oracle.validity_weights(v, S, flags)
    for a in range(Na):
        for b in range(a + 1):
            n = int(np.sum(v[a, :S] & v[b, :S]))
            assert W[a * (a + 1) // 2 + b] == (0 if 4 in (a, b) else n)
    W2 = oracle.validity_weights(v, S)
    assert W2[4 * 5 // 2 + 4] == v[4, :S].sum()


def test_common_loss_equals_correlating_the_kept_spectra():
    """When every antenna loses the same samples, the masked visibility is
    the correlation of the spectra that stay valid, and every weight is
    their number."""
    rng = np.random.default_rng(9)
    Na, S = 4, 50
    n_pk = (S + T - 1) * P // Q
    pkt = np.ones((n_pk, Na), np.uint8)
    pkt[100:103, :] = 0
    v = oracle.spectrum_validity(pkt, Q, P, T, S)
    kept = np.flatnonzero(v[0])
    assert 0 < kept.size < S and np.all(v == v[0])
    z = rng.standard_normal((S, 2 * Na)) + 1j * rng.standard_normal((S, 2 * Na))
    Vm, _ = oracle.xcorr(oracle.zero_invalid(z, v))
    Vk, _ = oracle.xcorr(z[kept])
    np.testing.assert_allclose(Vm, Vk, rtol=1e-12, atol=1e-12)
    assert np.all(oracle.validity_weights(v, S) == kept.size)


def test_no_loss_is_the_plain_correlation():
    rng = np.random.default_rng(10)
    Na, S = 3, 20
    pkt = np.ones(((S + T - 1) * P // Q, Na), np.uint8)
    v = oracle.spectrum_validity(pkt, Q, P, T, S)
    assert np.all(v == 1)
    z = rng.standard_normal((S, 2 * Na)) + 1j * rng.standard_normal((S, 2 * Na))
    np.testing.assert_array_equal(oracle.zero_invalid(z, v), z)
    assert np.all(oracle.validity_weights(v, S) == S)
