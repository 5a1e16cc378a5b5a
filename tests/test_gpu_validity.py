"""GPU parity of the lost-packet path (afc_validity, afc_zero_invalid,
afc_validity_weights, afc_normalise_visibilities) against the CPU oracle:
bit-exact masks, zeroed samples and weights; the masked chain within the
chain tolerances (int8 exact against the device's own samples)."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import log, normalised_error, vis_to_complex

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def afc():
    import paper_1609_04205_amd as afc
    return afc


def _unpack(bits, S):
    """int32 [B][Wd][Na] -> uint8 [B][Na][S]."""
    u = bits.cpu().numpy().view(np.uint32)
    B, Wd, Na = u.shape
    s = np.arange(S)
    return ((u[:, s // 32, :] >> (s % 32)[None, :, None]) & 1).astype(np.uint8).transpose(0, 2, 1)


@pytest.mark.parametrize("Na,B,S,Q,Ps,rate", [(50, 2, 100, 16, 64, 0.01), (7, 3, 37, 16, 256, 0.02),
                                              (70, 1, 64, 7, 64, 0.005), (300, 1, 33, 100, 256, 0.01)])
def test_validity_bits(afc, dev, Na, B, S, Q, Ps, rate):
    n_rows = (S + 15) * Ps
    pkt = W.packet_loss(B, Na, n_rows, seed=Na + S, rate=rate, packet_samples=Q, dead=[(B - 1, 0)])
    if Na > 1:
        pkt[0, -1, 1] = 0                                   # the last packet of one antenna
    log(f"validity Na={Na} B={B} S={S} Q={Q} Ps={Ps}")
    bits = afc.validity(torch.from_numpy(pkt).to(dev), S, Q, Ps)
    got = _unpack(bits, S)
    for b in range(B):
        ref = oracle.spectrum_validity(pkt[b], Q, Ps, 16, S)
        np.testing.assert_array_equal(got[b], ref)
    raw = bits.cpu().numpy().view(np.uint32)
    if S % 32:
        assert np.all(raw[:, -1, :] >> (S % 32) == 0)        # bits of s >= S are clear
    log(f"  invalid fraction {1 - got.mean():.3f}")


@pytest.mark.parametrize("dtype", ["f32", "f16", "i8"])
def test_zero_invalid(afc, dev, dtype):
    B, Na, S = 2, 40, 90
    N = 2 * Na
    Sb = (S + 7) // 8
    pkt = W.packet_loss(B, Na, (S + 15) * 64, seed=3, rate=0.02, dead=[(1, 0)])
    bits = afc.validity(torch.from_numpy(pkt).to(dev), S, 16)
    z = W.make_channelised(B, 64, S, N, dtype, seed=5, device=dev)
    before = z.cpu().numpy().copy()
    afc.zero_invalid(z, bits, S)
    after = z.cpu().numpy()
    v = np.stack([oracle.spectrum_validity(pkt[b], 16, 64, 16, S) for b in range(B)])       # [B][Na][S]
    # samples kept: valid spectra, and the pad slots of spectra >= S (not touched)
    keep = np.ones((B, Sb * 8, N), bool)
    keep[:, :S, :] = np.repeat(v.transpose(0, 2, 1), 2, axis=2).astype(bool)
    keep = keep.reshape(B, Sb, 8, N).transpose(0, 1, 3, 2)                                  # [B][Sb][N][8]
    expect = np.where(keep[:, None, :, :, :, None], before, np.zeros_like(before))
    np.testing.assert_array_equal(after, expect)
    assert (before != after).any()


def test_weights_with_flags_and_ragged_S(afc, dev):
    B, Na, S = 3, 70, 130
    pkt = W.packet_loss(B, Na, (S + 15) * 64, seed=8, rate=0.02, dead=[(2, 1)])
    bits = afc.validity(torch.from_numpy(pkt).to(dev), S, 16)
    flags = np.zeros((B, Na), np.uint8)
    flags[1, [3, 50]] = 1
    Sb_list = [130, 77, 101]
    W_gpu = afc.validity_weights(bits, S, Sb_list, torch.from_numpy(flags).to(dev)).cpu().numpy()
    for b in range(B):
        v = oracle.spectrum_validity(pkt[b], 16, 64, 16, S)
        ref = oracle.validity_weights(v, Sb_list[b], flags[b])
        np.testing.assert_array_equal(W_gpu[b], ref)


@pytest.mark.parametrize("dtype", ["f32", "i8"])
def test_masked_chain(afc, dev, dtype):
    """channelise -> validity -> zero_invalid -> correlate -> weights, against
    the oracle's channeliser with the invalid spectra zeroed."""
    cfg = W.Config("masked", 24, 1, n_spectra=200, sigma_n=64.0, source_sigmas=(32.0,), seed=12)
    x = W.make_voltages(cfg, device=dev)
    taps = W.prototype_taps()
    S, Na = cfg.n_spectra, cfg.n_antennas
    pkt = W.packet_loss(1, Na, cfg.n_rows, seed=13, rate=0.01)
    pkt[0, 300:305, 5] = 0
    gain = W.requant_gain(cfg, taps)
    z = afc.channelise(x, torch.from_numpy(taps).to(dev), S, dtype, gain)
    bits = afc.validity(torch.from_numpy(pkt).to(dev), S, 16)
    afc.zero_invalid(z, bits, S)
    vis, _ = afc.correlate(z, n_spectra=S)
    Wt = afc.validity_weights(bits, S)
    v = oracle.spectrum_validity(pkt[0], 16, 64, 16, S)
    np.testing.assert_array_equal(Wt.cpu().numpy()[0], oracle.validity_weights(v, S))
    vv = vis_to_complex(vis.cpu().numpy())[0]
    log(f"masked chain {dtype}: invalid fraction {1 - v.mean():.3f}")
    if dtype == "i8":
        zz = z.cpu().numpy()[0]                                           # [P][Sb][N][8][2]
        for ch in (0, 9, 63):
            rows = zz[ch].transpose(0, 2, 1, 3).reshape(-1, 2 * Na, 2)[:S]
            # the device's own samples are zero where invalid
            zc = rows[..., 0].astype(np.float64) + 1j * rows[..., 1]
            assert np.all(oracle.zero_invalid(zc, v) == zc)
            Vi, _ = oracle.xcorr_int(rows)
            np.testing.assert_array_equal(vis.cpu().numpy()[0, ch], Vi)
    else:
        y = oracle.ppf_subband(x[0].cpu().numpy(), taps, 64, 16, S)       # [P][S][N]
        worst = 0.0
        for ch in (0, 9, 31, 63):
            Vref, _ = oracle.xcorr(oracle.zero_invalid(y[ch], v))
            worst = max(worst, float(normalised_error(vv[ch], Vref, Na).max()))
        log(f"  max normalised error {worst:.3e}")
        assert worst <= 1e-5


@pytest.mark.parametrize("dtype", ["f32", "i8"])
def test_normalise(afc, dev, dtype):
    B, Na = 2, 20
    nbl = Na * (Na + 1) // 2
    rng = np.random.default_rng(4)
    Wt = rng.integers(0, 3000, size=(B, nbl)).astype(np.int32)
    Wt[0, :5] = 0
    if dtype == "i8":
        vis = rng.integers(-2 ** 30, 2 ** 30, size=(B, 64, nbl, 2, 2, 2)).astype(np.int32)
        expect = (vis.astype(np.float64) / np.maximum(Wt, 1)[:, None, :, None, None, None]).astype(np.float32)
    else:
        vis = rng.standard_normal((B, 64, nbl, 2, 2, 2)).astype(np.float32) * 1e4
        expect = vis / np.maximum(Wt, 1).astype(np.float32)[:, None, :, None, None, None]
    expect[np.broadcast_to(Wt[:, None, :, None, None, None] == 0, expect.shape)] = 0
    out = afc.normalise_visibilities(torch.from_numpy(vis).to(dev), torch.from_numpy(Wt).to(dev)).cpu().numpy()
    np.testing.assert_array_equal(out, expect)


def test_validity_full_size_sampled(afc, dev):
    """AARTFAAC-12 shape: 16 subbands x 576 antennas x 3051 spectra, 0.1%
    packet loss plus one dead station; sampled antennas against the oracle,
    weights of sampled baselines against the oracle's count."""
    cfg = W.A12
    B, Na, S = cfg.n_subbands, cfg.n_antennas, cfg.n_spectra
    pkt = W.packet_loss(B, Na, cfg.n_rows, seed=3, dead=[(5, 7)])
    pt = torch.from_numpy(pkt).to(dev)
    bits = afc.validity(pt, S, 16)
    Wt = afc.validity_weights(bits, S).cpu().numpy()
    got = bits.cpu().numpy().view(np.uint32)
    rng = np.random.default_rng(0)
    for b in (0, 5, 15):
        ants = sorted(rng.choice(Na, size=4, replace=False).tolist()) + [7 * 48, Na - 1]
        v = np.stack([oracle.spectrum_validity(pkt[b], 16, 64, 16, S, antennas=(a, a + 1))[0] for a in ants])
        s = np.arange(S)
        g = ((got[b][s // 32][:, ants] >> (s % 32)[:, None]) & 1).T
        np.testing.assert_array_equal(g, v)
        for i, a in enumerate(ants):
            for j, c in enumerate(ants[:i + 1]):
                hi, lo = max(a, c), min(a, c)
                assert Wt[b, hi * (hi + 1) // 2 + lo] == int(np.sum(v[i] & v[j]))
        log(f"  sb={b} antennas={ants} valid fraction {v.mean():.4f}")
