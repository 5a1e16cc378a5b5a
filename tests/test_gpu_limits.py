"""GPU parity at the library's largest shapes: 4096 antennas (8192 receivers,
the limit of one launch), and the longest integration a subband of that many
receivers can hold (2^31 input values)."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import gather_rows, log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

NA_MAX = 4096


@pytest.fixture(scope="module")
def afc():
    import paper_1609_04205_amd as afc
    return afc


def _sampled_pairs(ants, inputs):
    """Receiver pairs (positions in `inputs`) of the baselines a >= b of
    `ants`, with (baseline index, p, q, a, b) of each."""
    pos = {i: k for k, i in enumerate(inputs)}
    pairs, where = [], []
    for ia, a in enumerate(ants):
        for b in ants[: ia + 1]:
            for p in range(2):
                for q in range(2):
                    pairs.append((pos[2 * a + p], pos[2 * b + q]))
                    where.append((a * (a + 1) // 2 + b, p, q, a, b))
    return np.array(pairs), where


@pytest.mark.parametrize("dtype", ["i8", "f32"])
def test_correlate_max_antennas(afc, dev, dtype):
    """8192 receivers, 20 spectra (a partial last block): 8.4 M baselines per
    channel, 17 GB of visibilities.  Sampled baselines at the array's ends
    and at 64- and 128-receiver tile edges against the oracle; flagged
    antennas (the last one among them) give exact zeros and weight 0."""
    Na, S = NA_MAX, 20
    log(f"xengine {dtype} Na={Na} S={S}")
    z = W.make_channelised(1, 64, S, 2 * Na, dtype, seed=41, device=dev)
    flagged = [5, 2047, Na - 1]
    fl = torch.zeros((1, Na), dtype=torch.uint8, device=dev)
    fl[0, flagged] = 1
    vis, w = afc.correlate(z, n_spectra=S, flags=fl)
    torch.cuda.synchronize()
    ants = [0, 5, 31, 32, 63, 64, 1000, 2047, 2048, 3071, 4031, 4032, Na - 2, Na - 1]
    inputs = [2 * a + p for a in ants for p in range(2)]
    pairs, where = _sampled_pairs(ants, inputs)
    blv = torch.as_tensor([x[0] for x in where], device=dev)
    hit = np.array([x[3] in flagged or x[4] in flagged for x in where])
    wv = w[0, blv].cpu().numpy()
    np.testing.assert_array_equal(wv, np.where(hit, 0, S))
    for ch in (0, 63):
        rows = gather_rows(z, 0, ch, inputs, S)
        got = vis[0, ch, blv].cpu().numpy()
        gp = np.array([got[k, where[k][1], where[k][2]] for k in range(len(where))])
        assert np.all(gp[hit] == 0)
        if dtype == "i8":
            ref = oracle.xcorr_pairs_int(rows, pairs)
            np.testing.assert_array_equal(gp[~hit].astype(np.int64), ref[~hit])
        else:
            r64 = rows.astype(np.float64)
            ref = oracle.xcorr_pairs(r64, pairs)
            auto = {k: oracle.xcorr_pairs(r64, np.array([[k, k]]))[0].real for k in range(len(inputs))}
            den = np.sqrt([auto[i] * auto[j] for i, j in pairs])
            err = np.abs((gp[:, 0] + 1j * gp[:, 1]) - ref) / den
            log(f"  ch {ch} max err {err[~hit].max():.2e}")
            assert err[~hit].max() <= 1e-5
    del z, vis, w
    torch.cuda.empty_cache()


def test_channelise_longest_integration_max_antennas(afc, dev):
    """8192 receivers and 2032 spectra: (2032 + 15) * 64 rows of 8192 complex
    int16 receivers is the most one subband may hold (just below 2^31 int16
    values); fp32 output 8.5 GB.  Sampled receivers, all channels and
    spectra, against the oracle."""
    Na, S = NA_MAX, 2032
    assert (S + 15) * 64 * 2 * Na * 2 < 2 ** 31 <= (S + 16) * 64 * 2 * Na * 2
    cfg = W.Config("max-na", Na, 1, n_spectra=S, sigma_n=32.0, n_sources=1, seed=43)
    log(f"ppf f32 Na={Na} S={S}")
    x = W.make_voltages(cfg, device=dev)
    taps_np = W.prototype_taps()
    taps = torch.from_numpy(taps_np).to(dev)
    z = afc.channelise(x, taps, S, "f32", 1.0)
    torch.cuda.synchronize()
    inputs = [0, 1, 4095, 4096, 2 * Na - 2, 2 * Na - 1]
    idx = torch.as_tensor(inputs, device=dev)
    xs = x[0].view(x.shape[1], 2 * Na, 2).index_select(1, idx).cpu().numpy()     # [L][R][2]
    ref = oracle.ppf_subband(xs, taps_np, 64, 16, S)                                  # [P][S][R]
    got = z[0].index_select(2, idx).permute(0, 1, 3, 2, 4).reshape(64, -1, len(inputs), 2)[:, :S].cpu().numpy()
    got = got[..., 0].astype(np.float64) + 1j * got[..., 1]
    sigma = np.sqrt(np.mean(np.abs(ref) ** 2) / 2)
    err = np.abs(got - ref).max() / sigma
    log(f"  max |dy|/sigma_y = {err:.3e}")
    assert err <= 1e-5
    del x, z
    torch.cuda.empty_cache()
