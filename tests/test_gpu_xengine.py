"""GPU parity of the correlator (afc_correlate) against the CPU oracle.

Inputs are seeded channelised samples drawn directly in the block layout
(workloads.make_channelised); the oracle receives the same values in its
natural [S][N] layout.  int8: bit-exact against exact integer sums.  fp16 and
fp32: float32 accumulation of exactly representable products, compared per
baseline with the error normalised by sqrt(V_ii V_jj).
"""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import gather_rows, log, normalised_error, vis_to_complex

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def afc():
    import paper_1609_04205_amd as afc
    return afc


def _oracle_channel(zn, dtype, flags=None):
    if dtype == "i8":
        V, W_ = oracle.xcorr_int(zn, flags)
        return V, W_
    V, W_ = oracle.xcorr(zn.astype(np.float64), flags)
    return V, W_


CASES = [
    # (dtype, B, Na, S, per-subband S or None, flagged antennas or None, channels to check)
    ("i8", 2, 48, 1024, None, None, range(64)),
    ("f16", 2, 48, 1024, None, None, range(0, 64, 7)),
    ("f32", 2, 48, 1024, None, None, range(0, 64, 7)),
    ("i8", 1, 70, 37, None, [3, 69], range(0, 64, 9)),        # N = 140: ragged against 128 and 64 tiles
    ("f16", 1, 70, 37, None, [0], range(0, 64, 9)),
    ("f32", 1, 70, 37, None, [1], range(0, 64, 9)),
    ("i8", 2, 33, 100, [100, 61], [5], range(0, 64, 13)),     # spectra >= S_b ignored although nonzero
    ("f32", 2, 33, 100, [3, 100], None, range(0, 64, 13)),
    ("i8", 1, 1, 5, None, None, range(64)),                   # one antenna
    ("f16", 1, 64, 16, None, None, range(0, 64, 21)),         # exactly one 128 tile
    # three 128-row tiles (off-diagonal tiles load their column operands
    # directly) with stage counts that are not a multiple of the register ring
    ("i8", 2, 150, 300, [300, 171], [7], range(0, 64, 13)),
    ("f16", 1, 150, 77, None, None, range(0, 64, 13)),
    # one spectrum block (one real stage, the rest of the register ring padding)
    ("i8", 2, 100, 8, [8, 1], [99], range(0, 64, 17)),
    ("f16", 1, 100, 3, None, None, range(0, 64, 17)),
]


@pytest.mark.parametrize("dtype,B,Na,S,S_sb,flagged,chans", CASES)
def test_correlate_matches_oracle(afc, dev, dtype, B, Na, S, S_sb, flagged, chans):
    log(f"xengine {dtype} B={B} Na={Na} S={S} S_sb={S_sb} flagged={flagged}")
    z = W.make_channelised(B, 64, S, 2 * Na, dtype, seed=Na * 7 + S, device=dev)
    if S_sb is not None:
        # fill the slots beyond each subband's S_b with nonzero values: they must be ignored
        zf = W.make_channelised(B, 64, S, 2 * Na, dtype, seed=99, device=dev)
        z = torch.where(z == 0, zf, z)
    fl = None
    if flagged is not None:
        fl_np = np.zeros((B, Na), np.uint8)
        fl_np[:, flagged] = 1
        fl = torch.from_numpy(fl_np).to(dev)
    vis, w = afc.correlate(z, n_spectra=S, n_spectra_per_sb=S_sb, flags=fl)
    torch.cuda.synchronize()
    vis_np = vis.cpu().numpy()
    w_np = w.cpu().numpy()
    zn_all = W.blocked_to_natural(z.cpu(), z.shape[2] * 8).numpy()
    for b in range(B):
        Sb_ = S if S_sb is None else S_sb[b]
        fb = None if fl is None else fl_np[b]
        for ch in chans:
            zn = zn_all[b, ch, :Sb_]
            Vref, Wref = _oracle_channel(zn, dtype, fb)
            if dtype == "i8":
                np.testing.assert_array_equal(vis_np[b, ch].astype(np.int64), Vref)
            else:
                got = vis_to_complex(vis_np[b, ch])
                ref = Vref
                err = normalised_error(got, ref, Na)
                if fb is not None:
                    a_, b_ = np.tril_indices(Na)
                    hit = (fb[a_] == 1) | (fb[b_] == 1)
                    assert np.all(got[hit] == 0)
                    err = err[~hit]
                assert err.max() <= 1e-5, (b, ch, err.max())
            np.testing.assert_array_equal(w_np[b], Wref)


def test_autocorrelations_exactly_real(afc, dev):
    z = W.make_channelised(1, 64, 200, 96, "f32", seed=3, device=dev)
    vis, _ = afc.correlate(z, n_spectra=200)
    v = vis.cpu().numpy()
    d = np.array([a * (a + 1) // 2 + a for a in range(48)])
    assert np.all(v[:, :, d, 0, 0, 1] == 0) and np.all(v[:, :, d, 1, 1, 1] == 0)
    assert np.all(v[:, :, d, 0, 0, 0] >= 0) and np.all(v[:, :, d, 1, 1, 0] >= 0)


def test_int8_extreme_values_exact(afc, dev):
    """All samples at +-127 (the largest products) stay exact; -128 is never produced."""
    g = torch.Generator(device=dev)
    g.manual_seed(11)
    S = 3051
    bits = torch.randint(0, 2, (1, 64, (S + 7) // 8, 96, 8, 2), generator=g, device=dev)
    z = (bits * 254 - 127).to(torch.int8)
    z[:, :, -1, :, S % 8:, :] = 0
    vis, _ = afc.correlate(z, n_spectra=S)
    v = vis.cpu().numpy()
    zn = W.blocked_to_natural(z.cpu(), z.shape[2] * 8).numpy()
    for ch in (0, 33):
        Vref, _ = oracle.xcorr_int(zn[0, ch, :S])
        np.testing.assert_array_equal(v[0, ch].astype(np.int64), Vref)


@pytest.mark.parametrize("dtype,B,Na,S", [("i8", 2, 576, 3051), ("f16", 1, 576, 763), ("i8", 2, 150, 300),
                                          ("f16", 1, 150, 77), ("i8", 1, 70, 37)])
def test_repeated_launches_bit_identical(afc, dev, dtype, B, Na, S):
    """The DMA ring's stage barrier orders the refill of a stage buffer after
    every wave's reads of it; a missing wait would show as launches that
    differ.  Every repeat (with other work queued in between) must equal the
    first bit for bit, on 128-wide diagonal and off-diagonal tiles and
    ragged tails."""
    log(f"xengine repeats {dtype} B={B} Na={Na} S={S}")
    z = W.make_channelised(B, 64, S, 2 * Na, dtype, seed=12, device=dev)
    fl = torch.zeros((B, Na), dtype=torch.uint8, device=dev)
    fl[:, Na // 3] = 1
    vis = torch.empty(afc.visibility_shape(B, Na), dtype=torch.int32 if dtype == "i8" else torch.float32,
                      device=dev)
    afc.correlate(z, n_spectra=S, out=vis, flags=fl, want_weights=False)
    torch.cuda.synchronize()
    first = vis.view(torch.int32).clone()
    for _ in range(6):
        vis.fill_(-1)
        _ = torch.randn(4096, device=dev).sum()
        afc.correlate(z, n_spectra=S, out=vis, flags=fl, want_weights=False)
        torch.cuda.synchronize()
        assert torch.equal(vis.view(torch.int32), first)
    del z, vis, first
    torch.cuda.empty_cache()


@pytest.mark.parametrize("dtype", ["i8", "f16"])
def test_checked_and_check_free_stores_agree(afc, dev, dtype):
    """Channel 0's tiles store through the checked path when weights are
    asked for and through the check-free one otherwise (interior
    off-diagonal 128-wide tiles): the visibilities are the same bit for bit,
    with and without flagged antennas."""
    Na, S = 576, 300
    z = W.make_channelised(2, 64, S, 2 * Na, dtype, seed=21, device=dev)
    for flagged in ([], [0, 200, 575]):
        fl = torch.zeros((2, Na), dtype=torch.uint8, device=dev)
        if flagged:
            fl[:, flagged] = 1
        v_w, _ = afc.correlate(z, n_spectra=S, flags=fl)
        v_n, _ = afc.correlate(z, n_spectra=S, flags=fl, want_weights=False)
        torch.cuda.synchronize()
        assert torch.equal(v_w.view(torch.int32), v_n.view(torch.int32)), flagged
    del z, v_w, v_n
    torch.cuda.empty_cache()


@pytest.mark.parametrize("dtype", ["i8", "f16", "f32"])
def test_full_size_sampled(afc, dev, dtype):
    """AARTFAAC-12 shape: 1152 receivers, 16 subbands, 3051 spectra, sampled baselines."""
    Na, B, S = 576, 16, 3051
    log(f"xengine full size {dtype}")
    z = W.make_channelised(B, 64, S, 2 * Na, dtype, seed=5, device=dev)
    vis, w = afc.correlate(z, n_spectra=S)
    torch.cuda.synchronize()
    rng = np.random.default_rng(1)
    for _ in range(6):
        sb = int(rng.integers(B))
        ch = int(rng.integers(64))
        ants = sorted(set(rng.choice(Na, size=5, replace=False).tolist() + [Na - 1, 0]))
        inputs = [2 * a + p for a in ants for p in range(2)]
        rows = gather_rows(z, sb, ch, inputs, S)
        pos = {i: k for k, i in enumerate(inputs)}
        pairs, where = [], []
        for ia, a in enumerate(ants):
            for b in ants[: ia + 1]:
                for p in range(2):
                    for q in range(2):
                        pairs.append((pos[2 * a + p], pos[2 * b + q]))
                        where.append((a * (a + 1) // 2 + b, p, q))
        pairs = np.array(pairs)
        blv = np.array([x[0] for x in where])
        got = vis[sb, ch, torch.as_tensor(blv, device=dev)].cpu().numpy()     # [n][2][2][2]
        gp = np.array([got[k, where[k][1], where[k][2]] for k in range(len(where))])
        if dtype == "i8":
            ref = oracle.xcorr_pairs_int(rows, pairs)
            np.testing.assert_array_equal(gp.astype(np.int64), ref)
        else:
            ref = oracle.xcorr_pairs(rows.astype(np.float64), pairs)
            autos = {pos[i]: oracle.xcorr_pairs(rows.astype(np.float64), np.array([[pos[i], pos[i]]]))[0].real
                     for i in inputs}
            den = np.sqrt([autos[i] * autos[j] for i, j in pairs])
            err = np.abs((gp[:, 0] + 1j * gp[:, 1]) - ref) / den
            assert err.max() <= 1e-5
    assert int(w.min()) == S and int(w.max()) == S
    del z, vis
    torch.cuda.empty_cache()
