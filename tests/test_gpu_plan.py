"""Batching form: one graph (channeliser + correlator launches) over subbands
with their own integration length, sample type and antenna flags."""
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


def _plain(afc, x, taps, S_b, dt, gain, fl, Na):
    """Reference through the plain entry points for one subband."""
    L = (S_b + 15) * 64
    xs = x[:, :L].contiguous()
    z = afc.channelise(xs, taps, S_b, dt, gain)
    vis, w = afc.correlate(z, n_spectra=S_b, flags=fl)
    return z, vis, w


def _run_plan(afc, dev, Na, S_list, dts, flags_np, tune_cache=None, check_oracle=True):
    B = len(S_list)
    Smax = max(S_list)
    cfg = W.Config("plan", Na, B, n_spectra=Smax, sigma_n=32.0, n_sources=2, seed=31)
    x = W.make_voltages(cfg, device=dev)
    taps_np = W.prototype_taps()
    taps = torch.from_numpy(taps_np).to(dev)
    gain = W.requant_gain(cfg, taps_np)
    plan = afc.Plan(Na, S_list, dts, tune_cache=tune_cache)
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=dev)
    nbl = Na * (Na + 1) // 2
    vis = torch.zeros((B, 64, nbl, 2, 2, 2), dtype=torch.int32, device=dev)
    w = torch.zeros((B, nbl), dtype=torch.int32, device=dev)
    fl = torch.from_numpy(flags_np).to(dev)
    gains = [gain] * B
    plan.launch(x, taps, gains, ws, vis, flags=fl, weights=w)
    torch.cuda.synchronize()
    first = vis.clone()
    # replay the graph with eager work in between; every replay must match
    for _ in range(3):
        vis.zero_()
        _ = torch.randn(1000, device=dev).sum()
        torch.cuda.synchronize()
        plan.launch(x, taps, gains, ws, vis, flags=fl, weights=w)
        torch.cuda.synchronize()
        assert torch.equal(vis, first)
    info = plan.info()
    log(f"  plan tile={info.tile} wgs={info.n_workgroups} items={info.n_work_items}")
    return_info = info
    for b in range(B):
        fb = fl[b:b + 1]
        zr, vr, wr = _plain(afc, x[b:b + 1], taps, S_list[b], dts[b], gain, fb, Na)
        got = vis[b]
        if dts[b] != "i8":
            got = got.view(torch.float32)
        assert torch.equal(got, vr[0]), f"subband {b} differs from the plain path"
        assert torch.equal(w[b], wr[0])
        if check_oracle and b < 3:
            _check_subband_against_oracle(x[b], zr, got, w[b], S_list[b], dts[b], flags_np[b], Na, taps_np)
    plan.close()
    return return_info


def _check_subband_against_oracle(xb, zr, got, wb, S_b, dt, flags_b, Na, taps_np, channels=(0, 31)):
    """One subband of the plan against the oracle: int8 exactly against the
    integer correlator on the int8 samples the channeliser produced; fp32
    (<= 1e-5) and fp16 (<= 2e-3) against the FP64 chain, normalised by
    sqrt(V_ii V_jj).  Flagged baselines are exactly zero."""
    a_, b_ = np.tril_indices(Na)
    hit = (flags_b[a_] == 1) | (flags_b[b_] == 1)
    if dt == "i8":
        for ch in channels:
            rows = gather_rows(zr, 0, ch, range(2 * Na), S_b)
            Vref, Wref = oracle.xcorr_int(rows, flags_b)
            np.testing.assert_array_equal(got[ch].cpu().numpy(), Vref.astype(np.int32))
    else:
        y = oracle.ppf_subband(xb.cpu().numpy(), taps_np, 64, 16, S_b)
        v = vis_to_complex(got.cpu().numpy())
        for ch in channels:
            Vref, Wref = oracle.xcorr(y[ch], flags_b)
            e = normalised_error(v[ch], Vref, Na)
            assert np.all(v[ch][hit] == 0)
            tol = 1e-5 if dt == "f32" else 2e-3
            assert e[~hit].max() <= tol, (dt, ch, float(e[~hit].max()))
    np.testing.assert_array_equal(wb.cpu().numpy(), Wref)


def test_plan_small_mixed(afc, dev, tmp_path):
    log("plan small mixed")
    Na = 40
    S_list = [1024, 77, 500, 16, 333, 1]
    dts = ["f16", "i8", "f16", "i8", "i8", "f16"]
    flags = np.zeros((6, Na), np.uint8)
    flags[0, [2, 39]] = 1
    flags[3, 0] = 1
    flags[4, :] = 1
    _run_plan(afc, dev, Na, S_list, dts, flags, tune_cache=str(tmp_path / "tune.json"))
    assert (tmp_path / "tune.json").exists()


def test_plan_f32_subbands(afc, dev):
    log("plan fp32 + int8")
    Na = 24
    _run_plan(afc, dev, Na, [200, 64, 129], ["f32", "i8", "f32"], np.zeros((3, Na), np.uint8))


def test_plan_large_subband_output(afc, dev):
    """2304 receivers and 2000 spectra: a subband's channeliser output could
    reach 2.4 GB in fp32, above 2^31 bytes, so the batched channeliser
    stores through one buffer descriptor per channel; the plan equals the
    plain path (whose int8 subband output, 0.6 GB, takes the per-subband
    descriptor) bit for bit."""
    log("plan 2304 receivers, 2000 spectra")
    Na = 1152
    flags = np.zeros((1, Na), np.uint8)
    flags[0, [0, 600, 1151]] = 1
    _run_plan(afc, dev, Na, [2000], ["i8"], flags, check_oracle=False)


def test_plan_forced_small_tiles(afc, dev, tmp_path):
    """A tune cache entry selects 64-wide tiles at 4 workgroups per CU."""
    log("plan forced 64 tiles")
    Na = 72
    S_list = [300, 1000, 9]
    dts = ["i8", "f16", "f16"]
    key = f"N{2 * Na}_i8x1_f16x2_f32x0_S9-1000"
    path = tmp_path / "tune.json"
    path.write_text('{"%s": [64, 4]}\n' % key)
    flags = np.zeros((3, Na), np.uint8)
    flags[1, 70] = 1
    info = _run_plan(afc, dev, Na, S_list, dts, flags, tune_cache=str(path))
    assert info.tile == 64


def test_plan_split_launches(afc, dev, tmp_path):
    """A tune cache entry puts int8 and fp16 subbands in correlator launches
    of their own; results are unchanged."""
    log("plan split int8 / fp16 launches")
    Na = 56
    S_list = [700, 64, 333, 5]
    dts = ["i8", "f16", "i8", "f16"]
    key = f"N{2 * Na}_i8x2_f16x2_f32x0_S5-700"
    path = tmp_path / "tune.json"
    path.write_text('{"%s": [128, 2, 1]}\n' % key)
    flags = np.zeros((4, Na), np.uint8)
    flags[2, [3, 30, 55]] = 1
    _run_plan(afc, dev, Na, S_list, dts, flags, tune_cache=str(path))


def test_plan_full_size_a12_batched(afc, dev, tmp_path):
    """AARTFAAC-12 batching workload: 32 subbands, S_b in 500..3051, 0-10% flagged, mixed fp16/int8."""
    log("plan full size a12_batched")
    cfg = W.A12_BATCHED
    bp = W.batch_params(cfg)
    dts = ["f16" if d == 1 else "i8" for d in bp.dtypes]
    B = cfg.n_subbands
    Na = cfg.n_antennas
    x = W.make_voltages(cfg, device=dev)
    taps_np = W.prototype_taps()
    taps = torch.from_numpy(taps_np).to(dev)
    gain = W.requant_gain(cfg, taps_np)
    plan = afc.Plan(Na, bp.n_spectra.tolist(), dts, tune_cache=str(tmp_path / "tune.json"),
                    n_spectra=cfg.n_spectra)
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=dev)
    nbl = Na * (Na + 1) // 2
    vis = torch.empty((B, 64, nbl, 2, 2, 2), dtype=torch.int32, device=dev)
    w = torch.empty((B, nbl), dtype=torch.int32, device=dev)
    fl = torch.from_numpy(bp.flags).to(dev)
    plan.launch(x, taps, [gain] * B, ws, vis, flags=fl, weights=w)
    torch.cuda.synchronize()
    log(f"  plan info {plan.info()}")
    rng = np.random.default_rng(5)
    for b in (0, 13, 31):
        S_b = int(bp.n_spectra[b])
        zr, vr, wr = _plain(afc, x[b:b + 1], taps, S_b, dts[b], gain, fl[b:b + 1], Na)
        got = vis[b] if dts[b] == "i8" else vis[b].view(torch.float32)
        assert torch.equal(got, vr[0])
        assert torch.equal(w[b], wr[0])
        # sampled baselines against the oracle: int8 exactly on the GPU's own
        # int8 samples, fp16 against the FP64 chain (<= 2e-3 normalised)
        ants = np.sort(rng.choice(Na, size=12, replace=False))
        inputs = np.stack([2 * ants, 2 * ants + 1], 1).reshape(-1)
        fl_b = bp.flags[b]
        y = None if dts[b] == "i8" else oracle.ppf_subband(x[b].cpu().numpy(), taps_np, 64, 16, S_b, inputs=inputs)
        for ch in (3, 40):
            g = got[ch].cpu().numpy()
            if dts[b] == "i8":
                rows = gather_rows(zr, 0, ch, inputs, S_b)
            for ia in range(len(ants)):
                for ib in range(ia + 1):
                    a, c = ants[ia], ants[ib]
                    blx = a * (a + 1) // 2 + c
                    if fl_b[a] or fl_b[c]:
                        assert np.all(g[blx] == 0) and int(w[b, blx]) == 0
                        continue
                    assert int(w[b, blx]) == S_b
                    pairs = [(2 * ia + p, 2 * ib + q) for p in range(2) for q in range(2)]
                    if dts[b] == "i8":
                        ref = oracle.xcorr_pairs_int(rows, np.array(pairs)).reshape(2, 2, 2)
                        np.testing.assert_array_equal(g[blx], ref.astype(np.int32))
                    else:
                        ref = oracle.xcorr_pairs(y[ch], np.array(pairs)).reshape(2, 2)
                        auto_a = oracle.xcorr_pairs(y[ch], np.array([(2 * ia, 2 * ia), (2 * ia + 1, 2 * ia + 1)])).real
                        auto_c = oracle.xcorr_pairs(y[ch], np.array([(2 * ib, 2 * ib), (2 * ib + 1, 2 * ib + 1)])).real
                        den = np.sqrt(np.outer(auto_a, auto_c))
                        e = np.abs(vis_to_complex(g[blx]) - ref) / den
                        assert e.max() <= 2e-3, (b, ch, a, c, float(e.max()))
        del zr, vr, wr
    plan.close()
    del x, ws, vis
    torch.cuda.empty_cache()


def test_plan_relaunch_new_gains_on_side_stream(afc, dev):
    """Two launches on a side stream with different int8 gains and different
    output buffers, back to back without synchronisation, then a third with
    the first gains again: each result equals the plain channelise +
    correlate path with its own gains (a launch in flight never sees the
    next launch's gains)."""
    log("plan relaunch with new gains on a side stream")
    Na, S_list, dts = 20, [400, 90, 257], ["i8", "f16", "i8"]
    B = len(S_list)
    cfg = W.Config("plan2", Na, B, n_spectra=max(S_list), sigma_n=32.0, n_sources=1, seed=33)
    x = W.make_voltages(cfg, device=dev)
    taps_np = W.prototype_taps()
    taps = torch.from_numpy(taps_np).to(dev)
    g1 = W.requant_gain(cfg, taps_np)
    gains = [[g1] * B, [g1 * 0.37] * B, [g1] * B]
    plan = afc.Plan(Na, S_list, dts)
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=dev)
    nbl = Na * (Na + 1) // 2
    outs = [torch.full((B, 64, nbl, 2, 2, 2), -1, dtype=torch.int32, device=dev) for _ in range(3)]
    side = torch.cuda.Stream(device=dev)
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        for k in range(3):
            plan.launch(x, taps, gains[k], ws, outs[k])
    side.synchronize()
    for k in range(3):
        for b in range(B):
            _, vr, _ = _plain(afc, x[b:b + 1], taps, S_list[b], dts[b], gains[k][b], None, Na)
            got = outs[k][b] if dts[b] == "i8" else outs[k][b].view(torch.float32)
            assert torch.equal(got, vr[0]), f"launch {k} subband {b} differs from the plain path"
    assert not torch.equal(outs[0][0], outs[1][0])        # the gains really differ
    plan.close()
