"""Batching form: one graph (channeliser + correlator launches) over subbands
with their own integration length, sample type and antenna flags."""
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
        if check_oracle and dts[b] == "f16" and b < 2:
            y = oracle.ppf_subband(x[b].cpu().numpy(), taps_np, 64, 16, S_list[b])
            v = vis_to_complex(got.cpu().numpy())
            for ch in (0, 31):
                Vref, Wref = oracle.xcorr(y[ch], flags_np[b])
                e = normalised_error(v[ch], Vref, Na)
                a_, b_ = np.tril_indices(Na)
                hit = (flags_np[b][a_] == 1) | (flags_np[b][b_] == 1)
                assert np.all(v[ch][hit] == 0)
                assert e[~hit].max() <= 2e-3
            np.testing.assert_array_equal(w[b].cpu().numpy(), Wref)
    plan.close()
    return return_info


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
    for b in (0, 13, 31):
        zr, vr, wr = _plain(afc, x[b:b + 1], taps, int(bp.n_spectra[b]), dts[b], gain, fl[b:b + 1], Na)
        got = vis[b] if dts[b] == "i8" else vis[b].view(torch.float32)
        assert torch.equal(got, vr[0])
        assert torch.equal(w[b], wr[0])
        del zr, vr, wr
    plan.close()
    del x, ws, vis
    torch.cuda.empty_cache()
