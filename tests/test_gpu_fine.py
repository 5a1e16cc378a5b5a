"""GPU parity of the fine channeliser (afc_channelise_fine: 256-channel bank,
delay and bandpass compensation, 4:1 channel integration) against the CPU
oracle, plus the delayed-tone property and the chain into the correlator.
FP32 <= 1e-5 of the per-component output sigma; fp16 and int8 follow the
rounding rules of the 64-channel bank's tests."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import log, normalised_error, vis_to_complex

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

PF, T, R = 256, 16, 4
DF = W.F_SUBBAND / PF


@pytest.fixture(scope="module")
def afc():
    import paper_1609_04205_amd as afc
    return afc


def _inputs(dev, Na, B, S, seed, sigma_n=500.0, source_sigma=100.0):
    cfg = W.Config("fine", Na, B, n_spectra=S, sigma_n=sigma_n, source_sigmas=(source_sigma,), seed=seed)
    x = W.make_voltages(cfg, device=dev, n_rows=W.fine_rows(S))
    taps = W.prototype_taps(PF, T)
    tau = W.cable_delays(2 * Na, seed=seed)
    w = W.bandpass_weights(PF, seed=seed)
    nu = [W.subband_frequency(b) for b in range(B)]
    return cfg, x, taps, tau, w, nu


def _run(afc, dev, x, taps, tau, w, nu, S, dtype, gain=1.0):
    z = afc.channelise_fine(x, torch.from_numpy(taps).to(dev), S, torch.from_numpy(tau).to(dev),
                            torch.from_numpy(w).to(dev), nu, W.F_SUBBAND, dtype, gain)
    torch.cuda.synchronize()
    return z


def _natural(z, S):
    """[B][64][Sb][N][8][2] -> numpy complex [B][64][S][N] plus the pad slots."""
    zn = z.float().cpu().numpy()
    B, P, Sb, N = zn.shape[:4]
    full = zn.transpose(0, 1, 2, 4, 3, 5).reshape(B, P, Sb * 8, N, 2)
    c = full[..., 0].astype(np.float64) + 1j * full[..., 1]
    return c[:, :, :S], c[:, :, S:]


def _oracle(x_np, taps, tau, w, nu_b, S, inputs=None):
    return oracle.fine_subband(x_np, taps, PF, T, S, tau, nu_b, DF, w, R, inputs=inputs)   # [64][S][R']


def test_f32_small_all_outputs(afc, dev):
    """96 receivers, 200 spectra: two spectrum chunks and a ragged last phase."""
    S = 200
    cfg, x, taps, tau, w, nu = _inputs(dev, 48, 1, S, seed=21)
    log(f"fine f32 Na=48 S={S}")
    z = _run(afc, dev, x, taps, tau, w, nu, S, "f32")
    y, pad = _natural(z, S)
    ref = _oracle(x[0].cpu().numpy(), taps, tau, w, nu[0], S)
    sigma = np.sqrt(np.mean(np.abs(ref) ** 2) / 2)
    err = np.abs(y[0] - ref).max() / sigma
    log(f"  max |dz|/sigma_z = {err:.3e}")
    assert err <= 1e-5
    assert pad.size == 0 or np.all(pad == 0)


@pytest.mark.parametrize("Na,S,B", [(5, 37, 2), (1, 1, 1), (3, 17, 3)])
def test_f32_ragged(afc, dev, Na, S, B):
    """Receivers not a multiple of the workgroup's 4, spectra not a multiple of 8 or 16."""
    cfg, x, taps, tau, w, nu = _inputs(dev, Na, B, S, seed=7 + Na)
    log(f"fine f32 ragged: Na={Na} S={S} B={B}")
    z = _run(afc, dev, x, taps, tau, w, nu, S, "f32")
    y, pad = _natural(z, S)
    xs = x.cpu().numpy()
    for b in range(B):
        ref = _oracle(xs[b], taps, tau, w, nu[b], S)
        sigma = np.sqrt(np.mean(np.abs(ref) ** 2) / 2)
        assert np.abs(y[b] - ref).max() / sigma <= 1e-5
    assert np.all(pad == 0)


def test_f16(afc, dev):
    S = 64
    # the bank's gain is about 20 in amplitude: input sigmas of 32 and 16 keep
    # every output far inside the fp16 range (the AARTFAAC-12 workload uses 32)
    cfg, x, taps, tau, w, nu = _inputs(dev, 16, 1, S, seed=31, sigma_n=32.0, source_sigma=16.0)
    log("fine f16")
    z = _run(afc, dev, x, taps, tau, w, nu, S, "f16")
    y, _ = _natural(z, S)
    ref = _oracle(x[0].cpu().numpy(), taps, tau, w, nu[0], S)
    sigma = np.sqrt(np.mean(np.abs(ref) ** 2) / 2)
    for comp in (np.real, np.imag):
        d = np.abs(comp(y[0]) - comp(ref))
        assert np.all(d <= 2.0 ** -11 * np.abs(comp(ref)) * 1.0001 + 2e-5 * sigma)


def test_i8_requant(afc, dev):
    S = 64
    cfg, x, taps, tau, w, nu = _inputs(dev, 16, 1, S, seed=41)
    z32 = _run(afc, dev, x, taps, tau, w, nu, S, "f32")
    ref = _oracle(x[0].cpu().numpy(), taps, tau, w, nu[0], S)
    sigma = np.sqrt(np.mean(np.abs(ref) ** 2) / 2)
    gain = float(np.float32(127.0 / (4.0 * sigma)))
    log(f"fine i8 gain={gain}")
    z8 = _run(afc, dev, x, taps, tau, w, nu, S, "i8", gain)
    q = z8.cpu().numpy()
    y32 = z32.cpu().numpy()
    # the int8 output is the requantised float32 output of the same kernel
    # (the exact product, exact in float64, rounded once)
    ref_q = np.clip(np.rint(y32.astype(np.float64) * np.float64(np.float32(gain))), -127, 127).astype(np.int8)
    np.testing.assert_array_equal(q, ref_q)
    # against the float64 oracle: at most one step, only next to a rounding boundary
    yq, _ = _natural(z8.float(), S)
    for comp in (np.real, np.imag):
        v = comp(ref) * gain
        r = np.clip(np.rint(v), -127, 127)
        d = np.abs(comp(yq[0]) - r)
        assert d.max() <= 1
        near = np.abs(np.abs(v - np.floor(v)) - 0.5)
        assert np.all(near[d == 1] <= 1e-5 * sigma * gain)


def test_delayed_tones_are_realigned(afc, dev):
    """Tones at fine-channel centres, received with per-receiver delays tau_i
    (baseband phase exp(-2 pi i (nu + f_k) tau_i) per tone): after the
    compensation every receiver carries the same channelised signal."""
    Na, S = 6, 48
    N = 2 * Na
    nu = W.subband_frequency(3)
    tau = W.cable_delays(N, seed=12)
    n = np.arange(W.fine_rows(S))
    rng = np.random.default_rng(13)
    ks = [3, 40, 131, 200, 255]
    amp = rng.uniform(800, 2000, len(ks)) * np.exp(2j * np.pi * rng.random(len(ks)))
    x = np.zeros((1, n.size, N, 2), np.int16)
    for i in range(N):
        sig = np.zeros(n.size, np.complex128)
        for a, k in zip(amp, ks):
            fk = (k if k < PF // 2 else k - PF) * DF
            sig += a * np.exp(2j * np.pi * fk * n / W.F_SUBBAND) * np.exp(-2j * np.pi * (nu + fk) * tau[i])
        x[0, :, i, 0] = np.rint(sig.real)
        x[0, :, i, 1] = np.rint(sig.imag)
    taps = W.prototype_taps(PF, T)
    w = np.ones(PF, np.float32)
    z = _run(afc, dev, torch.from_numpy(x).to(dev), taps, tau, w, [nu], S, "f32")
    y, _ = _natural(z, S)
    y = y[0]                                              # [64][S][N]
    peak = np.abs(y).max()
    spread = np.abs(y - y[:, :, :1]).max() / peak
    log(f"  max |z_i - z_0| / peak = {spread:.2e}")
    # int16 rounding of the inputs (|e| <= 0.5 per component) is the only difference
    assert spread < 1e-3
    for k in ks:
        assert np.abs(y[k // R]).min() > 0.1 * peak


def test_chain_into_correlator(afc, dev):
    """The fine output feeds afc_correlate as is: visibilities against the
    oracle's float64 fine channeliser and float64 correlator."""
    S = 96
    cfg, x, taps, tau, w, nu = _inputs(dev, 24, 1, S, seed=51)
    z = _run(afc, dev, x, taps, tau, w, nu, S, "f32")
    vis, wts = afc.correlate(z, n_spectra=S)
    v = vis_to_complex(vis.cpu().numpy())[0]
    ref = _oracle(x[0].cpu().numpy(), taps, tau, w, nu[0], S)
    worst = 0.0
    for ch in (0, 1, 17, 32, 63):
        Vref, _ = oracle.xcorr(ref[ch])
        worst = max(worst, float(normalised_error(v[ch], Vref, 24).max()))
    log(f"  fine chain max normalised error {worst:.3e}")
    assert worst <= 1e-5
    assert np.all(wts.cpu().numpy() == S)


def test_f32_full_size_sampled(afc, dev):
    """AARTFAAC-12 shape, 1 s of 256-sample spectra (1152 receivers, 16
    subbands, 762 spectra): sampled receivers of three subbands."""
    Na, B, S = 576, 16, 762
    cfg = W.A12
    log("fine f32 full size")
    x = W.make_voltages(cfg, device=dev, n_rows=W.fine_rows(S))
    taps = W.prototype_taps(PF, T)
    tau = W.cable_delays(2 * Na)
    w = W.bandpass_weights(PF)
    nu = [W.subband_frequency(b) for b in range(B)]
    z = _run(afc, dev, x, taps, tau, w, nu, S, "f32")
    rng = np.random.default_rng(0)
    for sb in (0, 7, 15):
        inputs = sorted(rng.choice(2 * Na, size=3, replace=False).tolist()) + [2 * Na - 1]
        ref = _oracle(x[sb].cpu().numpy(), taps, tau, w, nu[sb], S, inputs=inputs)
        zz = z[sb].index_select(2, torch.tensor(inputs, device=dev))          # [64][Sb][R][8][2]
        got = zz.permute(0, 1, 3, 2, 4).reshape(64, -1, len(inputs), 2)[:, :S].cpu().numpy()
        got = got[..., 0].astype(np.float64) + 1j * got[..., 1]
        sigma = np.sqrt(np.mean(np.abs(ref) ** 2) / 2)
        err = np.abs(got - ref).max() / sigma
        log(f"  sb={sb} inputs={inputs} max err {err:.3e}")
        assert err <= 1e-5
    del x, z
    torch.cuda.empty_cache()


def test_run_length_does_not_change_results(afc, dev):
    """The host picks the spectra per workgroup from the launch size: the
    16-subband AARTFAAC-12 launch runs 768 spectra per workgroup, a launch of
    one of its subbands shorter runs (more workgroups for the CUs).  Each
    output's FIR is the same 16 products in the same order wherever a run
    starts, so the subband's fp32 and int8 outputs are identical bit for bit."""
    Na, B, S = 576, 16, 762
    log("fine run lengths: 16 subbands against single subbands")
    x = W.make_voltages(W.A12, device=dev, n_rows=W.fine_rows(S))
    taps = W.prototype_taps(PF, T)
    tau = W.cable_delays(2 * Na)
    w = W.bandpass_weights(PF)
    nu = [W.subband_frequency(b) for b in range(B)]
    for dtype, gain in (("f32", 1.0), ("i8", 0.05)):
        z = _run(afc, dev, x, taps, tau, w, nu, S, dtype, gain)
        for sb in (0, 15):
            z1 = _run(afc, dev, x[sb:sb + 1].contiguous(), taps, tau, w, [nu[sb]], S, dtype, gain)
            assert torch.equal(z1[0].view(torch.int8), z[sb].view(torch.int8)), (dtype, sb)
        del z, z1
    del x
    torch.cuda.empty_cache()
