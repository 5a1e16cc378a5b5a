"""GPU parity of the channeliser (afc_channelise) against the CPU oracle."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def afc():
    import paper_1609_04205_amd as afc
    return afc


def _run(afc, dev, cfg, dtype, gain=1.0, n_rows=None):
    x = W.make_voltages(cfg, device=dev, n_rows=n_rows)
    taps_np = W.prototype_taps()
    taps = torch.from_numpy(taps_np).to(dev)
    z = afc.channelise(x, taps, cfg.n_spectra, dtype, gain)
    torch.cuda.synchronize()
    return x, taps_np, z


def _natural(z, S):
    """[B][P][Sb][N][8][2] -> numpy complex [B][P][S][N] plus the pad slots."""
    zn = z.float().cpu().numpy()
    B, P, Sb, N = zn.shape[:4]
    full = zn.transpose(0, 1, 2, 4, 3, 5).reshape(B, P, Sb * 8, N, 2)
    c = full[..., 0].astype(np.float64) + 1j * full[..., 1]
    return c[:, :, :S], c[:, :, S:]


def test_f32_small_all_outputs(afc, dev):
    cfg = W.SMALL
    log("ppf f32 small: Na=48 S=1024")
    x, taps, z = _run(afc, dev, cfg, "f32")
    y, pad = _natural(z, cfg.n_spectra)
    ref = oracle.ppf_subband(x[0].cpu().numpy(), taps, 64, 16, cfg.n_spectra)      # [P][S][N]
    sigma = np.sqrt(np.mean(np.abs(ref) ** 2) / 2)
    err = np.abs(y[0] - ref).max() / sigma
    log(f"  max |dy|/sigma_y = {err:.3e}")
    assert err <= 1e-5
    assert pad.size == 0 or np.all(pad == 0)


@pytest.mark.parametrize("Na,S,B", [(5, 37, 2), (1, 1, 1), (24, 130, 1)])
def test_f32_ragged(afc, dev, Na, S, B):
    """Receivers not a multiple of the workgroup's 16, spectra not a multiple of 8 or 16."""
    cfg = W.Config("ragged", Na, B, n_spectra=S, sigma_n=500.0, source_sigmas=(100.0,), seed=7)
    log(f"ppf f32 ragged: Na={Na} S={S} B={B}")
    x, taps, z = _run(afc, dev, cfg, "f32")
    y, pad = _natural(z, S)
    xs = x.cpu().numpy()
    for b in range(B):
        ref = oracle.ppf_subband(xs[b], taps, 64, 16, S)
        sigma = np.sqrt(np.mean(np.abs(ref) ** 2) / 2)
        assert np.abs(y[b] - ref).max() / sigma <= 1e-5
    assert np.all(pad == 0)


@pytest.mark.parametrize("tap_scale", [1.0, 3.7e-4, 2.9e3])
def test_f32_full_scale_samples_and_tap_scales(afc, dev, tap_scale):
    """Samples over the whole int16 range (both bytes of every sample carry
    signal) and taps far from unit scale: the FIR's exact sample split and
    its power-of-two tap scaling keep the float32 bound."""
    rng = np.random.default_rng(11)
    Na, S = 8, 40
    N = 2 * Na
    L = (S + 15) * 64
    xs = rng.integers(-32768, 32768, size=(1, L, N, 2)).astype(np.int16)
    xs[0, :64, 0, 0] = -32768                       # extremes of the range
    xs[0, 64:128, 1, 1] = 32767
    taps = (W.prototype_taps() * tap_scale).astype(np.float32)
    log(f"ppf f32 full-scale samples, taps x {tap_scale}")
    z = afc.channelise(torch.from_numpy(xs).to(dev), torch.from_numpy(taps).to(dev), S, "f32")
    y, _ = _natural(z, S)
    ref = oracle.ppf_subband(xs[0], taps, 64, 16, S)
    sigma = np.sqrt(np.mean(np.abs(ref) ** 2) / 2)
    err = np.abs(y[0] - ref).max() / sigma
    log(f"  max |dy|/sigma_y = {err:.3e}")
    assert err <= 1e-5


def test_f16_small(afc, dev):
    cfg = W.SMALL
    log("ppf f16 small")
    x, taps, z = _run(afc, dev, cfg, "f16")
    y, _ = _natural(z, cfg.n_spectra)
    ref = oracle.ppf_subband(x[0].cpu().numpy(), taps, 64, 16, cfg.n_spectra)
    sigma = np.sqrt(np.mean(np.abs(ref) ** 2) / 2)
    # each component: fp16 rounding (half an ulp, 2^-11 relative) + float32 error
    for comp in (np.real, np.imag):
        d = np.abs(comp(y[0]) - comp(ref))
        assert np.all(d <= 2.0 ** -11 * np.abs(comp(ref)) * 1.0001 + 2e-5 * sigma)


def test_i8_requant_small(afc, dev):
    cfg = W.SMALL
    taps = W.prototype_taps()
    gain = W.requant_gain(cfg, taps)
    log(f"ppf i8 small gain={gain}")
    x = W.make_voltages(cfg, device=dev)
    tt = torch.from_numpy(taps).to(dev)
    z8 = afc.channelise(x, tt, cfg.n_spectra, "i8", gain)
    z32 = afc.channelise(x, tt, cfg.n_spectra, "f32")
    torch.cuda.synchronize()
    q = z8.cpu().numpy()
    y32 = z32.cpu().numpy()
    # property: the int8 output is the requantised float32 output of the same
    # kernel (the exact product, exact in float64, rounded once)
    ref_q = np.clip(np.rint(y32.astype(np.float64) * np.float64(np.float32(gain))), -127, 127).astype(np.int8)
    np.testing.assert_array_equal(q, ref_q)
    assert q.min() >= -127
    # against the float64 oracle: at most one step, and only next to a rounding boundary
    yq, _ = _natural(z8.float(), cfg.n_spectra)
    ref = oracle.ppf_subband(x[0].cpu().numpy(), taps, 64, 16, cfg.n_spectra)
    for comp in (np.real, np.imag):
        v = comp(ref) * gain
        r = np.clip(np.rint(v), -127, 127)
        d = np.abs(comp(yq[0]) - r)
        assert d.max() <= 1
        near = np.abs(np.abs(v - np.floor(v)) - 0.5)
        sigma = np.sqrt(np.mean(np.abs(ref) ** 2) / 2)
        assert np.all(near[d == 1] <= 1e-5 * sigma * gain)
        log(f"  off-by-one fraction {np.mean(d == 1):.2e}")


def test_i8_requant_rounds_the_exact_product_once(afc, dev):
    """A single unit tap (branch 0, tap 0) makes every channel of spectrum s
    equal to the sample x[64 s] exactly; with gain fp32(1/6) the product
    15 * gain = 2.50000007... rounds to 3 when rounded once, but a float32
    product rounds to 2.5 first and then to 2 (ties to even).  Also the
    clamp at +-127 and the zero pad slots."""
    Na, S = 8, 24
    N = 2 * Na
    L = (S + 15) * 64
    xs = np.zeros((1, L, N, 2), np.int16)
    xs[0, ::64, :, 0] = 15
    xs[0, ::64, :, 1] = -15
    xs[0, 64 * 5, 3, 0] = 32767                     # spectrum 5, receiver 3: clamps
    taps = np.zeros(64 * 16, np.float32)
    taps[0] = 1.0
    gain = float(np.float32(1.0 / 6.0))
    assert np.rint(np.float32(15) * np.float32(gain)) == 2.0          # the float32 product's rounding
    z8 = afc.channelise(torch.from_numpy(xs).to(dev), torch.from_numpy(taps).to(dev), S, "i8", gain)
    q, pad = _natural(z8.float(), S)
    q = q[0]
    assert np.all(pad == 0)
    expect = np.full(q.shape, 3 - 3j)
    expect[:, 5, 3] = 127 - 3j
    np.testing.assert_array_equal(q, expect)


def test_f32_full_size_sampled(afc, dev):
    """AARTFAAC-12 shape (1152 receivers, 16 subbands, 3051 spectra): sampled receivers."""
    cfg = W.A12
    log("ppf f32 AARTFAAC-12 full size")
    x, taps, z = _run(afc, dev, cfg, "f32")
    rng = np.random.default_rng(0)
    for sb in (0, 7, 15):
        inputs = sorted(rng.choice(cfg.n_inputs, size=3, replace=False).tolist()) + [cfg.n_inputs - 1]
        xs = x[sb].cpu().numpy()
        ref = oracle.ppf_subband(xs, taps, 64, 16, cfg.n_spectra, inputs=inputs)
        zz = z[sb].index_select(2, torch.tensor(inputs, device=dev))          # [P][Sb][R][8][2]
        got = zz.permute(0, 1, 3, 2, 4).reshape(64, -1, len(inputs), 2)[:, :cfg.n_spectra].cpu().numpy()
        got = got[..., 0].astype(np.float64) + 1j * got[..., 1]
        sigma = np.sqrt(np.mean(np.abs(ref) ** 2) / 2)
        err = np.abs(got - ref).max() / sigma
        log(f"  sb={sb} inputs={inputs} max err {err:.3e}")
        assert err <= 1e-5
    del x, z
    torch.cuda.empty_cache()


@pytest.mark.parametrize("dtype", ["f32", "f16"])
def test_output_above_2gib_per_subband(afc, dev, dtype):
    """1152 antennas (2304 receivers), 3051 spectra: one subband's fp32 output
    is 3.6 GB and fp16 1.8 GB.  Above 2^31 bytes the channeliser stores
    through one buffer descriptor per channel instead of one per subband
    (fp32 here); sampled receivers, every channel, against the oracle."""
    cfg = W.Config("a24-1sb", 1152, 1, n_spectra=3051, sigma_n=32.0)
    log(f"ppf {dtype} 2304 receivers, output {64 * 382 * 2304 * 8 * (8 if dtype == 'f32' else 4) / 1e9:.2f} GB")
    x, taps, z = _run(afc, dev, cfg, dtype)
    inputs = [0, 777, 1500, cfg.n_inputs - 1]
    ref = oracle.ppf_subband(x[0].cpu().numpy(), taps, 64, 16, cfg.n_spectra, inputs=inputs)
    zz = z[0].index_select(2, torch.tensor(inputs, device=dev))
    got = zz.permute(0, 1, 3, 2, 4).reshape(64, -1, len(inputs), 2)[:, :cfg.n_spectra].float().cpu().numpy()
    got = got[..., 0].astype(np.float64) + 1j * got[..., 1]
    sigma = np.sqrt(np.mean(np.abs(ref) ** 2) / 2)
    err = np.abs(got - ref).max() / sigma
    log(f"  max err {err:.3e}")
    if dtype == "f32":
        assert err <= 1e-5
    else:
        # each component: fp16 rounding (2^-11 relative) + float32 error
        for comp in (np.real, np.imag):
            d = np.abs(comp(got) - comp(ref))
            assert np.all(d <= 2.0 ** -11 * np.abs(comp(ref)) * 1.0001 + 2e-5 * sigma)
    del x, z
    torch.cuda.empty_cache()
