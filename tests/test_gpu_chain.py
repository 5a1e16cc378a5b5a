"""End-to-end parity of the hot path: channeliser -> correlator, against the
oracle's float64 channeliser -> float64 correlator on the same int16 input.
FP32 chain <= 1e-5 and FP16 chain <= 2e-3 per baseline, normalised by
sqrt(V_ii V_jj); the int8 chain is reported against its quantisation level.
"""
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


@pytest.fixture(scope="module")
def small_case(dev):
    cfg = W.SMALL
    x = W.make_voltages(cfg, device=dev)
    taps = W.prototype_taps()
    y = oracle.ppf_subband(x[0].cpu().numpy(), taps, 64, 16, cfg.n_spectra)       # [P][S][N]
    return cfg, x, taps, y


@pytest.mark.parametrize("dtype,tol", [("f32", 1e-5), ("f16", 2e-3)])
def test_chain_small(afc, dev, small_case, dtype, tol):
    cfg, x, taps, y = small_case
    log(f"chain {dtype} small_case")
    z = afc.channelise(x, torch.from_numpy(taps).to(dev), cfg.n_spectra, dtype)
    vis, w = afc.correlate(z, n_spectra=cfg.n_spectra)
    v = vis_to_complex(vis.cpu().numpy())[0]
    worst = 0.0
    for ch in range(64):
        Vref, _ = oracle.xcorr(y[ch])
        e = normalised_error(v[ch], Vref, cfg.n_antennas)
        worst = max(worst, float(e.max()))
    log(f"  max normalised error {worst:.3e}")
    assert worst <= tol
    assert np.all(w.cpu().numpy() == cfg.n_spectra)


def test_chain_i8_small_closeness(afc, dev, small_case):
    """int8 chain: the visibility of the requantised samples, scaled back by 1/gain^2,
    stays within the quantisation noise of the float64 chain."""
    cfg, x, taps, y = small_case
    gain = W.requant_gain(cfg, taps)
    z = afc.channelise(x, torch.from_numpy(taps).to(dev), cfg.n_spectra, "i8", gain)
    vis, _ = afc.correlate(z, n_spectra=cfg.n_spectra)
    v = vis_to_complex(vis.cpu().numpy())[0] / gain ** 2
    Vref, _ = oracle.xcorr(y[5])
    e = normalised_error(v[5], Vref, cfg.n_antennas)
    # uniform quantisation noise of step 1/gain against sigma_y = 127/(4 gain): about 1e-2
    log(f"  int8 chain max normalised deviation {e.max():.3e}")
    assert e.max() < 0.05


def test_chain_plane_wave(afc, dev):
    """Noise-free plane wave at the centre of channel 0: V_ab = S |A|^2 (sum h)^2 e^{i(phi_a - phi_b)}."""
    Na, S = 8, 256
    cfg = W.Config("tone", Na, 1, n_spectra=S)
    L = cfg.n_rows
    rng = np.random.default_rng(4)
    phi = rng.uniform(0, 2 * np.pi, 2 * Na)
    A = 1000.0
    # a constant (DC) signal per receiver, integer-valued so int16 holds it exactly
    amp = np.round(A * np.exp(1j * phi))
    x = np.zeros((1, L, Na, 2, 2), np.int16)
    x[0, :, :, :, 0] = amp.real.reshape(Na, 2)
    x[0, :, :, :, 1] = amp.imag.reshape(Na, 2)
    taps = W.prototype_taps()
    xt = torch.from_numpy(x).to(dev)
    z = afc.channelise(xt, torch.from_numpy(taps).to(dev), S, "f32")
    vis, _ = afc.correlate(z, n_spectra=S)
    v = vis_to_complex(vis.cpu().numpy())[0, 0]
    hs = float(np.sum(taps.astype(np.float64)))
    a_, b_ = np.tril_indices(Na)
    for p in range(2):
        for q in range(2):
            ref = S * hs * hs * amp[2 * a_ + p] * np.conj(amp[2 * b_ + q])
            assert np.allclose(v[:, p, q], ref, rtol=2e-6, atol=2e-6 * np.abs(ref).max())


@pytest.mark.parametrize("cfg,dtype,tol", [(W.A6, "f32", 1e-5), (W.A12, "f16", 2e-3), (W.A12, "f32", 1e-5)],
                         ids=["a6-f32", "a12-f16", "a12-f32"])
def test_chain_full_size_sampled(afc, dev, cfg, dtype, tol):
    """Full shape (AARTFAAC-6: 576 receivers, 8 subbands; AARTFAAC-12: 1152
    receivers, 16 subbands; 3051 spectra), the chain in fp32 or fp16 against
    the FP64 chain on sampled antennas, normalised by sqrt(V_ii V_jj).  The
    max and RMS error are logged."""
    log(f"chain {dtype} {cfg.name} full size")
    x = W.make_voltages(cfg, device=dev)
    taps = W.prototype_taps()
    z = afc.channelise(x, torch.from_numpy(taps).to(dev), cfg.n_spectra, dtype)
    vis, _ = afc.correlate(z, n_spectra=cfg.n_spectra)
    torch.cuda.synchronize()
    del z
    rng = np.random.default_rng(2)
    errs = []
    for sb in (0, cfg.n_subbands - 1):
        ants = sorted(set(rng.choice(cfg.n_antennas, size=5, replace=False).tolist() + [cfg.n_antennas - 1]))
        inputs = [2 * a + p for a in ants for p in range(2)]
        y = oracle.ppf_subband(x[sb].cpu().numpy(), taps, 64, 16, cfg.n_spectra, inputs=inputs)  # [P][S][R]
        bls = [a * (a + 1) // 2 + b for ia, a in enumerate(ants) for b in ants[: ia + 1]]
        got = vis_to_complex(vis[sb][:, torch.as_tensor(bls, device=dev)].cpu().numpy())    # [P][n][2][2]
        pos = {i: k for k, i in enumerate(inputs)}
        pairs, slots = [], []
        for ia, a in enumerate(ants):
            for b in ants[: ia + 1]:
                for p in range(2):
                    for q in range(2):
                        pairs.append((pos[2 * a + p], pos[2 * b + q]))
                        slots.append((len(slots) // 4, p, q))
        pairs = np.array(pairs)
        autos = np.array([[k, k] for k in range(len(inputs))])
        for ch in range(0, 64, 3):
            ref = oracle.xcorr_pairs(y[ch], pairs)
            pw = oracle.xcorr_pairs(y[ch], autos).real
            den = np.sqrt(pw[pairs[:, 0]] * pw[pairs[:, 1]])
            g = np.array([got[ch, k, p, q] for (k, p, q) in slots])
            errs.append(np.abs(g - ref) / den)
    e = np.concatenate(errs)
    log(f"  max normalised error {e.max():.3e}, rms {np.sqrt(np.mean(e * e)):.3e} over {e.size} visibilities")
    assert e.max() <= tol
    del x, vis
    torch.cuda.empty_cache()
