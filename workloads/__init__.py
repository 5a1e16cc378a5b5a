"""Seeded synthetic inputs for the FX-correlator hot path.

This module is shared by the tests, the benchmark and the oracle checks.  It
only *draws* inputs: antenna layouts, complex int16 subband voltages with
injected plane-wave point sources, prototype-filter coefficients, int8/fp16/
fp32 channelised samples, gains and model visibilities.  It holds none of the
channeliser or correlator arithmetic; both the HIP path and the CPU oracle
receive the arrays produced here.

Shapes follow the paper's arrays: 48 dual-polarised antennas per station
(Sec. "LOFAR Telescope Architecture"), 6 or 12 stations (AARTFAAC-6 / -12,
Table 1), 195312.5 Hz subbands of complex 16-bit samples (Sec. "LOFAR Digital
Processing"), 3 kHz channels and 1 s integrations (Table 1).  The real
observations are not available, so everything here is synthetic: seeded
Gaussian noise per input plus point sources with known geometric phases.

Array layouts (all C order):
  x   int16  [B][L][Na][2][2]   time-major subband samples, inputs i = 2a+p
                                contiguous, re/im interleaved; L = (S+T-1)*P
  z   dtype  [B][P][Sb][N][8][2] channelised samples in spectrum blocks of 8
                                (Sb = ceil(S/8)); spectra >= S are zero
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

F_SUBBAND = 195312.5          # Hz, subband width (= sample rate per subband)
C_LIGHT = 299792458.0         # m/s
NU0 = 60.0e6                  # Hz, centre of the first subband
SPECTRUM_BLOCK = 8            # spectra per block in the channelised layout


# --------------------------------------------------------------------------
# configurations
# --------------------------------------------------------------------------
@dataclass
class Config:
    name: str
    n_antennas: int
    n_subbands: int
    n_channels: int = 64
    n_taps: int = 16
    n_spectra: int = 3051
    sigma_n: float = 32.0
    source_sigmas: Sequence[float] = ()
    n_sources: int = 0            # drawn log-uniform in [4, 16] when > 0
    layout: str = "disc"          # "disc" | "stations6" | "stations12"
    seed: int = 1
    # batching form
    ragged: bool = False          # per-subband S drawn from U{500..n_spectra}
    flag_max: float = 0.0         # per-subband flagged fraction ~ U[0, flag_max]
    mixed_dtype: bool = False     # per-subband dtype ~ Bernoulli(1/2) fp16 / int8

    @property
    def n_inputs(self) -> int:
        return 2 * self.n_antennas

    @property
    def n_rows(self) -> int:
        return (self.n_spectra + self.n_taps - 1) * self.n_channels


# small: 48 antennas in a 30 m disc, 1 subband, 1024 spectra
SMALL = Config("small-48ant", 48, 1, n_spectra=1024, sigma_n=64.0,
               source_sigmas=(16.0,), layout="disc", seed=1)
# AARTFAAC-6 shape: 6 stations x 48 antennas, 8 subbands, 1 s
A6 = Config("a6-288ant-8sb", 288, 8, n_spectra=3051, sigma_n=32.0,
            n_sources=3, layout="stations6", seed=2)
# AARTFAAC-12 shape: 12 stations x 48 antennas, 16 subbands, 1 s
A12 = Config("a12-576ant-16sb", 576, 16, n_spectra=3051, sigma_n=32.0,
             n_sources=3, layout="stations12", seed=3)
# batching: 32 subbands, ragged integration, flags, mixed fp16/int8
A12_BATCHED = Config("a12-576ant-32sb-batched", 576, 32, n_spectra=3051, sigma_n=32.0,
                     n_sources=3, layout="stations12", seed=4,
                     ragged=True, flag_max=0.10, mixed_dtype=True)


# --------------------------------------------------------------------------
# prototype filter: an INPUT of the channeliser (the paper gives none)
# --------------------------------------------------------------------------
def prototype_taps(n_channels: int = 64, n_taps: int = 16) -> np.ndarray:
    """Hann-windowed sinc prototype, length M = P*T, rounded to float32.

    h[m] = w[m] * sinc((m - (M-1)/2) / P), w[m] = 0.5 - 0.5 cos(2 pi m/(M-1)).
    The paper names a 16-tap polyphase filter bank but prints no
    coefficients, so the taps are a workload input; the channeliser is
    defined for any h.  Returned as float32 in the order h[t*P + p].
    """
    M = n_channels * n_taps
    m = np.arange(M, dtype=np.float64)
    w = 0.5 - 0.5 * np.cos(2.0 * np.pi * m / (M - 1))
    arg = (m - (M - 1) / 2.0) / n_channels
    h = w * np.sin(np.pi * arg) / (np.pi * arg)
    return h.astype(np.float32)


def requant_gain(cfg: Config, taps: np.ndarray, clip_sigmas: float = 4.0) -> float:
    """Gain that maps the channelised per-component sigma to 127/clip_sigmas.

    sigma_y = sigma_in * sqrt(sum h^2), with sigma_in the per-component input
    sigma (noise and sources added in power).  Analytic, from the generator
    parameters, so it does not depend on the data.
    """
    s2 = cfg.sigma_n ** 2 + sum(s * s for s in source_sigmas(cfg))
    sigma_y = math.sqrt(s2) * math.sqrt(float(np.sum(taps.astype(np.float64) ** 2)))
    return float(np.float32(127.0 / (clip_sigmas * sigma_y)))


# --------------------------------------------------------------------------
# inputs of the fine channeliser: cable delays and bandpass weights
# --------------------------------------------------------------------------
N_FINE = 256                  # channels of the paper's filter bank
FINE_RATIO = 4                # fine channels per output channel


def fine_rows(n_spectra: int, n_taps: int = 16) -> int:
    """Input rows of the fine channeliser for n_spectra 256-sample spectra."""
    return (n_spectra + n_taps - 1) * N_FINE


def cable_delays(n_inputs: int, seed: int = 5, max_delay: float = 6.0e-7) -> np.ndarray:
    """Per-receiver fixed cable delays in seconds, float64 [N].

    The paper reads them from calibration tables it does not print; a
    dual-polarised antenna's two receivers share one cable run, so both get
    the antenna's delay U[0, max_delay] plus an independent 0..2 ns offset
    (0.6 us is about 120 m of coax).
    """
    rng = np.random.default_rng([seed, 606])
    Na = n_inputs // 2
    base = rng.uniform(0.0, max_delay, size=Na)
    return (np.repeat(base, 2) + rng.uniform(0.0, 2.0e-9, size=2 * Na)).astype(np.float64)


def bandpass_weights(n_fine: int = N_FINE, seed: int = 6) -> np.ndarray:
    """Real positive weights per fine channel (natural FFT order), float32.

    Stand-in for the correction of the first-stage filter bank's ripple
    across a subband, which the paper applies from fixed tables it does not
    print: the inverse of a smooth response that falls by about 30 % towards
    the subband edges, with a 2 % ripple.
    """
    rng = np.random.default_rng([seed, 707])
    k = np.arange(n_fine)
    f = np.where(k < n_fine // 2, k, k - n_fine) / n_fine          # -0.5 .. 0.5
    ph = rng.uniform(0.0, 2.0 * np.pi)
    resp = (1.0 - 1.2 * f * f) * (1.0 + 0.02 * np.cos(2.0 * np.pi * 7.0 * f + ph))
    return (1.0 / resp).astype(np.float32)


def fine_requant_gain(cfg: Config, taps: np.ndarray, w: np.ndarray, ratio: int = FINE_RATIO,
                      clip_sigmas: float = 4.0) -> float:
    """Gain that maps the fine channeliser's per-component output sigma, in
    its loudest output channel, to 127/clip_sigmas.

    A fine channel of white input has sigma_in * sqrt(sum h^2) per component;
    an output channel sums `ratio` of them, weighted by w (the delay phases
    leave the power unchanged), so its variance carries sum_j w[4c+j]^2.
    Analytic, from the generator parameters.
    """
    s2 = cfg.sigma_n ** 2 + sum(s * s for s in source_sigmas(cfg))
    w2 = (w.astype(np.float64) ** 2).reshape(-1, ratio).sum(1).max()
    sigma_z = math.sqrt(s2) * math.sqrt(float(np.sum(taps.astype(np.float64) ** 2))) * math.sqrt(w2)
    return float(np.float32(127.0 / (clip_sigmas * sigma_z)))


# --------------------------------------------------------------------------
# lost packets (per station, per subband)
# --------------------------------------------------------------------------
PACKET_SAMPLES = 16           # time samples per station packet
ANTENNAS_PER_STATION = 48


def packet_loss(n_subbands: int, n_antennas: int, n_rows: int, seed: int, rate: float = 1e-3,
                mean_burst: float = 8.0, dead: Sequence[tuple] = (),
                packet_samples: int = PACKET_SAMPLES) -> np.ndarray:
    """Packet arrival flags uint8 [B][n_packets][Na] (1 = arrived).

    A station's packets carry all of its 48 antennas, so loss is drawn per
    (subband, station): bursts of lost packets starting with probability
    `rate / mean_burst` per packet, lengths geometric with mean
    `mean_burst` (about `rate` of the packets lost); `dead` lists
    (subband, station) pairs whose packets are all lost.
    """
    rng = np.random.default_rng([seed, 808])
    n_pk = -(-n_rows // packet_samples)
    n_st = -(-n_antennas // ANTENNAS_PER_STATION)
    ok = np.ones((n_subbands, n_pk, n_st), np.uint8)
    p_start = rate / mean_burst
    for b in range(n_subbands):
        for st in range(n_st):
            starts = np.flatnonzero(rng.random(n_pk) < p_start)
            lens = rng.geometric(1.0 / mean_burst, size=starts.size)
            for s0, ln in zip(starts, lens):
                ok[b, s0:s0 + ln, st] = 0
    for b, st in dead:
        ok[b, :, st] = 0
    ant_station = np.arange(n_antennas) // ANTENNAS_PER_STATION
    return np.ascontiguousarray(ok[:, :, ant_station])


# --------------------------------------------------------------------------
# array geometry and sky
# --------------------------------------------------------------------------
def _disc(rng: np.random.Generator, n: int, radius: float) -> np.ndarray:
    r = radius * np.sqrt(rng.random(n))
    phi = 2.0 * np.pi * rng.random(n)
    return np.stack([r * np.cos(phi), r * np.sin(phi)], axis=1)


def antenna_positions(cfg: Config) -> np.ndarray:
    """[Na][2] east/north positions in metres (seeded)."""
    rng = np.random.default_rng([cfg.seed, 101])
    if cfg.layout == "disc":
        return _disc(rng, cfg.n_antennas, 30.0)
    n_st = {"stations6": 6, "stations12": 12}[cfg.layout]
    counts = [cfg.n_antennas // n_st + (1 if k < cfg.n_antennas % n_st else 0) for k in range(n_st)]
    centres = []
    for k in range(n_st):
        ring = 150.0 if k < 6 else 588.0
        ang = 2.0 * np.pi * (k % 6) / 6.0 + (0.0 if k < 6 else np.pi / 6.0)
        centres.append((ring * np.cos(ang), ring * np.sin(ang)))
    pos = [np.asarray(c)[None, :] + _disc(rng, n, 30.0) for c, n in zip(centres, counts)]
    return np.concatenate(pos, axis=0)


def source_sigmas(cfg: Config) -> List[float]:
    if cfg.source_sigmas:
        return list(cfg.source_sigmas)
    rng = np.random.default_rng([cfg.seed, 202])
    return list(np.exp(rng.uniform(np.log(4.0), np.log(16.0), cfg.n_sources)))


def source_directions(cfg: Config, n: Optional[int] = None) -> np.ndarray:
    """[n][2] direction cosines (l, m), uniform in the unit disc (seeded)."""
    rng = np.random.default_rng([cfg.seed, 303])
    n = len(source_sigmas(cfg)) if n is None else n
    return _disc(rng, n, 1.0)


def subband_frequency(sb: int) -> float:
    return NU0 + sb * F_SUBBAND


def geometric_phases(pos: np.ndarray, lm: np.ndarray, nu: float) -> np.ndarray:
    """[n_src][Na] complex exp(+2 pi i nu (l x + m y) / c)."""
    d = lm[:, 0:1] * pos[None, :, 0] + lm[:, 1:2] * pos[None, :, 1]
    return np.exp(2j * np.pi * nu * d / C_LIGHT)


# --------------------------------------------------------------------------
# per-subband parameters of the batching form
# --------------------------------------------------------------------------
@dataclass
class BatchParams:
    n_spectra: np.ndarray        # int32 [B]
    flags: np.ndarray            # uint8 [B][Na]
    dtypes: np.ndarray           # int32 [B]  1 = fp16, 2 = int8


def batch_params(cfg: Config) -> BatchParams:
    B, Na = cfg.n_subbands, cfg.n_antennas
    rng = np.random.default_rng([cfg.seed, 404])
    if cfg.ragged:
        S = rng.integers(500, cfg.n_spectra + 1, size=B).astype(np.int32)
    else:
        S = np.full(B, cfg.n_spectra, np.int32)
    flags = np.zeros((B, Na), np.uint8)
    if cfg.flag_max > 0:
        for b in range(B):
            f = rng.uniform(0.0, cfg.flag_max)
            k = int(round(f * Na))
            flags[b, rng.choice(Na, size=k, replace=False)] = 1
    if cfg.mixed_dtype:
        dt = np.where(rng.random(B) < 0.5, 1, 2).astype(np.int32)
    else:
        dt = np.full(B, 0, np.int32)
    return BatchParams(S, flags, dt)


# --------------------------------------------------------------------------
# int16 subband voltages
# --------------------------------------------------------------------------
def make_voltages(cfg: Config, device="cpu", subbands: Optional[Sequence[int]] = None,
                  n_rows: Optional[int] = None):
    """Complex int16 voltages, torch tensor [B'][L][Na][2][2] on `device`.

    Each component is round(N(0, sigma_n^2) + sources), clipped to int16.
    A source is a complex Gaussian signal per polarisation (unpolarised:
    X and Y independent) with per-component sigma sigma_s, arriving at
    antenna a with phase exp(+2 pi i nu (l x_a + m y_a)/c), nu the subband
    centre.  Uses torch's generator on `device`: the values on a GPU differ
    from those on the CPU for the same seed, so every consumer takes the
    array itself, never a regeneration.
    """
    import torch
    sbs = list(range(cfg.n_subbands)) if subbands is None else list(subbands)
    L = cfg.n_rows if n_rows is None else n_rows
    Na = cfg.n_antennas
    pos = antenna_positions(cfg)
    sig = source_sigmas(cfg)
    lm = source_directions(cfg)
    out = torch.empty((len(sbs), L, Na, 2, 2), dtype=torch.int16, device=device)
    gen = torch.Generator(device=device)
    chunk = max(1, (1 << 26) // (Na * 4))
    for k, sb in enumerate(sbs):
        gen.manual_seed(cfg.seed * 100003 + sb)
        ph = geometric_phases(pos, lm, subband_frequency(sb))        # [src][Na]
        ph_t = torch.from_numpy(np.stack([ph.real, ph.imag], -1)).to(device=device, dtype=torch.float32)
        for r0 in range(0, L, chunk):
            r1 = min(L, r0 + chunk)
            n = r1 - r0
            v = torch.randn((n, Na, 2, 2), generator=gen, device=device, dtype=torch.float32)
            v.mul_(cfg.sigma_n)
            for si, s in enumerate(sig):
                sgl = torch.randn((n, 1, 2, 2), generator=gen, device=device, dtype=torch.float32) * s
                pr = ph_t[si][None, :, None, 0]       # [1][Na][1]
                pi = ph_t[si][None, :, None, 1]
                sr = sgl[..., 0]                      # [n][1][2]
                sim = sgl[..., 1]
                v[..., 0] += sr * pr - sim * pi
                v[..., 1] += sr * pi + sim * pr
            out[k, r0:r1] = torch.round(v).clamp_(-32768, 32767).to(torch.int16)
    return out


# --------------------------------------------------------------------------
# channelised samples for correlator-only tests (ABI block layout)
# --------------------------------------------------------------------------
def make_channelised(B: int, P: int, S: int, N: int, dtype: str, seed: int,
                     device="cpu", sigma: float = 31.75, corr: float = 0.3):
    """Random channelised samples in the block layout [B][P][Sb][N][8][2].

    Values are Gaussian with per-component `sigma` plus a common component
    (weight `corr`) shared by all inputs, so cross-correlations are not
    trivially small.  int8 values are rounded and clipped to [-127, 127]
    (the requantiser never emits -128); fp16 values are rounded to fp16.
    Spectra s >= S inside the last block are zero.
    """
    import torch
    Sb = (S + SPECTRUM_BLOCK - 1) // SPECTRUM_BLOCK
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    v = torch.randn((B, P, Sb, N, SPECTRUM_BLOCK, 2), generator=gen, device=device)
    c = torch.randn((B, P, Sb, 1, SPECTRUM_BLOCK, 2), generator=gen, device=device)
    v = (v * math.sqrt(1.0 - corr * corr) + c * corr) * sigma
    s_idx = torch.arange(Sb * SPECTRUM_BLOCK, device=device).view(Sb, SPECTRUM_BLOCK)
    mask = (s_idx < S).to(v.dtype)[None, None, :, None, :, None]
    v = v * mask
    if dtype == "i8":
        return torch.round(v).clamp_(-127, 127).to(torch.int8)
    if dtype == "f16":
        return v.to(torch.float16)
    if dtype == "f32":
        return v.to(torch.float32)
    raise ValueError(dtype)


def blocked_to_natural(z, S: int):
    """[..][Sb][N][8][2] block layout -> [..][S][N][2] (pure index permutation)."""
    Sb, N = z.shape[-4], z.shape[-3]
    lead = z.shape[:-4]
    zz = z.movedim(-3, -2) if hasattr(z, "movedim") else np.moveaxis(z, -3, -2)
    zz = zz.reshape(*lead, Sb * SPECTRUM_BLOCK, N, 2)
    return zz[..., :S, :, :]


# --------------------------------------------------------------------------
# calibration workload: model and observed visibilities, gains
# --------------------------------------------------------------------------
def baseline_count(Na: int) -> int:
    return Na * (Na + 1) // 2


def channel_offset(k: int, P: int) -> int:
    """Frequency offset (in channels) of FFT channel k: natural FFT order."""
    return k if k < P // 2 else k - P


def make_calibration(Na: int = 576, P: int = 64, n_src: int = 5, snr: float = 20.0,
                     seed: int = 5, layout: str = "stations12"):
    """Model M, observed V = G M G^H + noise, true gains g (numpy).

    Returns (V, M, g_true) with V, M float32 [P][Nbl][2][2][2] (the correlator
    output layout; XX = [0][0], YY = [1][1], XY = YX = 0) and g float32
    [P][Na][2][2] (complex gain per channel, antenna, polarisation).
    Sources: flux log-uniform in [10, 1000] Jy, directions uniform in the
    unit disc.  Noise: Hermitian (E + E^H)/2 with E complex Gaussian, scaled
    per (channel, pol) so that ||G M G^H||_F / ||noise||_F = snr.
    """
    cfg = Config("cal", Na, 1, n_channels=P, layout=layout, seed=seed)
    pos = antenna_positions(cfg)
    rng = np.random.default_rng([seed, 505])
    flux = np.exp(rng.uniform(np.log(10.0), np.log(1000.0), n_src))
    lm = _disc(rng, n_src, 1.0)
    amp = rng.uniform(0.8, 1.2, (P, Na, 2))
    pha = rng.uniform(0.0, 2.0 * np.pi, (P, Na, 2))
    g = amp * np.exp(1j * pha)
    tri_a, tri_b = np.tril_indices(Na)
    nbl = baseline_count(Na)
    # np.tril_indices enumerates row by row: bl(a, b) = a(a+1)/2 + b
    V = np.zeros((P, nbl, 2, 2), np.complex64)
    Mo = np.zeros((P, nbl, 2, 2), np.complex64)
    for k in range(P):
        nu = NU0 + channel_offset(k, P) * F_SUBBAND / P
        ph = geometric_phases(pos, lm, nu)                      # [src][Na]
        Mfull = np.einsum("s,sa,sb->ab", flux, ph, np.conj(ph))
        for pol in range(2):
            gg = g[k, :, pol]
            S_ = gg[:, None] * Mfull * np.conj(gg)[None, :]
            E = rng.standard_normal((Na, Na)) + 1j * rng.standard_normal((Na, Na))
            Nn = 0.5 * (E + E.conj().T)
            Nn *= np.linalg.norm(S_) / (snr * np.linalg.norm(Nn))
            V[k, :, pol, pol] = (S_ + Nn)[tri_a, tri_b]
            Mo[k, :, pol, pol] = Mfull[tri_a, tri_b]
    as_f = lambda c: np.ascontiguousarray(np.stack([c.real, c.imag], -1).astype(np.float32))
    return as_f(V), as_f(Mo), as_f(g.astype(np.complex64))
