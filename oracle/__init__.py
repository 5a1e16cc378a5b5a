"""CPU oracle for the FX-correlator hot path: TEST INFRASTRUCTURE ONLY.

Only `tests/`, `__graft_entry__.smoke()` and the CPU-baseline leg of
`bench.py` may import this package.  The product library never loads it and
shares no code with it.  The arithmetic lives in `afc_oracle.c` (double
precision, exact int64 for the int8 path); this module only marshals numpy
arrays through ctypes.  Each function cites the passage of the paper it
follows; see afc_oracle.c for the definitions.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liborc.so")
_lib = None

_p = C.c_void_p
_i64 = C.c_int64
_f32 = C.c_float


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = C.CDLL(_LIB_PATH)
    lib.orc_ppf_stream.argtypes = [_p, _i64, _i64, _i64, _p, _i64, _i64, _i64, _i64, _p]
    lib.orc_ppf_stream.restype = C.c_int
    lib.orc_ppf_stream_direct.argtypes = lib.orc_ppf_stream.argtypes
    lib.orc_ppf_stream_direct.restype = C.c_int
    lib.orc_requant.argtypes = [_p, _i64, _f32, _p]
    lib.orc_requant.restype = None
    lib.orc_xcorr_pairs_f64.argtypes = [_p, _i64, _i64, _i64, _p, _p]
    lib.orc_xcorr_pairs_f64.restype = None
    lib.orc_xcorr_pairs_i64.argtypes = [_p, _i64, _i64, _i64, _p, _p]
    lib.orc_xcorr_pairs_i64.restype = None
    lib.orc_xcorr_f64.argtypes = [_p, _i64, _i64, _p, _p, _p]
    lib.orc_xcorr_f64.restype = None
    lib.orc_xcorr_i64.argtypes = [_p, _i64, _i64, _p, _p, _p]
    lib.orc_xcorr_i64.restype = C.c_int
    lib.orc_cal_loss_grad.argtypes = [_p, _p, _p, _i64, _i64, _p, _p]
    lib.orc_cal_loss_grad.restype = C.c_int
    lib.orc_cal_loss_grad_w.argtypes = [_p, _p, _p, _p, _i64, _i64, _p, _p]
    lib.orc_cal_loss_grad_w.restype = C.c_int
    lib.orc_fine_channelise.argtypes = [_p, _i64, _i64, _i64, _p, _i64, _i64, _i64, _i64,
                                        C.c_double, C.c_double, C.c_double, _p, _i64, _p]
    lib.orc_fine_channelise.restype = C.c_int
    lib.orc_spectrum_validity.argtypes = [_p, _i64, _i64, _i64, _i64, _i64, _i64, _i64, _i64, _p]
    lib.orc_spectrum_validity.restype = None
    lib.orc_validity_weights.argtypes = [_p, _i64, _i64, _i64, _p, _p]
    lib.orc_validity_weights.restype = None
    _lib = lib
    return lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(np.asarray(a), dtype=dtype)


def _to_complex(a: np.ndarray) -> np.ndarray:
    return a[..., 0] + 1j * a[..., 1]


# --------------------------------------------------------------------------
# channeliser (Sec. "Polyphase Filterbank")
# --------------------------------------------------------------------------
def ppf_stream(x: np.ndarray, taps: np.ndarray, input: int, P: int, T: int,
               s0: int, s1: int, direct: bool = False) -> np.ndarray:
    """Channelised spectra s0..s1-1 of one input: complex128 [s1-s0][P].

    x: int16 [L][R][2] (one subband, R receivers) or [L][Na][2][2].
    """
    x = _c(x, np.int16)
    L = x.shape[0]
    R = x.size // (2 * L)
    taps = _c(taps, np.float32)
    assert taps.size == P * T
    y = np.empty((s1 - s0, P, 2), np.float64)
    fn = _load().orc_ppf_stream_direct if direct else _load().orc_ppf_stream
    rc = fn(_ptr(x), L, R, input, _ptr(taps), P, T, s0, s1, _ptr(y))
    if rc != 0:
        raise ValueError("orc_ppf_stream: invalid range or sizes")
    return _to_complex(y)


def ppf_subband(x: np.ndarray, taps: np.ndarray, P: int, T: int, S: int,
                inputs=None) -> np.ndarray:
    """All (or the listed) inputs of one subband: complex128 [P][S][R']."""
    x = _c(x, np.int16)
    L = x.shape[0]
    R = x.size // (2 * L)
    inputs = range(R) if inputs is None else list(inputs)
    out = np.empty((P, S, len(inputs)), np.complex128)
    for n, i in enumerate(inputs):
        out[:, :, n] = ppf_stream(x, taps, i, P, T, 0, S).T
    return out


def fine_channelise(x: np.ndarray, taps: np.ndarray, input: int, Pf: int, T: int, s0: int, s1: int,
                    tau: float, nu_c: float, df: float, w: np.ndarray, R: int) -> np.ndarray:
    """Fine channeliser + delay/bandpass compensation + R:1 channel
    integration of one input (Sec. "Polyphase Filterbank", Sec. "Delay,
    Bandpass Compensation and Transpose Kernel"): complex128 [s1-s0][Pf/R]."""
    x = _c(x, np.int16)
    L = x.shape[0]
    Rr = x.size // (2 * L)
    taps = _c(taps, np.float32)
    w = _c(w, np.float32)
    assert taps.size == Pf * T and w.size == Pf and Pf % R == 0
    out = np.empty((s1 - s0, Pf // R, 2), np.float64)
    rc = _load().orc_fine_channelise(_ptr(x), L, Rr, input, _ptr(taps), Pf, T, s0, s1, float(tau), float(nu_c),
                                     float(df), _ptr(w), R, _ptr(out))
    if rc != 0:
        raise ValueError("orc_fine_channelise: invalid range or sizes")
    return _to_complex(out)


def fine_subband(x: np.ndarray, taps: np.ndarray, Pf: int, T: int, S: int, tau: np.ndarray, nu_c: float,
                 df: float, w: np.ndarray, R: int, inputs=None) -> np.ndarray:
    """All (or the listed) inputs of one subband: complex128 [Pf/R][S][R']."""
    x = _c(x, np.int16)
    L = x.shape[0]
    Rr = x.size // (2 * L)
    inputs = range(Rr) if inputs is None else list(inputs)
    out = np.empty((Pf // R, S, len(inputs)), np.complex128)
    for n, i in enumerate(inputs):
        out[:, :, n] = fine_channelise(x, taps, i, Pf, T, 0, S, tau[i], nu_c, df, w, R).T
    return out


# --------------------------------------------------------------------------
# requantiser (Sec. "LOFAR Digital Processing", bit modes)
# --------------------------------------------------------------------------
def requant(y: np.ndarray, gain: float) -> np.ndarray:
    """float32 values (any shape) -> int8, clamp(rint(y*gain), +-127) of the
    exact product (rounded once, ties to even)."""
    y = _c(y, np.float32)
    q = np.empty(y.shape, np.int8)
    _load().orc_requant(_ptr(y), y.size, float(np.float32(gain)), _ptr(q))
    return q


# --------------------------------------------------------------------------
# correlator (Sec. "Correlation Kernel")
# --------------------------------------------------------------------------
def xcorr_pairs(rows: np.ndarray, pairs: np.ndarray) -> np.ndarray:
    """rows: complex [S][R] (or float [S][R][2]); pairs int [n][2] -> complex128 [n]."""
    if np.iscomplexobj(rows):
        rows = np.stack([rows.real, rows.imag], -1)
    rows = _c(rows, np.float64)
    S, R = rows.shape[0], rows.shape[1]
    pairs = _c(pairs, np.int32).reshape(-1, 2)
    out = np.empty((pairs.shape[0], 2), np.float64)
    _load().orc_xcorr_pairs_f64(_ptr(rows), S, R, pairs.shape[0], _ptr(pairs), _ptr(out))
    return _to_complex(out)


def xcorr_pairs_int(rows: np.ndarray, pairs: np.ndarray) -> np.ndarray:
    """rows: int8 [S][R][2]; pairs [n][2] -> int64 [n][2] exact sums."""
    rows = _c(rows, np.int8)
    S, R = rows.shape[0], rows.shape[1]
    pairs = _c(pairs, np.int32).reshape(-1, 2)
    out = np.empty((pairs.shape[0], 2), np.int64)
    _load().orc_xcorr_pairs_i64(_ptr(rows), S, R, pairs.shape[0], _ptr(pairs), _ptr(out))
    return out


def xcorr(z: np.ndarray, flags: Optional[np.ndarray] = None) -> Tuple[np.ndarray, np.ndarray]:
    """Lower triangle of one channel.

    z: complex [S][2*Na] (or float [S][2*Na][2]).
    Returns V complex128 [Nbl][2][2] and W int32 [Nbl].
    """
    if np.iscomplexobj(z):
        z = np.stack([z.real, z.imag], -1)
    z = _c(z, np.float64)
    S, R = z.shape[0], z.shape[1]
    Na = R // 2
    nbl = Na * (Na + 1) // 2
    V = np.empty((nbl, 2, 2, 2), np.float64)
    W = np.empty(nbl, np.int32)
    fl = None if flags is None else _c(flags, np.uint8)
    _load().orc_xcorr_f64(_ptr(z), S, Na, _ptr(fl), _ptr(V), _ptr(W))
    return _to_complex(V), W


def xcorr_int(z: np.ndarray, flags: Optional[np.ndarray] = None) -> Tuple[np.ndarray, np.ndarray]:
    """Exact integer lower triangle: z int8 [S][2*Na][2] -> V int64 [Nbl][2][2][2], W."""
    z = _c(z, np.int8)
    S, R = z.shape[0], z.shape[1]
    Na = R // 2
    nbl = Na * (Na + 1) // 2
    V = np.empty((nbl, 2, 2, 2), np.int64)
    W = np.empty(nbl, np.int32)
    fl = None if flags is None else _c(flags, np.uint8)
    rc = _load().orc_xcorr_i64(_ptr(z), S, Na, _ptr(fl), _ptr(V), _ptr(W))
    if rc != 0:
        raise OverflowError("integer visibility does not fit in int32")
    return V, W


# --------------------------------------------------------------------------
# lost packets and the weighting matrix (Sec. "CPU Data Collation";
# Sec. "Calibration Pipeline", weighting)
# --------------------------------------------------------------------------
def spectrum_validity(pkt: np.ndarray, Q: int, P: int, T: int, S: int, antennas=None) -> np.ndarray:
    """pkt uint8 [n_packets][Na] (nonzero = arrived), Q samples per packet ->
    uint8 [Na'][S]: spectrum s valid iff samples s*P .. (s+T)*P-1 all arrived."""
    pkt = _c(pkt, np.uint8)
    n_pk, Na = pkt.shape
    a0, a1 = (0, Na) if antennas is None else antennas
    v = np.empty((a1 - a0, S), np.uint8)
    _load().orc_spectrum_validity(_ptr(pkt), n_pk, Na, Q, P, T, S, a0, a1, _ptr(v))
    return v


def validity_weights(v: np.ndarray, S: int, flags: Optional[np.ndarray] = None) -> np.ndarray:
    """v uint8 [Na][>=S] -> int32 [Nbl]: spectra s < S valid for both antennas."""
    v = _c(v, np.uint8)
    Na = v.shape[0]
    W = np.empty(Na * (Na + 1) // 2, np.int32)
    fl = None if flags is None else _c(flags, np.uint8)
    _load().orc_validity_weights(_ptr(v), Na, v.shape[1], S, _ptr(fl), _ptr(W))
    return W


def zero_invalid(z: np.ndarray, v: np.ndarray) -> np.ndarray:
    """z [S][2*Na] (complex) with the samples of invalid spectra set to zero:
    z'[s][2a+p] = z[s][2a+p] if v[a][s] else 0 (both polarisations)."""
    keep = np.repeat(np.asarray(v, bool).T[:, :, None], 2, axis=2).reshape(z.shape[0], -1)
    return np.where(keep, z, 0)


# --------------------------------------------------------------------------
# gain calibration (Sec. "Calibration Pipeline")
# --------------------------------------------------------------------------
def cal_weights(P: int, nbl: int, flags: Optional[np.ndarray] = None,
                weights: Optional[np.ndarray] = None) -> np.ndarray:
    """Per-baseline calibration weights float64 [P][Nbl][2] (XX, YY) (Sec.
    "Real-time Flagging, Calibration and Imaging": the calibration works on
    the flagged visibilities, re-weighted for lost data): 0 where flags
    (uint8 [P][Nbl][2], nonzero = flagged) is set, else the given weight
    (float [P][Nbl][2]) or 1."""
    w = np.ones((P, nbl, 2), np.float64) if weights is None else np.asarray(weights, np.float64).copy()
    if flags is not None:
        w[np.asarray(flags) != 0] = 0.0
    return w


def cal_loss_grad(V: np.ndarray, M: np.ndarray, g: np.ndarray,
                  want_grad: bool = True, weights: Optional[np.ndarray] = None
                  ) -> Tuple[np.ndarray, Optional[np.ndarray]]:
    """V, M float32 [P][Nbl][2][2][2]; g float32 [P][Na][2][2]; optional
    weights float64 [P][Nbl][2] (the weighted loss sum w_ab |R_ab|^2).

    Returns loss float64 [P][2] and grad complex128 [P][Na][2] (or None).
    """
    V = _c(V, np.float32)
    M = _c(M, np.float32)
    g = _c(g, np.float32)
    P, Na = g.shape[0], g.shape[1]
    assert V.shape[:2] == (P, Na * (Na + 1) // 2) and M.shape == V.shape
    loss = np.empty((P, 2), np.float64)
    grad = np.empty((P, Na, 2, 2), np.float64) if want_grad else None
    if weights is None:
        rc = _load().orc_cal_loss_grad(_ptr(V), _ptr(M), _ptr(g), Na, P, _ptr(loss), _ptr(grad))
    else:
        w = _c(weights, np.float64)
        assert w.shape == (P, Na * (Na + 1) // 2, 2)
        rc = _load().orc_cal_loss_grad_w(_ptr(V), _ptr(M), _ptr(w), _ptr(g), Na, P, _ptr(loss), _ptr(grad))
    if rc != 0:
        raise MemoryError("orc_cal_loss_grad")
    return loss, (None if grad is None else _to_complex(grad))


# --------------------------------------------------------------------------
# calibration solver and flagging (Sec. "Calibration Pipeline")
# --------------------------------------------------------------------------
def _full(T_lower: np.ndarray, Na: int, pol: int) -> np.ndarray:
    """Hermitian Na x Na matrix (complex128) of polarisation pol (0 = XX,
    1 = YY) from a lower triangle float [Nbl][2][2][2]: entry (a, b), a >= b,
    at bl = a(a+1)/2 + b; the upper triangle is the conjugate."""
    t = T_lower[:, pol, pol, 0].astype(np.float64) + 1j * T_lower[:, pol, pol, 1].astype(np.float64)
    F = np.zeros((Na, Na), np.complex128)
    a, b = np.tril_indices(Na)
    F[a, b] = t
    F[b, a] = np.conj(t)
    return F


def cal_solve(V: np.ndarray, M: np.ndarray, g0: np.ndarray, n_iter: int,
              weights: Optional[np.ndarray] = None) -> np.ndarray:
    """Per-channel complex gains minimising L = ||V - G M G^H||_F^2 for XX and
    YY (Sec. "Calibration Pipeline": amplitude and phase calibration per
    channel against a point-source model; least-squares reading).

    Alternating least squares with averaging (the StEFCal iteration of
    Salvini & Wijnholds, 2014): with every other gain fixed, the best g_a is
    sum_b V_ab conj(z_ab) / sum_b |z_ab|^2, z_ab = M_ab conj(g_b); all gains
    are updated from the previous iterate at once, and on every second
    iteration the new iterate is averaged with the previous one.  After
    n_iter iterations the common phase is removed so that g_0 is real and
    positive.

    With weights (float [P][Nbl][2], the weighted loss of cal_loss_grad)
    the same update minimises sum_b w_ab |V_ab - g_a z_ab|^2 over g_a:
    sum_b w_ab V_ab conj(z_ab) / sum_b w_ab |z_ab|^2.

    V, M float32 [P][Nbl][2][2][2]; g0 complex [P][Na][2] -> complex128 [P][Na][2].
    """
    P, nbl = V.shape[0], V.shape[1]
    Na = int(round((np.sqrt(8 * nbl + 1) - 1) / 2))
    out = np.empty((P, Na, 2), np.complex128)
    for ch in range(P):
        for pol in range(2):
            Vf = _full(V[ch], Na, pol)
            Mf = _full(M[ch], Na, pol)
            Wf = np.ones((Na, Na))
            if weights is not None:
                a_, b_ = np.tril_indices(Na)
                Wf[a_, b_] = weights[ch, :, pol]
                Wf[b_, a_] = weights[ch, :, pol]
            g = np.asarray(g0[ch, :, pol], np.complex128).copy()
            for it in range(1, n_iter + 1):
                z = Mf * np.conj(g)[None, :]
                num = (Wf * Vf * np.conj(z)).sum(axis=1)
                den = (Wf * np.abs(z) ** 2).sum(axis=1)
                g_new = np.where(den > 0, num / np.where(den > 0, den, 1.0), g)
                if it % 2 == 0:
                    g_new = 0.5 * (g_new + g)
                g = g_new
            if abs(g[0]) > 0:
                g = g * (np.conj(g[0]) / abs(g[0]))
            out[ch, :, pol] = g
    return out


def sigma_clip(V: np.ndarray, k: float) -> np.ndarray:
    """Flags uint8 [P][Nbl][2] (XX, YY) of the real-time flagger (Sec.
    "Calibration Pipeline", flagging): sigma clipping of visibility
    amplitudes against the locally computed RMS, first across the
    visibilities of each channel, then across the channels of each
    visibility.

    Stage 1, per channel and polarisation: RMS^2 = mean |V|^2 over the
    cross-correlations; flag those with |V| > k RMS.  Stage 2, per
    cross-correlation and polarisation: RMS^2 = mean |V|^2 over the channels
    not flagged in stage 1; flag the channels with |V| > k RMS.
    Autocorrelations are neither used nor flagged.  V float32
    [P][Nbl][2][2][2].
    """
    P, nbl = V.shape[0], V.shape[1]
    Na = int(round((np.sqrt(8 * nbl + 1) - 1) / 2))
    a, b = np.tril_indices(Na)
    cross = a != b
    flags = np.zeros((P, nbl, 2), np.uint8)
    k2 = float(k) * float(k)
    for pol in range(2):
        re = V[:, :, pol, pol, 0].astype(np.float64)
        im = V[:, :, pol, pol, 1].astype(np.float64)
        a2 = re * re + im * im                                     # [P][Nbl]
        for ch in range(P):
            m = a2[ch, cross].mean()
            flags[ch, cross & (a2[ch] > k2 * m), pol] = 1
        keep = flags[:, :, pol] == 0                               # [P][Nbl]
        n = keep.sum(axis=0)
        m = np.where(keep, a2, 0.0).sum(axis=0) / np.maximum(n, 1)   # per baseline
        hit = (a2 > k2 * m[None, :]) & (cross & (n > 0))[None, :]
        flags[:, :, pol] |= hit.astype(np.uint8)
    return flags


def apply_vis_flags(T: np.ndarray, flags: np.ndarray) -> np.ndarray:
    """Copy of T float [P][Nbl][2][2][2] with the flagged XX / YY entries set
    to zero (a zeroed visibility and model drop out of the loss)."""
    T = np.array(T, copy=True)
    for pol in range(2):
        T[:, :, pol, pol, :] *= (flags[:, :, pol] == 0)[:, :, None]
    return T


# --------------------------------------------------------------------------
# gridding and imaging (Sec. "Imaging Pipeline")
# --------------------------------------------------------------------------
C_LIGHT = 299792458.0


def grid_visibilities(V: np.ndarray, W, pos: np.ndarray, freq: np.ndarray, N: int, du: float):
    """Spectral integration by bilinear gridding (Sec. "Imaging Pipeline":
    the visibilities of several subbands are gridded onto one grid with
    bilinear interpolation).

    V float [B][P][Nbl][2][2][2] (calibrated, afc_correlate layout), W int
    [B][Nbl] weights or None (1), pos [Na][2] east/north metres, freq [B][P]
    sky frequency of each channel in Hz, N grid size (N % 4 == 0), du cell
    size in wavelengths.  For every cross-correlation a > c with weight w > 0,
    I = (XX + YY) / 2 sits at u = (x_a - x_c) nu / c, v = (y_a - y_c) nu / c;
    with (pu, pv) = (u, v) / du + N/2, i0 = floor(pu), fu = pu - i0 (and j0,
    fv), w I is spread over cells (j0 + dj, i0 + di), di, dj in {0, 1}, with
    weights (1-fu or fu)(1-fv or fv), and w conj(I) over the mirrored cells
    (N - j0 - dj, N - i0 - di) (the visibility at -u, -v).  A visibility is
    gridded only if all eight cells lie inside the grid (1 <= i0, j0 and
    i0, j0 <= N - 2).  Returns (G complex128 [N][N] indexed [v][u], norm = sum
    of 2 w over the gridded visibilities)."""
    V = np.asarray(V)
    B, P, nbl = V.shape[0], V.shape[1], V.shape[2]
    Na = pos.shape[0]
    a, c = np.tril_indices(Na)
    cross = a != c
    a, c = a[cross], c[cross]
    blx = np.flatnonzero(cross)
    dx = pos[a, 0] - pos[c, 0]
    dy = pos[a, 1] - pos[c, 1]
    G = np.zeros((N, N), np.complex128)
    norm = 0.0
    for b in range(B):
        w = np.ones(blx.size) if W is None else np.asarray(W[b], np.float64)[blx]
        for k in range(P):
            I = 0.5 * ((V[b, k, blx, 0, 0, 0].astype(np.float64) + V[b, k, blx, 1, 1, 0])
                       + 1j * (V[b, k, blx, 0, 0, 1].astype(np.float64) + V[b, k, blx, 1, 1, 1]))
            nu = float(freq[b, k])
            pu = dx * nu / C_LIGHT / du + N / 2
            pv = dy * nu / C_LIGHT / du + N / 2
            i0 = np.floor(pu).astype(np.int64)
            j0 = np.floor(pv).astype(np.int64)
            fu = pu - i0
            fv = pv - j0
            ok = (w > 0) & (i0 >= 1) & (j0 >= 1) & (i0 <= N - 2) & (j0 <= N - 2)
            for dj in (0, 1):
                for di in (0, 1):
                    wt = (fu if di else 1.0 - fu) * (fv if dj else 1.0 - fv) * w
                    np.add.at(G, (j0[ok] + dj, i0[ok] + di), wt[ok] * I[ok])
                    np.add.at(G, (N - j0[ok] - dj, N - i0[ok] - di), wt[ok] * np.conj(I[ok]))
            norm += 2.0 * w[ok].sum()
    return G, norm


def image_from_grid(G: np.ndarray, norm: float) -> np.ndarray:
    """Snapshot image (Sec. "Imaging Pipeline": the gridded visibilities are
    Fourier transformed): for N % 4 == 0,
        img[j][i] = Re sum_{q,p} G[q][p] exp(-2 pi i ((p - N/2)(i - N/2)
                    + (q - N/2)(j - N/2)) / N) / norm,
    pixel (i, j) at l = (i - N/2) / (N du), m = (j - N/2) / (N du).
    Evaluated as (-1)^(i+j) Re FFT2[(-1)^(p+q) G] with numpy's FFT (the
    exponent expands to pi + pi*i... terms that give these signs)."""
    N = G.shape[0]
    assert N % 4 == 0
    s = (-1.0) ** np.add.outer(np.arange(N), np.arange(N))
    F = np.fft.fft2(G * s)
    return (s * F.real) / (norm if norm > 0 else 1.0)
