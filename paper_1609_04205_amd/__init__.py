"""Python binding of the MI355X FX-correlator library (libafc.so).

Argument marshalling only: every step of the channeliser, the correlator and
the calibration gradient runs in the HIP kernels behind the C ABI declared in
include/afc.h.  PyTorch provides device memory and the current stream.  If
the built library is missing, importing this package raises: there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional, Sequence, Tuple

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("AFC_LIBRARY", os.path.join(HERE, "libafc.so"))

AFC_F32, AFC_F16, AFC_I8 = 0, 1, 2
DTYPES = {"f32": AFC_F32, "f16": AFC_F16, "i8": AFC_I8}
SPECTRUM_BLOCK = 8
N_CHANNELS = 64
N_TAPS = 16
N_FINE = 256          # channels of the fine bank, integrated 4:1 to N_CHANNELS
SUBBAND_HZ = 195312.5

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run paper_1609_04205_amd/build.py (or __graft_entry__.build())")

_lib = C.CDLL(LIB_PATH)


class Dims(C.Structure):
    _fields_ = [("n_antennas", C.c_int32), ("n_pols", C.c_int32), ("n_subbands", C.c_int32),
                ("n_channels", C.c_int32), ("n_taps", C.c_int32), ("n_spectra", C.c_int32)]


_vp, _i32, _f32, _sz = C.c_void_p, C.c_int32, C.c_float, C.c_size_t
_lib.afc_last_error.restype = C.c_char_p
_lib.afc_channelised_bytes.argtypes = [C.POINTER(Dims), C.c_int]
_lib.afc_channelised_bytes.restype = _sz
_lib.afc_visibility_bytes.argtypes = [C.POINTER(Dims)]
_lib.afc_visibility_bytes.restype = _sz
_lib.afc_channelise.argtypes = [C.POINTER(Dims), _vp, _vp, C.c_int, _f32, _vp, _vp]
_lib.afc_correlate.argtypes = [C.POINTER(Dims), C.c_int, _vp, _vp, _vp, _vp, _vp, _vp]
_lib.afc_validity_words.argtypes = [C.POINTER(Dims)]
_lib.afc_validity_words.restype = _sz
_lib.afc_validity.argtypes = [C.POINTER(Dims), _vp, _i32, _i32, _i32, _vp, _vp]
_lib.afc_zero_invalid.argtypes = [C.POINTER(Dims), C.c_int, _vp, _vp, _vp]
_lib.afc_validity_weights.argtypes = [C.POINTER(Dims), _vp, _vp, _vp, _vp, _vp]
_lib.afc_normalise_visibilities.argtypes = [C.POINTER(Dims), C.c_int, _vp, _vp, _vp, _vp]
_lib.afc_channelise_fine_workspace_bytes.argtypes = [C.POINTER(Dims)]
_lib.afc_channelise_fine_workspace_bytes.restype = _sz
_lib.afc_channelise_fine.argtypes = [C.POINTER(Dims), _vp, _vp, _vp, _vp, C.POINTER(C.c_double), C.c_double,
                                     C.c_int, _f32, _vp, _vp, _vp]
_lib.afc_calibrate_workspace_bytes.argtypes = [_i32, _i32]
_lib.afc_calibrate_workspace_bytes.restype = _sz
_lib.afc_calibrate_grad.argtypes = [_i32, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
_lib.afc_calibrate_grad_noalloc.argtypes = [_i32, _i32, _vp, _vp, _vp, _vp, _vp, _vp]
_lib.afc_calibrate_solve_workspace_bytes.argtypes = [_i32, _i32]
_lib.afc_calibrate_solve_workspace_bytes.restype = _sz
_lib.afc_calibrate_solve.argtypes = [_i32, _i32, _vp, _vp, _vp, _i32, _vp, _vp, _vp]
_lib.afc_calibrate_grad_weighted.argtypes = [_i32, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
_lib.afc_calibrate_solve_weighted.argtypes = [_i32, _i32, _vp, _vp, _vp, _vp, _vp, _i32, _vp, _vp, _vp]
_lib.afc_sigma_clip_workspace_bytes.argtypes = [_i32, _i32]
_lib.afc_sigma_clip_workspace_bytes.restype = _sz
_lib.afc_sigma_clip.argtypes = [_i32, _i32, _vp, _f32, _vp, _vp, _vp]
_lib.afc_apply_vis_flags.argtypes = [_i32, _i32, _vp, _vp, _vp, _vp]
_lib.afc_imaging_workspace_bytes.argtypes = [_i32, _i32, _i32]
_lib.afc_imaging_workspace_bytes.restype = _sz
_lib.afc_grid_visibilities.argtypes = [_i32, _i32, _vp, _vp, _vp, _vp, _i32, C.c_double, _vp, _vp, _vp, _vp]
_lib.afc_image_from_grid.argtypes = [_i32, _vp, _vp, _vp, _vp, _vp]
_lib.afc_plan_create.argtypes = [C.POINTER(Dims), _vp, _vp, C.c_char_p, C.POINTER(_vp)]
_lib.afc_plan_workspace_bytes.argtypes = [_vp]
_lib.afc_plan_workspace_bytes.restype = _sz
_lib.afc_plan_launch.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
_lib.afc_plan_info.argtypes = [_vp, C.POINTER(_i32), C.POINTER(_i32), C.POINTER(_i32), C.POINTER(_i32)]
_lib.afc_plan_destroy.argtypes = [_vp]
_lib.afc_plan_destroy.restype = None
_lib.afc_set_checked_mode.argtypes = [C.c_int]
_lib.afc_set_checked_mode.restype = None
_lib.afc_checked_mode.restype = C.c_int
_lib.afc_count_nonfinite.argtypes = [_vp, _sz, C.c_int, C.POINTER(C.c_uint64), _vp]

EXPORTS = ["afc_channelised_bytes", "afc_visibility_bytes", "afc_channelise",
           "afc_channelise_fine_workspace_bytes", "afc_channelise_fine", "afc_correlate",
           "afc_validity_words", "afc_validity", "afc_zero_invalid", "afc_validity_weights",
           "afc_normalise_visibilities", "afc_calibrate_solve_workspace_bytes", "afc_calibrate_solve",
           "afc_sigma_clip_workspace_bytes", "afc_sigma_clip", "afc_apply_vis_flags",
           "afc_imaging_workspace_bytes", "afc_grid_visibilities", "afc_image_from_grid",
           "afc_calibrate_workspace_bytes", "afc_calibrate_grad", "afc_calibrate_grad_noalloc",
           "afc_calibrate_grad_weighted", "afc_calibrate_solve_weighted", "afc_plan_create",
           "afc_plan_workspace_bytes", "afc_plan_launch", "afc_plan_info", "afc_plan_destroy",
           "afc_set_checked_mode", "afc_checked_mode", "afc_count_nonfinite", "afc_last_error"]

AFC_VALUES_F32, AFC_VALUES_F16, AFC_VALUES_F64 = 0, 1, 3


class AfcError(RuntimeError):
    pass


def _check(rc: int, what: str):
    if rc != 0:
        raise AfcError(f"{what} failed ({rc}): {_lib.afc_last_error().decode()}")


def set_checked_mode(on: bool) -> None:
    """Checked (debug) mode, process-wide: every entry point refuses
    non-finite floating-point inputs (and waits for its stream to count
    them).  Off by default."""
    _lib.afc_set_checked_mode(1 if on else 0)


def checked_mode() -> bool:
    return bool(_lib.afc_checked_mode())


def count_nonfinite(t) -> int:
    """Number of NaN / Inf values of a float32, float16 or float64 GPU tensor."""
    torch = _torch()
    kinds = {torch.float32: AFC_VALUES_F32, torch.float16: AFC_VALUES_F16, torch.float64: AFC_VALUES_F64}
    if t.dtype not in kinds:
        raise AfcError(f"count_nonfinite: float32, float16 or float64 tensor expected, got {t.dtype}")
    _require(t, t.dtype, "values")
    out = C.c_uint64(0)
    _check(_lib.afc_count_nonfinite(_ptr(t), t.numel(), kinds[t.dtype], C.byref(out), _stream(t)),
           "afc_count_nonfinite")
    return int(out.value)


def dims(n_antennas: int, n_subbands: int, n_spectra: int, n_channels: int = N_CHANNELS,
         n_taps: int = N_TAPS) -> Dims:
    return Dims(n_antennas, 2, n_subbands, n_channels, n_taps, n_spectra)


def _torch():
    import torch
    return torch


def _stream(*tensors):
    """Current stream of the first tensor's GPU, after checking that every
    buffer of the call (None skipped) lives on that GPU.  Called last, after
    the shape checks, right before the library call."""
    torch = _torch()
    ts = [t for t in tensors if t is not None]
    dev = ts[0].device
    for t in ts:
        if not t.is_cuda:
            raise AfcError(f"every buffer must be a GPU tensor (got one on {t.device})")
        if t.device != dev:
            raise AfcError(f"buffers on {dev} and {t.device}: one GPU per call")
    return C.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def _ptr(t) -> Optional[C.c_void_p]:
    return None if t is None else C.c_void_p(t.data_ptr())


def _require(t, dtype, name, shape=None):
    """Type, shape and layout of a caller buffer (a buffer of the wrong size
    is a host-side error, never an out-of-bounds device access).  Devices are
    checked by _stream()."""
    if t.dtype != dtype:
        raise AfcError(f"{name} must be {dtype}, got {t.dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise AfcError(f"{name} shape {tuple(t.shape)} != {tuple(shape)}")
    if not t.is_contiguous():
        raise AfcError(f"{name} must be contiguous")


_TORCH_OF = {"f32": "float32", "f16": "float16", "i8": "int8"}


def channelised_shape(n_subbands, n_spectra, n_inputs):
    sb = (n_spectra + SPECTRUM_BLOCK - 1) // SPECTRUM_BLOCK
    return (n_subbands, N_CHANNELS, sb, n_inputs, SPECTRUM_BLOCK, 2)


def channelise(x, taps, n_spectra: int, out_dtype: str = "f32", gain: float = 1.0, out=None):
    """x int16 [B][L][Na][2][2] (or [B][L][N][2]) -> z [B][P][Sb][N][8][2]."""
    torch = _torch()
    if out_dtype not in DTYPES:
        raise AfcError(f"out_dtype must be one of {sorted(DTYPES)}, got {out_dtype!r}")
    _require(x, torch.int16, "x")
    B, L = x.shape[0], x.shape[1]
    N = x[0, 0].numel() // 2
    if x.dim() < 3 or x.shape[-1] != 2 or N % 2:
        raise AfcError(f"x shape {tuple(x.shape)} is not [B][L][N][2] with N even")
    _require(taps, torch.float32, "taps", (N_TAPS * N_CHANNELS,))
    Na = N // 2
    d = dims(Na, B, n_spectra)
    if L != (n_spectra + N_TAPS - 1) * N_CHANNELS:
        raise AfcError(f"x has {L} rows, expected (S+T-1)*P = {(n_spectra + N_TAPS - 1) * N_CHANNELS}")
    shape = channelised_shape(B, n_spectra, N)
    tdt = getattr(torch, _TORCH_OF[out_dtype])
    if out is None:
        out = torch.empty(shape, dtype=tdt, device=x.device)
    _require(out, tdt, "out", shape)
    _check(_lib.afc_channelise(C.byref(d), _ptr(x), _ptr(taps), DTYPES[out_dtype], float(gain), _ptr(out),
                               _stream(x, taps, out)), "afc_channelise")
    return out


def fine_workspace_bytes(n_antennas: int, n_subbands: int, n_spectra: int) -> int:
    d = dims(n_antennas, n_subbands, n_spectra)
    return int(_lib.afc_channelise_fine_workspace_bytes(C.byref(d)))


def channelise_fine(x, taps, n_spectra: int, delays, bandpass, center_hz: Sequence[float],
                    subband_hz: float = SUBBAND_HZ, out_dtype: str = "f32", gain: float = 1.0, out=None,
                    workspace=None):
    """256-channel bank, delay and bandpass compensation, 4:1 channel
    integration: x int16 [B][L][N][2], L = (S+15)*256 -> z [B][64][Sb][N][8][2]
    (the layout of channelise).  delays float64 [N] seconds and bandpass
    float32 [256] on the GPU; center_hz: B sky frequencies (host)."""
    torch = _torch()
    if out_dtype not in DTYPES:
        raise AfcError(f"out_dtype must be one of {sorted(DTYPES)}, got {out_dtype!r}")
    _require(x, torch.int16, "x")
    B, L = x.shape[0], x.shape[1]
    N = x[0, 0].numel() // 2
    if x.dim() < 3 or x.shape[-1] != 2 or N % 2:
        raise AfcError(f"x shape {tuple(x.shape)} is not [B][L][N][2] with N even")
    _require(taps, torch.float32, "taps", (N_TAPS * N_FINE,))
    _require(delays, torch.float64, "delays", (N,))
    _require(bandpass, torch.float32, "bandpass", (N_FINE,))
    d = dims(N // 2, B, n_spectra)
    if L != (n_spectra + N_TAPS - 1) * N_FINE:
        raise AfcError(f"x has {L} rows, expected (S+T-1)*256 = {(n_spectra + N_TAPS - 1) * N_FINE}")
    if len(center_hz) != B:
        raise AfcError(f"center_hz has {len(center_hz)} entries, expected {B}")
    nu = (C.c_double * B)(*[float(v) for v in center_hz])
    shape = channelised_shape(B, n_spectra, N)
    tdt = getattr(torch, _TORCH_OF[out_dtype])
    if out is None:
        out = torch.empty(shape, dtype=tdt, device=x.device)
    _require(out, tdt, "out", shape)
    need = _lib.afc_channelise_fine_workspace_bytes(C.byref(d))
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=x.device)
    _require(workspace, torch.uint8, "workspace")
    if workspace.numel() < need:
        raise AfcError(f"workspace holds {workspace.numel()} bytes, {need} needed")
    _check(_lib.afc_channelise_fine(C.byref(d), _ptr(x), _ptr(taps), _ptr(delays), _ptr(bandpass), nu,
                                    float(subband_hz), DTYPES[out_dtype], float(gain), _ptr(workspace),
                                    _ptr(out), _stream(x, taps, delays, bandpass, workspace, out)), "afc_channelise_fine")
    return out


def validity_shape(n_subbands, n_spectra, n_antennas):
    return (n_subbands, (n_spectra + 31) // 32, n_antennas)


def validity(packet_valid, n_spectra: int, packet_samples: int, samples_per_spectrum: int = N_CHANNELS,
             out=None):
    """packet_valid uint8 [B][n_packets][Na] -> spectrum validity bits, int32
    [B][ceil(S/32)][Na] (bit s % 32 of word s // 32 = spectrum s valid)."""
    torch = _torch()
    if packet_valid.dim() != 3:
        raise AfcError(f"packet_valid shape {tuple(packet_valid.shape)} is not [B][n_packets][Na]")
    _require(packet_valid, torch.uint8, "packet_valid")
    B, n_pk, Na = packet_valid.shape
    d = dims(Na, B, n_spectra)
    shape = validity_shape(B, n_spectra, Na)
    if out is None:
        out = torch.empty(shape, dtype=torch.int32, device=packet_valid.device)
    _require(out, torch.int32, "out", shape)
    _check(_lib.afc_validity(C.byref(d), _ptr(packet_valid), int(n_pk), int(packet_samples),
                             int(samples_per_spectrum), _ptr(out), _stream(packet_valid, out)), "afc_validity")
    return out


def zero_invalid(z, spec_valid, n_spectra: int):
    """Zero, in place, the samples of z [B][64][Sb][N][8][2] whose spectrum is
    invalid for their antenna."""
    torch = _torch()
    dt = {torch.float32: "f32", torch.float16: "f16", torch.int8: "i8"}.get(z.dtype)
    if dt is None or z.dim() != 6:
        raise AfcError(f"z must be float32, float16 or int8 [B][64][Sb][N][8][2], got {z.dtype} {tuple(z.shape)}")
    B, N = z.shape[0], z.shape[3]
    _require(z, z.dtype, "z", channelised_shape(B, n_spectra, N))
    _require(spec_valid, torch.int32, "spec_valid", validity_shape(B, n_spectra, N // 2))
    d = dims(N // 2, B, n_spectra)
    _check(_lib.afc_zero_invalid(C.byref(d), DTYPES[dt], _ptr(spec_valid), _ptr(z), _stream(z, spec_valid)),
           "afc_zero_invalid")
    return z


def validity_weights(spec_valid, n_spectra: int, n_spectra_per_sb: Optional[Sequence[int]] = None, flags=None,
                     out=None):
    """Weighting matrix int32 [B][Nbl]: spectra valid for both antennas of each baseline."""
    torch = _torch()
    B, _, Na = spec_valid.shape
    _require(spec_valid, torch.int32, "spec_valid", validity_shape(B, n_spectra, Na))
    d = dims(Na, B, n_spectra)
    if out is None:
        out = torch.empty((B, Na * (Na + 1) // 2), dtype=torch.int32, device=spec_valid.device)
    _require(out, torch.int32, "out", (B, Na * (Na + 1) // 2))
    if flags is not None:
        _require(flags, torch.uint8, "flags", (B, Na))
    sp = None
    if n_spectra_per_sb is not None:
        if len(n_spectra_per_sb) != B:
            raise AfcError(f"n_spectra_per_sb has {len(n_spectra_per_sb)} entries, expected {B}")
        arr = (C.c_int32 * B)(*[int(v) for v in n_spectra_per_sb])
        sp = C.cast(arr, C.c_void_p)
    _check(_lib.afc_validity_weights(C.byref(d), _ptr(spec_valid), sp, _ptr(flags), _ptr(out),
                                     _stream(spec_valid, flags, out)), "afc_validity_weights")
    return out


def normalise_visibilities(vis, weights, out=None):
    """vis [B][64][Nbl][2][2][2] (int32 or float32) / weights [B][Nbl] -> float32, 0 where W = 0."""
    torch = _torch()
    if vis.dtype not in (torch.int32, torch.float32):
        raise AfcError(f"vis must be int32 or float32, got {vis.dtype}")
    dt = "i8" if vis.dtype == torch.int32 else "f32"
    B, nbl = vis.shape[0], vis.shape[2]
    Na = int(round(((8 * nbl + 1) ** 0.5 - 1) / 2))
    _require(vis, vis.dtype, "vis", visibility_shape(B, Na))
    _require(weights, torch.int32, "weights", (B, nbl))
    if out is None:
        out = torch.empty(vis.shape, dtype=torch.float32, device=vis.device)
    _require(out, torch.float32, "out", vis.shape)
    if out.data_ptr() == vis.data_ptr():
        raise AfcError("out may not alias vis")
    d = dims(Na, B, 1)
    _check(_lib.afc_normalise_visibilities(C.byref(d), DTYPES[dt], _ptr(vis), _ptr(weights), _ptr(out),
                                           _stream(vis, weights, out)), "afc_normalise_visibilities")
    return out


def visibility_shape(n_subbands, n_antennas):
    return (n_subbands, N_CHANNELS, n_antennas * (n_antennas + 1) // 2, 2, 2, 2)


def correlate(z, n_spectra: Optional[int] = None, n_spectra_per_sb: Optional[Sequence[int]] = None,
              flags=None, want_weights: bool = True, out=None, weights=None):
    """z [B][P][Sb][N][8][2] -> (vis [B][P][Nbl][2][2][2] float32 or int32, weights [B][Nbl] int32)."""
    torch = _torch()
    dt = {torch.float32: "f32", torch.float16: "f16", torch.int8: "i8"}.get(z.dtype)
    if dt is None or z.dim() != 6:
        raise AfcError(f"z must be float32, float16 or int8 [B][64][Sb][N][8][2], got {z.dtype} {tuple(z.shape)}")
    B, P, Sb, N = z.shape[0], z.shape[1], z.shape[2], z.shape[3]
    if P != N_CHANNELS or z.shape[4] != SPECTRUM_BLOCK or z.shape[5] != 2 or N % 2:
        raise AfcError(f"z shape {tuple(z.shape)} is not [B][64][Sb][N][8][2] with N even")
    _require(z, z.dtype, "z")
    S = n_spectra if n_spectra is not None else Sb * SPECTRUM_BLOCK
    if (S + SPECTRUM_BLOCK - 1) // SPECTRUM_BLOCK != Sb:
        raise AfcError("n_spectra does not match the number of spectrum blocks")
    Na = N // 2
    d = dims(Na, B, S)
    vdt = torch.int32 if dt == "i8" else torch.float32
    if out is None:
        out = torch.empty(visibility_shape(B, Na), dtype=vdt, device=z.device)
    _require(out, vdt, "out", visibility_shape(B, Na))
    if want_weights and weights is None:
        weights = torch.empty((B, Na * (Na + 1) // 2), dtype=torch.int32, device=z.device)
    if weights is not None:
        _require(weights, torch.int32, "weights", (B, Na * (Na + 1) // 2))
    if flags is not None:
        _require(flags, torch.uint8, "flags", (B, Na))
    sp = None
    if n_spectra_per_sb is not None:
        if len(n_spectra_per_sb) != B:
            raise AfcError(f"n_spectra_per_sb has {len(n_spectra_per_sb)} entries, expected {B}")
        arr = (C.c_int32 * B)(*[int(v) for v in n_spectra_per_sb])
        sp = C.cast(arr, C.c_void_p)
    _check(_lib.afc_correlate(C.byref(d), DTYPES[dt], _ptr(z), sp, _ptr(flags), _ptr(out), _ptr(weights),
                              _stream(z, flags, out, weights)), "afc_correlate")
    return out, weights


def _cal_shapes(V, M, g):
    """(P, Na) of calibration buffers V, M [P][Nbl][2][2][2] and g [P][Na][2][2]."""
    torch = _torch()
    if g.dim() != 4:
        raise AfcError(f"g shape {tuple(g.shape)} is not [P][Na][2][2]")
    P, Na = g.shape[0], g.shape[1]
    nbl = Na * (Na + 1) // 2
    _require(g, torch.float32, "g", (P, Na, 2, 2))
    _require(V, torch.float32, "V", (P, nbl, 2, 2, 2))
    _require(M, torch.float32, "M", (P, nbl, 2, 2, 2))
    return P, Na


def _workspace(ws, nbytes: int, device):
    """A caller's workspace (uint8, at least nbytes) or a new one."""
    torch = _torch()
    if ws is None:
        return torch.empty(max(1, nbytes), dtype=torch.uint8, device=device)
    _require(ws, torch.uint8, "workspace")
    if ws.numel() < nbytes:
        raise AfcError(f"workspace holds {ws.numel()} bytes, {nbytes} needed")
    return ws


def _cal_weights(P: int, Na: int, flags, weights):
    torch = _torch()
    nbl = Na * (Na + 1) // 2
    if flags is not None:
        _require(flags, torch.uint8, "flags", (P, nbl, 2))
    if weights is not None:
        _require(weights, torch.float32, "weights", (P, nbl, 2))


def calibrate_grad(V, M, g, want_grad: bool = True, workspace=None, flags=None, weights=None):
    """V, M float32 [P][Nbl][2][2][2]; g float32 [P][Na][2][2] -> (loss float64 [P][2], grad [P][Na][2][2]).
    With flags (uint8 [P][Nbl][2], nonzero = flagged) and/or weights (float32
    [P][Nbl][2]): the weighted loss (afc_calibrate_grad_weighted)."""
    torch = _torch()
    P, Na = _cal_shapes(V, M, g)
    loss = torch.empty((P, 2), dtype=torch.float64, device=V.device)
    grad = torch.empty_like(g) if want_grad else None
    wsb = _lib.afc_calibrate_workspace_bytes(Na, P)
    workspace = _workspace(workspace, wsb, V.device)
    if flags is None and weights is None:
        _check(_lib.afc_calibrate_grad(Na, P, _ptr(V), _ptr(M), _ptr(g), _ptr(loss), _ptr(grad), _ptr(workspace),
                                       _stream(V, M, g, loss, grad, workspace)), "afc_calibrate_grad")
    else:
        _cal_weights(P, Na, flags, weights)
        _check(_lib.afc_calibrate_grad_weighted(Na, P, _ptr(V), _ptr(M), _ptr(flags), _ptr(weights), _ptr(g),
                                                _ptr(loss), _ptr(grad), _ptr(workspace),
                                                _stream(V, M, flags, weights, g, loss, grad, workspace)),
               "afc_calibrate_grad_weighted")
    return loss, grad


CAL_NOALLOC_MAX_BYTES = 16 << 20


def calibrate_grad_noalloc(V, M, g, loss, grad=None):
    """afc_calibrate_grad_noalloc: as calibrate_grad into caller-provided
    loss float64 [P][2] and grad float32 [P][Na][2][2] (or None), with the
    library's fixed per-GPU scratch instead of a workspace.  Allocates
    nothing; calls that overlap on one GPU race."""
    torch = _torch()
    P, Na = _cal_shapes(V, M, g)
    _require(loss, torch.float64, "loss", (P, 2))
    if grad is not None:
        _require(grad, torch.float32, "grad", (P, Na, 2, 2))
    _check(_lib.afc_calibrate_grad_noalloc(Na, P, _ptr(V), _ptr(M), _ptr(g), _ptr(loss), _ptr(grad),
                                           _stream(V, M, g, loss, grad)), "afc_calibrate_grad_noalloc")
    return loss, grad


def calibrate_solve(V, M, g, n_iter: int = 40, want_loss: bool = True, workspace=None, flags=None,
                    weights=None):
    """Gains minimising ||V - G M G^H||_F^2 per (channel, XX/YY): g float32
    [P][Na][2][2] is updated in place (initial gains in, phase-referenced
    solution out).  Returns the loss float64 [P][2] of the solution (or None).
    flags / weights as in calibrate_grad select the weighted loss."""
    torch = _torch()
    P, Na = _cal_shapes(V, M, g)
    loss = torch.empty((P, 2), dtype=torch.float64, device=V.device) if want_loss else None
    wsb = _lib.afc_calibrate_solve_workspace_bytes(Na, P)
    workspace = _workspace(workspace, wsb, V.device)
    if flags is None and weights is None:
        _check(_lib.afc_calibrate_solve(Na, P, _ptr(V), _ptr(M), _ptr(g), int(n_iter), _ptr(loss), _ptr(workspace),
                                        _stream(V, M, g, loss, workspace)), "afc_calibrate_solve")
    else:
        _cal_weights(P, Na, flags, weights)
        _check(_lib.afc_calibrate_solve_weighted(Na, P, _ptr(V), _ptr(M), _ptr(flags), _ptr(weights), _ptr(g),
                                                 int(n_iter), _ptr(loss), _ptr(workspace),
                                                 _stream(V, M, flags, weights, g, loss, workspace)),
               "afc_calibrate_solve_weighted")
    return loss


def sigma_clip(V, threshold: float = 5.0, out=None, workspace=None):
    """Two-stage sigma clipping of XX / YY: V float32 [P][Nbl][2][2][2] -> uint8 flags [P][Nbl][2]."""
    torch = _torch()
    if V.dim() != 5:
        raise AfcError("sigma_clip: V must be [P][Nbl][2][2][2]")
    P, nbl = V.shape[0], V.shape[1]
    Na = int(round(((8 * nbl + 1) ** 0.5 - 1) / 2))
    if Na * (Na + 1) // 2 != nbl:
        raise AfcError(f"sigma_clip: {nbl} is not a baseline count Na(Na+1)/2")
    _require(V, torch.float32, "V", (P, nbl, 2, 2, 2))
    if out is None:
        out = torch.empty((P, nbl, 2), dtype=torch.uint8, device=V.device)
    _require(out, torch.uint8, "out", (P, nbl, 2))
    wsb = _lib.afc_sigma_clip_workspace_bytes(Na, P)
    workspace = _workspace(workspace, wsb, V.device)
    _check(_lib.afc_sigma_clip(Na, P, _ptr(V), float(threshold), _ptr(out), _ptr(workspace), _stream(V, out, workspace)),
           "afc_sigma_clip")
    return out


def apply_vis_flags(flags, V=None, M=None):
    """Zero, in place, the flagged XX / YY entries of V and / or M."""
    torch = _torch()
    if flags.dim() != 3:
        raise AfcError(f"flags shape {tuple(flags.shape)} is not [P][Nbl][2]")
    P, nbl = flags.shape[0], flags.shape[1]
    Na = int(round(((8 * nbl + 1) ** 0.5 - 1) / 2))
    if Na * (Na + 1) // 2 != nbl:
        raise AfcError(f"apply_vis_flags: {nbl} is not a baseline count Na(Na+1)/2")
    _require(flags, torch.uint8, "flags", (P, nbl, 2))
    for t, n in ((V, "V"), (M, "M")):
        if t is not None:
            _require(t, torch.float32, n, (P, nbl, 2, 2, 2))
    _check(_lib.afc_apply_vis_flags(Na, P, _ptr(flags), _ptr(V), _ptr(M), _stream(flags, V, M)),
           "afc_apply_vis_flags")


class Imager:
    """Bilinear gridding of calibrated visibilities and the snapshot image
    (afc_grid_visibilities + afc_image_from_grid) for one array: positions
    float64 [Na][2] metres, grid N x N cells of `cell_wavelengths`."""

    def __init__(self, positions, n_subbands: int, grid_size: int, cell_wavelengths: float = 0.5):
        torch = _torch()
        if positions.dim() != 2:
            raise AfcError(f"positions shape {tuple(positions.shape)} is not [Na][2]")
        _require(positions, torch.float64, "positions", (positions.shape[0], 2))
        self.Na = positions.shape[0]
        self.B = int(n_subbands)
        self.N = int(grid_size)
        self.du = float(cell_wavelengths)
        self.pos = positions
        wsb = _lib.afc_imaging_workspace_bytes(self.Na, self.B, self.N)
        if wsb == 0:
            raise AfcError(f"imaging: unsupported shape (Na={self.Na}, B={self.B}, N={self.N})")
        self.ws = torch.empty(wsb, dtype=torch.uint8, device=positions.device)
        self.norm = torch.empty(1, dtype=torch.float64, device=positions.device)

    def grid(self, vis, freq_hz, weights=None, out=None):
        """vis float32 [B][64][Nbl][2][2][2], freq_hz float64 [B][64] -> complex grid float32 [N][N][2]."""
        torch = _torch()
        nbl = self.Na * (self.Na + 1) // 2
        dev = self.pos.device
        _require(vis, torch.float32, "vis", (self.B, N_CHANNELS, nbl, 2, 2, 2))
        _require(freq_hz, torch.float64, "freq_hz", (self.B, N_CHANNELS))
        if weights is not None:
            _require(weights, torch.int32, "weights", (self.B, nbl))
        if out is None:
            out = torch.empty((self.N, self.N, 2), dtype=torch.float32, device=dev)
        _require(out, torch.float32, "out", (self.N, self.N, 2))
        _check(_lib.afc_grid_visibilities(self.Na, self.B, _ptr(vis), _ptr(weights), _ptr(self.pos), _ptr(freq_hz),
                                          self.N, self.du, _ptr(out), _ptr(self.norm), _ptr(self.ws),
                                          _stream(self.pos, vis, weights, freq_hz, out)), "afc_grid_visibilities")
        return out

    def image(self, grid, out=None):
        """grid float32 [N][N][2] (from grid()) -> image float32 [N][N], normalised by the gridded weight."""
        torch = _torch()
        dev = self.pos.device
        _require(grid, torch.float32, "grid", (self.N, self.N, 2))
        if out is None:
            out = torch.empty((self.N, self.N), dtype=torch.float32, device=dev)
        _require(out, torch.float32, "out", (self.N, self.N))
        _check(_lib.afc_image_from_grid(self.N, _ptr(grid), _ptr(self.norm), _ptr(out), _ptr(self.ws),
                                        _stream(self.pos, grid, out)), "afc_image_from_grid")
        return out


def _make_cal_loss():
    torch = _torch()

    class CalLoss(torch.autograd.Function):
        """L[k][pol] = ||V - G M G^H||_F^2 with the hand-written adjoint kernel.

        g is complex64 [P][Na][2]; V, M float32 [P][Nbl][2][2][2]; optional
        flags / weights [P][Nbl][2] select the weighted loss.  The forward
        kernel computes the gradient together with the loss; the backward
        scales it by the incoming gradient of each (channel, pol).
        """

        @staticmethod
        def forward(ctx, V, M, g, flags=None, weights=None):
            gr = torch.view_as_real(g.contiguous())
            loss, grad = calibrate_grad(V, M, gr, want_grad=True, flags=flags, weights=weights)
            ctx.save_for_backward(torch.view_as_complex(grad))
            return loss

        @staticmethod
        def backward(ctx, grad_out):
            (grad,) = ctx.saved_tensors
            gg = grad * grad_out.to(torch.float32)[:, None, :]
            return None, None, gg, None, None

    return CalLoss


_cal_loss_cls = None


def cal_loss(V, M, g, flags=None, weights=None):
    """Differentiable calibration loss [P][2] (float64) with respect to complex
    g; with flags / weights the weighted loss."""
    global _cal_loss_cls
    if _cal_loss_cls is None:
        _cal_loss_cls = _make_cal_loss()
    return _cal_loss_cls.apply(V, M, g, flags, weights)


@dataclass
class PlanInfo:
    tile: int
    n_workgroups: int
    n_work_items: int


class Plan:
    """Batching form: one graph of one channeliser launch and one correlator launch per sample-type family."""

    def __init__(self, n_antennas: int, n_spectra_per_sb: Sequence[int], dtypes: Sequence[str],
                 tune_cache: Optional[str] = None, n_spectra: Optional[int] = None):
        """n_spectra: the row count of x is (n_spectra + 15) * 64 (default max of n_spectra_per_sb)."""
        B = len(n_spectra_per_sb)
        self.n_antennas = n_antennas
        self.S = [int(s) for s in n_spectra_per_sb]
        self.dtypes = list(dtypes)
        self.dims = dims(n_antennas, B, max(self.S) if n_spectra is None else int(n_spectra))
        dt = (C.c_int * B)(*[DTYPES[t] for t in self.dtypes])
        sp = (C.c_int32 * B)(*self.S)
        h = C.c_void_p()
        _check(_lib.afc_plan_create(C.byref(self.dims), C.cast(dt, C.c_void_p), C.cast(sp, C.c_void_p),
                                    tune_cache.encode() if tune_cache else None, C.byref(h)), "afc_plan_create")
        self._h = h

    @property
    def workspace_bytes(self) -> int:
        return int(_lib.afc_plan_workspace_bytes(self._h))

    def info(self) -> PlanInfo:
        a, b, c, d = _i32(), _i32(), _i32(), _i32()
        _check(_lib.afc_plan_info(self._h, C.byref(a), C.byref(b), C.byref(c), C.byref(d)), "afc_plan_info")
        return PlanInfo(a.value, c.value, d.value)

    def launch(self, x, taps, gains, workspace, vis, flags=None, weights=None):
        """x int16 [B][L][Na][2][2]; gains host [B] (int8 subbands); workspace
        uint8 of workspace_bytes; vis int32 or float32 [B][64][Nbl][2][2][2]
        (8 bytes per complex value whatever each subband's type); flags uint8
        [B][Na] or None; weights int32 [B][Nbl] or None."""
        torch = _torch()
        if not getattr(self, "_h", None):
            raise AfcError("plan is closed")
        B, Na = len(self.S), self.n_antennas
        nbl = Na * (Na + 1) // 2
        rows = (self.dims.n_spectra + N_TAPS - 1) * N_CHANNELS
        if x.dim() < 3 or x.shape[0] != B or x.shape[1] != rows or x[0, 0].numel() != 4 * Na:
            raise AfcError(f"x must be [{B}][{rows}][{Na}][2][2]: got {tuple(x.shape)}")
        _require(x, torch.int16, "x")
        dev = x.device
        _require(taps, torch.float32, "taps", (N_TAPS * N_CHANNELS,))
        if vis.dtype not in (torch.int32, torch.float32):
            raise AfcError(f"vis must be int32 or float32, got {vis.dtype}")
        _require(vis, vis.dtype, "vis", visibility_shape(B, Na))
        if flags is not None:
            _require(flags, torch.uint8, "flags", (B, Na))
        if weights is not None:
            _require(weights, torch.int32, "weights", (B, nbl))
        _workspace(workspace, self.workspace_bytes, dev)
        if len(gains) != B:
            raise AfcError(f"gains has {len(gains)} entries, expected {B}")
        g = (C.c_float * B)(*[float(v) for v in gains])
        _check(_lib.afc_plan_launch(self._h, _ptr(x), _ptr(taps), C.cast(g, C.c_void_p), _ptr(workspace),
                                    _ptr(flags), _ptr(vis), _ptr(weights), _stream(x, taps, workspace, flags, vis, weights)), "afc_plan_launch")

    def close(self):
        if getattr(self, "_h", None):
            _lib.afc_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
