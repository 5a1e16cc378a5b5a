"""C-ABI checks that need no GPU: the library loads, exports every entry point
declared in include/afc.h, sizes its buffers correctly and rejects invalid
arguments on the host before anything is launched."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "afc.h")


def _declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"AFC_API\s+[\w\s\*]+?\b(afc_\w+)\s*\(", src)))


@pytest.fixture(scope="module")
def afc():
    import paper_1609_04205_amd as afc
    return afc


def test_header_declares_entry_points():
    names = _declared()
    for n in ["afc_channelise", "afc_correlate", "afc_calibrate_grad", "afc_plan_create", "afc_plan_launch",
              "afc_plan_destroy", "afc_last_error"]:
        assert n in names


def test_library_exports_every_declared_symbol(afc):
    lib = C.CDLL(afc.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(afc.EXPORTS) == _declared()


def test_sizes(afc):
    d = afc.dims(576, 16, 3051)
    Sb = (3051 + 7) // 8
    assert afc._lib.afc_channelised_bytes(C.byref(d), afc.AFC_I8) == 16 * 64 * Sb * 1152 * 8 * 2
    assert afc._lib.afc_channelised_bytes(C.byref(d), afc.AFC_F32) == 16 * 64 * Sb * 1152 * 8 * 8
    assert afc._lib.afc_visibility_bytes(C.byref(d)) == 16 * 64 * (576 * 577 // 2) * 32
    bad = afc.dims(576, 16, 3051, n_channels=256)
    assert afc._lib.afc_channelised_bytes(C.byref(bad), afc.AFC_I8) == 0
    assert afc._lib.afc_calibrate_workspace_bytes(576, 64) > 0
    assert afc._lib.afc_calibrate_workspace_bytes(0, 64) == 0


def test_size_limits(afc):
    """4096 antennas is the largest array; one subband holds below 2^31 int16
    input values, so 4096 antennas allow 2032 spectra and not 2033."""
    lib = afc._lib
    ok = afc.dims(4096, 1, 2032)
    assert lib.afc_channelised_bytes(C.byref(ok), afc.AFC_F32) == 64 * 254 * 8192 * 8 * 8
    assert lib.afc_channelised_bytes(C.byref(afc.dims(4096, 1, 2033)), afc.AFC_F32) == 0
    assert lib.afc_visibility_bytes(C.byref(afc.dims(4096, 1, 20))) == 64 * (4096 * 4097 // 2) * 32
    assert lib.afc_visibility_bytes(C.byref(afc.dims(4097, 1, 20))) == 0
    dummy = C.c_void_p(0x1000)          # never dereferenced: validation fails first
    too_long = afc.dims(4096, 1, 2033)
    assert lib.afc_channelise(C.byref(too_long), dummy, dummy, afc.AFC_F32, 1.0, dummy, None) == -2
    assert b"2^31" in lib.afc_last_error()


def test_invalid_arguments_are_rejected_on_host(afc):
    lib = afc._lib
    d = afc.dims(48, 1, 1024)
    dummy = C.c_void_p(0x1000)          # never dereferenced: validation fails first
    assert lib.afc_channelise(None, dummy, dummy, afc.AFC_F32, 1.0, dummy, None) == -1
    assert b"dims" in lib.afc_last_error()
    assert lib.afc_channelise(C.byref(d), None, dummy, afc.AFC_F32, 1.0, dummy, None) == -1
    assert lib.afc_channelise(C.byref(d), dummy, dummy, 7, 1.0, dummy, None) == -1
    assert lib.afc_channelise(C.byref(d), dummy, dummy, afc.AFC_I8, 0.0, dummy, None) == -1
    p256 = afc.dims(48, 1, 1024, n_channels=256)
    assert lib.afc_channelise(C.byref(p256), dummy, dummy, afc.AFC_F32, 1.0, dummy, None) == -2
    t8 = afc.dims(48, 1, 1024, n_taps=8)
    assert lib.afc_correlate(C.byref(t8), afc.AFC_F32, dummy, None, None, dummy, None, None) == -2
    pol1 = afc.Dims(48, 1, 1, 64, 16, 1024)
    assert lib.afc_correlate(C.byref(pol1), afc.AFC_F32, dummy, None, None, dummy, None, None) == -2
    s_bad = (C.c_int32 * 1)(2000)
    assert lib.afc_correlate(C.byref(d), afc.AFC_F32, dummy, C.cast(s_bad, C.c_void_p), None, dummy, None, None) == -1
    odd = C.c_void_p(0x1008)           # 8- but not 16-byte aligned: the visibility stores are 16 bytes wide
    assert lib.afc_correlate(C.byref(d), afc.AFC_F32, dummy, None, None, odd, None, None) == -1
    assert b"aligned" in lib.afc_last_error()
    big = afc.dims(48, 1, 70000)       # int8 sums could overflow int32
    assert lib.afc_correlate(C.byref(big), afc.AFC_I8, dummy, None, None, dummy, None, None) == -2
    assert lib.afc_calibrate_grad(48, 4, dummy, dummy, dummy, dummy, None, None, None) == -4
    assert lib.afc_calibrate_grad(0, 4, dummy, dummy, dummy, dummy, None, dummy, None) == -1
    # weighted calibration: flags 2-byte and weights 8-byte aligned
    f_odd, w_odd = C.c_void_p(0x1001), C.c_void_p(0x1004)
    assert lib.afc_calibrate_grad_weighted(48, 4, dummy, dummy, f_odd, None, dummy, dummy, None, dummy, None) == -1
    assert b"aligned" in lib.afc_last_error()
    assert lib.afc_calibrate_solve_weighted(48, 4, dummy, dummy, None, w_odd, dummy, 5, None, dummy, None) == -1
    assert b"aligned" in lib.afc_last_error()
    assert lib.afc_calibrate_solve_weighted(48, 4, dummy, dummy, None, None, dummy, -1, None, dummy, None) == -1
    out = C.c_void_p()
    assert lib.afc_plan_create(C.byref(d), None, None, None, C.byref(out)) == -1
    assert not out.value


def test_fine_channeliser_sizes_and_argument_checks(afc):
    lib = afc._lib
    d = afc.dims(576, 16, 762)
    N, B = 1152, 16
    assert lib.afc_channelise_fine_workspace_bytes(C.byref(d)) == (256 + N * 256 + B * N) * 8
    bad = afc.dims(576, 16, 762, n_channels=256)
    assert lib.afc_channelise_fine_workspace_bytes(C.byref(bad)) == 0
    dummy = C.c_void_p(0x1000)          # never dereferenced: validation fails first
    nu = (C.c_double * 16)(*([60e6] * 16))
    ok = dict(x=dummy, taps=dummy, delays=dummy, bp=dummy, nu=nu, width=195312.5, dt=afc.AFC_F32, gain=1.0,
              ws=dummy, out=dummy)

    def call(dims=d, **kw):
        a = dict(ok, **kw)
        return lib.afc_channelise_fine(C.byref(dims), a["x"], a["taps"], a["delays"], a["bp"], a["nu"],
                                       a["width"], a["dt"], a["gain"], a["ws"], a["out"], None)

    assert call(delays=None) == -1
    assert call(bp=None) == -1
    assert call(nu=None) == -1
    assert call(ws=None) == -4
    assert call(width=0.0) == -1
    assert call(width=float("nan")) == -1
    assert call(dt=afc.AFC_I8, gain=0.0) == -1
    assert call(dt=9) == -1
    nan_nu = (C.c_double * 16)(*([float("inf")] * 16))
    assert call(nu=nan_nu) == -1
    assert call(dims=bad) == -2
    # (S + 15) * 256 rows of 2 N int16 values must stay below 2^31 per subband
    huge = afc.dims(576, 1, 4000)
    assert call(dims=huge) == -2
    assert b"2^31" in lib.afc_last_error()


def _meta(shape, dtype):
    import torch
    return torch.empty(shape, dtype=dtype, device="meta")


def _raises(afc, fn, *words):
    with pytest.raises(afc.AfcError) as e:
        fn()
    msg = str(e.value)
    for w in words:
        assert w in msg, msg
    return msg


def test_binding_rejects_wrong_buffer_sizes_on_host(afc):
    """Every caller buffer's size is checked before its device: a buffer of
    the wrong shape is an AfcError naming the shape, never a launch.  (Meta
    tensors carry shapes without memory; a buffer of the right shape then
    fails only because it is not on a GPU.)"""
    import torch
    B, Na, S = 2, 6, 20
    N, nbl = 2 * Na, Na * (Na + 1) // 2
    z = _meta(afc.channelised_shape(B, S, N), torch.int8)
    vis_ok = _meta(afc.visibility_shape(B, Na), torch.int32)
    # correlate: out, weights, flags, per-subband S
    _raises(afc, lambda: afc.correlate(z, S, out=_meta(afc.visibility_shape(B, Na - 1), torch.int32)), "out shape")
    _raises(afc, lambda: afc.correlate(z, S, out=vis_ok, weights=_meta((B, nbl + 1), torch.int32)), "weights shape")
    _raises(afc, lambda: afc.correlate(z, S, out=vis_ok, flags=_meta((B, Na + 1), torch.uint8)), "flags shape")
    _raises(afc, lambda: afc.correlate(z, S, n_spectra_per_sb=[S], out=vis_ok), "entries")
    _raises(afc, lambda: afc.correlate(z, S, out=_meta(afc.visibility_shape(B, Na), torch.float32)), "int32")
    _raises(afc, lambda: afc.correlate(z, S + 8), "blocks")
    _raises(afc, lambda: afc.correlate(z, S, out=vis_ok), "GPU tensor")          # right sizes: only the device
    # zero_invalid: block count of z against n_spectra, validity words
    sv = _meta(afc.validity_shape(B, S, Na), torch.int32)
    _raises(afc, lambda: afc.zero_invalid(z, sv, S + 16), "z shape")
    _raises(afc, lambda: afc.zero_invalid(z, _meta(afc.validity_shape(B, S + 40, Na), torch.int32), S),
            "spec_valid shape")
    # validity weights and normalisation
    _raises(afc, lambda: afc.validity_weights(sv, S, out=_meta((B, nbl - 1), torch.int32)), "out shape")
    _raises(afc, lambda: afc.validity_weights(sv, S, out=_meta((B, nbl), torch.int32),
                                              flags=_meta((B, 3), torch.uint8)), "flags shape")
    _raises(afc, lambda: afc.normalise_visibilities(vis_ok, _meta((B, nbl - 1), torch.int32)), "weights shape")
    _raises(afc, lambda: afc.normalise_visibilities(vis_ok, _meta((B, nbl), torch.int32),
                                                    out=_meta(afc.visibility_shape(B + 1, Na), torch.float32)),
            "out shape")
    # channelise: taps and out
    x = _meta((B, (S + 15) * 64, Na, 2, 2), torch.int16)
    _raises(afc, lambda: afc.channelise(x, _meta((1000,), torch.float32), S), "taps shape")
    _raises(afc, lambda: afc.channelise(x, _meta((1024,), torch.float32), S, "i8",
                                        out=_meta(afc.channelised_shape(B, S + 8, N), torch.int8)), "out shape")
    # calibration: V, M, g, workspace
    P = 3
    g = _meta((P, Na, 2, 2), torch.float32)
    V = _meta((P, nbl, 2, 2, 2), torch.float32)
    _raises(afc, lambda: afc.calibrate_grad(_meta((P, nbl + 1, 2, 2, 2), torch.float32), V, g), "V shape")
    _raises(afc, lambda: afc.calibrate_grad(V, _meta((P - 1, nbl, 2, 2, 2), torch.float32), g), "M shape")
    _raises(afc, lambda: afc.calibrate_solve(V, V, _meta((P, Na, 2), torch.float32)), "g shape")
    _raises(afc, lambda: afc.calibrate_grad(V, V, g, flags=_meta((P, nbl, 3), torch.uint8)), "flags shape")
    _raises(afc, lambda: afc.calibrate_solve(V, V, g, weights=_meta((P, nbl + 1, 2), torch.float32)),
            "weights shape")
    _raises(afc, lambda: afc.calibrate_grad(V, V, g, weights=_meta((P, nbl, 2), torch.float64)), "float32")
    _raises(afc, lambda: afc.sigma_clip(V, out=_meta((P, nbl, 3), torch.uint8)), "out shape")
    _raises(afc, lambda: afc.apply_vis_flags(_meta((P, nbl, 2), torch.uint8), V=_meta((P, nbl, 2, 2), torch.float32)),
            "V shape")


def test_plan_launch_rejects_wrong_buffer_sizes_on_host(afc):
    """Plan.launch checks x, taps, vis, weights, flags, gains and the
    workspace before calling the library (the plan's handle is never reached
    here: every call below fails first)."""
    import torch
    B, Na, S = 2, 6, 40
    nbl = Na * (Na + 1) // 2

    class FakePlan(afc.Plan):
        workspace_bytes = 1000

        def __init__(self):
            self._h = C.c_void_p(1)
            self.n_antennas, self.S, self.dims = Na, [S, S], afc.dims(Na, B, S)

        def close(self):
            self._h = None

    plan = FakePlan()
    try:
        x = _meta((B, (S + 15) * 64, Na, 2, 2), torch.int16)
        taps = _meta((1024,), torch.float32)
        ws = _meta((1000,), torch.uint8)
        vis = _meta(afc.visibility_shape(B, Na), torch.int32)
        g = [1.0, 1.0]
        _raises(afc, lambda: plan.launch(_meta((B, (S + 15) * 64 - 1, Na, 2, 2), torch.int16), taps, g, ws, vis),
                "x must be")
        _raises(afc, lambda: plan.launch(x, _meta((512,), torch.float32), g, ws, vis), "taps shape")
        _raises(afc, lambda: plan.launch(x, taps, g, ws, _meta(afc.visibility_shape(B, Na + 1), torch.int32)),
                "vis shape")
        _raises(afc, lambda: plan.launch(x, taps, g, ws, vis, flags=_meta((B, Na - 1), torch.uint8)), "flags shape")
        _raises(afc, lambda: plan.launch(x, taps, g, ws, vis, weights=_meta((B + 1, nbl), torch.int32)),
                "weights shape")
        _raises(afc, lambda: plan.launch(x, taps, g, _meta((999,), torch.uint8), vis), "workspace holds")
        _raises(afc, lambda: plan.launch(x, taps, [1.0], ws, vis), "gains has")
        _raises(afc, lambda: plan.launch(x, taps, g, ws, vis), "GPU tensor")     # right sizes: only the device
    finally:
        plan.close()


def test_degenerate_sizes_are_rejected_on_host(afc):
    """No antennas, no subbands or no spectra (and negative sizes) are
    invalid arguments (the header asks Na >= 1, 1 <= B <= 256, S >= 1) for the
    channeliser and the correlator, with a message naming the size; the size
    queries return 0 for them."""
    lib = afc._lib
    dummy = C.c_void_p(0x1000)          # never dereferenced: validation fails first
    for (Na, B, S, word) in [(0, 1, 16, b"n_antennas"), (-1, 1, 16, b"n_antennas"), (48, 0, 16, b"n_subbands"),
                             (48, 257, 16, b"n_subbands"), (48, 1, 0, b"n_spectra")]:
        d = afc.Dims(Na, 2, B, 64, 16, S)
        assert lib.afc_channelise(C.byref(d), dummy, dummy, afc.AFC_I8, 1.0, dummy, None) == -1
        assert word in lib.afc_last_error()
        assert lib.afc_correlate(C.byref(d), afc.AFC_I8, dummy, None, None, dummy, None, None) == -1
        assert word in lib.afc_last_error()
        assert lib.afc_channelised_bytes(C.byref(d), afc.AFC_I8) == 0
        assert lib.afc_visibility_bytes(C.byref(d)) == 0
