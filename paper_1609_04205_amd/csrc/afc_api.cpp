// C ABI of the FX-correlator library: argument checks, launch set-up, the
// batching plan (XCD-balanced work lists, HIP graph replay and
// the tile tuner).  See include/afc.h for the contract of each entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <initializer_list>
#include <map>
#include <queue>
#include <sstream>
#include <string>
#include <vector>

#include "afc_internal.h"

using namespace afc;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(AFC_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

// Checked mode: refuse non-finite floating-point inputs (counted on the
// device; the call then waits for its stream).  No-op when the mode is off.
struct FloatInput {
    const void* p;
    size_t n;          // values
    int kind;          // afc_value_type
    const char* name;
};
int check_inputs(std::initializer_list<FloatInput> ins, hipStream_t stream) {
    if (!checked_mode()) return AFC_OK;
    for (const FloatInput& in : ins) {
        if (!in.p || in.n == 0) continue;
        unsigned long long c = 0;
        const hipError_t e = count_nonfinite(in.p, in.n, in.kind, &c, stream);
        if (e != hipSuccess) return hip_fail(e, "checked mode");
        if (c) return fail(AFC_ERR_INVALID, "checked mode: %llu non-finite values in %s", c, in.name);
    }
    return AFC_OK;
}

int check_dims(const afc_dims* d) {
    if (!d) return fail(AFC_ERR_INVALID, "dims is NULL");
    if (d->n_antennas < 1) return fail(AFC_ERR_INVALID, "n_antennas = %d < 1", d->n_antennas);
    if (d->n_pols != 2) return fail(AFC_ERR_UNSUPPORTED, "n_pols = %d (only 2 is built)", d->n_pols);
    if (d->n_subbands < 1 || d->n_subbands > AFC_MAX_SUBBANDS)
        return fail(AFC_ERR_INVALID, "n_subbands = %d outside 1..%d", d->n_subbands, AFC_MAX_SUBBANDS);
    if (d->n_channels != kP) return fail(AFC_ERR_UNSUPPORTED, "n_channels = %d (only 64 is built)", d->n_channels);
    if (d->n_taps != kT) return fail(AFC_ERR_UNSUPPORTED, "n_taps = %d (only 16 is built)", d->n_taps);
    if (d->n_spectra < 1) return fail(AFC_ERR_INVALID, "n_spectra = %d < 1", d->n_spectra);
    const int64_t N = 2LL * d->n_antennas;
    const int64_t L = ((int64_t)d->n_spectra + kT - 1) * kP;
    if (L * N * 2 >= (1LL << 31))
        return fail(AFC_ERR_UNSUPPORTED, "one subband of input holds %lld int16 values (limit 2^31)",
                    (long long)(L * N * 2));
    if (N > 8192) return fail(AFC_ERR_UNSUPPORTED, "n_antennas = %d > 4096", d->n_antennas);
    return AFC_OK;
}

bool dtype_ok(afc_dtype t) { return t == AFC_F32 || t == AFC_F16 || t == AFC_I8; }

int64_t blocks_of(int64_t S) { return ceil_div(S, kSBlk); }

// samples of one subband of z
int64_t z_sb_samples(int64_t N, int64_t S) { return (int64_t)kP * blocks_of(S) * N * kSBlk; }

int64_t nbl_of(int64_t Na) { return Na * (Na + 1) / 2; }

}  // namespace

extern "C" {

AFC_API const char* afc_last_error(void) { return g_err.c_str(); }

AFC_API void afc_set_checked_mode(int on) { set_checked_mode(on != 0); }

AFC_API int afc_checked_mode(void) { return checked_mode() ? 1 : 0; }

AFC_API int afc_count_nonfinite(const void* values, size_t n, afc_value_type type, uint64_t* count,
                                hipStream_t stream) {
    g_err.clear();
    if (!count) return fail(AFC_ERR_INVALID, "count is NULL");
    *count = 0;
    if (n == 0) return AFC_OK;
    if (!values) return fail(AFC_ERR_INVALID, "values is NULL");
    if (type != AFC_VALUES_F32 && type != AFC_VALUES_F16 && type != AFC_VALUES_F64)
        return fail(AFC_ERR_INVALID, "unknown value type %d", (int)type);
    unsigned long long c = 0;
    const hipError_t e = count_nonfinite(values, n, type, &c, stream);
    if (e != hipSuccess) return hip_fail(e, "non-finite count");
    *count = (uint64_t)c;
    return AFC_OK;
}

AFC_API size_t afc_channelised_bytes(const afc_dims* d, afc_dtype dt) {
    if (check_dims(d) != AFC_OK || !dtype_ok(dt)) return 0;
    return (size_t)d->n_subbands * z_sb_samples(2LL * d->n_antennas, d->n_spectra) * sample_bytes(dt);
}

AFC_API size_t afc_visibility_bytes(const afc_dims* d) {
    if (check_dims(d) != AFC_OK) return 0;
    return (size_t)d->n_subbands * kP * nbl_of(d->n_antennas) * 4 * 8;
}

AFC_API int afc_channelise(const afc_dims* d, const int16_t* x, const float* taps, afc_dtype out_dtype,
                           float requant_gain, void* out, hipStream_t stream) {
    g_err.clear();
    int rc = check_dims(d);
    if (rc != AFC_OK) return rc;
    if (!x || !taps || !out) return fail(AFC_ERR_INVALID, "NULL pointer (x, taps or out)");
    if (!dtype_ok(out_dtype)) return fail(AFC_ERR_INVALID, "unknown out_dtype %d", (int)out_dtype);
    if (out_dtype == AFC_I8 && !(std::isfinite(requant_gain) && requant_gain > 0.0f))
        return fail(AFC_ERR_INVALID, "requant_gain must be finite and > 0 for AFC_I8");
    const int64_t N = 2LL * d->n_antennas;
    const int64_t z_sb = z_sb_samples(N, d->n_spectra);
    if (z_sb * sample_bytes(out_dtype) >= (1LL << 40)) return fail(AFC_ERR_UNSUPPORTED, "output too large");
    rc = check_inputs({{taps, (size_t)kT * kP, AFC_VALUES_F32, "taps"}}, stream);
    if (rc != AFC_OK) return rc;
    PpfLaunch a{};
    a.x = x;
    a.taps = taps;
    a.z = out;
    a.x_sb_stride = ((int64_t)d->n_spectra + kT - 1) * kP * N * 2;
    a.z_sb_stride = z_sb;
    a.N = (int)N;
    a.S = d->n_spectra;
    a.Sb = (int)blocks_of(d->n_spectra);
    a.B = d->n_subbands;
    a.gain = requant_gain;
    a.dt = out_dtype;
    hipError_t e = launch_ppf(a, stream);
    if (e != hipSuccess) return hip_fail(e, "channeliser launch");
    return AFC_OK;
}

namespace {
// int16 values of one subband of fine-channeliser input: (S + T - 1) * 256 rows
int64_t fine_x_values(const afc_dims* d) {
    return ((int64_t)d->n_spectra + kT - 1) * kPFine * 2LL * d->n_antennas * 2;
}
}  // namespace

AFC_API size_t afc_channelise_fine_workspace_bytes(const afc_dims* d) {
    if (check_dims(d) != AFC_OK) return 0;
    return fine_workspace_bytes(2 * d->n_antennas, d->n_subbands);
}

AFC_API int afc_channelise_fine(const afc_dims* d, const int16_t* x, const float* taps, const double* delays,
                                const float* bandpass, const double* center_hz, double subband_width_hz,
                                afc_dtype out_dtype, float requant_gain, void* workspace, void* out,
                                hipStream_t stream) {
    g_err.clear();
    int rc = check_dims(d);
    if (rc != AFC_OK) return rc;
    if (!x || !taps || !delays || !bandpass || !center_hz || !out)
        return fail(AFC_ERR_INVALID, "NULL pointer (x, taps, delays, bandpass, center_hz or out)");
    if (!workspace) return fail(AFC_ERR_WORKSPACE, "workspace is NULL");
    if (!dtype_ok(out_dtype)) return fail(AFC_ERR_INVALID, "unknown out_dtype %d", (int)out_dtype);
    if (out_dtype == AFC_I8 && !(std::isfinite(requant_gain) && requant_gain > 0.0f))
        return fail(AFC_ERR_INVALID, "requant_gain must be finite and > 0 for AFC_I8");
    if (!(std::isfinite(subband_width_hz) && subband_width_hz > 0.0))
        return fail(AFC_ERR_INVALID, "subband_width_hz must be finite and > 0");
    for (int b = 0; b < d->n_subbands; ++b)
        if (!std::isfinite(center_hz[b])) return fail(AFC_ERR_INVALID, "center_hz[%d] is not finite", b);
    if (fine_x_values(d) >= (1LL << 31))
        return fail(AFC_ERR_UNSUPPORTED, "one subband of input holds %lld int16 values (limit 2^31)",
                    (long long)fine_x_values(d));
    const int64_t N = 2LL * d->n_antennas;
    const int64_t z_sb = z_sb_samples(N, d->n_spectra);
    if (z_sb * sample_bytes(out_dtype) >= (1LL << 40)) return fail(AFC_ERR_UNSUPPORTED, "output too large");
    rc = check_inputs({{taps, (size_t)kT * kPFine, AFC_VALUES_F32, "taps"},
                       {bandpass, (size_t)kPFine, AFC_VALUES_F32, "bandpass"},
                       {delays, (size_t)N, AFC_VALUES_F64, "delays"}},
                      stream);
    if (rc != AFC_OK) return rc;
    FineLaunch l{};
    l.x = x;
    l.taps = taps;
    l.tau = delays;
    l.bandpass = bandpass;
    l.nu_center = center_hz;
    l.subband_hz = subband_width_hz;
    l.workspace = workspace;
    l.z = out;
    l.x_sb_stride = fine_x_values(d);
    l.z_sb_stride = z_sb;
    l.N = (int)N;
    l.S = d->n_spectra;
    l.Sb = (int)blocks_of(d->n_spectra);
    l.B = d->n_subbands;
    l.gain = requant_gain;
    l.dt = out_dtype;
    hipError_t e = launch_ppf_fine(l, stream);
    if (e != hipSuccess) return hip_fail(e, "fine channeliser launch");
    return AFC_OK;
}

AFC_API size_t afc_validity_words(const afc_dims* d) {
    if (check_dims(d) != AFC_OK) return 0;
    return (size_t)d->n_subbands * ceil_div(d->n_spectra, 32) * d->n_antennas;
}

AFC_API int afc_validity(const afc_dims* d, const uint8_t* packet_valid, int32_t n_packets, int32_t packet_samples,
                         int32_t samples_per_spectrum, uint32_t* spec_valid, hipStream_t stream) {
    g_err.clear();
    int rc = check_dims(d);
    if (rc != AFC_OK) return rc;
    if (!packet_valid || !spec_valid) return fail(AFC_ERR_INVALID, "NULL pointer (packet_valid or spec_valid)");
    if (n_packets < 1 || packet_samples < 1)
        return fail(AFC_ERR_INVALID, "n_packets = %d and packet_samples = %d must be >= 1", n_packets, packet_samples);
    if (samples_per_spectrum != kP && samples_per_spectrum != kPFine)
        return fail(AFC_ERR_INVALID, "samples_per_spectrum = %d (64 or 256)", samples_per_spectrum);
    hipError_t e = launch_validity(packet_valid, spec_valid, d->n_subbands, d->n_antennas, d->n_spectra, n_packets,
                                   packet_samples, samples_per_spectrum, stream);
    if (e != hipSuccess) return hip_fail(e, "validity launch");
    return AFC_OK;
}

AFC_API int afc_zero_invalid(const afc_dims* d, afc_dtype dt, const uint32_t* spec_valid, void* z,
                             hipStream_t stream) {
    g_err.clear();
    int rc = check_dims(d);
    if (rc != AFC_OK) return rc;
    if (!spec_valid || !z) return fail(AFC_ERR_INVALID, "NULL pointer (spec_valid or z)");
    if (!dtype_ok(dt)) return fail(AFC_ERR_INVALID, "unknown dtype %d", (int)dt);
    hipError_t e = launch_zero_invalid(spec_valid, z, dt, d->n_subbands, d->n_antennas, d->n_spectra, stream);
    if (e != hipSuccess) return hip_fail(e, "zero-invalid launch");
    return AFC_OK;
}

AFC_API int afc_validity_weights(const afc_dims* d, const uint32_t* spec_valid, const int32_t* n_spectra_per_sb,
                                 const uint8_t* flags, int32_t* weights, hipStream_t stream) {
    g_err.clear();
    int rc = check_dims(d);
    if (rc != AFC_OK) return rc;
    if (!spec_valid || !weights) return fail(AFC_ERR_INVALID, "NULL pointer (spec_valid or weights)");
    if (n_spectra_per_sb)
        for (int b = 0; b < d->n_subbands; ++b)
            if (n_spectra_per_sb[b] < 1 || n_spectra_per_sb[b] > d->n_spectra)
                return fail(AFC_ERR_INVALID, "n_spectra_per_sb[%d] = %d outside 1..%d", b, n_spectra_per_sb[b],
                            d->n_spectra);
    hipError_t e = launch_validity_weights(spec_valid, flags, weights, d->n_subbands, d->n_antennas, d->n_spectra,
                                           n_spectra_per_sb, stream);
    if (e != hipSuccess) return hip_fail(e, "validity-weights launch");
    return AFC_OK;
}

AFC_API int afc_normalise_visibilities(const afc_dims* d, afc_dtype vis_dtype, const void* vis,
                                       const int32_t* weights, void* out, hipStream_t stream) {
    g_err.clear();
    int rc = check_dims(d);
    if (rc != AFC_OK) return rc;
    if (!vis || !weights || !out) return fail(AFC_ERR_INVALID, "NULL pointer (vis, weights or out)");
    if (!dtype_ok(vis_dtype)) return fail(AFC_ERR_INVALID, "unknown vis_dtype %d", (int)vis_dtype);
    if (vis_dtype != AFC_I8) {
        rc = check_inputs({{vis, (size_t)d->n_subbands * kP * nbl_of(d->n_antennas) * 8, AFC_VALUES_F32, "vis"}}, stream);
        if (rc != AFC_OK) return rc;
    }
    hipError_t e = launch_normalise(vis, vis_dtype == AFC_I8, weights, out, d->n_subbands, d->n_antennas, stream);
    if (e != hipSuccess) return hip_fail(e, "normalise launch");
    return AFC_OK;
}

AFC_API int afc_correlate(const afc_dims* d, afc_dtype in_dtype, const void* z, const int32_t* n_spectra_per_sb,
                          const uint8_t* flags, void* vis, int32_t* weights, hipStream_t stream) {
    g_err.clear();
    int rc = check_dims(d);
    if (rc != AFC_OK) return rc;
    if (!z || !vis) return fail(AFC_ERR_INVALID, "NULL pointer (z or vis)");
    if (reinterpret_cast<uintptr_t>(vis) % 16) return fail(AFC_ERR_INVALID, "vis is not 16-byte aligned");
    if (!dtype_ok(in_dtype)) return fail(AFC_ERR_INVALID, "unknown in_dtype %d", (int)in_dtype);
    std::vector<int32_t> S(d->n_subbands, d->n_spectra);
    if (n_spectra_per_sb) {
        for (int b = 0; b < d->n_subbands; ++b) {
            if (n_spectra_per_sb[b] < 1 || n_spectra_per_sb[b] > d->n_spectra)
                return fail(AFC_ERR_INVALID, "n_spectra_per_sb[%d] = %d outside 1..%d", b, n_spectra_per_sb[b],
                            d->n_spectra);
            S[b] = n_spectra_per_sb[b];
        }
    }
    if (in_dtype == AFC_I8) {
        for (int b = 0; b < d->n_subbands; ++b)
            if (2LL * 127 * 127 * S[b] >= (1LL << 31))
                return fail(AFC_ERR_UNSUPPORTED, "int8 sums over %d spectra may overflow int32", S[b]);
    }
    const int64_t N = 2LL * d->n_antennas;
    if (in_dtype != AFC_I8) {
        const size_t nz = (size_t)d->n_subbands * z_sb_samples(N, d->n_spectra) * 2;
        rc = check_inputs({{z, nz, in_dtype == AFC_F32 ? AFC_VALUES_F32 : AFC_VALUES_F16, "z"}}, stream);
        if (rc != AFC_OK) return rc;
    }
    XLaunch a{};
    a.z = z;
    a.vis = vis;
    a.weights = weights;
    a.flags = flags;
    a.Sb = (int)blocks_of(d->n_spectra);
    a.z_ch_stride = (int64_t)a.Sb * N * kSBlk;
    a.z_sb_stride = a.z_ch_stride * kP;
    a.N = (int)N;
    a.Na = d->n_antennas;
    a.B = d->n_subbands;
    a.S_host = S.data();
    a.dt = in_dtype;
    hipError_t e = launch_xengine(a, stream);
    if (e != hipSuccess) return hip_fail(e, "correlator launch");
    return AFC_OK;
}

AFC_API size_t afc_calibrate_workspace_bytes(int32_t n_antennas, int32_t n_channels) {
    if (n_antennas < 1 || n_antennas > 4096 || n_channels < 1) return 0;
    return cal_workspace_bytes(n_antennas, n_channels);
}

namespace {
int check_cal_inputs(int32_t Na, int32_t P, const void* V, const void* M, const void* g, hipStream_t stream) {
    const size_t nv = (size_t)P * nbl_of(Na) * 8;
    return check_inputs({{V, nv, AFC_VALUES_F32, "V"}, {M, nv, AFC_VALUES_F32, "M"},
                         {g, (size_t)P * Na * 4, AFC_VALUES_F32, "g"}},
                        stream);
}
}  // namespace

AFC_API int afc_calibrate_grad(int32_t n_antennas, int32_t n_channels, const void* V, const void* M, const void* g,
                               double* loss, void* grad, void* workspace, hipStream_t stream) {
    g_err.clear();
    if (n_antennas < 1 || n_antennas > 4096) return fail(AFC_ERR_INVALID, "n_antennas = %d outside 1..4096", n_antennas);
    if (n_channels < 1 || n_channels > 65535) return fail(AFC_ERR_INVALID, "n_channels = %d outside 1..65535", n_channels);
    if (!V || !M || !g || !loss) return fail(AFC_ERR_INVALID, "NULL pointer (V, M, g or loss)");
    if (!workspace) return fail(AFC_ERR_WORKSPACE, "workspace is NULL (need %zu bytes)",
                                cal_workspace_bytes(n_antennas, n_channels));
    const int rc = check_cal_inputs(n_antennas, n_channels, V, M, g, stream);
    if (rc != AFC_OK) return rc;
    hipError_t e = launch_calibrate(n_antennas, n_channels, reinterpret_cast<const float2*>(V),
                                    reinterpret_cast<const float2*>(M), reinterpret_cast<const float2*>(g), loss,
                                    reinterpret_cast<float2*>(grad), workspace, stream);
    if (e != hipSuccess) return hip_fail(e, "calibration launch");
    return AFC_OK;
}

AFC_API int afc_calibrate_grad_noalloc(int32_t n_antennas, int32_t n_channels, const void* V, const void* M,
                                       const void* g, double* loss, void* grad, hipStream_t stream) {
    g_err.clear();
    if (n_antennas < 1 || n_antennas > 4096) return fail(AFC_ERR_INVALID, "n_antennas = %d outside 1..4096", n_antennas);
    if (n_channels < 1 || n_channels > 65535) return fail(AFC_ERR_INVALID, "n_channels = %d outside 1..65535", n_channels);
    if (!V || !M || !g || !loss) return fail(AFC_ERR_INVALID, "NULL pointer (V, M, g or loss)");
    const size_t need = cal_workspace_bytes(n_antennas, n_channels);
    if (need > kCalScratchBytes)
        return fail(AFC_ERR_UNSUPPORTED, "%d antennas x %d channels need %zu bytes of scratch, more than the %zu built in",
                    n_antennas, n_channels, need, kCalScratchBytes);
    const int rc = check_cal_inputs(n_antennas, n_channels, V, M, g, stream);
    if (rc != AFC_OK) return rc;
    void* scratch = nullptr;
    hipError_t e = cal_scratch_address(&scratch);
    if (e != hipSuccess) return hip_fail(e, "scratch address");
    e = launch_calibrate(n_antennas, n_channels, reinterpret_cast<const float2*>(V), reinterpret_cast<const float2*>(M),
                         reinterpret_cast<const float2*>(g), loss, reinterpret_cast<float2*>(grad), scratch, stream);
    if (e != hipSuccess) return hip_fail(e, "calibration launch");
    return AFC_OK;
}

AFC_API int afc_calibrate_grad_weighted(int32_t n_antennas, int32_t n_channels, const void* V, const void* M,
                                        const uint8_t* vis_flags, const float* weights, const void* g, double* loss,
                                        void* grad, void* workspace, hipStream_t stream) {
    g_err.clear();
    if (n_antennas < 1 || n_antennas > 4096) return fail(AFC_ERR_INVALID, "n_antennas = %d outside 1..4096", n_antennas);
    if (n_channels < 1 || n_channels > 65535) return fail(AFC_ERR_INVALID, "n_channels = %d outside 1..65535", n_channels);
    if (!V || !M || !g || !loss) return fail(AFC_ERR_INVALID, "NULL pointer (V, M, g or loss)");
    if (!workspace) return fail(AFC_ERR_WORKSPACE, "workspace is NULL (need %zu bytes)",
                                cal_workspace_bytes(n_antennas, n_channels));
    if (reinterpret_cast<uintptr_t>(vis_flags) % 2 || reinterpret_cast<uintptr_t>(weights) % 8)
        return fail(AFC_ERR_INVALID, "vis_flags must be 2-byte and weights 8-byte aligned");
    int rc = check_cal_inputs(n_antennas, n_channels, V, M, g, stream);
    if (rc != AFC_OK) return rc;
    if (weights) {
        rc = check_inputs({{weights, (size_t)n_channels * nbl_of(n_antennas) * 2, AFC_VALUES_F32, "weights"}}, stream);
        if (rc != AFC_OK) return rc;
    }
    hipError_t e = launch_calibrate(n_antennas, n_channels, reinterpret_cast<const float2*>(V),
                                    reinterpret_cast<const float2*>(M), reinterpret_cast<const float2*>(g), loss,
                                    reinterpret_cast<float2*>(grad), workspace, stream, vis_flags, weights);
    if (e != hipSuccess) return hip_fail(e, "calibration launch");
    return AFC_OK;
}

AFC_API size_t afc_calibrate_solve_workspace_bytes(int32_t n_antennas, int32_t n_channels) {
    if (n_antennas < 1 || n_antennas > 4096 || n_channels < 1 || n_channels > 65535) return 0;
    return cal_solve_workspace_bytes(n_antennas, n_channels);
}

AFC_API int afc_calibrate_solve(int32_t n_antennas, int32_t n_channels, const void* V, const void* M, void* g,
                                int32_t n_iter, double* loss, void* workspace, hipStream_t stream) {
    g_err.clear();
    if (n_antennas < 1 || n_antennas > 4096) return fail(AFC_ERR_INVALID, "n_antennas = %d outside 1..4096", n_antennas);
    if (n_channels < 1 || n_channels > 65535) return fail(AFC_ERR_INVALID, "n_channels = %d outside 1..65535", n_channels);
    if (n_iter < 0 || n_iter > 100000) return fail(AFC_ERR_INVALID, "n_iter = %d outside 0..100000", n_iter);
    if (!V || !M || !g) return fail(AFC_ERR_INVALID, "NULL pointer (V, M or g)");
    if (!workspace) return fail(AFC_ERR_WORKSPACE, "workspace is NULL (need %zu bytes)",
                                cal_solve_workspace_bytes(n_antennas, n_channels));
    const int rc = check_cal_inputs(n_antennas, n_channels, V, M, g, stream);
    if (rc != AFC_OK) return rc;
    hipError_t e = launch_calibrate_solve(n_antennas, n_channels, reinterpret_cast<const float2*>(V),
                                          reinterpret_cast<const float2*>(M), reinterpret_cast<float2*>(g), n_iter,
                                          loss, workspace, stream);
    if (e != hipSuccess) return hip_fail(e, "calibration solver launch");
    return AFC_OK;
}

AFC_API int afc_calibrate_solve_weighted(int32_t n_antennas, int32_t n_channels, const void* V, const void* M,
                                         const uint8_t* vis_flags, const float* weights, void* g, int32_t n_iter,
                                         double* loss, void* workspace, hipStream_t stream) {
    g_err.clear();
    if (n_antennas < 1 || n_antennas > 4096) return fail(AFC_ERR_INVALID, "n_antennas = %d outside 1..4096", n_antennas);
    if (n_channels < 1 || n_channels > 65535) return fail(AFC_ERR_INVALID, "n_channels = %d outside 1..65535", n_channels);
    if (n_iter < 0 || n_iter > 100000) return fail(AFC_ERR_INVALID, "n_iter = %d outside 0..100000", n_iter);
    if (!V || !M || !g) return fail(AFC_ERR_INVALID, "NULL pointer (V, M or g)");
    if (!workspace) return fail(AFC_ERR_WORKSPACE, "workspace is NULL (need %zu bytes)",
                                cal_solve_workspace_bytes(n_antennas, n_channels));
    if (reinterpret_cast<uintptr_t>(vis_flags) % 2 || reinterpret_cast<uintptr_t>(weights) % 8)
        return fail(AFC_ERR_INVALID, "vis_flags must be 2-byte and weights 8-byte aligned");
    int rc = check_cal_inputs(n_antennas, n_channels, V, M, g, stream);
    if (rc != AFC_OK) return rc;
    if (weights) {
        rc = check_inputs({{weights, (size_t)n_channels * nbl_of(n_antennas) * 2, AFC_VALUES_F32, "weights"}}, stream);
        if (rc != AFC_OK) return rc;
    }
    hipError_t e = launch_calibrate_solve(n_antennas, n_channels, reinterpret_cast<const float2*>(V),
                                          reinterpret_cast<const float2*>(M), reinterpret_cast<float2*>(g), n_iter,
                                          loss, workspace, stream, vis_flags, weights);
    if (e != hipSuccess) return hip_fail(e, "calibration solver launch");
    return AFC_OK;
}

AFC_API size_t afc_sigma_clip_workspace_bytes(int32_t n_antennas, int32_t n_channels) {
    if (n_antennas < 1 || n_antennas > 4096 || n_channels < 1 || n_channels > 65535) return 0;
    return sigma_clip_workspace_bytes(n_antennas, n_channels);
}

AFC_API int afc_sigma_clip(int32_t n_antennas, int32_t n_channels, const void* V, float threshold,
                           uint8_t* vis_flags, void* workspace, hipStream_t stream) {
    g_err.clear();
    if (n_antennas < 1 || n_antennas > 4096) return fail(AFC_ERR_INVALID, "n_antennas = %d outside 1..4096", n_antennas);
    if (n_channels < 1 || n_channels > 65535) return fail(AFC_ERR_INVALID, "n_channels = %d outside 1..65535", n_channels);
    if (!V || !vis_flags) return fail(AFC_ERR_INVALID, "NULL pointer (V or vis_flags)");
    if (!(std::isfinite(threshold) && threshold > 0.0f)) return fail(AFC_ERR_INVALID, "threshold must be finite and > 0");
    if (!workspace) return fail(AFC_ERR_WORKSPACE, "workspace is NULL (need %zu bytes)",
                                sigma_clip_workspace_bytes(n_antennas, n_channels));
    const int rc = check_inputs({{V, (size_t)n_channels * nbl_of(n_antennas) * 8, AFC_VALUES_F32, "V"}}, stream);
    if (rc != AFC_OK) return rc;
    hipError_t e = launch_sigma_clip(n_antennas, n_channels, reinterpret_cast<const float2*>(V), threshold, vis_flags,
                                     workspace, stream);
    if (e != hipSuccess) return hip_fail(e, "sigma-clip launch");
    return AFC_OK;
}

AFC_API int afc_apply_vis_flags(int32_t n_antennas, int32_t n_channels, const uint8_t* vis_flags, void* V, void* M,
                                hipStream_t stream) {
    g_err.clear();
    if (n_antennas < 1 || n_antennas > 4096) return fail(AFC_ERR_INVALID, "n_antennas = %d outside 1..4096", n_antennas);
    if (n_channels < 1 || n_channels > 65535) return fail(AFC_ERR_INVALID, "n_channels = %d outside 1..65535", n_channels);
    if (!vis_flags || (!V && !M)) return fail(AFC_ERR_INVALID, "NULL pointer (vis_flags, or both V and M)");
    hipError_t e = launch_apply_vis_flags(n_antennas, n_channels, vis_flags, reinterpret_cast<float2*>(V),
                                          reinterpret_cast<float2*>(M), stream);
    if (e != hipSuccess) return hip_fail(e, "apply-flags launch");
    return AFC_OK;
}

namespace {
int check_grid(int32_t n_antennas, int32_t n_subbands, int32_t grid_size) {
    if (n_antennas < 1 || n_antennas > 4096) return fail(AFC_ERR_INVALID, "n_antennas = %d outside 1..4096", n_antennas);
    if (n_subbands < 1 || n_subbands > AFC_MAX_SUBBANDS)
        return fail(AFC_ERR_INVALID, "n_subbands = %d outside 1..%d", n_subbands, AFC_MAX_SUBBANDS);
    if (grid_size < 32 || grid_size > 4096 || (grid_size & (grid_size - 1)))
        return fail(AFC_ERR_UNSUPPORTED, "grid_size = %d (a power of two in 32..4096)", grid_size);
    return AFC_OK;
}
}  // namespace

AFC_API size_t afc_imaging_workspace_bytes(int32_t n_antennas, int32_t n_subbands, int32_t grid_size) {
    if (check_grid(n_antennas, n_subbands, grid_size) != AFC_OK) return 0;
    return imaging_workspace_bytes(n_antennas, n_subbands, grid_size);
}

AFC_API int afc_grid_visibilities(int32_t n_antennas, int32_t n_subbands, const void* vis, const int32_t* weights,
                                  const double* positions, const double* freq_hz, int32_t grid_size,
                                  double cell_wavelengths, void* grid, double* norm, void* workspace,
                                  hipStream_t stream) {
    g_err.clear();
    int rc = check_grid(n_antennas, n_subbands, grid_size);
    if (rc != AFC_OK) return rc;
    if (!vis || !positions || !freq_hz || !grid || !norm)
        return fail(AFC_ERR_INVALID, "NULL pointer (vis, positions, freq_hz, grid or norm)");
    if (!(std::isfinite(cell_wavelengths) && cell_wavelengths > 0.0))
        return fail(AFC_ERR_INVALID, "cell_wavelengths must be finite and > 0");
    if (!workspace) return fail(AFC_ERR_WORKSPACE, "workspace is NULL");
    rc = check_inputs({{vis, (size_t)n_subbands * kP * nbl_of(n_antennas) * 8, AFC_VALUES_F32, "vis"},
                       {positions, (size_t)n_antennas * 2, AFC_VALUES_F64, "positions"},
                       {freq_hz, (size_t)n_subbands * kP, AFC_VALUES_F64, "freq_hz"}},
                      stream);
    if (rc != AFC_OK) return rc;
    hipError_t e = launch_grid(reinterpret_cast<const float2*>(vis), weights, positions, freq_hz, n_antennas,
                               n_subbands, grid_size, cell_wavelengths, reinterpret_cast<float2*>(grid), norm,
                               workspace, stream);
    if (e != hipSuccess) return hip_fail(e, "gridding launch");
    return AFC_OK;
}

AFC_API int afc_image_from_grid(int32_t grid_size, const void* grid, const double* norm, float* image, void* workspace,
                                hipStream_t stream) {
    g_err.clear();
    int rc = check_grid(1, 1, grid_size);
    if (rc != AFC_OK) return rc;
    if (!grid || !norm || !image) return fail(AFC_ERR_INVALID, "NULL pointer (grid, norm or image)");
    if (!workspace) return fail(AFC_ERR_WORKSPACE, "workspace is NULL");
    rc = check_inputs({{grid, (size_t)grid_size * grid_size * 2, AFC_VALUES_F32, "grid"}}, stream);
    if (rc != AFC_OK) return rc;
    hipError_t e = launch_image(reinterpret_cast<const float2*>(grid), norm, image, grid_size, workspace, stream);
    if (e != hipSuccess) return hip_fail(e, "imaging launch");
    return AFC_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// batching plan
// ---------------------------------------------------------------------------
struct afc_plan {
    afc_dims d{};
    std::vector<int32_t> dt, S;
    std::vector<int64_t> z_off;
    size_t ws_bytes = 0;
    int N = 0, Na = 0;
    int64_t L = 0;
    // device tables (d_sbs and the work lists never change after creation)
    XSubband* d_sbs = nullptr;
    struct Mode {
        bool used = false;
        int tile = 128;
        int n_wg = 0;
        int n_items = 0;
        XWork* d_work = nullptr;
        XcdRanges ranges{};
    } mode[3];    // 0: int8 and fp16 subbands (int8 only when split), 1: fp32, 2: fp16 when split
    bool split = false;     // int8 and fp16 subbands in launches of their own
    std::vector<PpfItem> items;
    // A captured graph with the channeliser's item table it reads (the table
    // holds the int8 gains, so each capture has its own).  `done` is recorded
    // on the caller's stream after every launch of the graph: a retired
    // capture is freed once its last launch has completed.
    struct Capture {
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        PpfItem* d_items = nullptr;
        std::vector<PpfItem> h_items;   // source of the table's async upload
        hipEvent_t done = nullptr;
        std::vector<const void*> key_ptrs;
        std::vector<float> key_gains;
    };
    hipStream_t cap_stream = nullptr;
    Capture* cur = nullptr;
    std::vector<Capture*> retired;
};

namespace {

// Time of one tile item in MFMA cycles (per SIMD), from the instruction
// rates: an int8 16x16x64 and an fp16 16x16x32 MFMA take the same cycles,
// the int8 one covering twice the spectra (4 and 8 cycles per spectrum for
// the real and imaginary parts of a 32 x 32 area); fp32 32x32x2 blocks take
// 128.  The waves of a tile run in parallel, so a diagonal tile takes the
// time of its busiest wave: 9 of 16 blocks (128-wide), 3 of 4 (64-wide
// int8 / fp16), all of it for fp32 (one block per wave either way).
double tile_cost(int dt, int tile, int S, bool diag) {
    const double diag_frac = dt == AFC_F32 ? 1.0 : tile == 128 ? 9.0 / 16.0 : 3.0 / 4.0;
    const double blocks = (tile / 32.0) * (tile / 32.0) * (diag ? diag_frac : 1.0);
    const double per_spec = dt == AFC_I8 ? 4.0 : dt == AFC_F16 ? 8.0 : 128.0;   // cycles per 32x32 area-spectrum
    return blocks * per_spec * S + 2000.0;                                      // + fixed cost (epilogue)
}

// Build the work list of one mode: the (subband, channel) groups are spread
// over the 8 XCDs by cost (longest first onto the least loaded XCD), and each
// XCD's items are stored contiguously, group after group, tiles in row order.
bool in_mode(const afc_plan& p, int m, int dt) {
    if (m == 0) return dt == AFC_I8 || (!p.split && dt == AFC_F16);
    if (m == 1) return dt == AFC_F32;
    return p.split && dt == AFC_F16;
}

void build_work(const afc_plan& p, int m, int tile, std::vector<XWork>& work_out, XcdRanges& ranges) {
    const int nT = (int)ceil_div(p.N, tile);
    struct G {
        int sb, ch;
        double cost;
    };
    std::vector<G> groups;
    for (int b = 0; b < p.d.n_subbands; ++b) {
        if (!in_mode(p, m, p.dt[b])) continue;
        double c = 0;
        for (int ti = 0; ti < nT; ++ti)
            for (int tj = 0; tj <= ti; ++tj) c += tile_cost(p.dt[b], tile, p.S[b], ti == tj);
        for (int ch = 0; ch < kP; ++ch) groups.push_back({b, ch, c});
    }
    const int n_xcd = 8;
    std::vector<double> xload(n_xcd, 0.0);
    std::vector<std::vector<int>> xgroups(n_xcd);
    std::vector<int> order(groups.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return groups[a].cost > groups[b].cost; });
    for (int gi : order) {
        int best = (int)(std::min_element(xload.begin(), xload.end()) - xload.begin());
        xload[best] += groups[gi].cost;
        xgroups[best].push_back(gi);
    }
    work_out.clear();
    for (int x = 0; x < n_xcd; ++x) {
        ranges.begin[x] = (int32_t)work_out.size();
        for (int gi : xgroups[x])
            for (int ti = 0; ti < nT; ++ti)
                for (int tj = 0; tj <= ti; ++tj) work_out.push_back(XWork{groups[gi].sb, groups[gi].ch, ti, tj});
        ranges.count[x] = (int32_t)work_out.size() - ranges.begin[x];
    }
}

int upload_mode(afc_plan* p, int m, int tile) {
    afc_plan::Mode& md = p->mode[m];
    std::vector<XWork> work;
    XcdRanges ranges{};
    build_work(*p, m, tile, work, ranges);
    if (md.d_work) hipFree(md.d_work);
    md.d_work = nullptr;
    md.used = !work.empty();
    md.tile = tile;
    md.ranges = ranges;
    md.n_wg = xengine_list_grid(ranges);
    md.n_items = (int)work.size();
    if (!md.used) return AFC_OK;
    hipError_t e = hipMalloc(&md.d_work, work.size() * sizeof(XWork));
    if (e == hipSuccess) e = hipMemcpy(md.d_work, work.data(), work.size() * sizeof(XWork), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "plan work upload");
    return AFC_OK;
}

std::string tune_key(const afc_plan& p) {
    int n8 = 0, n16 = 0, n32 = 0;
    int smin = 1 << 30, smax = 0;
    for (int b = 0; b < p.d.n_subbands; ++b) {
        n8 += p.dt[b] == AFC_I8;
        n16 += p.dt[b] == AFC_F16;
        n32 += p.dt[b] == AFC_F32;
        smin = std::min(smin, p.S[b]);
        smax = std::max(smax, p.S[b]);
    }
    std::ostringstream o;
    o << "N" << p.N << "_i8x" << n8 << "_f16x" << n16 << "_f32x" << n32 << "_S" << smin << "-" << smax;
    return o.str();
}

// The tune cache is a flat JSON object {"key": [tile, wg_per_cu, split], ...}
// (split: int8 and fp16 subbands in separate correlator launches; entries
// with two values are read as split = 0).
struct TuneChoice {
    int tile = 128, wpc = 2, split = 0;
};
std::map<std::string, TuneChoice> read_cache(const char* path) {
    std::map<std::string, TuneChoice> m;
    std::ifstream f(path);
    if (!f) return m;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string s = ss.str();
    size_t i = 0;
    while ((i = s.find('"', i)) != std::string::npos) {
        const size_t j = s.find('"', i + 1);
        if (j == std::string::npos) break;
        const std::string key = s.substr(i + 1, j - i - 1);
        const size_t lb = s.find('[', j), rb = s.find(']', j);
        if (lb == std::string::npos || rb == std::string::npos) break;
        int a = 0, b = 0, c = 0;
        const int n = sscanf(s.c_str() + lb, "[ %d , %d , %d ]", &a, &b, &c);
        if (n >= 2) m[key] = TuneChoice{a, b, n == 3 ? c : 0};
        i = rb + 1;
    }
    return m;
}

void write_cache(const char* path, const std::map<std::string, TuneChoice>& m) {
    std::ofstream f(path);
    f << "{\n";
    size_t k = 0;
    for (const auto& kv : m) {
        f << "  \"" << kv.first << "\": [" << kv.second.tile << ", " << kv.second.wpc << ", " << kv.second.split << "]"
          << (++k < m.size() ? ",\n" : "\n");
    }
    f << "}\n";
}

// Time the int8/fp16 correlator of the plan's own work for each candidate
// -- tile 128 wide at 2 workgroups per CU or 64 wide at 4, int8 and fp16
// subbands in one launch or in one launch each (when both types are
// present) -- on scratch buffers holding random samples; returns the best.
int tune_mode0(afc_plan* p, TuneChoice& out) {
    bool has8 = false, has16 = false;
    for (int b = 0; b < p->d.n_subbands; ++b) {
        has8 |= p->dt[b] == AFC_I8;
        has16 |= p->dt[b] == AFC_F16;
    }
    std::vector<TuneChoice> cands = {{128, 2, 0}, {64, 4, 0}};
    if (has8 && has16) {
        cands.push_back({128, 2, 1});
        cands.push_back({64, 4, 1});
    }
    size_t vis_bytes = (size_t)p->d.n_subbands * kP * nbl_of(p->Na) * 32;
    void* z = nullptr;
    void* vis = nullptr;
    hipError_t e = hipMalloc(&z, std::max<size_t>(p->ws_bytes, 256));
    if (e == hipSuccess) e = hipMalloc(&vis, vis_bytes);
    if (e != hipSuccess) {
        if (z) hipFree(z);
        return hip_fail(e, "tuner scratch allocation");
    }
    // random samples: the MFMA rate (and clock) depends on the data, so zeros
    // would time the candidates unrepresentatively
    e = launch_fill_scratch(z, p->ws_bytes, nullptr);
    if (e != hipSuccess) {
        hipFree(z);
        hipFree(vis);
        return hip_fail(e, "tuner scratch fill");
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    float best = 1e30f;
    out = cands[0];
    int rc = e == hipSuccess ? AFC_OK : hip_fail(e, "tuner events");
    // every launch and event call is checked: a candidate that failed to
    // launch would otherwise time as the fastest
    for (size_t ci = 0; rc == AFC_OK && ci < cands.size(); ++ci) {
        const TuneChoice& c = cands[ci];
        p->split = c.split != 0;
        rc = upload_mode(p, 0, c.tile);
        if (rc == AFC_OK) rc = upload_mode(p, 2, c.tile);
        if (rc != AFC_OK) break;
        float tmin = 1e30f;
        for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
            e = hipEventRecord(e0, nullptr);
            for (int m : {0, 2}) {
                const afc_plan::Mode& md = p->mode[m];
                if (e == hipSuccess && md.used)
                    e = launch_xengine_list(z, vis, nullptr, nullptr, p->d_sbs, md.d_work, md.ranges, p->N, p->Na, 0,
                                            md.tile, nullptr);
            }
            if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e == hipSuccess && rep > 0) tmin = std::min(tmin, ms);
        }
        if (e != hipSuccess) {
            rc = hip_fail(e, "tuner candidate launch");
            break;
        }
        if (tmin < best) {
            best = tmin;
            out = c;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(z);
    (void)hipFree(vis);
    return rc;
}

void free_capture(afc_plan::Capture* c) {
    if (!c) return;
    if (c->exec) hipGraphExecDestroy(c->exec);
    if (c->graph) hipGraphDestroy(c->graph);
    if (c->d_items) hipFree(c->d_items);
    if (c->done) hipEventDestroy(c->done);
    delete c;
}

// Free the retired captures whose last launch has completed (or, with
// wait, all of them after their last launch).
void reap_captures(afc_plan* p, bool wait) {
    std::vector<afc_plan::Capture*> keep;
    for (afc_plan::Capture* c : p->retired) {
        if (wait) hipEventSynchronize(c->done);
        if (wait || hipEventQuery(c->done) == hipSuccess)
            free_capture(c);
        else
            keep.push_back(c);
    }
    p->retired.swap(keep);
}

// Capture the plan's launches into a new graph for these buffers and gains.
// The item table is uploaded on the caller's stream, so it is in place
// before the graph's first launch there and no earlier launch can see it.
int capture_plan(afc_plan* p, const int16_t* x, const float* taps, const std::vector<float>& gains, void* z_workspace,
                 const uint8_t* flags, void* vis, int32_t* weights, hipStream_t stream,
                 const std::vector<const void*>& key) {
    const int B = p->d.n_subbands;
    auto* c = new afc_plan::Capture();
    c->h_items = p->items;
    for (int b = 0; b < B; ++b) c->h_items[b].gain = gains[b];
    hipError_t e = hipMalloc(&c->d_items, B * sizeof(PpfItem));
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->done, hipEventDisableTiming);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->d_items, c->h_items.data(), B * sizeof(PpfItem), hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) {
        free_capture(c);
        return hip_fail(e, "plan item table upload");
    }
    e = hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        free_capture(c);
        return hip_fail(e, "graph capture begin");
    }
    hipError_t le = launch_ppf_batched(x, taps, z_workspace, c->d_items, B, p->N, p->d.n_spectra, p->cap_stream);
    for (int m = 0; m < 3 && le == hipSuccess; ++m) {
        const afc_plan::Mode& md = p->mode[m];
        if (!md.used) continue;
        le = launch_xengine_list(z_workspace, vis, weights, flags, p->d_sbs, md.d_work, md.ranges, p->N, p->Na,
                                 m == 1 ? 1 : 0, md.tile, p->cap_stream);
    }
    e = hipStreamEndCapture(p->cap_stream, &c->graph);
    if (le != hipSuccess || e != hipSuccess) {
        free_capture(c);
        return hip_fail(le != hipSuccess ? le : e, "plan graph capture");
    }
    e = hipGraphInstantiate(&c->exec, c->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        free_capture(c);
        return hip_fail(e, "graph instantiate");
    }
    c->key_ptrs = key;
    c->key_gains = gains;
    if (p->cur) p->retired.push_back(p->cur);
    p->cur = c;
    return AFC_OK;
}

}  // namespace

extern "C" {

AFC_API int afc_plan_create(const afc_dims* d, const afc_dtype* dtype_per_sb, const int32_t* n_spectra_per_sb,
                            const char* tune_cache_path, afc_plan** out) {
    g_err.clear();
    if (!out) return fail(AFC_ERR_INVALID, "out is NULL");
    *out = nullptr;
    int rc = check_dims(d);
    if (rc != AFC_OK) return rc;
    if (!dtype_per_sb || !n_spectra_per_sb) return fail(AFC_ERR_INVALID, "dtype_per_sb and n_spectra_per_sb are required");
    afc_plan* p = new afc_plan();
    p->d = *d;
    p->N = 2 * d->n_antennas;
    p->Na = d->n_antennas;
    p->L = ((int64_t)d->n_spectra + kT - 1) * kP;
    const int B = d->n_subbands;
    p->dt.resize(B);
    p->S.resize(B);
    p->z_off.resize(B);
    int64_t off = 0;
    for (int b = 0; b < B; ++b) {
        if (!dtype_ok(dtype_per_sb[b])) {
            delete p;
            return fail(AFC_ERR_INVALID, "dtype_per_sb[%d] = %d unknown", b, (int)dtype_per_sb[b]);
        }
        if (n_spectra_per_sb[b] < 1 || n_spectra_per_sb[b] > d->n_spectra) {
            delete p;
            return fail(AFC_ERR_INVALID, "n_spectra_per_sb[%d] = %d outside 1..%d", b, n_spectra_per_sb[b], d->n_spectra);
        }
        if (dtype_per_sb[b] == AFC_I8 && 2LL * 127 * 127 * n_spectra_per_sb[b] >= (1LL << 31)) {
            delete p;
            return fail(AFC_ERR_UNSUPPORTED, "int8 sums over %d spectra may overflow int32", n_spectra_per_sb[b]);
        }
        p->dt[b] = dtype_per_sb[b];
        p->S[b] = n_spectra_per_sb[b];
        p->z_off[b] = off;
        off += z_sb_samples(p->N, p->S[b]) * sample_bytes((afc_dtype)p->dt[b]);
        off = (off + 255) / 256 * 256;
    }
    p->ws_bytes = (size_t)off;
    // per-subband tables
    std::vector<XSubband> sbs(B);
    p->items.resize(B);
    const int64_t nbl = nbl_of(p->Na);
    for (int b = 0; b < B; ++b) {
        sbs[b] = XSubband{p->z_off[b], (int64_t)b * kP * nbl * 32, p->S[b], (int32_t)blocks_of(p->S[b]), p->dt[b], 0};
        p->items[b] = PpfItem{(int64_t)b * p->L * p->N * 2, p->z_off[b], p->S[b], (int32_t)blocks_of(p->S[b]),
                              p->dt[b], 1.0f};
    }
    hipError_t e = hipMalloc(&p->d_sbs, B * sizeof(XSubband));
    if (e == hipSuccess) e = hipMemcpy(p->d_sbs, sbs.data(), B * sizeof(XSubband), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        afc_plan_destroy(p);
        return hip_fail(e, "plan allocation");
    }
    // int8 / fp16 subbands: tile choice from the tune cache or the tuner
    bool any0 = false, any1 = false;
    for (int b = 0; b < B; ++b) {
        any0 |= p->dt[b] != AFC_F32;
        any1 |= p->dt[b] == AFC_F32;
    }
    if (any0) {
        TuneChoice ch;
        if (tune_cache_path && *tune_cache_path) {
            auto cache = read_cache(tune_cache_path);
            const std::string key = tune_key(*p);
            auto it = cache.find(key);
            if (it != cache.end() && (it->second.tile == 64 || it->second.tile == 128) && it->second.wpc >= 1 &&
                it->second.wpc <= 8 && (it->second.split == 0 || it->second.split == 1)) {
                ch = it->second;
            } else {
                rc = tune_mode0(p, ch);
                if (rc != AFC_OK) {
                    afc_plan_destroy(p);
                    return rc;
                }
                cache[key] = ch;
                write_cache(tune_cache_path, cache);
            }
        }
        p->split = ch.split != 0;
        rc = upload_mode(p, 0, ch.tile);
        if (rc == AFC_OK) rc = upload_mode(p, 2, ch.tile);
        if (rc != AFC_OK) {
            afc_plan_destroy(p);
            return rc;
        }
    }
    if (any1) {
        rc = upload_mode(p, 1, 64);
        if (rc != AFC_OK) {
            afc_plan_destroy(p);
            return rc;
        }
    }
    *out = p;
    return AFC_OK;
}

AFC_API size_t afc_plan_workspace_bytes(const afc_plan* p) { return p ? p->ws_bytes : 0; }

AFC_API int afc_plan_info(const afc_plan* p, int32_t* tile_rows, int32_t* tile_cols, int32_t* n_workgroups,
                          int32_t* n_work_items) {
    if (!p) return fail(AFC_ERR_INVALID, "plan is NULL");
    const afc_plan::Mode& md = p->mode[0].used ? p->mode[0] : p->mode[2].used ? p->mode[2] : p->mode[1];
    if (tile_rows) *tile_rows = md.tile;
    if (tile_cols) *tile_cols = md.tile;
    if (n_workgroups) *n_workgroups = md.n_wg;
    if (n_work_items) *n_work_items = p->mode[0].n_items + p->mode[1].n_items + p->mode[2].n_items;
    return AFC_OK;
}

AFC_API int afc_plan_launch(afc_plan* p, const int16_t* x, const float* taps, const float* gain_per_sb,
                            void* z_workspace, const uint8_t* flags, void* vis, int32_t* weights, hipStream_t stream) {
    g_err.clear();
    if (!p) return fail(AFC_ERR_INVALID, "plan is NULL");
    if (!x || !taps || !z_workspace || !vis) return fail(AFC_ERR_INVALID, "NULL pointer (x, taps, workspace or vis)");
    if (reinterpret_cast<uintptr_t>(vis) % 16) return fail(AFC_ERR_INVALID, "vis is not 16-byte aligned");
    const int B = p->d.n_subbands;
    std::vector<float> gains(B, 1.0f);
    for (int b = 0; b < B; ++b) {
        if (p->dt[b] == AFC_I8) {
            if (!gain_per_sb) return fail(AFC_ERR_INVALID, "gain_per_sb is required with int8 subbands");
            if (!(std::isfinite(gain_per_sb[b]) && gain_per_sb[b] > 0.0f))
                return fail(AFC_ERR_INVALID, "gain_per_sb[%d] must be finite and > 0", b);
            gains[b] = gain_per_sb[b];
        }
    }
    const int rc0 = check_inputs({{taps, (size_t)kT * kP, AFC_VALUES_F32, "taps"}}, stream);
    if (rc0 != AFC_OK) return rc0;
    const std::vector<const void*> key = {x, taps, z_workspace, flags, vis, weights};
    const bool same = p->cur && key == p->cur->key_ptrs && gains == p->cur->key_gains;
    reap_captures(p, false);
    if (!same) {
        const int rc = capture_plan(p, x, taps, gains, z_workspace, flags, vis, weights, stream, key);
        if (rc != AFC_OK) return rc;
    }
    hipError_t e = hipGraphLaunch(p->cur->exec, stream);
    if (e == hipSuccess) e = hipEventRecord(p->cur->done, stream);
    if (e != hipSuccess) return hip_fail(e, "graph launch");
    return AFC_OK;
}

AFC_API void afc_plan_destroy(afc_plan* p) {
    if (!p) return;
    if (p->cur) p->retired.push_back(p->cur);
    p->cur = nullptr;
    reap_captures(p, true);
    for (auto& md : p->mode)
        if (md.d_work) hipFree(md.d_work);
    if (p->d_sbs) hipFree(p->d_sbs);
    if (p->cap_stream) hipStreamDestroy(p->cap_stream);
    delete p;
}

}  // extern "C"
