// Internal declarations shared by the kernels and the C ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "afc.h"

namespace afc {

constexpr int kP = 64;                 // channels
constexpr int kT = 16;                 // taps per branch
constexpr int kPFine = 256;            // channels of the fine bank
constexpr int kSBlk = AFC_SPECTRUM_BLOCK;

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int sample_bytes(afc_dtype t) { return t == AFC_F32 ? 8 : t == AFC_F16 ? 4 : 2; }

// ---------------------------------------------------------------- PPF
struct PpfLaunch {
    const int16_t* x;       // subband 0 base
    const float* taps;      // [T*P]
    void* z;                // subband 0 base of the channelised output
    int64_t x_sb_stride;    // int16 elements between subbands
    int64_t z_sb_stride;    // samples between subbands (complex elements)
    int N;                  // receivers
    int S;                  // spectra (per subband, same for all in one launch)
    int Sb;                 // blocks allocated per channel
    int B;                  // subbands
    float gain;
    afc_dtype dt;
};
hipError_t launch_ppf(const PpfLaunch& a, hipStream_t stream);

// Per-subband descriptor for the batched channeliser.
struct PpfItem {
    int64_t x_off;          // int16 elements from x base to this subband
    int64_t z_off;          // bytes from workspace base to this subband
    int32_t S;              // spectra
    int32_t Sb;             // blocks allocated
    int32_t dt;             // afc_dtype
    float gain;
};
hipError_t launch_ppf_batched(const int16_t* x, const float* taps, void* z_ws, const PpfItem* items_dev,
                              int n_items, int N, int max_S, hipStream_t stream);

// Fine channeliser: 256-channel bank, delay and bandpass compensation,
// coherent 4:1 integration to 64 channels, stored in the layout of the
// 64-channel bank (one table launch, then one channeliser launch).
struct FineLaunch {
    const int16_t* x;       // subband 0 base, rows of 256 samples per spectrum
    const float* taps;      // [T*256]
    const double* tau;      // device [N] delays in seconds
    const float* bandpass;  // device [256] weights, natural FFT order
    const double* nu_center;// host [B] subband centre frequencies in Hz
    double subband_hz;      // subband width in Hz
    void* workspace;        // fine_workspace_bytes(N, B)
    void* z;
    int64_t x_sb_stride;    // int16 elements between subbands
    int64_t z_sb_stride;    // samples between subbands
    int N, S, Sb, B;
    float gain;
    afc_dtype dt;
};
size_t fine_workspace_bytes(int N, int B);
hipError_t launch_ppf_fine(const FineLaunch& l, hipStream_t stream);

// ---------------------------------------------------------------- X-engine
struct XLaunch {
    const void* z;          // subband 0 base
    void* vis;              // subband 0 base
    int32_t* weights;       // or nullptr
    const uint8_t* flags;   // [B][Na] or nullptr
    int64_t z_ch_stride;    // samples between channels
    int64_t z_sb_stride;    // samples between subbands
    int N, Na, Sb, B;
    const int32_t* S_host;  // [B] host
    afc_dtype dt;
};
hipError_t launch_xengine(const XLaunch& a, hipStream_t stream);

// Batched X-engine work item (one lower-triangle tile of one channel of one
// subband).
struct XWork {
    int32_t sb;             // subband index
    int32_t ch;             // channel
    int32_t ti, tj;         // tile row / column (ti >= tj)
};
struct XSubband {
    int64_t z_off;          // bytes from workspace base
    int64_t vis_off;        // bytes from vis base
    int32_t S;
    int32_t Sb;
    int32_t dt;
    int32_t pad;
};
// The work list is laid out XCD by XCD: XCD x owns items
// [begin[x], begin[x] + count[x]).
struct XcdRanges {
    int32_t begin[8];
    int32_t count[8];
};
// One workgroup per work item (workgroup ids go round-robin over the 8
// XCDs); mode 0: int8 / fp16 subbands with tile-wide tiles (128 or 64),
// mode 1: fp32 subbands (64).  Returns the grid size through n_wg_out.
hipError_t launch_xengine_list(const void* z_ws, void* vis, int32_t* weights, const uint8_t* flags,
                               const XSubband* sbs_dev, const XWork* work_dev, const XcdRanges& ranges,
                               int N, int Na, int mode, int tile, hipStream_t stream);
int xengine_list_grid(const XcdRanges& ranges);
// Fill `bytes` (a multiple of 4) of device memory with hashed bytes that are
// valid int8 samples and finite fp16 values (bit 6 of every byte clear).
hipError_t launch_fill_scratch(void* p, size_t bytes, hipStream_t stream);
int xengine_tile(afc_dtype dt);

// ---------------------------------------------------------------- validity
// spectrum validity bits [B][ceil(S/32)][Na] from packet flags [B][n_pk][Na]
hipError_t launch_validity(const uint8_t* pkt, uint32_t* v, int B, int Na, int S, int64_t n_pk, int Q, int Ps,
                           hipStream_t stream);
hipError_t launch_zero_invalid(const uint32_t* v, void* z, afc_dtype dt, int B, int Na, int S, hipStream_t stream);
hipError_t launch_validity_weights(const uint32_t* v, const uint8_t* flags, int32_t* W, int B, int Na, int S,
                                   const int32_t* S_host, hipStream_t stream);
hipError_t launch_normalise(const void* vis, bool is_int, const int32_t* W, void* out, int B, int Na,
                            hipStream_t stream);

// ---------------------------------------------------------------- imaging
size_t imaging_workspace_bytes(int Na, int B, int N);
hipError_t launch_grid(const float2* vis, const int32_t* weights, const double* pos, const double* freq, int Na, int B,
                       int N, double du, float2* grid_out, double* norm, void* ws, hipStream_t stream);
hipError_t launch_image(const float2* grid, const double* norm, float* image, int N, void* ws, hipStream_t stream);

// ---------------------------------------------------------------- calibration
size_t cal_workspace_bytes(int Na, int P);
// checked (debug) mode: a process-wide switch and the count of non-finite
// values of a device buffer (kind: afc_value_type), read back to the host
void set_checked_mode(bool on);
bool checked_mode();
hipError_t count_nonfinite(const void* p, size_t n, int kind, unsigned long long* count, hipStream_t stream);
// Fixed device scratch of afc_calibrate_grad_noalloc (one per GPU) and its
// address on the current device.
constexpr size_t kCalScratchBytes = (size_t)AFC_CAL_NOALLOC_MAX_BYTES;
hipError_t cal_scratch_address(void** out);
// fl (uint8 [P][Nbl][2], nonzero = flagged) and wt (float [P][Nbl][2]) weight
// the loss per baseline and polarisation; both NULL = the unweighted loss
hipError_t launch_calibrate(int Na, int P, const float2* V, const float2* M, const float2* g,
                            double* loss, float2* grad, void* ws, hipStream_t stream,
                            const uint8_t* fl = nullptr, const float* wt = nullptr);
// gain solver: n_iter preconditioned-gradient (alternating least-squares)
// iterations from g, result phase-referenced to antenna 0, written to g
size_t cal_solve_workspace_bytes(int Na, int P);
hipError_t launch_calibrate_solve(int Na, int P, const float2* V, const float2* M, float2* g, int n_iter,
                                  double* loss, void* ws, hipStream_t stream, const uint8_t* fl = nullptr,
                                  const float* wt = nullptr);
// two-stage sigma clipping of XX / YY visibility amplitudes -> flags [P][Nbl][2]
size_t sigma_clip_workspace_bytes(int Na, int P);
hipError_t launch_sigma_clip(int Na, int P, const float2* V, float k, uint8_t* flags, void* ws, hipStream_t stream);
hipError_t launch_apply_vis_flags(int Na, int P, const uint8_t* flags, float2* V, float2* M, hipStream_t stream);

}  // namespace afc

namespace afc {
// Workgroup barrier that orders LDS only: waits for this wave's LDS
// operations, then s_barrier.  Unlike __syncthreads() it does not wait for
// outstanding global loads and stores, so prefetches stay in flight across it.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}
}  // namespace afc
