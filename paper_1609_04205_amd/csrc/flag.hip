// Real-time flagging by sigma clipping (Sec. "Calibration Pipeline",
// flagging: visibility amplitudes are clipped against a threshold above the
// locally computed RMS, first across the visibilities of a channel, then
// across the channels of each visibility), on the XX and YY correlations.
//
//   stage 1, per (channel, pol):  RMS^2 = mean over cross-correlations of
//            |V|^2; flag |V|^2 > k^2 RMS^2
//   stage 2, per (baseline, pol): RMS^2 = mean over the channels not flagged
//            in stage 1; flag the channels with |V|^2 > k^2 RMS^2
// Autocorrelations are neither used nor flagged.  |V|^2 is formed in float64
// (exact products of the float32 components); every sum runs in a fixed
// order, so the flags are reproducible.
#include "afc_internal.h"

namespace afc {
namespace {

constexpr int kClipChunk = 4096;   // baselines per partial sum of stage 1

// antenna pair of a lower-triangle index, bl = a(a+1)/2 + b
__device__ __forceinline__ bool is_auto(int64_t bl) {
    int64_t a = (int64_t)((sqrt(8.0 * (double)bl + 1.0) - 1.0) * 0.5);
    while (a * (a + 1) / 2 > bl) --a;
    while ((a + 1) * (a + 2) / 2 <= bl) ++a;
    return bl - a * (a + 1) / 2 == a;
}

__device__ __forceinline__ double abs2(float2 v) { return (double)v.x * v.x + (double)v.y * v.y; }

__global__ __launch_bounds__(256) void clip_partial_kernel(int64_t nbl, const float2* __restrict__ V,
                                                           double* __restrict__ part, int n_chunks) {
    __shared__ double red[256];
    const int c = blockIdx.x, ch = blockIdx.y, pol = blockIdx.z;
    const int64_t bl0 = (int64_t)c * kClipChunk, bl1 = min(nbl, bl0 + kClipChunk);
    double acc = 0.0;
    for (int64_t bl = bl0 + threadIdx.x; bl < bl1; bl += 256)
        if (!is_auto(bl)) acc += abs2(V[((int64_t)ch * nbl + bl) * 4 + pol * 3]);
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(int64_t)(ch * 2 + pol) * n_chunks + c] = red[0];
}

__global__ void clip_mean_kernel(int P, int n_chunks, int64_t n_cross, const double* __restrict__ part,
                                 double* __restrict__ mean) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= P * 2) return;
    double s = 0.0;
    for (int c = 0; c < n_chunks; ++c) s += part[(int64_t)e * n_chunks + c];
    mean[e] = n_cross > 0 ? s / (double)n_cross : 0.0;
}

// stage 1: one thread per (channel, baseline), both polarisations
__global__ void clip_stage1_kernel(int P, int64_t nbl, const float2* __restrict__ V, const double* __restrict__ mean,
                                   double k2, uint8_t* __restrict__ flags) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)P * nbl) return;
    const int ch = (int)(e / nbl);
    const int64_t bl = e % nbl;
    const bool au = is_auto(bl);
#pragma unroll
    for (int pol = 0; pol < 2; ++pol) {
        const double a2 = abs2(V[e * 4 + pol * 3]);
        flags[e * 2 + pol] = (!au && a2 > k2 * mean[ch * 2 + pol]) ? 1 : 0;
    }
}

// stage 2: one thread per (baseline, polarisation), channels in order
__global__ void clip_stage2_kernel(int P, int64_t nbl, const float2* __restrict__ V, double k2,
                                   uint8_t* __restrict__ flags) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nbl * 2) return;
    const int64_t bl = e >> 1;
    const int pol = (int)(e & 1);
    if (is_auto(bl)) return;
    double s = 0.0;
    int n = 0;
    for (int ch = 0; ch < P; ++ch) {
        const int64_t i = (int64_t)ch * nbl + bl;
        if (flags[i * 2 + pol] == 0) {
            s += abs2(V[i * 4 + pol * 3]);
            ++n;
        }
    }
    if (n == 0) return;
    const double m = s / (double)n;
    for (int ch = 0; ch < P; ++ch) {
        const int64_t i = (int64_t)ch * nbl + bl;
        if (abs2(V[i * 4 + pol * 3]) > k2 * m) flags[i * 2 + pol] = 1;
    }
}

__global__ void apply_flags_kernel(int64_t n, const uint8_t* __restrict__ flags, float2* __restrict__ V,
                                   float2* __restrict__ M) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
#pragma unroll
    for (int pol = 0; pol < 2; ++pol)
        if (flags[e * 2 + pol]) {
            if (V) V[e * 4 + pol * 3] = make_float2(0.0f, 0.0f);
            if (M) M[e * 4 + pol * 3] = make_float2(0.0f, 0.0f);
        }
}

int clip_chunks(int64_t nbl) { return (int)ceil_div(nbl, kClipChunk); }

}  // namespace

size_t sigma_clip_workspace_bytes(int Na, int P) {
    const int64_t nbl = (int64_t)Na * (Na + 1) / 2;
    return ((size_t)P * 2 * clip_chunks(nbl) + (size_t)P * 2) * sizeof(double);
}

hipError_t launch_sigma_clip(int Na, int P, const float2* V, float k, uint8_t* flags, void* ws, hipStream_t stream) {
    const int64_t nbl = (int64_t)Na * (Na + 1) / 2;
    const int nc = clip_chunks(nbl);
    double* part = reinterpret_cast<double*>(ws);
    double* mean = part + (size_t)P * 2 * nc;
    const double k2 = (double)k * (double)k;
    hipLaunchKernelGGL(clip_partial_kernel, dim3(nc, P, 2), dim3(256), 0, stream, nbl, V, part, nc);
    hipLaunchKernelGGL(clip_mean_kernel, dim3((unsigned)ceil_div(P * 2, 256)), dim3(256), 0, stream, P, nc,
                       nbl - Na, part, mean);
    hipLaunchKernelGGL(clip_stage1_kernel, dim3((unsigned)ceil_div((int64_t)P * nbl, 256)), dim3(256), 0, stream, P,
                       nbl, V, mean, k2, flags);
    hipLaunchKernelGGL(clip_stage2_kernel, dim3((unsigned)ceil_div(nbl * 2, 256)), dim3(256), 0, stream, P, nbl, V,
                       k2, flags);
    return hipGetLastError();
}

hipError_t launch_apply_vis_flags(int Na, int P, const uint8_t* flags, float2* V, float2* M, hipStream_t stream) {
    const int64_t n = (int64_t)P * Na * (Na + 1) / 2;
    hipLaunchKernelGGL(apply_flags_kernel, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, stream, n, flags, V, M);
    return hipGetLastError();
}

}  // namespace afc
