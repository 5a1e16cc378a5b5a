// Antenna flags in the batching form (Sec. "CPU Data Collation": flagged
// data carry weight 0 in the weighting matrix).  Instead of multiplying the
// baselines of flagged antennas and zeroing them afterwards, the plan's
// graph compacts the flagged antennas out of each subband: the channeliser
// stores only the receivers of unflagged antennas (in antenna order, at the
// front of the subband's rows), the X-engine correlates those and maps the
// compact indices back to the visibility layout, and one small kernel
// writes V = 0 and W = 0 for every baseline that touches a flagged antenna.
#include <hip/hip_runtime.h>

#include "afc_internal.h"

namespace afc {
namespace {

constexpr int kCompactThreads = 256;

// One workgroup per subband; the flags are scanned in antenna order, 256 at
// a time, with wave ballots for the prefix counts.
__global__ __launch_bounds__(kCompactThreads) void plan_compact_kernel(const uint8_t* __restrict__ flags, int Na,
                                                                     int32_t* __restrict__ inv,
                                                                     int32_t* __restrict__ amap,
                                                                     int32_t* __restrict__ flagged,
                                                                     int32_t* __restrict__ counts) {
    __shared__ int wave_act[kCompactThreads / 64], wave_fl[kCompactThreads / 64];
    const int b = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
    int base_act = 0, base_fl = 0;
    for (int a0 = 0; a0 < Na; a0 += kCompactThreads) {
        const int a = a0 + tid;
        const bool in = a < Na;
        const bool f = in && flags[(int64_t)b * Na + a] != 0;
        const bool act = in && !f;
        const uint64_t ma = __ballot(act), mf = __ballot(f);
        if (lane == 0) {
            wave_act[wv] = __popcll(ma);
            wave_fl[wv] = __popcll(mf);
        }
        __syncthreads();
        int pa = base_act, pf = base_fl, ta = 0, tf = 0;
        for (int w = 0; w < kCompactThreads / 64; ++w) {
            if (w < wv) {
                pa += wave_act[w];
                pf += wave_fl[w];
            }
            ta += wave_act[w];
            tf += wave_fl[w];
        }
        if (act) {
            const int c = pa + __popcll(ma & below);
            inv[(int64_t)b * Na + a] = c;
            amap[(int64_t)b * Na + c] = a;
        } else if (f) {
            inv[(int64_t)b * Na + a] = -1;
            flagged[(int64_t)b * Na + pf + __popcll(mf & below)] = a;
        }
        base_act += ta;
        base_fl += tf;
        __syncthreads();
    }
    if (tid == 0) {
        counts[2 * b] = base_act;
        counts[2 * b + 1] = base_fl;
    }
}

// Block (k, b): the k-th flagged antenna f of subband b zeroes its Na
// baselines (f, c) / (c, f) in all 64 channels, 32 bytes each, and their
// weights.  Baselines of two flagged antennas are zeroed twice, with the
// same value.
__global__ __launch_bounds__(256) void plan_zero_flagged_kernel(const int32_t* __restrict__ flagged,
                                                                const int32_t* __restrict__ counts, int Na,
                                                                char* __restrict__ vis, int32_t* __restrict__ weights) {
    const int k = blockIdx.x, b = blockIdx.y;
    if (k >= counts[2 * b + 1]) return;                       // uniform
    const int f = flagged[(int64_t)b * Na + k];
    const int64_t nbl = (int64_t)Na * (Na + 1) / 2;
    char* vb = vis + (int64_t)b * kP * nbl * 32;
    for (int e = threadIdx.x; e < Na * kP; e += blockDim.x) {
        const int c = e % Na, ch = e / Na;
        const int hi = max(f, c), lo = min(f, c);
        const int64_t bl = (int64_t)hi * (hi + 1) / 2 + lo;
        uint4* dst = reinterpret_cast<uint4*>(vb + ((int64_t)ch * nbl + bl) * 32);
        dst[0] = make_uint4(0u, 0u, 0u, 0u);
        dst[1] = make_uint4(0u, 0u, 0u, 0u);
        if (weights && ch == 0) weights[(int64_t)b * nbl + bl] = 0;
    }
}

}  // namespace

hipError_t launch_plan_compact(const uint8_t* flags, int B, int Na, int32_t* inv, int32_t* amap, int32_t* flagged,
                               int32_t* counts, hipStream_t stream) {
    hipLaunchKernelGGL(plan_compact_kernel, dim3(B), dim3(kCompactThreads), 0, stream, flags, Na, inv, amap, flagged,
                       counts);
    return hipGetLastError();
}

hipError_t launch_plan_zero_flagged(const int32_t* flagged, const int32_t* counts, int B, int Na, void* vis,
                                    int32_t* weights, hipStream_t stream) {
    hipLaunchKernelGGL(plan_zero_flagged_kernel, dim3(Na, B), dim3(256), 0, stream, flagged, counts, Na,
                       reinterpret_cast<char*>(vis), weights);
    return hipGetLastError();
}

}  // namespace afc
