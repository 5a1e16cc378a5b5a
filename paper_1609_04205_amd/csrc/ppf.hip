// Polyphase filter bank (FIR + 64-point FFT) with the corner turn fused into
// the store.  Sec. "Polyphase Filterbank" (a bank of 16-tap FIR filters per
// receiver subband stream, then a complex FFT of the filter outputs) and
// Sec. "Delay, Bandpass Compensation and Transpose Kernel" (exchange of the
// parallel axis from channels to receivers).
//
//   u[s][p] = sum_{t<16} h[t*64 + p] x[(s+t)*64 + p]
//   y[s][k] = sum_{p<64} u[s][p] exp(-2 pi i k p / 64)
//
// Mapping (one workgroup = 16 receivers x a run of spectra, 16 waves):
//  * FIR phase: wave w owns the four branches p = w + 16 j (j = 0..3).  Lane
//    (il, j) owns both components of receiver i0 + il for branch j (one
//    32-bit load per spectrum).  The 16-deep windows live in registers and
//    slide by one sample per spectrum; loads are coalesced rows of the
//    time-major input.
//  * The first radix-4 stage of the FFT (over j) runs across each lane quad
//    in two DPP exchanges (sums and differences with the lane at j ^ 2, then
//    the +-1, +-i combinations with the lane at j ^ 1); quad lane j then owns
//    k1 = the bit reverse of j and applies the twiddle exp(-2 pi i p1 k1 / 64).
//    Results go to LDS as [spectrum][k1][p1][il] for 16 spectra.
//  * FFT phase: a lane owns (receiver, spectrum, k1) and does the remaining
//    16-point FFT over p1 in registers (radix-4 x radix-4), producing
//    channels k = k1 + 4 k2.  Lanes are ordered so that each store writes
//    8 receivers x 8 spectra contiguously in the [k][block][receiver][slot]
//    output layout.
#include <hip/hip_fp16.h>

#include "afc_internal.h"
#include "ppf_common.h"

namespace afc {
namespace {
using namespace ppfk;

constexpr int kNi = 16;                      // receivers per workgroup
constexpr int kThreads = 1024;               // 16 waves
// LDS rows padded so that the FIR-phase stores (16 lanes: 4 receivers x 4 k1)
// and the FFT-phase loads (16 lanes: 8 spectra x 2 receivers) hit 32
// distinct banks: k1 rows start 8 banks apart, spectrum rows 4 banks apart
constexpr int kKStride = 16 * 16 + 4;        // float2 per k1 row
constexpr int kSStride = 4 * kKStride + 2;   // float2 per spectrum
constexpr int kSpectraPerPhase = 16;
constexpr int kChunk = 768;                  // spectra per workgroup, a multiple of 16
constexpr int kDepth = 4;                    // spectra of loads in flight per lane (divides 16)

// One workgroup: receivers [i0, i0+16) of one subband, spectra [s_begin, s_end).
template <int DT>
__device__ __forceinline__ void ppf_body(const int16_t* __restrict__ xs, const float* __restrict__ taps,
                                         void* __restrict__ zs, const Tw64& tw, int N, int S, int Sb,
                                         int i0, int s_begin, int s_end, float gain, float2* lds,
                                         float* ltaps) {
    const int tid = threadIdx.x;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;

    // ---- FIR-phase roles: lane = il * 4 + j, branch p = p1 + 16 j of
    // receiver i0 + il, both components (one 32-bit load per spectrum)
    const int j = lane & 3, il = lane >> 2;
    // Receivers beyond N read receiver N-1 and spectra beyond S read the last
    // valid samples: every load is in bounds and unconditional (no load waits
    // on another); such lanes and spectra are never stored.
    const int rcv = min(i0 + il, N - 1);
    const int p1 = wv;
    const int row_stride = N * 2;
    const int lane_off = (p1 + 16 * j) * row_stride + rcv * 2;          // branch p at row 0, re/im pair
    const int64_t spec_stride = (int64_t)kP * row_stride;               // int16 elements per spectrum row

    // taps staged in LDS as [branch][t]; each FIR phase reloads its 32 taps,
    // so they do not occupy registers during the FFT phase
    for (int e = tid; e < kT * kP; e += kThreads) {
        const int t = e / kP, p = e % kP;
        ltaps[p * kT + t] = taps[e];
    }
    lds_barrier();
    const float4* tp = reinterpret_cast<const float4*>(ltaps + (p1 + 16 * j) * kT);

    // radix-4 over j across the lane quad: step 1 (partner j ^ 2) gives
    // u0+u2, u1+u3, u0-u2, u1-u3 in lanes 0..3, step 2 (partner j ^ 1)
    // own * al + partner * be gives A[k1o], k1o the bit reverse of j
    const int k1o = ((j & 1) << 1) | (j >> 1);
    const float s1 = (j >> 1) ? -1.0f : 1.0f;
    const float2 al = j == 0 ? make_float2(1.0f, 0.0f) : j == 1 ? make_float2(-1.0f, 0.0f)
                    : j == 2 ? make_float2(1.0f, 0.0f) : make_float2(0.0f, 1.0f);
    const float2 be = j == 2 ? make_float2(0.0f, -1.0f) : make_float2(1.0f, 0.0f);
    // twiddle exp(-2 pi i p1 k1o / 64) (uniform loads of the four candidates, then a per-lane select)
    const float2 tw1 = tw.w[p1 & 63], tw2 = tw.w[(2 * p1) & 63], tw3 = tw.w[(3 * p1) & 63];
    const float2 tw_o = k1o == 0 ? make_float2(1.0f, 0.0f) : k1o == 1 ? tw1 : k1o == 2 ? tw2 : tw3;

    // re/im pair of branch p at spectrum-row m (wave-uniform 64-bit row
    // pointer + 32-bit lane offset); converted to float only where it enters
    // the window, so that a load in flight is not waited on before it is needed
    auto ld = [&](int m) -> int {
        const int16_t* rowp = xs + (int64_t)min(m, S + kT - 2) * spec_stride;
        return *reinterpret_cast<const int*>(rowp + lane_off);
    };
    float win[2][16];
    auto put = [&](int slot, int d) {
        win[0][slot] = (float)(int)(short)(d & 0xFFFF);
        win[1][slot] = (float)(d >> 16);
    };

    // history: window slot m % 16 holds x_p[m]; s_begin is a multiple of 16
#pragma unroll
    for (int m = 0; m < 15; ++m) put(m, ld(s_begin + m));
    win[0][15] = win[1][15] = 0.0f;

    // ---- FFT-phase roles
    const int k1 = wv & 3, rh = (wv >> 2) & 1, bh = wv >> 3;
    const int sl = lane & 7, ii = lane >> 3;
    const int ilf = rh * 8 + ii;
    const int rf = i0 + ilf;

    // software pipeline of the per-spectrum loads, kDepth spectra ahead
    int pf[kDepth];
#pragma unroll
    for (int d = 0; d < kDepth; ++d) pf[d] = ld(s_begin + d + 15);

    for (int sg = s_begin; sg < s_end; sg += kSpectraPerPhase) {
        float h[16];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const float4 a0 = tp[v];
            h[4 * v] = a0.x; h[4 * v + 1] = a0.y; h[4 * v + 2] = a0.z; h[4 * v + 3] = a0.w;
        }
#pragma unroll
        for (int q = 0; q < kSpectraPerPhase; ++q) {
            put((q + 15) & 15, pf[q % kDepth]);
            pf[q % kDepth] = ld(sg + q + kDepth + 15);
            float u[2];
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                float acc = 0.0f;
#pragma unroll
                for (int t = 0; t < 16; ++t) acc = fmaf(h[t], win[c][(q + t) & 15], acc);
                u[c] = acc;
            }
            const float e0 = fmaf(s1, u[0], quad_xor<2>(u[0]));
            const float e1 = fmaf(s1, u[1], quad_xor<2>(u[1]));
            const float f0 = quad_xor<1>(e0), f1 = quad_xor<1>(e1);
            float2 v;
            v.x = al.x * e0 - al.y * e1 + be.x * f0 - be.y * f1;
            v.y = al.x * e1 + al.y * e0 + be.x * f1 + be.y * f0;
            const float2 o = cmul(v, tw_o);
            lds[q * kSStride + k1o * kKStride + p1 * 16 + il] = o;
            __builtin_amdgcn_sched_barrier(0);
        }
        lds_barrier();
        {
            float2 a[16];
            const float2* src = lds + (8 * bh + sl) * kSStride + k1 * kKStride + ilf;
#pragma unroll
            for (int p = 0; p < 16; ++p) a[p] = src[p * 16];
            dft16(a);
            const int s = sg + 8 * bh + sl;
            const int blk = (sg >> 3) + bh;
            if (rf < N && blk < Sb) {
                const bool live = s < S;
                const unsigned lane_zoff = (blk * N + rf) * kSBlk + sl;     // samples within a channel
                const int64_t ch_stride = (int64_t)Sb * N * kSBlk;          // samples per channel
                // spectra >= S are stored as zeros (int8: through a zero gain)
                const float g = live ? gain : 0.0f;
#pragma unroll
                for (int ga = 0; ga < 4; ++ga)
#pragma unroll
                    for (int de = 0; de < 4; ++de) {
                        const int k = k1 + 4 * (ga + 4 * de);
                        float2 y = a[4 * ga + de];
                        if constexpr (DT != AFC_I8)
                            if (!live) y = make_float2(0.0f, 0.0f);
                        store_sample<DT>(zs, (int64_t)k * ch_stride, lane_zoff, y, g);
                    }
            }
        }
        lds_barrier();
    }
}

template <int DT>
__global__ __launch_bounds__(kThreads) void ppf_kernel(const int16_t* __restrict__ x, const float* __restrict__ taps,
                                                       void* __restrict__ z, Tw64 tw, int64_t x_sb_stride,
                                                       int64_t z_sb_bytes, int N, int S, int Sb, int n_groups,
                                                       int n_chunks, int total, int per_xcd, float gain) {
    __shared__ float2 lds[kSpectraPerPhase * kSStride];
    __shared__ __attribute__((aligned(16))) float ltaps[kT * kP];
    // workgroups go round-robin over the 8 XCDs: give each XCD a contiguous
    // range with neighbouring receiver groups (which share 128-byte lines of
    // the input rows) adjacent in time
    const int w = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
    if (w >= total) return;
    const int grp = w % n_groups;
    const int chunk = (w / n_groups) % n_chunks;
    const int sb = w / (n_groups * n_chunks);
    const int s_begin = chunk * kChunk;
    const int s_end = min(S, s_begin + kChunk);
    ppf_body<DT>(x + sb * x_sb_stride, taps, reinterpret_cast<char*>(z) + sb * z_sb_bytes, tw, N, S, Sb,
                 grp * kNi, s_begin, s_end, gain, lds, ltaps);
}

// Batched form: one launch over per-subband jobs with their own S, type and gain.
__global__ __launch_bounds__(kThreads) void ppf_batched_kernel(const int16_t* __restrict__ x,
                                                              const float* __restrict__ taps, void* __restrict__ z,
                                                              Tw64 tw, const PpfItem* __restrict__ items,
                                                              int N, int n_groups, int n_chunks, int total,
                                                              int per_xcd) {
    __shared__ float2 lds[kSpectraPerPhase * kSStride];
    __shared__ __attribute__((aligned(16))) float ltaps[kT * kP];
    // XCD-aware order as in ppf_kernel: neighbouring receiver groups (which
    // share 128-byte lines of the input rows) run on one XCD at one time
    const int w = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
    if (w >= total) return;
    const int grp = w % n_groups;
    const int chunk = (w / n_groups) % n_chunks;
    const int it = w / (n_groups * n_chunks);
    const PpfItem item = items[it];
    const int s_begin = chunk * kChunk;
    if (s_begin >= item.S) return;                       // uniform over the workgroup
    const int s_end = min(item.S, s_begin + kChunk);
    const int16_t* xs = x + item.x_off;
    void* zs = reinterpret_cast<char*>(z) + item.z_off;
    if (item.dt == AFC_F32)
        ppf_body<AFC_F32>(xs, taps, zs, tw, N, item.S, item.Sb, grp * kNi, s_begin, s_end, item.gain, lds, ltaps);
    else if (item.dt == AFC_F16)
        ppf_body<AFC_F16>(xs, taps, zs, tw, N, item.S, item.Sb, grp * kNi, s_begin, s_end, item.gain, lds, ltaps);
    else
        ppf_body<AFC_I8>(xs, taps, zs, tw, N, item.S, item.Sb, grp * kNi, s_begin, s_end, item.gain, lds, ltaps);
}

}  // namespace

hipError_t launch_ppf(const PpfLaunch& a, hipStream_t stream) {
    static const Tw64 tw = make_twiddles();
    const int n_groups = (int)ceil_div(a.N, kNi);
    const int n_chunks = (int)ceil_div(a.S, kChunk);
    const int total = (int)((int64_t)a.B * n_groups * n_chunks);
    const int per_xcd = (int)ceil_div(total, 8);
    const dim3 grid((unsigned)(per_xcd * 8));
    const int64_t z_sb_bytes = a.z_sb_stride * sample_bytes(a.dt);
    switch (a.dt) {
        case AFC_F32:
            hipLaunchKernelGGL(ppf_kernel<AFC_F32>, grid, dim3(kThreads), 0, stream, a.x, a.taps, a.z, tw,
                               a.x_sb_stride, z_sb_bytes, a.N, a.S, a.Sb, n_groups, n_chunks, total, per_xcd, a.gain);
            break;
        case AFC_F16:
            hipLaunchKernelGGL(ppf_kernel<AFC_F16>, grid, dim3(kThreads), 0, stream, a.x, a.taps, a.z, tw,
                               a.x_sb_stride, z_sb_bytes, a.N, a.S, a.Sb, n_groups, n_chunks, total, per_xcd, a.gain);
            break;
        default:
            hipLaunchKernelGGL(ppf_kernel<AFC_I8>, grid, dim3(kThreads), 0, stream, a.x, a.taps, a.z, tw,
                               a.x_sb_stride, z_sb_bytes, a.N, a.S, a.Sb, n_groups, n_chunks, total, per_xcd, a.gain);
            break;
    }
    return hipGetLastError();
}

hipError_t launch_ppf_batched(const int16_t* x, const float* taps, void* z_ws, const PpfItem* items_dev,
                              int n_items, int N, int max_S, hipStream_t stream) {
    static const Tw64 tw = make_twiddles();
    const int n_groups = (int)ceil_div(N, kNi);
    const int n_chunks = (int)ceil_div(max_S, kChunk);
    const int64_t total64 = (int64_t)n_items * n_groups * n_chunks;
    if (total64 > (1LL << 30)) return hipErrorInvalidValue;
    const int total = (int)total64;
    const int per_xcd = (int)ceil_div(total, 8);
    const dim3 grid((unsigned)(per_xcd * 8));
    hipLaunchKernelGGL(ppf_batched_kernel, grid, dim3(kThreads), 0, stream, x, taps, z_ws, tw, items_dev, N,
                       n_groups, n_chunks, total, per_xcd);
    return hipGetLastError();
}

}  // namespace afc
