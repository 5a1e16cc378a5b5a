// Lost packets and the weighting matrix (Sec. "CPU Data Collation": the
// correlator handles lost UDP packets and produces a weighting matrix with
// the visibilities; Sec. "Calibration Pipeline": the visibilities are
// re-weighted for the lost data).
//
// A spectrum of antenna a is valid iff every input sample of its FIR window
// (spectrum s reads samples s*Ps .. (s+T)*Ps - 1) arrived.  Invalid spectra
// are zeroed in the channelised array, so that the X-engine's sums run over
// the spectra valid for both antennas of a baseline, and the weight of a
// baseline is the number of those spectra.
//
//   validity_kernel   packet flags -> bit masks [B][ceil(S/32)][Na]
//   zero_kernel       zero the channelised samples of invalid spectra
//   weights_kernel    W[b][bl(a,c)] = popcount of (v_a & v_c) over s < S_b
//   normalise_kernel  V / W per baseline, float2 out
#include "afc_internal.h"

namespace afc {
namespace {

// floor(n / d) for d > 0 and any sign of n
__device__ __forceinline__ int64_t floor_div(int64_t n, int64_t d) {
    return n >= 0 ? n / d : -((-n + d - 1) / d);
}

// One thread = one antenna and one word of 32 spectra; threads of a block
// take consecutive antennas, so the packet flags of one packet row and the
// output words are read and written contiguously.
__global__ void validity_kernel(const uint8_t* __restrict__ pkt, uint32_t* __restrict__ v, int Na, int S,
                                int Wd, int64_t n_pk, int Q, int Ps) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    const int wd = blockIdx.y;
    const int b = blockIdx.z;
    if (a >= Na) return;
    const int s0 = wd * 32;
    const int n = min(32, S - s0);
    uint32_t bits = n == 32 ? 0xFFFFFFFFu : ((1u << n) - 1u);
    // packets touched by the windows of spectra s0 .. s0+n-1
    const int64_t k_lo = (int64_t)s0 * Ps / Q;
    const int64_t k_hi = ((int64_t)(s0 + n - 1 + kT) * Ps - 1) / Q;
    const uint8_t* pb = pkt + (int64_t)b * n_pk * Na + a;
    for (int64_t k = k_lo; k <= k_hi; ++k) {
        const bool arrived = k < n_pk && pb[k * Na] != 0;
        if (arrived) continue;
        // spectra whose window [s Ps, (s+T) Ps - 1] meets [k Q, (k+1) Q - 1]
        const int64_t lo = max(floor_div(k * Q - (int64_t)kT * Ps, Ps) + 1, (int64_t)s0);
        const int64_t hi = min(floor_div((k + 1) * Q - 1, Ps), (int64_t)(s0 + n - 1));
        for (int64_t s = lo; s <= hi; ++s) bits &= ~(1u << (s - s0));
    }
    v[((int64_t)b * Wd + wd) * Na + a] = bits;
}

// One thread = one antenna and one word of 32 spectra; it writes zeros
// only where a spectrum is invalid (lost data is rare), over both
// receivers of the antenna and all channels.
template <typename SampleT>
__global__ void zero_kernel(const uint32_t* __restrict__ v, SampleT* __restrict__ z, int Na, int S, int Wd,
                            int Sb) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    const int wd = blockIdx.y;
    const int b = blockIdx.z;
    if (a >= Na) return;
    const int s0 = wd * 32;
    const int n = min(32, S - s0);
    const uint32_t all = n == 32 ? 0xFFFFFFFFu : ((1u << n) - 1u);
    uint32_t bad = ~v[((int64_t)b * Wd + wd) * Na + a] & all;
    const int N = 2 * Na;
    const int64_t ch_stride = (int64_t)Sb * N * kSBlk;
    SampleT* zb = z + (int64_t)b * kP * ch_stride;
    const SampleT zero{};
    while (bad) {
        const int j = __builtin_ctz(bad);
        bad &= bad - 1u;
        const int s = s0 + j;
        const int64_t off = ((int64_t)(s >> 3) * N + 2 * a) * kSBlk + (s & 7);
        for (int k = 0; k < kP; ++k) {
            zb[k * ch_stride + off] = zero;
            zb[k * ch_stride + off + kSBlk] = zero;
        }
    }
}

struct WeightArgs {
    const uint32_t* v;
    const uint8_t* flags;
    int32_t* W;
    int Na, Wd, n_tiles;
    int S[AFC_MAX_SUBBANDS];
};

constexpr int kWT = 32;          // antennas per tile side
constexpr int kWChunk = 128;     // words of 32 spectra staged per pass

// One workgroup (256 threads) = one 32 x 32 tile (a-tile >= c-tile) of one
// subband; each thread sums four (a, c) pairs, masks staged in LDS.
__global__ __launch_bounds__(256) void weights_kernel(WeightArgs w) {
    __shared__ uint32_t la[kWChunk][kWT], lc[kWChunk][kWT];
    const int b = blockIdx.y;
    // tile pair from the linear index: ta >= tc
    int t = blockIdx.x, ta = 0;
    while (t > ta) { t -= ta + 1; ++ta; }
    const int tc = t;
    const int Na = w.Na, Wd = w.Wd, S = w.S[b];
    const int tid = threadIdx.x;
    const int ci = tid & 15, ai = tid >> 4;
    int cnt[2][2] = {{0, 0}, {0, 0}};
    const uint32_t* vb = w.v + (int64_t)b * Wd * Na;
    for (int w0 = 0; w0 < Wd; w0 += kWChunk) {
        const int nw = min(kWChunk, Wd - w0);
        for (int e = tid; e < nw * kWT; e += 256) {
            const int wd = e / kWT, j = e % kWT;
            const int s0 = (w0 + wd) * 32;
            // spectra >= S of this subband do not count
            const int n = max(0, min(32, S - s0));
            const uint32_t m = n == 32 ? 0xFFFFFFFFu : ((1u << n) - 1u);
            const int a = ta * kWT + j, c = tc * kWT + j;
            la[wd][j] = a < Na ? vb[(int64_t)(w0 + wd) * Na + a] & m : 0u;
            lc[wd][j] = c < Na ? vb[(int64_t)(w0 + wd) * Na + c] & m : 0u;
        }
        __syncthreads();
        for (int wd = 0; wd < nw; ++wd) {
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y)
                    cnt[x][y] += __popc(la[wd][ai + 16 * x] & lc[wd][ci + 16 * y]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
            const int a = ta * kWT + ai + 16 * x, c = tc * kWT + ci + 16 * y;
            if (a >= Na || c > a) continue;
            const bool flagged = w.flags && (w.flags[(int64_t)b * Na + a] || w.flags[(int64_t)b * Na + c]);
            w.W[(int64_t)b * ((int64_t)Na * (Na + 1) / 2) + (int64_t)a * (a + 1) / 2 + c] = flagged ? 0 : cnt[x][y];
        }
}

// out = vis / W per baseline (0 where W = 0); one thread = one baseline's
// 2 x 2 block of one channel; blockIdx.y = subband * P + channel, so the
// indices need no 64-bit division.  Every byte is touched once: loads and
// stores are non-temporal.
typedef int nv4i __attribute__((ext_vector_type(4)));
typedef float nv4f __attribute__((ext_vector_type(4)));

template <bool kInt>
__global__ void normalise_kernel(const void* __restrict__ vis, const int32_t* __restrict__ W,
                                 float2* __restrict__ out, int nbl, int P) {
    const int bl = blockIdx.x * blockDim.x + threadIdx.x;
    if (bl >= nbl) return;
    const int slice = blockIdx.y;                           // subband * P + channel
    const int64_t e = (int64_t)slice * nbl + bl;
    const int32_t wt = W[(int64_t)(slice / P) * nbl + bl];
    float2 r[4];
    if constexpr (kInt) {
        const nv4i* src = reinterpret_cast<const nv4i*>(vis) + e * 2;
        const nv4i u0 = __builtin_nontemporal_load(src), u1 = __builtin_nontemporal_load(src + 1);
        const int vv[8] = {u0.x, u0.y, u0.z, u0.w, u1.x, u1.y, u1.z, u1.w};
#pragma unroll
        for (int j = 0; j < 4; ++j)
            r[j] = wt > 0 ? make_float2((float)((double)vv[2 * j] / wt), (float)((double)vv[2 * j + 1] / wt))
                          : make_float2(0.0f, 0.0f);
    } else {
        const nv4f* src = reinterpret_cast<const nv4f*>(vis) + e * 2;
        const nv4f f0 = __builtin_nontemporal_load(src), f1 = __builtin_nontemporal_load(src + 1);
        const float vv[8] = {f0.x, f0.y, f0.z, f0.w, f1.x, f1.y, f1.z, f1.w};
        const float fw = (float)wt;
#pragma unroll
        for (int j = 0; j < 4; ++j)
            r[j] = wt > 0 ? make_float2(vv[2 * j] / fw, vv[2 * j + 1] / fw) : make_float2(0.0f, 0.0f);
    }
    nv4f* dst = reinterpret_cast<nv4f*>(out) + e * 2;
    __builtin_nontemporal_store(nv4f{r[0].x, r[0].y, r[1].x, r[1].y}, dst);
    __builtin_nontemporal_store(nv4f{r[2].x, r[2].y, r[3].x, r[3].y}, dst + 1);
}

struct alignas(4) Half2Raw { uint16_t x, y; };
struct alignas(2) I8x2 { int8_t x, y; };

}  // namespace

hipError_t launch_validity(const uint8_t* pkt, uint32_t* v, int B, int Na, int S, int64_t n_pk, int Q, int Ps,
                           hipStream_t stream) {
    const int Wd = (int)ceil_div(S, 32);
    const dim3 grid((unsigned)ceil_div(Na, 256), (unsigned)Wd, (unsigned)B);
    hipLaunchKernelGGL(validity_kernel, grid, dim3(256), 0, stream, pkt, v, Na, S, Wd, n_pk, Q, Ps);
    return hipGetLastError();
}

hipError_t launch_zero_invalid(const uint32_t* v, void* z, afc_dtype dt, int B, int Na, int S, hipStream_t stream) {
    const int Wd = (int)ceil_div(S, 32);
    const int Sb = (int)ceil_div(S, kSBlk);
    const dim3 grid((unsigned)ceil_div(Na, 256), (unsigned)Wd, (unsigned)B);
    if (dt == AFC_F32)
        hipLaunchKernelGGL(zero_kernel<float2>, grid, dim3(256), 0, stream, v, reinterpret_cast<float2*>(z), Na, S,
                           Wd, Sb);
    else if (dt == AFC_F16)
        hipLaunchKernelGGL(zero_kernel<Half2Raw>, grid, dim3(256), 0, stream, v, reinterpret_cast<Half2Raw*>(z), Na,
                           S, Wd, Sb);
    else
        hipLaunchKernelGGL(zero_kernel<I8x2>, grid, dim3(256), 0, stream, v, reinterpret_cast<I8x2*>(z), Na, S, Wd,
                           Sb);
    return hipGetLastError();
}

hipError_t launch_validity_weights(const uint32_t* v, const uint8_t* flags, int32_t* W, int B, int Na, int S,
                                   const int32_t* S_host, hipStream_t stream) {
    WeightArgs w{};
    w.v = v;
    w.flags = flags;
    w.W = W;
    w.Na = Na;
    w.Wd = (int)ceil_div(S, 32);
    const int nt = (int)ceil_div(Na, kWT);
    w.n_tiles = nt;
    for (int b = 0; b < B; ++b) w.S[b] = S_host ? S_host[b] : S;
    const dim3 grid((unsigned)(nt * (nt + 1) / 2), (unsigned)B);
    hipLaunchKernelGGL(weights_kernel, grid, dim3(256), 0, stream, w);
    return hipGetLastError();
}

hipError_t launch_normalise(const void* vis, bool is_int, const int32_t* W, void* out, int B, int Na,
                            hipStream_t stream) {
    const int64_t nbl = (int64_t)Na * (Na + 1) / 2;
    if (nbl > (1 << 30) || (int64_t)B * kP > 65535) return hipErrorInvalidValue;
    const dim3 grid((unsigned)ceil_div(nbl, 256), (unsigned)(B * kP));
    if (is_int)
        hipLaunchKernelGGL(normalise_kernel<true>, grid, dim3(256), 0, stream, vis, W,
                           reinterpret_cast<float2*>(out), (int)nbl, kP);
    else
        hipLaunchKernelGGL(normalise_kernel<false>, grid, dim3(256), 0, stream, vis, W,
                           reinterpret_cast<float2*>(out), (int)nbl, kP);
    return hipGetLastError();
}

}  // namespace afc
