// Polyphase filter bank (FIR + 64-point FFT) with the corner turn fused into
// the store.  Sec. "Polyphase Filterbank" (a bank of 16-tap FIR filters per
// receiver subband stream, then a complex FFT of the filter outputs) and
// Sec. "Delay, Bandpass Compensation and Transpose Kernel" (exchange of the
// parallel axis from channels to receivers).
//
//   u[s][p] = sum_{t<16} h[t*64 + p] x[(s+t)*64 + p]
//   y[s][k] = sum_{p<64} u[s][p] exp(-2 pi i k p / 64)
//
// Mapping (one workgroup = 16 receivers x a run of spectra, 16 waves; 8 in
// the batched kernel):
//  * FIR phase on the matrix cores.  For one branch p and a phase of 16
//    spectra the filter is a banded matrix product: U[m][n] =
//    sum_k H[m][k] X[k][n] over the 32 input times k of the phase's window
//    (spectrum m uses times m .. m+15, so H[m][k] = h[(k-m)*64 + p] inside
//    the band and 0 outside), n = the 16 receivers, one product for the real
//    and one for the imaginary components.  It runs as fp16 MFMAs (16x16x32)
//    on exact splits with float32 sums: each int16 sample is 256 hb + lo,
//    entered as the fp16 parts hb and lo / 256 (both exact; the factor 256
//    goes into the unscaling), and each tap, scaled by a power of two 2^E
//    (per workgroup, so that the largest is near 2^15), is the sum of two
//    fp16 parts (22 significant bits, the rest below float32 rounding of
//    the sums); 2^(8-E) is folded into the twiddles.  Wave w owns the
//    branches p = p1 + 16 j with p1 = w (16 waves) or p1 in {w, w+8} (8
//    waves); lane (n, g) reads its band rows of H from tables of fp16 tap
//    pairs in LDS and loads the int16 pairs of receiver n at 4 times per
//    branch and phase (window slot k = 8 g + e <-> time 16 (e / 4) + 4 g +
//    e % 4: the first half is the previous phase's second half, so every
//    sample is loaded and converted once; odd phases swap the two halves'
//    slots, so that the converted parts stay in place in their registers).
//  * The product leaves U for 4 spectra of receiver n in each lane, for all
//    four branches p1 + 16 j, so the first radix-4 stage of the FFT (over j)
//    is lane-local; then the twiddle exp(-2 pi i p1 k1 / 64).  Results go to
//    LDS as [spectrum][k1][p1][receiver] for 16 spectra.
//  * FFT phase: a lane owns (receiver, spectrum, k1) and does the remaining
//    16-point FFT over p1 in registers (radix-4 x radix-4), producing
//    channels k = k1 + 4 k2 (two such jobs per lane with 8 waves).  Lanes
//    are ordered so that each store writes 8 receivers x 8 spectra
//    contiguously in the [k][block][receiver][slot] output layout.
#include <hip/hip_fp16.h>

#include <type_traits>

#include "afc_internal.h"
#include "ppf_common.h"

namespace afc {
namespace {
using namespace ppfk;

typedef float v4f __attribute__((ext_vector_type(4)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef _Float16 v4h __attribute__((ext_vector_type(4)));
typedef _Float16 h2 __attribute__((ext_vector_type(2)));
typedef unsigned v4u __attribute__((ext_vector_type(4)));
constexpr h2 kInv256 = {(_Float16)0.00390625f, (_Float16)0.00390625f};
constexpr h2 kMinus4 = {(_Float16)-4.0f, (_Float16)-4.0f};
constexpr h2 kMinus1152 = {(_Float16)-1152.0f, (_Float16)-1152.0f};

constexpr int kNi = 16;                      // receivers per workgroup
// Waves per workgroup: 16 (four branches per wave, 128 registers per lane)
// for the single-type kernel; 8 (eight branches per wave, 256 registers) for
// the batched kernel, which holds all three output types in one body.
constexpr int kWavesMain = 16, kWavesBatched = 8;
// LDS rows padded so that the FIR-phase stores (16 lanes: 16 receivers)
// and the FFT-phase loads (16 lanes: 8 spectra x 2 receivers) hit 32
// distinct banks: k1 rows start 8 banks apart, spectrum rows 4 banks apart
constexpr int kKStride = 16 * 16 + 4;        // float2 per k1 row
constexpr int kSStride = 4 * kKStride + 2;   // float2 per spectrum
constexpr int kSpectraPerPhase = 16;
constexpr int kChunk = 768;                  // spectra per workgroup, a multiple of 16
constexpr int kTT = 18;                      // tap pairs per branch and part (t = 0..17, cyclic)

// One workgroup: receivers [i0, i0+16) of one subband, spectra [s_begin, s_end).
template <int DT, int kWaves, bool kOne>
__device__ __forceinline__ void ppf_body(const int16_t* __restrict__ xs, const float* __restrict__ taps,
                                         void* __restrict__ zs, const Tw64& tw, int N, int S, int Sb,
                                         int i0, int s_begin, int s_end, float gain, float2* lds,
                                         unsigned* ltp) {
    constexpr int kThreads = 64 * kWaves;
    constexpr int kGrp = 16 / kWaves;            // branch groups p1 per wave
    constexpr int kFftJobs = 16 / kWaves;        // 16-point FFT jobs per lane and phase
    static_assert(kWaves == 8 || kWaves == 16, "8 or 16 waves");
    const int tid = threadIdx.x;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;

    // ---- FIR-phase roles: lane = 16 g + n; receiver n (clamped: receivers
    // beyond N read receiver N-1 and are never stored), window k-group g
    const int n = lane & 15, g = lane >> 4;
    const int rcv = min(i0 + n, N - 1);
    const unsigned row_bytes = (unsigned)N * 4u;                     // one time row of one branch
    const unsigned time_bytes = (unsigned)kP * row_bytes;            // one time step, all branches
    const int t_last = S + kT - 2;                                   // last input time row
    const char* xb = reinterpret_cast<const char*>(xs);

    // scale 2^E for the taps: the largest |h| lands in [2^14, 2^15), inside
    // the fp16 range with room for the parts (one value per workgroup: each
    // wave's maximum goes through the exchange buffer, unused until the
    // first phase)
    float hmax = 0.0f;
    for (int e = tid; e < kT * kP; e += kThreads) hmax = fmaxf(hmax, fabsf(taps[e]));
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) hmax = fmaxf(hmax, __shfl_xor(hmax, d));
    float* wmax = reinterpret_cast<float*>(lds);
    if (lane == 0) wmax[wv] = hmax;
    lds_barrier();
#pragma unroll
    for (int w = 0; w < kWaves; ++w) hmax = fmaxf(hmax, wmax[w]);
    int ex = 0;
    (void)frexpf(hmax, &ex);
    const int E = hmax > 0.0f ? min(max(15 - ex, -100), 100) : 0;
    const float up = ldexpf(1.0f, E), down = ldexpf(1.0f, 8 - E);     // 2^8: the samples enter as x / 256
    // The unscaling 2^(8-E) rides on the twiddles; for int8 output it goes
    // into the gain instead (exact: a power of two), and the FFT runs on the
    // scaled values.
    const float unscale = DT == AFC_I8 ? 1.0f : down;
    const float gain_u = DT == AFC_I8 ? gain * down : gain;
    // Band row m = n of H for this lane's k-group g, as two fp16 parts of
    // h 2^E.  Slot e <-> time offset 16 (e / 4) + 4 g + e % 4, tap t =
    // offset - n; for each i = e % 4 exactly one of the slots i and 4 + i is
    // inside the band (slot i when 4 g + i >= n), and its tap is t = (4 g - n
    // + i) mod 16.  So the lane reads the 4 taps (d + i) mod 16, d = (4 g -
    // n) mod 16, as two dwords of tables of tap pairs (part q of h[t] and of
    // h[(t+1) mod 16], t = 0..17) and places them with a mask.
    for (int e = tid; e < kP * kTT; e += kThreads) {
        const int p = e / kTT, t = e % kTT;
        const float ha = taps[(t & 15) * kP + p] * up, hb = taps[((t + 1) & 15) * kP + p] * up;
        const _Float16 a1 = (_Float16)ha, b1 = (_Float16)hb;
        const _Float16 a2 = (_Float16)(ha - (float)a1), b2 = (_Float16)(hb - (float)b1);
        ltp[e] = __builtin_bit_cast(unsigned, h2{a1, b1});
        ltp[kP * kTT + e] = __builtin_bit_cast(unsigned, h2{a2, b2});
    }
    lds_barrier();
    const int tq0 = (4 * g - n) & 15;                             // this lane's first tap pair
    unsigned band[2];                                               // halves of slots 0-3 inside the band
#pragma unroll
    for (int q = 0; q < 2; ++q)
        band[q] = (4 * g + 2 * q >= n ? 0x0000FFFFu : 0u) | (4 * g + 2 * q + 1 >= n ? 0xFFFF0000u : 0u);
    // (with the window's halves swapped between slots 0-3 and 4-7 when odd)
    auto band_row = [&](uint2 u, bool odd) -> v8h {
        const uint2 in = make_uint2(u.x & band[0], u.y & band[1]), out = make_uint2(u.x & ~band[0], u.y & ~band[1]);
        return odd ? __builtin_bit_cast(v8h, make_uint4(out.x, out.y, in.x, in.y))
                   : __builtin_bit_cast(v8h, make_uint4(in.x, in.y, out.x, out.y));
    };

    // int16 (re, im) pairs of receiver rcv, branch p, at the 4 times
    // t0 + 4 g + i of one half-window (rows beyond the input repeat the last
    // row: they only feed spectra >= S, which are never stored as data)
    const unsigned toff = (unsigned)(4 * g) * time_bytes + (unsigned)rcv * 4u;
    // One raw buffer per half-window with its scalar base at the first row:
    // the per-lane offset (time 4 g, receiver) and the scalar one (branch and
    // time i) stay below 16 rows of 64 branches, far below 2^31 bytes.
    auto load_half = [&](int (&r)[kGrp][4][4], int t0) {
        const int tb = min(t0, t_last);
#if defined(__HIP_DEVICE_COMPILE__)
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            (void*)(xb + (int64_t)tb * time_bytes), (short)0, 0x7FFFFFFF, 0x00020000);
        if (t0 + 15 <= t_last) {                                     // uniform: no row beyond the input
#pragma unroll
            for (int gr = 0; gr < kGrp; ++gr)
#pragma unroll
                for (int j = 0; j < 4; ++j)
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        r[gr][j][i] = (int)__builtin_amdgcn_raw_buffer_load_b32(
                            rs, toff, (unsigned)(wv + kWaves * gr + 16 * j) * row_bytes + (unsigned)i * time_bytes, 0);
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const unsigned vo = (unsigned)(min(t0 + 4 * g + i, t_last) - tb) * time_bytes + (unsigned)rcv * 4u;
#pragma unroll
                for (int gr = 0; gr < kGrp; ++gr)
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        r[gr][j][i] = (int)__builtin_amdgcn_raw_buffer_load_b32(
                            rs, vo, (unsigned)(wv + kWaves * gr + 16 * j) * row_bytes, 0);
            }
        }
#endif
    };

    // ---- FFT-phase roles (spectra 0-7 and 8-15: two jobs per lane with 8
    // waves, one with 16)
    const int k1 = wv & 3, rh = (wv >> 2) & 1;
    const int sl = lane & 7, ii = lane >> 3;
    const int ilf = rh * 8 + ii;
    const int rf = i0 + ilf;

    // Exact fp16 parts of the int16 (re, im) words wa, wb of two times
    // (x = 256 hb + lo): o = {re lo / 256, im lo / 256, re hb, im hb}, each
    // packed (time a, time b).  A byte pair gathered by v_perm is placed in
    // the mantissa of 1024 (fp16 bits 0x6400 | byte), then one packed fp16
    // operation, exact: lo: (1024 + lo) / 256 - 4; hb: flipping the sign bit
    // of the byte gives 1152 + hb.  The products then sum to x / 256 (the 256
    // goes into the unscaling).
    auto convert2 = [](unsigned wa, unsigned wb, unsigned (&o)[4]) __attribute__((always_inline)) {
        const h2 vrl = __builtin_bit_cast(h2, __builtin_amdgcn_perm(wb, wa, 0x0C040C00u) | 0x64006400u);
        const h2 vil = __builtin_bit_cast(h2, __builtin_amdgcn_perm(wb, wa, 0x0C060C02u) | 0x64006400u);
        const h2 vrh = __builtin_bit_cast(h2, __builtin_amdgcn_perm(wb, wa, 0x0C050C01u) ^ 0x64806480u);
        const h2 vih = __builtin_bit_cast(h2, __builtin_amdgcn_perm(wb, wa, 0x0C070C03u) ^ 0x64806480u);
        o[0] = __builtin_bit_cast(unsigned, vrl * kInv256 + kMinus4);
        o[1] = __builtin_bit_cast(unsigned, vil * kInv256 + kMinus4);
        o[2] = __builtin_bit_cast(unsigned, vrh + kMinus1152);
        o[3] = __builtin_bit_cast(unsigned, vih + kMinus1152);
    };
    // Operand tuples of branch (gr, j): op[part] (re lo, im lo, re hb, im
    // hb) holds slots 0-1, 2-3, 4-5, 6-7 in .x .. .w.  One half-window of
    // samples w goes into .xy (second = false) or .zw (second = true).
    auto convert_half = [&](const int (&w)[4], v4u (&op)[4], bool second) __attribute__((always_inline)) {
        unsigned o0[4], o1[4];
        convert2((unsigned)w[0], (unsigned)w[1], o0);
        convert2((unsigned)w[2], (unsigned)w[3], o1);
#pragma unroll
        for (int part = 0; part < 4; ++part) {
            if (second) {
                op[part].z = o0[part];
                op[part].w = o1[part];
            } else {
                op[part].x = o0[part];
                op[part].y = o1[part];
            }
        }
    };

    // One phase of 16 spectra starting at sg.  Each sample is converted once
    // and stays in its operand tuple for two phases; the window's halves
    // alternate between the tuple halves: in an even phase slots 0-3 hold
    // the first half (times sg ..) and the second half (sg + 16 ..) is
    // converted from `raw` into slots 4-7; in an odd phase slots 4-7 hold the
    // first half and the second goes into slots 0-3, and the band rows swap
    // their halves to match.  `raw` is then refilled with the next phase's
    // second half (sg + 32 ..).
    auto phase = [&](int sg, int (&raw)[kGrp][4][4], v4u (&ops)[kGrp][4][4],
                     auto odd_tag) __attribute__((always_inline)) {
        constexpr bool kOdd = decltype(odd_tag)::value;
        // the table index and masks pass through an empty asm each phase, so
        // the band rows are read and formed per use instead of being hoisted
        // out of the loop into registers (the index, not the pointer: a
        // pointer out of an asm loses its LDS address space, and the reads
        // would become flat loads that wait for every outstanding global
        // access)
        int tqi = tq0;
        __asm__ volatile("" : "+v"(tqi), "+v"(band[0]), "+v"(band[1]));
        const unsigned* tq = ltp + tqi;
#pragma unroll
        for (int gr = 0; gr < kGrp; ++gr) {
            const int p1 = wv + kWaves * gr;
            v4f ur[4], ui[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                convert_half(raw[gr][j], ops[gr][j], !kOdd);
                const v8h rl = __builtin_bit_cast(v8h, ops[gr][j][0]);
                const v8h il = __builtin_bit_cast(v8h, ops[gr][j][1]);
                const v8h rh = __builtin_bit_cast(v8h, ops[gr][j][2]);
                const v8h ih = __builtin_bit_cast(v8h, ops[gr][j][3]);
                const int pt = (p1 + 16 * j) * kTT;
                const v8h a1 = band_row(make_uint2(tq[pt], tq[pt + 2]), kOdd);
                const v8h a2 = band_row(make_uint2(tq[kP * kTT + pt], tq[kP * kTT + pt + 2]), kOdd);
                v4f ar = {0.0f, 0.0f, 0.0f, 0.0f}, ai = {0.0f, 0.0f, 0.0f, 0.0f};
                ar = __builtin_amdgcn_mfma_f32_16x16x32_f16(a2, rl, ar, 0, 0, 0);
                ai = __builtin_amdgcn_mfma_f32_16x16x32_f16(a2, il, ai, 0, 0, 0);
                ar = __builtin_amdgcn_mfma_f32_16x16x32_f16(a2, rh, ar, 0, 0, 0);
                ai = __builtin_amdgcn_mfma_f32_16x16x32_f16(a2, ih, ai, 0, 0, 0);
                ar = __builtin_amdgcn_mfma_f32_16x16x32_f16(a1, rl, ar, 0, 0, 0);
                ai = __builtin_amdgcn_mfma_f32_16x16x32_f16(a1, il, ai, 0, 0, 0);
                ar = __builtin_amdgcn_mfma_f32_16x16x32_f16(a1, rh, ar, 0, 0, 0);
                ai = __builtin_amdgcn_mfma_f32_16x16x32_f16(a1, ih, ai, 0, 0, 0);
                ur[j] = ar;
                ui[j] = ai;
                // one branch at a time: keeps its operands' live ranges short
                __builtin_amdgcn_sched_barrier(0);
            }
            if (gr == kGrp - 1) load_half(raw, sg + 32);
            // radix-4 over j (lane-local), then the twiddle exp(-2 pi i p1 k1 / 64)
            // times the unscaling (exact)
            const float2 w1 = tw.w[p1 & 63] * unscale, w2 = tw.w[(2 * p1) & 63] * unscale;
            const float2 w3 = tw.w[(3 * p1) & 63] * unscale;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float2 u0 = make_float2(ur[0][r], ui[0][r]), u1 = make_float2(ur[1][r], ui[1][r]);
                const float2 u2 = make_float2(ur[2][r], ui[2][r]), u3 = make_float2(ur[3][r], ui[3][r]);
                const float2 s02 = u0 + u2, d02 = u0 - u2, s13 = u1 + u3, d13 = u1 - u3;
                const float2 a0 = s02 + s13, a2 = s02 - s13;
                const float2 a1 = make_float2(d02.x + d13.y, d02.y - d13.x);      // d02 - i d13
                const float2 a3 = make_float2(d02.x - d13.y, d02.y + d13.x);      // d02 + i d13
                float2* dst = lds + (4 * g + r) * kSStride + p1 * 16 + n;
                dst[0] = DT == AFC_I8 ? a0 : a0 * down;
                dst[kKStride] = cmul(a1, w1);
                dst[2 * kKStride] = cmul(a2, w2);
                dst[3 * kKStride] = cmul(a3, w3);
            }
        }
        lds_barrier();
#pragma unroll
        for (int jb = 0; jb < kFftJobs; ++jb) {
            const int bh = kFftJobs == 2 ? jb : wv >> 3;
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
                const float gq = live ? gain_u : 0.0f;
#pragma unroll
                for (int ga = 0; ga < 4; ++ga)
#pragma unroll
                    for (int de = 0; de < 4; ++de) {
                        const int k = k1 + 4 * (ga + 4 * de);
                        float2 y = a[4 * ga + de];
                        if constexpr (DT != AFC_I8)
                            if (!live) y = make_float2(0.0f, 0.0f);
                        store_sample<DT, kOne>(zs, (int64_t)k * ch_stride, lane_zoff, y, gq);
                    }
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        lds_barrier();
    };

    // s_begin is a multiple of 16; the loop body holds an even and an odd
    // phase
    int raw[kGrp][4][4];
    v4u ops[kGrp][4][4];
    load_half(raw, s_begin);
#pragma unroll
    for (int gr = 0; gr < kGrp; ++gr)
#pragma unroll
        for (int j = 0; j < 4; ++j) convert_half(raw[gr][j], ops[gr][j], false);
    load_half(raw, s_begin + 16);
    for (int sg = s_begin; sg < s_end; sg += 2 * kSpectraPerPhase) {
        phase(sg, raw, ops, std::false_type{});
        if (sg + kSpectraPerPhase >= s_end) break;
        phase(sg + kSpectraPerPhase, raw, ops, std::true_type{});
    }
}

template <int DT, bool kOne>
__global__ __launch_bounds__(64 * kWavesMain) void ppf_kernel(const int16_t* __restrict__ x, const float* __restrict__ taps,
                                                       void* __restrict__ z, Tw64 tw, int64_t x_sb_stride,
                                                       int64_t z_sb_bytes, int N, int S, int Sb, int n_groups,
                                                       int n_chunks, int total, int per_xcd, float gain) {
    __shared__ float2 lds[kSpectraPerPhase * kSStride];
    __shared__ __attribute__((aligned(16))) unsigned ltp[2 * kP * kTT];
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
    ppf_body<DT, kWavesMain, kOne>(x + sb * x_sb_stride, taps, reinterpret_cast<char*>(z) + sb * z_sb_bytes, tw, N, S, Sb,
                 grp * kNi, s_begin, s_end, gain, lds, ltp);
}

// Batched form: one launch over per-subband jobs with their own S, type and gain.
template <bool kOne>
__global__ __launch_bounds__(64 * kWavesBatched) void ppf_batched_kernel(const int16_t* __restrict__ x,
                                                              const float* __restrict__ taps, void* __restrict__ z,
                                                              Tw64 tw, const PpfItem* __restrict__ items,
                                                              int N, int n_groups, int n_chunks, int total,
                                                              int per_xcd) {
    __shared__ float2 lds[kSpectraPerPhase * kSStride];
    __shared__ __attribute__((aligned(16))) unsigned ltp[2 * kP * kTT];
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
        ppf_body<AFC_F32, kWavesBatched, kOne>(xs, taps, zs, tw, N, item.S, item.Sb, grp * kNi, s_begin, s_end, item.gain, lds, ltp);
    else if (item.dt == AFC_F16)
        ppf_body<AFC_F16, kWavesBatched, kOne>(xs, taps, zs, tw, N, item.S, item.Sb, grp * kNi, s_begin, s_end, item.gain, lds, ltp);
    else
        ppf_body<AFC_I8, kWavesBatched, kOne>(xs, taps, zs, tw, N, item.S, item.Sb, grp * kNi, s_begin, s_end, item.gain, lds, ltp);
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
    // one store descriptor per subband when its output is below 2^31 bytes
    const bool one = (int64_t)kP * a.Sb * a.N * kSBlk * sample_bytes(a.dt) <= 0x7FFFFFFFLL;
#define AFC_PPF_LAUNCH(DT)                                                                                       \
    if (one)                                                                                                     \
        hipLaunchKernelGGL((ppf_kernel<DT, true>), grid, dim3(64 * kWavesMain), 0, stream, a.x, a.taps, a.z, tw,  \
                           a.x_sb_stride, z_sb_bytes, a.N, a.S, a.Sb, n_groups, n_chunks, total, per_xcd, a.gain); \
    else                                                                                                         \
        hipLaunchKernelGGL((ppf_kernel<DT, false>), grid, dim3(64 * kWavesMain), 0, stream, a.x, a.taps, a.z, tw, \
                           a.x_sb_stride, z_sb_bytes, a.N, a.S, a.Sb, n_groups, n_chunks, total, per_xcd, a.gain);
    switch (a.dt) {
        case AFC_F32: AFC_PPF_LAUNCH(AFC_F32) break;
        case AFC_F16: AFC_PPF_LAUNCH(AFC_F16) break;
        default: AFC_PPF_LAUNCH(AFC_I8) break;
    }
#undef AFC_PPF_LAUNCH
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
    // one store descriptor per subband when the largest possible subband
    // output (fp32 samples at the longest integration) is below 2^31 bytes
    const bool one = (int64_t)kP * ceil_div(max_S, kSBlk) * N * kSBlk * 8 <= 0x7FFFFFFFLL;
    if (one)
        hipLaunchKernelGGL((ppf_batched_kernel<true>), grid, dim3(64 * kWavesBatched), 0, stream, x, taps, z_ws, tw,
                           items_dev, N, n_groups, n_chunks, total, per_xcd);
    else
        hipLaunchKernelGGL((ppf_batched_kernel<false>), grid, dim3(64 * kWavesBatched), 0, stream, x, taps, z_ws, tw,
                           items_dev, N, n_groups, n_chunks, total, per_xcd);
    return hipGetLastError();
}

}  // namespace afc
