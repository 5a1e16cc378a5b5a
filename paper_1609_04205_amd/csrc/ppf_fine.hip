// Fine channeliser: a 256-channel polyphase filter bank, per-receiver delay
// and per-channel bandpass compensation, and coherent integration of 4
// adjacent channels into one of 64 (Sec. "Polyphase Filterbank": a bank of
// 256 16-tap FIR filters and a 256-point complex FFT; Sec. "Delay, Bandpass
// Compensation and Transpose Kernel": fixed cable delays applied as phase
// rotations, a fixed real weight per channel, channels integrated to the
// output resolution, then the exchange of the parallel axis from channels to
// receivers).
//
//   u[s][p] = sum_{t<16} h[t*256 + p] x[(s+t)*256 + p]
//   y[s][k] = sum_{p<256} u[s][p] exp(-2 pi i k p / 256)
//   z[s][c] = sum_{j<4} C_i[4c + j] y[s][4c + j]                  (c < 64)
//   C_i[k] = w[k] exp(2 pi i (nu_b + f_k) tau_i),
//   f_k = (k < 128 ? k : k - 256) * (subband width / 256)
//
// 256 = 4 x 64 with p = p1 + 64 j, k = k1 + 4 k', k' = k2 + 16 k3.
// One workgroup = 8 receivers x a run of spectra of one subband, 512 threads
// (8 waves, two per SIMD, so that a lane may hold 256 registers): a row of
// the time-major input gives the workgroup 32 contiguous bytes (with 4
// receivers per workgroup the rate of L1-to-L2 line requests bounded the
// kernel; 8 halve it, and the vector instructions bound it now).
//  * FIR phase: lane (p1, receiver half, j) owns branch p = p1 + 64 j of 4
//    receivers: its taps (16 registers), the 16-deep windows of 4 receivers x
//    2 components (128 registers), one 16-byte load per spectrum.  The radix-4
//    stage over j runs across the lane quad in two DPP exchanges (sums and
//    differences, then the +-1, +-i rotations), leaving A[k1] in quad lane j
//    with k1 the bit reverse of j, times exp(-2 pi i p1 k1 / 256).
//  * FFT phase 1: a lane takes two (spectrum, k1, receiver, qd) jobs: the
//    16-point DFT over r (p1 = qd + 4 r) and the twiddle exp(-2 pi i qd k2 / 64).
//  * FFT phase 2 (after an LDS exchange): lane (receiver, spectrum) of wave
//    k2 (and k2 + 8) does the radix-4 over qd for each k1 (fine channels
//    k = k1 + 4 k2 + 64 k3), weighs them with C and sums over k1: coarse
//    channel c = k2 + 16 k3, stored as 8 receivers x 8 spectra, contiguous in
//    the block layout.
// A phase covers 8 spectra, one block of the output.
#include <algorithm>
#include <cmath>

#include "afc_internal.h"
#include "ppf_common.h"

namespace afc {
namespace {
using namespace ppfk;

constexpr int kPF = kPFine;                  // fine channels
constexpr int kRF = 4;                       // fine channels per output channel
constexpr int kNiF = 8;                      // receivers per workgroup
constexpr int kThreadsF = 512;               // 8 waves
constexpr int kQF = 8;                       // spectra per phase
constexpr int kK1S = 64 * kNiF + 2;          // float2 per k1 row of the phase buffer (+2: the 4 k1 rows start 4 banks apart)
constexpr int kQS = 4 * kK1S;                // float2 per spectrum of the phase buffer
constexpr int kXR = 16 * kNiF;               // float2 per (spectrum, k2) row of the exchange buffer
constexpr int kChunkQ = 16;                  // a workgroup's run of spectra is a multiple of this
constexpr int kDepthF = 2;                   // spectra of loads in flight per lane (divides 8)
static_assert(kQF * 16 * kXR <= kQF * kQS, "the exchange fits the phase buffer");
static_assert(kChunkQ % kQF == 0 && kQF % kDepthF == 0, "phase and pipeline shapes");

struct FineArgs {
    const int16_t* x;
    const float* taps;
    void* z;
    const float2* W;                         // [256] exp(-2 pi i m / 256)
    const float2* E;                         // [N][256] w[k] exp(2 pi i f_k tau_i)
    const float2* A;                         // [B][N] exp(2 pi i nu_b tau_i)
    int64_t x_sb_stride;                     // int16 elements between subbands
    int64_t z_sb_bytes;
    int N, S, Sb, n_groups, chunk, n_chunks, total, per_xcd;   // chunk: spectra per workgroup
    float gain;
};

template <int DT, bool kVec4, bool kOne>
__global__ __launch_bounds__(kThreadsF) void ppf_fine_kernel(FineArgs a, Tw64 tw64) {
    __shared__ __attribute__((aligned(16))) float2 lds[kQF * kQS];
    // rows padded by one element: the receivers' rows start in different banks
    __shared__ float2 lcomp[kNiF * (kPF + 1)];
    __shared__ float2 ltw[4 * 17];               // [qd][k2] exp(-2 pi i qd k2 / 64)
    // XCD-aware order: neighbouring receiver groups (which share 128-byte
    // lines of the input rows) run on one XCD at one time
    const int w = (blockIdx.x & 7) * a.per_xcd + (blockIdx.x >> 3);
    if (w >= a.total) return;
    const int grp = w % a.n_groups;
    const int chunk = (w / a.n_groups) % a.n_chunks;
    const int sb = w / (a.n_groups * a.n_chunks);
    const int N = a.N, S = a.S;
    const int i0 = grp * kNiF;
    const int s_begin = chunk * a.chunk;
    const int s_end = min(S, s_begin + a.chunk);
    const int16_t* xs = a.x + sb * a.x_sb_stride;
    void* zs = reinterpret_cast<char*>(a.z) + sb * a.z_sb_bytes;

    const int tid = threadIdx.x;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;

    // compensation factors C = E A of this subband, [receiver][fine channel]
    // (receivers beyond N repeat receiver N-1 and are never stored)
    for (int e = tid; e < kNiF * kPF; e += kThreadsF) {
        const int il = e / kPF, k = e % kPF;
        const int i = min(i0 + il, N - 1);
        lcomp[il * (kPF + 1) + k] = cmul(a.E[(int64_t)i * kPF + k], a.A[(int64_t)sb * N + i]);
    }
    if (tid < 64) ltw[(tid >> 4) * 17 + (tid & 15)] = tw64.w[((tid >> 4) * (tid & 15)) & 63];

    // ---- FIR roles: lane = x * 8 + rh * 4 + j
    const int j = lane & 3, rh = (lane >> 2) & 1, x = lane >> 3;
    const int p1 = 8 * wv + x;
    const int p = p1 + 64 * j;
    const int k1o = ((j & 1) << 1) | (j >> 1);                 // this lane ends with A[k1o]
    const float2 tw_o = a.W[p1 * k1o];
    // radix-4 over j: step 1 (partner j ^ 2) own * s1 + partner gives
    // u0+u2, u1+u3, u0-u2, u1-u3 in lanes 0..3; step 2 (partner j ^ 1)
    // alpha own + beta partner gives A0, A2, A1, A3
    const float s1 = (j >> 1) ? -1.0f : 1.0f;
    const float2 al = j == 0 ? make_float2(1.0f, 0.0f) : j == 1 ? make_float2(-1.0f, 0.0f)
                    : j == 2 ? make_float2(1.0f, 0.0f) : make_float2(0.0f, 1.0f);
    const float2 be = j == 2 ? make_float2(0.0f, -1.0f) : make_float2(1.0f, 0.0f);
    // with the twiddle folded in (al and be are 1, -1, i or -i: exact)
    const float2 alw = cmul(al, tw_o), bew = cmul(be, tw_o);
    float h[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) h[t] = a.taps[t * kPF + p];
    // first receiver of this lane's four; loads clamped into the row (the
    // clamped receivers are never stored)
    const int rb = i0 + 4 * rh;
    const int64_t row_stride = 2LL * N;                        // int16 per input row
    const int64_t spec_stride = (int64_t)kPF * row_stride;
    const int16_t* lane_base = xs + (int64_t)p * row_stride;
    const int rq0 = kVec4 ? min(rb, N - 4) : min(rb, N - 2);
    const int rq1 = min(rb + 2, N - 2);
    auto ld = [&](int m) -> int4 {
        const int16_t* rowp = lane_base + (int64_t)min(m, S + kT - 2) * spec_stride;
        if constexpr (kVec4) {
            return *reinterpret_cast<const int4*>(rowp + 2 * rq0);
        } else {
            const int2 u0 = *reinterpret_cast<const int2*>(rowp + 2 * rq0);
            const int2 u1 = *reinterpret_cast<const int2*>(rowp + 2 * rq1);
            return make_int4(u0.x, u0.y, u1.x, u1.y);
        }
    };

    float win[4][2][16];
    auto put = [&](int slot, int4 d) {
        const int dd[4] = {d.x, d.y, d.z, d.w};
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            win[r][0][slot] = (float)(int)(short)(dd[r] & 0xFFFF);
            win[r][1][slot] = (float)(dd[r] >> 16);
        }
    };
#pragma unroll
    for (int m = 0; m < 15; ++m) put(m, ld(s_begin + m));
#pragma unroll
    for (int r = 0; r < 4; ++r) win[r][0][15] = win[r][1][15] = 0.0f;

    int4 pf[kDepthF];
#pragma unroll
    for (int d = 0; d < kDepthF; ++d) pf[d] = ld(s_begin + d + 15);

    // ---- FFT phase 1 jobs: T = tid + 512 t, receiver = T % 8, qd = (T / 8) % 4,
    // k1 = (T / 32) % 4, spectrum = T / 128
    const int rc1 = tid & 7, qd1 = (tid >> 3) & 3, k11 = (tid >> 5) & 3, q1 = tid >> 7;   // t = 0; t = 1 adds 4 to q
    // ---- FFT phase 2 roles: lane = spectrum * 8 + receiver, k2 = wave (+ 8)
    const int rc2 = lane & 7, q2 = lane >> 3;
    const int rf = i0 + rc2;
    const float2* comp2 = lcomp + rc2 * (kPF + 1);

    for (int sg = s_begin; sg < s_end; sg += 16) {
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            const int sp = sg + 8 * half;                      // first spectrum of this phase
#pragma unroll
            for (int ql = 0; ql < kQF; ++ql) {
                const int q = 8 * half + ql;                   // window slot of spectrum sg + q
                put((q + 15) & 15, pf[ql % kDepthF]);
                pf[ql % kDepthF] = ld(sp + ql + kDepthF + 15);
                float u[4][2];
#pragma unroll
                for (int r = 0; r < 4; ++r)
#pragma unroll
                    for (int c = 0; c < 2; ++c) {
                        float acc = 0.0f;
#pragma unroll
                        for (int t = 0; t < 16; ++t) acc = fmaf(h[t], win[r][c][(q + t) & 15], acc);
                        u[r][c] = acc;
                    }
                float2 o[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    // step 1: with the lane at j ^ 2
                    const float e0 = fmaf(s1, u[r][0], quad_xor<2>(u[r][0]));
                    const float e1 = fmaf(s1, u[r][1], quad_xor<2>(u[r][1]));
                    // step 2: with the lane at j ^ 1
                    const float f0 = quad_xor<1>(e0), f1 = quad_xor<1>(e1);
                    // (al e + be f) exp(-2 pi i p1 k1o / 256)
                    o[r].x = alw.x * e0 - alw.y * e1 + bew.x * f0 - bew.y * f1;
                    o[r].y = alw.x * e1 + alw.y * e0 + bew.x * f1 + bew.y * f0;
                }
                float4* dst = reinterpret_cast<float4*>(lds + ql * kQS + k1o * kK1S + p1 * kNiF + 4 * rh);
                dst[0] = make_float4(o[0].x, o[0].y, o[1].x, o[1].y);
                dst[1] = make_float4(o[2].x, o[2].y, o[3].x, o[3].y);
                __builtin_amdgcn_sched_barrier(0);
            }
            lds_barrier();
            // 16-point DFT over r (p1 = qd + 4 r), spectra q1 then q1 + 4: the
            // exchange rows of spectra 0..3 end before the phase-buffer rows
            // of spectra 4..7 begin, so the second job's reads may overlap the
            // first job's writes
            static_assert(4 * 16 * kXR <= 4 * kQS, "exchange rows of spectra 0..3 precede phase rows 4..7");
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const int q = q1 + 4 * t;
                float2 v[16];
                const float2* src = lds + q * kQS + k11 * kK1S + qd1 * kNiF + rc1;
#pragma unroll
                for (int r = 0; r < 16; ++r) v[r] = src[r * 4 * kNiF];
                lds_barrier();
                dft16(v);
                // exchange [spectrum][k2][(k1 * 4 + qd) ^ (spectrum & 1)][receiver]
                float2* dst = lds + (q * 16) * kXR + (((k11 * 4 + qd1) ^ (q & 1)) * kNiF) + rc1;
#pragma unroll
                for (int ga = 0; ga < 4; ++ga)
#pragma unroll
                    for (int de = 0; de < 4; ++de) {
                        const int kk = ga + 4 * de;                    // k2
                        float2 y = v[4 * ga + de];
                        if (kk != 0) y = cmul(y, ltw[qd1 * 17 + kk]);
                        dst[kk * kXR] = y;
                    }
            }
            lds_barrier();
            {
                const int blk = sp >> 3;
                const bool live = sp + q2 < S;
                const float g = live ? a.gain : 0.0f;
                const int64_t ch_stride = (int64_t)a.Sb * N * kSBlk;
                const unsigned lane_zoff = (unsigned)((blk * N + rf) * kSBlk + q2);
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    const int k2 = wv + 8 * t;
                    const float2* src = lds + (q2 * 16 + k2) * kXR + rc2;
                    const int sw = q2 & 1;
                    float2 v[4][4];
#pragma unroll
                    for (int m = 0; m < 16; ++m) v[m >> 2][m & 3] = src[(m ^ sw) * kNiF];
                    float2 c4[4];
#pragma unroll
                    for (int k3 = 0; k3 < 4; ++k3) c4[k3] = make_float2(0.0f, 0.0f);
#pragma unroll
                    for (int k1 = 0; k1 < kRF; ++k1) {
                        dft4(v[k1][0], v[k1][1], v[k1][2], v[k1][3]);
#pragma unroll
                        for (int k3 = 0; k3 < 4; ++k3)
                            c4[k3] = c4[k3] + cmul(v[k1][k3], comp2[k1 + 4 * k2 + 64 * k3]);
                    }
                    if (rf < N && blk < a.Sb) {
#pragma unroll
                        for (int k3 = 0; k3 < 4; ++k3) {
                            float2 y = c4[k3];
                            if constexpr (DT != AFC_I8)
                                if (!live) y = make_float2(0.0f, 0.0f);
                            store_sample<DT, kOne>(zs, (int64_t)(k2 + 16 * k3) * ch_stride, lane_zoff, y, g);
                        }
                    }
                }
            }
            lds_barrier();
        }
    }
}

// Tables in double precision, rounded to float: W[m] = exp(-2 pi i m / 256),
// E[i][k] = w[k] exp(2 pi i f_k tau_i), A[b][i] = exp(2 pi i nu_b tau_i).
struct TableArgs {
    const double* tau;
    const float* w;
    float2* W;
    float2* E;
    float2* A;
    double df;
    int N, B;
    double nu[AFC_MAX_SUBBANDS];
};

__global__ void fine_table_kernel(TableArgs t) {
    const int64_t n_e = (int64_t)t.N * kPF, n_a = (int64_t)t.B * t.N;
    const double pi = 3.14159265358979323846;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < kPF + n_e + n_a;
         e += (int64_t)gridDim.x * blockDim.x) {
        if (e < kPF) {
            const double ang = -2.0 * pi * (double)e / kPF;
            t.W[e] = make_float2((float)cos(ang), (float)sin(ang));
        } else if (e < kPF + n_e) {
            const int64_t r = e - kPF;
            const int i = (int)(r / kPF), k = (int)(r % kPF);
            const double fk = (double)(k < kPF / 2 ? k : k - kPF) * t.df;
            const double turns = fk * t.tau[i];
            const double ang = 2.0 * pi * (turns - floor(turns));
            t.E[r] = make_float2((float)((double)t.w[k] * cos(ang)), (float)((double)t.w[k] * sin(ang)));
        } else {
            const int64_t r = e - kPF - n_e;
            const int b = (int)(r / t.N), i = (int)(r % t.N);
            // nu tau is many turns: reduce to a fraction of a turn first
            const double turns = t.nu[b] * t.tau[i];
            const double ang = 2.0 * pi * (turns - floor(turns));
            t.A[r] = make_float2((float)cos(ang), (float)sin(ang));
        }
    }
}

// Spectra per workgroup: each run re-reads and re-filters the 15 spectra
// before it, and the launch runs one workgroup per CU at a time, so the
// time goes as (waves of workgroups over the CUs) x (run + 15 spectra).
// The run is the multiple of 16 that minimises that (the longer on ties):
// 768 for 16 subbands x 1152 antennas x 762 spectra (3% faster than runs of
// 192), shorter runs when few subbands or receivers would leave CUs idle.
int fine_chunk(int B, int n_groups, int S) {
    int dev = 0, n_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n_cu <= 0)
        n_cu = 256;
    const int s16 = (int)ceil_div(S, kChunkQ) * kChunkQ;
    int best = kChunkQ;
    double best_cost = 1e300;
    for (int c = kChunkQ; c <= std::min(s16, 2048); c += kChunkQ) {
        const double wgs = (double)B * n_groups * (double)ceil_div(S, c);
        const double cost = std::ceil(wgs / n_cu) * (double)(std::min(c, S) + kT - 1);
        if (cost <= best_cost) {
            best_cost = cost;
            best = c;
        }
    }
    return best;
}

}  // namespace

size_t fine_workspace_bytes(int N, int B) {
    return ((size_t)kPF + (size_t)N * kPF + (size_t)B * N) * sizeof(float2);
}

hipError_t launch_ppf_fine(const FineLaunch& l, hipStream_t stream) {
    static const Tw64 tw64 = make_twiddles();
    float2* W = reinterpret_cast<float2*>(l.workspace);
    float2* E = W + kPF;
    float2* A = E + (size_t)l.N * kPF;
    TableArgs t{};
    t.tau = l.tau;
    t.w = l.bandpass;
    t.W = W;
    t.E = E;
    t.A = A;
    t.df = l.subband_hz / kPF;
    t.N = l.N;
    t.B = l.B;
    for (int b = 0; b < l.B; ++b) t.nu[b] = l.nu_center[b];
    const int64_t n_tab = kPF + (int64_t)l.N * kPF + (int64_t)l.B * l.N;
    hipLaunchKernelGGL(fine_table_kernel, dim3((unsigned)std::min<int64_t>(ceil_div(n_tab, 256), 2048)),
                       dim3(256), 0, stream, t);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;

    FineArgs a{};
    a.x = l.x;
    a.taps = l.taps;
    a.z = l.z;
    a.W = W;
    a.E = E;
    a.A = A;
    a.x_sb_stride = l.x_sb_stride;
    a.z_sb_bytes = l.z_sb_stride * sample_bytes(l.dt);
    a.N = l.N;
    a.S = l.S;
    a.Sb = l.Sb;
    a.gain = l.gain;
    a.n_groups = (int)ceil_div(l.N, kNiF);
    a.chunk = fine_chunk(l.B, a.n_groups, l.S);
    a.n_chunks = (int)ceil_div(l.S, a.chunk);
    const int64_t total = (int64_t)l.B * a.n_groups * a.n_chunks;
    if (total > (1LL << 30)) return hipErrorInvalidValue;
    a.total = (int)total;
    a.per_xcd = (int)ceil_div(total, 8);
    const dim3 grid((unsigned)(a.per_xcd * 8));
    // 16-byte row loads need 16-byte aligned rows: N a multiple of 4
    const bool vec4 = l.N % 4 == 0;
    // one store descriptor per subband when its output is below 2^31 bytes
    const bool one = (int64_t)64 * l.Sb * l.N * kSBlk * sample_bytes(l.dt) <= 0x7FFFFFFFLL;
#define AFC_FINE_LAUNCH(DT)                                                                                  \
    if (vec4 && one)                                                                                         \
        hipLaunchKernelGGL((ppf_fine_kernel<DT, true, true>), grid, dim3(kThreadsF), 0, stream, a, tw64);     \
    else if (vec4)                                                                                           \
        hipLaunchKernelGGL((ppf_fine_kernel<DT, true, false>), grid, dim3(kThreadsF), 0, stream, a, tw64);    \
    else if (one)                                                                                            \
        hipLaunchKernelGGL((ppf_fine_kernel<DT, false, true>), grid, dim3(kThreadsF), 0, stream, a, tw64);    \
    else                                                                                                     \
        hipLaunchKernelGGL((ppf_fine_kernel<DT, false, false>), grid, dim3(kThreadsF), 0, stream, a, tw64);
    switch (l.dt) {
        case AFC_F32: AFC_FINE_LAUNCH(AFC_F32) break;
        case AFC_F16: AFC_FINE_LAUNCH(AFC_F16) break;
        default: AFC_FINE_LAUNCH(AFC_I8) break;
    }
#undef AFC_FINE_LAUNCH
    return hipGetLastError();
}

}  // namespace afc
