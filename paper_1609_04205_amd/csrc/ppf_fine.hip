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
//  * FIR phase: as in the 64-channel bank, a lane keeps the 16-deep windows
//    of two branches in registers; a lane quad holds the four branches
//    p1 + 64 j of one receiver and after two DPP exchanges each quad lane owns
//    one k1 of the radix-4 stage over j, times exp(-2 pi i p1 k1 / 256).
//    16 waves x 4 branch groups cover p1 < 64, 16 lanes per branch group
//    cover 4 receivers x 4 quad lanes.
//  * FFT phase 1: lane (receiver, k1, qd), wave = spectrum, does the 16-point
//    DFT over r (p1 = qd + 4 r) and the twiddle exp(-2 pi i qd k2 / 64).
//  * FFT phase 2 (after an LDS exchange): lane (receiver, spectrum, k2) does
//    the radix-4 over qd for each k1, which gives fine channels
//    k = k1 + 4 k2 + 64 k3, weighs them with C and sums over k1: coarse
//    channel c = k2 + 16 k3.
// Both LDS buffers are XOR-swizzled instead of padded so that they fit in
// 160 KB beside the taps and the compensation factors.
#include "afc_internal.h"
#include "ppf_common.h"

namespace afc {
namespace {
using namespace ppfk;

constexpr int kPF = kPFine;                  // fine channels
constexpr int kRF = 4;                       // fine channels per output channel
constexpr int kNiF = 4;                      // receivers per workgroup
constexpr int kThreadsF = 1024;              // 16 waves
constexpr int kKSF = 64 * kNiF;              // float2 per k1 row of the FIR-phase buffer
constexpr int kSSF = 4 * kKSF;               // float2 per spectrum
constexpr int kSppF = 16;                    // spectra per phase
constexpr int kChunkF = 192;                 // spectra per workgroup, a multiple of 16
constexpr int kDepthF = 4;                   // spectra of loads in flight per lane (divides 16)
constexpr int kXS = 64 * kSppF;              // float2 per k2 plane of the exchange buffer
static_assert(16 * kXS <= kSppF * kSSF, "the exchange of the FFT phase fits the LDS buffer");
static_assert(kChunkF % kSppF == 0 && kSppF % kDepthF == 0, "phase and pipeline shapes");

struct FineArgs {
    const int16_t* x;
    const float* taps;
    void* z;
    const float2* W;                         // [256] exp(-2 pi i m / 256)
    const float2* E;                         // [N][256] w[k] exp(2 pi i f_k tau_i)
    const float2* A;                         // [B][N] exp(2 pi i nu_b tau_i)
    int64_t x_sb_stride;                     // int16 elements between subbands
    int64_t z_sb_bytes;
    int N, S, Sb, n_groups, n_chunks, total, per_xcd;
    float gain;
};

template <int DT>
__global__ __launch_bounds__(kThreadsF) void ppf_fine_kernel(FineArgs a, Tw64 tw64) {
    __shared__ __attribute__((aligned(16))) float2 lds[kSppF * kSSF];
    __shared__ __attribute__((aligned(16))) float ltaps[kT * kPF];
    // rows padded by one element: the four receivers' rows start in
    // different banks
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
    const int s_begin = chunk * kChunkF;
    const int s_end = min(S, s_begin + kChunkF);
    const int16_t* xs = a.x + sb * a.x_sb_stride;
    void* zs = reinterpret_cast<char*>(a.z) + sb * a.z_sb_bytes;

    const int tid = threadIdx.x;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;

    // taps as [branch][t]; compensation factors C = E A of this subband as
    // [receiver][fine channel] (receivers beyond N repeat receiver N-1 and
    // are never stored)
    for (int e = tid; e < kT * kPF; e += kThreadsF) {
        const int t = e / kPF, p = e % kPF;
        ltaps[p * kT + t] = a.taps[e];
    }
    {
        const int il = tid / kPF, k = tid % kPF;
        const int i = min(i0 + il, N - 1);
        lcomp[il * (kPF + 1) + k] = cmul(a.E[(int64_t)i * kPF + k], a.A[(int64_t)sb * N + i]);
        if (tid < 64) ltw[(tid >> 4) * 17 + (tid & 15)] = tw64.w[((tid >> 4) * (tid & 15)) & 63];
    }

    // ---- FIR-phase roles: lane = il * 16 + ps * 4 + jh * 2 + comp
    const int comp = lane & 1, jh = (lane >> 1) & 1, ps = (lane >> 2) & 3, il = lane >> 4;
    const int p1 = 4 * wv + ps;
    const int rcv = min(i0 + il, N - 1);
    const int row_stride = N * 2;
    const int lane_off = (p1 + 128 * jh) * row_stride + rcv * 2 + comp;   // branch p1 + 64 (2 jh) at row 0
    const int64_t spec_stride = (int64_t)kPF * row_stride;
    const int k1o = comp + 2 * jh;
    const float2 tw_o = a.W[p1 * k1o];
    const float2 rtw_o = k1o == 0 ? tw_o : k1o == 1 ? make_float2(tw_o.y, -tw_o.x)
                       : k1o == 2 ? make_float2(-tw_o.x, -tw_o.y) : make_float2(-tw_o.y, tw_o.x);
    const float sgn = (k1o & 1) ? -1.0f : 1.0f;
    // [spectrum][k1][p1 * 4 + (receiver ^ k1)], bit 4 of the index flipped
    // for odd k1: the 16 lanes of (branch group, k1) of one receiver, and the
    // 32 of two receivers, write to distinct banks
    const int fir_w = k1o * kKSF + ((p1 * kNiF + (il ^ k1o)) ^ ((k1o & 1) << 4));

    lds_barrier();
    const float4* tp0 = reinterpret_cast<const float4*>(ltaps + (p1 + 128 * jh) * kT);
    const float4* tp1 = reinterpret_cast<const float4*>(ltaps + (p1 + 128 * jh + 64) * kT);

    // raw int16 sample of branch p1 + 64 (2 jh + jj) at spectrum-row m
    // (clamped: every load is in bounds and unconditional)
    auto ld = [&](int m, int jj) -> int {
        const int16_t* rowp = xs + (int64_t)min(m, S + kT - 2) * spec_stride;
        return rowp[jj * (64 * row_stride) + lane_off];
    };

    float win[2][16];
#pragma unroll
    for (int m = 0; m < 15; ++m)
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) win[jj][m] = (float)ld(s_begin + m, jj);
#pragma unroll
    for (int jj = 0; jj < 2; ++jj) win[jj][15] = 0.0f;

    // ---- FFT phase 1 roles: lane = k1 * 16 + qd * 4 + receiver, wave = spectrum
    const int il1 = lane & 3, qd1 = (lane >> 2) & 3, k1f = lane >> 4, q1 = wv;
    const int b1 = k1f & 1;
    const int il1s = il1 ^ k1f;
    const float2* src1e = lds + q1 * kSSF + k1f * kKSF + 4 * qd1 + il1s + 16 * b1;   // r even
    const float2* src1o = lds + q1 * kSSF + k1f * kKSF + 4 * qd1 + il1s - 16 * b1;   // r odd
    // exchange buffer [k2][spectrum][(k1 * 4 + qd) * 4 + receiver], the
    // (k1 * 4 + qd) index XOR spectrum % 8
    const int xw = q1 * 64 + (((k1f * 4 + qd1) * 4 + il1) ^ ((q1 & 7) << 2));
    const float2* tw1 = ltw + qd1 * 17;
    // ---- FFT phase 2 roles: lane = k2lo * 32 + (spectrum % 8) * 4 + receiver
    const int il2 = lane & 3, ql2 = (lane >> 2) & 7, k2lo = lane >> 5;
    const int q2 = (wv & 1) * 8 + ql2, k2 = (wv >> 1) * 2 + k2lo;
    const float2* src2 = lds + k2 * kXS + q2 * 64 + il2;
    const float2* comp2 = lcomp + il2 * (kPF + 1) + 4 * k2;
    const int rf = i0 + il2;

    int pf[kDepthF][2];
    auto fetch = [&](int s, int (&dst)[2]) {
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) dst[jj] = ld(s + 15, jj);
    };
#pragma unroll
    for (int d = 0; d < kDepthF; ++d) fetch(s_begin + d, pf[d]);

    for (int sg = s_begin; sg < s_end; sg += kSppF) {
        float h[2][16];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const float4 a0 = tp0[v], a1 = tp1[v];
            h[0][4 * v] = a0.x; h[0][4 * v + 1] = a0.y; h[0][4 * v + 2] = a0.z; h[0][4 * v + 3] = a0.w;
            h[1][4 * v] = a1.x; h[1][4 * v + 1] = a1.y; h[1][4 * v + 2] = a1.z; h[1][4 * v + 3] = a1.w;
        }
#pragma unroll
        for (int q = 0; q < kSppF; ++q) {
#pragma unroll
            for (int jj = 0; jj < 2; ++jj) win[jj][(q + 15) & 15] = (float)pf[q % kDepthF][jj];
            fetch(sg + q + kDepthF, pf[q % kDepthF]);
            float u[2];
#pragma unroll
            for (int jj = 0; jj < 2; ++jj) {
                float acc = 0.0f;
#pragma unroll
                for (int t = 0; t < 16; ++t) acc = fmaf(h[jj][t], win[jj][(q + t) & 15], acc);
                u[jj] = acc;
            }
            // quad lane (comp, jh) holds component comp of branches j = 2 jh + jj
            const float2 u0 = make_float2(quad_bcast<0>(u[0]), quad_bcast<1>(u[0]));
            const float2 u1 = make_float2(quad_bcast<0>(u[1]), quad_bcast<1>(u[1]));
            const float2 u2 = make_float2(quad_bcast<2>(u[0]), quad_bcast<3>(u[0]));
            const float2 u3 = make_float2(quad_bcast<2>(u[1]), quad_bcast<3>(u[1]));
            // A[k1] = (u0 + (-1)^k1 u2) + (-i)^k1 (u1 + (-1)^k1 u3), times the twiddle
            const float2 E = make_float2(fmaf(sgn, u2.x, u0.x), fmaf(sgn, u2.y, u0.y));
            const float2 Od = make_float2(fmaf(sgn, u3.x, u1.x), fmaf(sgn, u3.y, u1.y));
            float2 o = cmul(E, tw_o);
            o.x = fmaf(Od.x, rtw_o.x, fmaf(-Od.y, rtw_o.y, o.x));
            o.y = fmaf(Od.x, rtw_o.y, fmaf(Od.y, rtw_o.x, o.y));
            lds[q * kSSF + fir_w] = o;
            __builtin_amdgcn_sched_barrier(0);
        }
        lds_barrier();
        {
            float2 v[16];
#pragma unroll
            for (int r = 0; r < 16; ++r) v[r] = (r & 1) ? src1o[16 * r] : src1e[16 * r];
            dft16(v);
            lds_barrier();
#pragma unroll
            for (int ga = 0; ga < 4; ++ga)
#pragma unroll
                for (int de = 0; de < 4; ++de) {
                    const int kk = ga + 4 * de;            // k2
                    float2 y = v[4 * ga + de];
                    if (kk != 0) y = cmul(y, tw1[kk]);
                    lds[kk * kXS + xw] = y;
                }
        }
        lds_barrier();
        {
            float2 v[4][4];
            // the swizzle is per lane: keep its 8 addresses out of the
            // registers that live across the loop
            int sw = ql2;
            asm volatile("" : "+v"(sw));
#pragma unroll
            for (int m = 0; m < 16; ++m) v[m >> 2][m & 3] = src2[(m & 8) * 4 + (((m & 7) ^ sw) << 2)];
            float2 c4[4];
#pragma unroll
            for (int k3 = 0; k3 < 4; ++k3) c4[k3] = make_float2(0.0f, 0.0f);
#pragma unroll
            for (int k1 = 0; k1 < kRF; ++k1) {
                dft4(v[k1][0], v[k1][1], v[k1][2], v[k1][3]);
#pragma unroll
                for (int k3 = 0; k3 < 4; ++k3) c4[k3] = c4[k3] + cmul(v[k1][k3], comp2[k1 + 64 * k3]);
            }
            const int s = sg + q2;
            const int blk = s >> 3;
            if (rf < N && blk < a.Sb) {
                const bool live = s < S;
                const float g = live ? a.gain : 0.0f;
                // channel c = k2 + 16 k3: the wave-uniform part (k2 - k2lo +
                // 16 k3) goes to the store's scalar base, k2lo to the lane
                // offset (a channel pair spans far less than 4 GiB: one
                // subband of input is bounded to 2^31 values)
                const int64_t ch_stride = (int64_t)a.Sb * N * kSBlk;
                const unsigned lane_zoff = (unsigned)((blk * N + rf) * kSBlk + ql2 + k2lo * ch_stride);
                const int k2u = (wv >> 1) * 2;
#pragma unroll
                for (int k3 = 0; k3 < 4; ++k3) {
                    float2 y = c4[k3];
                    if constexpr (DT != AFC_I8)
                        if (!live) y = make_float2(0.0f, 0.0f);
                    store_sample<DT>(zs, (int64_t)(k2u + 16 * k3) * ch_stride, lane_zoff, y, g);
                }
            }
        }
        lds_barrier();
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
    a.n_chunks = (int)ceil_div(l.S, kChunkF);
    const int64_t total = (int64_t)l.B * a.n_groups * a.n_chunks;
    if (total > (1LL << 30)) return hipErrorInvalidValue;
    a.total = (int)total;
    a.per_xcd = (int)ceil_div(total, 8);
    const dim3 grid((unsigned)(a.per_xcd * 8));
    switch (l.dt) {
        case AFC_F32:
            hipLaunchKernelGGL(ppf_fine_kernel<AFC_F32>, grid, dim3(kThreadsF), 0, stream, a, tw64);
            break;
        case AFC_F16:
            hipLaunchKernelGGL(ppf_fine_kernel<AFC_F16>, grid, dim3(kThreadsF), 0, stream, a, tw64);
            break;
        default:
            hipLaunchKernelGGL(ppf_fine_kernel<AFC_I8>, grid, dim3(kThreadsF), 0, stream, a, tw64);
            break;
    }
    return hipGetLastError();
}

}  // namespace afc
