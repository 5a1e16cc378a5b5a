// X-engine: lower triangle of the time-integrated Hermitian visibility matrix
// on MFMA.  Sec. "Correlation Kernel": the covariance matrix of every channel
// is split into tiles with only one triangle computed, and visibilities are
// accumulated over time in registers before a single write.
//
//   V_ij = sum_s z_i(s) conj(z_j(s))
//   Re V = sum (re_i re_j + im_i im_j),   Im V = sum (im_i re_j - re_i im_j)
//
// The complex product is mapped onto real MFMAs with the (re, im) pairs of
// each spectrum laid along the contraction axis: Re V = A B^T with A, B the
// interleaved samples, Im V = A B''^T with B'' = (-im, re) per spectrum,
// formed in registers from B.  No Gauss 3-multiply trick (its 9-bit sums do
// not fit int8).
//
// Work: one workgroup = one TILE x TILE tile (ti >= tj) of one channel of
// one subband; 4 waves in 2 x 2, each owning (TILE/2)^2 outputs as 32 x 32
// MFMA blocks.  Tiles wholly above the diagonal are never launched; inside a
// diagonal tile the wave and the MFMA blocks above the diagonal are skipped.
// Samples stream through LDS in stages of 2-4 spectrum blocks, double-buffered, copied with 16-byte coalesced loads of the block layout
// [block][receiver][8 spectra] and stored with an XOR swizzle of the 16-byte
// chunks so that the MFMA operand reads are bank-conflict free.
//
// Sample types (gfx950 MFMA):
//   int8  v_mfma_i32_32x32x32_i8  (16 spectra per K-step), exact int32 sums
//   fp16  v_mfma_f32_32x32x16_f16 ( 8 spectra per K-step), fp32 sums
//   fp32  v_mfma_f32_32x32x2_f32  ( 2 spectra per K-step), fp32 sums, summed
//         in two levels (blocks of 64 spectra into a second accumulator) to
//         keep the rounding error of 3051-term sums near 1e-7 relative
#include "afc_internal.h"

namespace afc {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef float v16f __attribute__((ext_vector_type(16)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));

constexpr int kThreads = 256;
constexpr int kF32Inner = 8;         // fp32: blocks summed before folding into the outer accumulator

template <int DT> struct XT;
// RB: bytes of one receiver in one spectrum block; PLANES: 16-byte chunks per RB.
template <> struct XT<AFC_I8> {
    static constexpr int RB = 16, PLANES = 1;
    using acc_t = v16i;
};
template <> struct XT<AFC_F16> {
    static constexpr int RB = 32, PLANES = 2;
    using acc_t = v16f;
};
template <> struct XT<AFC_F32> {
    static constexpr int RB = 64, PLANES = 4;
    using acc_t = v16f;
};
// spectrum blocks per LDS stage (fp16 at 128 keeps its prefetch registers down)
template <int DT, int TILE>
constexpr int stage_blocks() { return (DT == AFC_F16 && TILE == 128) ? 2 : 4; }
template <int DT, int TILE>
constexpr int lds_bytes() { return 2 * 2 * stage_blocks<DT, TILE>() * TILE * XT<DT>::RB; }

// 16-byte chunk q of receiver row r lives at chunk slot q ^ swz(r)
template <int RB, int PLANES>
__device__ __forceinline__ int swz(int r) {
    if constexpr (PLANES == 1) return 0;
    else return (r / (256 / RB)) % PLANES;
}

// (re, im) -> (-im, re) on packed int8 pairs
__device__ __forceinline__ int jswap_i8(int w) {
    const unsigned u = (unsigned)w;
    const unsigned t = ((u & 0x00FF00FFu) << 8) | ((u >> 8) & 0x00FF00FFu);   // (im, re) per pair
    return (int)((t & 0xFF00FF00u) | ((0x01000100u - (t & 0x00FF00FFu)) & 0x00FF00FFu));
}
// (re, im) -> (-im, re) on packed fp16 pairs
__device__ __forceinline__ int jswap_f16(int w) {
    const unsigned u = (unsigned)w;
    return (int)(((u >> 16) | (u << 16)) ^ 0x00008000u);
}

// Zero the spectra >= valid (1..8) of a 16-byte chunk of plane q.
template <int DT>
__device__ __forceinline__ uint4 mask_tail(uint4 v, int q, int valid) {
    unsigned d[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        if constexpr (DT == AFC_I8) {
            const int s0 = 2 * e;                       // two spectra per dword
            unsigned m = (s0 < valid ? 0x0000FFFFu : 0u) | (s0 + 1 < valid ? 0xFFFF0000u : 0u);
            d[e] &= m;
        } else if constexpr (DT == AFC_F16) {
            if (4 * q + e >= valid) d[e] = 0u;          // one spectrum per dword
        } else {
            if (2 * q + e / 2 >= valid) d[e] = 0u;      // half a spectrum per dword
        }
    }
    return make_uint4(d[0], d[1], d[2], d[3]);
}

struct XArgs {
    const char* z;              // subband 0, channel 0
    char* vis;
    int32_t* weights;
    const uint8_t* flags;
    int64_t z_ch_bytes;         // bytes between channels
    int64_t z_sb_bytes;         // bytes between subbands
    int N, Na, Sb, B, P;
    int n_tiles_side, n_tiles;
    int total, per_xcd;
    int S[AFC_MAX_SUBBANDS];
};

__device__ __forceinline__ void tile_rc(int t, int& ti, int& tj) {
    int r = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
    while (r * (r + 1) / 2 > t) --r;
    while ((r + 1) * (r + 2) / 2 <= t) ++r;
    ti = r;
    tj = t - r * (r + 1) / 2;
}

// One tile of one (subband, channel).  `z` points at channel ch of subband sb.
template <int DT, int TILE>
__device__ __forceinline__ void xtile(const char* __restrict__ z, char* __restrict__ vis_ch,
                                      int32_t* __restrict__ w_sb, const uint8_t* __restrict__ fl_sb,
                                      int N, int Na, int S, int ti, int tj, bool write_weights,
                                      char* lds_raw) {
    using Tr = XT<DT>;
    constexpr int RB = Tr::RB, PLANES = Tr::PLANES, kStg = stage_blocks<DT, TILE>();
    constexpr int WT = TILE / 2, MB = WT / 32;
    constexpr int PANEL = kStg * TILE * RB;                  // bytes of one panel in one stage
    constexpr int CHUNKS = kStg * TILE * PLANES;             // 16-byte chunks per panel per stage
    constexpr int CPT = CHUNKS / kThreads;
    using acc_t = typename Tr::acc_t;

    const int tid = threadIdx.x, lane = tid & 63;
    const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wr = wid >> 1, wc = wid & 1;
    const int i0 = ti * TILE, j0 = tj * TILE;
    const bool diag = ti == tj;
    const bool wave_on = !(diag && wr < wc);
    const int nb = (S + kSBlk - 1) / kSBlk;
    const int tail_valid = S - (nb - 1) * kSBlk;             // spectra in the last block
    const int n_stages = (nb + kStg - 1) / kStg;

    acc_t accR[MB][MB], accI[MB][MB];
    acc_t outR[MB][MB], outI[MB][MB];                        // fp32 only: outer level
#pragma unroll
    for (int m = 0; m < MB; ++m)
#pragma unroll
        for (int n = 0; n < MB; ++n) {
            accR[m][n] = acc_t{};
            accI[m][n] = acc_t{};
            outR[m][n] = acc_t{};
            outI[m][n] = acc_t{};
        }

    uint4 pre[2][CPT];
    auto load_stage = [&](int st) {
#pragma unroll
        for (int pn = 0; pn < 2; ++pn) {
            if (pn == 1 && diag) break;
            const int r0 = pn == 0 ? i0 : j0;
#pragma unroll
            for (int c = 0; c < CPT; ++c) {
                const int chunk = tid + c * kThreads;
                const int bl = chunk / (TILE * PLANES);
                const int rem = chunk % (TILE * PLANES);
                const int row = rem / PLANES, q = rem % PLANES;
                const int blk = st * kStg + bl;
                const int rg = r0 + row;
                uint4 v = make_uint4(0u, 0u, 0u, 0u);
                if (blk < nb && rg < N) {
                    v = *reinterpret_cast<const uint4*>(z + ((int64_t)blk * N + rg) * RB + q * 16);
                    if (blk == nb - 1 && tail_valid < kSBlk) v = mask_tail<DT>(v, q, tail_valid);
                }
                pre[pn][c] = v;
            }
        }
    };
    auto store_stage = [&](int buf) {
#pragma unroll
        for (int pn = 0; pn < 2; ++pn) {
            if (pn == 1 && diag) break;
            char* base = lds_raw + (buf * 2 + pn) * PANEL;
#pragma unroll
            for (int c = 0; c < CPT; ++c) {
                const int chunk = tid + c * kThreads;
                const int bl = chunk / (TILE * PLANES);
                const int rem = chunk % (TILE * PLANES);
                const int row = rem / PLANES, q = rem % PLANES;
                *reinterpret_cast<uint4*>(base + bl * TILE * RB + row * RB + ((q ^ swz<RB, PLANES>(row)) * 16)) =
                    pre[pn][c];
            }
        }
    };
    auto rd = [&](const char* panel, int bl, int row, int q) -> uint4 {
        return *reinterpret_cast<const uint4*>(panel + bl * TILE * RB + row * RB + ((q ^ swz<RB, PLANES>(row)) * 16));
    };

    const int lr = lane & 31, lh = lane >> 5;
    int fold = 0;

    load_stage(0);
    store_stage(0);
    __syncthreads();
    for (int st = 0; st < n_stages; ++st) {
        const int buf = st & 1;
        if (st + 1 < n_stages) load_stage(st + 1);
        const char* PA = lds_raw + (buf * 2 + 0) * PANEL;
        const char* PB = lds_raw + (buf * 2 + (diag ? 0 : 1)) * PANEL;
        if (wave_on) {
            if constexpr (DT == AFC_I8) {
#pragma unroll
                for (int kk = 0; kk < kStg / 2; ++kk) {
                    v4i a[MB], b[MB], bj[MB];
#pragma unroll
                    for (int m = 0; m < MB; ++m) {
                        const uint4 u = rd(PA, 2 * kk + lh, wr * WT + m * 32 + lr, 0);
                        a[m] = v4i{(int)u.x, (int)u.y, (int)u.z, (int)u.w};
                        const uint4 w = rd(PB, 2 * kk + lh, wc * WT + m * 32 + lr, 0);
                        b[m] = v4i{(int)w.x, (int)w.y, (int)w.z, (int)w.w};
                        bj[m] = v4i{jswap_i8((int)w.x), jswap_i8((int)w.y), jswap_i8((int)w.z), jswap_i8((int)w.w)};
                    }
#pragma unroll
                    for (int m = 0; m < MB; ++m)
#pragma unroll
                        for (int n = 0; n < MB; ++n) {
                            if (diag && wr == wc && m < n) continue;
                            accR[m][n] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[m], b[n], accR[m][n], 0, 0, 0);
                            accI[m][n] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[m], bj[n], accI[m][n], 0, 0, 0);
                        }
                }
            } else if constexpr (DT == AFC_F16) {
#pragma unroll
                for (int kk = 0; kk < kStg; ++kk) {
                    v8h a[MB], b[MB], bj[MB];
#pragma unroll
                    for (int m = 0; m < MB; ++m) {
                        const uint4 u = rd(PA, kk, wr * WT + m * 32 + lr, lh);
                        a[m] = __builtin_bit_cast(v8h, u);
                        const uint4 w = rd(PB, kk, wc * WT + m * 32 + lr, lh);
                        b[m] = __builtin_bit_cast(v8h, w);
                        const uint4 wj = make_uint4((unsigned)jswap_f16((int)w.x), (unsigned)jswap_f16((int)w.y),
                                                    (unsigned)jswap_f16((int)w.z), (unsigned)jswap_f16((int)w.w));
                        bj[m] = __builtin_bit_cast(v8h, wj);
                    }
#pragma unroll
                    for (int m = 0; m < MB; ++m)
#pragma unroll
                        for (int n = 0; n < MB; ++n) {
                            if (diag && wr == wc && m < n) continue;
                            accR[m][n] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a[m], b[n], accR[m][n], 0, 0, 0);
                            accI[m][n] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a[m], bj[n], accI[m][n], 0, 0, 0);
                        }
                }
            } else {
#pragma unroll
                for (int kk = 0; kk < kStg; ++kk) {
#pragma unroll
                    for (int r2 = 0; r2 < 2; ++r2) {
                        float4 a[MB], b[MB];
#pragma unroll
                        for (int m = 0; m < MB; ++m) {
                            a[m] = __builtin_bit_cast(float4, rd(PA, kk, wr * WT + m * 32 + lr, 2 * r2 + lh));
                            b[m] = __builtin_bit_cast(float4, rd(PB, kk, wc * WT + m * 32 + lr, 2 * r2 + lh));
                        }
#pragma unroll
                        for (int m = 0; m < MB; ++m)
#pragma unroll
                            for (int n = 0; n < MB; ++n) {
                                if (diag && wr == wc && m < n) continue;
                                acc_t R = accR[m][n], I = accI[m][n];
                                R = __builtin_amdgcn_mfma_f32_32x32x2f32(a[m].x, b[n].x, R, 0, 0, 0);
                                R = __builtin_amdgcn_mfma_f32_32x32x2f32(a[m].y, b[n].y, R, 0, 0, 0);
                                I = __builtin_amdgcn_mfma_f32_32x32x2f32(a[m].y, b[n].x, I, 0, 0, 0);
                                I = __builtin_amdgcn_mfma_f32_32x32x2f32(a[m].x, -b[n].y, I, 0, 0, 0);
                                R = __builtin_amdgcn_mfma_f32_32x32x2f32(a[m].z, b[n].z, R, 0, 0, 0);
                                R = __builtin_amdgcn_mfma_f32_32x32x2f32(a[m].w, b[n].w, R, 0, 0, 0);
                                I = __builtin_amdgcn_mfma_f32_32x32x2f32(a[m].w, b[n].z, I, 0, 0, 0);
                                I = __builtin_amdgcn_mfma_f32_32x32x2f32(a[m].z, -b[n].w, I, 0, 0, 0);
                                accR[m][n] = R;
                                accI[m][n] = I;
                            }
                    }
                    if (++fold == kF32Inner) {
                        fold = 0;
#pragma unroll
                        for (int m = 0; m < MB; ++m)
#pragma unroll
                            for (int n = 0; n < MB; ++n) {
                                outR[m][n] += accR[m][n];
                                outI[m][n] += accI[m][n];
                                accR[m][n] = acc_t{};
                                accI[m][n] = acc_t{};
                            }
                    }
                }
            }
        }
        __syncthreads();
        if (st + 1 < n_stages) {
            store_stage(buf ^ 1);
            __syncthreads();
        }
    }
    if constexpr (DT == AFC_F32) {
#pragma unroll
        for (int m = 0; m < MB; ++m)
#pragma unroll
            for (int n = 0; n < MB; ++n) {
                accR[m][n] += outR[m][n];
                accI[m][n] += outI[m][n];
            }
    }
    if (!wave_on) return;

    // ---- epilogue: 2x2 polarisation blocks of antennas a >= b
    const int64_t nbl = (int64_t)Na * (Na + 1) / 2;
    (void)nbl;
#pragma unroll
    for (int m = 0; m < MB; ++m)
#pragma unroll
        for (int n = 0; n < MB; ++n) {
            if (diag && wr == wc && m < n) continue;
            const int J = j0 + wc * WT + n * 32 + lr;
            if (J >= N) continue;
            const int b = J >> 1, qq = J & 1;
            const bool fb = fl_sb ? fl_sb[b] != 0 : false;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int I = i0 + wr * WT + m * 32 + 8 * (r >> 2) + 4 * lh + (r & 3);
                if (I >= N) continue;
                const int a = I >> 1, p = I & 1;
                if (a < b) continue;
                const bool flagged = fb || (fl_sb ? fl_sb[a] != 0 : false);
                const int64_t bl = (int64_t)a * (a + 1) / 2 + b;
                const int64_t e = bl * 4 + p * 2 + qq;
                if constexpr (DT == AFC_I8) {
                    int re = accR[m][n][r], im = accI[m][n][r];
                    if (I == J) im = 0;
                    if (flagged) re = im = 0;
                    reinterpret_cast<int2*>(vis_ch)[e] = make_int2(re, im);
                } else {
                    float re = accR[m][n][r], im = accI[m][n][r];
                    if (I == J) im = 0.0f;
                    if (flagged) re = im = 0.0f;
                    reinterpret_cast<float2*>(vis_ch)[e] = make_float2(re, im);
                }
                if (write_weights && p == 0 && qq == 0) w_sb[bl] = flagged ? 0 : S;
            }
        }
}

template <int DT, int TILE>
__global__ __launch_bounds__(kThreads, 2) void xengine_kernel(XArgs a) {
    __shared__ __attribute__((aligned(16))) char lds[lds_bytes<DT, TILE>()];
    // XCD-aware order: consecutive workgroup ids go round-robin over the 8
    // XCDs; give each XCD a contiguous range of work so that the tiles of one
    // channel share that XCD's L2.
    const int bid = blockIdx.x;
    const int w = (bid & 7) * a.per_xcd + (bid >> 3);
    if (w >= a.total) return;
    const int t = w % a.n_tiles;
    const int rest = w / a.n_tiles;
    const int ch = rest % a.P;
    const int sb = rest / a.P;
    int ti, tj;
    tile_rc(t, ti, tj);
    const char* z = a.z + sb * a.z_sb_bytes + ch * a.z_ch_bytes;
    const int64_t nbl = (int64_t)a.Na * (a.Na + 1) / 2;
    char* vis = a.vis + ((int64_t)sb * a.P + ch) * nbl * 4 * 8;
    int32_t* wsb = a.weights ? a.weights + (int64_t)sb * nbl : nullptr;
    const uint8_t* fl = a.flags ? a.flags + (int64_t)sb * a.Na : nullptr;
    xtile<DT, TILE>(z, vis, wsb, fl, a.N, a.Na, a.S[sb], ti, tj, wsb != nullptr && ch == 0, lds);
}

// Persistent batched form: a fixed grid walks a host-balanced list of work
// items; each item is one tile of one channel of one subband with its own
// sample type and integration length.  MODE 0 serves int8 and fp16 subbands
// (mixed in one launch) with TILE-wide tiles, MODE 1 fp32 subbands (64).
template <int MODE, int TILE, int WPC>
__global__ __launch_bounds__(kThreads, WPC) void xengine_persistent_kernel(
    const char* __restrict__ z_ws, char* __restrict__ vis, int32_t* __restrict__ weights,
    const uint8_t* __restrict__ flags, const XSubband* __restrict__ sbs, const XWork* __restrict__ work,
    const int32_t* __restrict__ wg_begin, int N, int Na) {
    constexpr int kLds = MODE == 0 ? (lds_bytes<AFC_I8, TILE>() > lds_bytes<AFC_F16, TILE>() ? lds_bytes<AFC_I8, TILE>()
                                                                                            : lds_bytes<AFC_F16, TILE>())
                                   : lds_bytes<AFC_F32, TILE>();
    __shared__ __attribute__((aligned(16))) char lds[kLds];
    const int64_t nbl = (int64_t)Na * (Na + 1) / 2;
    const int b = blockIdx.x;
    const int e0 = wg_begin[b], e1 = wg_begin[b + 1];
    for (int e = e0; e < e1; ++e) {
        const XWork wk = work[e];
        const XSubband sd = sbs[wk.sb];
        char* vis_ch = vis + sd.vis_off + (int64_t)wk.ch * nbl * 4 * 8;
        int32_t* wsb = weights ? weights + (int64_t)wk.sb * nbl : nullptr;
        const uint8_t* fl = flags ? flags + (int64_t)wk.sb * Na : nullptr;
        const bool ww = wsb != nullptr && wk.ch == 0;
        if constexpr (MODE == 0) {
            if (sd.dt == AFC_I8) {
                const char* z = z_ws + sd.z_off + (int64_t)wk.ch * sd.Sb * N * kSBlk * 2;
                xtile<AFC_I8, TILE>(z, vis_ch, wsb, fl, N, Na, sd.S, wk.ti, wk.tj, ww, lds);
            } else {
                const char* z = z_ws + sd.z_off + (int64_t)wk.ch * sd.Sb * N * kSBlk * 4;
                xtile<AFC_F16, TILE>(z, vis_ch, wsb, fl, N, Na, sd.S, wk.ti, wk.tj, ww, lds);
            }
        } else {
            const char* z = z_ws + sd.z_off + (int64_t)wk.ch * sd.Sb * N * kSBlk * 8;
            xtile<AFC_F32, TILE>(z, vis_ch, wsb, fl, N, Na, sd.S, wk.ti, wk.tj, ww, lds);
        }
        __syncthreads();
    }
}

}  // namespace

int xengine_tile(afc_dtype dt) { return dt == AFC_F32 ? 64 : 128; }

hipError_t launch_xengine(const XLaunch& l, hipStream_t stream) {
    XArgs a{};
    a.z = reinterpret_cast<const char*>(l.z);
    a.vis = reinterpret_cast<char*>(l.vis);
    a.weights = l.weights;
    a.flags = l.flags;
    const int sbytes = sample_bytes(l.dt);
    a.z_ch_bytes = l.z_ch_stride * sbytes;
    a.z_sb_bytes = l.z_sb_stride * sbytes;
    a.N = l.N;
    a.Na = l.Na;
    a.Sb = l.Sb;
    a.B = l.B;
    a.P = kP;
    const int tile = xengine_tile(l.dt);
    a.n_tiles_side = (int)ceil_div(l.N, tile);
    a.n_tiles = a.n_tiles_side * (a.n_tiles_side + 1) / 2;
    const int64_t total = (int64_t)a.n_tiles * kP * l.B;
    if (total > (1LL << 30)) return hipErrorInvalidValue;
    a.total = (int)total;
    a.per_xcd = (int)ceil_div(total, 8);
    for (int b = 0; b < l.B; ++b) a.S[b] = l.S_host[b];
    const dim3 grid((unsigned)(a.per_xcd * 8));
    switch (l.dt) {
        case AFC_I8: hipLaunchKernelGGL((xengine_kernel<AFC_I8, 128>), grid, dim3(kThreads), 0, stream, a); break;
        case AFC_F16: hipLaunchKernelGGL((xengine_kernel<AFC_F16, 128>), grid, dim3(kThreads), 0, stream, a); break;
        default: hipLaunchKernelGGL((xengine_kernel<AFC_F32, 64>), grid, dim3(kThreads), 0, stream, a); break;
    }
    return hipGetLastError();
}

hipError_t launch_xengine_persistent(const void* z_ws, void* vis, int32_t* weights, const uint8_t* flags,
                                     const XSubband* sbs_dev, const XWork* work_dev, const int32_t* wg_begin_dev,
                                     int n_wg, int N, int Na, int mode, int tile, hipStream_t stream) {
    const char* z = reinterpret_cast<const char*>(z_ws);
    char* v = reinterpret_cast<char*>(vis);
    const dim3 grid((unsigned)n_wg), block(kThreads);
    if (mode == 1)  // fp32 subbands
        hipLaunchKernelGGL((xengine_persistent_kernel<1, 64, 2>), grid, block, 0, stream, z, v, weights, flags,
                           sbs_dev, work_dev, wg_begin_dev, N, Na);
    else if (tile == 128)
        hipLaunchKernelGGL((xengine_persistent_kernel<0, 128, 2>), grid, block, 0, stream, z, v, weights, flags,
                           sbs_dev, work_dev, wg_begin_dev, N, Na);
    else
        hipLaunchKernelGGL((xengine_persistent_kernel<0, 64, 4>), grid, block, 0, stream, z, v, weights, flags,
                           sbs_dev, work_dev, wg_begin_dev, N, Na);
    return hipGetLastError();
}

}  // namespace afc
