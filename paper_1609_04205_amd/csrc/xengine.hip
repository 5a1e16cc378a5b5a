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
#include <type_traits>

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
#ifndef AFC_I8_STAGE_BLOCKS
#define AFC_I8_STAGE_BLOCKS 4
#endif
template <int DT, int TILE>
constexpr int stage_blocks() {
    return (DT == AFC_F16 && TILE == 128) ? 2 : (DT == AFC_I8 && TILE == 128) ? AFC_I8_STAGE_BLOCKS : 4;
}
#ifndef AFC_PREFETCH_DEPTH
#define AFC_PREFETCH_DEPTH 2
#endif
template <int DT, int TILE>
constexpr int prefetch_depth() { return (DT == AFC_F16 && TILE == 128) ? 1 : AFC_PREFETCH_DEPTH; }
// int8 and fp16 stage through direct global-to-LDS loads (three buffers);
// fp32 through registers (two buffers)
template <int DT>
constexpr bool uses_dma() { return DT != AFC_F32; }
#ifndef AFC_DMA_DEPTH
#define AFC_DMA_DEPTH 2
#endif
constexpr int kDmaDepth = AFC_DMA_DEPTH;      // stages of global-to-LDS loads in flight
template <int DT, int TILE>
constexpr int lds_bytes() {
    return (uses_dma<DT>() ? kDmaDepth + 1 : 2) * 2 * stage_blocks<DT, TILE>() * TILE * XT<DT>::RB;
}


// Workgroup barrier for the DMA pipeline: no memory fence (which would wait
// for every outstanding global-to-LDS load); a compiler-level memory clobber
// keeps LDS accesses on their side of it.
__device__ __forceinline__ void dma_barrier() {
    __asm__ volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// s_waitcnt vmcnt(N) with the other counters left at their maximum
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
    static_assert(N >= 0 && N < 64, "vmcnt");
    __builtin_amdgcn_s_waitcnt((N & 15) | (((N >> 4) & 3) << 14) | 0x0F70);
}

// s_waitcnt vmcnt(PER * k) for a runtime k in [0, kDmaDepth - 1] (uniform)
template <int PER>
__device__ __forceinline__ void wait_vmcnt_runtime(int k) {
    if (k <= 0) wait_vmcnt<0>();
    else if (k == 1 || kDmaDepth <= 2) wait_vmcnt<PER>();
    else if (k == 2 || kDmaDepth <= 3) wait_vmcnt<(2 * PER < 63 ? 2 * PER : 63)>();
    else wait_vmcnt<(3 * PER < 63 ? 3 * PER : 63)>();
}

// 16-byte chunk q of receiver row r lives at chunk slot q ^ swz(r)
template <int RB, int PLANES>
__device__ __forceinline__ int swz(int r) {
    if constexpr (PLANES == 1) return 0;
    else return (r / (256 / RB)) % PLANES;
}

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

// (re, im) -> (-im, re) on packed int8 pairs: swap the bytes of each pair,
// negate each pair as a 16-bit number (its low byte becomes -im mod 256),
// keep the low bytes of that and the high bytes (re) of the swapped word.
__device__ __forceinline__ int jswap_i8(int w) {
    const unsigned t = __builtin_amdgcn_perm((unsigned)w, (unsigned)w, 0x02030001u);   // (im, re) per pair
    const u16x2 n = (u16x2)0 - __builtin_bit_cast(u16x2, t);
    const unsigned nb = __builtin_bit_cast(unsigned, n);
    return (int)((nb & 0x00FF00FFu) | (t & 0xFF00FF00u));
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
    constexpr bool kDma = uses_dma<DT>();
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

    // Loads are issued unconditionally from clamped addresses (always in
    // bounds) so that none of them waits on another; rows beyond N, blocks
    // beyond the subband's spectra and the tail spectra of the last block are
    // zeroed when the staged registers are written to LDS, after the compute
    // of the current stage has hidden the load latency.
    constexpr int DEPTH = prefetch_depth<DT, TILE>();   // stages of loads in flight
    uint4 pre[DEPTH][2][CPT];
    auto load_stage = [&](int st, auto slot_tag) {
        constexpr int slot = decltype(slot_tag)::value;
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
                const int blk = min(st * kStg + bl, nb - 1);
                const int rg = min(r0 + row, N - 1);
                pre[slot][pn][c] = *reinterpret_cast<const uint4*>(z + ((int64_t)blk * N + rg) * RB + q * 16);
            }
        }
    };
    // a stage needs no masking when all its blocks are whole and in range and
    // both panels' rows are below N (uniform over the workgroup)
    const bool rows_full = i0 + TILE <= N && j0 + TILE <= N;
    const int full_blocks = tail_valid < kSBlk ? nb - 1 : nb;
    auto store_stage = [&](int st, int buf, auto slot_tag) {
        constexpr int slot = decltype(slot_tag)::value;
        const bool clean = rows_full && (st + 1) * kStg <= full_blocks;
#pragma unroll
        for (int pn = 0; pn < 2; ++pn) {
            if (pn == 1 && diag) break;
            const int r0 = pn == 0 ? i0 : j0;
            char* base = lds_raw + (buf * 2 + pn) * PANEL;
#pragma unroll
            for (int c = 0; c < CPT; ++c) {
                const int chunk = tid + c * kThreads;
                const int bl = chunk / (TILE * PLANES);
                const int rem = chunk % (TILE * PLANES);
                const int row = rem / PLANES, q = rem % PLANES;
                const int blk = st * kStg + bl;
                uint4 v = pre[slot][pn][c];
                if (!clean) {
                    if (blk >= nb || r0 + row >= N) v = make_uint4(0u, 0u, 0u, 0u);
                    else if (blk == nb - 1 && tail_valid < kSBlk) v = mask_tail<DT>(v, q, tail_valid);
                }
                *reinterpret_cast<uint4*>(base + bl * TILE * RB + row * RB + ((q ^ swz<RB, PLANES>(row)) * 16)) = v;
            }
        }
    };
    auto rd = [&](const char* panel, int bl, int row, int q) -> uint4 {
        return *reinterpret_cast<const uint4*>(panel + bl * TILE * RB + row * RB + ((q ^ swz<RB, PLANES>(row)) * 16));
    };

    const int lr = lane & 31, lh = lane >> 5;
    int fold = 0;

    // MFMAs of one stage from the panels PA (rows) and PB (columns)
    auto compute = [&](const char* PA, const char* PB) {
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
    };

    if constexpr (kDma) {
        // Stages made of whole blocks go straight from global memory to LDS
        // (global_load_lds: lane L of a wave writes 16 bytes at M0 + 16 L),
        // kDmaDepth stages ahead, in a ring of kDmaDepth + 1 buffers.  Rows
        // beyond N read row N-1: they only feed outputs that are never
        // stored.  The remaining (partial) stage goes through registers with
        // masking.
        constexpr int NB = kDmaDepth + 1;
        const int n_clean = full_blocks / kStg;
        auto issue = [&](int st) {
            const int bq = st % NB;
#pragma unroll
            for (int pn = 0; pn < 2; ++pn) {
                if (pn == 1 && diag) break;
                const int r0 = pn == 0 ? i0 : j0;
#pragma unroll
                for (int c = 0; c < CPT; ++c) {
                    const int chunk = tid + c * kThreads;
                    const int bl = chunk / (TILE * PLANES);
                    const int rem = chunk % (TILE * PLANES);
                    const int row = rem / PLANES, sl = rem % PLANES;
                    const int q = sl ^ swz<RB, PLANES>(row);
                    const int blk = st * kStg + bl;
                    const char* src = z + ((int64_t)blk * N + min(r0 + row, N - 1)) * RB + q * 16;
                    char* dst = lds_raw + (bq * 2 + pn) * PANEL + (c * kThreads + wid * 64) * 16;
                    __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)dst, 16, 0, 0);
                }
            }
        };
#pragma unroll
        for (int d = 0; d < kDmaDepth; ++d)
            if (d < n_clean) issue(d);
        for (int st = 0; st < n_clean; ++st) {
            // this wave's loads of stage st have landed once at most the
            // later stages already issued (up to kDmaDepth - 1) are outstanding
            const int later = min(n_clean - 1 - st, kDmaDepth - 1);
            if (diag) wait_vmcnt_runtime<CPT>(later);
            else wait_vmcnt_runtime<2 * CPT>(later);
            // plain s_barrier: the explicit wait above already covers the
            // LDS written by this wave's DMA loads (an LDS fence here would
            // also wait for the stages still in flight)
            dma_barrier();
            if (st + kDmaDepth < n_clean) issue(st + kDmaDepth);
            const int bq = st % NB;
            compute(lds_raw + (bq * 2) * PANEL, lds_raw + (bq * 2 + (diag ? 0 : 1)) * PANEL);
        }
        using S0 = std::integral_constant<int, 0>;
        for (int st = n_clean; st < n_stages; ++st) {
            load_stage(st, S0{});
            lds_barrier();
            store_stage(st, 0, S0{});
            lds_barrier();
            compute(lds_raw, lds_raw + (diag ? 0 : 1) * PANEL);
        }
        lds_barrier();
    } else {
        // Register staging with one barrier per stage: at stage st the
        // registers hold the samples of the next DEPTH stages; stage st+1 goes
        // to the other LDS buffer first, its register slot is refilled with
        // stage st+1+DEPTH, then stage st is multiplied from its buffer.  The
        // barrier at the end of the stage orders both the buffer just written
        // (read at st+1) and the buffer just read (written at st+1).  Stage k
        // lives in register slot k % DEPTH; the loop is unrolled by DEPTH so
        // that every slot index is a constant.
        using S0 = std::integral_constant<int, 0>;
        using S1 = std::integral_constant<int, (DEPTH > 1 ? 1 : 0)>;
        load_stage(0, S0{});
        store_stage(0, 0, S0{});
        if (n_stages > 1) load_stage(1, S1{});
        if (DEPTH > 1 && n_stages > 2) load_stage(2, S0{});
        lds_barrier();
        auto step = [&](int st, auto slot_tag) {
            const int buf = st & 1;
            if (st + 1 < n_stages) {
                store_stage(st + 1, buf ^ 1, slot_tag);
                if (st + 1 + DEPTH < n_stages) load_stage(st + 1 + DEPTH, slot_tag);
            }
            compute(lds_raw + (buf * 2 + 0) * PANEL, lds_raw + (buf * 2 + (diag ? 0 : 1)) * PANEL);
            lds_barrier();
        };
        // stage st consumes slot (st + 1) % DEPTH
        for (int st = 0; st < n_stages; st += 2) {
            step(st, S1{});
            if (st + 1 < n_stages) step(st + 1, S0{});
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
    // flags of this lane's row antennas (8 per 32-row block) and column
    // antennas, fetched together before the stores
    bool frow[MB][8], fcol[MB];
#pragma unroll
    for (int m = 0; m < MB; ++m) {
        fcol[m] = false;
#pragma unroll
        for (int k = 0; k < 8; ++k) frow[m][k] = false;
    }
    if (fl_sb) {
        uint8_t fc[MB], fr[MB][8];
#pragma unroll
        for (int m = 0; m < MB; ++m) {
            fc[m] = fl_sb[min(j0 + wc * WT + m * 32 + lr, N - 1) >> 1];
#pragma unroll
            for (int k = 0; k < 8; ++k)
                fr[m][k] = fl_sb[min(i0 + wr * WT + m * 32 + 8 * (k >> 1) + 4 * lh + 2 * (k & 1), N - 1) >> 1];
        }
#pragma unroll
        for (int m = 0; m < MB; ++m) {
            fcol[m] = fc[m] != 0;
#pragma unroll
            for (int k = 0; k < 8; ++k) frow[m][k] = fr[m][k] != 0;
        }
    }
#pragma unroll
    for (int m = 0; m < MB; ++m)
#pragma unroll
        for (int n = 0; n < MB; ++n) {
            if (diag && wr == wc && m < n) continue;
            const int J = j0 + wc * WT + n * 32 + lr;
            if (J >= N) continue;
            const int b = J >> 1, qq = J & 1;
            const bool fb = fcol[n];
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int I = i0 + wr * WT + m * 32 + 8 * (r >> 2) + 4 * lh + (r & 3);
                if (I >= N) continue;
                const int a = I >> 1, p = I & 1;
                if (a < b) continue;
                const bool flagged = fb || frow[m][((r >> 2) << 1) | ((r >> 1) & 1)];
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
#ifdef AFC_NO_XCD_ORDER
    const int w = bid;
#else
    const int w = (bid & 7) * a.per_xcd + (bid >> 3);
#endif
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
        lds_barrier();
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
