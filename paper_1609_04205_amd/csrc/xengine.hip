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
// one subband, 4 waves.  int8 / fp16 outputs are 16 x 16 MFMA blocks (on
// noise-like operands the power limit lets these shapes run ~15% more
// operations per second than the 32 x 32 ones, for the same operand bytes
// per operation).  128-wide tiles: off the diagonal wave w owns column blocks
// 2w, 2w+1 against the eight row blocks (128 x 32 outputs); a diagonal tile
// gives wave w the column blocks w and 7-w, nine blocks on or below the
// diagonal each.  64-wide tiles: four row blocks x column block w off the
// diagonal, ten blocks split 3/3/2/2 on it.  fp32: 32 x 32 blocks, 2 x 2
// waves of one quarter each, the wave above the diagonal idle on a diagonal
// tile.  Tiles wholly above the diagonal are never launched.
// int8 / fp16: the row panel of a tile streams through LDS in stages of one
// MFMA k-step (direct global-to-LDS loads of the block layout
// [block][receiver][8 spectra], XOR-swizzled 16-byte chunks so that the MFMA
// operand reads are bank-conflict free); off the diagonal each wave loads
// its own column blocks straight into registers.  fp32 stages both panels
// through registers into LDS.
//
// Sample types (gfx950 MFMA):
//   int8  v_mfma_i32_16x16x64_i8  (32 spectra per k-step), exact int32 sums
//   fp16  v_mfma_f32_16x16x32_f16 (16 spectra per k-step), fp32 sums
//   fp32  v_mfma_f32_32x32x2_f32  ( 2 spectra per k-step), fp32 sums, summed
//         in two levels (blocks of 64 spectra into a second accumulator) to
//         keep the rounding error of 3051-term sums near 1e-7 relative
#include <algorithm>
#include <type_traits>
#include <utility>

#include "afc_internal.h"

namespace afc {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef float v16f __attribute__((ext_vector_type(16)));
typedef float v4f __attribute__((ext_vector_type(4)));
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
// spectrum blocks per LDS stage: int8 / fp16 one 16 x 16 MFMA k-step (64
// bytes of each receiver), fp32 four blocks
template <int DT, int TILE>
constexpr int stage_blocks() {
    return DT == AFC_F32 ? 4 : 64 / XT<DT>::RB;
}
// fp32: stages of register-staged loads in flight
template <int DT, int TILE>
constexpr int prefetch_depth() { return 2; }
// int8 and fp16 stage through direct global-to-LDS loads, fp32 through registers
template <int DT>
constexpr bool uses_dma() { return DT != AFC_F32; }
// stages of global-to-LDS loads in flight beyond the next one: one stage is
// 32 spectra for int8 and 16 for fp16
#ifndef AFC_I8_DMA_DEPTH
#define AFC_I8_DMA_DEPTH 2
#endif
#ifndef AFC_F16_DMA_DEPTH
#define AFC_F16_DMA_DEPTH 3
#endif
template <int DT>
constexpr int dma_depth() { return DT == AFC_I8 ? AFC_I8_DMA_DEPTH : AFC_F16_DMA_DEPTH; }
// DMA ring: the stage being multiplied, the next one (landed before its
// operands are read) and dma_depth - 1 further stages in flight, plus the
// buffer being refilled
template <int DT>
constexpr int dma_buffers() { return dma_depth<DT>() + 2; }
template <int DT, int TILE>
constexpr int lds_bytes() {
    // 128-wide int8 / fp16 tiles stage only the row panel (their column
    // operands are loaded into registers, or, on the diagonal, are the row
    // panel); the others stage both
    constexpr int panels = uses_dma<DT>() && TILE == 128 ? 1 : 2;
    return (uses_dma<DT>() ? dma_buffers<DT>() : 2) * panels * stage_blocks<DT, TILE>() * TILE * XT<DT>::RB;
}

// Workgroup barrier for the DMA pipeline: no memory fence (which would wait
// for every outstanding global-to-LDS load) and no wait for the wave's LDS
// reads: the buffer refilled after it is the one the previous stage read,
// and each of those reads has fed an MFMA or an operand conversion of that
// stage before the wave reaches the barrier; the reads still in flight are
// of the next stage's buffer.  A compiler-level memory clobber keeps LDS
// accesses on their side of it.
__device__ __forceinline__ void dma_barrier() {
    __asm__ volatile("s_barrier" ::: "memory");
}

// 16 bytes per lane from base + voff + soff (a raw buffer of `bytes` bytes)
// into LDS: lane L of the wave writes dst + 16 L (dst wave-uniform)
__device__ __forceinline__ void buffer_load_lds16(const char* base, int bytes, char* dst, int voff, int soff) {
#if defined(__HIP_DEVICE_COMPILE__)
    const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, bytes, 0x00020000);
    __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (__attribute__((address_space(3))) void*)dst, 16, voff, soff, 0, 0);
#endif
}

// 16 bytes from base + voff + soff (a raw buffer of `bytes` bytes) into
// registers.  A buffer load, unlike a flat one, cannot touch LDS, so the
// compiler's LDS wait counts stay exact around it.
__device__ __forceinline__ uint4 buffer_load16(const char* base, int bytes, int voff, int soff) {
#if defined(__HIP_DEVICE_COMPILE__)
    const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, bytes, 0x00020000);
    const v4i v = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
    return make_uint4((unsigned)v.x, (unsigned)v.y, (unsigned)v.z, (unsigned)v.w);
#else
    return make_uint4(0u, 0u, 0u, 0u);
#endif
}

template <class F, int... I>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}
// f(integral_constant<int, 0>) ... f(integral_constant<int, N - 1>)
template <int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
    static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// s_waitcnt vmcnt(N) with the other counters left at their maximum
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
    static_assert(N >= 0 && N < 64, "vmcnt");
    __builtin_amdgcn_s_waitcnt((N & 15) | (((N >> 4) & 3) << 14) | 0x0F70);
}

// s_waitcnt vmcnt(PER * k) for a runtime k in [0, DEPTH - 1] (uniform)
template <int PER, int DEPTH>
__device__ __forceinline__ void wait_vmcnt_runtime(int k) {
    static_assert(DEPTH >= 1 && DEPTH <= 4, "DMA depth 1..4");
    if (k <= 0) wait_vmcnt<0>();
    else if (k == 1 || DEPTH <= 2) wait_vmcnt<PER>();
    else if (k == 2 || DEPTH <= 3) wait_vmcnt<(2 * PER < 63 ? 2 * PER : 63)>();
    else wait_vmcnt<(3 * PER < 63 ? 3 * PER : 63)>();
}

// 16-byte chunk q of receiver row r lives at chunk slot q ^ swz(r)
template <int RB, int PLANES>
__device__ __forceinline__ int swz(int r) {
    if constexpr (PLANES == 1) return 0;
    else return (r / (256 / RB)) % PLANES;
}

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

// value of the lane at (this lane xor 1) (DPP quad_perm [1,0,3,2])
__device__ __forceinline__ int pair_swap(int v) {
    return __builtin_amdgcn_mov_dpp(v, 1 | (0 << 2) | (3 << 4) | (2 << 6), 0xF, 0xF, false);
}
__device__ __forceinline__ float pair_swap(float v) { return __int_as_float(pair_swap(__float_as_int(v))); }

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

// ---------------------------------------------------------------------------
// int8 / fp16 tiles in 16 x 16 MFMA blocks (int8 16x16x64, fp16 16x16x32).
//
// One stage of the DMA ring is exactly one k-step (64 bytes of K per lane
// group: int8 4 spectrum blocks, fp16 2).  A lane supplies row (or column)
// lane % 16 and the 16-byte K chunk lane / 16; the output block leaves
// column lane % 16, rows 4 (lane / 16) + 0..3 in the lane.
//
// Jobs: NP blocks pairing row operand IA[p] with column operand IB[p]; the
// blocks of one row operand are consecutive, so that the operand's register
// can take the next stage's value right after its last MFMA (a rolling
// reload instead of a second operand set: the 128-tile's 8 x 2 job holds 128
// accumulator registers).
struct JobTab {
    int IA[16], IB[16], AM[8], BN[2];
};
constexpr JobTab rows_by_cols(int na, int nb) {
    JobTab t{};
    int p = 0;
    for (int i = 0; i < na; ++i)
        for (int j = 0; j < nb; ++j) {
            t.IA[p] = i;
            t.IB[p] = j;
            ++p;
        }
    for (int i = 0; i < na; ++i) t.AM[i] = i;
    return t;
}
// diagonal 128-tile (8 x 8 blocks, 36 on or below the diagonal): wave w takes
// column blocks w (rows w..7) and 7 - w (rows 7-w..7), 9 blocks each
constexpr JobTab diag8(int w) {
    JobTab t{};
    int p = 0;
    for (int i = w; i < 8; ++i) {
        t.IA[p] = i - w;
        t.IB[p] = 0;
        ++p;
        if (i >= 7 - w) {
            t.IA[p] = i - w;
            t.IB[p] = 1;
            ++p;
        }
    }
    for (int k = 0; k < 8 - w; ++k) t.AM[k] = w + k;
    t.BN[0] = w;
    t.BN[1] = 7 - w;
    return t;
}
// diagonal 64-tile (4 x 4 blocks, 10 on or below the diagonal) split 3/3/2/2
constexpr JobTab diag4(int w) {
    JobTab t{};
    if (w == 0) {          // (0,0) (1,0) (2,0)
        t = rows_by_cols(3, 1);
    } else if (w == 1) {   // (3,0) (1,1) (2,1)
        t.IA[0] = 0, t.IB[0] = 0, t.IA[1] = 1, t.IB[1] = 1, t.IA[2] = 2, t.IB[2] = 1;
        t.AM[0] = 3, t.AM[1] = 1, t.AM[2] = 2;
        t.BN[0] = 0, t.BN[1] = 1;
    } else if (w == 2) {   // (3,1) (2,2)
        t.IA[0] = 0, t.IB[0] = 0, t.IA[1] = 1, t.IB[1] = 1;
        t.AM[0] = 3, t.AM[1] = 2;
        t.BN[0] = 1, t.BN[1] = 2;
    } else {               // (3,2) (3,3)
        t.IA[0] = 0, t.IB[0] = 0, t.IA[1] = 0, t.IB[1] = 1;
        t.AM[0] = 3;
        t.BN[0] = 2, t.BN[1] = 3;
    }
    return t;
}
template <int NA_, int NB_, int NP_, bool kDiag_, bool kDirectB_>
struct Job16Base {
    static constexpr int NA = NA_, NB = NB_, NP = NP_;
    static constexpr bool kDiag = kDiag_, kDirectB = kDirectB_;
};
// off-diagonal 128-tile: all 8 row blocks x this wave's 2 column blocks
struct Job16R8C2 : Job16Base<8, 2, 16, false, true> {
    static constexpr JobTab T = rows_by_cols(8, 2);
};
template <int W>
struct Job16D8 : Job16Base<8 - W, 2, 9, true, false> {
    static constexpr JobTab T = diag8(W);
};
// off-diagonal 64-tile: all 4 row blocks x this wave's column block
struct Job16R4C1 : Job16Base<4, 1, 4, false, false> {
    static constexpr JobTab T = rows_by_cols(4, 1);
};
template <int W>
struct Job16D4 : Job16Base<W == 0 ? 3 : W == 1 ? 3 : W == 2 ? 2 : 1, W == 0 ? 1 : 2, W < 2 ? 3 : 2, true, false> {
    static constexpr JobTab T = diag4(W);
};

// the last block of job J that uses row operand i / column operand j
template <class J>
constexpr int last_use(int i) {
    int last = -1;
    for (int p = 0; p < J::NP; ++p)
        if (J::T.IA[p] == i) last = p;
    return last;
}
template <class J>
constexpr int last_use_b(int j) {
    int last = -1;
    for (int p = 0; p < J::NP; ++p)
        if (J::T.IB[p] == j) last = p;
    return last;
}

template <int DT, int TILE, class J>
__device__ __forceinline__ void xtile_mm16(const char* __restrict__ z, char* __restrict__ vis_ch,
                                           int32_t* __restrict__ w_sb, const uint8_t* __restrict__ fl_sb,
                                           int N, int Na, int S, int ti, int tj, bool write_weights,
                                           char* lds_raw, const int (&am)[8], const int (&bn)[2]) {
    using Tr = XT<DT>;
    using acc_t = std::conditional_t<DT == AFC_I8, v4i, v4f>;
    using V = std::conditional_t<DT == AFC_I8, v4i, v8h>;
    constexpr int RB = Tr::RB, PLANES = Tr::PLANES, kStg = stage_blocks<DT, TILE>();
    static_assert(kStg * RB == 64, "one stage is one 16 x 16 MFMA k-step");
    constexpr int PANEL = kStg * TILE * RB;                  // bytes of panel A in one stage
    constexpr int PANEL_B = PANEL;                           // bytes of panel B in one stage
    constexpr int CPT = kStg * TILE * PLANES / kThreads;     // 16-byte chunks of A per thread per stage
    constexpr int CPT_B = CPT;
    static_assert((kStg * TILE * PLANES) % kThreads == 0, "a stage must split evenly over the threads");
    constexpr int NA = J::NA, NBO = J::NB, NP = J::NP;
    constexpr int kDmaDepth = dma_depth<DT>();
    constexpr int NB = dma_buffers<DT>();
    constexpr bool kDiagJob = J::kDiag;
    // off-diagonal 128-tiles load their column operands straight into
    // registers (each wave alone uses its two column blocks), in a ring of RS
    // register slots: the stage in use and kDmaDepth in flight
    constexpr bool BD = J::kDirectB;
    constexpr int RS = BD ? kDmaDepth + 1 : 1;
    static_assert(RS <= 4, "register ring of at most four stages");
    constexpr int BUF = PANEL + (BD || kDiagJob ? 0 : PANEL_B);

    const int tid = threadIdx.x, lane = tid & 63, lc = lane & 15, lg = lane >> 4;
    const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int i0 = ti * TILE, j0 = tj * TILE;
    const bool diag = ti == tj;
    const int nb = (S + kSBlk - 1) / kSBlk;
    const int tail_valid = S - (nb - 1) * kSBlk;
    const int n_st = (nb + kStg * RS - 1) / (kStg * RS) * RS;
    const int n_final = n_st - RS;
    // this lane's K chunk: spectrum block lbl of the stage, plane q of it
    const int lbl = DT == AFC_I8 ? lg : lg >> 1;
    const int q = DT == AFC_I8 ? 0 : lg & 1;

    acc_t accR[NP], accI[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        accR[p] = acc_t{};
        accI[p] = acc_t{};
    }
    auto rd = [&](const char* panel, int row) -> uint4 {
        return *reinterpret_cast<const uint4*>(panel + lbl * TILE * RB + row * RB + ((q ^ swz<RB, PLANES>(row)) * 16));
    };
    auto cvt = [](uint4 u) -> V {
        if constexpr (DT == AFC_I8) return v4i{(int)u.x, (int)u.y, (int)u.z, (int)u.w};
        else return __builtin_bit_cast(v8h, u);
    };
    auto jsw = [](uint4 u) -> V {
        if constexpr (DT == AFC_I8)
            return v4i{jswap_i8((int)u.x), jswap_i8((int)u.y), jswap_i8((int)u.z), jswap_i8((int)u.w)};
        else
            return __builtin_bit_cast(v8h, make_uint4((unsigned)jswap_f16((int)u.x), (unsigned)jswap_f16((int)u.y),
                                                      (unsigned)jswap_f16((int)u.z), (unsigned)jswap_f16((int)u.w)));
    };
    auto op = [&](acc_t& acc, V x, V y) {
        if constexpr (DT == AFC_I8) acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(x, y, acc, 0, 0, 0);
        else acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(x, y, acc, 0, 0, 0);
    };
    // zero the spectra >= S of an operand chunk of stage st
    auto mask_op = [&](int st, uint4& v) {
        const int blk = st * kStg + lbl;
        if (blk < nb - 1 || (blk == nb - 1 && tail_valid == kSBlk)) return;
        v = mask_tail<DT>(v, q, blk == nb - 1 ? tail_valid : 0);
    };

    // Samples go straight from global memory to LDS (buffer loads with the
    // LDS bit: lane L of a wave writes 16 bytes at M0 + 16 L) through a ring
    // of NB stage buffers.  Buffer rather than global loads: the compiler
    // must assume that global (flat) ones may also touch LDS and would then
    // wait for every LDS read at once.  Rows beyond N read row N-1 (they only
    // feed outputs that are never stored); blocks beyond the data read the
    // last block again, and the operands of the partial last block are
    // masked in registers.
    //
    // One barrier per stage, after the stage's first MFMAs: by then every
    // wave has waited for its own loads of the next stage and has finished
    // the previous stage, so the DMA of stage st + 1 + depth refills the
    // previous stage's buffer and the next stage's operands may be read.
    const int z_bytes = nb * N * RB;
    auto chunk_src = [&](int c, int r0) {
        const int chunk = tid + c * kThreads;
        const int bl = chunk / (TILE * PLANES);
        const int rem = chunk % (TILE * PLANES);
        const int row = rem / PLANES, sl = rem % PLANES;
        const int qq = sl ^ swz<RB, PLANES>(row);
        return (bl * N + min(r0 + row, N - 1)) * RB + qq * 16;
    };
    int src_a[CPT], src_b[CPT_B];
#pragma unroll
    for (int c = 0; c < CPT; ++c) src_a[c] = chunk_src(c, i0);
#pragma unroll
    for (int c = 0; c < CPT_B; ++c) src_b[c] = chunk_src(c, j0);
    const int stage_bytes = kStg * N * RB;
    // A stage whose blocks all lie in the data takes its offset as the
    // scalar part of the load; past the end (the last stages) the block is
    // clamped to nb - 1 per lane, and every offset then lies in the channel's
    // data (the scalar part of a buffer offset is not range-checked).  Only
    // the offsets sit behind the (uniform) branch, not the loads.  The clamp
    // tag is false only where the stage is known to be whole: the loads the
    // main loop of the register-ring form issues.
    auto issue_panel = [&](auto clamp_tag, int st, char* panel, int c, int src) {
        char* dst = panel + (c * kThreads + wid * 64) * 16;
        int voff = src, soff = st * stage_bytes;
        if (decltype(clamp_tag)::value && (st + 1) * kStg > nb) {
            const int bl = (tid + c * kThreads) / (TILE * PLANES);
            voff += (min(st * kStg + bl, nb - 1) - bl) * N * RB;
            soff = 0;
        }
        buffer_load_lds16(z, z_bytes, dst, voff, soff);
    };
    // the column operands' per-lane offsets within a stage
    int b_off[NBO];
#pragma unroll
    for (int x = 0; x < NBO; ++x) b_off[x] = (lbl * N + min(j0 + bn[x] * 16 + lc, N - 1)) * RB + q * 16;
    uint4 bdir[RS][BD ? NBO : 1];
    auto issue_b = [&](auto clamp_tag, auto slot_tag, int st) {
        constexpr int slot = decltype(slot_tag)::value;
        int soff = st * stage_bytes, dv = 0;
        if (decltype(clamp_tag)::value && (st + 1) * kStg > nb) {
            dv = (min(st * kStg + lbl, nb - 1) - lbl) * N * RB;
            soff = 0;
        }
#pragma unroll
        for (int x = 0; x < NBO; ++x) bdir[slot][x] = buffer_load16(z, z_bytes, b_off[x] + dv, soff);
    };
    auto issue_a = [&](auto clamp_tag, int st) {
        char* buf = lds_raw + (st % NB) * BUF;
#pragma unroll
        for (int c = 0; c < CPT; ++c) issue_panel(clamp_tag, st, buf, c, src_a[c]);
        if constexpr (!BD) {
            if (!diag) {
#pragma unroll
                for (int c = 0; c < CPT_B; ++c) issue_panel(clamp_tag, st, buf + PANEL, c, src_b[c]);
            }
        }
    };
    auto issue = [&](auto slot_tag, int st) {
        issue_a(std::true_type{}, st);
        if constexpr (BD) issue_b(std::true_type{}, slot_tag, st);
    };
    auto wait_landed = [&](int s) {
        const int later = min(n_st - 1 - s, kDmaDepth - 1);
        if (diag) wait_vmcnt_runtime<CPT, kDmaDepth>(later);
        else wait_vmcnt_runtime<CPT + CPT_B, kDmaDepth>(later);
    };
    auto wait_landed_bd = [&](auto later_tag) { wait_vmcnt<(CPT + NBO) * decltype(later_tag)::value>(); };
    auto buf_a = [&](int st) -> const char* { return lds_raw + (st % NB) * BUF; };
    auto buf_b = [&](int st) -> const char* { return lds_raw + (st % NB) * BUF + (diag ? 0 : PANEL); };

    // this stage's operands: rows as read, columns as read and J-swapped;
    // each is replaced by the next stage's right after its last MFMA
    uint4 a_op[NA];
    V bv[NBO], bj[NBO];
    uint4 b_raw[NBO];                  // the next stage's columns as read (LDS-staged forms)
    auto read_b = [&](int st) {
#pragma unroll
        for (int x = 0; x < NBO; ++x) b_raw[x] = rd(buf_b(st), bn[x] * 16 + lc);
    };

    // stage st in ring slot R; kMask: the stage is in the final group (its
    // wait counts are those of the last stages); kMaskNext: the operands it
    // loads for stage st + 1 may hold blocks at or past the partial one
    auto run_stage = [&](auto r_tag, int st, auto has_next_tag, auto mask_tag, auto mask_next_tag, auto clamp_tag) {
        constexpr int R = decltype(r_tag)::value;
        constexpr int RN = (R + 1) % RS;
        constexpr bool kNext = decltype(has_next_tag)::value;
        constexpr bool kMask = decltype(mask_tag)::value;
        constexpr bool kMaskNext = decltype(mask_next_tag)::value;
        static_for<NP>([&](auto p_tag) {
            constexpr int p = decltype(p_tag)::value;
            constexpr int ia = J::T.IA[p], ib = J::T.IB[p];
            const V av = cvt(a_op[ia]);
            op(accR[p], av, bv[ib]);
            op(accI[p], av, bj[ib]);
            __builtin_amdgcn_sched_barrier(0);
            if constexpr (kNext && p == 0) {
                // stage st + 1 has landed for every wave, and every wave has
                // finished stage st - 1, whose buffer the next DMA refills
                if constexpr (BD) {
                    // (clamped: the count is formed even where the branch
                    // is discarded, on the last stage)
                    constexpr int later = kMask ? (RS - 2 - R > 0 ? RS - 2 - R : 0) : kDmaDepth - 1;
                    wait_landed_bd(std::integral_constant<int, later>{});
                    dma_barrier();
                    if constexpr (!kMask) issue_a(clamp_tag, st + 1 + kDmaDepth);
                } else {
                    wait_landed(st + 1);
                    dma_barrier();
                    // (with a ring of one stage the main loop also issues the
                    // last stages, so the offsets are always checked)
                    if (st + 1 + kDmaDepth < n_st) issue_a(std::true_type{}, st + 1 + kDmaDepth);
                    read_b(st + 1);
                }
                __builtin_amdgcn_sched_barrier(0);
            }
            if constexpr (kNext && last_use<J>(ia) == p) {
                a_op[ia] = rd(buf_a(st + 1), am[ia] * 16 + lc);
                if constexpr (kMaskNext) mask_op(st + 1, a_op[ia]);
                __builtin_amdgcn_sched_barrier(0);
            }
            if constexpr (kNext && last_use_b<J>(ib) == p) {
                uint4 u;
                if constexpr (BD) u = bdir[RN][ib];
                else u = b_raw[ib];
                if constexpr (kMaskNext) mask_op(st + 1, u);
                bv[ib] = cvt(u);
                bj[ib] = jsw(u);
                __builtin_amdgcn_sched_barrier(0);
            }
            // the column loads of stage st + 1 + kDmaDepth go into this
            // stage's ring slot once its last MFMA is issued, so that the
            // operands can be used from the slot itself
            if constexpr (BD && kNext && !kMask && p == NP - 1) {
                issue_b(clamp_tag, r_tag, st + 1 + kDmaDepth);
                __builtin_amdgcn_sched_barrier(0);
            }
        });
    };
    __builtin_amdgcn_s_waitcnt(0xC07F);
    static_for<kDmaDepth>([&](auto d) {
        if (BD || d < n_st) issue(std::integral_constant<int, decltype(d)::value % RS>{}, d);
    });
    if constexpr (BD) wait_landed_bd(std::integral_constant<int, kDmaDepth - 1>{});
    else wait_landed(0);
    dma_barrier();
    if (BD || kDmaDepth < n_st) issue(std::integral_constant<int, kDmaDepth % RS>{}, kDmaDepth);
#pragma unroll
    for (int i = 0; i < NA; ++i) {
        a_op[i] = rd(buf_a(0), am[i] * 16 + lc);
        if (n_final == 0) mask_op(0, a_op[i]);
    }
    if constexpr (!BD) read_b(0);
#pragma unroll
    for (int x = 0; x < NBO; ++x) {
        uint4 u;
        if constexpr (BD) u = bdir[0][x];
        else u = b_raw[x];
        if (n_final == 0) mask_op(0, u);
        bv[x] = cvt(u);
        bj[x] = jsw(u);
    }
    // main loop, then the group that ends with the stage loading the first
    // stage of the final group (all stages before the final group hold whole
    // blocks), then the final group
    for (int st = 0; st < n_final - RS; st += RS)
        static_for<RS>([&](auto r) {
            run_stage(r, st + r, std::true_type{}, std::false_type{}, std::false_type{}, std::false_type{});
        });
    if (n_final >= RS)
        static_for<RS>([&](auto r) {
            run_stage(r, n_final - RS + r, std::true_type{}, std::false_type{},
                      std::integral_constant<bool, (decltype(r)::value + 1 == RS)>{}, std::true_type{});
        });
    static_for<RS>([&](auto r) {
        run_stage(r, n_final + r, std::integral_constant<bool, (decltype(r)::value + 1 < RS)>{}, std::true_type{},
                  std::true_type{}, std::true_type{});
    });
    lds_barrier();

    // ---- epilogue: 2 x 2 polarisation blocks of antennas a >= b.  Rows
    // 4 (lane / 16) + {0, 1} and {2, 3} of a lane are the two polarisations
    // of two antennas, lanes lc, lc ^ 1 the two of one antenna b: a lane pair
    // holds the four values of a baseline, swaps one value so that the even
    // lane owns (p, q) = (0, 0), (0, 1) and the odd lane (1, 0), (1, 1), and
    // each lane stores 16 contiguous bytes.
    using E = std::conditional_t<DT == AFC_I8, int, float>;
    const bool odd = (lc & 1) != 0;
    // rows I, I + 1 (the two polarisations of antenna I / 2) of receiver Jc
    auto store_pair = [&](E r0, E i0v, E r1, E i1v, int I, int Jc, bool flagged) {
        // the even lane sends its p = 1 values, the odd lane its p = 0 values
        const E yr = pair_swap(odd ? r0 : r1), yi = pair_swap(odd ? i0v : i1v);
        E o0 = odd ? yr : r0, o1 = odd ? yi : i0v, o2 = odd ? r1 : yr, o3 = odd ? i1v : yi;
        const int a = I >> 1, b = Jc >> 1;
        if (Jc >= N || I >= N || a < b) return;
        if (a == b) {             // inputs equal for (0, 0) and (1, 1)
            if (odd) o3 = E(0);
            else o1 = E(0);
        }
        if (flagged) o0 = o1 = o2 = o3 = E(0);
        const int64_t bl = (int64_t)a * (a + 1) / 2 + b;
        // written once and not read again by this kernel: a streaming
        // (non-temporal) store
        typedef E ev4 __attribute__((ext_vector_type(4)));
        __builtin_nontemporal_store(ev4{o0, o1, o2, o3}, reinterpret_cast<ev4*>(vis_ch) + bl * 2 + (odd ? 1 : 0));
        if (write_weights && !odd) w_sb[bl] = flagged ? 0 : S;
    };
    auto flag_of = [&](int rcv) { return fl_sb[min(rcv, N - 1) >> 1] != 0; };
    auto to_u = [](E v) -> unsigned {
        if constexpr (DT == AFC_I8) return (unsigned)v;
        else return __float_as_uint(v);
    };
    auto from_u = [](unsigned u) -> E {
        if constexpr (DT == AFC_I8) return (int)u;
        else return __uint_as_float(u);
    };
    if constexpr (std::is_same_v<J, Job16R8C2>) {
        // Off the diagonal the wave's two column blocks are 16 consecutive
        // antennas.  One permlane16 swap per value pair gives the lanes of
        // rows 0 and 2 (of 16 lanes) column block 0 and the lanes of rows 1
        // and 3 column block 1, each for the rows of both, so that a store
        // instruction writes two runs of 16 whole baselines (512 bytes)
        // instead of four runs of 8.
        const int cbk = lg & 1, gb = lg & 2;
        const int Jc = j0 + bn[cbk] * 16 + lc;
        // [rows 4 gb + r, rows 4 (gb + 1) + r][r] of the two column blocks'
        // row block i
        auto swap_rows = [&](int i, E (&hr)[2][4], E (&hi)[2][4]) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                // (elements into scalars first: a bit cast of a vector element
                // passed straight to the builtin read element 0 for every r)
                const E xr = accR[2 * i][r], yr = accR[2 * i + 1][r];
                const E xi = accI[2 * i][r], yi = accI[2 * i + 1][r];
                const auto sr = __builtin_amdgcn_permlane16_swap(to_u(xr), to_u(yr), false, false);
                const auto si = __builtin_amdgcn_permlane16_swap(to_u(xi), to_u(yi), false, false);
                hr[0][r] = from_u(sr[0]);
                hr[1][r] = from_u(sr[1]);
                hi[0][r] = from_u(si[0]);
                hi[1][r] = from_u(si[1]);
            }
        };
        if (!write_weights && i0 + TILE <= N) {
            // Interior tile that writes no weights (uniform): every baseline
            // of it exists (a > b, all rows and columns below N), so the
            // stores need no checks, and flagged baselines are zeroed by
            // selection.  The lane's row antennas are a0 + k,
            // k = 8 i + 2 h + r / 2, and bl(a0 + k, b) - bl(a0, b) =
            // k a0 + k (k + 1) / 2, so each store's offset is one multiply-add
            // on the lane's base (32-bit: a channel's visibilities are below
            // 2^31 bytes at the antenna limit).
            const int a0 = (i0 >> 1) + 2 * gb, b = Jc >> 1;
            const int nbl = Na * (Na + 1) / 2;
            const unsigned vbase = (unsigned)(a0 * (a0 + 1) / 2 + b) * 32u + (odd ? 16u : 0u);
            const unsigned a32 = (unsigned)a0 * 32u;
#if defined(__HIP_DEVICE_COMPILE__)
            const __amdgpu_buffer_rsrc_t rs =
                __builtin_amdgcn_make_buffer_rsrc((void*)vis_ch, (short)0, nbl * 32, 0x00020000);
#endif
            // the lane's flags, all loaded before the first store (stores and
            // loads share the wave's memory counter, so a flag load waited for
            // between stores would also wait for every store before it)
            bool fz[8][2][2] = {};
            if (fl_sb) {
                const bool fc = flag_of(Jc);
#pragma unroll
                for (int i = 0; i < 8; ++i)
#pragma unroll
                    for (int h = 0; h < 2; ++h)
#pragma unroll
                        for (int k = 0; k < 2; ++k) fz[i][h][k] = fc || flag_of(i0 + am[i] * 16 + 4 * (gb + h) + 2 * k);
            }
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                E hr[2][4], hi[2][4];
                swap_rows(i, hr, hi);
#pragma unroll
                for (int h = 0; h < 2; ++h)
#pragma unroll
                    for (int r = 0; r < 4; r += 2) {
                        // the even lane keeps (p, q) = (0, 0), (0, 1), the odd
                        // lane (1, 0), (1, 1), as in store_pair
                        const E r0 = hr[h][r], i0v = hi[h][r], r1 = hr[h][r + 1], i1v = hi[h][r + 1];
                        const E yr = pair_swap(odd ? r0 : r1), yi = pair_swap(odd ? i0v : i1v);
                        v4i o{(int)to_u(odd ? yr : r0), (int)to_u(odd ? yi : i0v), (int)to_u(odd ? r1 : yr),
                              (int)to_u(odd ? i1v : yi)};
                        if (fz[i][h][r >> 1]) o = v4i{0, 0, 0, 0};
                        const int k = 8 * am[i] + 2 * h + r / 2;
                        const unsigned voff = vbase + (unsigned)k * a32 + (unsigned)(k * (k + 1) / 2) * 32u;
#if defined(__HIP_DEVICE_COMPILE__)
                        // non-temporal (cache policy bit 1), as the checked stores
                        __builtin_amdgcn_raw_buffer_store_b128(o, rs, (int)voff, 0, 2);
#else
                        (void)o;
                        (void)voff;
#endif
                    }
            }
        } else {
            const bool fc = fl_sb ? flag_of(Jc) : false;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                bool fr[2][2] = {{false, false}, {false, false}};
                if (fl_sb) {
#pragma unroll
                    for (int h = 0; h < 2; ++h)
#pragma unroll
                        for (int k = 0; k < 2; ++k) fr[h][k] = flag_of(i0 + am[i] * 16 + 4 * (gb + h) + 2 * k);
                }
                E hr[2][4], hi[2][4];
                swap_rows(i, hr, hi);
#pragma unroll
                for (int h = 0; h < 2; ++h)
#pragma unroll
                    for (int r = 0; r < 4; r += 2)
                        store_pair(hr[h][r], hi[h][r], hr[h][r + 1], hi[h][r + 1], i0 + am[i] * 16 + 4 * (gb + h) + r,
                                   Jc, fc || fr[h][r >> 1]);
            }
        }
    } else {
        bool frow[NA][2], fcol[NBO];
#pragma unroll
        for (int x = 0; x < NBO; ++x) fcol[x] = fl_sb ? flag_of(j0 + bn[x] * 16 + lc) : false;
#pragma unroll
        for (int i = 0; i < NA; ++i)
#pragma unroll
            for (int k = 0; k < 2; ++k) frow[i][k] = fl_sb ? flag_of(i0 + am[i] * 16 + 4 * lg + 2 * k) : false;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const int ia = J::T.IA[p], ib = J::T.IB[p];
#pragma unroll
            for (int r = 0; r < 4; r += 2)
                store_pair(accR[p][r], accI[p][r], accR[p][r + 1], accI[p][r + 1], i0 + am[ia] * 16 + 4 * lg + r,
                           j0 + bn[ib] * 16 + lc, fcol[ib] || frow[ia][r >> 1]);
        }
    }
}

// One fp32 tile of one (subband, channel): 2 x 2 waves of one 32 x 32 block
// each, samples staged through registers.  `z` points at channel ch of
// subband sb.
template <int DT, int TILE>
__device__ __forceinline__ void xtile_f32(const char* __restrict__ z, char* __restrict__ vis_ch,
                                      int32_t* __restrict__ w_sb, const uint8_t* __restrict__ fl_sb,
                                      int N, int Na, int S, int ti, int tj, bool write_weights,
                                      char* lds_raw) {
    using Tr = XT<DT>;
    constexpr int RB = Tr::RB, PLANES = Tr::PLANES, kStg = stage_blocks<DT, TILE>();
    constexpr int WT = TILE / 2, MB = WT / 32;
    constexpr int PANEL = kStg * TILE * RB;                  // bytes of one panel in one stage
    constexpr int CHUNKS = kStg * TILE * PLANES;             // 16-byte chunks per panel per stage
    constexpr int CPT = CHUNKS / kThreads;
    static_assert(CHUNKS % kThreads == 0, "a stage must split evenly over the threads");
    static_assert(DT == AFC_F32, "fp32 only");
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
            {
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

    {
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
#pragma unroll
    for (int m = 0; m < MB; ++m)
#pragma unroll
        for (int n = 0; n < MB; ++n) {
            accR[m][n] += outR[m][n];
            accI[m][n] += outI[m][n];
        }
    if (!wave_on) return;

    // ---- epilogue: 2x2 polarisation blocks of antennas a >= b
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
                float re = accR[m][n][r], im = accI[m][n][r];
                if (I == J) im = 0.0f;
                if (flagged) re = im = 0.0f;
                reinterpret_cast<float2*>(vis_ch)[e] = make_float2(re, im);
                if (write_weights && p == 0 && qq == 0) w_sb[bl] = flagged ? 0 : S;
            }
        }
}

// One tile of one (subband, channel).  int8 / fp16: each wave computes its
// job of 16 x 16 blocks (diagonal tiles spread their lower-triangle blocks
// over the waves); fp32: 2 x 2 waves of one 32 x 32 block each.
template <int DT, int TILE>
__device__ __forceinline__ void xtile(const char* __restrict__ z, char* __restrict__ vis_ch,
                                      int32_t* __restrict__ w_sb, const uint8_t* __restrict__ fl_sb,
                                      int N, int Na, int S, int ti, int tj, bool write_weights, char* lds_raw) {
    if constexpr (DT == AFC_F32) {
        xtile_f32<DT, TILE>(z, vis_ch, w_sb, fl_sb, N, Na, S, ti, tj, write_weights, lds_raw);
    } else {
        const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
        auto run = [&](auto job, const int (&am)[8], const int (&bn)[2]) {
            xtile_mm16<DT, TILE, decltype(job)>(z, vis_ch, w_sb, fl_sb, N, Na, S, ti, tj, write_weights, lds_raw,
                                                am, bn);
        };
        if constexpr (TILE == 128) {
            if (ti != tj) {
                const int am[8] = {0, 1, 2, 3, 4, 5, 6, 7}, bn[2] = {2 * wid, 2 * wid + 1};
                run(Job16R8C2{}, am, bn);
            } else if (wid == 0) {
                run(Job16D8<0>{}, Job16D8<0>::T.AM, Job16D8<0>::T.BN);
            } else if (wid == 1) {
                run(Job16D8<1>{}, Job16D8<1>::T.AM, Job16D8<1>::T.BN);
            } else if (wid == 2) {
                run(Job16D8<2>{}, Job16D8<2>::T.AM, Job16D8<2>::T.BN);
            } else {
                run(Job16D8<3>{}, Job16D8<3>::T.AM, Job16D8<3>::T.BN);
            }
        } else {
            static_assert(TILE == 64, "int8 / fp16 tiles are 128 or 64 wide");
            if (ti != tj) {
                const int am[8] = {0, 1, 2, 3, 0, 0, 0, 0}, bn[2] = {wid, 0};
                run(Job16R4C1{}, am, bn);
            } else if (wid == 0) {
                run(Job16D4<0>{}, Job16D4<0>::T.AM, Job16D4<0>::T.BN);
            } else if (wid == 1) {
                run(Job16D4<1>{}, Job16D4<1>::T.AM, Job16D4<1>::T.BN);
            } else if (wid == 2) {
                run(Job16D4<2>{}, Job16D4<2>::T.AM, Job16D4<2>::T.BN);
            } else {
                run(Job16D4<3>{}, Job16D4<3>::T.AM, Job16D4<3>::T.BN);
            }
        }
    }
}

template <int DT, int TILE>
__global__ __launch_bounds__(kThreads, 2) void xengine_kernel(XArgs a) {
    __shared__ __attribute__((aligned(16))) char lds[lds_bytes<DT, TILE>()];
    // XCD-aware order: consecutive workgroup ids go round-robin over the 8
    // XCDs; give each XCD a contiguous range of work so that the tiles of one
    // channel share that XCD's L2.  (One tile per workgroup: the hardware
    // dispatcher then keeps the tiles in flight on an XCD a contiguous
    // window, which a static persistent schedule does not.)
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

// Batched form: one workgroup per work item of a host-built list; each item
// is one tile of one channel of one subband with its own sample type and
// integration length.  MODE 0 serves int8 and fp16 subbands (mixed in one
// launch) with TILE-wide tiles, MODE 1 fp32 subbands (64).  Workgroup ids go
// round-robin over the 8 XCDs and the list holds each XCD's items (whole
// channels, cost-balanced across XCDs) contiguously, so that the hardware
// dispatcher keeps the tiles in flight on an XCD a window of few channels.
template <int MODE, int TILE, int WPC>
__global__ __launch_bounds__(kThreads, WPC) void xengine_list_kernel(
    const char* __restrict__ z_ws, char* __restrict__ vis, int32_t* __restrict__ weights,
    const uint8_t* __restrict__ flags, const XSubband* __restrict__ sbs, const XWork* __restrict__ work,
    XcdRanges r, int N, int Na) {
    constexpr int kLds = MODE == 0 ? (lds_bytes<AFC_I8, TILE>() > lds_bytes<AFC_F16, TILE>() ? lds_bytes<AFC_I8, TILE>()
                                                                                            : lds_bytes<AFC_F16, TILE>())
                                   : lds_bytes<AFC_F32, TILE>();
    __shared__ __attribute__((aligned(16))) char lds[kLds];
    const int x = blockIdx.x & 7, k = blockIdx.x >> 3;
    if (k >= r.count[x]) return;
    const int64_t nbl = (int64_t)Na * (Na + 1) / 2;
    const XWork wk = work[r.begin[x] + k];
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
}

}  // namespace

namespace {
__global__ void fill_scratch_kernel(uint32_t* p, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        uint32_t h = (uint32_t)i * 0x9E3779B9u ^ (uint32_t)(i >> 32);
        h ^= h >> 16;
        h *= 0x85EBCA6Bu;
        h ^= h >> 13;
        h *= 0xC2B2AE35u;
        h ^= h >> 16;
        p[i] = h & 0xBFBFBFBFu;
    }
}
}  // namespace

hipError_t launch_fill_scratch(void* p, size_t bytes, hipStream_t stream) {
    const size_t n = bytes / 4;
    if (n == 0) return hipSuccess;
    const unsigned grid = (unsigned)std::min<size_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(fill_scratch_kernel, dim3(grid), dim3(256), 0, stream, reinterpret_cast<uint32_t*>(p), n);
    return hipGetLastError();
}

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

int xengine_list_grid(const XcdRanges& r) {
    int mx = 0;
    for (int x = 0; x < 8; ++x) mx = std::max(mx, (int)r.count[x]);
    return mx * 8;
}

hipError_t launch_xengine_list(const void* z_ws, void* vis, int32_t* weights, const uint8_t* flags,
                               const XSubband* sbs_dev, const XWork* work_dev, const XcdRanges& ranges, int N,
                               int Na, int mode, int tile, hipStream_t stream) {
    const char* z = reinterpret_cast<const char*>(z_ws);
    char* v = reinterpret_cast<char*>(vis);
    const int g = xengine_list_grid(ranges);
    if (g == 0) return hipSuccess;
    const dim3 grid((unsigned)g), block(kThreads);
    if (mode == 1)  // fp32 subbands
        hipLaunchKernelGGL((xengine_list_kernel<1, 64, 2>), grid, block, 0, stream, z, v, weights, flags, sbs_dev,
                           work_dev, ranges, N, Na);
    else if (tile == 128)
        hipLaunchKernelGGL((xengine_list_kernel<0, 128, 2>), grid, block, 0, stream, z, v, weights, flags, sbs_dev,
                           work_dev, ranges, N, Na);
    else
        hipLaunchKernelGGL((xengine_list_kernel<0, 64, 4>), grid, block, 0, stream, z, v, weights, flags, sbs_dev,
                           work_dev, ranges, N, Na);
    return hipGetLastError();
}

}  // namespace afc
