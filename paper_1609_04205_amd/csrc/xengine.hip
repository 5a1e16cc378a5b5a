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
// one subband, 4 waves, outputs in 32 x 32 MFMA blocks.  128-wide int8 /
// fp16 tiles: off the diagonal wave w owns column block w against the four
// row blocks; a diagonal tile spreads its ten lower-triangle blocks 3/3/2/2
// over the waves.  64-wide tiles and fp32: 2 x 2 waves of one quarter each,
// the wave above the diagonal idle on a diagonal tile.  Tiles wholly above
// the diagonal are never launched.
// int8 / fp16: the row panel of a tile streams through LDS in stages of 2-4
// spectrum blocks (direct global-to-LDS loads of the block layout
// [block][receiver][8 spectra], XOR-swizzled 16-byte chunks so that the MFMA
// operand reads are bank-conflict free); off the diagonal each wave loads
// its own column block straight into registers.  fp32 stages both panels
// through registers into LDS.
//
// Sample types (gfx950 MFMA):
//   int8  v_mfma_i32_32x32x32_i8  (16 spectra per K-step), exact int32 sums
//   fp16  v_mfma_f32_32x32x16_f16 ( 8 spectra per K-step), fp32 sums
//   fp32  v_mfma_f32_32x32x2_f32  ( 2 spectra per K-step), fp32 sums, summed
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
// spectrum blocks per LDS stage
#ifndef AFC_I8_STAGE_BLOCKS
#define AFC_I8_STAGE_BLOCKS 4
#endif
#ifndef AFC_F16_STAGE_BLOCKS
#define AFC_F16_STAGE_BLOCKS 2
#endif
template <int DT, int TILE>
constexpr int stage_blocks() {
    return DT == AFC_F32 ? 4 : TILE != 128 ? (DT == AFC_I8 ? 4 : 2)
                                           : DT == AFC_I8 ? AFC_I8_STAGE_BLOCKS : AFC_F16_STAGE_BLOCKS;
}
// fp32: stages of register-staged loads in flight
template <int DT, int TILE>
constexpr int prefetch_depth() { return 2; }
// int8 and fp16 stage through direct global-to-LDS loads, fp32 through registers
template <int DT>
constexpr bool uses_dma() { return DT != AFC_F32; }
#ifndef AFC_DMA_DEPTH
#define AFC_DMA_DEPTH 3
#endif
constexpr int kDmaDepth = AFC_DMA_DEPTH;      // stages of global-to-LDS loads in flight
#ifndef AFC_XENGINE_BDIRECT
#define AFC_XENGINE_BDIRECT 1
#endif
// off-diagonal square tiles load their B operands into registers (1) or
// stage them through LDS with the A panel (0)
constexpr bool kBDirect = AFC_XENGINE_BDIRECT != 0;
// DMA ring: the stage being multiplied, the next one (already landed when
// its first operands are read) and kDmaDepth - 1 further stages in flight,
// plus the buffer being refilled
constexpr int kDmaBuffers = kDmaDepth + 2;
template <int DT, int TILE>
constexpr int lds_bytes() {
    // 128-wide int8 / fp16 tiles stage only the row panel (their column
    // operands are loaded into registers, or, on the diagonal, are the row
    // panel); the others stage both
    constexpr int panels = uses_dma<DT>() && TILE == 128 && kBDirect ? 1 : 2;
    return (uses_dma<DT>() ? kDmaBuffers : 2) * panels * stage_blocks<DT, TILE>() * TILE * XT<DT>::RB;
}

// Workgroup barrier for the DMA pipeline: no memory fence (which would wait
// for every outstanding global-to-LDS load); a compiler-level memory clobber
// keeps LDS accesses on their side of it.
__device__ __forceinline__ void dma_barrier() {
    __asm__ volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
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

// Work of one wave in an int8 / fp16 tile: NP blocks of 32 x 32 outputs,
// block p pairing row block am[IA[p]] of panel A with column block
// bn[IB[p]] of panel B (am, bn hold NA and NB block indices).
struct JobRows4 {      // off-diagonal 128-tile: every row block x this wave's column block
    static constexpr int NA = 4, NB = 1, NP = 4;
    static constexpr int IA[8] = {0, 1, 2, 3}, IB[8] = {0, 0, 0, 0};
};
// diagonal 128-tile: its ten lower-triangle blocks (m >= n) split 3/3/2/2
struct JobDiag0 {      // (0,0) (1,0) (2,0)
    static constexpr int NA = 3, NB = 1, NP = 3;
    static constexpr int IA[8] = {0, 1, 2, 0}, IB[8] = {0, 0, 0, 0};
    static constexpr int AM[4] = {0, 1, 2, 0}, BN[2] = {0, 0};
};
struct JobDiag1 {      // (3,0) (1,1) (2,1)
    static constexpr int NA = 3, NB = 2, NP = 3;
    static constexpr int IA[8] = {0, 1, 2, 0}, IB[8] = {0, 1, 1, 0};
    static constexpr int AM[4] = {3, 1, 2, 0}, BN[2] = {0, 1};
};
struct JobDiag2 {      // (3,1) (2,2)
    static constexpr int NA = 2, NB = 2, NP = 2;
    static constexpr int IA[8] = {0, 1, 0, 0}, IB[8] = {0, 1, 0, 0};
    static constexpr int AM[4] = {3, 2, 0, 0}, BN[2] = {1, 2};
};
struct JobDiag3 {      // (3,2) (3,3)
    static constexpr int NA = 1, NB = 2, NP = 2;
    static constexpr int IA[8] = {0, 0, 0, 0}, IB[8] = {0, 1, 0, 0};
    static constexpr int AM[4] = {3, 0, 0, 0}, BN[2] = {2, 3};
};
struct JobOne {        // 64-tile: one block per wave
    static constexpr int NA = 1, NB = 1, NP = 1;
    static constexpr int IA[8] = {0, 0, 0, 0}, IB[8] = {0, 0, 0, 0};
};
struct JobIdle {       // 64-tile, the wave above the diagonal
    static constexpr int NA = 1, NB = 1, NP = 0;
    static constexpr int IA[8] = {0, 0, 0, 0}, IB[8] = {0, 0, 0, 0};
};

// One int8 / fp16 tile of one (subband, channel) for one wave's job.  All
// waves of the workgroup stage the panels together; `z` points at channel ch
// of subband sb.
//
// The row panel A is TILE receivers tall (rows ti*TILE ..), the column panel B
// as wide (columns tj*TILE ..).  A stage buffer holds A then B; a diagonal
// tile (ti == tj) stages A only and reads both operands from it.
template <int DT, int TILE, class J>
__device__ __forceinline__ void xtile_mm(const char* __restrict__ z, char* __restrict__ vis_ch,
                                         int32_t* __restrict__ w_sb, const uint8_t* __restrict__ fl_sb,
                                         int N, int Na, int S, int ti, int tj, bool write_weights,
                                         char* lds_raw, const int (&am)[4], const int (&bn)[2]) {
    using Tr = XT<DT>;
    using acc_t = typename Tr::acc_t;
    using V = std::conditional_t<DT == AFC_I8, v4i, v8h>;
    constexpr int RB = Tr::RB, PLANES = Tr::PLANES, kStg = stage_blocks<DT, TILE>();
    constexpr int PANEL = kStg * TILE * RB;                  // bytes of panel A in one stage
    constexpr int PANEL_B = PANEL;                           // bytes of panel B in one stage
    constexpr int CPT = kStg * TILE * PLANES / kThreads;     // 16-byte chunks of A per thread per stage
    constexpr int CPT_B = CPT;                               // of B
    static_assert((kStg * TILE * PLANES) % kThreads == 0, "a stage must split evenly over the threads");
    // k-steps per stage (int8: 16 spectra, fp16: 8 spectra each)
    constexpr int NKK = DT == AFC_I8 ? kStg / 2 : kStg;
    static_assert(NKK % 2 == 0, "k-steps per stage must be even");
    constexpr int NA = J::NA, NBO = J::NB, NP = J::NP;
    constexpr int NB = kDmaBuffers;
    // a stage buffer holds panel A and, where it is staged, panel B (not for
    // the diagonal jobs, whose operands all come from panel A, nor for the
    // direct-B form)
    constexpr bool kDiagJob = std::is_same_v<J, JobDiag0> || std::is_same_v<J, JobDiag1> ||
                              std::is_same_v<J, JobDiag2> || std::is_same_v<J, JobDiag3>;
    // Off-diagonal square tiles take their B operands straight from global
    // memory into registers: wave w alone uses column block w, so staging it
    // through LDS bought no sharing and cost an LDS write and read per byte.
    // The loads of a stage go out with that stage's A panel and land in a
    // ring of RS register slots (the stage in use and kDmaDepth in flight).
    constexpr bool BD = kBDirect && std::is_same_v<J, JobRows4>;
    constexpr int RS = BD ? kDmaDepth + 1 : 1;
    static_assert(RS <= 4, "register ring of at most four stages");
    constexpr int BUF = PANEL + (BD || kDiagJob ? 0 : PANEL_B);   // bytes of one stage buffer

    const int tid = threadIdx.x, lane = tid & 63, lr = lane & 31, lh = lane >> 5;
    const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int i0 = ti * TILE, j0 = tj * TILE;
    const bool diag = ti == tj;
    const int nb = (S + kSBlk - 1) / kSBlk;
    const int tail_valid = S - (nb - 1) * kSBlk;             // spectra in the last block
    // stages, rounded up to a multiple of the register ring (the extra
    // stages read the last block again and are masked to zero)
    const int n_st = (nb + kStg * RS - 1) / (kStg * RS) * RS;
    const int n_final = n_st - RS;                           // first stage of the final group

    acc_t accR[NP > 0 ? NP : 1], accI[NP > 0 ? NP : 1];
#pragma unroll
    for (int p = 0; p < (NP > 0 ? NP : 1); ++p) {
        accR[p] = acc_t{};
        accI[p] = acc_t{};
    }

    // a panel of `rows` receivers holds block bl at bl * rows * RB
    auto rd = [&](const char* panel, int rows, int bl, int row, int q) -> uint4 {
        return *reinterpret_cast<const uint4*>(panel + bl * rows * RB + row * RB + ((q ^ swz<RB, PLANES>(row)) * 16));
    };
    // this wave's operands of k-step kk (unconditional, so that the LDS
    // wait counts stay exact across branches); a diagonal tile's B operands
    // come from panel A
    // B operands loaded directly: [ring slot][k-step of the stage]
    uint4 bdir[RS][BD ? NKK : 1];
    auto load_ops = [&](auto slot_tag, const char* PA, const char* PB, int kk, uint4 (&oa)[NA], uint4 (&ob)[NBO]) {
        constexpr int slot = decltype(slot_tag)::value;
        const int bl = DT == AFC_I8 ? 2 * kk + lh : kk;
        const int q = DT == AFC_I8 ? 0 : lh;
#pragma unroll
        for (int i = 0; i < NA; ++i) oa[i] = rd(PA, TILE, bl, am[i] * 32 + lr, q);
        if constexpr (BD) {
            ob[0] = bdir[slot][kk];
        } else {
#pragma unroll
            for (int i = 0; i < NBO; ++i) ob[i] = rd(PB, TILE, bl, bn[i] * 32 + lr, q);
        }
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
        if constexpr (DT == AFC_I8) acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(x, y, acc, 0, 0, 0);
        else acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(x, y, acc, 0, 0, 0);
    };
    // MFMAs of one k-step.  `mid` runs after the first block's two MFMAs
    // have been issued (the scheduler may not move work across it): loads
    // of the next operands issued there overlap the remaining MFMAs.
    // MFMAs of one k-step from A operands oa and the prepared B operands
    // (bv as loaded, bj J-swapped).  `mid1` runs after the first block's two
    // MFMAs have been issued (it issues the next k-step's LDS reads), `mid2`
    // after about half of the blocks (it masks and J-swaps the next k-step's
    // B operands, whose reads have had those MFMAs to land), so that the
    // VALU work of the next k-step overlaps this one's MFMAs instead of
    // standing between two k-steps.  The scheduler may not move work across
    // the fences.
    constexpr int SPLIT = NP >= 4 ? NP / 2 + 1 : (NP > 1 ? NP - 1 : 1);
    auto mma = [&](const uint4 (&oa)[NA], const V (&bv)[NBO], const V (&bj)[NBO], auto&& mid1, auto&& mid2) {
        if constexpr (NP > 0) {
            const V a0 = cvt(oa[J::IA[0]]);
            op(accR[0], a0, bv[J::IB[0]]);
            op(accI[0], a0, bj[J::IB[0]]);
        }
        __builtin_amdgcn_sched_barrier(0);
        mid1();
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int p = 1; p < SPLIT && p < NP; ++p) {
            const V a = cvt(oa[J::IA[p]]);
            op(accR[p], a, bv[J::IB[p]]);
            op(accI[p], a, bj[J::IB[p]]);
        }
        __builtin_amdgcn_sched_barrier(0);
        mid2();
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int p = SPLIT; p < NP; ++p) {
            const V a = cvt(oa[J::IA[p]]);
            op(accR[p], a, bv[J::IB[p]]);
            op(accI[p], a, bj[J::IB[p]]);
        }
        __builtin_amdgcn_sched_barrier(0);
    };
    // zero the spectra >= S of this lane's operands of k-step kk of stage st
    auto mask_tail_ops = [&](int st, int kk, uint4 (&a)[NA], uint4 (&b)[NBO]) {
        const int blk = st * kStg + (DT == AFC_I8 ? 2 * kk + lh : kk);
        const int q = DT == AFC_I8 ? 0 : lh;
        if (blk < nb - 1 || (blk == nb - 1 && tail_valid == kSBlk)) return;
        const int valid = blk == nb - 1 ? tail_valid : 0;
#pragma unroll
        for (int i = 0; i < NA; ++i) a[i] = mask_tail<DT>(a[i], q, valid);
#pragma unroll
        for (int i = 0; i < NBO; ++i) b[i] = mask_tail<DT>(b[i], q, valid);
    };

    // Samples go straight from global memory to LDS (buffer loads with the
    // LDS bit: lane L of a wave writes 16 bytes at M0 + 16 L) through a ring
    // of NB stage buffers.  Buffer rather than global loads: the compiler
    // must assume that global (flat) ones may also touch LDS and would then
    // wait for every LDS read at once.  Rows beyond N read row N-1 (they only
    // feed outputs that are never stored); in the last stage, blocks beyond
    // the data read the last block again, and the operands of the partial
    // last block are masked in registers.
    //
    // One barrier per stage st, placed before its last k-step: by then stage
    // st+1 has landed (each wave waits for its own loads first) and every
    // wave has finished stage st-1, so the loads of stage st+1+kDmaDepth
    // refill st-1's buffer, and the first operands of st+1 are read while the
    // last MFMAs of st run.  Operands are double-buffered one k-step ahead.
    //
    // Offsets within the channel: voffset = this thread's chunk in stage 0,
    // soffset = the stage (a channel of samples is far below 2 GiB: the entry
    // points bound one subband of input to 2^31 values).
    const int z_bytes = nb * N * RB;
    // source offset of chunk c of a panel of `rows` receivers starting at r0
    auto chunk_src = [&](int c, int rows, int r0) {
        const int chunk = tid + c * kThreads;
        const int bl = chunk / (rows * PLANES);
        const int rem = chunk % (rows * PLANES);
        const int row = rem / PLANES, sl = rem % PLANES;
        const int q = sl ^ swz<RB, PLANES>(row);
        return (bl * N + min(r0 + row, N - 1)) * RB + q * 16;
    };
    int src_a[CPT], src_b[CPT_B];
#pragma unroll
    for (int c = 0; c < CPT; ++c) src_a[c] = chunk_src(c, TILE, i0);
#pragma unroll
    for (int c = 0; c < CPT_B; ++c) src_b[c] = chunk_src(c, TILE, j0);
    const int stage_bytes = kStg * N * RB;
    auto issue_panel = [&](int st, char* panel, int c, int src, int rows) {
        char* dst = panel + (c * kThreads + wid * 64) * 16;
        const int bl = (tid + c * kThreads) / (rows * PLANES);
        if constexpr (BD) {           // branch-free: block clamped to nb - 1 in voffset
            buffer_load_lds16(z, z_bytes, dst, src + (min(st * kStg + bl, nb - 1) - bl) * N * RB, 0);
            return;
        }
        int voff = src, soff = st * stage_bytes;
        if ((st + 1) * kStg > nb) {   // past the end (uniform): whole offset in voffset, block clamped to nb - 1
            voff += (min(st * kStg + bl, nb - 1) - bl) * N * RB;
            soff = 0;
        }
        buffer_load_lds16(z, z_bytes, dst, voff, soff);
    };
    // this lane's B row and, per k-step of a stage, its block and chunk
    const int b_row = min(j0 + bn[0] * 32 + lr, N - 1);
    auto issue = [&](auto slot_tag, int st) {
        constexpr int slot = decltype(slot_tag)::value;
        char* buf = lds_raw + (st % NB) * BUF;
#pragma unroll
        for (int c = 0; c < CPT; ++c) issue_panel(st, buf, c, src_a[c], TILE);
        if constexpr (BD) {
            // no branch around these loads (the compiler's wait counts for
            // their registers stay exact): the block index is clamped to
            // nb - 1 arithmetically
#pragma unroll
            for (int kk = 0; kk < NKK; ++kk) {
                const int lbl = DT == AFC_I8 ? 2 * kk + lh : kk;
                const int q = DT == AFC_I8 ? 0 : lh;
                const int blk = min(st * kStg + lbl, nb - 1);
                bdir[slot][kk] = buffer_load16(z, z_bytes, (blk * N + b_row) * RB + q * 16, 0);
            }
        } else if (!diag) {
#pragma unroll
            for (int c = 0; c < CPT_B; ++c) issue_panel(st, buf + PANEL, c, src_b[c], TILE);
        }
    };
    // wait until this wave's loads of stage s have landed, given that the
    // stages up to min(s + kDmaDepth - 1, n_st - 1) have been issued
    auto wait_landed = [&](int s) {
        const int later = min(n_st - 1 - s, kDmaDepth - 1);
        if (diag) wait_vmcnt_runtime<CPT>(later);
        else wait_vmcnt_runtime<CPT + CPT_B>(later);
    };
    // the same for the direct-B form, where `later` is known at compile time
    auto wait_landed_bd = [&](auto later_tag) {
        wait_vmcnt<(CPT + NKK) * decltype(later_tag)::value>();
    };
    auto panels = [&](int st, const char*& PA, const char*& PB) {
        const char* buf = lds_raw + (st % NB) * BUF;
        PA = buf;
        PB = diag ? buf : buf + PANEL;
    };
    // operand set kk & 1 holds k-step kk of the current stage; the last
    // stage is peeled off so that the loop body has no branch around LDS
    // reads and the compiler's LDS wait counts stay exact
    uint4 oa[2][NA], ob[2][NBO];
    V bv[2][NBO], bj[2][NBO];
    // B operands of slot `slot` as MFMA values: as loaded and J-swapped
    auto prep = [&](uint4 (&b)[NBO], V (&v)[NBO], V (&j)[NBO]) {
#pragma unroll
        for (int i = 0; i < NBO; ++i) {
            v[i] = cvt(b[i]);
            j[i] = jsw(b[i]);
        }
    };
    // stage st (using register slot R of the direct B ring); the stages of
    // the final group mask the operands of blocks at or past the partial one
    auto run_stage = [&](auto r_tag, int st, auto has_next_tag, auto mask_tag) {
        constexpr int R = decltype(r_tag)::value;
        constexpr int RN = (R + 1) % RS;                     // slot of stage st + 1
        constexpr bool kNext = decltype(has_next_tag)::value;
        constexpr bool kMask = decltype(mask_tag)::value;
        const char *PA, *PB;
        panels(st, PA, PB);
#pragma unroll
        for (int kk = 0; kk + 1 < NKK; ++kk) {
            mma(oa[kk & 1], bv[kk & 1], bj[kk & 1],
                [&] { load_ops(r_tag, PA, PB, kk + 1, oa[(kk + 1) & 1], ob[(kk + 1) & 1]); },
                [&] {
                    if constexpr (kMask) mask_tail_ops(st, kk + 1, oa[(kk + 1) & 1], ob[(kk + 1) & 1]);
                    prep(ob[(kk + 1) & 1], bv[(kk + 1) & 1], bj[(kk + 1) & 1]);
                });
        }
        mma(oa[(NKK - 1) & 1], bv[(NKK - 1) & 1], bj[(NKK - 1) & 1],
            [&] {
                if constexpr (kNext) {
                    if constexpr (BD) {
                        // stages issued after st + 1: kDmaDepth - 1 before
                        // the final group, RS - 2 - R inside it
                        wait_landed_bd(std::integral_constant<int, kMask ? RS - 2 - R : kDmaDepth - 1>{});
                        dma_barrier();
                        // stage st + 1 + kDmaDepth reuses this stage's slot
                        // R; it exists exactly for the stages before the
                        // final group
                        if constexpr (!kMask) issue(r_tag, st + 1 + kDmaDepth);
                    } else {
                        wait_landed(st + 1);
                        dma_barrier();
                        if (st + 1 + kDmaDepth < n_st) issue(r_tag, st + 1 + kDmaDepth);
                    }
                    const char *NA_, *NB_;
                    panels(st + 1, NA_, NB_);
                    load_ops(std::integral_constant<int, RN>{}, NA_, NB_, 0, oa[0], ob[0]);
                }
            },
            [&] {
                if constexpr (kNext) {
                    if (st + 1 >= n_final) mask_tail_ops(st + 1, 0, oa[0], ob[0]);
                    prep(ob[0], bv[0], bj[0]);
                }
            });
    };
    // scalar loads still in flight would turn every LDS wait in the loop
    // into lgkmcnt(0): settle them here
    __builtin_amdgcn_s_waitcnt(0xC07F);
    static_for<kDmaDepth>([&](auto d) {
        // (the direct-B form always has at least RS stages)
        if (BD || d < n_st) issue(std::integral_constant<int, decltype(d)::value % RS>{}, d);
    });
    if constexpr (BD) wait_landed_bd(std::integral_constant<int, kDmaDepth - 1>{});
    else wait_landed(0);
    dma_barrier();
    if (BD || kDmaDepth < n_st) issue(std::integral_constant<int, kDmaDepth % RS>{}, kDmaDepth);
    {
        const char *PA, *PB;
        panels(0, PA, PB);
        load_ops(std::integral_constant<int, 0>{}, PA, PB, 0, oa[0], ob[0]);
        if (n_final == 0) mask_tail_ops(0, 0, oa[0], ob[0]);
        prep(ob[0], bv[0], bj[0]);
    }
    // the stage loop is unrolled by the ring size so that every slot index
    // is a constant; the final RS stages are peeled off
    for (int st = 0; st < n_final; st += RS)
        static_for<RS>([&](auto r) { run_stage(r, st + r, std::true_type{}, std::false_type{}); });
    static_for<RS>([&](auto r) {
        run_stage(r, n_final + r, std::integral_constant<bool, (decltype(r)::value + 1 < RS)>{}, std::true_type{});
    });
    lds_barrier();

    // ---- epilogue: 2x2 polarisation blocks of antennas a >= b
    if constexpr (NP > 0) {
        // flags of this lane's row antennas (8 per row block) and column
        // antennas, fetched together before the stores
        bool frow[NA][8], fcol[NBO];
#pragma unroll
        for (int i = 0; i < NBO; ++i) fcol[i] = false;
#pragma unroll
        for (int i = 0; i < NA; ++i)
#pragma unroll
            for (int k = 0; k < 8; ++k) frow[i][k] = false;
        if (fl_sb) {
            uint8_t fc[NBO], fr[NA][8];
#pragma unroll
            for (int i = 0; i < NBO; ++i) fc[i] = fl_sb[min(j0 + bn[i] * 32 + lr, N - 1) >> 1];
#pragma unroll
            for (int i = 0; i < NA; ++i)
#pragma unroll
                for (int k = 0; k < 8; ++k)
                    fr[i][k] = fl_sb[min(i0 + am[i] * 32 + 8 * (k >> 1) + 4 * lh + 2 * (k & 1), N - 1) >> 1];
#pragma unroll
            for (int i = 0; i < NBO; ++i) fcol[i] = fc[i] != 0;
#pragma unroll
            for (int i = 0; i < NA; ++i)
#pragma unroll
                for (int k = 0; k < 8; ++k) frow[i][k] = fr[i][k] != 0;
        }
        // Rows r, r + 1 of a lane are the two polarisations of one antenna a
        // and lanes lr, lr ^ 1 the two of one antenna b, so a lane pair holds
        // the four values of baseline (a, b).  The pair swaps one value so
        // that the even lane owns (p, q) = (0, 0), (0, 1) and the odd lane
        // (1, 0), (1, 1): each lane then stores 16 contiguous bytes and the
        // pair the whole 32-byte baseline.  Validity, flags and the antenna
        // indices are uniform over the pair.
        using E = std::conditional_t<DT == AFC_I8, int, float>;
        const bool odd = (lr & 1) != 0;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const int Jc = j0 + bn[J::IB[p]] * 32 + lr;
            const int b = Jc >> 1;
            const bool fb = fcol[J::IB[p]];
#pragma unroll
            for (int r = 0; r < 16; r += 2) {
                const E r0 = accR[p][r], i0v = accI[p][r], r1 = accR[p][r + 1], i1v = accI[p][r + 1];
                // the even lane sends its p = 1 values, the odd lane its p = 0 values
                const E yr = pair_swap(odd ? r0 : r1), yi = pair_swap(odd ? i0v : i1v);
                E o0 = odd ? yr : r0, o1 = odd ? yi : i0v, o2 = odd ? r1 : yr, o3 = odd ? i1v : yi;
                const int I = i0 + am[J::IA[p]] * 32 + 8 * (r >> 2) + 4 * lh + (r & 3);
                const int a = I >> 1;
                if (Jc >= N || I >= N || a < b) continue;
                if (a == b) {             // inputs equal for (0, 0) and (1, 1)
                    if (odd) o3 = E(0);
                    else o1 = E(0);
                }
                const bool flagged = fb || frow[J::IA[p]][((r >> 2) << 1) | ((r >> 1) & 1)];
                if (flagged) o0 = o1 = o2 = o3 = E(0);
                const int64_t bl = (int64_t)a * (a + 1) / 2 + b;
                // written once and not read again by this kernel: a streaming
                // (non-temporal) store
                typedef E ev4 __attribute__((ext_vector_type(4)));
                __builtin_nontemporal_store(ev4{o0, o1, o2, o3}, reinterpret_cast<ev4*>(vis_ch) + bl * 2 + (odd ? 1 : 0));
                if (write_weights && !odd) w_sb[bl] = flagged ? 0 : S;
            }
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
// job of 32 x 32 blocks (diagonal tiles spread their lower-triangle blocks
// over the waves); fp32: 2 x 2 waves of one block each.
template <int DT, int TILE>
__device__ __forceinline__ void xtile(const char* __restrict__ z, char* __restrict__ vis_ch,
                                      int32_t* __restrict__ w_sb, const uint8_t* __restrict__ fl_sb,
                                      int N, int Na, int S, int ti, int tj, bool write_weights, char* lds_raw) {
    if constexpr (DT == AFC_F32) {
        xtile_f32<DT, TILE>(z, vis_ch, w_sb, fl_sb, N, Na, S, ti, tj, write_weights, lds_raw);
    } else {
        const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
        auto run = [&](auto job, const int (&am)[4], const int (&bn)[2]) {
            xtile_mm<DT, TILE, decltype(job)>(z, vis_ch, w_sb, fl_sb, N, Na, S, ti, tj, write_weights, lds_raw,
                                              am, bn);
        };
        if constexpr (TILE == 128) {
            if (ti != tj) {
                const int am[4] = {0, 1, 2, 3}, bn[2] = {wid, 0};
                run(JobRows4{}, am, bn);
            } else if (wid == 0) {
                run(JobDiag0{}, JobDiag0::AM, JobDiag0::BN);
            } else if (wid == 1) {
                run(JobDiag1{}, JobDiag1::AM, JobDiag1::BN);
            } else if (wid == 2) {
                run(JobDiag2{}, JobDiag2::AM, JobDiag2::BN);
            } else {
                run(JobDiag3{}, JobDiag3::AM, JobDiag3::BN);
            }
        } else {
            static_assert(TILE == 64, "int8 / fp16 tiles are 128 or 64 wide");
            const int wr = wid >> 1, wc = wid & 1;
            const int am[4] = {wr, 0, 0, 0}, bn[2] = {wc, 0};
            if (ti == tj && wr < wc) run(JobIdle{}, am, bn);
            else run(JobOne{}, am, bn);
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
