// Gain-calibration loss and its gradient with respect to the complex gains.
// Sec. "Calibration Pipeline": per-channel amplitude and phase calibration of
// the XX and YY visibilities against a point-source sky model; read here as
// the least-squares loss
//
//   R_ab = V_ab - g_a M_ab conj(g_b),   L = sum_{a,b} |R_ab|^2
//   grad_a = dL/dRe g_a + i dL/dIm g_a = -2 sum_b [R_ab conj(M_ab) + conj(R_ba) M_ba] g_b
//
// With V and M stored as lower triangles (upper = conjugate), R is Hermitian
// off the diagonal and, for t_ab = R_ab conj(M_ab),
//   grad_a = -4 [ sum_{b<a} t_ab g_b + sum_{c>a} conj(t_ca) g_c + Re(t_aa) g_a ].
// Every stored element therefore feeds one row sum (antenna a) and one
// column sum (antenna b).
//
// Weighted form (Sec. "Real-time Flagging, Calibration and Imaging": the
// calibration works on the flagged visibilities, re-weighted for lost data):
// L = sum_{a,b} w_ab |R_ab|^2 with a real weight w_ab = w_ba per stored
// baseline and polarisation (0 where flagged), and t_ab = w_ab R_ab conj(M_ab).
//
// Pass 1: one workgroup per 64 x 64 antenna tile of the lower triangle and
// channel, both polarisations.  Each thread owns 4 rows x 4 columns;
// the residual is formed in float32 with error-free product and sum
// transformations, so that R keeps full float32 relative accuracy even when
// V and G M G^H cancel to a few percent.  Row sums (shuffles over the 16
// lanes of a row) and column sums (shuffles, then LDS across the waves) are
// accumulated in float64 and written to the workspace; the tile's loss is a
// float32 tree sum.
// Pass 2: one thread per antenna adds its row and column partials over the
// tiles in a fixed order (float64) and writes -4 x the sum; the first block
// of each (channel, polarisation) adds the tile losses in a fixed order.
// No atomics: the result is bitwise reproducible.
#include <mutex>
#include <utility>
#include <vector>

#include "afc_internal.h"

// The error-free transformations below need every product and sum rounded
// on its own: this file is compiled with -ffp-contract=off (the fma in
// two_prod is explicit), and the pragma keeps the intent visible.
#pragma clang fp contract(off)

namespace afc {
namespace {

constexpr int kTileA = 64;      // antennas per tile side
constexpr int kThreads = 256;   // 4 waves: rows r, r+4, ...

struct ff {
    float hi, lo;
};
__device__ __forceinline__ ff two_prod(float a, float b) {
    const float p = __fmul_rn(a, b);
    return {p, fmaf(a, b, -p)};
}
__device__ __forceinline__ ff two_sum(float a, float b) {
    const float s = __fadd_rn(a, b);
    const float bb = __fsub_rn(s, a);
    const float e = __fadd_rn(__fsub_rn(a, __fsub_rn(s, bb)), __fsub_rn(b, bb));
    return {s, e};
}
// a*b + c*d as hi + lo
__device__ __forceinline__ ff dot2(float a, float b, float c, float d) {
    const ff p = two_prod(a, b), q = two_prod(c, d);
    const ff s = two_sum(p.hi, q.hi);
    return {s.hi, __fadd_rn(s.lo, __fadd_rn(p.lo, q.lo))};
}

// R = V - g_a M conj(g_b), each component rounded once to float32.
__device__ __forceinline__ float2 residual(float2 v, float2 m, float2 ga, float2 gb) {
    // q = g_a conj(g_b)
    const ff qr = dot2(ga.x, gb.x, ga.y, gb.y);
    const ff qi = dot2(ga.y, gb.x, -ga.x, gb.y);
    // w = q M
    ff wr = dot2(qr.hi, m.x, -qi.hi, m.y);
    ff wi = dot2(qr.hi, m.y, qi.hi, m.x);
    wr.lo = __fadd_rn(wr.lo, __fsub_rn(__fmul_rn(qr.lo, m.x), __fmul_rn(qi.lo, m.y)));
    wi.lo = __fadd_rn(wi.lo, __fadd_rn(__fmul_rn(qr.lo, m.y), __fmul_rn(qi.lo, m.x)));
    // R = V - w
    const ff rr = two_sum(v.x, -wr.hi);
    const ff ri = two_sum(v.y, -wi.hi);
    return make_float2(__fadd_rn(rr.hi, __fsub_rn(rr.lo, wr.lo)), __fadd_rn(ri.hi, __fsub_rn(ri.lo, wi.lo)));
}

__device__ __forceinline__ float wave_sumf(float v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ void tile_rc(int t, int& ti, int& tj) {
    int r = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
    while (r * (r + 1) / 2 > t) --r;
    while ((r + 1) * (r + 2) / 2 <= t) ++r;
    ti = r;
    tj = t - r * (r + 1) / 2;
}

// workspace layout: rowpart, colpart double2 [P][2][n_tiles][64]; loss float [P][2][n_tiles];
// with kDiag also rowd, cold double [P][2][n_tiles][64]: the partial sums of
// D_a = sum_b |M_ab|^2 |g_b|^2 over the full Hermitian matrix (the diagonal
// of the Gauss-Newton normal matrix of the row-wise least-squares problem)
//
// V and M element (channel ch, polarisation pol, baseline bl) at
// ch * ch_stride + pol * pol_off + bl * el_stride float2: the correlator's
// [P][Nbl][2][2] layout (nbl * 4, 3, 4) or the solver's compact XX / YY
// copy [P][2][Nbl] (2 nbl, nbl, 1).
//
// Thread (r4, c4) of the tile owns rows 4 r4 .. 4 r4 + 3 and columns c4,
// c4 + 16, c4 + 32, c4 + 48 for both polarisations (a load of 16 lanes
// covers 16 consecutive baselines): a row's 16 column threads are 16
// consecutive lanes (xor-shuffle sum in 4 steps), a column's 16 row threads
// are 4 per wave (2 steps) times 4 waves (LDS).
// kRec: V and M in the correlator's 32-byte records (el_stride 4, pol_off 3)
// at 16-byte aligned addresses: each element is read as two 16-byte halves,
// (XX, XY) and (YX, YY), which the hardware fetches whole anyway (6% faster
// than two 8-byte loads).
// kW: weighted loss sum_{a,b} w_ab |R_ab|^2 with w from the visibility
// flags fl (uint8 [P][Nbl][2], nonzero = weight 0) and the weights wt (float
// [P][Nbl][2]; either may be NULL): every per-element term (loss, the
// gradient's t = w R conj(M), the solver's w |M|^2) is scaled by w.
template <bool kDiag, bool kRec, bool kW>
__global__ __launch_bounds__(kThreads) void cal_tiles_kernel(int Na, int P, int n_tiles, int64_t ch_stride,
                                                             int64_t pol_off, int el_stride,
                                                             const float2* __restrict__ V,
                                                             const float2* __restrict__ M, const float2* __restrict__ g,
                                                             double2* __restrict__ rowpart, double2* __restrict__ colpart,
                                                             float* __restrict__ losspart, double* __restrict__ rowd,
                                                             double* __restrict__ cold, const uint8_t* __restrict__ fl,
                                                             const float* __restrict__ wt) {
    constexpr int NV = kDiag ? 3 : 2;                         // re, im (and D) per sum
    __shared__ double col_lds[4][kTileA][2][NV];
    __shared__ float loss_lds[4][2];
    const int t = blockIdx.x, ch = blockIdx.y;
    int ti, tj;
    tile_rc(t, ti, tj);
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int c4 = tid & 15, r4 = tid >> 4;
    const float2* Vc = V + (int64_t)ch * ch_stride;
    const float2* Mc = M + (int64_t)ch * ch_stride;
    const int64_t nbl_w = (int64_t)Na * (Na + 1) / 2;        // baselines of the weight arrays
    const float2* gc = g + (int64_t)ch * Na * 2;              // [a][2]

    float2 gb[4][2];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int b = tj * kTileA + c4 + 16 * q;
#pragma unroll
        for (int p = 0; p < 2; ++p) gb[q][p] = b < Na ? gc[(int64_t)b * 2 + p] : make_float2(0.0f, 0.0f);
    }
    double col[4][2][NV];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int k = 0; k < NV; ++k) col[q][p][k] = 0.0;
    float lsum[2] = {0.0f, 0.0f};
    const int64_t slot0 = ((int64_t)(ch * 2) * n_tiles + t) * kTileA;            // pol 0
    const int64_t slot1 = ((int64_t)(ch * 2 + 1) * n_tiles + t) * kTileA;        // pol 1

#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int r = 4 * r4 + i;
        const int a = ti * kTileA + r;
        float2 ga[2];
#pragma unroll
        for (int p = 0; p < 2; ++p) ga[p] = a < Na ? gc[(int64_t)a * 2 + p] : make_float2(0.0f, 0.0f);
        double row[2][NV];
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int k = 0; k < NV; ++k) row[p][k] = 0.0;
        // all loads of the row first (clamped to element 0 where the
        // element is outside the triangle; such elements contribute nothing)
        float2 vv[4][2], mv[4][2];
        float ww[4][2];
        bool ok[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int b = tj * kTileA + c4 + 16 * q;
            ok[q] = a < Na && b < Na && b <= a;
            const int64_t e = ok[q] ? ((int64_t)a * (a + 1) / 2 + b) * el_stride : 0;
            if constexpr (kW) {
                // the element's two weights (XX, YY); outside the triangle
                // the element contributes nothing anyway
                const int64_t wi = ok[q] ? ((int64_t)ch * nbl_w + (int64_t)a * (a + 1) / 2 + b) * 2 : 0;
                const unsigned short fp = fl ? *reinterpret_cast<const unsigned short*>(fl + wi) : (unsigned short)0;
                const float2 wp = wt ? *reinterpret_cast<const float2*>(wt + wi) : make_float2(1.0f, 1.0f);
                ww[q][0] = (fp & 0xFF) ? 0.0f : wp.x;
                ww[q][1] = (fp >> 8) ? 0.0f : wp.y;
            }
            if constexpr (kRec) {
                const float4 v0 = *reinterpret_cast<const float4*>(Vc + e);
                const float4 v1 = *reinterpret_cast<const float4*>(Vc + e + 2);
                const float4 m0 = *reinterpret_cast<const float4*>(Mc + e);
                const float4 m1 = *reinterpret_cast<const float4*>(Mc + e + 2);
                vv[q][0] = make_float2(v0.x, v0.y);
                vv[q][1] = make_float2(v1.z, v1.w);
                mv[q][0] = make_float2(m0.x, m0.y);
                mv[q][1] = make_float2(m1.z, m1.w);
            } else {
#pragma unroll
                for (int p = 0; p < 2; ++p) {
                    vv[q][p] = Vc[e + p * pol_off];
                    mv[q][p] = Mc[e + p * pol_off];
                }
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int b = tj * kTileA + c4 + 16 * q;
            if (ok[q]) {
#pragma unroll
                for (int p = 0; p < 2; ++p) {
                    const float2 v = vv[q][p], mm = mv[q][p];
                    const float2 R = residual(v, mm, ga[p], gb[q][p]);
                    const float wq = kW ? ww[q][p] : 1.0f;
                    const float r2 = wq * (R.x * R.x + R.y * R.y);
                    lsum[p] += a == b ? r2 : 2.0f * r2;
                    // t = w R conj(M)
                    const float tr = wq * (R.x * mm.x + R.y * mm.y);
                    const float tm = a == b ? 0.0f : wq * (R.y * mm.x - R.x * mm.y);   // diagonal: Re(t) only
                    // row a: t g_b
                    row[p][0] += (double)(tr * gb[q][p].x - tm * gb[q][p].y);
                    row[p][1] += (double)(tr * gb[q][p].y + tm * gb[q][p].x);
                    if (a != b) {                                  // column b: conj(t) g_a
                        col[q][p][0] += (double)(tr * ga[p].x + tm * ga[p].y);
                        col[q][p][1] += (double)(tr * ga[p].y - tm * ga[p].x);
                    }
                    if constexpr (kDiag) {
                        // |M|^2 |g_b|^2 to row a; |M|^2 |g_a|^2 to column b off the diagonal
                        const double m2 = (double)wq * ((double)mm.x * mm.x + (double)mm.y * mm.y);
                        row[p][2] += m2 * ((double)gb[q][p].x * gb[q][p].x + (double)gb[q][p].y * gb[q][p].y);
                        if (a != b) col[q][p][2] += m2 * ((double)ga[p].x * ga[p].x + (double)ga[p].y * ga[p].y);
                    }
                }
            }
        }
        // row sums over the 16 column threads (consecutive lanes)
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int k = 0; k < NV; ++k)
#pragma unroll
                for (int off = 1; off < 16; off <<= 1) row[p][k] += __shfl_xor(row[p][k], off, 64);
        if (c4 == 0) {
            rowpart[slot0 + r] = make_double2(row[0][0], row[0][1]);
            rowpart[slot1 + r] = make_double2(row[1][0], row[1][1]);
            if constexpr (kDiag) {
                rowd[slot0 + r] = row[0][2];
                rowd[slot1 + r] = row[1][2];
            }
        }
    }
    // column sums: the 4 row threads of this wave, then the 4 waves
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int k = 0; k < NV; ++k) {
                col[q][p][k] += __shfl_xor(col[q][p][k], 16, 64);
                col[q][p][k] += __shfl_xor(col[q][p][k], 32, 64);
            }
    if (lane < 16) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int p = 0; p < 2; ++p)
#pragma unroll
                for (int k = 0; k < NV; ++k) col_lds[wv][c4 + 16 * q][p][k] = col[q][p][k];
    }
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        const float l = wave_sumf(lsum[p]);
        if (lane == 0) loss_lds[wv][p] = l;
    }
    __syncthreads();
    if (tid < 2 * kTileA) {
        const int c = tid & (kTileA - 1), p = tid / kTileA;
        const int64_t slot = p ? slot1 : slot0;
        double s[NV];
#pragma unroll
        for (int k = 0; k < NV; ++k)
            s[k] = (col_lds[0][c][p][k] + col_lds[1][c][p][k]) + (col_lds[2][c][p][k] + col_lds[3][c][p][k]);
        colpart[slot + c] = make_double2(s[0], s[1]);
        if constexpr (kDiag) cold[slot + c] = s[2];
    }
    if (tid < 2) {
        const int p = tid;
        losspart[(int64_t)(ch * 2 + p) * n_tiles + t] = (loss_lds[0][p] + loss_lds[1][p]) + (loss_lds[2][p] + loss_lds[3][p]);
    }
}

template <bool kDiag>
__global__ __launch_bounds__(256) void cal_reduce_kernel(int Na, int P, int nT, int n_tiles,
                                                         const double2* __restrict__ rowpart,
                                                         const double2* __restrict__ colpart,
                                                         const float* __restrict__ losspart, double* __restrict__ loss,
                                                         float2* __restrict__ grad, const double* __restrict__ rowd,
                                                         const double* __restrict__ cold, double* __restrict__ D) {
    const int ch = blockIdx.y, pol = blockIdx.z;
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t base = (int64_t)(ch * 2 + pol) * n_tiles;
    if (grad && a < Na) {
        const int ta = a / kTileA, ra = a % kTileA;
        double sr = 0.0, si = 0.0;
        for (int tj = 0; tj <= ta; ++tj) {                   // row a: tiles (ta, tj)
            const double2 v = rowpart[(base + ta * (ta + 1) / 2 + tj) * kTileA + ra];
            sr += v.x;
            si += v.y;
        }
        for (int ti = ta; ti < nT; ++ti) {                   // column a: tiles (ti, ta)
            const double2 v = colpart[(base + ti * (ti + 1) / 2 + ta) * kTileA + ra];
            sr += v.x;
            si += v.y;
        }
        grad[((int64_t)ch * Na + a) * 2 + pol] = make_float2((float)(-4.0 * sr), (float)(-4.0 * si));
        if constexpr (kDiag) {
            double sd = 0.0;
            for (int tj = 0; tj <= ta; ++tj) sd += rowd[(base + ta * (ta + 1) / 2 + tj) * kTileA + ra];
            for (int ti = ta; ti < nT; ++ti) sd += cold[(base + ti * (ti + 1) / 2 + ta) * kTileA + ra];
            D[((int64_t)ch * Na + a) * 2 + pol] = sd;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        float s = 0.0f;
        for (int t = 0; t < n_tiles; ++t) s += losspart[base + t];
        loss[ch * 2 + pol] = (double)s;
    }
}

int n_tiles_side(int Na) { return (int)ceil_div(Na, kTileA); }

// One iteration of the gain solver per (channel, antenna, polarisation):
// g_new = g - grad / (4 D), which with grad = -4 (sum_b V_ab conj(z_ab) -
// g_a D_a), z_ab = M_ab conj(g_b), is the alternating least-squares update
// sum_b V_ab conj(z_ab) / D_a of each gain with all others fixed; on every
// second iteration the new gain is averaged with the previous one.
__global__ void cal_update_kernel(int n, const float2* __restrict__ g, const float2* __restrict__ grad,
                                  const double* __restrict__ D, float2* __restrict__ g_next, int average) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const float2 gc = g[e];
    const double d = D[e];
    double nr = gc.x, ni = gc.y;
    if (d > 0.0) {
        nr = (double)gc.x - (double)grad[e].x / (4.0 * d);
        ni = (double)gc.y - (double)grad[e].y / (4.0 * d);
    }
    if (average) {
        nr = 0.5 * (nr + (double)gc.x);
        ni = 0.5 * (ni + (double)gc.y);
    }
    g_next[e] = make_float2((float)nr, (float)ni);
}

// Remove the common phase of each (channel, polarisation): g_a conj(g_0) / |g_0|.
__global__ void cal_reference_kernel(int Na, int P, const float2* __restrict__ g, float2* __restrict__ out) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= P * Na * 2) return;
    const int pol = e & 1, ch = e / (2 * Na);
    const float2 g0 = g[(int64_t)ch * Na * 2 + pol];
    const float2 ga = g[e];
    const double m = sqrt((double)g0.x * g0.x + (double)g0.y * g0.y);
    if (m > 0.0) {
        const double cr = g0.x / m, ci = -(double)g0.y / m;
        out[e] = make_float2((float)(ga.x * cr - ga.y * ci), (float)(ga.x * ci + ga.y * cr));
    } else {
        out[e] = ga;
    }
}

// XX and YY of V and M from [P][Nbl][2][2] into [P][2][Nbl] (one thread per
// channel and baseline)
__global__ void cal_compact_kernel(int64_t total, int64_t nbl, const float2* __restrict__ V,
                                   const float2* __restrict__ M, float2* __restrict__ Vc, float2* __restrict__ Mc) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total) return;
    const int64_t ch = e / nbl, bl = e - ch * nbl;
    Vc[2 * ch * nbl + bl] = V[4 * e];                           // XX
    Vc[(2 * ch + 1) * nbl + bl] = V[4 * e + 3];                 // YY
    Mc[2 * ch * nbl + bl] = M[4 * e];
    Mc[(2 * ch + 1) * nbl + bl] = M[4 * e + 3];
}

}  // namespace

size_t cal_workspace_bytes(int Na, int P) {
    const int nT = n_tiles_side(Na);
    const size_t n_tiles = (size_t)nT * (nT + 1) / 2;
    return (size_t)P * 2 * n_tiles * (2 * kTileA * sizeof(double2) + sizeof(float)) + 256;
}

size_t cal_solve_workspace_bytes(int Na, int P) {
    const int nT = n_tiles_side(Na);
    const size_t n_tiles = (size_t)nT * (nT + 1) / 2;
    const size_t n_g = (size_t)P * Na * 2;
    const size_t nbl = (size_t)Na * (Na + 1) / 2;
    // gradient workspace (rounded up to 256 B), row and column partials of D,
    // D, the gradient, two gain buffers, the per-iteration loss (rounded up
    // to 256 B), the compact XX / YY copies of V and M
    const size_t solver = (size_t)P * 2 * n_tiles * kTileA * 2 * sizeof(double) + n_g * (sizeof(double) + 3 * sizeof(float2))
                          + (size_t)P * 2 * sizeof(double);
    return ((cal_workspace_bytes(Na, P) + 255) & ~(size_t)255) + ((solver + 255) & ~(size_t)255)
           + 2 * (size_t)P * 2 * nbl * sizeof(float2);
}

hipError_t launch_calibrate_solve(int Na, int P, const float2* V, const float2* M, float2* g, int n_iter,
                                  double* loss, void* ws, hipStream_t stream, const uint8_t* fl, const float* wt) {
    const int nT = n_tiles_side(Na);
    const int n_tiles = nT * (nT + 1) / 2;
    const size_t n_g = (size_t)P * Na * 2;
    char* w = reinterpret_cast<char*>(ws);
    double2* rowpart = reinterpret_cast<double2*>(w);
    double2* colpart = rowpart + (size_t)P * 2 * n_tiles * kTileA;
    float* losspart = reinterpret_cast<float*>(colpart + (size_t)P * 2 * n_tiles * kTileA);
    char* w2 = w + ((cal_workspace_bytes(Na, P) + 255) & ~(size_t)255);
    double* rowd = reinterpret_cast<double*>(w2);
    double* cold = rowd + (size_t)P * 2 * n_tiles * kTileA;
    double* D = cold + (size_t)P * 2 * n_tiles * kTileA;
    float2* grad = reinterpret_cast<float2*>(D + n_g);
    float2* ga = grad + n_g;
    float2* gb = ga + n_g;
    double* it_loss = reinterpret_cast<double*>(gb + n_g);
    // compact XX / YY copies of V and M: every iteration reads only what it
    // uses, contiguously
    const int64_t nbl = (int64_t)Na * (Na + 1) / 2;
    const size_t solver = (size_t)P * 2 * n_tiles * kTileA * 2 * sizeof(double) + n_g * (sizeof(double) + 3 * sizeof(float2))
                          + (size_t)P * 2 * sizeof(double);
    float2* Vc = reinterpret_cast<float2*>(w2 + ((solver + 255) & ~(size_t)255));
    float2* Mc = Vc + (size_t)P * 2 * nbl;
    hipError_t e = hipMemcpyAsync(ga, g, n_g * sizeof(float2), hipMemcpyDeviceToDevice, stream);
    if (e != hipSuccess) return e;
    if (n_iter > 0) {
        const int64_t total = (int64_t)P * nbl;
        hipLaunchKernelGGL(cal_compact_kernel, dim3((unsigned)ceil_div(total, 256)), dim3(256), 0, stream, total, nbl,
                           V, M, Vc, Mc);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const unsigned ug = (unsigned)ceil_div((int64_t)n_g, 256);
    for (int it = 1; it <= n_iter; ++it) {
        if (fl || wt)
            hipLaunchKernelGGL((cal_tiles_kernel<true, false, true>), dim3(n_tiles, P), dim3(kThreads), 0, stream, Na,
                               P, n_tiles, 2 * nbl, nbl, 1, Vc, Mc, ga, rowpart, colpart, losspart, rowd, cold, fl, wt);
        else
            hipLaunchKernelGGL((cal_tiles_kernel<true, false, false>), dim3(n_tiles, P), dim3(kThreads), 0, stream, Na,
                               P, n_tiles, 2 * nbl, nbl, 1, Vc, Mc, ga, rowpart, colpart, losspart, rowd, cold, nullptr,
                               nullptr);
        hipLaunchKernelGGL(cal_reduce_kernel<true>, dim3((unsigned)ceil_div(Na, 256), P, 2), dim3(256), 0, stream,
                           Na, P, nT, n_tiles, rowpart, colpart, losspart, it_loss, grad, rowd, cold, D);
        hipLaunchKernelGGL(cal_update_kernel, dim3(ug), dim3(256), 0, stream, (int)n_g, ga, grad, D, gb,
                           (int)(it % 2 == 0));
        std::swap(ga, gb);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(cal_reference_kernel, dim3(ug), dim3(256), 0, stream, Na, P, ga, g);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (loss) return launch_calibrate(Na, P, V, M, g, loss, nullptr, ws, stream, fl, wt);
    return hipSuccess;
}

// Scratch of the allocation-free gradient entry point: the per-tile partial
// sums (every element read is written earlier in the same call, so nothing
// has to start at zero).  Each GPU the library runs on holds its own copy
// until the process ends.  Host code never passes `cal_scratch` itself to a
// kernel (on the host it names a stand-in, not the device address): it uses
// the address hipGetSymbolAddress returns for the current device.
__device__ __align__(256) unsigned char cal_scratch[kCalScratchBytes];

hipError_t cal_scratch_address(void** out) {
    static std::mutex mu;
    static std::vector<void*> ptrs;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lock(mu);
    if ((int)ptrs.size() <= dev) ptrs.resize(dev + 1, nullptr);
    if (!ptrs[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(cal_scratch));
        if (e != hipSuccess) return e;
        ptrs[dev] = p;
    }
    *out = ptrs[dev];
    return hipSuccess;
}

hipError_t launch_calibrate(int Na, int P, const float2* V, const float2* M, const float2* g, double* loss,
                            float2* grad, void* ws, hipStream_t stream, const uint8_t* fl, const float* wt) {
    const int nT = n_tiles_side(Na);
    const int n_tiles = nT * (nT + 1) / 2;
    char* w = reinterpret_cast<char*>(ws);
    double2* rowpart = reinterpret_cast<double2*>(w);
    double2* colpart = rowpart + (size_t)P * 2 * n_tiles * kTileA;
    float* losspart = reinterpret_cast<float*>(colpart + (size_t)P * 2 * n_tiles * kTileA);
    const int64_t nbl = (int64_t)Na * (Na + 1) / 2;
    const bool aligned16 = (reinterpret_cast<uintptr_t>(V) | reinterpret_cast<uintptr_t>(M)) % 16 == 0;
    const bool weighted = fl || wt;
#define AFC_CAL_TILES(REC, W)                                                                                       \
    hipLaunchKernelGGL((cal_tiles_kernel<false, REC, W>), dim3(n_tiles, P), dim3(kThreads), 0, stream, Na, P,         \
                       n_tiles, nbl * 4, (int64_t)3, 4, V, M, g, rowpart, colpart, losspart, nullptr, nullptr, fl, wt)
    if (aligned16) {
        if (weighted) AFC_CAL_TILES(true, true);
        else AFC_CAL_TILES(true, false);
    } else {
        if (weighted) AFC_CAL_TILES(false, true);
        else AFC_CAL_TILES(false, false);
    }
#undef AFC_CAL_TILES
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(cal_reduce_kernel<false>, dim3((unsigned)ceil_div(Na, 256), P, 2), dim3(256), 0, stream, Na, P,
                       nT, n_tiles, rowpart, colpart, losspart, loss, grad, nullptr, nullptr, nullptr);
    return hipGetLastError();
}

}  // namespace afc
