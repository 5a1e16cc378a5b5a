// Gridding and imaging (Sec. "Imaging Pipeline": the calibrated
// visibilities of several subbands are gridded onto one grid with bilinear
// interpolation, which integrates them spectrally, and the grid is Fourier
// transformed into the snapshot image).
//
// Gridding, per cross-correlation a > c of subband b and channel k with
// weight w > 0: I = (XX + YY) / 2 at u = (x_a - x_c) nu / c, v = (y_a - y_c)
// nu / c; (pu, pv) = (u, v) / du + N/2, i0 = floor(pu), fu = pu - i0;
// w I goes to the four cells around (pu, pv) with bilinear weights and
// w conj(I) to the mirrored cells (N - j, N - i) (the point -u, -v).  A
// visibility is gridded only if all eight cells are inside the grid.
//
//  * grid_bound_kernel: per (subband, baseline) the sum of 2 w (|Re I| +
//    |Im I|) over its gridded channels (a bound on any cell) and of 2 w (the
//    normalisation), reduced in a fixed order.
//  * grid_kernel: one workgroup per (subband, pair of 48-antenna blocks),
//    one thread per baseline at a time.  Across the 64 channels of a
//    subband a baseline's uv point moves by a small fraction of its length,
//    so the thread accumulates its contributions in a 3 x 3 window of cells
//    in registers (float64) and only adds the window when the point leaves
//    it and at the end: to a 64 x 64-cell window in LDS around the blocks'
//    mean separation (added to the grid once per workgroup), or to the grid.  The grid accumulates in
//    64-bit fixed point (2^e scaled, e from the bound so that nothing can
//    overflow): integer atomics make the result independent of the order of
//    the additions, so the grid is bitwise reproducible.
//  * imaging: (-1)^(p+q) modulation, radix-2 Stockham FFT of each row in LDS,
//    transpose, row FFT again, and (-1)^(i+j) Re(.) / norm with the
//    transpose back.
#include "afc_internal.h"

namespace afc {
namespace {

constexpr double kC = 299792458.0;

struct GridArgs {
    const float2* vis;            // [B][64][Nbl][2][2]
    const int32_t* weights;       // [B][Nbl] or nullptr
    const double* pos;            // [Na][2]
    const double* freq;           // [B][64]
    int Na, B, N;
    double inv_du;
};

__device__ __forceinline__ void pair_of(int64_t t, int& a, int& c) {
    // t-th cross-correlation in lower-triangle order (a > c): a(a-1)/2 + c
    int x = (int)((sqrt(8.0 * (double)t + 1.0) + 1.0) * 0.5);
    while ((int64_t)x * (x - 1) / 2 > t) --x;
    while ((int64_t)(x + 1) * x / 2 <= t) ++x;
    a = x;
    c = (int)(t - (int64_t)x * (x - 1) / 2);
}

struct Vis1 {
    double re, im, w;
    double pu, pv;
    bool ok;
};

__device__ __forceinline__ Vis1 load_vis(const GridArgs& g, int b, int k, int a, int c, double dx, double dy,
                                         double w) {
    Vis1 r;
    const int64_t nbl = (int64_t)g.Na * (g.Na + 1) / 2;
    const int64_t bl = (int64_t)a * (a + 1) / 2 + c;
    const float2* v = g.vis + (((int64_t)b * kP + k) * nbl + bl) * 4;
    const float2 xx = v[0], yy = v[3];
    r.re = 0.5 * ((double)xx.x + (double)yy.x);
    r.im = 0.5 * ((double)xx.y + (double)yy.y);
    r.w = w;
    const double nu = g.freq[b * kP + k];
    r.pu = dx * nu / kC * g.inv_du + 0.5 * g.N;
    r.pv = dy * nu / kC * g.inv_du + 0.5 * g.N;
    const double i0 = floor(r.pu), j0 = floor(r.pv);
    r.ok = w > 0.0 && i0 >= 1.0 && j0 >= 1.0 && i0 <= g.N - 2.0 && j0 <= g.N - 2.0;
    return r;
}

// bound and normalisation: partial sums per block of 256 (subband, baseline)
// threads, tree-reduced in LDS
__global__ __launch_bounds__(256) void grid_bound_kernel(GridArgs g, double* __restrict__ part_abs,
                                                         double* __restrict__ part_w, int64_t n_cross) {
    __shared__ double ra[256], rw[256];
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double sa = 0.0, sw = 0.0;
    if (t < n_cross * g.B) {
        const int b = (int)(t / n_cross);
        int a, c;
        pair_of(t % n_cross, a, c);
        const double dx = g.pos[a * 2] - g.pos[c * 2], dy = g.pos[a * 2 + 1] - g.pos[c * 2 + 1];
        const double w = g.weights ? (double)g.weights[(int64_t)b * ((int64_t)g.Na * (g.Na + 1) / 2) +
                                                       (int64_t)a * (a + 1) / 2 + c]
                                   : 1.0;
        for (int k = 0; k < kP; ++k) {
            const Vis1 v = load_vis(g, b, k, a, c, dx, dy, w);
            if (!v.ok) continue;
            sa += 2.0 * w * (fabs(v.re) + fabs(v.im));
            sw += 2.0 * w;
        }
    }
    ra[threadIdx.x] = sa;
    rw[threadIdx.x] = sw;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            ra[threadIdx.x] += ra[threadIdx.x + s];
            rw[threadIdx.x] += rw[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part_abs[blockIdx.x] = ra[0];
        part_w[blockIdx.x] = rw[0];
    }
}

// one block: totals in a fixed order; scale = 2^e with bound * scale < 2^61
__global__ __launch_bounds__(256) void grid_total_kernel(const double* __restrict__ part_abs,
                                                         const double* __restrict__ part_w, int n_part,
                                                         double* __restrict__ scale, double* __restrict__ norm) {
    __shared__ double ra[256], rw[256];
    double sa = 0.0, sw = 0.0;
    for (int i = threadIdx.x; i < n_part; i += 256) {
        sa += part_abs[i];
        sw += part_w[i];
    }
    ra[threadIdx.x] = sa;
    rw[threadIdx.x] = sw;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            ra[threadIdx.x] += ra[threadIdx.x + s];
            rw[threadIdx.x] += rw[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        int e = 0;
        frexp(ra[0] > 0.0 ? ra[0] : 1.0, &e);              // bound < 2^e
        scale[0] = ldexp(1.0, 61 - e);
        norm[0] = rw[0];
    }
}

__global__ void zero_words_kernel(unsigned long long* __restrict__ p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

// Gridding work: one workgroup per (subband, pair of 48-antenna blocks; a
// block is one station of the array), so that the baselines of a workgroup
// land in a compact patch of the uv plane.  Cells inside a 64 x 64 window
// around the blocks' mean separation are summed in LDS (64-bit fixed point,
// the same integers as the grid's atomics) and added to the grid once per
// workgroup with their mirrors; cells outside the window (other layouts, a
// patch larger than the window) go to the grid directly.  Integer sums: the
// grid is the same whatever the routing.
constexpr int kGB = 48;                      // antennas per block
constexpr int kGW = 64;                      // LDS window side, cells
constexpr int kGThreads = 1024;

__device__ __forceinline__ void add_fixed(unsigned long long* cell, double v, double scale) {
    if (v != 0.0) atomicAdd(cell, (unsigned long long)llrint(v * scale));
}

// one baseline a > c of subband b: its 64 channels through a 3 x 3 window of
// cells in registers (float64), flushed to the LDS window or the grid when
// the point leaves it and at the end
__device__ __forceinline__ void grid_baseline(const GridArgs& g, int b, int a, int c, double scale,
                                              unsigned long long* __restrict__ grid, unsigned long long* win,
                                              int i0w, int j0w) {
    const double dx = g.pos[a * 2] - g.pos[c * 2], dy = g.pos[a * 2 + 1] - g.pos[c * 2 + 1];
    const double w = g.weights ? (double)g.weights[(int64_t)b * ((int64_t)g.Na * (g.Na + 1) / 2) +
                                                   (int64_t)a * (a + 1) / 2 + c]
                               : 1.0;
    if (w <= 0.0) return;
    const int N = g.N;
    double wr[3][3], wi[3][3];
    int ai = 0, aj = 0;
    bool open = false;
    auto flush = [&]() {
#pragma unroll
        for (int y = 0; y < 3; ++y)
#pragma unroll
            for (int x = 0; x < 3; ++x) {
                const int i = ai + x, j = aj + y;
                if (wr[y][x] == 0.0 && wi[y][x] == 0.0) continue;
                const unsigned li = (unsigned)(i - i0w), lj = (unsigned)(j - j0w);
                if (li < (unsigned)kGW && lj < (unsigned)kGW) {
                    unsigned long long* l = win + (lj * kGW + li) * 2;
                    if (wr[y][x] != 0.0) atomicAdd(l, (unsigned long long)llrint(wr[y][x] * scale));
                    if (wi[y][x] != 0.0) atomicAdd(l + 1, (unsigned long long)llrint(wi[y][x] * scale));
                } else {
                    // cells of gridded visibilities: 1 <= i, j <= N-1, mirrors likewise
                    unsigned long long* d = grid + ((int64_t)j * N + i) * 2;
                    unsigned long long* m = grid + ((int64_t)(N - j) * N + (N - i)) * 2;
                    add_fixed(d, wr[y][x], scale);
                    add_fixed(d + 1, wi[y][x], scale);
                    add_fixed(m, wr[y][x], scale);
                    add_fixed(m + 1, -wi[y][x], scale);
                }
            }
    };
    for (int k = 0; k < kP; ++k) {
        const Vis1 v = load_vis(g, b, k, a, c, dx, dy, w);
        if (!v.ok) continue;
        const int i0 = (int)floor(v.pu), j0 = (int)floor(v.pv);
        const double fu = v.pu - i0, fv = v.pv - j0;
        if (!open || i0 < ai || j0 < aj || i0 + 1 > ai + 2 || j0 + 1 > aj + 2) {
            if (open) flush();
            ai = i0;
            aj = j0;
            open = true;
#pragma unroll
            for (int y = 0; y < 3; ++y)
#pragma unroll
                for (int x = 0; x < 3; ++x) wr[y][x] = wi[y][x] = 0.0;
        }
        const int ox = i0 - ai, oy = j0 - aj;                 // 0 or 1
#pragma unroll
        for (int y = 0; y < 3; ++y) {
            const double wy = y == oy ? 1.0 - fv : y == oy + 1 ? fv : 0.0;
#pragma unroll
            for (int x = 0; x < 3; ++x) {
                const double wx = x == ox ? 1.0 - fu : x == ox + 1 ? fu : 0.0;
                const double f = wx * wy * w;
                wr[y][x] += f * v.re;
                wi[y][x] += f * v.im;
            }
        }
    }
    if (open) flush();
}

__global__ __launch_bounds__(kGThreads) void grid_kernel(GridArgs g, const double* __restrict__ scale_p,
                                                         unsigned long long* __restrict__ grid) {
    __shared__ unsigned long long win[kGW * kGW * 2];
    __shared__ double msum[2];
    const int b = blockIdx.y;
    int ba, bc;                                               // block pair ba >= bc
    {
        const int t = blockIdx.x;
        int r = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
        while (r * (r + 1) / 2 > t) --r;
        while ((r + 1) * (r + 2) / 2 <= t) ++r;
        ba = r;
        bc = t - r * (r + 1) / 2;
    }
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int a0 = ba * kGB, c0 = bc * kGB;
    const int nA = min(kGB, g.Na - a0), nC = min(kGB, g.Na - c0);
    for (int e = tid; e < kGW * kGW * 2; e += kGThreads) win[e] = 0ull;
    // window origin: the mean separation of the two blocks at the subband's
    // middle channel (wave 0 sums the positions)
    if (wv == 0) {
        double sx = 0.0, sy = 0.0, tx = 0.0, ty = 0.0;
        if (lane < nA) {
            sx = g.pos[(a0 + lane) * 2];
            sy = g.pos[(a0 + lane) * 2 + 1];
        }
        if (lane < nC) {
            tx = g.pos[(c0 + lane) * 2];
            ty = g.pos[(c0 + lane) * 2 + 1];
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            sx += __shfl_xor(sx, off, 64);
            sy += __shfl_xor(sy, off, 64);
            tx += __shfl_xor(tx, off, 64);
            ty += __shfl_xor(ty, off, 64);
        }
        if (lane == 0) {
            msum[0] = sx / nA - tx / nC;
            msum[1] = sy / nA - ty / nC;
        }
    }
    __syncthreads();
    const double nu = g.freq[b * kP + kP / 2];
    const double ur = msum[0] * nu / kC * g.inv_du + 0.5 * g.N;
    const double vr = msum[1] * nu / kC * g.inv_du + 0.5 * g.N;
    const int i0w = (int)floor(ur) - kGW / 2, j0w = (int)floor(vr) - kGW / 2;
    const double scale = scale_p[0];

    const int n_bl = ba == bc ? nA * (nA - 1) / 2 : nA * nC;
    for (int q = tid; q < n_bl; q += kGThreads) {
        int a, c;
        if (ba == bc) {
            pair_of(q, a, c);
            a += a0;
            c += c0;
        } else {
            a = a0 + q / nC;
            c = c0 + q % nC;
        }
        grid_baseline(g, b, a, c, scale, grid, win, i0w, j0w);
    }
    __syncthreads();
    const int N = g.N;
    for (int e = tid; e < kGW * kGW; e += kGThreads) {
        const long long re = (long long)win[e * 2], im = (long long)win[e * 2 + 1];
        if (re == 0 && im == 0) continue;
        // nonzero cells are cells of gridded visibilities: 1 <= i, j <= N-1
        const int i = i0w + e % kGW, j = j0w + e / kGW;
        unsigned long long* d = grid + ((int64_t)j * N + i) * 2;
        unsigned long long* m = grid + ((int64_t)(N - j) * N + (N - i)) * 2;
        if (re != 0) {
            atomicAdd(d, (unsigned long long)re);
            atomicAdd(m, (unsigned long long)re);
        }
        if (im != 0) {
            atomicAdd(d + 1, (unsigned long long)im);
            atomicAdd(m + 1, (unsigned long long)(-im));
        }
    }
}

// fixed point -> float2 grid (un-normalised), as the gridding's output
__global__ void grid_to_float_kernel(const unsigned long long* __restrict__ grid, const double* __restrict__ scale_p,
                                     float2* __restrict__ out, int64_t n) {
    const double inv = 1.0 / scale_p[0];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const long long re = (long long)grid[i * 2], im = (long long)grid[i * 2 + 1];
        out[i] = make_float2((float)((double)re * inv), (float)((double)im * inv));
    }
}

// ---------------------------------------------------------------- FFT
__device__ __forceinline__ float2 cmulf(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__global__ void twiddle_kernel(float2* __restrict__ tw, int N) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= N / 2) return;
    const double ang = -2.0 * 3.14159265358979323846 * (double)m / (double)N;
    tw[m] = make_float2((float)cos(ang), (float)sin(ang));
}

// Forward DFT of each row of `data` (N points, N a power of two) in place:
// X[k] = sum_n x[n] exp(-2 pi i k n / N).  Radix-2 Stockham: with sub-DFTs
// of size ns done, butterfly j (< N/2) takes x[j] and x[j + N/2], rotates
// the second by exp(-2 pi i (j mod ns) / (2 ns)) and writes the sum and the
// difference to positions (j / ns) 2 ns + j mod ns and that + ns.
// Optional (-1)^(row + column) modulation on load.
__global__ __launch_bounds__(256) void fft_rows_kernel(float2* __restrict__ data, const float2* __restrict__ tw,
                                                       int N, int log2N, int modulate) {
    extern __shared__ float2 buf[];
    float2* x = buf;
    float2* y = buf + N;
    const int row = blockIdx.x;
    float2* r = data + (int64_t)row * N;
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        float2 v = r[i];
        if (modulate && ((row + i) & 1)) v = make_float2(-v.x, -v.y);
        x[i] = v;
    }
    __syncthreads();
    const int half = N / 2;
    for (int l = 0; l < log2N; ++l) {
        const int ns = 1 << l;
        for (int j = threadIdx.x; j < half; j += blockDim.x) {
            const int k = j & (ns - 1);
            const float2 a = x[j];
            const float2 b = cmulf(x[j + half], tw[k << (log2N - 1 - l)]);
            const int o = ((j >> l) << (l + 1)) + k;
            y[o] = make_float2(a.x + b.x, a.y + b.y);
            y[o + ns] = make_float2(a.x - b.x, a.y - b.y);
        }
        __syncthreads();
        float2* t = x;
        x = y;
        y = t;
    }
    for (int i = threadIdx.x; i < N; i += blockDim.x) r[i] = x[i];
}

// out[c][r] = in[r][c] for an N x N float2 matrix; 32 x 32 tiles via LDS.
// finalize: out is float, (-1)^(r+c) Re(in[r][c]) / norm.
template <bool kFinal>
__global__ __launch_bounds__(256) void transpose_kernel(const float2* __restrict__ in, void* __restrict__ out, int N,
                                                        const double* __restrict__ norm_p) {
    __shared__ float2 tile[32][33];
    const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;       // 32 x 8
    for (int y = ty; y < 32; y += 8) tile[y][tx] = in[(int64_t)(by + y) * N + bx + tx];
    __syncthreads();
    if constexpr (kFinal) {
        const double nv = norm_p[0];
        const float inv = (float)(1.0 / (nv > 0.0 ? nv : 1.0));
        float* o = reinterpret_cast<float*>(out);
        for (int y = ty; y < 32; y += 8) {
            const int orow = bx + y, ocol = by + tx;                   // element in[ocol][orow]
            const float v = tile[tx][y].x * inv;
            o[(int64_t)orow * N + ocol] = ((orow + ocol) & 1) ? -v : v;
        }
    } else {
        float2* o = reinterpret_cast<float2*>(out);
        for (int y = ty; y < 32; y += 8) o[(int64_t)(bx + y) * N + by + tx] = tile[tx][y];
    }
}

}  // namespace

size_t imaging_workspace_bytes(int Na, int B, int N) {
    const int64_t n_cross = (int64_t)Na * (Na - 1) / 2;
    const int64_t n_part = ceil_div(std::max<int64_t>(1, n_cross * B), 256);
    return (size_t)N * N * 16                      // fixed-point grid
           + (size_t)N * N * 8 * 2                 // two float2 planes
           + (size_t)N / 2 * 8                     // twiddles
           + (size_t)n_part * 16 + 64;             // partial sums, scale
}

hipError_t launch_grid(const float2* vis, const int32_t* weights, const double* pos, const double* freq, int Na, int B,
                       int N, double du, float2* grid_out, double* norm, void* ws, hipStream_t stream) {
    const int64_t n_cross = (int64_t)Na * (Na - 1) / 2;
    const int64_t n_thr = std::max<int64_t>(1, n_cross * B);
    const int n_part = (int)ceil_div(n_thr, 256);
    char* w = reinterpret_cast<char*>(ws);
    unsigned long long* fixed = reinterpret_cast<unsigned long long*>(w);
    double* part_abs = reinterpret_cast<double*>(w + (size_t)N * N * 16 + (size_t)N * N * 16 + (size_t)N / 2 * 8);
    double* part_w = part_abs + n_part;
    double* scale = part_w + n_part;
    GridArgs g{vis, weights, pos, freq, Na, B, N, 1.0 / du};
    const int64_t n_words = (int64_t)N * N * 2;
    hipLaunchKernelGGL(zero_words_kernel, dim3((unsigned)std::min<int64_t>(ceil_div(n_words, 256), 4096)), dim3(256),
                       0, stream, fixed, n_words);
    hipLaunchKernelGGL(grid_bound_kernel, dim3(n_part), dim3(256), 0, stream, g, part_abs, part_w, n_cross);
    hipLaunchKernelGGL(grid_total_kernel, dim3(1), dim3(256), 0, stream, part_abs, part_w, n_part, scale, norm);
    const int n_blk = (int)ceil_div(Na, kGB);
    if (n_cross > 0 && B > 0)
        hipLaunchKernelGGL(grid_kernel, dim3((unsigned)(n_blk * (n_blk + 1) / 2), (unsigned)B), dim3(kGThreads), 0,
                           stream, g, scale, fixed);
    hipLaunchKernelGGL(grid_to_float_kernel, dim3((unsigned)std::min<int64_t>(ceil_div((int64_t)N * N, 256), 4096)),
                       dim3(256), 0, stream, fixed, scale, grid_out, (int64_t)N * N);
    return hipGetLastError();
}

hipError_t launch_image(const float2* grid, const double* norm, float* image, int N, void* ws, hipStream_t stream) {
    int log2N = 0;
    while ((1 << log2N) < N) ++log2N;
    char* w = reinterpret_cast<char*>(ws);
    float2* a = reinterpret_cast<float2*>(w + (size_t)N * N * 16);
    float2* b = a + (size_t)N * N;
    float2* tw = b + (size_t)N * N;
    hipLaunchKernelGGL(twiddle_kernel, dim3((unsigned)ceil_div(N / 2, 256)), dim3(256), 0, stream, tw, N);
    hipError_t e = hipMemcpyAsync(a, grid, (size_t)N * N * sizeof(float2), hipMemcpyDeviceToDevice, stream);
    if (e != hipSuccess) return e;
    const size_t lds = (size_t)2 * N * sizeof(float2);
    const dim3 tgrid((unsigned)(N / 32), (unsigned)(N / 32));
    hipLaunchKernelGGL(fft_rows_kernel, dim3(N), dim3(256), lds, stream, a, tw, N, log2N, 1);
    hipLaunchKernelGGL(transpose_kernel<false>, tgrid, dim3(256), 0, stream, a, b, N, norm);
    hipLaunchKernelGGL(fft_rows_kernel, dim3(N), dim3(256), lds, stream, b, tw, N, log2N, 0);
    hipLaunchKernelGGL(transpose_kernel<true>, tgrid, dim3(256), 0, stream, b, image, N, norm);
    return hipGetLastError();
}

}  // namespace afc
