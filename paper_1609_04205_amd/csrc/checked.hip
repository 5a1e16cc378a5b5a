// Checked (debug) mode: a count of the non-finite values (NaN, +-Inf) in a
// floating-point buffer.  With the mode on, the entry points count the
// non-finite values of their floating-point inputs before launching and
// refuse the call if there are any (the count is read back, so a checked
// call waits for its stream).  Off by default: the hot path never pays for
// it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <vector>

#include "afc_internal.h"

namespace afc {
namespace {

// Per-device counter of the checks (one word; each GPU holds its own copy).
// Host code uses the address hipGetSymbolAddress returns for the current
// device, never the name itself.
__device__ __align__(256) unsigned long long nonfinite_counter[64];

std::atomic<int> g_checked{0};

__global__ void counter_clear_kernel(unsigned long long* c) { c[threadIdx.x] = 0ull; }

template <int KIND>
__device__ __forceinline__ bool nonfinite_at(const void* p, size_t i) {
    if constexpr (KIND == AFC_VALUES_F32) {
        const unsigned u = reinterpret_cast<const unsigned*>(p)[i];
        return (u & 0x7F800000u) == 0x7F800000u;
    } else if constexpr (KIND == AFC_VALUES_F16) {
        const unsigned short u = reinterpret_cast<const unsigned short*>(p)[i];
        return (u & 0x7C00u) == 0x7C00u;
    } else {
        const unsigned long long u = reinterpret_cast<const unsigned long long*>(p)[i];
        return (u & 0x7FF0000000000000ull) == 0x7FF0000000000000ull;
    }
}

// exponent field all ones = Inf or NaN; grid-stride, one atomic per wave
template <int KIND>
__global__ void count_nonfinite_kernel(const void* __restrict__ p, size_t n, unsigned long long* c) {
    unsigned long long k = 0;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        k += nonfinite_at<KIND>(p, i) ? 1u : 0u;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) k += __shfl_xor(k, d);
    if ((threadIdx.x & 63) == 0 && k) atomicAdd(c, k);
}

hipError_t counter_address(unsigned long long** out) {
    static std::mutex mu;
    static std::vector<void*> ptrs;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lock(mu);
    if ((int)ptrs.size() <= dev) ptrs.resize(dev + 1, nullptr);
    if (!ptrs[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(nonfinite_counter));
        if (e != hipSuccess) return e;
        ptrs[dev] = p;
    }
    *out = reinterpret_cast<unsigned long long*>(ptrs[dev]);
    return hipSuccess;
}

}  // namespace

void set_checked_mode(bool on) { g_checked.store(on ? 1 : 0); }
bool checked_mode() { return g_checked.load() != 0; }

hipError_t count_nonfinite(const void* p, size_t n, int kind, unsigned long long* count, hipStream_t stream) {
    *count = 0;
    if (n == 0) return hipSuccess;
    // one counter per device: a count runs from its clear to its read-back
    // (the stream is synchronised) before another thread may start one
    static std::mutex busy;
    std::lock_guard<std::mutex> hold(busy);
    unsigned long long* c = nullptr;
    hipError_t e = counter_address(&c);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(counter_clear_kernel, dim3(1), dim3(64), 0, stream, c);
    const unsigned grid = (unsigned)std::min<size_t>((n + 255) / 256, 4096);
    if (kind == AFC_VALUES_F32)
        hipLaunchKernelGGL(count_nonfinite_kernel<AFC_VALUES_F32>, dim3(grid), dim3(256), 0, stream, p, n, c);
    else if (kind == AFC_VALUES_F16)
        hipLaunchKernelGGL(count_nonfinite_kernel<AFC_VALUES_F16>, dim3(grid), dim3(256), 0, stream, p, n, c);
    else
        hipLaunchKernelGGL(count_nonfinite_kernel<AFC_VALUES_F64>, dim3(grid), dim3(256), 0, stream, p, n, c);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    unsigned long long host = 0;
    e = hipMemcpyAsync(&host, c, sizeof host, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    *count = host;
    return e;
}

}  // namespace afc
