// Streaming ceilings of the HBM on the device the benchmark runs on: plain
// contiguous kernels with no method arithmetic, timed beside the AdamW-GS
// step so that its bandwidth can be read against what the memory system
// delivers for the same access mix, not only against the datasheet peak.
// Measurement support only: built as a library of its own, never linked
// into libgsopt.
//
// Each thread handles kItems 16-byte elements, 256 elements apart, and
// issues all of their loads before any store; loads and stores carry the
// non-temporal hint, as the step kernel's wide accesses do.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
constexpr int kThreads = 256;
constexpr int kItems = 4;

// The step's mix: four arrays read (parameter, gradient, two moments),
// three written back (parameter, two moments).
__global__ __launch_bounds__(kThreads) void rmw_4r3w_kernel(f4* p, const f4* g, f4* m, f4* v, int64_t n)
{
    const int64_t base = (int64_t)blockIdx.x * kThreads * kItems + threadIdx.x;
    f4 a[kItems], b[kItems], c[kItems], d[kItems];
#pragma unroll
    for (int u = 0; u < kItems; ++u) {
        const int64_t i = min(base + u * kThreads, n - 1);
        a[u] = __builtin_nontemporal_load(p + i);
        b[u] = __builtin_nontemporal_load(g + i);
        c[u] = __builtin_nontemporal_load(m + i);
        d[u] = __builtin_nontemporal_load(v + i);
    }
#pragma unroll
    for (int u = 0; u < kItems; ++u) {
        const int64_t i = base + u * kThreads;
        if (i >= n) break;
        const f4 mm = 0.875f * c[u] + 0.125f * b[u];
        const f4 vv = 0.5f * d[u] + 0.5f * b[u] * b[u];
        __builtin_nontemporal_store(a[u] - 0.0625f * mm, p + i);
        __builtin_nontemporal_store(mm, m + i);
        __builtin_nontemporal_store(vv, v + i);
    }
}

__global__ __launch_bounds__(kThreads) void copy_kernel(f4* dst, const f4* src, int64_t n)
{
    const int64_t base = (int64_t)blockIdx.x * kThreads * kItems + threadIdx.x;
    f4 a[kItems];
#pragma unroll
    for (int u = 0; u < kItems; ++u) a[u] = __builtin_nontemporal_load(src + min(base + u * kThreads, n - 1));
#pragma unroll
    for (int u = 0; u < kItems; ++u) {
        const int64_t i = base + u * kThreads;
        if (i < n) __builtin_nontemporal_store(a[u], dst + i);
    }
}

// Sums each thread's elements; one lane writes only if the sum equals a
// value it cannot take for the probe's data, so the loads are kept.
__global__ __launch_bounds__(kThreads) void read_kernel(const f4* src, int64_t n, float* sink)
{
    const int64_t base = (int64_t)blockIdx.x * kThreads * kItems + threadIdx.x;
    f4 s = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int u = 0; u < kItems; ++u) s += __builtin_nontemporal_load(src + min(base + u * kThreads, n - 1));
    if (s.x == -1.0e30f) sink[0] = s.y;
}

unsigned grid_for(int64_t n) { return (unsigned)((n + (int64_t)kThreads * kItems - 1) / ((int64_t)kThreads * kItems)); }

bool bad(const void* p) { return p == nullptr || (uintptr_t)p % 16 != 0; }

}  // namespace

// All pointers are device memory, 16-byte aligned; n16 counts 16-byte
// elements per array (1 .. 2^31).  Return 0 on success, -1 on a bad
// argument (nothing launched), else the HIP error of the launch.
extern "C" int gsprobe_rmw_4r3w(void* p, const void* g, void* m, void* v, int64_t n16, hipStream_t stream)
{
    if (bad(p) || bad(g) || bad(m) || bad(v) || n16 < 1 || n16 > ((int64_t)1 << 31)) return -1;
    hipLaunchKernelGGL(rmw_4r3w_kernel, dim3(grid_for(n16)), dim3(kThreads), 0, stream, static_cast<f4*>(p),
                       static_cast<const f4*>(g), static_cast<f4*>(m), static_cast<f4*>(v), n16);
    return (int)hipGetLastError();
}

extern "C" int gsprobe_copy(void* dst, const void* src, int64_t n16, hipStream_t stream)
{
    if (bad(dst) || bad(src) || n16 < 1 || n16 > ((int64_t)1 << 31)) return -1;
    hipLaunchKernelGGL(copy_kernel, dim3(grid_for(n16)), dim3(kThreads), 0, stream, static_cast<f4*>(dst),
                       static_cast<const f4*>(src), n16);
    return (int)hipGetLastError();
}

extern "C" int gsprobe_read(const void* src, int64_t n16, float* sink, hipStream_t stream)
{
    if (bad(src) || sink == nullptr || n16 < 1 || n16 > ((int64_t)1 << 31)) return -1;
    hipLaunchKernelGGL(read_kernel, dim3(grid_for(n16)), dim3(kThreads), 0, stream, static_cast<const f4*>(src), n16,
                       sink);
    return (int)hipGetLastError();
}
