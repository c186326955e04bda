// Streaming ceilings of the HBM on the device the benchmark runs on: plain
// contiguous kernels with no method arithmetic, timed beside the AdamW-GS
// step so that its bandwidth can be read against what the memory system
// delivers for the same access mix, not only against the datasheet peak.
// Measurement support only: built as a library of its own, never linked
// into libgsopt.
//
// Three access mixes over 16-byte-aligned arrays:
//   rmw_4r3w  four arrays read (parameter, gradient, two moments), three
//             written back (parameter, two moments): the step's mix;
//   copy      one array read, one written;
//   read      one array read (a reduction that keeps every load).
// Each comes in a family of launch shapes, so that the ceiling is the best
// over shapes and not one shape's figure:
//   width     bytes per access: 8 or 16;
//   items     accesses in flight per thread per array: 2, 4, 8 or 16 (all
//             loads of a tile are issued before any store);
//   nt_load / nt_store   the non-temporal hint on loads / stores; nt_load = 2
//             hints only the loads of arrays that are written back (the
//             4-read / 3-write mix's parameter and moments; its gradient
//             is loaded plainly);
//   blocks    0: one tile per block (the grid covers the arrays once);
//             > 0: that many blocks, each striding over the tiles.
// A tile is 256 threads x items accesses, 256 accesses apart per item, so
// each access instruction of a wave covers one contiguous 64 x width bytes.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f2 __attribute__((ext_vector_type(2)));
constexpr int kThreads = 256;

template <bool NT, typename T>
__device__ __forceinline__ T ld(const T* p)
{
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}

template <bool NT, typename T>
__device__ __forceinline__ void st(T x, T* p)
{
    if constexpr (NT) __builtin_nontemporal_store(x, p);
    else *p = x;
}

// NTL: 0 none, 1 every load, 2 the loads of the arrays written back
template <typename T, int ITEMS, int NTL, bool NTS>
__global__ __launch_bounds__(kThreads) void rmw_4r3w_kernel(T* p, const T* g, T* m, T* v, int64_t n, int64_t tiles)
{
    for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        const int64_t base = tile * kThreads * ITEMS + threadIdx.x;
        T a[ITEMS], b[ITEMS], c[ITEMS], d[ITEMS];
#pragma unroll
        for (int u = 0; u < ITEMS; ++u) {
            const int64_t i = min(base + u * kThreads, n - 1);
            a[u] = ld<NTL != 0>(p + i);
            b[u] = ld<NTL == 1>(g + i);
            c[u] = ld<NTL != 0>(m + i);
            d[u] = ld<NTL != 0>(v + i);
        }
#pragma unroll
        for (int u = 0; u < ITEMS; ++u) {
            const int64_t i = base + u * kThreads;
            if (i >= n) break;
            const T mm = 0.875f * c[u] + 0.125f * b[u];
            const T vv = 0.5f * d[u] + 0.5f * b[u] * b[u];
            st<NTS>(a[u] - 0.0625f * mm, p + i);
            st<NTS>(mm, m + i);
            st<NTS>(vv, v + i);
        }
    }
}

template <typename T, int ITEMS, int NTL, bool NTS>
__global__ __launch_bounds__(kThreads) void copy_kernel(T* dst, const T* src, int64_t n, int64_t tiles)
{
    for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        const int64_t base = tile * kThreads * ITEMS + threadIdx.x;
        T a[ITEMS];
#pragma unroll
        for (int u = 0; u < ITEMS; ++u) a[u] = ld<NTL == 1>(src + min(base + u * kThreads, n - 1));
#pragma unroll
        for (int u = 0; u < ITEMS; ++u) {
            const int64_t i = base + u * kThreads;
            if (i < n) st<NTS>(a[u], dst + i);
        }
    }
}

// Sums each thread's elements; one lane writes only if the sum equals a
// value it cannot take for the probe's data, so the loads are kept.
template <typename T, int ITEMS, int NTL, bool NTS>
__global__ __launch_bounds__(kThreads) void read_kernel(const T* src, int64_t n, int64_t tiles, float* sink)
{
    T s = {};
    for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        const int64_t base = tile * kThreads * ITEMS + threadIdx.x;
#pragma unroll
        for (int u = 0; u < ITEMS; ++u) s += ld<NTL == 1>(src + min(base + u * kThreads, n - 1));
    }
    if (s.x == -1.0e30f) sink[0] = s.y;
}

enum Mix { kRmw = 0, kCopy = 1, kRead = 2 };

struct Args {
    void* a;
    void* b;
    void* c;
    void* d;
    int64_t n16;
    int blocks;
};

template <typename T, int ITEMS, int NTL, bool NTS>
int launch(Mix mix, const Args& x, hipStream_t stream)
{
    constexpr int64_t per16 = 16 / sizeof(T);
    const int64_t n = x.n16 * per16;
    const int64_t tiles = (n + (int64_t)kThreads * ITEMS - 1) / ((int64_t)kThreads * ITEMS);
    const int64_t grid = x.blocks > 0 ? (x.blocks < tiles ? x.blocks : tiles) : tiles;
    if (grid > 0x7fffffff) return -1;
    const dim3 gd((unsigned)grid), bd(kThreads);
    if (mix == kRmw)
        hipLaunchKernelGGL((rmw_4r3w_kernel<T, ITEMS, NTL, NTS>), gd, bd, 0, stream, static_cast<T*>(x.a),
                           static_cast<const T*>(x.b), static_cast<T*>(x.c), static_cast<T*>(x.d), n, tiles);
    else if (mix == kCopy)
        hipLaunchKernelGGL((copy_kernel<T, ITEMS, NTL, NTS>), gd, bd, 0, stream, static_cast<T*>(x.a),
                           static_cast<const T*>(x.b), n, tiles);
    else
        hipLaunchKernelGGL((read_kernel<T, ITEMS, NTL, NTS>), gd, bd, 0, stream, static_cast<const T*>(x.a), n,
                           tiles, static_cast<float*>(x.b));
    return (int)hipGetLastError();
}

template <typename T, int ITEMS>
int by_hint(Mix mix, const Args& x, int ntl, int nts, hipStream_t s)
{
    if (ntl == 2) return nts ? launch<T, ITEMS, 2, true>(mix, x, s) : launch<T, ITEMS, 2, false>(mix, x, s);
    if (ntl == 1) return nts ? launch<T, ITEMS, 1, true>(mix, x, s) : launch<T, ITEMS, 1, false>(mix, x, s);
    return nts ? launch<T, ITEMS, 0, true>(mix, x, s) : launch<T, ITEMS, 0, false>(mix, x, s);
}

template <typename T>
int by_items(Mix mix, const Args& x, int items, int ntl, int nts, hipStream_t s)
{
    switch (items) {
    case 2: return by_hint<T, 2>(mix, x, ntl, nts, s);
    case 4: return by_hint<T, 4>(mix, x, ntl, nts, s);
    case 8: return by_hint<T, 8>(mix, x, ntl, nts, s);
    case 16: return by_hint<T, 16>(mix, x, ntl, nts, s);
    default: return -1;
    }
}

int dispatch(Mix mix, const Args& x, int width, int items, int ntl, int nts, hipStream_t s)
{
    if (width == 16) return by_items<f4>(mix, x, items, ntl, nts, s);
    if (width == 8) return by_items<f2>(mix, x, items, ntl, nts, s);
    return -1;
}

bool bad(const void* p) { return p == nullptr || (uintptr_t)p % 16 != 0; }
bool bad_n(int64_t n16) { return n16 < 1 || n16 > ((int64_t)1 << 31); }
bool bad_shape(int width, int items, int blocks, int ntl)
{
    return (width != 8 && width != 16) || (items != 2 && items != 4 && items != 8 && items != 16) || blocks < 0 ||
           ntl < 0 || ntl > 2;
}

}  // namespace

// All pointers are device memory, 16-byte aligned; n16 counts 16-byte
// elements per array (1 .. 2^31).  Return 0 on success, -1 on a bad
// argument (nothing launched), else the HIP error of the launch.

// The launch-shape family (see the top of this file).
extern "C" int gsprobe_rmw_4r3w_cfg(void* p, const void* g, void* m, void* v, int64_t n16, int width, int items,
                                    int nt_load, int nt_store, int blocks, hipStream_t stream)
{
    if (bad(p) || bad(g) || bad(m) || bad(v) || bad_n(n16) || bad_shape(width, items, blocks, nt_load)) return -1;
    return dispatch(kRmw, Args{p, const_cast<void*>(g), m, v, n16, blocks}, width, items, nt_load, nt_store, stream);
}

extern "C" int gsprobe_copy_cfg(void* dst, const void* src, int64_t n16, int width, int items, int nt_load,
                                int nt_store, int blocks, hipStream_t stream)
{
    if (bad(dst) || bad(src) || bad_n(n16) || bad_shape(width, items, blocks, nt_load)) return -1;
    return dispatch(kCopy, Args{dst, const_cast<void*>(src), nullptr, nullptr, n16, blocks}, width, items, nt_load,
                    nt_store, stream);
}

extern "C" int gsprobe_read_cfg(const void* src, int64_t n16, float* sink, int width, int items, int nt_load,
                                int blocks, hipStream_t stream)
{
    if (bad(src) || sink == nullptr || bad_n(n16) || bad_shape(width, items, blocks, nt_load)) return -1;
    return dispatch(kRead, Args{const_cast<void*>(src), sink, nullptr, nullptr, n16, blocks}, width, items, nt_load,
                    0, stream);
}

// The fixed shape the benchmark reports by default: 16-byte accesses, four
// in flight per thread, both hints, one tile per block.
extern "C" int gsprobe_rmw_4r3w(void* p, const void* g, void* m, void* v, int64_t n16, hipStream_t stream)
{
    return gsprobe_rmw_4r3w_cfg(p, g, m, v, n16, 16, 4, 1, 1, 0, stream);
}

extern "C" int gsprobe_copy(void* dst, const void* src, int64_t n16, hipStream_t stream)
{
    return gsprobe_copy_cfg(dst, src, n16, 16, 4, 1, 1, 0, stream);
}

extern "C" int gsprobe_read(const void* src, int64_t n16, float* sink, hipStream_t stream)
{
    return gsprobe_read_cfg(src, n16, sink, 16, 4, 1, 0, stream);
}
