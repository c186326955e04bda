// Streaming ceilings of the HBM on the device the benchmark runs on: plain
// contiguous kernels with no method arithmetic, timed beside the AdamW-GS
// step so that its bandwidth can be read against what the memory system
// delivers for the same access mix, not only against the datasheet peak.
// Measurement support only: built as a library of its own, never linked
// into libgsopt.
//
// Three access mixes over 16-byte-aligned arrays (and, further down, the
// masked step's own pattern of rows):
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

// ---------------------------------------------------------------- rows
// The masked step's access pattern without its arithmetic.  Each wave takes
// a window of primitives (32 in the step's shape) and keeps, in order, those
// whose mask byte is set; it bumps their 4-byte counters, then passes over
// each group: its lanes walk the kept rows' (row, chunk) items, a chunk
// being 4 floats when the group's width is a multiple of 4 and 1 float
// otherwise, and each lane issues the loads of its items (attribute,
// gradient and two moments; U chunk items or 2U single ones in flight)
// before it writes three back.
// 16-byte accesses carry the non-temporal hint, 4-byte ones do not.  The
// values written are plain blends of the ones read.
constexpr int kRowsWaves = 4;
constexpr int kMaxRowGroups = 8;

struct RowsArgs {
    const uint8_t* mask;
    int32_t* t;
    float* p[kMaxRowGroups];
    const float* g[kMaxRowGroups];
    void* m[kMaxRowGroups];
    void* v[kMaxRowGroups];
    int32_t dim[kMaxRowGroups];
    int32_t n_groups;
    int64_t n;
};

typedef uint32_t u2x32 __attribute__((ext_vector_type(2)));

// The values written back: blends of the ones read for FP32 moments; for
// BF16 moments (4 packed in 8 bytes, or 1 in 2 bytes) the bits read with
// each element's lowest bit flipped.
__device__ __forceinline__ f4 mix_m(f4 x, f4 b) { return 0.875f * x + 0.125f * b; }
__device__ __forceinline__ float mix_m(float x, float b) { return 0.875f * x + 0.125f * b; }
__device__ __forceinline__ f4 mix_v(f4 y, f4 b) { return 0.5f * y + 0.5f * b * b; }
__device__ __forceinline__ float mix_v(float y, float b) { return 0.5f * y + 0.5f * b * b; }
__device__ __forceinline__ u2x32 mix_m(u2x32 x, f4) { return x ^ 0x00010001u; }
__device__ __forceinline__ uint16_t mix_m(uint16_t x, float) { return (uint16_t)(x ^ 1u); }
__device__ __forceinline__ u2x32 mix_v(u2x32 y, f4) { return y ^ 0x00010001u; }
__device__ __forceinline__ uint16_t mix_v(uint16_t y, float) { return (uint16_t)(y ^ 1u); }

// T: an attribute chunk (V floats); MT: the moments of a chunk.  Accesses of
// 8 bytes and more carry the non-temporal hint.
template <typename T, typename MT, int V, int U>
__device__ __forceinline__ void rows_group(float* P, const float* G, void* M, void* W, int dim, const int* rows,
                                           int nrows, int lane)
{
    constexpr bool NT = sizeof(T) >= 8;
    constexpr bool NTM = sizeof(MT) >= 8;
    const int cpr = dim / V;
    const int items = nrows * cpr;
    int r = lane / cpr, c = lane - (lane / cpr) * cpr;
    const int dr = 64 / cpr, dc = 64 - (64 / cpr) * cpr;
    for (int k0 = lane; k0 < items; k0 += U * 64) {
        T a[U], b[U];
        MT x[U], y[U];
        int64_t e[U];
        bool ok[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            ok[u] = k0 + u * 64 < items;
            e[u] = ok[u] ? ((int64_t)rows[r] * dim + c * V) / V : 0;
            if (ok[u]) {
                a[u] = ld<NT>(reinterpret_cast<const T*>(P) + e[u]);
                b[u] = ld<NT>(reinterpret_cast<const T*>(G) + e[u]);
                x[u] = ld<NTM>(static_cast<const MT*>(M) + e[u]);
                y[u] = ld<NTM>(static_cast<const MT*>(W) + e[u]);
            }
            r += dr;
            c += dc;
            if (c >= cpr) {
                c -= cpr;
                ++r;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (!ok[u]) continue;
            st<NT>(a[u] - 0.0625f * b[u], reinterpret_cast<T*>(P) + e[u]);
            st<NTM>(mix_m(x[u], b[u]), static_cast<MT*>(M) + e[u]);
            st<NTM>(mix_v(y[u], b[u]), static_cast<MT*>(W) + e[u]);
        }
    }
}

template <int WIN, int U, bool BF16>
__global__ __launch_bounds__(kThreads) void rows_kernel(RowsArgs A)
{
    constexpr int R = (WIN + 63) / 64;
    __shared__ int s_row[kRowsWaves][WIN];
    const int wave = threadIdx.x / 64;
    const int lane = threadIdx.x % 64;
    const int64_t w0 = ((int64_t)blockIdx.x * kRowsWaves + wave) * WIN;
    if (w0 >= A.n) return;
    int nrows = 0;
#pragma unroll
    for (int b = 0; b < R; ++b) {
        const int j = b * 64 + lane;
        const int64_t i = w0 + j;
        const bool keep = j < WIN && i < A.n && A.mask[i] != 0;
        const uint64_t bal = __ballot(keep);
        if (keep) s_row[wave][nrows + __popcll(bal & ((1ull << lane) - 1))] = (int)i;
        nrows += __popcll(bal);
    }
    if (nrows == 0) return;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int j = lane; j < nrows; j += 64) {
        const int row = s_row[wave][j];
        A.t[row] = A.t[row] + 1;
    }
    for (int gi = 0; gi < A.n_groups; ++gi) {
        if (A.dim[gi] % 4 == 0) {
            if constexpr (BF16)
                rows_group<f4, u2x32, 4, U>(A.p[gi], A.g[gi], A.m[gi], A.v[gi], A.dim[gi], s_row[wave], nrows, lane);
            else
                rows_group<f4, f4, 4, U>(A.p[gi], A.g[gi], A.m[gi], A.v[gi], A.dim[gi], s_row[wave], nrows, lane);
        } else {
            if constexpr (BF16)
                rows_group<float, uint16_t, 1, 2 * U>(A.p[gi], A.g[gi], A.m[gi], A.v[gi], A.dim[gi], s_row[wave],
                                                      nrows, lane);
            else
                rows_group<float, float, 1, 2 * U>(A.p[gi], A.g[gi], A.m[gi], A.v[gi], A.dim[gi], s_row[wave],
                                                   nrows, lane);
        }
    }
}

template <int WIN, bool BF16>
int rows_launch(const RowsArgs& A, int items, hipStream_t stream)
{
    const int64_t units = (A.n + WIN - 1) / WIN;
    const dim3 gd((unsigned)((units + kRowsWaves - 1) / kRowsWaves)), bd(kThreads);
    switch (items) {
    case 2: hipLaunchKernelGGL((rows_kernel<WIN, 2, BF16>), gd, bd, 0, stream, A); break;
    case 4: hipLaunchKernelGGL((rows_kernel<WIN, 4, BF16>), gd, bd, 0, stream, A); break;
    case 8: hipLaunchKernelGGL((rows_kernel<WIN, 8, BF16>), gd, bd, 0, stream, A); break;
    default: return -1;
    }
    return (int)hipGetLastError();
}

template <bool BF16>
int rows_by_window(const RowsArgs& A, int window, int items, hipStream_t stream)
{
    switch (window) {
    case 32: return rows_launch<32, BF16>(A, items, stream);
    case 64: return rows_launch<64, BF16>(A, items, stream);
    case 128: return rows_launch<128, BF16>(A, items, stream);
    case 256: return rows_launch<256, BF16>(A, items, stream);
    default: return -1;
    }
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

// The masked step's access pattern (rows_kernel above).  mask: n bytes
// (device), t: n counters (device); p, g, m, v: host arrays of n_groups
// (1 .. 8) device pointers to arrays of n x dims[k] elements (dims 1 .. 64):
// FP32 attributes and gradients, moments in FP32 (bf16 = 0) or BF16 (1);
// where dims[k] is a multiple of 4, the attribute and gradient arrays are
// 16-byte aligned and the moment arrays 16-byte (FP32) or 8-byte (BF16)
// aligned; n in 1 .. 2^31 - 1; window: primitives per wave (32, 64, 128 or
// 256); items: chunk items in flight per lane (2, 4 or 8; twice that for
// single elements).  Return 0, -1 on a bad argument (nothing launched), else
// the HIP error of the launch.
extern "C" int gsprobe_rows_4r3w_cfg(const uint8_t* mask, int32_t* t, float* const* p, const float* const* g,
                                     void* const* m, void* const* v, const int32_t* dims, int n_groups, int64_t n,
                                     int window, int items, int bf16, hipStream_t stream)
{
    if (mask == nullptr || t == nullptr || p == nullptr || g == nullptr || m == nullptr || v == nullptr ||
        dims == nullptr || n_groups < 1 || n_groups > kMaxRowGroups || n < 1 || n > 0x7fffffff ||
        (items != 2 && items != 4 && items != 8) || (bf16 != 0 && bf16 != 1))
        return -1;
    const uintptr_t malign = bf16 ? 8 : 16;
    RowsArgs A{};
    A.mask = mask;
    A.t = t;
    A.n_groups = n_groups;
    A.n = n;
    for (int k = 0; k < n_groups; ++k) {
        if (dims[k] < 1 || dims[k] > 64 || p[k] == nullptr || g[k] == nullptr || m[k] == nullptr || v[k] == nullptr)
            return -1;
        if (dims[k] % 4 == 0 && (bad(p[k]) || bad(g[k]) || (uintptr_t)m[k] % malign != 0 ||
                                 (uintptr_t)v[k] % malign != 0))
            return -1;
        A.p[k] = p[k];
        A.g[k] = g[k];
        A.m[k] = m[k];
        A.v[k] = v[k];
        A.dim[k] = dims[k];
    }
    return bf16 ? rows_by_window<true>(A, window, items, stream) : rows_by_window<false>(A, window, items, stream);
}

// The shape of the masked FP32 step: windows of 32, four chunk items in flight.
extern "C" int gsprobe_rows_4r3w(const uint8_t* mask, int32_t* t, float* const* p, const float* const* g,
                                 void* const* m, void* const* v, const int32_t* dims, int n_groups, int64_t n,
                                 hipStream_t stream)
{
    return gsprobe_rows_4r3w_cfg(mask, t, p, g, m, v, dims, n_groups, n, 32, 4, 0, stream);
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
