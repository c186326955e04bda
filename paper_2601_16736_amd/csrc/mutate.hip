// Primitive-set mutation around the step: order-preserving pruning of every
// per-primitive array (theta, m, v, t), and appending clones with a fresh
// optimizer state.  Both are row copies driven by a per-wave row list in LDS,
// walked like the step's groups: consecutive lanes move consecutive chunks
// of a row, several chunks in flight per lane.
#include <algorithm>
#include <cstdio>
#include <cstring>

#include <rocprim/device/device_scan.hpp>

#include "device_common.h"
#include "trace.h"

namespace gs {

gs_status set_error(gs_status s, const char* msg);
void clear_error();

namespace {

#ifndef GS_MUT_UNIT
#define GS_MUT_UNIT 64
#endif
#ifndef GS_MUT_UNROLL
#define GS_MUT_UNROLL 8
#endif
// GS_MUT_UNIT: rows per wave of the prune.  GS_MUT_UNROLL: loads in flight
// per lane in the row moves.  Pruning 10 % of a 3M-row, 59-attribute FP32
// state took 838 us with 512 rows and 4 loads, 802 us with 128 and 8,
// 786 us with 64 and 8, 817 us with 256 and 8, and 846 us with 128 and 16.
constexpr int kMutUnit = GS_MUT_UNIT;
constexpr int kMaxArrays = 3 * GS_MAX_GROUPS + 1;
constexpr size_t kWsAlign = 256;

// One per-primitive array: rows of row_bytes, moved in chunks of w bytes
// (cpr chunks per row); consecutive rows start src_pitch / dst_pitch bytes
// apart (the row length, or a packed array's row).  src == nullptr: the
// destination rows are zeroed.
struct KArr {
    const char* src;
    char* dst;
    int64_t src_pitch;
    int64_t dst_pitch;
    int32_t row_bytes;
    int32_t w;
    int32_t cpr;
    int32_t pad;
};

struct KMut {
    KArr a[kMaxArrays];
    int32_t n_arr;
    int32_t pad;
    int64_t n;                 // source rows
    int64_t k;                 // append: new rows
    const uint8_t* keep;       // prune
    const int32_t* src_idx;    // append
    int32_t* counts;           // prune: kept rows per unit
    int32_t* offsets;          // prune: exclusive prefix of counts
    int32_t* kept_count;       // prune: total, device scalar
};

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <int W> struct Chunk;
template <> struct Chunk<16> { using T = u32x4; };
template <> struct Chunk<8> { using T = u32x2; };
template <> struct Chunk<4> { using T = uint32_t; };
template <> struct Chunk<2> { using T = uint16_t; };

// Moves the chunks of `nrows` rows: source row s_src[r] (skipped when < 0)
// to destination row dst0 + r.  Each lane issues U loads before its stores.
template <int W>
__device__ __forceinline__ void move_rows(const KArr& A, int nrows, const int* s_src, int64_t dst0, int lane)
{
    using T = typename Chunk<W>::T;
    constexpr bool NT = W >= 8;
    constexpr int U = GS_MUT_UNROLL;
    const int cpr = A.cpr;
    const int items = nrows * cpr;
    int r = lane / cpr;
    int c = lane - r * cpr;
    const int dr = kWave / cpr;
    const int dc = kWave - dr * cpr;
    for (int k0 = lane; k0 < items; k0 += U * kWave) {
        T x[U];
        int64_t d[U];
        bool ok[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool in = k0 + u * kWave < items;
            const int s = in ? s_src[r] : -1;
            ok[u] = in && (A.src == nullptr || s >= 0);
            d[u] = (dst0 + r) * A.dst_pitch + (int64_t)c * W;
            x[u] = T{};
            if (ok[u] && A.src != nullptr)
                x[u] = ld<T, NT>(reinterpret_cast<const T*>(A.src + (int64_t)s * A.src_pitch + (int64_t)c * W));
            r += dr;
            c += dc;
            if (c >= cpr) { c -= cpr; ++r; }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (ok[u]) st<T, NT>(reinterpret_cast<T*>(A.dst + d[u]), x[u]);
    }
}

__device__ __forceinline__ void move_all(const KMut& M, int nrows, const int* s_src, int64_t dst0, int lane)
{
    for (int j = 0; j < M.n_arr; ++j) {
        const KArr& A = M.a[j];
        switch (A.w) {
        case 16: move_rows<16>(A, nrows, s_src, dst0, lane); break;
        case 8: move_rows<8>(A, nrows, s_src, dst0, lane); break;
        case 4: move_rows<4>(A, nrows, s_src, dst0, lane); break;
        default: move_rows<2>(A, nrows, s_src, dst0, lane); break;
        }
    }
}

// kept rows of each unit of kMutUnit rows
__global__ __launch_bounds__(kBlock) void prune_count_kernel(KMut M)
{
    const int lane = threadIdx.x % kWave;
    const int64_t unit = (int64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
    const int64_t w0 = unit * kMutUnit;
    if (w0 >= M.n) return;
    int cnt = 0;
#pragma unroll
    for (int b = 0; b < kMutUnit / kWave; ++b) {
        const int64_t i = w0 + b * kWave + lane;
        cnt += __popcll(__ballot(i < M.n && M.keep[i] != 0));
    }
    if (lane == 0) M.counts[unit] = cnt;
}

// each unit stages its kept rows in order and moves them to offsets[unit]
__global__ __launch_bounds__(kBlock) void prune_move_kernel(KMut M, int64_t units)
{
    __shared__ int s_row[kWavesPerBlock][kMutUnit];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);   // the same on every lane
    const int lane = threadIdx.x % kWave;
    const int64_t unit = (int64_t)blockIdx.x * kWavesPerBlock + wave;
    if (unit >= units) return;
    const int nrows = build_rows_window<kMutUnit>(M.keep, M.n, unit * kMutUnit, s_row[wave], lane);
    const int64_t base = M.offsets[unit];
    if (unit == units - 1 && lane == 0) *M.kept_count = (int32_t)(base + nrows);
    if (nrows == 0) return;
    wave_sync();
    move_all(M, nrows, s_row[wave], base, lane);
}

__global__ void set_zero_kernel(int32_t* p) { *p = 0; }

// Rows per wave of the append: densification adds a few percent of the
// scene at a time, so the waves are kept short for enough of them to fill
// the device (150 000 new rows make 4 688 waves).  Appending 150 000 clone
// rows to a 3M-row, 59-attribute FP32 state took 49.1 us with 32 rows per
// wave, 53.4 us with 64 and 64.9 us with 16.
#ifndef GS_APPEND_UNIT
#define GS_APPEND_UNIT 32
#endif
constexpr int kAppendUnit = GS_APPEND_UNIT;
static_assert(kAppendUnit >= 1 && kAppendUnit <= 1024, "append unit");

// new rows n + [u*kAppendUnit, (u+1)*kAppendUnit) for each unit u of the
// wave: clones of src_idx, state zeroed.  The grid is capped at what one
// dispatch holds; a wave then takes every (grid waves)-th unit.
__global__ __launch_bounds__(kBlock) void append_kernel(KMut M, int64_t units)
{
    __shared__ int s_row[kWavesPerBlock][kAppendUnit];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);   // the same on every lane
    const int lane = threadIdx.x % kWave;
    for (int64_t u = (int64_t)blockIdx.x * kWavesPerBlock + wave; u < units;
         u += (int64_t)gridDim.x * kWavesPerBlock) {
        const int64_t j0 = u * kAppendUnit;
        const int nrows = (int)min((int64_t)kAppendUnit, M.k - j0);
        wave_sync();   // the previous unit's rows are done with
        for (int j = lane; j < nrows; j += kWave) {
            const int32_t s = M.src_idx[j0 + j];
            s_row[wave][j] = (s >= 0 && s < M.n) ? s : -1;
        }
        wave_sync();
        move_all(M, nrows, s_row[wave], M.n + j0, lane);
    }
}

size_t align_up(size_t x) { return (x + kWsAlign - 1) / kWsAlign * kWsAlign; }

int chunk_width(size_t row_bytes, size_t sp, size_t dp, const void* a, const void* b)
{
    for (int w = 16; w >= 2; w /= 2)
        if (row_bytes % (size_t)w == 0 && sp % (size_t)w == 0 && dp % (size_t)w == 0 &&
            (uintptr_t)a % (uintptr_t)w == 0 && (uintptr_t)b % (uintptr_t)w == 0)
            return w;
    return 0;
}

// src_pitch / dst_pitch 0: the row length
bool add_arr(KMut& M, const void* src, void* dst, size_t row_bytes, size_t src_pitch = 0, size_t dst_pitch = 0)
{
    const size_t sp = src_pitch != 0 ? src_pitch : row_bytes;
    const size_t dp = dst_pitch != 0 ? dst_pitch : row_bytes;
    const int w = chunk_width(row_bytes, sp, dp, src != nullptr ? src : dst, dst);
    if (w == 0 || M.n_arr >= kMaxArrays) return false;
    KArr& A = M.a[M.n_arr++];
    A.src = static_cast<const char*>(src);
    A.dst = static_cast<char*>(dst);
    A.src_pitch = (int64_t)sp;
    A.dst_pitch = (int64_t)dp;
    A.row_bytes = (int32_t)row_bytes;
    A.w = w;
    A.cpr = (int32_t)(row_bytes / (size_t)w);
    A.pad = 0;
    return true;
}

gs_status fail_fmt(const char* fmt, int a, int b = 0)
{
    char buf[256];
    snprintf(buf, sizeof buf, fmt, a, b);
    return set_error(GS_EINVAL, buf);
}

// elements from one row of a group to the next
int64_t row_pitch(const gs_group& G) { return G.row_stride != 0 ? G.row_stride : G.dim; }

gs_status check_group(const gs_group& G, int g, int64_t rows, size_t msz, bool need)
{
    if (G.dim < 1 || G.dim > 4096) return fail_fmt("group %d: dim = %d, must be in [1, 4096]", g, G.dim);
    if (G.row_stride != 0 && (G.row_stride < G.dim || G.row_stride > 65536))
        return fail_fmt("group %d: row_stride = %d, must be 0 or in [dim, 65536]", g, G.row_stride);
    if (row_pitch(G) * rows >= ((int64_t)1 << 40)) return fail_fmt("group %d: n * row stride too large", g);
    if (need && (G.param == nullptr || G.exp_avg == nullptr || G.exp_avg_sq == nullptr))
        return fail_fmt("group %d: param, exp_avg and exp_avg_sq must be non-NULL", g);
    if ((uintptr_t)G.param % 4 || (uintptr_t)G.exp_avg % msz || (uintptr_t)G.exp_avg_sq % msz)
        return fail_fmt("group %d: misaligned pointer (FP32 arrays need 4 bytes, BF16 moments %d)", g, (int)msz);
    return GS_OK;
}

size_t scan_temp_bytes(int64_t units)
{
    size_t bytes = 0;
    if (units <= 0) return 0;
    if (rocprim::exclusive_scan(nullptr, bytes, static_cast<const int32_t*>(nullptr), static_cast<int32_t*>(nullptr),
                                0, (size_t)units, rocprim::plus<int32_t>()) != hipSuccess)
        return 0;
    return bytes;
}

}  // namespace

}  // namespace gs

using namespace gs;

extern "C" size_t gs_prune_workspace_size(int64_t n)
{
    if (n <= 0) return 0;
    const int64_t units = (n + kMutUnit - 1) / kMutUnit;
    return kWsAlign + 2 * align_up((size_t)units * 4) + scan_temp_bytes(units);
}

extern "C" gs_status gs_prune(const uint8_t* keep, int64_t n, const gs_group* src, const gs_group* dst,
                              int32_t n_groups, int32_t moment_dtype, const int32_t* t_src, int32_t* t_dst,
                              int32_t* kept_count, void* ws, size_t ws_bytes, hipStream_t stream)
{
    clear_error();
    if (n < 0 || n >= ((int64_t)1 << 31)) return set_error(GS_EINVAL, "gs_prune: n must be in [0, 2^31)");
    if (src == nullptr || dst == nullptr) return set_error(GS_EINVAL, "gs_prune: src or dst is NULL");
    if (n_groups < 1 || n_groups > GS_MAX_GROUPS) return set_error(GS_EINVAL, "gs_prune: n_groups out of range");
    if (moment_dtype != GS_MOMENT_F32 && moment_dtype != GS_MOMENT_BF16)
        return set_error(GS_EINVAL, "gs_prune: unknown moment_dtype");
    if (kept_count == nullptr || (uintptr_t)kept_count % 4)
        return set_error(GS_EINVAL, "gs_prune: kept_count is NULL or misaligned");
    const size_t msz = moment_dtype == GS_MOMENT_BF16 ? 2 : 4;
    KMut M;
    memset(&M, 0, sizeof M);
    for (int g = 0; g < n_groups; ++g) {
        gs_status st = check_group(src[g], g, n, msz, n > 0);
        if (st == GS_OK) st = check_group(dst[g], g, n, msz, n > 0);
        if (st != GS_OK) return st;
        if (src[g].dim != dst[g].dim) return set_error(GS_EINVAL, "gs_prune: src and dst dims differ");
    }
    if (n == 0) {
        hipLaunchKernelGGL(set_zero_kernel, dim3(1), dim3(1), 0, stream, kept_count);
        const hipError_t e = hipGetLastError();
        return e == hipSuccess ? GS_OK : set_error(GS_EHIP, hipGetErrorString(e));
    }
    if (keep == nullptr || t_src == nullptr || t_dst == nullptr || (uintptr_t)t_src % 4 || (uintptr_t)t_dst % 4)
        return set_error(GS_EINVAL, "gs_prune: keep, t_src or t_dst is NULL or misaligned");
    const size_t need = gs_prune_workspace_size(n);
    if (ws == nullptr || ws_bytes < need) return set_error(GS_EINVAL, "gs_prune: workspace smaller than gs_prune_workspace_size(n)");
    for (int g = 0; g < n_groups; ++g) {
        const size_t d = (size_t)src[g].dim;
        const size_t sp = (size_t)row_pitch(src[g]), dp = (size_t)row_pitch(dst[g]);
        if (!add_arr(M, src[g].param, dst[g].param, d * 4, sp * 4, dp * 4) ||
            !add_arr(M, src[g].exp_avg, dst[g].exp_avg, d * msz, sp * msz, dp * msz) ||
            !add_arr(M, src[g].exp_avg_sq, dst[g].exp_avg_sq, d * msz, sp * msz, dp * msz))
            return set_error(GS_EINVAL, "gs_prune: misaligned rows");
    }
    if (!add_arr(M, t_src, t_dst, 4)) return set_error(GS_EINVAL, "gs_prune: misaligned step counts");
    const int64_t units = (n + kMutUnit - 1) / kMutUnit;
    char* base = reinterpret_cast<char*>(((uintptr_t)ws + kWsAlign - 1) / kWsAlign * kWsAlign);
    M.n = n;
    M.keep = keep;
    M.counts = reinterpret_cast<int32_t*>(base);
    M.offsets = reinterpret_cast<int32_t*>(base + align_up((size_t)units * 4));
    M.kept_count = kept_count;
    void* temp = base + 2 * align_up((size_t)units * 4);
    size_t temp_bytes = scan_temp_bytes(units);
    const unsigned blocks = (unsigned)((units + kWavesPerBlock - 1) / kWavesPerBlock);
    hipLaunchKernelGGL(prune_count_kernel, dim3(blocks), dim3(kBlock), 0, stream, M);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess)
        e = rocprim::exclusive_scan(temp, temp_bytes, M.counts, M.offsets, 0, (size_t)units, rocprim::plus<int32_t>(),
                                    stream);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(prune_move_kernel, dim3(blocks), dim3(kBlock), 0, stream, M, units);
        e = hipGetLastError();
    }
    return e == hipSuccess ? GS_OK : set_error(GS_EHIP, hipGetErrorString(e));
}

extern "C" gs_status gs_append(const gs_group* groups, int32_t n_groups, int32_t moment_dtype, int64_t n,
                               const int32_t* src_idx, int64_t k, int32_t* step_count, hipStream_t stream)
{
    clear_error();
    if (n < 0 || k < 0 || n + k >= ((int64_t)1 << 31))
        return set_error(GS_EINVAL, "gs_append: need n, k >= 0 and n + k < 2^31");
    if (groups == nullptr) return set_error(GS_EINVAL, "gs_append: groups is NULL");
    if (n_groups < 1 || n_groups > GS_MAX_GROUPS) return set_error(GS_EINVAL, "gs_append: n_groups out of range");
    if (moment_dtype != GS_MOMENT_F32 && moment_dtype != GS_MOMENT_BF16)
        return set_error(GS_EINVAL, "gs_append: unknown moment_dtype");
    const size_t msz = moment_dtype == GS_MOMENT_BF16 ? 2 : 4;
    for (int g = 0; g < n_groups; ++g) {
        const gs_status st = check_group(groups[g], g, n + k, msz, k > 0);
        if (st != GS_OK) return st;
    }
    if (k == 0) return GS_OK;
    if (src_idx == nullptr || step_count == nullptr || (uintptr_t)src_idx % 4 || (uintptr_t)step_count % 4)
        return set_error(GS_EINVAL, "gs_append: src_idx or step_count is NULL or misaligned");
    KMut M;
    memset(&M, 0, sizeof M);
    for (int g = 0; g < n_groups; ++g) {
        const size_t d = (size_t)groups[g].dim;
        const size_t p = (size_t)row_pitch(groups[g]);
        if (!add_arr(M, groups[g].param, groups[g].param, d * 4, p * 4, p * 4) ||
            !add_arr(M, nullptr, groups[g].exp_avg, d * msz, p * msz, p * msz) ||
            !add_arr(M, nullptr, groups[g].exp_avg_sq, d * msz, p * msz, p * msz))
            return set_error(GS_EINVAL, "gs_append: misaligned rows");
    }
    if (!add_arr(M, nullptr, step_count, 4)) return set_error(GS_EINVAL, "gs_append: misaligned step counts");
    M.n = n;
    M.k = k;
    M.src_idx = src_idx;
    const int64_t units = (k + kAppendUnit - 1) / kAppendUnit;
    const unsigned blocks = (unsigned)std::min<int64_t>((units + kWavesPerBlock - 1) / kWavesPerBlock, kMaxGridBlocks);
    hipLaunchKernelGGL(append_kernel, dim3(blocks), dim3(kBlock), 0, stream, M, units);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? GS_OK : set_error(GS_EHIP, hipGetErrorString(e));
}
