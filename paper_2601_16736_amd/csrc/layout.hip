// Spatial ordering of primitives (Morton / Z-order of the means) and row
// gather, used to lay a scene out so that the primitives one view sees sit in
// long contiguous index runs.
#include <cstring>

#include <rocprim/device/device_radix_sort.hpp>

#include "internal.h"

namespace gs {

gs_status set_error(gs_status s, const char* msg);
void clear_error();

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// order-preserving map of FP32 onto uint32 (for atomic min/max)
__device__ __forceinline__ uint32_t f2ord(float f)
{
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ float ord2f(uint32_t o)
{
    const uint32_t u = (o & 0x80000000u) ? (o & 0x7FFFFFFFu) : ~o;
    return __uint_as_float(u);
}

__global__ void bbox_init_kernel(uint32_t* box)
{
    if (threadIdx.x < 3) box[threadIdx.x] = 0xFFFFFFFFu;
    else if (threadIdx.x < 6) box[threadIdx.x] = 0u;
}

__global__ __launch_bounds__(256) void bbox_kernel(const float* __restrict__ means, int64_t ms, int64_t n,
                                                   uint32_t* box)
{
    uint32_t lo[3] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu}, hi[3] = {0u, 0u, 0u};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const float x = means[ms * i + a];
            if (x == x) {                      // NaN means take no part in the box
                const uint32_t o = f2ord(x);
                lo[a] = min(lo[a], o);
                hi[a] = max(hi[a], o);
            }
        }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        for (int off = 32; off > 0; off >>= 1) {
            lo[a] = min(lo[a], (uint32_t)__shfl_xor((int)lo[a], off));
            hi[a] = max(hi[a], (uint32_t)__shfl_xor((int)hi[a], off));
        }
    }
    // one set of six atomics per block, not per wave
    __shared__ uint32_t s_box[4][6];
    const int wave = threadIdx.x / 64;
    if ((threadIdx.x % 64) == 0) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            s_box[wave][a] = lo[a];
            s_box[wave][3 + a] = hi[a];
        }
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        const int a = threadIdx.x;
        uint32_t v = s_box[0][a];
        for (int w = 1; w < 4; ++w) v = a < 3 ? min(v, s_box[w][a]) : max(v, s_box[w][a]);
        if (a < 3) atomicMin(box + a, v);
        else atomicMax(box + a, v);
    }
}

// 10 bits spread to every third bit position
__device__ __forceinline__ uint32_t spread3(uint32_t x)
{
    x &= 0x3FFu;
    x = (x | (x << 16)) & 0x030000FFu;
    x = (x | (x << 8)) & 0x0300F00Fu;
    x = (x | (x << 4)) & 0x030C30C3u;
    x = (x | (x << 2)) & 0x09249249u;
    return x;
}

__global__ __launch_bounds__(256) void morton_kernel(const float* __restrict__ means, int64_t ms, int64_t n,
                                                     const uint32_t* box, uint32_t* __restrict__ keys,
                                                     int32_t* __restrict__ vals)
{
    float lo[3], scale[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        lo[a] = ord2f(box[a]);
        const float ext = ord2f(box[3 + a]) - lo[a];
        scale[a] = ext > 0.0f ? 1024.0f / ext : 0.0f;
    }
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        uint32_t q[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const float t = (means[ms * i + a] - lo[a]) * scale[a];
            q[a] = t >= 0.0f ? (uint32_t)min(t, 1023.0f) : 0u;        // NaN -> 0
        }
        keys[i] = spread3(q[0]) | (spread3(q[1]) << 1) | (spread3(q[2]) << 2);
        vals[i] = (int32_t)i;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void gather_kernel(const T* __restrict__ src, T* __restrict__ dst,
                                                     const int32_t* __restrict__ perm, int64_t n, int64_t per_row)
{
    const int64_t total = n * per_row;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total; k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = k / per_row;
        const int64_t c = k - i * per_row;
        const int32_t p = perm[i];
        if ((uint32_t)p < (uint64_t)n) dst[k] = src[(int64_t)p * per_row + c];   // out-of-range entries are skipped
    }
}

size_t sort_temp_bytes(int64_t n)
{
    size_t bytes = 0;
    (void)rocprim::radix_sort_pairs(nullptr, bytes, (const uint32_t*)nullptr, (uint32_t*)nullptr,
                                    (const int32_t*)nullptr, (int32_t*)nullptr, (size_t)n, 0, 30);
    return bytes;
}

}  // namespace

}  // namespace gs

using namespace gs;

extern "C" size_t gs_spatial_order_workspace_size(int64_t n)
{
    if (n < 0) return 0;
    return kAlign + 3 * align_up((size_t)n * 4) + align_up(sort_temp_bytes(n));
}

extern "C" gs_status gs_spatial_order(const float* means, int64_t means_stride, int64_t n, int32_t* perm,
                                      void* workspace, size_t workspace_bytes, hipStream_t stream)
{
    clear_error();
    if (n < 0 || n >= ((int64_t)1 << 31)) return set_error(GS_EINVAL, "gs_spatial_order: n must be in [0, 2^31)");
    const int64_t ms = means_stride == 0 ? 3 : means_stride;
    if (ms < 3 || ms > 65536 || ms * n >= ((int64_t)1 << 40))
        return set_error(GS_EINVAL, "gs_spatial_order: means_stride must be 0 or in [3, 65536]");
    if (n == 0) return GS_OK;
    if (means == nullptr || perm == nullptr || workspace == nullptr)
        return set_error(GS_EINVAL, "gs_spatial_order: means, perm and workspace are required");
    if ((uintptr_t)means % 4 || (uintptr_t)perm % 4 || (uintptr_t)workspace % kAlign)
        return set_error(GS_EINVAL, "gs_spatial_order: misaligned pointer (workspace needs 256 bytes)");
    if (workspace_bytes < gs_spatial_order_workspace_size(n))
        return set_error(GS_EINVAL, "gs_spatial_order: workspace too small");
    char* ws = static_cast<char*>(workspace);
    uint32_t* box = reinterpret_cast<uint32_t*>(ws);
    uint32_t* keys_in = reinterpret_cast<uint32_t*>(ws + kAlign);
    uint32_t* keys_out = reinterpret_cast<uint32_t*>(ws + kAlign + align_up((size_t)n * 4));
    int32_t* vals_in = reinterpret_cast<int32_t*>(ws + kAlign + 2 * align_up((size_t)n * 4));
    void* temp = ws + kAlign + 3 * align_up((size_t)n * 4);
    size_t temp_bytes = sort_temp_bytes(n);
    hipLaunchKernelGGL(bbox_init_kernel, dim3(1), dim3(64), 0, stream, box);
    const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(bbox_kernel, dim3(std::min(grid, 512u)), dim3(256), 0, stream, means, ms, n, box);
    hipLaunchKernelGGL(morton_kernel, dim3(grid), dim3(256), 0, stream, means, ms, n, box, keys_in, vals_in);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(GS_EHIP, hipGetErrorString(e));
    e = rocprim::radix_sort_pairs(temp, temp_bytes, keys_in, keys_out, vals_in, perm, (size_t)n, 0, 30, stream);
    if (e != hipSuccess) return set_error(GS_EHIP, hipGetErrorString(e));
    return GS_OK;
}

extern "C" gs_status gs_gather_rows(const void* src, void* dst, const int32_t* perm, int64_t n, int64_t row_bytes,
                                    hipStream_t stream)
{
    clear_error();
    if (n < 0 || n >= ((int64_t)1 << 31) || row_bytes < 1)
        return set_error(GS_EINVAL, "gs_gather_rows: bad n or row_bytes");
    if (n == 0) return GS_OK;
    if (src == nullptr || dst == nullptr || perm == nullptr)
        return set_error(GS_EINVAL, "gs_gather_rows: NULL pointer");
    if (src == dst) return set_error(GS_EINVAL, "gs_gather_rows: src and dst must differ");
    const uintptr_t align = (uintptr_t)src | (uintptr_t)dst | (uintptr_t)row_bytes;
    const unsigned grid = 8192;
    if (align % 16 == 0)
        hipLaunchKernelGGL(gather_kernel<uint4>, dim3(grid), dim3(256), 0, stream, (const uint4*)src, (uint4*)dst, perm,
                           n, row_bytes / 16);
    else if (align % 4 == 0)
        hipLaunchKernelGGL(gather_kernel<uint32_t>, dim3(grid), dim3(256), 0, stream, (const uint32_t*)src,
                           (uint32_t*)dst, perm, n, row_bytes / 4);
    else
        hipLaunchKernelGGL(gather_kernel<uint8_t>, dim3(grid), dim3(256), 0, stream, (const uint8_t*)src,
                           (uint8_t*)dst, perm, n, row_bytes);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? GS_OK : set_error(GS_EHIP, hipGetErrorString(e));
}
