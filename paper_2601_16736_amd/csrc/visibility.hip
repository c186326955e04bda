// Per-view visibility (frustum/radius cull of the projected means) and
// compaction of the visible indices (gfx950).
//
// Each block of 256 threads covers 4096 consecutive primitives in sixteen
// rounds.  Per round a wave ballots its 64 predicates; the block adds up its
// 64 (round, wave) counts and reserves one contiguous range of the index list
// with a single atomic, so the list holds ascending runs of up to 4096
// primitives and the one shared counter sees n/4096 atomics.
#include "device_common.h"
#include "predicate.h"

namespace gs {

#ifndef GS_VIS_ROUNDS
#define GS_VIS_ROUNDS 16
#endif
constexpr int kVisRounds = GS_VIS_ROUNDS;
constexpr int kVisPerBlock = kBlock * kVisRounds;
static_assert(kVisRounds * kWavesPerBlock <= kWave, "the block's (round, wave) counts fit one wave");

// Appends the visible primitives of this block (flags per round) to idx.
__device__ __forceinline__ void block_append(const bool (&vis)[kVisRounds], int64_t first, int32_t* idx,
                                             int32_t* count)
{
    __shared__ int s_cnt[kVisRounds * kWavesPerBlock];
    __shared__ int s_base;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);   // the same on every lane
    const int lane = threadIdx.x % kWave;
    uint64_t bal[kVisRounds];
#pragma unroll
    for (int s = 0; s < kVisRounds; ++s) {
        bal[s] = __ballot(vis[s]);
        if (lane == 0) s_cnt[s * kWavesPerBlock + wave] = __popcll(bal[s]);
    }
    __syncthreads();
    if (threadIdx.x < kWave) {
        // exclusive prefix of the (round, wave) counts across wave 0
        const int c = threadIdx.x < kVisRounds * kWavesPerBlock ? s_cnt[threadIdx.x] : 0;
        int incl = c;
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
            const int y = __shfl_up(incl, off);
            if ((int)threadIdx.x >= off) incl += y;
        }
        if (threadIdx.x < kVisRounds * kWavesPerBlock) s_cnt[threadIdx.x] = incl - c;
        const int total = __shfl(incl, kWave - 1);
        if (threadIdx.x == 0) s_base = total > 0 ? atomicAdd(count, total) : 0;
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < kVisRounds; ++s) {
        if (vis[s]) {
            const int off = s_base + s_cnt[s * kWavesPerBlock + wave] + lanes_below(bal[s]);
            idx[off] = (int32_t)(first + s * kBlock + threadIdx.x);
        }
    }
}

template <bool RADIUS>
__global__ __launch_bounds__(kBlock) void visibility_kernel(const float* __restrict__ means, int64_t ms,
                                                            const float* __restrict__ radius, int64_t n,
                                                            KCamera cam, uint8_t* __restrict__ mask,
                                                            int32_t* __restrict__ idx, int32_t* count)
{
    const int64_t first = (int64_t)blockIdx.x * kVisPerBlock;
    // every round's loads first (indices past the end read the last element
    // and are discarded), so the 16 rounds' loads are in flight together
    float x[kVisRounds], y[kVisRounds], z[kVisRounds], rho[kVisRounds];
#pragma unroll
    for (int s = 0; s < kVisRounds; ++s) {
        const int64_t i = min(first + s * kBlock + threadIdx.x, n - 1);
        x[s] = means[ms * i];
        y[s] = means[ms * i + 1];
        z[s] = means[ms * i + 2];
        rho[s] = RADIUS ? radius[i] : 0.0f;
    }
    bool vis[kVisRounds];
#pragma unroll
    for (int s = 0; s < kVisRounds; ++s) {
        const int64_t i = first + s * kBlock + threadIdx.x;
        vis[s] = i < n && visible_pred(x[s], y[s], z[s], RADIUS ? &rho[s] : nullptr, cam);
    }
    if (mask != nullptr) {
#pragma unroll
        for (int s = 0; s < kVisRounds; ++s) {
            const int64_t i = first + s * kBlock + threadIdx.x;
            if (i < n) mask[i] = (uint8_t)vis[s];
        }
    }
    if (idx != nullptr) block_append(vis, first, idx, count);
}

// Several views in one pass: bit v of a primitive's word is its predicate in
// view v; the union (any bit) feeds the mask and the index list.  The means
// are read once for all views.
template <bool RADIUS>
__global__ __launch_bounds__(kBlock) void visibility_multi_kernel(const float* __restrict__ means, int64_t ms,
                                                                  const float* __restrict__ radius, int64_t n,
                                                                  KCameras cams, uint8_t* __restrict__ mask,
                                                                  uint32_t* __restrict__ bits,
                                                                  int32_t* __restrict__ idx, int32_t* count)
{
    const int64_t first = (int64_t)blockIdx.x * kVisPerBlock;
    float x[kVisRounds], y[kVisRounds], z[kVisRounds], rho[kVisRounds];
#pragma unroll
    for (int s = 0; s < kVisRounds; ++s) {
        const int64_t i = min(first + s * kBlock + threadIdx.x, n - 1);
        x[s] = means[ms * i];
        y[s] = means[ms * i + 1];
        z[s] = means[ms * i + 2];
        rho[s] = RADIUS ? radius[i] : 0.0f;
    }
    uint32_t b[kVisRounds];
#pragma unroll
    for (int s = 0; s < kVisRounds; ++s) b[s] = 0u;
    for (int v = 0; v < cams.n; ++v) {
        const KCamera& c = cams.c[v];
#pragma unroll
        for (int s = 0; s < kVisRounds; ++s)
            if (visible_pred(x[s], y[s], z[s], RADIUS ? &rho[s] : nullptr, c)) b[s] |= 1u << v;
    }
    bool vis[kVisRounds];
#pragma unroll
    for (int s = 0; s < kVisRounds; ++s) {
        const int64_t i = first + s * kBlock + threadIdx.x;
        vis[s] = i < n && b[s] != 0u;
        if (i < n) {
            if (mask != nullptr) mask[i] = (uint8_t)vis[s];
            if (bits != nullptr) bits[i] = b[s];
        }
    }
    if (idx != nullptr) block_append(vis, first, idx, count);
}

__global__ __launch_bounds__(kBlock) void compact_kernel(const uint8_t* __restrict__ mask, int64_t n,
                                                         int32_t* __restrict__ idx, int32_t* count)
{
    const int64_t first = (int64_t)blockIdx.x * kVisPerBlock;
    uint8_t m[kVisRounds];
#pragma unroll
    for (int s = 0; s < kVisRounds; ++s) m[s] = mask[min(first + s * kBlock + threadIdx.x, n - 1)];
    bool vis[kVisRounds];
#pragma unroll
    for (int s = 0; s < kVisRounds; ++s) vis[s] = first + s * kBlock + threadIdx.x < n && m[s] != 0;
    block_append(vis, first, idx, count);
}

// Clears the visible count before the appends (a kernel rather than a memset
// so the sequence can sit inside a captured graph).
__global__ void clear_count_kernel(int32_t* count)
{
    if (threadIdx.x == 0) count[0] = 0;
}

hipError_t launch_visibility(const float* means, int64_t ms, const float* radius, int64_t n, const KCamera& cam,
                             uint8_t* mask, int32_t* idx, int32_t* count, hipStream_t stream)
{
    if (idx != nullptr) {
        hipLaunchKernelGGL(clear_count_kernel, dim3(1), dim3(kWave), 0, stream, count);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (n == 0) return hipSuccess;
    const unsigned blocks = (unsigned)((n + kVisPerBlock - 1) / kVisPerBlock);
    if (radius != nullptr)
        hipLaunchKernelGGL(visibility_kernel<true>, dim3(blocks), dim3(kBlock), 0, stream, means, ms, radius, n,
                           cam, mask, idx, count);
    else
        hipLaunchKernelGGL(visibility_kernel<false>, dim3(blocks), dim3(kBlock), 0, stream, means, ms, radius, n,
                           cam, mask, idx, count);
    return hipGetLastError();
}

hipError_t launch_compact(const uint8_t* mask, int64_t n, int32_t* idx, int32_t* count, hipStream_t stream)
{
    hipLaunchKernelGGL(clear_count_kernel, dim3(1), dim3(kWave), 0, stream, count);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || n == 0) return e;
    const unsigned blocks = (unsigned)((n + kVisPerBlock - 1) / kVisPerBlock);
    hipLaunchKernelGGL(compact_kernel, dim3(blocks), dim3(kBlock), 0, stream, mask, n, idx, count);
    return hipGetLastError();
}

hipError_t launch_visibility_multi(const float* means, int64_t ms, const float* radius, int64_t n,
                                   const KCameras& cams, uint8_t* mask, uint32_t* bits, int32_t* idx, int32_t* count,
                                   hipStream_t stream)
{
    if (idx != nullptr) {
        hipLaunchKernelGGL(clear_count_kernel, dim3(1), dim3(kWave), 0, stream, count);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (n == 0) return hipSuccess;
    const unsigned blocks = (unsigned)((n + kVisPerBlock - 1) / kVisPerBlock);
    if (radius != nullptr)
        hipLaunchKernelGGL(visibility_multi_kernel<true>, dim3(blocks), dim3(kBlock), 0, stream, means, ms, radius,
                           n, cams, mask, bits, idx, count);
    else
        hipLaunchKernelGGL(visibility_multi_kernel<false>, dim3(blocks), dim3(kBlock), 0, stream, means, ms, radius,
                           n, cams, mask, bits, idx, count);
    return hipGetLastError();
}

}  // namespace gs
