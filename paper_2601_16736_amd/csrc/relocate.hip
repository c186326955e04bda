// Relocation state reset: the k primitives with the smallest key (ties to the
// lower index) get zero moments (and optionally a zero step count), the
// optimizer-side half of relocating dead primitives.
//
// Selection is a most-significant-digit radix select over the keys mapped to
// order-preserving uint32: four 8-bit passes narrow the key of the k-th
// smallest element (K) and the number r of elements equal to K that still
// belong to the selection.  An ordered block scan then picks every key < K
// and the first r keys == K in index order, writing the selected indices in
// ascending order; a last kernel zeroes their state rows.
#include <cstring>

#include "device_common.h"

namespace gs {

gs_status set_error(gs_status s, const char* msg);
void clear_error();

namespace {

constexpr int kRelPerThread = 16;
constexpr int kRelPerBlock = kBlock * kRelPerThread;   // 4096 keys per block
constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct SelectState {
    uint32_t prefix;   // key bits decided so far
    uint32_t mask;     // which bits are decided
    int32_t rank;      // elements still to take among those matching prefix
    int32_t pad;
};

// -0.0 and +0.0 compare equal, so both map to the key of +0.0
__device__ __forceinline__ uint32_t key_ord(float f)
{
    const uint32_t u = f == 0.0f ? 0u : __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__global__ void select_init_kernel(SelectState* st, uint32_t* hist, int32_t k)
{
    if (threadIdx.x == 0) {
        st->prefix = 0u;
        st->mask = 0u;
        st->rank = k;
        st->pad = 0;
    }
    hist[threadIdx.x] = 0u;   // 256 threads
}

__global__ __launch_bounds__(kBlock) void select_hist_kernel(const float* __restrict__ key, int64_t n,
                                                             const SelectState* st, int shift, uint32_t* hist)
{
    __shared__ uint32_t s_hist[256];
    s_hist[threadIdx.x] = 0u;
    __syncthreads();
    const uint32_t prefix = st->prefix, mask = st->mask;
    const int64_t first = (int64_t)blockIdx.x * kRelPerBlock;
#pragma unroll 4
    for (int j = 0; j < kRelPerThread; ++j) {
        const int64_t i = first + (int64_t)j * kBlock + threadIdx.x;
        if (i < n) {
            const uint32_t o = key_ord(key[i]);
            if ((o & mask) == prefix) atomicAdd(&s_hist[(o >> shift) & 0xFFu], 1u);
        }
    }
    __syncthreads();
    const uint32_t c = s_hist[threadIdx.x];
    if (c) atomicAdd(&hist[threadIdx.x], c);
}

// One block of 256 threads: finds the digit bucket holding the rank-th
// element, narrows the state, clears the histogram for the next pass.
__global__ void select_digit_kernel(SelectState* st, uint32_t* hist, int shift)
{
    __shared__ uint32_t s_inc[256];
    const uint32_t c = hist[threadIdx.x];
    s_inc[threadIdx.x] = c;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const uint32_t y = threadIdx.x >= (unsigned)off ? s_inc[threadIdx.x - off] : 0u;
        __syncthreads();
        s_inc[threadIdx.x] += y;
        __syncthreads();
    }
    const uint32_t rank = (uint32_t)st->rank;
    const uint32_t before = s_inc[threadIdx.x] - c;
    __syncthreads();
    // the bucket where the running count first reaches `rank`
    if (rank > 0 && before < rank && s_inc[threadIdx.x] >= rank) {
        st->prefix |= (uint32_t)threadIdx.x << shift;
        st->mask |= 0xFFu << shift;
        st->rank = (int32_t)(rank - before);
    }
    hist[threadIdx.x] = 0u;
}

// Per block: keys below K and keys equal to K.
__global__ __launch_bounds__(kBlock) void select_count_kernel(const float* __restrict__ key, int64_t n,
                                                              const SelectState* st, int32_t* lt, int32_t* eq)
{
    __shared__ int s_lt[kWavesPerBlock], s_eq[kWavesPerBlock];
    const uint32_t K = st->prefix;
    const bool any = st->rank > 0;
    const int64_t first = (int64_t)blockIdx.x * kRelPerBlock;
    int nl = 0, ne = 0;
    for (int j = 0; j < kRelPerThread; ++j) {
        const int64_t i = first + (int64_t)j * kBlock + threadIdx.x;
        if (i < n && any) {
            const uint32_t o = key_ord(key[i]);
            nl += o < K;
            ne += o == K;
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        nl += __shfl_xor(nl, off);
        ne += __shfl_xor(ne, off);
    }
    const int wave = threadIdx.x / kWave;
    if (threadIdx.x % kWave == 0) {
        s_lt[wave] = nl;
        s_eq[wave] = ne;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int a = 0, b = 0;
        for (int w = 0; w < kWavesPerBlock; ++w) {
            a += s_lt[w];
            b += s_eq[w];
        }
        lt[blockIdx.x] = a;
        eq[blockIdx.x] = b;
    }
}

// One block: in-place exclusive scans of the per-block counts.
__global__ void select_scan_kernel(int32_t* lt, int32_t* eq, int nblocks)
{
    __shared__ int s_a[kBlock], s_b[kBlock];
    __shared__ int s_carry_a, s_carry_b;
    if (threadIdx.x == 0) {
        s_carry_a = 0;
        s_carry_b = 0;
    }
    __syncthreads();
    for (int base = 0; base < nblocks; base += kBlock) {
        const int i = base + threadIdx.x;
        const int a = i < nblocks ? lt[i] : 0;
        const int b = i < nblocks ? eq[i] : 0;
        s_a[threadIdx.x] = a;
        s_b[threadIdx.x] = b;
        __syncthreads();
        for (int off = 1; off < kBlock; off <<= 1) {
            const int ya = threadIdx.x >= (unsigned)off ? s_a[threadIdx.x - off] : 0;
            const int yb = threadIdx.x >= (unsigned)off ? s_b[threadIdx.x - off] : 0;
            __syncthreads();
            s_a[threadIdx.x] += ya;
            s_b[threadIdx.x] += yb;
            __syncthreads();
        }
        if (i < nblocks) {
            lt[i] = s_carry_a + s_a[threadIdx.x] - a;
            eq[i] = s_carry_b + s_b[threadIdx.x] - b;
        }
        __syncthreads();
        if (threadIdx.x == kBlock - 1) {
            s_carry_a += s_a[threadIdx.x];
            s_carry_b += s_b[threadIdx.x];
        }
        __syncthreads();
    }
}

// Per block, in index order: take every key < K and the first `rank` keys
// equal to K; write their indices at their place in the ascending list.
__global__ __launch_bounds__(kBlock) void select_write_kernel(const float* __restrict__ key, int64_t n,
                                                              const SelectState* st, const int32_t* lt_before,
                                                              const int32_t* eq_before, int32_t* sel)
{
    __shared__ int s_cnt[2][kWavesPerBlock];
    __shared__ int s_run_eq, s_run_sel;
    const uint32_t K = st->prefix;
    const int rank = st->rank;
    if (rank <= 0) return;
    const int wave = threadIdx.x / kWave;
    const int lane = threadIdx.x % kWave;
    const int64_t first = (int64_t)blockIdx.x * kRelPerBlock;
    const int eq0 = eq_before[blockIdx.x];
    // selected before this block: all smaller keys, plus the equal ones that fit
    const int sel0 = lt_before[blockIdx.x] + min(eq0, rank);
    if (threadIdx.x == 0) {
        s_run_eq = 0;
        s_run_sel = 0;
    }
    __syncthreads();
    for (int j = 0; j < kRelPerThread; ++j) {
        const int64_t i = first + (int64_t)j * kBlock + threadIdx.x;
        uint32_t o = 0xFFFFFFFFu;
        if (i < n) o = key_ord(key[i]);
        const bool is_eq = i < n && o == K;
        const bool is_lt = i < n && o < K;
        const uint64_t b_eq = __ballot(is_eq);
        if (lane == 0) s_cnt[0][wave] = __popcll(b_eq);
        __syncthreads();
        int eq_off = s_run_eq;
        for (int w = 0; w < wave; ++w) eq_off += s_cnt[0][w];
        const int my_eq_rank = eq0 + eq_off + lanes_below(b_eq);
        const bool pick = is_lt || (is_eq && my_eq_rank < rank);
        const uint64_t b_sel = __ballot(pick);
        if (lane == 0) s_cnt[1][wave] = __popcll(b_sel);
        __syncthreads();
        int sel_off = s_run_sel;
        for (int w = 0; w < wave; ++w) sel_off += s_cnt[1][w];
        if (pick && sel != nullptr) sel[sel0 + sel_off + lanes_below(b_sel)] = (int32_t)i;
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int w = 0; w < kWavesPerBlock; ++w) {
                s_run_eq += s_cnt[0][w];
                s_run_sel += s_cnt[1][w];
            }
        }
        __syncthreads();
    }
}

// Zeroes m and v of the selected rows in every group, and t if asked.
template <bool BF16>
__global__ __launch_bounds__(kBlock) void reset_rows_kernel(KScene S, const int32_t* sel, int64_t k, int reset_t)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int gi = 0; gi < S.n_groups; ++gi) {
        const KGroup& G = S.g[gi];
        const int64_t total = k * G.dim;
        for (int64_t x = tid; x < total; x += stride) {
            const int64_t j = x / G.dim;
            const int64_t c = x - j * G.dim;
            const int32_t i = sel[j];
            if ((uint64_t)i >= (uint64_t)S.n) continue;
            const int64_t e = (int64_t)i * G.dim + c;
            if constexpr (BF16) {
                static_cast<uint16_t*>(G.m)[e] = 0;
                static_cast<uint16_t*>(G.v)[e] = 0;
            } else {
                static_cast<float*>(G.m)[e] = 0.0f;
                static_cast<float*>(G.v)[e] = 0.0f;
            }
        }
    }
    if (reset_t && S.t != nullptr) {
        for (int64_t j = tid; j < k; j += stride) {
            const int32_t i = sel[j];
            if ((uint64_t)i < (uint64_t)S.n) S.t[i] = 0;
        }
    }
}

}  // namespace

size_t relocate_workspace_bytes(int64_t n)
{
    const size_t nblocks = (size_t)((n + kRelPerBlock - 1) / kRelPerBlock);
    return kAlign /* state */ + align_up(256 * 4) /* hist */ + 2 * align_up(nblocks * 4) +
           align_up((size_t)(n > 0 ? n : 1) * 4) /* selected list when the caller passes none */;
}

hipError_t launch_relocate(const float* key, int64_t n, int64_t k, const KScene& s, int reset_t, int32_t* selected,
                           void* ws, hipStream_t stream)
{
    const int nblocks = (int)((n + kRelPerBlock - 1) / kRelPerBlock);
    char* p = static_cast<char*>(ws);
    SelectState* st = reinterpret_cast<SelectState*>(p);
    uint32_t* hist = reinterpret_cast<uint32_t*>(p + kAlign);
    int32_t* lt = reinterpret_cast<int32_t*>(p + kAlign + align_up(256 * 4));
    int32_t* eq = reinterpret_cast<int32_t*>(p + kAlign + align_up(256 * 4) + align_up((size_t)nblocks * 4));
    int32_t* sel_ws = reinterpret_cast<int32_t*>(p + kAlign + align_up(256 * 4) + 2 * align_up((size_t)nblocks * 4));
    int32_t* sel = selected != nullptr ? selected : sel_ws;

    hipLaunchKernelGGL(select_init_kernel, dim3(1), dim3(256), 0, stream, st, hist, (int32_t)k);
    for (int shift = 24; shift >= 0; shift -= 8) {
        hipLaunchKernelGGL(select_hist_kernel, dim3(nblocks), dim3(kBlock), 0, stream, key, n, st, shift, hist);
        hipLaunchKernelGGL(select_digit_kernel, dim3(1), dim3(256), 0, stream, st, hist, shift);
    }
    hipLaunchKernelGGL(select_count_kernel, dim3(nblocks), dim3(kBlock), 0, stream, key, n, st, lt, eq);
    hipLaunchKernelGGL(select_scan_kernel, dim3(1), dim3(kBlock), 0, stream, lt, eq, nblocks);
    hipLaunchKernelGGL(select_write_kernel, dim3(nblocks), dim3(kBlock), 0, stream, key, n, st, lt, eq, sel);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || k == 0) return e;
    const unsigned grid = (unsigned)std::min<int64_t>((k * 64 + kBlock - 1) / kBlock, 4096);
    if (s.bf16) hipLaunchKernelGGL(reset_rows_kernel<true>, dim3(grid), dim3(kBlock), 0, stream, s, sel, k, reset_t);
    else hipLaunchKernelGGL(reset_rows_kernel<false>, dim3(grid), dim3(kBlock), 0, stream, s, sel, k, reset_t);
    return hipGetLastError();
}

gs_status build_groups(const gs_group* groups, int32_t n_groups, int64_t n, int32_t moment_dtype,
                       const gs_step_config* cfg, KScene* out, const char* prefix);

}  // namespace gs

using namespace gs;

extern "C" size_t gs_relocate_workspace_size(int64_t n)
{
    return n < 0 ? 0 : relocate_workspace_bytes(n);
}

extern "C" gs_status gs_relocate_reset(const float* key, int64_t n, int64_t k, const gs_group* groups,
                                       int32_t n_groups, int32_t moment_dtype, int32_t* step_count, int32_t reset_t,
                                       int32_t* selected, void* workspace, size_t workspace_bytes, hipStream_t stream)
{
    clear_error();
    if (n < 0 || n >= ((int64_t)1 << 31)) return set_error(GS_EINVAL, "gs_relocate_reset: n must be in [0, 2^31)");
    if (k < 0 || k > n) return set_error(GS_EINVAL, "gs_relocate_reset: k must be in [0, n]");
    if (moment_dtype != GS_MOMENT_F32 && moment_dtype != GS_MOMENT_BF16)
        return set_error(GS_EINVAL, "gs_relocate_reset: unknown moment_dtype");
    if (n == 0) return GS_OK;
    if (key == nullptr || workspace == nullptr) return set_error(GS_EINVAL, "gs_relocate_reset: key and workspace are required");
    if ((uintptr_t)key % 4 || (uintptr_t)workspace % kAlign || (uintptr_t)selected % 4 || (uintptr_t)step_count % 4)
        return set_error(GS_EINVAL, "gs_relocate_reset: misaligned pointer (workspace needs 256 bytes)");
    if (workspace_bytes < relocate_workspace_bytes(n)) return set_error(GS_EINVAL, "gs_relocate_reset: workspace too small");
    if (reset_t && step_count == nullptr) return set_error(GS_EINVAL, "gs_relocate_reset: reset_t needs step_count");
    gs_step_config cfg;
    memset(&cfg, 0, sizeof cfg);
    cfg.reg_norm = 1.0;
    KScene s;
    memset(&s, 0, sizeof s);
    const gs_status st = build_groups(groups, n_groups, n, moment_dtype, &cfg, &s, "gs_relocate_reset: ");
    if (st != GS_OK) return st;
    s.t = step_count;
    const hipError_t e = launch_relocate(key, n, k, s, reset_t, selected, workspace, stream);
    return e == hipSuccess ? GS_OK : set_error(GS_EHIP, hipGetErrorString(e));
}
