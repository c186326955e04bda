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
// st[p]: the state digit pass p starts from (p = 0..3); st[4]: the final one.
static_assert(5 * sizeof(SelectState) <= kAlign, "states fit the first aligned slot");

// -0.0 and +0.0 compare equal, so both map to the key of +0.0
__device__ __forceinline__ uint32_t key_ord(float f)
{
    const uint32_t u = f == 0.0f ? 0u : __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// st[0] = the initial state; the four pass histograms cleared.  256 threads.
__global__ void select_init_kernel(SelectState* st, uint32_t* hist, int32_t k)
{
    if (threadIdx.x == 0) {
        st[0].prefix = 0u;
        st[0].mask = 0u;
        st[0].rank = k;
        st[0].pad = 0;
    }
    for (int p = 0; p < 4; ++p) hist[p * 256 + threadIdx.x] = 0u;
}

// The state after a digit pass, from the state before it and the pass's
// histogram: the bucket where the running count first reaches `rank` fixes
// the digit.  Every block of the next kernel computes it (a 1 KB read and a
// 256-wide scan), so no kernel waits on another block; block 0 records it.
// Needs all 256 threads of the block.
__device__ SelectState narrow(const SelectState* prev, const uint32_t* hist, int shift)
{
    __shared__ uint32_t s_inc[256];
    __shared__ SelectState s_st;
    const uint32_t c = hist[threadIdx.x];
    s_inc[threadIdx.x] = c;
    if (threadIdx.x == 0) s_st = *prev;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const uint32_t y = threadIdx.x >= (unsigned)off ? s_inc[threadIdx.x - off] : 0u;
        __syncthreads();
        s_inc[threadIdx.x] += y;
        __syncthreads();
    }
    const uint32_t rank = (uint32_t)s_st.rank;
    const uint32_t before = s_inc[threadIdx.x] - c;
    __syncthreads();
    if (rank > 0 && before < rank && s_inc[threadIdx.x] >= rank) {
        s_st.prefix |= (uint32_t)threadIdx.x << shift;
        s_st.mask |= 0xFFu << shift;
        s_st.rank = (int32_t)(rank - before);
    }
    __syncthreads();
    return s_st;
}

// The block's keys, mapped to order-preserving uint32; entries past n get
// the largest key and are excluded by the callers through the index test.
__device__ __forceinline__ void load_keys(const float* __restrict__ key, int64_t n, int64_t first,
                                          uint32_t (&o)[kRelPerThread])
{
#pragma unroll
    for (int j = 0; j < kRelPerThread; ++j) o[j] = key_ord(key[min(first + (int64_t)j * kBlock + threadIdx.x, n - 1)]);
}

// Digit pass p (bits 31-8p .. 24-8p): histogram of the keys that match the
// state narrowed by passes 0 .. p-1.
__global__ __launch_bounds__(kBlock) void select_hist_kernel(const float* __restrict__ key, int64_t n,
                                                             SelectState* st, int pass, uint32_t* hist)
{
    // one private histogram per wave: the keys of a view are concentrated in
    // a few digits, and four copies cut the LDS atomic collisions fourfold
    __shared__ uint32_t s_hist[kWavesPerBlock][256];
    for (int w = 0; w < kWavesPerBlock; ++w) s_hist[w][threadIdx.x] = 0u;
    const int64_t first = (int64_t)blockIdx.x * kRelPerBlock;
    uint32_t o[kRelPerThread];
    load_keys(key, n, first, o);
    const int shift = 24 - 8 * pass;
    const SelectState cur = pass == 0 ? st[0] : narrow(&st[pass - 1], hist + (pass - 1) * 256, shift + 8);
    if (pass > 0 && blockIdx.x == 0 && threadIdx.x == 0) st[pass] = cur;
    __syncthreads();
    uint32_t* mine = s_hist[threadIdx.x / kWave];
#pragma unroll
    for (int j = 0; j < kRelPerThread; ++j) {
        const int64_t i = first + (int64_t)j * kBlock + threadIdx.x;
        if (i < n && (o[j] & cur.mask) == cur.prefix) atomicAdd(&mine[(o[j] >> shift) & 0xFFu], 1u);
    }
    __syncthreads();
    uint32_t c = 0;
    for (int w = 0; w < kWavesPerBlock; ++w) c += s_hist[w][threadIdx.x];
    if (c) atomicAdd(&hist[pass * 256 + threadIdx.x], c);
}

// Per block: keys below K and keys equal to K, K being the key of the k-th
// smallest (the state after the last pass, recorded in st[4] by block 0).
__global__ __launch_bounds__(kBlock) void select_count_kernel(const float* __restrict__ key, int64_t n,
                                                              SelectState* st, const uint32_t* hist, int32_t* lt,
                                                              int32_t* eq)
{
    __shared__ int s_lt[kWavesPerBlock], s_eq[kWavesPerBlock];
    const SelectState fin = narrow(&st[3], hist + 3 * 256, 0);
    if (blockIdx.x == 0 && threadIdx.x == 0) st[4] = fin;
    const uint32_t K = fin.prefix;
    const bool any = fin.rank > 0;
    const int64_t first = (int64_t)blockIdx.x * kRelPerBlock;
    uint32_t o[kRelPerThread];
    load_keys(key, n, first, o);
    int nl = 0, ne = 0;
#pragma unroll
    for (int j = 0; j < kRelPerThread; ++j) {
        const int64_t i = first + (int64_t)j * kBlock + threadIdx.x;
        if (i < n && any) {
            nl += o[j] < K;
            ne += o[j] == K;
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
    const uint32_t K = st[4].prefix;
    const int rank = st[4].rank;
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
    uint32_t o[kRelPerThread];
    load_keys(key, n, first, o);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kRelPerThread; ++j) {
        const int64_t i = first + (int64_t)j * kBlock + threadIdx.x;
        const bool is_eq = i < n && o[j] == K;
        const bool is_lt = i < n && o[j] < K;
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
// One wave per selected row at a time: its lanes clear the row's elements
// group by group (no index arithmetic beyond the row base).
template <bool BF16>
__global__ __launch_bounds__(kBlock) void reset_rows_kernel(KScene S, const int32_t* sel, int64_t k, int reset_t)
{
    const int lane = threadIdx.x % kWave;
    const int64_t waves = (int64_t)gridDim.x * kWavesPerBlock;
    for (int64_t j = (int64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave; j < k; j += waves) {
        const int32_t i = sel[j];
        if ((uint64_t)i >= (uint64_t)S.n) continue;
        for (int gi = 0; gi < S.n_groups; ++gi) {
            const KGroup& G = S.g[gi];
            const int64_t base = (int64_t)i * G.dim;
            for (int c = lane; c < G.dim; c += kWave) {
                if constexpr (BF16) {
                    static_cast<uint16_t*>(G.m)[base + c] = 0;
                    static_cast<uint16_t*>(G.v)[base + c] = 0;
                } else {
                    static_cast<float*>(G.m)[base + c] = 0.0f;
                    static_cast<float*>(G.v)[base + c] = 0.0f;
                }
            }
        }
        if (reset_t && S.t != nullptr && lane == 0) S.t[i] = 0;
    }
}

}  // namespace

size_t relocate_workspace_bytes(int64_t n)
{
    const size_t nblocks = (size_t)((n + kRelPerBlock - 1) / kRelPerBlock);
    return kAlign /* states */ + align_up(4 * 256 * 4) /* pass histograms */ + 2 * align_up(nblocks * 4) +
           align_up((size_t)(n > 0 ? n : 1) * 4) /* selected list when the caller passes none */;
}

hipError_t launch_relocate(const float* key, int64_t n, int64_t k, const KScene& s, int reset_t, int32_t* selected,
                           void* ws, hipStream_t stream)
{
    const int nblocks = (int)((n + kRelPerBlock - 1) / kRelPerBlock);
    const size_t hist_bytes = align_up(4 * 256 * 4);
    char* p = static_cast<char*>(ws);
    SelectState* st = reinterpret_cast<SelectState*>(p);
    uint32_t* hist = reinterpret_cast<uint32_t*>(p + kAlign);
    int32_t* lt = reinterpret_cast<int32_t*>(p + kAlign + hist_bytes);
    int32_t* eq = reinterpret_cast<int32_t*>(p + kAlign + hist_bytes + align_up((size_t)nblocks * 4));
    int32_t* sel_ws = reinterpret_cast<int32_t*>(p + kAlign + hist_bytes + 2 * align_up((size_t)nblocks * 4));
    int32_t* sel = selected != nullptr ? selected : sel_ws;

    hipLaunchKernelGGL(select_init_kernel, dim3(1), dim3(256), 0, stream, st, hist, (int32_t)k);
    for (int pass = 0; pass < 4; ++pass)
        hipLaunchKernelGGL(select_hist_kernel, dim3(nblocks), dim3(kBlock), 0, stream, key, n, st, pass, hist);
    hipLaunchKernelGGL(select_count_kernel, dim3(nblocks), dim3(kBlock), 0, stream, key, n, st, hist, lt, eq);
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
