// Relocation state reset: the k primitives with the smallest key (ties to the
// lower index) get zero moments (and optionally a zero step count), the
// optimizer-side half of relocating dead primitives.
//
// Selection is a most-significant-digit radix select over the keys mapped to
// order-preserving uint32: three passes over the keys narrow the key of the
// k-th smallest element (K) and the number r of elements equal to K that
// still belong to the selection, two 8-bit digits and then the last 16 bits
// at once (a 256-bin histogram of the third digit and a 65536-bin table of
// the last two, which only keys matching the 16-bit prefix reach).  Per-block counts of keys < K and == K, summed
// over the blocks before each block, let every block pick its keys < K and
// the first r keys == K in index order, writing the selected indices in
// ascending order and zeroing their state rows.
#include <cstring>
#include <mutex>

#include "device_common.h"

namespace gs {

gs_status set_error(gs_status s, const char* msg);
void clear_error();

namespace {

constexpr int kRelPerThread = 16;
constexpr int kRelPerBlock = kBlock * kRelPerThread;   // 4096 keys per block
constexpr size_t kAlign = 256;
// Each digit pass accumulates its histogram into kHistCopies global copies,
// one per XCD under the round-robin dispatch of blocks, kHistStride words
// apart: one shared copy serialises thousands of device-scope atomics on a
// few cache lines, and that, not the key reads, set the time of a pass.
constexpr int kHistCopies = 8;
constexpr int kHistStride = 1024;
constexpr int kHistWords = 4 * kHistCopies * kHistStride;
// LDS digit histograms of a pass block: one per kSubLanes lanes, kSubStride
// words apart (8 banks further on per copy)
constexpr int kSubLanes = 16;
constexpr int kSubHist = kBlock / kSubLanes;
constexpr int kSubStride = 264;

// The last pass's table of the last two digits: bin (d2 << 8) | d3.
constexpr int kFineWords = 1 << 16;
constexpr int kLastPass = 2;

constexpr size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Workspace layout for n keys: the select states (one aligned slot), the
// pass histograms, the last pass's 16-bit table, then the per-block counts
// below K and equal to K.
constexpr size_t workspace_bytes_for(int64_t n)
{
    return kAlign + align_up((size_t)kHistWords * 4) + align_up((size_t)kFineWords * 4) +
           2 * align_up((size_t)((n + kRelPerBlock - 1) / kRelPerBlock) * 4);
}

constexpr size_t kScratchBytes = workspace_bytes_for(GS_RELOCATE_NOALLOC_MAX_N);

}  // namespace
}  // namespace gs

// The no-allocation entry point's workspace: one copy per device, held
// until the process ends, sized for GS_RELOCATE_NOALLOC_MAX_N keys.  Host
// code uses its device address (scratch_address), never this name.
static __device__ __align__(256) unsigned char scratch[gs::kScratchBytes];

namespace gs {
namespace {

struct SelectState {
    uint32_t prefix;   // key bits decided so far
    uint32_t mask;     // which bits are decided
    int32_t rank;      // elements still to take among those matching prefix
    int32_t pad;
};
// st[p]: the state digit pass p starts from (p = 0..2); st[3]: after the
// third digit; st[4]: the final one.
static_assert(5 * sizeof(SelectState) <= kAlign, "states fit the first aligned slot");

// -0.0 and +0.0 compare equal, so both map to the key of +0.0
__device__ __forceinline__ uint32_t key_ord(float f)
{
    const uint32_t u = f == 0.0f ? 0u : __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// st[0] = the initial state; every copy of the pass histograms and the
// 16-bit table cleared.  One block of 256 threads per (pass, copy), then one
// per 256 words of the table.
constexpr int kInitBlocks = 4 * kHistCopies + kFineWords / 256;
__global__ void select_init_kernel(SelectState* st, uint32_t* hist, uint32_t* fine, int32_t k)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st[0].prefix = 0u;
        st[0].mask = 0u;
        st[0].rank = k;
        st[0].pad = 0;
    }
    if (blockIdx.x < 4 * kHistCopies) hist[blockIdx.x * kHistStride + threadIdx.x] = 0u;
    else fine[(blockIdx.x - 4 * kHistCopies) * 256 + threadIdx.x] = 0u;
}

__device__ __forceinline__ uint32_t* pass_hist(uint32_t* hist, int pass, int copy)
{
    return hist + (pass * kHistCopies + copy) * kHistStride;
}

// The state after a digit, from the state before it and the digit's 256
// counts (summed over `copies` arrays kHistStride words apart): the bucket
// where the running count first reaches `rank` fixes the digit.  Every block
// of the next kernel computes it (up to 8 KB read from L2 and a 256-wide
// scan), so no kernel waits on another block; block 0 records it.  Needs all
// 256 threads of the block; two calls in a row need a barrier between them.
__device__ SelectState narrow(const SelectState* prev, const uint32_t* counts, int copies, int shift)
{
    __shared__ uint32_t s_inc[256];
    __shared__ SelectState s_st;
    uint32_t c = 0;
    for (int cp = 0; cp < copies; ++cp) c += counts[cp * kHistStride + threadIdx.x];
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
__device__ __forceinline__ void load_keys(const float* __restrict__ key, int64_t ks, int64_t n, int64_t first,
                                          uint32_t (&o)[kRelPerThread])
{
#pragma unroll
    for (int j = 0; j < kRelPerThread; ++j)
        o[j] = key_ord(key[ks * min(first + (int64_t)j * kBlock + threadIdx.x, n - 1)]);
}

// The block's keys for passes that only count them (digit histograms, the
// counts below and equal to K), in no particular thread order: with unit
// stride, a 16-byte aligned array and the whole block inside [0, n), four
// 16-byte loads per thread instead of sixteen 4-byte ones.  Returns whether
// that form was taken; then every loaded key is in range, else load_keys'
// mapping and its index test apply.
__device__ __forceinline__ bool load_keys_counted(const float* __restrict__ key, int64_t ks, int64_t n,
                                                  int64_t first, uint32_t (&o)[kRelPerThread])
{
    if (ks == 1 && ((uintptr_t)key & 15u) == 0 && first + kRelPerBlock <= n) {
        const float4* k4 = reinterpret_cast<const float4*>(key + first);
#pragma unroll
        for (int q = 0; q < kRelPerThread / 4; ++q) {
            const float4 f = k4[q * kBlock + threadIdx.x];
            o[4 * q + 0] = key_ord(f.x);
            o[4 * q + 1] = key_ord(f.y);
            o[4 * q + 2] = key_ord(f.z);
            o[4 * q + 3] = key_ord(f.w);
        }
        return true;
    }
    load_keys(key, ks, n, first, o);
    return false;
}

// Digit pass p (bits 31-8p .. 24-8p): histogram of the keys that match the
// state narrowed by passes 0 .. p-1.
// The last pass (kLastPass) also adds every matching key to the 16-bit table.
__global__ __launch_bounds__(kBlock) void select_hist_kernel(const float* __restrict__ key, int64_t ks, int64_t n,
                                                             SelectState* st, int pass, uint32_t* hist,
                                                             uint32_t* fine)
{
    // one private histogram per quarter-wave: keys such as opacity logits
    // fall into a few adjacent top digits, and at most 16 lanes of an LDS
    // atomic then meet on one word; copies kSubStride words apart put the
    // four quarters' copies of neighbouring digits in different banks
    __shared__ uint32_t s_hist[kSubHist * kSubStride];
    for (int i = threadIdx.x; i < kSubHist * kSubStride; i += kBlock) s_hist[i] = 0u;
    const int64_t first = (int64_t)blockIdx.x * kRelPerBlock;
    uint32_t o[kRelPerThread];
    const bool whole = load_keys_counted(key, ks, n, first, o);
    const int shift = 24 - 8 * pass;
    const SelectState cur =
        pass == 0 ? st[0] : narrow(&st[pass - 1], pass_hist(hist, pass - 1, 0), kHistCopies, shift + 8);
    if (pass > 0 && blockIdx.x == 0 && threadIdx.x == 0) st[pass] = cur;
    __syncthreads();
    uint32_t* mine = s_hist + (threadIdx.x / kSubLanes) * kSubStride;
#pragma unroll
    for (int j = 0; j < kRelPerThread; ++j) {
        const bool in = whole || first + (int64_t)j * kBlock + threadIdx.x < n;
        if (in && (o[j] & cur.mask) == cur.prefix) atomicAdd(&mine[(o[j] >> shift) & 0xFFu], 1u);
    }
    if (pass == kLastPass) {
        // Few keys match a 16-bit prefix, but ties can make many: the wave
        // adds each distinct bin once, with the number of its lanes in it.
        const int lane = threadIdx.x % kWave;
#pragma unroll
        for (int j = 0; j < kRelPerThread; ++j) {
            const bool in = whole || first + (int64_t)j * kBlock + threadIdx.x < n;
            bool want = in && (o[j] & cur.mask) == cur.prefix;
            const int bin = (int)(o[j] & 0xFFFFu);
            uint64_t pend = __ballot(want);
            while (pend != 0) {
                const int src = __builtin_ctzll(pend);
                const int lb = __builtin_amdgcn_readlane(bin, src);
                const bool same = want && bin == lb;
                const uint64_t grp = __ballot(same);
                if (lane == src) atomicAdd(&fine[lb], (uint32_t)__popcll(grp));
                want = want && !same;
                pend &= ~grp;
            }
        }
    }
    __syncthreads();
    uint32_t c = 0;
#pragma unroll
    for (int h = 0; h < kSubHist; ++h) c += s_hist[h * kSubStride + threadIdx.x];
    if (c) atomicAdd(&pass_hist(hist, pass, blockIdx.x % kHistCopies)[threadIdx.x], c);
}

// Per block: keys below K and keys equal to K, K being the key of the k-th
// smallest: the third digit from the last pass's histogram copies, then the
// fourth from that digit's row of the 16-bit table (states recorded in st[3]
// and st[4] by block 0).
__global__ __launch_bounds__(kBlock) void select_count_kernel(const float* __restrict__ key, int64_t ks, int64_t n,
                                                              SelectState* st, uint32_t* hist,
                                                              const uint32_t* fine, int32_t* lt, int32_t* eq)
{
    __shared__ int s_lt[kWavesPerBlock], s_eq[kWavesPerBlock];
    const SelectState s3 = narrow(&st[kLastPass], pass_hist(hist, kLastPass, 0), kHistCopies, 8);
    __syncthreads();   // narrow's shared state is taken again below
    const SelectState fin = narrow(&s3, fine + ((s3.prefix >> 8) & 0xFFu) * 256, 1, 0);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st[3] = s3;
        st[4] = fin;
    }
    const uint32_t K = fin.prefix;
    const bool any = fin.rank > 0;
    const int64_t first = (int64_t)blockIdx.x * kRelPerBlock;
    uint32_t o[kRelPerThread];
    const bool whole = load_keys_counted(key, ks, n, first, o);
    int nl = 0, ne = 0;
#pragma unroll
    for (int j = 0; j < kRelPerThread; ++j) {
        const bool in = whole || first + (int64_t)j * kBlock + threadIdx.x < n;
        if (in && any) {
            nl += o[j] < K;
            ne += o[j] == K;
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        nl += __shfl_xor(nl, off);
        ne += __shfl_xor(ne, off);
    }
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);   // the same on every lane
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

// Up to this many blocks, each block of the write kernel sums the counts of
// the blocks before it itself (at most 16 KB of L2 reads) instead of a
// separate single-block scan kernel, whose run is mostly latency.
constexpr int kInlineScanBlocks = 2048;

// Sum over blocks j < blockIdx.x of lt[j] and eq[j].  Needs all threads.
__device__ __forceinline__ void counts_before(const int32_t* lt, const int32_t* eq, int* a_out, int* b_out)
{
    __shared__ int s_a[kWavesPerBlock], s_b[kWavesPerBlock];
    int a = 0, b = 0;
    for (int j = threadIdx.x; j < (int)blockIdx.x; j += kBlock) {
        a += lt[j];
        b += eq[j];
    }
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_xor(a, off);
        b += __shfl_xor(b, off);
    }
    if (threadIdx.x % kWave == 0) {
        s_a[threadIdx.x / kWave] = a;
        s_b[threadIdx.x / kWave] = b;
    }
    __syncthreads();
    a = 0;
    b = 0;
    for (int w = 0; w < kWavesPerBlock; ++w) {
        a += s_a[w];
        b += s_b[w];
    }
    *a_out = a;
    *b_out = b;
}

// Zeroes m and v of the wave's staged rows in every group, walking each
// group's flattened (row, chunk) space like the step does, so consecutive
// lanes clear consecutive chunks of a row even for 1- and 3-element groups.
template <bool BF16, int V>
__device__ __forceinline__ void zero_group(const KGroup& G, int nrows, const int* s_row, int lane)
{
    const int cpr = G.cpr;
    const int items = nrows * cpr;
    int r = lane / cpr;
    int c = lane - r * cpr;
    const int dr = kWave / cpr;
    const int dc = kWave - dr * cpr;
    const float zf[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    const uint32_t zh[4] = {0u, 0u, 0u, 0u};
    for (int k = lane; k < items; k += kWave) {
        const int64_t e = (int64_t)s_row[r] * G.stride + c * V;
        if constexpr (BF16) {
            store_h<V>(static_cast<uint16_t*>(G.m) + e, zh);
            store_h<V>(static_cast<uint16_t*>(G.v) + e, zh);
        } else {
            store_f<V>(static_cast<float*>(G.m) + e, zf);
            store_f<V>(static_cast<float*>(G.v) + e, zf);
        }
        r += dr;
        c += dc;
        if (c >= cpr) { c -= cpr; ++r; }
    }
}

// Per block, in index order: take every key < K and the first `rank` keys
// equal to K; write their indices at their place in the ascending list (if
// sel is given) and zero their state rows.  Key (round j, wave w, lane l) of
// the block is element first + 256 j + 64 w + l, so index order is round,
// then wave, then lane: the wave ballots of all rounds are taken first and
// two barriers give every wave its offsets.  INLINE: lt / eq are the
// per-block counts, summed here; else their exclusive scans.
template <bool INLINE, bool BF16>
__global__ __launch_bounds__(kBlock) void select_write_kernel(const float* __restrict__ key, int64_t ks, int64_t n,
                                                              const SelectState* st, const int32_t* lt,
                                                              const int32_t* eq, int32_t* sel, KScene S,
                                                              int reset_t)
{
    constexpr int J = kRelPerThread;
    __shared__ int s_eq[J][kWavesPerBlock], s_sel[J][kWavesPerBlock];
    __shared__ int s_row[kWavesPerBlock][J * kWave];
    const uint32_t K = st[4].prefix;
    const int rank = st[4].rank;
    if (rank <= 0) return;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);   // the same on every lane
    const int lane = threadIdx.x % kWave;
    const int64_t first = (int64_t)blockIdx.x * kRelPerBlock;
    uint32_t o[J];
    load_keys(key, ks, n, first, o);
    int lt0, eq0;
    if constexpr (INLINE) {
        counts_before(lt, eq, &lt0, &eq0);
    } else {
        lt0 = lt[blockIdx.x];
        eq0 = eq[blockIdx.x];
    }
    // selected before this block: all smaller keys, plus the equal ones that fit
    const int sel0 = lt0 + min(eq0, rank);

    uint64_t b_eq[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {
        const bool in = first + (int64_t)j * kBlock + threadIdx.x < n;
        b_eq[j] = __ballot(in && o[j] == K);
        if (lane == 0) s_eq[j][wave] = __popcll(b_eq[j]);
    }
    __syncthreads();
    uint32_t picks = 0;
    uint64_t b_sel[J];
    int run = eq0;   // equal keys before round j
#pragma unroll
    for (int j = 0; j < J; ++j) {
        const bool in = first + (int64_t)j * kBlock + threadIdx.x < n;
        int off = run, tot = 0;
        for (int w = 0; w < kWavesPerBlock; ++w) {
            const int c = s_eq[j][w];
            off += w < wave ? c : 0;
            tot += c;
        }
        run += tot;
        const bool is_eq = (b_eq[j] >> lane) & 1u;
        const bool pick = (in && o[j] < K) || (is_eq && off + lanes_below(b_eq[j]) < rank);
        picks |= (uint32_t)pick << j;
        b_sel[j] = __ballot(pick);
        if (lane == 0) s_sel[j][wave] = __popcll(b_sel[j]);
    }
    __syncthreads();
    run = sel0;
    int nrows = 0;   // the wave's picks, staged in index order
#pragma unroll
    for (int j = 0; j < J; ++j) {
        int off = run, tot = 0;
        for (int w = 0; w < kWavesPerBlock; ++w) {
            const int c = s_sel[j][w];
            off += w < wave ? c : 0;
            tot += c;
        }
        run += tot;
        if ((picks >> j) & 1u) {
            const int32_t i = (int32_t)(first + (int64_t)j * kBlock + threadIdx.x);
            if (sel != nullptr) sel[off + lanes_below(b_sel[j])] = i;
            s_row[wave][nrows + lanes_below(b_sel[j])] = i;
            if (reset_t && S.t != nullptr) S.t[i] = 0;
        }
        nrows += __popcll(b_sel[j]);
    }
    if (nrows == 0) return;
    wave_sync();
    for (int gi = 0; gi < S.n_groups; ++gi) {
        const KGroup& G = S.g[gi];
        if (G.vec == 4) zero_group<BF16, 4>(G, nrows, s_row[wave], lane);
        else if (G.vec == 2) zero_group<BF16, 2>(G, nrows, s_row[wave], lane);
        else zero_group<BF16, 1>(G, nrows, s_row[wave], lane);
    }
}

template <bool INLINE>
void launch_write(int nblocks, hipStream_t stream, const float* key, int64_t ks, int64_t n, const SelectState* st,
                  const int32_t* lt, const int32_t* eq, int32_t* sel, const KScene& s, int reset_t)
{
    if (s.bf16)
        hipLaunchKernelGGL((select_write_kernel<INLINE, true>), dim3(nblocks), dim3(kBlock), 0, stream, key, ks, n,
                           st, lt, eq, sel, s, reset_t);
    else
        hipLaunchKernelGGL((select_write_kernel<INLINE, false>), dim3(nblocks), dim3(kBlock), 0, stream, key, ks, n,
                           st, lt, eq, sel, s, reset_t);
}

}  // namespace

size_t relocate_workspace_bytes(int64_t n) { return workspace_bytes_for(n); }

// Device address of this device's `scratch`, looked up once per device with
// that device current (host code must not pass the array's own name, which
// is a host-side stand-in).  nullptr and the HIP error on failure.
constexpr int kMaxDevices = 64;
void* scratch_address(hipError_t* err)
{
    static std::mutex mu;
    static void* addr[kMaxDevices] = {};
    int dev = -1;
    *err = hipGetDevice(&dev);
    if (*err != hipSuccess) return nullptr;
    if (dev < 0 || dev >= kMaxDevices) {
        *err = hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(mu);
    if (addr[dev] == nullptr) {
        void* p = nullptr;
        *err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (*err != hipSuccess) return nullptr;
        addr[dev] = p;
    }
    return addr[dev];
}

hipError_t launch_relocate(const float* key, int64_t ks, int64_t n, int64_t k, const KScene& s, int reset_t,
                           int32_t* selected, void* ws, hipStream_t stream)
{
    const int nblocks = (int)((n + kRelPerBlock - 1) / kRelPerBlock);
    const size_t hist_bytes = align_up(kHistWords * 4);
    char* p = static_cast<char*>(ws);
    SelectState* st = reinterpret_cast<SelectState*>(p);
    uint32_t* hist = reinterpret_cast<uint32_t*>(p + kAlign);
    const size_t fine_bytes = align_up((size_t)kFineWords * 4);
    uint32_t* fine = reinterpret_cast<uint32_t*>(p + kAlign + hist_bytes);
    int32_t* lt = reinterpret_cast<int32_t*>(p + kAlign + hist_bytes + fine_bytes);
    int32_t* eq = reinterpret_cast<int32_t*>(p + kAlign + hist_bytes + fine_bytes + align_up((size_t)nblocks * 4));

    hipLaunchKernelGGL(select_init_kernel, dim3(kInitBlocks), dim3(256), 0, stream, st, hist, fine, (int32_t)k);
    for (int pass = 0; pass <= kLastPass; ++pass)
        hipLaunchKernelGGL(select_hist_kernel, dim3(nblocks), dim3(kBlock), 0, stream, key, ks, n, st, pass, hist,
                           fine);
    hipLaunchKernelGGL(select_count_kernel, dim3(nblocks), dim3(kBlock), 0, stream, key, ks, n, st, hist, fine, lt,
                       eq);
    if (nblocks <= kInlineScanBlocks) {
        launch_write<true>(nblocks, stream, key, ks, n, st, lt, eq, selected, s, reset_t);
    } else {
        hipLaunchKernelGGL(select_scan_kernel, dim3(1), dim3(kBlock), 0, stream, lt, eq, nblocks);
        launch_write<false>(nblocks, stream, key, ks, n, st, lt, eq, selected, s, reset_t);
    }
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

namespace {

// Host-side checks and group set-up shared by both entry points.
gs_status relocate_prepare(const char* who, const float* key, int64_t key_stride, int64_t n, int64_t k,
                           const gs_group* groups, int32_t n_groups, int32_t moment_dtype, int32_t* step_count,
                           int32_t reset_t, int32_t* selected, KScene* s, bool* empty)
{
    char msg[160];
    *empty = false;
    if (n < 0 || n >= ((int64_t)1 << 31)) {
        snprintf(msg, sizeof msg, "%s: n must be in [0, 2^31)", who);
        return set_error(GS_EINVAL, msg);
    }
    if (key_stride < 0 || key_stride > 65536 || key_stride * n >= ((int64_t)1 << 40)) {
        snprintf(msg, sizeof msg, "%s: key_stride must be 0 or in [1, 65536] (and n * stride < 2^40)", who);
        return set_error(GS_EINVAL, msg);
    }
    if (k < 0 || k > n) {
        snprintf(msg, sizeof msg, "%s: k must be in [0, n]", who);
        return set_error(GS_EINVAL, msg);
    }
    if (moment_dtype != GS_MOMENT_F32 && moment_dtype != GS_MOMENT_BF16) {
        snprintf(msg, sizeof msg, "%s: unknown moment_dtype", who);
        return set_error(GS_EINVAL, msg);
    }
    if (n == 0) {                      // nothing to select: no other argument is read
        *empty = true;
        return GS_OK;
    }
    if (key == nullptr) {
        snprintf(msg, sizeof msg, "%s: key is required", who);
        return set_error(GS_EINVAL, msg);
    }
    if ((uintptr_t)key % 4 || (uintptr_t)selected % 4 || (uintptr_t)step_count % 4) {
        snprintf(msg, sizeof msg, "%s: misaligned key, selected or step_count", who);
        return set_error(GS_EINVAL, msg);
    }
    if (reset_t && step_count == nullptr) {
        snprintf(msg, sizeof msg, "%s: reset_t needs step_count", who);
        return set_error(GS_EINVAL, msg);
    }
    gs_step_config cfg;
    memset(&cfg, 0, sizeof cfg);
    cfg.reg_norm = 1.0;
    memset(s, 0, sizeof *s);
    snprintf(msg, sizeof msg, "%s: ", who);
    const gs_status st = build_groups(groups, n_groups, n, moment_dtype, &cfg, s, msg);
    if (st != GS_OK) return st;
    s->t = step_count;
    return GS_OK;
}

}  // namespace

extern "C" gs_status gs_relocate_reset(const float* key, int64_t key_stride, int64_t n, int64_t k,
                                       const gs_group* groups, int32_t n_groups, int32_t moment_dtype,
                                       int32_t* step_count, int32_t reset_t, int32_t* selected, void* workspace,
                                       size_t workspace_bytes, hipStream_t stream)
{
    clear_error();
    KScene s;
    bool empty = false;
    gs_status st = relocate_prepare("gs_relocate_reset", key, key_stride, n, k, groups, n_groups, moment_dtype,
                                    step_count, reset_t, selected, &s, &empty);
    if (st != GS_OK || empty) return st;
    if (workspace == nullptr) return set_error(GS_EINVAL, "gs_relocate_reset: workspace is required");
    if ((uintptr_t)workspace % kAlign)
        return set_error(GS_EINVAL, "gs_relocate_reset: misaligned workspace (needs 256 bytes)");
    if (workspace_bytes < relocate_workspace_bytes(n)) return set_error(GS_EINVAL, "gs_relocate_reset: workspace too small");
    const hipError_t e = launch_relocate(key, key_stride == 0 ? 1 : key_stride, n, k, s, reset_t, selected, workspace,
                                         stream);
    return e == hipSuccess ? GS_OK : set_error(GS_EHIP, hipGetErrorString(e));
}

extern "C" gs_status gs_relocate_reset_noalloc(const float* key, int64_t key_stride, int64_t n, int64_t k,
                                               const gs_group* groups, int32_t n_groups, int32_t moment_dtype,
                                               int32_t* step_count, int32_t reset_t, int32_t* selected,
                                               hipStream_t stream)
{
    clear_error();
    if (n > GS_RELOCATE_NOALLOC_MAX_N)
        return set_error(GS_EINVAL, "gs_relocate_reset_noalloc: n exceeds GS_RELOCATE_NOALLOC_MAX_N "
                                    "(use gs_relocate_reset with a workspace)");
    KScene s;
    bool empty = false;
    gs_status st = relocate_prepare("gs_relocate_reset_noalloc", key, key_stride, n, k, groups, n_groups,
                                    moment_dtype, step_count, reset_t, selected, &s, &empty);
    if (st != GS_OK || empty) return st;
    hipError_t e = hipSuccess;
    void* ws = scratch_address(&e);
    if (ws == nullptr) return set_error(GS_EHIP, hipGetErrorString(e));
    e = launch_relocate(key, key_stride == 0 ? 1 : key_stride, n, k, s, reset_t, selected, ws, stream);
    return e == hipSuccess ? GS_OK : set_error(GS_EHIP, hipGetErrorString(e));
}
