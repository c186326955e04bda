// Many scenes in one launch.
//
// A plan holds the scenes' kernel views in device memory and, in the kernel
// arguments, each scene's first work unit: first every scene's step units
// (index-list slices or mask windows, per the scene's schedule), then, on
// Re-State or AIU iterations, every scene's windows of invisible sampled
// rows.  A wave takes a unit and finds its scene from those prefix sums (at
// most 64 of them), so the launch needs no queue, no atomics and no clearing
// between steps.  By default the grid has one wave per unit; a resident
// (persistent) grid sized to the device's occupancy, whose waves stride over
// the units, is the other choice (gs_batch_set_resident).  A compacted scene is given units for all its
// primitives; waves past its visible count exit at once.  The launch is a
// HIP graph with one kernel node whose arguments (the step's scalars and the
// grid, which grows on Re-State iterations) are replaced before each replay.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <vector>

#include "device_common.h"
#include "trace.h"

namespace gs {

gs_status set_error(gs_status s, const char* msg);
void clear_error();
gs_status build_groups(const gs_group* groups, int32_t n_groups, int64_t n, int32_t moment_dtype,
                       const gs_step_config* cfg, KScene* out, const char* prefix);
gs_status build_hyper(const gs_step_config* cfg, bool need_reg_norm, KHyper* h);
gs_status resolve_schedule(int requested, int unit, float hint, int64_t n, int n_groups, const int32_t* dims,
                           int dtype, const uint8_t* mask, const int32_t* idx, const int32_t* count,
                           int* sched_out, int* unit_out, const char* prefix);

namespace {

constexpr int kMaxScenes = 64;
constexpr int kBatchCap = 512;
constexpr int kInvWindow = 512;
// items per lane per trip in the step units (four would spill here)
constexpr int kBatchUnroll = 2;
// A packed scene's pass needs the 4-wave register budget (launch bounds of
// the PACKED instances); the per-group instances fit in fewer registers.
constexpr int kBatchMinWindow = 32;         // smallest masked window in a plan
constexpr int kBatchMinWindowPacked = 128;  // ... for a scene in packed rows
constexpr int kBatchMinSlice = 64;     // smallest compacted slice in a plan


struct KBatch {
    const KScene* scenes;
    int32_t n_scenes;
    int32_t inv;                              // 1: invisible units follow the step units
    int32_t step_first[kMaxScenes + 1];       // first step unit of each scene; [n_scenes] = total
    int32_t inv_first[kMaxScenes + 1];        // first invisible unit of each scene, after all step units
};

template <bool BF16, bool NOISE, bool PACKED>
__device__ __forceinline__ void step_unit(const KScene& S, const KHyper& H, int64_t local, int* s_row, float* s_rb1,
                                          float* s_rsb2, float* s_noise, int lane)
{
    int nrows = 0;
    if (S.sched == kSchedCompacted) {
        const int cnt = (int)min((int64_t)*to_global(S.count), S.n);
        const int64_t base = local * S.unit;
        switch (S.unit) {
        case 32: nrows = build_rows_slice<32>(S.idx, cnt, S.n, base, s_row, lane); break;
        case 64: nrows = build_rows_slice<64>(S.idx, cnt, S.n, base, s_row, lane); break;
        case 128: nrows = build_rows_slice<128>(S.idx, cnt, S.n, base, s_row, lane); break;
        case 256: nrows = build_rows_slice<256>(S.idx, cnt, S.n, base, s_row, lane); break;
        default: nrows = build_rows_slice<512>(S.idx, cnt, S.n, base, s_row, lane); break;
        }
    } else {
        const int64_t w0 = local * S.unit;
        const uint8_t* mask = S.sched == kSchedMasked ? S.mask : nullptr;
        switch (S.unit) {
        case 32: nrows = build_rows_window<32>(mask, S.n, w0, s_row, lane); break;
        case 64: nrows = build_rows_window<64>(mask, S.n, w0, s_row, lane); break;
        case 128: nrows = build_rows_window<128>(mask, S.n, w0, s_row, lane); break;
        case 256: nrows = build_rows_window<256>(mask, S.n, w0, s_row, lane); break;
        default: nrows = build_rows_window<512>(mask, S.n, w0, s_row, lane); break;
        }
    }
    if (nrows > 0) {
        const uint64_t seed = H.seed + (uint64_t)S.seed_offset;
        wave_sync();
        stage_step_rows(nrows, s_row, s_rb1, s_rsb2, S.t, H, d_stream(seed, kTagRsr, H.iteration), lane);
        wave_sync();
        step_all_groups<BF16, NOISE, kBatchUnroll, PACKED>(S, H, seed, nrows, s_row, s_rb1, s_rsb2, lane, s_noise);
    }
    wave_sync();   // the next unit reuses this wave's LDS rows
}

template <bool BF16>
__device__ __forceinline__ void invisible_unit(const KScene& S, const KHyper& H, int64_t local, int* s_row,
                                               float* s_rb1, float* s_rsb2, int lane)
{
    const uint64_t seed = H.seed + (uint64_t)S.seed_offset;
    const int nrows = build_rows_invisible<kInvWindow>(S.mask, S.n, local * kInvWindow, S.t, H,
                                                       d_stream(seed, kTagRsr, H.iteration),
                                                       d_stream(seed, kTagAiu, H.iteration), s_row, s_rb1, s_rsb2,
                                                       lane);
    if (nrows > 0) {
        wave_sync();
        invisible_all_groups<BF16>(S, H, seed, nrows, s_row, s_rb1, s_rsb2, lane);
    }
    wave_sync();
}

// The scene of unit u: the last s with first[s] <= u (first[] ascending).
__device__ __forceinline__ int scene_of(const int32_t* first, int n_scenes, int64_t u)
{
    int s = 0;
    while (s + 1 < n_scenes && first[s + 1] <= u) ++s;
    return s;
}

template <bool BF16, bool NOISE, bool PACKED>
__global__ __launch_bounds__(kBlock, PACKED ? 4 : 1) void batched_kernel(KBatch B, KHyper H)
{
    __shared__ int s_row[kWavesPerBlock][kBatchCap];
    __shared__ float s_rb1[kWavesPerBlock][kBatchCap];
    __shared__ float s_rsb2[kWavesPerBlock][kBatchCap];
    __shared__ float s_noise[kWavesPerBlock][NOISE ? 3 * kBatchCap : 1];   // position-noise displacements
    // the wave's index, and so its unit and scene, as a value the compiler
    // knows to be the same on every lane (scalar registers, scalar loads)
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int lane = threadIdx.x % kWave;
    const int64_t steps = B.step_first[B.n_scenes];
    const int64_t total = steps + (B.inv ? B.inv_first[B.n_scenes] : 0);
    const int64_t stride = (int64_t)gridDim.x * kWavesPerBlock;
    // The scene table is not written during the launch: read as constant
    // memory, its fields (the same for the whole wave) load as scalars.
    typedef const __attribute__((address_space(4))) KScene* scene_cptr;
    const scene_cptr scenes = (scene_cptr)B.scenes;
    for (int64_t u = (int64_t)blockIdx.x * kWavesPerBlock + wave; u < total; u += stride) {
        if (u < steps) {
            const int s = scene_of(B.step_first, B.n_scenes, u);
            step_unit<BF16, NOISE, PACKED>(*(const KScene*)(scenes + s), H, u - B.step_first[s], s_row[wave],
                                           s_rb1[wave], s_rsb2[wave], s_noise[wave], lane);
        } else {
            const int64_t v = u - steps;
            const int s = scene_of(B.inv_first, B.n_scenes, v);
            invisible_unit<BF16>(*(const KScene*)(scenes + s), H, v - B.inv_first[s], s_row[wave], s_rb1[wave],
                                 s_rsb2[wave], lane);
        }
    }
}

}  // namespace

}  // namespace gs

using namespace gs;

struct gs_batch {
    int32_t n_scenes = 0;
    int32_t moment_dtype = 0;
    bool any_adaptive = false;
    bool any_packed = false;                    // some scene has packed rows
    std::vector<KScene> h_scenes;
    std::vector<int32_t> sched;
    KScene* d_scenes = nullptr;
    int64_t persistent_blocks = 0;              // > 0: a resident grid whose waves loop over the units
    hipGraph_t graph[2] = {nullptr, nullptr};   // per kernel variant: [0] plain, [1] position noise
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    hipGraphNode_t node[2] = {nullptr, nullptr};
    hipEvent_t done = nullptr;
    KBatch kb{};
    KHyper kh{};
};

namespace {

// packed: some scene of the plan has packed rows (those kernels also carry
// the per-group passes, for the plan's other scenes)
void* kernel_for(int moment_dtype, int noise, bool packed)
{
    if (packed) {
        if (moment_dtype == GS_MOMENT_BF16)
            return noise ? reinterpret_cast<void*>(&batched_kernel<true, true, true>)
                         : reinterpret_cast<void*>(&batched_kernel<true, false, true>);
        return noise ? reinterpret_cast<void*>(&batched_kernel<false, true, true>)
                     : reinterpret_cast<void*>(&batched_kernel<false, false, true>);
    }
    if (moment_dtype == GS_MOMENT_BF16)
        return noise ? reinterpret_cast<void*>(&batched_kernel<true, true, false>)
                     : reinterpret_cast<void*>(&batched_kernel<true, false, false>);
    return noise ? reinterpret_cast<void*>(&batched_kernel<false, true, false>)
                 : reinterpret_cast<void*>(&batched_kernel<false, false, false>);
}

void free_batch(gs_batch* b)
{
    if (b == nullptr) return;
    for (int v = 0; v < 2; ++v) {
        if (b->exec[v]) (void)hipGraphExecDestroy(b->exec[v]);
        if (b->graph[v]) (void)hipGraphDestroy(b->graph[v]);
    }
    if (b->done) (void)hipEventDestroy(b->done);
    if (b->d_scenes) (void)hipFree(b->d_scenes);
    delete b;
}

gs_status fail_batch(gs_batch* b, gs_status s, const char* msg)
{
    free_batch(b);
    return set_error(s, msg);
}

}  // namespace

extern "C" gs_status gs_batch_create(const gs_scene* scenes, int32_t n_scenes, int32_t moment_dtype, gs_batch** out)
{
    clear_error();
    if (out == nullptr) return set_error(GS_EINVAL, "gs_batch_create: out is NULL");
    *out = nullptr;
    if (scenes == nullptr || n_scenes < 1 || n_scenes > kMaxScenes)
        return set_error(GS_EINVAL, "gs_batch_create: need 1..64 scenes");
    if (moment_dtype != GS_MOMENT_F32 && moment_dtype != GS_MOMENT_BF16)
        return set_error(GS_EINVAL, "gs_batch_create: unknown moment_dtype");
    gs_batch* b = new gs_batch();
    b->n_scenes = n_scenes;
    b->moment_dtype = moment_dtype;
    b->h_scenes.resize((size_t)n_scenes);
    b->sched.resize((size_t)n_scenes);
    gs_step_config dummy;
    memset(&dummy, 0, sizeof dummy);
    for (int s = 0; s < n_scenes; ++s) {
        const gs_scene& sc = scenes[s];
        char prefix[64];
        snprintf(prefix, sizeof prefix, "gs_batch_create: scene %d: ", s);
        if (sc.n < 0 || sc.n >= ((int64_t)1 << 31)) return fail_batch(b, GS_EINVAL, "gs_batch_create: scene n out of range");
        if (sc.reserved != 0) return fail_batch(b, GS_EINVAL, "gs_batch_create: reserved must be 0");
        if (sc.n > 0 && sc.step_count == nullptr) return fail_batch(b, GS_EINVAL, "gs_batch_create: step_count is NULL");
        if ((uintptr_t)sc.step_count % 4 || (uintptr_t)sc.vis_count % 4 || (uintptr_t)sc.vis_idx % 4)
            return fail_batch(b, GS_EINVAL, "gs_batch_create: misaligned step_count / vis_idx / vis_count");
        KScene& K = b->h_scenes[(size_t)s];
        memset(&K, 0, sizeof K);
        gs_status st = build_groups(sc.groups, sc.n_groups, sc.n, moment_dtype, &dummy, &K, prefix);
        if (st != GS_OK) {
            free_batch(b);
            return st;
        }
        if (K.pk_stride > 0) b->any_packed = true;
        int32_t dims[GS_MAX_GROUPS];
        for (int g = 0; g < sc.n_groups; ++g) {
            dims[g] = sc.groups[g].dim;
            if (sc.groups[g].dar_kind != GS_DAR_NONE && sc.groups[g].reg_mode == GS_REG_ADAPTIVE) b->any_adaptive = true;
        }
        int sched = 0, unit = 0;
        st = resolve_schedule(sc.schedule, 0, sc.visible_hint, sc.n, sc.n_groups, dims, moment_dtype, sc.visible,
                              sc.vis_idx, sc.vis_count, &sched, &unit, prefix);
        if (st != GS_OK) {
            free_batch(b);
            return st;
        }
        // a packed scene's pass serves whole rows: its windows measured
        // fastest at 128 primitives and more, a contiguous scene's at the
        // tuner's own sizes (down to 32)
        if (sched == kSchedMasked) unit = std::max(unit, K.pk_stride > 0 ? kBatchMinWindowPacked : kBatchMinWindow);
        if (sched == kSchedCompacted) unit = std::max(unit, kBatchMinSlice);
        K.sched = sched;
        K.unit = unit;
        K.seed_offset = s;
        K.mask = sc.visible;
        K.idx = sc.vis_idx;
        K.count = sc.vis_count;
        K.t = sc.step_count;
        b->sched[(size_t)s] = sched;
    }
    // each scene's first unit: step units (for a compacted scene, enough for
    // all its primitives), then the windows of its invisible rows
    int64_t acc = 0, acc_inv = 0;
    for (int s = 0; s < n_scenes; ++s) {
        const KScene& K = b->h_scenes[(size_t)s];
        b->kb.step_first[s] = (int32_t)acc;
        b->kb.inv_first[s] = (int32_t)acc_inv;
        acc += K.n > 0 ? (K.n + K.unit - 1) / K.unit : 0;
        if (K.sched != kSchedDense && K.mask != nullptr) acc_inv += (K.n + kInvWindow - 1) / kInvWindow;
        if (acc + acc_inv >= ((int64_t)1 << 31) - kWavesPerBlock)
            return fail_batch(b, GS_EINVAL, "gs_batch_create: too many work units in one plan");
    }
    b->kb.step_first[n_scenes] = (int32_t)acc;
    b->kb.inv_first[n_scenes] = (int32_t)acc_inv;
    if (hipMalloc(&b->d_scenes, sizeof(KScene) * (size_t)n_scenes) != hipSuccess)
        return fail_batch(b, GS_ENOMEM, "gs_batch_create: hipMalloc failed");
    if (hipMemcpy(b->d_scenes, b->h_scenes.data(), sizeof(KScene) * (size_t)n_scenes, hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipEventCreate(&b->done) != hipSuccess || hipDeviceSynchronize() != hipSuccess)
        return fail_batch(b, GS_EHIP, "gs_batch_create: upload failed");
    b->kb.scenes = b->d_scenes;
    b->kb.n_scenes = n_scenes;
    *out = b;
    return GS_OK;
}

extern "C" gs_status adamw_gs_step_batched(gs_batch* b, const gs_step_config* cfg, hipStream_t stream)
{
    clear_error();
    if (b == nullptr) return set_error(GS_EINVAL, "adamw_gs_step_batched: batch is NULL");
    if (cfg == nullptr) return set_error(GS_EINVAL, "adamw_gs_step_batched: cfg is NULL");
    if (cfg->moment_dtype != b->moment_dtype)
        return set_error(GS_EINVAL, "adamw_gs_step_batched: cfg->moment_dtype differs from the plan's");
    KHyper h;
    gs_status st = build_hyper(cfg, b->any_adaptive, &h);
    if (st != GS_OK) return st;
    if (cfg->noise_enable) {
        static const int dims[4] = {3, 3, 4, 1};
        for (const KScene& K : b->h_scenes)
            for (int k = 0; k < 4; ++k) {
                const int g = cfg->noise_groups[k];
                bool dup = false;
                for (int j = 0; j < k; ++j) dup = dup || cfg->noise_groups[j] == g;
                if (g < 0 || g >= K.n_groups || K.g[g].dim != dims[k] || dup)
                    return set_error(GS_EINVAL, "adamw_gs_step_batched: noise_groups do not fit every scene");
            }
    }
    if (h.rsr_thr > 0 || h.aiu_thr > 0)
        for (const KScene& K : b->h_scenes)
            if (K.n > 0 && K.sched != kSchedDense && K.mask == nullptr)
                return set_error(GS_EINVAL, "adamw_gs_step_batched: RSR or AIU needs every sparse scene's "
                                            "visibility mask (to find invisible rows)");
    // Each variant has its own graph: a kernel node keeps the function it
    // was created with.  The grid covers the step units, plus the invisible
    // windows on Re-State or AIU iterations.
    const int v = h.noise ? 1 : 0;
    b->kh = h;
    b->kb.inv = (h.rsr_thr > 0 || h.aiu_thr > 0) ? 1 : 0;
    const int64_t units = (int64_t)b->kb.step_first[b->n_scenes] + (b->kb.inv ? b->kb.inv_first[b->n_scenes] : 0);
    if (trace_on()) {
        int64_t n_all = 0;
        for (const KScene& K : b->h_scenes) n_all += K.n;
        int packed = 0;
        for (const KScene& K : b->h_scenes) packed += K.pk_stride > 0;
        char detail[96];
        snprintf(detail, sizeof detail, "scenes=%d waves=%lld packed=%d", b->n_scenes, (long long)units, packed);
        trace_step("adamw_gs_step_batched", n_all, b->h_scenes.empty() ? 0 : b->h_scenes[0].n_groups,
                   b->persistent_blocks > 0 ? "plan-resident" : "plan", 0, cfg, detail);
    }
    if (units == 0) {
        const hipError_t e = hipEventRecord(b->done, stream);
        return e == hipSuccess ? GS_OK : set_error(GS_EHIP, hipGetErrorString(e));
    }
    void* args[] = {&b->kb, &b->kh};
    hipKernelNodeParams p;
    memset(&p, 0, sizeof p);
    p.func = kernel_for(b->moment_dtype, v, b->any_packed);
    const int64_t blocks = (units + kWavesPerBlock - 1) / kWavesPerBlock;
    // the waves stride over the units, so a grid capped at one dispatch's
    // limit still covers them all
    int64_t grid = std::min<int64_t>(blocks, kMaxGridBlocks);
    if (b->persistent_blocks > 0) grid = std::min<int64_t>(grid, b->persistent_blocks);
    p.gridDim = dim3((unsigned)grid);
    p.blockDim = dim3(kBlock);
    p.sharedMemBytes = 0;
    p.kernelParams = args;
    p.extra = nullptr;
    hipError_t e = hipSuccess;
    if (b->exec[v] == nullptr) {
        e = hipGraphCreate(&b->graph[v], 0);
        if (e == hipSuccess) e = hipGraphAddKernelNode(&b->node[v], b->graph[v], nullptr, 0, &p);
        if (e == hipSuccess) e = hipGraphInstantiate(&b->exec[v], b->graph[v], nullptr, nullptr, 0);
    } else {
        e = hipGraphExecKernelNodeSetParams(b->exec[v], b->node[v], &p);
    }
    if (e == hipSuccess) e = hipGraphLaunch(b->exec[v], stream);
    if (e == hipSuccess) e = hipEventRecord(b->done, stream);
    if (e != hipSuccess) return set_error(GS_EHIP, hipGetErrorString(e));
    return GS_OK;
}

extern "C" gs_status gs_batch_set_resident(gs_batch* b, int32_t resident)
{
    clear_error();
    if (b == nullptr) return set_error(GS_EINVAL, "gs_batch_set_resident: batch is NULL");
    if (!resident) {
        b->persistent_blocks = 0;
        return GS_OK;
    }
    // as many blocks as fit on the device at once (the plain variant's
    // occupancy); the noise variant may fit fewer, which only makes some
    // blocks start later
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, reinterpret_cast<const void*>(kernel_for(b->moment_dtype, 0, b->any_packed)), kBlock, 0) != hipSuccess)
        return set_error(GS_EHIP, "gs_batch_set_resident: device query failed");
    b->persistent_blocks = (int64_t)cus * std::max(1, per_cu);
    return GS_OK;
}

extern "C" int32_t gs_batch_scene_schedule(const gs_batch* b, int32_t s)
{
    if (b == nullptr || s < 0 || s >= b->n_scenes) return -1;
    return b->sched[(size_t)s];
}

extern "C" gs_status gs_batch_destroy(gs_batch* b)
{
    if (b == nullptr) return GS_OK;
    if (b->done) (void)hipEventSynchronize(b->done);
    free_batch(b);
    return GS_OK;
}
