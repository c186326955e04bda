// Schedule tuner: times the compacted and masked schedules and their wave
// unit sizes on synthetic buffers and keeps the fastest per bucket of
// (primitive count, visible fraction, moment dtype).
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "device_common.h"
#include "trace.h"
#include "tuner.h"

namespace gs {

gs_status set_error(gs_status s, const char* msg);
void clear_error();

namespace {

std::mutex g_mu;
std::map<std::tuple<int, int, int>, std::pair<int, int>> g_table;

int n_bucket(int64_t n) { return n <= 1 ? 0 : (int)std::lround(std::log2((double)n)); }

// visible-fraction buckets, finer at low fractions where the schedules differ most
int f_bucket(float f)
{
    static const float edges[] = {0.01f, 0.02f, 0.04f, 0.07f, 0.1f, 0.15f, 0.2f, 0.3f, 0.4f, 0.5f, 0.65f, 0.8f};
    int b = 0;
    for (float e : edges)
        if (f > e) ++b;
    return b;
}

__global__ void bernoulli_mask_kernel(uint8_t* mask, int64_t n, uint64_t thr)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) mask[i] = (uint8_t)((d_splitmix(0x5EEDull, (uint64_t)i + 1) >> 32) < thr);
}

struct DevBuf {
    void* p = nullptr;
    ~DevBuf()
    {
        if (p) (void)hipFree(p);
    }
};

}  // namespace

bool tuner_lookup(int64_t n, float f, int dtype, int* sched, int* unit)
{
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_table.find({n_bucket(n), f_bucket(f), dtype});
    if (it == g_table.end()) return false;
    *sched = it->second.first;
    *unit = it->second.second;
    return true;
}

void tuner_record(int64_t n, float f, int dtype, int sched, int unit)
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_table[{n_bucket(n), f_bucket(f), dtype}] = {sched, unit};
}

}  // namespace gs

using namespace gs;

extern "C" void gs_tune_clear(void)
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_table.clear();
}

namespace {

// Argument checks shared by both tuner entry points.
gs_status check_tune_args(const char* who, int64_t n, const int32_t* dims, int32_t n_groups, int32_t moment_dtype)
{
    char msg[128];
    if (n < 1 || n >= ((int64_t)1 << 31)) {
        snprintf(msg, sizeof msg, "%s: n must be in [1, 2^31)", who);
        return set_error(GS_EINVAL, msg);
    }
    if (dims == nullptr || n_groups < 1 || n_groups > GS_MAX_GROUPS) {
        snprintf(msg, sizeof msg, "%s: bad dims / n_groups", who);
        return set_error(GS_EINVAL, msg);
    }
    if (moment_dtype != GS_MOMENT_F32 && moment_dtype != GS_MOMENT_BF16) {
        snprintf(msg, sizeof msg, "%s: unknown moment_dtype", who);
        return set_error(GS_EINVAL, msg);
    }
    for (int g = 0; g < n_groups; ++g)
        if (dims[g] < 1 || dims[g] > 4096) {
            snprintf(msg, sizeof msg, "%s: dim out of range", who);
            return set_error(GS_EINVAL, msg);
        }
    return GS_OK;
}

// Times every (schedule, unit) candidate on buffers of n zero rows and
// records the fastest.  user_mask == nullptr: the visibility is a synthetic
// Bernoulli(visible_fraction) mask; else it is that device mask (only read),
// and the entry is recorded under its own visible fraction.
gs_status tune(const char* who, int64_t n, const int32_t* dims, int32_t n_groups, float visible_fraction,
               const uint8_t* user_mask, int32_t moment_dtype, int32_t* best_schedule, int32_t* best_unit)
{

    const bool bf16 = moment_dtype == GS_MOMENT_BF16;
    const size_t msz = bf16 ? 2 : 4;
    std::vector<DevBuf> bufs((size_t)n_groups * 4 + 4);
    KScene s;
    memset(&s, 0, sizeof s);
    for (int g = 0; g < n_groups; ++g) {
        const size_t elems = (size_t)n * dims[g];
        const size_t bytes[4] = {elems * 4, elems * 4, elems * msz, elems * msz};
        for (int a = 0; a < 4; ++a) {
            DevBuf& b = bufs[(size_t)g * 4 + a];
            if (hipMalloc(&b.p, bytes[a]) != hipSuccess) return set_error(GS_ENOMEM, "gs_tune: hipMalloc failed");
            if (hipMemset(b.p, 0, bytes[a]) != hipSuccess) return set_error(GS_EHIP, "gs_tune: hipMemset failed");
        }
        KGroup& K = s.g[g];
        K.param = (float*)bufs[(size_t)g * 4].p;
        K.grad = (const float*)bufs[(size_t)g * 4 + 1].p;
        K.m = bufs[(size_t)g * 4 + 2].p;
        K.v = bufs[(size_t)g * 4 + 3].p;
        K.dim = dims[g];
        K.vec = dims[g] % 4 == 0 ? 4 : (dims[g] % 2 == 0 ? 2 : 1);
        K.cpr = dims[g] / K.vec;
        K.stride = dims[g];
        K.lr = 1e-3f;
    }
    DevBuf& bt = bufs[(size_t)n_groups * 4];
    DevBuf& bm = bufs[(size_t)n_groups * 4 + 1];
    DevBuf& bi = bufs[(size_t)n_groups * 4 + 2];
    DevBuf& bc = bufs[(size_t)n_groups * 4 + 3];
    if (hipMalloc(&bt.p, (size_t)n * 4) != hipSuccess ||
        (user_mask == nullptr && hipMalloc(&bm.p, (size_t)n) != hipSuccess) ||
        hipMalloc(&bi.p, (size_t)n * 4) != hipSuccess || hipMalloc(&bc.p, 256) != hipSuccess)
        return set_error(GS_ENOMEM, "gs_tune: hipMalloc failed");
    if (hipMemset(bt.p, 0, (size_t)n * 4) != hipSuccess) return set_error(GS_EHIP, "gs_tune: hipMemset failed");

    hipStream_t st;
    if (hipStreamCreate(&st) != hipSuccess) return set_error(GS_EHIP, "gs_tune: hipStreamCreate failed");
    const uint8_t* mask = user_mask;
    if (mask == nullptr) {
        const uint64_t thr = visible_fraction >= 1.0f
                                 ? ((uint64_t)1 << 32)
                                 : (uint64_t)std::floor((double)visible_fraction * 4294967296.0);
        hipLaunchKernelGGL(bernoulli_mask_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                           (uint8_t*)bm.p, n, thr);
        mask = (const uint8_t*)bm.p;
    }
    hipError_t e = launch_compact(mask, n, (int32_t*)bi.p, (int32_t*)bc.p, st);
    if (user_mask != nullptr) {
        // the mask's own visible fraction, for the record
        int32_t count = 0;
        if (e == hipSuccess) e = hipMemcpyAsync(&count, bc.p, 4, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e == hipSuccess && count <= 0) {
            (void)hipStreamDestroy(st);
            char msg[96];
            snprintf(msg, sizeof msg, "%s: the mask has no visible entry", who);
            return set_error(GS_EINVAL, msg);
        }
        visible_fraction = (float)((double)count / (double)n);
    }

    s.n_groups = n_groups;
    s.bf16 = bf16 ? 1 : 0;
    s.n = n;
    s.mask = mask;
    s.idx = (const int32_t*)bi.p;
    s.count = (const int32_t*)bc.p;
    s.t = (int32_t*)bt.p;
    KHyper h;
    memset(&h, 0, sizeof h);
    h.beta1 = 0.9f;
    h.omb1 = 0.1f;
    h.beta2 = 0.999f;
    h.omb2 = 0.001f;
    h.logb1 = std::log(0.9f);
    h.logb2 = std::log(0.999f);
    h.eps = 1e-15f;

    struct Cand { int sched, unit; };
    const Cand cands[] = {{kSchedCompacted, 32}, {kSchedCompacted, 64}, {kSchedCompacted, 128},
                          {kSchedCompacted, 256}, {kSchedCompacted, 512}, {kSchedMasked, 32},
                          {kSchedMasked, 64},     {kSchedMasked, 128},    {kSchedMasked, 256},
                          {kSchedMasked, 512}};
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    float best_ms = INFINITY;
    Cand best = cands[0];
    const int reps = 5;
    for (const Cand& c : cands) {
        if (e != hipSuccess) break;
        if (fit_unit(n, c.unit, c.unit * 2) != c.unit) continue;      // its grid would not fit one dispatch
        s.sched = c.sched;
        s.unit = c.unit;
        for (int w = 0; w < 2 && e == hipSuccess; ++w) e = launch_step(s, h, st);
        (void)hipEventRecord(e0, st);
        for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch_step(s, h, st);
        (void)hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e == hipSuccess && ms < best_ms) {
            best_ms = ms;
            best = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
    if (e != hipSuccess) return set_error(GS_EHIP, hipGetErrorString(e));
    tuner_record(n, visible_fraction, moment_dtype, best.sched, best.unit);
    if (best_schedule) *best_schedule = best.sched;
    if (best_unit) *best_unit = best.unit;
    return GS_OK;
}

}  // namespace

extern "C" gs_status gs_tune(int64_t n, const int32_t* dims, int32_t n_groups, float visible_fraction,
                             int32_t moment_dtype, int32_t* best_schedule, int32_t* best_unit)
{
    clear_error();
    const gs_status st = check_tune_args("gs_tune", n, dims, n_groups, moment_dtype);
    if (st != GS_OK) return st;
    if (!(visible_fraction > 0.0f && visible_fraction <= 1.0f))
        return set_error(GS_EINVAL, "gs_tune: visible_fraction must be in (0, 1]");
    return tune("gs_tune", n, dims, n_groups, visible_fraction, nullptr, moment_dtype, best_schedule, best_unit);
}

extern "C" gs_status gs_tune_mask(int64_t n, const int32_t* dims, int32_t n_groups, const uint8_t* mask,
                                  int32_t moment_dtype, int32_t* best_schedule, int32_t* best_unit)
{
    clear_error();
    const gs_status st = check_tune_args("gs_tune_mask", n, dims, n_groups, moment_dtype);
    if (st != GS_OK) return st;
    if (mask == nullptr) return set_error(GS_EINVAL, "gs_tune_mask: mask is NULL");
    return tune("gs_tune_mask", n, dims, n_groups, 0.0f, mask, moment_dtype, best_schedule, best_unit);
}
