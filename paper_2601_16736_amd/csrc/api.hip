// Host side of the C ABI: argument validation, FP32 constants prepared in
// double, schedule choice and launches.  Declarations and contracts: gsopt.h.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>

#include "internal.h"
#include "trace.h"
#include "tuner.h"

namespace gs {

namespace {

thread_local std::string t_err;

gs_status fail(gs_status s, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    t_err = buf;
    return s;
}

gs_status hip_fail(hipError_t e, const char* what)
{
    return fail(GS_EHIP, "%s: %s (%s)", what, hipGetErrorName(e), hipGetErrorString(e));
}

bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

bool finite_d(double x) { return std::isfinite(x); }

}  // namespace

bool trace_on()
{
    const char* v = getenv("GSOPT_TRACE");
    return v != nullptr && v[0] != '\0' && strcmp(v, "0") != 0;
}

void trace_step(const char* entry, int64_t n, int n_groups, const char* schedule, int unit,
                const gs_step_config* cfg, const char* detail)
{
    if (!trace_on()) return;
    fprintf(stderr, "gsopt: %s n=%lld groups=%d schedule=%s unit=%d moments=%s iteration=%lld rsr=%d aiu=%d noise=%d%s%s\n",
            entry, (long long)n, n_groups, schedule, unit,
            cfg->moment_dtype == GS_MOMENT_BF16 ? (cfg->stochastic_round ? "bf16-sr" : "bf16-rne") : "f32",
            (long long)cfg->iteration, cfg->rsr_enable, cfg->aiu_enable, cfg->noise_enable, detail[0] ? " " : "",
            detail);
}

int fit_unit(int64_t rows, int unit, int max_unit)
{
    while (unit < max_unit) {
        const int64_t units = (rows + unit - 1) / unit;
        if ((units + kWavesPerBlock - 1) / kWavesPerBlock <= kMaxGridBlocks) break;
        unit *= 2;
    }
    return unit;
}

uint64_t splitmix_output(uint64_t s, uint64_t k)
{
    uint64_t z = s + k * kGamma;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

gs_status set_error(gs_status s, const char* msg)
{
    t_err = msg;
    return s;
}

void clear_error() { t_err.clear(); }

// Row stride of a means array: 0 means 3 (contiguous [n][3]); otherwise at
// least 3, and the rows must stay inside 2^40 elements.
static bool means_rows(int64_t stride, int64_t n, int64_t* out)
{
    const int64_t ms = stride == 0 ? 3 : stride;
    if (ms < 3 || ms > 65536 || ms * n >= ((int64_t)1 << 40)) return false;
    *out = ms;
    return true;
}

void plan_packed_rows(KScene& s, size_t msz)
{
    s.pk_stride = 0;
    s.pk_param = nullptr;
    s.pk_grad = nullptr;
    s.pk_m = nullptr;
    s.pk_v = nullptr;
    for (int g = 0; g < GS_MAX_GROUPS; ++g) s.pk_col[g] = 0;
    if (s.n_groups < 1) return;
    const int32_t S = s.g[0].stride;
    if (S < 4 || S > 256 || (S & (S - 1)) != 0) return;
    uintptr_t bp = UINTPTR_MAX, bg = UINTPTR_MAX, bm = UINTPTR_MAX, bv = UINTPTR_MAX;
    for (int g = 0; g < s.n_groups; ++g) {
        const KGroup& G = s.g[g];
        if (G.stride != S || G.param == nullptr) return;
        bp = std::min(bp, (uintptr_t)G.param);
        bg = std::min(bg, (uintptr_t)G.grad);
        bm = std::min(bm, (uintptr_t)G.m);
        bv = std::min(bv, (uintptr_t)G.v);
    }
    if (bp % 16 || bg % 16 || bm % (4 * msz) || bv % (4 * msz)) return;
    uint64_t used = 0;                  // columns 0..63 taken so far
    uint64_t used_hi[3] = {0, 0, 0};    // columns 64..255
    for (int g = 0; g < s.n_groups; ++g) {
        const KGroup& G = s.g[g];
        const uintptr_t dp = (uintptr_t)G.param - bp;
        if (dp % 4) return;
        const int64_t col = (int64_t)(dp / 4);
        if (col + G.dim > S) return;
        if ((uintptr_t)G.grad - bg != dp || (uintptr_t)G.m - bm != (uintptr_t)col * msz ||
            (uintptr_t)G.v - bv != (uintptr_t)col * msz)
            return;
        for (int64_t c = col; c < col + G.dim; ++c) {
            uint64_t& word = c < 64 ? used : used_hi[c / 64 - 1];
            const uint64_t bit = (uint64_t)1 << (c % 64);
            if (word & bit) return;                  // two groups share a column
            word |= bit;
        }
        s.pk_col[g] = (int32_t)col;
    }
    s.pk_stride = S;
    s.pk_param = reinterpret_cast<float*>(bp);
    s.pk_grad = reinterpret_cast<const float*>(bg);
    s.pk_m = reinterpret_cast<void*>(bm);
    s.pk_v = reinterpret_cast<void*>(bv);
}

// Validates one scene's groups and fills the kernel view.  Prefix names the
// scene in messages.
gs_status build_groups(const gs_group* groups, int32_t n_groups, int64_t n, int32_t moment_dtype,
                       const gs_step_config* cfg, KScene* out, const char* prefix)
{
    if (groups == nullptr) return fail(GS_EINVAL, "%sgroups is NULL", prefix);
    if (n_groups < 1 || n_groups > GS_MAX_GROUPS)
        return fail(GS_EINVAL, "%sn_groups = %d, must be in [1, %d]", prefix, n_groups, GS_MAX_GROUPS);
    const bool bf16 = moment_dtype == GS_MOMENT_BF16;
    const size_t msz = bf16 ? 2 : 4;
    for (int g = 0; g < n_groups; ++g) {
        const gs_group& G = groups[g];
        if (G.dim < 1 || G.dim > 4096) return fail(GS_EINVAL, "%sgroup %d: dim = %d, must be in [1, 4096]", prefix, g, G.dim);
        if (G.row_stride != 0 && (G.row_stride < G.dim || G.row_stride > 65536))
            return fail(GS_EINVAL, "%sgroup %d: row_stride = %d, must be 0 or in [dim, 65536]", prefix, g, G.row_stride);
        const int32_t stride = G.row_stride != 0 ? G.row_stride : G.dim;
        if ((int64_t)stride * n >= ((int64_t)1 << 40))
            return fail(GS_EINVAL, "%sgroup %d: n * row stride too large", prefix, g);
        if (n > 0 && (G.param == nullptr || G.grad == nullptr || G.exp_avg == nullptr || G.exp_avg_sq == nullptr))
            return fail(GS_EINVAL, "%sgroup %d: param, grad, exp_avg and exp_avg_sq must be non-NULL", prefix, g);
        if (!aligned(G.param, 4) || !aligned(G.grad, 4) || !aligned(G.exp_avg, msz) || !aligned(G.exp_avg_sq, msz))
            return fail(GS_EINVAL, "%sgroup %d: misaligned pointer (FP32 arrays need 4 bytes, BF16 moments 2)", prefix, g);
        if (G.dar_kind < GS_DAR_NONE || G.dar_kind > GS_DAR_LOGSCALE_EXP)
            return fail(GS_EINVAL, "%sgroup %d: unknown dar_kind %d", prefix, g, G.dar_kind);
        if (G.reg_mode < GS_REG_ADAPTIVE || G.reg_mode > GS_REG_CONSTANT_CLIPPED)
            return fail(GS_EINVAL, "%sgroup %d: unknown reg_mode %d", prefix, g, G.reg_mode);
        if (!finite_d(G.lr)) return fail(GS_EINVAL, "%sgroup %d: lr must be finite", prefix, g);
        if (!(G.dar_lambda >= 0.0) || !finite_d(G.dar_lambda))
            return fail(GS_EINVAL, "%sgroup %d: dar_lambda must be finite and >= 0", prefix, g);
        if (!(G.dar_clip >= 0.0)) return fail(GS_EINVAL, "%sgroup %d: dar_clip must be >= 0", prefix, g);

        KGroup& K = out->g[g];
        K.param = G.param;
        K.grad = G.grad;
        K.m = G.exp_avg;
        K.v = G.exp_avg_sq;
        K.dim = G.dim;
        // a row's accesses are as wide as its length, stride and pointers allow
        int vec = 1;
        if (G.dim % 4 == 0 && stride % 4 == 0 && aligned(G.param, 16) && aligned(G.grad, 16) &&
            aligned(G.exp_avg, 4 * msz) && aligned(G.exp_avg_sq, 4 * msz))
            vec = 4;
        else if (G.dim % 2 == 0 && stride % 2 == 0 && aligned(G.param, 8) && aligned(G.grad, 8) &&
                 aligned(G.exp_avg, 2 * msz) && aligned(G.exp_avg_sq, 2 * msz))
            vec = 2;
        K.vec = vec;
        K.cpr = G.dim / vec;
        K.lr = (float)G.lr;
        K.dar_kind = G.dar_kind;
        K.reg_mode = G.reg_mode;
        K.dar_clip = std::isinf(G.dar_clip) ? INFINITY : (float)G.dar_clip;
        K.stride = stride;
        K.dar_lambda = G.dar_lambda;
    }
    (void)cfg;
    for (int g = n_groups; g < GS_MAX_GROUPS; ++g) memset(&out->g[g], 0, sizeof(KGroup));
    out->n_groups = n_groups;
    out->bf16 = bf16 ? 1 : 0;
    out->n = n;
    plan_packed_rows(*out, msz);
    return GS_OK;
}

// Bernoulli(p) sampling threshold on the top 32 bits of a draw.
static uint64_t sample_threshold(double p)
{
    if (p >= 1.0) return (uint64_t)1 << 32;
    if (p > 0.0) return (uint64_t)std::floor(p * 4294967296.0);
    return 0;
}

gs_status build_hyper(const gs_step_config* cfg, bool need_reg_norm, KHyper* h)
{
    if (cfg == nullptr) return fail(GS_EINVAL, "cfg is NULL");
    if (!(cfg->beta1 >= 0.0 && cfg->beta1 < 1.0)) return fail(GS_EINVAL, "beta1 = %g, must be in [0, 1)", cfg->beta1);
    if (!(cfg->beta2 >= 0.0 && cfg->beta2 < 1.0)) return fail(GS_EINVAL, "beta2 = %g, must be in [0, 1)", cfg->beta2);
    if (!(cfg->eps > 0.0) || !finite_d(cfg->eps) || !((float)cfg->eps > 0.0f))
        return fail(GS_EINVAL, "eps = %g, must be > 0 and representable in FP32", cfg->eps);
    if (need_reg_norm && !(cfg->reg_norm > 0.0 && finite_d(cfg->reg_norm)))
        return fail(GS_EINVAL, "reg_norm = %g, must be finite and > 0 for adaptive DAR groups", cfg->reg_norm);
    if (cfg->moment_dtype != GS_MOMENT_F32 && cfg->moment_dtype != GS_MOMENT_BF16)
        return fail(GS_EINVAL, "unknown moment_dtype %d", cfg->moment_dtype);
    if (cfg->iteration < 0) return fail(GS_EINVAL, "iteration must be >= 0");
    if (cfg->rsr_enable) {
        if (!(cfg->rsr_alpha1 >= 0.0 && cfg->rsr_alpha1 < 1.0))
            return fail(GS_EINVAL, "rsr_alpha1 = %g, must be in [0, 1)", cfg->rsr_alpha1);
        if (!(cfg->rsr_alpha2 >= 0.0 && cfg->rsr_alpha2 < 1.0))
            return fail(GS_EINVAL, "rsr_alpha2 = %g, must be in [0, 1)", cfg->rsr_alpha2);
        if (!(cfg->rsr_ratio >= 0.0 && cfg->rsr_ratio <= 1.0))
            return fail(GS_EINVAL, "rsr_ratio = %g, must be in [0, 1]", cfg->rsr_ratio);
    }
    h->beta1 = (float)cfg->beta1;
    h->omb1 = (float)(1.0 - cfg->beta1);
    h->beta2 = (float)cfg->beta2;
    h->omb2 = (float)(1.0 - cfg->beta2);
    h->logb1 = cfg->beta1 > 0.0 ? (float)std::log(cfg->beta1) : -INFINITY;
    h->logb2 = cfg->beta2 > 0.0 ? (float)std::log(cfg->beta2) : -INFINITY;
    h->eps = (float)cfg->eps;
    h->rsr_a1 = (float)cfg->rsr_alpha1;
    h->rsr_a2 = (float)cfg->rsr_alpha2;
    h->c1_rsr = (float)(cfg->beta1 * cfg->rsr_alpha1);
    h->c2_rsr = (float)(cfg->beta2 * cfg->rsr_alpha2);
    h->sr = (cfg->moment_dtype == GS_MOMENT_BF16 && cfg->stochastic_round) ? 1 : 0;
    h->rsr_thr = cfg->rsr_enable ? sample_threshold(cfg->rsr_ratio) : 0;
    if (cfg->aiu_enable && (!(cfg->aiu_ratio >= 0.0 && cfg->aiu_ratio <= 1.0) || !(cfg->aiu_scale >= 0.0) ||
                            !finite_d(cfg->aiu_scale)))
        return fail(GS_EINVAL, "aiu_ratio must be in [0, 1] and aiu_scale finite and >= 0");
    h->aiu_thr = cfg->aiu_enable ? sample_threshold(cfg->aiu_ratio) : 0;
    h->aiu_scale = cfg->aiu_enable ? cfg->aiu_scale : 0.0;
    h->seed = cfg->seed;
    h->reg_norm = cfg->reg_norm;
    h->iteration = cfg->iteration;
    h->noise = cfg->noise_enable ? 1 : 0;
    for (int k = 0; k < 4; ++k) h->noise_g[k] = cfg->noise_enable ? cfg->noise_groups[k] : 0;
    h->noise_lr = cfg->noise_enable ? cfg->noise_lr : 0.0;
    h->noise_k = (float)cfg->noise_k;
    h->noise_t = (float)cfg->noise_t;
    if (cfg->noise_enable && (!(cfg->noise_lr >= 0.0) || !finite_d(cfg->noise_lr) || !finite_d(cfg->noise_k) ||
                              !finite_d(cfg->noise_t)))
        return fail(GS_EINVAL, "noise_lr must be finite and >= 0; noise_k, noise_t finite");
    return GS_OK;
}

// Position noise reads the quaternion, log-scale and opacity groups of the
// scene: their indices and dims must fit.
gs_status check_noise_groups(const gs_step_config* cfg, const gs_group* groups, int32_t n_groups, const char* prefix)
{
    if (!cfg->noise_enable) return GS_OK;
    static const int dims[4] = {3, 3, 4, 1};
    for (int k = 0; k < 4; ++k) {
        const int g = cfg->noise_groups[k];
        if (g < 0 || g >= n_groups) return fail(GS_EINVAL, "%snoise_groups[%d] = %d out of range", prefix, k, g);
        if (groups[g].dim != dims[k])
            return fail(GS_EINVAL, "%snoise_groups[%d] = %d has dim %d, expected %d", prefix, k, g, groups[g].dim, dims[k]);
        for (int j = 0; j < k; ++j)
            if (cfg->noise_groups[j] == g) return fail(GS_EINVAL, "%snoise_groups must be distinct", prefix);
    }
    return GS_OK;
}

bool any_adaptive(const gs_group* groups, int32_t n_groups)
{
    if (groups == nullptr) return false;
    for (int g = 0; g < n_groups && g < GS_MAX_GROUPS; ++g)
        if (groups[g].dar_kind != GS_DAR_NONE && groups[g].reg_mode == GS_REG_ADAPTIVE) return true;
    return false;
}

bool valid_unit(int sched, int unit)
{
    if (sched == kSchedCompacted) return unit == 32 || unit == 64 || unit == 128 || unit == 256 || unit == 512;
    if (sched == kSchedMasked) return unit == 32 || unit == 64 || unit == 128 || unit == 256 || unit == 512;
    if (sched == kSchedDense) return unit == 64 || unit == 256 || unit == 512;
    return false;
}

// Units that were fastest on the 3M-primitive scene (Morton order, 29 % visible).
int default_unit(int sched) { return sched == kSchedCompacted ? 64 : sched == kSchedMasked ? 32 : 64; }

// Resolves the schedule and unit of a scene from what the caller supplied.
gs_status resolve_schedule(int requested, int unit, float hint, int64_t n, int n_groups, const int32_t* dims,
                           int dtype, const uint8_t* mask, const int32_t* idx, const int32_t* count,
                           int* sched_out, int* unit_out, const char* prefix)
{
    int sched = requested;
    if (sched == GS_SCHED_AUTO) {
        int tuned_s = 0, tuned_u = 0;
        if (hint > 0.0f && tuner_lookup(n, hint, dtype, &tuned_s, &tuned_u) &&
            ((tuned_s == kSchedCompacted && idx && count) || (tuned_s == kSchedMasked && mask))) {
            sched = tuned_s;
            if (unit == 0) unit = tuned_u;
        } else if (idx != nullptr && count != nullptr) {
            sched = kSchedCompacted;
        } else if (mask != nullptr) {
            sched = kSchedMasked;
        } else {
            sched = kSchedDense;
        }
    }
    (void)n_groups;
    (void)dims;
    if (n > 0 && sched == kSchedCompacted && (idx == nullptr || count == nullptr))
        return fail(GS_EINVAL, "%scompacted schedule needs vis_idx and vis_count", prefix);
    if (n > 0 && sched == kSchedMasked && mask == nullptr)
        return fail(GS_EINVAL, "%smasked schedule needs visible", prefix);
    if (sched != kSchedCompacted && sched != kSchedMasked && sched != kSchedDense)
        return fail(GS_EINVAL, "%sunknown schedule %d", prefix, requested);
    if (unit == 0) unit = default_unit(sched);
    if (!valid_unit(sched, unit)) return fail(GS_EINVAL, "%sunit %d not available for schedule %d", prefix, unit, sched);
    if (sched == kSchedCompacted && !aligned(idx, 4)) return fail(GS_EINVAL, "%svis_idx misaligned", prefix);
    *sched_out = sched;
    *unit_out = unit;
    return GS_OK;
}

}  // namespace gs

using namespace gs;

extern "C" {

const char* gs_last_error(void) { return t_err.c_str(); }

int32_t gs_version(void) { return GSOPT_VERSION; }

double gs_reg_norm(double n_pixels)
{
    if (!(n_pixels >= 1.0) || !std::isfinite(n_pixels)) return 0.0;
    uint64_t v = (uint64_t)n_pixels;
    uint64_t p = 1;
    while (v / p >= 10) p *= 10;
    return (double)((v / p) * p) / 10.0;
}

// Validates a camera and fills its kernel view (prefix names it in messages).
static gs_status to_kcamera(const gs_camera* cam, KCamera* k, const char* prefix)
{
    if (cam->width < 1 || cam->height < 1) return fail(GS_EINVAL, "%scamera width/height must be >= 1", prefix);
    if (!(cam->z_near >= 0.0f) || !(cam->z_far > cam->z_near))
        return fail(GS_EINVAL, "%scamera needs 0 <= z_near < z_far", prefix);
    for (int j = 0; j < 12; ++j)
        if (!std::isfinite(cam->view[j])) return fail(GS_EINVAL, "%scamera view matrix must be finite", prefix);
    if (!std::isfinite(cam->fx) || !std::isfinite(cam->fy) || !std::isfinite(cam->cx) || !std::isfinite(cam->cy))
        return fail(GS_EINVAL, "%scamera intrinsics must be finite", prefix);
    memcpy(k->R, cam->view, sizeof k->R);
    k->fx = cam->fx;
    k->fy = cam->fy;
    k->cx = cam->cx;
    k->cy = cam->cy;
    k->W = (float)cam->width;
    k->H = (float)cam->height;
    k->z_near = cam->z_near;
    k->z_far = cam->z_far;
    k->r_min = cam->r_min_px;
    k->f_max = cam->fx > cam->fy ? cam->fx : cam->fy;
    return GS_OK;
}

gs_status gs_visibility(const float* means, int64_t means_stride, const float* radius, int64_t n,
                        const gs_camera* cam, uint8_t* mask, int32_t* vis_idx, int32_t* vis_count, hipStream_t stream)
{
    clear_error();
    if (n < 0 || n >= ((int64_t)1 << 31)) return fail(GS_EINVAL, "n = %lld, must be in [0, 2^31)", (long long)n);
    int64_t ms = 0;
    if (!means_rows(means_stride, n, &ms)) return fail(GS_EINVAL, "means_stride = %lld: must be 0 or >= 3 (and n * stride < 2^40)", (long long)means_stride);
    if (cam == nullptr) return fail(GS_EINVAL, "cam is NULL");
    if (mask == nullptr && vis_idx == nullptr) return fail(GS_EINVAL, "mask and vis_idx are both NULL");
    if (vis_idx != nullptr && vis_count == nullptr) return fail(GS_EINVAL, "vis_idx needs vis_count");
    if (n > 0 && means == nullptr) return fail(GS_EINVAL, "means is NULL");
    if (!aligned(means, 4) || !aligned(radius, 4) || !aligned(vis_idx, 4) || !aligned(vis_count, 4))
        return fail(GS_EINVAL, "misaligned pointer (4-byte alignment required)");
    KCamera k;
    const gs_status st = to_kcamera(cam, &k, "");
    if (st != GS_OK) return st;
    const hipError_t e = launch_visibility(means, ms, radius, n, k, mask, vis_idx, vis_count, stream);
    return e == hipSuccess ? GS_OK : hip_fail(e, "gs_visibility launch");
}

gs_status gs_visibility_multi(const float* means, int64_t means_stride, const float* radius, int64_t n,
                              const gs_camera* cams, int32_t n_cams, uint8_t* mask, uint32_t* view_bits,
                              int32_t* vis_idx, int32_t* vis_count, hipStream_t stream)
{
    clear_error();
    if (n < 0 || n >= ((int64_t)1 << 31)) return fail(GS_EINVAL, "n = %lld, must be in [0, 2^31)", (long long)n);
    int64_t ms = 0;
    if (!means_rows(means_stride, n, &ms)) return fail(GS_EINVAL, "means_stride = %lld: must be 0 or >= 3 (and n * stride < 2^40)", (long long)means_stride);
    if (cams == nullptr) return fail(GS_EINVAL, "cams is NULL");
    if (n_cams < 1 || n_cams > kMaxViews) return fail(GS_EINVAL, "n_cams = %d, must be in [1, %d]", n_cams, kMaxViews);
    if (mask == nullptr && view_bits == nullptr && vis_idx == nullptr)
        return fail(GS_EINVAL, "mask, view_bits and vis_idx are all NULL");
    if (vis_idx != nullptr && vis_count == nullptr) return fail(GS_EINVAL, "vis_idx needs vis_count");
    if (n > 0 && means == nullptr) return fail(GS_EINVAL, "means is NULL");
    if (!aligned(means, 4) || !aligned(radius, 4) || !aligned(view_bits, 4) || !aligned(vis_idx, 4) ||
        !aligned(vis_count, 4))
        return fail(GS_EINVAL, "misaligned pointer (4-byte alignment required)");
    KCameras k;
    memset(&k, 0, sizeof k);
    for (int v = 0; v < n_cams; ++v) {
        char prefix[32];
        snprintf(prefix, sizeof prefix, "view %d: ", v);
        const gs_status st = to_kcamera(&cams[v], &k.c[v], prefix);
        if (st != GS_OK) return st;
    }
    k.n = n_cams;
    const hipError_t e = launch_visibility_multi(means, ms, radius, n, k, mask, view_bits, vis_idx, vis_count, stream);
    return e == hipSuccess ? GS_OK : hip_fail(e, "gs_visibility_multi launch");
}

gs_status gs_compact(const uint8_t* mask, int64_t n, int32_t* vis_idx, int32_t* vis_count, hipStream_t stream)
{
    clear_error();
    if (n < 0 || n >= ((int64_t)1 << 31)) return fail(GS_EINVAL, "n = %lld, must be in [0, 2^31)", (long long)n);
    if (vis_idx == nullptr || vis_count == nullptr) return fail(GS_EINVAL, "vis_idx and vis_count are required");
    if (n > 0 && mask == nullptr) return fail(GS_EINVAL, "mask is NULL");
    if (!aligned(vis_idx, 4) || !aligned(vis_count, 4)) return fail(GS_EINVAL, "misaligned pointer");
    const hipError_t e = launch_compact(mask, n, vis_idx, vis_count, stream);
    return e == hipSuccess ? GS_OK : hip_fail(e, "gs_compact launch");
}

gs_status adamw_gs_step(const gs_group* groups, int32_t n_groups, int64_t n, const uint8_t* visible,
                        const int32_t* vis_idx, const int32_t* vis_count, int32_t* step_count,
                        const gs_step_config* cfg, hipStream_t stream)
{
    clear_error();
    if (n < 0 || n >= ((int64_t)1 << 31)) return fail(GS_EINVAL, "n = %lld, must be in [0, 2^31)", (long long)n);
    if (n > 0 && step_count == nullptr) return fail(GS_EINVAL, "step_count is NULL");
    if (!aligned(step_count, 4) || !aligned(vis_count, 4)) return fail(GS_EINVAL, "misaligned step_count/vis_count");
    KHyper h;
    gs_status st = build_hyper(cfg, any_adaptive(groups, n_groups), &h);
    if (st != GS_OK) return st;
    KScene s;
    memset(&s, 0, sizeof s);
    st = build_groups(groups, n_groups, n, cfg->moment_dtype, cfg, &s, "");
    if (st != GS_OK) return st;
    st = check_noise_groups(cfg, groups, n_groups, "");
    if (st != GS_OK) return st;
    int32_t dims[GS_MAX_GROUPS];
    for (int g = 0; g < n_groups; ++g) dims[g] = groups[g].dim;
    int sched = 0, unit = 0;
    st = resolve_schedule(cfg->schedule, cfg->unit, cfg->visible_hint, n, n_groups, dims, cfg->moment_dtype, visible,
                          vis_idx, vis_count, &sched, &unit, "");
    if (st != GS_OK) return st;
    if (n > 0 && (h.rsr_thr > 0 || h.aiu_thr > 0) && sched != kSchedDense && visible == nullptr)
        return fail(GS_EINVAL, "RSR or AIU with a sparse schedule needs the visibility mask (to find invisible rows)");
    // masked windows of 32 are the default; with position noise 64 is faster
    if (cfg->unit == 0 && cfg->noise_enable && sched == kSchedMasked && unit == 32) unit = 64;
    if (sched != kSchedDense) unit = fit_unit(n, unit, 512);
    s.sched = sched;
    s.unit = unit;
    s.mask = visible;
    s.idx = vis_idx;
    s.count = vis_count;
    s.t = step_count;
    if (trace_on()) {
        char detail[32] = "";
        if (s.pk_stride > 0) snprintf(detail, sizeof detail, "rows=packed%d", s.pk_stride);
        trace_step("adamw_gs_step", n, n_groups,
                   sched == kSchedCompacted ? "compacted" : sched == kSchedMasked ? "masked" : "dense", unit, cfg,
                   detail);
    }
    const hipError_t e = launch_step(s, h, stream);
    return e == hipSuccess ? GS_OK : hip_fail(e, "adamw_gs_step launch");
}

gs_status adamw_gs_step_view(const gs_group* groups, int32_t n_groups, int64_t n, const float* means,
                             int64_t means_stride, const float* radius, const gs_camera* cams, int32_t n_cams,
                             uint8_t* visible_out, int32_t* step_count, const gs_step_config* cfg, hipStream_t stream)
{
    clear_error();
    if (n < 0 || n >= ((int64_t)1 << 31)) return fail(GS_EINVAL, "n = %lld, must be in [0, 2^31)", (long long)n);
    int64_t ms = 0;
    if (!means_rows(means_stride, n, &ms)) return fail(GS_EINVAL, "means_stride = %lld: must be 0 or >= 3 (and n * stride < 2^40)", (long long)means_stride);
    if (cams == nullptr) return fail(GS_EINVAL, "cams is NULL");
    if (n_cams < 1 || n_cams > kMaxViews) return fail(GS_EINVAL, "n_cams = %d, must be in [1, %d]", n_cams, kMaxViews);
    if (n > 0 && (step_count == nullptr || means == nullptr)) return fail(GS_EINVAL, "step_count or means is NULL");
    if (!aligned(step_count, 4) || !aligned(means, 4) || !aligned(radius, 4))
        return fail(GS_EINVAL, "misaligned step_count/means/radius");
    KCameras k;
    memset(&k, 0, sizeof k);
    gs_status st = GS_OK;
    for (int v = 0; v < n_cams && st == GS_OK; ++v) {
        char prefix[32] = "";
        if (n_cams > 1) snprintf(prefix, sizeof prefix, "view %d: ", v);
        st = to_kcamera(&cams[v], &k.c[v], prefix);
    }
    if (st != GS_OK) return st;
    k.n = n_cams;
    KHyper h;
    st = build_hyper(cfg, any_adaptive(groups, n_groups), &h);
    if (st != GS_OK) return st;
    KScene s;
    memset(&s, 0, sizeof s);
    st = build_groups(groups, n_groups, n, cfg->moment_dtype, cfg, &s, "");
    if (st != GS_OK) return st;
    st = check_noise_groups(cfg, groups, n_groups, "");
    if (st != GS_OK) return st;
    // the fastest windows on the 3M scene: 32 for the plain step; 64 with
    // position noise (its per-row arithmetic runs on twice as many lanes) and
    // on Re-State or AIU calls (each wave's pass over its window's sampled
    // invisible rows then serves twice as many rows)
    const bool wide = cfg->noise_enable || cfg->rsr_enable || cfg->aiu_enable;
    const int unit = cfg->unit != 0 ? cfg->unit : wide ? 64 : 32;
    if (unit != 32 && unit != 64 && unit != 128 && unit != 256)
        return fail(GS_EINVAL, "unit = %d: the view step takes 32, 64, 128 or 256 primitives per wave", cfg->unit);
    s.sched = kSchedMasked;
    s.unit = fit_unit(n, unit, 256);
    s.t = step_count;
    if (trace_on()) {
        char detail[48];
        if (s.pk_stride > 0) snprintf(detail, sizeof detail, "views=%d rows=packed%d", n_cams, s.pk_stride);
        else snprintf(detail, sizeof detail, "views=%d", n_cams);
        trace_step("adamw_gs_step_view", n, n_groups, "view", s.unit, cfg, detail);
    }
    const hipError_t e = launch_step_view(s, h, k, means, ms, radius, visible_out, stream);
    return e == hipSuccess ? GS_OK : hip_fail(e, "adamw_gs_step_view launch");
}

}  // extern "C"
