// Internal declarations of the gfx950 AdamW-GS library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gsopt.h"

namespace gs {

constexpr int kWave = 64;            // CDNA wavefront
constexpr int kWavesPerBlock = 4;
constexpr int kBlock = kWave * kWavesPerBlock;
constexpr int kCap = 512;            // max rows a wave stages per unit
constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;

enum : uint64_t { kTagRsr = 1, kTagSrStep = 16, kTagSrRsr = 32 };   // kTagSrRsr: rounding in the invisible pass
enum : int { kSchedCompacted = 1, kSchedMasked = 2, kSchedDense = 3 };

// One attribute group as the kernels see it.
struct KGroup {
    float* param;
    const float* grad;
    void* m;
    void* v;
    int32_t dim;
    int32_t vec;         // elements per access: 4, 2 or 1
    int32_t cpr;         // accesses per row = dim / vec
    float lr;
    int32_t dar_kind;
    int32_t reg_mode;
    float dar_clip;
    int32_t stride;      // elements from one row to the next (>= dim)
    double dar_lambda;   // lambda; the kernels form lambda / N_I' in double, as the host would
};

// Per-call scalars.
struct KHyper {
    float beta1, omb1, beta2, omb2;   // beta and (1 - beta), both rounded from double
    float logb1, logb2;               // log(beta) rounded from double (-inf for beta = 0)
    float eps;
    float rsr_a1, rsr_a2;
    float c1_rsr, c2_rsr;             // beta1*alpha1, beta2*alpha2: moment decay of a sampled visible row
    int32_t sr;                       // stochastic rounding of BF16 moments
    uint64_t rsr_thr;                 // sampled iff draw >> 32 < rsr_thr
    uint64_t seed;                    // draws of scene s use seed + s (see KScene::seed_offset)
    double reg_norm;                  // N_I'
    int64_t iteration;
    // position noise on the mean group
    int32_t noise;                    // 1 = on
    int32_t noise_g[4];               // groups: mean, log-scale, quaternion, opacity logit
    double noise_lr;                  // eta_{R_o} (multiplied by the mean group's lr on the device, in double)
    float noise_k, noise_t;           // lambda_mu, lambda_t
    // Artificial Implicit Update of sampled invisible rows
    uint64_t aiu_thr;                 // sampled iff draw >> 32 < aiu_thr; 0 = off
    double aiu_scale;                 // eta_AIU (multiplied by each group's lr on the device, in double)
};

enum : uint64_t { kTagNoise = 48, kTagAiu = 64 };

// One scene: its groups, visibility inputs and schedule.
struct KScene {
    KGroup g[GS_MAX_GROUPS];
    int32_t n_groups;
    int32_t sched;
    int32_t unit;                      // rows (compacted) or primitives (masked/dense) per wave unit
    int32_t bf16;
    int64_t seed_offset;               // added to the call's seed: 0, or the scene's place in a batch
    int64_t n;
    const uint8_t* mask;
    const int32_t* idx;
    const int32_t* count;
    int32_t* t;
    // Packed rows: every group is a column range of the same [n][pk_stride]
    // arrays (pk_param, pk_grad, pk_m, pk_v), pk_stride a power of two in
    // [4, 256]; the step then takes each row in one pass (set by
    // plan_packed_rows; pk_stride = 0 otherwise).
    int32_t pk_stride;
    int32_t pk_col[GS_MAX_GROUPS];     // first column of each group
    float* pk_param;
    const float* pk_grad;
    void* pk_m;
    void* pk_v;
};

// Sets the packed-row fields of a scene whose groups are set (msz: bytes
// per moment element): packed when all groups share one row stride that is
// a power of two in [4, 256], lie at the same column in the attribute,
// gradient and both moment arrays, do not overlap, and the arrays' row
// starts allow 16-byte attribute and 4-element moment accesses.
void plan_packed_rows(KScene& s, size_t msz);

struct KCamera {
    float R[12];
    float fx, fy, cx, cy;
    float W, H;
    float z_near, z_far;
    float r_min, f_max;
};

// up to 32 views for the multi-view visibility pass (kernel argument)
constexpr int kMaxViews = 32;
struct KCameras {
    KCamera c[kMaxViews];
    int32_t n;
};

// host-side helpers shared by the library's translation units
uint64_t splitmix_output(uint64_t s, uint64_t k);

// means: rows ms elements apart (ms >= 3)
hipError_t launch_visibility(const float* means, int64_t ms, const float* radius, int64_t n, const KCamera& cam,
                             uint8_t* mask, int32_t* idx, int32_t* count, hipStream_t stream);
hipError_t launch_step_view(const KScene& s, const KHyper& h, const KCameras& cams, const float* means, int64_t ms,
                            const float* radius, uint8_t* mask_out, hipStream_t stream);
hipError_t launch_visibility_multi(const float* means, int64_t ms, const float* radius, int64_t n,
                                   const KCameras& cams, uint8_t* mask, uint32_t* bits, int32_t* idx, int32_t* count,
                                   hipStream_t stream);
hipError_t launch_compact(const uint8_t* mask, int64_t n, int32_t* idx, int32_t* count, hipStream_t stream);
// The invisible-row pass (Re-State / AIU samples) runs first when either is on.
hipError_t launch_step(const KScene& s, const KHyper& h, hipStream_t stream);
hipError_t launch_invisible(const KScene& s, const KHyper& h, hipStream_t stream);
size_t step_kernel_units(const KScene& s);


// batched
struct BatchDevice;  // defined in batched.hip
hipError_t launch_batched(const KScene* d_scenes, int32_t n_scenes, const int64_t* d_unit_prefix_max,
                          int32_t* d_queue, int grid, const KHyper& h, int rsr, hipStream_t stream);

// relocation
size_t relocate_workspace_bytes(int64_t n);
hipError_t launch_relocate(const float* key, int64_t key_stride, int64_t n, int64_t k, const KScene& s, int reset_t,
                           int32_t* selected, void* ws, hipStream_t stream);

}  // namespace gs
