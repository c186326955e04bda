/*
 * gsopt.h -- C ABI of the MI355X (gfx950) AdamW-GS optimizer step.
 *
 * Method: "A Step to Decouple Optimization in 3DGS" (ICLR 2026, arXiv
 * 2601.16736).  AdamW-GS recouples three parts (Sec. "Recoupling: AdamW-GS"):
 *   - Sparse Adam: only primitives visible from the current view advance
 *     their moments, step count and attributes (Sec. "Characteristics of
 *     Sparse Adam", sparse-beta equation), each with its own step count t_i
 *     (asynchronous indexing, Sec. "Update-step decoupling");
 *   - Re-State Regularization (RSR): at scheduled iterations a uniform sample
 *     of the existing primitives has its moments rescaled, m <- alpha1 m,
 *     v <- alpha2 v (Re-State equation);
 *   - Decoupled Attribute Regularization (DAR): the moments see only the
 *     photometric gradient (decoupled-moment equation) and the regulariser
 *     enters the update outside them, preconditioned by sqrt(v_hat) and
 *     clamped at C (DAR update equation; per-attribute forms for opacity and
 *     log-scale in Sec. "Implementation Details / AdamW-GS").
 *
 * Conventions shared by every entry point:
 *   - Array arguments are DEVICE pointers owned by the caller; the library
 *     never frees them and keeps no reference after the call is enqueued.
 *     Structs passed by pointer (gs_camera, gs_group, gs_step_config,
 *     gs_scene) are HOST memory, read during the call only.
 *   - Every call is asynchronous on `stream` (0 = the null stream).
 *   - Argument errors are found on the host before anything is enqueued and
 *     return GS_EINVAL; nothing is launched then.  A failed launch returns
 *     GS_EHIP.  gs_last_error() gives the calling thread's last message.
 *   - NaN and Inf propagate per element; nothing is clamped or "repaired".
 *   - Indices are int32: n must be below 2^31.
 *   - Attribute groups are row-major [n][dim] (the 3DGS convention of one
 *     tensor per attribute group), or, with gs_group.row_stride, column
 *     ranges of wider row-major arrays: several groups may then share one
 *     packed [n][row_stride] array per role (attributes, gradients, each
 *     moment), so that all of a primitive's state sits in one line-aligned
 *     row.  Rows of one group are updated independently; no two groups may
 *     overlap.  When every group of a scene lies in the same packed arrays
 *     (one row stride, a power of two from 4 to 256, each group at the same
 *     column in the attribute, gradient and both moment arrays, row starts
 *     16-byte aligned for the attributes and 4-element aligned for the
 *     moments) the step takes each visible row in one pass, and writes whole
 *     rows: the columns no group covers are read and written back with the
 *     bits they held, so nothing else may write them during a step.
 *   - A `means` argument is [n][3] FP32 with rows means_stride elements
 *     apart (0 = 3), so the means may be the mean group's columns of a
 *     packed array.
 */
#ifndef GSOPT_H
#define GSOPT_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GSOPT_VERSION 2
#define GS_MAX_GROUPS 8

typedef enum {
    GS_OK = 0,
    GS_EINVAL = 1,        /* invalid argument; nothing enqueued */
    GS_EHIP = 2,          /* a HIP call or kernel launch failed */
    GS_ENOMEM = 3,        /* allocation failed (plans and the tuner only) */
    GS_EUNSUPPORTED = 4   /* valid but not supported here (e.g. no gfx950 device) */
} gs_status;

/* Last error message of the calling thread ("" if none).  Never NULL. */
const char* gs_last_error(void);

/* GSOPT_VERSION of the built library. */
int32_t gs_version(void);

/* ------------------------------------------------------------------------
 * Visibility (the filter V of the sparse-beta equation).
 *
 * The paper takes V from the rasterizer ("visible from the current
 * viewpoint").  Here V is the frustum/radius cull of each projected mean,
 * defined as an FP32 computation in this exact order, one rounding per
 * operation and no fused multiply-add, so that a reimplementation anywhere
 * reproduces the mask bit for bit:
 *   p = R mu + t           each row as ((R_k0*x + R_k1*y) + R_k2*z) + t_k
 *   visible requires  z_near < p_z < z_far
 *   u = (fx*p_x)/p_z + cx,   v = (fy*p_y)/p_z + cy
 *   r = (max(fx,fy)*rho_i)/p_z and r >= r_min_px   if radius != NULL, else r = 0
 *   u + r >= 0,  u - r <= width,  v + r >= 0,  v - r <= height
 * A NaN anywhere makes the primitive invisible.
 * ---------------------------------------------------------------------- */
typedef struct {
    float view[12];          /* row-major 3x4 [R|t], world -> camera; camera looks along +z,
                                image x right, y down */
    float fx, fy, cx, cy;    /* pixels */
    int32_t width, height;   /* pixels, >= 1 */
    float z_near, z_far;     /* 0 <= z_near < z_far; z_far may be +INFINITY */
    float r_min_px;          /* radius cull threshold; used only when radius != NULL */
} gs_camera;

/*
 * means   [n][3] FP32, 4-byte aligned, rows means_stride elements apart
 *         (0 = 3; otherwise >= 3).
 * radius  [n] FP32 world-space bounding radius per primitive, or NULL.
 * mask    [n] uint8 out (1 visible, 0 not), or NULL.
 * vis_idx [n] int32 out: indices of the visible primitives, or NULL.  The
 *         order is unspecified (rows are updated independently, so it does
 *         not change any result); each visible index appears exactly once.
 * vis_count  device int32 scalar out (number of visible primitives); required
 *         when vis_idx != NULL.  It is overwritten, not accumulated.
 * At least one of mask and vis_idx must be non-NULL.
 */
gs_status gs_visibility(const float* means, int64_t means_stride, const float* radius, int64_t n,
                        const gs_camera* cam, uint8_t* mask, int32_t* vis_idx,
                        int32_t* vis_count, hipStream_t stream);

/*
 * Several views in one pass (a batch of training views; the paper trains on
 * one view per iteration and is silent on batches).  The predicate above is
 * evaluated for each of the n_cams (1..32) cameras:
 * view_bits [n] uint32 out, bit v = visible in cams[v], or NULL;
 * mask      [n] uint8 out, 1 where any view sees the primitive (the union, the
 *           V of a step over the batch), or NULL;
 * vis_idx / vis_count: the union's indices, as for gs_visibility, or NULL.
 * At least one output must be non-NULL.  cams is a host array.
 */
gs_status gs_visibility_multi(const float* means, int64_t means_stride, const float* radius, int64_t n,
                              const gs_camera* cams, int32_t n_cams, uint8_t* mask,
                              uint32_t* view_bits, int32_t* vis_idx, int32_t* vis_count,
                              hipStream_t stream);

/*
 * Compaction alone: vis_idx/vis_count from an existing mask ([n] uint8,
 * nonzero = visible).  Same output contract as gs_visibility.
 */
gs_status gs_compact(const uint8_t* mask, int64_t n, int32_t* vis_idx, int32_t* vis_count,
                     hipStream_t stream);

/* ------------------------------------------------------------------------
 * The step.
 * ---------------------------------------------------------------------- */
typedef enum {
    GS_DAR_NONE = 0,               /* plain sparse Adam ("other attributes" equation) */
    GS_DAR_OPACITY_SIGMOID = 1,    /* theta = opacity logit tau, R'(tau) = sigma(tau)(1 - sigma(tau)) */
    GS_DAR_LOGSCALE_EXP = 2        /* theta = log-scale kappa,  R'(kappa) = exp(kappa) */
} gs_dar_kind;

typedef enum {
    GS_REG_ADAPTIVE = 0,           /* DAR: + min(lambda R'/N_I' / (sqrt(v_hat)+eps), C)   (AdamW-GS) */
    GS_REG_CONSTANT = 1,           /* AdamW-style constant penalty: + lambda R'            (comparison variant) */
    GS_REG_CONSTANT_CLIPPED = 2    /* AdamW-style, clipped: + min(lambda R', C)            (comparison variant) */
} gs_reg_mode;

typedef enum { GS_MOMENT_F32 = 0, GS_MOMENT_BF16 = 1 } gs_moment_dtype;

typedef enum {
    GS_SCHED_AUTO = 0,       /* the tuner's choice for (n, visible_hint, dtype), else by inputs */
    GS_SCHED_COMPACTED = 1,  /* waves take slices of vis_idx (needs vis_idx, vis_count) */
    GS_SCHED_MASKED = 2,     /* waves sweep windows of the mask (needs visible) */
    GS_SCHED_DENSE = 3       /* V = 1 for all n primitives: synchronous Adam + DAR */
} gs_schedule;

typedef struct {
    float* param;            /* theta [n][dim] FP32, updated in place */
    const float* grad;       /* photometric gradient [n][dim] FP32; read on visible rows only */
    void* exp_avg;           /* m [n][dim], FP32 or BF16 per moment_dtype, updated in place */
    void* exp_avg_sq;        /* v [n][dim], same dtype as exp_avg */
    int32_t dim;             /* >= 1 */
    int32_t dar_kind;        /* gs_dar_kind */
    int32_t reg_mode;        /* gs_reg_mode (ignored when dar_kind == GS_DAR_NONE) */
    int32_t row_stride;      /* elements from the start of one row to the next, the same in param, grad,
                                exp_avg and exp_avg_sq: 0 = dim (contiguous rows), else >= dim (the group
                                is dim columns of [n][row_stride] arrays) */
    double lr;               /* eta of this attribute group, finite */
    double dar_lambda;       /* lambda_theta >= 0 */
    double dar_clip;         /* C >= 0 (the paper's C_t, a constant per group) */
} gs_group;

typedef struct {
    double beta1, beta2;     /* 0 <= beta < 1 */
    double eps;              /* > 0, added outside the square root */
    double reg_norm;         /* N_I' > 0: pixel normaliser of DAR; see gs_reg_norm() */
    uint64_t seed;           /* key of the RSR sampler and the stochastic-rounding draws */
    int64_t iteration;       /* training iteration; keys the draws together with seed */
    int32_t moment_dtype;    /* gs_moment_dtype */
    int32_t stochastic_round;/* BF16 only: 1 = stochastic rounding of moment writes, 0 = nearest-even */
    int32_t rsr_enable;      /* 1 = apply Re-State Regularization in this call */
    int32_t schedule;        /* gs_schedule */
    double rsr_alpha1;       /* 0 <= alpha1 < 1 */
    double rsr_alpha2;       /* 0 <= alpha2 < 1 (the paper uses alpha2 = alpha1^2) */
    double rsr_ratio;        /* sampling probability p in [0, 1] */
    float visible_hint;      /* expected visible fraction for GS_SCHED_AUTO (<= 0: unknown) */
    int32_t unit;            /* rows (compacted: 32, 64, 128, 256, 512) / primitives (masked: 32, 64,
                                128, 256, 512; dense: 64, 256, 512) per wave; 0 = default (compacted 64,
                                masked 32 or, with position noise, 64; dense 64).  A scene too
                                large for one dispatch at this unit (above 2^31 - 128 rows at 32) runs
                                at the next size, with the same results */
    /* Position noise (Implementation Details, position equations): each
     * visible primitive's mean also moves by -eta_{R_o} R_mu, R_mu =
     * eta_mu sigma(-lambda_mu (sigma(tau) - lambda_t)) Sigma gamma, with
     * Sigma = R(q) diag(exp(2 kappa)) R(q)^T from the pre-update quaternion
     * q = (w, x, y, z) (normalised) and log-scale kappa, tau the pre-update
     * opacity logit, eta_mu the mean group's lr, and gamma ~ N(0, I3) by the
     * Box-Muller transform of two draws d1, d2 (outputs 2i+1, 2i+2 of the
     * stream keyed by (seed, tag 48, iteration)): u = (top 24 bits + 1)/2^24,
     * a = (bits 31..8)/2^24, gamma = (r1 cos 2 pi a1, r1 sin 2 pi a1,
     * r2 cos 2 pi a2), r = sqrt(-2 ln u).  The paper takes lambda_mu,
     * lambda_t and eta_{R_o} from 3DGS-MCMC without printing them. */
    int32_t noise_enable;    /* 1 = on */
    int32_t noise_groups[4]; /* group indices of the mean (dim 3), log-scale (dim 3),
                                quaternion (dim 4) and opacity logit (dim 1) */
    double noise_lr;         /* eta_{R_o} >= 0 */
    double noise_k;          /* lambda_mu */
    double noise_t;          /* lambda_t */
    /* Artificial Implicit Update (Sec. "Update-step decoupling", AIU): each
     * invisible primitive is sampled with probability aiu_ratio (Pro_AIU) by
     * the Re-State rule on stream tag 64, and a sampled one with t_i > 0
     * takes theta <- theta - lr aiu_scale (m/b1)/(sqrt(v/b2) + eps) from its
     * moments after this call's Re-State rescale, with b1, b2 from its
     * current t_i; m, v and t_i stay unchanged, and no regulariser term is
     * added.  The paper's comparison tool; AdamW-GS itself runs without it. */
    int32_t aiu_enable;      /* 1 = on */
    double aiu_ratio;        /* Pro_AIU in [0, 1] */
    double aiu_scale;        /* eta_AIU >= 0 */
} gs_step_config;

/*
 * N_I' from the image pixel count N_I: the most significant decimal digit
 * of N_I is kept and the result divided by ten (DAR paragraph of Sec.
 * "Hyperparameter Selection"); e.g. 1000*1000 -> 1e5.  Returns 0 for N_I < 1.
 */
double gs_reg_norm(double n_pixels);

/*
 * One AdamW-GS step over the groups of one scene (Sec. "Recoupling:
 * AdamW-GS"; equations referenced at the top of this file).
 *
 * For every primitive i, in this order:
 *  1. if rsr_enable and i is sampled (below), m <- alpha1 m and v <- alpha2 v
 *     on every element of every group, visible or not; t_i is unchanged;
 *  2. if i is not visible nothing else changes (theta, m, v, t_i);
 *  3. t_i <- t_i + 1, b1 = 1 - beta1^t_i, b2 = 1 - beta2^t_i;
 *  4. per element: m <- beta1 m + (1-beta1) g;  v <- beta2 v + (1-beta2) g^2;
 *     d = sqrt(v/b2) + eps;  u = (m/b1)/d;
 *     DAR groups add min(lambda R'(theta)/N_I'/d, C) (or the reg_mode
 *     variant), with R' at the pre-update theta;
 *     theta <- theta - lr u;
 *  5. with position noise on, visible means also move by -eta_{R_o} R_mu;
 *  6. with AIU on, sampled invisible rows move as stated at aiu_enable.
 * Sampling: the k-th output of a SplitMix64 stream with state s is
 * mix64(s + k*0x9E3779B97F4A7C15) (Steele, Lea & Flood 2014).  With
 * s1 = output (1+1) of the stream seeded with `seed` (tag 1) and
 * s2 = output (iteration+1) of the stream with state s1, primitive i is
 * sampled iff (output (i+1) of the stream with state s2) >> 32 is below
 * floor(rsr_ratio * 2^32) (2^32 when rsr_ratio = 1).
 * BF16 moments are computed in FP32 and rounded once on store, to
 * nearest-even or stochastically: 16 random bits are added below the kept
 * bits, then truncated.  The bits of element e = row*dim+col of group g come
 * from output (floor(e/2)+1) of the stream keyed by (seed, tag 16+g,
 * iteration): for even e bits 63..48 for m and 47..32 for v, for odd e bits
 * 31..16 for m and 15..0 for v.  A sampled visible row is rescaled inside
 * the step (in FP32, before its moment update, no extra rounding); a sampled
 * invisible row is rescaled and rounded with the stream of tag 32+g.
 *
 * visible     [n] uint8 mask (nonzero = visible), or NULL;
 * vis_idx     [n] int32 visible indices (any order, no duplicates), or NULL;
 * vis_count   device int32 scalar, length of vis_idx, or NULL;
 * step_count  [n] int32 t_i, updated in place.
 * GS_SCHED_MASKED needs `visible`; GS_SCHED_COMPACTED needs vis_idx and
 * vis_count, and the index list must match the mask's visible set when both
 * are given (entries outside [0, n) are ignored); GS_SCHED_DENSE ignores all
 * three.  RSR or AIU with a sparse schedule also needs `visible`, to find
 * the invisible sampled rows.  Pointers: 4-byte aligned
 * (BF16 moments 2-byte); wider alignment lets rows use 64/128-bit accesses.
 * Distinct groups must not overlap; overlapping arrays give undefined results.
 */
gs_status adamw_gs_step(const gs_group* groups, int32_t n_groups, int64_t n,
                        const uint8_t* visible, const int32_t* vis_idx, const int32_t* vis_count,
                        int32_t* step_count, const gs_step_config* cfg, hipStream_t stream);

/*
 * Visibility and step in one launch: the predicate of gs_visibility
 * (optional radius) decides V for every primitive from `means` [n][3] as
 * they are when the call starts, then the step above runs with that V.
 * With several cameras (n_cams in 1..32, a host array; a batch of training
 * views) V is their union, as the mask of gs_visibility_multi.  Each wave
 * takes a window of cfg->unit primitives (32, 64, 128 or 256; 0 = 32, or 64
 * with position noise, Re-State or AIU on): it
 * culls the window, steps its visible rows and, when Re-State or AIU is
 * on, treats its invisible sampled rows, so no mask or index list passes
 * through memory in between.  Results equal the visibility call followed
 * by adamw_gs_step with that mask, bit for bit.  cfg->schedule and
 * cfg->visible_hint are ignored.  means is normally the mean group's param
 * array with its row stride (any [n][3] FP32 rows work); visible_out [n] uint8 receives V, or
 * is NULL.  Other arguments as for adamw_gs_step.
 */
gs_status adamw_gs_step_view(const gs_group* groups, int32_t n_groups, int64_t n,
                             const float* means, int64_t means_stride, const float* radius, const gs_camera* cams,
                             int32_t n_cams, uint8_t* visible_out, int32_t* step_count,
                             const gs_step_config* cfg, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Many scenes in one launch.
 * ---------------------------------------------------------------------- */
typedef struct {
    const gs_group* groups;  /* host array of n_groups descriptors (device arrays inside) */
    int32_t n_groups;
    int32_t schedule;        /* GS_SCHED_* for this scene (AUTO: tuner by visible_hint) */
    int64_t n;
    const uint8_t* visible;  /* as in adamw_gs_step */
    const int32_t* vis_idx;
    const int32_t* vis_count;
    int32_t* step_count;
    float visible_hint;      /* expected visible fraction (AUTO only) */
    int32_t reserved;        /* must be 0 */
} gs_scene;

typedef struct gs_batch gs_batch;

/*
 * Builds a plan for 1..64 scenes whose moments are all stored as
 * moment_dtype: validates them, picks each scene's schedule (and wave unit),
 * uploads the scene table to device memory and lays out each scene's range
 * of work units.  Allocates the device table and synchronizes the device;
 * the step calls below do not allocate.  The
 * arrays the scenes point to must stay alive and in place while the plan is
 * used; vis_count values are read on the device at each step.
 */
gs_status gs_batch_create(const gs_scene* scenes, int32_t n_scenes, int32_t moment_dtype, gs_batch** out);

/*
 * One AdamW-GS step for every scene of the plan, as if adamw_gs_step were
 * called once per scene s with cfg->seed + s as the seed (so the scenes'
 * RSR samples and rounding draws are independent); the results are bit for
 * bit those of the per-scene calls.  cfg->schedule, cfg->unit and
 * cfg->visible_hint are ignored (the plan fixed them); cfg->moment_dtype must
 * equal the plan's.  One kernel launch serves every scene's step units and,
 * when Re-State or AIU runs, every scene's windows of invisible rows: each
 * wave takes one unit and finds its scene from the plan's unit ranges.  It
 * is replayed from a HIP graph (the first call instantiates it, later calls
 * only replace its arguments and grid).  Calls on one plan may be issued
 * back to back on one stream; from several host threads at once they race
 * on the plan's host-side argument buffers.
 */
gs_status adamw_gs_step_batched(gs_batch* batch, const gs_step_config* cfg, hipStream_t stream);

/*
 * Launch shape of the plan's steps.  resident = 0 (the default): one wave
 * per work unit, the hardware dispatcher balancing them.  resident = 1: a
 * persistent grid of as many blocks as the device holds at once, whose
 * waves stride over the work units.  Results are the same bits either way.
 * Takes effect at the next adamw_gs_step_batched call.
 */
gs_status gs_batch_set_resident(gs_batch* batch, int32_t resident);

/* Schedule chosen for scene s of the plan (GS_SCHED_*), or -1. */
int32_t gs_batch_scene_schedule(const gs_batch* batch, int32_t s);

/* Frees the plan (synchronizes with its last launch first). NULL is a no-op. */
gs_status gs_batch_destroy(gs_batch* batch);

/* ------------------------------------------------------------------------
 * Relocation state reset (Sec. "Hyperparameter Selection", scaling in RSR:
 * a reallocated primitive starts from zero optimizer state, i.e. RSR with
 * alpha1 = alpha2 = 0).
 * ---------------------------------------------------------------------- */

/* Bytes of device workspace gs_relocate_reset needs for n primitives. */
size_t gs_relocate_workspace_size(int64_t n);

/*
 * Selects the k primitives with the smallest key (e.g. the opacity logit),
 * ties broken by the lower index, and zeroes their m and v in every group;
 * with reset_t also their step count.  key [n] FP32 device (finite values),
 * entries key_stride elements apart (0 = 1; e.g. the opacity column of a
 * packed attribute array), 0 <= k <= n.  selected [k] int32 out (ascending indices) or NULL.
 * workspace: device memory of gs_relocate_workspace_size(n) bytes, 256-byte
 * aligned; contents on entry are ignored.  key must not overlap any group's
 * m or v, step_count or selected: rows are zeroed while keys are still read.
 */
gs_status gs_relocate_reset(const float* key, int64_t key_stride, int64_t n, int64_t k, const gs_group* groups,
                            int32_t n_groups, int32_t moment_dtype, int32_t* step_count,
                            int32_t reset_t, int32_t* selected, void* workspace,
                            size_t workspace_bytes, hipStream_t stream);

/*
 * For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): gs_relocate_reset with
 * no workspace argument.  Same selection, results and argument rules; the
 * workspace is instead a device array of fixed size inside the library
 * (about 640 KB, one copy on each device the library runs on, held until the
 * process ends), so n is limited to GS_RELOCATE_NOALLOC_MAX_N (GS_EINVAL
 * above it; gs_relocate_reset serves larger n).  The call allocates nothing:
 * its first call on a device looks up that device's copy (with the device
 * current, as for any call: the stream must belong to the current device).
 * Every call on one device shares that copy, and each call clears what it
 * needs on the device before using it: calls that overlap on one device
 * (on two streams, or from two host threads) race and give undefined
 * results; calls issued one after another on one stream do not.
 */
#define GS_RELOCATE_NOALLOC_MAX_N ((int64_t)1 << 27)
gs_status gs_relocate_reset_noalloc(const float* key, int64_t key_stride, int64_t n, int64_t k,
                                    const gs_group* groups,
                                    int32_t n_groups, int32_t moment_dtype, int32_t* step_count,
                                    int32_t reset_t, int32_t* selected, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Schedule tuner.
 * ---------------------------------------------------------------------- */

/*
 * Times the schedules (compacted, masked) and their wave-unit sizes on
 * synthetic buffers of n primitives with the given group dims, at the given
 * visible fraction and moment dtype, and records the fastest for
 * GS_SCHED_AUTO.  Allocates and frees its own buffers; synchronizes the
 * device.  Entries are kept per (log2 n, visible-fraction bucket, dtype).
 * best_schedule / best_unit (host, may be NULL) receive the winner.
 */
gs_status gs_tune(int64_t n, const int32_t* dims, int32_t n_groups, float visible_fraction,
                  int32_t moment_dtype, int32_t* best_schedule, int32_t* best_unit);

/*
 * As gs_tune, but the candidates are timed with the caller's own visibility
 * mask (mask [n] uint8, device, read only; nonzero = visible) instead of an
 * i.i.d. Bernoulli one.  In a spatially ordered scene the visible rows come
 * in runs, which favours other schedules and units than isolated rows at
 * the same fraction.  The winner is recorded for GS_SCHED_AUTO under the
 * mask's own visible fraction.  GS_EINVAL for a NULL mask or one with no
 * visible entry; otherwise as gs_tune (own buffers, synchronizes the device).
 */
gs_status gs_tune_mask(int64_t n, const int32_t* dims, int32_t n_groups, const uint8_t* mask,
                       int32_t moment_dtype, int32_t* best_schedule, int32_t* best_unit);

/* Removes every tuner entry. */
void gs_tune_clear(void);

/* ------------------------------------------------------------------------
 * Spatial layout.  The step touches every attribute row of each visible
 * primitive; when the primitives a view sees are scattered over the index
 * range, each small row drags a whole 128-byte line (and a DRAM page) with it.
 * Ordering the primitives along a Z-order (Morton) curve of their means puts
 * what one view sees into long contiguous index runs.  These two calls compute
 * such an order and apply it to any per-primitive array; they are meant for
 * scene set-up and for the moments when the primitive set changes anyway
 * (densification), not for every step.
 * ---------------------------------------------------------------------- */

/* Bytes of device workspace gs_spatial_order needs for n primitives. */
size_t gs_spatial_order_workspace_size(int64_t n);

/*
 * perm [n] int32 out: primitive indices sorted by the 30-bit Morton code of
 * their mean (10 bits per axis over the bounding box of the means; NaN
 * coordinates take part as the box minimum), ties in index order.
 * means [n][3] FP32, rows means_stride elements apart (0 = 3).  workspace:
 * gs_spatial_order_workspace_size(n) bytes, 256-byte aligned.
 */
gs_status gs_spatial_order(const float* means, int64_t means_stride, int64_t n, int32_t* perm, void* workspace,
                           size_t workspace_bytes, hipStream_t stream);

/*
 * dst row i = src row perm[i] for n rows of row_bytes bytes (dst != src).
 * Entries of perm outside [0, n) leave their dst row untouched.
 */
gs_status gs_gather_rows(const void* src, void* dst, const int32_t* perm, int64_t n,
                         int64_t row_bytes, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Primitive-set mutation around the step.  Densification removes primitives
 * and generates new ones (Sec. "Preliminaries"; Optimization paragraph of
 * the appendix); a newly generated primitive's optimizer state is that of
 * RSR with alpha1 = alpha2 = 0 ("Scaling in RSR", Sec. "Hyperparameter
 * Selection").  The policy that decides what to prune or clone, and how a
 * clone is then moved or rescaled, is the caller's.  Gradients are not
 * carried: they belong to one iteration.
 * ---------------------------------------------------------------------- */

/* Bytes of device workspace gs_prune needs for n primitives (0 for n = 0). */
size_t gs_prune_workspace_size(int64_t n);

/*
 * Pruning: the rows i with keep[i] != 0, in ascending order, are copied with
 * their theta, m, v (each group of src to the same group of dst) and t_src[i]
 * to the front of the destination arrays; *kept_count (a device int32)
 * receives their number.  Out of place: no dst array may overlap a src
 * array.  The destination arrays must hold as many rows as will be kept (n
 * is always enough); rows beyond the kept count are not written.
 * keep [n] uint8; t_src, t_dst [n] int32; group dims equal in src and dst;
 * the grad pointers are ignored (may be NULL).  workspace:
 * gs_prune_workspace_size(n) bytes (any alignment; 256 bytes of it are slack
 * for alignment), used only during the call's kernels.
 */
gs_status gs_prune(const uint8_t* keep, int64_t n, const gs_group* src, const gs_group* dst,
                   int32_t n_groups, int32_t moment_dtype, const int32_t* t_src, int32_t* t_dst,
                   int32_t* kept_count, void* workspace, size_t workspace_bytes, hipStream_t stream);

/*
 * New primitives: for j in [0, k), row n + j of every group takes theta of
 * row src_idx[j] (a clone) and a fresh state, m = v = 0 and step_count = 0.
 * The arrays must hold n + k rows; rows below n do not change.  src_idx [k]
 * int32 (device); an entry outside [0, n) leaves that new row's theta as it
 * was (its state is still cleared).  The grad pointers are ignored.
 */
gs_status gs_append(const gs_group* groups, int32_t n_groups, int32_t moment_dtype, int64_t n,
                    const int32_t* src_idx, int64_t k, int32_t* step_count, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* GSOPT_H */
