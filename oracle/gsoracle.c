/*
 * gsoracle.c -- plain, slow, FP64 CPU oracle for the AdamW-GS optimizer step.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker of the HIP library, not
 * part of it: only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark load it.  It shares no source, header, table or helper with the
 * GPU path (paper_2601_16736_amd/csrc); the two meet only through the seeded
 * input generators, which hold none of the method's arithmetic.
 *
 * Paper: "A Step to Decouple Optimization in 3DGS" (ICLR 2026, arXiv
 * 2601.16736).  Every function cites the passage it follows.  Floating point
 * is FP64 throughout, except the visibility predicate, whose definition is an
 * FP32 computation in a fixed operation order (built with -ffp-contract=off,
 * SSE arithmetic, no fast-math, so each operation is one IEEE-754 binary32
 * round-to-nearest-even step).
 *
 * No blocking, fusion or reordering: one primitive at a time, one element at
 * a time, in the order the method states.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Counter-based random numbers: SplitMix64 (Steele, Lea & Flood, "Fast      */
/* splittable pseudorandom number generators", OOPSLA 2014).                 */
/*                                                                           */
/* A SplitMix64 stream with state s yields, as its k-th output (k >= 1),     */
/* mix64(s + k * GAMMA).  The draws used by the step are nested streams:     */
/*   s1 = 1 + tag-th      output of the stream with state `seed`            */
/*   s2 = 1 + iteration-th output of the stream with state s1              */
/*   draw(e) = (e+1)-th   output of the stream with state s2               */
/* so every (seed, tag, iteration, element) has its own 64 random bits and   */
/* no state is carried between calls.                                        */
/* ------------------------------------------------------------------------ */
#define ORC_GAMMA 0x9E3779B97F4A7C15ULL

uint64_t orc_mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* k-th output (k >= 1) of the SplitMix64 stream whose state is s. */
uint64_t orc_splitmix_output(uint64_t s, uint64_t k)
{
    return orc_mix64(s + k * ORC_GAMMA);
}

uint64_t orc_stream_state(uint64_t seed, uint64_t tag, int64_t iteration)
{
    uint64_t s1 = orc_splitmix_output(seed, tag + 1);
    return orc_splitmix_output(s1, (uint64_t)iteration + 1);
}

uint64_t orc_draw(uint64_t seed, uint64_t tag, int64_t iteration, uint64_t element)
{
    return orc_splitmix_output(orc_stream_state(seed, tag, iteration), element + 1);
}

/* Tag of the Re-State sampling stream. */
#define ORC_TAG_RSR 1ULL

/*
 * State Sampling Schedule (Sec. "Update-step decoupling: Re-State
 * Regularization"): at an RSR iteration every existing primitive is sampled
 * uniformly and independently with probability `ratio`.  Primitive i is
 * sampled iff the top 32 bits of its draw are below floor(ratio * 2^32); an
 * integer compare, so the decision is exact on every platform.
 */
uint64_t orc_rsr_threshold(double ratio)
{
    if (!(ratio > 0.0)) return 0;
    if (ratio >= 1.0) return 1ULL << 32;
    return (uint64_t)floor(ratio * 4294967296.0);
}

int orc_rsr_sampled(uint64_t seed, int64_t iteration, int64_t i, double ratio)
{
    uint64_t u = orc_draw(seed, ORC_TAG_RSR, iteration, (uint64_t)i) >> 32;
    return u < orc_rsr_threshold(ratio);
}

/* Sample flags of n primitives (ids[k], or k when ids is NULL). */
void orc_rsr_sample_mask(uint64_t seed, int64_t iteration, const int64_t* ids, int64_t n,
                         double ratio, uint8_t* out)
{
    for (int64_t k = 0; k < n; ++k)
        out[k] = (uint8_t)orc_rsr_sampled(seed, iteration, ids ? ids[k] : k, ratio);
}

/* ------------------------------------------------------------------------ */
/* DAR pixel-count normaliser (Sec. "Hyperparameter Selection", DAR          */
/* paragraph): keep only the most significant decimal digit of N_I, then     */
/* divide by ten.  1000*1000 -> 1e6 -> 1e5; 1089480 -> 1e6 -> 1e5;           */
/* 779*519 = 404301 -> 4e5 -> 4e4.                                           */
/* ------------------------------------------------------------------------ */
double orc_reg_norm(double n_pixels)
{
    if (!(n_pixels >= 1.0)) return 0.0;
    /* exact integer digit extraction, no log10 rounding at powers of ten */
    uint64_t v = (uint64_t)n_pixels;
    uint64_t p = 1;
    while (v / p >= 10) p *= 10;
    uint64_t msd = v / p;
    return (double)(msd * p) / 10.0;
}

/* ------------------------------------------------------------------------ */
/* Visibility filter V (Sec. "Characteristics of Sparse Adam", Eq. of the    */
/* sparse beta): 1 for primitives visible from the current view.  The paper */
/* takes V from the rasterizer; here it is the frustum/radius cull of the    */
/* projected mean, defined as this FP32 computation (one rounding per        */
/* operation, no fused multiply-add):                                        */
/*   p = R mu + t, row k as ((R_k0*x + R_k1*y) + R_k2*z) + t_k              */
/*   z_near < p_z < z_far                                                    */
/*   u = (fx*p_x)/p_z + cx,  v = (fy*p_y)/p_z + cy                           */
/*   r = (max(fx,fy)*rho)/p_z if a radius is given (and r >= r_min), else 0  */
/*   u + r >= 0, u - r <= W, v + r >= 0, v - r <= H                          */
/* Any NaN makes a comparison false, hence invisible.                        */
/* ------------------------------------------------------------------------ */
typedef struct {
    float view[12];   /* row-major 3x4 [R|t], world -> camera, camera looks along +z */
    float fx, fy, cx, cy;
    int32_t width, height;
    float z_near, z_far;
    float r_min;
} orc_camera;

int orc_visible_f32(const float* mu, const float* rho, const orc_camera* c)
{
    const float* M = c->view;
    float px = ((M[0] * mu[0] + M[1] * mu[1]) + M[2] * mu[2]) + M[3];
    float py = ((M[4] * mu[0] + M[5] * mu[1]) + M[6] * mu[2]) + M[7];
    float pz = ((M[8] * mu[0] + M[9] * mu[1]) + M[10] * mu[2]) + M[11];
    if (!(pz > c->z_near)) return 0;
    if (!(pz < c->z_far)) return 0;
    float u = (c->fx * px) / pz + c->cx;
    float v = (c->fy * py) / pz + c->cy;
    float r = 0.0f;
    if (rho) {
        float f = c->fx > c->fy ? c->fx : c->fy;
        r = (f * rho[0]) / pz;
        if (!(r >= c->r_min)) return 0;
    }
    float W = (float)c->width, H = (float)c->height;
    if (!(u + r >= 0.0f)) return 0;
    if (!(u - r <= W)) return 0;
    if (!(v + r >= 0.0f)) return 0;
    if (!(v - r <= H)) return 0;
    return 1;
}

void orc_visibility(const float* means, const float* radius, int64_t n,
                    const orc_camera* cam, uint8_t* mask)
{
    for (int64_t i = 0; i < n; ++i)
        mask[i] = (uint8_t)orc_visible_f32(means + 3 * i, radius ? radius + i : NULL, cam);
}

/* Same predicate in FP64: a diagnostic only (the mask is defined in FP32).  */
void orc_visibility_f64(const float* means, const float* radius, int64_t n,
                        const orc_camera* c, uint8_t* mask)
{
    const float* M = c->view;
    for (int64_t i = 0; i < n; ++i) {
        const float* mu = means + 3 * i;
        double px = (double)M[0] * mu[0] + (double)M[1] * mu[1] + (double)M[2] * mu[2] + M[3];
        double py = (double)M[4] * mu[0] + (double)M[5] * mu[1] + (double)M[6] * mu[2] + M[7];
        double pz = (double)M[8] * mu[0] + (double)M[9] * mu[1] + (double)M[10] * mu[2] + M[11];
        int vis = pz > c->z_near && pz < c->z_far;
        if (vis) {
            double u = (double)c->fx * px / pz + c->cx;
            double v = (double)c->fy * py / pz + c->cy;
            double r = 0.0;
            if (radius) {
                double f = c->fx > c->fy ? c->fx : c->fy;
                r = f * radius[i] / pz;
                vis = r >= c->r_min;
            }
            vis = vis && u + r >= 0.0 && u - r <= c->width && v + r >= 0.0 && v - r <= c->height;
        }
        mask[i] = (uint8_t)vis;
    }
}

/* Visible index list in ascending order; returns its length. */
int64_t orc_compact(const uint8_t* mask, int64_t n, int32_t* idx)
{
    int64_t k = 0;
    for (int64_t i = 0; i < n; ++i)
        if (mask[i]) idx[k++] = (int32_t)i;
    return k;
}

/* ------------------------------------------------------------------------ */
/* The AdamW-GS step (Sec. "Recoupling: AdamW-GS" with the per-attribute     */
/* forms of Sec. "Implementation Details / AdamW-GS").                       */
/* ------------------------------------------------------------------------ */
enum { ORC_DAR_NONE = 0, ORC_DAR_OPACITY_SIGMOID = 1, ORC_DAR_LOGSCALE_EXP = 2 };
/* Variants from Sec. "AdamW Style Decoupling" (constant penalty, unclipped
 * and clipped); not part of AdamW-GS itself. */
enum { ORC_REG_ADAPTIVE = 0, ORC_REG_CONSTANT = 1, ORC_REG_CONSTANT_CLIPPED = 2 };

typedef struct {
    double* param;        /* theta [n][dim] */
    const double* grad;   /* photometric gradient only [n][dim] */
    double* m;            /* first moment  [n][dim] */
    double* v;            /* second moment [n][dim] */
    int32_t dim;
    double lr;            /* eta of this attribute group */
    int32_t dar_kind;     /* which regulariser gradient R'(theta) the group carries */
    double dar_lambda;    /* lambda_theta */
    double dar_clip;      /* C_t */
    int32_t reg_mode;     /* ORC_REG_* */
} orc_group;

typedef struct {
    double beta1, beta2, eps;
    double reg_norm;      /* N_I' (see orc_reg_norm) */
    uint64_t seed;
    int64_t iteration;
    int32_t rsr_enable;
    double rsr_alpha1, rsr_alpha2, rsr_ratio;
} orc_config;

/* Gradient of the L1 regulariser through the activation (Sec. "Implementation
 * Details / AdamW-GS"): the L1 gradient of a positive quantity is +1, so what
 * remains is the activation's derivative at the stored value. */
static double reg_grad(int kind, double theta)
{
    if (kind == ORC_DAR_OPACITY_SIGMOID) {         /* o = sigma(tau) */
        double s = 1.0 / (1.0 + exp(-theta));
        return s * (1.0 - s);
    }
    if (kind == ORC_DAR_LOGSCALE_EXP)              /* s = exp(kappa) */
        return exp(theta);
    return 0.0;
}

/*
 * One AdamW-GS step.  For each primitive i, in this order:
 *  1. Re-State Regularization (RSR equation): if RSR runs this iteration and
 *     i is sampled, m <- alpha1 m and v <- alpha2 v for every element of
 *     every group, whether or not i is visible.  The step count is not
 *     touched.
 *  2. Sparse Adam (sparse beta equation, beta' = 1 where V = 0): an invisible
 *     primitive keeps theta, m, v and t unchanged.
 *  3. Asynchronous step index: t_i <- t_i + 1; bias corrections
 *     b1 = 1 - beta1^t_i, b2 = 1 - beta2^t_i (Kingma & Ba).
 *  4. Per element, decoupled moments of the photometric gradient only, then
 *     the DAR update:
 *       m <- beta1 m + (1-beta1) g,   v <- beta2 v + (1-beta2) g^2
 *       d = sqrt(v/b2) + eps,  u = (m/b1) / d
 *       u += min(lambda * R'(theta) / N_I' / d, C)   (groups with DAR)
 *       theta <- theta - lr * u
 *     R' is taken at the pre-update theta; d is this step's denominator.
 * The rows may be a subset of a scene: ids[i] (NULL: i) is row i's index in
 * the scene, which keys its Re-State draw.
 */
void orc_adamw_gs_step_rows(const orc_group* groups, int32_t n_groups, int64_t n,
                            const int64_t* ids, const uint8_t* visible, int32_t* t,
                            const orc_config* cfg)
{
    uint64_t thr = cfg->rsr_enable ? orc_rsr_threshold(cfg->rsr_ratio) : 0;
    uint64_t rsr_state = orc_stream_state(cfg->seed, ORC_TAG_RSR, cfg->iteration);

    for (int64_t i = 0; i < n; ++i) {
        if (cfg->rsr_enable) {
            /* the sample is keyed by the primitive's index in its scene */
            uint64_t id = ids ? (uint64_t)ids[i] : (uint64_t)i;
            uint64_t u32 = orc_splitmix_output(rsr_state, id + 1) >> 32;
            if (u32 < thr) {
                for (int g = 0; g < n_groups; ++g) {
                    const orc_group* G = &groups[g];
                    for (int c = 0; c < G->dim; ++c) {
                        G->m[i * G->dim + c] *= cfg->rsr_alpha1;
                        G->v[i * G->dim + c] *= cfg->rsr_alpha2;
                    }
                }
            }
        }

        if (visible && !visible[i]) continue;

        t[i] += 1;
        double b1 = 1.0 - pow(cfg->beta1, (double)t[i]);
        double b2 = 1.0 - pow(cfg->beta2, (double)t[i]);

        for (int g = 0; g < n_groups; ++g) {
            const orc_group* G = &groups[g];
            for (int c = 0; c < G->dim; ++c) {
                int64_t e = i * G->dim + c;
                double gr = G->grad[e];
                double m = cfg->beta1 * G->m[e] + (1.0 - cfg->beta1) * gr;
                double v = cfg->beta2 * G->v[e] + (1.0 - cfg->beta2) * gr * gr;
                G->m[e] = m;
                G->v[e] = v;
                double mhat = m / b1;
                double vhat = v / b2;
                double d = sqrt(vhat) + cfg->eps;
                double u = mhat / d;
                double theta = G->param[e];
                if (G->dar_kind != ORC_DAR_NONE) {
                    double rg = reg_grad(G->dar_kind, theta);
                    double r;
                    if (G->reg_mode == ORC_REG_CONSTANT)
                        r = G->dar_lambda * rg;
                    else if (G->reg_mode == ORC_REG_CONSTANT_CLIPPED)
                        r = fmin(G->dar_lambda * rg, G->dar_clip);
                    else
                        r = fmin(G->dar_lambda * rg / cfg->reg_norm / d, G->dar_clip);
                    u += r;
                }
                G->param[e] = theta - G->lr * u;
            }
        }
    }
}

/* All n primitives of a scene: row i is primitive i. */
void orc_adamw_gs_step(const orc_group* groups, int32_t n_groups, int64_t n,
                       const uint8_t* visible, int32_t* t, const orc_config* cfg)
{
    orc_adamw_gs_step_rows(groups, n_groups, n, NULL, visible, t, cfg);
}

/* ------------------------------------------------------------------------ */
/* Relocation state reset (Sec. "Hyperparameter Selection", scaling in RSR:  */
/* a reallocated primitive starts from zero optimizer state, i.e. RSR with   */
/* alpha1 = alpha2 = 0).  The k primitives with the smallest opacity logit   */
/* are selected, ties broken by the lower index; their m and v are zeroed    */
/* and, if reset_t, their step count too.                                    */
/* ------------------------------------------------------------------------ */
typedef struct { float key; int64_t idx; } orc_key_idx;

static int cmp_key_idx(const void* a, const void* b)
{
    const orc_key_idx* x = (const orc_key_idx*)a;
    const orc_key_idx* y = (const orc_key_idx*)b;
    if (x->key < y->key) return -1;
    if (x->key > y->key) return 1;
    return (x->idx > y->idx) - (x->idx < y->idx);
}

/* Writes the selected indices in ascending order.  NaN keys are not
 * supported (the caller's opacities are finite). */
void orc_select_smallest(const float* key, int64_t n, int64_t k, int64_t* sel)
{
    orc_key_idx* a = (orc_key_idx*)malloc(sizeof(orc_key_idx) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) { a[i].key = key[i]; a[i].idx = i; }
    qsort(a, (size_t)n, sizeof(orc_key_idx), cmp_key_idx);
    uint8_t* pick = (uint8_t*)calloc((size_t)(n > 0 ? n : 1), 1);
    for (int64_t j = 0; j < k && j < n; ++j) pick[a[j].idx] = 1;
    int64_t w = 0;
    for (int64_t i = 0; i < n; ++i) if (pick[i]) sel[w++] = i;
    free(pick);
    free(a);
}

void orc_reset_state(const orc_group* groups, int32_t n_groups, const int64_t* sel,
                     int64_t k, int32_t* t, int32_t reset_t)
{
    for (int64_t j = 0; j < k; ++j) {
        int64_t i = sel[j];
        for (int g = 0; g < n_groups; ++g) {
            const orc_group* G = &groups[g];
            for (int c = 0; c < G->dim; ++c) {
                G->m[i * G->dim + c] = 0.0;
                G->v[i * G->dim + c] = 0.0;
            }
        }
        if (reset_t && t) t[i] = 0;
    }
}

/* ------------------------------------------------------------------------ */
/* bfloat16 storage rounding, by definition of the format (top 16 bits of a  */
/* binary32).  Round-to-nearest-even, and stochastic rounding with 16 given  */
/* random bits: add them below the kept bits, then truncate.  Used to check  */
/* reduced-precision moment storage; the oracle's own state stays FP64.     */
/* ------------------------------------------------------------------------ */
static uint32_t f32_bits(float x) { uint32_t b; memcpy(&b, &x, 4); return b; }

uint16_t orc_bf16_rne(float x)
{
    uint32_t b = f32_bits(x);
    if ((b & 0x7F800000u) == 0x7F800000u && (b & 0x007FFFFFu))
        return (uint16_t)((b >> 16) | 0x0040u);           /* quiet NaN */
    uint32_t lsb = (b >> 16) & 1u;
    return (uint16_t)((b + 0x7FFFu + lsb) >> 16);
}

uint16_t orc_bf16_sr(float x, uint32_t r16)
{
    uint32_t b = f32_bits(x);
    if ((b & 0x7F800000u) == 0x7F800000u)                   /* Inf/NaN unchanged */
        return (uint16_t)((b >> 16) | ((b & 0x007FFFFFu) ? 0x0040u : 0u));
    return (uint16_t)((b + (r16 & 0xFFFFu)) >> 16);
}
