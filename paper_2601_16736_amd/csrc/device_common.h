// Device-side building blocks of the AdamW-GS step kernels (gfx950, wave64).
//
// Work is organised per wavefront: a wave takes one "unit" (a window of the
// mask, or a slice of the visible-index list), stages the unit's visible row
// indices and per-row bias corrections in its own slice of LDS, then sweeps
// each attribute group once.  Inside a group the wave's 64 lanes walk the
// flattened (row, chunk) space of the staged rows, so consecutive lanes touch
// consecutive 4/8/16-byte chunks of one row before moving to the next row:
// every group is one coalesced read-modify-write pass.
#pragma once

#include "internal.h"

namespace gs {

// ---------------------------------------------------------------- draws
// SplitMix64 output function and stream (Steele, Lea & Flood 2014): the
// k-th output of the stream with state s is mix64(s + k * gamma).
__device__ __forceinline__ uint64_t d_mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t d_splitmix(uint64_t s, uint64_t k) { return d_mix64(s + k * kGamma); }

// State of the stream keyed by (seed, tag, iteration): output (tag+1) of the
// stream seeded with `seed`, then output (iteration+1) of that one.
__device__ __forceinline__ uint64_t d_stream(uint64_t seed, uint64_t tag, int64_t iteration)
{
    return d_splitmix(d_splitmix(seed, tag + 1), (uint64_t)iteration + 1);
}

// ---------------------------------------------------------------- bf16 storage
__device__ __forceinline__ float bf16_to_f32(uint32_t h) { return __uint_as_float(h << 16); }

// round-to-nearest-even; NaN stays a quiet NaN
__device__ __forceinline__ uint32_t f32_to_bf16_rne(float x)
{
    const uint32_t b = __float_as_uint(x);
    if ((b & 0x7F800000u) == 0x7F800000u && (b & 0x007FFFFFu)) return (b >> 16) | 0x40u;
    return (b + 0x7FFFu + ((b >> 16) & 1u)) >> 16;
}

// stochastic rounding: add 16 random bits below the kept bits, truncate
__device__ __forceinline__ uint32_t f32_to_bf16_sr(float x, uint32_t r16)
{
    const uint32_t b = __float_as_uint(x);
    if ((b & 0x7F800000u) == 0x7F800000u) return (b >> 16) | ((b & 0x007FFFFFu) ? 0x40u : 0u);
    return (b + r16) >> 16;
}

// ---------------------------------------------------------------- wave helpers
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// number of set bits of `mask` in lanes below this one
__device__ __forceinline__ int lanes_below(uint64_t mask)
{
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                          __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// ---------------------------------------------------------------- vector access
// Attribute and moment streams are touched once per step.  Their 8- and
// 16-byte accesses carry the non-temporal hint; 2- and 4-byte ones do not
// (on the 3M-primitive scene, hinting no access made the step 29 % slower
// and hinting every access 7 % slower than this split).
constexpr bool kNtWide = true;     // 8- and 16-byte loads and stores
constexpr bool kNtNarrow = false;  // 2- and 4-byte loads and stores

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// Every array the kernels read or write lives in device (global) memory.  A
// pointer that a kernel reads from memory, as the batched plan reads its
// scenes' descriptors, is a generic pointer to the compiler, whose accesses
// it would issue as flat instructions (slower to wait for: they count against
// the LDS counter too).  The accessors below name the address space.
template <typename T> using gptr = __attribute__((address_space(1))) T*;
template <typename T> __device__ __forceinline__ gptr<T> to_global(T* p) { return (gptr<T>)p; }

template <typename T, bool NT> __device__ __forceinline__ T ld(const T* p)
{
    if constexpr (NT) return __builtin_nontemporal_load(to_global(p));
    else return *to_global(p);
}

template <typename T, bool NT> __device__ __forceinline__ void st(T* p, T x)
{
    if constexpr (NT) __builtin_nontemporal_store(x, to_global(p));
    else *to_global(p) = x;
}

template <int V> __device__ __forceinline__ void load_f(const float* p, float* x)
{
    if constexpr (V == 4) {
        const f32x4 t = ld<f32x4, kNtWide>(reinterpret_cast<const f32x4*>(p));
        x[0] = t.x; x[1] = t.y; x[2] = t.z; x[3] = t.w;
    } else if constexpr (V == 2) {
        const f32x2 t = ld<f32x2, kNtWide>(reinterpret_cast<const f32x2*>(p));
        x[0] = t.x; x[1] = t.y;
    } else {
        x[0] = ld<float, kNtNarrow>(p);
    }
}

template <int V> __device__ __forceinline__ void store_f(float* p, const float* x)
{
    if constexpr (V == 4) {
        f32x4 t;
        t.x = x[0]; t.y = x[1]; t.z = x[2]; t.w = x[3];
        st<f32x4, kNtWide>(reinterpret_cast<f32x4*>(p), t);
    } else if constexpr (V == 2) {
        f32x2 t;
        t.x = x[0]; t.y = x[1];
        st<f32x2, kNtWide>(reinterpret_cast<f32x2*>(p), t);
    } else {
        st<float, kNtNarrow>(p, x[0]);
    }
}

template <int V> __device__ __forceinline__ void load_h(const uint16_t* p, float* x)
{
    if constexpr (V == 4) {
        const u32x2 t = ld<u32x2, kNtWide>(reinterpret_cast<const u32x2*>(p));
        x[0] = bf16_to_f32(t.x & 0xFFFFu); x[1] = bf16_to_f32(t.x >> 16);
        x[2] = bf16_to_f32(t.y & 0xFFFFu); x[3] = bf16_to_f32(t.y >> 16);
    } else if constexpr (V == 2) {
        const uint32_t t = ld<uint32_t, kNtNarrow>(reinterpret_cast<const uint32_t*>(p));
        x[0] = bf16_to_f32(t & 0xFFFFu); x[1] = bf16_to_f32(t >> 16);
    } else {
        x[0] = bf16_to_f32(ld<uint16_t, kNtNarrow>(p));
    }
}

template <int V> __device__ __forceinline__ void store_h(uint16_t* p, const uint32_t* h)
{
    if constexpr (V == 4) {
        u32x2 t;
        t.x = h[0] | (h[1] << 16); t.y = h[2] | (h[3] << 16);
        st<u32x2, kNtWide>(reinterpret_cast<u32x2*>(p), t);
    } else if constexpr (V == 2) {
        st<uint32_t, kNtNarrow>(reinterpret_cast<uint32_t*>(p), h[0] | (h[1] << 16));
    } else {
        st<uint16_t, kNtNarrow>(p, (uint16_t)h[0]);
    }
}

template <bool BF16, int V> __device__ __forceinline__ void load_moment(const void* base, int64_t e, float* x)
{
    if constexpr (BF16) load_h<V>(static_cast<const uint16_t*>(base) + e, x);
    else load_f<V>(static_cast<const float*>(base) + e, x);
}

// The 32 rounding bits of element e from draw d = output (e/2 + 1) of
// stream s2: bits 63..32 of d for even e, 31..0 for odd e (m takes the
// upper 16, v the lower 16), so one draw serves two consecutive elements.
__device__ __forceinline__ uint32_t sr_word(uint64_t d, int64_t e) { return (e & 1) ? (uint32_t)d : (uint32_t)(d >> 32); }

// Stores m and v of V consecutive elements at array offset e; el is the
// first one's element index row * dim + column in its group, which keys its
// rounding bits (for V > 1 both are multiples of V: vector access needs
// dim % V == 0 and a row stride that is a multiple of V).  BF16 with
// stochastic rounding takes the bits of sr_word.
template <bool BF16, int V>
__device__ __forceinline__ void store_moments(void* mb, void* vb, int64_t e, int64_t el, const float* m,
                                              const float* v, bool sr, uint64_t s2)
{
    if constexpr (BF16) {
        uint32_t hm[V], hv[V];
        if (sr) {
            if constexpr (V == 1) {
                const uint32_t w = sr_word(d_splitmix(s2, (uint64_t)(el >> 1) + 1), el);
                hm[0] = f32_to_bf16_sr(m[0], w >> 16);
                hv[0] = f32_to_bf16_sr(v[0], w & 0xFFFFu);
            } else {
#pragma unroll
                for (int q = 0; q < V; q += 2) {
                    const uint64_t d = d_splitmix(s2, (uint64_t)((el + q) >> 1) + 1);
                    const uint32_t hi = (uint32_t)(d >> 32), lo = (uint32_t)d;
                    hm[q] = f32_to_bf16_sr(m[q], hi >> 16);
                    hv[q] = f32_to_bf16_sr(v[q], hi & 0xFFFFu);
                    hm[q + 1] = f32_to_bf16_sr(m[q + 1], lo >> 16);
                    hv[q + 1] = f32_to_bf16_sr(v[q + 1], lo & 0xFFFFu);
                }
            }
        } else {
#pragma unroll
            for (int q = 0; q < V; ++q) {
                hm[q] = f32_to_bf16_rne(m[q]);
                hv[q] = f32_to_bf16_rne(v[q]);
            }
        }
        store_h<V>(static_cast<uint16_t*>(mb) + e, hm);
        store_h<V>(static_cast<uint16_t*>(vb) + e, hv);
    } else {
        store_f<V>(static_cast<float*>(mb) + e, m);
        store_f<V>(static_cast<float*>(vb) + e, v);
    }
}

// ---------------------------------------------------------------- the update
// Regulariser term added to the Adam direction u (DAR update equation and
// the AdamW-style variants).  R' is the activation derivative at the
// pre-update theta: sigma(tau)(1 - sigma(tau)), computed in the equivalent
// form e/(1+e)^2 with e = exp(-|tau|) (no cancellation), or exp(kappa).
__device__ __forceinline__ float reg_term(int kind, int mode, float scale, float clip, float th, float d)
{
    float R;
    if (kind == GS_DAR_OPACITY_SIGMOID) {
        const float e = expf(-fabsf(th));
        const float q = 1.0f + e;
        R = e / (q * q);
    } else {
        R = expf(th);
    }
    if (mode == GS_REG_ADAPTIVE) return fminf(scale * R / d, clip);
    if (mode == GS_REG_CONSTANT) return scale * R;
    return fminf(scale * R, clip);
}

struct NoiseArgs {
    const float* q;      // quaternion group's attributes
    const float* kappa;  // log-scale group's attributes
    const float* tau;    // opacity-logit group's attributes
    int64_t sq, sk, st;  // their row strides in elements
    uint64_t s2;         // stream (seed, tag 48, iteration)
    float scale;         // eta_{R_o} * eta_mu
};

// Position-noise displacement eta_{R_o} R_mu of primitive i (definition in
// gsopt.h), all three components: Sigma gamma from the pre-update quaternion
// and log-scale, gated by the pre-update opacity.  `nz.scale` = eta_{R_o}
// eta_mu.
__device__ __forceinline__ void noise_row(const NoiseArgs& nz, int64_t i, float k, float t0, float* out)
{
    // gamma ~ N(0, I3): Box-Muller on 24-bit uniforms of two draws
    const uint64_t d1 = d_splitmix(nz.s2, 2 * (uint64_t)i + 1);
    const uint64_t d2 = d_splitmix(nz.s2, 2 * (uint64_t)i + 2);
    const float u1 = (float)((uint32_t)(d1 >> 40) + 1u) * 0x1p-24f;
    const float a1 = (float)((uint32_t)(d1 >> 8) & 0xFFFFFFu) * 0x1p-24f;
    const float u2 = (float)((uint32_t)(d2 >> 40) + 1u) * 0x1p-24f;
    const float a2 = (float)((uint32_t)(d2 >> 8) & 0xFFFFFFu) * 0x1p-24f;
    const float r1 = __fsqrt_rn(-2.0f * logf(u1));
    const float r2 = __fsqrt_rn(-2.0f * logf(u2));
    float sn1, cs1, sn2, cs2;
    sincospif(2.0f * a1, &sn1, &cs1);
    sincospif(2.0f * a2, &sn2, &cs2);
    const float g0 = r1 * cs1, g1 = r1 * sn1, g2 = r2 * cs2;
    // rotation of the normalised quaternion (w, x, y, z)
    const gptr<const float> qp = to_global(nz.q);
    const gptr<const float> kp = to_global(nz.kappa);
    float w = qp[nz.sq * i], x = qp[nz.sq * i + 1], y = qp[nz.sq * i + 2], z = qp[nz.sq * i + 3];
    const float inv = 1.0f / __fsqrt_rn(w * w + x * x + y * y + z * z);
    w *= inv; x *= inv; y *= inv; z *= inv;
    const float R00 = 1.0f - 2.0f * (y * y + z * z), R01 = 2.0f * (x * y - w * z), R02 = 2.0f * (x * z + w * y);
    const float R10 = 2.0f * (x * y + w * z), R11 = 1.0f - 2.0f * (x * x + z * z), R12 = 2.0f * (y * z - w * x);
    const float R20 = 2.0f * (x * z - w * y), R21 = 2.0f * (y * z + w * x), R22 = 1.0f - 2.0f * (x * x + y * y);
    // Sigma gamma = R diag(exp(2 kappa)) R^T gamma
    const float e0 = (R00 * g0 + R10 * g1 + R20 * g2) * expf(2.0f * kp[nz.sk * i]);
    const float e1 = (R01 * g0 + R11 * g1 + R21 * g2) * expf(2.0f * kp[nz.sk * i + 1]);
    const float e2 = (R02 * g0 + R12 * g1 + R22 * g2) * expf(2.0f * kp[nz.sk * i + 2]);
    const float o = 1.0f / (1.0f + expf(-to_global(nz.tau)[nz.st * i]));
    const float gate = 1.0f / (1.0f + expf(k * (o - t0)));            // sigma(-k (o - t))
    out[0] = nz.scale * gate * (R00 * e0 + R01 * e1 + R02 * e2);
    out[1] = nz.scale * gate * (R10 * e0 + R11 * e1 + R12 * e2);
    out[2] = nz.scale * gate * (R20 * e0 + R21 * e1 + R22 * e2);
}


// The update of one visible element (sparse-beta, decoupled-moment, Adam
// and DAR update equations): the moments from the photometric gradient g
// (c1, c2: beta, or beta*alpha for a row in this iteration's Re-State
// sample), the Adam direction from the bias corrections rb1 = 1/(1-beta1^t)
// and rsb2 = 1/sqrt(1-beta2^t), the regulariser term at the pre-update
// theta (dar: kind != GS_DAR_NONE), and theta.  Every schedule calls this
// one function, so they all round alike.
__device__ __forceinline__ void update_element(float& th, float g, float& m, float& v, float c1, float c2, float rb1,
                                               float rsb2, const KHyper& H, bool dar, int kind, int mode, float scale,
                                               float clip, float lr)
{
    const float mm = c1 * m + H.omb1 * g;
    const float vv = c2 * v + H.omb2 * (g * g);
    const float d = __fsqrt_rn(vv) * rsb2 + H.eps;       // sqrt(v / b2) + eps
    float uu = (mm * rb1) / d;                            // (m / b1) / d
    if (dar) uu += reg_term(kind, mode, scale, clip, th, d);
    th = th - lr * uu;
    m = mm;
    v = vv;
}

// One group's read-modify-write pass over the wave's staged rows.  Each
// lane takes U (row, chunk) items per trip and issues all their loads before
// any store, so a wave keeps U x 4 vector loads in flight.  NOISE (mean
// group only, V = 1) subtracts the position-noise displacement, staged per
// row in s_noise, after the Adam update.
template <bool BF16, int V, int U, bool NOISE = false>
__device__ __forceinline__ void step_group(const KGroup& G, const KHyper& H, int nrows,
                                           const int* s_row, const float* s_rb1, const float* s_rsb2,
                                           int lane, float dar_scale, uint64_t sr_s2, const float* s_noise = nullptr)
{
    const int cpr = G.cpr;
    const int dim = G.dim;
    const int64_t stride = G.stride;
    const int items = nrows * cpr;
    int r = lane / cpr;
    int c = lane - r * cpr;
    const int dr = kWave / cpr;
    const int dc = kWave - dr * cpr;
    const bool dar = G.dar_kind != GS_DAR_NONE;
    for (int k0 = lane; k0 < items; k0 += U * kWave) {
        int64_t e[U], el[U];   // array offset, element index in the group
        float c1[U], c2[U], rb1[U], rsb2[U];
        bool ok[U];
        int nidx[U];      // NOISE: the item's slot in s_noise
#pragma unroll
        for (int u = 0; u < U; ++u) {
            ok[u] = k0 + u * kWave < items;
            nidx[u] = 3 * r + c;
            const int raw = ok[u] ? s_row[r] : 0;
            // a row in this iteration's Re-State sample decays by alpha before
            // the moment update: beta*(alpha*m) folded into (beta*alpha)*m
            c1[u] = raw < 0 ? H.c1_rsr : H.beta1;
            c2[u] = raw < 0 ? H.c2_rsr : H.beta2;
            rb1[u] = ok[u] ? s_rb1[r] : 1.0f;
            rsb2[u] = ok[u] ? s_rsb2[r] : 1.0f;
            e[u] = (int64_t)(raw & 0x7FFFFFFF) * stride + c * V;
            el[u] = (int64_t)(raw & 0x7FFFFFFF) * dim + c * V;
            r += dr;
            c += dc;
            if (c >= cpr) { c -= cpr; ++r; }
        }
        float th[U][V], g[U][V], m[U][V], v[U][V];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (ok[u]) {
                load_f<V>(G.param + e[u], th[u]);
                load_f<V>(G.grad + e[u], g[u]);
                load_moment<BF16, V>(G.m, e[u], m[u]);
                load_moment<BF16, V>(G.v, e[u], v[u]);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (!ok[u]) continue;
#pragma unroll
            for (int q = 0; q < V; ++q) {
                update_element(th[u][q], g[u][q], m[u][q], v[u][q], c1[u], c2[u], rb1[u], rsb2[u], H, dar,
                               G.dar_kind, G.reg_mode, dar_scale, G.dar_clip, G.lr);
                if constexpr (NOISE) th[u][q] -= s_noise[nidx[u]];     // the mean group: dim 3, V = 1
            }
            store_f<V>(G.param + e[u], th[u]);
            store_moments<BF16, V>(G.m, G.v, e[u], el[u], m[u], v[u], H.sr != 0, sr_s2);
        }
    }
}

// One group's pass over the wave's staged invisible rows.  A row tagged in
// its sign bit is in this iteration's Re-State sample: m <- a1 m, v <- a2 v,
// stored.  A row with rb1 > 0 is in the AIU sample: theta moves by
// -lr eta_AIU (m rb1)/(sqrt(v) rsb2 + eps) from the (rescaled) moments,
// which are not stored again unless the row was rescaled.
template <bool BF16, int V>
__device__ __forceinline__ void invisible_group(const KGroup& G, const KHyper& H, int nrows, const int* s_row,
                                                const float* s_rb1, const float* s_rsb2, int lane, uint64_t sr_s2,
                                                float lr_aiu)
{
    const int cpr = G.cpr;
    const int dim = G.dim;
    const int64_t stride = G.stride;
    const int items = nrows * cpr;
    int r = lane / cpr;
    int c = lane - r * cpr;
    const int dr = kWave / cpr;
    const int dc = kWave - dr * cpr;
    for (int k = lane; k < items; k += kWave) {
        const int raw = s_row[r];
        const float rb1 = s_rb1[r];
        const float rsb2 = s_rsb2[r];
        const bool rsr = raw < 0;
        const bool aiu = rb1 > 0.0f;
        const int64_t e = (int64_t)(raw & 0x7FFFFFFF) * stride + c * V;
        const int64_t el = (int64_t)(raw & 0x7FFFFFFF) * dim + c * V;
        float m[V], v[V], th[V];
        load_moment<BF16, V>(G.m, e, m);
        load_moment<BF16, V>(G.v, e, v);
        if (aiu) load_f<V>(G.param + e, th);
        if (rsr) {
#pragma unroll
            for (int q = 0; q < V; ++q) {
                m[q] = H.rsr_a1 * m[q];
                v[q] = H.rsr_a2 * v[q];
            }
            store_moments<BF16, V>(G.m, G.v, e, el, m, v, H.sr != 0, sr_s2);
        }
        if (aiu) {
#pragma unroll
            for (int q = 0; q < V; ++q) {
                const float d = __fsqrt_rn(v[q]) * rsb2 + H.eps;
                th[q] = th[q] - lr_aiu * ((m[q] * rb1) / d);
            }
            store_f<V>(G.param + e, th);
        }
        r += dr;
        c += dc;
        if (c >= cpr) { c -= cpr; ++r; }
    }
}

// ---------------------------------------------------------------- staging
// Rows of a window [w0, w0 + UNIT) that pass the mask (mask == nullptr: all
// rows below n), in ascending order.  Returns the row count.
template <int UNIT>
__device__ __forceinline__ int build_rows_window(const uint8_t* mask, int64_t n, int64_t w0, int* s_row,
                                                 int lane)
{
    // a 32-primitive window leaves the upper half-wave idle
    constexpr int R = (UNIT + kWave - 1) / kWave;
    bool vis[R];
#pragma unroll
    for (int b = 0; b < R; ++b) {
        const int64_t i = w0 + b * kWave + lane;
        vis[b] = b * kWave + lane < UNIT && i < n;
        if (mask != nullptr && vis[b]) vis[b] = to_global(mask)[i] != 0;
    }
    int nrows = 0;
#pragma unroll
    for (int b = 0; b < R; ++b) {
        const uint64_t bal = __ballot(vis[b]);
        if (vis[b]) s_row[nrows + lanes_below(bal)] = (int)(w0 + b * kWave + lane);
        nrows += __popcll(bal);
    }
    return nrows;
}

// Re-State sample: primitive i is sampled iff the top 32 bits of draw (i+1)
// of stream s2 are below thr.
__device__ __forceinline__ bool rsr_sampled(uint64_t s2, uint64_t thr, int64_t i)
{
    return (d_splitmix(s2, (uint64_t)i + 1) >> 32) < thr;
}

// Invisible rows of a window (mask == 0) in this iteration's Re-State sample
// or, with t > 0, in its AIU sample, in ascending order.  Re-State rows get
// the sign bit; AIU rows get their bias factors from the unchanged t, other
// rows rb1 = 0.
template <int UNIT>
__device__ __forceinline__ int build_rows_invisible(const uint8_t* mask, int64_t n, int64_t w0, const int32_t* t,
                                                    const KHyper& H, uint64_t rsr_s2, uint64_t aiu_s2, int* s_row,
                                                    float* s_rb1, float* s_rsb2, int lane)
{
    int nrows = 0;
#pragma unroll
    for (int b = 0; b < UNIT / kWave; ++b) {
        const int64_t i = w0 + b * kWave + lane;
        const bool inv = i < n && to_global(mask)[i] == 0;
        const bool rsr = inv && H.rsr_thr != 0 && rsr_sampled(rsr_s2, H.rsr_thr, i);
        int ti = 0;
        if (inv && H.aiu_thr != 0 && rsr_sampled(aiu_s2, H.aiu_thr, i)) ti = to_global(t)[i];
        const bool aiu = ti > 0;
        const bool pick = rsr || aiu;
        const uint64_t bal = __ballot(pick);
        if (pick) {
            const int j = nrows + lanes_below(bal);
            s_row[j] = rsr ? (int)((uint32_t)i | 0x80000000u) : (int)i;
            float rb1 = 0.0f, rsb2 = 0.0f;
            if (aiu) {
                const float ft = (float)ti;
                rb1 = 1.0f / -expm1f(ft * H.logb1);
                rsb2 = 1.0f / __fsqrt_rn(-expm1f(ft * H.logb2));
            }
            s_rb1[j] = rb1;
            s_rsb2[j] = rsb2;
        }
        nrows += __popcll(bal);
    }
    return nrows;
}

// Entries [base, base + UNIT) of the visible-index list (cnt entries in all).
// Entries outside [0, n) are dropped, so a corrupt list cannot send the
// step outside the arrays.
template <int UNIT>
__device__ __forceinline__ int build_rows_slice(const int32_t* idx, int cnt, int64_t n, int64_t base, int* s_row,
                                                int lane)
{
    // a 32-entry slice leaves the upper half-wave idle (avail <= UNIT)
    constexpr int R = (UNIT + kWave - 1) / kWave;
    const int avail = (int)min((int64_t)UNIT, (int64_t)cnt - base);
    int32_t v[R];
#pragma unroll
    for (int b = 0; b < R; ++b) {
        const int j = b * kWave + lane;
        v[b] = j < avail ? to_global(idx)[base + j] : -1;
    }
    int nrows = 0;
#pragma unroll
    for (int b = 0; b < R; ++b) {
        const bool ok = v[b] >= 0 && v[b] < n;
        const uint64_t bal = __ballot(ok);
        if (ok) s_row[nrows + lanes_below(bal)] = v[b];
        nrows += __popcll(bal);
    }
    return nrows;
}

// t_i <- t_i + 1 for each staged row and its bias corrections:
// 1/(1 - beta1^t) and 1/sqrt(1 - beta2^t), with 1 - beta^t = -expm1(t log beta).
// A row in the Re-State sample gets its sign bit set (indices are < 2^31).
__device__ __forceinline__ void stage_step_rows(int nrows, int* s_row, float* s_rb1, float* s_rsb2,
                                                int32_t* t, const KHyper& H, uint64_t rsr_s2, int lane)
{
    for (int j = lane; j < nrows; j += kWave) {
        const int i = s_row[j];
        if (H.rsr_thr != 0 && rsr_sampled(rsr_s2, H.rsr_thr, i)) s_row[j] = (int)((uint32_t)i | 0x80000000u);
        const int tn = to_global(t)[i] + 1;
        to_global(t)[i] = tn;
        const float ft = (float)tn;
        const float b1 = -expm1f(ft * H.logb1);
        const float b2 = -expm1f(ft * H.logb2);
        s_rb1[j] = 1.0f / b1;
        s_rsb2[j] = 1.0f / __fsqrt_rn(b2);
    }
}

// ---------------------------------------------------------------- packed rows
// The packed pass (KScene::pk_stride > 0): every group is a column range of
// the same [n][S] arrays, so the step takes each staged row in one pass of
// 4-column chunks (16-byte attribute, 4-element moment accesses) instead of
// one pass per group.  S / 4 divides the wave, so a lane meets the same
// chunk in every row it visits: the group of each of its 4 columns and that
// group's hyper-parameters are set up once per pass.  A column outside every
// group is read and written back unchanged (the same bits), so that every
// chunk is stored with one access per array and a row's lines are written
// whole: the HBM has no byte masks, and a line written in part costs its
// controller a read-modify-write.  Each element's update is step_group's;
// a BF16 element's rounding bits come from its index row * dim + column in
// its own group, exactly as in the per-group passes, so both schedules give
// the same bits.
template <bool BF16, int U, bool NOISE>
__device__ __forceinline__ void step_packed(const KScene& S, const KHyper& H, uint64_t seed, int nrows,
                                            const int* s_row, const float* s_rb1, const float* s_rsb2, int lane,
                                            const float* s_noise)
{
    const int cpr = S.pk_stride >> 2;          // chunks per row, a power of two up to 64
    const int chunk = lane & (cpr - 1);
    const int rstep = kWave / cpr;             // rows that one wave-wide trip covers
    // the lane's 4 columns: group (-1: none), DAR, lr, rounding stream and
    // place in the group (element index = row * dim + off)
    int gid[4], kind[4], mode[4], dim[4], off[4];
    float lr[4], scale[4], clip[4];
    uint64_t s2[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        gid[q] = -1;
        kind[q] = GS_DAR_NONE;
        mode[q] = GS_REG_ADAPTIVE;
        dim[q] = 1;
        off[q] = 0;
        lr[q] = 0.0f;
        scale[q] = 0.0f;
        clip[q] = 0.0f;
        s2[q] = 0;
    }
    for (int gi = 0; gi < S.n_groups; ++gi) {
        const KGroup& G = S.g[gi];
        const int lo = S.pk_col[gi];
        // lambda / N_I' rounded once from double, exactly as a host would form it
        const float sc = (G.dar_kind != GS_DAR_NONE && G.reg_mode == GS_REG_ADAPTIVE)
                             ? (float)(G.dar_lambda / H.reg_norm)
                             : (float)G.dar_lambda;
        const uint64_t gs2 = BF16 ? d_stream(seed, kTagSrStep + (uint64_t)gi, H.iteration) : 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int col = 4 * chunk + q;
            if (col >= lo && col < lo + G.dim) {
                gid[q] = gi;
                kind[q] = G.dar_kind;
                mode[q] = G.reg_mode;
                dim[q] = G.dim;
                off[q] = col - lo;
                lr[q] = G.lr;
                scale[q] = sc;
                clip[q] = G.dar_clip;
                s2[q] = gs2;
            }
        }
    }
    const bool sr = H.sr != 0;
    const int64_t stride = S.pk_stride;
    for (int r0 = lane / cpr; r0 < nrows; r0 += U * rstep) {
        int rr[U];
        bool ok[U];
        int64_t row[U];
        float th[U][4], g[U][4], m[U][4], v[U][4];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            rr[u] = r0 + u * rstep;
            ok[u] = rr[u] < nrows;
            row[u] = ok[u] ? (int64_t)(s_row[rr[u]] & 0x7FFFFFFF) : 0;
            if (ok[u]) {
                const int64_t e = row[u] * stride + 4 * chunk;
                load_f<4>(S.pk_param + e, th[u]);
                load_f<4>(S.pk_grad + e, g[u]);
                load_moment<BF16, 4>(S.pk_m, e, m[u]);
                load_moment<BF16, 4>(S.pk_v, e, v[u]);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (!ok[u]) continue;
            const int raw = s_row[rr[u]];
            // a row in this iteration's Re-State sample decays by alpha before
            // the moment update: beta*(alpha*m) folded into (beta*alpha)*m
            const float c1 = raw < 0 ? H.c1_rsr : H.beta1;
            const float c2 = raw < 0 ? H.c2_rsr : H.beta2;
            const float rb1 = s_rb1[rr[u]];
            const float rsb2 = s_rsb2[rr[u]];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (gid[q] < 0) continue;
                update_element(th[u][q], g[u][q], m[u][q], v[u][q], c1, c2, rb1, rsb2, H, kind[q] != GS_DAR_NONE,
                               kind[q], mode[q], scale[q], clip[q], lr[q]);
                if (NOISE && gid[q] == H.noise_g[0]) th[u][q] -= s_noise[3 * rr[u] + off[q]];
            }
            const int64_t e = row[u] * stride + 4 * chunk;
            if constexpr (BF16) {
                uint32_t hm[4], hv[4];
                if (sr) {
                    // one draw serves m and v of an element and of its pair
                    // partner (sr_word): the chunk's columns reuse the draw
                    // of the column before them when it is the same pair
                    uint64_t d = 0;
                    int64_t key_prev = -1;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int64_t el = row[u] * dim[q] + off[q];
                        const int64_t key = el >> 1;
                        if (gid[q] >= 0 && (q == 0 || gid[q] != gid[q - 1] || key != key_prev))
                            d = d_splitmix(s2[q], (uint64_t)key + 1);
                        key_prev = key;
                        const uint32_t w = sr_word(d, el);
                        hm[q] = f32_to_bf16_sr(m[u][q], w >> 16);
                        hv[q] = f32_to_bf16_sr(v[u][q], w & 0xFFFFu);
                    }
                } else {
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        hm[q] = f32_to_bf16_rne(m[u][q]);
                        hv[q] = f32_to_bf16_rne(v[u][q]);
                    }
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (gid[q] < 0) {             // not a group's column: its own bits again
                        hm[q] = __float_as_uint(m[u][q]) >> 16;
                        hv[q] = __float_as_uint(v[u][q]) >> 16;
                    }
                }
                store_f<4>(S.pk_param + e, th[u]);
                store_h<4>(static_cast<uint16_t*>(S.pk_m) + e, hm);
                store_h<4>(static_cast<uint16_t*>(S.pk_v) + e, hv);
            } else {
                store_f<4>(S.pk_param + e, th[u]);
                store_f<4>(static_cast<float*>(S.pk_m) + e, m[u]);
                store_f<4>(static_cast<float*>(S.pk_v) + e, v[u]);
            }
        }
    }
}

// Every group's pass over the staged rows.  U: (row, chunk) items per lane
// per trip for the 16/8-byte groups (twice that for 4-byte ones, the noise
// group included).
template <bool BF16, bool NOISE, int U, bool PACKED>
__device__ __forceinline__ void step_all_groups(const KScene& S, const KHyper& H, uint64_t seed, int nrows,
                                                const int* s_row, const float* s_rb1, const float* s_rsb2,
                                                int lane, float* s_noise = nullptr)
{
    // With position noise the mean group goes first, so the quaternion,
    // log-scale and opacity rows it reads are still the pre-update ones.
    // Groups are indexed directly (no switch over constant indices): the
    // by-value scene then stays in the kernel arguments instead of being
    // copied to private memory.  The noise code is compiled only into the
    // NOISE kernels, so the plain step keeps its register budget.
    const int first = NOISE ? H.noise_g[0] : -1;
    if constexpr (NOISE) {
        const KGroup& G = S.g[first];
        NoiseArgs nz;
        nz.q = S.g[H.noise_g[2]].param;
        nz.kappa = S.g[H.noise_g[1]].param;
        nz.tau = S.g[H.noise_g[3]].param;
        nz.sq = S.g[H.noise_g[2]].stride;
        nz.sk = S.g[H.noise_g[1]].stride;
        nz.st = S.g[H.noise_g[3]].stride;
        nz.s2 = d_stream(seed, kTagNoise, H.iteration);
        nz.scale = (float)(H.noise_lr * (double)G.lr);
        const float dar_scale = (G.dar_kind != GS_DAR_NONE && G.reg_mode == GS_REG_ADAPTIVE)
                                    ? (float)(G.dar_lambda / H.reg_norm)
                                    : (float)G.dar_lambda;
        const uint64_t s2 = BF16 ? d_stream(seed, kTagSrStep + (uint64_t)first, H.iteration) : 0;
        // each lane forms whole rows' displacements (3 floats per staged row),
        // then the mean group's items read their component
        for (int j = lane; j < nrows; j += kWave)
            noise_row(nz, (int64_t)(s_row[j] & 0x7FFFFFFF), H.noise_k, H.noise_t, &s_noise[3 * j]);
        wave_sync();
        if (!PACKED || S.pk_stride == 0)
            step_group<BF16, 1, U * 2, true>(G, H, nrows, s_row, s_rb1, s_rsb2, lane, dar_scale, s2, s_noise);
    }
    // the packed pass is compiled only into the kernels for packed scenes, so
    // the per-group kernels keep their register budget
    if constexpr (PACKED) {
        if (S.pk_stride > 0) {
            step_packed<BF16, U, NOISE>(S, H, seed, nrows, s_row, s_rb1, s_rsb2, lane, s_noise);
            return;
        }
    }
    for (int gi = 0; gi < S.n_groups; ++gi) {
        if (gi == first) continue;
        const KGroup& G = S.g[gi];
        // lambda / N_I' rounded once from double, exactly as a host would form it
        const float dar_scale = (G.dar_kind != GS_DAR_NONE && G.reg_mode == GS_REG_ADAPTIVE)
                                    ? (float)(G.dar_lambda / H.reg_norm)
                                    : (float)G.dar_lambda;
        const uint64_t s2 = BF16 ? d_stream(seed, kTagSrStep + (uint64_t)gi, H.iteration) : 0;
        if (G.vec == 4) step_group<BF16, 4, U>(G, H, nrows, s_row, s_rb1, s_rsb2, lane, dar_scale, s2);
        else if (G.vec == 2) step_group<BF16, 2, U>(G, H, nrows, s_row, s_rb1, s_rsb2, lane, dar_scale, s2);
        else step_group<BF16, 1, U * 2>(G, H, nrows, s_row, s_rb1, s_rsb2, lane, dar_scale, s2);
    }
}

template <bool BF16>
__device__ __forceinline__ void invisible_all_groups(const KScene& S, const KHyper& H, uint64_t seed, int nrows,
                                                     const int* s_row, const float* s_rb1, const float* s_rsb2,
                                                     int lane)
{
    for (int gi = 0; gi < S.n_groups; ++gi) {
        const KGroup& G = S.g[gi];
        const uint64_t s2 = BF16 ? d_stream(seed, kTagSrRsr + (uint64_t)gi, H.iteration) : 0;
        const float lr_aiu = (float)((double)G.lr * H.aiu_scale);
        if (G.vec == 4) invisible_group<BF16, 4>(G, H, nrows, s_row, s_rb1, s_rsb2, lane, s2, lr_aiu);
        else if (G.vec == 2) invisible_group<BF16, 2>(G, H, nrows, s_row, s_rb1, s_rsb2, lane, s2, lr_aiu);
        else invisible_group<BF16, 1>(G, H, nrows, s_row, s_rb1, s_rsb2, lane, s2, lr_aiu);
    }
}

}  // namespace gs
