// Visibility fused into the step: one launch evaluates the FP32 predicate of
// every primitive of a wave's window from its pre-update mean, steps the
// visible rows and, on Re-State or AIU iterations, treats the window's
// invisible sampled rows.  Nothing goes through HBM between the cull and
// the update (no mask or index list, no counter to clear), and the results
// are those of gs_visibility followed by the masked step, bit for bit.
#include "device_common.h"
#include "predicate.h"

namespace gs {

#ifndef GS_STEP_UNROLL
#define GS_STEP_UNROLL 4
#endif
#ifndef GS_STEP_UNROLL_BF16
#define GS_STEP_UNROLL_BF16 2
#endif

// Visible from the one camera, or (CAMS = KCameras) from any camera of the batch.
__device__ __forceinline__ bool visible_any(float x, float y, float z, const float* rho, const KCamera& c)
{
    return visible_pred(x, y, z, rho, c);
}

__device__ __forceinline__ bool visible_any(float x, float y, float z, const float* rho, const KCameras& cs)
{
    bool v = false;
    for (int k = 0; k < cs.n; ++k) v = v || visible_pred(x, y, z, rho, cs.c[k]);
    return v;
}

template <bool BF16, int UNIT, bool NOISE, bool RADIUS, bool PACKED, typename CAMS>
__global__ __launch_bounds__(kBlock) void step_view_kernel(KScene S, KHyper H, CAMS cam,
                                                           const float* __restrict__ means, int64_t ms,
                                                           const float* __restrict__ radius,
                                                           uint8_t* __restrict__ mask_out)
{
    // rounds of 64 primitives per lane group; a 32-primitive window leaves the
    // upper half of the lanes idle during the cull
    constexpr int R = (UNIT + kWave - 1) / kWave;
    __shared__ int s_row[kWavesPerBlock][UNIT];
    __shared__ float s_rb1[kWavesPerBlock][UNIT];
    __shared__ float s_rsb2[kWavesPerBlock][UNIT];
    __shared__ float s_noise[kWavesPerBlock][NOISE ? 3 * UNIT : 1];   // position-noise displacements
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);   // the same on every lane
    const int lane = threadIdx.x % kWave;
    const int64_t w0 = ((int64_t)blockIdx.x * kWavesPerBlock + wave) * UNIT;
    if (w0 >= S.n) return;

    // the window's means (all loads first; past the end: the last one, discarded)
    float x[R], y[R], z[R], rho[R];
#pragma unroll
    for (int b = 0; b < R; ++b) {
        const int64_t i = min(w0 + b * kWave + lane, S.n - 1);
        x[b] = means[ms * i];
        y[b] = means[ms * i + 1];
        z[b] = means[ms * i + 2];
        rho[b] = RADIUS ? radius[i] : 0.0f;
    }
    bool vis[R], in[R];
#pragma unroll
    for (int b = 0; b < R; ++b) {
        in[b] = b * kWave + lane < UNIT && w0 + b * kWave + lane < S.n;
        vis[b] = in[b] && visible_any(x[b], y[b], z[b], RADIUS ? &rho[b] : nullptr, cam);
        if (mask_out != nullptr && in[b]) mask_out[w0 + b * kWave + lane] = (uint8_t)vis[b];
    }

    const uint64_t seed = H.seed + (uint64_t)S.seed_offset;
    int nrows = 0;
#pragma unroll
    for (int b = 0; b < R; ++b) {
        const uint64_t bal = __ballot(vis[b]);
        if (vis[b]) s_row[wave][nrows + lanes_below(bal)] = (int)(w0 + b * kWave + lane);
        nrows += __popcll(bal);
    }
    if (nrows > 0) {
        wave_sync();
        stage_step_rows(nrows, s_row[wave], s_rb1[wave], s_rsb2[wave], S.t, H,
                        d_stream(seed, kTagRsr, H.iteration), lane);
        wave_sync();
        step_all_groups<BF16, NOISE, BF16 ? GS_STEP_UNROLL_BF16 : GS_STEP_UNROLL, PACKED>(S, H, seed, nrows, s_row[wave],
                                                                                  s_rb1[wave], s_rsb2[wave], lane,
                                                                                  s_noise[wave]);
    }
    if (H.rsr_thr == 0 && H.aiu_thr == 0) return;

    // invisible rows of the window in this iteration's Re-State or AIU sample
    wave_sync();   // the staged visible rows are done with
    const uint64_t rsr_s2 = d_stream(seed, kTagRsr, H.iteration);
    const uint64_t aiu_s2 = d_stream(seed, kTagAiu, H.iteration);
    nrows = 0;
#pragma unroll
    for (int b = 0; b < R; ++b) {
        const int64_t i = w0 + b * kWave + lane;
        const bool inv = in[b] && !vis[b];
        const bool rsr = inv && H.rsr_thr != 0 && rsr_sampled(rsr_s2, H.rsr_thr, i);
        int ti = 0;
        if (inv && H.aiu_thr != 0 && rsr_sampled(aiu_s2, H.aiu_thr, i)) ti = S.t[i];
        const bool aiu = ti > 0;
        const bool pick = rsr || aiu;
        const uint64_t bal = __ballot(pick);
        if (pick) {
            const int j = nrows + lanes_below(bal);
            s_row[wave][j] = rsr ? (int)((uint32_t)i | 0x80000000u) : (int)i;
            float rb1 = 0.0f, rsb2 = 0.0f;
            if (aiu) {
                const float ft = (float)ti;
                rb1 = 1.0f / -expm1f(ft * H.logb1);
                rsb2 = 1.0f / __fsqrt_rn(-expm1f(ft * H.logb2));
            }
            s_rb1[wave][j] = rb1;
            s_rsb2[wave][j] = rsb2;
        }
        nrows += __popcll(bal);
    }
    if (nrows == 0) return;
    wave_sync();
    invisible_all_groups<BF16>(S, H, seed, nrows, s_row[wave], s_rb1[wave], s_rsb2[wave], lane);
}

namespace {

template <typename CAMS>
using ViewFn = void (*)(KScene, KHyper, CAMS, const float*, int64_t, const float*, uint8_t*);

template <bool BF16, bool NOISE, bool RADIUS, bool PACKED, typename CAMS>
ViewFn<CAMS> pick_view(int unit)
{
    switch (unit) {
    case 32: return step_view_kernel<BF16, 32, NOISE, RADIUS, PACKED, CAMS>;
    case 64: return step_view_kernel<BF16, 64, NOISE, RADIUS, PACKED, CAMS>;
    case 128: return step_view_kernel<BF16, 128, NOISE, RADIUS, PACKED, CAMS>;
    case 256: return step_view_kernel<BF16, 256, NOISE, RADIUS, PACKED, CAMS>;
    default: return nullptr;
    }
}

template <bool PACKED, typename CAMS>
ViewFn<CAMS> pick_view(bool bf16, int unit, bool noise, bool radius)
{
    if (bf16) {
        if (noise)
            return radius ? pick_view<true, true, true, PACKED, CAMS>(unit) : pick_view<true, true, false, PACKED, CAMS>(unit);
        return radius ? pick_view<true, false, true, PACKED, CAMS>(unit) : pick_view<true, false, false, PACKED, CAMS>(unit);
    }
    if (noise)
        return radius ? pick_view<false, true, true, PACKED, CAMS>(unit) : pick_view<false, true, false, PACKED, CAMS>(unit);
    return radius ? pick_view<false, false, true, PACKED, CAMS>(unit) : pick_view<false, false, false, PACKED, CAMS>(unit);
}

template <typename CAMS>
hipError_t launch_view(const KScene& s, const KHyper& h, const CAMS& cams, const float* means, int64_t ms,
                       const float* radius, uint8_t* mask_out, hipStream_t stream)
{
    if (s.n == 0) return hipSuccess;
    ViewFn<CAMS> fn = s.pk_stride > 0 ? pick_view<true, CAMS>(s.bf16 != 0, s.unit, h.noise != 0, radius != nullptr)
                                      : pick_view<false, CAMS>(s.bf16 != 0, s.unit, h.noise != 0, radius != nullptr);
    if (fn == nullptr) return hipErrorInvalidValue;
    const int64_t units = (s.n + s.unit - 1) / s.unit;
    const unsigned blocks = (unsigned)((units + kWavesPerBlock - 1) / kWavesPerBlock);
    hipLaunchKernelGGL(fn, dim3(blocks), dim3(kBlock), 0, stream, s, h, cams, means, ms, radius, mask_out);
    return hipGetLastError();
}

}  // namespace

// One camera: the camera itself is the kernel argument; several: the batch.
hipError_t launch_step_view(const KScene& s, const KHyper& h, const KCameras& cams, const float* means, int64_t ms,
                            const float* radius, uint8_t* mask_out, hipStream_t stream)
{
    if (cams.n == 1) return launch_view(s, h, cams.c[0], means, ms, radius, mask_out, stream);
    return launch_view(s, h, cams, means, ms, radius, mask_out, stream);
}

}  // namespace gs
