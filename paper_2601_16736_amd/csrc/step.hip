// Single-scene AdamW-GS step kernels: the fused Sparse-Adam + DAR pass and
// the Re-State Regularization pass (gfx950).
#include "device_common.h"

namespace gs {

// One wave per unit.  SCHED picks where the unit's rows come from:
//   compacted: entries [unit*UNIT, unit*UNIT + UNIT) of the visible-index list
//   masked:    visible primitives of the window [unit*UNIT, unit*UNIT + UNIT)
//   dense:     every primitive of that window (V = 1)
// The grid covers the largest possible unit count; waves past the end exit.
// NOISE adds the position-noise displacement to the mean group.
// Items in flight per lane: four with FP32 moments (faster than two on the
// 3M scene; 126 VGPRs, no scratch), two with BF16 moments (four spills there).
#ifndef GS_STEP_UNROLL
#define GS_STEP_UNROLL 4
#endif
#ifndef GS_STEP_UNROLL_BF16
#define GS_STEP_UNROLL_BF16 2
#endif

template <bool BF16, int SCHED, int UNIT, bool NOISE, bool PACKED>
__global__ __launch_bounds__(kBlock) void step_kernel(KScene S, KHyper H)
{
    __shared__ int s_row[kWavesPerBlock][UNIT];
    __shared__ float s_rb1[kWavesPerBlock][UNIT];
    __shared__ float s_rsb2[kWavesPerBlock][UNIT];
    __shared__ float s_noise[kWavesPerBlock][NOISE ? 3 * UNIT : 1];   // position-noise displacements
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);   // the same on every lane
    const int lane = threadIdx.x % kWave;
    const int64_t unit = (int64_t)blockIdx.x * kWavesPerBlock + wave;
    int nrows;
    if constexpr (SCHED == kSchedCompacted) {
        const int cnt = (int)min((int64_t)*S.count, S.n);   // the list holds at most n entries
        const int64_t base = unit * UNIT;
        if (base >= cnt) return;
        nrows = build_rows_slice<UNIT>(S.idx, cnt, S.n, base, s_row[wave], lane);
    } else {
        const int64_t w0 = unit * UNIT;
        if (w0 >= S.n) return;
        nrows = build_rows_window<UNIT>(SCHED == kSchedMasked ? S.mask : nullptr, S.n, w0, s_row[wave], lane);
    }
    if (nrows == 0) return;
    const uint64_t seed = H.seed + (uint64_t)S.seed_offset;
    wave_sync();
    stage_step_rows(nrows, s_row[wave], s_rb1[wave], s_rsb2[wave], S.t, H, d_stream(seed, kTagRsr, H.iteration),
                    lane);
    wave_sync();
    step_all_groups<BF16, NOISE, BF16 ? GS_STEP_UNROLL_BF16 : GS_STEP_UNROLL, PACKED>(S, H, seed, nrows, s_row[wave],
                                                                            s_rb1[wave], s_rsb2[wave], lane,
                                                                            s_noise[wave]);
}

// Pass over the primitives the step does not visit (mask == 0): each wave
// takes a window of 512, stages the invisible rows in this iteration's
// Re-State or AIU sample and applies both in every group.  Sampled visible
// rows are rescaled inside the step kernel, in registers, before their
// moment update.
constexpr int kInvUnit = 512;

template <bool BF16>
__global__ __launch_bounds__(kBlock) void invisible_kernel(KScene S, KHyper H)
{
    __shared__ int s_row[kWavesPerBlock][kInvUnit];
    __shared__ float s_rb1[kWavesPerBlock][kInvUnit];
    __shared__ float s_rsb2[kWavesPerBlock][kInvUnit];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);   // the same on every lane
    const int lane = threadIdx.x % kWave;
    const int64_t w0 = ((int64_t)blockIdx.x * kWavesPerBlock + wave) * kInvUnit;
    if (w0 >= S.n) return;
    const uint64_t seed = H.seed + (uint64_t)S.seed_offset;
    const int nrows = build_rows_invisible<kInvUnit>(S.mask, S.n, w0, S.t, H, d_stream(seed, kTagRsr, H.iteration),
                                                     d_stream(seed, kTagAiu, H.iteration), s_row[wave],
                                                     s_rb1[wave], s_rsb2[wave], lane);
    if (nrows == 0) return;
    wave_sync();
    invisible_all_groups<BF16>(S, H, seed, nrows, s_row[wave], s_rb1[wave], s_rsb2[wave], lane);
}

namespace {

using StepFn = void (*)(KScene, KHyper);

template <bool BF16, bool NOISE, bool PACKED>
StepFn pick(int sched, int unit)
{
    if (sched == kSchedCompacted) {
        switch (unit) {
        case 32: return step_kernel<BF16, kSchedCompacted, 32, NOISE, PACKED>;
        case 64: return step_kernel<BF16, kSchedCompacted, 64, NOISE, PACKED>;
        case 128: return step_kernel<BF16, kSchedCompacted, 128, NOISE, PACKED>;
        case 256: return step_kernel<BF16, kSchedCompacted, 256, NOISE, PACKED>;
        case 512: return step_kernel<BF16, kSchedCompacted, 512, NOISE, PACKED>;
        default: return nullptr;
        }
    }
    if (sched == kSchedMasked) {
        switch (unit) {
        case 32: return step_kernel<BF16, kSchedMasked, 32, NOISE, PACKED>;
        case 64: return step_kernel<BF16, kSchedMasked, 64, NOISE, PACKED>;
        case 128: return step_kernel<BF16, kSchedMasked, 128, NOISE, PACKED>;
        case 256: return step_kernel<BF16, kSchedMasked, 256, NOISE, PACKED>;
        case 512: return step_kernel<BF16, kSchedMasked, 512, NOISE, PACKED>;
        default: return nullptr;
        }
    }
    if (sched == kSchedDense) {
        switch (unit) {
        case 64: return step_kernel<BF16, kSchedDense, 64, NOISE, PACKED>;
        case 256: return step_kernel<BF16, kSchedDense, 256, NOISE, PACKED>;
        case 512: return step_kernel<BF16, kSchedDense, 512, NOISE, PACKED>;
        default: return nullptr;
        }
    }
    return nullptr;
}

}  // namespace

size_t step_kernel_units(const KScene& s)
{
    return (size_t)((s.n + s.unit - 1) / s.unit);
}

hipError_t launch_step(const KScene& s, const KHyper& h, hipStream_t stream)
{
    if (s.n == 0) return hipSuccess;
    if (s.sched != kSchedDense) {
        const hipError_t e = launch_invisible(s, h, stream);
        if (e != hipSuccess) return e;
    }
    StepFn fn;
    if (s.pk_stride > 0)
        fn = s.bf16 ? (h.noise ? pick<true, true, true>(s.sched, s.unit) : pick<true, false, true>(s.sched, s.unit))
                    : (h.noise ? pick<false, true, true>(s.sched, s.unit) : pick<false, false, true>(s.sched, s.unit));
    else
        fn = s.bf16 ? (h.noise ? pick<true, true, false>(s.sched, s.unit) : pick<true, false, false>(s.sched, s.unit))
                    : (h.noise ? pick<false, true, false>(s.sched, s.unit)
                               : pick<false, false, false>(s.sched, s.unit));
    if (fn == nullptr) return hipErrorInvalidValue;
    const size_t units = step_kernel_units(s);
    const unsigned blocks = (unsigned)((units + kWavesPerBlock - 1) / kWavesPerBlock);
    hipLaunchKernelGGL(fn, dim3(blocks), dim3(kBlock), 0, stream, s, h);
    return hipGetLastError();
}

hipError_t launch_invisible(const KScene& s, const KHyper& h, hipStream_t stream)
{
    if (s.n == 0 || (h.rsr_thr == 0 && h.aiu_thr == 0) || s.mask == nullptr) return hipSuccess;
    const size_t units = (size_t)((s.n + kInvUnit - 1) / kInvUnit);
    const unsigned blocks = (unsigned)((units + kWavesPerBlock - 1) / kWavesPerBlock);
    if (s.bf16) hipLaunchKernelGGL(invisible_kernel<true>, dim3(blocks), dim3(kBlock), 0, stream, s, h);
    else hipLaunchKernelGGL(invisible_kernel<false>, dim3(blocks), dim3(kBlock), 0, stream, s, h);
    return hipGetLastError();
}

}  // namespace gs
