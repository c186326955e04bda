// The FP32 visibility predicate shared by the visibility kernels and the
// fused view step (definition in gsopt.h, "Visibility").
#pragma once

#include "internal.h"

namespace gs {

// The FP32 predicate, one rounding per operation in the stated order (no
// contraction into fused multiply-add).
__device__ __forceinline__ bool visible_pred(float x, float y, float z, const float* rho, const KCamera& c)
{
#pragma clang fp contract(off)
    const float px = ((c.R[0] * x + c.R[1] * y) + c.R[2] * z) + c.R[3];
    const float py = ((c.R[4] * x + c.R[5] * y) + c.R[6] * z) + c.R[7];
    const float pz = ((c.R[8] * x + c.R[9] * y) + c.R[10] * z) + c.R[11];
    if (!(pz > c.z_near)) return false;
    if (!(pz < c.z_far)) return false;
    const float u = (c.fx * px) / pz + c.cx;
    const float v = (c.fy * py) / pz + c.cy;
    float r = 0.0f;
    if (rho != nullptr) {
        r = (c.f_max * *rho) / pz;
        if (!(r >= c.r_min)) return false;
    }
    if (!(u + r >= 0.0f)) return false;
    if (!(u - r <= c.W)) return false;
    if (!(v + r >= 0.0f)) return false;
    if (!(v - r <= c.H)) return false;
    return true;
}

}  // namespace gs
