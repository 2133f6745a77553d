// Device helpers shared by the CSR kernels (streaming step and resident
// loop): the nonlinearity f of Eq. 8, operand byte packing, and the update of
// Eqs. 6-7 with the wall (one routine, so that every CSR kernel produces the
// same bits).
#pragma once

#include "sbqa_internal.h"

namespace sbqa {
namespace csr {

__device__ __forceinline__ float f_value(int fmode, float x, float delta) {
    if (fmode == 2) return x;
    const float d = (fmode == 1) ? 0.0f : delta;
    if (fabsf(x) <= d) return 0.0f;
    return x > 0.0f ? 1.0f : -1.0f;
}

__device__ __forceinline__ uint32_t pack_ternary(float a, float b, float c, float d) {
    auto q = [](float v) -> uint32_t { return (uint32_t)(uint8_t)(int8_t)(v > 0.0f ? 1 : (v < 0.0f ? -1 : 0)); };
    return q(a) | (q(b) << 8) | (q(c) << 16) | (q(d) << 24);
}

// Update of one element (Eqs. 6-7 and the wall): kick with the pump term, the
// coupling sum plus field and the ring, then drift, then clamp. Shared by both
// CSR kernels so that they produce identical bits. so = copysign(1, x_new),
// the same before and after the clamp (which keeps the sign), so f of Eq. 8
// is |x_new| > Delta ? so : 0.
__device__ __forceinline__ void update_elem(float x, float y, float phi, float hv, float xl, float xr, float jpr,
                                            float kA, float kB, float dt, float kD, float &xo, float &yo,
                                            float &so) {
#pragma clang fp contract(off)
    // force = -kA x + kB (phi + h) + J_perp (x_left + x_right), with explicit
    // fused multiply-adds so every kernel that calls this rounds identically
    const float force = __builtin_fmaf(jpr, xl + xr, __builtin_fmaf(kB, phi + hv, -kA * x));
    float yn = __builtin_fmaf(dt, force, y);
    float xn = __builtin_fmaf(kD, yn, x);
    const float sg = __builtin_copysignf(1.0f, xn);
    if (fabsf(xn) > 1.0f) {  // |x| > 1 (NaN excluded): the clamp is the sign
        xn = sg;
        yn = 0.0f;
    }
    xo = xn;
    yo = yn;
    so = sg;
}
__device__ __forceinline__ void update_elem(float x, float y, float phi, float hv, float xl, float xr, float jpr,
                                            float kA, float kB, float dt, float kD, float &xo, float &yo) {
    float so;
    update_elem(x, y, phi, hv, xl, xr, jpr, kA, kB, dt, kD, xo, yo, so);
}

__device__ __forceinline__ uint32_t ternary_byte(float x, float d) {
    return (uint32_t)(uint8_t)(int8_t)(x > d ? 1 : (x < -d ? -1 : 0));
}

}  // namespace csr
}  // namespace sbqa
