// O(n) bond activation with Wolff's embedding (Sec. 2 of the paper), shared
// by the tiled pyrochlore sweep and the generic graph sweep:
//   sigma = fmaf(s_z, r_z, fmaf(s_y, r_y, s_x * r_x))      (XY: no z term)
//   x     = (x0 * sigma_a) * sigma_b,   x0 = (float)(2 J / T)
//   bond active iff (double)x > -log1p(-u), u = (r32 + 0.5) 2^-32.
// The FP64 log1p is evaluated only when x lies within 1e-4 (1 + t) of
// t = -ln(1 - u) computed in FP32 with the native base-2 logarithm: that
// margin exceeds the FP32 error by orders of magnitude, so outside it the
// FP32 comparison gives the same answer as the exact one.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace pyro {

template <int NV>
__device__ __forceinline__ float project(const float v[NV], const float r[NV])
{
    float sig = __fmul_rn(v[0], r[0]);
    sig = __fmaf_rn(v[1], r[1], sig);
    if (NV == 3) sig = __fmaf_rn(v[NV - 1], r[NV - 1], sig);
    return sig;
}

// The exact comparison, out of line: it is rarely reached, and 48 inlined
// copies per cell would swell the tile kernel's code.
static __device__ __noinline__ bool on_bond_exact(float x, double u) { return (double)x > -log1p(-u); }

// Exact activation decision of one bond (see the file comment).  1 - u is
// exact in FP64 and at least 2^-33, so its FP32 rounding is a normal number
// within a relative 2^-24.
__device__ __forceinline__ bool on_bond_active(float x, uint32_t r32)
{
    if (!(x > 0.0f)) return false;
    const double u = ((double)r32 + 0.5) * 0x1p-32;
    const float t = -0.6931472f * __log2f((float)(1.0 - u));  // native base-2 logarithm
    const float m = 1e-4f * (1.0f + t);
    if (x > t + m) return true;
    if (x < t - m) return false;
    return on_bond_exact(x, u);
}

}  // namespace pyro
