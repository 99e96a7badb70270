// Uniform unit n-vector (n = 2, 3) by rejection from the cube [-1, 1]^n:
// attempt a uses Philox counter (c0, c1, stream, a); coordinates are
// (float)(int32)w_k * 2^-31; the draw is accepted when 1e-12 < |v|^2 <= 1
// and normalised with IEEE-rounded square root and division; after 64
// rejections (probability below 1e-17) the x unit vector is returned.
// Used for the random initial state (stream INIT, c0 = site) and for the
// embedding axis of each sweep (stream AXIS, c0 = 0, c1 = sweep).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "philox.hpp"

namespace pyro {

__device__ inline void unit_vector(uint32_t c0, uint32_t c1, uint32_t stream, int n, PhiloxKey key, float out[3])
{
    for (uint32_t a = 0; a < 64u; ++a) {
        const uint4 w = philox4x32_10(c0, c1, stream, a, key);
        const float v0 = (float)(int32_t)w.x * 0x1p-31f;
        const float v1 = (float)(int32_t)w.y * 0x1p-31f;
        const float v2 = (float)(int32_t)w.z * 0x1p-31f;
        float r2 = __fmul_rn(v0, v0);
        r2 = __fmaf_rn(v1, v1, r2);
        if (n == 3) r2 = __fmaf_rn(v2, v2, r2);
        if (r2 > 1e-12f && r2 <= 1.0f) {
            // sqrtf and '/' are correctly rounded under HIP's default
            // -fhip-fp32-correctly-rounded-divide-sqrt
            const float nr = sqrtf(r2);
            out[0] = v0 / nr;
            out[1] = v1 / nr;
            out[2] = n == 3 ? v2 / nr : 0.0f;
            return;
        }
    }
    out[0] = 1.0f;
    out[1] = 0.0f;
    out[2] = 0.0f;
}

}  // namespace pyro
