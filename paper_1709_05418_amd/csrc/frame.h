// Light-oriented local frame of a shading configuration (Sec. 4.2): z toward the
// light, x perpendicular to the plane spanned by z and the view direction, y
// orthogonal to both; gamma = acos(omega . omega_l).  Device code, FP32.
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/deepscatter.h"

namespace ds {

struct Frame {
    float X[3], Y[3], Z[3];
    float gamma;
};

// Unit vector of v; false if v is zero or not finite.  Scaling by the largest
// component first keeps tiny and huge inputs usable.
__device__ __forceinline__ bool unit3(const float *v, float *u)
{
    float a = v[0], b = v[1], c = v[2];
    if (!(isfinite(a) && isfinite(b) && isfinite(c)))
        return false;
    float m = fmaxf(fabsf(a), fmaxf(fabsf(b), fabsf(c)));
    if (m == 0.f)
        return false;
    a /= m;
    b /= m;
    c /= m;
    float l = sqrtf(a * a + b * b + c * c);
    u[0] = a / l;
    u[1] = b / l;
    u[2] = c / l;
    return true;
}

__device__ __forceinline__ bool light_frame(const float *view, const float *light, Frame &f)
{
    float w[3];
    if (!unit3(view, w) || !unit3(light, f.Z))
        return false;
    const float *Z = f.Z;
    float xp[3] = {w[1] * Z[2] - w[2] * Z[1], w[2] * Z[0] - w[0] * Z[2], w[0] * Z[1] - w[1] * Z[0]};
    float s = sqrtf(xp[0] * xp[0] + xp[1] * xp[1] + xp[2] * xp[2]);
    if (s >= 1e-6f) {
        f.X[0] = xp[0] / s;
        f.X[1] = xp[1] / s;
        f.X[2] = xp[2] / s;
    } else {
        // view parallel to the light: any x axis perpendicular to z will do; use the
        // branchless orthonormal basis of Duff et al. (2017)
        float sg = copysignf(1.f, Z[2]);
        float a = -1.f / (sg + Z[2]);
        float b = Z[0] * Z[1] * a;
        f.X[0] = 1.f + sg * Z[0] * Z[0] * a;
        f.X[1] = sg * b;
        f.X[2] = -sg * Z[0];
    }
    const float *X = f.X;
    f.Y[0] = Z[1] * X[2] - Z[2] * X[1];
    f.Y[1] = Z[2] * X[0] - Z[0] * X[2];
    f.Y[2] = Z[0] * X[1] - Z[1] * X[0];
    float c = w[0] * Z[0] + w[1] * Z[1] + w[2] * Z[2];
    c = fminf(1.f, fmaxf(-1.f, c));
    f.gamma = acosf(c);
    return true;
}

// OUTSIDE: x lies outside the grid box.  FALLBACK: a corner of the level-1 stencil
// box ([-1,1]^2 x [-1,3] mean free paths in the light frame) lies outside it.
__device__ __forceinline__ uint8_t point_flags(const float *x, const Frame &f, const float *amin,
                                               const float *amax, float inv_mean)
{
    uint8_t fl = 0;
#pragma unroll
    for (int c = 0; c < 3; ++c)
        if (x[c] < amin[c] || x[c] > amax[c])
            fl |= DS_FLAG_OUTSIDE;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        float ox = (k & 1) ? 1.f : -1.f, oy = (k & 2) ? 1.f : -1.f, oz = (k & 4) ? 3.f : -1.f;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            float q = x[c] + inv_mean * (ox * f.X[c] + oy * f.Y[c] + oz * f.Z[c]);
            if (q < amin[c] || q > amax[c])
                fl |= DS_FLAG_FALLBACK;
        }
    }
    return fl;
}

}  // namespace ds
