// Plain-form descriptor gather (Sec. 4.2, Fig. 5): per shading point the K levels of
// the 5x5x9 light-oriented stencil, trilinearly interpolated from float32 mip levels,
// written row by row to HBM together with gamma.
#include "internal.h"
#include "frame.h"

namespace ds {
namespace {

constexpr int kThreads = 256;

template <typename T>
__device__ __forceinline__ void store(T *z, int64_t i, float v);
template <>
__device__ __forceinline__ void store<float>(float *z, int64_t i, float v)
{
    z[i] = v;
}
template <>
__device__ __forceinline__ void store<uint16_t>(uint16_t *z, int64_t i, float v)
{
    uint32_t u = __float_as_uint(v);
    u += 0x7FFFu + ((u >> 16) & 1u);
    z[i] = (uint16_t)(u >> 16);
}

// Voxel-centred trilinear interpolation with zero outside the level grid.
__device__ __forceinline__ float trilinear(const float *__restrict__ d, int nx, int ny, int nz,
                                           float ux, float uy, float uz)
{
    float fx0 = floorf(ux), fy0 = floorf(uy), fz0 = floorf(uz);
    float fx = ux - fx0, fy = uy - fy0, fz = uz - fz0;
    int ix = (int)fx0, iy = (int)fy0, iz = (int)fz0;
    float acc = 0.f;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        int dx = c & 1, dy = (c >> 1) & 1, dz = (c >> 2) & 1;
        int a = ix + dx, b = iy + dy, e = iz + dz;
        if (a >= 0 && b >= 0 && e >= 0 && a < nx && b < ny && e < nz) {
            float w = (dx ? fx : 1.f - fx) * (dy ? fy : 1.f - fy) * (dz ? fz : 1.f - fz);
            acc += w * d[((int64_t)e * ny + b) * nx + a];
        }
    }
    return acc;
}

// One block per point: the block's threads stride over the 225 K samples.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_gather(GatherArgs a, int64_t p0, T *z, int64_t ldz,
                                                     uint8_t *flags)
{
    int64_t p = p0 + blockIdx.x;
    if (p >= a.P)
        return;
    T *row = z + (int64_t)blockIdx.x * ldz;
    float x[3] = {a.pos[3 * p], a.pos[3 * p + 1], a.pos[3 * p + 2]};
    Frame f;
    bool ok = isfinite(x[0]) && isfinite(x[1]) && isfinite(x[2]) &&
              light_frame(&a.view[3 * p], &a.light[3 * p], f);
    const int D = kStencil * a.K + 1;
    if (!ok) {
        for (int i = threadIdx.x; i < D; i += kThreads)
            store<T>(row, i, 0.f);
        if (flags && threadIdx.x == 0)
            flags[p] = DS_FLAG_INVALID;
        return;
    }
    for (int i = threadIdx.x; i < D - 1; i += kThreads) {
        int k = i / kStencil, n = i - k * kStencil;
        const GatherLevel L = a.lv[k];
        int ix = n % 5, iy = (n / 5) % 5, iz = n / 25;
        float ox = -1.f + 0.5f * ix, oy = -1.f + 0.5f * iy, oz = -1.f + 0.5f * iz;
        float u[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            float q = x[c] + L.step * (ox * f.X[c] + oy * f.Y[c] + oz * f.Z[c]);
            u[c] = (q - a.amin[c]) * L.inv_h - 0.5f;
        }
        store<T>(row, i, trilinear(L.data, L.nx, L.ny, L.nz, u[0], u[1], u[2]));
    }
    if (threadIdx.x == 0) {
        store<T>(row, D - 1, f.gamma);
        if (flags)
            flags[p] = point_flags(x, f, a.amin, a.amax, a.inv_mean);
    }
}

// Outputs of points flagged invalid are defined as zero.
__global__ void __launch_bounds__(256) k_mask(const uint8_t *__restrict__ flags, int64_t n,
                                              float *out, float *pre)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && (flags[i] & DS_FLAG_INVALID)) {
        out[i] = 0.f;
        if (pre)
            pre[i] = 0.f;
    }
}

}  // namespace

ds_status mask_invalid(hipStream_t s, const uint8_t *flags, int64_t n, float *out, float *pre)
{
    if (n <= 0)
        return DS_OK;
    k_mask<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(flags, n, out, pre);
    DS_HIP(hipGetLastError());
    return DS_OK;
}

ds_status gather_plain(hipStream_t s, const GatherArgs &a, int64_t p0, int64_t np, ds_dtype odt,
                       void *z, int64_t ldz, uint8_t *flags)
{
    if (np <= 0)
        return DS_OK;
    if (odt == DS_F32)
        k_gather<float><<<(unsigned)np, kThreads, 0, s>>>(a, p0, (float *)z, ldz, flags);
    else
        k_gather<uint16_t><<<(unsigned)np, kThreads, 0, s>>>(a, p0, (uint16_t *)z, ldz, flags);
    DS_HIP(hipGetLastError());
    return DS_OK;
}

}  // namespace ds
