// Plain-form descriptor gather (Sec. 4.2, Fig. 5): per shading point the K levels of
// the 5x5x9 light-oriented stencil, trilinearly interpolated from corner-packed float32
// copies of the mip levels, written row by row to HBM together with gamma.
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

// Voxel-centred trilinear interpolation with zero outside the level grid, at the cell
// coordinate u (the voxel-centred coordinate plus one).  Clamping u to [0, n + 1] changes
// nothing inside the grid and puts every sample outside it on all-zero border cells, so
// the eight corners need no bounds tests; they arrive in two 16-byte loads.
__device__ __forceinline__ float trilinear_cells(const GatherLevel &L, float ux, float uy,
                                                 float uz)
{
    ux = __builtin_amdgcn_fmed3f(ux, 0.f, L.hx);
    uy = __builtin_amdgcn_fmed3f(uy, 0.f, L.hy);
    uz = __builtin_amdgcn_fmed3f(uz, 0.f, L.hz);
    const uint32_t i = (uint32_t)ux, j = (uint32_t)uy, k = (uint32_t)uz;
    const float fx = __builtin_amdgcn_fractf(ux), fy = __builtin_amdgcn_fractf(uy),
                fz = __builtin_amdgcn_fractf(uz);
    const int64_t cell = (int64_t)i + (int64_t)L.cx * ((int64_t)j + (int64_t)L.cy * k);
    const float4 lo = L.cells[2 * cell], hi = L.cells[2 * cell + 1];
    // corner c = dx + 2 dy + 4 dz
    const float a00 = fmaf(fx, lo.y - lo.x, lo.x), a10 = fmaf(fx, lo.w - lo.z, lo.z);
    const float a01 = fmaf(fx, hi.y - hi.x, hi.x), a11 = fmaf(fx, hi.w - hi.z, hi.z);
    const float b0 = fmaf(fy, a10 - a00, a00), b1 = fmaf(fy, a11 - a01, a01);
    return fmaf(fz, b1 - b0, b0);
}

constexpr int kGatherPts = 64;  // shading points per workgroup, one per lane of each wave

// Lattice geometry of one point at one stencil level, in cell coordinates:
// lattice point (ix, iy, iz) sits at u0 + ix a + iy b + iz c.
struct LatticeGeom {
    float u0[3], a[3], b[3], c[3];
};

// kGatherPts points per workgroup, lane l of every wave on point l.  For each stencil level
// the four waves split the 25 columns (ix, iy) (wave w takes the columns c = w mod 4) and
// each lane walks the nine samples iz = 0..8 of a column of its point, so the 64 addresses
// of a load are the same lattice offset of 64 neighbouring points, which share cache lines
// when the points do (points in camera order); the level's 225 values per point are staged
// in LDS and leave as one contiguous run per point.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_gather(GatherArgs a, int64_t p0, int64_t np, T *z,
                                                     int64_t ldz, uint8_t *flags)
{
    __shared__ float rows[kGatherPts * kStencil];  // one level: [point][25 iz + column]
    const int K = a.K, D = kStencil * K + 1, tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6;
    const int64_t pb = (int64_t)blockIdx.x * kGatherPts;  // first point (chunk-relative)
    const int64_t pl = pb + lane;
    const int n = (int)(np - pb < kGatherPts ? np - pb : kGatherPts);
    float x[3] = {0.f, 0.f, 0.f};
    Frame f = {};
    bool ok = false;
    if (pl < np) {
        const int64_t p = p0 + pl;
        x[0] = a.pos[3 * p];
        x[1] = a.pos[3 * p + 1];
        x[2] = a.pos[3 * p + 2];
        ok = isfinite(x[0]) && isfinite(x[1]) && isfinite(x[2]) &&
             light_frame(&a.view[3 * p], &a.light[3 * p], f);
        if (w == 0) {
            store<T>(z, pl * ldz + (D - 1), ok ? f.gamma : 0.f);
            if (flags)
                flags[p] = ok ? point_flags(x, f, a.amin, a.amax, a.inv_mean)
                              : (uint8_t)DS_FLAG_INVALID;
        }
    }
    for (int k = 0; k < K; ++k) {
        const GatherLevel L = a.lv[k];
        LatticeGeom G = {};
        if (ok) {
            const float hs = 0.5f * L.step * L.inv_h;  // half a lattice unit, in voxels
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                // lattice point (0, 0, 0) has offset (-1, -1, -1) mean free paths
                const float q = x[c] - L.step * (f.X[c] + f.Y[c] + f.Z[c]);
                G.u0[c] = (q - a.amin[c]) * L.inv_h + 0.5f;
                G.a[c] = hs * f.X[c];
                G.b[c] = hs * f.Y[c];
                G.c[c] = hs * f.Z[c];
            }
        }
        float *out = rows + lane * kStencil;
        for (int col = w; col < 25; col += 4) {
            const float ix = (float)(col % 5), iy = (float)(col / 5);
            float ub[3];
#pragma unroll
            for (int c = 0; c < 3; ++c)
                ub[c] = fmaf(iy, G.b[c], fmaf(ix, G.a[c], G.u0[c]));
#pragma unroll
            for (int iz = 0; iz < 9; ++iz)
                out[25 * iz + col] = ok ? trilinear_cells(L, fmaf((float)iz, G.c[0], ub[0]),
                                                          fmaf((float)iz, G.c[1], ub[1]),
                                                          fmaf((float)iz, G.c[2], ub[2]))
                                        : 0.f;
        }
        __syncthreads();
        for (int e = tid; e < n * kStencil; e += kThreads) {
            const int i = e / kStencil, j = e - i * kStencil;
            store<T>(z, (pb + i) * ldz + (int64_t)k * kStencil + j, rows[e]);
        }
        __syncthreads();
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
    const int64_t blocks = (np + kGatherPts - 1) / kGatherPts;
    if (odt == DS_F32)
        k_gather<float><<<(unsigned)blocks, kThreads, 0, s>>>(a, p0, np, (float *)z, ldz, flags);
    else
        k_gather<uint16_t><<<(unsigned)blocks, kThreads, 0, s>>>(a, p0, np, (uint16_t *)z, ldz,
                                                                 flags);
    DS_HIP(hipGetLastError());
    return DS_OK;
}

}  // namespace ds
