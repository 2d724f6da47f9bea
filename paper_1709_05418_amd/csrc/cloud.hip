// Per-cloud precompute: mean extinction over non-zero voxels (Sec. 4.2, 5) and the
// Gaussian density mipmap with sigma_i = 2^i base voxels (Sec. 6), plus the
// corner-packed FP16 copy of every level read by the fused prediction kernel.
#include <math.h>

#include <vector>

#include "internal.h"

namespace ds {
namespace {

__device__ __forceinline__ float load_density(const void *d, ds_dtype dt, int64_t i)
{
    if (dt == DS_F32)
        return static_cast<const float *>(d)[i];
    uint32_t b = static_cast<uint32_t>(static_cast<const uint16_t *>(d)[i]) << 16;
    return __uint_as_float(b);
}

// Error-free sum of two floats (Knuth's two-sum), used to combine (hi, lo) pairs.
__device__ __forceinline__ void two_sum(float a, float b, float &s, float &e)
{
    s = a + b;
    float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

__device__ __forceinline__ void dd_add(float &hi, float &lo, float bhi, float blo)
{
    float s, e;
    two_sum(hi, bhi, s, e);
    e += lo + blo;
    hi = s + e;
    lo = e - (hi - s);
}

constexpr int kMeanBlocks = 1024;
constexpr int kMeanThreads = 256;

// Block-level (hi, lo, count) reduction in LDS; deterministic order.
__device__ void block_reduce(float &hi, float &lo, unsigned long long &cnt)
{
    __shared__ float shi[kMeanThreads], slo[kMeanThreads];
    __shared__ unsigned long long sc[kMeanThreads];
    int t = threadIdx.x;
    shi[t] = hi;
    slo[t] = lo;
    sc[t] = cnt;
    __syncthreads();
    for (int w = kMeanThreads / 2; w > 0; w >>= 1) {
        if (t < w) {
            float h = shi[t], l = slo[t];
            dd_add(h, l, shi[t + w], slo[t + w]);
            shi[t] = h;
            slo[t] = l;
            sc[t] += sc[t + w];
        }
        __syncthreads();
    }
    hi = shi[0];
    lo = slo[0];
    cnt = sc[0];
}

__global__ void __launch_bounds__(kMeanThreads) k_mean_partial(const void *d, ds_dtype dt,
                                                               int64_t n, float2 *part,
                                                               unsigned long long *pcnt)
{
    float sum = 0.f, c = 0.f;  // Kahan-compensated per-thread sum of d over d > 0
    unsigned long long cnt = 0;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        float v = load_density(d, dt, i);
        if (v > 0.f) {
            float y = v - c;
            float t = sum + y;
            c = (t - sum) - y;
            sum = t;
            ++cnt;
        }
    }
    float hi = sum, lo = -c;
    block_reduce(hi, lo, cnt);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = make_float2(hi, lo);
        pcnt[blockIdx.x] = cnt;
    }
}

__global__ void __launch_bounds__(kMeanThreads) k_mean_final(const float2 *part,
                                                             const unsigned long long *pcnt,
                                                             int nb, float2 *out,
                                                             unsigned long long *ocnt)
{
    float hi = 0.f, lo = 0.f;
    unsigned long long cnt = 0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) {
        dd_add(hi, lo, part[i].x, part[i].y);
        cnt += pcnt[i];
    }
    block_reduce(hi, lo, cnt);
    if (threadIdx.x == 0) {
        out[0] = make_float2(hi, lo);
        ocnt[0] = cnt;
    }
}

// One separable Gaussian pass along AXIS with decimation by s = 2^level:
// out[.., m, ..] = sum_e w[e] * in[.., m*s + emin + e, ..], zero outside the input.
// Input dims (n0, n1, n2) = (x, y, z); output has `nout` samples along AXIS.
template <int AXIS, bool FROM_DENSITY>
__global__ void __launch_bounds__(256) k_blur(const void *in, ds_dtype dt, float scale, float *out,
                                              int n0, int n1, int n2, int nout, int s, int emin,
                                              int ntaps, const float *__restrict__ w)
{
    int64_t o0 = AXIS == 0 ? nout : n0;
    int64_t o1 = AXIS == 1 ? nout : n1;
    int64_t o2 = AXIS == 2 ? nout : n2;
    int64_t total = o0 * o1 * o2;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t in_stride = AXIS == 0 ? 1 : (AXIS == 1 ? (int64_t)n0 : (int64_t)n0 * n1);
    int nax = AXIS == 0 ? n0 : (AXIS == 1 ? n1 : n2);
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += stride) {
        int64_t x = idx % o0;
        int64_t r = idx / o0;
        int64_t y = r % o1;
        int64_t z = r / o1;
        int64_t m = AXIS == 0 ? x : (AXIS == 1 ? y : z);
        int64_t base = (AXIS == 0 ? 0 : x) + (AXIS == 1 ? 0 : y * n0) +
                       (AXIS == 2 ? 0 : z * (int64_t)n0 * n1);
        int64_t j0 = m * s + emin;
        int e0 = j0 < 0 ? (int)(-j0) : 0;
        int e1 = ntaps;
        if (j0 + e1 > nax)
            e1 = (int)(nax - j0);
        float sum = 0.f, c = 0.f;
        for (int e = e0; e < e1; ++e) {
            int64_t ii = base + (j0 + e) * in_stride;
            float v = FROM_DENSITY ? load_density(in, dt, ii) * scale
                                   : static_cast<const float *>(in)[ii];
            float y2 = w[e] * v - c;
            float t = sum + y2;
            c = (t - sum) - y2;
            sum = t;
        }
        out[idx] = sum;
    }
}

// FP16 bits of f, round to nearest even, saturated at the largest finite magnitude.
__device__ __forceinline__ uint32_t f16_sat(float f)
{
    const _Float16 h = (_Float16)fmaxf(fminf(f, 65504.f), -65504.f);
    return (uint32_t)__builtin_bit_cast(uint16_t, h);
}

// Corner-packed level with a zero border of bd cells: cell (i, j, k) covers the lattice
// cell whose lower corner is voxel (i - bd, j - bd, k - bd), values zero outside the level
// grid.  Its trilinear function is stored as polynomial coefficients in the fractions
// (tx, ty, tz):  v(t) = P0(ty, tz) + tx P1(ty, tz),  P = A + B ty + tz (C + D ty),
// with P0 the bilinear function of the x0 face and P1 that of the x1 face minus the x0
// face.  FP16, word 0 = (A0, A1), 1 = (B0, B1), 2 = (C0, C1), 3 = (D0, D1), the P0
// coefficient in the low half; the coefficients are formed in FP32 from the level and
// rounded once.  Evaluating this form takes three packed FMAs and one mixed FMA.
__global__ void __launch_bounds__(256) k_pack(const float *__restrict__ lv, int nx, int ny, int nz,
                                              int bd, uint4 *__restrict__ cells)
{
    const int64_t cx = nx + 2 * bd, cy = ny + 2 * bd, cz = nz + 2 * bd;
    const int64_t total = cx * cy * cz;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += stride) {
        const int64_t i = idx % cx - bd, r = idx / cx;
        const int64_t j = r % cy - bd, k = r / cy - bd;
        float v[8];  // corner dx + 2 dy + 4 dz
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int64_t a = i + (c & 1), b = j + ((c >> 1) & 1), e = k + ((c >> 2) & 1);
            const bool in = a >= 0 && b >= 0 && e >= 0 && a < nx && b < ny && e < nz;
            v[c] = in ? lv[(e * ny + b) * nx + a] : 0.f;
        }
        uint32_t w[4];
        float co[2][4];
#pragma unroll
        for (int x = 0; x < 2; ++x) {  // bilinear coefficients of the x = 0 and x = 1 faces
            const float f00 = v[x], f10 = v[x + 2], f01 = v[x + 4], f11 = v[x + 6];
            co[x][0] = f00;
            co[x][1] = f10 - f00;
            co[x][2] = f01 - f00;
            co[x][3] = (f11 - f01) - (f10 - f00);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
            w[q] = f16_sat(co[0][q]) | (f16_sat(co[1][q] - co[0][q]) << 16);
        cells[idx] = make_uint4(w[0], w[1], w[2], w[3]);
    }
}

// Corner-packed float32 level (the plain gather's copy): cell (i, j, k) holds the 8
// corners of the lattice cell whose lower corner is voxel (i - 1, j - 1, k - 1), corner
// c = dx + 2 dy + 4 dz at float c of the cell's 32 bytes, zero outside the grid.
__global__ void __launch_bounds__(256) k_pack32(const float *__restrict__ lv, int nx, int ny,
                                                int nz, float4 *__restrict__ cells)
{
    const int64_t cx = nx + 2, cy = ny + 2, cz = nz + 2;
    const int64_t total = cx * cy * cz;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += stride) {
        const int64_t i = idx % cx - 1, r = idx / cx;
        const int64_t j = r % cy - 1, k = r / cy - 1;
        float v[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int64_t a = i + (c & 1), b = j + ((c >> 1) & 1), e = k + ((c >> 2) & 1);
            const bool in = a >= 0 && b >= 0 && e >= 0 && a < nx && b < ny && e < nz;
            v[c] = in ? lv[(e * ny + b) * nx + a] : 0.f;
        }
        cells[2 * idx] = make_float4(v[0], v[1], v[2], v[3]);
        cells[2 * idx + 1] = make_float4(v[4], v[5], v[6], v[7]);
    }
}

int grid_for(int64_t n)
{
    int64_t b = (n + 255) / 256;
    if (b > 65536)
        b = 65536;
    return (int)(b < 1 ? 1 : b);
}

// Normalised 1-D Gaussian taps of level i: weights for base offsets e = j - m 2^i
// in [emin, emin + ntaps), where t = e + 1/2 - 2^i / 2 lies within 3 sigma.  The
// normaliser runs over all such offsets, so grid borders are darkened, not renormalised.
void level_taps(int i, int *emin, std::vector<float> &w)
{
    double s = ldexp(1.0, i);
    int lo = (int)floor(-3.0 * s - 1.0 + 0.5 * s), hi = (int)ceil(3.0 * s + 1.0 + 0.5 * s);
    std::vector<double> wd;
    int first = 0;
    bool have = false;
    for (int e = lo; e <= hi; ++e) {
        double t = e + 0.5 - 0.5 * s;
        if (fabs(t) <= 3.0 * s) {
            if (!have) {
                first = e;
                have = true;
            }
            wd.push_back(exp(-t * t / (2.0 * s * s)));
        }
    }
    double z = 0.0;
    for (double v : wd)
        z += v;
    w.resize(wd.size());
    for (size_t k = 0; k < wd.size(); ++k)
        w[k] = (float)(wd[k] / z);
    *emin = first;
}

}  // namespace

ds_status cloud_mean(hipStream_t s, const void *d, ds_dtype dt, int64_t n, double *sum,
                     int64_t *count)
{
    float2 *part = nullptr;
    unsigned long long *pc = nullptr;
    DS_HIP(hipMalloc(&part, sizeof(float2) * (kMeanBlocks + 1)));
    if (hipMalloc(&pc, sizeof(unsigned long long) * (kMeanBlocks + 1)) != hipSuccess) {
        (void)hipFree(part);
        set_error("out of device memory for the mean reduction");
        return DS_ERR_OOM;
    }
    k_mean_partial<<<kMeanBlocks, kMeanThreads, 0, s>>>(d, dt, n, part, pc);
    k_mean_final<<<1, kMeanThreads, 0, s>>>(part, pc, kMeanBlocks, part + kMeanBlocks,
                                            pc + kMeanBlocks);
    float2 h;
    unsigned long long c;
    hipError_t e = hipGetLastError();
    if (e == hipSuccess)
        e = hipMemcpyAsync(&h, part + kMeanBlocks, sizeof(h), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(&c, pc + kMeanBlocks, sizeof(c), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    (void)hipFree(part);
    (void)hipFree(pc);
    if (e != hipSuccess)
        return hip_fail(e, "mean reduction");
    *sum = (double)h.x + (double)h.y;
    *count = (int64_t)c;
    return DS_OK;
}

ds_status cloud_pyramid(hipStream_t s, const void *d, ds_dtype dt, int nx, int ny, int nz,
                        float scale, int L, const Level *lv, float *pyr)
{
    // scratch for the x and x-y filtered volumes (sized for level 0)
    size_t na = (size_t)nx * ny * nz, nb = na;
    float *A = nullptr, *B = nullptr, *w = nullptr;
    DS_HIP(hipMalloc(&A, na * sizeof(float)));
    if (hipMalloc(&B, nb * sizeof(float)) != hipSuccess) {
        (void)hipFree(A);
        set_error("out of device memory for the pyramid build");
        return DS_ERR_OOM;
    }
    ds_status st = DS_OK;
    std::vector<float> taps;
    for (int i = 0; i < L && st == DS_OK; ++i) {
        int emin = 0;
        level_taps(i, &emin, taps);
        hipError_t e = hipMalloc(&w, taps.size() * sizeof(float));
        if (e == hipSuccess)
            e = hipMemcpy(w, taps.data(), taps.size() * sizeof(float), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            st = hip_fail(e, "pyramid taps");
            break;
        }
        int sI = 1 << i, nt = (int)taps.size();
        const Level &l = lv[i];
        k_blur<0, true><<<grid_for((int64_t)l.nx * ny * nz), 256, 0, s>>>(
            d, dt, scale, A, nx, ny, nz, l.nx, sI, emin, nt, w);
        k_blur<1, false><<<grid_for((int64_t)l.nx * l.ny * nz), 256, 0, s>>>(
            A, dt, 1.f, B, l.nx, ny, nz, l.ny, sI, emin, nt, w);
        k_blur<2, false><<<grid_for((int64_t)l.nx * l.ny * l.nz), 256, 0, s>>>(
            B, dt, 1.f, pyr + l.off, l.nx, l.ny, nz, l.nz, sI, emin, nt, w);
        e = hipGetLastError();
        if (e == hipSuccess)
            e = hipStreamSynchronize(s);
        (void)hipFree(w);
        w = nullptr;
        if (e != hipSuccess)
            st = hip_fail(e, "pyramid level");
    }
    (void)hipFree(A);
    (void)hipFree(B);
    return st;
}

ds_status cloud_pack32(hipStream_t s, const float *pyr, int L, const Level *lv, float4 *cells)
{
    for (int i = 0; i < L; ++i) {
        const Level &l = lv[i];
        int64_t n = (int64_t)(l.nx + 2) * (l.ny + 2) * (l.nz + 2);
        k_pack32<<<grid_for(n), 256, 0, s>>>(pyr + l.off, l.nx, l.ny, l.nz,
                                             cells + 2 * l.cell32_off);
    }
    DS_HIP(hipGetLastError());
    return DS_OK;
}

ds_status cloud_pack(hipStream_t s, const float *pyr, int L, const Level *lv, uint4 *cells)
{
    for (int i = 0; i < L; ++i) {
        const Level &l = lv[i];
        int64_t n = (int64_t)(l.nx + 2 * l.bd) * (l.ny + 2 * l.bd) * (l.nz + 2 * l.bd);
        k_pack<<<grid_for(n), 256, 0, s>>>(pyr + l.off, l.nx, l.ny, l.nz, l.bd,
                                           cells + l.cell_off);
    }
    DS_HIP(hipGetLastError());
    return DS_OK;
}

}  // namespace ds
