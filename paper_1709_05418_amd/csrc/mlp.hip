// Plain FP32 form of the network layers (Sec. 4.3): one LDS-tiled FP32 GEMM per
// layer on the matrix cores, with bias, optional rank-1 term (the gamma input),
// optional residual and ReLU fused into the epilogue.
#include "internal.h"

namespace ds {
namespace {

constexpr int BM = 64, BN = 64, BK = 16;

typedef float f4v __attribute__((ext_vector_type(4)));

// Elements of the staged A and B tiles: thread t stages elements e = t + 256 q (q < 4)
// of the 64 x 16 tiles, row e / 16 and column k0 + e % 16; the A1/B1 pair covers k < K1,
// the A2/B2 pair the K2 columns after it.
__device__ __forceinline__ void stage_load(const GemmArgs &a, int m0, int n0, int k0, int t,
                                           float (&av)[4], float (&bv)[4])
{
    const int Ktot = a.K1 + a.K2;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int e = t + q * 256;
        const int r = e / BK, k = k0 + e % BK;
        const int m = m0 + r, n = n0 + r;
        av[q] = 0.f;
        bv[q] = 0.f;
        if (k < a.K1) {
            if (m < a.M)
                av[q] = a.A1[(int64_t)m * a.lda1 + k];
            if (n < a.N)
                bv[q] = a.B1[(int64_t)n * a.ldb1 + k];
        } else if (k < Ktot) {
            const int k2 = k - a.K1;
            if (m < a.M)
                av[q] = a.A2[(int64_t)m * a.lda2 + k2];
            if (n < a.N)
                bv[q] = a.B2[(int64_t)n * a.ldb2 + k2];
        }
    }
}

// C = A B^T on the FP32 matrix cores (v_mfma_f32_16x16x4_f32): a 64 x 64 tile per
// workgroup, each wave a 32 x 32 quarter of it as 2 x 2 products of 16 x 16, k steps of
// 16 staged through LDS with the next step's operands loaded into registers meanwhile.
// Lane l supplies A(row l % 16, k l / 16) and B(k l / 16, column l % 16) and receives
// C(rows 4 (l / 16) .. + 3, column l % 16).  (Measured on the plain form's layers, this
// shape at seven waves per SIMD beat k steps of 32 and a variant holding all 200
// columns of a layer per workgroup, both at lower occupancy.)
__global__ void __launch_bounds__(256) k_gemm(GemmArgs a)
{
    __shared__ float As[BK][BM + 4];
    __shared__ float Bs[BK][BN + 4];
    const int t = threadIdx.x;
    const int lane = t & 63, w = t >> 6;
    const int wm = (w & 1) * 32, wn = (w >> 1) * 32;
    const int li = lane & 15, lk = lane >> 4;
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    const int Ktot = a.K1 + a.K2;
    f4v acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
            acc[i][j] = f4v{0.f, 0.f, 0.f, 0.f};
    float av[4], bv[4];
    stage_load(a, m0, n0, 0, t, av, bv);
    for (int k0 = 0; k0 < Ktot; k0 += BK) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = t + q * 256;
            As[e % BK][e / BK] = av[q];
            Bs[e % BK][e / BK] = bv[q];
        }
        __syncthreads();
        if (k0 + BK < Ktot)
            stage_load(a, m0, n0, k0 + BK, t, av, bv);
#pragma unroll
        for (int ks = 0; ks < BK; ks += 4) {
            float x[2], y[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                x[i] = As[ks + lk][wm + 16 * i + li];
                y[i] = Bs[ks + lk][wn + 16 * i + li];
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(x[i], y[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int m = m0 + wm + 16 * i + 4 * lk + v;
                const int n = n0 + wn + 16 * j + li;
                if (m >= a.M || n >= a.N)
                    continue;
                float c = acc[i][j][v];
                if (a.g)
                    c += a.g[(int64_t)m * a.ldg] * a.gw[(int64_t)n * a.ldgw];
                if (a.bias)
                    c += a.bias[n];
                if (a.R)
                    c += a.R[(int64_t)m * a.ldr + n];
                if (a.pre)
                    a.pre[(int64_t)m * a.ldpre + n] = c;
                a.C[(int64_t)m * a.ldc + n] = a.relu ? fmaxf(c, 0.f) : c;
            }
}

// Largest magnitude of x, merged into *out as the bits of a non-negative float (whose
// order as unsigned integers is the order of the values).
__global__ void __launch_bounds__(256) k_amax(const float *__restrict__ x, int64_t n,
                                              unsigned *out)
{
    __shared__ float part[4];
    float m = 0.f;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        m = fmaxf(m, fabsf(x[i]));
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        m = fmaxf(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0)
        part[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        m = fmaxf(fmaxf(part[0], part[1]), fmaxf(part[2], part[3]));
        atomicMax(out, __float_as_uint(m));
    }
}

}  // namespace

ds_status amax_into(hipStream_t s, const float *x, int64_t n, unsigned *out)
{
    if (n <= 0)
        return DS_OK;
    int64_t blocks = (n + 255) / 256;
    k_amax<<<(unsigned)(blocks < 1024 ? blocks : 1024), 256, 0, s>>>(x, n, out);
    DS_HIP(hipGetLastError());
    return DS_OK;
}

ds_status gemm_f32(hipStream_t s, const GemmArgs &a)
{
    if (a.M <= 0 || a.N <= 0)
        return DS_OK;
    dim3 grid((a.N + BN - 1) / BN, (a.M + BM - 1) / BM);
    k_gemm<<<grid, 256, 0, s>>>(a);
    DS_HIP(hipGetLastError());
    return DS_OK;
}

}  // namespace ds
