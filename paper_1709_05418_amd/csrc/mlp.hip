// Plain FP32 form of the network layers (Sec. 4.3): one LDS-tiled FP32 GEMM per
// layer with bias, optional rank-1 term (the gamma input), optional residual and
// ReLU fused into the epilogue.
#include "internal.h"

namespace ds {
namespace {

constexpr int BM = 64, BN = 64, BK = 16, TM = 4, TN = 4;

__global__ void __launch_bounds__(256) k_gemm(GemmArgs a)
{
    __shared__ float As[BK][BM + 4];
    __shared__ float Bs[BK][BN + 4];
    const int t = threadIdx.x;
    const int tx = t % 16, ty = t / 16;
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    float acc[TM][TN] = {};
    const int Ktot = a.K1 + a.K2;
    for (int k0 = 0; k0 < Ktot; k0 += BK) {
        // stage A and B tiles: 64 x 16 each, 4 elements per thread
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            int e = t + q * 256;      // 0..1023
            int r = e / BK, kk = e % BK;
            int k = k0 + kk;
            float av = 0.f, bv = 0.f;
            int m = m0 + r, n = n0 + r;
            if (k < a.K1) {
                if (m < a.M)
                    av = a.A1[(int64_t)m * a.lda1 + k];
                if (n < a.N)
                    bv = a.B1[(int64_t)n * a.ldb1 + k];
            } else if (k < Ktot) {
                int k2 = k - a.K1;
                if (m < a.M)
                    av = a.A2[(int64_t)m * a.lda2 + k2];
                if (n < a.N)
                    bv = a.B2[(int64_t)n * a.ldb2 + k2];
            }
            As[kk][r] = av;
            Bs[kk][r] = bv;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < BK; ++kk) {
            float av[TM], bv[TN];
#pragma unroll
            for (int i = 0; i < TM; ++i)
                av[i] = As[kk][ty * TM + i];
#pragma unroll
            for (int j = 0; j < TN; ++j)
                bv[j] = Bs[kk][tx * TN + j];
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j)
                    acc[i][j] += av[i] * bv[j];
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < TM; ++i) {
        int m = m0 + ty * TM + i;
        if (m >= a.M)
            continue;
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            int n = n0 + tx * TN + j;
            if (n >= a.N)
                continue;
            float v = acc[i][j];
            if (a.g)
                v += a.g[(int64_t)m * a.ldg] * a.gw[(int64_t)n * a.ldgw];
            if (a.bias)
                v += a.bias[n];
            if (a.R)
                v += a.R[(int64_t)m * a.ldr + n];
            if (a.pre)
                a.pre[(int64_t)m * a.ldpre + n] = v;
            a.C[(int64_t)m * a.ldc + n] = a.relu ? fmaxf(v, 0.f) : v;
        }
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
