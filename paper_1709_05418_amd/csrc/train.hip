// Training step of the network (Sec. 5.2): loss on log(1 + g), backpropagation
// through the progressive residual blocks and trailing layers, Adam on the FP32
// master parameters.  Every reduction over the batch runs in a fixed order, so a
// step is bitwise reproducible.
#include "internal.h"

namespace ds {
namespace {

constexpr int BM = 64, BN = 64, BK = 16;

// C[m][n] (+)= sum_k A(m, k) B(k, n) with A(m, k) = A[m sam + k sak] and
// B(k, n) = B[k sbk + n sbn]; each output element sums over k in order.
__global__ void __launch_bounds__(256) k_gemm_strided(StridedGemm g)
{
    __shared__ float As[BK][BM + 4];
    __shared__ float Bs[BK][BN + 4];
    const int t = threadIdx.x, tx = t % 16, ty = t / 16;
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    float acc[4][4] = {};
    for (int k0 = 0; k0 < g.K; k0 += BK) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = t + q * 256;
            const int r = e % BM, kk = e / BM;  // consecutive threads walk m (or n)
            const int k = k0 + kk;
            float av = 0.f, bv = 0.f;
            if (k < g.K) {
                if (m0 + r < g.M)
                    av = g.A[(int64_t)(m0 + r) * g.sam + (int64_t)k * g.sak];
                if (n0 + r < g.N)
                    bv = g.B[(int64_t)k * g.sbk + (int64_t)(n0 + r) * g.sbn];
            }
            As[kk][r] = av;
            Bs[kk][r] = bv;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < BK; ++kk) {
            float a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                a[i] = As[kk][ty * 4 + i];
                b[i] = Bs[kk][tx * 4 + i];
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[i][j] += a[i] * b[j];
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int m = m0 + ty * 4 + i;
        if (m >= g.M)
            continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int n = n0 + tx * 4 + j;
            if (n >= g.N)
                continue;
            float *c = g.C + (int64_t)m * g.ldc + n;
            *c = g.accumulate ? *c + acc[i][j] : acc[i][j];
        }
    }
}

// x[r][c] *= (pre[r][c] > 0) for an [R][C] block with row strides.
__global__ void __launch_bounds__(256) k_relu_mask(float *x, int ldx, const float *pre, int ldp,
                                                   int R, int C)
{
    const int64_t n = (int64_t)R * C;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / C, c = i % C;
        if (!(pre[r * ldp + c] > 0.f))
            x[r * ldx + c] = 0.f;
    }
}

// db[c] (+)= sum_r d[r][c], rows in order.
__global__ void __launch_bounds__(256) k_colsum(const float *d, int ldd, int R, int C, float *db)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C)
        return;
    float s = 0.f;
    for (int r = 0; r < R; ++r)
        s += d[(int64_t)r * ldd + c];
    db[c] = s;
}

// Output layer: g = relu(pre), residual r = log(1 + g) - t, per-sample loss r^2 and
// d loss / d pre = 2 r / (B (1 + g)) for pre > 0 (else 0).
__global__ void __launch_bounds__(256) k_loss_head(const float *pre, const float *t, int B,
                                                   float *dpre, float *sq)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B)
        return;
    const float p = pre[b];
    const float g = fmaxf(p, 0.f);
    const float r = log1pf(g) - t[b];
    sq[b] = r * r;
    dpre[b] = p > 0.f ? 2.f * r / ((float)B * (1.f + g)) : 0.f;
}

// Mean of the per-sample losses, summed in a fixed tree order.
__global__ void __launch_bounds__(256) k_loss_mean(const float *sq, int B, float *loss)
{
    __shared__ float s[256];
    float acc = 0.f;
    for (int i = threadIdx.x; i < B; i += 256)
        acc += sq[i];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        *loss = s[0] / (float)B;
}

// Adam (Kingma and Ba, Alg. 1) with the bias corrections folded into c1, c2.
__global__ void __launch_bounds__(256) k_adam(float *theta, float *m, float *v, const float *grad,
                                              int64_t n, float lr, float b1, float b2, float eps,
                                              float c1, float c2)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = grad[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        theta[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

int grid1(int64_t n)
{
    int64_t b = (n + 255) / 256;
    return (int)(b > 4096 ? 4096 : (b < 1 ? 1 : b));
}

}  // namespace

ds_status gemm_strided(hipStream_t s, const StridedGemm &g)
{
    if (g.M <= 0 || g.N <= 0)
        return DS_OK;
    dim3 grid((g.N + BN - 1) / BN, (g.M + BM - 1) / BM);
    k_gemm_strided<<<grid, 256, 0, s>>>(g);
    DS_HIP(hipGetLastError());
    return DS_OK;
}

ds_status relu_mask(hipStream_t s, float *x, int ldx, const float *pre, int ldp, int R, int C)
{
    k_relu_mask<<<grid1((int64_t)R * C), 256, 0, s>>>(x, ldx, pre, ldp, R, C);
    DS_HIP(hipGetLastError());
    return DS_OK;
}

ds_status colsum(hipStream_t s, const float *d, int ldd, int R, int C, float *db)
{
    k_colsum<<<(C + 255) / 256, 256, 0, s>>>(d, ldd, R, C, db);
    DS_HIP(hipGetLastError());
    return DS_OK;
}

ds_status loss_head(hipStream_t s, const float *pre, const float *t, int B, float *dpre, float *sq,
                    float *loss)
{
    k_loss_head<<<(B + 255) / 256, 256, 0, s>>>(pre, t, B, dpre, sq);
    if (loss)
        k_loss_mean<<<1, 256, 0, s>>>(sq, B, loss);
    DS_HIP(hipGetLastError());
    return DS_OK;
}

ds_status adam_update(hipStream_t s, float *theta, float *m, float *v, const float *grad,
                      int64_t n, float lr, float b1, float b2, float eps, float c1, float c2)
{
    k_adam<<<grid1(n), 256, 0, s>>>(theta, m, v, grad, n, lr, b1, b2, eps, c1, c2);
    DS_HIP(hipGetLastError());
    return DS_OK;
}

}  // namespace ds
