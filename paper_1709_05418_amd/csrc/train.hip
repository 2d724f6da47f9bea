// Training step of the network (Sec. 5.2): loss on log(1 + g), backpropagation
// through the progressive residual blocks and trailing layers, Adam on the FP32
// master parameters.  Every reduction over the batch runs in a fixed order, so a
// step is bitwise reproducible.
#include "internal.h"

namespace ds {
namespace {

constexpr int BM = 64, BN = 64, BK = 32;
constexpr int NF = BK / 4;  // elements of each operand a thread stages per k step
typedef float f4v __attribute__((ext_vector_type(4)));

// One operand's share of a k step of the FP32 GEMM: NF values of one row (m of A, n of B)
// at k = k0 + kq + j with unit k stride (kc), else at k = k0 + kq + 4 j, zero outside.
struct StageF {
    const float *p;   // element (row, kbeg + kq)
    int64_t sk;
    int kbeg, kq, row;
    bool kc, ok;

    __device__ __forceinline__ void load(int k0, int kend, float (&v)[NF]) const
    {
        const float *q = p + (int64_t)(k0 - kbeg) * sk;
        if (kc) {
#pragma unroll
            for (int j = 0; j < NF; ++j)
                v[j] = ok && k0 + kq + j < kend ? q[j] : 0.f;
        } else {
#pragma unroll
            for (int j = 0; j < NF; ++j)
                v[j] = ok && k0 + kq + 4 * j < kend ? q[(int64_t)4 * j * sk] : 0.f;
        }
    }
    // stored k-major: T[k][row]
    __device__ __forceinline__ void store(float (*T)[BM + 4], const float (&v)[NF]) const
    {
#pragma unroll
        for (int j = 0; j < NF; ++j)
            T[kc ? kq + j : kq + 4 * j][row] = v[j];
    }
};

__device__ __forceinline__ StageF stage_f(const float *base, int64_t s_row, int64_t s_k, int row0,
                                          int rows, int kbeg, int tid)
{
    StageF st;
    st.kc = s_k == 1;
    st.row = st.kc ? tid >> 2 : tid & 63;
    st.kq = st.kc ? NF * (tid & 3) : tid >> 6;
    st.ok = row0 + st.row < rows;
    st.sk = s_k;
    st.kbeg = kbeg;
    st.p = base + (int64_t)(st.ok ? row0 + st.row : 0) * s_row + (int64_t)(kbeg + st.kq) * s_k;
    return st;
}

// C[m][n] (+)= sum_k A(m, k) B(k, n) with A(m, k) = A[m sam + k sak] and
// B(k, n) = B[k sbk + n sbn], in FP32 on the matrix cores (v_mfma_f32_16x16x4_f32): a
// 64 x 64 tile per block, each wave a 32 x 32 quarter as 2 x 2 products of 16 x 16 (lane
// l supplies A(row l % 16, k l / 16) and B(k l / 16, column l % 16) and holds C(rows
// 4 (l / 16) .. + 3, column l % 16)).  Operands are read along their contiguous index and
// the next k step is prefetched into registers.  Split s (blockIdx.z) covers k in
// [s kc, (s+1) kc) in order; several splits write partial tiles to P[s][M][N], which
// k_splitk_sum adds in split order, so every result is reproducible.
__global__ void __launch_bounds__(256) k_gemm_strided(StridedGemm g, int kc, float *P)
{
    __shared__ float As[BK][BM + 4];
    __shared__ float Bs[BK][BN + 4];
    const int t = threadIdx.x;
    const int lane = t & 63, w = t >> 6;
    const int wm = (w & 1) * 32, wn = (w >> 1) * 32;
    const int li = lane & 15, lk = lane >> 4;
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    const int kbeg = blockIdx.z * kc;
    const int kend = min(g.K, kbeg + kc);
    const StageF sa = stage_f(g.A, g.sam, g.sak, m0, g.M, kbeg, t);
    const StageF sb = stage_f(g.B, g.sbn, g.sbk, n0, g.N, kbeg, t);
    f4v acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
            acc[i][j] = f4v{0.f, 0.f, 0.f, 0.f};
    float va[NF], vb[NF];
    if (kbeg < kend) {
        sa.load(kbeg, kend, va);
        sb.load(kbeg, kend, vb);
    }
    for (int k0 = kbeg; k0 < kend; k0 += BK) {
        sa.store(As, va);
        sb.store(Bs, vb);
        __syncthreads();
        if (k0 + BK < kend) {
            sa.load(k0 + BK, kend, va);
            sb.load(k0 + BK, kend, vb);
        }
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
                if (m >= g.M || n >= g.N)
                    continue;
                if (P) {
                    P[((int64_t)blockIdx.z * g.M + m) * g.N + n] = acc[i][j][v];
                } else {
                    float *c = g.C + (int64_t)m * g.ldc + n;
                    *c = g.accumulate ? *c + acc[i][j][v] : acc[i][j][v];
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

constexpr int kColBlocks = 64;  // row blocks of a column sum (pass-1 partials per column)

// Column sums db[c] = sum_r d[r][c] in a fixed order, in two passes.  Pass 1: workgroup
// (x, y) covers 64 columns and the y-th block of `rows` rows, split over 4 slices of
// consecutive rows (each summed in order) that are then added in slice order; pass 2
// adds the row blocks of every column in block order.
__global__ void __launch_bounds__(256) k_colsum_part(const float *__restrict__ d, int ldd, int R,
                                                     int C, int rows, float *__restrict__ part)
{
    __shared__ float red[4][64];
    const int c = blockIdx.x * 64 + (threadIdx.x & 63);
    const int slice = threadIdx.x >> 6;
    const int per = (rows + 3) / 4;
    const int r0 = blockIdx.y * rows + slice * per;
    int r1 = r0 + per;
    r1 = r1 < (int)(blockIdx.y + 1) * rows ? r1 : (int)(blockIdx.y + 1) * rows;
    r1 = r1 < R ? r1 : R;
    float s = 0.f;
    if (c < C) {
#pragma unroll 8
        for (int r = r0; r < r1; ++r)
            s += d[(int64_t)r * ldd + c];
    }
    red[slice][threadIdx.x & 63] = s;
    __syncthreads();
    if (slice == 0 && c < C) {
        const int t = threadIdx.x;
        part[(int64_t)blockIdx.y * C + c] = ((red[0][t] + red[1][t]) + red[2][t]) + red[3][t];
    }
}

__global__ void __launch_bounds__(256) k_colsum_final(const float *__restrict__ part, int RB, int C,
                                                      float *__restrict__ db)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= C)
        return;
    float s = 0.f;
    for (int b = 0; b < RB; ++b)
        s += part[(int64_t)b * C + c];
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
        if ((int)threadIdx.x < w)
            s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        *loss = s[0] / (float)B;
}

// Adam (Kingma and Ba, Alg. 1) with the bias corrections folded into c1, c2.
// Advances the step count and forms the bias corrections of Adam (Kingma and Ba, Alg. 1)
// for it, in FP64, stored as FP32: state = {lr, 1 - b1^t, 1 - b2^t}.
__global__ void k_adam_prep(int64_t *steps, float *state, float b1, float b2)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const int64_t t = *steps + 1;
        *steps = t;
        state[1] = (float)(1.0 - pow((double)b1, (double)t));
        state[2] = (float)(1.0 - pow((double)b2, (double)t));
    }
}

__global__ void __launch_bounds__(256) k_adam(float *theta, float *m, float *v, const float *grad,
                                              int64_t n, float b1, float b2, float eps,
                                              const float *state)
{
    const float lr = state[0], c1 = state[1], c2 = state[2];
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

// ---------------------------------------------------------------- BF16 MFMA GEMM
// C (+)= A B with the strided operands of StridedGemm, every operand rounded to BF16
// (nearest even) as it is staged into LDS, products accumulated in FP32 by
// v_mfma_f32_16x16x32_bf16.  A 256-thread block computes a 64 x 64 tile of C, each
// wave a 32 x 32 quarter (2 x 2 MFMA tiles), over k steps of TK = 128.  Each operand is
// read along its contiguous index: with unit k stride a thread loads 32 consecutive k
// of one row (constant offsets from one pointer, 16-byte LDS stores); with unit row
// stride the 64 threads of a wave cover 64 consecutive rows and a thread walks 32 k
// values 4 apart.  The next step's values are loaded into registers before the
// current step's products, so their latency overlaps the matrix-core work.  Split s
// (blockIdx.z) covers k in [s kc, (s+1) kc); with several splits the partial tiles go
// to P[s][M][N] and k_splitk_sum adds them in split order, so results do not depend
// on timing.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));
constexpr int TM = 64, TN = 64, TK = 128, TKP = TK + 8;
constexpr int NE = TK / 4;  // elements of each operand a thread stages per k step

// One operand's share of a k step: NE values of one row at k = k0 + kq + j (kc: unit k
// stride) or k = k0 + kq + 4 j (otherwise), zero outside.
struct Stage {
    const float *p;   // element (row, kbeg + kq)
    int64_t sk;       // k stride
    int kbeg;         // first k of the split
    int kq;           // first k of this thread inside a step
    bool kc, ok;      // unit k stride; row inside the matrix

    __device__ __forceinline__ void load(int k0, int kend, float (&v)[NE]) const
    {
        const float *q = p + (int64_t)(k0 - kbeg) * sk;
        if (kc) {
            if (ok && k0 + kq + NE <= kend) {
#pragma unroll
                for (int j = 0; j < NE; ++j)
                    v[j] = q[j];
            } else {
#pragma unroll
                for (int j = 0; j < NE; ++j)
                    v[j] = ok && k0 + kq + j < kend ? q[j] : 0.f;
            }
        } else if (ok && k0 + kq + 4 * (NE - 1) < kend) {
            const int64_t s4 = 4 * sk;
#pragma unroll
            for (int j = 0; j < NE; ++j) {
                v[j] = *q;
                q += s4;
            }
        } else {
#pragma unroll
            for (int j = 0; j < NE; ++j)
                v[j] = ok && k0 + kq + 4 * j < kend ? q[(int64_t)4 * j * sk] : 0.f;
        }
    }
};

__device__ __forceinline__ Stage stage_of(const float *base, int64_t s_row, int64_t s_k, int row0,
                                          int rows, int kbeg, int tid)
{
    Stage st;
    st.kc = s_k == 1;
    int r;
    if (st.kc) {
        r = tid >> 2;
        st.kq = NE * (tid & 3);
    } else {
        r = tid & 63;
        st.kq = tid >> 6;
    }
    st.ok = row0 + r < rows;
    st.sk = s_k;
    st.kbeg = kbeg;
    st.p = base + (int64_t)(st.ok ? row0 + r : 0) * s_row + (int64_t)(kbeg + st.kq) * s_k;
    return st;
}

// Stores one operand's NE values (as BF16) at [row][k] of an LDS tile; with L, also the
// rounding remainder v - bf16(v) as a second BF16 term (the pair carries about 16
// significant bits).
template <bool X3>
__device__ __forceinline__ void stage_store(__bf16 (*T)[TKP], __bf16 (*L)[TKP], const Stage &st,
                                            int tid, const float (&v)[NE])
{
    if (st.kc) {
#pragma unroll
        for (int h = 0; h < NE; h += 8) {
            bf16x8 x, y;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                x[j] = (__bf16)v[h + j];
                if (X3)
                    y[j] = (__bf16)(v[h + j] - (float)x[j]);
            }
            *reinterpret_cast<bf16x8 *>(&T[tid >> 2][st.kq + h]) = x;
            if (X3)
                *reinterpret_cast<bf16x8 *>(&L[tid >> 2][st.kq + h]) = y;
        }
    } else {
#pragma unroll
        for (int j = 0; j < NE; ++j) {
            const __bf16 x = (__bf16)v[j];
            T[tid & 63][st.kq + 4 * j] = x;
            if (X3)
                L[tid & 63][st.kq + 4 * j] = (__bf16)(v[j] - (float)x);
        }
    }
}

// X3: both operands as BF16 pairs (hi + lo) and three products per step, hi hi + hi lo +
// lo hi, on the same matrix cores (the lo lo product is below FP32 rounding of the sum).
template <bool X3>
__global__ void __launch_bounds__(256) k_gemm_bf16(StridedGemm g, int kc, float *P)
{
    __shared__ __attribute__((aligned(16))) __bf16 As[TM][TKP];  // [row][k]
    __shared__ __attribute__((aligned(16))) __bf16 Bt[TN][TKP];  // [col][k]
    __shared__ __attribute__((aligned(16))) __bf16 Al[X3 ? TM : 1][TKP];  // remainders
    __shared__ __attribute__((aligned(16))) __bf16 Bl[X3 ? TN : 1][TKP];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int g4 = lane >> 4, n16 = lane & 15;
    const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
    const int kbeg = blockIdx.z * kc;
    const int kend = min(g.K, kbeg + kc);
    const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
    // A as rows m over k; B read as columns n over k (B(k, n) = B[k sbk + n sbn])
    const Stage sa = stage_of(g.A, g.sam, g.sak, m0, g.M, kbeg, tid);
    const Stage sb = stage_of(g.B, g.sbn, g.sbk, n0, g.N, kbeg, tid);
    f4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
            acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
    float va[NE], vb[NE];
    if (kbeg < kend) {
        sa.load(kbeg, kend, va);
        sb.load(kbeg, kend, vb);
    }
    for (int k0 = kbeg; k0 < kend; k0 += TK) {
        stage_store<X3>(As, Al, sa, tid, va);
        stage_store<X3>(Bt, Bl, sb, tid, vb);
        __syncthreads();
        if (k0 + TK < kend) {  // the next step's values, in flight during the products
            sa.load(k0 + TK, kend, va);
            sb.load(k0 + TK, kend, vb);
        }
#pragma unroll
        for (int ks = 0; ks < TK; ks += 32) {
            bf16x8 a[2], b[2];
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                a[t] = *reinterpret_cast<const bf16x8 *>(&As[wr + 16 * t + n16][ks + 8 * g4]);
                b[t] = *reinterpret_cast<const bf16x8 *>(&Bt[wc + 16 * t + n16][ks + 8 * g4]);
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] =
                        __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
            if (X3) {
                bf16x8 al[2], bl[2];
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    al[t] = *reinterpret_cast<const bf16x8 *>(&Al[wr + 16 * t + n16][ks + 8 * g4]);
                    bl[t] = *reinterpret_cast<const bf16x8 *>(&Bl[wc + 16 * t + n16][ks + 8 * g4]);
                }
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j) {
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], bl[j], acc[i][j],
                                                                            0, 0, 0);
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], b[j], acc[i][j],
                                                                            0, 0, 0);
                    }
            }
        }
        __syncthreads();
    }
    // lane 16 g4 + n16 holds rows 4 g4 .. 4 g4 + 3, column n16 of each 16 x 16 tile
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = m0 + wr + 16 * i + 4 * g4 + q, col = n0 + wc + 16 * j + n16;
                if (row >= g.M || col >= g.N)
                    continue;
                const float v = acc[i][j][q];
                if (P) {
                    P[((int64_t)blockIdx.z * g.M + row) * g.N + col] = v;
                } else {
                    float *c = g.C + (int64_t)row * g.ldc + col;
                    *c = g.accumulate ? *c + v : v;
                }
            }
}

__global__ void __launch_bounds__(256) k_splitk_sum(const float *P, int S, StridedGemm g)
{
    const int64_t n = (int64_t)g.M * g.N;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        float v = 0.f;
        for (int z = 0; z < S; ++z)
            v += P[z * n + i];
        const int64_t row = i / g.N, col = i % g.N;
        float *c = g.C + row * g.ldc + col;
        *c = g.accumulate ? *c + v : v;
    }
}

// Forward epilogue of a layer whose GEMM part is already in pre:
// pre += g[m] gw[n] + bias[n] + R[m][n]; out = relu(pre).
__global__ void __launch_bounds__(256) k_epilogue(int M, int N, float *pre, int ldp,
                                                  const float *gv, int ldg, const float *gw,
                                                  int ldgw, const float *bias, const float *R,
                                                  int ldr, float *out, int ldo)
{
    const int64_t n = (int64_t)M * N;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t m = i / N, c = i % N;
        float v = pre[m * ldp + c];
        if (gv)
            v += gv[m * ldg] * gw[c * ldgw];
        v += bias[c];
        if (R)
            v += R[m * ldr + c];
        pre[m * ldp + c] = v;
        out[m * ldo + c] = fmaxf(v, 0.f);
    }
}

int grid1(int64_t n)
{
    int64_t b = (n + 255) / 256;
    return (int)(b > 4096 ? 4096 : (b < 1 ? 1 : b));
}

}  // namespace

ds_status gemm_strided(hipStream_t s, const StridedGemm &g, float *split_ws, size_t ws_floats)
{
    if (g.M <= 0 || g.N <= 0)
        return DS_OK;
    const int64_t tiles = (int64_t)((g.N + BN - 1) / BN) * ((g.M + BM - 1) / BM);
    const int ksteps = (g.K + BK - 1) / BK;
    int S = 1;
    if (split_ws && tiles < 64)  // few output tiles: split k, at least four k steps each
        while (S < 16 && tiles * S < 256 && ksteps >= 8 * S)
            S *= 2;
    const bool split = S > 1 && (size_t)S * g.M * g.N <= ws_floats;
    const int kc = split ? ((ksteps + S - 1) / S) * BK : ksteps * BK;
    dim3 grid((g.N + BN - 1) / BN, (g.M + BM - 1) / BM, split ? S : 1);
    k_gemm_strided<<<grid, 256, 0, s>>>(g, kc, split ? split_ws : nullptr);
    if (split)
        k_splitk_sum<<<grid1((int64_t)g.M * g.N), 256, 0, s>>>(split_ws, S, g);
    DS_HIP(hipGetLastError());
    return DS_OK;
}

int splitk_count(const StridedGemm &g)
{
    const int64_t tiles = (int64_t)((g.N + TN - 1) / TN) * ((g.M + TM - 1) / TM);
    const int ksteps = (g.K + TK - 1) / TK;
    if (tiles >= 64)  // enough blocks already: no extra pass over partial sums
        return 1;
    int S = 1;
    while (S < 16 && tiles * S < 256 && ksteps >= 2 * S)
        S *= 2;
    return S;
}

ds_status gemm_bf16(hipStream_t s, const StridedGemm &g, float *split_ws, size_t ws_floats, bool x3)
{
    if (g.M <= 0 || g.N <= 0)
        return DS_OK;
    const int S = split_ws ? splitk_count(g) : 1;
    const int ksteps = (g.K + TK - 1) / TK;
    const int kc = ((ksteps + S - 1) / S) * TK;
    const bool split = S > 1 && (size_t)S * g.M * g.N <= ws_floats;
    dim3 grid((g.N + TN - 1) / TN, (g.M + TM - 1) / TM, split ? S : 1);
    if (x3)
        k_gemm_bf16<true><<<grid, 256, 0, s>>>(g, split ? kc : ksteps * TK, split ? split_ws : nullptr);
    else
        k_gemm_bf16<false><<<grid, 256, 0, s>>>(g, split ? kc : ksteps * TK, split ? split_ws : nullptr);
    if (split)
        k_splitk_sum<<<grid1((int64_t)g.M * g.N), 256, 0, s>>>(split_ws, S, g);
    DS_HIP(hipGetLastError());
    return DS_OK;
}

ds_status layer_epilogue(hipStream_t s, int M, int N, float *pre, int ldp, const float *gv, int ldg,
                         const float *gw, int ldgw, const float *bias, const float *R, int ldr,
                         float *out, int ldo)
{
    k_epilogue<<<grid1((int64_t)M * N), 256, 0, s>>>(M, N, pre, ldp, gv, ldg, gw, ldgw, bias, R, ldr,
                                                     out, ldo);
    DS_HIP(hipGetLastError());
    return DS_OK;
}

ds_status relu_mask(hipStream_t s, float *x, int ldx, const float *pre, int ldp, int R, int C)
{
    k_relu_mask<<<grid1((int64_t)R * C), 256, 0, s>>>(x, ldx, pre, ldp, R, C);
    DS_HIP(hipGetLastError());
    return DS_OK;
}

int colsum_scratch(int C) { return kColBlocks * C; }

ds_status colsum(hipStream_t s, const float *d, int ldd, int R, int C, float *db, float *scratch)
{
    if (C <= 0)
        return DS_OK;
    // at most kColBlocks row blocks of at least 64 rows each
    int rows = (R + kColBlocks - 1) / kColBlocks;
    rows = rows < 64 ? 64 : rows;
    const int RB = R > 0 ? (R + rows - 1) / rows : 0;
    if (RB == 0) {
        DS_HIP(hipMemsetAsync(db, 0, sizeof(float) * C, s));
        return DS_OK;
    }
    k_colsum_part<<<dim3((C + 63) / 64, RB), 256, 0, s>>>(d, ldd, R, C, rows, scratch);
    k_colsum_final<<<(C + 255) / 256, 256, 0, s>>>(scratch, RB, C, db);
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
                      int64_t n, float b1, float b2, float eps, int64_t *steps, float *state)
{
    k_adam_prep<<<1, 64, 0, s>>>(steps, state, b1, b2);
    k_adam<<<grid1(n), 256, 0, s>>>(theta, m, v, grad, n, b1, b2, eps, state);
    DS_HIP(hipGetLastError());
    return DS_OK;
}

__global__ void __launch_bounds__(256) k_copy(float *dst, const float *src, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

ds_status copy_f32(hipStream_t s, float *dst, const float *src, int64_t n)
{
    if (n <= 0)
        return DS_OK;
    k_copy<<<grid1(n), 256, 0, s>>>(dst, src, n);
    DS_HIP(hipGetLastError());
    return DS_OK;
}

}  // namespace ds
