// Fused prediction kernel: light-oriented stencil gather (Sec. 4.2) feeding the
// progressive residual network (Sec. 4.3, Fig. 6) on the gfx950 matrix cores.
//
// Formulation.  Every layer is computed transposed, out^T = Wmat * in^T, with the
// weights as the MFMA A operand (16 output features x 32 inputs per fragment) and
// the activations of 16 shading points as the B operand (32 inputs x 16 points).
// v_mfma_f32_16x16x32_bf16 leaves lane l = 16 g + n holding output features
// 4g..4g+3 of an M tile for point n; two such tiles give that lane exactly 8 inputs
// of point n, which is the B operand of the next layer.  So activations never
// leave registers: the residual stream o^k stays in FP32 in the accumulator
// layout, and the order in which inputs enter the 32-wide reduction is a fixed
// permutation that the host folds into the packed weight fragments.
//
// The stencil part of each block's first layer is gathered straight into B
// operands: lane (g, n) samples stencil points 32c + 8g + j (j = 0..7) of point n
// for chunk c = 0..6; chunk 7 carries sample 224, gamma and, when the number of M
// tiles is odd, the last tile of o^{k-1}.  Samples come from a corner-packed BF16
// copy of the mip level (8 corners per 16-byte cell, one load per sample) with the
// coordinates clamped to [-1, n], which reproduces zero outside the grid.
#include <string.h>

#include <vector>

#include "internal.h"
#include "frame.h"

namespace ds {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kWaves = 4;

__device__ __forceinline__ f4 mfma_bf16(const uint4 &a, const bf16x8 &b, const f4 &c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), b, c, 0, 0, 0);
}

__device__ __forceinline__ float bf_lo(uint32_t v) { return __uint_as_float(v << 16); }
__device__ __forceinline__ float bf_hi(uint32_t v) { return __uint_as_float(v & 0xffff0000u); }

// Per point and level: voxel coordinate of lattice point (0,0,0) and the
// coordinate steps along the three lattice axes.
struct PtLevel {
    float u0[3], a[3], b[3], c[3];
};

__device__ __forceinline__ float lerp(float a, float b, float t) { return fmaf(t, b - a, a); }

__device__ __forceinline__ float sample(const FusedLevel &L, const PtLevel &q, float ix, float iy,
                                        float iz)
{
    float ux = q.u0[0] + ix * q.a[0] + iy * q.b[0] + iz * q.c[0];
    float uy = q.u0[1] + ix * q.a[1] + iy * q.b[1] + iz * q.c[1];
    float uz = q.u0[2] + ix * q.a[2] + iy * q.b[2] + iz * q.c[2];
    ux = fminf(fmaxf(ux, -1.f), L.hi_x);
    uy = fminf(fmaxf(uy, -1.f), L.hi_y);
    uz = fminf(fmaxf(uz, -1.f), L.hi_z);
    float fx0 = floorf(ux), fy0 = floorf(uy), fz0 = floorf(uz);
    float fx = ux - fx0, fy = uy - fy0, fz = uz - fz0;
    int i = (int)fx0 + 1, j = (int)fy0 + 1, k = (int)fz0 + 1;
    int64_t idx = ((int64_t)k * L.cy + j) * L.cx + i;
    uint4 v = L.cells[idx];
    float x00 = lerp(bf_lo(v.x), bf_hi(v.x), fx);
    float x10 = lerp(bf_lo(v.y), bf_hi(v.y), fx);
    float x01 = lerp(bf_lo(v.z), bf_hi(v.z), fx);
    float x11 = lerp(bf_lo(v.w), bf_hi(v.w), fx);
    return lerp(lerp(x00, x10, fy), lerp(x01, x11, fy), fz);
}

__device__ __forceinline__ bf16x8 pack8(const f4 &lo, const f4 &hi)
{
    bf16x8 r;
    r[0] = (__bf16)lo[0];
    r[1] = (__bf16)lo[1];
    r[2] = (__bf16)lo[2];
    r[3] = (__bf16)lo[3];
    r[4] = (__bf16)hi[0];
    r[5] = (__bf16)hi[1];
    r[6] = (__bf16)hi[2];
    r[7] = (__bf16)hi[3];
    return r;
}

template <int MT, int NT>
__device__ __forceinline__ void dense(const uint4 *__restrict__ frags, const float *__restrict__ bias,
                                      int lane, const f4 (&in)[MT][NT], f4 (&out)[MT][NT])
{
    constexpr int C2 = (MT + 1) / 2;
    const int g = lane >> 4;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
        f4 b = *reinterpret_cast<const f4 *>(bias + 16 * mt + 4 * g);
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
            out[mt][nt] = b;
    }
#pragma unroll
    for (int q = 0; q < C2; ++q) {
        bf16x8 B[NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
            B[nt] = pack8(in[2 * q][nt], (2 * q + 1 < MT) ? in[2 * q + 1 < MT ? 2 * q + 1 : 0][nt]
                                                          : f4{0.f, 0.f, 0.f, 0.f});
        const uint4 *fr = frags + (size_t)(q * MT) * 64 + lane;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            uint4 a = fr[mt * 64];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
                out[mt][nt] = mfma_bf16(a, B[nt], out[mt][nt]);
        }
    }
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                out[mt][nt][i] = fmaxf(out[mt][nt][i], 0.f);
}

template <int MT, int NT>
__global__ void __launch_bounds__(64 * kWaves) k_fused(FusedArgs a, const FusedLevel *__restrict__ lvt,
                                                       const uint4 *__restrict__ frags,
                                                       const float *__restrict__ vec)
{
    constexpr int C1 = 8 + MT / 2;     // first-layer chunks
    constexpr int C2 = (MT + 1) / 2;   // chunks of a W-wide input
    constexpr int WP = 16 * MT;        // padded width
    __shared__ float4 tab[224];        // lattice coordinates (ix, iy, iz) of stencil point s
    for (int s = threadIdx.x; s < 224; s += blockDim.x)
        tab[s] = make_float4((float)(s % 5), (float)((s / 5) % 5), (float)(s / 25), 0.f);
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int g = lane >> 4, n = lane & 15;
    const int64_t pbase = ((int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6)) * (16 * NT);

    float x[NT][3];
    Frame fr[NT];
    bool valid[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        int64_t p = pbase + 16 * nt + n;
        valid[nt] = false;
        if (p < a.P) {
            x[nt][0] = a.pos[3 * p];
            x[nt][1] = a.pos[3 * p + 1];
            x[nt][2] = a.pos[3 * p + 2];
            valid[nt] = isfinite(x[nt][0]) && isfinite(x[nt][1]) && isfinite(x[nt][2]) &&
                        light_frame(&a.view[3 * p], &a.light[3 * p], fr[nt]);
        }
        if (!valid[nt]) {
            x[nt][0] = x[nt][1] = x[nt][2] = 0.f;
#pragma unroll
            for (int c = 0; c < 3; ++c)
                fr[nt].X[c] = fr[nt].Y[c] = fr[nt].Z[c] = 0.f;
            fr[nt].gamma = 0.f;
        }
    }

    f4 O[MT][NT], F[MT][NT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
            O[mt][nt] = f4{0.f, 0.f, 0.f, 0.f};

    for (int k = 0; k < a.K; ++k) {
        const FusedLevel L = lvt[k];
        PtLevel q[NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            float st = L.step * L.inv_h;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                float X = fr[nt].X[c], Y = fr[nt].Y[c], Z = fr[nt].Z[c];
                q[nt].u0[c] = (x[nt][c] - a.amin[c]) * L.inv_h - 0.5f - st * (X + Y + Z);
                q[nt].a[c] = 0.5f * st * X;
                q[nt].b[c] = 0.5f * st * Y;
                q[nt].c[c] = 0.5f * st * Z;
            }
            if (!valid[nt])
                q[nt].u0[0] = q[nt].u0[1] = q[nt].u0[2] = -4.f;  // clamps to the zero border
        }
        const uint4 *f1 = frags + (size_t)k * (C1 + C2) * MT * 64 + lane;
        const uint4 *f2 = f1 + (size_t)C1 * MT * 64;
        const float *b1 = vec + (size_t)k * 2 * WP;
        const float *b2 = b1 + WP;

#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
                F[mt][nt] = f4{0.f, 0.f, 0.f, 0.f};

        // stencil chunks 0..6: 32 samples per point each
#pragma unroll 1
        for (int c = 0; c < 7; ++c) {
            bf16x8 B[NT];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    float4 o = tab[32 * c + 8 * g + j];
                    B[nt][j] = (__bf16)sample(L, q[nt], o.x, o.y, o.z);
                }
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                uint4 af = f1[(c * MT + mt) * 64];
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
                    F[mt][nt] = mfma_bf16(af, B[nt], F[mt][nt]);
            }
        }
        // chunk 7: sample 224, gamma, and the odd tile of o^{k-1}
        {
            bf16x8 B[NT];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                float s224 = sample(L, q[nt], 4.f, 4.f, 8.f);
                f4 lo = f4{g == 0 ? s224 : 0.f, g == 0 ? fr[nt].gamma : 0.f, 0.f, 0.f};
                f4 hi = (MT & 1) ? O[MT - 1][nt] : f4{0.f, 0.f, 0.f, 0.f};
                B[nt] = pack8(lo, hi);
            }
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                uint4 af = f1[(7 * MT + mt) * 64];
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
                    F[mt][nt] = mfma_bf16(af, B[nt], F[mt][nt]);
            }
        }
        // o^{k-1} pairs (o^0 = 0, so block 1 skips them)
        if (k > 0) {
#pragma unroll
            for (int qq = 0; qq < MT / 2; ++qq) {
                bf16x8 B[NT];
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
                    B[nt] = pack8(O[2 * qq][nt], O[2 * qq + 1][nt]);
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) {
                    uint4 af = f1[((8 + qq) * MT + mt) * 64];
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt)
                        F[mt][nt] = mfma_bf16(af, B[nt], F[mt][nt]);
                }
            }
        }
        // F1 = relu(. + b1)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            f4 bb = *reinterpret_cast<const f4 *>(b1 + 16 * mt + 4 * g);
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    F[mt][nt][i] = fmaxf(F[mt][nt][i] + bb[i], 0.f);
        }
        // o^k = relu(W2 F1 + b2 + o^{k-1}), accumulated in place
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            f4 bb = *reinterpret_cast<const f4 *>(b2 + 16 * mt + 4 * g);
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
                O[mt][nt] += bb;
        }
#pragma unroll
        for (int qq = 0; qq < C2; ++qq) {
            bf16x8 B[NT];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
                B[nt] = pack8(F[2 * qq][nt], (2 * qq + 1 < MT) ? F[2 * qq + 1 < MT ? 2 * qq + 1 : 0][nt]
                                                                : f4{0.f, 0.f, 0.f, 0.f});
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                uint4 af = f2[(qq * MT + mt) * 64];
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
                    O[mt][nt] = mfma_bf16(af, B[nt], O[mt][nt]);
            }
        }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    O[mt][nt][i] = fmaxf(O[mt][nt][i], 0.f);
    }

    // trailing layers: H-1 dense W -> W layers, ping-ponging between O and F
    const uint4 *fh = frags + (size_t)a.K * (C1 + C2) * MT * 64;  // dense() adds the lane
    const float *bh = vec + (size_t)a.K * 2 * WP;
    int h = 0;
    for (; h + 1 < a.H - 1; h += 2) {
        dense<MT, NT>(fh + (size_t)h * C2 * MT * 64, bh + (size_t)h * WP, lane, O, F);
        dense<MT, NT>(fh + (size_t)(h + 1) * C2 * MT * 64, bh + (size_t)(h + 1) * WP, lane, F, O);
    }
    if (h < a.H - 1) {
        dense<MT, NT>(fh + (size_t)h * C2 * MT * 64, bh + (size_t)h * WP, lane, O, F);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
                O[mt][nt] = F[mt][nt];
    }
    // final scalar layer in FP32 on the vector ALUs
    const float *wl = bh + (size_t)(a.H - 1) * WP;
    const float bl = wl[WP];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        float s = 0.f;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            f4 w = *reinterpret_cast<const f4 *>(wl + 16 * mt + 4 * g);
            f4 v = O[mt][nt];
            s += w[0] * v[0] + w[1] * v[1] + w[2] * v[2] + w[3] * v[3];
        }
        s += __shfl_xor(s, 16, 64);
        s += __shfl_xor(s, 32, 64);
        int64_t p = pbase + 16 * nt + n;
        if (g == 0 && p < a.P) {
            float pre = s + bl;
            a.out[p] = valid[nt] ? fmaxf(pre, 0.f) : 0.f;
            if (a.pre)
                a.pre[p] = valid[nt] ? pre : 0.f;
            if (a.flags)
                a.flags[p] = valid[nt] ? point_flags(x[nt], fr[nt], a.amin, a.amax, a.inv_mean)
                                       : (uint8_t)DS_FLAG_INVALID;
        }
    }
}

uint16_t bf16_host(float f)
{
    uint32_t u;
    memcpy(&u, &f, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// Input index feeding slot (g, j) of chunk q of a W-wide layer: tiles 2q and 2q+1
// of the previous output, 4 features per lane group each; -1 if padding.
int pair_slot(int MT, int q, int g, int j)
{
    int t = 2 * q + (j >= 4 ? 1 : 0);
    if (t >= MT)
        return -1;
    return 16 * t + 4 * g + (j & 3);
}

template <int MT, int NT>
ds_status launch(hipStream_t s, const ds_net *net, const FusedArgs &a, const FusedLevel *lvt)
{
    int64_t per = (int64_t)kWaves * 16 * NT;
    int64_t blocks = (a.P + per - 1) / per;
    if (blocks <= 0)
        return DS_OK;
    k_fused<MT, NT><<<(unsigned)blocks, 64 * kWaves, 0, s>>>(a, lvt, net->frag_bf16, net->vec);
    DS_HIP(hipGetLastError());
    return DS_OK;
}

}  // namespace

int fused_tiles(int W)
{
    int mt = (W + 15) / 16;
    static const int inst[] = {1, 2, 4, 8, 13, 16};
    for (int v : inst)
        if (v >= mt)
            return v;
    return -1;
}

// Host packing of the BF16 weight fragments and FP32 vectors in kernel order.
ds_status fused_pack_bf16(ds_net *net, const float *theta)
{
    const int K = net->K, W = net->W, H = net->H;
    const int MT = fused_tiles(W);
    DS_CHECK(MT > 0, DS_ERR_UNSUPPORTED, "width %d is not supported by the fused kernel", W);
    const int C1 = 8 + MT / 2, C2 = (MT + 1) / 2, WP = 16 * MT;
    // parameter offsets (canonical order)
    std::vector<int64_t> oV(K), oW1(K), ob1(K), oW2(K), ob2(K), ohw(H), ohb(H);
    int64_t off = 0;
    for (int k = 0; k < K; ++k) {
        oV[k] = off;
        off += (int64_t)W * 226;
        oW1[k] = k ? off : -1;
        if (k)
            off += (int64_t)W * W;
        ob1[k] = off;
        off += W;
        oW2[k] = off;
        off += (int64_t)W * W;
        ob2[k] = off;
        off += W;
    }
    for (int m = 0; m < H; ++m) {
        int rows = m == H - 1 ? 1 : W;
        ohw[m] = off;
        off += (int64_t)rows * W;
        ohb[m] = off;
        off += rows;
    }
    const int64_t nfr = (int64_t)K * (C1 + C2) * MT + (int64_t)(H - 1) * C2 * MT;
    std::vector<uint16_t> fr((size_t)nfr * 64 * 8, 0);
    auto put = [&](int64_t frag, int mt, int g, int r, int j, float v) {
        fr[((size_t)frag * 64 + 16 * g + r) * 8 + j] = bf16_host(v);
    };
    for (int k = 0; k < K; ++k) {
        int64_t base1 = (int64_t)k * (C1 + C2) * MT, base2 = base1 + (int64_t)C1 * MT;
        for (int c = 0; c < C1; ++c)
            for (int mt = 0; mt < MT; ++mt)
                for (int g = 0; g < 4; ++g)
                    for (int r = 0; r < 16; ++r) {
                        int row = 16 * mt + r;
                        if (row >= W)
                            continue;
                        for (int j = 0; j < 8; ++j) {
                            float v = 0.f;
                            if (c < 7) {
                                v = theta[oV[k] + (int64_t)row * 226 + 32 * c + 8 * g + j];
                            } else if (c == 7) {
                                if (j < 4) {
                                    int sidx = 224 + 8 * g + j;
                                    if (sidx <= 225)
                                        v = theta[oV[k] + (int64_t)row * 226 + sidx];
                                } else if ((MT & 1) && k > 0) {
                                    int col = 16 * (MT - 1) + 4 * g + (j - 4);
                                    if (col < W)
                                        v = theta[oW1[k] + (int64_t)row * W + col];
                                }
                            } else if (k > 0) {
                                int col = pair_slot(MT, c - 8, g, j);
                                if (col >= 0 && col < W)
                                    v = theta[oW1[k] + (int64_t)row * W + col];
                            }
                            put(base1 + (int64_t)c * MT + mt, mt, g, r, j, v);
                        }
                    }
        for (int q = 0; q < C2; ++q)
            for (int mt = 0; mt < MT; ++mt)
                for (int g = 0; g < 4; ++g)
                    for (int r = 0; r < 16; ++r) {
                        int row = 16 * mt + r;
                        if (row >= W)
                            continue;
                        for (int j = 0; j < 8; ++j) {
                            int col = pair_slot(MT, q, g, j);
                            float v = (col >= 0 && col < W)
                                          ? theta[oW2[k] + (int64_t)row * W + col] : 0.f;
                            put(base2 + (int64_t)q * MT + mt, mt, g, r, j, v);
                        }
                    }
    }
    for (int h = 0; h < H - 1; ++h) {
        int64_t base = (int64_t)K * (C1 + C2) * MT + (int64_t)h * C2 * MT;
        for (int q = 0; q < C2; ++q)
            for (int mt = 0; mt < MT; ++mt)
                for (int g = 0; g < 4; ++g)
                    for (int r = 0; r < 16; ++r) {
                        int row = 16 * mt + r;
                        if (row >= W)
                            continue;
                        for (int j = 0; j < 8; ++j) {
                            int col = pair_slot(MT, q, g, j);
                            float v = (col >= 0 && col < W)
                                          ? theta[ohw[h] + (int64_t)row * W + col] : 0.f;
                            put(base + (int64_t)q * MT + mt, mt, g, r, j, v);
                        }
                    }
    }
    // vectors: per block b1, b2; per dense trailing layer its bias; final weights + bias
    const int64_t nvec = (int64_t)K * 2 * WP + (int64_t)(H - 1) * WP + WP + 4;
    std::vector<float> vec((size_t)nvec, 0.f);
    for (int k = 0; k < K; ++k)
        for (int r = 0; r < W; ++r) {
            vec[(size_t)k * 2 * WP + r] = theta[ob1[k] + r];
            vec[(size_t)k * 2 * WP + WP + r] = theta[ob2[k] + r];
        }
    for (int h = 0; h < H - 1; ++h)
        for (int r = 0; r < W; ++r)
            vec[(size_t)K * 2 * WP + (size_t)h * WP + r] = theta[ohb[h] + r];
    size_t wl = (size_t)K * 2 * WP + (size_t)(H - 1) * WP;
    for (int c = 0; c < W; ++c)
        vec[wl + c] = theta[ohw[H - 1] + c];
    vec[wl + WP] = theta[ohb[H - 1]];

    if (net->frag_bf16 && net->frag_count != nfr * 64) {
        (void)hipFree(net->frag_bf16);
        net->frag_bf16 = nullptr;
    }
    if (net->vec && net->vec_count != nvec) {
        (void)hipFree(net->vec);
        net->vec = nullptr;
    }
    if (!net->frag_bf16) {
        DS_CHECK(hipMalloc(&net->frag_bf16, (size_t)nfr * 64 * 16) == hipSuccess, DS_ERR_OOM,
                 "out of device memory for the packed weights");
        net->frag_count = nfr * 64;
    }
    if (!net->vec) {
        DS_CHECK(hipMalloc(&net->vec, (size_t)nvec * 4) == hipSuccess, DS_ERR_OOM,
                 "out of device memory for the packed biases");
        net->vec_count = nvec;
    }
    DS_HIP(hipMemcpy(net->frag_bf16, fr.data(), fr.size() * 2, hipMemcpyHostToDevice));
    DS_HIP(hipMemcpy(net->vec, vec.data(), vec.size() * 4, hipMemcpyHostToDevice));
    return DS_OK;
}

ds_status fused_predict_bf16(hipStream_t s, const ds_net *net, const FusedArgs &a,
                             const FusedLevel *lvt)
{
    switch (fused_tiles(net->W)) {
    case 1: return launch<1, 2>(s, net, a, lvt);
    case 2: return launch<2, 2>(s, net, a, lvt);
    case 4: return launch<4, 2>(s, net, a, lvt);
    case 8: return launch<8, 1>(s, net, a, lvt);
    case 13: return launch<13, 1>(s, net, a, lvt);
    case 16: return launch<16, 1>(s, net, a, lvt);
    default:
        set_error("width %d is not supported by the fused kernel", net->W);
        return DS_ERR_UNSUPPORTED;
    }
}

}  // namespace ds
