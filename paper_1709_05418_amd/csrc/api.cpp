// Host side of the C ABI: argument validation, object lifetime, device memory and
// kernel dispatch.  Every entry point returns a status and never throws.
#include <math.h>

#include <cmath>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <new>
#include <utility>
#include <algorithm>
#include <vector>

#include "internal.h"

namespace ds {

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

ds_status hip_fail(hipError_t e, const char *what)
{
    set_error("%s: %s", what, hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? DS_ERR_OOM : DS_ERR_DEVICE;
}

bool unit_host(const float *v, float *u)
{
    double a = v[0], b = v[1], c = v[2];
    if (!(std::isfinite(a) && std::isfinite(b) && std::isfinite(c)))
        return false;
    const double l = std::sqrt(a * a + b * b + c * c);
    if (!(l > 0.0))
        return false;
    u[0] = (float)(a / l);
    u[1] = (float)(b / l);
    u[2] = (float)(c / l);
    return true;
}

namespace {

int level_dim(int n, int i)
{
    int64_t s = (int64_t)1 << i;
    int64_t d = ((int64_t)n + s - 1) / s;
    return d < 1 ? 1 : (int)d;
}

struct ParamOffsets {
    std::vector<int64_t> V, W1, b1, W2, b2, hw, hb;
};

ParamOffsets param_offsets(int K, int W, int H)
{
    ParamOffsets o;
    int64_t off = 0;
    for (int k = 0; k < K; ++k) {
        o.V.push_back(off);
        off += (int64_t)W * 226;
        o.W1.push_back(k ? off : -1);
        if (k)
            off += (int64_t)W * W;
        o.b1.push_back(off);
        off += W;
        o.W2.push_back(off);
        off += (int64_t)W * W;
        o.b2.push_back(off);
        off += W;
    }
    for (int m = 0; m < H; ++m) {
        int rows = m == H - 1 ? 1 : W;
        o.hw.push_back(off);
        off += (int64_t)rows * W;
        o.hb.push_back(off);
        off += rows;
    }
    return o;
}

bool desc_ok(const ds_net_desc *d)
{
    return d && d->K >= 1 && d->K <= kMaxK && d->W >= 1 && d->W <= 256 && d->H >= 1 && d->H <= 8;
}

ds_status ensure_ws(ds_ctx *ctx, size_t bytes)
{
    if (ctx->ws_bytes >= bytes)
        return DS_OK;
    if (ctx->ws) {
        DS_HIP(hipStreamSynchronize(ctx->stream));
        (void)hipFree(ctx->ws);
        ctx->ws = nullptr;
        ctx->ws_bytes = 0;
    }
    DS_HIP(hipMalloc(&ctx->ws, bytes));
    ctx->ws_bytes = bytes;
    return DS_OK;
}

ds_status ensure_ws2(ds_ctx *ctx, size_t bytes)
{
    if (ctx->ws2_bytes >= bytes)
        return DS_OK;
    if (ctx->ws2) {
        DS_HIP(hipStreamSynchronize(ctx->stream));
        (void)hipFree(ctx->ws2);
        ctx->ws2 = nullptr;
        ctx->ws2_bytes = 0;
    }
    DS_HIP(hipMalloc(&ctx->ws2, bytes));
    ctx->ws2_bytes = bytes;
    return DS_OK;
}

// Carves aligned sub-buffers out of one workspace.
struct Carve {
    char *base;
    size_t off = 0;
    explicit Carve(void *b) : base(static_cast<char *>(b)) {}
    template <class T> T *take(size_t n)
    {
        off = (off + 255) & ~size_t(255);
        T *p = reinterpret_cast<T *>(base + off);
        off += n * sizeof(T);
        return p;
    }
};

// Philox key of the path-tracing streams derived from a caller seed, kept apart from
// the key of the record and camera streams.
uint64_t derived_key(uint64_t seed, uint64_t which)
{
    uint64_t z = seed + 0x9E3779B97F4A7C15ull * (which + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

void gather_args(const ds_cloud *c, const float *pos, const float *view, const float *light,
                 int64_t P, GatherArgs &a)
{
    a.pos = pos;
    a.view = view;
    a.light = light;
    a.P = P;
    int n[3] = {c->nx, c->ny, c->nz};
    for (int i = 0; i < 3; ++i) {
        a.amin[i] = c->aabb_min[i];
        a.amax[i] = (float)((double)c->aabb_min[i] + (double)n[i] * c->h0);
    }
    a.inv_mean = (float)(1.0 / c->mean);
    a.K = c->K;
    a.lv = static_cast<const GatherLevel *>(c->tables);
}

// Builds the corner-packed float32 levels of the cloud if they do not exist yet and points
// the gather table at them (synchronises the context stream the first time).
ds_status gather_cells(ds_ctx *ctx, const ds_cloud *c)
{
    if (c->cells32)
        return DS_OK;
    float4 *cells = nullptr;
    DS_CHECK(hipMalloc(&cells, sizeof(float4) * 2 * (size_t)c->n_cells32) == hipSuccess,
             DS_ERR_OOM, "out of device memory for the float32 corner cells (%lld cells of 32 bytes)",
             (long long)c->n_cells32);
    ds_status st = cloud_pack32(ctx->stream, c->pyr, c->L, c->lv, cells);
    std::vector<GatherLevel> gl((size_t)c->K);
    hipError_t e = st ? hipSuccess
                      : hipMemcpyAsync(gl.data(), c->tables, sizeof(GatherLevel) * c->K,
                                       hipMemcpyDeviceToHost, ctx->stream);
    if (!st && e == hipSuccess)
        e = hipStreamSynchronize(ctx->stream);
    if (!st && e == hipSuccess) {
        for (int k = 0; k < c->K; ++k)
            gl[k].cells = cells + 2 * c->lv[c->mips[k]].cell32_off;
        e = hipMemcpy(c->tables, gl.data(), sizeof(GatherLevel) * c->K, hipMemcpyHostToDevice);
    }
    if (!st && e != hipSuccess)
        st = hip_fail(e, "building the float32 corner cells");
    if (st) {
        (void)hipFree(cells);
        return st;
    }
    c->cells32 = cells;
    return DS_OK;
}

#define DS_TRY(expr)          \
    do {                      \
        ds_status s_ = (expr); \
        if (s_)               \
            return s_;        \
    } while (0)

constexpr int64_t kChunk = 65536;  // points per plain-form chunk

// All-at-once MLP over `rows` descriptor rows in FP32: per layer one GEMM and a
// bias + ReLU epilogue, ping-ponging between O and F (rows x W each); the scalar
// output layer's pre-activation goes to pre (or T).
static ds_status mlp_forward(ds_ctx *ctx, const ds_net *net, const float *z, int64_t rows,
                             float *out, float *pre, float *O, float *F, float *T)
{
    hipStream_t s = ctx->stream;
    const std::vector<int> &wd = net->mlp_widths;
    const int L = (int)wd.size() - 1, D = wd[0];
    for (int64_t r0 = 0; r0 < rows; r0 += kChunk) {
        const int M = (int)((rows - r0) < kChunk ? (rows - r0) : kChunk);
        const float *in = z + r0 * D;
        int ld = D;
        const float *th = net->theta;
        for (int l = 0; l < L; ++l) {
            const int ni = wd[l], no = wd[l + 1];
            const float *Wl = th, *bl = th + (int64_t)no * ni;
            th = bl + no;
            const bool last = l == L - 1;
            float *C = last ? (pre ? pre + r0 : T) : (l & 1 ? F : O);
            DS_TRY(gemm_strided(s, {M, no, ni, in, ld, 1, Wl, 1, ni, C, no, 0}));
            DS_TRY(layer_epilogue(s, M, no, C, no, nullptr, 0, nullptr, 0, bl, nullptr, 0,
                                  last ? out + r0 : C, no));
            in = C;
            ld = no;
        }
    }
    return DS_OK;
}

// Plain FP32 network over `rows` descriptor rows (ldz = 225K + 1).
// amax (may be NULL): running maxima of |activation| per layer, as float bits: the first
// layer of every block (K), the residual stream over all blocks (1), the dense trailing
// layers (H - 1).
ds_status forward_plain(ds_ctx *ctx, const ds_net *net, const float *z, int64_t rows, float *out,
                        float *pre, float *O, float *F, float *T, unsigned *amax = nullptr)
{
    if (net->kind == 1)
        return mlp_forward(ctx, net, z, rows, out, pre, O, F, T);
    const int K = net->K, W = net->W, H = net->H;
    const int D = kStencil * K + 1;
    const float *th = net->theta;
    ParamOffsets po = param_offsets(K, W, H);
    for (int64_t r0 = 0; r0 < rows; r0 += kChunk) {
        int M = (int)((rows - r0) < kChunk ? (rows - r0) : kChunk);
        const float *zc = z + r0 * D;
        for (int k = 0; k < K; ++k) {
            GemmArgs g1 = {};
            g1.M = M;
            g1.N = W;
            g1.A1 = zc + (int64_t)k * kStencil;
            g1.lda1 = D;
            g1.K1 = kStencil;
            g1.B1 = th + po.V[k];
            g1.ldb1 = 226;
            if (k > 0) {
                g1.A2 = O;
                g1.lda2 = W;
                g1.K2 = W;
                g1.B2 = th + po.W1[k];
                g1.ldb2 = W;
            }
            g1.g = zc + (int64_t)kStencil * K;
            g1.ldg = D;
            g1.gw = th + po.V[k] + 225;
            g1.ldgw = 226;
            g1.bias = th + po.b1[k];
            g1.C = F;
            g1.ldc = W;
            g1.relu = 1;
            ds_status st = gemm_f32(ctx->stream, g1);
            if (!st && amax)
                st = amax_into(ctx->stream, F, (int64_t)M * W, amax + k);
            if (st)
                return st;
            GemmArgs g2 = {};
            g2.M = M;
            g2.N = W;
            g2.A1 = F;
            g2.lda1 = W;
            g2.K1 = W;
            g2.B1 = th + po.W2[k];
            g2.ldb1 = W;
            g2.bias = th + po.b2[k];
            if (k > 0) {
                g2.R = O;
                g2.ldr = W;
            }
            g2.C = O;
            g2.ldc = W;
            g2.relu = 1;
            st = gemm_f32(ctx->stream, g2);
            if (!st && amax)
                st = amax_into(ctx->stream, O, (int64_t)M * W, amax + K);
            if (st)
                return st;
        }
        const float *in = O;
        float *bufs[2] = {T, F};
        for (int m = 0; m < H; ++m) {
            bool last = m == H - 1;
            GemmArgs g = {};
            g.M = M;
            g.N = last ? 1 : W;
            g.A1 = in;
            g.lda1 = W;
            g.K1 = W;
            g.B1 = th + po.hw[m];
            g.ldb1 = W;
            g.bias = th + po.hb[m];
            g.C = last ? out + r0 : bufs[m & 1];
            g.ldc = last ? 1 : W;
            if (last && pre) {
                g.pre = pre + r0;
                g.ldpre = 1;
            }
            g.relu = 1;
            ds_status st = gemm_f32(ctx->stream, g);
            if (!st && amax && !last)
                st = amax_into(ctx->stream, bufs[m & 1], (int64_t)M * W, amax + K + 1 + m);
            if (st)
                return st;
            in = bufs[m & 1];
        }
    }
    return DS_OK;
}

// Workspace of one minibatch: per block the first-layer pre-activations H, their
// ReLU F1, the second-layer pre-activations A and the block outputs O; per
// trailing layer its pre-activations and outputs; gradient scratch.
struct TrainWs {
    float *H, *F1, *A, *O, *HA, *HO, *dcur, *dnext, *dh, *dpre, *sq;
    float *split;          // split-K partial products (BF16 training)
    size_t split_floats;
};

// Training workspace of a minibatch of B samples, in floats (both network kinds).
size_t train_ws_floats(const ds_net *net, int B)
{
    if (net->kind == 1) {
        const std::vector<int> &wd = net->mlp_widths;
        size_t act = 0;
        for (size_t l = 1; l < wd.size(); ++l)
            act += (size_t)B * wd[l];
        size_t split = (size_t)16 * net->W * 226;
        const size_t csum = (size_t)colsum_scratch(net->W);
        split = split > csum ? split : csum;
        return 2 * act + 2 * (size_t)B * net->W + 2 * (size_t)B + split;
    }
    const size_t BW = (size_t)B * net->W, K = net->K, Hh = net->H;
    const size_t split = (size_t)16 * net->W * 226;
    return 4 * K * BW + 2 * Hh * BW + 3 * BW + 2 * (size_t)B + split;
}

ds_status train_ws(ds_net *net, int B, TrainWs &w)
{
    const size_t BW = (size_t)B * net->W, K = net->K, Hh = net->H;
    const size_t split = (size_t)16 * net->W * 226;
    const size_t need = train_ws_floats(net, B);
    if (net->tws_floats < need) {
        if (net->tws) {
            DS_HIP(hipStreamSynchronize(net->ctx->stream));
            (void)hipFree(net->tws);
            net->tws = nullptr;
            net->tws_floats = 0;
        }
        DS_HIP(hipMalloc(&net->tws, need * sizeof(float)));
        net->tws_floats = need;
    }
    float *p = net->tws;
    w.H = p;
    p += K * BW;
    w.F1 = p;
    p += K * BW;
    w.A = p;
    p += K * BW;
    w.O = p;
    p += K * BW;
    w.HA = p;
    p += Hh * BW;
    w.HO = p;
    p += Hh * BW;
    w.dcur = p;
    p += BW;
    w.dnext = p;
    p += BW;
    w.dh = p;
    p += BW;
    w.dpre = p;
    p += B;
    w.sq = p;
    p += B;
    w.split = p;
    w.split_floats = split;
    return DS_OK;
}

// Loss and gradient of the all-at-once MLP: per layer its pre-activations and outputs
// are kept, then backpropagation last layer first (FP32, or BF16 GEMM operands with FP32
// accumulation as for the RPNN).
static ds_status mlp_loss_grad(ds_net *net, const float *z, const float *target, int B,
                               float *loss, float *grad)
{
    hipStream_t s = net->ctx->stream;
    const bool bf = net->train_prec == DS_PREC_BF16;
    const std::vector<int> &wd = net->mlp_widths;
    const int L = (int)wd.size() - 1, D = wd[0], Wm = net->W;
    size_t split = (size_t)16 * Wm * 226;
    const size_t csum = (size_t)colsum_scratch(Wm);
    split = split > csum ? split : csum;
    const size_t need = train_ws_floats(net, B);
    if (net->tws_floats < need) {
        if (net->tws) {
            DS_HIP(hipStreamSynchronize(s));
            (void)hipFree(net->tws);
            net->tws = nullptr;
            net->tws_floats = 0;
        }
        DS_HIP(hipMalloc(&net->tws, need * sizeof(float)));
        net->tws_floats = need;
    }
    std::vector<float *> A(L), Y(L);
    std::vector<int64_t> ow(L), ob(L);
    float *p = net->tws;
    int64_t at = 0;
    for (int l = 0; l < L; ++l) {
        A[l] = p;
        p += (size_t)B * wd[l + 1];
        Y[l] = p;
        p += (size_t)B * wd[l + 1];
        ow[l] = at;
        at += (int64_t)wd[l + 1] * wd[l];
        ob[l] = at;
        at += wd[l + 1];
    }
    const size_t wide = (size_t)B * Wm;  // d loss / d (hidden layer), at most W wide
    float *dcur = p, *dnext = p + wide;
    p += 2 * wide;
    float *dpre = p, *sq = p + B;
    p += 2 * (size_t)B;
    float *sp = p;
    auto mm = [&](const StridedGemm &g) {
        return bf ? gemm_bf16(s, g, sp, split) : gemm_strided(s, g, sp, split);
    };
    const float *th = net->theta;
    // forward
    const float *in = z;
    int ld = D;
    for (int l = 0; l < L; ++l) {
        const int ni = wd[l], no = wd[l + 1];
        // hidden-layer products with BF16 operand pairs, as the RPNN's W x W layers
        const StridedGemm gl = {B, no, ni, in, ld, 1, th + ow[l], 1, ni, A[l], no, 0};
        DS_TRY(bf && l > 0 ? gemm_bf16(s, gl, sp, split, true) : mm(gl));
        DS_TRY(layer_epilogue(s, B, no, A[l], no, nullptr, 0, nullptr, 0, th + ob[l], nullptr, 0,
                              Y[l], no));
        in = Y[l];
        ld = no;
    }
    DS_TRY(loss_head(s, A[L - 1], target, B, dpre, sq, loss));
    if (!grad)
        return DS_OK;
    // backward; dY = d loss / d (pre-activation of layer l)
    const float *dY = dpre;
    int ldy = 1;
    for (int l = L - 1; l >= 0; --l) {
        const int ni = wd[l], no = wd[l + 1];
        if (l < L - 1) {
            DS_TRY(relu_mask(s, dcur, no, A[l], no, B, no));
            dY = dcur;
            ldy = no;
        }
        const float *x = l == 0 ? z : Y[l - 1];
        const int ldx = l == 0 ? D : ni;
        DS_TRY(mm({no, ni, B, dY, 1, ldy, x, ldx, 1, grad + ow[l], ni, 0}));
        DS_TRY(colsum(s, dY, ldy, B, no, grad + ob[l], sp));
        if (l > 0) {
            DS_TRY(mm({B, ni, no, dY, ldy, 1, th + ow[l], ni, 1, dnext, ni, 0}));
            std::swap(dcur, dnext);
        }
    }
    return DS_OK;
}

// Loss and gradient of a minibatch: forward keeping pre-activations, then
// backpropagation layer by layer; every parameter gradient is written exactly once.
// FP32 arithmetic, or (train_prec BF16) every GEMM on the BF16 matrix cores with FP32
// accumulation (operands rounded once, or as hi + lo pairs for the forward W x W products);
// epilogues, reductions and the loss stay FP32.
ds_status loss_grad(ds_net *net, const float *z, const float *target, int B, float *loss,
                    float *grad)
{
    if (net->kind == 1)
        return mlp_loss_grad(net, z, target, B, loss, grad);
    hipStream_t s = net->ctx->stream;
    const bool bf = net->train_prec == DS_PREC_BF16;
    const int K = net->K, W = net->W, Hn = net->H, D = kStencil * K + 1;
    const float *th = net->theta;
    ParamOffsets po = param_offsets(K, W, Hn);
    TrainWs w;
    DS_TRY(train_ws(net, B, w));
    auto mm = [&](const StridedGemm &g) {
        return bf ? gemm_bf16(s, g, w.split, w.split_floats)
                  : gemm_strided(s, g, w.split, w.split_floats);
    };
    // forward products of the W x W layers (W1, W2, trailing): in BF16 their operands as
    // hi + lo pairs.  A single BF16 rounding of these operands, carried through the residual
    // stream of all blocks, moves the loss and thus every gradient; the descriptor layers
    // and the backward products keep one BF16 term
    auto mmw = [&](const StridedGemm &g) {
        return bf ? gemm_bf16(s, g, w.split, w.split_floats, true)
                  : gemm_strided(s, g, w.split, w.split_floats);
    };
    const size_t BW = (size_t)B * W;
    auto H = [&](int k) { return w.H + k * BW; };
    auto F1 = [&](int k) { return w.F1 + k * BW; };
    auto A = [&](int k) { return w.A + k * BW; };
    auto O = [&](int k) { return w.O + k * BW; };  // output of block k
    auto HA = [&](int m) { return w.HA + m * BW; };
    auto HO = [&](int m) { return w.HO + m * BW; };
    // ---- forward
    for (int k = 0; k < K; ++k) {
        GemmArgs g1 = {};
        g1.M = B;
        g1.N = W;
        g1.A1 = z + (int64_t)k * kStencil;
        g1.lda1 = D;
        g1.K1 = kStencil;
        g1.B1 = th + po.V[k];
        g1.ldb1 = 226;
        if (k > 0) {
            g1.A2 = O(k - 1);
            g1.lda2 = W;
            g1.K2 = W;
            g1.B2 = th + po.W1[k];
            g1.ldb2 = W;
        }
        g1.g = z + (int64_t)kStencil * K;
        g1.ldg = D;
        g1.gw = th + po.V[k] + 225;
        g1.ldgw = 226;
        g1.bias = th + po.b1[k];
        g1.C = F1(k);
        g1.ldc = W;
        g1.pre = H(k);
        g1.ldpre = W;
        g1.relu = 1;
        if (bf) {
            DS_TRY(mm({B, W, kStencil, z + (int64_t)k * kStencil, D, 1, th + po.V[k], 1, 226, H(k), W,
                       0}));
            if (k > 0)
                DS_TRY(mmw({B, W, W, O(k - 1), W, 1, th + po.W1[k], 1, W, H(k), W, 1}));
            DS_TRY(layer_epilogue(s, B, W, H(k), W, z + (int64_t)kStencil * K, D,
                                  th + po.V[k] + 225, 226, th + po.b1[k], nullptr, 0, F1(k), W));
        } else {
            DS_TRY(gemm_f32(s, g1));
        }
        GemmArgs g2 = {};
        g2.M = B;
        g2.N = W;
        g2.A1 = F1(k);
        g2.lda1 = W;
        g2.K1 = W;
        g2.B1 = th + po.W2[k];
        g2.ldb1 = W;
        g2.bias = th + po.b2[k];
        if (k > 0) {
            g2.R = O(k - 1);
            g2.ldr = W;
        }
        g2.C = O(k);
        g2.ldc = W;
        g2.pre = A(k);
        g2.ldpre = W;
        g2.relu = 1;
        if (bf) {
            DS_TRY(mmw({B, W, W, F1(k), W, 1, th + po.W2[k], 1, W, A(k), W, 0}));
            DS_TRY(layer_epilogue(s, B, W, A(k), W, nullptr, 0, nullptr, 0, th + po.b2[k],
                                  k > 0 ? O(k - 1) : nullptr, W, O(k), W));
        } else {
            DS_TRY(gemm_f32(s, g2));
        }
    }
    for (int m = 0; m < Hn; ++m) {
        const bool last = m == Hn - 1;
        GemmArgs g = {};
        g.M = B;
        g.N = last ? 1 : W;
        g.A1 = m == 0 ? O(K - 1) : HO(m - 1);
        g.lda1 = W;
        g.K1 = W;
        g.B1 = th + po.hw[m];
        g.ldb1 = W;
        g.bias = th + po.hb[m];
        g.C = HO(m);
        g.ldc = last ? 1 : W;
        g.pre = HA(m);
        g.ldpre = last ? 1 : W;
        g.relu = 1;
        if (bf) {
            const int N = last ? 1 : W;
            DS_TRY(mmw({B, N, W, g.A1, W, 1, th + po.hw[m], 1, W, HA(m), N, 0}));
            DS_TRY(layer_epilogue(s, B, N, HA(m), N, nullptr, 0, nullptr, 0, th + po.hb[m], nullptr,
                                  0, HO(m), N));
        } else {
            DS_TRY(gemm_f32(s, g));
        }
    }
    // ---- loss and d loss / d (final pre-activation)
    DS_TRY(loss_head(s, HA(Hn - 1), target, B, w.dpre, w.sq, loss));
    if (!grad)
        return DS_OK;
    // ---- trailing layers, last first; dcur = d loss / d (layer pre-activation)
    const float *dY = w.dpre;
    int ldy = 1;
    for (int m = Hn - 1; m >= 0; --m) {
        const int rows = m == Hn - 1 ? 1 : W;
        const float *in = m == 0 ? O(K - 1) : HO(m - 1);
        if (m < Hn - 1) {
            DS_TRY(relu_mask(s, w.dcur, W, HA(m), W, B, W));
            dY = w.dcur;
            ldy = W;
        }
        // dW = dY^T in, db = column sums of dY
        DS_TRY(mm({rows, W, B, dY, 1, ldy, in, W, 1, grad + po.hw[m], W, 0}));
        DS_TRY(colsum(s, dY, ldy, B, rows, grad + po.hb[m], w.split));
        // d in = dY W
        DS_TRY(mm({B, W, rows, dY, ldy, 1, th + po.hw[m], W, 1, w.dnext, W, 0}));
        std::swap(w.dcur, w.dnext);
    }
    // ---- blocks, last first; dcur = d loss / d o^k
    for (int k = K - 1; k >= 0; --k) {
        float *da = w.dcur;
        DS_TRY(relu_mask(s, da, W, A(k), W, B, W));
        DS_TRY(mm({W, W, B, da, 1, W, F1(k), W, 1, grad + po.W2[k], W, 0}));
        DS_TRY(colsum(s, da, W, B, W, grad + po.b2[k], w.split));
        // dh = (da W2) masked by h > 0
        DS_TRY(mm({B, W, W, da, W, 1, th + po.W2[k], W, 1, w.dh, W, 0}));
        DS_TRY(relu_mask(s, w.dh, W, H(k), W, B, W));
        // dV over the 225 stencil columns and the gamma column
        DS_TRY(mm({W, kStencil, B, w.dh, 1, W, z + (int64_t)k * kStencil, D, 1,
                                grad + po.V[k], 226, 0}));
        DS_TRY(mm({W, 1, B, w.dh, 1, W, z + (int64_t)kStencil * K, D, 1,
                                grad + po.V[k] + 225, 226, 0}));
        DS_TRY(colsum(s, w.dh, W, B, W, grad + po.b1[k], w.split));
        if (k > 0) {
            DS_TRY(mm({W, W, B, w.dh, 1, W, O(k - 1), W, 1, grad + po.W1[k], W, 0}));
            // d o^{k-1} = da + dh W1
            DS_TRY(copy_f32(s, w.dnext, da, (int64_t)BW));
            DS_TRY(mm({B, W, W, w.dh, W, 1, th + po.W1[k], W, 1, w.dnext, W, 1}));
            std::swap(w.dcur, w.dnext);
        }
    }
    return DS_OK;
}

}  // namespace
}  // namespace ds

using namespace ds;

// ---------------------------------------------------------------- allocation-free plain form
// Scratch of ds_predict_f32_noalloc: the descriptor rows, activations and flags of one
// chunk of points.  Every GPU the library runs on holds its own copy of this array from
// module load until the process ends.  In host code its name is only a stand-in: kernels
// get the device address that hipGetSymbolAddress gives for the current device, taken
// once per device at ds_create and kept in g_scratch.
static constexpr size_t kScratchBytes = (size_t)32 << 20;
static constexpr int kScratchDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
static void *g_scratch[kScratchDevices];
static std::mutex g_scratch_mutex;

// With `device` current: its address of `scratch`, once.
static ds_status scratch_setup(int device)
{
    DS_CHECK(device >= 0 && device < kScratchDevices, DS_ERR_UNSUPPORTED,
             "device %d: the scratch table covers devices 0..%d", device, kScratchDevices - 1);
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (g_scratch[device])
        return DS_OK;
    void *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess)
        return hip_fail(e, "scratch address");
    DS_CHECK(ptr, DS_ERR_DEVICE, "scratch address: NULL");
    g_scratch[device] = ptr;
    return DS_OK;
}

// A distant emitter as m directional lights (Sec. 4.4): per light the unit direction and
// the weight E_j / p_j (device float4), and the selection thresholds (device).
// A tabulated phase function on the device (FP32 copies of the host FP64 table).
struct ds_phase {
    ds_ctx *ctx = nullptr;
    int n = 0;
    float *p = nullptr, *cdf = nullptr;
    double removed = 0.0, mean_cos = 0.0;
};

constexpr int kMaxLights = 65536;  // members of a light set
constexpr int kMaxDraws = 256;     // lights drawn per camera sample

struct ds_lights {
    ds_ctx *ctx = nullptr;
    int m = 0;
    float4 *dw = nullptr;
    uint32_t *thr = nullptr;
};

namespace {

// Selection table of a light set: thr[j] = the running FP64 sum of E to j over the
// total, times 2^24, rounded half up, kept one above thr[j-1] and low enough to leave
// one step per later light (so thr[m-1] = 2^24 and each p_j > 0); w[j] = E_j / p_j with
// p_j = (thr[j] - thr[j-1]) / 2^24.
void light_table(const double *E, int m, uint32_t *thr, double *w)
{
    double total = 0.0;
    for (int j = 0; j < m; ++j)
        total += E[j];
    double run = 0.0;
    int64_t prev = 0;
    for (int j = 0; j < m; ++j) {
        run += E[j];
        int64_t t = (int64_t)std::floor(run / total * 16777216.0 + 0.5);
        t = t < prev + 1 ? prev + 1 : t;
        const int64_t cap = ((int64_t)1 << 24) - (m - 1 - j);
        t = t > cap ? cap : t;
        thr[j] = (uint32_t)t;
        w[j] = E[j] / ((double)(t - prev) / 16777216.0);
        prev = t;
    }
}

}  // namespace

extern "C" {

const char *ds_last_error(void) { return g_err; }

const char *ds_version(void) { return "deepscatter-mi355x 0.1 (gfx950)"; }

ds_status ds_create(int device, void *hip_stream, ds_ctx **out)
{
    DS_CHECK(out, DS_ERR_INVALID_ARG, "ds_create: out is NULL");
    int n = 0;
    DS_HIP(hipGetDeviceCount(&n));
    DS_CHECK(device >= 0 && device < n, DS_ERR_INVALID_ARG, "ds_create: device %d of %d", device,
             n);
    DS_HIP(hipSetDevice(device));
    ds_status st = scratch_setup(device);
    if (st)
        return st;
    ds_ctx *c = new (std::nothrow) ds_ctx();
    DS_CHECK(c, DS_ERR_OOM, "ds_create: out of host memory");
    c->device = device;
    c->stream = static_cast<hipStream_t>(hip_stream);
    if (hipMalloc(&c->truncated, sizeof(unsigned long long)) != hipSuccess ||
        hipMemset(c->truncated, 0, sizeof(unsigned long long)) != hipSuccess) {
        (void)hipFree(c->truncated);
        delete c;
        set_error("ds_create: out of device memory for the tracer counter");
        return DS_ERR_OOM;
    }
    *out = c;
    return DS_OK;
}

ds_status ds_tracer_truncated(ds_ctx *ctx, int64_t *count, int reset)
{
    DS_CHECK(ctx && count, DS_ERR_INVALID_ARG, "ds_tracer_truncated: NULL argument");
    unsigned long long h = 0;
    DS_HIP(hipMemcpyAsync(&h, ctx->truncated, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
    DS_HIP(hipStreamSynchronize(ctx->stream));
    *count = (int64_t)h;
    if (reset) {
        DS_HIP(hipMemsetAsync(ctx->truncated, 0, sizeof(h), ctx->stream));
        DS_HIP(hipStreamSynchronize(ctx->stream));
    }
    return DS_OK;
}

ds_status ds_set_stream(ds_ctx *ctx, void *hip_stream)
{
    DS_CHECK(ctx, DS_ERR_INVALID_ARG, "ds_set_stream: ctx is NULL");
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    return DS_OK;
}

ds_status ds_synchronize(ds_ctx *ctx)
{
    DS_CHECK(ctx, DS_ERR_INVALID_ARG, "ds_synchronize: ctx is NULL");
    DS_HIP(hipStreamSynchronize(ctx->stream));
    return DS_OK;
}

ds_status ds_destroy(ds_ctx *ctx)
{
    if (!ctx)
        return DS_OK;
    if (ctx->ws || ctx->ws2)
        (void)hipStreamSynchronize(ctx->stream);
    (void)hipFree(ctx->ws);
    (void)hipFree(ctx->ws2);
    (void)hipFree(ctx->truncated);
    delete ctx;
    return DS_OK;
}

// ---------------------------------------------------------------- cloud
ds_status ds_cloud_create(ds_ctx *ctx, const void *density_dev, ds_dtype dtype, int nx, int ny,
                          int nz, float sigma_max, const float aabb_min[3], float voxel_size,
                          int n_levels, const int *mip_of_level, int K, ds_cloud **out)
{
    DS_CHECK(ctx && density_dev && aabb_min && out, DS_ERR_INVALID_ARG,
             "ds_cloud_create: NULL argument");
    DS_CHECK(dtype == DS_F32 || dtype == DS_BF16, DS_ERR_INVALID_ARG,
             "ds_cloud_create: dtype must be DS_F32 or DS_BF16");
    DS_CHECK(nx > 0 && ny > 0 && nz > 0 && nx <= 4096 && ny <= 4096 && nz <= 4096,
             DS_ERR_INVALID_ARG, "ds_cloud_create: bad grid size %d x %d x %d", nx, ny, nz);
    DS_CHECK(sigma_max > 0.f && isfinite(sigma_max) && voxel_size > 0.f && isfinite(voxel_size),
             DS_ERR_INVALID_ARG, "ds_cloud_create: sigma_max and voxel_size must be positive");
    DS_CHECK(isfinite(aabb_min[0]) && isfinite(aabb_min[1]) && isfinite(aabb_min[2]),
             DS_ERR_INVALID_ARG, "ds_cloud_create: aabb_min must be finite");
    DS_CHECK(n_levels >= 1 && n_levels <= kMaxLevels, DS_ERR_INVALID_ARG,
             "ds_cloud_create: n_levels %d outside 1..%d", n_levels, kMaxLevels);
    DS_CHECK(K >= 1 && K <= kMaxK, DS_ERR_INVALID_ARG, "ds_cloud_create: K %d outside 1..%d", K,
             kMaxK);
    if (mip_of_level)
        for (int k = 0; k < K; ++k)
            DS_CHECK(mip_of_level[k] >= 0 && mip_of_level[k] < n_levels, DS_ERR_INVALID_ARG,
                     "ds_cloud_create: mip_of_level[%d] = %d outside [0, %d)", k, mip_of_level[k],
                     n_levels);
    DS_HIP(hipSetDevice(ctx->device));
    const int64_t nvox = (int64_t)nx * ny * nz;
    double sum = 0.0;
    int64_t count = 0;
    ds_status st = cloud_mean(ctx->stream, density_dev, dtype, nvox, &sum, &count);
    if (st)
        return st;
    DS_CHECK(count > 0 && sum > 0.0, DS_ERR_INVALID_ARG,
             "ds_cloud_create: the density grid has no positive voxel");

    ds_cloud *c = new (std::nothrow) ds_cloud();
    DS_CHECK(c, DS_ERR_OOM, "ds_cloud_create: out of host memory");
    c->ctx = ctx;
    c->nx = nx;
    c->ny = ny;
    c->nz = nz;
    c->sigma_max = sigma_max;
    memcpy(c->aabb_min, aabb_min, sizeof(float) * 3);
    c->h0 = voxel_size;
    c->mean = (double)sigma_max * sum / (double)count;
    c->L = n_levels;
    c->K = K;
    int64_t off = 0, coff32 = 0;
    for (int i = 0; i < n_levels; ++i) {
        Level &l = c->lv[i];
        l.nx = level_dim(nx, i);
        l.ny = level_dim(ny, i);
        l.nz = level_dim(nz, i);
        l.off = off;
        l.cell32_off = coff32;
        l.h = (float)ldexp((double)voxel_size, i);
        off += (int64_t)l.nx * l.ny * l.nz;
        coff32 += (int64_t)(l.nx + 2) * (l.ny + 2) * (l.nz + 2);
    }
    c->pyr_elems = off;
    c->n_cells32 = coff32;
    if (mip_of_level) {
        memcpy(c->mips, mip_of_level, sizeof(int) * K);
    } else {
        // the level whose voxel best matches the level-1 spacing of half a mean free path
        int delta = (int)floor(log2(0.5 / (c->mean * (double)voxel_size)) + 0.5);
        for (int k = 0; k < K; ++k) {
            int m = k + delta;
            c->mips[k] = m < 0 ? 0 : (m > n_levels - 1 ? n_levels - 1 : m);
        }
    }
    // Zero borders of the FP16 cells.  A stencil sample lies at most sqrt(1 + 1 + 9) mean
    // free paths times 2^(k-1) from its point along any axis (offsets within [-1, 1]^2 x
    // [-1, 3], scaled by 2^(k-1) on the orthonormal light frame), so a point inside the grid
    // box reads cells within E = 3.3167 * step / h voxels of the grid: a border of
    // ceil(E + 1/2) + 1 cells holds all of them and the kernel can skip the per-sample
    // clamp.  Levels whose border would grow the cells too much keep a border of one and
    // the clamp.
    int64_t coff = 0;
    for (int i = 0; i < n_levels; ++i) {
        Level &l = c->lv[i];
        double ext = 0.0;
        for (int k = 0; k < K; ++k)
            if (c->mips[k] == i)
                ext = std::max(ext, 3.3166248 * ldexp(1.0, k) / c->mean / (double)l.h);
        int bd = 1;
        l.fast = true;
        if (ext > 0.0) {
            const double want = ceil(ext + 0.5) + 1.0;
            const double base = (double)(l.nx + 2) * (l.ny + 2) * (l.nz + 2);
            const double grown = (l.nx + 2 * want) * (l.ny + 2 * want) * (l.nz + 2 * want);
            if (want <= 256.0 && (grown <= 1.5 * base || grown <= (double)(1 << 21)))
                bd = (int)want;
            else
                l.fast = false;
        }
        l.bd = bd;
        l.cell_off = coff;
        coff += (int64_t)(l.nx + 2 * bd) * (l.ny + 2 * bd) * (l.nz + 2 * bd);
    }
    c->n_cells = coff;
    auto fail = [&](ds_status s) {
        ds_cloud_destroy(c);
        return s;
    };
    if (hipMalloc(&c->pyr, sizeof(float) * c->pyr_elems) != hipSuccess) {
        set_error("ds_cloud_create: out of device memory for the float32 pyramid (%lld floats)",
                  (long long)c->pyr_elems);
        return fail(DS_ERR_OOM);
    }
    if (hipMalloc(&c->cells, sizeof(uint4) * c->n_cells) != hipSuccess) {
        set_error("ds_cloud_create: out of device memory for the packed pyramid (%lld cells)",
                  (long long)c->n_cells);
        return fail(DS_ERR_OOM);
    }
    float scale = (float)((double)sigma_max / c->mean);
    st = cloud_pyramid(ctx->stream, density_dev, dtype, nx, ny, nz, scale, n_levels, c->lv, c->pyr);
    if (st)
        return fail(st);
    st = cloud_pack(ctx->stream, c->pyr, n_levels, c->lv, c->cells);
    if (st)
        return fail(st);
    st = tracer_prepare(c, density_dev, dtype);
    if (st)
        return fail(st);
    // device-side per-stencil-level tables
    std::vector<GatherLevel> gl(K);
    std::vector<FusedLevel> fl(K);
    for (int k = 0; k < K; ++k) {
        const Level &l = c->lv[c->mips[k]];
        double h = ldexp((double)voxel_size, c->mips[k]);
        double step = ldexp(1.0, k) / c->mean;
        gl[k].cells = nullptr;  // set by gather_cells on the first plain-form call
        gl[k].cx = l.nx + 2;
        gl[k].cy = l.ny + 2;
        gl[k].hx = (float)(l.nx + 1);  // cell coordinates are shifted by one
        gl[k].hy = (float)(l.ny + 1);
        gl[k].hz = (float)(l.nz + 1);
        gl[k].inv_h = (float)(1.0 / h);
        gl[k].step = (float)step;
        fl[k].cells = c->cells + l.cell_off;
        fl[k].cx = l.nx + 2 * l.bd;
        fl[k].cy = l.ny + 2 * l.bd;
        fl[k].hi_x = (float)(l.nx + 2 * l.bd - 1);  // cell coordinates are shifted by bd
        fl[k].hi_y = (float)(l.ny + 2 * l.bd - 1);
        fl[k].hi_z = (float)(l.nz + 2 * l.bd - 1);
        fl[k].inv_h = (float)(1.0 / h);
        fl[k].step = (float)step;
        fl[k].shift = (float)l.bd - 0.5f;
        fl[k].fast = l.fast ? 1 : 0;
    }
    size_t tb = sizeof(GatherLevel) * K + sizeof(FusedLevel) * K + 64;
    if (hipMalloc(&c->tables, tb) != hipSuccess) {
        set_error("ds_cloud_create: out of device memory for the level tables");
        return fail(DS_ERR_OOM);
    }
    std::vector<char> host(tb, 0);
    memcpy(host.data(), gl.data(), sizeof(GatherLevel) * K);
    size_t foff = (sizeof(GatherLevel) * K + 63) / 64 * 64;
    memcpy(host.data() + foff, fl.data(), sizeof(FusedLevel) * K);
    hipError_t e = hipMemcpy(c->tables, host.data(), tb, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess)
        return fail(hip_fail(e, "ds_cloud_create"));
    *out = c;
    return DS_OK;
}

static const FusedLevel *fused_table(const ds_cloud *c)
{
    size_t foff = (sizeof(GatherLevel) * c->K + 63) / 64 * 64;
    return reinterpret_cast<const FusedLevel *>(static_cast<const char *>(c->tables) + foff);
}

static const FusedVariant kDefaultVariant = {DS_KERNEL_REGISTER, 4, 0};

static void fused_args(const float *pos, const float *view, const float *light, float *out,
                       float *pre, uint8_t *flags, int K, int W, int H, FusedArgs &a)
{
    a.pos = pos;
    a.view = view;
    a.light = light;
    a.out = out;
    a.pre = pre;
    a.flags = flags;
    a.perm = nullptr;
    a.K = K;
    a.W = W;
    a.H = H;
    a.n_clouds = 0;
    a.n_tiles = 0;
}

// Appends a cloud whose points are rows [p_begin, p_begin + P) of the point arrays.
static void add_cloud(FusedArgs &a, const ds_cloud *c, int64_t p_begin, int64_t P)
{
    FusedCloud &f = a.cl[a.n_clouds++];
    GatherArgs ga;
    gather_args(c, nullptr, nullptr, nullptr, 0, ga);
    f.lvt = fused_table(c);
    memcpy(f.amin, ga.amin, sizeof(f.amin));
    memcpy(f.amax, ga.amax, sizeof(f.amax));
    f.inv_mean = ga.inv_mean;
    f.fast = 1;
    for (int k = 0; k < c->K; ++k)
        if (!c->lv[c->mips[k]].fast)
            f.fast = 0;
    f.p_begin = p_begin;
    f.P = P;
    f.tile_begin = 0;
}

ds_status ds_cloud_info(const ds_cloud *c, double *mean_mu_t, int *n_levels, int *dims,
                        int *mip_of_level, int *K)
{
    DS_CHECK(c, DS_ERR_INVALID_ARG, "ds_cloud_info: cloud is NULL");
    if (mean_mu_t)
        *mean_mu_t = c->mean;
    if (n_levels)
        *n_levels = c->L;
    if (dims)
        for (int i = 0; i < c->L; ++i) {
            dims[3 * i] = c->lv[i].nx;
            dims[3 * i + 1] = c->lv[i].ny;
            dims[3 * i + 2] = c->lv[i].nz;
        }
    if (mip_of_level)
        memcpy(mip_of_level, c->mips, sizeof(int) * c->K);
    if (K)
        *K = c->K;
    return DS_OK;
}

ds_status ds_cloud_level(ds_ctx *ctx, const ds_cloud *c, int level, float *dst_dev)
{
    DS_CHECK(ctx && c && dst_dev, DS_ERR_INVALID_ARG, "ds_cloud_level: NULL argument");
    DS_CHECK(level >= 0 && level < c->L, DS_ERR_INVALID_ARG, "ds_cloud_level: level %d of %d",
             level, c->L);
    const Level &l = c->lv[level];
    DS_HIP(hipMemcpyAsync(dst_dev, c->pyr + l.off, sizeof(float) * l.nx * l.ny * l.nz,
                          hipMemcpyDeviceToDevice, ctx->stream));
    return DS_OK;
}

ds_status ds_cloud_destroy(ds_cloud *c)
{
    if (!c)
        return DS_OK;
    if (c->ctx)
        (void)hipStreamSynchronize(c->ctx->stream);
    (void)hipFree(c->pyr);
    (void)hipFree(c->cells32);
    (void)hipFree(c->mu_cells);
    (void)hipFree(c->cells);
    (void)hipFree(c->tables);
    (void)hipFree(c->mu);
    delete c;
    return DS_OK;
}

// ---------------------------------------------------------------- network
int64_t ds_net_param_count(const ds_net_desc *d)
{
    if (!desc_ok(d))
        return -1;
    int64_t n = 0;
    for (int k = 0; k < d->K; ++k)
        n += (int64_t)d->W * 226 + (k ? (int64_t)d->W * d->W : 0) + d->W + (int64_t)d->W * d->W +
             d->W;
    for (int m = 0; m < d->H; ++m) {
        int rows = m == d->H - 1 ? 1 : d->W;
        n += (int64_t)rows * d->W + rows;
    }
    return n;
}

ds_status ds_net_create(ds_ctx *ctx, const ds_net_desc *desc, ds_net **out)
{
    DS_CHECK(ctx && out, DS_ERR_INVALID_ARG, "ds_net_create: NULL argument");
    DS_CHECK(desc_ok(desc), DS_ERR_INVALID_ARG,
             "ds_net_create: need 1 <= K <= 16, 1 <= W <= 256, 1 <= H <= 8");
    ds_net *n = new (std::nothrow) ds_net();
    DS_CHECK(n, DS_ERR_OOM, "ds_net_create: out of host memory");
    n->ctx = ctx;
    n->K = desc->K;
    n->W = desc->W;
    n->H = desc->H;
    n->n_params = ds_net_param_count(desc);
    if (hipMalloc(&n->theta, sizeof(float) * n->n_params) != hipSuccess) {
        delete n;
        set_error("ds_net_create: out of device memory");
        return DS_ERR_OOM;
    }
    hipError_t e = hipMemsetAsync(n->theta, 0, sizeof(float) * n->n_params, ctx->stream);
    if (e != hipSuccess) {
        (void)hipFree(n->theta);
        delete n;
        return hip_fail(e, "ds_net_create");
    }
    *out = n;
    return DS_OK;
}

int64_t ds_net_param_count_mlp(int32_t K, int32_t n_layers, const int32_t *widths)
{
    if (!widths || K < 1 || K > kMaxK || n_layers < 1 || n_layers > 64 || widths[n_layers - 1] != 1)
        return -1;
    int64_t n = 0, in = (int64_t)kStencil * K + 1;
    for (int l = 0; l < n_layers; ++l) {
        if (widths[l] < 1 || widths[l] > 1024)
            return -1;
        n += (int64_t)widths[l] * in + widths[l];
        in = widths[l];
    }
    return n;
}

ds_status ds_net_create_mlp(ds_ctx *ctx, int32_t K, int32_t n_layers, const int32_t *widths,
                            ds_net **out)
{
    DS_CHECK(ctx && widths && out, DS_ERR_INVALID_ARG, "ds_net_create_mlp: NULL argument");
    const int64_t np = ds_net_param_count_mlp(K, n_layers, widths);
    DS_CHECK(np > 0, DS_ERR_INVALID_ARG,
             "ds_net_create_mlp: need 1 <= K <= %d, 1 <= n_layers <= 64, widths in 1..1024 and "
             "a last width of 1", kMaxK);
    ds_net *n = new (std::nothrow) ds_net();
    DS_CHECK(n, DS_ERR_OOM, "ds_net_create_mlp: out of host memory");
    n->ctx = ctx;
    n->kind = 1;
    n->K = K;
    n->H = n_layers;
    n->mlp_widths.push_back(kStencil * K + 1);
    for (int l = 0; l < n_layers; ++l) {
        n->mlp_widths.push_back(widths[l]);
        n->W = widths[l] > n->W ? widths[l] : n->W;
    }
    n->n_params = np;
    if (hipMalloc(&n->theta, sizeof(float) * np) != hipSuccess) {
        delete n;
        set_error("ds_net_create_mlp: out of device memory");
        return DS_ERR_OOM;
    }
    hipError_t e = hipMemsetAsync(n->theta, 0, sizeof(float) * np, ctx->stream);
    if (e != hipSuccess) {
        (void)hipFree(n->theta);
        delete n;
        return hip_fail(e, "ds_net_create_mlp");
    }
    *out = n;
    return DS_OK;
}

ds_status ds_net_set_params(ds_net *net, const float *theta_host, int64_t n)
{
    DS_CHECK(net && theta_host, DS_ERR_INVALID_ARG, "ds_net_set_params: NULL argument");
    DS_CHECK(n == net->n_params, DS_ERR_INVALID_ARG,
             "ds_net_set_params: %lld parameters given, %lld expected", (long long)n,
             (long long)net->n_params);
    for (int64_t i = 0; i < n; ++i)
        DS_CHECK(isfinite(theta_host[i]), DS_ERR_INVALID_ARG,
                 "ds_net_set_params: parameter %lld is not finite", (long long)i);
    DS_HIP(hipStreamSynchronize(net->ctx->stream));
    DS_HIP(hipMemcpy(net->theta, theta_host, sizeof(float) * n, hipMemcpyHostToDevice));
    net->fp8_ready = false;
    if (net->kind == 0 && fused_tiles(net->W) > 0) {
        ds_status st = fused_pack_bf16(net->ctx->stream, net);
        if (st)
            return st;
        DS_HIP(hipStreamSynchronize(net->ctx->stream));
    }
    return DS_OK;
}

ds_status ds_net_get_params(ds_net *net, float *theta_host, int64_t n)
{
    DS_CHECK(net && theta_host, DS_ERR_INVALID_ARG, "ds_net_get_params: NULL argument");
    DS_CHECK(n == net->n_params, DS_ERR_INVALID_ARG,
             "ds_net_get_params: %lld parameters requested, %lld held", (long long)n,
             (long long)net->n_params);
    DS_HIP(hipStreamSynchronize(net->ctx->stream));
    DS_HIP(hipMemcpy(theta_host, net->theta, sizeof(float) * n, hipMemcpyDeviceToHost));
    return DS_OK;
}

ds_status ds_net_destroy(ds_net *net)
{
    if (!net)
        return DS_OK;
    (void)hipStreamSynchronize(net->ctx->stream);
    (void)hipFree(net->theta);
    (void)hipFree(net->frag_bf16);
    (void)hipFree(net->vec);
    (void)hipFree(net->fmap);
    (void)hipFree(net->vmap);
    (void)hipFree(net->frag_fp8);
    (void)hipFree(net->vec8);
    (void)hipFree(net->tws);
    delete net;
    return DS_OK;
}

// ---------------------------------------------------------------- hot path
ds_status ds_gather(ds_ctx *ctx, const ds_cloud *cloud, const float *pos, const float *view_dir,
                    const float *light_dir, int64_t P, ds_dtype out_dtype, void *z_out,
                    uint8_t *flags)
{
    DS_CHECK(ctx && cloud, DS_ERR_INVALID_ARG, "ds_gather: NULL context or cloud");
    DS_CHECK(P >= 0 && P <= ((int64_t)1 << 31), DS_ERR_INVALID_ARG, "ds_gather: bad P %lld",
             (long long)P);
    DS_CHECK(out_dtype == DS_F32 || out_dtype == DS_BF16, DS_ERR_INVALID_ARG,
             "ds_gather: bad output dtype");
    if (P == 0)
        return DS_OK;
    DS_CHECK(pos && view_dir && light_dir && z_out, DS_ERR_INVALID_ARG,
             "ds_gather: NULL device pointer");
    ds_status st = gather_cells(ctx, cloud);
    if (st)
        return st;
    GatherArgs a;
    gather_args(cloud, pos, view_dir, light_dir, P, a);
    return gather_plain(ctx->stream, a, 0, P, out_dtype, z_out, kStencil * cloud->K + 1, flags);
}

ds_status ds_gather_packed(ds_ctx *ctx, const ds_cloud *cloud, const float *pos,
                           const float *view_dir, const float *light_dir, int64_t P, float *z_out)
{
    DS_CHECK(ctx && cloud, DS_ERR_INVALID_ARG, "ds_gather_packed: NULL context or cloud");
    DS_CHECK(P >= 0 && P <= ((int64_t)1 << 31), DS_ERR_INVALID_ARG, "ds_gather_packed: bad P");
    if (P == 0)
        return DS_OK;
    DS_CHECK(pos && view_dir && light_dir && z_out, DS_ERR_INVALID_ARG,
             "ds_gather_packed: NULL device pointer");
    FusedArgs a = {};
    fused_args(pos, view_dir, light_dir, nullptr, nullptr, nullptr, cloud->K, 0, 0, a);
    add_cloud(a, cloud, 0, P);
    return fused_gather_packed(ctx->stream, a, z_out);
}

ds_status ds_forward(ds_ctx *ctx, const ds_net *net, const float *z, int64_t P, float *out,
                     float *pre_out)
{
    DS_CHECK(ctx && net, DS_ERR_INVALID_ARG, "ds_forward: NULL context or network");
    DS_CHECK(P >= 0 && P <= ((int64_t)1 << 31), DS_ERR_INVALID_ARG, "ds_forward: bad P");
    if (P == 0)
        return DS_OK;
    DS_CHECK(z && out, DS_ERR_INVALID_ARG, "ds_forward: NULL device pointer");
    const int64_t rows = P < kChunk ? P : kChunk;
    size_t need = sizeof(float) * (size_t)rows * net->W * 3;
    ds_status st = ensure_ws(ctx, need);
    if (st)
        return st;
    float *O = static_cast<float *>(ctx->ws);
    return forward_plain(ctx, net, z, P, out, pre_out, O, O + rows * net->W,
                         O + 2 * rows * net->W);
}

// The plain FP32 form in chunks of kChunk points: descriptor rows to HBM, then one GEMM
// per layer (amax: see forward_plain).
static ds_status predict_plain(ds_ctx *ctx, const ds_cloud *cloud, const ds_net *net,
                               const float *pos, const float *view_dir, const float *light_dir,
                               int64_t P, float *out, float *pre_out, uint8_t *flags,
                               unsigned *amax)
{
    const int D = kStencil * net->K + 1;
    const int64_t rows = P < kChunk ? P : kChunk;
    size_t need = sizeof(float) * (size_t)rows * ((size_t)D + 3 * net->W) + (size_t)rows;
    ds_status st = ensure_ws(ctx, need);
    if (!st)
        st = gather_cells(ctx, cloud);
    if (st)
        return st;
    float *z = static_cast<float *>(ctx->ws);
    float *O = z + rows * D;
    uint8_t *fl_ws = reinterpret_cast<uint8_t *>(O + 3 * rows * net->W);
    GatherArgs a;
    gather_args(cloud, pos, view_dir, light_dir, P, a);
    for (int64_t p0 = 0; p0 < P; p0 += kChunk) {
        int64_t np = (P - p0) < kChunk ? (P - p0) : kChunk;
        // the gather writes flags at absolute point indices
        uint8_t *fl = flags ? flags : fl_ws - p0;
        st = gather_plain(ctx->stream, a, p0, np, DS_F32, z, D, fl);
        if (st)
            return st;
        st = forward_plain(ctx, net, z, np, out + p0, pre_out ? pre_out + p0 : nullptr, O,
                           O + rows * net->W, O + 2 * rows * net->W, amax);
        if (st)
            return st;
        st = mask_invalid(ctx->stream, fl + p0, np, out + p0, pre_out ? pre_out + p0 : nullptr);
        if (st)
            return st;
    }
    return DS_OK;
}

ds_status ds_predict_reserve(ds_ctx *ctx, const ds_cloud *cloud, const ds_net *net,
                             ds_precision precision, int64_t P)
{
    DS_CHECK(ctx && cloud && net, DS_ERR_INVALID_ARG,
             "ds_predict_reserve: NULL context, cloud or net");
    DS_CHECK(cloud->K == net->K, DS_ERR_INVALID_ARG,
             "ds_predict_reserve: the cloud has %d stencil levels, the network %d", cloud->K,
             net->K);
    DS_CHECK(P >= 0 && P <= ((int64_t)1 << 31), DS_ERR_INVALID_ARG, "ds_predict_reserve: bad P");
    DS_CHECK(precision == DS_PREC_F32 || precision == DS_PREC_BF16 || precision == DS_PREC_FP8,
             DS_ERR_INVALID_ARG, "ds_predict_reserve: unknown precision %d", (int)precision);
    if (precision != DS_PREC_F32 || P == 0)
        return DS_OK;
    DS_HIP(hipSetDevice(ctx->device));
    const int64_t rows = P < kChunk ? P : kChunk;
    const size_t D = (size_t)kStencil * net->K + 1;
    DS_TRY(ensure_ws(ctx, sizeof(float) * (size_t)rows * (D + 3 * (size_t)net->W) + (size_t)rows));
    DS_TRY(gather_cells(ctx, cloud));
    DS_HIP(hipStreamSynchronize(ctx->stream));
    return DS_OK;
}

ds_status ds_predict_f32_noalloc(ds_ctx *ctx, const ds_cloud *cloud, const ds_net *net,
                                 const float *pos, const float *view_dir, const float *light_dir,
                                 int64_t P, float *out, float *pre_out, uint8_t *flags)
{
    DS_CHECK(ctx && cloud && net, DS_ERR_INVALID_ARG,
             "ds_predict_f32_noalloc: NULL context, cloud or net");
    DS_CHECK(cloud->K == net->K, DS_ERR_INVALID_ARG,
             "ds_predict_f32_noalloc: the cloud has %d stencil levels, the network %d", cloud->K,
             net->K);
    DS_CHECK(P >= 0 && P <= ((int64_t)1 << 31), DS_ERR_INVALID_ARG,
             "ds_predict_f32_noalloc: bad P");
    if (P == 0)
        return DS_OK;
    DS_CHECK(pos && view_dir && light_dir && out, DS_ERR_INVALID_ARG,
             "ds_predict_f32_noalloc: NULL device pointer");
    DS_CHECK(ctx->device >= 0 && ctx->device < kScratchDevices && g_scratch[ctx->device],
             DS_ERR_STATE, "ds_predict_f32_noalloc: no scratch address for device %d",
             ctx->device);
    DS_CHECK(cloud->cells32, DS_ERR_STATE,
             "ds_predict_f32_noalloc: the cloud's float32 corner cells do not exist (building "
             "them allocates): call ds_predict_reserve with DS_PREC_F32 once first");
    // a chunk: descriptor rows [rows][D], three activation buffers [rows][W], flags [rows]
    const int D = kStencil * net->K + 1;
    const size_t per_point = sizeof(float) * ((size_t)D + 3 * (size_t)net->W) + 1;
    const int64_t fit = (int64_t)((kScratchBytes - 256) / per_point) / 64 * 64;
    DS_CHECK(fit >= 64, DS_ERR_INVALID_ARG,
             "ds_predict_f32_noalloc: a point needs %zu bytes of scratch, %zu bytes hold fewer "
             "than 64 points", per_point, kScratchBytes);
    const int64_t rows = P < fit ? P : fit;
    float *z = static_cast<float *>(g_scratch[ctx->device]);
    float *O = z + rows * D;
    uint8_t *fl_ws = reinterpret_cast<uint8_t *>(O + 3 * rows * net->W);
    GatherArgs a;
    gather_args(cloud, pos, view_dir, light_dir, P, a);
    for (int64_t p0 = 0; p0 < P; p0 += rows) {
        const int64_t np = (P - p0) < rows ? (P - p0) : rows;
        uint8_t *fl = flags ? flags : fl_ws - p0;  // the gather writes absolute indices
        ds_status st = gather_plain(ctx->stream, a, p0, np, DS_F32, z, D, fl);
        if (!st)
            st = forward_plain(ctx, net, z, np, out + p0, pre_out ? pre_out + p0 : nullptr, O,
                               O + rows * net->W, O + 2 * rows * net->W);
        if (!st)
            st = mask_invalid(ctx->stream, fl + p0, np, out + p0, pre_out ? pre_out + p0 : nullptr);
        if (st)
            return st;
    }
    return DS_OK;
}

ds_status ds_predict(ds_ctx *ctx, const ds_cloud *cloud, const ds_net *net,
                     ds_precision precision, const float *pos, const float *view_dir,
                     const float *light_dir, int64_t P, float *out, float *pre_out,
                     uint8_t *flags)
{
    DS_CHECK(ctx && cloud && net, DS_ERR_INVALID_ARG, "ds_predict: NULL context, cloud or net");
    DS_CHECK(cloud->K == net->K, DS_ERR_INVALID_ARG,
             "ds_predict: the cloud has %d stencil levels, the network %d", cloud->K, net->K);
    DS_CHECK(P >= 0 && P <= ((int64_t)1 << 31), DS_ERR_INVALID_ARG, "ds_predict: bad P");
    if (P == 0)
        return DS_OK;
    DS_CHECK(pos && view_dir && light_dir && out, DS_ERR_INVALID_ARG,
             "ds_predict: NULL device pointer");
    if (precision == DS_PREC_F32)
        return predict_plain(ctx, cloud, net, pos, view_dir, light_dir, P, out, pre_out, flags,
                             nullptr);
    if (precision == DS_PREC_BF16 || precision == DS_PREC_FP8) {
        DS_CHECK(net->kind == 0, DS_ERR_UNSUPPORTED,
                 "ds_predict: the all-at-once MLP runs in DS_PREC_F32 only");
        FusedArgs a = {};
        fused_args(pos, view_dir, light_dir, out, pre_out, flags, net->K, net->W, net->H, a);
        add_cloud(a, cloud, 0, P);
        return fused_predict(ctx->stream, net, a, kDefaultVariant, precision);
    }
    set_error("ds_predict: unknown precision %d", (int)precision);
    return DS_ERR_INVALID_ARG;
}

// ---------------------------------------------------------------- batched prediction
static void batch_args(const ds_batch *b, const float *pos, const float *view, const float *light,
                       float *out, float *pre, uint8_t *flags, FusedArgs &a)
{
    fused_args(pos, view, light, out, pre, flags, b->net->K, b->net->W, b->net->H, a);
    for (int c = 0; c < b->n; ++c)
        add_cloud(a, b->clouds[c], b->offsets[c], b->offsets[c + 1] - b->offsets[c]);
}

static void batch_drop_graph(ds_batch *b)
{
    if (b->exec) {
        (void)hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
    }
}

static ds_status batch_fused(ds_batch *b, hipStream_t s, ds_precision prec, const float *pos,
                             const float *view, const float *light, float *out, float *pre,
                             uint8_t *flags, const FusedVariant &v)
{
    DS_CHECK(prec == DS_PREC_BF16 || prec == DS_PREC_FP8, DS_ERR_INVALID_ARG,
             "batched launch: precision %d is not a fused precision", (int)prec);
    FusedArgs a = {};
    batch_args(b, pos, view, light, out, pre, flags, a);
    if (b->order == DS_ORDER_SPATIAL) {
        ds_status st = batch_order(s, a, b->offsets[b->n], b->perm, b->slot, b->counts, b->sums);
        if (st)
            return st;
        a.perm = b->perm;
    }
    return fused_predict(s, b->net, a, v, prec);
}

static void batch_free_order(ds_batch *b)
{
    int32_t **bufs[4] = {&b->perm, &b->slot, &b->counts, &b->sums};
    for (int32_t **q : bufs) {
        if (*q)
            (void)hipFree(*q);
        *q = nullptr;
    }
}

ds_status ds_batch_create(ds_ctx *ctx, const ds_net *net, int n_clouds,
                          const ds_cloud *const *clouds, const int64_t *offsets, ds_batch **out)
{
    DS_CHECK(ctx && net && clouds && offsets && out, DS_ERR_INVALID_ARG,
             "ds_batch_create: NULL argument");
    DS_CHECK(n_clouds >= 1 && n_clouds <= kMaxBatch, DS_ERR_INVALID_ARG,
             "ds_batch_create: n_clouds %d outside 1..%d", n_clouds, kMaxBatch);
    DS_CHECK(net->kind == 0, DS_ERR_UNSUPPORTED,
             "ds_batch_create: batched prediction runs the RPNN's fused kernel");
    DS_CHECK(offsets[0] == 0, DS_ERR_INVALID_ARG, "ds_batch_create: offsets[0] must be 0");
    for (int c = 0; c < n_clouds; ++c) {
        DS_CHECK(clouds[c], DS_ERR_INVALID_ARG, "ds_batch_create: cloud %d is NULL", c);
        DS_CHECK(clouds[c]->K == net->K, DS_ERR_INVALID_ARG,
                 "ds_batch_create: cloud %d has %d stencil levels, the network %d", c,
                 clouds[c]->K, net->K);
        DS_CHECK(offsets[c + 1] >= offsets[c], DS_ERR_INVALID_ARG,
                 "ds_batch_create: offsets must not decrease");
    }
    DS_CHECK(offsets[n_clouds] <= ((int64_t)1 << 31), DS_ERR_INVALID_ARG,
             "ds_batch_create: more than 2^31 points");
    ds_batch *b = new (std::nothrow) ds_batch();
    DS_CHECK(b, DS_ERR_OOM, "ds_batch_create: out of host memory");
    b->ctx = ctx;
    b->net = net;
    b->n = n_clouds;
    for (int c = 0; c < n_clouds; ++c)
        b->clouds[c] = clouds[c];
    memcpy(b->offsets, offsets, sizeof(int64_t) * (n_clouds + 1));
    b->kind = kDefaultVariant.kind;
    b->waves = kDefaultVariant.waves;
    b->grid = kDefaultVariant.grid;
    *out = b;
    return DS_OK;
}

ds_status ds_batch_destroy(ds_batch *b)
{
    if (!b)
        return DS_OK;
    batch_drop_graph(b);
    if (b->cap_stream)
        (void)hipStreamDestroy(b->cap_stream);
    if (b->perm)
        (void)hipSetDevice(b->ctx->device);
    batch_free_order(b);
    delete b;
    return DS_OK;
}

ds_status ds_batch_set_order(ds_batch *b, int32_t order)
{
    DS_CHECK(b, DS_ERR_INVALID_ARG, "ds_batch_set_order: batch is NULL");
    DS_CHECK(order == DS_ORDER_INPUT || order == DS_ORDER_SPATIAL, DS_ERR_INVALID_ARG,
             "ds_batch_set_order: unknown order %d", (int)order);
    if (order == b->order)
        return DS_OK;
    DS_HIP(hipSetDevice(b->ctx->device));
    DS_HIP(hipStreamSynchronize(b->ctx->stream));  // no launch may still read the workspace
    batch_drop_graph(b);
    batch_free_order(b);
    b->order = DS_ORDER_INPUT;
    if (order == DS_ORDER_SPATIAL) {
        const int64_t total = b->offsets[b->n];
        const size_t sizes[4] = {(size_t)std::max<int64_t>(total, 1),
                                 (size_t)std::max<int64_t>(total, 1),
                                 (size_t)order_buckets(b->n), (size_t)order_sums(b->n)};
        int32_t **bufs[4] = {&b->perm, &b->slot, &b->counts, &b->sums};
        for (int i = 0; i < 4; ++i) {
            hipError_t e = hipMalloc((void **)bufs[i], sizes[i] * sizeof(int32_t));
            if (e != hipSuccess) {
                *bufs[i] = nullptr;
                batch_free_order(b);
                return hip_fail(e, "ds_batch_set_order: workspace");
            }
        }
        b->order = DS_ORDER_SPATIAL;
    }
    return DS_OK;
}

ds_status ds_batch_set_config(ds_batch *b, int32_t kernel, int32_t waves, int32_t grid)
{
    DS_CHECK(b, DS_ERR_INVALID_ARG, "ds_batch_set_config: batch is NULL");
    FusedVariant v = {kernel, waves, grid};
    DS_CHECK(fused_variant_ok(b->net, v), DS_ERR_INVALID_ARG,
             "ds_batch_set_config: variant (kernel %d, %d waves, grid %d) not available", kernel,
             waves, grid);
    b->kind = kernel;
    b->waves = waves;
    b->grid = grid;
    b->tuned_ms = -1.f;
    batch_drop_graph(b);
    return DS_OK;
}

ds_status ds_batch_get_config(const ds_batch *b, int32_t *kernel, int32_t *waves, int32_t *grid,
                              float *ms)
{
    DS_CHECK(b, DS_ERR_INVALID_ARG, "ds_batch_get_config: batch is NULL");
    if (kernel)
        *kernel = b->kind;
    if (waves)
        *waves = b->waves;
    if (grid)
        *grid = b->grid;
    if (ms)
        *ms = b->tuned_ms;
    return DS_OK;
}

ds_status ds_batch_predict(ds_batch *b, ds_precision precision, const float *pos,
                           const float *view_dir, const float *light_dir, float *out,
                           float *pre_out, uint8_t *flags)
{
    DS_CHECK(b, DS_ERR_INVALID_ARG, "ds_batch_predict: batch is NULL");
    const int64_t total = b->offsets[b->n];
    if (total == 0)
        return DS_OK;
    DS_CHECK(pos && view_dir && light_dir && out, DS_ERR_INVALID_ARG,
             "ds_batch_predict: NULL device pointer");
    DS_HIP(hipSetDevice(b->ctx->device));
    if (precision == DS_PREC_F32) {
        for (int c = 0; c < b->n; ++c) {
            const int64_t o = b->offsets[c], P = b->offsets[c + 1] - o;
            ds_status st = ds_predict(b->ctx, b->clouds[c], b->net, DS_PREC_F32, pos + 3 * o,
                                      view_dir + 3 * o, light_dir + 3 * o, P, out + o,
                                      pre_out ? pre_out + o : nullptr, flags ? flags + o : nullptr);
            if (st)
                return st;
        }
        return DS_OK;
    }
    return batch_fused(b, b->ctx->stream, precision, pos, view_dir, light_dir, out, pre_out, flags,
                       FusedVariant{b->kind, b->waves, b->grid});
}

ds_status ds_batch_autotune(ds_batch *b, ds_precision precision, const float *pos,
                            const float *view_dir, const float *light_dir, float *out, int reps)
{
    DS_CHECK(b, DS_ERR_INVALID_ARG, "ds_batch_autotune: batch is NULL");
    DS_CHECK(reps >= 1 && reps <= 1000, DS_ERR_INVALID_ARG, "ds_batch_autotune: reps 1..1000");
    DS_CHECK(precision != DS_PREC_F32, DS_ERR_UNSUPPORTED,
             "ds_batch_autotune: only the fused precisions have variants");
    if (b->offsets[b->n] == 0)
        return DS_OK;
    DS_CHECK(pos && view_dir && light_dir && out, DS_ERR_INVALID_ARG,
             "ds_batch_autotune: NULL device pointer");
    DS_HIP(hipSetDevice(b->ctx->device));
    int cus = 0;
    DS_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->ctx->device));
    hipStream_t s = b->ctx->stream;
    hipEvent_t e0, e1;
    DS_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_fail(hipErrorOutOfMemory, "ds_batch_autotune: event");
    }
    ds_status st = DS_OK;
    // the candidates, each warmed up once; then kTuneRounds interleaved rounds of reps
    // launches per candidate, keeping each candidate's fastest round, so that a clock that
    // drifts during the sweep does not favour the candidates timed last
    constexpr int kTuneRounds = 3;
    FusedVariant cand[32];
    float tbest[32];
    int nc = 0;
    const int grids[4] = {0, cus, 2 * cus, 4 * cus};
    for (int kind = 0; kind < 4 && !st; ++kind)
        for (int waves = 4; waves <= 8 && !st; waves += 4)
            for (int gi = 0; gi < 4 && !st; ++gi) {
                FusedVariant v = {kind, waves, grids[gi]};
                if (!(precision == DS_PREC_FP8 ? fused_variant_ok_fp8(b->net, v)
                                               : fused_variant_ok(b->net, v)))
                    continue;
                st = batch_fused(b, s, precision, pos, view_dir, light_dir, out, nullptr, nullptr,
                                 v);
                cand[nc] = v;
                tbest[nc++] = -1.f;
            }
    for (int round = 0; round < kTuneRounds && !st; ++round)
        for (int c = 0; c < nc && !st; ++c) {
            hipError_t e = hipEventRecord(e0, s);
            for (int r = 0; r < reps && !st && e == hipSuccess; ++r)
                st = batch_fused(b, s, precision, pos, view_dir, light_dir, out, nullptr, nullptr,
                                 cand[c]);
            if (e == hipSuccess)
                e = hipEventRecord(e1, s);
            if (e == hipSuccess)
                e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess)
                e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess && !st)
                st = hip_fail(e, "ds_batch_autotune");
            if (!st && (tbest[c] < 0.f || ms / reps < tbest[c]))
                tbest[c] = ms / reps;
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st)
        return st;
    float best = -1.f;
    FusedVariant bestv = {b->kind, b->waves, b->grid};
    for (int c = 0; c < nc; ++c)
        if (best < 0.f || tbest[c] < best) {
            best = tbest[c];
            bestv = cand[c];
        }
    b->kind = bestv.kind;
    b->waves = bestv.waves;
    b->grid = bestv.grid;
    b->tuned_ms = best;
    batch_drop_graph(b);
    return DS_OK;
}

ds_status ds_batch_capture(ds_batch *b, ds_precision precision, const float *pos,
                           const float *view_dir, const float *light_dir, float *out,
                           float *pre_out, uint8_t *flags)
{
    DS_CHECK(b, DS_ERR_INVALID_ARG, "ds_batch_capture: batch is NULL");
    DS_CHECK(precision != DS_PREC_F32, DS_ERR_UNSUPPORTED,
             "ds_batch_capture: the plain FP32 form is not captured");
    DS_CHECK(b->offsets[b->n] == 0 || (pos && view_dir && light_dir && out), DS_ERR_INVALID_ARG,
             "ds_batch_capture: NULL device pointer");
    DS_CHECK(precision == DS_PREC_BF16 || precision == DS_PREC_FP8, DS_ERR_INVALID_ARG,
             "ds_batch_capture: precision %d is not available", (int)precision);
    DS_CHECK(precision == DS_PREC_FP8 ? b->net->fp8_ready : b->net->frag_bf16 != nullptr,
             DS_ERR_STATE, "ds_batch_capture: the network has no %s form",
             precision == DS_PREC_FP8 ? "FP8 (quantize it first)" : "BF16 (set its parameters)");
    DS_HIP(hipSetDevice(b->ctx->device));
    batch_drop_graph(b);
    if (!b->cap_stream)
        DS_HIP(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
    // the capture stream starts after the context stream's pending work
    DS_HIP(hipStreamSynchronize(b->ctx->stream));
    DS_HIP(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
    ds_status st = b->offsets[b->n] == 0
                       ? DS_OK
                       : batch_fused(b, b->cap_stream, precision, pos, view_dir, light_dir, out,
                                     pre_out, flags, FusedVariant{b->kind, b->waves, b->grid});
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
    if (st) {
        if (g)
            (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess)
        return hip_fail(e, "ds_batch_capture: end of capture");
    e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        b->exec = nullptr;
        return hip_fail(e, "ds_batch_capture: instantiate");
    }
    return DS_OK;
}

ds_status ds_batch_replay(ds_batch *b)
{
    DS_CHECK(b, DS_ERR_INVALID_ARG, "ds_batch_replay: batch is NULL");
    DS_CHECK(b->exec, DS_ERR_STATE, "ds_batch_replay: nothing captured");
    DS_HIP(hipSetDevice(b->ctx->device));
    DS_HIP(hipGraphLaunch(b->exec, b->ctx->stream));
    return DS_OK;
}

// ---------------------------------------------------------------- training (Sec. 5.2)
ds_status ds_net_set_train_precision(ds_net *net, ds_precision precision)
{
    DS_CHECK(net, DS_ERR_INVALID_ARG, "ds_net_set_train_precision: net is NULL");
    DS_CHECK(precision == DS_PREC_F32 || precision == DS_PREC_BF16,
             precision == DS_PREC_FP8 ? DS_ERR_UNSUPPORTED : DS_ERR_INVALID_ARG,
             "ds_net_set_train_precision: training runs in FP32 or BF16");
    net->train_prec = precision;
    return DS_OK;
}

// ---------------------------------------------------------------- FP8 form
ds_status ds_net_quantize(ds_ctx *ctx, ds_net *net, const ds_cloud *cloud, ds_precision precision,
                          const float *pos, const float *view_dir, const float *light_dir,
                          int64_t n_calib)
{
    DS_CHECK(ctx && net && cloud, DS_ERR_INVALID_ARG, "ds_net_quantize: NULL argument");
    DS_CHECK(precision == DS_PREC_FP8, DS_ERR_INVALID_ARG,
             "ds_net_quantize: only DS_PREC_FP8 is built by this call (the BF16 form follows "
             "every parameter change)");
    DS_CHECK(net->kind == 0, DS_ERR_UNSUPPORTED,
             "ds_net_quantize: the FP8 form exists for the RPNN only");
    DS_CHECK(fused_tiles(net->W) > 0, DS_ERR_UNSUPPORTED,
             "ds_net_quantize: width %d is not supported by the fused kernel", net->W);
    DS_CHECK(net->frag_bf16, DS_ERR_STATE, "ds_net_quantize: network parameters were never set");
    DS_CHECK(cloud->K == net->K, DS_ERR_INVALID_ARG,
             "ds_net_quantize: cloud has %d stencil levels, the network %d", cloud->K, net->K);
    DS_CHECK(n_calib >= 1 && n_calib <= ((int64_t)1 << 31), DS_ERR_INVALID_ARG,
             "ds_net_quantize: calibration count %lld outside 1..2^31", (long long)n_calib);
    DS_CHECK(pos && view_dir && light_dir, DS_ERR_INVALID_ARG,
             "ds_net_quantize: NULL device pointer");
    DS_HIP(hipSetDevice(ctx->device));
    const int K = net->K, H = net->H;
    const int na = K + H;  // activation maxima, see forward_plain
    // calibration: the FP32 plain form, recording the largest activation of every layer
    unsigned *amax = nullptr;
    float *out = nullptr;
    DS_CHECK(hipMalloc(&amax, sizeof(unsigned) * na) == hipSuccess, DS_ERR_OOM,
             "ds_net_quantize: out of device memory");
    ds_status st = DS_OK;
    if (hipMalloc(&out, sizeof(float) * (size_t)n_calib) != hipSuccess) {
        st = DS_ERR_OOM;
        set_error("ds_net_quantize: out of device memory");
    }
    if (!st) {
        hipError_t e = hipMemsetAsync(amax, 0, sizeof(unsigned) * na, ctx->stream);
        if (e != hipSuccess)
            st = hip_fail(e, "ds_net_quantize: clear");
    }
    if (!st)
        st = predict_plain(ctx, cloud, net, pos, view_dir, light_dir, n_calib, out, nullptr,
                           nullptr, amax);
    std::vector<unsigned> bits(na);
    std::vector<float> theta((size_t)net->n_params);
    if (!st) {
        hipError_t e = hipStreamSynchronize(ctx->stream);
        if (e == hipSuccess)
            e = hipMemcpy(bits.data(), amax, sizeof(unsigned) * na, hipMemcpyDeviceToHost);
        if (e == hipSuccess)
            e = hipMemcpy(theta.data(), net->theta, sizeof(float) * theta.size(),
                          hipMemcpyDeviceToHost);
        if (e != hipSuccess)
            st = hip_fail(e, "ds_net_quantize");
    }
    (void)hipFree(amax);
    (void)hipFree(out);
    if (st)
        return st;
    std::vector<float> act(na);
    for (int i = 0; i < na; ++i)
        memcpy(&act[i], &bits[i], 4);
    return fused_quantize_fp8(net, theta.data(), act.data());
}

ds_status ds_net_fp8_scales(const ds_net *net, int32_t *log2_scales, int32_t n)
{
    DS_CHECK(net && log2_scales, DS_ERR_INVALID_ARG, "ds_net_fp8_scales: NULL argument");
    DS_CHECK(net->fp8_ready, DS_ERR_STATE, "ds_net_fp8_scales: the network has no FP8 form");
    DS_CHECK(n == fp8_exp_count(net->K, net->H), DS_ERR_INVALID_ARG,
             "ds_net_fp8_scales: %d entries given, %d expected", n,
             fp8_exp_count(net->K, net->H));
    memcpy(log2_scales, net->fp8_exps.data(), sizeof(int32_t) * n);
    return DS_OK;
}

ds_status ds_fp8_e4m3_encode(const float *x, int64_t n, int32_t log2_scale, uint8_t *codes)
{
    DS_CHECK(n >= 0, DS_ERR_INVALID_ARG, "ds_fp8_e4m3_encode: negative count");
    if (n == 0)
        return DS_OK;
    DS_CHECK(x && codes, DS_ERR_INVALID_ARG, "ds_fp8_e4m3_encode: NULL argument");
    DS_CHECK(log2_scale >= -64 && log2_scale <= 64, DS_ERR_INVALID_ARG,
             "ds_fp8_e4m3_encode: scale exponent %d outside -64..64", log2_scale);
    for (int64_t i = 0; i < n; ++i)
        codes[i] = e4m3_encode((float)ldexp((double)x[i], log2_scale));
    return DS_OK;
}

ds_status ds_adam_create(ds_net *net, float lr, float beta1, float beta2, float eps, ds_adam **out)
{
    DS_CHECK(net && out, DS_ERR_INVALID_ARG, "ds_adam_create: NULL argument");
    DS_CHECK(lr > 0.f && beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && eps > 0.f,
             DS_ERR_INVALID_ARG, "ds_adam_create: bad hyper-parameters");
    ds_adam *a = new (std::nothrow) ds_adam();
    DS_CHECK(a, DS_ERR_OOM, "ds_adam_create: out of host memory");
    a->net = net;
    a->lr = lr;
    a->b1 = beta1;
    a->b2 = beta2;
    a->eps = eps;
    const size_t n = (size_t)net->n_params;
    if (hipMalloc(&a->m, n * 4) != hipSuccess || hipMalloc(&a->v, n * 4) != hipSuccess ||
        hipMalloc(&a->grad, n * 4) != hipSuccess || hipMalloc(&a->steps, 8) != hipSuccess ||
        hipMalloc(&a->state, 16) != hipSuccess) {
        ds_adam_destroy(a);
        set_error("ds_adam_create: out of device memory");
        return DS_ERR_OOM;
    }
    hipStream_t s = net->ctx->stream;
    const int64_t t0 = 0;
    const float st0[4] = {lr, 1.f, 1.f, 0.f};
    if (hipMemsetAsync(a->m, 0, n * 4, s) != hipSuccess ||
        hipMemsetAsync(a->v, 0, n * 4, s) != hipSuccess ||
        hipMemcpyAsync(a->steps, &t0, 8, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(a->state, st0, 16, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        ds_adam_destroy(a);
        set_error("ds_adam_create: initialising the optimiser state failed");
        return DS_ERR_DEVICE;
    }
    *out = a;
    return DS_OK;
}

ds_status ds_adam_set_lr(ds_adam *a, float lr)
{
    DS_CHECK(a, DS_ERR_INVALID_ARG, "ds_adam_set_lr: optimiser is NULL");
    DS_CHECK(lr > 0.f && std::isfinite(lr), DS_ERR_INVALID_ARG,
             "ds_adam_set_lr: learning rate must be positive and finite");
    a->lr = lr;
    hipStream_t s = a->net->ctx->stream;
    DS_HIP(hipMemcpyAsync(a->state, &lr, sizeof(float), hipMemcpyHostToDevice, s));
    DS_HIP(hipStreamSynchronize(s));
    return DS_OK;
}

ds_status ds_adam_destroy(ds_adam *a)
{
    if (!a)
        return DS_OK;
    (void)hipStreamSynchronize(a->net->ctx->stream);
    if (a->exec)
        (void)hipGraphExecDestroy(a->exec);
    (void)hipFree(a->m);
    (void)hipFree(a->v);
    (void)hipFree(a->grad);
    (void)hipFree(a->steps);
    (void)hipFree(a->state);
    delete a;
    return DS_OK;
}

ds_status ds_adam_steps(const ds_adam *a, int64_t *t)
{
    DS_CHECK(a && t, DS_ERR_INVALID_ARG, "ds_adam_steps: NULL argument");
    hipStream_t s = a->net->ctx->stream;
    DS_HIP(hipMemcpyAsync(t, a->steps, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    DS_HIP(hipStreamSynchronize(s));
    return DS_OK;
}

ds_status ds_loss_grad(ds_net *net, const float *z, const float *target_log1p, int B,
                       float *loss_dev, float *grad_dev)
{
    DS_CHECK(net && z && target_log1p, DS_ERR_INVALID_ARG, "ds_loss_grad: NULL argument");
    DS_CHECK(B >= 1 && B <= (1 << 20), DS_ERR_INVALID_ARG, "ds_loss_grad: batch %d outside 1..2^20",
             B);
    return loss_grad(net, z, target_log1p, B, loss_dev, grad_dev);
}

// Loss, gradient, Adam update and refresh of the matrix-core weights: kernels only, so the
// body can be captured once the training workspace exists.
static ds_status train_step_body(ds_net *net, ds_adam *opt, const float *z,
                                 const float *target_log1p, int B, float *loss_dev)
{
    ds_status st = loss_grad(net, z, target_log1p, B, loss_dev, opt->grad);
    if (st)
        return st;
    st = adam_update(net->ctx->stream, net->theta, opt->m, opt->v, opt->grad, net->n_params,
                     opt->b1, opt->b2, opt->eps, opt->steps, opt->state);
    if (st)
        return st;
    net->fp8_ready = false;
    if (net->kind == 0 && fused_tiles(net->W) > 0)
        return fused_pack_bf16(net->ctx->stream, net);
    return DS_OK;
}

ds_status ds_train_step(ds_net *net, ds_adam *opt, const float *z, const float *target_log1p,
                        int B, float *loss_dev)
{
    DS_CHECK(net && opt && z && target_log1p, DS_ERR_INVALID_ARG, "ds_train_step: NULL argument");
    DS_CHECK(opt->net == net, DS_ERR_INVALID_ARG, "ds_train_step: optimiser of another network");
    DS_CHECK(B >= 1 && B <= (1 << 20), DS_ERR_INVALID_ARG,
             "ds_train_step: batch %d outside 1..2^20", B);
    return train_step_body(net, opt, z, target_log1p, B, loss_dev);
}

ds_status ds_train_capture(ds_net *net, ds_adam *opt, const float *z, const float *target_log1p,
                           int B, float *loss_dev)
{
    DS_CHECK(net && opt && z && target_log1p, DS_ERR_INVALID_ARG,
             "ds_train_capture: NULL argument");
    DS_CHECK(opt->net == net, DS_ERR_INVALID_ARG, "ds_train_capture: optimiser of another network");
    DS_CHECK(B >= 1 && B <= (1 << 20), DS_ERR_INVALID_ARG,
             "ds_train_capture: batch %d outside 1..2^20", B);
    DS_CHECK(net->tws && net->tws_floats >= train_ws_floats(net, B), DS_ERR_STATE,
             "ds_train_capture: no training workspace for a batch of %d yet (growing it "
             "allocates): run ds_train_step or ds_loss_grad with this batch size first", B);
    DS_HIP(hipSetDevice(net->ctx->device));
    hipStream_t s = net->ctx->stream;
    DS_CHECK(s, DS_ERR_STATE, "ds_train_capture: the context uses the default stream, which "
                              "cannot be captured");
    if (opt->exec) {
        (void)hipGraphExecDestroy(opt->exec);
        opt->exec = nullptr;
    }
    DS_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    ds_status st = train_step_body(net, opt, z, target_log1p, B, loss_dev);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(s, &g);
    if (st) {
        if (g)
            (void)hipGraphDestroy(g);
        return st;
    }
    if (e == hipSuccess)
        e = hipGraphInstantiate(&opt->exec, g, nullptr, nullptr, 0);
    if (g)
        (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        opt->exec = nullptr;
        return hip_fail(e, "ds_train_capture");
    }
    return DS_OK;
}

ds_status ds_train_replay(ds_adam *opt)
{
    DS_CHECK(opt, DS_ERR_INVALID_ARG, "ds_train_replay: optimiser is NULL");
    DS_CHECK(opt->exec, DS_ERR_STATE, "ds_train_replay: no captured step (ds_train_capture)");
    DS_HIP(hipGraphLaunch(opt->exec, opt->net->ctx->stream));
    opt->net->fp8_ready = false;
    return DS_OK;
}

// ---------------------------------------------------------------- Monte Carlo
static ds_status tracer_params(const ds_tracer_params *p, TracerParams &tp, const char *fn)
{
    DS_CHECK(p, DS_ERR_INVALID_ARG, "%s: params is NULL", fn);
    tp.ph_p = p->phase ? p->phase->p : nullptr;
    tp.ph_cdf = p->phase ? p->phase->cdf : nullptr;
    tp.ph_n = p->phase ? p->phase->n : 0;
    tp.pf_p = p->phase_first ? p->phase_first->p : nullptr;
    tp.pf_cdf = p->phase_first ? p->phase_first->cdf : nullptr;
    tp.pf_n = p->phase_first ? p->phase_first->n : 0;
    DS_CHECK(p->albedo >= 0.f && p->albedo <= 1.f, DS_ERR_INVALID_ARG,
             "%s: albedo %g outside [0, 1]", fn, (double)p->albedo);
    // Sec. 3.1: chopping the forward peak removes the fraction f of the scattering, which
    // then travels on as unscattered light, so the medium gets optically thinner by the
    // scattering removed: extinction mu_t (1 - a f), albedo a (1 - f) / (1 - a f) for the
    // single-scattering albedo a the caller passes
    const double f = p->phase ? p->phase->removed : 0.0;
    const double s = 1.0 - (double)p->albedo * f;
    tp.ext_scale = (float)s;
    tp.albedo = f > 0.0 ? (float)((double)p->albedo * (1.0 - f) / s) : p->albedo;
    // a table chopped with removed fraction f carries 1 - f of the scattering: the
    // first-collision table is weighed against the scattering table by the ratio, so
    // that the thinner medium's scattering a (1 - f) mu_t times the weight is the
    // unreduced scattering a mu_t (times 1 - f_first for a chopped first table)
    tp.pf_scale = (p->phase_first && p->phase)
                      ? (float)((1.0 - p->phase_first->removed) / (1.0 - f))
                      : 1.f;
    DS_CHECK(p->g > -1.f && p->g < 1.f, DS_ERR_INVALID_ARG, "%s: g %g outside (-1, 1)", fn,
             (double)p->g);
    DS_CHECK(std::isfinite(p->irradiance), DS_ERR_INVALID_ARG, "%s: irradiance not finite", fn);
    DS_CHECK(p->light_mode == DS_LIGHT_DIRECTIONAL || p->light_mode == DS_LIGHT_ENVIRONMENT,
             DS_ERR_INVALID_ARG, "%s: unknown light_mode %d", fn, p->light_mode);
    DS_CHECK(p->max_interactions >= 0, DS_ERR_INVALID_ARG, "%s: max_interactions < 0", fn);
    DS_CHECK(p->include_direct == 0 || p->include_direct == 1, DS_ERR_INVALID_ARG,
             "%s: include_direct must be 0 or 1", fn);
    tp.g = p->g;
    tp.irradiance = p->irradiance;
    tp.light_mode = p->light_mode;
    tp.max_interactions = p->max_interactions;
    tp.include_direct = p->include_direct;
    return DS_OK;
}

// The render calls add the direct term themselves: L_s estimates are for records only.
static ds_status render_params(const ds_tracer_params *p, TracerParams &tp, const char *fn)
{
    ds_status st = tracer_params(p, tp, fn);
    if (st)
        return st;
    DS_CHECK(!tp.include_direct, DS_ERR_INVALID_ARG,
             "%s: include_direct is for record estimates; the renderer adds the direct term", fn);
    return DS_OK;
}

static ds_status adaptive_params(const ds_adaptive *a, const char *fn)
{
    DS_CHECK(a, DS_ERR_INVALID_ARG, "%s: adaptive is NULL", fn);
    DS_CHECK(a->batch_spp >= 2 && a->max_spp >= a->batch_spp && a->max_spp <= (1 << 20) &&
                 a->max_spp % a->batch_spp == 0,
             DS_ERR_INVALID_ARG,
             "%s: need 2 <= batch_spp <= max_spp <= 2^20 with max_spp a multiple of batch_spp "
             "(got %d, %d)", fn, a->batch_spp, a->max_spp);
    DS_CHECK(std::isfinite(a->rel) && a->rel > 0.0 && std::isfinite(a->z) && a->z > 0.0,
             DS_ERR_INVALID_ARG, "%s: rel and z must be finite and > 0", fn);
    return DS_OK;
}

static ds_status set_params(const ds_tracer_params *params, const ds_lights *lights, TracerParams &tp,
                     const char *fn)
{
    DS_CHECK(lights && lights->dw, DS_ERR_INVALID_ARG, "%s: NULL light set", fn);
    ds_status st = render_params(params, tp, fn);
    if (st)
        return st;
    DS_CHECK(tp.light_mode == DS_LIGHT_DIRECTIONAL, DS_ERR_INVALID_ARG,
             "%s: the members of a light set are directional lights (light_mode must be "
             "DS_LIGHT_DIRECTIONAL)", fn);
    tp.light_mode = kLightSetMode;
    tp.set_dw = lights->dw;
    tp.set_thr = lights->thr;
    tp.set_m = lights->m;
    return DS_OK;
}

ds_status ds_cloud_majorant(const ds_cloud *c, float *majorant)
{
    DS_CHECK(c && majorant, DS_ERR_INVALID_ARG, "ds_cloud_majorant: NULL argument");
    *majorant = c->majorant;
    return DS_OK;
}

ds_status ds_trace_li(ds_ctx *ctx, const ds_cloud *cloud, const ds_tracer_params *params,
                      const float *pos, const float *view_dir, const float *light_dir, int64_t P,
                      int spp, uint64_t seed, double *mean_out, double *var_out)
{
    DS_CHECK(ctx && cloud && (P == 0 || (pos && view_dir && light_dir && mean_out)),
             DS_ERR_INVALID_ARG, "ds_trace_li: NULL argument");
    DS_CHECK(P >= 0 && P < (int64_t(1) << 40), DS_ERR_INVALID_ARG, "ds_trace_li: P out of range");
    DS_CHECK(spp >= 1 && spp <= (1 << 20), DS_ERR_INVALID_ARG,
             "ds_trace_li: spp %d outside [1, 2^20]", spp);
    TracerParams tp;
    ds_status st = tracer_params(params, tp, "ds_trace_li");
    if (st || P == 0)
        return st;
    DS_HIP(hipSetDevice(ctx->device));
    st = ensure_ws(ctx, sizeof(double) * 2 * (size_t)P * tracer_blocks(spp));
    if (st)
        return st;
    return tracer_li(ctx->stream, cloud, tp, pos, view_dir, light_dir, P, spp, seed,
                     static_cast<double *>(ctx->ws), mean_out, var_out);
}

// Workspace of the progressive estimate: partial sums in ws, the rest carved from cv.
static ds_status adaptive_li(ds_ctx *ctx, const ds_cloud *cloud, const TracerParams &tp,
                             const ds_adaptive *ad, const float *pos, const float *view,
                             const float *light, int64_t P, uint64_t seed, Carve &cv,
                             double *mean, double *var, int32_t *n_out)
{
    const int ahead = tracer_adaptive_ahead(P, ad->batch_spp, ad->max_spp);
    ds_status st = ensure_ws(ctx, sizeof(double) * 2 * (size_t)P * tracer_blocks(ad->batch_spp) *
                                      (size_t)ahead);
    if (st)
        return st;
    uint8_t *active = cv.take<uint8_t>((size_t)P);
    double *sums = cv.take<double>(2 * (size_t)P);
    unsigned long long *left = cv.take<unsigned long long>(1);
    return tracer_li_adaptive(ctx->stream, cloud, tp, pos, view, light, P, ad->batch_spp,
                              ad->max_spp, ahead, ad->rel, ad->z, seed,
                              static_cast<double *>(ctx->ws), active, sums, left, mean, var, n_out,
                              nullptr);
}

static size_t adaptive_ws2(int64_t P) { return (size_t)P * (1 + 2 * sizeof(double)) + 4 * 256; }

ds_status ds_trace_li_adaptive(ds_ctx *ctx, const ds_cloud *cloud, const ds_tracer_params *params,
                               const ds_adaptive *adaptive, const float *pos,
                               const float *view_dir, const float *light_dir, int64_t P,
                               uint64_t seed, double *mean_out, double *var_out,
                               int32_t *spp_out)
{
    DS_CHECK(ctx && cloud && (P == 0 || (pos && view_dir && light_dir && mean_out)),
             DS_ERR_INVALID_ARG, "ds_trace_li_adaptive: NULL argument");
    DS_CHECK(P >= 0 && P <= ((int64_t)1 << 31) - 1, DS_ERR_INVALID_ARG,
             "ds_trace_li_adaptive: P out of range");
    TracerParams tp;
    ds_status st = tracer_params(params, tp, "ds_trace_li_adaptive");
    if (st)
        return st;
    if ((st = adaptive_params(adaptive, "ds_trace_li_adaptive")) || P == 0)
        return st;
    DS_HIP(hipSetDevice(ctx->device));
    if ((st = ensure_ws2(ctx, adaptive_ws2(P))))
        return st;
    Carve cv(ctx->ws2);
    return adaptive_li(ctx, cloud, tp, adaptive, pos, view_dir, light_dir, P, seed, cv, mean_out,
                       var_out, spp_out);
}

ds_status ds_sample_records(ds_ctx *ctx, const ds_cloud *cloud, int64_t N, uint64_t seed,
                            float *pos, float *view_dir, float *light_dir, int32_t *attempts)
{
    DS_CHECK(ctx && cloud && (N == 0 || (pos && view_dir && light_dir)), DS_ERR_INVALID_ARG,
             "ds_sample_records: NULL argument");
    DS_CHECK(N >= 0 && N < (int64_t(1) << 40), DS_ERR_INVALID_ARG,
             "ds_sample_records: N out of range");
    if (N == 0)
        return DS_OK;
    DS_HIP(hipSetDevice(ctx->device));
    return tracer_records(ctx->stream, cloud, N, seed, pos, view_dir, light_dir, attempts);
}

ds_status ds_render_mc(ds_ctx *ctx, const ds_cloud *cloud, const ds_tracer_params *params,
                       const float light_dir[3], const float *ray_o, const float *ray_d,
                       int64_t N, int spp, uint64_t seed, double *mean_out, double *var_out)
{
    DS_CHECK(ctx && cloud && light_dir && (N == 0 || (ray_o && ray_d && mean_out)),
             DS_ERR_INVALID_ARG, "ds_render_mc: NULL argument");
    DS_CHECK(N >= 0 && N < (int64_t(1) << 40), DS_ERR_INVALID_ARG, "ds_render_mc: N out of range");
    DS_CHECK(spp >= 1 && spp <= (1 << 20), DS_ERR_INVALID_ARG,
             "ds_render_mc: spp %d outside [1, 2^20]", spp);
    TracerParams tp;
    ds_status st = render_params(params, tp, "ds_render_mc");
    if (st)
        return st;
    float l[3];
    DS_CHECK(unit_host(light_dir, l), DS_ERR_INVALID_ARG, "ds_render_mc: unusable light_dir");
    if (N == 0)
        return DS_OK;
    DS_HIP(hipSetDevice(ctx->device));
    st = ensure_ws(ctx, sizeof(double) * 2 * (size_t)N * tracer_blocks(spp));
    if (st)
        return st;
    return tracer_render(ctx->stream, cloud, tp, light_dir, ray_o, ray_d, N, spp, seed,
                         static_cast<double *>(ctx->ws), mean_out, var_out);
}

ds_status ds_first_hits(ds_ctx *ctx, const ds_cloud *cloud, const ds_tracer_params *params,
                        const float light_dir[3], const float *ray_o, const float *ray_d,
                        int64_t N, uint64_t seed, uint64_t sample, float *pos, float *view_dir,
                        float *direct, uint8_t *hit)
{
    DS_CHECK(ctx && cloud && light_dir &&
                 (N == 0 || (ray_o && ray_d && pos && view_dir && direct && hit)),
             DS_ERR_INVALID_ARG, "ds_first_hits: NULL argument");
    DS_CHECK(N >= 0 && N < (int64_t(1) << 40), DS_ERR_INVALID_ARG,
             "ds_first_hits: N out of range");
    DS_CHECK(sample < (uint64_t(1) << 20), DS_ERR_INVALID_ARG,
             "ds_first_hits: sample index must be below 2^20");
    TracerParams tp;
    ds_status st = render_params(params, tp, "ds_first_hits");
    if (st)
        return st;
    float l[3];
    DS_CHECK(unit_host(light_dir, l), DS_ERR_INVALID_ARG, "ds_first_hits: unusable light_dir");
    if (N == 0)
        return DS_OK;
    DS_HIP(hipSetDevice(ctx->device));
    return tracer_first_hits(ctx->stream, cloud, tp, light_dir, ray_o, ray_d, N, seed, sample, pos,
                             view_dir, direct, hit);
}

// Training pairs with fixed (ad == NULL) or progressive path counts.
static ds_status make_records(ds_ctx *ctx, const ds_cloud *cloud, const ds_tracer_params *params,
                              const ds_adaptive *ad, int64_t N, int spp, uint64_t seed,
                              int64_t stride, float *z, float *target_log1p, float *pos,
                              float *view_dir, float *light_dir, double *li_mean, double *li_var,
                              int32_t *spp_out, const char *fn)
{
    DS_CHECK(ctx && cloud && (N == 0 || (z && target_log1p)), DS_ERR_INVALID_ARG,
             "%s: NULL argument", fn);
    DS_CHECK(N >= 0 && N <= ((int64_t)1 << 31) - 1, DS_ERR_INVALID_ARG, "%s: N out of range", fn);
    DS_CHECK(stride >= 1, DS_ERR_INVALID_ARG, "%s: stride must be >= 1", fn);
    TracerParams tp;
    ds_status st = tracer_params(params, tp, fn);
    if (st)
        return st;
    if (ad) {
        if ((st = adaptive_params(ad, fn)))
            return st;
    } else {
        DS_CHECK(spp >= 1 && spp <= (1 << 20), DS_ERR_INVALID_ARG, "%s: spp %d outside [1, 2^20]",
                 fn, spp);
    }
    DS_CHECK(tp.light_mode == DS_LIGHT_DIRECTIONAL, DS_ERR_INVALID_ARG,
             "%s: records need a directional light", fn);
    if (N == 0)
        return DS_OK;
    DS_HIP(hipSetDevice(ctx->device));
    st = ensure_ws2(ctx, 3 * 3 * sizeof(float) * (size_t)N + 2 * sizeof(double) * (size_t)N +
                             5 * 256 + (ad ? adaptive_ws2(N) : 0));
    if (st)
        return st;
    Carve cv(ctx->ws2);
    float *p = pos ? pos : cv.take<float>(3 * (size_t)N);
    float *v = view_dir ? view_dir : cv.take<float>(3 * (size_t)N);
    float *l = light_dir ? light_dir : cv.take<float>(3 * (size_t)N);
    double *m = li_mean ? li_mean : cv.take<double>((size_t)N);
    hipStream_t s = ctx->stream;
    st = tracer_records(s, cloud, N, seed, p, v, l, nullptr);
    if (st)
        return st;
    if (ad) {
        st = adaptive_li(ctx, cloud, tp, ad, p, v, l, N, derived_key(seed, 0), cv, m, li_var,
                         spp_out);
    } else {
        st = ensure_ws(ctx, sizeof(double) * 2 * (size_t)N * tracer_blocks(spp));
        if (st)
            return st;
        st = tracer_li(s, cloud, tp, p, v, l, N, spp, derived_key(seed, 0),
                       static_cast<double *>(ctx->ws), m, li_var);
    }
    if (st)
        return st;
    st = gather_cells(ctx, cloud);
    if (st)
        return st;
    GatherArgs ga;
    gather_args(cloud, p, v, l, N, ga);
    st = gather_plain(s, ga, 0, N, DS_F32, z, (int64_t)(kStencil * cloud->K + 1) * stride,
                      nullptr);
    if (st)
        return st;
    return tracer_targets(s, m, N, stride, target_log1p);
}

ds_status ds_make_records(ds_ctx *ctx, const ds_cloud *cloud, const ds_tracer_params *params,
                          int64_t N, int spp, uint64_t seed, int64_t stride, float *z,
                          float *target_log1p, float *pos, float *view_dir, float *light_dir,
                          double *li_mean, double *li_var)
{
    return make_records(ctx, cloud, params, nullptr, N, spp, seed, stride, z, target_log1p, pos,
                        view_dir, light_dir, li_mean, li_var, nullptr, "ds_make_records");
}

ds_status ds_make_records_adaptive(ds_ctx *ctx, const ds_cloud *cloud,
                                   const ds_tracer_params *params, const ds_adaptive *adaptive,
                                   int64_t N, uint64_t seed, int64_t stride, float *z,
                                   float *target_log1p, float *pos, float *view_dir,
                                   float *light_dir, double *li_mean, double *li_var,
                                   int32_t *spp_out)
{
    return make_records(ctx, cloud, params, adaptive, N, 0, seed, stride, z, target_log1p, pos,
                        view_dir, light_dir, li_mean, li_var, spp_out,
                        "ds_make_records_adaptive");
}

ds_status ds_render_rpnn(ds_ctx *ctx, const ds_cloud *cloud, const ds_net *net,
                         ds_precision precision, const ds_tracer_params *params,
                         const float light_dir[3], const float *ray_o, const float *ray_d,
                         int64_t N, int spp, uint64_t seed, int fallback_spp, double *mean_out,
                         double *var_out, double *direct_out, int64_t *n_fallback)
{
    DS_CHECK(ctx && cloud && net && light_dir && (N == 0 || (ray_o && ray_d && mean_out)),
             DS_ERR_INVALID_ARG, "ds_render_rpnn: NULL argument");
    DS_CHECK(N >= 0 && N <= ((int64_t)1 << 31), DS_ERR_INVALID_ARG,
             "ds_render_rpnn: N out of range");
    DS_CHECK(spp >= 1 && spp <= (1 << 20), DS_ERR_INVALID_ARG,
             "ds_render_rpnn: spp %d outside [1, 2^20]", spp);
    DS_CHECK(fallback_spp >= 0 && fallback_spp <= (1 << 20), DS_ERR_INVALID_ARG,
             "ds_render_rpnn: fallback_spp %d outside [0, 2^20]", fallback_spp);
    DS_CHECK(cloud->K == net->K, DS_ERR_INVALID_ARG,
             "ds_render_rpnn: the cloud has %d stencil levels, the network %d", cloud->K, net->K);
    TracerParams tp;
    ds_status st = render_params(params, tp, "ds_render_rpnn");
    if (st)
        return st;
    DS_CHECK(tp.light_mode == DS_LIGHT_DIRECTIONAL, DS_ERR_INVALID_ARG,
             "ds_render_rpnn: the network predicts radiance from a directional light");
    float l[3];
    DS_CHECK(unit_host(light_dir, l), DS_ERR_INVALID_ARG, "ds_render_rpnn: unusable light_dir");
    if (n_fallback)
        *n_fallback = 0;
    if (N == 0)
        return DS_OK;
    DS_HIP(hipSetDevice(ctx->device));
    const size_t n = (size_t)N;
    st = ensure_ws2(ctx, n * (9 * sizeof(float) + 2 * sizeof(float) + 2 + 5 * sizeof(double)) +
                             16 * 256);
    if (st)
        return st;
    Carve cv(ctx->ws2);
    float *pos = cv.take<float>(3 * n), *view = cv.take<float>(3 * n);
    float *light = cv.take<float>(3 * n);
    float *direct = cv.take<float>(n), *li = cv.take<float>(n);
    uint8_t *hit = cv.take<uint8_t>(n), *flags = cv.take<uint8_t>(n);
    double *li_mc = cv.take<double>(n), *sums = cv.take<double>(2 * n);
    double *dsum = direct_out ? cv.take<double>(2 * n) : nullptr;
    unsigned long long *cnt = cv.take<unsigned long long>(1);
    hipStream_t s = ctx->stream;
    if ((st = tracer_fill3(s, light, N, l)) || (st = tracer_zero(s, sums, 2 * N)) ||
        (dsum && (st = tracer_zero(s, dsum, 2 * N))) ||
        (st = tracer_zero(s, reinterpret_cast<double *>(cnt), 1)))
        return st;
    for (int smp = 0; smp < spp; ++smp) {
        st = tracer_first_hits(s, cloud, tp, l, ray_o, ray_d, N, seed, (uint64_t)smp, pos, view,
                               direct, hit);
        if (st)
            return st;
        st = ds_predict(ctx, cloud, net, precision, pos, view, light, N, li, nullptr, flags);
        if (st)
            return st;
        const double *mc = nullptr;
        if (fallback_spp > 0) {
            st = ensure_ws(ctx, sizeof(double) * 2 * n * tracer_blocks(fallback_spp));
            if (st)
                return st;
            st = tracer_li(s, cloud, tp, pos, view, light, N, fallback_spp,
                           derived_key(seed, 1 + (uint64_t)smp), static_cast<double *>(ctx->ws),
                           li_mc, nullptr, flags, DS_FLAG_FALLBACK);
            if (st)
                return st;
            mc = li_mc;
        }
        st = tracer_accumulate(s, N, hit, direct, li, flags, mc, tp.albedo, tp.irradiance, sums,
                               dsum, n_fallback ? cnt : nullptr);
        if (st)
            return st;
    }
    st = tracer_finish(s, sums, N, spp, mean_out, var_out);
    if (st)
        return st;
    if (direct_out) {
        st = tracer_finish(s, dsum, N, spp, direct_out, nullptr);
        if (st)
            return st;
    }
    if (n_fallback) {
        unsigned long long h = 0;
        DS_HIP(hipMemcpyAsync(&h, cnt, sizeof(h), hipMemcpyDeviceToHost, s));
        DS_HIP(hipStreamSynchronize(s));
        *n_fallback = (int64_t)h;
    }
    return DS_OK;
}

// ---------------------------------------------------------------- phase tables
ds_status ds_phase_build(int32_t n, const double *p, double chop_deg, double *p_out,
                         double *cdf_out, double *removed, double *mean_cos)
{
    DS_CHECK(p, DS_ERR_INVALID_ARG, "ds_phase_build: NULL table");
    DS_CHECK(n >= 3 && n <= 65536, DS_ERR_INVALID_ARG, "ds_phase_build: %d nodes outside 3..65536",
             n);
    DS_CHECK(std::isfinite(chop_deg) && chop_deg >= 0.0 && chop_deg < 180.0, DS_ERR_INVALID_ARG,
             "ds_phase_build: chop angle %g outside [0, 180)", chop_deg);
    for (int i = 0; i < n; ++i)
        DS_CHECK(std::isfinite(p[i]) && p[i] >= 0.0, DS_ERR_INVALID_ARG,
                 "ds_phase_build: value %d is negative or not finite", i);
    const double dth = M_PI / (n - 1);
    std::vector<double> q(p, p + n), f(n);
    auto integral = [&](const std::vector<double> &v) {
        double acc = 0.0;
        for (int i = 0; i < n; ++i)
            f[i] = 2.0 * M_PI * v[i] * std::sin(i * dth);
        for (int i = 0; i + 1 < n; ++i)
            acc += 0.5 * (f[i] + f[i + 1]) * dth;
        return acc;
    };
    const double tot = integral(q);
    DS_CHECK(tot > 0.0, DS_ERR_INVALID_ARG, "ds_phase_build: the table integrates to zero");
    for (double &v : q)
        v /= tot;
    double rem = 0.0;
    if (chop_deg > 0.0) {
        const int ic = (int)std::lround(chop_deg * M_PI / 180.0 / dth);
        for (int i = 0; i < ic && i < n; ++i)
            q[i] = q[ic < n ? ic : n - 1];
        rem = 1.0 - integral(q);
        DS_CHECK(rem < 1.0, DS_ERR_INVALID_ARG, "ds_phase_build: chopping removes everything");
        for (double &v : q)
            v /= 1.0 - rem;
    }
    for (int i = 0; i < n; ++i)
        f[i] = 2.0 * M_PI * q[i] * std::sin(i * dth);
    std::vector<double> c(n, 0.0);
    double g = 0.0;
    for (int i = 0; i + 1 < n; ++i) {
        c[i + 1] = c[i] + 0.5 * (f[i] + f[i + 1]) * dth;
        g += 0.5 * (f[i] * std::cos(i * dth) + f[i + 1] * std::cos((i + 1) * dth)) * dth;
    }
    for (int i = 0; i < n; ++i) {
        if (p_out)
            p_out[i] = q[i];
        if (cdf_out)
            cdf_out[i] = c[i] / c[n - 1];
    }
    if (removed)
        *removed = rem;
    if (mean_cos)
        *mean_cos = g;
    return DS_OK;
}

ds_status ds_phase_create(ds_ctx *ctx, int32_t n, const double *p, double chop_deg,
                          ds_phase **out)
{
    DS_CHECK(ctx && p && out, DS_ERR_INVALID_ARG, "ds_phase_create: NULL argument");
    *out = nullptr;
    std::vector<double> q((size_t)(n > 0 ? n : 0)), c((size_t)(n > 0 ? n : 0));
    double rem = 0.0, g = 0.0;
    ds_status st = ds_phase_build(n, p, chop_deg, q.data(), c.data(), &rem, &g);
    if (st)
        return st;
    std::vector<float> hf(2 * (size_t)n);
    for (int i = 0; i < n; ++i) {
        hf[i] = (float)q[i];
        hf[n + i] = (float)c[i];
    }
    hf[2 * (size_t)n - 1] = 1.f;
    ds_phase *ph = new (std::nothrow) ds_phase;
    DS_CHECK(ph, DS_ERR_OOM, "ds_phase_create: out of host memory");
    ph->ctx = ctx;
    ph->n = n;
    ph->removed = rem;
    ph->mean_cos = g;
    hipError_t e = hipSetDevice(ctx->device);
    if (e == hipSuccess)
        e = hipMalloc(&ph->p, sizeof(float) * 2 * (size_t)n);
    if (e == hipSuccess)
        e = hipMemcpy(ph->p, hf.data(), sizeof(float) * 2 * (size_t)n, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(ph->p);
        delete ph;
        return hip_fail(e, "ds_phase_create");
    }
    ph->cdf = ph->p + n;
    *out = ph;
    return DS_OK;
}

ds_status ds_phase_info(const ds_phase *phase, double *removed, double *mean_cos)
{
    DS_CHECK(phase, DS_ERR_INVALID_ARG, "ds_phase_info: NULL table");
    if (removed)
        *removed = phase->removed;
    if (mean_cos)
        *mean_cos = phase->mean_cos;
    return DS_OK;
}

ds_status ds_phase_destroy(ds_phase *phase)
{
    if (!phase)
        return DS_OK;
    (void)hipSetDevice(phase->ctx->device);
    (void)hipStreamSynchronize(phase->ctx->stream);
    (void)hipFree(phase->p);
    delete phase;
    return DS_OK;
}

// ---------------------------------------------------------------- light sets
ds_status ds_lights_create(ds_ctx *ctx, int32_t m, const float *dirs, const double *irradiance,
                           ds_lights **out)
{
    DS_CHECK(ctx && dirs && irradiance && out, DS_ERR_INVALID_ARG,
             "ds_lights_create: NULL argument");
    *out = nullptr;
    DS_CHECK(m >= 1 && m <= kMaxLights, DS_ERR_INVALID_ARG,
             "ds_lights_create: %d lights outside [1, %d]", m, kMaxLights);
    std::vector<float4> dw((size_t)m);
    for (int j = 0; j < m; ++j) {
        float u[3];
        DS_CHECK(unit_host(dirs + 3 * j, u), DS_ERR_INVALID_ARG,
                 "ds_lights_create: light %d has an unusable direction", j);
        DS_CHECK(std::isfinite(irradiance[j]) && irradiance[j] > 0.0, DS_ERR_INVALID_ARG,
                 "ds_lights_create: light %d has irradiance %g (must be finite and > 0)", j,
                 irradiance[j]);
        dw[j] = make_float4(u[0], u[1], u[2], 0.f);
    }
    std::vector<uint32_t> thr((size_t)m);
    std::vector<double> w((size_t)m);
    light_table(irradiance, m, thr.data(), w.data());
    for (int j = 0; j < m; ++j)
        dw[j].w = (float)w[j];
    ds_lights *L = new (std::nothrow) ds_lights;
    DS_CHECK(L, DS_ERR_OOM, "ds_lights_create: out of host memory");
    L->ctx = ctx;
    L->m = m;
    hipError_t e = hipSetDevice(ctx->device);
    if (e == hipSuccess)
        e = hipMalloc(&L->dw, sizeof(float4) * (size_t)m);
    if (e == hipSuccess)
        e = hipMalloc(&L->thr, sizeof(uint32_t) * (size_t)m);
    if (e == hipSuccess)
        e = hipMemcpy(L->dw, dw.data(), sizeof(float4) * (size_t)m, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(L->thr, thr.data(), sizeof(uint32_t) * (size_t)m, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(L->dw);
        (void)hipFree(L->thr);
        delete L;
        return hip_fail(e, "ds_lights_create");
    }
    *out = L;
    return DS_OK;
}

ds_status ds_light_table(int32_t m, const double *irradiance, uint32_t *thresholds,
                         double *weights)
{
    DS_CHECK(irradiance && thresholds && weights, DS_ERR_INVALID_ARG,
             "ds_light_table: NULL argument");
    DS_CHECK(m >= 1 && m <= kMaxLights, DS_ERR_INVALID_ARG,
             "ds_light_table: %d lights outside [1, %d]", m, kMaxLights);
    for (int j = 0; j < m; ++j)
        DS_CHECK(std::isfinite(irradiance[j]) && irradiance[j] > 0.0, DS_ERR_INVALID_ARG,
                 "ds_light_table: light %d has irradiance %g (must be finite and > 0)", j,
                 irradiance[j]);
    light_table(irradiance, m, thresholds, weights);
    return DS_OK;
}

ds_status ds_lights_destroy(ds_lights *lights)
{
    if (!lights)
        return DS_OK;
    (void)hipSetDevice(lights->ctx->device);
    (void)hipStreamSynchronize(lights->ctx->stream);
    (void)hipFree(lights->dw);
    (void)hipFree(lights->thr);
    delete lights;
    return DS_OK;
}

ds_status ds_render_mc_lights(ds_ctx *ctx, const ds_cloud *cloud, const ds_tracer_params *params,
                              const ds_lights *lights, const float *ray_o, const float *ray_d,
                              int64_t N, int spp, uint64_t seed, double *mean_out,
                              double *var_out)
{
    DS_CHECK(ctx && cloud && (N == 0 || (ray_o && ray_d && mean_out)), DS_ERR_INVALID_ARG,
             "ds_render_mc_lights: NULL argument");
    DS_CHECK(N >= 0 && N < (int64_t(1) << 40), DS_ERR_INVALID_ARG,
             "ds_render_mc_lights: N out of range");
    DS_CHECK(spp >= 1 && spp <= (1 << 20), DS_ERR_INVALID_ARG,
             "ds_render_mc_lights: spp %d outside [1, 2^20]", spp);
    TracerParams tp;
    ds_status st = set_params(params, lights, tp, "ds_render_mc_lights");
    if (st)
        return st;
    if (N == 0)
        return DS_OK;
    DS_HIP(hipSetDevice(ctx->device));
    st = ensure_ws(ctx, sizeof(double) * 2 * (size_t)N * tracer_blocks(spp));
    if (st)
        return st;
    const float unused[3] = {0.f, 0.f, 1.f};
    return tracer_render(ctx->stream, cloud, tp, unused, ray_o, ray_d, N, spp, seed,
                         static_cast<double *>(ctx->ws), mean_out, var_out);
}

ds_status ds_first_hits_lights(ds_ctx *ctx, const ds_cloud *cloud, const ds_tracer_params *params,
                               const ds_lights *lights, int32_t draws, const float *ray_o,
                               const float *ray_d, int64_t N, uint64_t seed, uint64_t sample,
                               float *pos, float *view_dir, float *light_dir, float *weight,
                               float *direct, uint8_t *hit)
{
    DS_CHECK(ctx && cloud &&
                 (N == 0 || (ray_o && ray_d && pos && view_dir && light_dir && weight && direct &&
                             hit)),
             DS_ERR_INVALID_ARG, "ds_first_hits_lights: NULL argument");
    DS_CHECK(draws >= 1 && draws <= kMaxDraws, DS_ERR_INVALID_ARG,
             "ds_first_hits_lights: draws %d outside [1, %d]", draws, kMaxDraws);
    DS_CHECK(N >= 0 && N * (int64_t)draws <= ((int64_t)1 << 31), DS_ERR_INVALID_ARG,
             "ds_first_hits_lights: N * draws above 2^31");
    DS_CHECK(sample < (uint64_t(1) << 20), DS_ERR_INVALID_ARG,
             "ds_first_hits_lights: sample index must be below 2^20");
    TracerParams tp;
    ds_status st = set_params(params, lights, tp, "ds_first_hits_lights");
    if (st)
        return st;
    if (N == 0)
        return DS_OK;
    DS_HIP(hipSetDevice(ctx->device));
    return tracer_first_hits_set(ctx->stream, cloud, tp, draws, ray_o, ray_d, N, seed, sample, pos,
                                 view_dir, light_dir, weight, direct, hit);
}

ds_status ds_render_rpnn_lights(ds_ctx *ctx, const ds_cloud *cloud, const ds_net *net,
                                ds_precision precision, const ds_tracer_params *params,
                                const ds_lights *lights, int32_t draws, const float *ray_o,
                                const float *ray_d, int64_t N, int spp, uint64_t seed,
                                int fallback_spp, double *mean_out, double *var_out,
                                double *direct_out, int64_t *n_fallback)
{
    DS_CHECK(ctx && cloud && net && (N == 0 || (ray_o && ray_d && mean_out)), DS_ERR_INVALID_ARG,
             "ds_render_rpnn_lights: NULL argument");
    DS_CHECK(draws >= 1 && draws <= kMaxDraws, DS_ERR_INVALID_ARG,
             "ds_render_rpnn_lights: draws %d outside [1, %d]", draws, kMaxDraws);
    DS_CHECK(N >= 0 && N * (int64_t)draws <= ((int64_t)1 << 31), DS_ERR_INVALID_ARG,
             "ds_render_rpnn_lights: N * draws above 2^31");
    DS_CHECK(spp >= 1 && spp <= (1 << 20), DS_ERR_INVALID_ARG,
             "ds_render_rpnn_lights: spp %d outside [1, 2^20]", spp);
    DS_CHECK(fallback_spp >= 0 && fallback_spp <= (1 << 20), DS_ERR_INVALID_ARG,
             "ds_render_rpnn_lights: fallback_spp %d outside [0, 2^20]", fallback_spp);
    DS_CHECK(cloud->K == net->K, DS_ERR_INVALID_ARG,
             "ds_render_rpnn_lights: the cloud has %d stencil levels, the network %d", cloud->K,
             net->K);
    TracerParams tp;
    ds_status st = set_params(params, lights, tp, "ds_render_rpnn_lights");
    if (st)
        return st;
    if (n_fallback)
        *n_fallback = 0;
    if (N == 0)
        return DS_OK;
    DS_HIP(hipSetDevice(ctx->device));
    const size_t n = (size_t)N, r = n * (size_t)draws;
    st = ensure_ws2(ctx, r * (11 * sizeof(float) + 1 + sizeof(double)) +
                             n * (sizeof(float) + 1 + 4 * sizeof(double)) + 16 * 256);
    if (st)
        return st;
    Carve cv(ctx->ws2);
    float *pos = cv.take<float>(3 * r), *view = cv.take<float>(3 * r);
    float *light = cv.take<float>(3 * r), *weight = cv.take<float>(r), *li = cv.take<float>(r);
    uint8_t *flags = cv.take<uint8_t>(r);
    double *li_mc = cv.take<double>(r);
    float *direct = cv.take<float>(n);
    uint8_t *hit = cv.take<uint8_t>(n);
    double *sums = cv.take<double>(2 * n);
    double *dsum = direct_out ? cv.take<double>(2 * n) : nullptr;
    unsigned long long *cnt = cv.take<unsigned long long>(1);
    hipStream_t s = ctx->stream;
    if ((st = tracer_zero(s, sums, 2 * N)) || (dsum && (st = tracer_zero(s, dsum, 2 * N))) ||
        (st = tracer_zero(s, reinterpret_cast<double *>(cnt), 1)))
        return st;
    // the fallback estimates L_i per unit irradiance for each drawn direction
    TracerParams dir_tp = tp;
    dir_tp.light_mode = DS_LIGHT_DIRECTIONAL;
    dir_tp.irradiance = 1.f;
    const int64_t R = N * draws;
    for (int smp = 0; smp < spp; ++smp) {
        st = tracer_first_hits_set(s, cloud, tp, draws, ray_o, ray_d, N, seed, (uint64_t)smp, pos,
                                   view, light, weight, direct, hit);
        if (st)
            return st;
        st = ds_predict(ctx, cloud, net, precision, pos, view, light, R, li, nullptr, flags);
        if (st)
            return st;
        const double *mc = nullptr;
        if (fallback_spp > 0) {
            st = ensure_ws(ctx, sizeof(double) * 2 * r * tracer_blocks(fallback_spp));
            if (st)
                return st;
            st = tracer_li(s, cloud, dir_tp, pos, view, light, R, fallback_spp,
                           derived_key(seed, 1 + (uint64_t)smp), static_cast<double *>(ctx->ws),
                           li_mc, nullptr, flags, DS_FLAG_FALLBACK);
            if (st)
                return st;
            mc = li_mc;
        }
        st = tracer_accumulate_set(s, N, draws, hit, direct, li, flags, mc, weight, tp.albedo,
                                   tp.irradiance, sums, dsum, n_fallback ? cnt : nullptr);
        if (st)
            return st;
    }
    st = tracer_finish(s, sums, N, spp, mean_out, var_out);
    if (st)
        return st;
    if (direct_out) {
        st = tracer_finish(s, dsum, N, spp, direct_out, nullptr);
        if (st)
            return st;
    }
    if (n_fallback) {
        unsigned long long h = 0;
        DS_HIP(hipMemcpyAsync(&h, cnt, sizeof(h), hipMemcpyDeviceToHost, s));
        DS_HIP(hipStreamSynchronize(s));
        *n_fallback = (int64_t)h;
    }
    return DS_OK;
}

ds_status ds_philox4x32_10(ds_ctx *ctx, const uint32_t *ctr_key, int64_t n, uint32_t *out)
{
    DS_CHECK(ctx && (n == 0 || (ctr_key && out)), DS_ERR_INVALID_ARG,
             "ds_philox4x32_10: NULL argument");
    DS_CHECK(n >= 0 && n < (int64_t(1) << 40), DS_ERR_INVALID_ARG,
             "ds_philox4x32_10: n out of range");
    if (n == 0)
        return DS_OK;
    DS_HIP(hipSetDevice(ctx->device));
    return philox_blocks(ctx->stream, ctr_key, n, out);
}

}  // extern "C"
