// Internal declarations shared by the host API and the HIP kernels of
// libdeepscatter.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/deepscatter.h"

namespace ds {

// ------------------------------------------------------------------ errors
void set_error(const char *fmt, ...);
ds_status hip_fail(hipError_t e, const char *what);

#define DS_HIP(expr)                                                    \
    do {                                                                \
        hipError_t e_ = (expr);                                         \
        if (e_ != hipSuccess)                                           \
            return ::ds::hip_fail(e_, #expr);                           \
    } while (0)

#define DS_CHECK(cond, code, ...)                                       \
    do {                                                                \
        if (!(cond)) {                                                  \
            ::ds::set_error(__VA_ARGS__);                               \
            return (code);                                              \
        }                                                               \
    } while (0)

constexpr int kStencil = 225;   // 5 x 5 x 9 points per level
constexpr int kMaxLevels = 16;
constexpr int kMaxK = 16;

// ------------------------------------------------------------------ objects
struct Level {
    int nx, ny, nz;          // level dims (ceil(n / 2^i))
    int64_t off;             // offset in the float32 pyramid (elements)
    int64_t cell_off;        // offset in the corner-packed FP16 pyramid (cells)
    int64_t cell32_off;      // offset in the corner-packed float32 pyramid (cells)
    int bd;                  // zero border of the FP16 cells (cells per side, >= 1)
    bool fast;               // bd covers every stencil sample of a point inside the grid box
    float h;                 // voxel size (world units)
};

}  // namespace ds

struct ds_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    // workspace for the plain (materialised-descriptor) form
    void *ws = nullptr;
    size_t ws_bytes = 0;
    // second workspace for calls that chain other calls using the first
    void *ws2 = nullptr;
    size_t ws2_bytes = 0;
    // device: paths of the tracer calls stopped at the bound on tentative collisions
    unsigned long long *truncated = nullptr;
};

struct ds_cloud {
    ds_ctx *ctx = nullptr;
    int nx = 0, ny = 0, nz = 0;
    float sigma_max = 0.f;
    float aabb_min[3] = {0, 0, 0};
    float h0 = 0.f;
    double mean = 0.0;        // mean extinction over non-zero voxels
    int L = 0;
    ds::Level lv[ds::kMaxLevels];
    int K = 0;
    int mips[ds::kMaxK];
    float *pyr = nullptr;      // float32 levels, concatenated
    int64_t pyr_elems = 0;
    // corner-packed float32 levels for the plain gather (8 corners, 32 bytes per cell), built
    // on the first plain-form call; the gather table points at them from then on
    mutable float4 *cells32 = nullptr;
    uint4 *cells = nullptr;    // corner-packed FP16 levels (8 corners per cell)
    int64_t n_cells = 0;
    int64_t n_cells32 = 0;     // cells of the float32 corner-packed levels
    void *tables = nullptr;    // device: GatherLevel[K] then FusedLevel[K]
    float *mu = nullptr;       // extinction sigma_max * d on the base grid (tracer medium)
    // the same extinction corner-packed (8 float32 corners, 32 bytes per cell, zero border),
    // built on the cloud's first tracer call; the tracer reads one cell per lookup
    mutable float4 *mu_cells = nullptr;
    float majorant = 0.f;      // sigma_max * max(d)
};

struct ds_net {
    ds_ctx *ctx = nullptr;
    int K = 0, W = 0, H = 0;
    // 0: the progressive RPNN; 1: an all-at-once MLP on the whole descriptor (the
    // comparison networks of Sec. 7), layer widths in mlp_widths (input 225 K + 1 first,
    // output 1 last), W = the widest layer, H = the number of layers
    int kind = 0;
    std::vector<int> mlp_widths;
    int64_t n_params = 0;
    float *theta = nullptr;       // FP32 master parameters (canonical order), device
    // fused-kernel operands, see fused.hip for the layout
    uint4 *frag_bf16 = nullptr;   // packed weight fragments
    int64_t frag_count = 0;       // number of 16-byte lane entries
    float *vec = nullptr;         // packed biases and the final layer (fp32)
    int64_t vec_count = 0;
    int32_t *fmap = nullptr;      // parameter index of every fragment element (-1: zero)
    int32_t *vmap = nullptr;      // parameter index of every vector entry
    // FP8 form (DS_PREC_FP8): the W x W layers in E4M3 with power-of-two scales, the
    // descriptor layers in BF16 pre-multiplied by their output scale; see fused.hip
    uint4 *frag_fp8 = nullptr;    // packed fragments of the FP8 form (BF16 and E4M3 chunks)
    int64_t frag8_count = 0;
    float *vec8 = nullptr;        // biases and final layer, scaled to the FP8 form's units
    std::vector<int32_t> fp8_exps;  // log2 units of the activations, then matrix exponents
    bool fp8_ready = false;       // FP8 form matches the current parameters
    // training workspace (activations and gradients of one minibatch)
    float *tws = nullptr;
    size_t tws_floats = 0;
    ds_precision train_prec = DS_PREC_F32;  // arithmetic of ds_loss_grad / ds_train_step
};

struct ds_batch {
    ds_ctx *ctx = nullptr;
    const ds_net *net = nullptr;
    int n = 0;
    const ds_cloud *clouds[16] = {};
    int64_t offsets[17] = {};
    int kind = 0, waves = 4, grid = 0;
    float tuned_ms = -1.f;
    // DS_ORDER_SPATIAL: the launch reads points in a spatial order computed per call into
    // perm, with the counting sort's workspace (slot per point, counts per cell, scan sums)
    int order = 0;
    int32_t *perm = nullptr, *slot = nullptr, *counts = nullptr, *sums = nullptr;
    hipStream_t cap_stream = nullptr;  // capture stream (created on first capture)
    hipGraphExec_t exec = nullptr;
};

struct ds_adam {
    ds_net *net = nullptr;
    float lr = 1e-3f, b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    float *m = nullptr;  // first and second moments, FP32
    float *v = nullptr;
    float *grad = nullptr;
    // device: the step count and {lr, 1 - b1^t, 1 - b2^t}, advanced by the step itself, so
    // a captured step replays with the right bias correction and the current rate
    int64_t *steps = nullptr;
    float *state = nullptr;
    hipGraphExec_t exec = nullptr;  // captured training step (ds_train_capture)
};

namespace ds {

// ------------------------------------------------------------------ kernels (launchers)
// cloud.hip
ds_status cloud_mean(hipStream_t s, const void *d, ds_dtype dt, int64_t n, double *sum,
                     int64_t *count);
ds_status cloud_pyramid(hipStream_t s, const void *d, ds_dtype dt, int nx, int ny, int nz,
                        float scale, int L, const Level *lv, float *pyr);
ds_status cloud_pack(hipStream_t s, const float *pyr, int L, const Level *lv, uint4 *cells);
ds_status cloud_pack32(hipStream_t s, const float *pyr, int L, const Level *lv, float4 *cells);

// gather.hip
struct GatherLevel {
    const float4 *cells;  // corner-packed float32 level: cell c = entries 2c, 2c + 1
    int cx, cy;           // cell-grid dims in x and y (level dims + 2)
    float hx, hy, hz;     // clamp bounds of the shifted cell coordinate (level dims + 1)
    float inv_h;          // 1 / h_m
    float step;           // 2^(k-1) / mean  (world units per lattice unit of 1 mfp)
};
struct GatherArgs {
    const float *pos, *view, *light;
    int64_t P;
    float amin[3], amax[3];
    float inv_mean;     // 1 / mean (level-1 scale)
    int K;
    const GatherLevel *lv;  // device table, K entries
};
ds_status gather_plain(hipStream_t s, const GatherArgs &a, int64_t p0, int64_t np, ds_dtype odt,
                       void *z, int64_t ldz, uint8_t *flags);
ds_status mask_invalid(hipStream_t s, const uint8_t *flags, int64_t n, float *out, float *pre);

// mlp.hip: C = act(A1 B1^T + A2 B2^T + g (x) gw + bias + R), row-major, B rows = outputs
struct GemmArgs {
    int M, N;
    const float *A1; int lda1; int K1; const float *B1; int ldb1;
    const float *A2; int lda2; int K2; const float *B2; int ldb2;
    const float *g; int ldg; const float *gw; int ldgw;  // rank-1 term (may be null)
    const float *bias;
    const float *R; int ldr;                           // residual (may be null)
    float *C; int ldc;
    float *pre; int ldpre;                             // pre-activation copy (may be null)
    int relu;
};
ds_status gemm_f32(hipStream_t s, const GemmArgs &a);
// out = max(out, max |x|) over n floats, as the bit pattern of a non-negative float
ds_status amax_into(hipStream_t s, const float *x, int64_t n, unsigned *out);

// train.hip: C (+)= A B with A(m, k) = A[m sam + k sak], B(k, n) = B[k sbk + n sbn]
struct StridedGemm {
    int M, N, K;
    const float *A; int64_t sam, sak;
    const float *B; int64_t sbk, sbn;
    float *C; int64_t ldc;
    int accumulate;
};
// FP32 on the vector units; split_ws (ws_floats floats, may be NULL) enables
// deterministic split-K for products with few output tiles
ds_status gemm_strided(hipStream_t s, const StridedGemm &g, float *split_ws = nullptr,
                       size_t ws_floats = 0);
// same product with operands rounded to BF16 and FP32 accumulation on the matrix
// cores; split_ws (ws_floats floats, may be NULL) enables deterministic split-K.  x3:
// each operand as a BF16 pair hi + lo (lo = the rounding remainder), three products
// hi hi + hi lo + lo hi per step
ds_status gemm_bf16(hipStream_t s, const StridedGemm &g, float *split_ws, size_t ws_floats,
                    bool x3 = false);
int splitk_count(const StridedGemm &g);
ds_status layer_epilogue(hipStream_t s, int M, int N, float *pre, int ldp, const float *gv, int ldg,
                         const float *gw, int ldgw, const float *bias, const float *R, int ldr,
                         float *out, int ldo);
ds_status relu_mask(hipStream_t s, float *x, int ldx, const float *pre, int ldp, int R, int C);
// column sums in a fixed order; scratch holds colsum_scratch(C) floats
ds_status colsum(hipStream_t s, const float *d, int ldd, int R, int C, float *db, float *scratch);
int colsum_scratch(int C);
ds_status loss_head(hipStream_t s, const float *pre, const float *t, int B, float *dpre, float *sq,
                    float *loss);
// one Adam step: the step count and bias corrections advance on the device (state:
// {lr, 1 - b1^t, 1 - b2^t}), then every parameter is updated
ds_status adam_update(hipStream_t s, float *theta, float *m, float *v, const float *grad,
                      int64_t n, float b1, float b2, float eps, int64_t *steps, float *state);
// dst = src (n floats), as a kernel
ds_status copy_f32(hipStream_t s, float *dst, const float *src, int64_t n);

// fused.hip
int fused_tiles(int W);
ds_status fused_prepare(ds_net *net);
ds_status fused_pack_bf16(hipStream_t s, ds_net *net);
struct FusedLevel {
    const uint4 *cells;
    int cx, cy;          // cell-grid dims in x and y (level dims + 2 bd)
    float hi_x, hi_y, hi_z;  // clamp bounds of the shifted cell coordinate (dims + 2 bd - 1)
    float inv_h;
    float step;          // 2^(k-1) / mean
    float shift;         // bd - 1/2: voxel-centred coordinate to cell coordinate
    int fast;            // 1: samples of points inside the grid box need no clamp
};
constexpr int kMaxBatch = 16;  // clouds per fused launch
struct FusedCloud {
    const FusedLevel *lvt;   // device table, K entries
    float amin[3], amax[3];
    float inv_mean;
    int32_t fast;            // every stencil level's border holds points inside the box
    int64_t p_begin;         // first point of this cloud in the point arrays
    int64_t P;               // its point count
    int64_t tile_begin;      // first tile (set by the launcher for its tile size)
};
// Kernel arguments: the per-cloud records travel in the argument block, so the
// kernel reads them with scalar loads.
struct FusedArgs {
    const float *pos, *view, *light;
    float *out, *pre;
    uint8_t *flags;
    // NULL, or the point row read (and written) at each position of the launch: a
    // permutation that keeps every cloud's range (see batch_order)
    const int32_t *perm;
    int K, W, H;
    int n_clouds;
    int64_t n_tiles;
    FusedCloud cl[kMaxBatch];
};
// Kernel variant of the fused prediction: kind (register-resident residual stream,
// or LDS-resident with cross-chunk pipelining), waves per workgroup (16 points each)
// and grid (0: one workgroup per tile; else that many persistent workgroups).
struct FusedVariant {
    int kind, waves, grid;
};
bool fused_variant_ok(const ds_net *net, const FusedVariant &v);
// precision DS_PREC_BF16 or DS_PREC_FP8 (the latter needs net->fp8_ready)
ds_status fused_predict(hipStream_t s, const ds_net *net, const FusedArgs &a,
                        const FusedVariant &v, ds_precision precision);
bool fused_variant_ok_fp8(const ds_net *net, const FusedVariant &v);
// Number of log2 scales of the FP8 form: K + 1 + (H - 1) activation units (F of every
// block, the residual stream, the dense trailing layers), then (K - 1) + K + (H - 1)
// matrix exponents (W1 of blocks 2..K, W2 of every block, the dense trailing layers).
int fp8_exp_count(int K, int H);
// Build the FP8 form from host parameters and the activation maxima of a calibration
// pass (same order as the activation scales), and upload it.
ds_status fused_quantize_fp8(ds_net *net, const float *theta_host, const float *act_amax);
// Host encoder: x * 2^e to OCP E4M3 (round to nearest even, saturating at 448).
uint8_t e4m3_encode(float x);
ds_status fused_gather_packed(hipStream_t s, const FusedArgs &a, float *z);
// order.hip: spatial order of a batch (cells of a 2^kOrderBits-per-axis grid over each
// cloud's box, Morton order); perm and slot hold `total` entries, counts
// order_buckets(n_clouds), sums order_sums(n_clouds)
constexpr int kOrderBits = 5;
constexpr int kOrderBuckets = 1 << (3 * kOrderBits);
int64_t order_buckets(int n_clouds);
int64_t order_sums(int n_clouds);
ds_status batch_order(hipStream_t s, const FusedArgs &a, int64_t total, int32_t *perm,
                      int32_t *slot, int32_t *counts, int32_t *sums);

// tracer.hip
// light_mode 0: one directional light; 1: uniform environment; 2: a light set, one
// member drawn per next-event estimate (set_dw: unit direction and weight per light,
// set_thr: selection thresholds on the top 24 bits of a uniform, both device arrays).
constexpr int kLightSetMode = 2;
struct TracerParams {
    float albedo, g, irradiance;
    int light_mode, max_interactions;
    int include_direct = 0;  // record estimates of L_s = L_d + L_i instead of L_i
    // tabulated phase functions (device, n values at theta_i = i pi / (n - 1) and the
    // normalised CDF of theta at the same nodes); ph_n = 0: Henyey-Greenstein with g.
    // The first-collision table (pf) serves the direct term of camera rays only.
    const float *ph_p = nullptr, *ph_cdf = nullptr;
    int ph_n = 0;
    const float *pf_p = nullptr, *pf_cdf = nullptr;
    int pf_n = 0;
    // weight of the first-collision table against a chopped scattering table that removed
    // the fraction f: 1 / (1 - f), so that albedo x weight is the unreduced medium's
    // scattering over the reduced extinction
    float pf_scale = 1.f;
    // extinction scale of the medium (1 - a f with a chopped table, else 1); albedo above is
    // then the thinner medium's a (1 - f) / (1 - a f)
    float ext_scale = 1.f;
    const float4 *set_dw = nullptr;
    const uint32_t *set_thr = nullptr;
    int set_m = 0;
};
bool unit_host(const float *v, float *u);  // normalise a host 3-vector; false if unusable
ds_status tracer_prepare(ds_cloud *c, const void *density, ds_dtype dt);
int tracer_blocks(int spp);  // partial sums per record
// mask: when not NULL, only records with (mask[i] & mask_bits) == mask_bits are traced
// (the others get 0)
ds_status tracer_li(hipStream_t s, const ds_cloud *c, const TracerParams &tp, const float *pos,
                    const float *view, const float *light, int64_t P, int spp, uint64_t seed,
                    double *partial, double *mean, double *var, const uint8_t *mask = nullptr,
                    uint8_t mask_bits = 0);
// Progressive estimates: batches of `batch` paths per active record until
// zq * sqrt(var of mean) <= rel * |mean| or max_spp (a multiple of batch) paths; a round
// traces up to `ahead` batches of the records still running (tracer_adaptive_ahead) and
// checks the rule after each in order.  Workspace: partial (2 * P * tracer_blocks(batch) *
// ahead doubles), active (P bytes), sums (2 P doubles), left (one counter).  Synchronises
// once per round; rounds (may be NULL) gets the round count.
ds_status tracer_li_adaptive(hipStream_t s, const ds_cloud *c, const TracerParams &tp,
                             const float *pos, const float *view, const float *light, int64_t P,
                             int batch, int max_spp, int ahead, double rel, double zq,
                             uint64_t seed, double *partial, uint8_t *active, double *sums,
                             unsigned long long *left, double *mean, double *var, int32_t *n_out,
                             int *rounds);
int tracer_adaptive_ahead(int64_t P, int batch, int max_spp);
ds_status tracer_targets(hipStream_t s, const double *li, int64_t N, int64_t stride, float *t);
ds_status tracer_accumulate(hipStream_t s, int64_t N, const uint8_t *hit, const float *direct,
                            const float *li_net, const uint8_t *flags, const double *li_mc,
                            float albedo, float E, double *sums, double *dsum,
                            unsigned long long *n_fb);
ds_status tracer_fill3(hipStream_t s, float *v, int64_t N, const float *xyz);
ds_status tracer_zero(hipStream_t s, double *v, int64_t n);
ds_status tracer_finish(hipStream_t s, const double *sums, int64_t N, int spp, double *mean,
                        double *var);
ds_status tracer_records(hipStream_t s, const ds_cloud *c, int64_t N, uint64_t seed, float *pos,
                         float *view, float *light, int32_t *attempts);
ds_status tracer_render(hipStream_t s, const ds_cloud *c, const TracerParams &tp,
                        const float *light_dir, const float *ray_o, const float *ray_d, int64_t N,
                        int spp, uint64_t seed, double *partial, double *mean, double *var);
ds_status tracer_first_hits(hipStream_t s, const ds_cloud *c, const TracerParams &tp,
                            const float *light_dir, const float *ray_o, const float *ray_d,
                            int64_t N, uint64_t seed, uint64_t sample, float *pos, float *view,
                            float *direct, uint8_t *hit);
ds_status philox_blocks(hipStream_t s, const uint32_t *ctr_key, int64_t n, uint32_t *out);
// Light sets (tp.light_mode == kLightSetMode).  Camera samples: per ray the first
// collision, then `draws` lights, each with one ratio-tracking estimate; rows
// i * draws + q of pos / view / light / weight (pos and view repeated per draw);
// direct = albedo * E * mean over draws of weight * p * T.
ds_status tracer_first_hits_set(hipStream_t s, const ds_cloud *c, const TracerParams &tp,
                                int draws, const float *ray_o, const float *ray_d, int64_t N,
                                uint64_t seed, uint64_t sample, float *pos, float *view,
                                float *light, float *weight, float *direct, uint8_t *hit);
// Pixel sums of one camera sample under a light set: direct + albedo * E * mean over the
// draws of weight * L_i (network, or li_mc where the row's fallback flag is set).
ds_status tracer_accumulate_set(hipStream_t s, int64_t N, int draws, const uint8_t *hit,
                                const float *direct, const float *li_net, const uint8_t *flags,
                                const double *li_mc, const float *weight, float albedo, float E,
                                double *sums, double *dsum, unsigned long long *n_fb);

}  // namespace ds
