/*
 * deepscatter.h - C ABI of the MI355X (gfx950) radiance-prediction library.
 *
 * The library implements the per-shading-point hot path of Kallweit et al.,
 * "Deep Scattering: Rendering Atmospheric Clouds with Radiance-Predicting Neural
 * Networks": a hierarchical, light-oriented stencil descriptor gathered from a
 * Gaussian mipmap of the cloud density (Sec. 4.2, Sec. 6 "Implementation"), fed
 * progressively into a residual radiance-predicting network (Sec. 4.3, Fig. 6),
 * plus the Monte Carlo path tracer that produces its training data (Sec. 3.2,
 * Sec. 5.1) and the training step (Sec. 5.2).
 *
 * Conventions (all calls):
 *  - Every call returns a ds_status; DS_OK is 0 and every error is negative.
 *    ds_last_error() returns a thread-local message for the last failure.
 *    Nothing aborts and no exception crosses the ABI.  Argument checks happen
 *    before anything is enqueued; a failed call leaves its outputs untouched.
 *  - "device" pointers are HIP device memory owned by the caller, "host"
 *    pointers are ordinary host memory.  The library never keeps a caller
 *    pointer beyond the call.
 *  - Work is enqueued asynchronously on the context's stream (a caller-owned
 *    hipStream_t passed as void*; NULL is the default stream) unless a call says
 *    it synchronises.  Outputs are valid once the stream reaches that point.
 *  - A call with an item count of 0 does nothing after its argument checks;
 *    its per-item arrays may then be NULL.
 *  - Geometry: density grids are [nz][ny][nx] with x fastest; voxel (i, j, k)
 *    occupies aabb_min + [i, i+1] x [j, j+1] x [k, k+1] * voxel_size (world
 *    units).  Points and directions are float32 arrays of shape [P][3].
 *    view_dir is omega, the direction in which the radiance travels toward the
 *    viewer (the integration in Eq. (1) runs along x - u omega); light_dir is
 *    omega_l, pointing toward the light.  Neither needs unit length.
 *  - A context, and the clouds, networks and optimisers created from it, must
 *    not be used from two threads at once.
 */
#ifndef DEEPSCATTER_H
#define DEEPSCATTER_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ds_status;
#define DS_OK 0
#define DS_ERR_INVALID_ARG (-1)
#define DS_ERR_OOM (-2)
#define DS_ERR_DEVICE (-3)
#define DS_ERR_UNSUPPORTED (-4)
#define DS_ERR_STATE (-5)

typedef enum { DS_F32 = 0, DS_BF16 = 1 } ds_dtype;

/* Arithmetic of the network layers (Sec. 4.3).  DS_PREC_F32: plain form, every layer
 * in FP32 (descriptor materialised, one kernel per layer).  DS_PREC_BF16: fused
 * kernel, every layer's inputs and weights in BF16 on the matrix cores.  DS_PREC_FP8:
 * fused kernel with the W x W layers (W1, W2 of every block and the dense trailing
 * layers) in FP8 E4M3 (OCP) with power-of-two per-layer scales and the descriptor
 * layers V^k in BF16 (see ds_net_quantize).  Accumulation, biases and residual sums
 * are FP32 in every form. */
typedef enum { DS_PREC_F32 = 0, DS_PREC_BF16 = 1, DS_PREC_FP8 = 2 } ds_precision;

/* Per-point flag bits written by ds_gather / ds_predict. */
#define DS_FLAG_INVALID 1u  /* non-finite position or zero/non-finite direction: outputs are 0 */
#define DS_FLAG_OUTSIDE 2u  /* the point lies outside the grid box                           */
#define DS_FLAG_FALLBACK 4u /* the level-1 stencil box (from (-1,-1,-1) to (1,1,3) mean free
                               paths in the light frame) is not entirely inside the grid box  */

typedef struct ds_ctx ds_ctx;
typedef struct ds_cloud ds_cloud;
typedef struct ds_net ds_net;
typedef struct ds_adam ds_adam;

/* Message of the last failed call on this thread ("" if none). */
const char *ds_last_error(void);

/* Library version string. */
const char *ds_version(void);

/* ---------------------------------------------------------------- context */
/* Create a context on HIP device `device`, enqueueing on `hip_stream`
 * (a hipStream_t, or NULL for the default stream).  The stream stays owned by
 * the caller and must outlive the context. */
ds_status ds_create(int device, void *hip_stream, ds_ctx **out);
/* Change the stream of an existing context. */
ds_status ds_set_stream(ds_ctx *ctx, void *hip_stream);
/* Wait for all work on the context's stream. */
ds_status ds_synchronize(ds_ctx *ctx);
/* Destroy a context; clouds and networks created from it must be destroyed first. */
ds_status ds_destroy(ds_ctx *ctx);

/* ---------------------------------------------------------------- cloud (Sec. 4.2, 5, 6) */
/* Build the per-cloud state from a caller-owned device density grid d in [0, 1]
 * (dtype DS_F32 or DS_BF16) of nx*ny*nz voxels.  Extinction is
 * mu_t = sigma_max * d per world unit.  The call
 *  - computes the mean extinction over all voxels with mu_t > 0 (one mean free
 *    path = 1 / that mean; Sec. 4.2) and the scaled density rho = mu_t / mean;
 *  - builds n_levels mip levels, level i filtered with a Gaussian of standard
 *    deviation 2^i base voxels (Sec. 6), truncated at 3 sigma, zero outside the
 *    grid, sampled at the centres of voxels 2^i times larger
 *    (ceil(n / 2^i) per axis);
 *  - records which mip level stencil level k (1..K) reads: mip_of_level[k-1],
 *    or, when mip_of_level is NULL, the level whose voxel best matches the
 *    level-1 stencil spacing of half a mean free path, plus k-1, clamped.
 * The density buffer is read during the call only.  The call synchronises the
 * stream once (to read the mean back).  Errors: DS_ERR_INVALID_ARG for bad sizes,
 * n_levels outside 1..16, K outside 1..16, mip entries outside [0, n_levels), or a
 * grid without any positive voxel; DS_ERR_OOM if the pyramid does not fit. */
ds_status ds_cloud_create(ds_ctx *ctx, const void *density_dev, ds_dtype dtype, int nx, int ny,
                          int nz, float sigma_max, const float aabb_min[3], float voxel_size,
                          int n_levels, const int *mip_of_level, int K, ds_cloud **out);
/* Host-side description: mean extinction, level count, per-level dims [L][3] as
 * (nx, ny, nz), stencil-to-mip map [K] and K.  Any output pointer may be NULL. */
ds_status ds_cloud_info(const ds_cloud *cloud, double *mean_mu_t, int *n_levels, int *dims,
                        int *mip_of_level, int *K);
/* Copy mip level `level` (float32, [nz][ny][nx]) into caller device memory. */
ds_status ds_cloud_level(ds_ctx *ctx, const ds_cloud *cloud, int level, float *dst_dev);
ds_status ds_cloud_destroy(ds_cloud *cloud);

/* ---------------------------------------------------------------- network (Sec. 4.3) */
/* K residual blocks of width W, then H trailing layers (H-1 of width W and a
 * final scalar layer), ReLU everywhere.  The canonical parameter vector (float32)
 * holds, for k = 1..K: V^k [W][226] (225 stencil densities of level k, then the
 * angle gamma), W1^k [W][W] (absent for k = 1, whose input o^0 is zero), b1^k [W],
 * W2^k [W][W], b2^k [W]; then per trailing layer its matrix [out][in] and bias.
 * Matrices are row-major [out][in]. */
typedef struct {
    int K; /* 1..16 */
    int W; /* 1..256 */
    int H; /* 1..8 */
} ds_net_desc;

int64_t ds_net_param_count(const ds_net_desc *desc);
ds_status ds_net_create(ds_ctx *ctx, const ds_net_desc *desc, ds_net **out);
/* Upload / read back the FP32 master parameters (host arrays of exactly
 * ds_net_param_count() floats).  set_params also refreshes the BF16 copy and
 * invalidates the FP8 copy; both synchronise the stream. */
/* The comparison networks of Sec. 7 (Fig. 10): a plain MLP fed the whole descriptor
 * (225 K + 1 values) at its first layer, widths[0..n_layers-1] the output widths of its
 * layers (the last must be 1), every layer ReLU(W h + b) including the last, as the RPNN's
 * head.  Parameters: per layer W [out][in] row-major, then b [out].  The result is a
 * ds_net that ds_net_set_params / get_params, ds_forward, ds_loss_grad, ds_train_step,
 * ds_adam_*, ds_net_set_train_precision and ds_predict / ds_render_rpnn in DS_PREC_F32
 * accept; the fused BF16 / FP8 forms, ds_net_quantize and the batch API return
 * DS_ERR_UNSUPPORTED.  1 <= K <= 16, 1 <= n_layers <= 64, widths in 1..1024.  The count
 * function returns -1 for an invalid shape. */
int64_t ds_net_param_count_mlp(int32_t K, int32_t n_layers, const int32_t *widths);
ds_status ds_net_create_mlp(ds_ctx *ctx, int32_t K, int32_t n_layers, const int32_t *widths,
                            ds_net **out);
ds_status ds_net_set_params(ds_net *net, const float *theta_host, int64_t n);
ds_status ds_net_get_params(ds_net *net, float *theta_host, int64_t n);
ds_status ds_net_destroy(ds_net *net);

/* ---------------------------------------------------------------- hot path */
/* Plain-form descriptor (Sec. 4.2): per point the row
 * [Sigma^1 (225) ... Sigma^K (225), gamma] of 225K+1 values, Sigma^k_n the
 * trilinearly interpolated rho of mip level mip_of_level[k-1] at
 * q = x + 2^(k-1)/mean * (o_x X + o_y Y + o_z Z), o the lattice point
 * n = ix + 5 iy + 25 iz, o = (-1 + ix/2, -1 + iy/2, -1 + iz/2), (X, Y, Z) the
 * light frame (Z toward the light, X = normalize(omega x omega_l), Y = Z x X) and
 * gamma = acos(omega . omega_l) in radians.  Voxel-centred interpolation, zero
 * outside each level's grid.  z_out is device memory of P*(225K+1) elements of
 * out_dtype; flags (device, P bytes) may be NULL. */
ds_status ds_gather(ds_ctx *ctx, const ds_cloud *cloud, const float *pos, const float *view_dir,
                    const float *light_dir, int64_t P, ds_dtype out_dtype, void *z_out,
                    uint8_t *flags);

/* The descriptor as the fused kernel gathers it: the same samples as ds_gather,
 * interpolated from the corner-packed FP16 copy of the pyramid (eight corners per
 * 16-byte cell, values rounded to nearest even and saturated at the largest finite
 * FP16 value; the y and z lerps in FP16 arithmetic with the fractions rounded toward
 * zero, the x lerp in FP32), written as float32 rows of 225K+1 values in ds_gather's
 * order.  For checking the fused path; z_out is device memory of P*(225K+1) floats. */
ds_status ds_gather_packed(ds_ctx *ctx, const ds_cloud *cloud, const float *pos,
                           const float *view_dir, const float *light_dir, int64_t P,
                           float *z_out);

/* Network on materialised descriptors z (device, [P][225K+1] float32):
 * out[p] = g(z_p) (the predicted L_i per unit irradiance) and, if pre_out is not
 * NULL, the final layer's pre-activation.  FP32 plain form. */
ds_status ds_forward(ds_ctx *ctx, const ds_net *net, const float *z, int64_t P, float *out,
                     float *pre_out);

/* The hot path: for P shading points, the descriptor of `cloud` (K levels of the
 * cloud must equal the network's K) and the network prediction of the indirect
 * in-scattered radiance L_i(x, omega) per unit light irradiance (Sec. 4, 4.1).
 * DS_PREC_F32 runs the plain form (descriptor through HBM, FP32 layers, in
 * chunks of at most 65536 points, with library-owned workspace);
 * DS_PREC_BF16 / DS_PREC_FP8 run the fused kernel (descriptor stays on chip).
 * out (device, P floats), pre_out (device, P floats, may be NULL: final
 * pre-activation) and flags (device, P bytes, may be NULL).  Invalid points get
 * out = pre_out = 0.  FP8 needs ds_net_quantize first (else DS_ERR_STATE).
 * The fused forms allocate nothing and never synchronise, so they can be captured in
 * a stream graph.  The plain form does too once ds_predict_reserve has run for the
 * cloud, the context and at least P points; otherwise its first call builds the
 * cloud's float32 corner cells and grows the context workspace (allocating and
 * synchronising the stream). */
ds_status ds_predict(ds_ctx *ctx, const ds_cloud *cloud, const ds_net *net,
                     ds_precision precision, const float *pos, const float *view_dir,
                     const float *light_dir, int64_t P, float *out, float *pre_out,
                     uint8_t *flags);
/* Builds ahead of time what ds_predict on (ctx, cloud, net, precision) with at most P
 * points would otherwise create on first use: for DS_PREC_F32 the cloud's float32
 * corner-packed levels and the context workspace of min(P, 65536) points (about
 * 4 (225 K + 1 + 3 W) + 1 bytes per point); nothing for the fused forms.  Synchronises
 * the stream.  Later ds_predict calls within those bounds allocate nothing and can be
 * captured in a stream graph.  Errors as ds_predict, DS_ERR_OOM if memory runs out. */
ds_status ds_predict_reserve(ds_ctx *ctx, const ds_cloud *cloud, const ds_net *net,
                             ds_precision precision, int64_t P);
/* For callers that cannot allocate device memory (code under stream-graph capture,
 * serving loops, harnesses that forbid hipMalloc): ds_predict in DS_PREC_F32 with the
 * same results, whose descriptor rows, activations and flags live in a scratch area
 * the library holds on every GPU from module load until the process ends (32 MiB per
 * device; chunks of up to floor((32 MiB - 256) / (4 (225 K + 1 + 3 W) + 1) / 64) * 64
 * points, 2880 at K = 10, W = 200).  It calls no hipMalloc, hipFree or other allocating
 * routine and never synchronises.  Arguments as ds_predict.  Errors: as ds_predict;
 * DS_ERR_STATE if the cloud's float32 corner cells do not exist yet (run
 * ds_predict_reserve with DS_PREC_F32 once) or the device has no scratch address;
 * DS_ERR_INVALID_ARG if the network needs more than the scratch for 64 points.  All
 * calls on one GPU share its scratch: calls that overlap in time on one GPU (two
 * streams, two threads) race and must be serialised by the caller. */
ds_status ds_predict_f32_noalloc(ds_ctx *ctx, const ds_cloud *cloud, const ds_net *net,
                                 const float *pos, const float *view_dir, const float *light_dir,
                                 int64_t P, float *out, float *pre_out, uint8_t *flags);

/* ---------------------------------------------------------------- batched prediction */
/* Uneven sets of shading points from several clouds (each with its own pyramid,
 * all with the network's K) in one persistent launch of the fused kernel: the
 * points of every cloud are cut into tiles of 16 * waves points, a tile never
 * spans two clouds, and the workgroups walk the tiles of all clouds.  A batch
 * plan fixes the clouds and the per-cloud point ranges; the arrays are given per
 * call.  Kernel variants: */
#define DS_KERNEL_REGISTER 0  /* residual stream in registers, one chunk of samples in flight */
#define DS_KERNEL_PIPELINED 1 /* residual stream in LDS, the next chunk's samples in flight  */
#define DS_KERNEL_WIDE 2      /* one wave per SIMD with two 16-point tiles (4 waves only)     */
#define DS_KERNEL_TEAMS 3     /* 8 waves as two teams of 4 on 128-point tiles, one weight copy
                               * for both, the second team a fixed number of weight chunks
                               * behind the first (8 waves only, W <= 240, an even number
                               * of weight chunks per tile)                                    */
typedef struct ds_batch ds_batch;

/* n_clouds (1..16) clouds; the points of cloud c are rows offsets[c] ..
 * offsets[c+1]-1 of the concatenated point arrays (offsets: host, n_clouds + 1
 * non-decreasing values, offsets[0] = 0).  The plan keeps the cloud and network
 * handles (they must outlive it) and starts with the variant ds_predict uses
 * (DS_KERNEL_REGISTER, 4 waves, one workgroup per tile). */
ds_status ds_batch_create(ds_ctx *ctx, const ds_net *net, int n_clouds,
                          const ds_cloud *const *clouds, const int64_t *offsets, ds_batch **out);
ds_status ds_batch_destroy(ds_batch *batch);
/* Kernel variant of the plan: kernel DS_KERNEL_*, waves 4 or 8 (8 needs W <= 240 for
 * DS_KERNEL_REGISTER, W <= 192 for DS_KERNEL_PIPELINED and is not available for
 * DS_KERNEL_WIDE; DS_KERNEL_TEAMS takes 8 only),
 * grid 0 (one workgroup per tile) or the number of persistent workgroups.
 * Setting a variant drops a captured graph. */
ds_status ds_batch_set_config(ds_batch *batch, int32_t kernel, int32_t waves, int32_t grid);
/* Current variant and, after ds_batch_autotune, its measured time in ms (else -1). */
ds_status ds_batch_get_config(const ds_batch *batch, int32_t *kernel, int32_t *waves,
                              int32_t *grid, float *ms);
/* Prediction for all clouds of the plan: as ds_predict per cloud, on the
 * concatenated arrays (device, offsets[n] points).  DS_PREC_BF16 (and DS_PREC_FP8
 * once quantised, register and two-team kernels only: DS_ERR_UNSUPPORTED for the
 * others) runs
 * one launch; DS_PREC_F32 runs the plain form per cloud. */
ds_status ds_batch_predict(ds_batch *batch, ds_precision precision, const float *pos,
                           const float *view_dir, const float *light_dir, float *out,
                           float *pre_out, uint8_t *flags);
/* Times every available variant (kernel x waves x grid in {one per tile, 1, 2, 4
 * workgroups per compute unit}; for DS_PREC_FP8 the register and two-team kernels') on
 * these arrays: one warm-up launch each, then three rounds that time `reps` launches of
 * every variant in turn; a variant's time is its fastest round (the rounds interleave, so
 * a clock that drifts during the sweep favours no variant).  Keeps the fastest variant and
 * drops a captured graph.  Synchronises; writes out.  Results depend on the arrays'
 * contents only through timing. */
ds_status ds_batch_autotune(ds_batch *batch, ds_precision precision, const float *pos,
                            const float *view_dir, const float *light_dir, float *out, int reps);
/* Records the plan's launch for these arrays into a HIP graph (captured on a
 * stream of the plan's own) and instantiates it; ds_batch_replay enqueues the
 * graph on the context's stream.  The arrays must stay valid while the graph is
 * replayed.  Fused precisions only (DS_ERR_UNSUPPORTED for DS_PREC_F32). */
ds_status ds_batch_capture(ds_batch *batch, ds_precision precision, const float *pos,
                           const float *view_dir, const float *light_dir, float *out,
                           float *pre_out, uint8_t *flags);
ds_status ds_batch_replay(ds_batch *batch);
/* Point order of the plan's fused launches (not of its arrays: outputs always follow the
 * input rows).  DS_ORDER_INPUT (the default) cuts each cloud's rows into tiles as given,
 * which suits camera-ordered points.  DS_ORDER_SPATIAL first sorts each cloud's points,
 * on the device and on every call, by the cell of a 32^3 grid over the cloud's box that
 * holds their position, cells in Morton order (a counting sort; points outside the box or
 * with a non-finite position go to the nearest cell), so that a tile holds neighbouring
 * points whose stencils share pyramid cells; the launch then reads and writes each point
 * through that permutation.  Results are bitwise those of DS_ORDER_INPUT: a point's
 * prediction does not depend on its tile.  The sort adds four small launches and a
 * workspace of 8 bytes per point plus 128 KiB per cloud, allocated here (so later calls,
 * captures included, allocate nothing); capture records the sort with the launch.
 * Synchronises the context stream and drops a captured graph when the order changes. */
#define DS_ORDER_INPUT 0
#define DS_ORDER_SPATIAL 1
ds_status ds_batch_set_order(ds_batch *batch, int32_t order);

/* ---------------------------------------------------------------- FP8 form */
/* Builds the network's FP8 form from its current parameters (precision must be
 * DS_PREC_FP8).  Calibration: the P_cal points (device, as for ds_predict) of `cloud`
 * run through the FP32 plain form, recording the largest activation of every layer.
 * Each scaled tensor gets the power of two 2^e, e the largest integer with
 * amax * 2^e <= 448 (clamped to -32..32; 0 for an all-zero tensor): weights per matrix,
 * activations per layer (the first layer of every block, one scale for the residual
 * stream, the dense trailing layers).  Weights are encoded as E4M3(w * 2^e), round to
 * nearest even, saturating; activations the same way inside the kernel, saturating at
 * 448 (inputs beyond the calibrated range are clamped).  The descriptor layers V^k stay
 * BF16.  Synchronises the stream; a later parameter change (ds_net_set_params,
 * ds_train_step) drops the FP8 form until the next call. */
ds_status ds_net_quantize(ds_ctx *ctx, ds_net *net, const ds_cloud *cloud,
                          ds_precision precision, const float *pos, const float *view_dir,
                          const float *light_dir, int64_t P_cal);
/* The exponents e of the FP8 form (host array of exactly 3K + 2H - 2 entries): the
 * activation scales (first layer of blocks 1..K, residual stream, dense trailing layers
 * 1..H-1), then the weight scales (W1 of blocks 2..K, W2 of blocks 1..K, dense trailing
 * layers 1..H-1).  DS_ERR_STATE without an FP8 form. */
ds_status ds_net_fp8_scales(const ds_net *net, int32_t *log2_scales, int32_t n);
/* The library's host E4M3 encoder, as used for the weights: codes[i] = E4M3(x[i] * 2^e)
 * (OCP E4M3: bias 7, no infinities, 0x7F / 0xFF NaN; round to nearest even;
 * magnitudes from 464 up saturate to 448).  Host arrays; e in -64..64. */
ds_status ds_fp8_e4m3_encode(const float *x, int64_t n, int32_t log2_scale, uint8_t *codes);

/* ---------------------------------------------------------------- training (Sec. 5.2) */
/* Adam (Kingma and Ba; the paper uses the default learning rate and decay rates:
 * lr 1e-3, beta1 0.9, beta2 0.999, eps 1e-8) on the network's FP32 master
 * parameters.  The optimiser owns its moment buffers (FP32, zero-initialised). */
ds_status ds_adam_create(ds_net *net, float lr, float beta1, float beta2, float eps,
                         ds_adam **out);
ds_status ds_adam_destroy(ds_adam *opt);
/* Learning rate of the following updates, captured steps included (moments and step
 * count are kept).  Synchronises the stream. */
ds_status ds_adam_set_lr(ds_adam *opt, float lr);
/* Number of updates applied so far (read from the device; synchronises the stream). */
ds_status ds_adam_steps(const ds_adam *opt, int64_t *t);

/* Arithmetic of ds_loss_grad and ds_train_step: DS_PREC_F32 (default; every GEMM in
 * FP32) or DS_PREC_BF16 (every GEMM on the BF16 matrix cores with FP32 accumulation:
 * descriptors, back-propagated gradients and the operands of the weight-gradient
 * products rounded to BF16 once; the forward products of the W x W layers (W1, W2, the
 * trailing layers; an MLP's hidden layers) with each operand as a BF16 pair hi + lo,
 * lo = x - hi, summed as hi hi + hi lo + lo hi, since their rounding, carried along the
 * residual stream, moves every gradient; bias, residual, ReLU, loss and batch
 * reductions in FP32; the master parameters and Adam stay FP32).  DS_PREC_FP8 gives
 * DS_ERR_UNSUPPORTED. */
ds_status ds_net_set_train_precision(ds_net *net, ds_precision precision);

/* Minibatch loss (1/B) sum_b (log(1 + g(z_b)) - t_b)^2 with t_b = log(1 + L_i) and,
 * if grad_dev is not NULL, its gradient with respect to every parameter in
 * canonical order (FP32, device, ds_net_param_count floats).  z is device memory
 * [B][225K+1] float32 (as ds_gather writes it), target_log1p device [B];
 * loss_dev (device, 1 float) may be NULL.  Reductions over the batch run in a
 * fixed order, so results are bitwise reproducible.  1 <= B <= 2^20. */
ds_status ds_loss_grad(ds_net *net, const float *z, const float *target_log1p, int B,
                       float *loss_dev, float *grad_dev);
/* One training step: loss and gradient as ds_loss_grad, one Adam update of the
 * FP32 master parameters (step count t + 1, bias-corrected moments), then the
 * matrix-core copy of the weights is refreshed on the device.  The step count, the
 * bias corrections and the learning rate live on the device and advance with the
 * step, so the step is kernels only.  Asynchronous. */
ds_status ds_train_step(ds_net *net, ds_adam *opt, const float *z, const float *target_log1p,
                        int B, float *loss_dev);
/* Captures one ds_train_step with these arguments (same buffers, B and loss_dev) into
 * a graph owned by `opt`, replacing an earlier one; nothing runs.  ds_train_replay
 * launches it on the context's stream: each replay is one training step on whatever
 * the buffers then hold, bitwise equal to the eager call (ds_adam_set_lr changes the
 * rate of later replays too).  The context must use a created stream, not the default
 * one.  Errors: DS_ERR_STATE if the training workspace for B does not exist yet (run
 * one ds_train_step or ds_loss_grad with B first; growing it allocates) or, for replay,
 * if nothing was captured. */
ds_status ds_train_capture(ds_net *net, ds_adam *opt, const float *z, const float *target_log1p,
                           int B, float *loss_dev);
ds_status ds_train_replay(ds_adam *opt);

/* ---------------------------------------------------------------- Monte Carlo (Sec. 3.2, 4, 5.1) */
/* The medium of every tracer call is the cloud's base grid: extinction
 * mu_t = sigma_max * d, trilinear between voxel centres, zero outside the grid,
 * vacuum outside its box.  Free flights are delta-tracked against the global
 * majorant sigma_max * max(d); transmittance toward the light is ratio-tracked;
 * scattering follows Henyey-Greenstein; at each collision the path survives
 * with probability albedo (absorption by Russian roulette).  Randomness:
 * Philox4x32-10 with key = seed and counter = (stream id low, high, block, 0),
 * uniforms are the top 24 bits of each word times 2^-24; stream ids are stated
 * per call.  Path estimates are FP32; per-record sums are FP64 and reduced in a
 * fixed order, so every result is bitwise reproducible for a given seed.  A path
 * stops after 2^26 tentative collisions (free-flight and transmittance steps
 * together): its estimate keeps what it gathered so far and the context counts it (see
 * ds_tracer_truncated); the estimators of the paper have no such bound. */
#define DS_LIGHT_DIRECTIONAL 0 /* a directional light of irradiance E, next-event estimation */
#define DS_LIGHT_ENVIRONMENT 1 /* a uniform environment of radiance E, counted on escape     */

/* A tabulated phase function (Sec. 3.1 and Sec. 5.1: the paper renders and generates
 * data with a tabulated Lorenz-Mie function whose forward peak is chopped, the density
 * reduced accordingly, and uses the unchopped function for the first scattering event
 * while rendering).  p: host, n values (3 <= n <= 65536, finite, >= 0) at theta_i =
 * i pi / (n - 1) per steradian.  The table is normalised so that the trapezoid rule
 * on 2 pi p sin(theta) gives 1.  chop_deg > 0 holds p below the node nearest
 * chop_deg at that node's value; the fraction f of the scattering that this removes
 * is reported and the rest renormalised.  A chopped table used as
 * ds_tracer_params.phase makes the tracer calls trace the optically thinner medium
 * themselves (see ds_tracer_params).  The tracer
 * evaluates p linearly in theta between nodes and draws theta from the cumulative
 * trapezoid sums, linear density inside a node interval.  ds_phase_build does the
 * host part only: p_out and cdf_out (n doubles each, may be NULL), removed and
 * mean_cos (may be NULL).  ds_phase_create uploads the table (8 bytes per node) to
 * ctx's device. */
typedef struct ds_phase ds_phase;
ds_status ds_phase_build(int32_t n, const double *p, double chop_deg, double *p_out,
                         double *cdf_out, double *removed, double *mean_cos);
ds_status ds_phase_create(ds_ctx *ctx, int32_t n, const double *p, double chop_deg,
                          ds_phase **out);
ds_status ds_phase_info(const ds_phase *phase, double *removed, double *mean_cos);
/* Waits for the context's stream, then frees the table. */
ds_status ds_phase_destroy(ds_phase *phase);

/* Tracer settings.  With a chopped table as `phase` (removed fraction f > 0) every call
 * traces the thinner medium of Sec. 3.1 (the reduced density): extinction times
 * 1 - albedo f, survival probability albedo (1 - f) / (1 - albedo f); the removed peak
 * travels on unscattered.  That albedo is the library's reading (the paper names only
 * the reduced density): the scattering that is left, albedo (1 - f) mu_t, over the
 * thinner extinction.  The network renderers multiply their network term by the same
 * reduced albedo.  Record sampling (ds_sample_records) and the descriptors use the cloud
 * as created. */
typedef struct ds_tracer_params {
    float albedo;         /* single-scattering albedo of the medium, in [0, 1]; the
                             survival probability per collision (reduced as above with
                             a chopped table)                                          */
    float g;              /* HG mean cosine, in (-1, 1)                                   */
    float irradiance;     /* E of the light (DS_LIGHT_DIRECTIONAL) or of the environment */
    int32_t light_mode;   /* DS_LIGHT_DIRECTIONAL or DS_LIGHT_ENVIRONMENT                 */
    int32_t max_interactions; /* path length cap in collisions; 0 = unlimited          */
    int32_t include_direct;   /* 0: estimates of L_i; 1: of all in-scattered radiance L_s =
                                 L_d + L_i (Sec. 7's target ablation): ds_trace_li and the
                                 record calls only, the render calls reject it           */
    const ds_phase *phase;       /* NULL: Henyey-Greenstein with g; else this table for
                                    every scattering and next-event estimate             */
    const ds_phase *phase_first; /* NULL: as phase; else the table for the direct term at
                                    the first collision of camera rays (render calls),
                                    weighted by (1 - f_first) / (1 - f) with f, f_first the
                                    fractions the two tables' chops removed.  Sec. 3.1 uses
                                    the full function at the first bounce; weighing it by
                                    1 / (1 - f) against the thinner medium's scattering
                                    albedo (1 - f) mu_t restores the full scattering
                                    albedo mu_t (the library's reading)                  */
} ds_tracer_params;

/* Number of paths of this context's tracer calls that stopped at the bound of 2^26
 * tentative collisions, since ds_create or the last reset (reset != 0 clears it).
 * Synchronises the stream. */
ds_status ds_tracer_truncated(ds_ctx *ctx, int64_t *count, int reset);

/* The cloud's majorant sigma_max * max(d) (host write). */
ds_status ds_cloud_majorant(const ds_cloud *cloud, float *majorant);

/* Reference estimates of the indirect in-scattered radiance L_i(x, omega) of
 * Sec. 4 (light that reaches x after at least one collision, folded with the
 * phase function; Eq. (1) without its single-scattering term) for P records:
 * per record the mean of spp path estimates (mean_out, device, P doubles) and
 * the variance of that mean (var_out, device, P doubles, may be NULL).  Path s
 * of record i uses stream id i * 2^20 + s.  Records with an unusable direction
 * get 0.  In DS_LIGHT_DIRECTIONAL mode light_dir is omega_l per record; in
 * DS_LIGHT_ENVIRONMENT mode it is ignored but must still be a valid pointer.
 * 1 <= spp <= 2^20, P < 2^40.  Library-owned workspace: 16 * P * ceil(spp/64) bytes. */
ds_status ds_trace_li(ds_ctx *ctx, const ds_cloud *cloud, const ds_tracer_params *params,
                      const float *pos, const float *view_dir, const float *light_dir, int64_t P,
                      int spp, uint64_t seed, double *mean_out, double *var_out);

/* Progressive estimation (Sec. 5.1: paths are drawn until the mean lies within
 * +-rel of the true value at a given confidence).  Per record, batches of batch_spp
 * paths (path s on stream id i * 2^20 + s, as ds_trace_li) until
 * z * sqrt(variance of the mean) <= rel * |mean| after a whole batch, or max_spp
 * paths.  2 <= batch_spp, max_spp a multiple of batch_spp and <= 2^20, rel > 0,
 * z > 0 (1.96 for 95 %). */
typedef struct ds_adaptive {
    int32_t batch_spp;
    int32_t max_spp;
    double rel;
    double z;
} ds_adaptive;

/* ds_trace_li with progressive stopping: mean_out and var_out as ds_trace_li (var_out
 * may be NULL), spp_out (device, P int32, may be NULL) the number of paths used (0
 * for records with an unusable direction).  The estimate of a record that used n
 * paths is the one ds_trace_li gives at spp = n, up to summation order.  When batch_spp
 * is a multiple of 64, a round traces up to k batches at once for the records still
 * running (k grows as they thin out, at most 64): the rule is applied after each batch in
 * order and the paths past a record's stopping batch are discarded, so estimates and path
 * counts are those of one batch per round.  Synchronises once per round.  Library-owned
 * workspace: 16 * P * ceil(batch_spp / 64) * k + 17 * P bytes, k the largest round (1 if
 * batch_spp is not a multiple of 64; its partial sums are kept within 256 MiB). */
ds_status ds_trace_li_adaptive(ds_ctx *ctx, const ds_cloud *cloud, const ds_tracer_params *params,
                               const ds_adaptive *adaptive, const float *pos,
                               const float *view_dir, const float *light_dir, int64_t P,
                               uint64_t seed, double *mean_out, double *var_out,
                               int32_t *spp_out);

/* Training-record configurations (Sec. 5.1): per record a direction d uniform on
 * the sphere, a ray origin uniform over the disc of the box's bounding sphere
 * orthogonal to d, and a delta-tracked free flight along d into the cloud,
 * retried from scratch on escape (at most 10^6 tries; a record that never
 * collides gets NaN positions).  Writes pos (the collision), view_dir = -d and
 * a light direction uniform on the sphere (device, [N][3] float32 each) and,
 * if not NULL, the number of tries (device, N int32).  Record i uses stream id i. */
ds_status ds_sample_records(ds_ctx *ctx, const ds_cloud *cloud, int64_t N, uint64_t seed,
                            float *pos, float *view_dir, float *light_dir, int32_t *attempts);

/* Path-traced pixels (Sec. 4.4 with the network replaced by path estimates):
 * along each camera ray o + t d (device, [N][3] float32 each) a delta-tracked
 * first collision x (escaping rays see 0, or E in DS_LIGHT_ENVIRONMENT mode),
 * then albedo times the in-scattered radiance at x toward -d: direct single
 * scattering by next-event estimation plus L_i for the directional light
 * light_dir (host, 3 floats); all in-scattered environment light in the other
 * mode.  Per pixel the mean of spp samples and the variance of the mean
 * (device doubles; var_out may be NULL).  Sample s of pixel i uses stream id
 * i * 2^20 + s.  Same limits and workspace as ds_trace_li. */
ds_status ds_render_mc(ds_ctx *ctx, const ds_cloud *cloud, const ds_tracer_params *params,
                       const float light_dir[3], const float *ray_o, const float *ray_d,
                       int64_t N, int spp, uint64_t seed, double *mean_out, double *var_out);

/* One camera sample per ray for the network renderer (Sec. 4.4): the
 * delta-tracked first collision along o + t d (pos, device [N][3]), the view
 * direction there (view_dir = -d), the direct single scattering albedo * p *
 * T * E from the directional light light_dir (host, 3 floats) by one
 * ratio-tracking estimate (direct, device N floats), and hit (device N bytes,
 * 1 where the ray collided).  Rays that escape get hit = 0 and zero outputs.
 * Ray i uses stream id i * 2^20 + sample. */
ds_status ds_first_hits(ds_ctx *ctx, const ds_cloud *cloud, const ds_tracer_params *params,
                        const float light_dir[3], const float *ray_o, const float *ray_d,
                        int64_t N, uint64_t seed, uint64_t sample, float *pos, float *view_dir,
                        float *direct, uint8_t *hit);

/* Training pairs (Sec. 5.1, 5.2): N records of `cloud` as ds_sample_records
 * draws them (key seed), their reference L_i per unit irradiance as
 * ds_trace_li estimates it with spp paths (DS_LIGHT_DIRECTIONAL only; its key
 * is derived from seed by a SplitMix64 finaliser, so record and path streams
 * never coincide), the plain FP32 descriptor of each record and the target
 * log(1 + L_i) in FP32.  Record i goes to row i * stride of z (device, rows of
 * 225K+1 floats) and to target_log1p[i * stride] (device), so several calls with
 * offsets 0..stride-1 interleave clouds.  pos / view_dir / light_dir (device
 * [N][3]) and li_mean / li_var (device N doubles: the estimate and the variance
 * of that mean) are written when not NULL.  Records that never collide get a
 * zero row and target 0.  Library-owned workspace as ds_trace_li plus 52 B per
 * record. */
ds_status ds_make_records(ds_ctx *ctx, const ds_cloud *cloud, const ds_tracer_params *params,
                          int64_t N, int spp, uint64_t seed, int64_t stride, float *z,
                          float *target_log1p, float *pos, float *view_dir, float *light_dir,
                          double *li_mean, double *li_var);

/* ds_make_records with each target estimated progressively (ds_trace_li_adaptive's
 * rule, same derived key), as Sec. 5.1 does; spp_out (device, N int32, may be NULL)
 * receives the paths each record used.  Synchronises once per round (rounds and
 * workspace as ds_trace_li_adaptive). */
ds_status ds_make_records_adaptive(ds_ctx *ctx, const ds_cloud *cloud,
                                   const ds_tracer_params *params, const ds_adaptive *adaptive,
                                   int64_t N, uint64_t seed, int64_t stride, float *z,
                                   float *target_log1p, float *pos, float *view_dir,
                                   float *light_dir, double *li_mean, double *li_var,
                                   int32_t *spp_out);

/* Image formation with the network (Sec. 4.4): for each camera ray o + t d
 * (device [N][3] each) and each of spp samples s, a delta-tracked first
 * collision and its direct single scattering as ds_first_hits computes them
 * (sample index s), then radiance = direct + albedo * E * L_i with L_i the
 * network's prediction at `precision` for the directional light light_dir (host,
 * 3 floats).  Where the level-1 stencil leaves the grid (DS_FLAG_FALLBACK) and
 * fallback_spp > 0, L_i comes from fallback_spp path-traced estimates instead
 * (ds_trace_li, key derived from seed and s).  Escaping rays give 0.  Per pixel:
 * the mean over samples (mean_out, device N doubles), the variance of that mean
 * (var_out, may be NULL) and the mean of the direct term alone (direct_out, may
 * be NULL: the renderer without the network).  n_fallback (host, may be NULL)
 * receives the number of (pixel, sample) collisions that used the fallback; it
 * makes the call synchronise.  The cloud's K must equal the network's. */
ds_status ds_render_rpnn(ds_ctx *ctx, const ds_cloud *cloud, const ds_net *net,
                         ds_precision precision, const ds_tracer_params *params,
                         const float light_dir[3], const float *ray_o, const float *ray_d,
                         int64_t N, int spp, uint64_t seed, int fallback_spp, double *mean_out,
                         double *var_out, double *direct_out, int64_t *n_fallback);

/* ---------------------------------------------------------------- light sets
 * A distant emitter (a sun and sky, an environment map) approximated by m
 * directional lights (Sec. 4.4: the renderer handles any distant light by
 * drawing directional samples of it and querying the network once per sample,
 * having been trained for one directional light only).  Member j has a unit
 * direction toward the light and an irradiance E_j > 0.  Every next-event
 * estimate draws one member from the top 24 bits k of one uniform: the first j
 * with k < thr[j], where thr[j] is the running FP64 sum of E up to j divided by
 * the total, times 2^24, rounded half up, then kept at least thr[j-1] + 1 and at
 * most 2^24 - (m - 1 - j) (so thr[m-1] = 2^24 and every member can be drawn).
 * The drawn member's term is weighted by w_j = E_j / p_j with
 * p_j = (thr[j] - thr[j-1]) / 2^24, so one draw is an unbiased estimate of the
 * sum over the set.  params->light_mode must be DS_LIGHT_DIRECTIONAL in the
 * calls below; params->irradiance scales every member. */
typedef struct ds_lights ds_lights;

/* dirs: host [m][3] float32 (normalised here; zero or non-finite rejected);
 * irradiance: host m doubles, finite and > 0; 1 <= m <= 65536.  The set owns a
 * small device table on ctx's device (20 bytes per member), uploaded
 * synchronously. */
ds_status ds_lights_create(ds_ctx *ctx, int32_t m, const float *dirs, const double *irradiance,
                           ds_lights **out);
/* The selection table ds_lights_create builds, on the host (no device needed):
 * thresholds (m uint32) and the FP64 weights w_j (m doubles) of the irradiances
 * (host, m doubles, finite and > 0; 1 <= m <= 65536). */
ds_status ds_light_table(int32_t m, const double *irradiance, uint32_t *thresholds,
                         double *weights);
/* Waits for the context's stream, then frees the set. */
ds_status ds_lights_destroy(ds_lights *lights);

/* Path-traced pixels under a light set: as ds_render_mc in DS_LIGHT_DIRECTIONAL
 * mode, except that the direct term and every next-event estimate of the path
 * draw one member of the set (one uniform, taken just before that estimate's
 * ratio tracking) and weight it by w_j.  Escaping rays see 0.  Same streams,
 * limits and workspace as ds_render_mc. */
ds_status ds_render_mc_lights(ds_ctx *ctx, const ds_cloud *cloud, const ds_tracer_params *params,
                              const ds_lights *lights, const float *ray_o, const float *ray_d,
                              int64_t N, int spp, uint64_t seed, double *mean_out,
                              double *var_out);

/* Camera samples for the network renderer under a light set: per ray the first
 * collision as ds_first_hits, then `draws` members of the set (1 <= draws <=
 * 256), each drawn by one uniform and followed by one ratio-tracking estimate
 * T_q toward it, on the ray's stream in draw order.  Row i * draws + q of pos,
 * view_dir and light_dir (device, [N * draws][3] float32) and of weight (device,
 * N * draws floats) holds the collision, the view direction, the drawn
 * direction and its w_j; direct (device, N floats) = albedo * E * (1 / draws) *
 * sum_q w_q p(d . l_q) T_q; hit (device, N bytes).  Rays that escape get hit = 0
 * and zero rows.  N * draws <= 2^31. */
ds_status ds_first_hits_lights(ds_ctx *ctx, const ds_cloud *cloud, const ds_tracer_params *params,
                               const ds_lights *lights, int32_t draws, const float *ray_o,
                               const float *ray_d, int64_t N, uint64_t seed, uint64_t sample,
                               float *pos, float *view_dir, float *light_dir, float *weight,
                               float *direct, uint8_t *hit);

/* Image formation with the network under a light set (Sec. 4.4, Fig. 7): per
 * camera sample s, the rows of ds_first_hits_lights (sample index s), one
 * prediction per row at `precision` (N * draws points in one ds_predict), and
 * radiance = direct + albedo * E * (1 / draws) * sum_q w_q L_i(x, omega, l_q).
 * Where a row's stencil leaves the grid and fallback_spp > 0, its L_i comes from
 * fallback_spp path-traced estimates per unit irradiance toward l_q (streams as
 * ds_render_rpnn's fallback, over rows).  Outputs, n_fallback (counted per row)
 * and the synchronisation rule as ds_render_rpnn.  Library-owned workspace:
 * about 57 bytes per row plus 41 per pixel, plus the fallback's. */
ds_status ds_render_rpnn_lights(ds_ctx *ctx, const ds_cloud *cloud, const ds_net *net,
                                ds_precision precision, const ds_tracer_params *params,
                                const ds_lights *lights, int32_t draws, const float *ray_o,
                                const float *ray_d, int64_t N, int spp, uint64_t seed,
                                int fallback_spp, double *mean_out, double *var_out,
                                double *direct_out, int64_t *n_fallback);

/* The tracer's random generator itself: for n (counter, key) pairs
 * ctr_key (device, [n][6] uint32: c0 c1 c2 c3 k0 k1) the Philox4x32-10 block
 * (device out, [n][4] uint32), as defined by Salmon et al., SC'11. */
ds_status ds_philox4x32_10(ds_ctx *ctx, const uint32_t *ctr_key, int64_t n, uint32_t *out);

#ifdef __cplusplus
}
#endif
#endif /* DEEPSCATTER_H */
