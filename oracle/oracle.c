/*
 * FP64 CPU oracle for the Deep Scattering radiance-prediction path
 * (Kallweit et al., "Deep Scattering: Rendering Atmospheric Clouds with
 * Radiance-Predicting Neural Networks").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously-correct
 * statement of what the GPU library computes.  It is loaded by the tests, by the
 * smoke check and by the benchmark's CPU-baseline leg, never by the library.  It
 * shares no code, header, table or constant generator with the GPU path.
 *
 * Every function works on host memory in double precision.  Loops run over the
 * indices in increasing order; the only parallelism is an OpenMP loop over
 * independent points / records / levels, which never changes a result.
 *
 * Pinning status of each part (what fixes it other than this code) is listed in
 * the Python wrapper's docstrings and in the tests under tests/test_oracle_*.py.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define DSO_OK 0
#define DSO_ERR_INVALID -1
#define DSO_ERR_OOM -2

#define FLAG_INVALID 1u
#define FLAG_OUTSIDE 2u
#define FLAG_FALLBACK 4u

#define STENCIL_N 225 /* 5 x 5 x 9 points per level (Sec. 4.2) */

/* ------------------------------------------------------------------------------ */
/* density input: float32 (dtype 0) or bfloat16 bit patterns (dtype 1)             */
/* ------------------------------------------------------------------------------ */
static double density_at(const void *d, int dtype, int64_t i)
{
    if (dtype == 0)
        return (double)((const float *)d)[i];
    uint32_t bits = ((uint32_t)((const uint16_t *)d)[i]) << 16;
    float f;
    memcpy(&f, &bits, 4);
    return (double)f;
}

int dso_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void dso_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0)
        omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------------ */
/* O1  Scale normalisation (Sec. 4.2, Sec. 5): mu_t = sigma_max * d; the mean      */
/* extinction over all non-zero voxels defines one mean free path.                 */
/* ------------------------------------------------------------------------------ */
int dso_normalize(const void *dens, int dtype, int nx, int ny, int nz, double sigma_max,
                  double *mean_mu_t, int64_t *count)
{
    if (!dens || nx <= 0 || ny <= 0 || nz <= 0 || !(sigma_max > 0))
        return DSO_ERR_INVALID;
    int64_t n = (int64_t)nx * ny * nz;
    double sum = 0.0;
    int64_t cnt = 0;
#pragma omp parallel for reduction(+ : sum, cnt) schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double mu = sigma_max * density_at(dens, dtype, i);
        if (mu > 0.0) {
            sum += mu;
            cnt += 1;
        }
    }
    if (cnt == 0)
        return DSO_ERR_INVALID;
    *mean_mu_t = sum / (double)cnt;
    *count = cnt;
    return DSO_OK;
}

/* ------------------------------------------------------------------------------ */
/* O2  Gaussian density mipmap (Sec. 6, Implementation): level i is the scaled     */
/* density rho = mu_t / mean convolved with a Gaussian of standard deviation 2^i   */
/* base voxels, truncated at 3 sigma, zero outside the grid, normalised over the   */
/* full (unclipped) kernel lattice, and point-sampled at the centres of voxels     */
/* 2^i times larger.  Each level is filtered directly from the base grid.          */
/* ------------------------------------------------------------------------------ */
static int level_dim(int n, int i)
{
    int64_t s = (int64_t)1 << i;
    int64_t d = ((int64_t)n + s - 1) / s;
    return d < 1 ? 1 : (int)d;
}

int64_t dso_pyramid_layout(int nx, int ny, int nz, int L, int *dims, int64_t *offsets)
{
    int64_t off = 0;
    for (int i = 0; i < L; ++i) {
        int a = level_dim(nx, i), b = level_dim(ny, i), c = level_dim(nz, i);
        if (dims) {
            dims[3 * i + 0] = a;
            dims[3 * i + 1] = b;
            dims[3 * i + 2] = c;
        }
        if (offsets)
            offsets[i] = off;
        off += (int64_t)a * b * c;
    }
    return off;
}

/* 1-D weight of base sample j for level-i sample m (unnormalised), or 0 beyond 3 sigma. */
static double gauss_w(int i, int64_t j, int64_t m)
{
    double s = ldexp(1.0, i);
    double t = ((double)j + 0.5) - ((double)m + 0.5) * s;
    if (fabs(t) > 3.0 * s)
        return 0.0;
    return exp(-t * t / (2.0 * s * s));
}

/* Base-sample index window [j0, j1] that can lie within 3 sigma of level-i sample m. */
static void window(int i, int64_t m, int n, int64_t *j0, int64_t *j1)
{
    double s = ldexp(1.0, i);
    double c = ((double)m + 0.5) * s - 0.5;
    int64_t a = (int64_t)floor(c - 3.0 * s) - 1, b = (int64_t)ceil(c + 3.0 * s) + 1;
    *j0 = a < 0 ? 0 : a;
    *j1 = b > n - 1 ? n - 1 : b;
}

/* Normaliser: sum of the kernel over every lattice offset within 3 sigma, inside the
 * grid or not.  Offsets are integers at level 0 and half-integers above it. */
double dso_gauss_norm(int i)
{
    double s = ldexp(1.0, i);
    double z = 0.0;
    if (i == 0) {
        for (int t = -3; t <= 3; ++t)
            z += exp(-(double)t * t / 2.0);
    } else {
        int64_t h = (int64_t)(3.0 * s);
        for (int64_t k = -h; k < h; ++k) {
            double t = (double)k + 0.5;
            z += exp(-t * t / (2.0 * s * s));
        }
    }
    return z;
}

int dso_pyramid(const void *dens, int dtype, int nx, int ny, int nz, double sigma_max,
                double mean_mu_t, int L, double *out)
{
    if (!dens || !out || L <= 0 || L > 16 || !(mean_mu_t > 0))
        return DSO_ERR_INVALID;
    int64_t nb = (int64_t)nx * ny * nz;
    double *rho = (double *)malloc(sizeof(double) * nb);
    if (!rho)
        return DSO_ERR_OOM;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < nb; ++i)
        rho[i] = sigma_max * density_at(dens, dtype, i) / mean_mu_t;

    int dims[48];
    int64_t offs[16];
    dso_pyramid_layout(nx, ny, nz, L, dims, offs);
    int status = DSO_OK;
    for (int lv = 0; lv < L; ++lv) {
        int mx = dims[3 * lv], my = dims[3 * lv + 1], mz = dims[3 * lv + 2];
        double zn = dso_gauss_norm(lv);
        double *a = (double *)malloc(sizeof(double) * (int64_t)nz * ny * mx);
        double *b = (double *)malloc(sizeof(double) * (int64_t)nz * my * mx);
        if (!a || !b) {
            free(a);
            free(b);
            status = DSO_ERR_OOM;
            break;
        }
        /* pass along x */
#pragma omp parallel for collapse(2) schedule(static)
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int m = 0; m < mx; ++m) {
                    double acc = 0.0;
                    int64_t j0, j1;
                    window(lv, m, nx, &j0, &j1);
                    for (int64_t j = j0; j <= j1; ++j) {
                        double w = gauss_w(lv, j, m);
                        if (w != 0.0)
                            acc += w * rho[((int64_t)z * ny + y) * nx + j];
                    }
                    a[((int64_t)z * ny + y) * mx + m] = acc / zn;
                }
        /* pass along y */
#pragma omp parallel for collapse(2) schedule(static)
        for (int z = 0; z < nz; ++z)
            for (int m = 0; m < my; ++m)
                for (int x = 0; x < mx; ++x) {
                    double acc = 0.0;
                    int64_t j0, j1;
                    window(lv, m, ny, &j0, &j1);
                    for (int64_t j = j0; j <= j1; ++j) {
                        double w = gauss_w(lv, j, m);
                        if (w != 0.0)
                            acc += w * a[((int64_t)z * ny + j) * mx + x];
                    }
                    b[((int64_t)z * my + m) * mx + x] = acc / zn;
                }
        /* pass along z */
        double *o = out + offs[lv];
#pragma omp parallel for collapse(2) schedule(static)
        for (int m = 0; m < mz; ++m)
            for (int y = 0; y < my; ++y)
                for (int x = 0; x < mx; ++x) {
                    double acc = 0.0;
                    int64_t j0, j1;
                    window(lv, m, nz, &j0, &j1);
                    for (int64_t j = j0; j <= j1; ++j) {
                        double w = gauss_w(lv, j, m);
                        if (w != 0.0)
                            acc += w * b[(j * my + y) * mx + x];
                    }
                    o[((int64_t)m * my + y) * mx + x] = acc / zn;
                }
        free(a);
        free(b);
    }
    free(rho);
    return status;
}

/* Default stencil-level -> mip-level rule (the paper leaves it open): the level whose
 * voxel best matches the level-1 stencil spacing of half a mean free path, then one
 * mip level per stencil level, clamped to the pyramid. */
void dso_default_mips(double mean_mu_t, double h0, int K, int L, int *mips)
{
    int delta = (int)floor(log2(0.5 / (mean_mu_t * h0)) + 0.5);
    for (int k = 0; k < K; ++k) {
        int m = k + delta;
        mips[k] = m < 0 ? 0 : (m > L - 1 ? L - 1 : m);
    }
}

/* ------------------------------------------------------------------------------ */
/* O3  Light-oriented local frame (Sec. 4.2): z toward the light, x perpendicular  */
/* to the plane of z and the view direction, y orthogonal to both;                 */
/* gamma = acos(omega . omega_l).                                                  */
/* ------------------------------------------------------------------------------ */
static int unit3(const double v[3], double u[3])
{
    if (!isfinite(v[0]) || !isfinite(v[1]) || !isfinite(v[2]))
        return 0;
    double m = fmax(fabs(v[0]), fmax(fabs(v[1]), fabs(v[2])));
    if (m == 0.0)
        return 0;
    double a = v[0] / m, b = v[1] / m, c = v[2] / m;
    double l = sqrt(a * a + b * b + c * c);
    u[0] = a / l;
    u[1] = b / l;
    u[2] = c / l;
    return 1;
}

static void cross3(const double a[3], const double b[3], double c[3])
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

static double dot3(const double a[3], const double b[3])
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

/* Orthonormal basis around a unit vector n (Duff et al. 2017, branchless form). */
static void onb(const double n[3], double t1[3], double t2[3])
{
    double sign = copysign(1.0, n[2]);
    double a = -1.0 / (sign + n[2]);
    double b = n[0] * n[1] * a;
    t1[0] = 1.0 + sign * n[0] * n[0] * a;
    t1[1] = sign * b;
    t1[2] = -sign * n[0];
    t2[0] = b;
    t2[1] = sign + n[1] * n[1] * a;
    t2[2] = -n[1];
}

/* Returns 0 if the directions are unusable (zero, NaN or infinite). */
int dso_frame(const double *view, const double *light, double *X, double *Y, double *Z,
              double *gamma)
{
    double w[3];
    if (!unit3(view, w) || !unit3(light, Z))
        return 0;
    double xp[3];
    cross3(w, Z, xp);
    double s = sqrt(dot3(xp, xp));
    if (s >= 1e-6) {
        X[0] = xp[0] / s;
        X[1] = xp[1] / s;
        X[2] = xp[2] / s;
    } else {
        double t2[3];
        onb(Z, X, t2);
    }
    cross3(Z, X, Y);
    double c = dot3(w, Z);
    c = c > 1.0 ? 1.0 : (c < -1.0 ? -1.0 : c);
    *gamma = acos(c);
    return 1;
}

/* ------------------------------------------------------------------------------ */
/* O4+O5  Hierarchical stencil and descriptor (Sec. 4.2, Fig. 5).                  */
/* Point n = ix + 5 iy + 25 iz of the 5x5x9 lattice spanning the box from          */
/* (-1,-1,-1) to (1,1,3) mean free paths; level k (1-based) is scaled by 2^(k-1).  */
/* Densities are read from mip level mips[k-1] by voxel-centred trilinear          */
/* interpolation with zero outside the level's grid.                               */
/* Output row: [Sigma^1 (225), ..., Sigma^K (225), gamma].                          */
/* ------------------------------------------------------------------------------ */
static double tri_sample(const double *lv, int mx, int my, int mz, const double u[3])
{
    double f[3];
    int64_t i0[3];
    for (int a = 0; a < 3; ++a) {
        double fl = floor(u[a]);
        i0[a] = (int64_t)fl;
        f[a] = u[a] - fl;
    }
    int64_t dims[3] = {mx, my, mz};
    double acc = 0.0;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                int64_t c[3] = {i0[0] + dx, i0[1] + dy, i0[2] + dz};
                if (c[0] < 0 || c[1] < 0 || c[2] < 0 || c[0] >= dims[0] || c[1] >= dims[1] ||
                    c[2] >= dims[2])
                    continue;
                double w = (dx ? f[0] : 1.0 - f[0]) * (dy ? f[1] : 1.0 - f[1]) *
                           (dz ? f[2] : 1.0 - f[2]);
                acc += w * lv[(c[2] * my + c[1]) * mx + c[0]];
            }
    return acc;
}

void dso_stencil_offset(int n, double o[3])
{
    int ix = n % 5, iy = (n / 5) % 5, iz = n / 25;
    o[0] = -1.0 + 0.5 * ix;
    o[1] = -1.0 + 0.5 * iy;
    o[2] = -1.0 + 0.5 * iz;
}

int dso_gather(const double *pyr, const int *dims, const int64_t *offsets, int L,
               const double *aabb_min, double h0, int nx, int ny, int nz, double mean_mu_t, int K,
               const int *mips, const float *pos, const float *view, const float *light, int64_t P,
               double *zout, uint8_t *flags)
{
    if (!pyr || !dims || !offsets || !mips || K <= 0 || L <= 0 || !(mean_mu_t > 0))
        return DSO_ERR_INVALID;
    for (int k = 0; k < K; ++k)
        if (mips[k] < 0 || mips[k] >= L)
            return DSO_ERR_INVALID;
    const int64_t D = (int64_t)STENCIL_N * K + 1;
    double amax[3] = {aabb_min[0] + nx * h0, aabb_min[1] + ny * h0, aabb_min[2] + nz * h0};
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t p = 0; p < P; ++p) {
        double *z = zout + p * D;
        double x[3] = {pos[3 * p], pos[3 * p + 1], pos[3 * p + 2]};
        double w[3] = {view[3 * p], view[3 * p + 1], view[3 * p + 2]};
        double l[3] = {light[3 * p], light[3 * p + 1], light[3 * p + 2]};
        double X[3], Y[3], Z[3], gamma;
        uint8_t fl = 0;
        int ok = isfinite(x[0]) && isfinite(x[1]) && isfinite(x[2]) && dso_frame(w, l, X, Y, Z, &gamma);
        if (!ok) {
            for (int64_t i = 0; i < D; ++i)
                z[i] = 0.0;
            if (flags)
                flags[p] = FLAG_INVALID;
            continue;
        }
        for (int a = 0; a < 3; ++a)
            if (x[a] < aabb_min[a] || x[a] > amax[a])
                fl |= FLAG_OUTSIDE;
        for (int k = 0; k < K; ++k) {
            double s = ldexp(1.0, k) / mean_mu_t;
            int m = mips[k];
            int mx = dims[3 * m], my = dims[3 * m + 1], mz = dims[3 * m + 2];
            double hm = ldexp(h0, m);
            const double *lv = pyr + offsets[m];
            for (int n = 0; n < STENCIL_N; ++n) {
                double o[3], u[3];
                dso_stencil_offset(n, o);
                for (int a = 0; a < 3; ++a) {
                    double q = x[a] + s * (o[0] * X[a] + o[1] * Y[a] + o[2] * Z[a]);
                    u[a] = (q - aabb_min[a]) / hm - 0.5;
                }
                z[(int64_t)k * STENCIL_N + n] = tri_sample(lv, mx, my, mz, u);
            }
        }
        z[D - 1] = gamma;
        /* fallback: the level-1 stencil box is not entirely inside the grid box */
        double s1 = 1.0 / mean_mu_t;
        for (int c = 0; c < 8; ++c) {
            double o[3] = {(c & 1) ? 1.0 : -1.0, (c & 2) ? 1.0 : -1.0, (c & 4) ? 3.0 : -1.0};
            for (int a = 0; a < 3; ++a) {
                double q = x[a] + s1 * (o[0] * X[a] + o[1] * Y[a] + o[2] * Z[a]);
                if (q < aabb_min[a] || q > amax[a])
                    fl |= FLAG_FALLBACK;
            }
        }
        if (flags)
            flags[p] = fl;
    }
    return DSO_OK;
}

/* ------------------------------------------------------------------------------ */
/* O6  Network forward (Sec. 4.3, Fig. 6).  Parameters in canonical order:          */
/* for k = 1..K: V^k[W][226], W1^k[W][W] (k > 1; o^0 = 0 makes W1^1 void), b1^k[W], */
/* W2^k[W][W], b2^k[W]; then H trailing layers, H-1 of shape [W][W] + bias and a   */
/* final [1][W] + bias.  All matrices row-major [out][in]; f = ReLU everywhere.     */
/* ------------------------------------------------------------------------------ */
int64_t dso_param_count(int K, int W, int H)
{
    int64_t n = 0;
    for (int k = 0; k < K; ++k)
        n += (int64_t)W * 226 + (k ? (int64_t)W * W : 0) + W + (int64_t)W * W + W;
    for (int m = 0; m < H; ++m) {
        int rows = (m == H - 1) ? 1 : W;
        n += (int64_t)rows * W + rows;
    }
    return n;
}

typedef struct {
    int64_t V, W1, b1, W2, b2; /* offsets, W1 = -1 when absent */
} block_off;

static void param_offsets(int K, int W, int H, block_off *blk, int64_t *hw, int64_t *hb)
{
    int64_t off = 0;
    for (int k = 0; k < K; ++k) {
        blk[k].V = off;
        off += (int64_t)W * 226;
        if (k) {
            blk[k].W1 = off;
            off += (int64_t)W * W;
        } else {
            blk[k].W1 = -1;
        }
        blk[k].b1 = off;
        off += W;
        blk[k].W2 = off;
        off += (int64_t)W * W;
        blk[k].b2 = off;
        off += W;
    }
    for (int m = 0; m < H; ++m) {
        int rows = (m == H - 1) ? 1 : W;
        hw[m] = off;
        off += (int64_t)rows * W;
        hb[m] = off;
        off += rows;
    }
}

static double relu(double a) { return a > 0.0 ? a : 0.0; }

/* Activations of one sample, kept for the backward pass. */
typedef struct {
    double *zk;   /* [K][226] block inputs */
    double *h;    /* [K][W]   first-layer pre-activations */
    double *F1;   /* [K][W] */
    double *a;    /* [K][W]   second pre-activations (F2 + o^{k-1}) */
    double *o;    /* [K+1][W] block outputs, o[0] = 0 */
    double *ha;   /* [H][W]   head pre-activations */
    double *ho;   /* [H][W]   head outputs */
} acts;

static void forward_one(const double *th, const block_off *blk, const int64_t *hw,
                        const int64_t *hb, int K, int W, int H, const double *zrow, acts *A)
{
    memset(A->o, 0, sizeof(double) * W);
    for (int k = 0; k < K; ++k) {
        double *zk = A->zk + (int64_t)k * 226;
        for (int n = 0; n < STENCIL_N; ++n)
            zk[n] = zrow[(int64_t)k * STENCIL_N + n];
        zk[225] = zrow[(int64_t)K * STENCIL_N];
        const double *op = A->o + (int64_t)k * W;
        double *h = A->h + (int64_t)k * W, *F1 = A->F1 + (int64_t)k * W;
        double *a = A->a + (int64_t)k * W, *on = A->o + (int64_t)(k + 1) * W;
        for (int r = 0; r < W; ++r) {
            double acc = 0.0;
            const double *vr = th + blk[k].V + (int64_t)r * 226;
            for (int c = 0; c < 226; ++c)
                acc += vr[c] * zk[c];
            if (blk[k].W1 >= 0) {
                const double *wr = th + blk[k].W1 + (int64_t)r * W;
                for (int c = 0; c < W; ++c)
                    acc += wr[c] * op[c];
            }
            acc += th[blk[k].b1 + r];
            h[r] = acc;
            F1[r] = relu(acc);
        }
        for (int r = 0; r < W; ++r) {
            double acc = 0.0;
            const double *wr = th + blk[k].W2 + (int64_t)r * W;
            for (int c = 0; c < W; ++c)
                acc += wr[c] * F1[c];
            acc += th[blk[k].b2 + r];
            a[r] = acc + op[r];
            on[r] = relu(a[r]);
        }
    }
    const double *in = A->o + (int64_t)K * W;
    for (int m = 0; m < H; ++m) {
        int rows = (m == H - 1) ? 1 : W;
        double *ha = A->ha + (int64_t)m * W, *ho = A->ho + (int64_t)m * W;
        for (int r = 0; r < rows; ++r) {
            double acc = 0.0;
            const double *wr = th + hw[m] + (int64_t)r * W;
            for (int c = 0; c < W; ++c)
                acc += wr[c] * in[c];
            acc += th[hb[m] + r];
            ha[r] = acc;
            ho[r] = relu(acc);
        }
        in = ho;
    }
}

static int acts_alloc(acts *A, int K, int W, int H)
{
    size_t n = (size_t)K * 226 + 4 * (size_t)K * W + (size_t)W + 2 * (size_t)H * W;
    double *buf = (double *)calloc(n, sizeof(double));
    if (!buf)
        return 0;
    A->zk = buf;
    A->h = A->zk + (size_t)K * 226;
    A->F1 = A->h + (size_t)K * W;
    A->a = A->F1 + (size_t)K * W;
    A->o = A->a + (size_t)K * W;
    A->ha = A->o + (size_t)(K + 1) * W;
    A->ho = A->ha + (size_t)H * W;
    return 1;
}

int dso_forward(const double *theta, int K, int W, int H, const double *z, int64_t P, double *g,
                double *pre)
{
    if (!theta || !z || !g || K <= 0 || W <= 0 || H <= 0 || K > 64)
        return DSO_ERR_INVALID;
    block_off blk[64];
    int64_t hw[16], hb[16];
    if (H > 16)
        return DSO_ERR_INVALID;
    param_offsets(K, W, H, blk, hw, hb);
    const int64_t D = (int64_t)STENCIL_N * K + 1;
    int err = 0;
#pragma omp parallel
    {
        acts A;
        int ok = acts_alloc(&A, K, W, H);
        if (!ok) {
#pragma omp atomic write
            err = 1;
        }
#pragma omp for schedule(dynamic, 8)
        for (int64_t p = 0; p < P; ++p) {
            if (!ok)
                continue;
            forward_one(theta, blk, hw, hb, K, W, H, z + p * D, &A);
            g[p] = A.ho[(int64_t)(H - 1) * W];
            if (pre)
                pre[p] = A.ha[(int64_t)(H - 1) * W];
        }
        if (ok)
            free(A.zk);
    }
    return err ? DSO_ERR_OOM : DSO_OK;
}

/* ------------------------------------------------------------------------------ */
/* O7  Loss (Sec. 5.2) and its gradient by backpropagation.                         */
/* loss = mean over the batch of (log(1 + g) - t)^2 with t = log(1 + L_i).          */
/* ReLU'(a) = 1 for a > 0 and 0 otherwise.                                          */
/* ------------------------------------------------------------------------------ */
int dso_loss_grad(const double *theta, int K, int W, int H, const double *z,
                  const double *target, int64_t B, double *loss, double *grad)
{
    if (!theta || !z || !target || B <= 0 || K <= 0 || K > 64 || H <= 0 || H > 16)
        return DSO_ERR_INVALID;
    block_off blk[64];
    int64_t hw[16], hb[16];
    param_offsets(K, W, H, blk, hw, hb);
    int64_t NP = dso_param_count(K, W, H);
    const int64_t D = (int64_t)STENCIL_N * K + 1;
    acts A;
    if (!acts_alloc(&A, K, W, H))
        return DSO_ERR_OOM;
    double *dcur = (double *)calloc((size_t)W, sizeof(double)); /* grad wrt current output */
    double *dnext = (double *)calloc((size_t)W, sizeof(double));
    double *da = (double *)calloc((size_t)W, sizeof(double));
    double *dh = (double *)calloc((size_t)W, sizeof(double));
    if (!dcur || !dnext || !da || !dh) {
        free(A.zk);
        free(dcur);
        free(dnext);
        free(da);
        free(dh);
        return DSO_ERR_OOM;
    }
    if (grad)
        memset(grad, 0, sizeof(double) * NP);
    double L = 0.0;
    for (int64_t b = 0; b < B; ++b) {
        forward_one(theta, blk, hw, hb, K, W, H, z + b * D, &A);
        double gv = A.ho[(int64_t)(H - 1) * W];
        double r = log1p(gv) - target[b];
        L += r * r;
        if (!grad)
            continue;
        /* d loss / d g */
        double dg = 2.0 * r / ((double)B * (1.0 + gv));
        /* head, last layer first */
        memset(dcur, 0, sizeof(double) * W);
        dcur[0] = dg;
        for (int m = H - 1; m >= 0; --m) {
            int rows = (m == H - 1) ? 1 : W;
            const double *in = (m == 0) ? A.o + (int64_t)K * W : A.ho + (int64_t)(m - 1) * W;
            const double *ha = A.ha + (int64_t)m * W;
            memset(dnext, 0, sizeof(double) * W);
            for (int rr = 0; rr < rows; ++rr) {
                double d = ha[rr] > 0.0 ? dcur[rr] : 0.0;
                grad[hb[m] + rr] += d;
                for (int c = 0; c < W; ++c) {
                    grad[hw[m] + (int64_t)rr * W + c] += d * in[c];
                    dnext[c] += theta[hw[m] + (int64_t)rr * W + c] * d;
                }
            }
            memcpy(dcur, dnext, sizeof(double) * W);
        }
        /* blocks, last first; dcur = d loss / d o^k */
        for (int k = K - 1; k >= 0; --k) {
            const double *a = A.a + (int64_t)k * W, *h = A.h + (int64_t)k * W;
            const double *F1 = A.F1 + (int64_t)k * W, *op = A.o + (int64_t)k * W;
            const double *zk = A.zk + (int64_t)k * 226;
            for (int r = 0; r < W; ++r)
                da[r] = a[r] > 0.0 ? dcur[r] : 0.0;
            /* o^k = f(W2 F1 + b2 + o^{k-1}) */
            memset(dh, 0, sizeof(double) * W);
            for (int r = 0; r < W; ++r) {
                grad[blk[k].b2 + r] += da[r];
                for (int c = 0; c < W; ++c) {
                    grad[blk[k].W2 + (int64_t)r * W + c] += da[r] * F1[c];
                    dh[c] += theta[blk[k].W2 + (int64_t)r * W + c] * da[r];
                }
            }
            for (int c = 0; c < W; ++c)
                dh[c] = h[c] > 0.0 ? dh[c] : 0.0;
            /* F1 = f(V z + W1 o^{k-1} + b1); residual path passes da to o^{k-1} */
            for (int c = 0; c < W; ++c)
                dnext[c] = da[c];
            for (int r = 0; r < W; ++r) {
                grad[blk[k].b1 + r] += dh[r];
                for (int c = 0; c < 226; ++c)
                    grad[blk[k].V + (int64_t)r * 226 + c] += dh[r] * zk[c];
                if (blk[k].W1 >= 0)
                    for (int c = 0; c < W; ++c) {
                        grad[blk[k].W1 + (int64_t)r * W + c] += dh[r] * op[c];
                        dnext[c] += theta[blk[k].W1 + (int64_t)r * W + c] * dh[r];
                    }
            }
            memcpy(dcur, dnext, sizeof(double) * W);
        }
    }
    if (loss)
        *loss = L / (double)B;
    free(A.zk);
    free(dcur);
    free(dnext);
    free(da);
    free(dh);
    return DSO_OK;
}

/* ------------------------------------------------------------------------------ */
/* O8  Adam (Kingma and Ba 2014, Algorithm 1), as prescribed in Sec. 5.2.          */
/* t is the 1-based step number of this update.                                     */
/* ------------------------------------------------------------------------------ */
void dso_adam(double *theta, double *m, double *v, const double *grad, int64_t n, int64_t t,
              double lr, double b1, double b2, double eps)
{
    double c1 = 1.0 - pow(b1, (double)t);
    double c2 = 1.0 - pow(b2, (double)t);
    for (int64_t i = 0; i < n; ++i) {
        m[i] = b1 * m[i] + (1.0 - b1) * grad[i];
        v[i] = b2 * v[i] + (1.0 - b2) * grad[i] * grad[i];
        double mh = m[i] / c1;
        double vh = v[i] / c2;
        theta[i] -= lr * mh / (sqrt(vh) + eps);
    }
}

/* ------------------------------------------------------------------------------ */
/* Philox4x32-10 counter-based generator (Salmon et al., SC'11).                   */
/* ------------------------------------------------------------------------------ */
void dso_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0;
        c1 = n1;
        c2 = n2;
        c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

/* One random stream per (stream id): key = seed, counter = (id lo, id hi, block, 0). */
typedef struct {
    uint32_t key[2];
    uint32_t ctr[4];
    uint32_t buf[4];
    int used;
} rng_t;

static void rng_init(rng_t *r, uint64_t seed, uint64_t id)
{
    r->key[0] = (uint32_t)seed;
    r->key[1] = (uint32_t)(seed >> 32);
    r->ctr[0] = (uint32_t)id;
    r->ctr[1] = (uint32_t)(id >> 32);
    r->ctr[2] = 0;
    r->ctr[3] = 0;
    r->used = 4;
}

/* uniform in [0, 1) on a 2^-24 grid (the top 24 bits of a word) */
static double rng_u(rng_t *r)
{
    if (r->used == 4) {
        dso_philox4x32_10(r->ctr, r->key, r->buf);
        if (++r->ctr[2] == 0)
            ++r->ctr[3];
        r->used = 0;
    }
    return (double)(r->buf[r->used++] >> 8) * (1.0 / 16777216.0);
}

/* ------------------------------------------------------------------------------ */
/* O9  Monte Carlo transport (Sec. 3.2 Eq. 1, Sec. 4, Sec. 4.4, Sec. 5.1).         */
/* Medium: voxel-centred trilinear interpolation of mu_t = sigma_max * d on the    */
/* base grid, zero outside; vacuum outside the grid box.  Free flights by delta    */
/* tracking against the global majorant, transmittance by ratio tracking,          */
/* absorption by Russian roulette with survival probability albedo.               */
/* ------------------------------------------------------------------------------ */
typedef struct {
    const void *d;
    int dtype;
    int nx, ny, nz;
    double sigma_max;
    double amin[3], amax[3], h0;
    double maj;
} medium_t;

static double mu_at(const medium_t *M, const double p[3])
{
    double u[3], f[3];
    int64_t i0[3];
    for (int a = 0; a < 3; ++a) {
        u[a] = (p[a] - M->amin[a]) / M->h0 - 0.5;
        double fl = floor(u[a]);
        i0[a] = (int64_t)fl;
        f[a] = u[a] - fl;
    }
    int64_t dims[3] = {M->nx, M->ny, M->nz};
    double acc = 0.0;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                int64_t c[3] = {i0[0] + dx, i0[1] + dy, i0[2] + dz};
                if (c[0] < 0 || c[1] < 0 || c[2] < 0 || c[0] >= dims[0] || c[1] >= dims[1] ||
                    c[2] >= dims[2])
                    continue;
                double w = (dx ? f[0] : 1.0 - f[0]) * (dy ? f[1] : 1.0 - f[1]) *
                           (dz ? f[2] : 1.0 - f[2]);
                acc += w * density_at(M->d, M->dtype, (c[2] * M->ny + c[1]) * M->nx + c[0]);
            }
    return M->sigma_max * acc;
}

/* Parametric interval [t0, t1] of the ray o + t d inside the grid box; 0 if none. */
static int box_clip(const medium_t *M, const double o[3], const double d[3], double *t0,
                    double *t1)
{
    double lo = -INFINITY, hi = INFINITY;
    for (int a = 0; a < 3; ++a) {
        if (d[a] != 0.0) {
            double ta = (M->amin[a] - o[a]) / d[a], tb = (M->amax[a] - o[a]) / d[a];
            if (ta > tb) {
                double s = ta;
                ta = tb;
                tb = s;
            }
            lo = fmax(lo, ta);
            hi = fmin(hi, tb);
        } else if (o[a] < M->amin[a] || o[a] > M->amax[a]) {
            return 0;
        }
    }
    lo = fmax(lo, 0.0);
    if (!(hi > lo))
        return 0;
    *t0 = lo;
    *t1 = hi;
    return 1;
}

/* Delta tracking from o along unit d: 1 and the collision point, or 0 on escape. */
static int delta_track(const medium_t *M, const double o[3], const double d[3], rng_t *r,
                       double x[3])
{
    double t0, t1;
    if (!box_clip(M, o, d, &t0, &t1) || !(M->maj > 0))
        return 0;
    double t = t0;
    for (;;) {
        t += -log(1.0 - rng_u(r)) / M->maj;
        if (t >= t1)
            return 0;
        double p[3] = {o[0] + t * d[0], o[1] + t * d[1], o[2] + t * d[2]};
        if (rng_u(r) * M->maj < mu_at(M, p)) {
            x[0] = p[0];
            x[1] = p[1];
            x[2] = p[2];
            return 1;
        }
    }
}

/* Ratio tracking estimate of the transmittance from o along unit d to the box exit. */
static double ratio_track(const medium_t *M, const double o[3], const double d[3], rng_t *r)
{
    double t0, t1;
    if (!box_clip(M, o, d, &t0, &t1) || !(M->maj > 0))
        return 1.0;
    double T = 1.0, t = t0;
    for (;;) {
        t += -log(1.0 - rng_u(r)) / M->maj;
        if (t >= t1)
            return T;
        double p[3] = {o[0] + t * d[0], o[1] + t * d[1], o[2] + t * d[2]};
        T *= 1.0 - mu_at(M, p) / M->maj;
    }
}

/* Henyey-Greenstein phase function of the cosine between propagation directions. */
double dso_hg(double g, double mu)
{
    double den = 1.0 + g * g - 2.0 * g * mu;
    return (1.0 - g * g) / (4.0 * M_PI * den * sqrt(den));
}

/* Inverse-CDF sample of the HG cosine; isotropic for |g| < 1e-3. */
double dso_hg_sample_cos(double g, double u)
{
    if (fabs(g) < 1e-3)
        return 2.0 * u - 1.0;
    double s = (1.0 - g * g) / (1.0 - g + 2.0 * g * u);
    double c = (1.0 + g * g - s * s) / (2.0 * g);
    return c > 1.0 ? 1.0 : (c < -1.0 ? -1.0 : c);
}

/* Tabulated phase functions (a chopped Lorenz-Mie table for every scattering, and an
 * optional unchopped one for the direct term at the first collision of a camera ray):
 * p at theta_i = i pi / (n - 1), per steradian, and the normalised cumulative
 * distribution of theta at the same nodes (the trapezoid rule on 2 pi p sin theta).
 * Set for all later tracer calls by dso_set_phase; n = 0 clears (Henyey-Greenstein). */
typedef struct {
    int n;
    double dth;
    double *p, *cdf;
} phase_tab;

static phase_tab g_phase, g_first;
/* Fraction f of the scattering that the chop removed from the scattering table (0 for an
 * unchopped table or Henyey-Greenstein), and the first-collision table's own fraction. */
static double g_removed = 0.0, g_removed_first = 0.0;

/* The chop of Sec. 3.1: the removed forward peak is treated as unscattered light, so the
 * medium is made optically thinner "according to the fraction of scattered light contained
 * in the peak".  With single-scattering albedo a, the removed scattering a f leaves the
 * extinction, mu_t' = mu_t (1 - a f), and the scattering left is a (1 - f) mu_t, so the
 * albedo of the thinner medium is a (1 - f) / (1 - a f).  Applied to the medium and albedo
 * of every tracer call while a chopped scattering table is set. */
static void chop_reduce(double *sigma_max, double *albedo)
{
    if (!g_phase.n || !(g_removed > 0.0))
        return;
    double a = *albedo, s = 1.0 - a * g_removed;
    *sigma_max *= s;
    *albedo = a * (1.0 - g_removed) / s;
}

/* Weight of the first-collision table (Sec. 3.1: the full function at the first bounce,
 * then the chopped one in the thinner medium).  A table that removed f_first carries
 * (1 - f_first) of the scattering: its direct term in the thinner medium must weigh the
 * unreduced scattering a mu_t, which is (1 - f_first) / (1 - f) times the thinner medium's
 * a' mu_t' = a (1 - f) mu_t. */
static double first_scale(void)
{
    if (!g_phase.n || !g_first.n)
        return 1.0;
    return (1.0 - g_removed_first) / (1.0 - g_removed);
}

static void tab_set(phase_tab *t, int n, const double *p, const double *cdf)
{
    free(t->p);
    free(t->cdf);
    t->p = t->cdf = NULL;
    t->n = 0;
    if (n < 3 || !p || !cdf)
        return;
    t->p = malloc(sizeof(double) * n);
    t->cdf = malloc(sizeof(double) * n);
    memcpy(t->p, p, sizeof(double) * n);
    memcpy(t->cdf, cdf, sizeof(double) * n);
    t->n = n;
    t->dth = M_PI / (n - 1);
}

void dso_set_phase(int n, const double *p, const double *cdf, double removed, int n_first,
                   const double *p_first, const double *cdf_first, double removed_first)
{
    tab_set(&g_phase, n, p, cdf);
    tab_set(&g_first, n_first, p_first, cdf_first);
    g_removed = g_phase.n ? removed : 0.0;
    g_removed_first = g_first.n ? removed_first : 0.0;
}

/* p(mu): linear in theta between nodes */
static double tab_eval(const phase_tab *t, double mu)
{
    double th = acos(fmax(-1.0, fmin(1.0, mu))) / t->dth;
    int i = (int)th;
    if (i > t->n - 2)
        i = t->n - 2;
    double f = th - i;
    return t->p[i] + f * (t->p[i + 1] - t->p[i]);
}

/* The table's p(mu), as the tracer reads it, for a table of n >= 2 values at
 * theta_i = i pi / (n - 1). */
double dso_tab_eval(int n, const double *p, double mu)
{
    phase_tab t = {n, M_PI / (n - 1), (double *)p, NULL};
    return tab_eval(&t, mu);
}

/* cos(theta) drawn from the table: the node interval by the cumulative distribution,
 * then theta inside it from the density linear between the nodes' p sin(theta). */
double dso_tab_sample(int n, const double *p, const double *cdf, double u)
{
    int lo = 0, hi = n - 1; /* cdf[lo] <= u < cdf[hi] */
    while (hi - lo > 1) {
        int mid = (lo + hi) / 2;
        if (cdf[mid] <= u)
            lo = mid;
        else
            hi = mid;
    }
    double dth = M_PI / (n - 1);
    double fa = p[lo] * sin(lo * dth), fb = p[lo + 1] * sin((lo + 1) * dth);
    double q = (u - cdf[lo]) / (cdf[lo + 1] - cdf[lo]);
    double t;
    if (fabs(fb - fa) <= 1e-12 * (fa + fb))
        t = q;
    else
        t = (-fa + sqrt(fa * fa + (fb - fa) * q * (fa + fb))) / (fb - fa);
    t = fmin(1.0, fmax(0.0, t));
    return cos((lo + t) * dth);
}

static double ph_eval(double g, int first, double mu)
{
    if (first && g_first.n)
        return first_scale() * tab_eval(&g_first, mu);
    if (g_phase.n)
        return tab_eval(&g_phase, mu);
    return dso_hg(g, mu);
}

static double ph_sample(double g, double u)
{
    if (g_phase.n)
        return dso_tab_sample(g_phase.n, g_phase.p, g_phase.cdf, u);
    return dso_hg_sample_cos(g, u);
}

static void sample_dir_around(const double w[3], double cos_t, double u, double out[3])
{
    double t1[3], t2[3];
    onb(w, t1, t2);
    double sin_t = sqrt(fmax(0.0, 1.0 - cos_t * cos_t));
    double phi = 2.0 * M_PI * u;
    double cp = cos(phi), sp = sin(phi);
    for (int a = 0; a < 3; ++a)
        out[a] = sin_t * cp * t1[a] + sin_t * sp * t2[a] + cos_t * w[a];
    double l = sqrt(dot3(out, out));
    for (int a = 0; a < 3; ++a)
        out[a] /= l;
}

static void uniform_sphere(double u, double v, double out[3])
{
    double z = 1.0 - 2.0 * u;
    double r = sqrt(fmax(0.0, 1.0 - z * z));
    double phi = 2.0 * M_PI * v;
    out[0] = r * cos(phi);
    out[1] = r * sin(phi);
    out[2] = z;
}

/* A distant emitter as m directional lights (Sec. 4.4): unit directions dir[3j..3j+2]
 * toward the light, selection thresholds thr[j] and weights w[j] (see set_pick). */
typedef struct {
    int m;
    const double *dir;
    const uint32_t *thr;
    const double *w;
} light_set;

typedef struct {
    double albedo;
    double g;
    double irradiance;   /* E of the directional light, or radiance of the uniform environment */
    int light_mode;      /* 0: directional light with next-event estimation; 1: uniform environment;
                            2: a set of directional lights, one drawn per next-event estimate */
    int max_interactions; /* 0: unlimited */
    const light_set *set; /* mode 2 only */
} tracer_params;

/* Mode 2: light j is drawn with probability (thr[j] - thr[j-1]) / 2^24 (thr[-1] = 0) by the
 * top 24 bits k of one uniform, as the first j with k < thr[j]; its estimate is weighted by
 * w[j] = E_j / that probability, so each draw is unbiased for the sum over the set. */
static int set_pick(const light_set *ls, rng_t *r)
{
    uint32_t k = (uint32_t)(rng_u(r) * 16777216.0);
    for (int j = 0; j < ls->m; ++j)
        if (k < ls->thr[j])
            return j;
    return ls->m - 1; /* not reached: thr[m-1] = 2^24 */
}

/* One path estimate of the indirect in-scattered radiance L_i(x, w) (Sec. 4):
 * the light that reaches x travelling along w_hat, after at least one collision,
 * folded with p(w . w_hat).  Uncollided light is excluded by construction. */
static double li_path(const medium_t *M, const tracer_params *tp, const double x[3],
                      const double w[3], const double wl[3], int count_uncollided, rng_t *r)
{
    double wprev[3] = {w[0], w[1], w[2]}, p[3] = {x[0], x[1], x[2]};
    double sum = 0.0;
    for (int j = 1;; ++j) {
        if (tp->max_interactions > 0 && j > tp->max_interactions)
            break;
        double c = ph_sample(tp->g, rng_u(r));
        double wh[3];
        sample_dir_around(wprev, c, rng_u(r), wh);
        double back[3] = {-wh[0], -wh[1], -wh[2]}, xn[3];
        if (!delta_track(M, p, back, r, xn)) {
            if (tp->light_mode == 1 && (j > 1 || count_uncollided))
                sum += tp->irradiance;
            break;
        }
        p[0] = xn[0];
        p[1] = xn[1];
        p[2] = xn[2];
        if (rng_u(r) >= tp->albedo)
            break;
        if (tp->light_mode == 0) {
            double mu = -dot3(wh, wl);
            double T = ratio_track(M, p, wl, r);
            sum += ph_eval(tp->g, 0, mu) * T * tp->irradiance;
        } else if (tp->light_mode == 2) {
            int j = set_pick(tp->set, r);
            const double *lj = tp->set->dir + 3 * j;
            double mu = -dot3(wh, lj);
            double T = ratio_track(M, p, lj, r);
            sum += tp->set->w[j] * ph_eval(tp->g, 0, mu) * T * tp->irradiance;
        }
        wprev[0] = wh[0];
        wprev[1] = wh[1];
        wprev[2] = wh[2];
    }
    return sum;
}

static int medium_init(medium_t *M, const void *dens, int dtype, int nx, int ny, int nz,
                       double sigma_max, const double *aabb_min, double h0)
{
    if (!dens || nx <= 0 || ny <= 0 || nz <= 0 || !(h0 > 0))
        return 0;
    M->d = dens;
    M->dtype = dtype;
    M->nx = nx;
    M->ny = ny;
    M->nz = nz;
    M->sigma_max = sigma_max;
    M->h0 = h0;
    int64_t dims[3] = {nx, ny, nz};
    for (int a = 0; a < 3; ++a) {
        M->amin[a] = aabb_min[a];
        M->amax[a] = aabb_min[a] + dims[a] * h0;
    }
    double mx = 0.0;
    int64_t n = (int64_t)nx * ny * nz;
    for (int64_t i = 0; i < n; ++i) {
        double v = density_at(dens, dtype, i);
        if (v > mx)
            mx = v;
    }
    M->maj = sigma_max * mx;
    return 1;
}

/* Per record i: mean of spp path estimates and the variance of that mean
 * (sample variance / spp), accumulated in double.  Path s of record i uses
 * random stream id = i * 2^20 + s under key `seed`. */
/* One record estimate: the indirect in-scattered radiance L_i (li_path), or with
 * include_direct all in-scattered radiance L_s = L_d + L_i (Sec. 7): for the
 * directional light the direct term p(-w . w_l) T(x -> light) E by ratio tracking,
 * drawn before the path; for the uniform environment the light that reaches x
 * without a collision is counted as well. */
static double record_path(const medium_t *M, const tracer_params *tp, const double x[3],
                          const double w[3], const double wl[3], int include_direct, rng_t *r)
{
    if (!include_direct)
        return li_path(M, tp, x, w, wl, 0, r);
    if (tp->light_mode == 1)
        return li_path(M, tp, x, w, wl, 1, r);
    double d = ph_eval(tp->g, 0, -dot3(w, wl)) * ratio_track(M, x, wl, r) * tp->irradiance;
    return d + li_path(M, tp, x, w, wl, 0, r);
}

int dso_trace_li(const void *dens, int dtype, int nx, int ny, int nz, double sigma_max,
                 const double *aabb_min, double h0, double albedo, double g, double irradiance,
                 int light_mode, int max_interactions, int include_direct, int spp, uint64_t seed,
                 const float *pos, const float *view, const float *light, int64_t P,
                 double *mean_out, double *var_out)
{
    medium_t M;
    chop_reduce(&sigma_max, &albedo);
    if (!medium_init(&M, dens, dtype, nx, ny, nz, sigma_max, aabb_min, h0) || spp <= 0 ||
        spp > (1 << 20))
        return DSO_ERR_INVALID;
    tracer_params tp = {albedo, g, irradiance, light_mode, max_interactions, NULL};
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < P; ++i) {
        double x[3] = {pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]};
        double wv[3] = {view[3 * i], view[3 * i + 1], view[3 * i + 2]};
        double lv[3] = {light[3 * i], light[3 * i + 1], light[3 * i + 2]};
        double w[3], wl[3];
        if (!unit3(wv, w) || !unit3(lv, wl)) {
            mean_out[i] = 0.0;
            if (var_out)
                var_out[i] = 0.0;
            continue;
        }
        double s1 = 0.0, s2 = 0.0;
        for (int s = 0; s < spp; ++s) {
            rng_t r;
            rng_init(&r, seed, ((uint64_t)i << 20) + (uint64_t)s);
            double e = record_path(&M, &tp, x, w, wl, include_direct, &r);
            s1 += e;
            s2 += e * e;
        }
        double mean = s1 / spp;
        mean_out[i] = mean;
        if (var_out)
            var_out[i] = spp > 1 ? fmax(0.0, (s2 - spp * mean * mean) / (spp - 1)) / spp : 0.0;
    }
    return DSO_OK;
}

/* Progressive estimates (Sec. 5.1): paths are added one batch at a time until the
 * sample mean lies within +-rel of the true value at the confidence of the normal
 * quantile zq, i.e. zq * sqrt(variance of the mean) <= rel * |mean| after a whole
 * batch, or until max_spp paths.  Path s of record i uses stream id i * 2^20 + s as in
 * dso_trace_li, so the result at n paths is dso_trace_li's at spp = n.  n_out receives
 * the number of paths used (0 for records with an unusable direction). */
int dso_trace_li_adaptive(const void *dens, int dtype, int nx, int ny, int nz, double sigma_max,
                          const double *aabb_min, double h0, double albedo, double g,
                          double irradiance, int light_mode, int max_interactions,
                          int include_direct, int batch, int max_spp, double rel, double zq,
                          uint64_t seed, const float *pos, const float *view, const float *light,
                          int64_t P, double *mean_out, double *var_out, int32_t *n_out)
{
    medium_t M;
    chop_reduce(&sigma_max, &albedo);
    if (!medium_init(&M, dens, dtype, nx, ny, nz, sigma_max, aabb_min, h0) || batch < 2 ||
        max_spp < batch || max_spp > (1 << 20) || max_spp % batch != 0 || !(rel > 0) ||
        !(zq > 0))
        return DSO_ERR_INVALID;
    tracer_params tp = {albedo, g, irradiance, light_mode, max_interactions, NULL};
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < P; ++i) {
        double x[3] = {pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]};
        double wv[3] = {view[3 * i], view[3 * i + 1], view[3 * i + 2]};
        double lv[3] = {light[3 * i], light[3 * i + 1], light[3 * i + 2]};
        double w[3], wl[3];
        mean_out[i] = 0.0;
        var_out[i] = 0.0;
        n_out[i] = 0;
        if (!unit3(wv, w) || !unit3(lv, wl))
            continue;
        double s1 = 0.0, s2 = 0.0, mean = 0.0, vm = 0.0;
        int n = 0;
        while (n < max_spp) {
            rng_t r;
            rng_init(&r, seed, ((uint64_t)i << 20) + (uint64_t)n);
            double e = record_path(&M, &tp, x, w, wl, include_direct, &r);
            s1 += e;
            s2 += e * e;
            ++n;
            if (n % batch == 0) {
                mean = s1 / n;
                vm = fmax(0.0, (s2 - n * mean * mean) / (n - 1)) / n;
                if (zq * sqrt(vm) <= rel * fabs(mean))
                    break;
            }
        }
        mean_out[i] = mean;
        var_out[i] = vm;
        n_out[i] = n;
    }
    return DSO_OK;
}

/* Transmittance estimates along rays (for the slab test): per ray, the mean of spp
 * ratio-tracking estimates, and separately the fraction of delta-tracked flights
 * that escape. */
int dso_transmittance(const void *dens, int dtype, int nx, int ny, int nz, double sigma_max,
                      const double *aabb_min, double h0, const double *orig, const double *dir,
                      int64_t R, int spp, uint64_t seed, double *ratio_mean, double *escape_frac)
{
    medium_t M;
    if (!medium_init(&M, dens, dtype, nx, ny, nz, sigma_max, aabb_min, h0) || spp <= 0)
        return DSO_ERR_INVALID;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < R; ++i) {
        double o[3] = {orig[3 * i], orig[3 * i + 1], orig[3 * i + 2]}, d[3];
        if (!unit3(dir + 3 * i, d)) {
            ratio_mean[i] = escape_frac[i] = 0.0;
            continue;
        }
        double sr = 0.0;
        int64_t esc = 0;
        for (int s = 0; s < spp; ++s) {
            rng_t r;
            rng_init(&r, seed, ((uint64_t)i << 20) + (uint64_t)s);
            sr += ratio_track(&M, o, d, &r);
            double x[3];
            if (!delta_track(&M, o, d, &r, x))
                ++esc;
        }
        ratio_mean[i] = sr / spp;
        escape_frac[i] = (double)esc / spp;
    }
    return DSO_OK;
}

/* Record configurations (Sec. 5.1): a direction d uniform on the sphere; an origin
 * uniform over the bounding sphere's cross-section orthogonal to d; a free flight
 * into the cloud along d, retried from scratch on escape.  The stored view direction
 * is the radiance propagation direction -d; the light direction is uniform on the
 * sphere.  Record i uses stream id i under key `seed`. */
int dso_sample_records(const void *dens, int dtype, int nx, int ny, int nz, double sigma_max,
                       const double *aabb_min, double h0, int64_t N, uint64_t seed, float *pos,
                       float *view, float *light, int32_t *attempts)
{
    medium_t M;
    if (!medium_init(&M, dens, dtype, nx, ny, nz, sigma_max, aabb_min, h0) || !(M.maj > 0))
        return DSO_ERR_INVALID;
    double c[3], R = 0.0;
    for (int a = 0; a < 3; ++a) {
        c[a] = 0.5 * (M.amin[a] + M.amax[a]);
        double e = 0.5 * (M.amax[a] - M.amin[a]);
        R += e * e;
    }
    R = sqrt(R);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < N; ++i) {
        rng_t r;
        rng_init(&r, seed, (uint64_t)i);
        double d[3], x[3];
        int tries = 0;
        for (;;) {
            ++tries;
            double u0 = rng_u(&r), u1 = rng_u(&r);
            uniform_sphere(u0, u1, d);
            double t1[3], t2[3];
            onb(d, t1, t2);
            double rr = R * sqrt(rng_u(&r)), ph = 2.0 * M_PI * rng_u(&r);
            double o[3];
            for (int a = 0; a < 3; ++a)
                o[a] = c[a] - R * d[a] + rr * (cos(ph) * t1[a] + sin(ph) * t2[a]);
            if (delta_track(&M, o, d, &r, x))
                break;
            if (tries >= 1000000) { /* empty-looking cloud: give up on this record */
                x[0] = x[1] = x[2] = NAN;
                break;
            }
        }
        double l[3];
        double u0 = rng_u(&r), u1 = rng_u(&r);
        uniform_sphere(u0, u1, l);
        for (int a = 0; a < 3; ++a) {
            pos[3 * i + a] = (float)x[a];
            view[3 * i + a] = (float)(-d[a]);
            light[3 * i + a] = (float)l[a];
        }
        if (attempts)
            attempts[i] = tries;
    }
    return DSO_OK;
}

/* One camera sample per ray (Sec. 4.4): the delta-tracked first collision x along
 * o + t d, the view direction there (-d), and the direct single scattering
 * albedo * p(d . w_l) * T(x -> light) * E with T one ratio-tracking estimate;
 * hit = 0 and zeros for rays that escape.  Ray i, sample s uses stream id
 * i * 2^20 + s under key `seed`: the same streams, consumed in the same order, as
 * the first stage of dso_render_pixels in mode 0. */
int dso_first_hits(const void *dens, int dtype, int nx, int ny, int nz, double sigma_max,
                   const double *aabb_min, double h0, double albedo, double g, double irradiance,
                   const double *light_dir, const float *ray_o, const float *ray_d, int64_t N,
                   uint64_t seed, uint64_t sample, double *pos, double *view, double *direct,
                   uint8_t *hit)
{
    medium_t M;
    chop_reduce(&sigma_max, &albedo);
    if (!medium_init(&M, dens, dtype, nx, ny, nz, sigma_max, aabb_min, h0) || sample >= (1u << 20))
        return DSO_ERR_INVALID;
    double wl[3];
    if (!unit3(light_dir, wl))
        return DSO_ERR_INVALID;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < N; ++i) {
        double o[3] = {ray_o[3 * i], ray_o[3 * i + 1], ray_o[3 * i + 2]};
        double dv[3] = {ray_d[3 * i], ray_d[3 * i + 1], ray_d[3 * i + 2]}, d[3], x[3];
        int h = 0;
        double e = 0.0;
        if (unit3(dv, d)) {
            rng_t r;
            rng_init(&r, seed, ((uint64_t)i << 20) + sample);
            h = delta_track(&M, o, d, &r, x);
            if (h)
                e = albedo * ph_eval(g, 1, dot3(d, wl)) * ratio_track(&M, x, wl, &r) * irradiance;
        }
        for (int a = 0; a < 3; ++a) {
            pos[3 * i + a] = h ? x[a] : 0.0;
            view[3 * i + a] = h ? -d[a] : 0.0;
        }
        direct[i] = e;
        hit[i] = (uint8_t)h;
    }
    return DSO_OK;
}

/* One path-traced camera sample: the first collision x along o + t d (background 0,
 * or the environment radiance in mode 1), then albedo times the in-scattered radiance
 * at x toward the camera: direct single scattering by next-event estimation plus the
 * L_i path estimate in modes 0 and 2, the full in-scattered environment light in
 * mode 1. */
static double pixel_sample(const medium_t *M, const tracer_params *tp, const double wl[3],
                           const double o[3], const double d[3], rng_t *r)
{
    double x[3];
    if (!delta_track(M, o, d, r, x))
        return tp->light_mode == 1 ? tp->irradiance : 0.0;
    double w[3] = {-d[0], -d[1], -d[2]};
    if (tp->light_mode == 1)
        return tp->albedo * li_path(M, tp, x, w, wl, 1, r);
    double direct;
    if (tp->light_mode == 0) {
        direct = ph_eval(tp->g, 1, -dot3(w, wl)) * ratio_track(M, x, wl, r) * tp->irradiance;
    } else {
        int j = set_pick(tp->set, r);
        const double *lj = tp->set->dir + 3 * j;
        direct = tp->set->w[j] * ph_eval(tp->g, 1, -dot3(w, lj)) * ratio_track(M, x, lj, r) *
                 tp->irradiance;
    }
    return tp->albedo * (direct + li_path(M, tp, x, w, wl, 0, r));
}

/* Path-traced pixels (Sec. 4.4 with the network replaced by the path estimate):
 * a delta-tracked first collision x along each camera ray o + t d (background 0,
 * or the environment radiance in mode 1), then albedo times the in-scattered
 * radiance at x toward the camera: in mode 0 direct single scattering by
 * next-event estimation plus the L_i path estimate; in mode 1 the full
 * in-scattered environment light.  Ray (pixel i, sample s) uses stream id
 * i * 2^20 + s. */
int dso_render_pixels(const void *dens, int dtype, int nx, int ny, int nz, double sigma_max,
                      const double *aabb_min, double h0, double albedo, double g,
                      double irradiance, int light_mode, int max_interactions,
                      const double *light_dir, const float *ray_o, const float *ray_d,
                      int64_t NPix, int spp, uint64_t seed, double *mean_out, double *var_out)
{
    medium_t M;
    chop_reduce(&sigma_max, &albedo);
    if (!medium_init(&M, dens, dtype, nx, ny, nz, sigma_max, aabb_min, h0) || spp <= 0 ||
        spp > (1 << 20))
        return DSO_ERR_INVALID;
    tracer_params tp = {albedo, g, irradiance, light_mode, max_interactions, NULL};
    double wl[3];
    if (!unit3(light_dir, wl))
        return DSO_ERR_INVALID;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < NPix; ++i) {
        double o[3] = {ray_o[3 * i], ray_o[3 * i + 1], ray_o[3 * i + 2]};
        double dv[3] = {ray_d[3 * i], ray_d[3 * i + 1], ray_d[3 * i + 2]}, d[3];
        if (!unit3(dv, d)) {
            mean_out[i] = 0.0;
            if (var_out)
                var_out[i] = 0.0;
            continue;
        }
        double s1 = 0.0, s2 = 0.0;
        for (int s = 0; s < spp; ++s) {
            rng_t r;
            rng_init(&r, seed, ((uint64_t)i << 20) + (uint64_t)s);
            double e = pixel_sample(&M, &tp, wl, o, d, &r);
            s1 += e;
            s2 += e * e;
        }
        double mean = s1 / spp;
        mean_out[i] = mean;
        if (var_out)
            var_out[i] = spp > 1 ? fmax(0.0, (s2 - spp * mean * mean) / (spp - 1)) / spp : 0.0;
    }
    return DSO_OK;
}

/* The light-set forms (Sec. 4.4: a distant emitter approximated by directional
 * samples).  The set is m unit directions dir ([m][3]) with thresholds thr and
 * weights w as set_pick states; every directional term is scaled by irradiance. */
static int set_ok(int m, const double *dir, const uint32_t *thr, const double *w)
{
    if (m < 1 || !dir || !thr || !w || thr[m - 1] != (1u << 24))
        return 0;
    for (int j = 0; j < m; ++j)
        if ((j > 0 && thr[j] <= thr[j - 1]) || thr[j] == 0 || !(w[j] >= 0))
            return 0;
    return 1;
}

/* Path-traced pixels under a light set: per sample, the first collision, the direct
 * term of one light drawn from the set, and the L_i path estimate with one light
 * drawn at every collision.  Streams as dso_render_pixels. */
int dso_render_pixels_lights(const void *dens, int dtype, int nx, int ny, int nz, double sigma_max,
                             const double *aabb_min, double h0, double albedo, double g,
                             double irradiance, int max_interactions, int m, const double *dir,
                             const uint32_t *thr, const double *w, const float *ray_o,
                             const float *ray_d, int64_t NPix, int spp, uint64_t seed,
                             double *mean_out, double *var_out)
{
    medium_t M;
    chop_reduce(&sigma_max, &albedo);
    if (!medium_init(&M, dens, dtype, nx, ny, nz, sigma_max, aabb_min, h0) || spp <= 0 ||
        spp > (1 << 20) || !set_ok(m, dir, thr, w))
        return DSO_ERR_INVALID;
    light_set ls = {m, dir, thr, w};
    tracer_params tp = {albedo, g, irradiance, 2, max_interactions, &ls};
    const double wl[3] = {0.0, 0.0, 1.0}; /* unused in mode 2 */
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < NPix; ++i) {
        double o[3] = {ray_o[3 * i], ray_o[3 * i + 1], ray_o[3 * i + 2]};
        double dv[3] = {ray_d[3 * i], ray_d[3 * i + 1], ray_d[3 * i + 2]}, d[3];
        double s1 = 0.0, s2 = 0.0;
        if (unit3(dv, d)) {
            for (int s = 0; s < spp; ++s) {
                rng_t r;
                rng_init(&r, seed, ((uint64_t)i << 20) + (uint64_t)s);
                double e = pixel_sample(&M, &tp, wl, o, d, &r);
                s1 += e;
                s2 += e * e;
            }
        }
        double mean = s1 / spp;
        mean_out[i] = mean;
        if (var_out)
            var_out[i] = spp > 1 ? fmax(0.0, (s2 - spp * mean * mean) / (spp - 1)) / spp : 0.0;
    }
    return DSO_OK;
}

/* One camera sample per ray for the network renderer under a light set: the first
 * collision x and view direction as dso_first_hits, then D lights drawn from the set
 * (draw q of ray i goes to row i * D + q of light_out and weight_out: the direction
 * and w[j]), each with one ratio-tracking estimate T_q toward it; direct =
 * albedo * irradiance * (1/D) * sum_q w[j_q] p(d . l_q) T_q.  Rays that escape get
 * hit = 0 and zero rows.  The stream of ray i, sample s (id i * 2^20 + s) is used for
 * the flight, then for each draw its choice and its ratio tracking, in draw order. */
int dso_first_hits_lights(const void *dens, int dtype, int nx, int ny, int nz, double sigma_max,
                          const double *aabb_min, double h0, double albedo, double g,
                          double irradiance, int m, const double *dir, const uint32_t *thr,
                          const double *w, int D, const float *ray_o, const float *ray_d,
                          int64_t N, uint64_t seed, uint64_t sample, double *pos, double *view,
                          double *light_out, double *weight_out, double *direct, uint8_t *hit)
{
    medium_t M;
    chop_reduce(&sigma_max, &albedo);
    if (!medium_init(&M, dens, dtype, nx, ny, nz, sigma_max, aabb_min, h0) ||
        sample >= (1u << 20) || D < 1 || !set_ok(m, dir, thr, w))
        return DSO_ERR_INVALID;
    light_set ls = {m, dir, thr, w};
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < N; ++i) {
        double o[3] = {ray_o[3 * i], ray_o[3 * i + 1], ray_o[3 * i + 2]};
        double dv[3] = {ray_d[3 * i], ray_d[3 * i + 1], ray_d[3 * i + 2]}, d[3], x[3];
        int h = 0;
        double e = 0.0;
        rng_t r;
        if (unit3(dv, d)) {
            rng_init(&r, seed, ((uint64_t)i << 20) + sample);
            h = delta_track(&M, o, d, &r, x);
        }
        for (int q = 0; q < D; ++q) {
            double *lo = light_out + 3 * (i * D + q);
            if (!h) {
                lo[0] = lo[1] = lo[2] = 0.0;
                weight_out[i * D + q] = 0.0;
                continue;
            }
            int j = set_pick(&ls, &r);
            const double *lj = dir + 3 * j;
            double T = ratio_track(&M, x, lj, &r);
            e += w[j] * ph_eval(g, 1, dot3(d, lj)) * T;
            lo[0] = lj[0];
            lo[1] = lj[1];
            lo[2] = lj[2];
            weight_out[i * D + q] = w[j];
        }
        for (int a = 0; a < 3; ++a) {
            pos[3 * i + a] = h ? x[a] : 0.0;
            view[3 * i + a] = h ? -d[a] : 0.0;
        }
        direct[i] = albedo * irradiance * e / D;
        hit[i] = (uint8_t)h;
    }
    return DSO_OK;
}
