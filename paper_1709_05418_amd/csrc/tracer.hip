// Monte Carlo transport in the cloud (Sec. 3.2 Eq. (1), Sec. 4, Sec. 4.4, Sec. 5.1):
// delta tracking against a global majorant, ratio-tracked transmittance toward the
// light, Henyey-Greenstein scattering, absorption by Russian roulette.  One thread
// per path; per-record sums of the path estimates are accumulated in FP64 and
// reduced in a fixed order, so results are reproducible bit for bit.
#include <math.h>

#include "internal.h"

namespace ds {
namespace {

// Paths per block: one wave.  The per-record sums end in a block barrier, and at high
// albedo path lengths spread widely; with one wave per block a wave that has finished
// its paths leaves at once instead of holding its slot until the block's slowest wave
// ends (20 % more paths per second than 256-thread blocks on long paths).
constexpr int kPaths = 64;
constexpr int64_t kMaxSteps = 1ll << 26;    // hard bound on tentative collisions per path

// ------------------------------------------------------------------ Philox4x32-10
// Counter-based generator of Salmon et al. (SC'11): 10 rounds of two 32x32->64-bit
// multiplications mixing the four counter words, with a Weyl-sequence key schedule.
struct Rng {
    uint32_t k0, k1;        // key = seed
    uint32_t c0, c1, c2, c3; // counter = (stream id lo, hi, block, 0)
    uint32_t buf[4];
    int used;

    __device__ void init(uint64_t seed, uint64_t id)
    {
        k0 = (uint32_t)seed;
        k1 = (uint32_t)(seed >> 32);
        c0 = (uint32_t)id;
        c1 = (uint32_t)(id >> 32);
        c2 = 0;
        c3 = 0;
        used = 4;
    }
    __device__ void refill()
    {
        uint32_t x0 = c0, x1 = c1, x2 = c2, x3 = c3, a = k0, b = k1;
#pragma unroll
        for (int r = 0; r < 10; ++r) {
            const uint32_t lo0 = 0xD2511F53u * x0, hi0 = __umulhi(0xD2511F53u, x0);
            const uint32_t lo1 = 0xCD9E8D57u * x2, hi1 = __umulhi(0xCD9E8D57u, x2);
            const uint32_t y0 = hi1 ^ x1 ^ a, y2 = hi0 ^ x3 ^ b;
            x0 = y0;
            x1 = lo1;
            x2 = y2;
            x3 = lo0;
            a += 0x9E3779B9u;
            b += 0xBB67AE85u;
        }
        buf[0] = x0;
        buf[1] = x1;
        buf[2] = x2;
        buf[3] = x3;
        if (++c2 == 0)
            ++c3;
        used = 0;
    }
    // the top 24 bits of the next word
    __device__ uint32_t bits24()
    {
        if (used == 4)
            refill();
        return buf[used++] >> 8;
    }
    // uniform in [0, 1) on the 2^-24 grid
    __device__ float u() { return (float)bits24() * (1.f / 16777216.f); }
};

// Member of a light set drawn by one uniform's top 24 bits k: the first j with
// k < thr[j] (thresholds strictly increasing, the last 2^24), by binary search.
__device__ __forceinline__ int set_pick(const TracerParams &tp, Rng &r)
{
    const uint32_t k = r.bits24();
    int lo = 0, hi = tp.set_m - 1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (k < tp.set_thr[mid])
            hi = mid;
        else
            lo = mid + 1;
    }
    return lo;
}

// ------------------------------------------------------------------ geometry helpers
struct V3 {
    float x, y, z;
};
__host__ __device__ __forceinline__ V3 v3(float x, float y, float z) { return V3{x, y, z}; }
__device__ __forceinline__ float dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ V3 neg(V3 a) { return v3(-a.x, -a.y, -a.z); }
__device__ __forceinline__ V3 madd(V3 a, float t, V3 d) { return v3(a.x + t * d.x, a.y + t * d.y, a.z + t * d.z); }

__device__ __forceinline__ bool unit(const float *v, V3 &u)
{
    float a = v[0], b = v[1], c = v[2];
    if (!(isfinite(a) && isfinite(b) && isfinite(c)))
        return false;
    float m = fmaxf(fabsf(a), fmaxf(fabsf(b), fabsf(c)));
    if (m == 0.f)
        return false;
    a /= m;
    b /= m;
    c /= m;
    float l = sqrtf(a * a + b * b + c * c);
    u = v3(a / l, b / l, c / l);
    return true;
}

// Orthonormal pair around unit n (branchless construction of Duff et al. 2017).
__device__ __forceinline__ void basis(V3 n, V3 &t1, V3 &t2)
{
    const float sg = copysignf(1.f, n.z);
    const float a = -1.f / (sg + n.z);
    const float b = n.x * n.y * a;
    t1 = v3(1.f + sg * n.x * n.x * a, sg * b, -sg * n.x);
    t2 = v3(b, sg + n.y * n.y * a, -n.y);
}

// ------------------------------------------------------------------ medium
struct Medium {
    const float4 *cells;  // corner-packed extinction: cell c = entries 2c, 2c + 1
    int cx, cy;           // cell-grid dims in x and y (grid dims + 2)
    float hx, hy, hz;     // clamp bounds of the shifted cell coordinate (grid dims + 1)
    V3 amin, amax;
    float inv_h, maj;
    float inv_ff;         // mean free-flight length 1 / (maj * extinction scale); the scale
                          // thins the medium uniformly (the chop of a tabulated phase
                          // function), so collision and transmittance ratios keep maj
    unsigned long long *truncated;  // paths stopped at kMaxSteps (the context's counter)
};

// A path whose tentative collisions reach kMaxSteps stops there; the call that crosses
// the bound counts it once in the context's counter (s0: the path's count before the call).
__device__ __forceinline__ void note_cap(const Medium &M, int64_t s0, int64_t steps)
{
    if (steps >= kMaxSteps && s0 < kMaxSteps && M.truncated)
        atomicAdd(M.truncated, 1ull);
}

// Voxel-centred trilinear extinction, zero outside the grid.  The cell coordinate (the
// voxel-centred coordinate plus one), clamped to [0, n + 1], selects a cell whose eight
// corners are the lattice values around the point; the border cells hold zeros, so points
// outside the grid read zero without tests.
__device__ float mu_at(const Medium &M, V3 p)
{
    const float ux = __builtin_amdgcn_fmed3f((p.x - M.amin.x) * M.inv_h + 0.5f, 0.f, M.hx);
    const float uy = __builtin_amdgcn_fmed3f((p.y - M.amin.y) * M.inv_h + 0.5f, 0.f, M.hy);
    const float uz = __builtin_amdgcn_fmed3f((p.z - M.amin.z) * M.inv_h + 0.5f, 0.f, M.hz);
    const uint32_t i = (uint32_t)ux, j = (uint32_t)uy, k = (uint32_t)uz;
    const float fx = __builtin_amdgcn_fractf(ux), fy = __builtin_amdgcn_fractf(uy),
                fz = __builtin_amdgcn_fractf(uz);
    const int64_t cell = (int64_t)i + (int64_t)M.cx * ((int64_t)j + (int64_t)M.cy * k);
    const float4 lo = M.cells[2 * cell], hi = M.cells[2 * cell + 1];
    // corner c = dx + 2 dy + 4 dz
    const float a00 = fmaf(fx, lo.y - lo.x, lo.x), a10 = fmaf(fx, lo.w - lo.z, lo.z);
    const float a01 = fmaf(fx, hi.y - hi.x, hi.x), a11 = fmaf(fx, hi.w - hi.z, hi.z);
    const float b0 = fmaf(fy, a10 - a00, a00), b1 = fmaf(fy, a11 - a01, a01);
    return fmaf(fz, b1 - b0, b0);
}

// Parametric interval [t0, t1] of o + t d inside the grid box, t >= 0.
__device__ bool clip(const Medium &M, V3 o, V3 d, float &t0, float &t1)
{
    float lo = 0.f, hi = INFINITY;
    const float oo[3] = {o.x, o.y, o.z}, dd[3] = {d.x, d.y, d.z};
    const float mn[3] = {M.amin.x, M.amin.y, M.amin.z}, mx[3] = {M.amax.x, M.amax.y, M.amax.z};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (dd[a] != 0.f) {
            float ta = (mn[a] - oo[a]) / dd[a], tb = (mx[a] - oo[a]) / dd[a];
            if (ta > tb) {
                const float s = ta;
                ta = tb;
                tb = s;
            }
            lo = fmaxf(lo, ta);
            hi = fminf(hi, tb);
        } else if (oo[a] < mn[a] || oo[a] > mx[a]) {
            return false;
        }
    }
    t0 = lo;
    t1 = hi;
    return hi > lo;
}

// Exponential free-flight length in units of the mean free path, -ln(1 - u), for u on the
// 2^-24 grid in [0, 1): 1 - u is exact and at least 2^-24, so the hardware base-2 logarithm
// (v_log_f32, no denormal inputs here) times ln 2 serves.
__device__ __forceinline__ float exp_flight(float u)
{
    return -__builtin_amdgcn_logf(1.f - u) * 0.693147180559945f;
}

// Free flight from o along unit d: true and the collision point, false on escape.
__device__ bool delta_track(const Medium &M, V3 o, V3 d, Rng &r, V3 &x, int64_t &steps)
{
    float t0, t1;
    if (!clip(M, o, d, t0, t1) || !(M.maj > 0.f))
        return false;
    float t = t0;
    const float inv = M.inv_ff;
    const int64_t s0 = steps;
    while (steps < kMaxSteps) {
        ++steps;
        t += exp_flight(r.u()) * inv;
        if (t >= t1)
            return false;
        const V3 p = madd(o, t, d);
        if (r.u() * M.maj < mu_at(M, p)) {
            x = p;
            return true;
        }
    }
    note_cap(M, s0, steps);
    return false;
}

// Ratio-tracking estimate of the transmittance from o along unit d to the box exit.
__device__ float ratio_track(const Medium &M, V3 o, V3 d, Rng &r, int64_t &steps)
{
    float t0, t1;
    if (!clip(M, o, d, t0, t1) || !(M.maj > 0.f))
        return 1.f;
    float T = 1.f, t = t0;
    const float inv = 1.f / M.maj;
    const int64_t s0 = steps;
    while (steps < kMaxSteps) {
        ++steps;
        t += exp_flight(r.u()) * M.inv_ff;
        if (t >= t1)
            return T;
        T *= 1.f - mu_at(M, madd(o, t, d)) * inv;
    }
    note_cap(M, s0, steps);
    return T;
}

__device__ __forceinline__ float hg(float g, float mu)
{
    const float den = 1.f + g * g - 2.f * g * mu;
    return (1.f - g * g) / (4.f * (float)M_PI * den * sqrtf(den));
}

// Inverse-CDF sample of the Henyey-Greenstein cosine (isotropic for |g| < 1e-3).
__device__ __forceinline__ float hg_cos(float g, float u)
{
    if (fabsf(g) < 1e-3f)
        return 2.f * u - 1.f;
    const float s = (1.f - g * g) / (1.f - g + 2.f * g * u);
    return fminf(1.f, fmaxf(-1.f, (1.f + g * g - s * s) / (2.f * g)));
}

// Tabulated phase function p at theta_i = i pi / (n - 1): linear in theta between nodes.
__device__ __forceinline__ float tab_eval(const float *p, int n, float mu)
{
    const float th = acosf(fminf(1.f, fmaxf(-1.f, mu))) * ((float)(n - 1) / (float)M_PI);
    const int i = min((int)th, n - 2);
    const float f = th - (float)i;
    return fmaf(f, p[i + 1] - p[i], p[i]);
}

// cos(theta) from the table: the node interval by binary search of the CDF, then theta
// inside it from the density linear between the nodes' p sin(theta) (the root of the
// interval's quadratic CDF, in the form without cancellation).
__device__ __forceinline__ float tab_sample(const float *p, const float *cdf, int n, float u)
{
    int lo = 0, hi = n - 1;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (cdf[mid] <= u)
            lo = mid;
        else
            hi = mid;
    }
    const float dth = (float)M_PI / (float)(n - 1);
    const float fa = p[lo] * sinf((float)lo * dth), fb = p[lo + 1] * sinf((float)(lo + 1) * dth);
    const float den = cdf[lo + 1] - cdf[lo];
    const float q = den > 0.f ? (u - cdf[lo]) / den : 0.f;
    const float sq = sqrtf(fmaxf(0.f, fa * fa + (fb - fa) * q * (fa + fb)));
    const float t = fa + sq > 0.f ? fminf(1.f, fmaxf(0.f, q * (fa + fb) / (fa + sq))) : q;
    return cosf(((float)lo + t) * dth);
}

// Phase function of the medium: the table when one is set (first: the first-collision
// table of camera rays, else the scattering table), else Henyey-Greenstein.  TAB (any
// table set) is a compile-time choice, so the kernels without tables keep the registers
// (and the occupancy) of the plain Henyey-Greenstein code.
template <bool TAB>
__device__ __forceinline__ float phase_eval(const TracerParams &tp, bool first, float mu)
{
    if constexpr (TAB) {
        if (first && tp.pf_n)
            return tp.pf_scale * tab_eval(tp.pf_p, tp.pf_n, mu);
        if (tp.ph_n)
            return tab_eval(tp.ph_p, tp.ph_n, mu);
    }
    return hg(tp.g, mu);
}

template <bool TAB> __device__ __forceinline__ float phase_sample(const TracerParams &tp, float u)
{
    if constexpr (TAB) {
        if (tp.ph_n)
            return tab_sample(tp.ph_p, tp.ph_cdf, tp.ph_n, u);
    }
    return hg_cos(tp.g, u);
}

__device__ V3 around(V3 w, float c, float u)
{
    V3 t1, t2;
    basis(w, t1, t2);
    const float s = sqrtf(fmaxf(0.f, 1.f - c * c));
    float sp, cp;
    sincosf(2.f * (float)M_PI * u, &sp, &cp);
    V3 o = v3(s * cp * t1.x + s * sp * t2.x + c * w.x, s * cp * t1.y + s * sp * t2.y + c * w.y,
              s * cp * t1.z + s * sp * t2.z + c * w.z);
    const float l = sqrtf(dot(o, o));
    return v3(o.x / l, o.y / l, o.z / l);
}

// One path estimate of the indirect in-scattered radiance at x toward w
// (directional light: next-event estimation at every collision; uniform
// environment: the radiance of escaping paths after at least one collision, or
// any escape when count_uncollided).
template <bool TAB, bool SET>
__device__ float li_path(const Medium &M, const TracerParams &tp, V3 x, V3 w, V3 wl,
                         bool count_uncollided, Rng &r)
{
    V3 wprev = w, p = x;
    float sum = 0.f;
    int64_t steps = 0;
    for (int j = 1;; ++j) {
        if ((tp.max_interactions > 0 && j > tp.max_interactions) || steps >= kMaxSteps)
            break;
        const float c = phase_sample<TAB>(tp, r.u());
        const V3 wh = around(wprev, c, r.u());
        V3 xn;
        if (!delta_track(M, p, neg(wh), r, xn, steps)) {
            if (tp.light_mode == 1 && (j > 1 || count_uncollided))
                sum += tp.irradiance;
            break;
        }
        p = xn;
        if (r.u() >= tp.albedo)
            break;
        if constexpr (SET) {
            const float4 lw = tp.set_dw[set_pick(tp, r)];
            const V3 lj = v3(lw.x, lw.y, lw.z);
            sum += lw.w * phase_eval<TAB>(tp, false, -dot(wh, lj)) *
                   ratio_track(M, p, lj, r, steps) * tp.irradiance;
        } else if (tp.light_mode == 0) {
            sum += phase_eval<TAB>(tp, false, -dot(wh, wl)) * ratio_track(M, p, wl, r, steps) *
                   tp.irradiance;
        }
        wprev = wh;
    }
    return sum;
}

// Launch geometry of the per-record estimators: a block holds kPaths / seg
// records, each owning seg consecutive threads (seg a power of two); records with
// more than kPaths samples are split over nblk blocks (then seg = kPaths), whose
// partial sums k_finish_sums adds in block order.
struct Split {
    int seg, nblk;
};

// Deterministic segmented reduction of (sum, sum of squares) in FP64: thread
// t of each segment ends holding nothing; the segment leader writes the totals.
__device__ void segment_sums(double s1, double s2, int seg, bool write, double *out)
{
    __shared__ double a[kPaths], b[kPaths];
    const int t = threadIdx.x;
    a[t] = s1;
    b[t] = s2;
    __syncthreads();
    for (int w = seg >> 1; w > 0; w >>= 1) {
        if ((t & (seg - 1)) < w) {
            a[t] += a[t + w];
            b[t] += b[t + w];
        }
        __syncthreads();
    }
    if (write && (t & (seg - 1)) == 0) {
        out[0] = a[t];
        out[1] = b[t];
    }
}

// One record estimate: L_i, or with tp.include_direct all in-scattered radiance L_s =
// L_d + L_i (directional light: the direct term by ratio tracking, drawn before the path;
// uniform environment: uncollided light counted too).
template <bool TAB, bool DIRECT>
__device__ float record_path(const Medium &M, const TracerParams &tp, V3 x, V3 w, V3 wl, Rng &r)
{
    if constexpr (!DIRECT) {
        return li_path<TAB, false>(M, tp, x, w, wl, false, r);
    } else {
        if (tp.light_mode == 1)
            return li_path<TAB, false>(M, tp, x, w, wl, true, r);
        int64_t steps = 0;
        const float d =
            phase_eval<TAB>(tp, false, -dot(w, wl)) * ratio_track(M, x, wl, r, steps) * tp.irradiance;
        return d + li_path<TAB, false>(M, tp, x, w, wl, false, r);
    }
}

// Paths s0 .. s0 + spp - 1 of every record (path s on stream id rec * 2^20 + s).
template <bool TAB, bool DIRECT>
__global__ void __launch_bounds__(kPaths) k_trace_li(Medium M, TracerParams tp, const float *pos,
                                                     const float *view, const float *light,
                                                     int64_t P, int s0, int spp, Split sp,
                                                     uint64_t seed, const uint8_t *mask,
                                                     uint8_t mask_bits, double *partial)
{
    const int64_t group = blockIdx.x / sp.nblk;
    const int blk = blockIdx.x % sp.nblk;
    const int64_t rec = group * (kPaths / sp.seg) + threadIdx.x / sp.seg;
    const int s = blk * sp.seg + (threadIdx.x & (sp.seg - 1));
    double e = 0.0;
    V3 w, wl;
    const bool wanted = rec < P && (!mask || (mask[rec] & mask_bits) == mask_bits);
    if (wanted && s < spp && unit(view + 3 * rec, w) && unit(light + 3 * rec, wl)) {
        const V3 x = v3(pos[3 * rec], pos[3 * rec + 1], pos[3 * rec + 2]);
        Rng r;
        r.init(seed, ((uint64_t)rec << 20) + (uint64_t)(s0 + s));
        e = (double)record_path<TAB, DIRECT>(M, tp, x, w, wl, r);
    }
    segment_sums(e, e * e, sp.seg, rec < P, partial + 2 * ((size_t)rec * sp.nblk + blk));
}

__global__ void __launch_bounds__(256) k_finish_sums(const double *partial, int64_t P, int nblk,
                                                     int spp, double *mean, double *var)
{
    const int64_t rec = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (rec >= P)
        return;
    double s1 = 0.0, s2 = 0.0;
    for (int b = 0; b < nblk; ++b) {
        s1 += partial[2 * (rec * nblk + b)];
        s2 += partial[2 * (rec * nblk + b) + 1];
    }
    const double m = s1 / spp;
    mean[rec] = m;
    if (var)
        var[rec] = spp > 1 ? fmax(0.0, (s2 - spp * m * m) / (spp - 1)) / spp : 0.0;
}

// Progressive estimates (Sec. 5.1).  k_adapt_init marks the records with usable
// directions active and zeroes their sums; after each batch of paths k_adapt_step adds
// the batch's per-block partial sums (in block order), and a record stops once
// zq * sqrt(variance of the mean) <= rel * |mean| or max_spp paths are reached, writing
// its mean, variance of the mean and path count; records still active are counted.
__global__ void __launch_bounds__(256) k_adapt_init(const float *view, const float *light,
                                                    int64_t P, uint8_t *active, double *sums,
                                                    double *mean, double *var, int32_t *n_out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P)
        return;
    V3 w, wl;
    active[i] = unit(view + 3 * i, w) && unit(light + 3 * i, wl) ? 1 : 0;
    sums[2 * i] = 0.0;
    sums[2 * i + 1] = 0.0;
    mean[i] = 0.0;
    if (var)
        var[i] = 0.0;
    if (n_out)
        n_out[i] = 0;
}

// Batches j = 0 .. kb - 1 of one round, in order: batch j's nb block partials (blocks
// j nb .. j nb + nb - 1 of the round's kb nb) join the record's running sums, and the rule
// is checked after each, so a record stops at the same batch as with one batch per round;
// later batches of a stopped record are discarded.
__global__ void __launch_bounds__(256) k_adapt_step(const double *partial, int nb, int kb,
                                                    int64_t P, int n0, int batch, int max_spp,
                                                    double rel, double zq, uint8_t *active,
                                                    double *sums, double *mean, double *var,
                                                    int32_t *n_out, unsigned long long *left)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P || !active[i])
        return;
    double s1 = sums[2 * i], s2 = sums[2 * i + 1];
    const int64_t nblk = (int64_t)nb * kb;
    for (int j = 0; j < kb; ++j) {
        for (int b = j * nb; b < (j + 1) * nb; ++b) {
            s1 += partial[2 * (i * nblk + b)];
            s2 += partial[2 * (i * nblk + b) + 1];
        }
        const int n = n0 + (j + 1) * batch;
        const double m = s1 / n;
        const double vm = fmax(0.0, (s2 - n * m * m) / (n - 1)) / n;
        if (zq * sqrt(vm) <= rel * fabs(m) || n >= max_spp) {
            active[i] = 0;
            mean[i] = m;
            if (var)
                var[i] = vm;
            if (n_out)
                n_out[i] = n;
            return;
        }
    }
    sums[2 * i] = s1;
    sums[2 * i + 1] = s2;
    atomicAdd(left, 1ull);
}

// Record configurations (Sec. 5.1): direction d uniform on the sphere, origin
// uniform over the bounding sphere's cross-section orthogonal to d, a free flight
// along d into the cloud, retried on escape; view = -d, light uniform.
__global__ void __launch_bounds__(256) k_sample_records(Medium M, int64_t N, uint64_t seed,
                                                        float *pos, float *view, float *light,
                                                        int32_t *attempts)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N)
        return;
    const V3 c = v3(0.5f * (M.amin.x + M.amax.x), 0.5f * (M.amin.y + M.amax.y),
                    0.5f * (M.amin.z + M.amax.z));
    const V3 e = v3(0.5f * (M.amax.x - M.amin.x), 0.5f * (M.amax.y - M.amin.y),
                    0.5f * (M.amax.z - M.amin.z));
    const float R = sqrtf(dot(e, e));
    Rng r;
    r.init(seed, (uint64_t)i);
    V3 d = v3(0, 0, 1), x = v3(NAN, NAN, NAN);
    int tries = 0;
    int64_t steps = 0;
    while (tries < 1000000) {
        ++tries;
        const float u0 = r.u(), u1 = r.u();
        const float zc = 1.f - 2.f * u0, rr = sqrtf(fmaxf(0.f, 1.f - zc * zc));
        float sp, cp;
        sincosf(2.f * (float)M_PI * u1, &sp, &cp);
        d = v3(rr * cp, rr * sp, zc);
        V3 t1, t2;
        basis(d, t1, t2);
        const float rad = R * sqrtf(r.u());
        sincosf(2.f * (float)M_PI * r.u(), &sp, &cp);
        const V3 o = v3(c.x - R * d.x + rad * (cp * t1.x + sp * t2.x),
                        c.y - R * d.y + rad * (cp * t1.y + sp * t2.y),
                        c.z - R * d.z + rad * (cp * t1.z + sp * t2.z));
        steps = 0;
        if (delta_track(M, o, d, r, x, steps))
            break;
        x = v3(NAN, NAN, NAN);
    }
    const float u0 = r.u(), u1 = r.u();
    const float zc = 1.f - 2.f * u0, rr = sqrtf(fmaxf(0.f, 1.f - zc * zc));
    float sp, cp;
    sincosf(2.f * (float)M_PI * u1, &sp, &cp);
    pos[3 * i] = x.x;
    pos[3 * i + 1] = x.y;
    pos[3 * i + 2] = x.z;
    view[3 * i] = -d.x;
    view[3 * i + 1] = -d.y;
    view[3 * i + 2] = -d.z;
    light[3 * i] = rr * cp;
    light[3 * i + 1] = rr * sp;
    light[3 * i + 2] = zc;
    if (attempts)
        attempts[i] = tries;
}

// Path-traced pixels: first collision along each camera ray, then albedo times the
// in-scattered radiance there (direct by next-event estimation plus the indirect
// path estimate for a directional light; all in-scattered environment light in mode 1).
template <bool TAB, bool SET>
__global__ void __launch_bounds__(kPaths) k_render_mc(Medium M, TracerParams tp, V3 wl,
                                                      const float *ray_o, const float *ray_d,
                                                      int64_t N, int spp, Split sp, uint64_t seed,
                                                      double *partial)
{
    const int64_t group = blockIdx.x / sp.nblk;
    const int blk = blockIdx.x % sp.nblk;
    const int64_t px = group * (kPaths / sp.seg) + threadIdx.x / sp.seg;
    const int s = blk * sp.seg + (threadIdx.x & (sp.seg - 1));
    double e = 0.0;
    V3 d;
    if (px < N && s < spp && unit(ray_d + 3 * px, d)) {
        const V3 o = v3(ray_o[3 * px], ray_o[3 * px + 1], ray_o[3 * px + 2]);
        Rng r;
        r.init(seed, ((uint64_t)px << 20) + (uint64_t)s);
        V3 x;
        int64_t steps = 0;
        if (!delta_track(M, o, d, r, x, steps)) {
            e = tp.light_mode == 1 ? tp.irradiance : 0.0;
        } else {
            const V3 w = neg(d);
            if constexpr (SET) {
                const float4 lw = tp.set_dw[set_pick(tp, r)];
                const V3 lj = v3(lw.x, lw.y, lw.z);
                const float direct = lw.w * phase_eval<TAB>(tp, true, -dot(w, lj)) *
                                     ratio_track(M, x, lj, r, steps) * tp.irradiance;
                e = (double)tp.albedo *
                    (double)(direct + li_path<TAB, true>(M, tp, x, w, wl, false, r));
            } else if (tp.light_mode == 0) {
                const float direct = phase_eval<TAB>(tp, true, -dot(w, wl)) *
                                     ratio_track(M, x, wl, r, steps) * tp.irradiance;
                e = (double)tp.albedo *
                    (double)(direct + li_path<TAB, false>(M, tp, x, w, wl, false, r));
            } else {
                e = (double)tp.albedo * (double)li_path<TAB, false>(M, tp, x, w, wl, true, r);
            }
        }
    }
    segment_sums(e, e * e, sp.seg, px < N, partial + 2 * ((size_t)px * sp.nblk + blk));
}

// One camera sample per ray for the network renderer: the delta-tracked first
// collision, the view direction there, and the direct single scattering from the
// directional light (next-event estimation, times the albedo).  Rays that escape
// get hit = 0 and zero outputs.
__global__ void __launch_bounds__(256) k_first_hits(Medium M, TracerParams tp, V3 wl,
                                                    const float *ray_o, const float *ray_d,
                                                    int64_t N, uint64_t seed, uint64_t sample,
                                                    float *pos, float *view, float *direct,
                                                    uint8_t *hit)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N)
        return;
    V3 d;
    bool h = false;
    float dir = 0.f;
    V3 x = v3(0, 0, 0);
    if (unit(ray_d + 3 * i, d)) {
        const V3 o = v3(ray_o[3 * i], ray_o[3 * i + 1], ray_o[3 * i + 2]);
        Rng r;
        r.init(seed, ((uint64_t)i << 20) + sample);
        int64_t steps = 0;
        h = delta_track(M, o, d, r, x, steps);
        if (h)
            dir = tp.albedo * phase_eval<true>(tp, true, dot(d, wl)) * ratio_track(M, x, wl, r, steps) *
                  tp.irradiance;
    }
    pos[3 * i] = x.x;
    pos[3 * i + 1] = x.y;
    pos[3 * i + 2] = x.z;
    view[3 * i] = h ? -d.x : 0.f;
    view[3 * i + 1] = h ? -d.y : 0.f;
    view[3 * i + 2] = h ? -d.z : 0.f;
    direct[i] = dir;
    hit[i] = h ? 1 : 0;
}

// Camera samples under a light set: the first collision as k_first_hits, then `draws`
// members of the set, each drawn by one uniform and followed by one ratio-tracking
// estimate toward it, on the same stream in draw order.  Row i * draws + q receives the
// collision, the view direction, the drawn direction and its weight; rays that escape
// get zero rows.
__global__ void __launch_bounds__(256) k_first_hits_set(Medium M, TracerParams tp, int draws,
                                                        const float *ray_o, const float *ray_d,
                                                        int64_t N, uint64_t seed, uint64_t sample,
                                                        float *pos, float *view, float *light,
                                                        float *weight, float *direct, uint8_t *hit)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N)
        return;
    V3 d;
    bool h = false;
    V3 x = v3(0, 0, 0);
    Rng r;
    int64_t steps = 0;
    if (unit(ray_d + 3 * i, d)) {
        const V3 o = v3(ray_o[3 * i], ray_o[3 * i + 1], ray_o[3 * i + 2]);
        r.init(seed, ((uint64_t)i << 20) + sample);
        h = delta_track(M, o, d, r, x, steps);
    }
    float sum = 0.f;
    for (int q = 0; q < draws; ++q) {
        const int64_t row = i * draws + q;
        float4 lw = make_float4(0.f, 0.f, 0.f, 0.f);
        if (h) {
            lw = tp.set_dw[set_pick(tp, r)];
            const V3 lj = v3(lw.x, lw.y, lw.z);
            sum += lw.w * phase_eval<true>(tp, true, dot(d, lj)) * ratio_track(M, x, lj, r, steps);
        }
        pos[3 * row] = x.x;
        pos[3 * row + 1] = x.y;
        pos[3 * row + 2] = x.z;
        view[3 * row] = h ? -d.x : 0.f;
        view[3 * row + 1] = h ? -d.y : 0.f;
        view[3 * row + 2] = h ? -d.z : 0.f;
        light[3 * row] = lw.x;
        light[3 * row + 1] = lw.y;
        light[3 * row + 2] = lw.z;
        weight[row] = lw.w;
    }
    direct[i] = h ? tp.albedo * tp.irradiance * sum / (float)draws : 0.f;
    hit[i] = h ? 1 : 0;
}

__global__ void __launch_bounds__(256) k_mu(const void *d, ds_dtype dt, int64_t n, float sigma,
                                            float *mu)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        float v;
        if (dt == DS_F32)
            v = static_cast<const float *>(d)[i];
        else
            v = __uint_as_float((uint32_t) static_cast<const uint16_t *>(d)[i] << 16);
        mu[i] = sigma * v;
    }
}

__global__ void __launch_bounds__(256) k_max(const float *x, int64_t n, float *out)
{
    __shared__ float s[256];
    float m = 0.f;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        m = fmaxf(m, x[i]);
    s[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            s[threadIdx.x] = fmaxf(s[threadIdx.x], s[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0)
        out[blockIdx.x] = s[0];
}

__global__ void __launch_bounds__(256) k_philox(const uint32_t *ck, int64_t n, uint32_t *out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    Rng r;
    r.c0 = ck[6 * i];
    r.c1 = ck[6 * i + 1];
    r.c2 = ck[6 * i + 2];
    r.c3 = ck[6 * i + 3];
    r.k0 = ck[6 * i + 4];
    r.k1 = ck[6 * i + 5];
    r.refill();
#pragma unroll
    for (int j = 0; j < 4; ++j)
        out[4 * i + j] = r.buf[j];
}

// Training targets: t = log(1 + L_i) in FP32 at record stride `stride`.
__global__ void __launch_bounds__(256) k_targets(const double *li, int64_t N, int64_t stride,
                                                 float *t)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N)
        t[i * stride] = log1pf((float)li[i]);
}

// One camera sample per pixel added to the pixel sums (Sec. 4.4): radiance
// direct + albedo * E * L_i at a collision, with L_i from the network or, where
// the stencil leaves the grid (fallback flag), from the path-traced estimate; 0 for
// rays that escape.  sums holds (sum, sum of squares) per pixel in FP64; dsum the
// sum of the direct term alone.
__global__ void __launch_bounds__(256) k_accumulate(int64_t N, const uint8_t *hit,
                                                    const float *direct, const float *li_net,
                                                    const uint8_t *flags, const double *li_mc,
                                                    float albedo, float E, double *sums,
                                                    double *dsum, unsigned long long *n_fb)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N)
        return;
    double e = 0.0, d = 0.0;
    if (hit[i]) {
        const bool fb = li_mc && (flags[i] & DS_FLAG_FALLBACK);
        const double li = fb ? li_mc[i] : (double)E * (double)li_net[i];
        d = (double)direct[i];
        e = d + (double)albedo * li;
        if (fb && n_fb)
            atomicAdd(n_fb, 1ull);
    }
    sums[2 * i] += e;
    sums[2 * i + 1] += e * e;
    if (dsum)
        dsum[2 * i] += d;
}

// One camera sample per pixel under a light set: direct + albedo * E * (1 / draws) *
// sum over the draws of weight * L_i (the network's per unit irradiance, or the
// path-traced estimate where the row's fallback flag is set).
__global__ void __launch_bounds__(256) k_accumulate_set(int64_t N, int draws, const uint8_t *hit,
                                                        const float *direct, const float *li_net,
                                                        const uint8_t *flags, const double *li_mc,
                                                        const float *weight, float albedo, float E,
                                                        double *sums, double *dsum,
                                                        unsigned long long *n_fb)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N)
        return;
    double e = 0.0, d = 0.0;
    if (hit[i]) {
        double li = 0.0;
        unsigned long long nf = 0;
        for (int q = 0; q < draws; ++q) {
            const int64_t row = i * draws + q;
            const bool fb = li_mc && (flags[row] & DS_FLAG_FALLBACK);
            li += (double)weight[row] * (fb ? li_mc[row] : (double)li_net[row]);
            nf += fb ? 1 : 0;
        }
        d = (double)direct[i];
        e = d + (double)albedo * (double)E * li / draws;
        if (nf && n_fb)
            atomicAdd(n_fb, nf);
    }
    sums[2 * i] += e;
    sums[2 * i + 1] += e * e;
    if (dsum)
        dsum[2 * i] += d;
}

__global__ void __launch_bounds__(256) k_fill3(float *v, int64_t N, float x, float y, float z)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) {
        v[3 * i] = x;
        v[3 * i + 1] = y;
        v[3 * i + 2] = z;
    }
}

__global__ void __launch_bounds__(256) k_zero64(double *v, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        v[i] = 0.0;
}

#define DS_TRY_MEDIUM(s, c)                \
    do {                                   \
        ds_status st_ = medium_cells(s, c); \
        if (st_)                           \
            return st_;                    \
    } while (0)

// The corner-packed extinction of the cloud, built on the first tracer call.
ds_status medium_cells(hipStream_t s, const ds_cloud *c)
{
    if (c->mu_cells)
        return DS_OK;
    const int64_t n = (int64_t)(c->nx + 2) * (c->ny + 2) * (c->nz + 2);
    float4 *cells = nullptr;
    DS_CHECK(hipMalloc(&cells, sizeof(float4) * 2 * (size_t)n) == hipSuccess, DS_ERR_OOM,
             "out of device memory for the corner-packed extinction (%lld cells of 32 bytes)",
             (long long)n);
    Level base = {};
    base.nx = c->nx;
    base.ny = c->ny;
    base.nz = c->nz;
    ds_status st = cloud_pack32(s, c->mu, 1, &base, cells);
    if (st) {
        (void)hipFree(cells);
        return st;
    }
    c->mu_cells = cells;
    return DS_OK;
}

Medium medium(const ds_cloud *c, float ext_scale = 1.f)
{
    Medium M;
    M.cells = c->mu_cells;
    M.cx = c->nx + 2;
    M.cy = c->ny + 2;
    M.hx = (float)(c->nx + 1);
    M.hy = (float)(c->ny + 1);
    M.hz = (float)(c->nz + 1);
    M.amin = v3(c->aabb_min[0], c->aabb_min[1], c->aabb_min[2]);
    M.amax = v3((float)((double)c->aabb_min[0] + (double)c->nx * c->h0),
                (float)((double)c->aabb_min[1] + (double)c->ny * c->h0),
                (float)((double)c->aabb_min[2] + (double)c->nz * c->h0));
    M.inv_h = (float)(1.0 / (double)c->h0);
    M.maj = c->majorant;
    M.inv_ff = (float)(1.0 / ((double)c->majorant * (double)ext_scale));
    M.truncated = c->ctx->truncated;
    return M;
}

Split split(int spp)
{
    Split sp;
    sp.nblk = (spp + kPaths - 1) / kPaths;
    sp.seg = 1;
    while (sp.seg < spp && sp.seg < kPaths)
        sp.seg <<= 1;
    return sp;
}

unsigned grid_of(int64_t n, Split sp)
{
    const int64_t rpb = kPaths / sp.seg;
    return (unsigned)(((n + rpb - 1) / rpb) * sp.nblk);
}

ds_status reduce_records(hipStream_t s, const double *partial, int64_t P, int nblk, int spp,
                         double *mean, double *var)
{
    k_finish_sums<<<(unsigned)((P + 255) / 256), 256, 0, s>>>(partial, P, nblk, spp, mean, var);
    DS_HIP(hipGetLastError());
    return DS_OK;
}

// The specialisation of the path kernels a call needs: tabulated phase functions and
// L_s records (k_trace_li), tables and light sets (k_render_mc).
void launch_trace_li(hipStream_t s, const ds_cloud *c, const TracerParams &tp, const float *pos,
                     const float *view, const float *light, int64_t P, int s0, int spp, Split sp,
                     uint64_t seed, const uint8_t *mask, uint8_t mask_bits, double *partial)
{
    const bool tab = tp.ph_n > 0 || tp.pf_n > 0, dir = tp.include_direct != 0;
    auto k = tab ? (dir ? k_trace_li<true, true> : k_trace_li<true, false>)
                 : (dir ? k_trace_li<false, true> : k_trace_li<false, false>);
    k<<<grid_of(P, sp), kPaths, 0, s>>>(medium(c, tp.ext_scale), tp, pos, view, light, P, s0, spp, sp, seed,
                                         mask, mask_bits, partial);
}

void launch_render_mc(hipStream_t s, const ds_cloud *c, const TracerParams &tp, V3 wl,
                      const float *ray_o, const float *ray_d, int64_t N, int spp, Split sp,
                      uint64_t seed, double *partial)
{
    const bool tab = tp.ph_n > 0 || tp.pf_n > 0, set = tp.light_mode == kLightSetMode;
    auto k = tab ? (set ? k_render_mc<true, true> : k_render_mc<true, false>)
                 : (set ? k_render_mc<false, true> : k_render_mc<false, false>);
    k<<<grid_of(N, sp), kPaths, 0, s>>>(medium(c, tp.ext_scale), tp, wl, ray_o, ray_d, N, spp, sp, seed,
                                         partial);
}

}  // namespace

ds_status tracer_prepare(ds_cloud *c, const void *density, ds_dtype dt)
{
    const int64_t n = (int64_t)c->nx * c->ny * c->nz;
    DS_CHECK(hipMalloc(&c->mu, (size_t)n * sizeof(float)) == hipSuccess, DS_ERR_OOM,
             "out of device memory for the extinction grid");
    hipStream_t s = c->ctx->stream;
    int grid = (int)((n + 255) / 256 < 16384 ? (n + 255) / 256 : 16384);
    k_mu<<<grid, 256, 0, s>>>(density, dt, n, c->sigma_max, c->mu);
    float *part = nullptr;
    DS_HIP(hipMalloc(&part, 1024 * sizeof(float)));
    k_max<<<1024, 256, 0, s>>>(c->mu, n, part);
    k_max<<<1, 256, 0, s>>>(part, 1024, part);
    float mx = 0.f;
    hipError_t e = hipGetLastError();
    if (e == hipSuccess)
        e = hipMemcpyAsync(&mx, part, sizeof(float), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    (void)hipFree(part);
    if (e != hipSuccess)
        return hip_fail(e, "majorant");
    c->majorant = mx;
    return DS_OK;
}

ds_status tracer_li(hipStream_t s, const ds_cloud *c, const TracerParams &tp, const float *pos,
                    const float *view, const float *light, int64_t P, int spp, uint64_t seed,
                    double *partial, double *mean, double *var, const uint8_t *mask,
                    uint8_t mask_bits)
{
    const Split sp = split(spp);
    DS_TRY_MEDIUM(s, c);
    launch_trace_li(s, c, tp, pos, view, light, P, 0, spp, sp, seed, mask, mask_bits, partial);
    DS_HIP(hipGetLastError());
    return reduce_records(s, partial, P, sp.nblk, spp, mean, var);
}

// Batches a round of the progressive estimate traces: one while the records still running
// fill the GPU (kAheadThreads threads), more as they thin out, up to `ahead`.  Tracing
// several batches at once keeps every block partial and its order (the batch is a whole
// number of blocks), so estimates and path counts equal those of one batch per round.
constexpr int64_t kAheadThreads = 1ll << 21;

ds_status tracer_li_adaptive(hipStream_t s, const ds_cloud *c, const TracerParams &tp,
                             const float *pos, const float *view, const float *light, int64_t P,
                             int batch, int max_spp, int ahead, double rel, double zq,
                             uint64_t seed, double *partial, uint8_t *active, double *sums,
                             unsigned long long *left, double *mean, double *var, int32_t *n_out,
                             int *rounds)
{
    const Split sp1 = split(batch);
    const bool whole = batch % kPaths == 0;
    const unsigned g256 = (unsigned)((P + 255) / 256);
    DS_TRY_MEDIUM(s, c);
    k_adapt_init<<<g256, 256, 0, s>>>(view, light, P, active, sums, mean, var, n_out);
    DS_HIP(hipGetLastError());
    int r = 0;
    int64_t live = P;
    for (int n = 0; n < max_spp;) {
        int kb = 1;
        if (whole && ahead > 1) {
            const int64_t want = (kAheadThreads + live * batch - 1) / (live * batch);
            kb = (int)std::max<int64_t>(
                1, std::min<int64_t>(want, std::min<int64_t>(ahead, (max_spp - n) / batch)));
        }
        ++r;
        launch_trace_li(s, c, tp, pos, view, light, P, n, kb * batch,
                        kb == 1 ? sp1 : split(kb * batch), seed, active, 1, partial);
        DS_HIP(hipGetLastError());
        unsigned long long h = 0;
        DS_HIP(hipMemsetAsync(left, 0, sizeof(*left), s));
        k_adapt_step<<<g256, 256, 0, s>>>(partial, sp1.nblk, kb, P, n, batch, max_spp, rel, zq,
                                          active, sums, mean, var, n_out, left);
        DS_HIP(hipGetLastError());
        DS_HIP(hipMemcpyAsync(&h, left, sizeof(h), hipMemcpyDeviceToHost, s));
        DS_HIP(hipStreamSynchronize(s));
        n += kb * batch;
        if (h == 0)
            break;
        live = (int64_t)h;
    }
    if (rounds)
        *rounds = r;
    return DS_OK;
}

// Batches ahead a progressive estimate of P records may trace in one round: 1 unless a
// batch is a whole number of blocks; else up to 64 (and the cap), within 256 MiB of
// partial sums.
int tracer_adaptive_ahead(int64_t P, int batch, int max_spp)
{
    if (batch % kPaths != 0 || P <= 0)
        return 1;
    const int64_t per = 16 * P * (batch / kPaths);
    const int64_t k = std::min<int64_t>(std::min<int64_t>(64, max_spp / batch),
                                        (256ll << 20) / per);
    return (int)std::max<int64_t>(1, k);
}

ds_status tracer_records(hipStream_t s, const ds_cloud *c, int64_t N, uint64_t seed, float *pos,
                         float *view, float *light, int32_t *attempts)
{
    DS_TRY_MEDIUM(s, c);
    k_sample_records<<<(unsigned)((N + 255) / 256), 256, 0, s>>>(medium(c), N, seed, pos, view,
                                                                 light, attempts);
    DS_HIP(hipGetLastError());
    return DS_OK;
}

ds_status tracer_render(hipStream_t s, const ds_cloud *c, const TracerParams &tp,
                        const float *light_dir, const float *ray_o, const float *ray_d, int64_t N,
                        int spp, uint64_t seed, double *partial, double *mean, double *var)
{
    float l[3];
    DS_CHECK(light_dir && unit_host(light_dir, l), DS_ERR_INVALID_ARG,
             "the light direction is not a usable vector");
    const V3 wl = v3(l[0], l[1], l[2]);
    const Split sp = split(spp);
    DS_TRY_MEDIUM(s, c);
    launch_render_mc(s, c, tp, wl, ray_o, ray_d, N, spp, sp, seed, partial);
    DS_HIP(hipGetLastError());
    return reduce_records(s, partial, N, sp.nblk, spp, mean, var);
}

ds_status tracer_first_hits(hipStream_t s, const ds_cloud *c, const TracerParams &tp,
                            const float *light_dir, const float *ray_o, const float *ray_d,
                            int64_t N, uint64_t seed, uint64_t sample, float *pos, float *view,
                            float *direct, uint8_t *hit)
{
    float l[3];
    DS_CHECK(light_dir && unit_host(light_dir, l), DS_ERR_INVALID_ARG,
             "the light direction is not a usable vector");
    const V3 wl = v3(l[0], l[1], l[2]);
    DS_TRY_MEDIUM(s, c);
    k_first_hits<<<(unsigned)((N + 255) / 256), 256, 0, s>>>(medium(c, tp.ext_scale), tp, wl, ray_o, ray_d, N,
                                                             seed, sample, pos, view, direct, hit);
    DS_HIP(hipGetLastError());
    return DS_OK;
}

ds_status philox_blocks(hipStream_t s, const uint32_t *ctr_key, int64_t n, uint32_t *out)
{
    k_philox<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(ctr_key, n, out);
    DS_HIP(hipGetLastError());
    return DS_OK;
}

ds_status tracer_targets(hipStream_t s, const double *li, int64_t N, int64_t stride, float *t)
{
    k_targets<<<(unsigned)((N + 255) / 256), 256, 0, s>>>(li, N, stride, t);
    DS_HIP(hipGetLastError());
    return DS_OK;
}

ds_status tracer_accumulate(hipStream_t s, int64_t N, const uint8_t *hit, const float *direct,
                            const float *li_net, const uint8_t *flags, const double *li_mc,
                            float albedo, float E, double *sums, double *dsum,
                            unsigned long long *n_fb)
{
    k_accumulate<<<(unsigned)((N + 255) / 256), 256, 0, s>>>(N, hit, direct, li_net, flags, li_mc,
                                                             albedo, E, sums, dsum, n_fb);
    DS_HIP(hipGetLastError());
    return DS_OK;
}

ds_status tracer_fill3(hipStream_t s, float *v, int64_t N, const float *xyz)
{
    k_fill3<<<(unsigned)((N + 255) / 256), 256, 0, s>>>(v, N, xyz[0], xyz[1], xyz[2]);
    DS_HIP(hipGetLastError());
    return DS_OK;
}

ds_status tracer_zero(hipStream_t s, double *v, int64_t n)
{
    int64_t b = (n + 255) / 256;
    k_zero64<<<(unsigned)(b > 4096 ? 4096 : (b < 1 ? 1 : b)), 256, 0, s>>>(v, n);
    DS_HIP(hipGetLastError());
    return DS_OK;
}

ds_status tracer_finish(hipStream_t s, const double *sums, int64_t N, int spp, double *mean,
                        double *var)
{
    return reduce_records(s, sums, N, 1, spp, mean, var);
}

ds_status tracer_first_hits_set(hipStream_t s, const ds_cloud *c, const TracerParams &tp,
                                int draws, const float *ray_o, const float *ray_d, int64_t N,
                                uint64_t seed, uint64_t sample, float *pos, float *view,
                                float *light, float *weight, float *direct, uint8_t *hit)
{
    DS_CHECK(tp.light_mode == kLightSetMode && tp.set_dw && tp.set_thr && tp.set_m >= 1,
             DS_ERR_INVALID_ARG, "internal error: no light set");
    DS_TRY_MEDIUM(s, c);
    k_first_hits_set<<<(unsigned)((N + 255) / 256), 256, 0, s>>>(
        medium(c, tp.ext_scale), tp, draws, ray_o, ray_d, N, seed, sample, pos, view, light, weight, direct, hit);
    DS_HIP(hipGetLastError());
    return DS_OK;
}

ds_status tracer_accumulate_set(hipStream_t s, int64_t N, int draws, const uint8_t *hit,
                                const float *direct, const float *li_net, const uint8_t *flags,
                                const double *li_mc, const float *weight, float albedo, float E,
                                double *sums, double *dsum, unsigned long long *n_fb)
{
    k_accumulate_set<<<(unsigned)((N + 255) / 256), 256, 0, s>>>(
        N, draws, hit, direct, li_net, flags, li_mc, weight, albedo, E, sums, dsum, n_fb);
    DS_HIP(hipGetLastError());
    return DS_OK;
}

int tracer_blocks(int spp) { return split(spp).nblk; }

}  // namespace ds
