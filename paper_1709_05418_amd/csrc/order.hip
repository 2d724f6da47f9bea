// Spatial order of a batch's shading points.
//
// Neighbouring lanes of the fused kernel read the same pyramid cells when their points
// are close, which camera-ordered points are and points scattered through a cloud are
// not.  Before a batched launch the points of every cloud are therefore sorted by the
// cell of a 32^3 grid over the cloud's box that holds them, cells in Morton order, with
// a counting sort: count the points per cell (the atomic add also gives each point its
// slot within its cell), an exclusive scan of the counts gives each cell's first
// position, and each point is written to its cell's first position plus its slot.  The
// order inside a cell is the order in which the atomic adds landed and carries no
// meaning: every point's prediction is independent of which tile it lands in.  Clouds
// keep their ranges, since the counts of cloud c precede those of cloud c + 1 and sum to
// its number of points.  Every launch has a fixed shape and nothing is cleared with
// hipMemsetAsync, so the order can sit inside a captured graph.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace ds {
namespace {

constexpr int kScanBlock = 1024;  // counts per block of the two-level scan

// the low 5 bits of v spread to every third bit
__device__ __forceinline__ uint32_t spread3(uint32_t v)
{
    uint32_t r = 0;
#pragma unroll
    for (int i = 0; i < kOrderBits; ++i)
        r |= ((v >> i) & 1u) << (3 * i);
    return r;
}

__device__ __forceinline__ int cell_axis(float x, float lo, float hi)
{
    const float u = (x - lo) / (hi - lo) * (float)(1 << kOrderBits);
    // NaN and points outside the box go to the nearest cell
    const float c = fminf(fmaxf(u, 0.f), (float)((1 << kOrderBits) - 1));
    return c == c ? (int)c : 0;
}

// Bucket of point p: the cloud whose range holds it, then the Morton code of its cell.
__device__ __forceinline__ int bucket_of(const FusedArgs &a, int64_t p)
{
    int c = 0;
    for (int i = 1; i < a.n_clouds; ++i)
        if (p >= a.cl[i].p_begin)
            c = i;
    const FusedCloud &cl = a.cl[c];
    const int ix = cell_axis(a.pos[3 * p], cl.amin[0], cl.amax[0]);
    const int iy = cell_axis(a.pos[3 * p + 1], cl.amin[1], cl.amax[1]);
    const int iz = cell_axis(a.pos[3 * p + 2], cl.amin[2], cl.amax[2]);
    return c * kOrderBuckets +
           (int)(spread3((uint32_t)ix) | (spread3((uint32_t)iy) << 1) |
                 (spread3((uint32_t)iz) << 2));
}

__global__ void __launch_bounds__(256) k_order_clear(int32_t *counts, int n)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        counts[i] = 0;
}

__global__ void __launch_bounds__(256) k_order_count(FusedArgs a, int64_t total,
                                                     int32_t *__restrict__ counts,
                                                     int32_t *__restrict__ slot)
{
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < total;
         p += (int64_t)gridDim.x * blockDim.x)
        slot[p] = atomicAdd(&counts[bucket_of(a, p)], 1);
}

// Exclusive scan of kScanBlock counts per block, in place; the block's total to sums.
__global__ void __launch_bounds__(256) k_scan_block(int32_t *__restrict__ counts, int n,
                                                    int32_t *__restrict__ sums)
{
    __shared__ int32_t part[256];
    const int base = blockIdx.x * kScanBlock + threadIdx.x * 4;
    int32_t v[4], s = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        v[i] = base + i < n ? counts[base + i] : 0;
        s += v[i];
    }
    part[threadIdx.x] = s;
    __syncthreads();
    // inclusive scan of the 256 thread sums (Hillis-Steele)
    for (int d = 1; d < 256; d <<= 1) {
        const int32_t t = (int)threadIdx.x >= d ? part[threadIdx.x - d] : 0;
        __syncthreads();
        part[threadIdx.x] += t;
        __syncthreads();
    }
    int32_t run = part[threadIdx.x] - s;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if (base + i < n)
            counts[base + i] = run;
        run += v[i];
    }
    if (threadIdx.x == 255)
        sums[blockIdx.x] = part[255];
}

// Exclusive scan of the block totals (at most 512) by one block.
__global__ void __launch_bounds__(512) k_scan_sums(int32_t *sums, int nb)
{
    __shared__ int32_t part[512];
    const int t = threadIdx.x;
    const int32_t v = t < nb ? sums[t] : 0;
    part[t] = v;
    __syncthreads();
    for (int d = 1; d < 512; d <<= 1) {
        const int32_t u = t >= d ? part[t - d] : 0;
        __syncthreads();
        part[t] += u;
        __syncthreads();
    }
    if (t < nb)
        sums[t] = part[t] - v;
}

__global__ void __launch_bounds__(256) k_order_scatter(FusedArgs a, int64_t total,
                                                       const int32_t *__restrict__ start,
                                                       const int32_t *__restrict__ sums,
                                                       const int32_t *__restrict__ slot,
                                                       int32_t *__restrict__ perm)
{
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < total;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int b = bucket_of(a, p);
        perm[start[b] + sums[b / kScanBlock] + slot[p]] = (int32_t)p;
    }
}

}  // namespace

int64_t order_buckets(int n_clouds)
{
    return (int64_t)n_clouds * kOrderBuckets;
}

int64_t order_sums(int n_clouds)
{
    return (order_buckets(n_clouds) + kScanBlock - 1) / kScanBlock;
}

ds_status batch_order(hipStream_t s, const FusedArgs &a, int64_t total, int32_t *perm,
                      int32_t *slot, int32_t *counts, int32_t *sums)
{
    if (total == 0)
        return DS_OK;
    const int nb = (int)order_buckets(a.n_clouds);
    const int ns = (int)order_sums(a.n_clouds);
    if (ns > 512 || total > ((int64_t)1 << 31)) {
        set_error("batch order: %d clouds or %lld points exceed the order's limits",
                  a.n_clouds, (long long)total);
        return DS_ERR_INVALID_ARG;
    }
    const int gp = (int)std::min<int64_t>((total + 255) / 256, 8192);
    k_order_clear<<<(nb + 255) / 256, 256, 0, s>>>(counts, nb);
    k_order_count<<<gp, 256, 0, s>>>(a, total, counts, slot);
    k_scan_block<<<ns, 256, 0, s>>>(counts, nb, sums);
    k_scan_sums<<<1, 512, 0, s>>>(sums, ns);
    k_order_scatter<<<gp, 256, 0, s>>>(a, total, counts, sums, slot, perm);
    DS_HIP(hipGetLastError());
    return DS_OK;
}

}  // namespace ds
