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
// Work split.  A workgroup of NW waves (4 or 8) owns 16 NW points, 16 per wave,
// with two waves per SIMD.  The weight fragments of one 32-wide input chunk (MT KB)
// are staged once per workgroup in LDS, double-buffered: while the waves consume
// chunk i the next chunk is already in flight from L2.  Fragments are stored in
// consumption order, so staging is a linear walk.  The stencil samples are
// software-pipelined: each lane keeps two half-chunks (4 samples each) of loads in
// flight, and the first samples of level k+1 are issued before the second layer
// of block k runs.
//
// Stencil gather.  The first layer of block k reads 225 stencil densities plus
// gamma.  Lane group g of chunk c gathers 8 samples of its point: chunks 0..5 and
// the g = 0 part of chunk 6 cover the 25 stencil columns (ix, iy) with iz = 0..7,
// so consecutive samples differ by one fixed step vector; lanes g = 1..3 of chunk
// 6 take 24 of the 25 samples of the iz = 8 plane (five rows of four and one
// column of four), and chunk 7 carries the last plane sample (4, 4, 8), gamma and
// (for an odd tile count) the last tile of o^{k-1}.
// Densities come from a corner-packed FP16 copy of the mip level (the 8 corners
// of a cell in one 16-byte load) addressed in cell coordinates shifted by one and
// clamped to [0, n+1], which reproduces zero outside the grid.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "internal.h"
#include "frame.h"

namespace ds {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 mfma_bf16(const uint4 &a, const bf16x8 &b, const f4 &c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), b, c, 0, 0, 0);
}

// 32 E4M3 bytes: one lane's operand of the 16x16x128 FP8 MFMA
typedef int fp8x32 __attribute__((ext_vector_type(8)));

// FP8 E4M3 x E4M3 over 128 inputs, FP32 accumulation, no operand scales (constant
// zero scale arguments select the unscaled v_mfma_f32_16x16x128_f8f6f4; the scaled
// form with register scales makes the register allocator spill this kernel's
// accumulators).  Operand layout: lane 16 g + r holds row r of A at inputs (g, byte
// b), lane 16 g + n column n of B at the same (g, b); the pairing of (g, b) is all the
// packing relies on.
__device__ __forceinline__ f4 mfma_fp8(const fp8x32 &a, const fp8x32 &b, const f4 &c)
{
    return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b, c, 0, 0, 0, 0, 0, 0);
}

// Per point and level: cell coordinate (shifted by +1) of lattice point (0,0,0)
// and the coordinate steps along the three lattice axes.
struct PtLevel {
    float u0[3], a[3], b[3], c[3];
};


typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(1))) u32x4 *gcell_ptr;

// Four trilinear samples in flight: the 16-byte corner cells and the fractions.
struct Pending {
    u32x4 v[4];
    float fx[4];
    uint32_t t[4];  // (fy, fz) as packed FP16
};

// Clamp a shifted cell coordinate (CL) or take it as it is (the level's zero border holds
// every sample of the wave's points), start the cell load, keep the fractions.
template <bool CL = true>
__device__ __forceinline__ void issue_one(gcell_ptr cells, const FusedLevel &L, float ux, float uy,
                                          float uz, u32x4 &v, float &fx, uint32_t &tyz)
{
    if (CL) {
        ux = __builtin_amdgcn_fmed3f(ux, 0.f, L.hi_x);
        uy = __builtin_amdgcn_fmed3f(uy, 0.f, L.hi_y);
        uz = __builtin_amdgcn_fmed3f(uz, 0.f, L.hi_z);
    }
    const uint32_t i = (uint32_t)ux, j = (uint32_t)uy, k = (uint32_t)uz;
    fx = __builtin_amdgcn_fractf(ux);
    tyz = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pkrtz(__builtin_amdgcn_fractf(uy),
                                                                __builtin_amdgcn_fractf(uz)));
    // 24-bit multiply-adds: cell dims stay below 2^13 and j + cy k below 2^24.  The empty
    // asm statements keep both partial indices 32-bit values in registers, so the compiler
    // emits two full-rate v_mad_u32_u24 instead of widening one into v_mad_u64_u32.
    uint32_t t = j + __umul24((uint32_t)L.cy, k);
    asm volatile("" : "+v"(t));
    uint32_t idx = i + __umul24((uint32_t)L.cx, t);
    asm volatile("" : "+v"(idx));
    v = cells[idx];
}

// Trilinear value of a sample from its cell's polynomial coefficients (FP16, see k_pack):
// the two faces' bilinear functions P0, P1 as packed FP16 FMAs on the (P0, P1) coefficient
// pairs, then P0 + fx P1 in FP32 on the two halves in place.
__device__ __forceinline__ float finish_one(const u32x4 &v, float fx, uint32_t tyz)
{
    typedef _Float16 h2 __attribute__((ext_vector_type(2)));
    // element copies first: a bit cast applied to a vector element itself reads the
    // vector's first element (seen with this compiler)
    const uint32_t u0 = v[0], u1 = v[1], u2 = v[2], u3 = v[3];
    const h2 A = __builtin_bit_cast(h2, u0), B = __builtin_bit_cast(h2, u1);
    const h2 C = __builtin_bit_cast(h2, u2), D = __builtin_bit_cast(h2, u3);
    const h2 t = __builtin_bit_cast(h2, tyz);  // (fy, fz)
    const h2 p = B * t[0] + A;  // A + B ty for both faces
    const h2 q = D * t[0] + C;  // C + D ty
    const h2 r = q * t[1] + p;  // (P0, P1)
    return fmaf(fx, (float)r[1], (float)r[0]);
}

// Lattice tables shared by a workgroup: (ix, iy) of stencil columns 0..23 (the
// column walk of chunks 0..5) and the coordinates of halves 12, 13 (column 24 for
// lane group 0; the iz = 8 plane for lane groups 1..3, see issue_table_half).
__device__ __forceinline__ void init_tables(int tid, float4 *plane, float2 *cols)
{
    if (tid < 32) {
        const int gg = tid >> 3, j = tid & 7;
        if (gg == 0) {
            plane[tid] = make_float4(4.f, 4.f, (float)j, 0.f);
        } else {
            const int G = 2 * (gg - 1) + (j >> 2), jj = j & 3;
            plane[tid] = G < 5 ? make_float4((float)jj, (float)G, 8.f, 0.f)
                               : make_float4(4.f, (float)jj, 8.f, 0.f);
        }
    }
    if (tid < 24)
        cols[tid] = make_float2((float)(tid % 5), (float)(tid / 5));
}

// Four samples of a stencil column from the coordinate (bx, by, bz) of its first one:
// consecutive samples along z differ by the step vector c.
template <bool CL = true>
__device__ __forceinline__ void issue_four(gcell_ptr cells, const FusedLevel &L, const PtLevel &q,
                                           float bx, float by, float bz, Pending &p)
{
    issue_one<CL>(cells, L, bx, by, bz, p.v[0], p.fx[0], p.t[0]);
#pragma unroll
    for (int j = 1; j < 4; ++j)
        issue_one<CL>(cells, L, fmaf((float)j, q.c[0], bx), fmaf((float)j, q.c[1], by),
                  fmaf((float)j, q.c[2], bz), p.v[j], p.fx[j], p.t[j]);
}

// Coordinate of lattice point (ix, iy, 0) of stencil column 4 s + g, (ix, iy) from the
// table (see init_tables).
__device__ __forceinline__ float3 column_base(const PtLevel &q, int s, int g, const float2 *cols)
{
    const float2 xy = cols[4 * s + g];
    return make_float3(fmaf(xy.y, q.b[0], fmaf(xy.x, q.a[0], q.u0[0])),
                       fmaf(xy.y, q.b[1], fmaf(xy.x, q.a[1], q.u0[1])),
                       fmaf(xy.y, q.b[2], fmaf(xy.x, q.a[2], q.u0[2])));
}

// Both halves (iz = 0..3 into lo, 4..7 into hi) of column 4 s + g from one base.
template <bool CL = true>
__device__ __forceinline__ void issue_column(gcell_ptr cells, const FusedLevel &L,
                                             const PtLevel &q, int s, int g, const float2 *cols,
                                             Pending &lo, Pending &hi)
{
    const float3 b = column_base(q, s, g, cols);
    issue_four<CL>(cells, L, q, b.x, b.y, b.z, lo);
    issue_four<CL>(cells, L, q, fmaf(4.f, q.c[0], b.x), fmaf(4.f, q.c[1], b.y),
               fmaf(4.f, q.c[2], b.z), hi);
}

// Halves 0..11 (chunks 0..5): lane group g walks stencil column 4c + g along z,
// iz = 4 (h & 1) + j.
__device__ __forceinline__ void issue_column_half(gcell_ptr cells, const FusedLevel &L,
                                                  const PtLevel &q, int h, int g,
                                                  const float2 *cols, Pending &p)
{
    const float3 b = column_base(q, h >> 1, g, cols);
    const float iz0 = (float)(4 * (h & 1));
    issue_four(cells, L, q, fmaf(iz0, q.c[0], b.x), fmaf(iz0, q.c[1], b.y),
               fmaf(iz0, q.c[2], b.z), p);
}

// Halves 12, 13 (chunk 6) mix directions: lattice coordinates come from a table
// (column 24 for g = 0; the iz = 8 plane for g = 1..3: rows iy = 0..4 with
// ix = 0..3, then ix = 4 with iy = 0..3; its last point (4, 4, 8) goes to chunk 7).
template <bool CL = true>
__device__ __forceinline__ void issue_table_half(gcell_ptr cells, const FusedLevel &L,
                                                 const PtLevel &q, int hh, int g,
                                                 const float4 *tab, Pending &p)
{
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const float4 o = tab[8 * g + 4 * hh + j];
        issue_one<CL>(cells, L, q.u0[0] + o.x * q.a[0] + o.y * q.b[0] + o.z * q.c[0],
                  q.u0[1] + o.x * q.a[1] + o.y * q.b[1] + o.z * q.c[1],
                  q.u0[2] + o.x * q.a[2] + o.y * q.b[2] + o.z * q.c[2], p.v[j], p.fx[j], p.t[j]);
    }
}

// Position and light frame of point p; false (and a zero frame) if the lane has
// no point (in = false) or its inputs are unusable.  Recomputed where needed instead of being kept
// in registers for the whole kernel.
__device__ __forceinline__ bool point_frame(const FusedArgs &a, int64_t p, bool in, float *x,
                                            Frame &fr)
{
    bool ok = false;
    x[0] = x[1] = x[2] = 0.f;
    if (in) {
        x[0] = a.pos[3 * p];
        x[1] = a.pos[3 * p + 1];
        x[2] = a.pos[3 * p + 2];
        ok = isfinite(x[0]) && isfinite(x[1]) && isfinite(x[2]) &&
             light_frame(&a.view[3 * p], &a.light[3 * p], fr);
    }
    if (!ok) {
        x[0] = x[1] = x[2] = 0.f;
#pragma unroll
        for (int c = 0; c < 3; ++c)
            fr.X[c] = fr.Y[c] = fr.Z[c] = 0.f;
        fr.gamma = 0.f;
    }
    return ok;
}

// Tile of the v-th step of the launch's walk (workgroup b takes steps b, b + grid, ...),
// so that neighbouring tiles share an XCD.  Workgroups go to the eight XCDs in turn
// (workgroup b to XCD b mod 8), each XCD with its own L2, and consecutive tiles hold
// neighbouring points that read the same cells: blocks of kXcdBlock consecutive tiles are
// dealt to the XCDs in turn, so an XCD walks whole blocks while every XCD still sees every
// part of the launch (uneven clouds stay balanced).  A bijection of [0, n): steps past the
// last whole round of 8 blocks keep their own tile.  With a grid that is a multiple of 8
// every step of a workgroup stays on its XCD.
constexpr int kXcdBlock = 32;

__device__ __forceinline__ int64_t xcd_tile(int64_t v, int64_t n)
{
    constexpr int64_t R = 8 * kXcdBlock;
    if (v >= n / R * R)
        return v;
    const int64_t q = v >> 3;
    return ((q / kXcdBlock) * 8 + (v & 7)) * kXcdBlock + q % kXcdBlock;
}

// Row of the point arrays at launch position i (a lane past its cloud's points reads none)
__device__ __forceinline__ int64_t point_row(const FusedArgs &a, int64_t i, bool in)
{
    return a.perm && in ? (int64_t)a.perm[i] : i;
}

// Cloud of tile t: the last cloud whose first tile is not after t (clouds without
// points own no tiles).  Uniform across the workgroup.
__device__ __forceinline__ int tile_cloud(const FusedArgs &a, int64_t t)
{
    int c = 0;
    for (int i = 1; i < a.n_clouds; ++i)
        if (t >= a.cl[i].tile_begin)
            c = i;
    return __builtin_amdgcn_readfirstlane(c);
}

// Per-point geometry that every stencil level needs: the position relative to the
// grid corner (x'), the frame axes X, Y, Z and their sum S (the lattice origin sits
// at -S half steps), and whether the point is valid.  Computed once per tile and
// kept in LDS; layout [x'0 x'1 x'2 S0] [S1 S2 X0 X1] [X2 Y0 Y1 Y2] [Z0 Z1 Z2 ok].
struct PtGeom {
    float4 a, b, c, d;
};

__device__ __forceinline__ PtGeom make_geom(const float *x, const Frame &fr, const float *amin,
                                            bool valid)
{
    PtGeom G;
    const float S0 = fr.X[0] + fr.Y[0] + fr.Z[0];
    const float S1 = fr.X[1] + fr.Y[1] + fr.Z[1];
    const float S2 = fr.X[2] + fr.Y[2] + fr.Z[2];
    G.a = make_float4(x[0] - amin[0], x[1] - amin[1], x[2] - amin[2], S0);
    G.b = make_float4(S1, S2, fr.X[0], fr.X[1]);
    G.c = make_float4(fr.X[2], fr.Y[0], fr.Y[1], fr.Y[2]);
    G.d = make_float4(fr.Z[0], fr.Z[1], fr.Z[2], valid ? 1.f : 0.f);
    return G;
}

// Stencil origin and lattice steps of one level, in cell coordinates (the voxel-centred
// coordinate shifted by the level's border, so cell coordinates start at the first zero
// border cell).  A point without a usable frame reads the all-zero corner cell 0 for every
// sample, which needs no clamp.
__device__ __forceinline__ void level_from_geom(const FusedLevel &L, const PtGeom &G, PtLevel &q)
{
    const float st = L.step * L.inv_h, hs = 0.5f * st;
    const float xr[3] = {G.a.x, G.a.y, G.a.z}, S[3] = {G.a.w, G.b.x, G.b.y};
    const float X[3] = {G.b.z, G.b.w, G.c.x}, Y[3] = {G.c.y, G.c.z, G.c.w};
    const float Z[3] = {G.d.x, G.d.y, G.d.z};
    const bool ok = G.d.w > 0.f;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        q.u0[c] = ok ? fmaf(-st, S[c], fmaf(xr[c], L.inv_h, L.shift)) : 0.f;
        q.a[c] = ok ? hs * X[c] : 0.f;
        q.b[c] = ok ? hs * Y[c] : 0.f;
        q.c[c] = ok ? hs * Z[c] : 0.f;
    }
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

// pack8 with a ReLU: BF16 bit patterns read as signed 16-bit integers order every
// negative value (and -0) below +0, so one packed integer max per pair replaces the
// two FP32 max operations, with identical results.
__device__ __forceinline__ bf16x8 pack8_relu(const f4 &lo, const f4 &hi)
{
    typedef short s16x8 __attribute__((ext_vector_type(8)));
    const s16x8 v = __builtin_bit_cast(s16x8, pack8(lo, hi));
    return __builtin_bit_cast(bf16x8, __builtin_elementwise_max(v, (s16x8)0));
}

// Double-buffered staging of weight chunks (MT fragments of 64 x 16 bytes), G chunks
// per buffer.  The next group of chunks is copied from global memory straight into
// the idle LDS buffer (global_load_lds, 16 bytes per lane, lane l of a wave writing
// base + 16 l), so the copy holds no registers; one barrier per group publishes it.
// FR is a multiple of 64, so each wave copies whole 1 KB rows or none.
//   begin()  at the start of a tile: group 0 resident, group 1 pending
//   fetch()  issue the pending group's copy (call after the chunk's sample loads, so
//            waiting for a sample never waits for weights)
//   next()   after consuming a chunk; at the end of a group: wait, barrier, switch
typedef __attribute__((address_space(1))) void gvoid;
typedef __attribute__((address_space(3))) void lvoid;

// s_waitcnt vmcnt(N) with the other counters left alone (gfx9 encoding: vmcnt in
// bits 3:0 and 15:14, expcnt 6:4, lgkmcnt 11:8).
template <int N>
__device__ __forceinline__ void vm_wait()
{
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
    asm volatile("" ::: "memory");
}

// Copy of K consecutive 1 KB rows (K = 1..4) from global g into LDS at byte address l:
// lane l of row r moves 16 bytes from g + r KB + 16 l to l + r KB + 16 l.  The immediate
// offset of the instruction moves the global and the LDS address alike, so the rows of a
// run share one m0 and one base pointer.
template <int K>
__device__ __forceinline__ void dma_rows(const uint4 *g, uint32_t l, uint32_t voff)
{
    static_assert(K >= 1 && K <= 4, "one to four rows per base");
    if constexpr (K == 1)
        asm volatile("s_mov_b32 m0, %0\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %1, %2"
                     :
                     : "s"(l), "v"(voff), "s"(g)
                     : "memory", "m0");
    else if constexpr (K == 2)
        asm volatile("s_mov_b32 m0, %0\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %1, %2\n\t"
                     "global_load_lds_dwordx4 %1, %2 offset:1024"
                     :
                     : "s"(l), "v"(voff), "s"(g)
                     : "memory", "m0");
    else if constexpr (K == 3)
        asm volatile("s_mov_b32 m0, %0\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %1, %2\n\t"
                     "global_load_lds_dwordx4 %1, %2 offset:1024\n\t"
                     "global_load_lds_dwordx4 %1, %2 offset:2048"
                     :
                     : "s"(l), "v"(voff), "s"(g)
                     : "memory", "m0");
    else
        asm volatile("s_mov_b32 m0, %0\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %1, %2\n\t"
                     "global_load_lds_dwordx4 %1, %2 offset:1024\n\t"
                     "global_load_lds_dwordx4 %1, %2 offset:2048\n\t"
                     "global_load_lds_dwordx4 %1, %2 offset:3072"
                     :
                     : "s"(l), "v"(voff), "s"(g)
                     : "memory", "m0");
}

// N consecutive rows in runs of up to four
template <int N>
__device__ __forceinline__ void dma_run(const uint4 *g, uint32_t l, uint32_t voff)
{
    if constexpr (N > 0) {
        constexpr int K = N < 4 ? N : 4;
        dma_rows<K>(g, l, voff);
        dma_run<N - K>(g + K * 64, l + K * 1024u, voff);
    }
}

template <int MT, int NW>
struct WeightStage {
    // chunks per buffer: two workgroups of four waves share a compute unit's LDS;
    // an eight-wave workgroup has it alone and stages four chunks per barrier
    static constexpr int G = NW == 8 ? 4 : 2;
    static constexpr int FR = MT * 64;
    static constexpr int T = 64 * NW;
    static constexpr int SLOT = FR;            // LDS entries per chunk
    static constexpr int BUF = G * SLOT;       // entries per buffer
    static constexpr int ROWS = G * MT;        // 1 KB rows per group
    uint4 *buf;          // LDS, 2 * BUF entries
    const uint4 *src;    // first chunk of the next group to copy
    int cur, j;
    bool pending;

    __device__ __forceinline__ const uint4 *chunk() const { return buf + cur * BUF + j * SLOT; }
    // The copy is written out as the instruction itself: with the builtin the compiler
    // cannot tell the idle buffer from the one being read, and makes the next LDS read of
    // every wave wait for the whole copy.  Issued here, the copy is waited for only by the
    // explicit vm_wait before the group's closing barrier (and, as the counter is in
    // order, by waits for loads issued after it).  The instruction has no register
    // result: its data goes to LDS at m0 + offset + 16 lane.  Wave w copies a contiguous
    // run of RB or RB + 1 rows, so a group costs a few scalar instructions per four rows
    // instead of an address and an m0 per row.
    static constexpr int RB = ROWS / NW, RX = ROWS % NW;
    int r0;     // first row of this wave's run (uniform)
    bool more;  // the run has RB + 1 rows
    __device__ __forceinline__ void init(uint4 *lds, int tid)
    {
        buf = lds;
        const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
        r0 = w * RB + (w < RX ? w : RX);
        more = RX > 0 && w < RX;
    }
    __device__ __forceinline__ void copy_group(int tid, uint4 *dst)
    {
        const uint4 *g = src + r0 * 64;
        const uint32_t l = (uint32_t)(uintptr_t)(lvoid *)(dst + r0 * 64);
        const uint32_t voff = (uint32_t)(tid & 63) * 16u;
        if (more)
            dma_run<RB + 1>(g, l, voff);
        else
            dma_run<RB>(g, l, voff);
        src += BUF;
    }
    __device__ __forceinline__ void begin(const uint4 *frags, int tid)
    {
        // drain a copy still in flight from the previous tile before reusing the buffers
        vm_wait<0>();
        __syncthreads();
        src = frags;
        copy_group(tid, buf);
        vm_wait<0>();
        __syncthreads();
        cur = 0;
        j = 0;
        pending = true;
    }
    __device__ __forceinline__ void fetch(int tid)
    {
        if (pending) {
            copy_group(tid, buf + (cur ^ 1) * BUF);
            pending = false;
        }
    }
    // N: vector-memory loads this chunk issued after its fetch() that may stay in
    // flight across the barrier (the copy is older, so waiting until at most N loads
    // are outstanding completes it)
    template <int N = 0>
    __device__ __forceinline__ void next(int tid)
    {
        if (++j == G) {
            if (pending) {  // a group whose chunks never fetched: copy now, wait for all
                fetch(tid);
                vm_wait<0>();
            } else {
                vm_wait<N>();
            }
            __syncthreads();
            cur ^= 1;
            j = 0;
            pending = true;
        }
    }
};

// Weight chunks for two teams of four waves that walk one chunk stream (every tile's
// chunks in order, tile after tile) D chunks apart: team 0 (waves 0..3) leads, team 1
// (waves 4..7) follows.  The chunks live in a ring of R slots in LDS; in every period of
// G chunks the eight waves together copy the group that team 0 needs in the next period,
// and all of them meet at a barrier every G chunks.  One copy thus serves 128 points, twice a
// WeightStage's 64, which halves the weight bytes that pass through each compute unit's
// vector memory path, and the two waves on a SIMD run different phases of the network
// (the stencil chunks, heavy in vector ALU work, against the dense layers, heavy in
// matrix work) instead of the same phase in step.  At the barrier that opens period n,
// team 0 has consumed the chunks before nG and team 1 those before nG - D; during the
// period the waves copy chunks [nG + G, nG + 2G) into the slots of chunks
// [nG + G - R, nG + 2G - R), all consumed by team 1 when R >= D + 2G.  The stream
// wraps at the tile's chunk count nc (even, so a group never straddles two tiles), and
// a team with no point in a tile still walks its nc chunks (idle steps) so that the
// barriers of both teams stay paired.
template <int MT, int R, int D>
struct TeamRing {
    static constexpr int G = 2;
    static constexpr int SLOT = MT * 64;  // LDS entries per chunk
    static constexpr int ROWS = G * MT;   // 1 KB rows per group
    static constexpr int RB = ROWS / 8, RX = ROWS % 8;  // rows per wave, all eight copy
    static_assert(R >= D + 2 * G && R % G == 0 && D % G == 0, "ring too small for the lag");
    uint4 *ring;
    const uint4 *frags, *src, *src_end;  // the network's chunks, the next group, the end
    int slot;   // slot of this team's current chunk
    int cslot;  // slot of the next group to copy
    int k;      // steps since the last barrier (both teams alike)
    int team, r0;
    bool more, pending;

    __device__ __forceinline__ void init(uint4 *lds, const uint4 *f, int nc, int tid)
    {
        ring = lds;
        frags = src = f;
        src_end = f + (size_t)nc * SLOT;
        const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
        team = w >> 2;
        r0 = w * RB + (w < RX ? w : RX);
        more = RX > 0 && w < RX;
        slot = team == 0 ? 0 : (R - D) % R;  // team 1 starts D idle steps behind chunk 0
        cslot = 0;
        k = 0;
        pending = false;
    }
    __device__ __forceinline__ void copy_group(int tid)
    {
        uint4 *dst = ring + cslot * SLOT;
        const uint4 *g = src + r0 * 64;
        const uint32_t l = (uint32_t)(uintptr_t)(lvoid *)(dst + r0 * 64);
        const uint32_t voff = (uint32_t)(tid & 63) * 16u;
        if (more)
            dma_run<RB + 1>(g, l, voff);
        else
            dma_run<RB>(g, l, voff);
        src += G * SLOT;
        if (src == src_end)
            src = frags;
        cslot += G;
        if (cslot == R)
            cslot = 0;
    }
    // the first group; every wave waits for it (and for the tables)
    __device__ __forceinline__ void prologue(int tid)
    {
        copy_group(tid);
        vm_wait<0>();
        __syncthreads();
        pending = true;
    }
    __device__ __forceinline__ const uint4 *chunk() const { return ring + slot * SLOT; }
    __device__ __forceinline__ void begin(const uint4 *, int) {}  // the stream runs on
    __device__ __forceinline__ void fetch(int tid)
    {
        if (pending) {
            copy_group(tid);
            pending = false;
        }
    }
    template <int N = 0>
    __device__ __forceinline__ void next(int tid)
    {
        if (++slot == R)
            slot = 0;
        if (++k == G) {
            if (pending) {  // a group whose chunks never fetched: copy now, wait for all
                fetch(tid);
                vm_wait<0>();
            } else {
                vm_wait<N>();
            }
            __syncthreads();
            k = 0;
            pending = true;
        }
    }
    // n steps without consuming a chunk (copies and barriers as usual)
    __device__ __forceinline__ void idle(int tid, int n)
    {
#pragma unroll 1
        for (int i = 0; i < n; ++i) {
            fetch(tid);
            next<0>(tid);
        }
    }
};

template <int MT>
__device__ __forceinline__ void mfma_chunk(const uint4 *w, int lane, const bf16x8 &B, f4 (&acc)[MT])
{
    // keep the fragment reads next to their MFMAs (hoisting all of them above the
    // gather math costs more registers than the two waves per SIMD can spare), three
    // reads ahead of the product that consumes them, so an LDS read's latency spans
    // three products instead of one
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
        acc[mt] = mfma_bf16(w[mt * 64 + lane], B, acc[mt]);
    constexpr int AHEAD = MT < 3 ? MT : 3;
    __builtin_amdgcn_sched_group_barrier(0x100, AHEAD, 0);
#pragma unroll
    for (int mt = 0; mt < MT - AHEAD; ++mt) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
    }
    __builtin_amdgcn_sched_group_barrier(0x008, AHEAD, 0);
    __builtin_amdgcn_sched_barrier(0);
}

// B operand of FP8 chunk Q of a W-wide layer: tiles 8Q..8Q+7 of the input in
// accumulator layout, dword d holding tile 8Q + d's four features of this lane.  The
// hardware conversion rounds to nearest even but does not saturate (>= 464 gives
// NaN), so inputs that may exceed 448 are clamped first.
template <int MT, bool CLAMP, bool BIAS = false>
__device__ __forceinline__ fp8x32 pack_fp8(const f4 (&x)[MT], int Q, int g)
{
    fp8x32 r;
#pragma unroll
    for (int d = 0; d < 8; ++d) {
        const int t = 8 * Q + d;
        if (BIAS && t == MT) {  // inputs 0..2 of lane group 0 in the first free tile: E4M3 1.0
            r[d] = g == 0 ? 0x00383838 : 0;
        } else if (t < MT) {
            f4 v = x[t < MT ? t : 0];
            if (CLAMP) {  // inputs are ReLU outputs, >= 0
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    v[i] = __builtin_amdgcn_fmed3f(v[i], 0.f, 448.f);
            }
            int w = __builtin_amdgcn_cvt_pk_fp8_f32(v[0], v[1], 0, false);
            r[d] = __builtin_amdgcn_cvt_pk_fp8_f32(v[2], v[3], w, true);
        } else {
            r[d] = 0;
        }
    }
    return r;
}

// One FP8 chunk: its 32-byte A fragments are split over two consecutive staging
// slots (bytes 0..15 of every lane entry in the first, 16..31 in the second).
template <int MT>
__device__ __forceinline__ void mfma8_chunk(const uint4 *w, int lane, const fp8x32 &B,
                                            f4 (&acc)[MT])
{
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
        const uint4 lo = w[mt * 64 + lane], hi = w[(MT + mt) * 64 + lane];
        const fp8x32 A = {(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w,
                          (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
        acc[mt] = mfma_fp8(A, B, acc[mt]);
    }
    // each A operand is eight registers: interleave two fragment reads (LDS) with one
    // MFMA instead of letting the scheduler issue every read first
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
        __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
    }
    __builtin_amdgcn_sched_barrier(0);
}

// Consume one FP8 chunk (two staging slots) of a W-wide layer; BIAS: the layer's bias
// rides in the first free tile of its last chunk (three E4M3 parts, see fused_quantize_fp8),
// whose inputs pack_fp8 sets to 1.
template <int MT, int NW, bool CLAMP, class Stage, bool BIAS = false>
__device__ __forceinline__ void fp8_layer(Stage &ws, int tid, int lane,
                                          const f4 (&in)[MT], f4 (&acc)[MT])
{
    static_assert(!BIAS || MT % 8 != 0, "a folded bias needs a free tile in the last chunk");
#pragma unroll
    for (int Q = 0; Q < (MT + 7) / 8; ++Q) {
        ws.fetch(tid);
        mfma8_chunk<MT>(ws.chunk(), lane, pack_fp8<MT, CLAMP, BIAS>(in, Q, lane >> 4), acc);
        ws.template next<0>(tid);
        ws.template next<0>(tid);
    }
}

// Inputs of the free half of a layer's last chunk when the bias rides in it (odd MT): the
// fragments hold the bias split into BF16 high and low parts at inputs (g = 0, j = 4, 5)
// of that chunk (see build_pack_maps), so those two inputs are 1 and the product adds the
// bias; the vector loads of the bias, which pass through the same memory path as the
// samples and the weight copies, are not needed.
__device__ __forceinline__ f4 bias_ones(int g)
{
    const float one = g == 0 ? 1.f : 0.f;
    return f4{one, one, 0.f, 0.f};
}

// out = relu(Wmat in + bias) for a W-wide input held in accumulator layout; FOLD: the bias
// comes with the last chunk's fragments instead of a vector load (odd MT only).
template <int MT, int NW, class Stage, bool FOLD = false>
__device__ __forceinline__ void dense(Stage &ws, const float *__restrict__ bias,
                                      int tid, int lane, const f4 (&in)[MT], f4 (&out)[MT])
{
    static_assert(!FOLD || (MT & 1), "a folded bias needs the free half of an odd last chunk");
    constexpr int C2 = (MT + 1) / 2;
    const int g = lane >> 4;
    const f4 z4 = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
        out[mt] = FOLD ? z4 : *reinterpret_cast<const f4 *>(bias + 16 * mt + 4 * g);
#pragma unroll
    for (int q = 0; q < C2; ++q) {
        ws.fetch(tid);
        bf16x8 B = pack8(in[2 * q], (2 * q + 1 < MT) ? in[2 * q + 1 < MT ? 2 * q + 1 : 0]
                                                      : (FOLD ? bias_ones(g) : z4));
        mfma_chunk<MT>(ws.chunk(), lane, B, out);
        ws.template next<0>(tid);
    }
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i)
            out[mt][i] = fmaxf(out[mt][i], 0.f);
}

// FP8 form of dense(): the output stays in its scaled units (biases pre-scaled), and the
// ReLU clamps at 448 so that the next FP8 layer can take it unclamped.  FOLD: the bias
// comes with the last chunk (MT not a multiple of 8).
template <int MT, int NW, class Stage, bool FOLD = false>
__device__ __forceinline__ void dense8(Stage &ws, const float *__restrict__ bias,
                                       int tid, int lane, const f4 (&in)[MT], f4 (&out)[MT])
{
    const int g = lane >> 4;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
        out[mt] = FOLD ? f4{0.f, 0.f, 0.f, 0.f}
                       : *reinterpret_cast<const f4 *>(bias + 16 * mt + 4 * g);
    fp8_layer<MT, NW, true, Stage, FOLD>(ws, tid, lane, in, out);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i)
            out[mt][i] = __builtin_amdgcn_fmed3f(out[mt][i], 0.f, 448.f);
}

template <int MT, int NW>
__global__ void __launch_bounds__(64 * NW, 2) k_fused(FusedArgs a, const uint4 *__restrict__ frags,
                                                      const float *__restrict__ vec)
{
    constexpr int C2 = (MT + 1) / 2;   // chunks of a W-wide input
    constexpr int WP = 16 * MT;        // padded width
    __shared__ uint4 wbuf[2 * WeightStage<MT, NW>::BUF];
    __shared__ float4 plane[32];       // lattice coordinates of halves 12, 13 per (lane group, j)
    __shared__ float2 cols[24];
    // residual stream o^k of each wave in FP32, accumulator layout [tile][lane]; it
    // lives in LDS while the first layer runs and comes back for the second
    __shared__ f4 obuf[NW][MT][64];
    __shared__ PtGeom geom[16 * NW];   // per point of the tile, see make_geom

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int g = lane >> 4, n = lane & 15;
    init_tables(tid, plane, cols);

    WeightStage<MT, NW> ws;
    ws.init(wbuf, tid);
    // persistent loop over tiles of 16 NW points; a tile never spans two clouds
#pragma unroll 1
    for (int64_t v = blockIdx.x; v < a.n_tiles; v += gridDim.x) {
        const int64_t t = xcd_tile(v, a.n_tiles);
        // keeps tile-invariant LDS reads (the plane table) inside the loop: hoisted,
        // they would hold registers across the whole tile and force spills
        asm volatile("" ::: "memory");
        const FusedCloud &cl = a.cl[tile_cloud(a, t)];
        ws.begin(frags, tid);  // also orders the plane table

        const int64_t pl = (t - cl.tile_begin) * (16 * NW) + (tid >> 6) * 16 + n;
        const bool in = pl < cl.P;
        const int64_t p = point_row(a, cl.p_begin + pl, in);
        float gamma;
        bool valid;
        {
            float x[3];
            Frame fr;
            valid = point_frame(a, p, in, x, fr);
            gamma = fr.gamma;
            // the four lanes of a point write the same slot; each reads its own write
            geom[(tid >> 6) * 16 + n] = make_geom(x, fr, cl.amin, valid);
        }

        f4 F[MT];
        const f4 z4 = f4{0.f, 0.f, 0.f, 0.f};
        f4(*Os)[64] = obuf[tid >> 6];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
            Os[mt][lane] = z4;

        // the first two half-chunks of level 1 go out before the loop; later levels
        // start theirs while the previous level's second layer runs
        FusedLevel L = cl.lvt[0];
        gcell_ptr cells = (gcell_ptr)L.cells;
        PtLevel q;
        {
            level_from_geom(L, geom[(tid >> 6) * 16 + n], q);
        }
        Pending pa, pb;
        issue_column_half(cells, L, q, 0, g, cols, pa);
        issue_column_half(cells, L, q, 1, g, cols, pb);

        for (int k = 0; k < a.K; ++k) {
            const float *b1 = vec + (size_t)k * 2 * WP;
            const float *b2 = b1 + WP;
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
                F[mt] = z4;

            // stencil chunks 0..6, two halves of four samples each, two halves in flight:
            // step c finishes halves 2c, 2c+1 and issues halves 2c+2, 2c+3
#pragma unroll 1
            for (int c = 0; c < 5; ++c) {
                ws.fetch(tid);
                f4 lo, hi;
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    lo[j] = finish_one(pa.v[j], pa.fx[j], pa.t[j]);
                issue_column_half(cells, L, q, 2 * c + 2, g, cols, pa);
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    hi[j] = finish_one(pb.v[j], pb.fx[j], pb.t[j]);
                issue_column_half(cells, L, q, 2 * c + 3, g, cols, pb);
                mfma_chunk<MT>(ws.chunk(), lane, pack8(lo, hi), F);
                ws.template next<0>(tid);
            }
            {  // chunk 5: issues the table halves of chunk 6
                ws.fetch(tid);
                f4 lo, hi;
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    lo[j] = finish_one(pa.v[j], pa.fx[j], pa.t[j]);
                issue_table_half(cells, L, q, 0, g, plane, pa);
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    hi[j] = finish_one(pb.v[j], pb.fx[j], pb.t[j]);
                issue_table_half(cells, L, q, 1, g, plane, pb);
                mfma_chunk<MT>(ws.chunk(), lane, pack8(lo, hi), F);
                ws.template next<0>(tid);
            }
            {  // chunk 6: issues chunk 7's stencil sample (4, 4, 8)
                ws.fetch(tid);
                f4 lo, hi;
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    lo[j] = finish_one(pa.v[j], pa.fx[j], pa.t[j]);
                issue_one(cells, L, q.u0[0] + 4.f * (q.a[0] + q.b[0]) + 8.f * q.c[0],
                          q.u0[1] + 4.f * (q.a[1] + q.b[1]) + 8.f * q.c[1],
                          q.u0[2] + 4.f * (q.a[2] + q.b[2]) + 8.f * q.c[2], pa.v[0], pa.fx[0],
                          pa.t[0]);
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    hi[j] = finish_one(pb.v[j], pb.fx[j], pb.t[j]);
                mfma_chunk<MT>(ws.chunk(), lane, pack8(lo, hi), F);
                ws.template next<0>(tid);
            }
            // chunk 7: stencil sample (4, 4, 8), gamma, and the odd tile of o^{k-1}
            {
                ws.fetch(tid);
                float s = finish_one(pa.v[0], pa.fx[0], pa.t[0]);
                f4 lo = f4{g == 0 ? s : 0.f, g == 0 ? gamma : 0.f, 0.f, 0.f};
                bf16x8 B = pack8(lo, (MT & 1) ? Os[MT - 1][lane] : z4);
                mfma_chunk<MT>(ws.chunk(), lane, B, F);
                ws.template next<0>(tid);
            }
            // o^{k-1} in pairs of tiles (o^0 = 0: block 1 has no such chunks)
            if (k > 0) {
#pragma unroll
                for (int qq = 0; qq < MT / 2; ++qq) {
                    ws.fetch(tid);
                    mfma_chunk<MT>(ws.chunk(), lane, pack8(Os[2 * qq][lane], Os[2 * qq + 1][lane]), F);
                    ws.template next<0>(tid);
                }
            }
            // the next level's first samples fly while the second layer runs
            if (k + 1 < a.K) {
                L = cl.lvt[k + 1];
                cells = (gcell_ptr)L.cells;
                level_from_geom(L, geom[(tid >> 6) * 16 + n], q);
                issue_column_half(cells, L, q, 0, g, cols, pa);
                issue_column_half(cells, L, q, 1, g, cols, pb);
            }
            // F1 = relu(. + b1)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                f4 bb = *reinterpret_cast<const f4 *>(b1 + 16 * mt + 4 * g);
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    F[mt][i] = fmaxf(F[mt][i] + bb[i], 0.f);
            }
            // o^k = relu(W2 F1 + b2 + o^{k-1}), accumulated in place
            f4 O[MT];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
                O[mt] = Os[mt][lane] + *reinterpret_cast<const f4 *>(b2 + 16 * mt + 4 * g);
#pragma unroll
            for (int qq = 0; qq < C2; ++qq) {
                ws.fetch(tid);
                mfma_chunk<MT>(ws.chunk(), lane,
                               pack8(F[2 * qq], (2 * qq + 1 < MT) ? F[2 * qq + 1 < MT ? 2 * qq + 1 : 0] : z4),
                               O);
                ws.template next<0>(tid);
            }
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    O[mt][i] = fmaxf(O[mt][i], 0.f);
                Os[mt][lane] = O[mt];
            }
        }

        // trailing layers: H-1 dense W -> W layers, ping-ponging between O and F
        f4 O[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
            O[mt] = Os[mt][lane];
        const float *bh = vec + (size_t)a.K * 2 * WP;
        int h = 0;
        for (; h + 1 < a.H - 1; h += 2) {
            dense<MT, NW>(ws, bh + (size_t)h * WP, tid, lane, O, F);
            dense<MT, NW>(ws, bh + (size_t)(h + 1) * WP, tid, lane, F, O);
        }
        if (h < a.H - 1) {
            dense<MT, NW>(ws, bh + (size_t)h * WP, tid, lane, O, F);
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
                O[mt] = F[mt];
        }
        // final scalar layer in FP32 on the vector ALUs
        const float *wl = bh + (size_t)(a.H - 1) * WP;
        const float bl = wl[WP];
        float acc = 0.f;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            f4 w = *reinterpret_cast<const f4 *>(wl + 16 * mt + 4 * g);
            acc += w[0] * O[mt][0] + w[1] * O[mt][1] + w[2] * O[mt][2] + w[3] * O[mt][3];
        }
        acc += __shfl_xor(acc, 16, 64);
        acc += __shfl_xor(acc, 32, 64);
        if (g == 0 && in) {
            float pre = acc + bl;
            a.out[p] = valid ? fmaxf(pre, 0.f) : 0.f;
            if (a.pre)
                a.pre[p] = valid ? pre : 0.f;
            if (a.flags) {
                float x[3];
                Frame fr;
                point_frame(a, p, in, x, fr);
                a.flags[p] = valid ? point_flags(x, fr, cl.amin, cl.amax, cl.inv_mean)
                                   : (uint8_t)DS_FLAG_INVALID;
            }
        }
    }
}

// Register variant: 16 points per wave, two waves per SIMD, the residual stream in
// registers; samples pipelined across the stencil chunks of a level.
//
// F8: the FP8 form.  W1, W2 and the dense trailing layers run on the 16x16x128 E4M3
// MFMA; the descriptor layers stay BF16.  Activations live in power-of-two scaled
// units chosen on the host: block k's first-layer output in units of 2^f_k (its BF16
// weights and bias are pre-multiplied), the residual stream in units of 2^o, trailing
// layer m in units of 2^h_m.  An FP8 matrix is encoded at the exponent (output unit -
// input unit), so the unscaled product lands in the output's units.  ReLU outputs that
// feed an FP8 layer are clamped at 448, the residual stream only where it is
// converted.
// CL = false: the pass without per-sample clamps.  It runs the tiles of clouds whose every
// stencil level has a zero border wide enough for points inside the grid box (FusedCloud::
// fast); points outside the box get no frame there (all their samples read the zero cell)
// and are left to the second pass.  CL = true: the clamped pass, which computes the tiles
// of the other clouds and recomputes every tile that holds a point outside its grid box; it
// skips all other tiles after reading their positions.  Launched one after the other, the
// two passes give every point the clamped kernel's result.
// One tile's prediction for the calling wave's 16 points p (in: the lane has a point;
// outside: its usable position lies outside the grid box, which the unclamped pass CL =
// false treats as invalid).  Shared by the kernels that stage the weight chunks through a
// WeightStage (one workgroup's waves in step) and a TeamRing (two teams of four waves a
// fixed number of chunks apart); gslot is the wave's LDS slot of this point's geometry.
template <int MT, int NW, bool F8, bool CL, class Stage>
__device__ __forceinline__ void predict_points(const FusedArgs &a, const FusedCloud &cl,
                                               const float *__restrict__ vec, Stage &ws,
                                               int tid, PtGeom &gslot, const float4 *plane,
                                               const float2 *cols, int64_t p, bool in,
                                               bool outside)
{
    constexpr int C2 = (MT + 1) / 2;
    constexpr int WP = 16 * MT;
    // The first layer's bias b1 rides in stencil chunk 7 (inputs (g = 1, j = 0, 1), split
    // into BF16 high and low parts, in both forms); with an odd MT the BF16 form's b2 and
    // the dense layers' biases ride in the free half of their last chunk (bias_ones); when
    // MT is not a multiple of 8 the FP8 form's b2 and dense biases ride in the first free
    // tile of their last FP8 chunk (three E4M3 parts).  Otherwise they are vector loads.
    constexpr bool FOLD2 = !F8 && (MT & 1);
    constexpr bool FOLD8 = F8 && (MT % 8 != 0);
    const int lane = tid & 63;
    const int g = lane >> 4;
    float gamma;
    bool valid;
    {
        float x[3];
        Frame fr;
        valid = point_frame(a, p, in, x, fr);
        if (!CL && outside)
            valid = false;  // no frame: its samples read the zero cell
        gamma = valid ? fr.gamma : 0.f;
        // the four lanes of a point write the same slot; each reads its own write
        gslot = make_geom(x, fr, cl.amin, valid);
    }
    const f4 z4 = f4{0.f, 0.f, 0.f, 0.f};
    f4 O[MT], F[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
        O[mt] = z4;

    // Samples are software-pipelined within a level: each stencil chunk finishes
    // the samples the previous chunk issued and issues the next chunk's.  (Issuing
    // the next level's first samples before the second layer would keep them live
    // next to both accumulator sets, which costs more registers than there are.)
    for (int k = 0; k < a.K; ++k) {
        const FusedLevel L = cl.lvt[k];
        gcell_ptr cells = (gcell_ptr)L.cells;
        PtLevel q;
        level_from_geom(L, gslot, q);
        const float *b1 = vec + (size_t)k * 2 * WP;
        const float *b2 = b1 + WP;
        (void)b1;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
            F[mt] = z4;
        Pending pa, pb;
        issue_column<CL>(cells, L, q, 0, g, cols, pa, pb);
#pragma unroll 1
        for (int c = 0; c < 5; ++c) {  // chunks 0..4: halves 2c, 2c+1 in, 2c+2, 2c+3 out
            f4 lo, hi;
            // both halves of the next column share its base
            const float3 cb = column_base(q, c + 1, g, cols);
#pragma unroll
            for (int j = 0; j < 4; ++j)
                lo[j] = finish_one(pa.v[j], pa.fx[j], pa.t[j]);
            issue_four<CL>(cells, L, q, cb.x, cb.y, cb.z, pa);
#pragma unroll
            for (int j = 0; j < 4; ++j)
                hi[j] = finish_one(pb.v[j], pb.fx[j], pb.t[j]);
            // the weight copy goes out after the waits for this chunk's samples (the
            // empty statement keeps the finished samples from sinking below it)
            asm volatile("" ::"v"(lo), "v"(hi));
            ws.fetch(tid);
            issue_four<CL>(cells, L, q, fmaf(4.f, q.c[0], cb.x), fmaf(4.f, q.c[1], cb.y),
                       fmaf(4.f, q.c[2], cb.z), pb);
            mfma_chunk<MT>(ws.chunk(), lane, pack8(lo, hi), F);
            ws.template next<8>(tid);
        }
        {  // chunk 5: issues the table halves of chunk 6
            f4 lo, hi;
#pragma unroll
            for (int j = 0; j < 4; ++j)
                lo[j] = finish_one(pa.v[j], pa.fx[j], pa.t[j]);
            issue_table_half<CL>(cells, L, q, 0, g, plane, pa);
#pragma unroll
            for (int j = 0; j < 4; ++j)
                hi[j] = finish_one(pb.v[j], pb.fx[j], pb.t[j]);
            asm volatile("" ::"v"(lo), "v"(hi));
            ws.fetch(tid);
            issue_table_half<CL>(cells, L, q, 1, g, plane, pb);
            mfma_chunk<MT>(ws.chunk(), lane, pack8(lo, hi), F);
            ws.template next<8>(tid);
        }
        {  // chunk 6: issues chunk 7's stencil sample (4, 4, 8)
            f4 lo, hi;
#pragma unroll
            for (int j = 0; j < 4; ++j)
                lo[j] = finish_one(pa.v[j], pa.fx[j], pa.t[j]);
            issue_one<CL>(cells, L, q.u0[0] + 4.f * (q.a[0] + q.b[0]) + 8.f * q.c[0],
                      q.u0[1] + 4.f * (q.a[1] + q.b[1]) + 8.f * q.c[1],
                      q.u0[2] + 4.f * (q.a[2] + q.b[2]) + 8.f * q.c[2], pa.v[0], pa.fx[0],
                      pa.t[0]);
#pragma unroll
            for (int j = 0; j < 4; ++j)
                hi[j] = finish_one(pb.v[j], pb.fx[j], pb.t[j]);
            asm volatile("" ::"v"(lo), "v"(hi));
            ws.fetch(tid);
            mfma_chunk<MT>(ws.chunk(), lane, pack8(lo, hi), F);
            ws.template next<1>(tid);
        }
        {  // chunk 7: stencil sample (4, 4, 8), gamma, and the odd tile of o^{k-1}
            const float sv = finish_one(pa.v[0], pa.fx[0], pa.t[0]);
            asm volatile("" ::"v"(sv));
            ws.fetch(tid);
            const float one = g == 1 ? 1.f : 0.f;  // the inputs of b1's two parts
            const f4 lo = f4{g == 0 ? sv : one, g == 0 ? gamma : one, 0.f, 0.f};
            mfma_chunk<MT>(ws.chunk(), lane, pack8(lo, (!F8 && (MT & 1)) ? O[MT - 1] : z4),
                           F);
            ws.template next<0>(tid);
        }
        if (k > 0) {
            if constexpr (F8) {
                fp8_layer<MT, NW, true>(ws, tid, lane, O, F);
            } else {
#pragma unroll
                for (int qq = 0; qq < MT / 2; ++qq) {
                    ws.fetch(tid);
                    mfma_chunk<MT>(ws.chunk(), lane, pack8(O[2 * qq], O[2 * qq + 1]), F);
                    ws.template next<0>(tid);
                }
            }
        }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            if constexpr (F8) {  // the BF16 form applies this ReLU when packing
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    F[mt][i] = __builtin_amdgcn_fmed3f(F[mt][i], 0.f, 448.f);
            }
            if constexpr (!FOLD2 && !FOLD8)
                O[mt] += *reinterpret_cast<const f4 *>(b2 + 16 * mt + 4 * g);
        }
        if constexpr (F8) {
            fp8_layer<MT, NW, false, Stage, FOLD8>(ws, tid, lane, F, O);
        } else {
#pragma unroll
            for (int qq = 0; qq < C2; ++qq) {
                ws.fetch(tid);
                mfma_chunk<MT>(ws.chunk(), lane,
                               pack8_relu(F[2 * qq],
                                          (2 * qq + 1 < MT) ? F[2 * qq + 1 < MT ? 2 * qq + 1 : 0]
                                                            : (FOLD2 ? bias_ones(g) : z4)),
                               O);
                ws.template next<0>(tid);
            }
        }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                O[mt][i] = fmaxf(O[mt][i], 0.f);
    }
    const float *bh = vec + (size_t)a.K * 2 * WP;
    int h = 0;
    if constexpr (F8) {
        for (; h + 1 < a.H - 1; h += 2) {
            dense8<MT, NW, Stage, FOLD8>(ws, bh + (size_t)h * WP, tid, lane, O, F);
            dense8<MT, NW, Stage, FOLD8>(ws, bh + (size_t)(h + 1) * WP, tid, lane, F, O);
        }
        if (h < a.H - 1) {
            dense8<MT, NW, Stage, FOLD8>(ws, bh + (size_t)h * WP, tid, lane, O, F);
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
                O[mt] = F[mt];
        }
    } else {
        for (; h + 1 < a.H - 1; h += 2) {
            dense<MT, NW, Stage, FOLD2>(ws, bh + (size_t)h * WP, tid, lane, O, F);
            dense<MT, NW, Stage, FOLD2>(ws, bh + (size_t)(h + 1) * WP, tid, lane, F, O);
        }
        if (h < a.H - 1) {
            dense<MT, NW, Stage, FOLD2>(ws, bh + (size_t)h * WP, tid, lane, O, F);
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
                O[mt] = F[mt];
        }
    }
    const float *wl = bh + (size_t)(a.H - 1) * WP;
    const float bl = wl[WP];
    float acc = 0.f;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
        const f4 w = *reinterpret_cast<const f4 *>(wl + 16 * mt + 4 * g);
        acc += w[0] * O[mt][0] + w[1] * O[mt][1] + w[2] * O[mt][2] + w[3] * O[mt][3];
    }
    acc += __shfl_xor(acc, 16, 64);
    acc += __shfl_xor(acc, 32, 64);
    if (g == 0 && in) {
        const float pre = acc + bl;
        a.out[p] = valid ? fmaxf(pre, 0.f) : 0.f;
        if (a.pre)
            a.pre[p] = valid ? pre : 0.f;
        if (a.flags) {
            float x[3];
            Frame fr;
            point_frame(a, p, in, x, fr);
            a.flags[p] = valid ? point_flags(x, fr, cl.amin, cl.amax, cl.inv_mean)
                               : (uint8_t)DS_FLAG_INVALID;
        }
    }
}

// A usable position of point p outside its cloud's grid box (only the clamped pass
// computes such a point's tile).
__device__ __forceinline__ bool point_outside(const FusedArgs &a, const FusedCloud &cl, int64_t p,
                                              bool in)
{
    if (!in)
        return false;
    const float x0 = a.pos[3 * p], x1 = a.pos[3 * p + 1], x2 = a.pos[3 * p + 2];
    return isfinite(x0) && isfinite(x1) && isfinite(x2) &&
           !(x0 >= cl.amin[0] && x0 <= cl.amax[0] && x1 >= cl.amin[1] && x1 <= cl.amax[1] &&
             x2 >= cl.amin[2] && x2 <= cl.amax[2]);
}

// The clamped pass screens this many tiles of a workgroup at once: every lane keeps the
// position loads of its point in all of them in flight together, and one barrier ORs the
// tiles' needs over the workgroup.  Its grid is persistent and at most kClampGrid
// workgroups (two per compute unit): launched one workgroup per tile, the pass spent its
// time dispatching workgroups that only looked at their positions.
constexpr int kClampBatch = 32;
constexpr int kClampGrid = 512;

template <int MT, int NW, bool F8, bool CL>
__global__ void __launch_bounds__(64 * NW, 2) k_fused_reg(FusedArgs a,
                                                          const uint4 *__restrict__ frags,
                                                          const float *__restrict__ vec)
{
    __shared__ uint4 wbuf[2 * WeightStage<MT, NW>::BUF];
    __shared__ float4 plane[32];
    __shared__ float2 cols[24];
    __shared__ PtGeom geom[16 * NW];   // per point of the tile, see make_geom
    __shared__ uint32_t need[3];        // tiles of a screened batch that need this pass
    const int tid = threadIdx.x;
    const int n = tid & 15;
    init_tables(tid, plane, cols);
    WeightStage<MT, NW> ws;
    ws.init(wbuf, tid);
    if constexpr (!CL) {
        // persistent loop over tiles of 16 NW points; a tile never spans two clouds
#pragma unroll 1
        for (int64_t v = blockIdx.x; v < a.n_tiles; v += gridDim.x) {
            const int64_t t = xcd_tile(v, a.n_tiles);
            // keeps tile-invariant LDS reads (the tables) inside the loop: hoisted, they
            // would hold registers across the whole tile and force spills
            asm volatile("" ::: "memory");
            const FusedCloud &cl = a.cl[tile_cloud(a, t)];
            if (!cl.fast)
                continue;  // uniform: the clamped pass computes this cloud
            const int64_t pl = (t - cl.tile_begin) * (16 * NW) + (tid >> 6) * 16 + n;
            const bool in = pl < cl.P;
            const int64_t p = point_row(a, cl.p_begin + pl, in);
            const bool outside = point_outside(a, cl, p, in);
            ws.begin(frags, tid);
            predict_points<MT, NW, F8, false>(a, cl, vec, ws, tid, geom[(tid >> 6) * 16 + n],
                                              plane, cols, p, in, outside);
        }
    } else {
        // Batch b of the workgroup's tiles ORs its needs into need[b % 3] and reads it after
        // the barrier; thread 0 then clears need[(b + 2) % 3], whose last readers (batch
        // b - 1) and next writers (batch b + 2, after the next barrier) are both on the
        // other side of a barrier.
        if (tid < 3)
            need[tid] = 0;
        __syncthreads();
        int slot = 0;
#pragma unroll 1
        for (int64_t v0 = blockIdx.x; v0 < a.n_tiles; v0 += (int64_t)kClampBatch * gridDim.x) {
            uint32_t mine = 0;
#pragma unroll
            for (int j = 0; j < kClampBatch; ++j) {
                const int64_t v = v0 + (int64_t)j * gridDim.x;
                if (v < a.n_tiles) {  // uniform
                    const FusedCloud &cl = a.cl[tile_cloud(a, xcd_tile(v, a.n_tiles))];
                    const int64_t pl = (xcd_tile(v, a.n_tiles) - cl.tile_begin) * (16 * NW) +
                                       (tid >> 6) * 16 + n;
                    const bool in = pl < cl.P;
                    if (!cl.fast || point_outside(a, cl, point_row(a, cl.p_begin + pl, in), in))
                        mine |= 1u << j;
                }
            }
            if (mine)
                atomicOr(&need[slot], mine);
            __syncthreads();
            const uint32_t m = need[slot];
            if (tid == 0)
                need[slot == 0 ? 2 : slot - 1] = 0;  // (slot + 2) % 3
            slot = slot == 2 ? 0 : slot + 1;
#pragma unroll 1
            for (int j = 0; j < kClampBatch; ++j) {
                if (!((m >> j) & 1u))
                    continue;  // uniform
                const int64_t t = xcd_tile(v0 + (int64_t)j * gridDim.x, a.n_tiles);
                asm volatile("" ::: "memory");
                const FusedCloud &cl = a.cl[tile_cloud(a, t)];
                const int64_t pl = (t - cl.tile_begin) * (16 * NW) + (tid >> 6) * 16 + n;
                const bool in = pl < cl.P;
                const int64_t p = point_row(a, cl.p_begin + pl, in);
                const bool outside = point_outside(a, cl, p, in);
                ws.begin(frags, tid);
                predict_points<MT, NW, F8, true>(a, cl, vec, ws, tid, geom[(tid >> 6) * 16 + n],
                                                 plane, cols, p, in, outside);
            }
        }
    }
}

// Unclamped pass of the register kernel with two teams of four waves sharing one weight
// ring (TeamRing): tiles of 128 points, team 0 taking points 0..63 and team 1 points
// 64..127 of each, team 1 kTeamLag chunks behind.  Clouds that need the clamps and tiles
// with a point outside the grid box are left to the clamped pass of the four-wave kernel,
// whose 64-point tiles are these tiles' halves.
constexpr int kTeamRing = 10, kTeamLag = 6;

template <int MT, bool F8>
__global__ void __launch_bounds__(512, 2) k_fused_teams(FusedArgs a,
                                                        const uint4 *__restrict__ frags,
                                                        const float *__restrict__ vec, int nc)
{
    __shared__ uint4 ring[kTeamRing * MT * 64];
    __shared__ float4 plane[32];
    __shared__ float2 cols[24];
    __shared__ PtGeom geom[128];
    const int tid = threadIdx.x;
    const int n = tid & 15;
    init_tables(tid, plane, cols);
    TeamRing<MT, kTeamRing, kTeamLag> ws;
    ws.init(ring, frags, nc, tid);
    ws.prologue(tid);  // also publishes the tables
    if (ws.team == 1)
        ws.idle(tid, kTeamLag);
#pragma unroll 1
    for (int64_t v = blockIdx.x; v < a.n_tiles; v += gridDim.x) {
        const int64_t t = xcd_tile(v, a.n_tiles);
        asm volatile("" ::: "memory");
        const FusedCloud &cl = a.cl[tile_cloud(a, t)];
        if (!cl.fast) {  // uniform: the clamped pass computes this cloud
            ws.idle(tid, nc);
            continue;
        }
        const int64_t pl = (t - cl.tile_begin) * 128 + (tid >> 6) * 16 + n;
        const bool in = pl < cl.P;
        const int64_t p = point_row(a, cl.p_begin + pl, in);
        const bool outside = point_outside(a, cl, p, in);
        predict_points<MT, 8, F8, false>(a, cl, vec, ws, tid, geom[(tid >> 6) * 16 + n], plane,
                                         cols, p, in, outside);
    }
    if (ws.team == 0)
        ws.idle(tid, kTeamLag);
}

// Wide variant: one wave per SIMD holding two 16-point tiles, so every weight
// fragment read from LDS feeds two MFMAs and a workgroup covers 128 points (half the
// LDS fragment reads, weight copies and barriers per point).  With one wave per
// SIMD the accumulators of both tiles live in the accumulation registers; the two
// tiles' samples of a chunk are in flight together.
template <int MT, int NT>
__device__ __forceinline__ void mfma_chunk_nt(const uint4 *w, int lane, const bf16x8 (&B)[NT],
                                              f4 (&acc)[MT][NT])
{
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
        const uint4 wa = w[mt * 64 + lane];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
            acc[mt][nt] = mfma_bf16(wa, B[nt], acc[mt][nt]);
    }
}

template <int MT, int NW, int NT>
__device__ __forceinline__ void dense_nt(WeightStage<MT, NW> &ws, const float *__restrict__ bias,
                                         int tid, int lane, const f4 (&in)[MT][NT],
                                         f4 (&out)[MT][NT])
{
    constexpr int C2 = (MT + 1) / 2;
    const int g = lane >> 4;
    const f4 z4 = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
        const f4 b = *reinterpret_cast<const f4 *>(bias + 16 * mt + 4 * g);
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
            out[mt][nt] = b;
    }
#pragma unroll
    for (int q = 0; q < C2; ++q) {
        ws.fetch(tid);
        bf16x8 B[NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
            B[nt] = pack8(in[2 * q][nt], (2 * q + 1 < MT) ? in[2 * q + 1 < MT ? 2 * q + 1 : 0][nt] : z4);
        mfma_chunk_nt<MT, NT>(ws.chunk(), lane, B, out);
        ws.template next<0>(tid);
    }
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                out[mt][nt][i] = fmaxf(out[mt][nt][i], 0.f);
}

template <int MT, int NW>
__global__ void __launch_bounds__(64 * NW, 1) k_fused_wide(FusedArgs a,
                                                           const uint4 *__restrict__ frags,
                                                           const float *__restrict__ vec)
{
    constexpr int NT = 2;
    constexpr int C2 = (MT + 1) / 2;
    constexpr int WP = 16 * MT;
    constexpr int TP = 16 * NW * NT;   // points per tile
    __shared__ uint4 wbuf[2 * WeightStage<MT, NW>::BUF];
    __shared__ float4 plane[32];
    __shared__ float2 cols[24];
    __shared__ PtGeom geom[TP];        // per point of the tile, see make_geom
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int g = lane >> 4, n = lane & 15;
    const int wv = tid >> 6;
    init_tables(tid, plane, cols);
    WeightStage<MT, NW> ws;
    ws.init(wbuf, tid);
#pragma unroll 1
    for (int64_t v = blockIdx.x; v < a.n_tiles; v += gridDim.x) {
        const int64_t t = xcd_tile(v, a.n_tiles);
        asm volatile("" ::: "memory");
        const FusedCloud &cl = a.cl[tile_cloud(a, t)];
        ws.begin(frags, tid);
        bool in[NT], valid[NT];
        float gamma[NT];
        int64_t p[NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            const int64_t pl = (t - cl.tile_begin) * TP + (wv * NT + nt) * 16 + n;
            in[nt] = pl < cl.P;
            p[nt] = point_row(a, cl.p_begin + pl, in[nt]);
            float x[3];
            Frame fr;
            valid[nt] = point_frame(a, p[nt], in[nt], x, fr);
            gamma[nt] = fr.gamma;
            geom[(wv * NT + nt) * 16 + n] = make_geom(x, fr, cl.amin, valid[nt]);
        }
        const f4 z4 = f4{0.f, 0.f, 0.f, 0.f};
        f4 O[MT][NT], F[MT][NT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
                O[mt][nt] = z4;

        for (int k = 0; k < a.K; ++k) {
            const FusedLevel L = cl.lvt[k];
            gcell_ptr cells = (gcell_ptr)L.cells;
            PtLevel q[NT];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
                level_from_geom(L, geom[(wv * NT + nt) * 16 + n], q[nt]);
            const float *b1 = vec + (size_t)k * 2 * WP;
            const float *b2 = b1 + WP;
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                const f4 bb = *reinterpret_cast<const f4 *>(b1 + 16 * mt + 4 * g);
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
                    F[mt][nt] = bb;
            }
#pragma unroll 1
            for (int c = 0; c < 7; ++c) {
                Pending pa[NT], pb[NT];
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) {
                    if (c < 6) {
                        issue_column_half(cells, L, q[nt], 2 * c, g, cols, pa[nt]);
                        issue_column_half(cells, L, q[nt], 2 * c + 1, g, cols, pb[nt]);
                    } else {
                        issue_table_half(cells, L, q[nt], 0, g, plane, pa[nt]);
                        issue_table_half(cells, L, q[nt], 1, g, plane, pb[nt]);
                    }
                }
                ws.fetch(tid);
                bf16x8 B[NT];
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) {
                    f4 lo, hi;
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        lo[j] = finish_one(pa[nt].v[j], pa[nt].fx[j], pa[nt].t[j]);
                        hi[j] = finish_one(pb[nt].v[j], pb[nt].fx[j], pb[nt].t[j]);
                    }
                    B[nt] = pack8(lo, hi);
                }
                mfma_chunk_nt<MT, NT>(ws.chunk(), lane, B, F);
                ws.template next<0>(tid);
            }
            {
                Pending pa[NT];
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
                    issue_one(cells, L, q[nt].u0[0] + 4.f * (q[nt].a[0] + q[nt].b[0]) + 8.f * q[nt].c[0],
                              q[nt].u0[1] + 4.f * (q[nt].a[1] + q[nt].b[1]) + 8.f * q[nt].c[1],
                              q[nt].u0[2] + 4.f * (q[nt].a[2] + q[nt].b[2]) + 8.f * q[nt].c[2],
                              pa[nt].v[0], pa[nt].fx[0], pa[nt].t[0]);
                ws.fetch(tid);
                bf16x8 B[NT];
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) {
                    const float sv = finish_one(pa[nt].v[0], pa[nt].fx[0], pa[nt].t[0]);
                    const f4 lo = f4{g == 0 ? sv : 0.f, g == 0 ? gamma[nt] : 0.f, 0.f, 0.f};
                    B[nt] = pack8(lo, (MT & 1) ? O[MT - 1][nt] : z4);
                }
                mfma_chunk_nt<MT, NT>(ws.chunk(), lane, B, F);
                ws.template next<0>(tid);
            }
            if (k > 0) {
#pragma unroll
                for (int qq = 0; qq < MT / 2; ++qq) {
                    ws.fetch(tid);
                    bf16x8 B[NT];
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt)
                        B[nt] = pack8(O[2 * qq][nt], O[2 * qq + 1][nt]);
                    mfma_chunk_nt<MT, NT>(ws.chunk(), lane, B, F);
                    ws.template next<0>(tid);
                }
            }
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                const f4 cc = *reinterpret_cast<const f4 *>(b2 + 16 * mt + 4 * g);
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) {
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        F[mt][nt][i] = fmaxf(F[mt][nt][i], 0.f);
                    O[mt][nt] += cc;
                }
            }
#pragma unroll
            for (int qq = 0; qq < C2; ++qq) {
                ws.fetch(tid);
                bf16x8 B[NT];
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
                    B[nt] = pack8(F[2 * qq][nt],
                                  (2 * qq + 1 < MT) ? F[2 * qq + 1 < MT ? 2 * qq + 1 : 0][nt] : z4);
                mfma_chunk_nt<MT, NT>(ws.chunk(), lane, B, O);
                ws.template next<0>(tid);
            }
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        O[mt][nt][i] = fmaxf(O[mt][nt][i], 0.f);
        }
        const float *bh = vec + (size_t)a.K * 2 * WP;
        int h = 0;
        for (; h + 1 < a.H - 1; h += 2) {
            dense_nt<MT, NW, NT>(ws, bh + (size_t)h * WP, tid, lane, O, F);
            dense_nt<MT, NW, NT>(ws, bh + (size_t)(h + 1) * WP, tid, lane, F, O);
        }
        if (h < a.H - 1) {
            dense_nt<MT, NW, NT>(ws, bh + (size_t)h * WP, tid, lane, O, F);
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
                    O[mt][nt] = F[mt][nt];
        }
        const float *wl = bh + (size_t)(a.H - 1) * WP;
        const float bl = wl[WP];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            float acc = 0.f;
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                const f4 w = *reinterpret_cast<const f4 *>(wl + 16 * mt + 4 * g);
                acc += w[0] * O[mt][nt][0] + w[1] * O[mt][nt][1] + w[2] * O[mt][nt][2] +
                       w[3] * O[mt][nt][3];
            }
            acc += __shfl_xor(acc, 16, 64);
            acc += __shfl_xor(acc, 32, 64);
            if (g == 0 && in[nt]) {
                const float pre = acc + bl;
                a.out[p[nt]] = valid[nt] ? fmaxf(pre, 0.f) : 0.f;
                if (a.pre)
                    a.pre[p[nt]] = valid[nt] ? pre : 0.f;
                if (a.flags) {
                    float x[3];
                    Frame fr;
                    point_frame(a, p[nt], in[nt], x, fr);
                    a.flags[p[nt]] = valid[nt] ? point_flags(x, fr, cl.amin, cl.amax, cl.inv_mean)
                                               : (uint8_t)DS_FLAG_INVALID;
                }
            }
        }
    }
}

// The fused kernel's gather schedule on its own: every sample is written to its
// canonical descriptor position [k][ix + 5 iy + 25 iz] (and gamma last), so the
// BF16 gather path can be checked against the plain descriptor.
__device__ __forceinline__ int column_sample(int c, int g, int j)
{
    const int col = 4 * c + g;
    return (col % 5) + 5 * (col / 5) + 25 * j;
}

__global__ void __launch_bounds__(256) k_gather_packed(FusedArgs a, float *__restrict__ z)
{
    __shared__ float4 plane[32];
    __shared__ float2 cols[24];
    const int tid = threadIdx.x, lane = tid & 63, g = lane >> 4, n = lane & 15;
    init_tables(tid, plane, cols);
    __syncthreads();
    const FusedCloud &cl = a.cl[0];
    const int64_t p = (int64_t)blockIdx.x * 64 + (tid >> 6) * 16 + n;
    const bool in = p < cl.P;
    float x[3];
    Frame fr;
    const bool valid = point_frame(a, p, in, x, fr);
    const int64_t D = 225 * (int64_t)a.K + 1;
    for (int k = 0; k < a.K; ++k) {
        const FusedLevel L = cl.lvt[k];
        gcell_ptr cells = (gcell_ptr)L.cells;
        PtLevel q;
        level_from_geom(L, make_geom(x, fr, cl.amin, valid), q);
        Pending pa;
        for (int h = 0; h < 12; ++h) {
            issue_column_half(cells, L, q, h, g, cols, pa);
            for (int j = 0; j < 4; ++j) {
                float v = finish_one(pa.v[j], pa.fx[j], pa.t[j]);
                if (in)
                    z[p * D + 225 * k + column_sample(h >> 1, g, 4 * (h & 1) + j)] = v;
            }
        }
        for (int hh = 0; hh < 2; ++hh) {
            issue_table_half(cells, L, q, hh, g, plane, pa);
            for (int j = 0; j < 4; ++j) {
                float v = finish_one(pa.v[j], pa.fx[j], pa.t[j]);
                float4 o = plane[8 * g + 4 * hh + j];
                int sidx = (int)o.x + 5 * (int)o.y + 25 * (int)o.z;
                if (in)
                    z[p * D + 225 * k + sidx] = v;
            }
        }
        if (g == 0) {
            issue_one(cells, L, q.u0[0] + 4.f * (q.a[0] + q.b[0]) + 8.f * q.c[0],
                      q.u0[1] + 4.f * (q.a[1] + q.b[1]) + 8.f * q.c[1],
                      q.u0[2] + 4.f * (q.a[2] + q.b[2]) + 8.f * q.c[2], pa.v[0], pa.fx[0],
                      pa.t[0]);
            float v = finish_one(pa.v[0], pa.fx[0], pa.t[0]);
            if (in)
                z[p * D + 225 * k + 224] = v;
        }
    }
    if (g == 0 && in)
        z[p * D + D - 1] = fr.gamma;
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

// Inputs of a W-wide layer's chunk q that carry the layer's bias (high part at j = 4, low
// part at j = 5 of lane group 0): the free half of the last chunk when MT is odd.
bool bias_slot(int MT, int q, int g, int j)
{
    return (MT & 1) && q == (MT + 1) / 2 - 1 && g == 0 && (j == 4 || j == 5);
}

// fragment map entries of a bias's low part: the parameter index with this bit set; the
// packing stores bf16(v - bf16(v)) there (v the parameter), the high part stores bf16(v)
constexpr int64_t kLowPart = (int64_t)1 << 30;

// Chunks in consumption order: block 1 has 8 stencil chunks, later blocks also the
// o^{k-1} pairs; every block then its second layer; then the dense trailing layers.
int chunk_count(int MT, int K, int H)
{
    int C1 = 8 + MT / 2, C2 = (MT + 1) / 2;
    return (8 + C2) + (K - 1) * (C1 + C2) + (H - 1) * C2;
}

// staging slots per tile of the FP8 form: 8 stencil slots per block, two slots per FP8
// chunk of 128 inputs for W1 (blocks 2..K), W2 and the dense trailing layers
int fp8_slot_count(int MT, int K, int H)
{
    const int C8 = (MT + 7) / 8;
    return (8 + 2 * C8) + (K - 1) * (8 + 4 * C8) + (H - 1) * 2 * C8;
}

// zeroed entries after the last chunk: the copies run up to two groups (2 x 4 chunks of
// at most 16 x 64 entries) past the chunk being consumed
constexpr size_t kFragPad = 8192;

// Tile partition of the clouds for tiles of `per` points; returns the tile count.
int64_t assign_tiles(FusedArgs &a, int64_t per)
{
    int64_t t = 0;
    for (int c = 0; c < a.n_clouds; ++c) {
        a.cl[c].tile_begin = t;
        t += (a.cl[c].P + per - 1) / per;
    }
    a.n_tiles = t;
    return t;
}

template <int MT, int NW, int KIND, bool F8 = false>
ds_status launch_kind(hipStream_t s, const ds_net *net, FusedArgs a, int grid)
{
    const int64_t tiles = assign_tiles(a, 16 * NW * (KIND == DS_KERNEL_WIDE ? 2 : 1));
    if (tiles <= 0)
        return DS_OK;
    const int64_t g = grid > 0 && grid < tiles ? grid : tiles;
    DS_CHECK(g < ((int64_t)1 << 31), DS_ERR_INVALID_ARG, "too many tiles for one launch");
    const unsigned gc = (unsigned)std::min<int64_t>(g, kClampGrid);  // the clamped pass
    if constexpr (F8) {
        static_assert(KIND == DS_KERNEL_REGISTER, "the FP8 form has the register kernel only");
        k_fused_reg<MT, NW, true, false><<<(unsigned)g, 64 * NW, 0, s>>>(a, net->frag_fp8, net->vec8);
        k_fused_reg<MT, NW, true, true><<<gc, 64 * NW, 0, s>>>(a, net->frag_fp8, net->vec8);
    } else if constexpr (KIND == DS_KERNEL_PIPELINED) {
        k_fused<MT, NW><<<(unsigned)g, 64 * NW, 0, s>>>(a, net->frag_bf16, net->vec);
    } else if constexpr (KIND == DS_KERNEL_WIDE) {
        k_fused_wide<MT, NW><<<(unsigned)g, 64 * NW, 0, s>>>(a, net->frag_bf16, net->vec);
    } else {
        k_fused_reg<MT, NW, false, false><<<(unsigned)g, 64 * NW, 0, s>>>(a, net->frag_bf16, net->vec);
        k_fused_reg<MT, NW, false, true><<<gc, 64 * NW, 0, s>>>(a, net->frag_bf16, net->vec);
    }
    DS_HIP(hipGetLastError());
    return DS_OK;
}

// The two-team kernel's unclamped pass on 128-point tiles, then the clamped pass of the
// four-wave register kernel on 64-point tiles (the halves of those tiles).
template <int MT, bool F8>
ds_status launch_teams(hipStream_t s, const ds_net *net, FusedArgs a, int grid)
{
    const int nc = F8 ? fp8_slot_count(MT, a.K, a.H) : chunk_count(MT, a.K, a.H);
    const uint4 *frags = F8 ? net->frag_fp8 : net->frag_bf16;
    const float *vec = F8 ? net->vec8 : net->vec;
    FusedArgs a4 = a;
    const int64_t tiles = assign_tiles(a, 128), tiles4 = assign_tiles(a4, 64);
    if (tiles <= 0)
        return DS_OK;
    const int64_t g = grid > 0 && grid < tiles ? grid : tiles;
    const int64_t g4 = grid > 0 && grid < tiles4 ? grid : tiles4;
    DS_CHECK(g4 < ((int64_t)1 << 31) && nc % 2 == 0, DS_ERR_INVALID_ARG,
             "two-team launch: %lld tiles, %d chunks per tile", (long long)tiles4, nc);
    k_fused_teams<MT, F8><<<(unsigned)g, 512, 0, s>>>(a, frags, vec, nc);
    k_fused_reg<MT, 4, F8, true><<<(unsigned)std::min<int64_t>(g4, kClampGrid), 256, 0, s>>>(
        a4, frags, vec);
    DS_HIP(hipGetLastError());
    return DS_OK;
}

// Eight waves need LDS for twice the points: the register kernel fits below 16
// tiles, the pipelined one (residual stream in LDS) below 13; the wide kernel runs
// one wave per SIMD, so four waves only.
constexpr bool fits(int MT, int waves, int kind)
{
    if (kind == DS_KERNEL_WIDE)
        return waves == 4;
    return waves == 4 || (kind == DS_KERNEL_REGISTER ? MT < 16 : MT < 13);
}

template <int MT>
ds_status launch(hipStream_t s, const ds_net *net, const FusedArgs &a, const FusedVariant &v,
                 bool fp8)
{
    if (v.kind == DS_KERNEL_TEAMS) {
        if constexpr (MT < 16)
            return fp8 ? launch_teams<MT, true>(s, net, a, v.grid)
                       : launch_teams<MT, false>(s, net, a, v.grid);
        set_error("the two-team kernel does not fit width %d", net->W);
        return DS_ERR_UNSUPPORTED;
    }
    if (fp8) {
        if constexpr (fits(MT, 8, DS_KERNEL_REGISTER)) {
            if (v.waves == 8)
                return launch_kind<MT, 8, DS_KERNEL_REGISTER, true>(s, net, a, v.grid);
        }
        if (v.waves == 4)
            return launch_kind<MT, 4, DS_KERNEL_REGISTER, true>(s, net, a, v.grid);
        set_error("eight waves per workgroup do not fit this kernel at width %d", net->W);
        return DS_ERR_UNSUPPORTED;
    }
    if (v.waves == 8) {
        if constexpr (fits(MT, 8, DS_KERNEL_PIPELINED)) {
            if (v.kind == DS_KERNEL_PIPELINED)
                return launch_kind<MT, 8, DS_KERNEL_PIPELINED>(s, net, a, v.grid);
        }
        if constexpr (fits(MT, 8, DS_KERNEL_REGISTER)) {
            if (v.kind == DS_KERNEL_REGISTER)
                return launch_kind<MT, 8, DS_KERNEL_REGISTER>(s, net, a, v.grid);
        }
        set_error("eight waves per workgroup do not fit this kernel at width %d", net->W);
        return DS_ERR_UNSUPPORTED;
    }
    if (v.kind == DS_KERNEL_PIPELINED)
        return launch_kind<MT, 4, DS_KERNEL_PIPELINED>(s, net, a, v.grid);
    if (v.kind == DS_KERNEL_WIDE)
        return launch_kind<MT, 4, DS_KERNEL_WIDE>(s, net, a, v.grid);
    return launch_kind<MT, 4, DS_KERNEL_REGISTER>(s, net, a, v.grid);
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

namespace {
// Offsets of every parameter block in the canonical order: per block V [W][226],
// W1 [W][W] (not for the first block), b1, W2 [W][W], b2; then per trailing layer its
// matrix and bias (the last one has a single output).
struct ParamBlocks {
    std::vector<int64_t> V, W1, b1, W2, b2, hw, hb;
};
ParamBlocks param_blocks(int K, int W, int H)
{
    ParamBlocks o;
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

// Stencil sample (index n = ix + 5 iy + 25 iz) held by slot (g, j) of stencil chunk
// c < 7: chunks 0..5 and g = 0 of chunk 6 walk the 25 columns (iz = j); lanes g = 1..3
// of chunk 6 cover the iz = 8 plane as five rows of four and one column of four.
int stencil_slot(int c, int g, int j)
{
    if (c < 6 || g == 0) {
        int col = 4 * c + g;  // column (ix, iy), iz = j
        return (col % 5) + 5 * (col / 5) + 25 * j;
    }
    int G = 2 * (g - 1) + (j >> 2), jj = j & 3;  // plane iz = 8
    return G < 5 ? jj + 5 * G + 25 * 8 : 4 + 5 * jj + 25 * 8;
}
}  // namespace

// Packing maps: for every bf16 element of the weight fragments (in kernel order)
// and every FP32 entry of the bias / final-layer vector, the index of the
// canonical parameter it holds, or -1 for padding.
static void build_pack_maps(int K, int W, int H, std::vector<int32_t> &fmap,
                            std::vector<int32_t> &vmap)
{
    const int MT = fused_tiles(W);
    const int C1 = 8 + MT / 2, C2 = (MT + 1) / 2, WP = 16 * MT;
    const ParamBlocks pb = param_blocks(K, W, H);
    const std::vector<int64_t> &oV = pb.V, &oW1 = pb.W1, &ob1 = pb.b1, &oW2 = pb.W2,
                               &ob2 = pb.b2, &ohw = pb.hw, &ohb = pb.hb;
    const int64_t nfr = (int64_t)chunk_count(MT, K, H) * MT;
    fmap.assign((size_t)nfr * 64 * 8, -1);
    auto put = [&](int64_t frag, int g, int r, int j, int64_t idx) {
        fmap[((size_t)frag * 64 + 16 * g + r) * 8 + j] = (int32_t)idx;
    };
    int64_t frag = 0;
    for (int k = 0; k < K; ++k) {
        const int c1 = k == 0 ? 8 : C1;
        for (int c = 0; c < c1; ++c, frag += MT)
            for (int mt = 0; mt < MT; ++mt)
                for (int g = 0; g < 4; ++g)
                    for (int r = 0; r < 16; ++r) {
                        const int row = 16 * mt + r;
                        if (row >= W)
                            continue;
                        for (int j = 0; j < 8; ++j) {
                            int64_t idx = -1;
                            if (c < 7) {
                                idx = oV[k] + (int64_t)row * 226 + stencil_slot(c, g, j);
                            } else if (c == 7) {
                                if (g == 0 && j == 0)
                                    idx = oV[k] + (int64_t)row * 226 + 224;  // (4, 4, 8)
                                else if (g == 0 && j == 1)
                                    idx = oV[k] + (int64_t)row * 226 + 225;  // gamma
                                else if (g == 1 && j < 2)  // b1: high, low part
                                    idx = (ob1[k] + row) | (j ? kLowPart : 0);
                                else if (j >= 4 && (MT & 1) && k > 0) {
                                    const int col = 16 * (MT - 1) + 4 * g + (j - 4);
                                    if (col < W)
                                        idx = oW1[k] + (int64_t)row * W + col;
                                }
                            } else {
                                const int col = pair_slot(MT, c - 8, g, j);
                                if (col >= 0 && col < W)
                                    idx = oW1[k] + (int64_t)row * W + col;
                            }
                            put(frag + mt, g, r, j, idx);
                        }
                    }
        for (int q = 0; q < C2; ++q, frag += MT)
            for (int mt = 0; mt < MT; ++mt)
                for (int g = 0; g < 4; ++g)
                    for (int r = 0; r < 16; ++r) {
                        const int row = 16 * mt + r;
                        if (row >= W)
                            continue;
                        for (int j = 0; j < 8; ++j) {
                            const int col = pair_slot(MT, q, g, j);
                            int64_t idx = (col >= 0 && col < W) ? oW2[k] + (int64_t)row * W + col : -1;
                            if (bias_slot(MT, q, g, j))  // b2: high, low part
                                idx = (ob2[k] + row) | (j == 5 ? kLowPart : 0);
                            put(frag + mt, g, r, j, idx);
                        }
                    }
    }
    for (int h = 0; h < H - 1; ++h)
        for (int q = 0; q < C2; ++q, frag += MT)
            for (int mt = 0; mt < MT; ++mt)
                for (int g = 0; g < 4; ++g)
                    for (int r = 0; r < 16; ++r) {
                        const int row = 16 * mt + r;
                        if (row >= W)
                            continue;
                        for (int j = 0; j < 8; ++j) {
                            const int col = pair_slot(MT, q, g, j);
                            int64_t idx = (col >= 0 && col < W) ? ohw[h] + (int64_t)row * W + col : -1;
                            if (bias_slot(MT, q, g, j))  // the layer's bias: high, low part
                                idx = (ohb[h] + row) | (j == 5 ? kLowPart : 0);
                            put(frag + mt, g, r, j, idx);
                        }
                    }
    // vectors: per block b1, b2; per dense trailing layer its bias; final weights + bias
    const int64_t nvec = (int64_t)K * 2 * WP + (int64_t)(H - 1) * WP + WP + 4;
    vmap.assign((size_t)nvec, -1);
    for (int k = 0; k < K; ++k)
        for (int r = 0; r < W; ++r) {
            vmap[(size_t)k * 2 * WP + r] = (int32_t)(ob1[k] + r);
            vmap[(size_t)k * 2 * WP + WP + r] = (int32_t)(ob2[k] + r);
        }
    for (int h = 0; h < H - 1; ++h)
        for (int r = 0; r < W; ++r)
            vmap[(size_t)K * 2 * WP + (size_t)h * WP + r] = (int32_t)(ohb[h] + r);
    const size_t wl = (size_t)K * 2 * WP + (size_t)(H - 1) * WP;
    for (int c = 0; c < W; ++c)
        vmap[wl + c] = (int32_t)(ohw[H - 1] + c);
    vmap[wl + WP] = (int32_t)ohb[H - 1];
}

namespace {
__global__ void __launch_bounds__(256) k_pack_frags(const float *__restrict__ theta,
                                                    const int32_t *__restrict__ map, int64_t n,
                                                    uint16_t *__restrict__ out)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t idx = map[i];
        float v = 0.f;
        if (idx >= 0) {
            v = theta[idx & (int32_t)(kLowPart - 1)];
            if (idx & (int32_t)kLowPart) {  // low part: the remainder of the high part
                uint32_t h = __float_as_uint(v);
                h = (h + 0x7FFFu + ((h >> 16) & 1u)) & 0xFFFF0000u;
                v -= __uint_as_float(h);
            }
        }
        uint32_t u = __float_as_uint(v);
        u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
        out[i] = (uint16_t)(u >> 16);
    }
}
__global__ void __launch_bounds__(256) k_pack_vec(const float *__restrict__ theta,
                                                  const int32_t *__restrict__ map, int64_t n,
                                                  float *__restrict__ out)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t idx = map[i];
        out[i] = idx >= 0 ? theta[idx] : 0.f;
    }
}
}  // namespace

// Allocate the fused-kernel operands and their index maps (once per network).
ds_status fused_prepare(ds_net *net)
{
    if (net->frag_bf16)
        return DS_OK;
    DS_CHECK(fused_tiles(net->W) > 0, DS_ERR_UNSUPPORTED,
             "width %d is not supported by the fused kernel", net->W);
    DS_CHECK(net->n_params < kLowPart, DS_ERR_UNSUPPORTED,
             "%lld parameters: the fused kernel's packing map holds fewer than 2^30",
             (long long)net->n_params);
    std::vector<int32_t> fmap, vmap;
    build_pack_maps(net->K, net->W, net->H, fmap, vmap);
    const int64_t nf = (int64_t)fmap.size(), nv = (int64_t)vmap.size();
    // zeroed tail: the kernel's branch-free staging may read past the last chunk
    const size_t fbytes = (size_t)nf * 2 + kFragPad * 16;
    DS_CHECK(hipMalloc(&net->frag_bf16, fbytes) == hipSuccess, DS_ERR_OOM,
             "out of device memory for the packed weights");
    DS_HIP(hipMemset(net->frag_bf16, 0, fbytes));
    net->frag_count = nf / 8;
    DS_CHECK(hipMalloc(&net->vec, (size_t)nv * 4) == hipSuccess, DS_ERR_OOM,
             "out of device memory for the packed biases");
    net->vec_count = nv;
    DS_CHECK(hipMalloc(&net->fmap, (size_t)nf * 4) == hipSuccess, DS_ERR_OOM,
             "out of device memory for the packing map");
    DS_CHECK(hipMalloc(&net->vmap, (size_t)nv * 4) == hipSuccess, DS_ERR_OOM,
             "out of device memory for the packing map");
    DS_HIP(hipMemcpy(net->fmap, fmap.data(), (size_t)nf * 4, hipMemcpyHostToDevice));
    DS_HIP(hipMemcpy(net->vmap, vmap.data(), (size_t)nv * 4, hipMemcpyHostToDevice));
    return DS_OK;
}

// Refresh the BF16 fragments and the FP32 vectors from the device master parameters.
ds_status fused_pack_bf16(hipStream_t s, ds_net *net)
{
    ds_status st = fused_prepare(net);
    if (st)
        return st;
    const int64_t nf = net->frag_count * 8, nv = net->vec_count;
    k_pack_frags<<<(unsigned)((nf + 255) / 256 < 8192 ? (nf + 255) / 256 : 8192), 256, 0, s>>>(
        net->theta, net->fmap, nf, reinterpret_cast<uint16_t *>(net->frag_bf16));
    k_pack_vec<<<(unsigned)((nv + 255) / 256), 256, 0, s>>>(net->theta, net->vmap, nv, net->vec);
    DS_HIP(hipGetLastError());
    return DS_OK;
}

// ------------------------------------------------------------------ FP8 form
int fp8_exp_count(int K, int H) { return 3 * K + 2 * H - 2; }

uint8_t e4m3_encode(float x)
{
    if (isnan(x))
        return 0x7F;
    const uint8_t sign = signbit(x) ? 0x80 : 0x00;
    const double a = fabs((double)x);
    if (a >= 464.0)  // beyond the rounding range of 448 = 1.75 * 2^8: saturate
        return sign | 0x7E;
    if (a < 0.015625) {  // below 2^-6: subnormal, a multiple of 2^-9 (8 -> smallest normal)
        return sign | (uint8_t)nearbyint(a * 512.0);
    }
    int e;
    frexp(a, &e);
    e -= 1;                                        // a in [2^e, 2^(e+1)), e in -6..8
    int q = (int)nearbyint(ldexp(a, 3 - e));       // 8..16, ties to even
    if (q == 16) {
        q = 8;
        ++e;
    }
    const int code = ((e + 7) << 3) | (q - 8);
    return sign | (uint8_t)(code > 0x7E ? 0x7E : code);
}

namespace {
// Largest e with amax * 2^e <= 448 (0 for an all-zero tensor), kept within +-32 so that
// every E8M0 operand scale of the kernel stays inside its range.
int log2_scale(double amax)
{
    if (!(amax > 0.0) || !isfinite(amax))
        return 0;
    int e = (int)floor(log2(448.0 / amax));
    while (ldexp(amax, e) > 448.0)
        --e;
    while (ldexp(amax, e + 1) <= 448.0)
        ++e;
    return e < -32 ? -32 : (e > 32 ? 32 : e);
}

uint16_t bf16_rne(float x)
{
    uint32_t u;
    memcpy(&u, &x, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// value of an OCP E4M3 code (bias 7, subnormals below 2^-6; 0x7F/0xFF are NaN, never encoded)
double e4m3_value(uint8_t c)
{
    const double sgn = (c & 0x80) ? -1.0 : 1.0;
    const int e = (c >> 3) & 15, m = c & 7;
    return sgn * (e == 0 ? ldexp((double)m, -9) : ldexp(1.0 + m / 8.0, e - 7));
}

double tensor_amax(const float *th, int64_t off, int64_t n)
{
    double m = 0.0;
    for (int64_t i = 0; i < n; ++i)
        m = fmax(m, fabs((double)th[off + i]));
    return m;
}
}  // namespace

// The FP8 form in kernel order.  Per block: the 8 stencil chunks in BF16 with V and the
// gamma weights multiplied by 2^f_k (exact: a power of two), then (blocks 2..K) the W1
// chunks and the W2 chunks in E4M3, each FP8 chunk covering 128 inputs (8 tiles of the
// previous layer) in two 16-byte staging slots; then the dense trailing layers.  A
// matrix is encoded as RNE(w * 2^e), e = its output unit - its input unit.
ds_status fused_quantize_fp8(ds_net *net, const float *th, const float *act_amax)
{
    const int K = net->K, W = net->W, H = net->H, MT = fused_tiles(W);
    DS_CHECK(MT > 0, DS_ERR_UNSUPPORTED, "width %d is not supported by the fused kernel", W);
    const int C8 = (MT + 7) / 8, WP = 16 * MT;
    const ParamBlocks pb = param_blocks(K, W, H);
    // Range-filling exponents: activations from the calibration maxima, weights from
    // their own maxima.
    std::vector<int> eF(K), eH(H > 1 ? H - 1 : 1), wW1(K, 0), wW2(K), wH(H > 1 ? H - 1 : 1);
    for (int k = 0; k < K; ++k)
        eF[k] = log2_scale(act_amax[k]);
    const int eO = log2_scale(act_amax[K]);
    for (int m = 0; m < H - 1; ++m)
        eH[m] = log2_scale(act_amax[K + 1 + m]);
    for (int k = 1; k < K; ++k)
        wW1[k] = log2_scale(tensor_amax(th, pb.W1[k], (int64_t)W * W));
    for (int k = 0; k < K; ++k)
        wW2[k] = log2_scale(tensor_amax(th, pb.W2[k], (int64_t)W * W));
    for (int m = 0; m < H - 1; ++m)
        wH[m] = log2_scale(tensor_amax(th, pb.hw[m], (int64_t)W * W));
    // Units: f_k <= eF_k, o <= eO, h_m <= eH_m (activations fit under 448), with every
    // matrix exponent (output unit - input unit) at most its range-filling one (weights
    // fit under 448): f_k - o <= wW1_k, o - f_k <= wW2_k, h_m - in_m <= wH_m.  Lowering
    // o only lowers the bounds, so the loop ends.
    // A bias that rides in its layer's last FP8 chunk (MT not a multiple of 8) is three
    // E4M3 parts behind inputs of 1, so it must fit under 448 in its output unit as well.
    const bool fold = MT % 8 != 0;
    int o = eO;
    if (fold) {
        double bm = 0.0;
        for (int k = 0; k < K; ++k)
            bm = fmax(bm, tensor_amax(th, pb.b2[k], W));
        if (bm > 0.0 && log2_scale(bm) < o)
            o = log2_scale(bm);
    }
    std::vector<int> f(K);
    for (int it = 0;; ++it) {
        bool again = false;
        for (int k = 0; k < K && !again; ++k) {
            f[k] = k > 0 && o + wW1[k] < eF[k] ? o + wW1[k] : eF[k];
            if (o - f[k] > wW2[k]) {
                o = f[k] + wW2[k];
                again = true;
            }
        }
        if (!again)
            break;
        if (it > 4 * K + 8) {
            set_error("ds_net_quantize: no consistent FP8 scales for this network");
            return DS_ERR_STATE;
        }
    }
    std::vector<int> h(H > 1 ? H - 1 : 1);
    for (int m = 0; m < H - 1; ++m) {
        const int in = m == 0 ? o : h[m - 1];
        h[m] = in + wH[m] < eH[m] ? in + wH[m] : eH[m];
        const double bm = fold ? tensor_amax(th, pb.hb[m], W) : 0.0;
        if (bm > 0.0 && log2_scale(bm) < h[m])
            h[m] = log2_scale(bm);
    }
    // exported: units, then matrix exponents
    std::vector<int32_t> ex;
    for (int k = 0; k < K; ++k)
        ex.push_back(f[k]);
    ex.push_back(o);
    for (int m = 0; m < H - 1; ++m)
        ex.push_back(h[m]);
    for (int k = 1; k < K; ++k)
        ex.push_back(f[k] - o);
    for (int k = 0; k < K; ++k)
        ex.push_back(o - f[k]);
    for (int m = 0; m < H - 1; ++m)
        ex.push_back(h[m] - (m == 0 ? o : h[m - 1]));
    if ((int)ex.size() != fp8_exp_count(K, H)) {
        set_error("internal error: FP8 scale count");
        return DS_ERR_STATE;
    }

    const int64_t slots = fp8_slot_count(MT, K, H);
    std::vector<uint4> fr((size_t)(slots * MT * 64 + kFragPad), uint4{0, 0, 0, 0});
    auto entry = [&](int64_t slot, int mt, int lane) -> uint8_t * {
        return reinterpret_cast<uint8_t *>(&fr[(size_t)((slot * MT + mt) * 64 + lane)]);
    };
    // One FP8 matrix [W][W] at offset off, scale 2^e, starting at `slot`; with boff >= 0
    // its bias (offset boff, in units 2^be) goes to the first free tile t = MT of the last
    // chunk, inputs 0..2 of lane group 0, as three E4M3 parts: each part encodes what the
    // parts before it left over (about 12 significant bits in all).
    auto put_fp8 = [&](int64_t slot, int64_t off, int e, int64_t boff = -1, int be = 0) {
        auto part = [&](int row, int i) -> uint8_t {
            double r = ldexp((double)th[boff + row], be);
            uint8_t c = 0;
            for (int q = 0; q <= i; ++q) {
                c = e4m3_encode((float)r);
                r -= e4m3_value(c);
            }
            return c;
        };
        for (int Q = 0; Q < C8; ++Q)
            for (int h = 0; h < 2; ++h)
                for (int mt = 0; mt < MT; ++mt)
                    for (int g = 0; g < 4; ++g)
                        for (int r = 0; r < 16; ++r) {
                            const int row = 16 * mt + r;
                            if (row >= W)
                                continue;
                            uint8_t *dst = entry(slot + 2 * Q + h, mt, 16 * g + r);
                            for (int bb = 0; bb < 16; ++bb) {
                                const int b = 16 * h + bb, t = 8 * Q + b / 4;
                                const int col = 16 * t + 4 * g + (b & 3);
                                dst[bb] = (t < MT && col < W)
                                              ? e4m3_encode((float)ldexp(
                                                    (double)th[off + (int64_t)row * W + col], e))
                                              : 0;
                                if (boff >= 0 && t == MT && g == 0 && (b & 3) < 3)
                                    dst[bb] = part(row, b & 3);
                            }
                        }
    };
    int64_t slot = 0;
    for (int k = 0; k < K; ++k) {
        for (int c = 0; c < 8; ++c, ++slot)
            for (int mt = 0; mt < MT; ++mt)
                for (int g = 0; g < 4; ++g)
                    for (int r = 0; r < 16; ++r) {
                        const int row = 16 * mt + r;
                        if (row >= W)
                            continue;
                        uint16_t *dst = reinterpret_cast<uint16_t *>(entry(slot, mt, 16 * g + r));
                        for (int j = 0; j < 8; ++j) {
                            int col = -1;
                            if (c < 7)
                                col = stencil_slot(c, g, j);
                            else if (g == 0 && j < 2)
                                col = 224 + j;  // sample (4, 4, 8), gamma
                            if (c == 7 && g == 1 && j < 2) {  // b1 in block k's units: high, low
                                const float b = (float)ldexp((double)th[pb.b1[k] + row], f[k]);
                                const uint16_t hi = bf16_rne(b);
                                dst[j] = j == 0 ? hi
                                                : bf16_rne(b - __builtin_bit_cast(
                                                                   float, (uint32_t)hi << 16));
                                continue;
                            }
                            dst[j] = col < 0 ? 0
                                             : bf16_rne((float)ldexp(
                                                   (double)th[pb.V[k] + (int64_t)row * 226 + col],
                                                   f[k]));
                        }
                    }
        if (k > 0) {
            put_fp8(slot, pb.W1[k], f[k] - o);
            slot += 2 * C8;
        }
        put_fp8(slot, pb.W2[k], o - f[k], fold ? pb.b2[k] : -1, o);
        slot += 2 * C8;
    }
    for (int m = 0; m < H - 1; ++m) {
        put_fp8(slot, pb.hw[m], h[m] - (m == 0 ? o : h[m - 1]), fold ? pb.hb[m] : -1, h[m]);
        slot += 2 * C8;
    }
    if (slot != slots) {
        set_error("internal error: FP8 packing produced %lld slots, expected %lld",
                  (long long)slot, (long long)slots);
        return DS_ERR_STATE;
    }

    // vectors in the same layout as the BF16 form's, in the FP8 form's units
    const int64_t nvec = (int64_t)K * 2 * WP + (int64_t)(H - 1) * WP + WP + 4;
    std::vector<float> vec((size_t)nvec, 0.f);
    for (int k = 0; k < K; ++k)
        for (int r = 0; r < W; ++r) {
            vec[(size_t)k * 2 * WP + r] = (float)ldexp((double)th[pb.b1[k] + r], f[k]);
            vec[(size_t)k * 2 * WP + WP + r] = (float)ldexp((double)th[pb.b2[k] + r], o);
        }
    for (int m = 0; m < H - 1; ++m)
        for (int r = 0; r < W; ++r)
            vec[(size_t)K * 2 * WP + (size_t)m * WP + r] =
                (float)ldexp((double)th[pb.hb[m] + r], h[m]);
    const size_t wl = (size_t)K * 2 * WP + (size_t)(H - 1) * WP;
    const int e_last = H >= 2 ? h[H - 2] : o;  // units of the final layer's input
    for (int c = 0; c < W; ++c)
        vec[wl + c] = (float)ldexp((double)th[pb.hw[H - 1] + c], -e_last);
    vec[wl + WP] = th[pb.hb[H - 1]];

    if (!net->frag_fp8) {
        DS_CHECK(hipMalloc(&net->frag_fp8, fr.size() * sizeof(uint4)) == hipSuccess, DS_ERR_OOM,
                 "out of device memory for the FP8 weights");
        DS_CHECK(hipMalloc(&net->vec8, vec.size() * sizeof(float)) == hipSuccess, DS_ERR_OOM,
                 "out of device memory for the FP8 vectors");
        net->frag8_count = (int64_t)fr.size();
    }
    DS_HIP(hipMemcpy(net->frag_fp8, fr.data(), fr.size() * sizeof(uint4), hipMemcpyHostToDevice));
    DS_HIP(hipMemcpy(net->vec8, vec.data(), vec.size() * sizeof(float), hipMemcpyHostToDevice));
    net->fp8_exps = ex;
    net->fp8_ready = true;
    return DS_OK;
}

ds_status fused_gather_packed(hipStream_t s, const FusedArgs &a, float *z)
{
    int64_t blocks = (a.cl[0].P + 63) / 64;
    if (blocks <= 0)
        return DS_OK;
    k_gather_packed<<<(unsigned)blocks, 256, 0, s>>>(a, z);
    DS_HIP(hipGetLastError());
    return DS_OK;
}

// two-team kernel: eight waves, a ring of ten chunks below 16 tiles, a chunk stream of
// even length per tile
static bool teams_ok(const ds_net *net, const FusedVariant &v, bool fp8)
{
    const int MT = fused_tiles(net->W);
    if (v.waves != 8 || v.grid < 0 || MT < 1 || MT >= 16)
        return false;
    const int nc = fp8 ? fp8_slot_count(MT, net->K, net->H) : chunk_count(MT, net->K, net->H);
    return nc % 2 == 0;
}

bool fused_variant_ok(const ds_net *net, const FusedVariant &v)
{
    if (v.kind == DS_KERNEL_TEAMS)
        return teams_ok(net, v, false);
    if (v.kind != DS_KERNEL_REGISTER && v.kind != DS_KERNEL_PIPELINED && v.kind != DS_KERNEL_WIDE)
        return false;
    if (v.waves != 4 && v.waves != 8)
        return false;
    if (!fits(fused_tiles(net->W), v.waves, v.kind))
        return false;
    return v.grid >= 0;
}

bool fused_variant_ok_fp8(const ds_net *net, const FusedVariant &v)
{
    if (v.kind == DS_KERNEL_TEAMS)
        return teams_ok(net, v, true);
    return v.kind == DS_KERNEL_REGISTER && fused_variant_ok(net, v);
}

ds_status fused_predict(hipStream_t s, const ds_net *net, const FusedArgs &a,
                        const FusedVariant &v, ds_precision precision)
{
    DS_CHECK(a.n_clouds >= 1 && a.n_clouds <= kMaxBatch, DS_ERR_INVALID_ARG,
             "between 1 and %d clouds per launch", kMaxBatch);
    DS_CHECK(precision == DS_PREC_BF16 || precision == DS_PREC_FP8, DS_ERR_INVALID_ARG,
             "fused prediction: precision %d", (int)precision);
    const bool fp8 = precision == DS_PREC_FP8;
    if (fp8) {
        DS_CHECK(net->fp8_ready, DS_ERR_STATE,
                 "FP8 weights are not available: quantize the network (ds_net_quantize) after "
                 "its parameters were last set");
        DS_CHECK(fused_variant_ok_fp8(net, v), DS_ERR_UNSUPPORTED,
                 "kernel variant (kind %d, %d waves, grid %d) has no FP8 form at width %d", v.kind,
                 v.waves, v.grid, net->W);
    } else {
        DS_CHECK(net->frag_bf16, DS_ERR_STATE, "network parameters were never set");
        DS_CHECK(fused_variant_ok(net, v), DS_ERR_INVALID_ARG,
                 "kernel variant (kind %d, %d waves, grid %d) is not available at width %d",
                 v.kind, v.waves, v.grid, net->W);
    }
    switch (fused_tiles(net->W)) {
    case 1: return launch<1>(s, net, a, v, fp8);
    case 2: return launch<2>(s, net, a, v, fp8);
    case 4: return launch<4>(s, net, a, v, fp8);
    case 8: return launch<8>(s, net, a, v, fp8);
    case 13: return launch<13>(s, net, a, v, fp8);
    case 16: return launch<16>(s, net, a, v, fp8);
    default:
        set_error("width %d is not supported by the fused kernel", net->W);
        return DS_ERR_UNSUPPORTED;
    }
}

}  // namespace ds
