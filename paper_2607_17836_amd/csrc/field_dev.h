// Device-side building blocks shared by the step kernels (step.hip) and the
// adjoint kernels (adjoint.hip): block order, periodic cell arithmetic, the
// interpolation kernels of Sec. 3.4, the LDS field tiles and the FP64
// velocity evaluation.  Internal to liblpt.so.
#pragma once

#include "lpt_kernels.h"

#include <math.h>

namespace lpt {

constexpr int kMaxBlock = 512;
constexpr int kWave = 64;
constexpr float kCellClampF = 1073741824.0f;   // 2^30 cells
constexpr double kCellClampD = 1073741824.0;

// ---------------------------------------------------------------------------
// Block order.  The hardware deals consecutive workgroups round-robin over the
// 8 XCDs of the chip; remap so that XCD x processes one contiguous run of
// logical blocks (neighbouring cells after the cell sort) and its private L2
// sees their shared stencil rows.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int xcd_logical_block(int b, int G)
{
    constexpr int X = 8;
    const int x = b % X, k = b / X;
    const int q = G / X, r = G % X;
    return x < r ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

// Persistent launches: XCD x (= blockIdx.x mod X, X = min(8, grid)) owns the
// contiguous logical blocks [x T / X, (x + 1) T / X) and its workgroups
// stride through them.  Every workgroup's range ends, so the grid always
// drains, and every logical block has exactly one owner.
__device__ __forceinline__ void persistent_range(int T, int &first, int &stride, int &end)
{
    const int G = gridDim.x, b = blockIdx.x;
    const int X = G < 8 ? G : 8;
    const int x = b % X, k = b / X;
    const int gx = (G - x + X - 1) / X;   // workgroups on XCD x
    const int lo = (int)((int64_t)T * x / X), hi = (int)((int64_t)T * (x + 1) / X);
    first = lo + k;
    stride = gx;
    end = hi;
}

// Walk over the logical blocks of a launch over [base, base + count): each
// block is visited by exactly one workgroup, and the walk is uniform per
// workgroup (it depends on blockIdx alone), so block bodies may synchronise.
//   - with a block-order table (P.order), XCD x = blockIdx mod 8 walks its
//     list with a stride of its own workgroup count (one entry each when
//     the grid is 8 * order_len), skipping the -1 padding;
//   - otherwise one block per workgroup in XCD-contiguous order, or, in a
//     persistent launch, the XCD's contiguous range.
// Every workgroup's walk ends, so the grid always drains.  (A plain iterator
// rather than a callback: the kernel parameters stay in the kernel-argument
// segment instead of being copied to private memory for a closure.)
struct BlockWalk {
    const int32_t *list;   // this XCD's table list, or null
    int k, stride, end;
};

__device__ __forceinline__ BlockWalk block_walk(const StepParams &P, int base, int count)
{
    BlockWalk w;
    if (P.order) {
        constexpr int X = 8;
        const int G = gridDim.x, b = blockIdx.x, x = b % X;
        w.list = P.order + (int64_t)x * P.order_len;
        w.k = b / X;
        w.stride = (G - x + X - 1) / X;   // workgroups on XCD x
        w.end = P.order_len;
    } else if (!P.persistent) {
        w.list = nullptr;
        w.k = base + xcd_logical_block(blockIdx.x, gridDim.x);
        w.stride = 1;
        w.end = w.k + 1;
    } else {
        int first, stride, end;
        persistent_range(count, first, stride, end);
        w.list = nullptr;
        w.k = base + first;
        w.stride = stride;
        w.end = base + end;
    }
    return w;
}

// The next logical block of the walk into lb; false once it is done.
__device__ __forceinline__ bool block_next(BlockWalk &w, int &lb)
{
    while (w.k < w.end) {
        const int v = w.list ? w.list[w.k] : w.k;
        w.k += w.stride;
        if (v >= 0) {
            lb = v;
            return true;
        }
    }
    return false;
}

// Streaming (non-temporal) loads and stores of the particle state: each
// value is touched once per step, so it should not displace the field's node
// records from the caches.
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t ld_stream(const uint32_t *p)
{
    return __builtin_nontemporal_load(p);
}
__device__ __forceinline__ float2 ld_stream(const float2 *p)
{
    const f32x2 v = __builtin_nontemporal_load(reinterpret_cast<const f32x2 *>(p));
    return make_float2(v.x, v.y);
}
__device__ __forceinline__ double2 ld_stream(const double2 *p)
{
    const f64x2 v = __builtin_nontemporal_load(reinterpret_cast<const f64x2 *>(p));
    return make_double2(v.x, v.y);
}
__device__ __forceinline__ int2 ld_stream(const int2 *p)
{
    typedef int i32x2 __attribute__((ext_vector_type(2)));
    const i32x2 v = __builtin_nontemporal_load(reinterpret_cast<const i32x2 *>(p));
    return make_int2(v.x, v.y);
}
__device__ __forceinline__ void st_stream(uint32_t *p, uint32_t v) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void st_stream(int2 *p, int2 v)
{
    typedef int i32x2 __attribute__((ext_vector_type(2)));
    i32x2 w = {v.x, v.y};
    __builtin_nontemporal_store(w, reinterpret_cast<i32x2 *>(p));
}
__device__ __forceinline__ void st_stream(float2 *p, float2 v)
{
    f32x2 w = {v.x, v.y};
    __builtin_nontemporal_store(w, reinterpret_cast<f32x2 *>(p));
}
__device__ __forceinline__ void st_stream(double2 *p, double2 v)
{
    f64x2 w = {v.x, v.y};
    __builtin_nontemporal_store(w, reinterpret_cast<f64x2 *>(p));
}

__device__ __forceinline__ int species_of(const StepParams &P, int lb)
{
    int s = 0;
    for (int k = 1; k < P.nspecies; ++k)
        if (lb >= P.sp[k].block_begin && lb < P.sp[k].block_end) s = k;
    return s;
}

// ---------------------------------------------------------------------------
// Periodic cell index.  Cell coordinates are clamped to +-2^30 before the
// integer conversion (one v_med3), so that any input -- NaN and absurd
// displacements included -- yields an index inside [0, n) and no gather can
// leave the field; within +-2^30 cells the mapping is the exact periodic one.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int wrap_cell(int c, int n, int mask)
{
    if (mask >= 0) return c & mask;
    if (c < 0) c += n;
    if (c >= n) c -= n;
    if ((unsigned)c >= (unsigned)n) {
        c %= n;
        if (c < 0) c += n;
    }
    return c;
}

__device__ __forceinline__ int cell_plus(int c, float fl, int n, int mask)
{
    const float f = __builtin_amdgcn_fmed3f(fl, -kCellClampF, kCellClampF);
    return wrap_cell(c + (int)f, n, mask);
}

__device__ __forceinline__ int cell_of_floor(double fl, int n, int mask)
{
    double f = fmin(fmax(fl, -kCellClampD), kCellClampD);
    if (!(f == f)) f = 0.0;
    return wrap_cell((int)f, n, mask);
}

// Catmull-Rom kernel (eq. cr_kernel) and cubic B-spline kernel
// (eq. bspline_kernel), evaluated in Horner form.
template <typename T>
__device__ __forceinline__ void weights_cr(T s, T w[4])
{
    w[0] = s * (T(-0.5) + s * (T(1.0) + s * T(-0.5)));
    w[1] = T(1.0) + s * s * (T(-2.5) + s * T(1.5));
    w[2] = s * (T(0.5) + s * (T(2.0) + s * T(-1.5)));
    w[3] = s * s * (T(-0.5) + s * T(0.5));
}

template <typename T>
__device__ __forceinline__ void weights_bs(T s, T w[4])
{
    const T r = T(1.0) - s;
    const T sixth = T(1.0) / T(6.0);
    w[0] = r * r * r * sixth;
    w[1] = (T(4.0) + s * s * (T(-6.0) + s * T(3.0))) * sixth;
    w[2] = (T(1.0) + s * (T(3.0) + s * (T(3.0) + s * T(-3.0)))) * sixth;
    w[3] = s * s * s * sixth;
}

template <typename T>
__device__ __forceinline__ void bilinear_weights(T xi, T eta, T &w00, T &w10, T &w01, T &w11)
{
    w11 = xi * eta;
    w10 = xi - w11;            // xi (1 - eta)
    w01 = eta - w11;           // (1 - xi) eta
    w00 = (T(1.0) - xi) - w01; // (1 - xi)(1 - eta)
}

__device__ __forceinline__ bool edge_cell(int compat, int i, int j, int n)
{
    return compat && (i == 0 || i >= n - 2 || j == 0 || j >= n - 2);
}

// ===========================================================================
// LDS field tiles.  After the cell-order sort, the particles of one block sit
// in a compact patch of cells.  The block finds the bounding box of its
// particles' stored cells, widens it by a halo that covers every RK4 stage
// position (the largest displacement a step can make, from the largest node
// speed of the two time levels) plus the interpolation stencil, and copies
// the node records of that box into LDS with coalesced loads.  The four
// stages then gather from LDS.  Every gather checks that its whole stencil
// lies inside the tile and otherwise reads global memory, so the halo is a
// performance estimate, never a correctness assumption.
// ===========================================================================
struct Tile {
    int x0, y0;   // global node index of tile entry (0, 0)
    int w, h;     // tile extent in nodes
    int on;       // block-uniform: the tile is staged
};

__device__ __forceinline__ Tile no_tile() { return Tile{0, 0, 0, 0, 0}; }

// Tile index of stencil origin node (i0, j0) if the span x span stencil that
// starts there lies inside the tile.
__device__ __forceinline__ bool tile_index(const Tile &T, int i0, int j0, int span, int n,
                                           int mask, int &idx)
{
    const int rx = wrap_cell(i0 - T.x0, n, mask), ry = wrap_cell(j0 - T.y0, n, mask);
    idx = ry * T.w + rx;
    return T.on && rx <= T.w - span && ry <= T.h - span;
}

extern __shared__ __align__(32) unsigned char lpt_dyn_lds[];

// Halo in cells for one step of size dt: the largest stage displacement
// (velocity bound times dt, rounded up) -- Catmull-Rom can overshoot the node
// values by up to (1 + 1/4)^2 because its weights have |W| summing to
// 1 + s(1 - s) per axis; bilinear and B-spline weights are convex.
__device__ __forceinline__ int step_halo(const StepParams &P, int scheme, float dt)
{
    const float um = fmaxf(P.umax[0], P.umax[1]);   // cells per unit time
    const float cs = scheme == kCatmullRom ? 1.5625f : 1.0f;
    const float d = fminf(P.halo_scale * cs * um * dt, 16.0f);
    return d > 0.0f ? (int)ceilf(d) : 0;
}

// Wave-wide maximum of two packed unsigned 16-bit lanes by DPP: four row
// shifts reduce each 16-lane row, two row broadcasts combine the rows, and
// lane 63 ends with the result.  Lanes outside a shift read 0, the identity.
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t pmax16(uint32_t a, uint32_t b)
{
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(u16x2, a),
                                                                  __builtin_bit_cast(u16x2, b)));
}

template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp_pmax(uint32_t x)
{
    return pmax16(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, ROWS, 0xF, true));
}

__device__ __forceinline__ uint32_t wave_pmax16(uint32_t x)
{
    x = dpp_pmax<0x111, 0xF>(x);   // row_shr:1
    x = dpp_pmax<0x112, 0xF>(x);   // row_shr:2
    x = dpp_pmax<0x114, 0xF>(x);   // row_shr:4
    x = dpp_pmax<0x118, 0xF>(x);   // row_shr:8
    x = dpp_pmax<0x142, 0xA>(x);   // row_bcast:15
    x = dpp_pmax<0x143, 0xC>(x);   // row_bcast:31
    return (uint32_t)__builtin_amdgcn_readlane((int)x, 63);
}

// The same DPP pattern for a binary64 sum: each shift moves the two 32-bit
// halves, lanes outside a shift read 0 (the identity), and lane 63 ends with
// the sum of all 64 lanes, added in a fixed order (an inclusive scan of each
// 16-lane row, then the row totals), so the result does not depend on
// scheduling.  Every lane of the wave must be active.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_f64(double x)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, x);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, ROWS, 0xF, true);
    const uint32_t hi =
        (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, ROWS, 0xF, true);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Exchanges of 64-bit lane values between lane groups (gfx950 permlane
// swaps, one per 32-bit half).  swap32: x takes [x lanes 0-31 | y lanes
// 0-31], y takes [x lanes 32-63 | y lanes 32-63].  swap16, per 16-lane row r:
// x takes [x r0 | y r0 | x r2 | y r2], y takes [x r1 | y r1 | x r3 | y r3].
__device__ __forceinline__ void swap32_f64(double &x, double &y)
{
    const uint64_t bx = __builtin_bit_cast(uint64_t, x), by = __builtin_bit_cast(uint64_t, y);
    const auto lo = __builtin_amdgcn_permlane32_swap((uint32_t)bx, (uint32_t)by, false, false);
    const auto hi =
        __builtin_amdgcn_permlane32_swap((uint32_t)(bx >> 32), (uint32_t)(by >> 32), false, false);
    x = __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi[0] << 32) | (uint32_t)lo[0]);
    y = __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi[1] << 32) | (uint32_t)lo[1]);
}

__device__ __forceinline__ void swap16_f64(double &x, double &y)
{
    const uint64_t bx = __builtin_bit_cast(uint64_t, x), by = __builtin_bit_cast(uint64_t, y);
    const auto lo = __builtin_amdgcn_permlane16_swap((uint32_t)bx, (uint32_t)by, false, false);
    const auto hi =
        __builtin_amdgcn_permlane16_swap((uint32_t)(bx >> 32), (uint32_t)(by >> 32), false, false);
    x = __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi[0] << 32) | (uint32_t)lo[0]);
    y = __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi[1] << 32) | (uint32_t)lo[1]);
}

// Statistics partial of one wave (Sec. 3.2 and 5.5 quantities): the sums of
// dx^2 and dy^2 over its active lanes, and the sums of d and d^2 for
// d = r2 - K, r2 = dx^2 + dy^2, with K the r2 of the wave's first active
// lane.  The finalisation forms the wave's M2 = sum d^2 - (sum d)^2 / count,
// the sum of squared deviations of r2 about the wave's mean: shifted by a
// sample of the wave, it keeps its accuracy where the spread of r2 is small
// against its mean (uniform flow: every d is zero), unlike
// (sum r2^2 - N m^2) / (N - 1).  The four sums are reduced together: two
// swap-and-add levels leave one quantity per 16-lane row, a row reduction
// finishes them, and the last lane of each row stores its sum, so out
// receives (sum dx^2, sum dy^2, sum d, sum d^2).  Every lane of the wave must
// call it (inactive lanes with r2x = r2y = 0).
__device__ __forceinline__ void wave_stats(double r2x, double r2y, bool active, double *out)
{
    const uint64_t live = __ballot(active);
    const int first = live ? __builtin_ctzll(live) : 0;
    const double r2 = r2x + r2y;
    const uint64_t br = __builtin_bit_cast(uint64_t, r2);
    const uint32_t klo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)br, first);
    const uint32_t khi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(br >> 32), first);
    const double K = __builtin_bit_cast(double, ((uint64_t)khi << 32) | klo);
    const double d = active ? r2 - K : 0.0;
    double a = r2x, b = r2y, c = d, e = d * d;
    swap32_f64(a, b);
    swap32_f64(c, e);
    double x = a + b;   // lanes 0-31: sum dx^2 halves, lanes 32-63: sum dy^2 halves
    double y = c + e;   // likewise sum d, sum d^2
    swap16_f64(x, y);
    double z = x + y;   // rows: sum dx^2, sum d, sum dy^2, sum d^2 over 16 lanes each
    z += dpp_f64<0x111, 0xF>(z);   // row_shr:1
    z += dpp_f64<0x112, 0xF>(z);   // row_shr:2
    z += dpp_f64<0x114, 0xF>(z);   // row_shr:4
    z += dpp_f64<0x118, 0xF>(z);   // row_shr:8
    const int lane = (int)(threadIdx.x & (kWave - 1));
    if ((lane & 15) == 15) {
        const int row = lane >> 4;
        out[(row & 1) * 2 + (row >> 1)] = z;   // rows 0, 1, 2, 3 -> out[0], out[2], out[1], out[3]
    }
}

// Bounding box of the stored cells of a block's active particles, widened by
// lo cells before and hi cells after on each axis.  The box is reduced on
// offsets from (ax, ay), the cell of the block's first particle (which is
// always active), biased by 2^15 and packed two per word, as maxima of
// (r + 2^15) and (2^15 - r).  A thread first folds its own particles into a
// BoxAcc (box_add), then block_box_reduce combines the block's threads (all
// threads must call it; it returns with the block synchronised) and fills
// x0, y0, w, h of the result; `on` is left 0.
struct BoxAcc {
    uint32_t up, dn;
};

constexpr int kBoxBias = 1 << 15;

// The anchor's own offset (0, 0), which every box holds.
__device__ __forceinline__ BoxAcc box_init()
{
    constexpr uint32_t z = (uint32_t)kBoxBias | ((uint32_t)kBoxBias << 16);
    return BoxAcc{z, z};
}

// The box terms of the single cell (cx, cy).
__device__ __forceinline__ BoxAcc box_of(int cx, int cy, int ax, int ay, int n)
{
    const int half = n >> 1;
    int rx = cx - ax, ry = cy - ay;   // in (-n, n): map it to (-n/2, n/2]
    rx += rx < -half ? n : (rx > half ? -n : 0);
    ry += ry < -half ? n : (ry > half ? -n : 0);
    return BoxAcc{(uint32_t)(rx + kBoxBias) | ((uint32_t)(ry + kBoxBias) << 16),
                  (uint32_t)(kBoxBias - rx) | ((uint32_t)(kBoxBias - ry) << 16)};
}

__device__ __forceinline__ void box_add(BoxAcc &b, int cx, int cy, int ax, int ay, int n)
{
    const BoxAcc c = box_of(cx, cy, ax, ay, n);
    b.up = pmax16(b.up, c.up);
    b.dn = pmax16(b.dn, c.dn);
}

__device__ __forceinline__ Tile block_box_reduce(BoxAcc b, int ax, int ay, int n, int mask,
                                                 int lo, int hi)
{
    __shared__ uint32_t red[2][kMaxBlock / kWave];
    uint32_t up = wave_pmax16(b.up);
    uint32_t dn = wave_pmax16(b.dn);
    const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave, nw = blockDim.x / kWave;
    if (lane == 0) {
        red[0][wv] = up;
        red[1][wv] = dn;
    }
    __syncthreads();
    up = red[0][0];
    dn = red[1][0];
    for (int k = 1; k < nw; ++k) {
        up = pmax16(up, red[0][k]);
        dn = pmax16(dn, red[1][k]);
    }
    const int mxx = (int)(up & 0xFFFFu) - kBoxBias, mxy = (int)(up >> 16) - kBoxBias;
    const int mnx = kBoxBias - (int)(dn & 0xFFFFu), mny = kBoxBias - (int)(dn >> 16);
    Tile T = no_tile();
    T.w = mxx - mnx + 1 + lo + hi;
    T.h = mxy - mny + 1 + lo + hi;
    T.x0 = wrap_cell(ax + mnx - lo, n, mask);
    T.y0 = wrap_cell(ay + mny - lo, n, mask);
    return T;
}

// The box of one particle per thread: (cx, cy) is the thread's cell
// (ignored when !active).
__device__ __forceinline__ Tile block_box(bool active, int cx, int cy, int ax, int ay, int n,
                                          int mask, int lo, int hi)
{
    return block_box_reduce(active ? box_of(cx, cy, ax, ay, n) : box_init(), ax, ay, n, mask, lo,
                            hi);
}

// Tile fill by LDS DMA: the tile's flat index space is cut into chunks of 64
// entries; a wave takes every nw-th chunk, and lane l of chunk c loads the
// record of entry 64 c + l straight into LDS in 16-byte pieces (the wave's
// LDS destination is the chunk's first entry; lane l lands 16 l bytes after
// it), so the records never pass through registers.  A lane's tile column
// and row are divided out once per tile; from one of its chunks to the next
// its entry moves by 64 nw, a fixed number of rows and columns, so they are
// carried forward with one compare per chunk.  An FP32 record is one piece
// (one plane of records); an FP64 record is two, level 0 and level 1, into
// two planes `area` entries apart.  Lanes past the tile's area are switched
// off.  Ends with every wave's loads complete.
template <typename Rec>
__device__ __forceinline__ void fill_tile_dma(Rec *lds_rec, const Rec *__restrict__ rec0,
                                              const StepParams &P, const Tile &T)
{
    constexpr int kPieces = (int)sizeof(Rec) / 16;
    float4 *lds = reinterpret_cast<float4 *>(lds_rec);
    if (!T.on) return;
    const int n = P.n;
    const int w = __builtin_amdgcn_readfirstlane(T.w), h = __builtin_amdgcn_readfirstlane(T.h);
    const int x0 = __builtin_amdgcn_readfirstlane(T.x0);
    const int y0 = __builtin_amdgcn_readfirstlane(T.y0);
    const int area = w * h;
    const int lane = (int)threadIdx.x & (kWave - 1);
    const int wv = __builtin_amdgcn_readfirstlane((int)threadIdx.x / kWave);
    const int nw = (int)blockDim.x / kWave;
    const int chunks = (area + kWave - 1) / kWave;
    const int step = nw * kWave;                     // entries between a wave's chunks
    const int sy = step / w, sx = step - sy * w;     // ... as rows and columns
    int k = wv * kWave + lane;
    int ty = k / w, tx = k - ty * w;
    for (int c = wv; c < chunks; c += nw) {
        if (k < area) {
            int gx = x0 + tx, gy = y0 + ty;   // below 2 n: x0, y0 < n, tx < w < n, ty < h < n
            gx -= gx >= n ? n : 0;
            gy -= gy >= n ? n : 0;
            const float4 *src =
                reinterpret_cast<const float4 *>(rec0 + (__mul24(gy, P.pitch) + gx));
#pragma unroll
            for (int piece = 0; piece < kPieces; ++piece)
                __builtin_amdgcn_global_load_lds(
                    (const void *)(src + piece),
                    (void __attribute__((address_space(3))) *)(lds + piece * area + c * kWave), 16,
                    0, 0);
        }
        k += step;
        tx += sx;
        ty += sy;
        if (tx >= w) {
            tx -= w;
            ty += 1;
        }
    }
    __builtin_amdgcn_s_waitcnt(0);
}

// Cooperative tile set-up of one block (all threads must call it): the box
// of the block's particles (folded into b by each thread, see box_add),
// staged in LDS if it fits the capacity and is not much larger than the
// block's particle count.
template <typename Rec>
__device__ __forceinline__ Tile stage_tile_acc(Rec *lds, const Rec *__restrict__ rec0,
                                              const StepParams &P, BoxAcc b, int ax, int ay,
                                              int lo, int hi, int nactive)
{
    const int n = P.n;
    Tile T = block_box_reduce(b, ax, ay, n, P.mask, lo, hi);
    // A box beyond the capacity (a block whose particles have spread since
    // the last re-sort) is cut down about its centre to a window of the same
    // shape that fits: the stencils inside it still read LDS, the others
    // global memory, instead of the whole block losing its tile.  A window
    // narrower than the widest stencil (4 nodes) is not staged, so every
    // tile holds at least one whole stencil along each axis.
    bool fits = true;
    if (P.tile_cap > 0 && T.w * T.h > P.tile_cap && T.w < n && T.h < n) {
        const float f = sqrtf((float)P.tile_cap / (float)(T.w * T.h));
        const int w = max(1, (int)((float)T.w * f));
        const int h = min(T.h, P.tile_cap / w);
        T.x0 = wrap_cell(T.x0 + (T.w - w) / 2, n, P.mask);
        T.y0 = wrap_cell(T.y0 + (T.h - h) / 2, n, P.mask);
        T.w = w;
        T.h = h;
        fits = w >= 4 && h >= 4;
    }
    const int area = T.w * T.h;
    T.on = fits && P.tile_cap > 0 && area <= P.tile_cap && T.w < n && T.h < n &&
           area <= kTileWaste * nactive;
    fill_tile_dma<Rec>(lds, rec0, P, T);
    __syncthreads();
    return T;
}

template <typename Rec>
__device__ __forceinline__ Tile stage_tile(Rec *lds, const Rec *__restrict__ rec0,
                                          const StepParams &P, bool active, int cx, int cy,
                                          int ax, int ay, int lo, int hi, int nactive)
{
    return stage_tile_acc<Rec>(lds, rec0, P, active ? box_of(cx, cy, ax, ay, P.n) : box_init(), ax,
                               ay, lo, hi, nactive);
}

// Halo extents of a scheme: a bilinear stencil spans nodes i..i+1, a bicubic
// one i-1..i+2 (the compatibility fallback to bilinear stays inside both).
__device__ __forceinline__ void stencil_reach(int scheme, int &lo, int &hi)
{
    lo = scheme == kBilinear ? 0 : 1;
    hi = scheme == kBilinear ? 1 : 2;
}

// ===========================================================================
// FP64 path (physical units)
// ===========================================================================
// Time-blended (u, v) of one node from its two levels (level 0 at q0, level 1
// at q1; only the ones smode needs are read).
__device__ __forceinline__ void blend64(const double2 *q0, const double2 *q1, int smode,
                                        double wa, double wb, double &u, double &v)
{
    if (smode == kSlot0) {
        const double2 a = *q0;
        u = a.x;
        v = a.y;
    } else if (smode == kSlot1) {
        const double2 b = *q1;
        u = b.x;
        v = b.y;
    } else {
        const double2 a = *q0, b = *q1;
        u = wa * a.x + wb * b.x;
        v = wa * a.y + wb * b.y;
    }
}

// Time-blended (u, v) of one node record.
__device__ __forceinline__ void node64(const Rec64 *r, int smode, double wa, double wb, double &u,
                                       double &v)
{
    const double2 *q = reinterpret_cast<const double2 *>(r);
    blend64(q, q + 1, smode, wa, wb, u, v);
}

// Stencil nodes in global memory: whole records, node (a, b) at p + b pitch + a.
struct RecNodes64 {
    const Rec64 *p;
    int pitch;
    __device__ __forceinline__ void get(int a, int b, int smode, double wa, double wb, double &u,
                                        double &v) const
    {
        node64(p + (b * pitch + a), smode, wa, wb, u, v);
    }
};

// Stencil nodes in the LDS tile: two planes of (u, v), level 0 then level 1,
// `area` entries apart; node (a, b) at entry b pitch + a from p.
struct TileNodes64 {
    const double2 *p;
    int pitch, area;
    __device__ __forceinline__ void get(int a, int b, int smode, double wa, double wb, double &u,
                                        double &v) const
    {
        const double2 *q = p + (b * pitch + a);
        blend64(q, q + area, smode, wa, wb, u, v);
    }
};

// eq. bilinear_interp on nodes (0, 0), (1, 0), (0, 1), (1, 1) of N.
template <typename Nodes>
__device__ __forceinline__ void bil64(const Nodes &N, double xi, double eta, int smode,
                                      double wa, double wb, double &u, double &v)
{
    double u00, v00, u10, v10, u01, v01, u11, v11;
    N.get(0, 0, smode, wa, wb, u00, v00);
    N.get(1, 0, smode, wa, wb, u10, v10);
    N.get(0, 1, smode, wa, wb, u01, v01);
    N.get(1, 1, smode, wa, wb, u11, v11);
    double w00, w10, w01, w11;
    bilinear_weights(xi, eta, w00, w10, w01, w11);
    u = w00 * u00 + w10 * u10 + w01 * u01 + w11 * u11;
    v = w00 * v00 + w10 * v10 + w01 * v01 + w11 * v11;
}

// eqs. cr_interp / bspline_interp on the 4x4 nodes of N (node (0, 0) is grid
// node (i - 1, j - 1)).
template <typename Nodes>
__device__ __forceinline__ void cub64(const Nodes &N, const double wx[4], const double wy[4],
                                      int smode, double wa, double wb, double &u, double &v)
{
    double au = 0.0, av = 0.0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        double ru = 0.0, rv = 0.0;
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            double nu, nv;
            N.get(a, b, smode, wa, wb, nu, nv);
            ru += wx[a] * nu;
            rv += wx[a] * nv;
        }
        au += wy[b] * ru;
        av += wy[b] * rv;
    }
    u = au;
    v = av;
}

// Velocity at (x, y) (physical units, any real value) with temporal weights
// (wa, wb) on the two snapshot slots.  rec0 points at global node (0, 0);
// tile/T is the block's LDS tile, two planes (T.on == 0: global only).
template <bool CUBIC>
__device__ __forceinline__ void vel64(const Rec64 *__restrict__ rec0, const double2 *tile,
                                      const Tile &T, const StepParams &P, int scheme, double x,
                                      double y, double wa, double wb, int smode, double &u,
                                      double &v)
{
    const double sx = x * P.invh, sy = y * P.invh;
    const double fx = floor(sx), fy = floor(sy);
    const double xi = sx - fx, eta = sy - fy;
    const int n = P.n, mask = P.mask;
    const int i = cell_of_floor(fx, n, mask), j = cell_of_floor(fy, n, mask);
    int t;
    if (!CUBIC || scheme == kBilinear || edge_cell(P.compat_edge, i, j, n)) {
        if (tile_index(T, i, j, 2, n, mask, t))
            bil64(TileNodes64{tile + t, T.w, T.w * T.h}, xi, eta, smode, wa, wb, u, v);
        else
            bil64(RecNodes64{rec0 + (__mul24(j, P.pitch) + i), P.pitch}, xi, eta, smode, wa, wb,
                  u, v);
        return;
    }
    if constexpr (CUBIC) {
        double wx[4], wy[4];
        if (scheme == kCatmullRom) {
            weights_cr(xi, wx);
            weights_cr(eta, wy);
        } else {
            weights_bs(xi, wx);
            weights_bs(eta, wy);
        }
        if (tile_index(T, i - 1, j - 1, 4, n, mask, t))
            cub64(TileNodes64{tile + t, T.w, T.w * T.h}, wx, wy, smode, wa, wb, u, v);
        else
            cub64(RecNodes64{rec0 + (__mul24(j - 1, P.pitch) + (i - 1)), P.pitch}, wx, wy, smode,
                  wa, wb, u, v);
    }
}

__device__ __forceinline__ double wrap_pos(double z, double L)
{
    if (z >= L) z -= L;
    else if (z < 0.0) z += L;
    if (!(z >= 0.0 && z < L)) {
        if (z == z) {   // finite but far away, or +L after rounding
            z = z - L * floor(z / L);
            if (z < 0.0) z += L;
            if (z >= L) z -= L;
        }
    }
    return z;
}

// Displacement of one tracer over one RK4 step from x (eq. rk4_update, stages
// at t_n, t_n + dt/2, t_n + dt/2, t_n + dt with the temporal weights of P).
// The step kernel and the adjoint's recomputation share it, so recomputed
// trajectories repeat the forward ones bit for bit.
template <bool CUBIC>
__device__ __forceinline__ void rk4_tracer64(const Rec64 *__restrict__ rec0, const double2 *tile,
                                             const Tile &T, const StepParams &P, int scheme,
                                             double2 x, double &ddx, double &ddy)
{
    const double dt = P.dt, hdt = 0.5 * P.dt, dt6 = P.dt / 6.0;
    double k1x, k1y, k2x, k2y, k3x, k3y, k4x, k4y;
    vel64<CUBIC>(rec0, tile, T, P, scheme, x.x, x.y, P.wa[0], P.wb[0], P.smode[0], k1x, k1y);
    vel64<CUBIC>(rec0, tile, T, P, scheme, x.x + hdt * k1x, x.y + hdt * k1y, P.wa[1], P.wb[1],
                 P.smode[1], k2x, k2y);
    vel64<CUBIC>(rec0, tile, T, P, scheme, x.x + hdt * k2x, x.y + hdt * k2y, P.wa[2], P.wb[2],
                 P.smode[2], k3x, k3y);
    vel64<CUBIC>(rec0, tile, T, P, scheme, x.x + dt * k3x, x.y + dt * k3y, P.wa[3], P.wb[3],
                 P.smode[3], k4x, k4y);
    ddx = dt6 * (k1x + 2.0 * k2x + 2.0 * k3x + k4x);
    ddy = dt6 * (k1y + 2.0 * k2y + 2.0 * k3y + k4y);
}

}  // namespace lpt
