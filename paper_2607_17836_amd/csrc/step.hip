// gfx950 kernels of the particle step: snapshot packing, RK4 + interpolation
// (FP64 and FP32-split), initial state, velocity probe, readout and the
// statistics finalisation.
//
// One thread advances one particle by one RK4 step (Alg. coupled_EL, particle
// loop; eqs. rk4_update / rk4_inertial).  Each of the four stages gathers the
// 4 (bilinear) or 16 (bicubic) node records around the stage position; a node
// record carries both retained time levels, so one gather serves the temporal
// interpolation (eq. temporal_interp) too, and a stage whose temporal weight
// is (1, 0) or (0, 1) loads only the half it needs.  Records carry a periodic
// ghost border, so a stencil never wraps: its nodes are fixed offsets from one
// base address.  State is structure-of-arrays with interleaved (x, y) pairs,
// so the per-step state stream is fully coalesced; the gathers rely on
// cell-ordered particles (sort.hip) and an XCD-aware block order for L2 reuse.
#include "field_dev.h"

#include <map>
#include <mutex>
#include <tuple>

namespace lpt {

// One logical block of the FP64 step: the state of slot p is read from S and
// written to D, in place, or, on a step that follows a re-sort (GATHER), slot
// p of D takes the particle of slot perm[p] of S, id included.
template <bool CUBIC, bool INERTIAL, bool STATS, bool GATHER>
__device__ __forceinline__ void step64_block(const StepParams &P, const State64 &S,
                                             const State64 &D, const uint32_t *perm,
                                             const Rec64 *__restrict__ rec,
                                             double *__restrict__ partials, DevClock *clock,
                                             int lb)
{
    Rec64 *lds = reinterpret_cast<Rec64 *>(lpt_dyn_lds);
    const double2 *planes = reinterpret_cast<const double2 *>(lpt_dyn_lds);   // tile, two planes
    const SpeciesDev &sp = P.sp[species_of(P, lb)];
    const int64_t base = (int64_t)(lb - sp.block_begin) * blockDim.x;
    const int64_t local = base + threadIdx.x;
    const bool active = local < sp.count;
    const int64_t p = sp.offset + local;
    const Rec64 *rec0 = rec + P.pitch + 1;
    const double dt = P.dt, hdt = 0.5 * P.dt, dt6 = P.dt / 6.0;
    double r2x = 0.0, r2y = 0.0;

    int64_t q = p;
    double2 x = make_double2(0.0, 0.0);
    if (active) {
        if (GATHER) q = perm[p];
        x = S.pos[q];
    }
    Tile T = no_tile();
    if (P.tile_cap > 0) {
        const int64_t a0 = sp.offset + base;
        const double2 a = S.pos[GATHER ? (int64_t)perm[a0] : a0];
        const int n = P.n, mask = P.mask;
        const int ax = cell_of_floor(floor(a.x * P.invh), n, mask);
        const int ay = cell_of_floor(floor(a.y * P.invh), n, mask);
        const int cx = cell_of_floor(floor(x.x * P.invh), n, mask);
        const int cy = cell_of_floor(floor(x.y * P.invh), n, mask);
        int lo, hi;
        stencil_reach(sp.scheme, lo, hi);
        const int H = step_halo(P, sp.scheme, (float)dt);
        const int64_t left = sp.count - base;
        T = stage_tile<Rec64>(lds, rec0, P, active, cx, cy, ax, ay, lo + H, hi + H,
                              (int)(left < (int64_t)blockDim.x ? left : blockDim.x));
    }

    if (active) {
        double2 d = S.disp[q];
        double ddx, ddy;
        if (INERTIAL && sp.inertial) {
            // eqs. inertial_particle, drag_rk4, rk4_inertial
            const double2 vn = S.vel[q];
            const double is = sp.inv_st;
            double u, v;
            const double V1x = vn.x, V1y = vn.y;
            vel64<CUBIC>(rec0, planes, T, P, sp.scheme, x.x, x.y, P.wa[0], P.wb[0], P.smode[0], u, v);
            const double A1x = (u - V1x) * is, A1y = (v - V1y) * is;
            const double V2x = vn.x + hdt * A1x, V2y = vn.y + hdt * A1y;
            vel64<CUBIC>(rec0, planes, T, P, sp.scheme, x.x + hdt * V1x, x.y + hdt * V1y, P.wa[1],
                         P.wb[1], P.smode[1], u, v);
            const double A2x = (u - V2x) * is, A2y = (v - V2y) * is;
            const double V3x = vn.x + hdt * A2x, V3y = vn.y + hdt * A2y;
            vel64<CUBIC>(rec0, planes, T, P, sp.scheme, x.x + hdt * V2x, x.y + hdt * V2y, P.wa[2],
                         P.wb[2], P.smode[2], u, v);
            const double A3x = (u - V3x) * is, A3y = (v - V3y) * is;
            const double V4x = vn.x + dt * A3x, V4y = vn.y + dt * A3y;
            vel64<CUBIC>(rec0, planes, T, P, sp.scheme, x.x + dt * V3x, x.y + dt * V3y, P.wa[3],
                         P.wb[3], P.smode[3], u, v);
            const double A4x = (u - V4x) * is, A4y = (v - V4y) * is;
            ddx = dt6 * (V1x + 2.0 * V2x + 2.0 * V3x + V4x);
            ddy = dt6 * (V1y + 2.0 * V2y + 2.0 * V3y + V4y);
            D.vel[p] = make_double2(vn.x + dt6 * (A1x + 2.0 * A2x + 2.0 * A3x + A4x),
                                    vn.y + dt6 * (A1y + 2.0 * A2y + 2.0 * A3y + A4y));
        } else {
            rk4_tracer64<CUBIC>(rec0, planes, T, P, sp.scheme, x, ddx, ddy);
        }
        // wrapped coordinates for evaluation/output, unwrapped displacement
        // for statistics
        D.pos[p] = make_double2(wrap_pos(x.x + ddx, P.L), wrap_pos(x.y + ddy, P.L));
        d.x += ddx;
        d.y += ddy;
        D.disp[p] = d;
        if (GATHER) D.id[p] = S.id[q];
        r2x = d.x * d.x;
        r2y = d.y * d.y;
    }
    if (STATS)
        wave_stats(r2x, r2y, active,
                   partials + (int64_t)kStatTerms *
                                  ((int64_t)lb * (blockDim.x / kWave) + threadIdx.x / kWave));
    if (lb == 0 && threadIdx.x == 0) {
        clock->t += P.dt;
        clock->step += 1;
    }
}

template <bool CUBIC, bool INERTIAL, bool STATS>
__global__ __launch_bounds__(kMaxBlock) void step64_kernel(StepParams P, State64 S,
                                                           const Rec64 *__restrict__ rec,
                                                           double *__restrict__ partials,
                                                           DevClock *clock)
{
    BlockWalk w = block_walk(P, 0, P.total_blocks);
    for (int lb = 0; block_next(w, lb);)
        step64_block<CUBIC, INERTIAL, STATS, false>(P, S, S, nullptr, rec, partials, clock, lb);
}

// The FP64 step that follows a re-sort: reads S through perm, writes D.
template <bool CUBIC, bool INERTIAL, bool STATS>
__global__ __launch_bounds__(kMaxBlock) void step64_perm_kernel(StepParams P, State64 S,
                                                                State64 D, const uint32_t *perm,
                                                                const Rec64 *__restrict__ rec,
                                                                double *__restrict__ partials,
                                                                DevClock *clock)
{
    BlockWalk w = block_walk(P, 0, P.total_blocks);
    for (int lb = 0; block_next(w, lb);)
        step64_block<CUBIC, INERTIAL, STATS, true>(P, S, D, perm, rec, partials, clock, lb);
}

// ===========================================================================
// FP32 split path.  Positions are (cell, offset) with the offset in cell
// units; the packed field is in cells per unit time, so every stage works in
// cell units: q = offset + c*dt*k, cell = stored cell + floor(q), in-cell
// coordinate = fract(q).
// ===========================================================================
template <int SM>
__device__ __forceinline__ float2 half32(const float4 *r)
{
    return reinterpret_cast<const float2 *>(r)[SM];
}

__device__ __forceinline__ void bil32(const float4 *p, int pitch, float xi, float eta, int smode,
                                      float wa, float wb, float &u, float &v)
{
    float w00, w10, w01, w11;
    bilinear_weights(xi, eta, w00, w10, w01, w11);
    if (smode == kSlot0) {
        const float2 a = half32<0>(p), b = half32<0>(p + 1);
        const float2 c = half32<0>(p + pitch), d = half32<0>(p + pitch + 1);
        u = w00 * a.x + w10 * b.x + w01 * c.x + w11 * d.x;
        v = w00 * a.y + w10 * b.y + w01 * c.y + w11 * d.y;
    } else if (smode == kSlot1) {
        const float2 a = half32<1>(p), b = half32<1>(p + 1);
        const float2 c = half32<1>(p + pitch), d = half32<1>(p + pitch + 1);
        u = w00 * a.x + w10 * b.x + w01 * c.x + w11 * d.x;
        v = w00 * a.y + w10 * b.y + w01 * c.y + w11 * d.y;
    } else {
        const float4 a = p[0], b = p[1], c = p[pitch], d = p[pitch + 1];
        const float ua = w00 * a.x + w10 * b.x + w01 * c.x + w11 * d.x;
        const float va = w00 * a.y + w10 * b.y + w01 * c.y + w11 * d.y;
        const float ub = w00 * a.z + w10 * b.z + w01 * c.z + w11 * d.z;
        const float vb = w00 * a.w + w10 * b.w + w01 * c.w + w11 * d.w;
        u = wa * ua + wb * ub;
        v = wa * va + wb * vb;
    }
}

__device__ __forceinline__ void cub32(const float4 *p, int pitch, const float wx[4],
                                      const float wy[4], int smode, float wa, float wb, float &u,
                                      float &v)
{
    if (smode != kBlend) {
        const int h = smode;   // which half of the record
        float au = 0.f, av = 0.f;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const float2 *q = reinterpret_cast<const float2 *>(p) + h;
            float ru = 0.f, rv = 0.f;
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                const float2 r = q[2 * a];
                ru += wx[a] * r.x;
                rv += wx[a] * r.y;
            }
            au += wy[b] * ru;
            av += wy[b] * rv;
            p += pitch;
        }
        u = au;
        v = av;
    } else {
        float au = 0.f, av = 0.f, bu = 0.f, bv = 0.f;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            float ru = 0.f, rv = 0.f, su = 0.f, sv = 0.f;
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                const float4 r = p[a];
                ru += wx[a] * r.x;
                rv += wx[a] * r.y;
                su += wx[a] * r.z;
                sv += wx[a] * r.w;
            }
            au += wy[b] * ru;
            av += wy[b] * rv;
            bu += wy[b] * su;
            bv += wy[b] * sv;
            p += pitch;
        }
        u = wa * au + wb * bu;
        v = wa * av + wb * bv;
    }
}

template <bool CUBIC>
__device__ __forceinline__ void vel32(const float4 *__restrict__ rec0, const float4 *tile,
                                      const Tile &T, const StepParams &P, int scheme, int cx,
                                      int cy, float qx, float qy, float wa, float wb, int smode,
                                      float &u, float &v)
{
    const float fx = floorf(qx), fy = floorf(qy);
    const float xi = __builtin_amdgcn_fractf(qx), eta = __builtin_amdgcn_fractf(qy);
    const int n = P.n, mask = P.mask;
    const int i = cell_plus(cx, fx, n, mask), j = cell_plus(cy, fy, n, mask);
    int t;
    if (!CUBIC || scheme == kBilinear || edge_cell(P.compat_edge, i, j, n)) {
        if (tile_index(T, i, j, 2, n, mask, t))
            bil32(tile + t, T.w, xi, eta, smode, wa, wb, u, v);
        else
            bil32(rec0 + (__mul24(j, P.pitch) + i), P.pitch, xi, eta, smode, wa, wb, u, v);
        return;
    }
    if constexpr (CUBIC) {
        float wx[4], wy[4];
        if (scheme == kCatmullRom) {
            weights_cr(xi, wx);
            weights_cr(eta, wy);
        } else {
            weights_bs(xi, wx);
            weights_bs(eta, wy);
        }
        if (tile_index(T, i - 1, j - 1, 4, n, mask, t))
            cub32(tile + t, T.w, wx, wy, smode, wa, wb, u, v);
        else
            cub32(rec0 + (__mul24(j - 1, P.pitch) + (i - 1)), P.pitch, wx, wy, smode, wa, wb, u, v);
    }
}

// New (cell, offset) after a displacement of dq cells from offset o; the
// offset stays in [0, 1) (fract never returns 1).
__device__ __forceinline__ int advance_split(int &c, float &o, float dq, const StepParams &P)
{
    const float q = o + dq;
    const float f = __builtin_amdgcn_fmed3f(floorf(q), -kCellClampF, kCellClampF);
    float r = __builtin_amdgcn_fractf(q);
    if (!(r >= 0.0f)) r = 0.0f;   // NaN guard keeps the state in range
    const int m = (int)f;         // the cell move (0 for NaN)
    c = wrap_cell(c + m, P.n, P.mask);
    o = r;
    return m;
}

// Unwrapped cell plus a move, wrapping modulo 2^32 (moves are clamped, so
// only an absurd state, never a real trajectory, gets there).
__device__ __forceinline__ int ucell_plus(int u, int m)
{
    return (int)((uint32_t)u + (uint32_t)m);
}

// Split form of a binary64 position: the cell floor(x n / L) in [0, n) and the
// binary32 offset in [0, 1) (the initial state of a particle).
__device__ __forceinline__ void split_of(double x, const StepParams &P, int &c, float &o)
{
    const double s = x * P.invh;
    const double f = floor(s);
    float r = (float)(s - f);
    int ci = cell_of_floor(f, P.n, P.mask);
    if (r >= 1.0f) {
        r = 0.0f;
        ci = wrap_cell(ci + 1, P.n, P.mask);
    }
    if (!(r >= 0.0f)) r = 0.0f;
    c = ci;
    o = r;
}

// Counter-indexed SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): output k of
// the stream seeded with s is mix(s + (k + 1) * golden gamma).
__device__ __forceinline__ uint64_t splitmix_at(uint64_t seed, uint64_t k)
{
    uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

// Uniform initial position of particle k of a species drawn with `seed`:
// outputs 2k and 2k + 1 of the stream, top 53 bits as a fraction of L.  The
// one definition both the initialisation and the record steps use, so a
// position drawn again is the stored one, bit for bit.
__device__ __forceinline__ double2 draw_x0(uint64_t seed, uint64_t k, double L)
{
    const double ux = (double)(splitmix_at(seed, 2 * k) >> 11) * 0x1p-53;
    const double uy = (double)(splitmix_at(seed, 2 * k + 1) >> 11) * 0x1p-53;
    return make_double2(wrap_pos(L * ux, L), wrap_pos(L * uy, L));
}

// Initial position of particle g (global id) of species sp: drawn again
// where the species was initialised uniformly (a few integer operations
// instead of a gather in particle order, which is random after re-sorts),
// else read.
__device__ __forceinline__ double2 initial_pos(const SpeciesDev &sp, const double2 *x0, uint32_t g,
                                               const StepParams &P)
{
    if (sp.x0_drawn) return draw_x0(sp.x0_seed, (uint64_t)((int64_t)g - sp.offset), P.L);
    return x0[g];
}

// Displacement since initialisation (physical units) of a particle at
// unwrapped cell u, offset o, that started at x0.
__device__ __forceinline__ double2 split_disp(int2 u, float2 o, double2 x0, const StepParams &P)
{
    int cx, cy;
    float ox, oy;
    split_of(x0.x, P, cx, ox);
    split_of(x0.y, P, cy, oy);
    return make_double2(((double)(int)((uint32_t)u.x - (uint32_t)cx) + ((double)o.x - (double)ox)) * P.h,
                        ((double)(int)((uint32_t)u.y - (uint32_t)cy) + ((double)o.y - (double)oy)) * P.h);
}

// ---------------------------------------------------------------------------
// The FP32-split step, specialised per block on (scheme, particle kind).
// Stage positions are kept relative to the particle's stored cell: the stage
// cell is (cx + floor(qx), cy + floor(qy)) and, inside the LDS tile, its tile
// coordinate is (rx + floor(qx), ry + floor(qy)) with (rx, ry) the stored
// cell's tile coordinate, computed once per particle.  Only a stencil that
// leaves the tile needs the periodic wrap and a global gather.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int wrapn(int c, const StepParams &P)
{
    return wrap_cell(c, P.n, P.mask);
}

// Node accessors of the FP32 step.  Global memory holds one {u0, v0, u1, v1}
// record per node (ghost-bordered rows of `pitch` records); the LDS tile
// holds two planes of (u, v), one per time level, so that a stage reading a
// single level gathers 8 dense bytes per node.  Both are addressed from the
// stencil's origin node (a, b: column and row offsets from it).
struct GlobalNodes {
    const float4 *p;
    int pitch;
    __device__ __forceinline__ float2 level(int a, int b, int h) const
    {
        return reinterpret_cast<const float2 *>(p + (b * pitch + a))[h];
    }
    __device__ __forceinline__ float4 both(int a, int b) const { return p[b * pitch + a]; }
};

struct TileNodes {
    const float4 *p;   // origin node
    int pitch;         // tile width
    __device__ __forceinline__ float2 level(int a, int b, int h) const
    {
        return reinterpret_cast<const float2 *>(p + (b * pitch + a))[h];
    }
    __device__ __forceinline__ float4 both(int a, int b) const { return p[b * pitch + a]; }
};

// Velocity of one stencil (eqs. bilinear_interp, cr_interp, bspline_interp)
// with the temporal interpolation of eq. temporal_interp: ONE reads only
// level h (weight (1, 0) or (0, 1)); otherwise both levels blend with
// (wa, wb).
template <int SCH, typename Nodes>
__device__ __forceinline__ void eval32(const Nodes &N, float xi, float eta, bool one, int h,
                                       float wa, float wb, float &u, float &v)
{
    if constexpr (SCH == kBilinear) {
        float w00, w10, w01, w11;
        bilinear_weights(xi, eta, w00, w10, w01, w11);
        if (one) {
            const float2 a = N.level(0, 0, h), b = N.level(1, 0, h);
            const float2 c = N.level(0, 1, h), d = N.level(1, 1, h);
            u = w00 * a.x + w10 * b.x + w01 * c.x + w11 * d.x;
            v = w00 * a.y + w10 * b.y + w01 * c.y + w11 * d.y;
        } else {
            const float4 a = N.both(0, 0), b = N.both(1, 0), c = N.both(0, 1), d = N.both(1, 1);
            const float ua = w00 * a.x + w10 * b.x + w01 * c.x + w11 * d.x;
            const float va = w00 * a.y + w10 * b.y + w01 * c.y + w11 * d.y;
            const float ub = w00 * a.z + w10 * b.z + w01 * c.z + w11 * d.z;
            const float vb = w00 * a.w + w10 * b.w + w01 * c.w + w11 * d.w;
            u = wa * ua + wb * ub;
            v = wa * va + wb * vb;
        }
    } else {
        float wx[4], wy[4];
        if constexpr (SCH == kCatmullRom) {
            weights_cr(xi, wx);
            weights_cr(eta, wy);
        } else {
            weights_bs(xi, wx);
            weights_bs(eta, wy);
        }
        if (one) {
            float au = 0.f, av = 0.f;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                float ru = 0.f, rv = 0.f;
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    const float2 r = N.level(a, b, h);
                    ru += wx[a] * r.x;
                    rv += wx[a] * r.y;
                }
                au += wy[b] * ru;
                av += wy[b] * rv;
            }
            u = au;
            v = av;
        } else {
            float au = 0.f, av = 0.f, bu = 0.f, bv = 0.f;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                float ru = 0.f, rv = 0.f, su = 0.f, sv = 0.f;
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    const float4 r = N.both(a, b);
                    ru += wx[a] * r.x;
                    rv += wx[a] * r.y;
                    su += wx[a] * r.z;
                    sv += wx[a] * r.w;
                }
                au += wy[b] * ru;
                av += wy[b] * rv;
                bu += wy[b] * su;
                bv += wy[b] * sv;
            }
            u = wa * au + wb * bu;
            v = wa * av + wb * bv;
        }
    }
}

__device__ __forceinline__ TileNodes tile_nodes(const float4 *lds, const Tile &T, int tx, int ty)
{
    return TileNodes{lds + (__mul24(ty, T.w) + tx), T.w};
}

__device__ __forceinline__ GlobalNodes global_nodes(const float4 *rec0, const StepParams &P,
                                                    int i, int j)
{
    return GlobalNodes{rec0 + (__mul24(j, P.pitch) + i), P.pitch};
}

// Fluid velocity (cells per unit time) of one RK4 stage at stored cell
// (cx, cy) + q.  (rx, ry): tile coordinate of the stored cell.
template <int SCH>
__device__ __forceinline__ void stage32(const float4 *__restrict__ rec0, const float4 *lds,
                                        const Tile &T, const StepParams &P, int cx, int cy,
                                        int rx, int ry, float qx, float qy, bool one, int h,
                                        float wa, float wb, float &u, float &v)
{
    constexpr int c1 = SCH == kBilinear ? 0 : 1;
    constexpr int span = SCH == kBilinear ? 2 : 4;
    qx = __builtin_amdgcn_fmed3f(qx, -kCellClampF, kCellClampF);
    qy = __builtin_amdgcn_fmed3f(qy, -kCellClampF, kCellClampF);
    const float flx = floorf(qx), fly = floorf(qy);
    const int fx = (int)flx, fy = (int)fly;
    const float xi = qx - flx, eta = qy - fly;
    if constexpr (SCH != kBilinear) {
        if (P.compat_edge) {   // the paper's bilinear fallback near the grid edge
            const int i = wrapn(cx + fx, P), j = wrapn(cy + fy, P);
            if (edge_cell(1, i, j, P.n)) {
                eval32<kBilinear>(global_nodes(rec0, P, i, j), xi, eta, one, h, wa, wb, u, v);
                return;
            }
        }
    }
    const int tx = rx + fx - c1, ty = ry + fy - c1;
    if (T.on && (unsigned)tx <= (unsigned)(T.w - span) && (unsigned)ty <= (unsigned)(T.h - span)) {
        eval32<SCH>(tile_nodes(lds, T, tx, ty), xi, eta, one, h, wa, wb, u, v);
    } else {
        const int i = wrapn(cx + fx, P) - c1, j = wrapn(cy + fy, P) - c1;
        eval32<SCH>(global_nodes(rec0, P, i, j), xi, eta, one, h, wa, wb, u, v);
    }
}

// The first stage sits at the stored position itself: stored cell, in-cell
// coordinates = the stored offset in [0, 1) (so floor(q) = 0 and the general
// stage computes the same values).  The stored cell lies inside the block's
// box and the box adds the stencil reach, so the stencil is inside the tile
// unless the box was cut down to the tile's capacity.
template <int SCH, bool ONE>
__device__ __forceinline__ void stage32_first(const float4 *__restrict__ rec0, const float4 *lds,
                                              const Tile &T, const StepParams &P, int cx, int cy,
                                              int rx, int ry, float2 o, int h, float wa, float wb,
                                              float &u, float &v)
{
    constexpr int c1 = SCH == kBilinear ? 0 : 1;
    if (SCH != kBilinear && P.compat_edge) {
        stage32<SCH>(rec0, lds, T, P, cx, cy, rx, ry, o.x, o.y, ONE, h, wa, wb, u, v);
        return;
    }
    constexpr int span = SCH == kBilinear ? 2 : 4;
    if (T.on && (unsigned)(rx - c1) <= (unsigned)(T.w - span) &&
        (unsigned)(ry - c1) <= (unsigned)(T.h - span))
        eval32<SCH>(tile_nodes(lds, T, rx - c1, ry - c1), o.x, o.y, ONE, h, wa, wb, u, v);
    else
        eval32<SCH>(global_nodes(rec0, P, cx - c1, cy - c1), o.x, o.y, ONE, h, wa, wb, u, v);
}

// One RK4 step of one particle (eqs. rk4_update / rk4_inertial, Stokes drag
// of eq. drag_rk4), then the split-position update and the FP64
// displacement.  Returns the new displacement squared per axis.
// GATHER: the step after a re-sort, whose state reads are gathers through the
// permutation; the displacement is then loaded first, so that its latency
// overlaps the stages (in place it is loaded last, which keeps registers free).
template <int SCH, bool INERT, bool ONE, bool GATHER>
__device__ __forceinline__ void particle32(const StepParams &P, const State32 &S,
                                           const State32 &D, const float4 *__restrict__ rec0,
                                           const float4 *lds, const Tile &T, const SpeciesDev &sp,
                                           int64_t p, int64_t q, uint32_t cell, int2 &uc,
                                           float2 &o)
{
    int cx = (int)(cell & 0xFFFFu), cy = (int)(cell >> 16);
    int rx = 0, ry = 0;
    if (T.on) {   // cx - T.x0 lies in (-n, n)
        rx = cx - T.x0;
        ry = cy - T.y0;
        rx += rx < 0 ? P.n : 0;
        ry += ry < 0 ? P.n : 0;
    }
    const float dt = P.dtf, hdt = P.hdtf, dt6 = P.dt6f;
    constexpr bool one = ONE;   // first / last stage read a single time level
    float dqx, dqy;
    if constexpr (INERT) {
        const float2 vn = ld_stream(S.vel + q);
        const float is = (float)sp.inv_st;
        float u, v;
        const float V1x = vn.x, V1y = vn.y;
        stage32_first<SCH, ONE>(rec0, lds, T, P, cx, cy, rx, ry, o, P.h0, P.waf[0], P.wbf[0], u, v);
        const float A1x = (u - V1x) * is, A1y = (v - V1y) * is;
        const float V2x = vn.x + hdt * A1x, V2y = vn.y + hdt * A1y;
        stage32<SCH>(rec0, lds, T, P, cx, cy, rx, ry, o.x + hdt * V1x, o.y + hdt * V1y, false, 0,
                     P.waf[1], P.wbf[1], u, v);
        const float A2x = (u - V2x) * is, A2y = (v - V2y) * is;
        const float V3x = vn.x + hdt * A2x, V3y = vn.y + hdt * A2y;
        stage32<SCH>(rec0, lds, T, P, cx, cy, rx, ry, o.x + hdt * V2x, o.y + hdt * V2y, false, 0,
                     P.waf[2], P.wbf[2], u, v);
        const float A3x = (u - V3x) * is, A3y = (v - V3y) * is;
        const float V4x = vn.x + dt * A3x, V4y = vn.y + dt * A3y;
        stage32<SCH>(rec0, lds, T, P, cx, cy, rx, ry, o.x + dt * V3x, o.y + dt * V3y, one, P.h3,
                     P.waf[3], P.wbf[3], u, v);
        const float A4x = (u - V4x) * is, A4y = (v - V4y) * is;
        dqx = dt6 * (V1x + 2.0f * V2x + 2.0f * V3x + V4x);
        dqy = dt6 * (V1y + 2.0f * V2y + 2.0f * V3y + V4y);
        st_stream(D.vel + p, make_float2(vn.x + dt6 * (A1x + 2.0f * A2x + 2.0f * A3x + A4x),
                                         vn.y + dt6 * (A1y + 2.0f * A2y + 2.0f * A3y + A4y)));
    } else {
        float k1x, k1y, k2x, k2y, k3x, k3y, k4x, k4y;
        stage32_first<SCH, ONE>(rec0, lds, T, P, cx, cy, rx, ry, o, P.h0, P.waf[0], P.wbf[0], k1x,
                                k1y);
        stage32<SCH>(rec0, lds, T, P, cx, cy, rx, ry, o.x + hdt * k1x, o.y + hdt * k1y, false, 0,
                     P.waf[1], P.wbf[1], k2x, k2y);
        stage32<SCH>(rec0, lds, T, P, cx, cy, rx, ry, o.x + hdt * k2x, o.y + hdt * k2y, false, 0,
                     P.waf[2], P.wbf[2], k3x, k3y);
        stage32<SCH>(rec0, lds, T, P, cx, cy, rx, ry, o.x + dt * k3x, o.y + dt * k3y, one, P.h3,
                     P.waf[3], P.wbf[3], k4x, k4y);
        dqx = dt6 * (k1x + 2.0f * k2x + 2.0f * k3x + k4x);
        dqy = dt6 * (k1y + 2.0f * k2y + 2.0f * k3y + k4y);
    }
    float ox = o.x, oy = o.y;
    const int mx = advance_split(cx, ox, dqx, P);
    const int my = advance_split(cy, oy, dqy, P);
    uc = make_int2(ucell_plus(uc.x, mx), ucell_plus(uc.y, my));
    o = make_float2(ox, oy);
    st_stream(D.uc + p, uc);
    st_stream(D.off + p, o);
}

// The particle body for the block's kind.  SCHS: the scheme of every species
// of the launch (one launch per scheme), or kAnyScheme in a fused launch.
// KINDS: 0 tracers only (St == 0 included), 1 tracers and/or inertial
// species.
template <int SCHS, int KINDS, bool ONE, bool GATHER>
__device__ __forceinline__ void particle_dispatch(const StepParams &P, const State32 &S,
                                                  const State32 &D,
                                                  const float4 *__restrict__ rec0,
                                                  const float4 *lds, const Tile &T,
                                                  const SpeciesDev &sp, int64_t p, int64_t q,
                                                  uint32_t cell, int2 &uc, float2 &o)
{
    if constexpr (SCHS == kAnyScheme) {   // fused launch: the block's species decides
        if (sp.scheme == kBilinear)
            particle_dispatch<kBilinear, KINDS, ONE, GATHER>(P, S, D, rec0, lds, T, sp, p, q, cell,
                                                             uc, o);
        else if (sp.scheme == kCatmullRom)
            particle_dispatch<kCatmullRom, KINDS, ONE, GATHER>(P, S, D, rec0, lds, T, sp, p, q,
                                                               cell, uc, o);
        else
            particle_dispatch<kBSpline, KINDS, ONE, GATHER>(P, S, D, rec0, lds, T, sp, p, q, cell,
                                                            uc, o);
        return;
    }
    if (KINDS != 0 && sp.inertial)
        particle32<SCHS, KINDS != 0, ONE, GATHER>(P, S, D, rec0, lds, T, sp, p, q, cell, uc, o);
    else
        particle32<SCHS, false, ONE, GATHER>(P, S, D, rec0, lds, T, sp, p, q, cell, uc, o);
}

// One logical block at one particle per thread: step32_block with ROWS = 1,
// as a body of its own (the row loop's carried state would cost registers a
// single row does not need).
template <int SCHS, int KINDS, bool STATS, bool GATHER>
__device__ __forceinline__ void step32_block1(const StepParams &P, const State32 &S,
                                             const State32 &D, const uint32_t *perm,
                                             const float4 *__restrict__ rec,
                                             double *__restrict__ partials, DevClock *clock,
                                             int lb)
{
    float4 *lds = reinterpret_cast<float4 *>(lpt_dyn_lds);
    const SpeciesDev &sp = P.sp[P.nspecies > 1 ? species_of(P, lb) : 0];
    const int64_t base = (int64_t)(lb - sp.block_begin) * blockDim.x;
    const int64_t local = base + threadIdx.x;
    const bool active = local < sp.count;
    const int64_t p = sp.offset + local;
    const float4 *rec0 = rec + P.pitch + 1;
    double r2x = 0.0, r2y = 0.0;

    int64_t q = p;
    uint32_t cell = 0;   // the stored cell, (cy << 16) | cx
    int2 uc = make_int2(0, 0);
    float2 o = make_float2(0.f, 0.f);
    if (active) {
        if (GATHER) q = perm[p];
        uc = ld_stream(S.uc + q);
        o = ld_stream(S.off + q);
        cell = (uint32_t)wrapn(uc.x, P) | ((uint32_t)wrapn(uc.y, P) << 16);
    }
    Tile T = no_tile();
    if (P.tile_cap > 0) {
        int lo, hi;
        stencil_reach(sp.scheme, lo, hi);
        const int H = step_halo(P, sp.scheme, P.dtf);
        const int64_t left = sp.count - base;
        const int nact = (int)(left < (int64_t)blockDim.x ? left : blockDim.x);
        const int64_t a0 = sp.offset + base;
        const int2 a = S.uc[GATHER ? (int64_t)perm[a0] : a0];
        T = stage_tile<float4>(lds, rec0, P, active, (int)(cell & 0xFFFFu), (int)(cell >> 16),
                               wrapn(a.x, P), wrapn(a.y, P), lo + H, hi + H, nact);
    }
    if (active) {
        if (P.ends_one)
            particle_dispatch<SCHS, KINDS, true, GATHER>(P, S, D, rec0, lds, T, sp, p, q, cell, uc,
                                                         o);
        else
            particle_dispatch<SCHS, KINDS, false, GATHER>(P, S, D, rec0, lds, T, sp, p, q, cell,
                                                          uc, o);
        if (GATHER || STATS) {
            const uint32_t g = S.id[q];
            if (GATHER) D.id[p] = g;
            if (STATS) {   // the displacement since initialisation, from the new state
                const double2 d = split_disp(uc, o, initial_pos(sp, S.x0, g, P), P);
                r2x = d.x * d.x;
                r2y = d.y * d.y;
            }
        }
    }
    if (STATS)
        wave_stats(r2x, r2y, active,
                   partials + (int64_t)kStatTerms *
                                  ((int64_t)lb * (blockDim.x / kWave) + threadIdx.x / kWave));
    if (lb == 0 && threadIdx.x == 0) {
        clock->t += P.dt;
        clock->step += 1;
    }
}

// One logical block of the step.  The state of slot p is read from S and
// written to D: in place, or, on a step that follows a re-sort (GATHER),
// slot p of D takes the particle of slot perm[p] of S, id included, so that
// the step itself applies the sort's permutation.  A logical block holds
// ROWS rows of blockDim.x slots: thread t takes slot t of every row, so the
// block's set-up (its box, tile and launch bookkeeping) is shared by ROWS
// particles per thread.  Row 0 keeps its state in registers from the box to
// the step; the cells of later rows are read for the box and again for the
// step (the second read finds them in the cache).
template <int SCHS, int KINDS, bool STATS, bool GATHER, int ROWS>
__device__ __forceinline__ void step32_block(const StepParams &P, const State32 &S,
                                             const State32 &D, const uint32_t *perm,
                                             const float4 *__restrict__ rec,
                                             double *__restrict__ partials, DevClock *clock,
                                             int lb)
{
    if constexpr (ROWS == 1) {
        step32_block1<SCHS, KINDS, STATS, GATHER>(P, S, D, perm, rec, partials, clock, lb);
        return;
    }
    float4 *lds = reinterpret_cast<float4 *>(lpt_dyn_lds);
    const SpeciesDev &sp = P.sp[P.nspecies > 1 ? species_of(P, lb) : 0];
    const int threads = (int)blockDim.x;
    const int64_t slots = (int64_t)threads * ROWS;
    const int64_t base = (int64_t)(lb - sp.block_begin) * slots;
    const float4 *rec0 = rec + P.pitch + 1;

    const bool active0 = base + threadIdx.x < sp.count;
    int64_t q0 = sp.offset + base + threadIdx.x;
    uint32_t cell0 = 0;   // the stored cell, (cy << 16) | cx
    int2 uc0 = make_int2(0, 0);
    float2 o0 = make_float2(0.f, 0.f);
    if (active0) {
        if (GATHER) q0 = perm[q0];
        uc0 = ld_stream(S.uc + q0);
        o0 = ld_stream(S.off + q0);
        cell0 = (uint32_t)wrapn(uc0.x, P) | ((uint32_t)wrapn(uc0.y, P) << 16);
    }
    Tile T = no_tile();
    if (P.tile_cap > 0) {
        int lo, hi;
        stencil_reach(sp.scheme, lo, hi);
        const int H = step_halo(P, sp.scheme, P.dtf);
        const int64_t left = sp.count - base;
        const int nact = (int)(left < slots ? left : slots);
        const int64_t a0 = sp.offset + base;
        const int2 a = S.uc[GATHER ? (int64_t)perm[a0] : a0];
        const int ax = wrapn(a.x, P), ay = wrapn(a.y, P);
        BoxAcc b = active0 ? box_of((int)(cell0 & 0xFFFFu), (int)(cell0 >> 16), ax, ay, P.n)
                           : box_init();
#pragma unroll
        for (int r = 1; r < ROWS; ++r) {
            const int64_t local = base + (int64_t)r * threads + threadIdx.x;
            if (local < sp.count) {
                const int64_t p = sp.offset + local;
                const int2 u = S.uc[GATHER ? (int64_t)perm[p] : p];
                box_add(b, wrapn(u.x, P), wrapn(u.y, P), ax, ay, P.n);
            }
        }
        T = stage_tile_acc<float4>(lds, rec0, P, b, ax, ay, lo + H, hi + H, nact);
    }
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        const int64_t local = base + (int64_t)r * threads + threadIdx.x;
        const bool active = local < sp.count;
        const int64_t p = sp.offset + local;
        double r2x = 0.0, r2y = 0.0;
        if (active) {
            int64_t q = q0;
            int2 uc = uc0;
            float2 o = o0;
            uint32_t cell = cell0;
            if (r > 0) {
                q = GATHER ? (int64_t)perm[p] : p;
                uc = ld_stream(S.uc + q);
                o = ld_stream(S.off + q);
                cell = (uint32_t)wrapn(uc.x, P) | ((uint32_t)wrapn(uc.y, P) << 16);
            }
            if (P.ends_one)
                particle_dispatch<SCHS, KINDS, true, GATHER>(P, S, D, rec0, lds, T, sp, p, q, cell,
                                                             uc, o);
            else
                particle_dispatch<SCHS, KINDS, false, GATHER>(P, S, D, rec0, lds, T, sp, p, q,
                                                              cell, uc, o);
            if (GATHER || STATS) {
                const uint32_t g = S.id[q];
                if (GATHER) D.id[p] = g;
                if (STATS) {   // the displacement since initialisation, from the new state
                    const double2 d = split_disp(uc, o, initial_pos(sp, S.x0, g, P), P);
                    r2x = d.x * d.x;
                    r2y = d.y * d.y;
                }
            }
        }
        // one partial per 64 slots, in slot order: wave w of row r covers the
        // slots lb * slots + r * threads + 64 w + [0, 64)
        if (STATS)
            wave_stats(r2x, r2y, active,
                       partials + (int64_t)kStatTerms *
                                      (((int64_t)lb * slots + (int64_t)r * threads) / kWave +
                                       threadIdx.x / kWave));
    }
    if (lb == 0 && threadIdx.x == 0) {
        clock->t += P.dt;
        clock->step += 1;
    }
}

// One launch advances every particle of its logical blocks by one step
// (block_walk: one workgroup per logical block in XCD-aware order, a
// persistent walk, or a fused launch's block-order table).
// Bilinear blocks hold eight 256-thread blocks per CU (the LDS tile's
// budget), i.e. eight waves per SIMD, so their registers are bounded to fit
// that; the bicubic bodies, and the fused kernel that holds every body
// (SCHS = kAnyScheme), need more registers and keep the default bound.
template <int SCHS, int KINDS, bool STATS, int ROWS>
__global__ __launch_bounds__(kMaxBlock)
__attribute__((amdgpu_waves_per_eu(SCHS == kBilinear ? 8 : 6)))
void step32_kernel(StepParams P, State32 S, const float4 *__restrict__ rec,
                   double *__restrict__ partials, DevClock *clock)
{
    BlockWalk w = block_walk(P, P.block_base, P.launch_blocks);
    for (int lb = 0; block_next(w, lb);)
        step32_block<SCHS, KINDS, STATS, false, ROWS>(P, S, S, nullptr, rec, partials, clock, lb);
}

// The step that follows a re-sort: reads S through perm, writes D.  (A kernel
// of its own, so that the in-place kernel above keeps its argument list.)
template <int SCHS, int KINDS, bool STATS, int ROWS>
__global__ __launch_bounds__(kMaxBlock)
__attribute__((amdgpu_waves_per_eu(SCHS == kBilinear ? 8 : 6)))
void step32_perm_kernel(StepParams P, State32 S, State32 D, const uint32_t *perm,
                        const float4 *__restrict__ rec, double *__restrict__ partials,
                        DevClock *clock)
{
    BlockWalk w = block_walk(P, P.block_base, P.launch_blocks);
    for (int lb = 0; block_next(w, lb);)
        step32_block<SCHS, KINDS, STATS, true, ROWS>(P, S, D, perm, rec, partials, clock, lb);
}

// Grid of a launch: one workgroup per logical block (per table entry in a
// fused launch), or -- when the step parameters ask for a persistent launch
// -- as many workgroups as the device keeps resident (occupancy of this
// kernel at this block size and LDS size, times the CU count, capped at
// P.max_wg if set; a multiple of the XCD count in a fused launch), if that
// is fewer.
template <typename K>
static int launch_grid(K kernel, const StepParams &P, int block, size_t lds, int grid,
                       StepParams &Q)
{
    Q = P;
    Q.persistent = 0;
    if (P.order) grid = 8 * P.order_len;
    if (!P.persistent) return grid;
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, lds) != hipSuccess ||
        per_cu < 1) {
        (void)hipGetLastError();
        return grid;
    }
    int64_t resident = (int64_t)per_cu * cus;
    if (P.max_wg > 0 && resident > P.max_wg) resident = P.max_wg;
    if (P.order) resident = resident < 8 ? 8 : resident / 8 * 8;
    if (resident >= grid) return grid;
    Q.persistent = 1;
    return (int)resident;
}

// Automatic LDS tile capacity of an FP32 step kernel at a block size: the
// CU's LDS split between as many blocks as the kernel's registers let stay
// resident (less each block's static LDS), in whole 64-entry fill chunks,
// lowered while it would still cost a resident block.  planes: 16-byte
// entries per node record (one for FP32; two, plus one chunk of fill
// overrun, for FP64).  The occupancy queries run once per (kernel, block
// size, device).
template <typename K>
static int32_t auto_tile_cap(K kernel, int block, int planes, int32_t fallback)
{
    static std::mutex mu;
    static std::map<std::tuple<const void *, int, int>, int32_t> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return fallback;
    }
    const auto key = std::make_tuple(reinterpret_cast<const void *>(kernel), block, dev);
    std::lock_guard<std::mutex> lock(mu);
    const auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    auto lds_of = [planes](int32_t cap) {
        return planes == 1 ? (size_t)cap * 16 : (size_t)(2 * cap + kWave) * 16;
    };
    int lds_cu = 0, blocks = 0;
    hipFuncAttributes fa{};
    int32_t cap = fallback;
    if (hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) ==
            hipSuccess &&
        hipFuncGetAttributes(&fa, reinterpret_cast<const void *>(kernel)) == hipSuccess &&
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, kernel, block, 0) == hipSuccess &&
        blocks > 0 && lds_cu > 0) {
        const int64_t per_block = (int64_t)lds_cu / blocks - (int64_t)fa.sharedSizeBytes;
        const int64_t entries = per_block / 16 - (planes == 1 ? 0 : kWave);
        int64_t c = entries / planes / kWave * kWave;
        const int64_t most = (int64_t)(61440 / (16 * planes)) / kWave * kWave;
        c = c > most ? most : c;
        int resident = 0;
        while (c >= kWave &&
               (hipOccupancyMaxActiveBlocksPerMultiprocessor(&resident, kernel, block,
                                                             lds_of((int32_t)c)) != hipSuccess ||
                resident < blocks))
            c -= kWave;
        if (c >= kWave) cap = (int32_t)c;
    }
    (void)hipGetLastError();
    cache.emplace(key, cap);
    return cap;
}

template <bool C, bool I, bool S>
static hipError_t launch64_t(const StepParams &P, const State64 &St, const State64 &Dst,
                             const uint32_t *perm, const Rec64 *rec, double *partials,
                             DevClock *clock, int block, int grid, hipStream_t st)
{
    // The FP64 tile keeps its fixed capacity in automatic mode too: sized to
    // the register-bound occupancy it would leave too many boxes uncovered.
    const StepParams &P1 = P;
    // two planes of 16-byte entries; the fill writes whole 64-entry chunks of each
    const size_t lds = P1.tile_cap > 0 ? (size_t)(2 * P1.tile_cap + kWave) * 16 : 0;
    StepParams Q;
    if (perm) {
        const int g = launch_grid(step64_perm_kernel<C, I, S>, P1, block, lds, grid, Q);
        hipLaunchKernelGGL((step64_perm_kernel<C, I, S>), dim3(g), dim3(block), lds, st, Q, St,
                           Dst, perm, rec, partials, clock);
    } else {
        const int g = launch_grid(step64_kernel<C, I, S>, P1, block, lds, grid, Q);
        hipLaunchKernelGGL((step64_kernel<C, I, S>), dim3(g), dim3(block), lds, st, Q, St, rec,
                           partials, clock);
    }
    return hipGetLastError();
}

template <int SCHS, int KINDS, bool ST, int ROWS>
static hipError_t launch32_r(const StepParams &P, const State32 &S, const State32 &D,
                             const uint32_t *perm, const float4 *rec, double *partials,
                             DevClock *clock, int block, int grid, hipStream_t st)
{
    // a logical block of `block` slots runs on block / ROWS threads
    const int threads = block / ROWS;
    StepParams P1 = P;
    if (P.tile_auto && P.tile_cap > 0)
        P1.tile_cap = perm ? auto_tile_cap(step32_perm_kernel<SCHS, KINDS, ST, ROWS>, threads, 1,
                                           P.tile_cap)
                           : auto_tile_cap(step32_kernel<SCHS, KINDS, ST, ROWS>, threads, 1,
                                           P.tile_cap);
    // whole 64-entry chunks: the tile fill writes LDS a wave's chunk at a time
    const size_t lds =
        P1.tile_cap > 0 ? (size_t)((P1.tile_cap + kWave - 1) / kWave * kWave) * sizeof(float4) : 0;
    StepParams Q;
    if (perm) {
        const int g =
            launch_grid(step32_perm_kernel<SCHS, KINDS, ST, ROWS>, P1, threads, lds, grid, Q);
        hipLaunchKernelGGL((step32_perm_kernel<SCHS, KINDS, ST, ROWS>), dim3(g), dim3(threads),
                           lds, st, Q, S, D, perm, rec, partials, clock);
    } else {
        const int g = launch_grid(step32_kernel<SCHS, KINDS, ST, ROWS>, P1, threads, lds, grid, Q);
        hipLaunchKernelGGL((step32_kernel<SCHS, KINDS, ST, ROWS>), dim3(g), dim3(threads), lds, st,
                           Q, S, rec, partials, clock);
    }
    return hipGetLastError();
}

template <int SCHS, int KINDS, bool ST>
static hipError_t launch32_t(const StepParams &P, const State32 &S, const State32 &D,
                             const uint32_t *perm, const float4 *rec, double *partials,
                             DevClock *clock, int block, int grid, hipStream_t st)
{
    // two rows per thread exist for the bilinear tracer bodies only (the
    // bodies where the block's set-up is the largest share of the work);
    // every other body runs one row, whatever P.rows asks
    if constexpr (SCHS == kBilinear && KINDS == 0)
        if (P.rows == 2)
            return launch32_r<SCHS, KINDS, ST, 2>(P, S, D, perm, rec, partials, clock, block, grid,
                                                  st);
    return launch32_r<SCHS, KINDS, ST, 1>(P, S, D, perm, rec, partials, clock, block, grid, st);
}

template <int SCHS>
static hipError_t launch32_s(const StepParams &P, const State32 &S, const State32 &D,
                             const uint32_t *perm, const float4 *rec, double *partials,
                             DevClock *clock, bool stats, bool inertial, int block, int grid,
                             hipStream_t st)
{
    if (inertial)
        return stats ? launch32_t<SCHS, 1, true>(P, S, D, perm, rec, partials, clock, block, grid,
                                                 st)
                     : launch32_t<SCHS, 1, false>(P, S, D, perm, rec, partials, clock, block,
                                                  grid, st);
    return stats ? launch32_t<SCHS, 0, true>(P, S, D, perm, rec, partials, clock, block, grid, st)
                 : launch32_t<SCHS, 0, false>(P, S, D, perm, rec, partials, clock, block, grid,
                                              st);
}

#define LPT_DISPATCH(fn, ...)                                                        \
    do {                                                                             \
        const int sel = (cubic ? 4 : 0) | (inertial ? 2 : 0) | (stats ? 1 : 0);      \
        switch (sel) {                                                               \
        case 0: return fn<false, false, false>(__VA_ARGS__);                          \
        case 1: return fn<false, false, true>(__VA_ARGS__);                           \
        case 2: return fn<false, true, false>(__VA_ARGS__);                           \
        case 3: return fn<false, true, true>(__VA_ARGS__);                            \
        case 4: return fn<true, false, false>(__VA_ARGS__);                           \
        case 5: return fn<true, false, true>(__VA_ARGS__);                            \
        case 6: return fn<true, true, false>(__VA_ARGS__);                            \
        default: return fn<true, true, true>(__VA_ARGS__);                            \
        }                                                                            \
    } while (0)

hipError_t launch_step64(const StepParams &P, const State64 &S, const State64 &D,
                         const uint32_t *perm, const Rec64 *rec, double *partials,
                         DevClock *clock, bool stats, bool cubic, bool inertial, int block,
                         int grid, hipStream_t st)
{
    LPT_DISPATCH(launch64_t, P, S, D, perm, rec, partials, clock, block, grid, st);
}

hipError_t launch_step32(const StepParams &P, const State32 &S, const State32 &D,
                         const uint32_t *perm, const float4 *rec, double *partials,
                         DevClock *clock, bool stats, int schemes, bool inertial, int block,
                         int grid, hipStream_t st)
{
    switch (schemes) {
    case kBilinear:
        return launch32_s<kBilinear>(P, S, D, perm, rec, partials, clock, stats, inertial, block,
                                     grid, st);
    case kCatmullRom:
        return launch32_s<kCatmullRom>(P, S, D, perm, rec, partials, clock, stats, inertial,
                                       block, grid, st);
    case kBSpline:
        return launch32_s<kBSpline>(P, S, D, perm, rec, partials, clock, stats, inertial, block,
                                    grid, st);
    case kAnyScheme:
        return launch32_s<kAnyScheme>(P, S, D, perm, rec, partials, clock, stats, inertial,
                                      block, grid, st);
    default:
        return hipErrorInvalidValue;
    }
}
// ===========================================================================
// Statistics: fixed-order merge of the per-wave partials into one record per
// species (Sec. 3.2 and 5.5 quantities).  A wave's partial becomes (count,
// sum dx^2, sum dy^2, mean of r2, M2) with M2 = sum d^2 - (sum d)^2 / count
// the sum of squared deviations of r2 = dx^2 + dy^2 about the wave's mean (d
// is r2 shifted by a sample of the wave; see wave_stats).  Two partials
// merge by the pairwise update of Chan, Golub & LeVeque (1979):
// n = na + nb, delta = mean_b - mean_a, mean = mean_a + delta nb / n,
// M2 = M2a + M2b + delta^2 na nb / n.  Stage 1 merges runs of kFinChunk waves
// of one species per workgroup (sequentially per thread, then a butterfly
// over each wave, then the block's waves in order); stage 2 merges the runs
// of every species at once, one wave per species.  (A single launch whose
// last workgroup merges the runs needs agent-scope fences, whose L2
// write-backs cost more than the second launch.)  Every merge pairs the
// same operands in the same order whatever the scheduling, so the record
// does not depend on it.
// ===========================================================================
constexpr int kFinThreads = 256;
constexpr int kFinPerThread = 4;
constexpr int kFinChunk = kFinThreads * kFinPerThread;   // waves per stage-1 workgroup

struct Moments {
    double n, sx, sy, mean, m2;
};

__device__ __forceinline__ Moments merge_moments(const Moments &a, const Moments &b)
{
    if (b.n == 0.0) return a;
    if (a.n == 0.0) return b;
    const double n = a.n + b.n;
    const double f = b.n / n;
    const double d = b.mean - a.mean;
    return Moments{n, a.sx + b.sx, a.sy + b.sy, a.mean + d * f, a.m2 + b.m2 + d * d * (a.n * f)};
}

__device__ __forceinline__ double shfl_xor_f64(double v, int m)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)b, m);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(b >> 32), m);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Butterfly merge over a wave: at each level a lane pair merges (lower lane,
// higher lane), so both hold the same result; every lane ends with the merge
// of all 64 in a fixed tree order.
__device__ __forceinline__ Moments wave_merge(Moments m)
{
    const int lane = (int)(threadIdx.x & (kWave - 1));
#pragma unroll
    for (int k = 1; k < kWave; k <<= 1) {
        const Moments o{shfl_xor_f64(m.n, k), shfl_xor_f64(m.sx, k), shfl_xor_f64(m.sy, k),
                        shfl_xor_f64(m.mean, k), shfl_xor_f64(m.m2, k)};
        m = (lane & k) ? merge_moments(o, m) : merge_moments(m, o);
    }
    return m;
}

struct FinParams {
    int32_t nspecies;
    int32_t chunk_begin[kMaxSpecies + 1];   // first stage-1 chunk of each species
    int64_t wave_begin[kMaxSpecies];        // first wave partial of each species
    int64_t nwaves[kMaxSpecies];
    int64_t count[kMaxSpecies];
};

// Record of species s from the merged moments (lane 0 of the calling wave).
__device__ __forceinline__ void write_record(const FinParams &F, int s, const Moments &m, double t,
                                             double t0, int64_t idx, double *records, int64_t cap)
{
    if (idx >= cap) return;
    const double nn = (double)F.count[s];
    const double mx = m.sx / nn, my = m.sy / nn;
    const double var = F.count[s] > 1 ? m.m2 / (nn - 1.0) : 0.0;
    const double el = t - t0;
    double *r = records + ((int64_t)s * cap + idx) * 8;
    r[0] = t;
    r[1] = mx;
    r[2] = my;
    r[3] = mx + my;
    r[4] = el > 0.0 ? mx / (2.0 * el) : 0.0;
    r[5] = el > 0.0 ? my / (2.0 * el) : 0.0;
    r[6] = sqrt(var / nn);
    reinterpret_cast<int64_t *>(r)[7] = F.count[s];
}

__global__ __launch_bounds__(kFinThreads) void fin_chunks_kernel(FinParams F,
                                                                 const double *__restrict__ partials,
                                                                 double *__restrict__ chunks)
{
    __shared__ double sm[kFinThreads / kWave][5];
    const int c = blockIdx.x;
    int s = 0;
    while (s + 1 < F.nspecies && c >= F.chunk_begin[s + 1]) ++s;
    const int64_t w0 = (int64_t)(c - F.chunk_begin[s]) * kFinChunk;
    Moments m{0.0, 0.0, 0.0, 0.0, 0.0};
    for (int k = 0; k < kFinPerThread; ++k) {
        const int64_t lw = w0 + (int64_t)threadIdx.x * kFinPerThread + k;   // wave within the species
        if (lw >= F.nwaves[s]) break;
        const int64_t left = F.count[s] - lw * kWave;
        const int cnt = (int)(left < kWave ? (left > 0 ? left : 0) : kWave);
        if (cnt == 0) break;
        const double *q = partials + (int64_t)kStatTerms * (F.wave_begin[s] + lw);
        const double n = (double)cnt;
        const double m2 = fmax(q[3] - q[2] * (q[2] / n), 0.0);
        m = merge_moments(m, Moments{n, q[0], q[1], (q[0] + q[1]) / n, m2});
    }
    m = wave_merge(m);
    const int wv = (int)threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) {
        sm[wv][0] = m.n;
        sm[wv][1] = m.sx;
        sm[wv][2] = m.sy;
        sm[wv][3] = m.mean;
        sm[wv][4] = m.m2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        Moments r{sm[0][0], sm[0][1], sm[0][2], sm[0][3], sm[0][4]};
        for (int k = 1; k < kFinThreads / kWave; ++k)
            r = merge_moments(r, Moments{sm[k][0], sm[k][1], sm[k][2], sm[k][3], sm[k][4]});
        double *o = chunks + 5 * (int64_t)c;
        o[0] = r.n;
        o[1] = r.sx;
        o[2] = r.sy;
        o[3] = r.mean;
        o[4] = r.m2;
    }
}

// One wave per species (blockDim.x = 64 x nspecies): lane l merges the runs
// l, l + 64, ... of its species in order, then the wave's butterfly; lane 0
// writes the record.
__global__ __launch_bounds__(kWave * kMaxSpecies) void fin_records_kernel(
    FinParams F, const double *__restrict__ chunks, DevClock *clock, double *records,
    int64_t cap, double t0)
{
    const double t = clock->t;
    const int64_t idx = clock->nrec;
    const int s = (int)threadIdx.x / kWave, lane = (int)(threadIdx.x & (kWave - 1));
    Moments m{0.0, 0.0, 0.0, 0.0, 0.0};
    for (int c = F.chunk_begin[s] + lane; c < F.chunk_begin[s + 1]; c += kWave) {
        const double *q = chunks + 5 * (int64_t)c;
        m = merge_moments(m, Moments{q[0], q[1], q[2], q[3], q[4]});
    }
    m = wave_merge(m);
    if (lane == 0) write_record(F, s, m, t, t0, idx, records, cap);
    __syncthreads();   // every wave has read the record index
    if (threadIdx.x == 0) clock->nrec = idx + 1;
}

int64_t stat_partials_doubles(const StepParams &P, int block)
{
    const int64_t waves = (int64_t)P.total_blocks * (block / kWave);
    return (int64_t)kStatTerms * waves + 5 * (waves / kFinChunk + P.nspecies + 1);
}

hipError_t launch_finalize(const StepParams &P, double *partials, DevClock *clock,
                           double *records, int64_t rec_cap, double t0, int block,
                           hipStream_t st)
{
    const int wpb = block / kWave;
    FinParams F{};
    F.nspecies = P.nspecies;
    int chunks = 0;
    for (int s = 0; s < P.nspecies; ++s) {
        const SpeciesDev &d = P.sp[s];
        F.chunk_begin[s] = chunks;
        F.wave_begin[s] = (int64_t)d.block_begin * wpb;
        F.nwaves[s] = (int64_t)(d.block_end - d.block_begin) * wpb;
        F.count[s] = d.count;
        chunks += (int)((F.nwaves[s] + kFinChunk - 1) / kFinChunk);
    }
    F.chunk_begin[P.nspecies] = chunks;
    double *chunk_buf = partials + (int64_t)kStatTerms * P.total_blocks * wpb;
    if (chunks > 0)
        hipLaunchKernelGGL(fin_chunks_kernel, dim3(chunks), dim3(kFinThreads), 0, st, F, partials,
                           chunk_buf);
    hipLaunchKernelGGL(fin_records_kernel, dim3(1), dim3(kWave * P.nspecies), 0, st, F, chunk_buf,
                       clock, records, rec_cap, t0);
    return hipGetLastError();
}

// ===========================================================================
// Snapshot ingest: planar u, v of one time level into its half of the padded
// node records (ghost nodes are periodic images).
// ===========================================================================
__device__ __forceinline__ int ghost_source(int a, int n)
{
    int i = a - kGhostLo;
    if (i < 0) i += n;
    if (i >= n) i -= n;
    return i;
}

// Block-wide maximum of m folded into *out with an unsigned max on the
// binary32 bit pattern (non-negative floats order like their bits).  The
// atomic is skipped when *out already holds at least m: *out only grows, so
// a stale read can only cause an unneeded atomic, never a missed one (with a
// thousand blocks on one address the atomics are what costs).  Every thread
// of the block must call it.
__device__ __forceinline__ void block_max_to(float m, unsigned *out)
{
    __shared__ float red[kMaxBlock / kWave];
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, kWave));
    if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < (int)(blockDim.x / kWave); ++k) m = fmaxf(m, red[k]);
        const unsigned bits = __float_as_uint(m);
        if (bits > __atomic_load_n(out, __ATOMIC_RELAXED)) atomicMax(out, bits);
    }
}

// Grid centred differences of psi (eq. particle_velocity_reconstruction with
// the interpolation moved onto the grid): periodic neighbours.
__device__ __forceinline__ int nxt(int i, int n) { return i + 1 == n ? 0 : i + 1; }
__device__ __forceinline__ int prv(int i, int n) { return i == 0 ? n - 1 : i - 1; }

// One ingest pass: each node record's half for this level (ghost records
// are periodic images), and the level's largest |u| or |v| times vscale
// (cells per unit time), which the step kernel's LDS tile halo uses, folded
// into *umax.  PSI: the level is a stream function f = psi, and the node's
// velocity is its grid centred difference, u = (psi(j+1) - psi(j-1)) / 2h,
// v = -(psi(i+1) - psi(i-1)) / 2h, formed here (g is unused); else f = u,
// g = v.  Blocks walk columns a of the padded grid and stride over its rows,
// so the grid stays at about a thousand blocks (one atomic each); each
// thread issues the loads of kRows rows before it stores any of them.
template <bool FP64, bool PSI>
__global__ __launch_bounds__(256) void pack_kernel(void *rec, int slot, const double *__restrict__ f,
                                                   const double *__restrict__ g, int n,
                                                   double scale, double vscale, double inv2h,
                                                   unsigned *umax)
{
    constexpr int kRows = 4;
    const int pitch = n + kGhostLo + kGhostHi;
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    const int G = gridDim.y;
    float m = 0.0f;
    if (a < pitch) {
        const int i = ghost_source(a, n);
        for (int b0 = blockIdx.y; b0 < pitch; b0 += kRows * G) {
            double uu[kRows], vv[kRows];
#pragma unroll
            for (int k = 0; k < kRows; ++k) {
                const int b = b0 + k * G;
                uu[k] = vv[k] = 0.0;
                if (b < pitch) {
                    const int j = ghost_source(b, n);
                    if constexpr (PSI) {
                        uu[k] = (f[(int64_t)nxt(j, n) * n + i] - f[(int64_t)prv(j, n) * n + i]) * inv2h;
                        vv[k] = -(f[(int64_t)j * n + nxt(i, n)] - f[(int64_t)j * n + prv(i, n)]) * inv2h;
                    } else {
                        uu[k] = f[(int64_t)j * n + i];
                        vv[k] = g[(int64_t)j * n + i];
                    }
                }
            }
#pragma unroll
            for (int k = 0; k < kRows; ++k) {
                const int b = b0 + k * G;
                if (b >= pitch) break;
                const int64_t r = (int64_t)b * pitch + a;
                if constexpr (FP64)
                    reinterpret_cast<double2 *>(static_cast<Rec64 *>(rec) + r)[slot] =
                        make_double2(uu[k], vv[k]);
                else
                    reinterpret_cast<float2 *>(static_cast<float4 *>(rec) + r)[slot] =
                        make_float2((float)(uu[k] * scale), (float)(vv[k] * scale));
                m = fmaxf(m, (float)(fmax(fabs(uu[k]), fabs(vv[k])) * vscale));
            }
        }
    }
    block_max_to(m, umax);
}

template <bool PSI>
static void launch_pack_t(void *rec, bool fp64, int slot, const double *f, const double *g, int n,
                          double scale, double vscale, double inv2h, float *umax, hipStream_t st)
{
    const int pitch = n + kGhostLo + kGhostHi, b = 256;
    const dim3 grid((pitch + b - 1) / b, pitch < 128 ? pitch : 128);
    unsigned *out = reinterpret_cast<unsigned *>(umax);
    if (fp64)
        hipLaunchKernelGGL((pack_kernel<true, PSI>), grid, dim3(b), 0, st, rec, slot, f, g, n, scale,
                           vscale, inv2h, out);
    else
        hipLaunchKernelGGL((pack_kernel<false, PSI>), grid, dim3(b), 0, st, rec, slot, f, g, n,
                           scale, vscale, inv2h, out);
}

hipError_t launch_pack(void *rec, bool fp64, int slot, const double *u, const double *v, int n,
                       double scale, double vscale, float *umax, hipStream_t st)
{
    launch_pack_t<false>(rec, fp64, slot, u, v, n, scale, vscale, 0.0, umax, st);
    return hipGetLastError();
}

hipError_t launch_pack_psi(void *rec, bool fp64, int slot, const double *psi, int n, double h,
                           double scale, double vscale, float *umax, hipStream_t st)
{
    launch_pack_t<true>(rec, fp64, slot, psi, nullptr, n, scale, vscale, 1.0 / (2.0 * h), umax,
                        st);
    return hipGetLastError();
}

// ===========================================================================
// Initial state.  Positions come from x0 (original order); the velocity of an
// inertial species is taken from the field or from v0.
// ===========================================================================
__device__ __forceinline__ int smode_of(double wa, double wb)
{
    return wb == 0.0 && wa == 1.0 ? kSlot0 : (wa == 0.0 && wb == 1.0 ? kSlot1 : kBlend);
}

__global__ void init64_kernel(StepParams P, State64 S, const double2 *__restrict__ x0,
                              const double2 *__restrict__ v0, const Rec64 *__restrict__ rec,
                              int species, int64_t begin, int64_t count, double wa, double wb,
                              int vel_from_field)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= count) return;
    const int64_t p = begin + k;
    const SpeciesDev &sp = P.sp[species];
    const double2 x = x0[p];
    S.pos[p] = make_double2(wrap_pos(x.x, P.L), wrap_pos(x.y, P.L));
    S.disp[p] = make_double2(0.0, 0.0);
    S.id[p] = (uint32_t)p;
    if (sp.inertial) {
        if (vel_from_field) {
            double u, v;
            vel64<true>(rec + P.pitch + 1, nullptr, no_tile(), P, sp.scheme, x.x, x.y, wa, wb, smode_of(wa, wb), u, v);
            S.vel[p] = make_double2(u, v);
        } else {
            S.vel[p] = v0[p];
        }
    }
}

__global__ void init32_kernel(StepParams P, State32 S, const double2 *__restrict__ x0,
                              const double2 *__restrict__ v0, const float4 *__restrict__ rec,
                              int species, int64_t begin, int64_t count, double wa, double wb,
                              int vel_from_field)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= count) return;
    const int64_t p = begin + k;
    const SpeciesDev &sp = P.sp[species];
    const double2 x = x0[p];
    int cx, cy;
    float ox, oy;
    split_of(x.x, P, cx, ox);
    split_of(x.y, P, cy, oy);
    S.uc[p] = make_int2(cx, cy);
    S.off[p] = make_float2(ox, oy);
    S.id[p] = (uint32_t)p;
    if (sp.inertial) {
        if (vel_from_field) {
            float u, v;
            vel32<true>(rec + P.pitch + 1, nullptr, no_tile(), P, sp.scheme, cx, cy, ox, oy, (float)wa, (float)wb,
                        smode_of(wa, wb), u, v);
            S.vel[p] = make_float2(u, v);
        } else {
            S.vel[p] = make_float2((float)(v0[p].x * P.invh), (float)(v0[p].y * P.invh));
        }
    }
}

hipError_t launch_init64(const StepParams &P, const State64 &S, const double2 *x0,
                         const double2 *v0, const Rec64 *rec, int species, int64_t begin,
                         int64_t count, double wa, double wb, int vel_from_field,
                         hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    const int b = 256;
    hipLaunchKernelGGL(init64_kernel, dim3((unsigned)((count + b - 1) / b)), dim3(b), 0, st, P,
                       S, x0, v0, rec, species, begin, count, wa, wb, vel_from_field);
    return hipGetLastError();
}

hipError_t launch_init32(const StepParams &P, const State32 &S, const double2 *x0,
                         const double2 *v0, const float4 *rec, int species, int64_t begin,
                         int64_t count, double wa, double wb, int vel_from_field,
                         hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    const int b = 256;
    hipLaunchKernelGGL(init32_kernel, dim3((unsigned)((count + b - 1) / b)), dim3(b), 0, st, P,
                       S, x0, v0, rec, species, begin, count, wa, wb, vel_from_field);
    return hipGetLastError();
}

__global__ void interleave_kernel(double2 *dst, const double *__restrict__ a,
                                  const double *__restrict__ b, int64_t n)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) dst[k] = make_double2(a[k], b[k]);
}

hipError_t launch_interleave(double2 *dst, const double *a, const double *b, int64_t n,
                             hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const int bs = 256;
    hipLaunchKernelGGL(interleave_kernel, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, st,
                       dst, a, b, n);
    return hipGetLastError();
}

__global__ void splitmix_kernel(double2 *x0, int64_t count, uint64_t seed, double L)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= count) return;
    x0[k] = draw_x0(seed, (uint64_t)k, L);
}

hipError_t launch_splitmix(double2 *x0, int64_t count, uint64_t seed, double L, hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    const int b = 256;
    hipLaunchKernelGGL(splitmix_kernel, dim3((unsigned)((count + b - 1) / b)), dim3(b), 0, st,
                       x0, count, seed, L);
    return hipGetLastError();
}

// ===========================================================================
// Velocity probe at arbitrary points (verification entry point).
// ===========================================================================
__global__ void interp64_kernel(StepParams P, const Rec64 *__restrict__ rec, int scheme,
                                int64_t npts, const double *__restrict__ x,
                                const double *__restrict__ y, double wa, double wb, double *u,
                                double *v)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= npts) return;
    double uu, vv;
    vel64<true>(rec + P.pitch + 1, nullptr, no_tile(), P, scheme, x[k], y[k], wa, wb, smode_of(wa, wb), uu, vv);
    u[k] = uu;
    v[k] = vv;
}

__global__ void interp32_kernel(StepParams P, const float4 *__restrict__ rec, int scheme,
                                int64_t npts, const double *__restrict__ x,
                                const double *__restrict__ y, double wa, double wb, double *u,
                                double *v)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= npts) return;
    int cx, cy;
    float ox, oy;
    split_of(x[k], P, cx, ox);
    split_of(y[k], P, cy, oy);
    float uu, vv;
    vel32<true>(rec + P.pitch + 1, nullptr, no_tile(), P, scheme, cx, cy, ox, oy, (float)wa, (float)wb,
                smode_of(wa, wb), uu, vv);
    u[k] = (double)uu * P.h;
    v[k] = (double)vv * P.h;
}

hipError_t launch_interp64(const StepParams &P, const Rec64 *rec, int scheme, int64_t npts,
                           const double *x, const double *y, double wa, double wb, double *u,
                           double *v, hipStream_t st)
{
    if (npts <= 0) return hipSuccess;
    const int b = 256;
    hipLaunchKernelGGL(interp64_kernel, dim3((unsigned)((npts + b - 1) / b)), dim3(b), 0, st, P,
                       rec, scheme, npts, x, y, wa, wb, u, v);
    return hipGetLastError();
}

hipError_t launch_interp32(const StepParams &P, const float4 *rec, int scheme, int64_t npts,
                           const double *x, const double *y, double wa, double wb, double *u,
                           double *v, hipStream_t st)
{
    if (npts <= 0) return hipSuccess;
    const int b = 256;
    hipLaunchKernelGGL(interp32_kernel, dim3((unsigned)((npts + b - 1) / b)), dim3(b), 0, st, P,
                       rec, scheme, npts, x, y, wa, wb, u, v);
    return hipGetLastError();
}

// ===========================================================================
// Readout in original particle order.
// ===========================================================================
__global__ void readout64_kernel(State64 S, const double2 *__restrict__ x0, int64_t offset,
                                 int64_t count, double *xw, double *yw, double *xu, double *yu,
                                 double *vx, double *vy)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= count) return;
    const int64_t p = offset + k;
    const uint32_t g = S.id[p];
    const int64_t q = (int64_t)g - offset;
    if (q < 0 || q >= count) return;
    const double2 x = S.pos[p];
    if (xw) xw[q] = x.x;
    if (yw) yw[q] = x.y;
    if (xu || yu) {
        const double2 d = S.disp[p];
        const double2 a = x0[g];
        if (xu) xu[q] = a.x + d.x;
        if (yu) yu[q] = a.y + d.y;
    }
    if (vx || vy) {
        const double2 w = S.vel[p];
        if (vx) vx[q] = w.x;
        if (vy) vy[q] = w.y;
    }
}

__global__ void readout32_kernel(StepParams P, State32 S, int64_t offset, int64_t count,
                                 double *xw, double *yw, double *xu, double *yu, double *vx,
                                 double *vy)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= count) return;
    const int64_t p = offset + k;
    const uint32_t g = S.id[p];
    const int64_t q = (int64_t)g - offset;
    if (q < 0 || q >= count) return;
    const int2 u = S.uc[p];
    const float2 o = S.off[p];
    if (xw) xw[q] = ((double)wrap_cell(u.x, P.n, P.mask) + (double)o.x) * P.h;
    if (yw) yw[q] = ((double)wrap_cell(u.y, P.n, P.mask) + (double)o.y) * P.h;
    if (xu || yu) {
        const double2 a = S.x0[g];
        const double2 d = split_disp(u, o, a, P);
        if (xu) xu[q] = a.x + d.x;
        if (yu) yu[q] = a.y + d.y;
    }
    if (vx || vy) {
        const float2 w = S.vel[p];
        if (vx) vx[q] = (double)w.x * P.h;
        if (vy) vy[q] = (double)w.y * P.h;
    }
}

hipError_t launch_readout64(const State64 &S, const double2 *x0, int64_t offset, int64_t count,
                            double L, double *xw, double *yw, double *xu, double *yu,
                            double *vx, double *vy, hipStream_t st)
{
    (void)L;
    if (count <= 0) return hipSuccess;
    const int b = 256;
    hipLaunchKernelGGL(readout64_kernel, dim3((unsigned)((count + b - 1) / b)), dim3(b), 0, st,
                       S, x0, offset, count, xw, yw, xu, yu, vx, vy);
    return hipGetLastError();
}

hipError_t launch_readout32(const StepParams &P, const State32 &S, int64_t offset, int64_t count,
                            double *xw, double *yw, double *xu, double *yu, double *vx,
                            double *vy, hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    const int b = 256;
    hipLaunchKernelGGL(readout32_kernel, dim3((unsigned)((count + b - 1) / b)), dim3(b), 0, st,
                       P, S, offset, count, xw, yw, xu, yu, vx, vy);
    return hipGetLastError();
}

}  // namespace lpt
