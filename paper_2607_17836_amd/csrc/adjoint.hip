// gfx950 kernels of the reverse-mode derivatives of the FP64 tracer step.
//
// The paper has no adjoint; these are the derivatives of the discrete map the
// step kernel computes (eq. rk4_update with the spatial interpolation of
// Sec. 3.4 and the temporal interpolation of eq. temporal_interp), for
// finite-time Lyapunov exponents (dx_T/dx_0) and for gradients of a scalar
// loss with respect to the gridded velocity.  Inside a cell the cell index
// is constant, so d(xi)/dx = n/L; across a cell edge bilinear interpolation
// is only continuous, and its derivative is the one-sided one of the cell
// that holds the point.
//
// One thread carries one particle's adjoint vector(s) backwards through one
// step: it recomputes the four stage points from the step's start position
// (read from the segment tape), then applies the chain rule through the RK4
// combine, the stage states and the interpolation.  Grid gradients are
// scatter-added: by default with FP64 atomics (summation order, hence the
// last bits, depends on scheduling); in the deterministic mode as exact
// fixed-point integers (value = hi 2^-32 + lo 2^-64, each contribution
// rounded once to a multiple of 2^-64), whose sums do not depend on the
// order of the additions.
#include "field_dev.h"

namespace lpt {

struct Loc64 {
    int i, j;          // periodic cell
    double xi, eta;    // in-cell coordinates
};

__device__ __forceinline__ Loc64 locate64(const StepParams &P, double x, double y)
{
    const double sx = x * P.invh, sy = y * P.invh;
    const double fx = floor(sx), fy = floor(sy);
    Loc64 l;
    l.xi = sx - fx;
    l.eta = sy - fy;
    l.i = cell_of_floor(fx, P.n, P.mask);
    l.j = cell_of_floor(fy, P.n, P.mask);
    return l;
}

// Derivatives of the Catmull-Rom and B-spline kernels in s.
__device__ __forceinline__ void dweights_cr(double s, double w[4])
{
    w[0] = -0.5 + s * (2.0 - 1.5 * s);
    w[1] = s * (-5.0 + 4.5 * s);
    w[2] = 0.5 + s * (4.0 - 4.5 * s);
    w[3] = s * (-1.0 + 1.5 * s);
}

__device__ __forceinline__ void dweights_bs(double s, double w[4])
{
    const double r = 1.0 - s;
    w[0] = -0.5 * r * r;
    w[1] = s * (1.5 * s - 2.0);
    w[2] = 0.5 + s * (1.0 - 1.5 * s);
    w[3] = 0.5 * s * s;
}

// Stencil of the point: K x K nodes starting at (i0, j0) (K = 2 bilinear,
// 4 bicubic), with 1D weights and their derivatives per axis.  K is a
// compile-time size, so the arrays stay in registers.
template <int K>
struct Sten64 {
    int i0, j0;
    double wx[K], wy[K], dx[K], dy[K];
};

// Whether the point's stencil is bilinear (the scheme, or the paper's
// bilinear fallback near the grid edge).
__device__ __forceinline__ bool bilinear_at(const StepParams &P, int scheme, const Loc64 &l)
{
    return scheme == kBilinear || edge_cell(P.compat_edge, l.i, l.j, P.n);
}

template <int K>
__device__ __forceinline__ Sten64<K> stencil64(int scheme, const Loc64 &l)
{
    Sten64<K> s;
    if constexpr (K == 2) {
        s.i0 = l.i;
        s.j0 = l.j;
        s.wx[0] = 1.0 - l.xi;
        s.wx[1] = l.xi;
        s.wy[0] = 1.0 - l.eta;
        s.wy[1] = l.eta;
        s.dx[0] = -1.0;
        s.dx[1] = 1.0;
        s.dy[0] = -1.0;
        s.dy[1] = 1.0;
    } else {
        s.i0 = l.i - 1;
        s.j0 = l.j - 1;
        if (scheme == kCatmullRom) {
            weights_cr(l.xi, s.wx);
            weights_cr(l.eta, s.wy);
            dweights_cr(l.xi, s.dx);
            dweights_cr(l.eta, s.dy);
        } else {
            weights_bs(l.xi, s.wx);
            weights_bs(l.eta, s.wy);
            dweights_bs(l.xi, s.dx);
            dweights_bs(l.eta, s.dy);
        }
    }
    return s;
}

// Spatial Jacobian J = [du/dx, du/dy, dv/dx, dv/dy] of the time-blended
// interpolated velocity at a stencil, its K x K nodes read through N (the
// LDS tile or the ghost-bordered records, so the stencil never wraps).
template <int K, typename Nodes>
__device__ __forceinline__ void jacobian_nodes(const Nodes &N, const StepParams &P,
                                               const Sten64<K> &s, double wa, double wb,
                                               int smode, double J[4])
{
    double ux = 0.0, uy = 0.0, vx = 0.0, vy = 0.0;
#pragma unroll
    for (int b = 0; b < K; ++b) {
        double rux = 0.0, rvx = 0.0, ru = 0.0, rv = 0.0;
#pragma unroll
        for (int a = 0; a < K; ++a) {
            double u, v;
            N.get(a, b, smode, wa, wb, u, v);
            rux += s.dx[a] * u;
            rvx += s.dx[a] * v;
            ru += s.wx[a] * u;
            rv += s.wx[a] * v;
        }
        ux += s.wy[b] * rux;
        vx += s.wy[b] * rvx;
        uy += s.dy[b] * ru;
        vy += s.dy[b] * rv;
    }
    J[0] = ux * P.invh;
    J[1] = uy * P.invh;
    J[2] = vx * P.invh;
    J[3] = vy * P.invh;
}

// The Jacobian from the block's LDS tile when the stencil lies inside it,
// else from global memory.
template <int K>
__device__ __forceinline__ void jacobian64(const Rec64 *__restrict__ rec0, const double2 *tile,
                                           const Tile &T, const StepParams &P, const Sten64<K> &s,
                                           double wa, double wb, int smode, double J[4])
{
    int t;
    if (tile_index(T, s.i0, s.j0, K, P.n, P.mask, t))
        jacobian_nodes<K>(TileNodes64{tile + t, T.w, T.w * T.h}, P, s, wa, wb, smode, J);
    else
        jacobian_nodes<K>(RecNodes64{rec0 + (__mul24(s.j0, P.pitch) + s.i0), P.pitch}, P, s, wa,
                          wb, smode, J);
}

// Exact fixed-point form of a contribution c (|c| < 2^31): c ~ hi 2^-32 +
// lo 2^-64 with hi = floor(c 2^32) and 0 <= lo < 2^32 the next 32 bits
// (truncated).  The scaling by 2^32 and the fractional part are exact in
// binary64, so the pair depends on c alone; sums of pairs are integer sums
// (hi in two's complement, lo unsigned), exact and order-independent.
__device__ __forceinline__ void to_fixed(double c, unsigned long long &hi, unsigned long long &lo)
{
    const double f = c * 0x1p32;
    const double h = floor(f);
    hi = (unsigned long long)(long long)h;
    lo = (unsigned long long)((f - h) * 0x1p32);
}

__device__ __forceinline__ void add_fixed(unsigned long long *pair, double c)
{
    unsigned long long hi, lo;
    to_fixed(c, hi, lo);
    atomicAdd(pair, hi);
    atomicAdd(pair + 1, lo);
}

// Accumulator of dL/d(grid) for one block.  gU in global memory is laid out
// [slot][u, v][n * n]: doubles, or (DET) pairs of 64-bit fixed-point words.
// The block's box B of nodes in LDS holds
//   - by default, planes of the stencil weights times the adjoint stage
//     vector per RK4 time level (g = 0: the first stage, 1: the two middle
//     stages, which share a time, 2: the last), u then v: the two slots'
//     temporal weights are applied once per node when the box is flushed;
//   - DET: fixed-point pairs of the four (slot, component) planes.
template <bool DET>
struct GridGrad {
    void *gU;
    void *acc;   // LDS planes, used when B.on
    Tile B;
};

// The grid gradient of one stage's stencil, K x K nodes: node weight w times
// the stage's adjoint vector (lx, ly), times the temporal weight of each slot.
template <int K, bool DET>
__device__ __forceinline__ void scatter64(const GridGrad<DET> &G, const StepParams &P,
                                          const Sten64<K> &s, int grp, double wa, double wb,
                                          double lx, double ly)
{
    const int n = P.n;
    const int64_t nn = (int64_t)n * n;
    const int area = G.B.w * G.B.h;
    const double wt[2] = {wa, wb};
#pragma unroll
    for (int b = 0; b < K; ++b) {
        const int j = wrap_cell(s.j0 + b, n, P.mask);
        int ry = j - G.B.y0;
        ry += ry < 0 ? n : 0;
#pragma unroll
        for (int a = 0; a < K; ++a) {
            const int i = wrap_cell(s.i0 + a, n, P.mask);
            int rx = i - G.B.x0;
            rx += rx < 0 ? n : 0;
            const double w = s.wx[a] * s.wy[b];
            const bool local = G.B.on && rx < G.B.w && ry < G.B.h;
            const int k = ry * G.B.w + rx;
            if (local && !DET) {
                double *acc = static_cast<double *>(G.acc);
                atomicAdd(acc + (2 * grp) * area + k, w * lx);
                atomicAdd(acc + (2 * grp + 1) * area + k, w * ly);
                continue;
            }
#pragma unroll
            for (int sl = 0; sl < 2; ++sl) {
                const double c = wt[sl] * w;
                if (c == 0.0) continue;
                if constexpr (DET) {
                    unsigned long long *q =
                        local ? static_cast<unsigned long long *>(G.acc) + 2 * ((2 * sl) * area + k)
                              : static_cast<unsigned long long *>(G.gU) +
                                    2 * ((2 * sl) * nn + (int64_t)j * n + i);
                    const int64_t pl = local ? area : nn;   // plane stride
                    add_fixed(q, c * lx);
                    add_fixed(q + 2 * pl, c * ly);
                } else {
                    double *g = static_cast<double *>(G.gU);
                    const int64_t kk = (int64_t)j * n + i;
                    atomicAdd(g + (2 * sl) * nn + kk, c * lx);
                    atomicAdd(g + (2 * sl + 1) * nn + kk, c * ly);
                }
            }
        }
    }
}

__device__ __forceinline__ void add_jt(const double J[4], const double l[2], double out[2])
{
    out[0] = J[0] * l[0] + J[2] * l[1];
    out[1] = J[1] * l[0] + J[3] * l[1];
}

// Recompute one step of every particle's position: out = wrap(in + step),
// with the step kernel's LDS field tile of the block's box.
template <bool CUBIC>
__global__ __launch_bounds__(kMaxBlock) void recompute64_kernel(StepParams P,
                                                                const Rec64 *__restrict__ rec,
                                                                const double2 *__restrict__ in,
                                                                double2 *__restrict__ out)
{
    const int lb = blockIdx.x;
    const SpeciesDev &sp = P.sp[species_of(P, lb)];
    const int64_t base = (int64_t)(lb - sp.block_begin) * blockDim.x;
    const int64_t local = base + threadIdx.x;
    const bool active = local < sp.count;
    const int64_t p = sp.offset + local;
    const Rec64 *rec0 = rec + P.pitch + 1;
    const double2 x = active ? in[p] : make_double2(0.0, 0.0);
    Tile T = no_tile();
    if (P.tile_cap > 0) {
        const double2 a = in[sp.offset + base];
        const int n = P.n, mask = P.mask;
        const int ax = cell_of_floor(floor(a.x * P.invh), n, mask);
        const int ay = cell_of_floor(floor(a.y * P.invh), n, mask);
        const int cx = cell_of_floor(floor(x.x * P.invh), n, mask);
        const int cy = cell_of_floor(floor(x.y * P.invh), n, mask);
        int lo, hi;
        stencil_reach(sp.scheme, lo, hi);
        const int H = step_halo(P, sp.scheme, (float)P.dt);
        const int64_t left = sp.count - base;
        T = stage_tile<Rec64>(reinterpret_cast<Rec64 *>(lpt_dyn_lds), rec0, P, active, cx, cy, ax,
                              ay, lo + H, hi + H,
                              (int)(left < (int64_t)blockDim.x ? left : blockDim.x));
    }
    if (!active) return;
    const double2 *planes = reinterpret_cast<const double2 *>(lpt_dyn_lds);
    double ddx, ddy;
    if (!CUBIC || sp.scheme == kBilinear)
        rk4_tracer64<false>(rec0, planes, T, P, sp.scheme, x, ddx, ddy);
    else
        rk4_tracer64<true>(rec0, planes, T, P, sp.scheme, x, ddx, ddy);
    out[p] = make_double2(wrap_pos(x.x + ddx, P.L), wrap_pos(x.y + ddy, P.L));
}

// One reverse step.  lam holds NL adjoint vectors per particle
// (lam[p * NL + r]); gU (may be null) receives the grid gradient of the
// first one.  With AGG, the block first sums its contributions in an LDS box
// of the grid (its particles' cells widened by the step's displacement
// bound and the stencil reach; acc_cap nodes of LDS) and then adds the box
// to gU with one atomic per nonzero entry; contributions outside the box
// (particles faster than the bound, or a box beyond the LDS budget, which is
// trimmed) go to gU directly.  DET: gU holds fixed-point pairs (see
// to_fixed), and so does the box.
extern __shared__ __align__(32) unsigned char adj_dyn_lds[];

template <int NL, bool AGG, bool CUBIC, bool DET>
__global__ __launch_bounds__(kMaxBlock) void adjoint64_kernel(StepParams P,
                                                              const Rec64 *__restrict__ rec,
                                                              const double2 *__restrict__ tape,
                                                              double2 *__restrict__ lam,
                                                              void *gU, int lds_bytes)
{
    const int lb = blockIdx.x;
    const SpeciesDev &sp = P.sp[species_of(P, lb)];
    const int64_t base = (int64_t)(lb - sp.block_begin) * blockDim.x;
    const int64_t local = base + threadIdx.x;
    const bool active = local < sp.count;
    const int64_t p = sp.offset + local;
    const Rec64 *rec0 = rec + P.pitch + 1;
    const int scheme = sp.scheme;
    const double dt = P.dt, hdt = 0.5 * P.dt, dt6 = P.dt / 6.0, dt3 = P.dt / 3.0;
    const double2 x = active ? tape[p] : make_double2(0.0, 0.0);
    // LDS per box node: the field tile's two planes of (u, v) (32 bytes, when
    // tiles are on), then the accumulators: three time levels x (u, v)
    // doubles, or (DET) four (slot, component) planes of fixed-point pairs
    // The box is sized for the accumulators (the scatter's atomics are what
    // an oversized box sends to global memory); the tile is staged beside
    // them only where both fit.
    constexpr int kAccBytes = AGG ? (DET ? 64 : 48) : 0;
    const bool tiles_on = P.tile_cap > 0;
    const int box_bytes = AGG ? kAccBytes : (tiles_on ? 32 : 0);

    GridGrad<DET> G{gU, adj_dyn_lds, no_tile()};
    Tile T = no_tile();
    const double2 *planes = reinterpret_cast<const double2 *>(adj_dyn_lds);
    if (box_bytes > 0) {
        const int cap = lds_bytes / box_bytes;
        const Loc64 me = locate64(P, x.x, x.y);
        const double2 a0 = tape[sp.offset + base];
        const Loc64 an = locate64(P, a0.x, a0.y);
        int lo, hi;
        stencil_reach(scheme, lo, hi);
        const int H = step_halo(P, scheme, (float)dt);
        Tile B = block_box(active, me.i, me.j, an.i, an.j, P.n, P.mask, lo + H, hi + H);
        // a box beyond the LDS budget first loses halo, then rows: whatever
        // falls outside it is read and added in global memory directly
        int shrink = 0;
        while (shrink < H && (B.w - 2 * shrink) * (B.h - 2 * shrink) > cap) ++shrink;
        B.w -= 2 * shrink;
        B.h -= 2 * shrink;
        B.x0 = wrap_cell(B.x0 + shrink, P.n, P.mask);
        B.y0 = wrap_cell(B.y0 + shrink, P.n, P.mask);
        B.w = min(min(B.w, cap), P.n - 1);
        B.h = min(min(B.h, cap / B.w), P.n - 1);
        B.on = 1;
        const int area = B.w * B.h;
        const bool tiled = tiles_on && area * (32 + kAccBytes) <= lds_bytes;
        if (tiled) {
            T = B;
            fill_tile_dma<Rec64>(reinterpret_cast<Rec64 *>(adj_dyn_lds), rec0, P, T);
        }
        if constexpr (AGG) {
            G.B = B;
            G.acc = adj_dyn_lds + (tiled ? 32 * area : 0);
            const int words = (kAccBytes / 8) * area;
            if constexpr (DET) {
                unsigned long long *acc = static_cast<unsigned long long *>(G.acc);
                for (int k = threadIdx.x; k < words; k += blockDim.x) acc[k] = 0ull;
            } else {
                double *acc = static_cast<double *>(G.acc);
                for (int k = threadIdx.x; k < words; k += blockDim.x) acc[k] = 0.0;
            }
        }
        __syncthreads();
    }

    if (active) {
        // forward recomputation of the stage points, exactly as the step kernel
        double px[4], py[4];
        double k1x, k1y, k2x, k2y, k3x, k3y;
        px[0] = x.x;
        py[0] = x.y;
        vel64<CUBIC>(rec0, planes, T, P, scheme, px[0], py[0], P.wa[0], P.wb[0], P.smode[0],
                     k1x, k1y);
        px[1] = x.x + hdt * k1x;
        py[1] = x.y + hdt * k1y;
        vel64<CUBIC>(rec0, planes, T, P, scheme, px[1], py[1], P.wa[1], P.wb[1], P.smode[1],
                     k2x, k2y);
        px[2] = x.x + hdt * k2x;
        py[2] = x.y + hdt * k2y;
        vel64<CUBIC>(rec0, planes, T, P, scheme, px[2], py[2], P.wa[2], P.wb[2], P.smode[2],
                     k3x, k3y);
        px[3] = x.x + dt * k3x;
        py[3] = x.y + dt * k3y;

        // Back through x' = x + dt/6 (k1 + 2 k2 + 2 k3 + k4), k_q = U(x_q),
        // x_q = x + c_q dt k_(q-1) (c = 1/2, 1/2, 1): per adjoint vector r,
        // lx[r] collects dL/dx and lk[r][q] the adjoint of k_q; the stages are
        // taken newest first, one stencil at a time.
        double lx[NL][2], lk[NL][4][2];
#pragma unroll
        for (int r = 0; r < NL; ++r) {
            const double2 l = lam[p * NL + r];
            lx[r][0] = l.x;
            lx[r][1] = l.y;
            lk[r][0][0] = dt6 * l.x;
            lk[r][0][1] = dt6 * l.y;
            lk[r][1][0] = dt3 * l.x;
            lk[r][1][1] = dt3 * l.y;
            lk[r][2][0] = dt3 * l.x;
            lk[r][2][1] = dt3 * l.y;
            lk[r][3][0] = dt6 * l.x;
            lk[r][3][1] = dt6 * l.y;
        }
        const bool grid = gU != nullptr;
        const double back[4] = {0.0, hdt, hdt, dt};   // c_q dt
#pragma unroll
        for (int q = 3; q >= 0; --q) {
            const Loc64 loc = locate64(P, px[q], py[q]);
            const int grp = q == 0 ? 0 : (q == 3 ? 2 : 1);   // time level of the stage
            double J[4];
            if (!CUBIC || bilinear_at(P, scheme, loc)) {
                const Sten64<2> st = stencil64<2>(scheme, loc);
                if (grid)
                    scatter64<2, DET>(G, P, st, grp, P.wa[q], P.wb[q], lk[0][q][0], lk[0][q][1]);
                jacobian64<2>(rec0, planes, T, P, st, P.wa[q], P.wb[q], P.smode[q], J);
            } else if constexpr (CUBIC) {
                const Sten64<4> st = stencil64<4>(scheme, loc);
                if (grid)
                    scatter64<4, DET>(G, P, st, grp, P.wa[q], P.wb[q], lk[0][q][0], lk[0][q][1]);
                jacobian64<4>(rec0, planes, T, P, st, P.wa[q], P.wb[q], P.smode[q], J);
            }
#pragma unroll
            for (int r = 0; r < NL; ++r) {
                double ls[2];
                add_jt(J, lk[r][q], ls);
                lx[r][0] += ls[0];
                lx[r][1] += ls[1];
                if (q > 0) {
                    lk[r][q - 1][0] += back[q] * ls[0];
                    lk[r][q - 1][1] += back[q] * ls[1];
                }
            }
        }
#pragma unroll
        for (int r = 0; r < NL; ++r) lam[p * NL + r] = make_double2(lx[r][0], lx[r][1]);
    }

    if constexpr (AGG) {
        __syncthreads();
        const int n = P.n, area = G.B.w * G.B.h;
        const int64_t nn = (int64_t)n * n;
        for (int k = threadIdx.x; k < area; k += blockDim.x) {
            const int ty = k / G.B.w, tx = k - ty * G.B.w;
            int gx = G.B.x0 + tx, gy = G.B.y0 + ty;
            gx -= gx >= n ? n : 0;
            gy -= gy >= n ? n : 0;
            const int64_t g = (int64_t)gy * n + gx;
            if constexpr (DET) {
                const unsigned long long *acc = static_cast<const unsigned long long *>(G.acc);
                unsigned long long *out = static_cast<unsigned long long *>(gU);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const unsigned long long hi = acc[2 * (q * area + k)];
                    const unsigned long long lo = acc[2 * (q * area + k) + 1];
                    if (hi | lo) {
                        atomicAdd(out + 2 * (q * nn + g), hi);
                        atomicAdd(out + 2 * (q * nn + g) + 1, lo);
                    }
                }
            } else {
                const double *acc = static_cast<const double *>(G.acc);
                double *out = static_cast<double *>(gU);
                // time levels 0, 1, 2 were taken at the weights of stages 0, 1, 3
                const double wa[3] = {P.wa[0], P.wa[1], P.wa[3]};
                const double wb[3] = {P.wb[0], P.wb[1], P.wb[3]};
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    double s0 = 0.0, s1 = 0.0;
#pragma unroll
                    for (int g3 = 0; g3 < 3; ++g3) {
                        const double v = acc[(2 * g3 + c) * area + k];
                        s0 += wa[g3] * v;
                        s1 += wb[g3] * v;
                    }
                    if (s0 != 0.0) atomicAdd(out + c * nn + g, s0);
                    if (s1 != 0.0) atomicAdd(out + (2 + c) * nn + g, s1);
                }
            }
        }
    }
}

// lam[p * NL + r] from the caller's per-id seeds: NL == 1: (gx[id], gy[id]);
// NL == 2: the unit vectors (d x_T, d y_T).
__global__ void seed_adjoint_kernel(const uint32_t *__restrict__ id, int64_t np, int nl,
                                    const double *__restrict__ gx, const double *__restrict__ gy,
                                    double2 *lam)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    if (nl == 1) {
        const uint32_t g = id[p];
        lam[p] = make_double2(gx[g], gy[g]);
    } else {
        lam[2 * p] = make_double2(1.0, 0.0);
        lam[2 * p + 1] = make_double2(0.0, 1.0);
    }
}

// Finite-time Lyapunov exponent of one Jacobian F = [[a, b], [c, d]]:
// (1/T) ln sqrt(lambda_max(F^T F)), with the largest eigenvalue of the
// symmetric Cauchy-Green tensor [[p, r], [r, q]] (p = a^2 + c^2,
// q = b^2 + d^2, r = ab + cd) in closed form,
// lambda_max = (p + q)/2 + sqrt(((p - q)/2)^2 + r^2).
__device__ __forceinline__ double ftle_of(double a, double b, double c, double d, double T)
{
    const double p = a * a + c * c, q = b * b + d * d, r = a * b + c * d;
    const double h = 0.5 * (p - q);
    const double lam = 0.5 * (p + q) + sqrt(h * h + r * r);
    return 0.5 * log(lam) / T;
}

// Results back in original (id) order: NL == 1: gx0, gy0; NL == 2: the
// Jacobian F[id] = [[dx/dx0, dx/dy0], [dy/dx0, dy/dy0]] and/or its FTLE over
// the time T (any output may be null).
__global__ void gather_adjoint_kernel(const uint32_t *__restrict__ id, int64_t np, int nl,
                                      const double2 *__restrict__ lam, double *gx, double *gy,
                                      double *F, double *sigma, double T)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const uint32_t g = id[p];
    if (nl == 1) {
        const double2 l = lam[p];
        if (gx) gx[g] = l.x;
        if (gy) gy[g] = l.y;
    } else {
        const double2 r0 = lam[2 * p], r1 = lam[2 * p + 1];
        if (F) {
            F[4 * (int64_t)g + 0] = r0.x;
            F[4 * (int64_t)g + 1] = r0.y;
            F[4 * (int64_t)g + 2] = r1.x;
            F[4 * (int64_t)g + 3] = r1.y;
        }
        if (sigma) sigma[g] = ftle_of(r0.x, r0.y, r1.x, r1.y, T);
    }
}

hipError_t launch_recompute64(const StepParams &P, const Rec64 *rec, const double2 *in,
                              double2 *out, bool cubic, int block, hipStream_t st)
{
    // the step kernel's tile: two planes of 16-byte entries, whole 64-entry chunks
    const size_t lds = P.tile_cap > 0 ? (size_t)(2 * P.tile_cap + kWave) * 16 : 0;
    if (cubic)
        hipLaunchKernelGGL(recompute64_kernel<true>, dim3(P.total_blocks), dim3(block), lds, st, P,
                           rec, in, out);
    else
        hipLaunchKernelGGL(recompute64_kernel<false>, dim3(P.total_blocks), dim3(block), lds, st,
                           P, rec, in, out);
    return hipGetLastError();
}

// LDS of the adjoint kernel: 31 KiB, so that five 256-thread blocks (the
// bilinear kernel's register-bound occupancy) fit in a CU's 160 KiB.  The
// accumulator box holds up to 661 nodes (48 bytes each; 496 of fixed-point
// pairs), and the field tile joins it in boxes of up to 396 nodes (80
// bytes each; 330 with fixed-point pairs); without accumulators, 992 nodes
// of tile.
constexpr int kAdjLdsBytes = 31 * 1024;

template <bool CUBIC, bool DET>
static hipError_t launch_adjoint64_c(const StepParams &P, const Rec64 *rec, const double2 *tape,
                                     double2 *lam, int nl, void *gU, int block, hipStream_t st)
{
    const size_t lds = kAdjLdsBytes + 64;   // the tile fill writes whole 16-byte pieces
    if (nl == 1 && gU)
        hipLaunchKernelGGL((adjoint64_kernel<1, true, CUBIC, DET>), dim3(P.total_blocks),
                           dim3(block), lds, st, P, rec, tape, lam, gU, kAdjLdsBytes);
    else if (nl == 1)
        hipLaunchKernelGGL((adjoint64_kernel<1, false, CUBIC, false>), dim3(P.total_blocks),
                           dim3(block), P.tile_cap > 0 ? lds : 0, st, P, rec, tape, lam,
                           (void *)nullptr, kAdjLdsBytes);
    else
        hipLaunchKernelGGL((adjoint64_kernel<2, false, CUBIC, false>), dim3(P.total_blocks),
                           dim3(block), P.tile_cap > 0 ? lds : 0, st, P, rec, tape, lam,
                           (void *)nullptr, kAdjLdsBytes);
    return hipGetLastError();
}

hipError_t launch_adjoint64(const StepParams &P, const Rec64 *rec, const double2 *tape,
                            double2 *lam, int nl, void *gU, bool det, bool cubic, int block,
                            hipStream_t st)
{
    if (det)
        return cubic ? launch_adjoint64_c<true, true>(P, rec, tape, lam, nl, gU, block, st)
                     : launch_adjoint64_c<false, true>(P, rec, tape, lam, nl, gU, block, st);
    return cubic ? launch_adjoint64_c<true, false>(P, rec, tape, lam, nl, gU, block, st)
                 : launch_adjoint64_c<false, false>(P, rec, tape, lam, nl, gU, block, st);
}

// Fixed-point pairs (hi 2^-32 + lo 2^-64) to binary64, in place order.
__global__ void fixed_to_double_kernel(const unsigned long long *__restrict__ pairs, int64_t count,
                                       double *out)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= count) return;
    const long long hi = (long long)pairs[2 * k];
    const unsigned long long lo = pairs[2 * k + 1];
    out[k] = (double)hi * 0x1p-32 + (double)lo * 0x1p-64;
}

hipError_t launch_fixed_to_double(const void *pairs, int64_t count, double *out, hipStream_t st)
{
    const int b = 256;
    hipLaunchKernelGGL(fixed_to_double_kernel, dim3((unsigned)((count + b - 1) / b)), dim3(b), 0,
                       st, static_cast<const unsigned long long *>(pairs), count, out);
    return hipGetLastError();
}

__global__ void zero_words_kernel(unsigned long long *p, int64_t count)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < count) p[k] = 0ull;
}

hipError_t launch_zero_words(void *p, int64_t words, hipStream_t st)
{
    const int b = 256;
    hipLaunchKernelGGL(zero_words_kernel, dim3((unsigned)((words + b - 1) / b)), dim3(b), 0, st,
                       static_cast<unsigned long long *>(p), words);
    return hipGetLastError();
}

// Adjoint vectors from one segment's slot order to the previous segment's:
// the sort at the segment's start filled slot i from slot perm[i], so
// out[perm[i]] = in[i] (NL vectors per slot).
__global__ void unpermute_adjoint_kernel(const uint32_t *__restrict__ perm, int64_t np, int nl,
                                         const double2 *__restrict__ in, double2 *out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    const int64_t j = perm[i];
    for (int r = 0; r < nl; ++r) out[j * nl + r] = in[i * nl + r];
}

hipError_t launch_unpermute_adjoint(const uint32_t *perm, int64_t np, int nl, const double2 *in,
                                    double2 *out, hipStream_t st)
{
    const int b = 256;
    hipLaunchKernelGGL(unpermute_adjoint_kernel, dim3((unsigned)((np + b - 1) / b)), dim3(b), 0,
                       st, perm, np, nl, in, out);
    return hipGetLastError();
}

hipError_t launch_seed_adjoint(const uint32_t *id, int64_t np, int nl, const double *gx,
                               const double *gy, double2 *lam, hipStream_t st)
{
    const int b = 256;
    hipLaunchKernelGGL(seed_adjoint_kernel, dim3((unsigned)((np + b - 1) / b)), dim3(b), 0, st, id,
                       np, nl, gx, gy, lam);
    return hipGetLastError();
}

hipError_t launch_gather_adjoint(const uint32_t *id, int64_t np, int nl, const double2 *lam,
                                 double *gx, double *gy, double *F, double *sigma, double T,
                                 hipStream_t st)
{
    const int b = 256;
    hipLaunchKernelGGL(gather_adjoint_kernel, dim3((unsigned)((np + b - 1) / b)), dim3(b), 0, st,
                       id, np, nl, lam, gx, gy, F, sigma, T);
    return hipGetLastError();
}

}  // namespace lpt
