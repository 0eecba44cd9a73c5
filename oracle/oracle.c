/*
 * oracle.c -- plain, slow, FP64 CPU oracle of the Lagrangian particle path of
 * "A coupled Eulerian-Lagrangian approach for fluid and particle dynamics"
 * (Maiti & Ganesh).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * loads this file: only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no source, header, table or helper with
 * the HIP library; both sides only consume the same seeded input arrays.
 *
 * Everything is IEEE binary64, one particle at a time, in the order the paper
 * states the algorithm (Alg. "coupled_EL": for each step, for each particle,
 * for each RK4 stage: build the stage state, map it periodically, interpolate
 * both time levels in space, interpolate linearly in time, evaluate the
 * right-hand side; then combine, and store wrapped and unwrapped
 * coordinates).  No blocking, fusion or reordering.  Build flags:
 * -O2 -fno-fast-math -ffp-contract=off (no FMA contraction).  The CPU
 * timing build adds -O3 -march=native -fopenmp: the particle loop of a step
 * then runs on several threads (statistics stay serial), with the same
 * arithmetic per particle.
 *
 * Grid convention (the paper does not state it; this is the reading used
 * throughout): node (i, j) sits at (i*h, j*h), 0 <= i, j < n, h = L/n,
 * stored as f[j*n + i] (x fastest).
 *
 * Parity status of each entry point is listed in its comment and pinned by
 * tests/test_oracle_pins.py.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_BILINEAR 0
#define ORC_CATMULL_ROM 1
#define ORC_BSPLINE 2

#define ORC_TRACER 0
#define ORC_INERTIAL 1

#define ORC_SRC_GRID 0     /* velocity interpolated from gridded u, v      */
#define ORC_SRC_PSI 1      /* stream function interpolated + centred FD    */
#define ORC_SRC_UNIFORM 2  /* analytic uniform flow (U0, V0)               */
#define ORC_SRC_TG 3       /* analytic (oscillating) Taylor-Green flow      */

#define ORC_BRACKET 0      /* snapshot slot 0 at ta, slot 1 at tb           */
#define ORC_PINGPONG 1     /* step n: slot n%2 at t_n, other slot at t_n+dt */

/* Velocity source.  Field arrays are [n*n], x fastest. */
typedef struct orc_flow {
    int32_t source;        /* ORC_SRC_*                                       */
    int32_t scheme;        /* ORC_BILINEAR / ORC_CATMULL_ROM / ORC_BSPLINE     */
    int32_t time_mode;     /* ORC_BRACKET / ORC_PINGPONG                       */
    int32_t compat_edge;   /* 1: bicubic falls back to bilinear near the edge  */
    int32_t n;
    int32_t pad_;
    double length;         /* L; the domain is [0, L)^2                        */
    const double *u[2];    /* ORC_SRC_GRID: u per slot                         */
    const double *v[2];    /* ORC_SRC_GRID: v per slot                         */
    const double *psi[2];  /* ORC_SRC_PSI: psi per slot                        */
    double t_slot[2];      /* ORC_BRACKET: snapshot times                      */
    /* analytic parameters */
    double U0, V0;                          /* uniform flow                    */
    double alpha, k, eps, omega, phi;       /* eq. kinematic_flow             */
} orc_flow;

/* ------------------------------------------------------------------------ */
/* Periodic mapping (Sec. 3.2, 3.5): a coordinate outside the domain is      */
/* moved to the opposite side.  wrap(z) = z - L*floor(z/L), with the          */
/* result forced into [0, L) against rounding.                                */
/* ------------------------------------------------------------------------ */
double orc_wrap(double z, double L)
{
    double w = z - L * floor(z / L);
    if (w < 0.0) w += L;
    if (w >= L) w -= L;
    return w;
}

void orc_wrap_many(int64_t np, const double *z, double L, double *out)
{
    for (int64_t p = 0; p < np; ++p)
        out[p] = orc_wrap(z[p], L);
}

static int32_t imod(int64_t a, int32_t n)
{
    int64_t m = a % n;
    if (m < 0) m += n;
    return (int32_t)m;
}

/* Cell containing the (already wrapped) coordinate xm and the local
 * coordinate xi = (x_p - x_i)/(x_{i+1} - x_i) of eqs. bilinear_local,
 * cr_local and bspline_local. */
static void locate(double xm, int32_t n, double h, int32_t *i, double *xi)
{
    double c = floor(xm / h);
    int64_t ci = (int64_t)c;
    if (ci > n - 1) ci = n - 1;   /* xm/h rounded up to n */
    if (ci < 0) ci = 0;
    double xi_node = (double)ci * h;
    double xi_next = (double)(ci + 1) * h;
    *i = (int32_t)ci;
    *xi = (xm - xi_node) / (xi_next - xi_node);
}

static double node(const double *f, int32_t n, int64_t i, int64_t j)
{
    return f[(int64_t)imod(j, n) * n + imod(i, n)];
}

/* Catmull-Rom kernel, eq. cr_kernel. */
static void cr_weights(double s, double w[4])
{
    w[0] = -0.5 * s + s * s - 0.5 * s * s * s;
    w[1] = 1.0 - 2.5 * s * s + 1.5 * s * s * s;
    w[2] = 0.5 * s + 2.0 * s * s - 1.5 * s * s * s;
    w[3] = -0.5 * s * s + 0.5 * s * s * s;
}

/* Cubic B-spline kernel, eq. bspline_kernel (applied to raw grid values,
 * no prefilter: the scheme is approximating). */
static void bspline_weights(double s, double w[4])
{
    w[0] = (1.0 - s) * (1.0 - s) * (1.0 - s) / 6.0;
    w[1] = (3.0 * s * s * s - 6.0 * s * s + 4.0) / 6.0;
    w[2] = (-3.0 * s * s * s + 3.0 * s * s + 3.0 * s + 1.0) / 6.0;
    w[3] = s * s * s / 6.0;
}

static double bilinear(const double *f, int32_t n, int32_t i, int32_t j,
                       double xi, double eta)
{
    /* eq. bilinear_interp */
    return (1.0 - xi) * (1.0 - eta) * node(f, n, i, j)
         + xi * (1.0 - eta) * node(f, n, i + 1, j)
         + (1.0 - xi) * eta * node(f, n, i, j + 1)
         + xi * eta * node(f, n, i + 1, j + 1);
}

static double bicubic(const double *f, int32_t n, int32_t i, int32_t j,
                      const double wx[4], const double wy[4])
{
    /* eqs. cr_interp / bspline_interp: sum over m, n = 1..4 of
     * W_m(t) W_n(u) f_{i+m-2, j+n-2}. */
    double acc = 0.0;
    for (int m = 1; m <= 4; ++m)
        for (int q = 1; q <= 4; ++q)
            acc += wx[m - 1] * wy[q - 1] * node(f, n, (int64_t)i + m - 2, (int64_t)j + q - 2);
    return acc;
}

/* Spatial interpolation of one field at (x, y) (Sec. 3.4).  The point is
 * first mapped periodically onto the domain.  With compat_edge set, the two
 * bicubic schemes revert to bilinear in cells where the 4x4 stencil would
 * leave [0, n) (the paper's description of its own boundary handling; the
 * default is the fully periodic stencil). */
double orc_interp(const double *f, int32_t n, double L, int32_t scheme,
                  int32_t compat_edge, double x, double y)
{
    double h = L / (double)n;
    double xm = orc_wrap(x, L), ym = orc_wrap(y, L);
    int32_t i, j;
    double xi, eta;
    locate(xm, n, h, &i, &xi);
    locate(ym, n, h, &j, &eta);
    if (scheme == ORC_BILINEAR)
        return bilinear(f, n, i, j, xi, eta);
    if (compat_edge && (i - 1 < 0 || i + 2 > n - 1 || j - 1 < 0 || j + 2 > n - 1))
        return bilinear(f, n, i, j, xi, eta);
    double wx[4], wy[4];
    if (scheme == ORC_CATMULL_ROM) {
        cr_weights(xi, wx);
        cr_weights(eta, wy);
    } else {
        bspline_weights(xi, wx);
        bspline_weights(eta, wy);
    }
    return bicubic(f, n, i, j, wx, wy);
}

/* ------------------------------------------------------------------------ */
/* Fluid velocity at (x, y, t) for a step whose bracketing time levels are   */
/* (t_lo, slot_lo) and (t_hi, slot_hi).  Spatial interpolation of each time  */
/* level, then linear interpolation in time, eq. temporal_interp.            */
/* ------------------------------------------------------------------------ */
typedef struct bracket {
    int32_t lo, hi;     /* slots holding t^n and t^{n+1}   */
    double t_lo, t_hi;  /* t^n and t^{n+1}                 */
} bracket;

static double temporal(double fn, double fn1, double t, const bracket *b)
{
    double theta = (t - b->t_lo) / (b->t_hi - b->t_lo);
    return (1.0 - theta) * fn + theta * fn1;
}

static double interp_psi_at(const orc_flow *fl, const bracket *b, double x, double y, double t)
{
    double pn = orc_interp(fl->psi[b->lo], fl->n, fl->length, fl->scheme, fl->compat_edge, x, y);
    double pn1 = orc_interp(fl->psi[b->hi], fl->n, fl->length, fl->scheme, fl->compat_edge, x, y);
    return temporal(pn, pn1, t, b);
}

static void velocity(const orc_flow *fl, const bracket *b, double x, double y, double t,
                     double *u, double *v)
{
    switch (fl->source) {
    case ORC_SRC_GRID: {
        double un = orc_interp(fl->u[b->lo], fl->n, fl->length, fl->scheme, fl->compat_edge, x, y);
        double un1 = orc_interp(fl->u[b->hi], fl->n, fl->length, fl->scheme, fl->compat_edge, x, y);
        double vn = orc_interp(fl->v[b->lo], fl->n, fl->length, fl->scheme, fl->compat_edge, x, y);
        double vn1 = orc_interp(fl->v[b->hi], fl->n, fl->length, fl->scheme, fl->compat_edge, x, y);
        *u = temporal(un, un1, t, b);
        *v = temporal(vn, vn1, t, b);
        return;
    }
    case ORC_SRC_PSI: {
        /* eq. particle_velocity_reconstruction: psi at (x, y +- dy) and
         * (x +- dx, y), each mapped periodically, then centred differences
         * with the grid spacings. */
        double h = fl->length / (double)fl->n;
        double pyp = interp_psi_at(fl, b, x, orc_wrap(y + h, fl->length), t);
        double pym = interp_psi_at(fl, b, x, orc_wrap(y - h, fl->length), t);
        double pxp = interp_psi_at(fl, b, orc_wrap(x + h, fl->length), y, t);
        double pxm = interp_psi_at(fl, b, orc_wrap(x - h, fl->length), y, t);
        *u = (pyp - pym) / (2.0 * h);
        *v = -(pxp - pxm) / (2.0 * h);
        return;
    }
    case ORC_SRC_UNIFORM:
        *u = fl->U0;
        *v = fl->V0;
        return;
    case ORC_SRC_TG: {
        /* eq. kinematic_flow */
        double ax = fl->k * (x - fl->eps * sin(fl->omega * t));
        double ay = fl->k * (y - fl->eps * sin(fl->omega * t + fl->phi));
        *u = fl->alpha * sin(ax) * cos(ay);
        *v = -fl->alpha * cos(ax) * sin(ay);
        return;
    }
    default:
        *u = NAN;
        *v = NAN;
    }
}

static bracket bracket_for_step(const orc_flow *fl, int64_t step, double t_n, double dt)
{
    bracket b;
    if (fl->time_mode == ORC_PINGPONG) {
        b.lo = (int32_t)(step & 1);
        b.hi = 1 - b.lo;
        b.t_lo = t_n;
        b.t_hi = t_n + dt;
    } else {
        b.lo = 0;
        b.hi = 1;
        b.t_lo = fl->t_slot[0];
        b.t_hi = fl->t_slot[1];
    }
    return b;
}

/* Evaluate the interpolated fluid velocity at npts points at time t, with
 * the bracket of global step `step` starting at t_n (PINGPONG) or the fixed
 * snapshot bracket (BRACKET). */
void orc_velocity(const orc_flow *fl, int64_t npts, const double *x, const double *y,
                  double t, int64_t step, double t_n, double dt, double *u, double *v)
{
    bracket b = bracket_for_step(fl, step, t_n, dt);
    for (int64_t p = 0; p < npts; ++p)
        velocity(fl, &b, x[p], y[p], t, &u[p], &v[p]);
}

/* Scalar interpolation of one grid field at npts points (Sec. 3.4). */
void orc_interp_many(const double *f, int32_t n, double L, int32_t scheme, int32_t compat_edge,
                     int64_t npts, const double *x, const double *y, double *out)
{
    for (int64_t p = 0; p < npts; ++p)
        out[p] = orc_interp(f, n, L, scheme, compat_edge, x[p], y[p]);
}

/* ------------------------------------------------------------------------ */
/* One RK4 step of one particle.                                             */
/* ------------------------------------------------------------------------ */

/* Tracer, eq. rk4_update with stages at t_n, t_n + dt/2, t_n + dt/2,
 * t_n + dt (Sec. 3.2).  Returns the displacement. */
static void tracer_step(const orc_flow *fl, const bracket *b, double x, double y,
                        double t_n, double dt, double *dx, double *dy)
{
    double u1, v1, u2, v2, u3, v3, u4, v4;
    velocity(fl, b, x, y, t_n, &u1, &v1);
    velocity(fl, b, x + dt / 2.0 * u1, y + dt / 2.0 * v1, t_n + dt / 2.0, &u2, &v2);
    velocity(fl, b, x + dt / 2.0 * u2, y + dt / 2.0 * v2, t_n + dt / 2.0, &u3, &v3);
    velocity(fl, b, x + dt * u3, y + dt * v3, t_n + dt, &u4, &v4);
    *dx = dt / 6.0 * (u1 + 2.0 * u2 + 2.0 * u3 + u4);
    *dy = dt / 6.0 * (v1 + 2.0 * v2 + 2.0 * v3 + v4);
}

/* Inertial particle, eqs. inertial_particle, drag_rk4 and rk4_inertial:
 * stage s predicts position and particle velocity from the preceding
 * stage, a_s = (u(x_s, t_s) - v_s)/St. */
static void inertial_step(const orc_flow *fl, const bracket *b, double st,
                          double x, double y, double vx, double vy,
                          double t_n, double dt,
                          double *dx, double *dy, double *dvx, double *dvy)
{
    double u, v;
    /* stage 1 */
    double V1x = vx, V1y = vy;
    velocity(fl, b, x, y, t_n, &u, &v);
    double A1x = (u - V1x) / st, A1y = (v - V1y) / st;
    /* stage 2 */
    double V2x = vx + dt / 2.0 * A1x, V2y = vy + dt / 2.0 * A1y;
    velocity(fl, b, x + dt / 2.0 * V1x, y + dt / 2.0 * V1y, t_n + dt / 2.0, &u, &v);
    double A2x = (u - V2x) / st, A2y = (v - V2y) / st;
    /* stage 3 */
    double V3x = vx + dt / 2.0 * A2x, V3y = vy + dt / 2.0 * A2y;
    velocity(fl, b, x + dt / 2.0 * V2x, y + dt / 2.0 * V2y, t_n + dt / 2.0, &u, &v);
    double A3x = (u - V3x) / st, A3y = (v - V3y) / st;
    /* stage 4 */
    double V4x = vx + dt * A3x, V4y = vy + dt * A3y;
    velocity(fl, b, x + dt * V3x, y + dt * V3y, t_n + dt, &u, &v);
    double A4x = (u - V4x) / st, A4y = (v - V4y) / st;

    *dx = dt / 6.0 * (V1x + 2.0 * V2x + 2.0 * V3x + V4x);
    *dy = dt / 6.0 * (V1y + 2.0 * V2y + 2.0 * V3y + V4y);
    *dvx = dt / 6.0 * (A1x + 2.0 * A2x + 2.0 * A3x + A4x);
    *dvy = dt / 6.0 * (A1y + 2.0 * A2y + 2.0 * A3y + A4y);
}

/* ------------------------------------------------------------------------ */
/* Statistics on unwrapped displacements (Sec. 3.2 and 3.3: MSD and the      */
/* diffusion coefficients use open trajectories; Sec. 5.5: SEM of the MSD). */
/* Reading of the undefined quantities: MSD_x = <dx^2>, MSD_y = <dy^2>,      */
/* MSD = MSD_x + MSD_y, D_x = MSD_x/(2t), D_y = MSD_y/(2t),                  */
/* SEM = sqrt(var(dx^2+dy^2; ddof=1)/Np).  Sums are Neumaier-compensated.    */
/* ------------------------------------------------------------------------ */
typedef struct { double s, c; } nsum;

static void nadd(nsum *a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}

static double nval(const nsum *a) { return a->s + a->c; }

/* rec = {t, msd_x, msd_y, msd, d_x, d_y, sem, np} */
void orc_stats(int64_t np, const double *dxs, const double *dys, double t, double elapsed,
               double *rec)
{
    nsum sx = {0, 0}, sy = {0, 0};
    for (int64_t p = 0; p < np; ++p) {
        nadd(&sx, dxs[p] * dxs[p]);
        nadd(&sy, dys[p] * dys[p]);
    }
    double msd_x = nval(&sx) / (double)np;
    double msd_y = nval(&sy) / (double)np;
    double msd = msd_x + msd_y;
    /* two-pass sample variance of r^2 = dx^2 + dy^2 about its mean msd */
    nsum sv = {0, 0};
    for (int64_t p = 0; p < np; ++p) {
        double r2 = dxs[p] * dxs[p] + dys[p] * dys[p];
        double d = r2 - msd;
        nadd(&sv, d * d);
    }
    double var = np > 1 ? nval(&sv) / (double)(np - 1) : 0.0;
    rec[0] = t;
    rec[1] = msd_x;
    rec[2] = msd_y;
    rec[3] = msd;
    rec[4] = elapsed > 0.0 ? msd_x / (2.0 * elapsed) : 0.0;
    rec[5] = elapsed > 0.0 ? msd_y / (2.0 * elapsed) : 0.0;
    rec[6] = np > 0 ? sqrt(var / (double)np) : 0.0;
    rec[7] = (double)np;
}

/* ------------------------------------------------------------------------ */
/* Advance one species by nsteps (Alg. coupled_EL, particle part).           */
/*  kind: ORC_TRACER / ORC_INERTIAL; st == 0 integrates the tracer equations */
/*  (the St -> 0 limit, Sec. 3.3).  xw, yw: wrapped positions (in/out);       */
/*  dxs, dys: unwrapped displacements (in/out); vx, vy: particle velocity    */
/*  (inertial only, in/out).  The step with local index k has global index   */
/*  step0 + k and starts at t_n = t_start + k*dt.  After a step whose global */
/*  index + 1 is a multiple of stats_every (> 0), a record is appended, with */
/*  elapsed time t_{n+1} - t_origin.  Returns the number of records.         */
/* ------------------------------------------------------------------------ */
int64_t orc_run(const orc_flow *fl, int32_t kind, double st, int64_t np,
                double *xw, double *yw, double *dxs, double *dys, double *vx, double *vy,
                int64_t nsteps, double dt, double t_start, int64_t step0,
                int64_t stats_every, double t_origin, double *records, int64_t rec_cap)
{
    int64_t nrec = 0;
    int inertial = (kind == ORC_INERTIAL) && (st != 0.0);
    for (int64_t k = 0; k < nsteps; ++k) {
        double t_n = t_start + (double)k * dt;
        bracket b = bracket_for_step(fl, step0 + k, t_n, dt);
        /* particles are independent within a step: a build with OpenMP (the
         * CPU timing build only) shares them out statically; the arithmetic
         * per particle is the same either way */
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
        for (int64_t p = 0; p < np; ++p) {
            double ddx, ddy;
            if (inertial) {
                double dvx, dvy;
                inertial_step(fl, &b, st, xw[p], yw[p], vx[p], vy[p], t_n, dt,
                              &ddx, &ddy, &dvx, &dvy);
                vx[p] += dvx;
                vy[p] += dvy;
            } else {
                tracer_step(fl, &b, xw[p], yw[p], t_n, dt, &ddx, &ddy);
            }
            /* wrapped coordinates for field evaluation and output, unwrapped
             * displacement for transport statistics */
            xw[p] = orc_wrap(xw[p] + ddx, fl->length);
            yw[p] = orc_wrap(yw[p] + ddy, fl->length);
            dxs[p] += ddx;
            dys[p] += ddy;
        }
        int64_t g = step0 + k + 1;
        if (stats_every > 0 && g % stats_every == 0 && nrec < rec_cap) {
            double t1 = t_start + (double)(k + 1) * dt;
            orc_stats(np, dxs, dys, t1, t1 - t_origin, records + 8 * nrec);
            ++nrec;
        }
    }
    return nrec;
}

/* ------------------------------------------------------------------------ */
/* Initial positions: counter-indexed SplitMix64 (Steele, Lea & Flood,       */
/* "Fast splittable pseudorandom number generators", OOPSLA 2014).  Output   */
/* k of the stream seeded with s is mix(s + (k+1)*0x9E3779B97F4A7C15); the   */
/* unit variate is (z >> 11) * 2^-53.  Particle p takes outputs 2p (x) and   */
/* 2p+1 (y), then x = wrap(L*u).  The paper does not say how its initial     */
/* positions are drawn; this is the reading used by both sides.              */
/* ------------------------------------------------------------------------ */
uint64_t orc_splitmix64(uint64_t seed, uint64_t k)
{
    uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

void orc_init_uniform(uint64_t seed, int64_t np, double L, double *x, double *y)
{
    for (int64_t p = 0; p < np; ++p) {
        double ux = (double)(orc_splitmix64(seed, 2 * (uint64_t)p) >> 11) * 0x1p-53;
        double uy = (double)(orc_splitmix64(seed, 2 * (uint64_t)p + 1) >> 11) * 0x1p-53;
        x[p] = orc_wrap(L * ux, L);
        y[p] = orc_wrap(L * uy, L);
    }
}

/* ------------------------------------------------------------------------ */
/* Cell-order key of a stored cell (i, j): tiles of T x T cells, tiles in    */
/* row-major order, cells row-major inside a tile.  T = 1 (or T = n) is the  */
/* plain row-major order j*n + i.  With coarse = 1 the key is the tile index */
/* alone.  n must be a multiple of T.  The sort itself is a stable ascending */
/* argsort of these keys (a library primitive on the Python side).           */
/* ------------------------------------------------------------------------ */
void orc_cell_keys(int32_t n, int32_t tile, int32_t coarse, int64_t np,
                   const int32_t *ci, const int32_t *cj, uint32_t *keys)
{
    int64_t tiles_x = n / tile;
    for (int64_t p = 0; p < np; ++p) {
        int64_t ti = ci[p] / tile, tj = cj[p] / tile;
        int64_t tix = (int64_t)tj * tiles_x + ti;
        if (coarse)
            keys[p] = (uint32_t)tix;
        else
            keys[p] = (uint32_t)(tix * tile * tile + (int64_t)(cj[p] % tile) * tile + ci[p] % tile);
    }
}

/* Stored cell of an FP64 wrapped position: the cell of O-3 style location. */
void orc_cells_of(int32_t n, double L, int64_t np, const double *x, int32_t *ci)
{
    double h = L / (double)n;
    for (int64_t p = 0; p < np; ++p) {
        int32_t i;
        double xi;
        locate(orc_wrap(x[p], L), n, h, &i, &xi);
        ci[p] = i;
    }
}

/* ======================================================================== */
/* Derivatives of the discrete particle map (tracers).  The paper has no     */
/* adjoint; these are the plain derivatives of the steps above, for          */
/* finite-time Lyapunov exponents and for gradients with respect to the      */
/* gridded velocity.  The floor of the cell location is piecewise constant,  */
/* so d(cell)/dx = 0 and d(xi)/dx = 1/h inside a cell.                        */
/* ======================================================================== */

/* Derivatives of the Catmull-Rom and B-spline kernels (eqs. cr_kernel and
 * bspline_kernel differentiated in s). */
static void cr_dweights(double s, double w[4])
{
    w[0] = -0.5 + 2.0 * s - 1.5 * s * s;
    w[1] = -5.0 * s + 4.5 * s * s;
    w[2] = 0.5 + 4.0 * s - 4.5 * s * s;
    w[3] = -s + 1.5 * s * s;
}

static void bspline_dweights(double s, double w[4])
{
    w[0] = -0.5 * (1.0 - s) * (1.0 - s);
    w[1] = 1.5 * s * s - 2.0 * s;
    w[2] = -1.5 * s * s + s + 0.5;
    w[3] = 0.5 * s * s;
}

/* Stencil of one interpolation: up to 16 nodes (periodic indices into the
 * [n*n] field), their weights, and the weights' x- and y-derivatives. */
typedef struct {
    int32_t count;
    int64_t idx[16];
    double w[16], wx[16], wy[16];
} stencil;

static void make_stencil(int32_t n, double L, int32_t scheme, int32_t compat_edge, double x,
                         double y, stencil *st)
{
    double h = L / (double)n;
    double xm = orc_wrap(x, L), ym = orc_wrap(y, L);
    int32_t i, j;
    double xi, eta;
    locate(xm, n, h, &i, &xi);
    locate(ym, n, h, &j, &eta);
    int bil = scheme == ORC_BILINEAR ||
              (compat_edge && (i - 1 < 0 || i + 2 > n - 1 || j - 1 < 0 || j + 2 > n - 1));
    st->count = 0;
    if (bil) {
        /* eq. bilinear_interp: weights (1-xi)(1-eta), xi(1-eta), (1-xi)eta, xi eta */
        double wxs[2] = {1.0 - xi, xi}, wys[2] = {1.0 - eta, eta};
        double dxs[2] = {-1.0 / h, 1.0 / h}, dys[2] = {-1.0 / h, 1.0 / h};
        for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 2; ++a) {
                int k = st->count++;
                st->idx[k] = (int64_t)imod((int64_t)j + b, n) * n + imod((int64_t)i + a, n);
                st->w[k] = wxs[a] * wys[b];
                st->wx[k] = dxs[a] * wys[b];
                st->wy[k] = wxs[a] * dys[b];
            }
        return;
    }
    double wx4[4], wy4[4], dx4[4], dy4[4];
    if (scheme == ORC_CATMULL_ROM) {
        cr_weights(xi, wx4);
        cr_weights(eta, wy4);
        cr_dweights(xi, dx4);
        cr_dweights(eta, dy4);
    } else {
        bspline_weights(xi, wx4);
        bspline_weights(eta, wy4);
        bspline_dweights(xi, dx4);
        bspline_dweights(eta, dy4);
    }
    /* eqs. cr_interp / bspline_interp: node (i+m-2, j+q-2) has weight
     * W_m(xi) W_q(eta) */
    for (int q = 1; q <= 4; ++q)
        for (int m = 1; m <= 4; ++m) {
            int k = st->count++;
            st->idx[k] = (int64_t)imod((int64_t)j + q - 2, n) * n + imod((int64_t)i + m - 2, n);
            st->w[k] = wx4[m - 1] * wy4[q - 1];
            st->wx[k] = dx4[m - 1] / h * wy4[q - 1];
            st->wy[k] = wx4[m - 1] * dy4[q - 1] / h;
        }
}

/* Value and gradient of one interpolated grid field at (x, y). */
void orc_interp_grad(const double *f, int32_t n, double L, int32_t scheme, int32_t compat_edge,
                     double x, double y, double *val, double *dfdx, double *dfdy)
{
    stencil st;
    make_stencil(n, L, scheme, compat_edge, x, y, &st);
    double a = 0.0, b = 0.0, c = 0.0;
    for (int k = 0; k < st.count; ++k) {
        a += st.w[k] * f[st.idx[k]];
        b += st.wx[k] * f[st.idx[k]];
        c += st.wy[k] * f[st.idx[k]];
    }
    *val = a;
    *dfdx = b;
    *dfdy = c;
}

/* Fluid velocity U and its spatial Jacobian J = [[du/dx, du/dy], [dv/dx,
 * dv/dy]] at (x, y, t) within bracket b (grid, uniform and Taylor-Green
 * sources). */
static void velocity_jac(const orc_flow *fl, const bracket *b, double x, double y, double t,
                         double U[2], double J[4])
{
    if (fl->source == ORC_SRC_GRID) {
        double theta = (t - b->t_lo) / (b->t_hi - b->t_lo);
        double wt[2] = {1.0 - theta, theta};
        int32_t sl[2] = {b->lo, b->hi};
        U[0] = U[1] = 0.0;
        for (int q = 0; q < 4; ++q) J[q] = 0.0;
        for (int s = 0; s < 2; ++s) {
            double val, dx, dy;
            orc_interp_grad(fl->u[sl[s]], fl->n, fl->length, fl->scheme, fl->compat_edge, x, y,
                            &val, &dx, &dy);
            U[0] += wt[s] * val;
            J[0] += wt[s] * dx;
            J[1] += wt[s] * dy;
            orc_interp_grad(fl->v[sl[s]], fl->n, fl->length, fl->scheme, fl->compat_edge, x, y,
                            &val, &dx, &dy);
            U[1] += wt[s] * val;
            J[2] += wt[s] * dx;
            J[3] += wt[s] * dy;
        }
        return;
    }
    if (fl->source == ORC_SRC_UNIFORM) {
        U[0] = fl->U0;
        U[1] = fl->V0;
        J[0] = J[1] = J[2] = J[3] = 0.0;
        return;
    }
    if (fl->source == ORC_SRC_TG) {
        /* eq. kinematic_flow differentiated in x and y */
        double ax = fl->k * (x - fl->eps * sin(fl->omega * t));
        double ay = fl->k * (y - fl->eps * sin(fl->omega * t + fl->phi));
        double A = fl->alpha, k = fl->k;
        U[0] = A * sin(ax) * cos(ay);
        U[1] = -A * cos(ax) * sin(ay);
        J[0] = A * k * cos(ax) * cos(ay);
        J[1] = -A * k * sin(ax) * sin(ay);
        J[2] = A * k * sin(ax) * sin(ay);
        J[3] = -A * k * cos(ax) * cos(ay);
        return;
    }
    U[0] = U[1] = NAN;
    J[0] = J[1] = J[2] = J[3] = NAN;
}

/* 2x2 product C = A B (row-major). */
static void mat2(const double A[4], const double B[4], double C[4])
{
    double c0 = A[0] * B[0] + A[1] * B[2];
    double c1 = A[0] * B[1] + A[1] * B[3];
    double c2 = A[2] * B[0] + A[3] * B[2];
    double c3 = A[2] * B[1] + A[3] * B[3];
    C[0] = c0;
    C[1] = c1;
    C[2] = c2;
    C[3] = c3;
}

/* Forward tangent propagation of F = d x_n / d x_0 (row-major 2x2 per
 * particle, in/out) alongside the tracer RK4 step of eq. rk4_update: every
 * stage state carries its own tangent, X_s = F + c_s dt K_{s-1}, and
 * K_s = J(x_s) X_s.  Advances xw, yw, dxs, dys as orc_run does. */
void orc_tangent_run(const orc_flow *fl, int64_t np, double *xw, double *yw, double *dxs,
                     double *dys, double *F, int64_t nsteps, double dt, double t_start,
                     int64_t step0)
{
    for (int64_t k = 0; k < nsteps; ++k) {
        double t_n = t_start + (double)k * dt;
        bracket b = bracket_for_step(fl, step0 + k, t_n, dt);
        /* particles are independent within a step: a build with OpenMP (the
         * CPU timing build only) shares them out statically; the arithmetic
         * per particle is the same either way */
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
        for (int64_t p = 0; p < np; ++p) {
            double *Fp = F + 4 * p;
            double x = xw[p], y = yw[p];
            double U1[2], U2[2], U3[2], U4[2], J[4], K1[4], K2[4], K3[4], K4[4], X[4];
            velocity_jac(fl, &b, x, y, t_n, U1, J);
            mat2(J, Fp, K1);
            for (int q = 0; q < 4; ++q) X[q] = Fp[q] + dt / 2.0 * K1[q];
            velocity_jac(fl, &b, x + dt / 2.0 * U1[0], y + dt / 2.0 * U1[1], t_n + dt / 2.0, U2, J);
            mat2(J, X, K2);
            for (int q = 0; q < 4; ++q) X[q] = Fp[q] + dt / 2.0 * K2[q];
            velocity_jac(fl, &b, x + dt / 2.0 * U2[0], y + dt / 2.0 * U2[1], t_n + dt / 2.0, U3, J);
            mat2(J, X, K3);
            for (int q = 0; q < 4; ++q) X[q] = Fp[q] + dt * K3[q];
            velocity_jac(fl, &b, x + dt * U3[0], y + dt * U3[1], t_n + dt, U4, J);
            mat2(J, X, K4);
            for (int q = 0; q < 4; ++q)
                Fp[q] += dt / 6.0 * (K1[q] + 2.0 * K2[q] + 2.0 * K3[q] + K4[q]);
            double ddx = dt / 6.0 * (U1[0] + 2.0 * U2[0] + 2.0 * U3[0] + U4[0]);
            double ddy = dt / 6.0 * (U1[1] + 2.0 * U2[1] + 2.0 * U3[1] + U4[1]);
            xw[p] = orc_wrap(x + ddx, fl->length);
            yw[p] = orc_wrap(y + ddy, fl->length);
            dxs[p] += ddx;
            dys[p] += ddy;
        }
    }
}

/* Scatter lam (dL/dU at one stage point) into the grid gradient: the stage
 * velocity is sum over time levels s and stencil nodes k of
 * wt_s w_k (u_s[k], v_s[k]). */
static void scatter_stage(const orc_flow *fl, const bracket *b, double x, double y, double t,
                          const double lam[2], double *gU)
{
    int64_t nn = (int64_t)fl->n * fl->n;
    double theta = (t - b->t_lo) / (b->t_hi - b->t_lo);
    double wt[2] = {1.0 - theta, theta};
    int32_t sl[2] = {b->lo, b->hi};
    stencil st;
    make_stencil(fl->n, fl->length, fl->scheme, fl->compat_edge, x, y, &st);
    for (int s = 0; s < 2; ++s) {
        double *gu = gU + (int64_t)(2 * sl[s]) * nn;      /* [slot][u] */
        double *gv = gU + (int64_t)(2 * sl[s] + 1) * nn;  /* [slot][v] */
        for (int k = 0; k < st.count; ++k) {
            gu[st.idx[k]] += wt[s] * st.w[k] * lam[0];
            gv[st.idx[k]] += wt[s] * st.w[k] * lam[1];
        }
    }
}

/* Reverse sweep for L = sum_p (a_p x_T,p + b_p y_T,p) over nsteps tracer RK4
 * steps from (x0, y0): the forward pass keeps every step's start position
 * (a full tape), the reverse pass recomputes each step's stages and applies
 * the chain rule through the combine, the stage states and the spatial and
 * temporal interpolation.  Outputs dL/dx0, dL/dy0 and, for a grid source,
 * adds dL/d(grid value) into gU laid out [slot][component u, v][n*n]
 * (caller zeroes it).  tape: caller buffer of 2*np*nsteps doubles. */
void orc_adjoint_run(const orc_flow *fl, int64_t np, const double *x0, const double *y0,
                     const double *a, const double *bb, int64_t nsteps, double dt,
                     double t_start, int64_t step0, double *gx0, double *gy0, double *gU,
                     double *tape)
{
    for (int64_t p = 0; p < np; ++p) {
        double x = orc_wrap(x0[p], fl->length), y = orc_wrap(y0[p], fl->length);
        for (int64_t k = 0; k < nsteps; ++k) {
            double t_n = t_start + (double)k * dt;
            bracket b = bracket_for_step(fl, step0 + k, t_n, dt);
            tape[2 * (k * np + p)] = x;
            tape[2 * (k * np + p) + 1] = y;
            double ddx, ddy;
            tracer_step(fl, &b, x, y, t_n, dt, &ddx, &ddy);
            x = orc_wrap(x + ddx, fl->length);
            y = orc_wrap(y + ddy, fl->length);
        }
    }
    for (int64_t p = 0; p < np; ++p) {
        double lam[2] = {a[p], bb[p]};
        for (int64_t k = nsteps - 1; k >= 0; --k) {
            double t_n = t_start + (double)k * dt;
            bracket b = bracket_for_step(fl, step0 + k, t_n, dt);
            double x = tape[2 * (k * np + p)], y = tape[2 * (k * np + p) + 1];
            /* recompute the stages */
            double U1[2], U2[2], U3[2], U4[2], J1[4], J2[4], J3[4], J4[4];
            double t2 = t_n + dt / 2.0, t4 = t_n + dt;
            velocity_jac(fl, &b, x, y, t_n, U1, J1);
            double x2 = x + dt / 2.0 * U1[0], y2 = y + dt / 2.0 * U1[1];
            velocity_jac(fl, &b, x2, y2, t2, U2, J2);
            double x3 = x + dt / 2.0 * U2[0], y3 = y + dt / 2.0 * U2[1];
            velocity_jac(fl, &b, x3, y3, t2, U3, J3);
            double x4 = x + dt * U3[0], y4 = y + dt * U3[1];
            velocity_jac(fl, &b, x4, y4, t4, U4, J4);
            /* x' = x + dt/6 (k1 + 2 k2 + 2 k3 + k4) */
            double lx[2] = {lam[0], lam[1]};
            double l1[2] = {dt / 6.0 * lam[0], dt / 6.0 * lam[1]};
            double l2[2] = {dt / 3.0 * lam[0], dt / 3.0 * lam[1]};
            double l3[2] = {dt / 3.0 * lam[0], dt / 3.0 * lam[1]};
            double l4[2] = {dt / 6.0 * lam[0], dt / 6.0 * lam[1]};
            double ls[2];
            /* k4 = U(x4, t4), x4 = x + dt k3 */
            if (gU && fl->source == ORC_SRC_GRID) scatter_stage(fl, &b, x4, y4, t4, l4, gU);
            ls[0] = J4[0] * l4[0] + J4[2] * l4[1];
            ls[1] = J4[1] * l4[0] + J4[3] * l4[1];
            lx[0] += ls[0];
            lx[1] += ls[1];
            l3[0] += dt * ls[0];
            l3[1] += dt * ls[1];
            /* k3 = U(x3, t2), x3 = x + dt/2 k2 */
            if (gU && fl->source == ORC_SRC_GRID) scatter_stage(fl, &b, x3, y3, t2, l3, gU);
            ls[0] = J3[0] * l3[0] + J3[2] * l3[1];
            ls[1] = J3[1] * l3[0] + J3[3] * l3[1];
            lx[0] += ls[0];
            lx[1] += ls[1];
            l2[0] += dt / 2.0 * ls[0];
            l2[1] += dt / 2.0 * ls[1];
            /* k2 = U(x2, t2), x2 = x + dt/2 k1 */
            if (gU && fl->source == ORC_SRC_GRID) scatter_stage(fl, &b, x2, y2, t2, l2, gU);
            ls[0] = J2[0] * l2[0] + J2[2] * l2[1];
            ls[1] = J2[1] * l2[0] + J2[3] * l2[1];
            lx[0] += ls[0];
            lx[1] += ls[1];
            l1[0] += dt / 2.0 * ls[0];
            l1[1] += dt / 2.0 * ls[1];
            /* k1 = U(x, t_n) */
            if (gU && fl->source == ORC_SRC_GRID) scatter_stage(fl, &b, x, y, t_n, l1, gU);
            lx[0] += J1[0] * l1[0] + J1[2] * l1[1];
            lx[1] += J1[1] * l1[0] + J1[3] * l1[1];
            lam[0] = lx[0];
            lam[1] = lx[1];
        }
        gx0[p] = lam[0];
        gy0[p] = lam[1];
    }
}
