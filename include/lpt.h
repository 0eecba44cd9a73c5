/*
 * lpt.h -- C ABI of the MI355X (gfx950) Lagrangian particle library, liblpt.so.
 *
 * The library advances passive tracers and Stokes-drag inertial particles
 * through gridded 2D velocity snapshots on the doubly periodic [0, L)^2 domain,
 * as in the particle half of the one-way coupled Eulerian-Lagrangian method of
 * Maiti & Ganesh, "A coupled Eulerian-Lagrangian approach for fluid and
 * particle dynamics":
 *   - spatial interpolation of the velocity: bilinear (eq. bilinear_interp),
 *     bicubic Catmull-Rom (eqs. cr_interp, cr_kernel) or bicubic B-spline
 *     without prefilter (eqs. bspline_interp, bspline_kernel), Sec. 3.4;
 *   - linear interpolation in time between the two snapshots that bracket
 *     each RK4 stage (eq. temporal_interp);
 *   - classical RK4 for tracers (eqs. adv_eqn, rk4_update, Sec. 3.2) and for
 *     inertial particles (eqs. inertial_particle, drag_rk4, rk4_inertial,
 *     Sec. 3.3), stages at t_n, t_n + dt/2, t_n + dt/2, t_n + dt;
 *   - wrapped positions for field evaluation and output, unwrapped
 *     displacements for the transport statistics (Sec. 3.2, Alg. coupled_EL);
 *   - mean-square displacement, diffusion coefficients and the standard error
 *     of the MSD (Sec. 3.2, 5.5, 6.2).
 *
 * Grid convention: node (i, j) sits at (i*h, j*h), h = L/n, 0 <= i, j < n;
 * every field array is [n][n] with x fastest (element j*n + i).
 *
 * Conventions for every entry point:
 *   - The return value is an lpt_status; no C++ exception crosses the ABI.
 *   - Arguments are validated before anything is enqueued: on any error the
 *     context is left exactly as it was, and lpt_last_error() says why.
 *   - Work is enqueued on the context's HIP stream and the call returns
 *     without waiting, unless it copies results into host memory (then it
 *     synchronises the stream first).  An asynchronous GPU fault surfaces as
 *     LPT_E_HIP at the next call that synchronises.
 *   - "on_device" = 1 means the pointer is device memory (readable on the
 *     context's device); 0 means host memory.  Inputs are copied (in stream
 *     order), so the caller keeps ownership; outputs go into caller buffers.
 *   - A context is not thread-safe; use one per host thread / stream.
 */
#ifndef LPT_H
#define LPT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lpt_ctx lpt_ctx;

typedef enum {
    LPT_OK = 0,
    LPT_E_ARG = 1,     /* invalid argument (NULL, out of range, NaN, ...)      */
    LPT_E_STATE = 2,   /* call not valid in the current state                 */
    LPT_E_RANGE = 3,   /* a stage time falls outside the snapshot bracket     */
    LPT_E_NOMEM = 4,   /* device or host allocation failed                    */
    LPT_E_HIP = 5      /* HIP runtime error (message in lpt_last_error)       */
} lpt_status;

typedef enum { LPT_BILINEAR = 0, LPT_CATMULL_ROM = 1, LPT_BSPLINE = 2 } lpt_scheme;

/* LPT_FP64: fields, positions and all arithmetic in binary64.
 * LPT_FP32_SPLIT: fields and interpolation in binary32; a position is an
 * unwrapped integer cell (its residue mod n is the periodic cell) plus a
 * binary32 offset in cell units, so the unwrapped displacement is that
 * position minus the split form of the initial one, formed in binary64 with
 * the offset's resolution (about 6e-8 cells) however far the particle has
 * gone; velocities are binary32; the statistics are binary64. */
typedef enum { LPT_FP64 = 0, LPT_FP32_SPLIT = 1 } lpt_precision;

typedef enum { LPT_TRACER = 0, LPT_INERTIAL = 1 } lpt_kind;

/* LPT_TIME_BRACKET: slot 0 holds the level at t_a, slot 1 the level at t_b;
 *   every stage time must lie in [t_a, t_b].
 * LPT_TIME_PINGPONG: step number s (counted from context creation) uses slot
 *   s % 2 as the level at t_n and the other slot as the level at t_n + dt,
 *   so that a caller can stream a new snapshot into the older slot after every
 *   step (the two retained time levels of Alg. coupled_EL); requires
 *   dt == |t_b - t_a| of the two set snapshots. */
typedef enum { LPT_TIME_BRACKET = 0, LPT_TIME_PINGPONG = 1 } lpt_time_mode;

/* flags */
#define LPT_FLAG_COMPAT_EDGE 0x1u  /* bicubic reverts to bilinear in cells whose
                                      4x4 stencil leaves [0, n) (Sec. 3.4); off:
                                      fully periodic stencil                    */
#define LPT_FLAG_TIME_KERNELS 0x2u /* record HIP events around every step-kernel
                                      launch and every re-sort, on the context
                                      stream (see lpt_get_timing)               */
#define LPT_FLAG_DETERMINISTIC_GRAD 0x4u /* lpt_adjoint sums the grid gradient
                                      exactly in fixed point (each contribution
                                      rounded once to a multiple of 2^-64, |entries|
                                      below 2^31): the same bits on every run and
                                      launch shape; needs 64 n^2 bytes of device
                                      memory more during the sweep              */

typedef struct {
    int32_t n;              /* grid points per side, 4 <= n <= 32768          */
    int32_t precision;      /* lpt_precision                                  */
    double length;          /* domain side L > 0; 0 selects 2*pi              */
    double t0;              /* initial time; statistics use t - t0            */
    void *hip_stream;       /* hipStream_t to enqueue on; NULL = null stream  */
    int32_t sort_interval;  /* steps between cell-order re-sorts; 0 = never   */
    int32_t sort_tile;      /* tile side T of the cell-order key (power of
                               two dividing n); 0 selects 16                  */
    int32_t block_size;     /* particles per logical block of the step
                               kernel (its threads, at one particle per
                               thread; see lpt_tuning.rows): 64, 128, 256 or
                               512; 0 selects 256 (else LPT_E_ARG)            */
    uint32_t flags;         /* LPT_FLAG_*                                     */
    int32_t tile_records;   /* capacity, in node records, of the per-block
                               LDS field tile of the step kernel: 0 selects
                               the default (FP32-split: per launch, the
                               largest capacity that keeps the kernel's
                               register-bound occupancy; FP64: 1200 records,
                               38400 bytes), -1 disables tiles (every
                               stencil gathers from global memory), else at
                               least 16 records and at most 61440 bytes of
                               records (rounded up to whole 64-entry fill
                               chunks); else LPT_E_ARG                      */
} lpt_config;

/* One statistics record of one species (Sec. 3.2, 5.5):
 *   msd_x = <dx^2>, msd_y = <dy^2>, msd = msd_x + msd_y over the species,
 *   d_x = msd_x / (2 (t - t0)), d_y = msd_y / (2 (t - t0)),
 *   sem = sqrt(var(dx^2 + dy^2; ddof = 1) / n),
 * where (dx, dy) is the unwrapped displacement since initialisation. */
typedef struct {
    double t, msd_x, msd_y, msd, d_x, d_y, sem;
    int64_t n;
} lpt_stat;

/* ---- context ------------------------------------------------------------ */

/* Create a context on the current HIP device.  *out receives the handle. */
lpt_status lpt_create(const lpt_config *cfg, lpt_ctx **out);
/* Release every device and host resource of the context (NULL is a no-op). */
void lpt_destroy(lpt_ctx *ctx);
/* Message of the last failed call on this context ("" if none).  The string
 * lives until the next call on the context. */
const char *lpt_last_error(const lpt_ctx *ctx);
/* Static name of a status code. */
const char *lpt_status_string(lpt_status s);
/* Block until all work enqueued by the context has finished. */
lpt_status lpt_synchronize(lpt_ctx *ctx);

/* ---- fields ------------------------------------------------------------- */

/* Store one velocity snapshot (u, v at time t) in slot 0 or 1 -- the two
 * retained time levels of Alg. coupled_EL.  u and v are [n][n], x fastest,
 * double for LPT_FP64 and LPT_FP32_SPLIT alike (the FP32 path rounds them).
 * May be called between steps to stream a new level into a slot. */
lpt_status lpt_set_snapshot(lpt_ctx *ctx, int32_t slot, double t,
                            const double *u, const double *v, int32_t on_device);
lpt_status lpt_set_time_mode(lpt_ctx *ctx, lpt_time_mode mode);

/* Store a stream-function snapshot psi [n][n] in slot 0 or 1 instead of a
 * velocity: the library forms the centred-difference velocity on the grid,
 * u = (psi(j+1) - psi(j-1))/(2h), v = -(psi(i+1) - psi(i-1))/(2h), which equals
 * interpolating psi at (x, y +- dy), (x +- dx, y) and differencing
 * (eq. particle_velocity_reconstruction) for every scheme, because the four
 * shifted points share the particle's in-cell coordinates. */
lpt_status lpt_set_snapshot_psi(lpt_ctx *ctx, int32_t slot, double t,
                                const double *psi, int32_t on_device);

/* ---- particles ---------------------------------------------------------- */

/* Add a species of `count` particles of one kind, Stokes number and scheme.
 * st must be >= 0; st == 0 integrates the tracer equations (the St -> 0 limit,
 * Sec. 3.3) whatever the kind.  x0, y0: initial positions (binary64, any real
 * value; they are mapped periodically).  vx0, vy0: initial particle velocity
 * of an inertial species; NULL sets it to the interpolated fluid velocity at
 * (x0, t0) (both snapshots must then be set).  Must be called before the
 * first step.  *species_id receives the species index (0, 1, ...). */
lpt_status lpt_add_species(lpt_ctx *ctx, lpt_kind kind, double st, lpt_scheme scheme,
                           int64_t count, const double *x0, const double *y0,
                           const double *vx0, const double *vy0, int32_t on_device,
                           int32_t *species_id);

/* Overwrite the initial positions of a species with uniform random points:
 * particle p takes outputs 2p and 2p+1 of the counter-indexed SplitMix64
 * stream seeded with `seed`, u = (z >> 11) * 2^-53, x = L*u.  Resets the
 * displacements (and the velocity, if it was taken from the field).  Only
 * before the first step.  In FP32-split mode the statistics steps draw these
 * positions again from the seed (the same bits) instead of reading them,
 * until lpt_set_state replaces them. */
lpt_status lpt_init_uniform(lpt_ctx *ctx, int32_t species_id, uint64_t seed);

/* Advance every species by nsteps RK4 steps of size dt (Alg. coupled_EL,
 * particle loop).  If stats_every > 0, a statistics record of every species
 * is taken after each step whose global step number (counted from context
 * creation, 1-based) is a multiple of stats_every.  Cell-order re-sorting
 * happens before every step whose global number is a multiple of
 * sort_interval.  Errors: LPT_E_STATE (no species / snapshots),
 * LPT_E_RANGE (BRACKET: a stage time outside [t_a, t_b]), LPT_E_ARG. */
lpt_status lpt_step(lpt_ctx *ctx, int64_t nsteps, double dt, int32_t stats_every);

/* Re-sort the particles into cell order now (stable; ties keep the current
 * order).  Per-particle results are unchanged by sorting. */
lpt_status lpt_sort(lpt_ctx *ctx);

/* Positions of a species in the original particle order: wrapped (xw, yw in
 * [0, L)) and unwrapped (xu = x0 + dx, yu = y0 + dy).  Any pointer may be
 * NULL.  Each array holds `count` doubles. */
lpt_status lpt_get_positions(lpt_ctx *ctx, int32_t species_id, double *xw, double *yw,
                             double *xu, double *yu, int32_t on_device);
/* Particle velocity of an inertial species (original order, binary64). */
lpt_status lpt_get_velocities(lpt_ctx *ctx, int32_t species_id, double *vx, double *vy,
                              int32_t on_device);
/* Copy up to `cap` statistics records of a species into host memory;
 * *n_written receives the number copied (oldest first). */
lpt_status lpt_get_stats(lpt_ctx *ctx, int32_t species_id, lpt_stat *out, int64_t cap,
                         int64_t *n_written);

/* Current slot order of a species: ids[k] receives the original index
 * (0 .. count-1) of the particle stored in slot k of the species' range, so
 * that a caller can see the cell order produced by lpt_sort.  `count` int32
 * values; device or host memory per on_device. */
lpt_status lpt_get_order(lpt_ctx *ctx, int32_t species_id, int32_t *ids, int32_t on_device);

/* Device time spent in the step kernel and in re-sorting since the last
 * reset, measured with HIP events on the context stream (needs
 * LPT_FLAG_TIME_KERNELS; synchronises the stream).  A step that follows a
 * re-sort also applies the sort's permutation to the state (a kernel of its
 * own); it is counted under perm_step_ms, not step_kernel_ms.  A step that
 * takes a statistics record (and is no permuting step) runs the step
 * kernel's statistics variant, counted under stats_step_ms; the merge of its
 * partials into the records under finalize_ms. */
typedef struct {
    double step_kernel_ms;    /* sum over in-place step launches without a
                                 statistics record                           */
    int64_t step_launches;
    double sort_ms;           /* sum over re-sorts (keys, radix sort; and the
                                 permutation where lpt_sort applies it)      */
    int64_t sorts;
    double perm_step_ms;      /* sum over steps that apply a permutation     */
    int64_t perm_steps;
    double stats_step_ms;     /* sum over in-place steps taking a record     */
    int64_t stats_steps;
    double finalize_ms;       /* sum over the records' merge kernels         */
} lpt_timing;
lpt_status lpt_get_timing(lpt_ctx *ctx, lpt_timing *out, int32_t reset);

/* Number of steps taken and current time. */
lpt_status lpt_get_time(lpt_ctx *ctx, int64_t *steps, double *t);

/* ---- checkpoint / resume --------------------------------------------------- */
/* Serialise everything lpt_step evolves: the particle state of every species
 * in the context's current slot order together with the slot -> particle
 * map (so the cell-order sort and the statistics' summation order carry
 * over), the initial positions and velocities, the time and step count, the
 * statistics records and the device clock.
 * Velocity snapshots are inputs, not state: set them again after a resume.
 * With blob == NULL only *size (the bytes needed) is returned; otherwise
 * cap must be at least that.  Host memory. */
lpt_status lpt_get_state(lpt_ctx *ctx, void *blob, size_t cap, size_t *size);
/* Restore a blob from lpt_get_state into a context created with the same n
 * and precision and given the same species (kind, St, scheme, count) in the
 * same order; anything else is LPT_E_ARG and leaves the context unchanged.
 * Stepping on from the restored context gives the same bits as stepping on
 * from the saved one. */
lpt_status lpt_set_state(lpt_ctx *ctx, const void *blob, size_t size);

/* ---- launch tuning -------------------------------------------------------- */
/* Launch-shape choices of the step path.  None of them changes a
 * per-particle result (positions, displacements and velocities are the same
 * bits with any choice), so an autotuner may pick them for speed.  The
 * statistics are summed per wave of 64 slots and merged in slot order, so the
 * block size and launch shape leave them unchanged too; a different sort
 * interval or sort key reorders the slots and so may change their last bits.
 * They are run-to-run reproducible for fixed choices. */
typedef struct {
    int32_t block_size;     /* particles (slots) per logical block of the step
                               kernel, 64, 128, 256 or 512 (0 selects 256);
                               the threads of its workgroup, unless `rows`
                               below splits it                               */
    int32_t tile_records;   /* as lpt_config.tile_records (0 default, -1 off) */
    int32_t sort_interval;  /* steps between cell-order re-sorts; 0 = never   */
    int32_t persistent;     /* 1: launch only as many workgroups as stay
                               resident; each loops over a contiguous range of
                               blocks of its own XCD                           */
    int32_t graph_chunk;    /* > 0: in PINGPONG mode without
                               LPT_FLAG_TIME_KERNELS, lpt_step captures runs of
                               this many steps (sorts and statistics included)
                               into a hipGraph once and replays it             */
    float halo_scale;       /* LDS tile halo as a multiple of the largest
                               displacement a step can make at the largest node
                               speed, in (0, 4], rounded up to whole cells;
                               0 selects 0.125 (one cell for displacements of
                               up to eight cells a step, 5.1 for Catmull-Rom).
                               Particles whose stencil leaves the tile gather
                               from global memory, so it never affects
                               results                                        */
    int32_t max_workgroups; /* > 0: a persistent launch holds at most this many
                               workgroups (below the resident capacity), so
                               that each walks several logical blocks; 0:
                               the resident capacity                          */
    int32_t fused;          /* with several species, 1 (default) or 2: one
                               step launch covers them all, each XCD taking
                               the same share of every species, species
                               after species (1) or interleaved along the
                               cell order (2); 0: one launch per species
                               (LPT_FP32_SPLIT) or one launch in species
                               order (LPT_FP64)                               */
    int32_t sort_cells;     /* 1: every re-sort key orders the cells inside
                               each T x T tile too (row-major), so that
                               neighbouring slots sit in neighbouring cells;
                               the key grows by 2 log2 T bits and must stay
                               within 32 bits (else LPT_E_ARG); 0: tiles only,
                               ties keep their order; 2 (default): cells on
                               the first re-sort after the particles are
                               placed (where the key fits), tiles after it --
                               the later tile sorts, being stable, keep most
                               of that order                                 */
    int32_t rows;           /* LPT_FP32_SPLIT bilinear tracer step kernels:
                               particles per thread, 1 (0 selects 1) or 2.
                               The block_size slots of a logical block are
                               then run by block_size / rows threads (at
                               least 64), which share one box, tile and
                               set-up; a smaller workgroup holds less LDS at
                               the same occupancy, so the tile's capacity per
                               particle halves.  Other bodies (bicubic,
                               inertial, fused, LPT_FP64) run one particle per
                               thread.  Results do not depend on it          */
} lpt_tuning;

lpt_status lpt_get_tuning(lpt_ctx *ctx, lpt_tuning *out);
/* Validated as a whole; on error nothing changes.  Takes effect at the next
 * step.  Changing the block size reallocates the statistics partials. */
lpt_status lpt_set_tuning(lpt_ctx *ctx, const lpt_tuning *tuning);

/* lpt_step with HIP events recorded on the context stream before and after
 * it; *ms receives the elapsed device time (synchronises).  The autotuner's
 * clock: it covers every launch of the steps, graph replays included. */
lpt_status lpt_time_steps(lpt_ctx *ctx, int64_t nsteps, double dt, int32_t stats_every,
                          double *ms);

/* ---- derivatives of the discrete tracer map (FP64) ---------------------- */
/* The paper has no adjoint.  These entry points differentiate exactly the
 * discrete map that lpt_step computes for tracers (eq. rk4_update with the
 * interpolation of Sec. 3.4 and eq. temporal_interp): inside a cell the cell
 * index is constant, so d(xi)/dx = n/L.  LPT_FP64 contexts whose species are
 * all tracers (or St = 0) only; otherwise LPT_E_STATE. */

/* Advance every species by nsteps steps like lpt_step (no statistics; with
 * sort_interval > 0, a cell-order re-sort at the start of every segment of
 * ckpt_every steps, whose permutation is kept), keeping the positions at
 * every ckpt_every-th step and each step's temporal weights, so that
 * lpt_adjoint / lpt_jacobian can recompute the trajectory segment by
 * segment.  Device memory: ceil(nsteps / ckpt_every) * 16 bytes per particle
 * for the checkpoints (plus 4 bytes per particle and segment for the
 * permutations when re-sorting), and min(ckpt_every, nsteps) * 16 bytes per
 * particle during a reverse sweep. */
lpt_status lpt_forward_checkpointed(lpt_ctx *ctx, int64_t nsteps, double dt, int32_t ckpt_every);

/* Reverse sweep of the last lpt_forward_checkpointed run (no step may follow
 * it) for L = sum_p (gx_T[p] x_T,p + gy_T[p] y_T,p), x_T the final
 * unwrapped position, p the global particle index (species concatenated in
 * the order they were added).  Outputs (any may be NULL):
 *   gx_0, gy_0: dL/dx_0, dL/dy_0 per particle (np doubles each);
 *   gU: dL/d(grid value), [slot 0, 1][u, v][n][n] doubles (4 n^2),
 *       x fastest; summed with FP64 atomics, so the last bits depend on
 *       scheduling, unless the context has LPT_FLAG_DETERMINISTIC_GRAD
 *       (then bit-reproducible).
 * All arrays are host or device memory per on_device. */
lpt_status lpt_adjoint(lpt_ctx *ctx, const double *gx_T, const double *gy_T, double *gx_0,
                       double *gy_0, double *gU, int32_t on_device);

/* Jacobian F = d x_T / d x_0 of every particle of the last
 * lpt_forward_checkpointed run, by a reverse sweep with two adjoint vectors:
 * F[4p + 0..3] = dx_T/dx_0, dx_T/dy_0, dy_T/dx_0, dy_T/dy_0 (row-major
 * 2x2; finite-time Lyapunov exponent (1/T) ln sqrt(lambda_max(F^T F))).
 * np * 4 doubles, host or device memory per on_device. */
lpt_status lpt_jacobian(lpt_ctx *ctx, double *F, int32_t on_device);

/* Finite-time Lyapunov exponent of every particle over the last
 * lpt_forward_checkpointed run of nsteps steps of size dt:
 * sigma[p] = (1/T) ln sqrt(lambda_max(F^T F)), T = nsteps * dt, F the
 * Jacobian of lpt_jacobian (from the same reverse sweep; F may be NULL,
 * else it receives the Jacobians as lpt_jacobian writes them).  np doubles
 * (4 np for F) in original particle order, host or device memory per
 * on_device.  Errors as lpt_jacobian. */
lpt_status lpt_ftle(lpt_ctx *ctx, double *sigma, double *F, int32_t on_device);

/* ---- primitives exposed for verification -------------------------------- */

/* Evaluate the interpolated fluid velocity at npts points with the given
 * temporal weights (u = w_a * I[slot 0] + w_b * I[slot 1]), through the same
 * device code the step kernel uses, in the context's precision.  x, y, u, v:
 * npts doubles each. */
lpt_status lpt_interp(lpt_ctx *ctx, lpt_scheme scheme, int64_t npts, const double *x,
                      const double *y, double w_a, double w_b, double *u, double *v,
                      int32_t on_device);

/* Stable ascending sort of npts 32-bit keys by the library's LSD radix sort
 * (8-bit digits over the low key_bits bits, 1 <= key_bits <= 32).  keys_out
 * and perm (perm[r] = input index of the r-th smallest key) may be NULL.
 * All pointers are device memory. */
lpt_status lpt_radix_sort(lpt_ctx *ctx, int64_t npts, int32_t key_bits,
                          const uint32_t *keys_in, uint32_t *keys_out, uint32_t *perm);

/* lpt_radix_sort for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same stable sort and the same results, through a fixed scratch array
 * that the library holds on every GPU it runs on (16.3 MiB, for the life
 * of the process), so the call allocates nothing and does not synchronise.
 * npts <= LPT_STATIC_SORT_MAX, else LPT_E_ARG.  All pointers are device
 * memory; the results are in keys_out / perm once the context's stream has
 * reached the call.  Every call on one GPU uses the same scratch: calls that
 * overlap on one GPU (other streams, other threads, other contexts) race. */
#define LPT_STATIC_SORT_MAX 1048576
lpt_status lpt_radix_sort_static(lpt_ctx *ctx, int64_t npts, int32_t key_bits,
                                 const uint32_t *keys_in, uint32_t *keys_out, uint32_t *perm);

/* Achievable device-memory bandwidth: a plain copy of `bytes` (rounded down
 * to a multiple of 16) between two device buffers, and a STREAM triad
 * a = b + s*c over three such buffers, each repeated `iters` times on the
 * context stream.  GB/s counts bytes read plus bytes written (copy: 2*bytes
 * per pass, triad: 3*bytes).  The buffers are allocated and freed inside. */
lpt_status lpt_bw_probe(lpt_ctx *ctx, int64_t bytes, int32_t iters, double *copy_gbps,
                        double *triad_gbps);

#ifdef __cplusplus
}
#endif
#endif /* LPT_H */
