/*
 * ns2d.h -- C ABI of the MI355X (gfx950) Eulerian field producer, libns2d.so.
 *
 * Decaying two-dimensional incompressible Navier-Stokes flow on the doubly
 * periodic square [0, L)^2 in vorticity-streamfunction form, advanced by the
 * Fourier pseudospectral method of Sec. 3.1 of Maiti & Ganesh, "A coupled
 * Eulerian-Lagrangian approach for fluid and particle dynamics":
 *   - spectral derivatives of the vorticity (eq. spectral_vorticity_derivatives);
 *   - the stream function from omega = -lap psi, zero mode zero
 *     (eq. poisson_spectral); the velocity u = dpsi/dy, v = -dpsi/dx
 *     (eq. spectral_velocity);
 *   - the advection term u domega/dx + v domega/dy formed on the grid and
 *     transformed forward (eq. spectral_nonlinear_term), 2/3-dealiased;
 *   - the viscous term -nu |k|^2 omega_hat (eq. spectral_vorticity_evolution,
 *     isotropic nu);
 *   - second-order Adams-Bashforth in spectral space (eq. ab2_fluid); the
 *     first step after ns2d_set_vorticity is forward Euler (the method has
 *     no earlier right-hand side);
 *   - FP64 real-to-complex / complex-to-real transforms; the fields on the
 *     grid carry the 1/(n*n) normalisation.
 * Dealiasing keeps a mode when 3|m| < n on both axes (m the signed integer
 * mode index, wavenumber k = 2 pi m / L), the largest alias-free band; the
 * state is kept inside it (the initial vorticity is truncated to it).
 *
 * It is the step before the particle path: after each ns2d_step the velocity
 * on the grid (ns2d_velocity) is the next time level for lpt_set_snapshot
 * with on_device = 1, in stream order, without a copy to the host.
 *
 * Grid convention (the same as lpt.h): node (i, j) at (i*h, j*h), h = L/n;
 * every field array is [n][n] with x fastest (element j*n + i).
 *
 * Conventions for every entry point:
 *   - The return value is an ns2d_status; no C++ exception crosses the ABI.
 *   - Arguments are validated before anything is enqueued; on an error the
 *     context is left as it was and ns2d_last_error() says why.
 *   - Work is enqueued on the context's HIP stream and the call returns
 *     without waiting, unless it copies into host memory (then it
 *     synchronises the stream first).
 *   - "on_device" = 1: the pointer is device memory on the context's device;
 *     0: host memory.  Inputs are copied; outputs go into caller buffers.
 *   - A context is not thread-safe.
 */
#ifndef NS2D_H
#define NS2D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ns2d_ctx ns2d_ctx;

typedef enum {
    NS2D_OK = 0,
    NS2D_E_ARG = 1,     /* invalid argument                                    */
    NS2D_E_STATE = 2,   /* call not valid in the current state                 */
    NS2D_E_NOMEM = 4,   /* device allocation failed                            */
    NS2D_E_HIP = 5,     /* HIP runtime error                                   */
    NS2D_E_FFT = 6      /* hipFFT plan or execution error                      */
} ns2d_status;

typedef struct {
    int32_t n;          /* grid points per side: even, 8 <= n <= 16384          */
    double length;      /* domain side L > 0; 0 selects 2*pi                    */
    double nu;          /* kinematic viscosity >= 0                             */
    double dt;          /* time step > 0                                        */
    void *hip_stream;   /* hipStream_t to enqueue on; NULL = null stream        */
    int32_t transforms; /* 0 (default) or 2: the library's own LDS
                           transforms, fused with the pointwise work, for n
                           a power of two from 64 to 4096 (else NS2D_E_ARG);
                           1: hipFFT, for any even n (a cross-check path,
                           and the only one for other n)                    */
} ns2d_config;

/* Create a context on the current HIP device: allocates the spectral state,
 * the AB2 history, four spectral and five grid work fields (about 11 n^2
 * doubles in total, 1.5 GB at n = 4096) and either the twiddle table of the
 * built-in transforms or the three hipFFT plans and their work areas.
 * NS2D_E_ARG for a size or option outside the limits. */
ns2d_status ns2d_create(const ns2d_config *cfg, ns2d_ctx **out);
/* Release every resource of the context (NULL is a no-op). */
void ns2d_destroy(ns2d_ctx *ctx);
/* Message of the last failed call ("" if none); lives until the next call. */
const char *ns2d_last_error(const ns2d_ctx *ctx);
/* Block until all work enqueued by the context has finished. */
ns2d_status ns2d_synchronize(ns2d_ctx *ctx);

/* Initial vorticity omega [n][n] (host or device).  Transforms it, keeps the
 * dealiased band, resets the AB2 history and the step count, and
 * reconstructs the velocity on the grid. */
ns2d_status ns2d_set_vorticity(ns2d_ctx *ctx, const double *omega, int32_t on_device);

/* Advance `count` >= 0 steps of dt (eq. ab2_fluid).  NS2D_E_STATE before
 * ns2d_set_vorticity. */
ns2d_status ns2d_step(ns2d_ctx *ctx, int32_t count);

/* Device pointers to the current velocity components on the grid, [n][n]
 * each.  They stay valid until ns2d_destroy, and their contents change at
 * the next ns2d_step or ns2d_set_vorticity: a consumer on another stream must
 * finish reading them first. */
ns2d_status ns2d_velocity(ns2d_ctx *ctx, const double **u, const double **v);

/* Copy the current fields on the grid into caller buffers of n*n doubles:
 * velocity (u, v), vorticity and stream function.  Any pointer may be NULL. */
ns2d_status ns2d_get_fields(ns2d_ctx *ctx, double *u, double *v, double *omega, double *psi,
                            int32_t on_device);

/* *builtin = 1 when the context uses its own transforms, 0 for hipFFT. */
ns2d_status ns2d_get_transforms(const ns2d_ctx *ctx, int32_t *builtin);

/* Steps taken since the last ns2d_set_vorticity. */
ns2d_status ns2d_get_steps(const ns2d_ctx *ctx, int64_t *steps);

#ifdef __cplusplus
}
#endif
#endif
