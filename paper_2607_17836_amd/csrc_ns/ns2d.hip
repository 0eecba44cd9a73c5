// Eulerian field producer: pseudospectral vorticity-streamfunction solver of
// Sec. 3.1 on gfx950 (C ABI in ns2d.h).
//
// One step, with the grid fields (u, v, dw/dx, dw/dy) of the current level
// already resident:
//   1. product kernel: N = u dw/dx + v dw/dy on the grid (one pass over HBM);
//   2. hipFFT D2Z of N;
//   3. spectral kernel, one thread per half-plane mode: the 2/3 band, the
//      right-hand side -N - nu k^2 w (eq. spectral_vorticity_evolution), the
//      AB2 update (eq. ab2_fluid) with the previous right-hand side kept in
//      HBM, then the Poisson solve (eq. poisson_spectral) and the four
//      spectral fields i k_y psi, -i k_x psi (eq. spectral_velocity),
//      i k_x w, i k_y w (eq. spectral_vorticity_derivatives), pre-scaled by
//      1/n^2 so that the inverse transforms come out normalised;
//   4. one batched hipFFT Z2D of the four fields.
// Every pointwise operation lives in the two kernels, so each step reads and
// writes each spectral array once.
//
// For every power of two n from 64 to 4096 (the default) the built-in
// transforms (fft_lds.h) replace the library's (which stay available as an
// explicit cross-check, and for other n) and fuse with the pointwise work,
// in four kernels a step
// over a transposed spectral layout (entry (row jy, column ix) of a
// half-plane spectrum at ix * n + jy, so that every column is contiguous)
// that holds only the columns inside the 2/3 band:
//   a. fwd_rows_kernel: the grid product of a slab of rows, two real rows
//      packed into one complex transform along x, unpacked into two half
//      spectra;
//   b. column_fwd_kernel: per band column, the transform along y, the band
//      and the AB2 update; column_emit_kernel: per band column and field,
//      the field's values and its inverse transform along y;
//   c. inv_rows_kernel: two rows of each field packed into one complex
//      inverse transform along x (Hermitian extension), written as grid rows.
// Each spectral array is read and written once per step and the grid
// advection term never reaches HBM.
#include <hip/hip_runtime.h>
#include <hipfft/hipfft.h>

#include <cmath>
#include <cstdio>
#include <new>
#include <string>
#include <vector>

#include "fft_lds.h"
#include "ns2d.h"

namespace {

constexpr int kBlock = 256;

struct Spec {
    int n, nh;        // grid side, half-plane width n/2 + 1
    double kscale;    // 2 pi / L
    double nu, dt;
    double inv_nn;    // 1 / n^2
    size_t plane;     // n * nh complex entries per spectral field
};

// Signed mode index of row j of a length-n transform (rows n/2 .. n-1 hold
// the negative modes).
__device__ __forceinline__ int signed_mode(int j, int n) { return j < n / 2 ? j : j - n; }

// 2/3 rule: a mode is kept when 3|m| < n on both axes.
__device__ __forceinline__ bool in_band(int mx, int my, int n)
{
    return 3 * abs(mx) < n && 3 * abs(my) < n;
}

// The four spectral fields of vorticity w at wavenumber (kx, ky), scaled by
// 1/n^2, into the four planes of `out`.
__device__ __forceinline__ void emit_fields(double2 *__restrict__ out, size_t idx, size_t plane,
                                            double kx, double ky, double2 w, double s)
{
    const double k2 = kx * kx + ky * ky;
    double2 p = make_double2(0.0, 0.0);
    if (k2 > 0.0) p = make_double2(w.x / k2, w.y / k2);
    // i a z = (-a z.y, a z.x)
    out[idx] = make_double2(-ky * p.y * s, ky * p.x * s);                  // u  =  i k_y psi
    out[idx + plane] = make_double2(kx * p.y * s, -kx * p.x * s);          // v  = -i k_x psi
    out[idx + 2 * plane] = make_double2(-kx * w.y * s, kx * w.x * s);      // dw/dx
    out[idx + 3 * plane] = make_double2(-ky * w.y * s, ky * w.x * s);      // dw/dy
}

__global__ __launch_bounds__(kBlock) void product_kernel(const double2 *__restrict__ u,
                                                         const double2 *__restrict__ v,
                                                         const double2 *__restrict__ wx,
                                                         const double2 *__restrict__ wy,
                                                         double2 *__restrict__ out, size_t count2)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count2; i += stride) {
        const double2 a = u[i], b = v[i], c = wx[i], d = wy[i];
        out[i] = make_double2(a.x * c.x + b.x * d.x, a.y * c.y + b.y * d.y);
    }
}

// After the forward transform of the initial vorticity: keep the band and
// emit the fields of that state.
__global__ __launch_bounds__(kBlock) void init_kernel(double2 *__restrict__ w_hat,
                                                      double2 *__restrict__ fields, Spec S)
{
    const int ix = blockIdx.x * kBlock + threadIdx.x, jy = blockIdx.y;
    if (ix >= S.nh) return;
    const size_t idx = (size_t)jy * S.nh + ix;
    const int my = signed_mode(jy, S.n);
    double2 w = w_hat[idx];
    if (!in_band(ix, my, S.n)) w = make_double2(0.0, 0.0);
    w_hat[idx] = w;
    emit_fields(fields, idx, S.plane, S.kscale * ix, S.kscale * my, w, S.inv_nn);
}

// One AB2 step in spectral space.  Plane 0 of `fields` holds the forward
// transform of the advection term on entry; all four planes are overwritten
// with the new level's fields (each thread reads its entry before writing).
template <bool FIRST>
__global__ __launch_bounds__(kBlock) void ab2_kernel(double2 *__restrict__ w_hat,
                                                     double2 *__restrict__ r_prev,
                                                     double2 *__restrict__ fields, Spec S)
{
    const int ix = blockIdx.x * kBlock + threadIdx.x, jy = blockIdx.y;
    if (ix >= S.nh) return;
    const size_t idx = (size_t)jy * S.nh + ix;
    const int my = signed_mode(jy, S.n);
    const double kx = S.kscale * ix, ky = S.kscale * my;
    const double k2 = kx * kx + ky * ky;
    const double2 w = w_hat[idx];
    double2 N = fields[idx];
    if (!in_band(ix, my, S.n)) N = make_double2(0.0, 0.0);
    const double visc = S.nu * k2;
    const double2 r = make_double2(-N.x - visc * w.x, -N.y - visc * w.y);
    const double2 r_old = FIRST ? r : r_prev[idx];
    const double2 wn = make_double2(w.x + S.dt * (1.5 * r.x - 0.5 * r_old.x),
                                    w.y + S.dt * (1.5 * r.y - 0.5 * r_old.y));
    w_hat[idx] = wn;
    r_prev[idx] = r;
    emit_fields(fields, idx, S.plane, kx, ky, wn, S.inv_nn);
}

// omega_hat / n^2 (which = 0) or psi_hat / n^2 (which = 1) into one plane.
__global__ __launch_bounds__(kBlock) void scaled_kernel(const double2 *__restrict__ w_hat,
                                                        double2 *__restrict__ out, Spec S,
                                                        int which)
{
    const int ix = blockIdx.x * kBlock + threadIdx.x, jy = blockIdx.y;
    if (ix >= S.nh) return;
    const size_t idx = (size_t)jy * S.nh + ix;
    const int my = signed_mode(jy, S.n);
    const double kx = S.kscale * ix, ky = S.kscale * my;
    const double k2 = kx * kx + ky * ky;
    double2 w = w_hat[idx];
    if (which == 1) w = k2 > 0.0 ? make_double2(w.x / k2, w.y / k2) : make_double2(0.0, 0.0);
    out[idx] = make_double2(w.x * S.inv_nn, w.y * S.inv_nn);
}

// ---- built-in transform path (n = 64, 128, ..., 4096) ---------------------

// Grid rows per row-pass block: four (two packed complex rows, 2N entries of
// LDS) at N = 2048, two (one packed row) elsewhere: below 2048 twice as many
// blocks fill the chip better (measured: 1024^2 step 71.9 -> 61.1 us; 2048^2
// step 163 -> 167 us with two), and at 4096 one packed row is 64 KiB of LDS.
template <int N>
constexpr int rows_per_block() { return N == 2048 ? 4 : 2; }

// Inverse row pass: one block per field and slab (1024^2 step 56.1 -> 52.3
// us, 512^2 33.1 -> 30.7 us), except at 2048, where one block per slab walks
// the four fields (161 us a step against 185 with a block per field).
template <int N>
constexpr bool field_blocks() { return N != 2048; }

// Contiguous logical block ranges per XCD (workgroups go to the eight XCDs
// round-robin): XCD x = b mod 8 takes logical blocks [x G/8, (x+1) G/8) up to
// the remainder, so consecutive logical blocks share an L2.
__device__ __forceinline__ int xcd_block(int b, int G)
{
    const int x = b % 8, k = b / 8, q = G / 8, r = G % 8;
    return x < r ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

// Row slab of a row-pass block.  Workgroups go to the eight XCDs round-robin;
// XCD x takes the contiguous slabs [x G/8, (x+1) G/8) (G = N / rows per
// block, a multiple of 8 for every built-in size), so the two slabs that share each
// 128-byte line of a transposed column run on one XCD and share its L2.
template <int N>
__device__ __forceinline__ int row_slab()
{
    constexpr int G = N / rows_per_block<N>();
    static_assert(G % 8 == 0, "slabs split evenly over the XCDs");
    return (int)(blockIdx.x % 8) * (G / 8) + (int)(blockIdx.x / 8);
}

// Columns ix = 0 .. band_cols(N) - 1 are the ones with 3 ix < N.  Every other
// column of the band-limited state, of the four fields and of the read-back
// fields is zero, so the built-in path neither transforms nor stores it:
// the row passes skip it and the inverse row pass supplies the zeros.
constexpr int band_cols(int N) { return (N - 1) / 3 + 1; }

// One slab of rows (rows_per_block) of the advection term (PRODUCT: u dw/dx + v dw/dy from the
// four grid fields at g) or of one grid field (g), transformed along x:
// rows (a, b) form z = a + i b, Z = FFT(z), and the half spectra are
// A(k) = (Z(k) + conj Z(-k)) / 2, B(k) = (Z(k) - conj Z(-k)) / (2i).
template <int N, bool PRODUCT>
__global__ __launch_bounds__(N / 8) void fwd_rows_kernel(const double *__restrict__ g,
                                                        double2 *__restrict__ specT,
                                                        const double2 *__restrict__ W)
{
    extern __shared__ double2 lds_rows[];   // kPairs packed rows of N entries
    constexpr int T = N / 8;
    constexpr size_t cells = (size_t)N * N;
    constexpr int kPairs = rows_per_block<N>() / 2;
    const int jy0 = row_slab<N>() * rows_per_block<N>();
    for (int p = 0; p < kPairs; ++p) {
        double2 *buf = lds_rows + p * N;
        const double *ra = g + (size_t)(jy0 + 2 * p) * N;
        const double *rb = ra + N;
        for (int x = threadIdx.x; x < N; x += T) {
            double a, b;
            if constexpr (PRODUCT) {
                a = ra[x] * ra[x + 2 * cells] + ra[x + cells] * ra[x + 3 * cells];
                b = rb[x] * rb[x + 2 * cells] + rb[x + cells] * rb[x + 3 * cells];
            } else {
                a = ra[x];
                b = rb[x];
            }
            buf[x] = make_double2(a, b);
        }
    }
    __syncthreads();
    for (int p = 0; p < kPairs; ++p) ns_fft::fft<N, false>(lds_rows + p * N, W);
    constexpr int KB = band_cols(N);
    for (int e = threadIdx.x; e < kPairs * KB; e += T) {
        const int k = e / kPairs, p = e % kPairs;
        const double2 *buf = lds_rows + p * N;
        const double2 z = buf[k], zc = buf[(N - k) & (N - 1)];
        double2 *dst = specT + (size_t)k * N + jy0 + 2 * p;
        dst[0] = make_double2(0.5 * (z.x + zc.x), 0.5 * (z.y - zc.y));
        dst[1] = make_double2(0.5 * (z.y + zc.y), -0.5 * (z.x - zc.x));
    }
}

enum ColumnMode { kColInit = 0, kColFirst = 1, kColStep = 2 };

// Column ix < band_cols(N) of the transposed spectra, one block per column:
// plane 0 of `fields` (the x-transformed rows) transformed along y, the band
// taken, and the state stored (init) or advanced by AB2 (step).
template <int N, int MODE>
__global__ __launch_bounds__(N / 8) void column_fwd_kernel(double2 *__restrict__ w_hat,
                                                          double2 *__restrict__ r_prev,
                                                          const double2 *__restrict__ fields,
                                                          Spec S, const double2 *__restrict__ W)
{
    extern __shared__ double2 lds_col[];   // N entries
    constexpr int T = N / 8;
    const int ix = blockIdx.x, t = threadIdx.x;
    const size_t col = (size_t)ix * N;
    const double kx = S.kscale * ix;
#pragma unroll
    for (int q = 0; q < 8; ++q) lds_col[t + q * T] = fields[col + t + q * T];
    __syncthreads();
    ns_fft::fft<N, false>(lds_col, W);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int jy = t + q * T;
        const size_t idx = col + jy;
        const int my = signed_mode(jy, N);
        const double2 Nh = in_band(ix, my, N) ? lds_col[jy] : make_double2(0.0, 0.0);
        if constexpr (MODE == kColInit) {
            w_hat[idx] = Nh;
        } else {
            const double ky = S.kscale * my;
            const double visc = S.nu * (kx * kx + ky * ky);
            const double2 w = w_hat[idx];
            const double2 r = make_double2(-Nh.x - visc * w.x, -Nh.y - visc * w.y);
            const double2 r_old = MODE == kColFirst ? r : r_prev[idx];
            w_hat[idx] = make_double2(w.x + S.dt * (1.5 * r.x - 0.5 * r_old.x),
                                      w.y + S.dt * (1.5 * r.y - 0.5 * r_old.y));
            r_prev[idx] = r;
        }
    }
}

enum EmitMode { kEmitFields = 0, kEmitW = 1, kEmitPsi = 2 };

// One field of one band column, transformed back along y: the four fields
// u = i k_y psi, v = -i k_x psi, dw/dx = i k_x w, dw/dy = i k_y w (emit
// mode), or omega or psi alone (read-back modes), each scaled by 1/n^2.
// Logical block l = column * nf + field, so a column's fields run on one XCD
// and re-read its state from that L2.
template <int N, int MODE>
__global__ __launch_bounds__(N / 8) void column_emit_kernel(const double2 *__restrict__ w_hat,
                                                           double2 *__restrict__ fields, Spec S,
                                                           const double2 *__restrict__ W)
{
    extern __shared__ double2 lds_col[];   // N entries
    constexpr int T = N / 8;
    constexpr int nf = MODE == kEmitFields ? 4 : 1;
    const int l = xcd_block(blockIdx.x, band_cols(N) * nf);
    const int ix = l / nf, f = l % nf, t = threadIdx.x;
    const size_t col = (size_t)ix * N;
    const double kx = S.kscale * ix, s = S.inv_nn;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int jy = t + q * T;
        const double ky = S.kscale * signed_mode(jy, N);
        const double k2 = kx * kx + ky * ky;
        const double2 w = w_hat[col + jy];
        double2 p = make_double2(0.0, 0.0);
        if (k2 > 0.0) p = make_double2(w.x / k2, w.y / k2);
        double2 v;
        if constexpr (MODE == kEmitW) v = make_double2(w.x * s, w.y * s);
        else if constexpr (MODE == kEmitPsi) v = make_double2(p.x * s, p.y * s);
        else if (f == 0) v = make_double2(-ky * p.y * s, ky * p.x * s);    // u  =  i k_y psi
        else if (f == 1) v = make_double2(kx * p.y * s, -kx * p.x * s);    // v  = -i k_x psi
        else if (f == 2) v = make_double2(-kx * w.y * s, kx * w.x * s);    // dw/dx
        else v = make_double2(-ky * w.y * s, ky * w.x * s);                // dw/dy
        lds_col[jy] = v;
    }
    __syncthreads();
    ns_fft::fft<N, true>(lds_col, W);
    double2 *dst = fields + (size_t)f * S.plane + col;
#pragma unroll
    for (int q = 0; q < 8; ++q) dst[t + q * T] = lds_col[t + q * T];
}

// One slab of rows (rows_per_block) of one or all nf fields (planes of the
// transposed spectra, already transformed along y; see field_blocks) back
// to the grid: rows (a, b) of a field form
// Z(k) = A(k) + i B(k) and Z(N-k) = conj A(k) + i conj B(k) for the band
// columns k < KB (the imaginary parts at k = 0 dropped as in any
// complex-to-real transform) and zero elsewhere; z = IFFT(Z) gives a = Re z,
// b = Im z.
template <int N>
__global__ __launch_bounds__(N / 8) void inv_rows_kernel(const double2 *__restrict__ fields,
                                                        double *__restrict__ grid, int nf,
                                                        size_t plane,
                                                        const double2 *__restrict__ W)
{
    extern __shared__ double2 lds_rows[];   // kPairs packed rows of N entries
    constexpr int T = N / 8, KB = band_cols(N);
    constexpr int kPairs = rows_per_block<N>() / 2, G = N / rows_per_block<N>();
    constexpr size_t cells = (size_t)N * N;
    int f0, f1, jy0;
    if constexpr (field_blocks<N>()) {
        // one block per (field, slab); a field's adjacent slabs share an XCD
        const int l = xcd_block(blockIdx.x, nf * G);
        f0 = l / G;
        f1 = f0 + 1;
        jy0 = (l % G) * rows_per_block<N>();
    } else {
        f0 = 0;
        f1 = nf;
        jy0 = row_slab<N>() * rows_per_block<N>();
    }
    for (int f = f0; f < f1; ++f) {
        const double2 *src = fields + (size_t)f * plane;
        for (int e = threadIdx.x; e < kPairs * KB; e += T) {
            const int k = e / kPairs, p = e % kPairs;
            const double2 *sp = src + (size_t)k * N + jy0 + 2 * p;
            double2 A = sp[0], B = sp[1];
            if (k == 0) {
                A.y = 0.0;
                B.y = 0.0;
            }
            double2 *buf = lds_rows + p * N;
            buf[k] = make_double2(A.x - B.y, A.y + B.x);
            if (k > 0) buf[N - k] = make_double2(A.x + B.y, B.x - A.y);
        }
        // columns KB .. N/2 and their mirrors N/2 .. N-KB are zero
        for (int x = KB + threadIdx.x; x <= N - KB; x += T)
            for (int p = 0; p < kPairs; ++p) lds_rows[p * N + x] = make_double2(0.0, 0.0);
        __syncthreads();
        for (int p = 0; p < kPairs; ++p) ns_fft::fft<N, true>(lds_rows + p * N, W);
        for (int p = 0; p < kPairs; ++p) {
            double *ra = grid + (size_t)f * cells + (size_t)(jy0 + 2 * p) * N;
            for (int x = threadIdx.x; x < N; x += T) {
                const double2 z = lds_rows[p * N + x];
                ra[x] = z.x;
                ra[x + N] = z.y;
            }
        }
        __syncthreads();   // lds_rows is refilled for the next field
    }
}

}  // namespace

struct ns2d_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int n = 0, nh = 0;
    double L = 0, nu = 0, dt = 0;
    double2 *w_hat = nullptr, *r_prev = nullptr, *fields = nullptr;   // fields: 4 planes
    double *grid = nullptr;   // 4 grid fields: u, v, dw/dx, dw/dy
    double *tmp = nullptr;    // grid scratch: advection term, read-back transforms
    hipfftHandle r2c = 0, c2r4 = 0, c2r1 = 0;
    bool r2c_ok = false, c2r4_ok = false, c2r1_ok = false;
    bool builtin = false;        // built-in transforms, transposed spectral layout
    double2 *twiddle = nullptr;  // exp(-2 pi i m / n), m < n (built-in path)
    bool have_state = false, first = true;
    int64_t steps = 0;
    std::string err;
};

namespace {

ns2d_status fail(ns2d_ctx *c, ns2d_status s, const std::string &msg)
{
    if (c) c->err = msg;
    return s;
}

#define NS_HIP(c, expr)                                                                  \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail((c), NS2D_E_HIP, std::string(#expr ": ") + hipGetErrorString(e_)); \
    } while (0)

#define NS_FFT(c, expr)                                                                  \
    do {                                                                                 \
        hipfftResult r_ = (expr);                                                        \
        if (r_ != HIPFFT_SUCCESS)                                                        \
            return fail((c), NS2D_E_FFT, std::string(#expr " failed, hipfftResult ") +     \
                                             std::to_string((int)r_));                   \
    } while (0)

Spec make_spec(const ns2d_ctx *c)
{
    Spec S;
    S.n = c->n;
    S.nh = c->nh;
    S.kscale = 2.0 * M_PI / c->L;
    S.nu = c->nu;
    S.dt = c->dt;
    S.inv_nn = 1.0 / ((double)c->n * (double)c->n);
    S.plane = (size_t)c->n * c->nh;
    return S;
}

dim3 spectral_grid(const ns2d_ctx *c) { return dim3((c->nh + kBlock - 1) / kBlock, c->n); }

void release(ns2d_ctx *c)
{
    if (c->r2c_ok) hipfftDestroy(c->r2c);
    if (c->c2r4_ok) hipfftDestroy(c->c2r4);
    if (c->c2r1_ok) hipfftDestroy(c->c2r1);
    if (c->w_hat) (void)hipFree(c->w_hat);
    if (c->r_prev) (void)hipFree(c->r_prev);
    if (c->fields) (void)hipFree(c->fields);
    if (c->grid) (void)hipFree(c->grid);
    if (c->tmp) (void)hipFree(c->tmp);
    if (c->twiddle) (void)hipFree(c->twiddle);
}

enum BuiltinOp { kOpInit, kOpStep, kOpReadW, kOpReadPsi };

template <int N>
ns2d_status run_builtin_n(ns2d_ctx *c, BuiltinOp op)
{
    constexpr int T = N / 8;
    constexpr int kPairs = rows_per_block<N>() / 2;
    const size_t rows_lds = kPairs * (size_t)N * sizeof(double2);
    const size_t col_lds = (size_t)N * sizeof(double2);
    const dim3 rows_grid(N / rows_per_block<N>()), col_grid(band_cols(N));
    const Spec S = make_spec(c);
    hipStream_t st = c->stream;
    const double2 *Wt = c->twiddle;
    const dim3 emit4_grid(4 * band_cols(N)), emit1_grid(band_cols(N));
    const dim3 inv4_grid(field_blocks<N>() ? 4 * rows_grid.x : rows_grid.x);
    switch (op) {
    case kOpInit:
        fwd_rows_kernel<N, false><<<rows_grid, T, rows_lds, st>>>(c->tmp, c->fields, Wt);
        column_fwd_kernel<N, kColInit><<<col_grid, T, col_lds, st>>>(c->w_hat, c->r_prev, c->fields, S, Wt);
        column_emit_kernel<N, kEmitFields><<<emit4_grid, T, col_lds, st>>>(c->w_hat, c->fields, S, Wt);
        inv_rows_kernel<N><<<inv4_grid, T, rows_lds, st>>>(c->fields, c->grid, 4, S.plane, Wt);
        break;
    case kOpStep:
        fwd_rows_kernel<N, true><<<rows_grid, T, rows_lds, st>>>(c->grid, c->fields, Wt);
        if (c->first)
            column_fwd_kernel<N, kColFirst><<<col_grid, T, col_lds, st>>>(c->w_hat, c->r_prev, c->fields, S, Wt);
        else
            column_fwd_kernel<N, kColStep><<<col_grid, T, col_lds, st>>>(c->w_hat, c->r_prev, c->fields, S, Wt);
        column_emit_kernel<N, kEmitFields><<<emit4_grid, T, col_lds, st>>>(c->w_hat, c->fields, S, Wt);
        inv_rows_kernel<N><<<inv4_grid, T, rows_lds, st>>>(c->fields, c->grid, 4, S.plane, Wt);
        break;
    case kOpReadW:
    case kOpReadPsi:
        if (op == kOpReadW)
            column_emit_kernel<N, kEmitW><<<emit1_grid, T, col_lds, st>>>(c->w_hat, c->fields, S, Wt);
        else
            column_emit_kernel<N, kEmitPsi><<<emit1_grid, T, col_lds, st>>>(c->w_hat, c->fields, S, Wt);
        inv_rows_kernel<N><<<rows_grid, T, rows_lds, st>>>(c->fields, c->tmp, 1, S.plane, Wt);
        break;
    }
    NS_HIP(c, hipGetLastError());
    return NS2D_OK;
}

ns2d_status run_builtin(ns2d_ctx *c, BuiltinOp op)
{
    switch (c->n) {
    case 64: return run_builtin_n<64>(c, op);
    case 128: return run_builtin_n<128>(c, op);
    case 256: return run_builtin_n<256>(c, op);
    case 512: return run_builtin_n<512>(c, op);
    case 1024: return run_builtin_n<1024>(c, op);
    case 2048: return run_builtin_n<2048>(c, op);
    case 4096: return run_builtin_n<4096>(c, op);
    default: return fail(c, NS2D_E_STATE, "no built-in transform for this n");
    }
}

// The four spectral planes to the four grid fields.
ns2d_status to_grid4(ns2d_ctx *c)
{
    NS_FFT(c, hipfftExecZ2D(c->c2r4, reinterpret_cast<hipfftDoubleComplex *>(c->fields), c->grid));
    return NS2D_OK;
}

ns2d_status copy_out(ns2d_ctx *c, double *dst, const double *src, int32_t on_device)
{
    const size_t bytes = (size_t)c->n * c->n * sizeof(double);
    NS_HIP(c, hipMemcpyAsync(dst, src, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                             c->stream));
    return NS2D_OK;
}

}  // namespace

extern "C" {

ns2d_status ns2d_create(const ns2d_config *cfg, ns2d_ctx **out)
{
    if (!cfg || !out) return NS2D_E_ARG;
    *out = nullptr;
    const int n = cfg->n;
    const double L = cfg->length == 0.0 ? 2.0 * M_PI : cfg->length;
    if (n < 8 || n > 16384 || (n & 1)) return NS2D_E_ARG;
    if (!(L > 0.0) || !std::isfinite(L)) return NS2D_E_ARG;
    if (!(cfg->nu >= 0.0) || !std::isfinite(cfg->nu)) return NS2D_E_ARG;
    if (!(cfg->dt > 0.0) || !std::isfinite(cfg->dt)) return NS2D_E_ARG;
    if (cfg->transforms < 0 || cfg->transforms > 2) return NS2D_E_ARG;
    // the built-in transforms (transforms 0 or 2) exist for powers of two
    // from 64 to 4096; hipFFT only on request (transforms 1)
    const bool own = cfg->transforms != 1;
    if (own && (n < 64 || n > 4096 || (n & (n - 1)))) return NS2D_E_ARG;
    ns2d_ctx *c = new (std::nothrow) ns2d_ctx;
    if (!c) return NS2D_E_NOMEM;
    c->n = n;
    c->nh = n / 2 + 1;
    c->L = L;
    c->nu = cfg->nu;
    c->dt = cfg->dt;
    c->stream = reinterpret_cast<hipStream_t>(cfg->hip_stream);
    auto bail = [&](ns2d_status s) {
        release(c);
        delete c;
        return s;
    };
    if (hipGetDevice(&c->device) != hipSuccess) return bail(NS2D_E_HIP);
    const size_t plane = (size_t)n * c->nh, cells = (size_t)n * n;
    if (hipMalloc(&c->w_hat, plane * sizeof(double2)) != hipSuccess ||
        hipMalloc(&c->r_prev, plane * sizeof(double2)) != hipSuccess ||
        hipMalloc(&c->fields, 4 * plane * sizeof(double2)) != hipSuccess ||
        hipMalloc(&c->grid, 4 * cells * sizeof(double)) != hipSuccess ||
        hipMalloc(&c->tmp, cells * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        return bail(NS2D_E_NOMEM);
    }
    // measured faster than hipFFT at the sizes compared (2048^2: 161 vs 337
    // us a step; 1024^2: 53 vs 101; 512^2: 31 vs 43)
    c->builtin = own;
    if (c->builtin) {
        // twiddles from the long-double cosine and sine, rounded once
        std::vector<double2> w(n);
        for (int m = 0; m < n; ++m) {
            const long double a = 2.0L * 3.14159265358979323846264338327950288L * m / n;
            w[m] = make_double2((double)cosl(a), (double)-sinl(a));
        }
        if (hipMalloc(&c->twiddle, n * sizeof(double2)) != hipSuccess) {
            (void)hipGetLastError();
            return bail(NS2D_E_NOMEM);
        }
        if (hipMemcpy(c->twiddle, w.data(), n * sizeof(double2), hipMemcpyHostToDevice) != hipSuccess)
            return bail(NS2D_E_HIP);
        *out = c;
        return NS2D_OK;
    }
    int dims[2] = {n, n};
    if (hipfftPlan2d(&c->r2c, n, n, HIPFFT_D2Z) != HIPFFT_SUCCESS) return bail(NS2D_E_FFT);
    c->r2c_ok = true;
    if (hipfftPlanMany(&c->c2r4, 2, dims, nullptr, 1, 0, nullptr, 1, 0, HIPFFT_Z2D, 4) != HIPFFT_SUCCESS)
        return bail(NS2D_E_FFT);
    c->c2r4_ok = true;
    if (hipfftPlan2d(&c->c2r1, n, n, HIPFFT_Z2D) != HIPFFT_SUCCESS) return bail(NS2D_E_FFT);
    c->c2r1_ok = true;
    if (hipfftSetStream(c->r2c, c->stream) != HIPFFT_SUCCESS ||
        hipfftSetStream(c->c2r4, c->stream) != HIPFFT_SUCCESS ||
        hipfftSetStream(c->c2r1, c->stream) != HIPFFT_SUCCESS)
        return bail(NS2D_E_FFT);
    *out = c;
    return NS2D_OK;
}

void ns2d_destroy(ns2d_ctx *ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    release(ctx);
    delete ctx;
}

const char *ns2d_last_error(const ns2d_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

ns2d_status ns2d_synchronize(ns2d_ctx *c)
{
    if (!c) return NS2D_E_ARG;
    NS_HIP(c, hipSetDevice(c->device));
    NS_HIP(c, hipStreamSynchronize(c->stream));
    return NS2D_OK;
}

ns2d_status ns2d_set_vorticity(ns2d_ctx *c, const double *omega, int32_t on_device)
{
    if (!c) return NS2D_E_ARG;
    if (!omega) return fail(c, NS2D_E_ARG, "omega is NULL");
    if (on_device != 0 && on_device != 1) return fail(c, NS2D_E_ARG, "on_device is 0 or 1");
    NS_HIP(c, hipSetDevice(c->device));
    const size_t bytes = (size_t)c->n * c->n * sizeof(double);
    NS_HIP(c, hipMemcpyAsync(c->tmp, omega, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                             c->stream));
    if (c->builtin) {
        const ns2d_status st = run_builtin(c, kOpInit);
        if (st != NS2D_OK) return st;
    } else {
        NS_FFT(c, hipfftExecD2Z(c->r2c, c->tmp, reinterpret_cast<hipfftDoubleComplex *>(c->w_hat)));
        const Spec S = make_spec(c);
        init_kernel<<<spectral_grid(c), kBlock, 0, c->stream>>>(c->w_hat, c->fields, S);
        NS_HIP(c, hipGetLastError());
        const ns2d_status st = to_grid4(c);
        if (st != NS2D_OK) return st;
    }
    if (!on_device) NS_HIP(c, hipStreamSynchronize(c->stream));   // host buffer read before return
    c->have_state = true;
    c->first = true;
    c->steps = 0;
    return NS2D_OK;
}

ns2d_status ns2d_step(ns2d_ctx *c, int32_t count)
{
    if (!c) return NS2D_E_ARG;
    if (count < 0) return fail(c, NS2D_E_ARG, "count must be >= 0");
    if (!c->have_state) return fail(c, NS2D_E_STATE, "ns2d_set_vorticity has not been called");
    NS_HIP(c, hipSetDevice(c->device));
    const Spec S = make_spec(c);
    const size_t cells = (size_t)c->n * c->n, count2 = cells / 2;
    const double2 *g = reinterpret_cast<const double2 *>(c->grid);
    int cus = 256;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device);
    const size_t want = (count2 + kBlock - 1) / kBlock;
    const unsigned pgrid = (unsigned)(want < (size_t)cus * 16 ? want : (size_t)cus * 16);
    if (c->builtin) {
        for (int32_t s = 0; s < count; ++s) {
            const ns2d_status st = run_builtin(c, kOpStep);
            if (st != NS2D_OK) return st;
            c->first = false;
            ++c->steps;
        }
        return NS2D_OK;
    }
    for (int32_t s = 0; s < count; ++s) {
        product_kernel<<<pgrid, kBlock, 0, c->stream>>>(g, g + count2, g + 2 * count2, g + 3 * count2,
                                                        reinterpret_cast<double2 *>(c->tmp), count2);
        NS_HIP(c, hipGetLastError());
        NS_FFT(c, hipfftExecD2Z(c->r2c, c->tmp, reinterpret_cast<hipfftDoubleComplex *>(c->fields)));
        if (c->first)
            ab2_kernel<true><<<spectral_grid(c), kBlock, 0, c->stream>>>(c->w_hat, c->r_prev, c->fields, S);
        else
            ab2_kernel<false><<<spectral_grid(c), kBlock, 0, c->stream>>>(c->w_hat, c->r_prev, c->fields, S);
        NS_HIP(c, hipGetLastError());
        const ns2d_status st = to_grid4(c);
        if (st != NS2D_OK) return st;
        c->first = false;
        ++c->steps;
    }
    return NS2D_OK;
}

ns2d_status ns2d_velocity(ns2d_ctx *c, const double **u, const double **v)
{
    if (!c) return NS2D_E_ARG;
    if (!u || !v) return fail(c, NS2D_E_ARG, "u and v must not be NULL");
    if (!c->have_state) return fail(c, NS2D_E_STATE, "ns2d_set_vorticity has not been called");
    const size_t cells = (size_t)c->n * c->n;
    *u = c->grid;
    *v = c->grid + cells;
    return NS2D_OK;
}

ns2d_status ns2d_get_fields(ns2d_ctx *c, double *u, double *v, double *omega, double *psi,
                            int32_t on_device)
{
    if (!c) return NS2D_E_ARG;
    if (on_device != 0 && on_device != 1) return fail(c, NS2D_E_ARG, "on_device is 0 or 1");
    if (!c->have_state) return fail(c, NS2D_E_STATE, "ns2d_set_vorticity has not been called");
    NS_HIP(c, hipSetDevice(c->device));
    const size_t cells = (size_t)c->n * c->n;
    ns2d_status st;
    if (u && (st = copy_out(c, u, c->grid, on_device)) != NS2D_OK) return st;
    if (v && (st = copy_out(c, v, c->grid + cells, on_device)) != NS2D_OK) return st;
    const Spec S = make_spec(c);
    double *outs[2] = {omega, psi};
    for (int which = 0; which < 2; ++which) {
        if (!outs[which]) continue;
        // plane 0 of the spectral fields is free between steps (the next
        // step's forward transform rewrites it before it is read)
        if (c->builtin) {
            if ((st = run_builtin(c, which == 0 ? kOpReadW : kOpReadPsi)) != NS2D_OK) return st;
        } else {
            scaled_kernel<<<spectral_grid(c), kBlock, 0, c->stream>>>(c->w_hat, c->fields, S, which);
            NS_HIP(c, hipGetLastError());
            NS_FFT(c, hipfftExecZ2D(c->c2r1, reinterpret_cast<hipfftDoubleComplex *>(c->fields), c->tmp));
        }
        if ((st = copy_out(c, outs[which], c->tmp, on_device)) != NS2D_OK) return st;
    }
    if (!on_device) NS_HIP(c, hipStreamSynchronize(c->stream));
    return NS2D_OK;
}

ns2d_status ns2d_get_transforms(const ns2d_ctx *c, int32_t *builtin)
{
    if (!c || !builtin) return NS2D_E_ARG;
    *builtin = c->builtin ? 1 : 0;
    return NS2D_OK;
}

ns2d_status ns2d_get_steps(const ns2d_ctx *c, int64_t *steps)
{
    if (!c || !steps) return NS2D_E_ARG;
    *steps = c->steps;
    return NS2D_OK;
}

}  // extern "C"
