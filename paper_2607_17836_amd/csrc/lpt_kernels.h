// Internal interface between the host runtime (runtime.cpp) and the gfx950
// kernels (step.hip, sort.hip, misc.hip) of liblpt.so.  Not installed.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lpt {

constexpr int kMaxSpecies = 16;
// per wave: sum dx^2, sum dy^2, and the sums of d and d^2 for
// d = r2 - K, r2 = dx^2 + dy^2, K = r2 of the wave's first active lane
constexpr int kStatTerms = 4;

enum Scheme : int32_t { kBilinear = 0, kCatmullRom = 1, kBSpline = 2 };
// a fused FP32 launch whose blocks take their species' scheme at run time
constexpr int kAnyScheme = -1;

// One species as the step kernel sees it.  A species owns the contiguous
// particle range [offset, offset + count) of the state arrays and the logical
// blocks [block_begin, block_end) of the step grid.
struct SpeciesDev {
    int32_t inertial;      // 1: Stokes drag with inv_st; 0: tracer (St == 0 too)
    int32_t scheme;        // Scheme
    double inv_st;         // 1/St (inertial only)
    int64_t offset;
    int64_t count;
    int32_t block_begin;
    int32_t block_end;
    uint64_t x0_seed;      // with x0_drawn: the seed the initial positions were drawn from
    int32_t x0_drawn;      // 1: initial positions are the SplitMix64 draws of x0_seed
    int32_t pad_;
};

// Node records are stored with a periodic ghost border: one node before and
// two after the grid on each axis, so that every stencil (bilinear: i..i+1,
// bicubic: i-1..i+2) of a cell i in [0, n) is contiguous and never wraps.
// Node (i, j), -1 <= i, j <= n + 1, lives at index (j + 1) * pitch + (i + 1)
// with pitch = n + 3.
constexpr int kGhostLo = 1;
constexpr int kGhostHi = 2;
inline int64_t padded_pitch(int n) { return (int64_t)n + kGhostLo + kGhostHi; }

// A block stages an LDS tile only if it holds at most this many node records
// per particle of the block (sparse species gather from global memory).
constexpr int kTileWaste = 8;

// Which time levels a stage needs: weights (1, 0), (0, 1), or a blend.
enum SlotMode : int32_t { kSlot0 = 0, kSlot1 = 1, kBlend = 2 };

struct StepParams {
    int32_t n;             // grid points per side
    int32_t pitch;         // n + 3 (padded row length)
    int32_t mask;          // n - 1 if n is a power of two, else -1
    int32_t nspecies;
    int32_t total_blocks;  // logical blocks over all species
    int32_t compat_edge;   // bicubic reverts to bilinear near the grid edge
    double L, h, invh;     // domain side, spacing, n/L
    double dt;
    double wa[4], wb[4];   // temporal weights of slot 0 / slot 1 per RK4 stage
    int32_t smode[4];      // SlotMode per RK4 stage
    // binary32 copies for the FP32-split kernel, rounded once on the host
    float dtf, hdtf, dt6f; // dt, dt/2, dt/6
    float waf[4], wbf[4];
    int32_t ends_one;      // stages 1 and 4 read one level each: h0 and h3
    int32_t h0, h3;
    int32_t persistent;    // grid sized to residency; workgroups loop over blocks
    int32_t tile_cap;      // LDS tile capacity in node records (0: no tile)
    float halo_scale;      // tile halo = halo_scale x the largest-speed displacement
    const float *umax;     // device: largest node speed of slot 0 / 1, cells per unit time
    SpeciesDev sp[kMaxSpecies];
    // the logical blocks [block_base, block_base + launch_blocks) of one FP32
    // launch (one launch per species)
    int32_t block_base;
    int32_t launch_blocks;
    // fused launches over all species: one list of order_len logical blocks
    // per XCD (device memory, XCD-major; -1 pads a shorter list), or null
    const int32_t *order;
    int32_t order_len;
    int32_t max_wg;        // > 0: persistent grids hold at most this many workgroups
    int32_t tile_auto;     // 1: each step launch replaces tile_cap by the largest
                           // capacity that keeps its kernel's register-bound occupancy
    int32_t rows;          // FP32 bilinear tracer step: rows of blockDim.x slots per block
};

// Block-order table of a fused launch over species whose logical blocks are
// [begin[s], end[s]): XCD x receives the slice [B x / 8, B (x + 1) / 8) of
// every species' B blocks, so every XCD carries the same share of each
// species.  Its list holds those slices species after species (a CU then
// runs one species' code at a time), or, with `interleave`, merged by the
// position of each block along its species' cell order, so that the blocks
// an XCD runs together cover one region of the grid for every species.
// Returns order_len; `out` receives 8 * order_len entries.
int32_t build_block_order(int nspecies, const int32_t *begin, const int32_t *end, bool interleave,
                          int32_t *out /* may be null: length only */);

// Device-resident clock so that captured step chunks can be replayed.
struct DevClock {
    double t;          // time after the last enqueued step
    int64_t step;      // steps taken
    int64_t nrec;      // statistics records written per species
    int64_t pad_;
};

// FP64 state, structure of arrays, pairs interleaved (x, y).
struct State64 {
    double2 *pos;      // wrapped position in [0, L)
    double2 *disp;     // unwrapped displacement since initialisation
    double2 *vel;      // particle velocity (inertial species)
    uint32_t *id;      // global particle index (species offset + local index)
};

// FP32 split state: the unwrapped integer cell (x, y) -- the stored cell is
// its residue mod n -- and the binary32 offset in [0, 1) cell units, so that
// the position unwrapped since initialisation is (uc + off) h exactly and no
// displacement is stored; binary32 velocity in cells per unit time.  16 bytes
// a tracer, 24 an inertial particle, read and written once a step; the id is
// moved only by the step after a re-sort.  x0: the initial positions by
// original index (binary64, read by record steps and readout: the
// displacement is (uc + off) - split(x0), in cells).
struct State32 {
    int2 *uc;
    float2 *off;
    float2 *vel;
    uint32_t *id;
    const double2 *x0;
};

// Snapshot records: both time levels of one node side by side.
// FP64: {u0, v0, u1, v1} in physical units.  FP32: {u0, v0, u1, v1} in
// cells per unit time (u * n / L).
struct alignas(32) Rec64 { double u0, v0, u1, v1; };

// ---- launch wrappers (return hipGetLastError of the launch) -------------
// rec: the padded record array ((n + 3)^2 records).
// One level's half of every record (FP64: Rec64 doubles; FP32: float4
// records of u * scale) and its largest |u| or |v| times vscale folded into
// *umax (which the caller zeroes first).
hipError_t launch_pack(void *rec, bool fp64, int slot, const double *u, const double *v, int n,
                       double scale, double vscale, float *umax, hipStream_t st);
// The same from a stream-function level: the node velocity is the grid
// centred difference of psi (spacing h), formed in the same pass.
hipError_t launch_pack_psi(void *rec, bool fp64, int slot, const double *psi, int n, double h,
                           double scale, double vscale, float *umax, hipStream_t st);

// The step works in place on S; with perm (the permutation of a re-sort, dst
// slot -> src slot) it reads S through perm and writes D, a different buffer,
// so that it also applies the permutation (id included).
hipError_t launch_step64(const StepParams &P, const State64 &S, const State64 &D,
                         const uint32_t *perm, const Rec64 *rec, double *partials,
                         DevClock *clock, bool stats, bool cubic, bool inertial, int block,
                         int grid, hipStream_t st);
// One launch over the logical blocks [P.block_base, P.block_base +
// P.launch_blocks) (= grid) of one species, whose scheme is `schemes`, or,
// with P.order set and schemes = kAnyScheme (or the one scheme they share),
// a fused launch over every species.  S, D and perm as for launch_step64.
hipError_t launch_step32(const StepParams &P, const State32 &S, const State32 &D,
                         const uint32_t *perm, const float4 *rec, double *partials,
                         DevClock *clock, bool stats, int schemes, bool inertial, int block,
                         int grid, hipStream_t st);

// Statistics record of every species from the per-wave partials of a step
// kernel launched with `block` threads per block (two fixed-order merge
// kernels; the buffer holds stat_partials_doubles(P, block) doubles: the wave
// partials, then the merge stage's own partials).
int64_t stat_partials_doubles(const StepParams &P, int block);
hipError_t launch_finalize(const StepParams &P, double *partials, DevClock *clock,
                           double *records, int64_t rec_cap, double t0, int block,
                           hipStream_t st);

// Initial state of particles [begin, begin + count) from x0 and v0 (both in
// original order, indexed by global particle index).  An inertial species
// takes its velocity from the field (vel_from_field) or from v0.
hipError_t launch_init64(const StepParams &P, const State64 &S, const double2 *x0,
                         const double2 *v0, const Rec64 *rec, int species, int64_t begin,
                         int64_t count, double wa, double wb, int vel_from_field,
                         hipStream_t st);
hipError_t launch_init32(const StepParams &P, const State32 &S, const double2 *x0,
                         const double2 *v0, const float4 *rec, int species, int64_t begin,
                         int64_t count, double wa, double wb, int vel_from_field,
                         hipStream_t st);
hipError_t launch_interleave(double2 *dst, const double *a, const double *b, int64_t n,
                             hipStream_t st);
hipError_t launch_splitmix(double2 *x0, int64_t count, uint64_t seed, double L, hipStream_t st);

hipError_t launch_interp64(const StepParams &P, const Rec64 *rec, int scheme, int64_t npts,
                           const double *x, const double *y, double wa, double wb, double *u,
                           double *v, hipStream_t st);
hipError_t launch_interp32(const StepParams &P, const float4 *rec, int scheme, int64_t npts,
                           const double *x, const double *y, double wa, double wb, double *u,
                           double *v, hipStream_t st);

// Readout in original particle order (id - offset).
hipError_t launch_readout64(const State64 &S, const double2 *x0, int64_t offset, int64_t count,
                            double L, double *xw, double *yw, double *xu, double *yu,
                            double *vx, double *vy, hipStream_t st);
hipError_t launch_readout32(const StepParams &P, const State32 &S, int64_t offset, int64_t count,
                            double *xw, double *yw, double *xu, double *yu, double *vx,
                            double *vy, hipStream_t st);

hipError_t launch_order(const uint32_t *id, int64_t offset, int64_t count, int32_t *out,
                        hipStream_t st);

// reverse-mode derivatives of the FP64 tracer step (adjoint.hip); block is
// the step kernel's block size (P's species block layout)
hipError_t launch_recompute64(const StepParams &P, const Rec64 *rec, const double2 *in,
                              double2 *out, bool cubic, int block, hipStream_t st);
// cubic: some species uses a bicubic scheme (else every stencil is bilinear).
// det: gU holds fixed-point pairs of 64-bit words (4 n^2 pairs; value =
// hi 2^-32 + lo 2^-64), summed exactly with integer atomics; else doubles.
hipError_t launch_adjoint64(const StepParams &P, const Rec64 *rec, const double2 *tape,
                            double2 *lam, int nl, void *gU, bool det, bool cubic, int block,
                            hipStream_t st);
// out[perm[i] * nl + r] = in[i * nl + r]: adjoint vectors back through a sort
hipError_t launch_unpermute_adjoint(const uint32_t *perm, int64_t np, int nl, const double2 *in,
                                    double2 *out, hipStream_t st);
hipError_t launch_fixed_to_double(const void *pairs, int64_t count, double *out, hipStream_t st);
hipError_t launch_zero_words(void *p, int64_t words, hipStream_t st);
hipError_t launch_seed_adjoint(const uint32_t *id, int64_t np, int nl, const double *gx,
                               const double *gy, double2 *lam, hipStream_t st);
// sigma (with nl == 2): the FTLE of each Jacobian over the time T
hipError_t launch_gather_adjoint(const uint32_t *id, int64_t np, int nl, const double2 *lam,
                                 double *gx, double *gy, double *F, double *sigma, double T,
                                 hipStream_t st);

// bandwidth probe (bytes: per buffer, multiple of 16)
hipError_t launch_copy(const void *src, void *dst, int64_t bytes, hipStream_t st);
hipError_t launch_triad(const void *b, const void *c, void *a, int64_t bytes, hipStream_t st);

// ---- cell-order sort -------------------------------------------------------
struct SortWork {
    uint32_t *keys[2];
    uint32_t *vals[2];
    uint32_t *hist;        // 256 * max_tiles counters
    uint32_t *scan_tmp;    // per-digit totals of a radix pass (256)
    int64_t capacity;      // keys
};
// Keys per radix-sort tile: each tile holds one row of digit histograms.
constexpr int kSortTileKeys = 4096;
int64_t sort_hist_entries(int64_t n);
int64_t sort_scan_blocks(int64_t n);
// p[0 .. n) = v (a kernel, so that it can sit in a captured graph)
hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t st);

// keys[0] = (species << tile_bits) | tile index of the stored cell -- with
// `cells`, shifted up by 2 log2(tile) bits over the cell's row-major index
// inside its tile -- plus the histogram of the first radix digit (of a
// key_bits-bit sort) in W.hist.  Keys of at most 16 bits are stored as
// uint16_t (see radix_sort's narrow).
hipError_t launch_keys64(const StepParams &P, const State64 &S, int tile, int tile_bits,
                         bool cells, int key_bits, SortWork &W, hipStream_t st);
hipError_t launch_keys32(const StepParams &P, const State32 &S, int tile, int tile_bits,
                         bool cells, int key_bits, SortWork &W, hipStream_t st);
// Stable LSD radix sort of keys[0] over the low key_bits bits, carrying each
// key's input index as its value (vals[0] is not read).  first_hist: W.hist
// already holds the first digit's histogram (from launch_keys*).  narrow:
// keys of at most 16 bits are stored as uint16_t (as launch_keys* writes
// them); else uint32_t.  *result receives the buffer index (0 or 1) holding
// the sorted keys and values.
hipError_t radix_sort(SortWork &W, int64_t n, int key_bits, bool first_hist, bool narrow,
                      int *result, hipStream_t st);
hipError_t launch_permute64(const State64 &src, const State64 &dst, const uint32_t *perm,
                            int64_t n, bool with_vel, hipStream_t st);
hipError_t launch_permute32(const State32 &src, const State32 &dst, const uint32_t *perm,
                            int64_t n, bool with_vel, hipStream_t st);

}  // namespace lpt
