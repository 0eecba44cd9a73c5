// Cell-order re-sorting of the particle state: key generation, a stable LSD
// radix sort with 8-bit digits, and the structure-of-arrays permutation.
//
// Radix pass = histogram (per 4096-key tile) -> one kernel scanning each
// digit's row of tile counts -> stable scatter, which adds the start of each
// digit's output run (the sum of the smaller digits' totals, scanned by every
// scatter block from the 256 totals).  Inside a tile, each wave
// owns a contiguous run of 1024 keys and ranks them with 8 ballots per
// 64 keys (lanes with an equal digit form a match mask); per-wave running
// counts live in LDS and are turned into scatter bases by one scan over the
// waves.  Equal digits therefore keep input order: tile order, then wave,
// then iteration, then lane -- which is the input order.  (The match masks
// come from peeling the wave's distinct digits one ballot at a time when
// there are at most 8 of them, as for the nearly sorted keys of a re-sort.)
//
// The key kernel also builds the first pass's histogram, and the first
// scatter takes the input index as the value, so the sort reads no value
// array it did not write.  Histograms count runs: each thread takes 16
// consecutive keys and adds one LDS increment per run of equal digits, since
// the keys of a state sorted a few steps ago arrive nearly in order (where
// one LDS bin per lane increment would serialise a wave on one address).
#include "lpt_kernels.h"

namespace lpt {

constexpr int kSortThreads = 256;
constexpr int kSortWaves = kSortThreads / 64;
constexpr int kItems = 16;                             // keys per thread
constexpr int kTile = kSortThreads * kItems;           // 4096 keys
static_assert(kTile == kSortTileKeys, "the tile the histogram buffers are sized for");
constexpr int kWaveRun = kTile / kSortWaves;           // 1024 keys per wave
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;

int64_t sort_hist_entries(int64_t n) { return 256 * ((n + kTile - 1) / kTile); }
int64_t sort_scan_blocks(int64_t n)
{
    (void)n;
    return 256;   // per-digit totals
}

// ---------------------------------------------------------------------------
// keys
// ---------------------------------------------------------------------------
__device__ __forceinline__ int cell_of_pos(double x, double invh, int n)
{
    double c = floor(x * invh);
    if (!(c >= 0.0)) c = 0.0;            // NaN / tiny negative
    int ci = (int)fmin(c, (double)(n - 1));
    return ci;
}

// The stored cell of an unwrapped cell coordinate: its residue in [0, n).
__device__ __forceinline__ int stored_cell(int u, int n, int mask)
{
    if (mask >= 0) return u & mask;
    int c = u % n;
    return c < 0 ? c + n : c;
}

__device__ __forceinline__ int species_of_particle(const StepParams &P, int64_t p)
{
    int s = 0;
    for (int k = 1; k < P.nspecies; ++k)
        if (p >= P.sp[k].offset) s = k;
    return s;
}

// Cell-order key of the stored cell (ci, cj): the species, then the T x T
// tile (T = 2^tile_shift) in row-major tile order, then -- with `cells` --
// the cell row-major inside its tile (2 tile_shift more low bits).
__device__ __forceinline__ uint32_t tile_key(int ci, int cj, int n, int tile_shift, int tile_bits,
                                             int cells, int species)
{
    const uint32_t tx = (uint32_t)ci >> tile_shift, ty = (uint32_t)cj >> tile_shift;
    const uint32_t tiles_x = (uint32_t)n >> tile_shift;
    uint32_t k = ((uint32_t)species << tile_bits) | (ty * tiles_x + tx);
    if (cells) {
        const uint32_t m = (1u << tile_shift) - 1u;
        k = (k << (2 * tile_shift)) | (((uint32_t)cj & m) << tile_shift) | ((uint32_t)ci & m);
    }
    return k;
}

// Adds the digits of v[0 .. cnt) to the LDS histogram h, one increment per
// run of equal digits.
template <int CNT>
__device__ __forceinline__ void count_runs(const uint32_t *v, int cnt, int shift, uint32_t mask,
                                           uint32_t *h)
{
    if (cnt <= 0) return;
    uint32_t cur = (v[0] >> shift) & mask, run = 1;
#pragma unroll
    for (int k = 1; k < CNT; ++k) {
        if (k >= cnt) break;
        const uint32_t d = (v[k] >> shift) & mask;
        if (d != cur) {
            atomicAdd(&h[cur], run);
            cur = d;
            run = 0;
        }
        ++run;
    }
    atomicAdd(&h[cur], run);
}

// 16 consecutive keys of type K (uint32_t, or uint16_t when keys fit in 16
// bits) from / to 16-byte aligned memory, widened to / narrowed from uint32.
template <typename K>
__device__ __forceinline__ void load16(const K *p, uint32_t k[kItems])
{
    const uint4 *q = reinterpret_cast<const uint4 *>(p);
    if constexpr (sizeof(K) == 4) {
#pragma unroll
        for (int c = 0; c < kItems / 4; ++c) {
            const uint4 w = q[c];
            k[4 * c] = w.x;
            k[4 * c + 1] = w.y;
            k[4 * c + 2] = w.z;
            k[4 * c + 3] = w.w;
        }
    } else {
#pragma unroll
        for (int c = 0; c < kItems / 8; ++c) {
            const uint4 w = q[c];
            const uint32_t h[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                k[8 * c + 2 * m] = h[m] & 0xFFFFu;
                k[8 * c + 2 * m + 1] = h[m] >> 16;
            }
        }
    }
}

template <typename K>
__device__ __forceinline__ void store16(K *p, const uint32_t k[kItems])
{
    uint4 *q = reinterpret_cast<uint4 *>(p);
    if constexpr (sizeof(K) == 4) {
#pragma unroll
        for (int c = 0; c < kItems / 4; ++c)
            q[c] = make_uint4(k[4 * c], k[4 * c + 1], k[4 * c + 2], k[4 * c + 3]);
    } else {
#pragma unroll
        for (int c = 0; c < kItems / 8; ++c) {
            uint32_t h[4];
#pragma unroll
            for (int m = 0; m < 4; ++m) h[m] = k[8 * c + 2 * m] | (k[8 * c + 2 * m + 1] << 16);
            q[c] = make_uint4(h[0], h[1], h[2], h[3]);
        }
    }
}

// Keys of the 16 consecutive particles of each thread, written to keys[], and
// the tile's histogram of the low `mask` digit.  load(i0, cnt, k) fills
// k[0 .. cnt) with the keys of particles i0 ...
template <typename K, typename Load>
__device__ __forceinline__ void keys_tile(Load load, int64_t total, K *keys, uint32_t mask,
                                          uint32_t *hist, int ntiles)
{
    __shared__ uint32_t h[256];
    const int tid = threadIdx.x;
    h[tid] = 0;
    __syncthreads();
    const int64_t i0 = (int64_t)blockIdx.x * kTile + (int64_t)tid * kItems;
    const int cnt = (int)(total - i0 < kItems ? (total - i0 > 0 ? total - i0 : 0) : kItems);
    uint32_t k[kItems];
    load(i0, cnt, k);
    if (cnt == kItems)
        store16<K>(keys + i0, k);
    else
        for (int j = 0; j < cnt; ++j) keys[i0 + j] = (K)k[j];
    count_runs<kItems>(k, cnt, 0, mask, h);
    __syncthreads();
    hist[(int64_t)tid * ntiles + blockIdx.x] = h[tid];
}

template <typename K>
__global__ __launch_bounds__(kSortThreads) void keys64_kernel(StepParams P, State64 S,
                                                              int tile_shift, int tile_bits,
                                                              int cells, K *keys, int64_t total,
                                                              uint32_t mask, uint32_t *hist,
                                                              int ntiles)
{
    keys_tile<K>(
        [&](int64_t i0, int cnt, uint32_t *k) {
#pragma unroll
            for (int j = 0; j < kItems; ++j) {
                if (j >= cnt) break;
                const double2 x = S.pos[i0 + j];
                const int ci = cell_of_pos(x.x, P.invh, P.n), cj = cell_of_pos(x.y, P.invh, P.n);
                k[j] = tile_key(ci, cj, P.n, tile_shift, tile_bits, cells,
                                species_of_particle(P, i0 + j));
            }
        },
        total, keys, mask, hist, ntiles);
}

template <typename K>
__global__ __launch_bounds__(kSortThreads) void keys32_kernel(StepParams P, State32 S,
                                                              int tile_shift, int tile_bits,
                                                              int cells, K *keys, int64_t total,
                                                              uint32_t mask, uint32_t *hist,
                                                              int ntiles)
{
    keys_tile<K>(
        [&](int64_t i0, int cnt, uint32_t *k) {
            int2 c[kItems];   // unwrapped cells; the stored cell is their residue mod n
            if (cnt == kItems) {
#pragma unroll
                for (int j = 0; j < kItems; j += 2) {
                    const int4 q = *reinterpret_cast<const int4 *>(S.uc + i0 + j);
                    c[j] = make_int2(q.x, q.y);
                    c[j + 1] = make_int2(q.z, q.w);
                }
            } else {
#pragma unroll
                for (int j = 0; j < kItems; ++j) c[j] = j < cnt ? S.uc[i0 + j] : make_int2(0, 0);
            }
#pragma unroll
            for (int j = 0; j < kItems; ++j)
                k[j] = tile_key(stored_cell(c[j].x, P.n, P.mask), stored_cell(c[j].y, P.n, P.mask),
                                P.n, tile_shift, tile_bits, cells, species_of_particle(P, i0 + j));
        },
        total, keys, mask, hist, ntiles);
}

static int64_t total_particles(const StepParams &P)
{
    const SpeciesDev &s = P.sp[P.nspecies - 1];
    return s.offset + s.count;
}

static int ilog2(int t)
{
    int s = 0;
    while ((1 << s) < t) ++s;
    return s;
}

static uint32_t first_mask(int key_bits) { return key_bits >= 8 ? 0xFFu : (1u << key_bits) - 1u; }

hipError_t launch_keys64(const StepParams &P, const State64 &S, int tile, int tile_bits,
                         bool cells, int key_bits, SortWork &W, hipStream_t st)
{
    const int64_t total = total_particles(P);
    const int ntiles = (int)((total + kTile - 1) / kTile);
    if (key_bits <= 16)
        hipLaunchKernelGGL(keys64_kernel<uint16_t>, dim3(ntiles), dim3(kSortThreads), 0, st, P, S,
                           ilog2(tile), tile_bits, (int)cells,
                           reinterpret_cast<uint16_t *>(W.keys[0]), total,
                           first_mask(key_bits), W.hist, ntiles);
    else
        hipLaunchKernelGGL(keys64_kernel<uint32_t>, dim3(ntiles), dim3(kSortThreads), 0, st, P, S,
                           ilog2(tile), tile_bits, (int)cells, W.keys[0], total,
                           first_mask(key_bits), W.hist, ntiles);
    return hipGetLastError();
}

hipError_t launch_keys32(const StepParams &P, const State32 &S, int tile, int tile_bits,
                         bool cells, int key_bits, SortWork &W, hipStream_t st)
{
    const int64_t total = total_particles(P);
    const int ntiles = (int)((total + kTile - 1) / kTile);
    if (key_bits <= 16)
        hipLaunchKernelGGL(keys32_kernel<uint16_t>, dim3(ntiles), dim3(kSortThreads), 0, st, P, S,
                           ilog2(tile), tile_bits, (int)cells,
                           reinterpret_cast<uint16_t *>(W.keys[0]), total,
                           first_mask(key_bits), W.hist, ntiles);
    else
        hipLaunchKernelGGL(keys32_kernel<uint32_t>, dim3(ntiles), dim3(kSortThreads), 0, st, P, S,
                           ilog2(tile), tile_bits, (int)cells, W.keys[0], total,
                           first_mask(key_bits), W.hist, ntiles);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// radix pass kernels
// ---------------------------------------------------------------------------
template <typename K>
__global__ __launch_bounds__(kSortThreads) void hist_kernel(const K *__restrict__ keys, int64_t n,
                                                            int shift, uint32_t mask,
                                                            uint32_t *hist, int ntiles)
{
    __shared__ uint32_t h[256];
    const int tid = threadIdx.x;
    h[tid] = 0;
    __syncthreads();
    const int64_t i0 = (int64_t)blockIdx.x * kTile + (int64_t)tid * kItems;
    const int cnt = (int)(n - i0 < kItems ? (n - i0 > 0 ? n - i0 : 0) : kItems);
    uint32_t k[kItems];
    if (cnt == kItems) {
        load16<K>(keys + i0, k);
    } else {
#pragma unroll
        for (int j = 0; j < kItems; ++j) k[j] = j < cnt ? (uint32_t)keys[i0 + j] : 0u;
    }
    count_runs<kItems>(k, cnt, shift, mask, h);
    __syncthreads();
    hist[(int64_t)tid * ntiles + blockIdx.x] = h[tid];
}

// Inclusive block scan of one value per thread (256 threads, 4 waves).
__device__ __forceinline__ uint32_t block_scan_incl(uint32_t x, uint32_t *wsum, uint32_t &total)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    uint32_t before = 0, tot = 0;
    const int nw = blockDim.x >> 6;
    for (int k = 0; k < nw; ++k) {
        if (k < w) before += wsum[k];
        tot += wsum[k];
    }
    total = tot;
    __syncthreads();
    return x + before;
}

// Exclusive scan of digit d's row of the histogram table (its count in every
// tile, in tile order), in place, in chunks of 2048 with a running carry;
// totals[d] receives the row's sum.  One block per digit.
__global__ __launch_bounds__(kScanThreads) void row_scan_kernel(uint32_t *hist, int ntiles,
                                                                uint32_t *totals)
{
    __shared__ uint32_t wsum[kScanThreads / 64];
    uint32_t *row = hist + (int64_t)blockIdx.x * ntiles;
    uint32_t carry = 0;
    for (int base = 0; base < ntiles; base += kScanThreads * kScanItems) {
        const int i0 = base + (int)threadIdx.x * kScanItems;
        uint32_t v[kScanItems];
        uint32_t sum = 0;
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            v[k] = i0 + k < ntiles ? row[i0 + k] : 0u;
            sum += v[k];
        }
        uint32_t total;
        const uint32_t incl = block_scan_incl(sum, wsum, total);
        uint32_t run = carry + incl - sum;
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            if (i0 + k < ntiles) row[i0 + k] = run;
            run += v[k];
        }
        carry += total;
    }
    if (threadIdx.x == 0) totals[blockIdx.x] = carry;
}

// offsets: the row-scanned histogram table; totals: each digit's count (the
// start of digit d's output run is the sum of the totals of smaller digits).
template <typename K>
__global__ __launch_bounds__(kSortThreads) void scatter_kernel(
    const K *__restrict__ keys_in, const uint32_t *vals_in,
    K *__restrict__ keys_out, uint32_t *__restrict__ vals_out, int64_t n, int shift,
    uint32_t mask, const uint32_t *__restrict__ offsets, const uint32_t *__restrict__ totals,
    int ntiles)
{
    __shared__ uint32_t wcount[kSortWaves][256];
    __shared__ uint32_t wsum[kSortWaves];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
#pragma unroll
    for (int k = 0; k < kSortWaves; ++k) wcount[k][tid] = 0;
    __syncthreads();

    const int64_t run0 = (int64_t)blockIdx.x * kTile + (int64_t)w * kWaveRun;
    const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    uint32_t key[kItems], val[kItems], rank[kItems];
#pragma unroll
    for (int it = 0; it < kItems; ++it) {
        const int64_t i = run0 + (int64_t)it * 64 + lane;
        const bool valid = i < n;
        key[it] = valid ? (uint32_t)keys_in[i] : 0u;
        val[it] = !valid ? 0u : vals_in ? vals_in[i] : (uint32_t)i;
        const uint32_t d = (key[it] >> shift) & mask;
        // m = the valid lanes whose digit equals this lane's.  Nearly sorted
        // keys give a wave few distinct digits: peel them one at a time
        // (one ballot each); past 8, match all 8 digit bits instead.
        const uint64_t act = __ballot(valid);
        uint64_t m = 0, left = act;
        for (int peel = 0; left != 0 && peel < 8; ++peel) {
            const uint32_t dl = (uint32_t)__builtin_amdgcn_readlane(
                (int)d, (int)__builtin_ctzll((unsigned long long)left));
            const uint64_t eq = __ballot(d == dl) & act;
            if (d == dl) m = eq;
            left &= ~eq;
        }
        if (left != 0) {
            m = act;
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const bool bit = (d >> b) & 1u;
                const uint64_t bal = __ballot(bit);
                m &= bit ? bal : ~bal;
            }
        }
        const uint32_t before = wcount[w][d];
        rank[it] = before + (uint32_t)__popcll(m & lt);
        if (valid && lane == __ffsll((unsigned long long)m) - 1)
            wcount[w][d] = before + (uint32_t)__popcll(m);
    }
    // block_scan_incl synchronises the block, which also publishes wcount
    const uint32_t tot = (uint32_t)tid <= mask ? totals[tid] : 0u;
    uint32_t all;
    const uint32_t dstart = block_scan_incl(tot, wsum, all) - tot;
    {
        uint32_t runv = dstart + offsets[(int64_t)tid * ntiles + blockIdx.x];
#pragma unroll
        for (int k = 0; k < kSortWaves; ++k) {
            const uint32_t c = wcount[k][tid];
            wcount[k][tid] = runv;
            runv += c;
        }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kItems; ++it) {
        const int64_t i = run0 + (int64_t)it * 64 + lane;
        if (i < n) {
            const uint32_t d = (key[it] >> shift) & mask;
            const uint32_t pos = wcount[w][d] + rank[it];
            keys_out[pos] = (K)key[it];
            vals_out[pos] = val[it];
        }
    }
}

template <typename K>
static hipError_t radix_sort_t(SortWork &W, int64_t n, int key_bits, bool first_hist, int *result,
                               hipStream_t st)
{
    const int ntiles = (int)((n + kTile - 1) / kTile);
    K *keys[2] = {reinterpret_cast<K *>(W.keys[0]), reinterpret_cast<K *>(W.keys[1])};
    int cur = 0;
    for (int shift = 0; shift < key_bits; shift += 8) {
        const int bits = key_bits - shift < 8 ? key_bits - shift : 8;
        const uint32_t mask = (1u << bits) - 1u;
        if (shift > 0 || !first_hist)
            hipLaunchKernelGGL(hist_kernel<K>, dim3(ntiles), dim3(kSortThreads), 0, st, keys[cur],
                               n, shift, mask, W.hist, ntiles);
        hipLaunchKernelGGL(row_scan_kernel, dim3(mask + 1), dim3(kScanThreads), 0, st, W.hist,
                           ntiles, W.scan_tmp);
        // the first pass takes each key's input index as its value
        hipLaunchKernelGGL(scatter_kernel<K>, dim3(ntiles), dim3(kSortThreads), 0, st, keys[cur],
                           shift == 0 ? (const uint32_t *)nullptr : W.vals[cur], keys[1 - cur],
                           W.vals[1 - cur], n, shift, mask, W.hist, W.scan_tmp, ntiles);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        cur = 1 - cur;
    }
    *result = cur;
    return hipSuccess;
}

hipError_t radix_sort(SortWork &W, int64_t n, int key_bits, bool first_hist, bool narrow,
                      int *result, hipStream_t st)
{
    *result = 0;
    if (n <= 1) return hipSuccess;
    return narrow && key_bits <= 16
               ? radix_sort_t<uint16_t>(W, n, key_bits, first_hist, result, st)
               : radix_sort_t<uint32_t>(W, n, key_bits, first_hist, result, st);
}

__global__ void fill_u32_kernel(uint32_t *p, int64_t n, uint32_t v)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) p[k] = v;
}

hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const int b = 256;
    hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)((n + b - 1) / b)), dim3(b), 0, st, p, n, v);
    return hipGetLastError();
}

__global__ void order_kernel(const uint32_t *__restrict__ id, int64_t offset, int64_t count,
                             int32_t *out)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < count) out[k] = (int32_t)((int64_t)id[offset + k] - offset);
}

hipError_t launch_order(const uint32_t *id, int64_t offset, int64_t count, int32_t *out,
                        hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    const int b = 256;
    hipLaunchKernelGGL(order_kernel, dim3((unsigned)((count + b - 1) / b)), dim3(b), 0, st, id,
                       offset, count, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// permutation of the state: dst[p] = src[perm[p]]
// ---------------------------------------------------------------------------
__global__ void permute64_kernel(State64 src, State64 dst, const uint32_t *__restrict__ perm,
                                 int64_t n, int with_vel)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const uint32_t q = perm[p];
    dst.pos[p] = src.pos[q];
    dst.disp[p] = src.disp[q];
    dst.id[p] = src.id[q];
    if (with_vel) dst.vel[p] = src.vel[q];
}

__global__ void permute32_kernel(State32 src, State32 dst, const uint32_t *__restrict__ perm,
                                 int64_t n, int with_vel)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const uint32_t q = perm[p];
    dst.uc[p] = src.uc[q];
    dst.off[p] = src.off[q];
    dst.id[p] = src.id[q];
    if (with_vel) dst.vel[p] = src.vel[q];
}

hipError_t launch_permute64(const State64 &src, const State64 &dst, const uint32_t *perm,
                            int64_t n, bool with_vel, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const int b = 256;
    hipLaunchKernelGGL(permute64_kernel, dim3((unsigned)((n + b - 1) / b)), dim3(b), 0, st, src,
                       dst, perm, n, (int)with_vel);
    return hipGetLastError();
}

hipError_t launch_permute32(const State32 &src, const State32 &dst, const uint32_t *perm,
                            int64_t n, bool with_vel, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const int b = 256;
    hipLaunchKernelGGL(permute32_kernel, dim3((unsigned)((n + b - 1) / b)), dim3(b), 0, st, src,
                       dst, perm, n, (int)with_vel);
    return hipGetLastError();
}

}  // namespace lpt
