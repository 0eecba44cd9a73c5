// Host runtime of liblpt.so: the C ABI of include/lpt.h on top of the gfx950
// kernels.  Validation happens before anything is enqueued so that a failed
// call leaves the context unchanged; every HIP failure is reported as
// LPT_E_HIP with the runtime's message.
#include "lpt.h"
#include "lpt_kernels.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <map>
#include <mutex>
#include <tuple>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

using namespace lpt;

int32_t lpt::build_block_order(int nspecies, const int32_t *begin, const int32_t *end,
                               bool interleave, int32_t *out)
{
    constexpr int X = 8;
    std::vector<std::pair<double, int32_t>> lists[X];
    size_t len = 0;
    for (int x = 0; x < X; ++x) {
        for (int s = 0; s < nspecies; ++s) {
            const int64_t B = end[s] - begin[s];
            for (int64_t k = B * x / X; k < B * (x + 1) / X; ++k)
                lists[x].emplace_back(((double)k + 0.5) / (double)B, begin[s] + (int32_t)k);
        }
        // interleaved: by position along the cell order (ties keep the species
        // order); else species after species
        if (interleave)
            std::stable_sort(lists[x].begin(), lists[x].end(),
                             [](const auto &a, const auto &b) { return a.first < b.first; });
        len = std::max(len, lists[x].size());
    }
    if (out)
        for (int x = 0; x < X; ++x)
            for (size_t k = 0; k < len; ++k)
                out[x * len + k] = k < lists[x].size() ? lists[x][k].second : -1;
    return (int32_t)len;
}

namespace {

// Capacity of the field tile, in node records, of the FP64 step kernel and
// the adjoint's recompute kernel when the tuning asks for the default (0):
// 38400 bytes (four 256-thread blocks per CU; a smaller FP64 tile leaves too
// many blocks' boxes uncovered, which costs more than the lost occupancy).
// The FP32 step kernels then size their tile per launch to the occupancy
// their registers allow (1216 records for the bilinear kernel's eight blocks
// per CU, more for the bicubic and fused kernels, which hold fewer).
constexpr int32_t kTileRecordsDefault = 1200;
constexpr size_t kTileBytesMax = 61440;
// Default tile halo, as a fraction of the largest per-step displacement: small
// enough that the halo rounds up to one cell at displacements of up to eight
// cells a step (5.1 for Catmull-Rom).  One cell was fastest at every scheme,
// precision and species mix measured: a wider halo grows every block's fill
// by a ring per cell for the few particles that leave it, and no halo sends
// every stage that steps past the stored cells to global memory.
constexpr float kHaloScaleDefault = 0.125f;

struct StepWeights {
    double wa[4], wb[4];
};

struct SpeciesHost {
    int32_t kind;
    double st;
    int32_t scheme;
    int64_t count;
    int64_t offset;
    bool vel_from_field;
    // the initial positions are still the SplitMix64 draws of x0_seed
    // (lpt_init_uniform), so a record step can draw them again instead of
    // gathering them in particle order
    bool x0_drawn = false;
    uint64_t x0_seed = 0;
};

template <typename T>
void dfree(T *&p)
{
    if (p) (void)hipFree((void *)p);
    p = nullptr;
}

}  // namespace

struct lpt_ctx {
    lpt_config cfg{};
    hipStream_t stream = nullptr;
    int device = 0;
    int32_t n = 0;
    double L = 0, h = 0, invh = 0;
    int32_t precision = LPT_FP64;
    int32_t block = 256;
    int32_t sort_interval = 0;
    int32_t sort_tile = 16;
    int32_t sort_cells = 2;  // 1: the key also orders cells inside each tile; 2: on
                             // the first re-sort only
    bool sorted_once = false;   // a re-sort has put the present particles in order
    int32_t tile_cap = 0;    // LDS tile capacity of the step kernel, node records
    int32_t tile_auto = 0;   // 1: step launches size the tile to their occupancy
    int32_t rows = 1;        // FP32 bilinear tracer step: particles per thread
                             // (tile_cap is then the adjoint kernels' capacity)
    int32_t persistent = 0;  // persistent step launches
    float halo_scale = kHaloScaleDefault; // LDS tile halo relative to the largest-speed bound
    int32_t graph_chunk = 0; // steps per captured hipGraph (0: eager launches)
    int32_t fused = 1;       // one launch over every species (block-order table):
                             // 1 species-major per XCD, 2 interleaved in cell order
    int32_t max_wg = 0;      // cap on persistent workgroups (0: residency only)
    int32_t *order = nullptr;   // device block-order table of fused launches
    size_t order_cap = 0;       // entries allocated
    int32_t order_len = 0;      // entries per XCD list
    bool order_ok = false;      // the table matches the species and block size
    // executable graphs of step chunks, keyed by (step phase, state buffer,
    // chunk length, dt bits, stats_every, buffer epoch, first re-sort done)
    std::map<std::tuple<int64_t, int, int64_t, uint64_t, int32_t, uint64_t, bool>, hipGraphExec_t>
        graphs;
    uint64_t epoch = 0;      // bumped whenever a buffer a graph may hold changes
    hipStream_t own_stream = nullptr;   // capture stream when the context uses the null stream
    bool compat_edge = false;
    uint32_t *static_sort = nullptr;   // this device's fixed sort scratch
    bool det_grad = false;       // grid gradients in exact fixed point
    unsigned long long *det_acc = nullptr;   // fixed-point pairs of the grid gradient
    int64_t det_acc_words = 0;
    std::string err;

    // snapshots
    void *rec = nullptr;   // padded Rec64 or float4 records, (n + 3)^2
    float *umax = nullptr; // largest node speed per slot, cells per unit time
    bool slot_set[2] = {false, false};
    double t_slot[2] = {0, 0};
    int32_t time_mode = LPT_TIME_BRACKET;

    // particles
    std::vector<SpeciesHost> sp;
    int64_t np = 0;
    State64 s64[2]{};
    State32 s32[2]{};
    int cur = 0;
    double2 *x0 = nullptr;   // initial positions, original order
    double2 *v0 = nullptr;   // given initial velocities, original order
    bool has_inertial = false, has_cubic = false;

    // statistics
    double *partials = nullptr;   // per-wave statistics partials + merge stage
    int64_t partial_cap = 0;      // doubles
    double *records = nullptr;
    int64_t rec_cap = 0;
    int64_t nrec = 0;
    DevClock *clock = nullptr;

    // sort workspace
    SortWork sw{};

    int64_t steps = 0;
    double t = 0;

    // checkpointed forward run for the derivatives
    double2 *ck = nullptr;       // positions at segment starts, [segment][np]
    size_t ck_bytes = 0;
    int32_t ck_every = 0;
    int64_t ck_nsteps = 0, ck_step0 = 0;
    double ck_dt = 0, ck_t0 = 0;
    std::vector<StepWeights> ck_w;   // temporal weights of every recorded step
    bool ck_valid = false;
    // with re-sorting, every segment starts from cell order: the permutation
    // applied at the start of segment s >= 1 (new slot -> previous slot),
    // and the slot -> particle ids of segment 0
    bool ck_sorted = false;
    uint32_t *ck_perm = nullptr;
    size_t ck_perm_bytes = 0;
    uint32_t *ck_id0 = nullptr;
    size_t ck_id0_bytes = 0;

    // optional event timing of step kernels and re-sorts
    bool time_kernels = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_step, ev_sort, ev_perm, ev_stat, ev_fin;
};

namespace {

lpt_status fail(lpt_ctx *c, lpt_status s, const std::string &msg)
{
    if (c) c->err = msg;
    return s;
}

#define HIP_TRY(ctx, expr)                                                                  \
    do {                                                                                    \
        const hipError_t e_ = (expr);                                                       \
        if (e_ != hipSuccess)                                                               \
            return fail((ctx), LPT_E_HIP,                                                   \
                        std::string(#expr) + ": " + hipGetErrorString(e_));                 \
    } while (0)

template <typename T>
hipError_t dalloc(T *&p, size_t count)
{
    void *q = nullptr;
    const hipError_t e = hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T));
    p = static_cast<T *>(q);
    return e;
}

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

int ilog2i(int64_t v)
{
    int s = 0;
    while ((int64_t(1) << s) < v) ++s;
    return s;
}

void free_state(lpt_ctx *c)
{
    for (int k = 0; k < 2; ++k) {
        dfree(c->s64[k].pos);
        dfree(c->s64[k].disp);
        dfree(c->s64[k].vel);
        dfree(c->s64[k].id);
        dfree(c->s32[k].uc);
        dfree(c->s32[k].off);
        dfree(c->s32[k].vel);
        dfree(c->s32[k].id);
    }
}

void free_sort(lpt_ctx *c)
{
    dfree(c->sw.keys[0]);
    dfree(c->sw.keys[1]);
    dfree(c->sw.vals[0]);
    dfree(c->sw.vals[1]);
    dfree(c->sw.hist);
    dfree(c->sw.scan_tmp);
    c->sw.capacity = 0;
}

StepParams make_params(const lpt_ctx *c)
{
    StepParams P{};
    P.n = c->n;
    P.pitch = (int32_t)padded_pitch(c->n);
    P.mask = is_pow2(c->n) ? c->n - 1 : -1;
    for (int q = 0; q < 4; ++q) {
        P.wa[q] = 1.0;
        P.wb[q] = 0.0;
        P.smode[q] = kSlot0;
    }
    P.nspecies = (int32_t)c->sp.size();
    P.tile_cap = c->tile_cap;
    P.persistent = c->persistent;
    P.halo_scale = c->halo_scale;
    P.umax = c->umax;
    P.compat_edge = c->compat_edge ? 1 : 0;
    P.L = c->L;
    P.h = c->h;
    P.invh = c->invh;
    int32_t blk = 0;
    for (size_t s = 0; s < c->sp.size(); ++s) {
        const SpeciesHost &h = c->sp[s];
        SpeciesDev &d = P.sp[s];
        d.inertial = (h.kind == LPT_INERTIAL && h.st > 0.0) ? 1 : 0;
        d.scheme = h.scheme;
        d.inv_st = d.inertial ? 1.0 / h.st : 0.0;
        d.offset = h.offset;
        d.count = h.count;
        d.block_begin = blk;
        blk += (int32_t)((h.count + c->block - 1) / c->block);
        d.block_end = blk;
        d.x0_seed = h.x0_seed;
        d.x0_drawn = h.x0_drawn ? 1 : 0;
        d.pad_ = 0;
    }
    P.total_blocks = blk;
    P.block_base = 0;
    P.launch_blocks = blk;
    P.max_wg = c->max_wg;
    P.tile_auto = c->tile_auto;
    P.rows = c->precision == LPT_FP64 ? 1 : c->rows;
    if (c->fused && c->sp.size() > 1 && c->order_ok) {
        P.order = c->order;
        P.order_len = c->order_len;
    }
    return P;
}

// Temporal weights of slot 0 / slot 1 at time t for the step with 0-based
// number `step` starting at t_n.
void weights_at(const lpt_ctx *c, int64_t step, double t_n, double t, double dt, double &wa,
                double &wb)
{
    if (c->time_mode == LPT_TIME_PINGPONG) {
        // t is t_n + c dt with c in {0, 1/2, 1}; take the fraction exactly
        const double theta = (t - t_n) / dt < 0.25 ? 0.0 : ((t - t_n) / dt < 0.75 ? 0.5 : 1.0);
        const bool slot0_first = (step & 1) == 0;
        wa = slot0_first ? 1.0 - theta : theta;
        wb = slot0_first ? theta : 1.0 - theta;
    } else {
        const double ta = c->t_slot[0], tb = c->t_slot[1];
        double theta = (t - ta) / (tb - ta);
        theta = std::min(1.0, std::max(0.0, theta));
        wa = 1.0 - theta;
        wb = theta;
    }
}

int32_t slot_mode(double wa, double wb)
{
    if (wa == 1.0 && wb == 0.0) return kSlot0;
    if (wa == 0.0 && wb == 1.0) return kSlot1;
    return kBlend;
}

// The scheme every species uses, or 3 if they differ.
int species_bits(const lpt_ctx *c) { return c->sp.size() > 1 ? ilog2i((int64_t)c->sp.size()) : 0; }
int tile_bits(const lpt_ctx *c) { return 2 * ilog2i(c->n / c->sort_tile); }
// Width of the cell-order key: species, tile and (with sort_cells) the cell
// inside the tile.
int key_width(int n, int tile, int cells, int nspecies)
{
    return 2 * ilog2i(n / tile) + (cells ? 2 * ilog2i(tile) : 0) +
           (nspecies > 1 ? ilog2i(nspecies) : 0);
}

lpt_status ensure_sort_work(lpt_ctx *c)
{
    if (c->sw.capacity >= c->np) return LPT_OK;
    free_sort(c);
    HIP_TRY(c, dalloc(c->sw.keys[0], c->np));
    HIP_TRY(c, dalloc(c->sw.keys[1], c->np));
    HIP_TRY(c, dalloc(c->sw.vals[0], c->np));
    HIP_TRY(c, dalloc(c->sw.vals[1], c->np));
    HIP_TRY(c, dalloc(c->sw.hist, (size_t)sort_hist_entries(c->np)));
    HIP_TRY(c, dalloc(c->sw.scan_tmp, (size_t)sort_scan_blocks(c->np)));
    c->sw.capacity = c->np;
    return LPT_OK;
}

// Device copy of the fused launches' block-order table (set-up only: never
// called while a graph is being captured).
lpt_status ensure_order(lpt_ctx *c)
{
    if (!c->fused || c->sp.size() < 2 || c->order_ok) return LPT_OK;
    StepParams P = make_params(c);
    int32_t begin[kMaxSpecies], end[kMaxSpecies];
    for (int s = 0; s < P.nspecies; ++s) {
        begin[s] = P.sp[s].block_begin;
        end[s] = P.sp[s].block_end;
    }
    const bool il = c->fused == 2;
    const int32_t len = build_block_order(P.nspecies, begin, end, il, nullptr);
    std::vector<int32_t> h((size_t)8 * len);
    build_block_order(P.nspecies, begin, end, il, h.data());
    if (h.size() > c->order_cap) {
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        dfree(c->order);
        c->order_cap = 0;
        HIP_TRY(c, dalloc(c->order, h.size()));
        c->order_cap = h.size();
    }
    HIP_TRY(c, hipMemcpyAsync(c->order, h.data(), h.size() * sizeof(int32_t),
                              hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->order_len = len;
    c->order_ok = true;
    for (auto &g : c->graphs) (void)hipGraphExecDestroy(g.second);
    c->graphs.clear();
    c->epoch += 1;
    return LPT_OK;
}

// Next timing event of the pool (created on first use).
hipError_t next_event(lpt_ctx *c, hipEvent_t &ev)
{
    if (c->ev_used == c->ev_pool.size()) {
        hipEvent_t e;
        const hipError_t r = hipEventCreate(&e);
        if (r != hipSuccess) return r;
        c->ev_pool.push_back(e);
    }
    ev = c->ev_pool[c->ev_used++];
    return hipSuccess;
}

hipError_t mark(lpt_ctx *c, hipEvent_t &ev)
{
    const hipError_t r = next_event(c, ev);
    return r != hipSuccess ? r : hipEventRecord(ev, c->stream);
}

// Cell-order re-sort: keys, radix sort, then the permutation of the state
// into the other buffer.  With `perm_out`, the permutation is left to the
// caller's next step kernel instead, which reads through it:
// *perm_out receives the permutation (dst slot -> src slot; null if nothing
// was sorted) and the state buffer does not change here.
lpt_status do_sort(lpt_ctx *c, const uint32_t **perm_out = nullptr,
                   const uint32_t **applied = nullptr)
{
    if (perm_out) *perm_out = nullptr;
    if (applied) *applied = nullptr;
    if (c->np <= 1) return LPT_OK;
    lpt_status s = ensure_sort_work(c);
    if (s != LPT_OK) return s;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (c->time_kernels) HIP_TRY(c, mark(c, e0));
    const StepParams P = make_params(c);
    const int tb = tile_bits(c);
    // the cell-inside-tile key on every re-sort (1), or on the first one (2),
    // where it fits in 32 bits; tiles only otherwise
    bool cells = c->sort_cells == 1 || (c->sort_cells == 2 && !c->sorted_once);
    if (cells && key_width(c->n, c->sort_tile, 1, (int)c->sp.size()) > 32) cells = false;
    c->sorted_once = true;
    const int kb = std::max(1, key_width(c->n, c->sort_tile, cells, (int)c->sp.size()));
    if (c->precision == LPT_FP64)
        HIP_TRY(c, launch_keys64(P, c->s64[c->cur], c->sort_tile, tb, cells, kb, c->sw,
                                 c->stream));
    else
        HIP_TRY(c, launch_keys32(P, c->s32[c->cur], c->sort_tile, tb, cells, kb, c->sw,
                                 c->stream));
    int res = 0;
    HIP_TRY(c, radix_sort(c->sw, c->np, kb, true, true, &res, c->stream));
    const uint32_t *perm = c->sw.vals[res];
    if (perm_out) {
        *perm_out = perm;
        if (c->time_kernels) {
            HIP_TRY(c, mark(c, e1));
            c->ev_sort.emplace_back(e0, e1);
        }
        return LPT_OK;
    }
    if (c->precision == LPT_FP64)
        HIP_TRY(c, launch_permute64(c->s64[c->cur], c->s64[1 - c->cur], perm, c->np,
                                    c->has_inertial, c->stream));
    else
        HIP_TRY(c, launch_permute32(c->s32[c->cur], c->s32[1 - c->cur], perm, c->np,
                                    c->has_inertial, c->stream));
    c->cur = 1 - c->cur;
    if (applied) *applied = perm;   // valid until the next sort
    if (c->time_kernels) {
        HIP_TRY(c, mark(c, e1));
        c->ev_sort.emplace_back(e0, e1);
    }
    return LPT_OK;
}

bool is_finite(double v) { return std::isfinite(v); }

}  // namespace

// ---- allocation-free radix sort: a fixed scratch array per GPU -------------
// Room for the sort of up to kStaticSortMax keys: two key and two value
// buffers, the per-tile digit histograms and the per-digit totals (16.3 MiB).
// Each GPU that loads the library holds its own copy for the life of the
// process; every lpt_radix_sort_static call on that GPU shares it.
namespace {
constexpr int64_t kStaticSortMax = LPT_STATIC_SORT_MAX;
constexpr int64_t kStaticSortHist = 256 * ((kStaticSortMax + kSortTileKeys - 1) / kSortTileKeys);
constexpr int64_t kStaticSortWords = 4 * kStaticSortMax + kStaticSortHist + 256;
}  // namespace

static __device__ __align__(256) uint32_t scratch[kStaticSortWords];

namespace {
std::mutex g_scratch_mu;
std::map<int, uint32_t *> g_scratch;   // device -> address of that device's scratch

// Device address of the scratch on the current device (device `dev`), looked
// up once per device.  The array's host-side name is only a handle for the
// lookup: kernels and copies take the returned address.
hipError_t bind_scratch(int dev, uint32_t **out)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    auto it = g_scratch.find(dev);
    if (it != g_scratch.end()) {
        *out = it->second;
        return hipSuccess;
    }
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[dev] = static_cast<uint32_t *>(p);
    *out = static_cast<uint32_t *>(p);
    return hipSuccess;
}
}  // namespace

extern "C" {

const char *lpt_status_string(lpt_status s)
{
    switch (s) {
    case LPT_OK: return "LPT_OK";
    case LPT_E_ARG: return "LPT_E_ARG";
    case LPT_E_STATE: return "LPT_E_STATE";
    case LPT_E_RANGE: return "LPT_E_RANGE";
    case LPT_E_NOMEM: return "LPT_E_NOMEM";
    case LPT_E_HIP: return "LPT_E_HIP";
    }
    return "LPT_E_UNKNOWN";
}

const char *lpt_last_error(const lpt_ctx *ctx) { return ctx ? ctx->err.c_str() : ""; }

static thread_local std::string g_create_error;

lpt_status lpt_create(const lpt_config *cfg, lpt_ctx **out)
{
    if (!cfg || !out) return LPT_E_ARG;
    *out = nullptr;
    const int32_t n = cfg->n;
    if (n < 4 || n > 32768) return LPT_E_ARG;
    if (cfg->precision != LPT_FP64 && cfg->precision != LPT_FP32_SPLIT) return LPT_E_ARG;
    const double L = cfg->length == 0.0 ? 2.0 * M_PI : cfg->length;
    if (!(L > 0.0) || !std::isfinite(L) || !std::isfinite(cfg->t0)) return LPT_E_ARG;
    if (cfg->sort_interval < 0) return LPT_E_ARG;
    int32_t tile = cfg->sort_tile;
    if (tile == 0) {
        tile = 16;
        while (tile > 1 && n % tile) tile >>= 1;
    }
    if (!is_pow2(tile) || n % tile) return LPT_E_ARG;
    const int32_t block = cfg->block_size == 0 ? 256 : cfg->block_size;
    if (block != 64 && block != 128 && block != 256 && block != 512) return LPT_E_ARG;
    if (cfg->flags & ~(LPT_FLAG_COMPAT_EDGE | LPT_FLAG_TIME_KERNELS | LPT_FLAG_DETERMINISTIC_GRAD))
        return LPT_E_ARG;
    const size_t rec_size = cfg->precision == LPT_FP64 ? sizeof(Rec64) : sizeof(float4);
    const int32_t tile_max = (int32_t)(kTileBytesMax / rec_size);
    int32_t tile_cap = cfg->tile_records;
    const int32_t tile_auto = tile_cap == 0;
    if (tile_cap == 0) tile_cap = kTileRecordsDefault;
    else if (tile_cap == -1) tile_cap = 0;
    else if (tile_cap < 16 || tile_cap > tile_max) return LPT_E_ARG;

    lpt_ctx *c = new (std::nothrow) lpt_ctx();
    if (!c) return LPT_E_NOMEM;
    c->cfg = *cfg;
    c->stream = static_cast<hipStream_t>(cfg->hip_stream);
    c->n = n;
    c->L = L;
    c->h = L / n;
    c->invh = n / L;
    c->precision = cfg->precision;
    c->block = block;
    c->sort_interval = cfg->sort_interval;
    c->sort_tile = tile;
    c->tile_cap = tile_cap;
    c->tile_auto = tile_auto;
    c->compat_edge = (cfg->flags & LPT_FLAG_COMPAT_EDGE) != 0;
    c->det_grad = (cfg->flags & LPT_FLAG_DETERMINISTIC_GRAD) != 0;
    c->time_kernels = (cfg->flags & LPT_FLAG_TIME_KERNELS) != 0;
    c->t = cfg->t0;

    auto bail = [&](hipError_t e) {
        g_create_error = hipGetErrorString(e);
        lpt_destroy(c);
        return LPT_E_HIP;
    };
    hipError_t e = hipGetDevice(&c->device);
    if (e != hipSuccess) return bail(e);
    e = bind_scratch(c->device, &c->static_sort);
    if (e != hipSuccess) return bail(e);
    const size_t np2 = (size_t)padded_pitch(n) * (size_t)padded_pitch(n);
    const size_t rec_bytes = np2 * (c->precision == LPT_FP64 ? sizeof(Rec64) : sizeof(float4));
    e = hipMalloc(&c->rec, rec_bytes);
    if (e != hipSuccess) return bail(e);
    e = hipMemsetAsync(c->rec, 0, rec_bytes, c->stream);
    if (e != hipSuccess) return bail(e);
    e = dalloc(c->umax, 2);
    if (e == hipSuccess) e = hipMemsetAsync(c->umax, 0, 2 * sizeof(float), c->stream);
    if (e != hipSuccess) return bail(e);
    e = dalloc(c->clock, 1);
    if (e != hipSuccess) return bail(e);
    DevClock ck{cfg->t0, 0, 0, 0};
    e = hipMemcpyAsync(c->clock, &ck, sizeof ck, hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) return bail(e);
    e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return bail(e);
    *out = c;
    return LPT_OK;
}

void lpt_destroy(lpt_ctx *c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    free_state(c);
    free_sort(c);
    dfree(c->x0);
    dfree(c->v0);
    dfree(c->partials);
    dfree(c->records);
    dfree(c->clock);
    dfree(c->umax);
    dfree(c->ck);
    dfree(c->order);
    dfree(c->ck_perm);
    dfree(c->ck_id0);
    dfree(c->det_acc);
    for (auto &g : c->graphs) (void)hipGraphExecDestroy(g.second);
    c->graphs.clear();
    if (c->own_stream) (void)hipStreamDestroy(c->own_stream);
    if (c->rec) (void)hipFree(c->rec);
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    delete c;
}

lpt_status lpt_synchronize(lpt_ctx *c)
{
    if (!c) return LPT_E_ARG;
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return LPT_OK;
}

// Device copies of caller arrays: `count` doubles per pointer.
namespace {
// Temporary device buffers of one call, freed when the call returns.  A
// copy or kernel enqueued on them may still be in flight when an error path
// returns early, so the stream is drained before they are released.
struct Staged {
    hipStream_t stream = nullptr;
    std::vector<double *> bufs;
    explicit Staged(hipStream_t s) : stream(s) {}
    ~Staged()
    {
        if (bufs.empty()) return;
        (void)hipStreamSynchronize(stream);
        for (double *p : bufs) (void)hipFree(p);
    }
};

lpt_status stage_in(lpt_ctx *c, Staged &st, const double *src, int64_t count, int32_t on_device,
                    const double *&dst)
{
    if (!src) {
        dst = nullptr;
        return LPT_OK;
    }
    if (on_device) {
        dst = src;
        return LPT_OK;
    }
    double *d = nullptr;
    HIP_TRY(c, dalloc(d, (size_t)count));
    st.bufs.push_back(d);
    HIP_TRY(c, hipMemcpyAsync(d, src, (size_t)count * sizeof(double), hipMemcpyHostToDevice,
                              c->stream));
    dst = d;
    return LPT_OK;
}
}  // namespace

lpt_status lpt_set_snapshot(lpt_ctx *c, int32_t slot, double t, const double *u, const double *v,
                            int32_t on_device)
{
    if (!c) return LPT_E_ARG;
    if (slot != 0 && slot != 1) return fail(c, LPT_E_ARG, "slot must be 0 or 1");
    if (!is_finite(t)) return fail(c, LPT_E_ARG, "snapshot time must be finite");
    if (!u || !v) return fail(c, LPT_E_ARG, "u and v must not be NULL");
    HIP_TRY(c, hipSetDevice(c->device));
    const int64_t nn = (int64_t)c->n * c->n;
    Staged st(c->stream);
    const double *du = nullptr, *dv = nullptr;
    lpt_status s = stage_in(c, st, u, nn, on_device, du);
    if (s == LPT_OK) s = stage_in(c, st, v, nn, on_device, dv);
    if (s != LPT_OK) return s;
    HIP_TRY(c, hipMemsetAsync(c->umax + slot, 0, sizeof(float), c->stream));
    HIP_TRY(c, launch_pack(c->rec, c->precision == LPT_FP64, slot, du, dv, c->n, c->invh, c->invh,
                           c->umax + slot, c->stream));
    if (!st.bufs.empty()) HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->slot_set[slot] = true;
    c->t_slot[slot] = t;
    c->ck_valid = false;   // a reverse sweep must see the fields of its forward run
    return LPT_OK;
}

lpt_status lpt_set_snapshot_psi(lpt_ctx *c, int32_t slot, double t, const double *psi,
                                int32_t on_device)
{
    if (!c) return LPT_E_ARG;
    if (slot != 0 && slot != 1) return fail(c, LPT_E_ARG, "slot must be 0 or 1");
    if (!is_finite(t)) return fail(c, LPT_E_ARG, "snapshot time must be finite");
    if (!psi) return fail(c, LPT_E_ARG, "psi must not be NULL");
    HIP_TRY(c, hipSetDevice(c->device));
    const int64_t nn = (int64_t)c->n * c->n;
    Staged st(c->stream);
    const double *dp = nullptr;
    lpt_status s = stage_in(c, st, psi, nn, on_device, dp);
    if (s != LPT_OK) return s;
    // the centred differences are formed inside the ingest pass
    HIP_TRY(c, hipMemsetAsync(c->umax + slot, 0, sizeof(float), c->stream));
    HIP_TRY(c, launch_pack_psi(c->rec, c->precision == LPT_FP64, slot, dp, c->n, c->h, c->invh,
                               c->invh, c->umax + slot, c->stream));
    if (!st.bufs.empty()) HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->slot_set[slot] = true;
    c->t_slot[slot] = t;
    c->ck_valid = false;
    return LPT_OK;
}

lpt_status lpt_set_time_mode(lpt_ctx *c, lpt_time_mode mode)
{
    if (!c) return LPT_E_ARG;
    if (mode != LPT_TIME_BRACKET && mode != LPT_TIME_PINGPONG)
        return fail(c, LPT_E_ARG, "unknown time mode");
    c->time_mode = mode;
    return LPT_OK;
}

namespace {

lpt_status init_species_state(lpt_ctx *c, int sid)
{
    c->sorted_once = false;   // new positions: the next re-sort starts from scratch
    const StepParams P = make_params(c);
    const SpeciesHost &s = c->sp[sid];
    double wa = 1.0, wb = 0.0;
    if (c->slot_set[0] && c->slot_set[1]) weights_at(c, c->steps, c->t, c->t, 1.0, wa, wb);
    const int field = s.vel_from_field ? 1 : 0;
    if (c->precision == LPT_FP64)
        HIP_TRY(c, launch_init64(P, c->s64[c->cur], c->x0, c->v0, static_cast<Rec64 *>(c->rec),
                                 sid, s.offset, s.count, wa, wb, field, c->stream));
    else
        HIP_TRY(c, launch_init32(P, c->s32[c->cur], c->x0, c->v0, static_cast<float4 *>(c->rec),
                                 sid, s.offset, s.count, wa, wb, field, c->stream));
    return LPT_OK;
}

// Grow every state array to `np` particles, keeping the first `old` ones.
lpt_status grow_state(lpt_ctx *c, int64_t np, int64_t old, bool inertial)
{
    const bool fp64 = c->precision == LPT_FP64;
    State64 n64[2]{};
    State32 n32[2]{};
    double2 *nx0 = nullptr, *nv0 = nullptr;
    auto cleanup = [&]() {
        for (int k = 0; k < 2; ++k) {
            dfree(n64[k].pos); dfree(n64[k].disp); dfree(n64[k].vel); dfree(n64[k].id);
            dfree(n32[k].uc); dfree(n32[k].off); dfree(n32[k].vel); dfree(n32[k].id);
        }
        dfree(nx0);
        dfree(nv0);
    };
    bool ok = true;
    const bool vel = inertial || c->has_inertial;
    for (int k = 0; k < 2 && ok; ++k) {
        if (fp64) {
            ok = dalloc(n64[k].pos, np) == hipSuccess && dalloc(n64[k].disp, np) == hipSuccess &&
                 dalloc(n64[k].id, np) == hipSuccess &&
                 (!vel || dalloc(n64[k].vel, np) == hipSuccess);
        } else {
            ok = dalloc(n32[k].uc, np) == hipSuccess && dalloc(n32[k].off, np) == hipSuccess &&
                 dalloc(n32[k].id, np) == hipSuccess &&
                 (!vel || dalloc(n32[k].vel, np) == hipSuccess);
        }
    }
    ok = ok && dalloc(nx0, np) == hipSuccess && (!vel || dalloc(nv0, np) == hipSuccess);
    if (!ok) {
        cleanup();
        (void)hipGetLastError();
        return fail(c, LPT_E_NOMEM, "device allocation of the particle state failed");
    }
    {
        // touch every page of both state buffers now, so that the first
        // steps (whose re-sort writes the other buffer) meet no first-touch
        // cost
        hipError_t e = hipSuccess;
        auto z = [&](void *d, size_t bytes) {
            if (e == hipSuccess && d) e = hipMemsetAsync(d, 0, bytes, c->stream);
        };
        const size_t n = (size_t)np;
        for (int k = 0; k < 2; ++k) {
            if (fp64) {
                z(n64[k].pos, n * sizeof(double2));
                z(n64[k].disp, n * sizeof(double2));
                z(n64[k].vel, n * sizeof(double2));
                z(n64[k].id, n * sizeof(uint32_t));
            } else {
                z(n32[k].uc, n * sizeof(int2));
                z(n32[k].off, n * sizeof(float2));
                z(n32[k].vel, n * sizeof(float2));
                z(n32[k].id, n * sizeof(uint32_t));
            }
        }
        if (e != hipSuccess) {
            cleanup();
            return fail(c, LPT_E_HIP, std::string("state clear: ") + hipGetErrorString(e));
        }
    }
    if (old > 0) {
        const int k = c->cur;
        hipError_t e = hipSuccess;
        auto cp = [&](void *d, const void *s, size_t bytes) {
            if (e == hipSuccess && s && d)
                e = hipMemcpyAsync(d, s, bytes, hipMemcpyDeviceToDevice, c->stream);
        };
        if (fp64) {
            cp(n64[k].pos, c->s64[k].pos, old * sizeof(double2));
            cp(n64[k].disp, c->s64[k].disp, old * sizeof(double2));
            cp(n64[k].vel, c->s64[k].vel, old * sizeof(double2));
            cp(n64[k].id, c->s64[k].id, old * sizeof(uint32_t));
        } else {
            cp(n32[k].uc, c->s32[k].uc, old * sizeof(int2));
            cp(n32[k].off, c->s32[k].off, old * sizeof(float2));
            cp(n32[k].vel, c->s32[k].vel, old * sizeof(float2));
            cp(n32[k].id, c->s32[k].id, old * sizeof(uint32_t));
        }
        cp(nx0, c->x0, old * sizeof(double2));
        cp(nv0, c->v0, old * sizeof(double2));
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) {
            cleanup();
            return fail(c, LPT_E_HIP, std::string("state copy: ") + hipGetErrorString(e));
        }
    }
    free_state(c);
    dfree(c->x0);
    dfree(c->v0);
    for (int k = 0; k < 2; ++k) {
        c->s64[k] = n64[k];
        c->s32[k] = n32[k];
    }
    c->x0 = nx0;
    c->v0 = nv0;
    c->s32[0].x0 = c->s32[1].x0 = nx0;   // the split state's displacement reference
    return LPT_OK;
}

}  // namespace

lpt_status lpt_add_species(lpt_ctx *c, lpt_kind kind, double st, lpt_scheme scheme, int64_t count,
                           const double *x0, const double *y0, const double *vx0,
                           const double *vy0, int32_t on_device, int32_t *species_id)
{
    if (!c) return LPT_E_ARG;
    if (kind != LPT_TRACER && kind != LPT_INERTIAL) return fail(c, LPT_E_ARG, "unknown kind");
    if (!(st >= 0.0) || !is_finite(st)) return fail(c, LPT_E_ARG, "St must be finite and >= 0");
    if (scheme < LPT_BILINEAR || scheme > LPT_BSPLINE) return fail(c, LPT_E_ARG, "unknown scheme");
    if (count < 1) return fail(c, LPT_E_ARG, "count must be >= 1");
    if (!x0 || !y0) return fail(c, LPT_E_ARG, "x0 and y0 must not be NULL");
    if ((vx0 == nullptr) != (vy0 == nullptr))
        return fail(c, LPT_E_ARG, "give both vx0 and vy0 or neither");
    if (c->steps > 0) return fail(c, LPT_E_STATE, "species must be added before the first step");
    if ((int)c->sp.size() >= kMaxSpecies) return fail(c, LPT_E_ARG, "too many species");
    if (c->np + count > (int64_t)0x7FFFFFFF) return fail(c, LPT_E_ARG, "too many particles");
    const bool inertial = kind == LPT_INERTIAL && st > 0.0;
    if (inertial && !vx0 && !(c->slot_set[0] && c->slot_set[1]))
        return fail(c, LPT_E_STATE, "v0 from the field needs both snapshots set");
    int32_t nsp = (int32_t)c->sp.size() + 1;
    if (key_width(c->n, c->sort_tile, c->sort_cells == 1, nsp) > 32)
        return fail(c, LPT_E_ARG, "sort key wider than 32 bits; raise sort_tile");
    HIP_TRY(c, hipSetDevice(c->device));

    Staged stg(c->stream);
    const double *dx = nullptr, *dy = nullptr, *dvx = nullptr, *dvy = nullptr;
    lpt_status s = stage_in(c, stg, x0, count, on_device, dx);
    if (s == LPT_OK) s = stage_in(c, stg, y0, count, on_device, dy);
    if (s == LPT_OK && inertial) s = stage_in(c, stg, vx0, count, on_device, dvx);
    if (s == LPT_OK && inertial) s = stage_in(c, stg, vy0, count, on_device, dvy);
    if (s != LPT_OK) return s;

    const int64_t old = c->np;
    s = grow_state(c, old + count, old, inertial);
    if (s != LPT_OK) return s;
    // partial sums: one slot per logical block of every species
    SpeciesHost h{(int32_t)kind, st, (int32_t)scheme, count, old, inertial && !vx0};
    c->sp.push_back(h);
    c->order_ok = false;
    c->np = old + count;
    c->has_inertial = c->has_inertial || inertial;
    c->has_cubic = c->has_cubic || scheme != LPT_BILINEAR;
    const StepParams P = make_params(c);
    const int64_t need = stat_partials_doubles(P, c->block);
    if (need > c->partial_cap) {
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        dfree(c->partials);
        c->partial_cap = 0;
        HIP_TRY(c, dalloc(c->partials, (size_t)need));
        c->partial_cap = need;
    }
    HIP_TRY(c, launch_interleave(c->x0 + old, dx, dy, count, c->stream));
    if (inertial && dvx) HIP_TRY(c, launch_interleave(c->v0 + old, dvx, dvy, count, c->stream));
    s = init_species_state(c, (int)c->sp.size() - 1);
    if (s != LPT_OK) return s;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (species_id) *species_id = (int32_t)c->sp.size() - 1;
    return LPT_OK;
}

lpt_status lpt_init_uniform(lpt_ctx *c, int32_t sid, uint64_t seed)
{
    if (!c) return LPT_E_ARG;
    if (sid < 0 || sid >= (int32_t)c->sp.size()) return fail(c, LPT_E_ARG, "unknown species");
    if (c->steps > 0) return fail(c, LPT_E_STATE, "initialisation only before the first step");
    HIP_TRY(c, hipSetDevice(c->device));
    SpeciesHost &s = c->sp[sid];
    HIP_TRY(c, launch_splitmix(c->x0 + s.offset, s.count, seed, c->L, c->stream));
    s.x0_drawn = true;
    s.x0_seed = seed;
    // a previous sort may have moved particles of this species around inside
    // its range: re-initialising writes the state in original order again
    return init_species_state(c, sid);
}

namespace {

void invalidate_graphs(lpt_ctx *c)
{
    for (auto &g : c->graphs) (void)hipGraphExecDestroy(g.second);
    c->graphs.clear();
    c->epoch += 1;
}

// Argument and state checks shared by lpt_step and lpt_forward_checkpointed.
lpt_status check_steps(lpt_ctx *c, int64_t nsteps, double dt, int32_t stats_every)
{
    if (nsteps < 0) return fail(c, LPT_E_ARG, "nsteps must be >= 0");
    if (!(dt > 0.0) || !is_finite(dt)) return fail(c, LPT_E_ARG, "dt must be finite and > 0");
    if (stats_every < 0) return fail(c, LPT_E_ARG, "stats_every must be >= 0");
    if (c->sp.empty()) return fail(c, LPT_E_STATE, "no species");
    if (!c->slot_set[0] || !c->slot_set[1])
        return fail(c, LPT_E_STATE, "both snapshot slots must be set");
    if (nsteps == 0) return LPT_OK;
    if (c->time_mode == LPT_TIME_PINGPONG) {
        const double gap = std::fabs(c->t_slot[1] - c->t_slot[0]);
        if (std::fabs(gap - dt) > 1e-9 * dt)
            return fail(c, LPT_E_ARG, "ping-pong mode needs dt equal to the snapshot spacing");
    } else {
        const double ta = c->t_slot[0], tb = c->t_slot[1];
        if (!(tb > ta)) return fail(c, LPT_E_STATE, "bracket mode needs t(slot 1) > t(slot 0)");
        const double tol = 1e-9 * (tb - ta);
        double tt = c->t;
        for (int64_t k = 0; k < nsteps; ++k) {
            if (tt < ta - tol || tt + dt > tb + tol) {
                char buf[160];
                std::snprintf(buf, sizeof buf,
                              "step %lld spans [%.17g, %.17g], outside the bracket [%.17g, %.17g]",
                              (long long)(c->steps + k), tt, tt + dt, ta, tb);
                return fail(c, LPT_E_RANGE, buf);
            }
            tt += dt;
        }
    }
    return LPT_OK;
}

lpt_status grow_records(lpt_ctx *c, int64_t nsteps, int32_t stats_every)
{
    int64_t new_rec = 0;
    if (stats_every > 0) new_rec = (c->steps + nsteps) / stats_every - c->steps / stats_every;
    if (c->nrec + new_rec <= c->rec_cap) return LPT_OK;
    const int64_t cap = std::max<int64_t>(2 * c->rec_cap, c->nrec + new_rec + 64);
    const int64_t ns = (int64_t)c->sp.size();
    double *nr = nullptr;
    HIP_TRY(c, dalloc(nr, (size_t)(ns * cap * 8)));
    for (int64_t s = 0; s < ns && c->nrec > 0; ++s)
        HIP_TRY(c, hipMemcpyAsync(nr + s * cap * 8, c->records + s * c->rec_cap * 8,
                                  (size_t)c->nrec * 8 * sizeof(double), hipMemcpyDeviceToDevice,
                                  c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    dfree(c->records);
    c->records = nr;
    c->rec_cap = cap;
    invalidate_graphs(c);
    return LPT_OK;
}

// Temporal weights of the step about to be taken (global number c->steps,
// starting at c->t).
void step_weights(const lpt_ctx *c, double dt, StepParams &P)
{
    const double stage_c[4] = {0.0, 0.5, 0.5, 1.0};
    for (int q = 0; q < 4; ++q) {
        weights_at(c, c->steps, c->t, c->t + stage_c[q] * dt, dt, P.wa[q], P.wb[q]);
        P.smode[q] = slot_mode(P.wa[q], P.wb[q]);
        P.waf[q] = (float)P.wa[q];
        P.wbf[q] = (float)P.wb[q];
    }
    P.ends_one = P.smode[0] != kBlend && P.smode[3] != kBlend;
    P.h0 = P.smode[0] == kSlot1 ? 1 : 0;
    P.h3 = P.smode[3] == kSlot1 ? 1 : 0;
}

void set_dt(StepParams &P, double dt)
{
    P.dt = dt;
    P.dtf = (float)dt;
    P.hdtf = (float)(0.5 * dt);
    P.dt6f = (float)(dt / 6.0);
}

// Enqueue nsteps steps.  With `ckpt`, no re-sort happens, the position of
// every particle is saved before each step whose index in the run is a
// multiple of c->ck_every, and every step's temporal weights are kept.
lpt_status run_steps(lpt_ctx *c, int64_t nsteps, double dt, int32_t stats_every, bool ckpt,
                     bool launch = true)
{
    StepParams P = make_params(c);
    set_dt(P, dt);
    for (int64_t k = 0; k < nsteps; ++k) {
        // the step right after a re-sort applies its permutation itself
        const uint32_t *perm = nullptr;
        if (!ckpt && c->sort_interval > 0 && c->steps % c->sort_interval == 0) {
            if (launch) {
                const lpt_status s = do_sort(c, &perm);
                if (s != LPT_OK) return s;
            } else if (c->np > 1) {
                c->cur = 1 - c->cur;   // where the sort leaves the host state
                c->sorted_once = true;
            }
        }
        if (ckpt && k % c->ck_every == 0) {
            const int64_t seg = k / c->ck_every;
            if (c->ck_sorted) {
                // each segment starts from cell order; its permutation (or,
                // for the first, the slot -> id map) is kept for the sweep
                const uint32_t *applied = nullptr;
                const lpt_status s = do_sort(c, nullptr, &applied);
                if (s != LPT_OK) return s;
                if (seg == 0)
                    HIP_TRY(c, hipMemcpyAsync(c->ck_id0, c->s64[c->cur].id,
                                              (size_t)c->np * sizeof(uint32_t),
                                              hipMemcpyDeviceToDevice, c->stream));
                else
                    HIP_TRY(c, hipMemcpyAsync(c->ck_perm + (seg - 1) * c->np, applied,
                                              (size_t)c->np * sizeof(uint32_t),
                                              hipMemcpyDeviceToDevice, c->stream));
            }
            HIP_TRY(c, hipMemcpyAsync(c->ck + seg * c->np, c->s64[c->cur].pos,
                                      (size_t)c->np * sizeof(double2), hipMemcpyDeviceToDevice,
                                      c->stream));
        }
        step_weights(c, dt, P);
        if (ckpt) {
            StepWeights w;
            for (int q = 0; q < 4; ++q) {
                w.wa[q] = P.wa[q];
                w.wb[q] = P.wb[q];
            }
            c->ck_w.push_back(w);
        }
        const bool rec = stats_every > 0 && (c->steps + 1) % stats_every == 0;
        if (!launch) {
            c->nrec += rec ? 1 : 0;
            c->t += dt;
            c->steps += 1;
            continue;
        }
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (c->time_kernels) HIP_TRY(c, mark(c, e0));
        if (c->precision == LPT_FP64) {
            HIP_TRY(c, launch_step64(P, c->s64[c->cur], c->s64[perm ? 1 - c->cur : c->cur], perm,
                                     static_cast<const Rec64 *>(c->rec), c->partials, c->clock,
                                     rec, c->has_cubic, c->has_inertial, c->block,
                                     P.total_blocks, c->stream));
            if (perm) c->cur = 1 - c->cur;
        } else if (P.order) {
            // one fused launch over every species: the block-order table
            // gives each XCD the same share of every species, in cell order
            int sch = P.sp[0].scheme;
            for (int s = 1; s < P.nspecies; ++s)
                if (P.sp[s].scheme != sch) sch = kAnyScheme;
            HIP_TRY(c, launch_step32(P, c->s32[c->cur], c->s32[perm ? 1 - c->cur : c->cur], perm,
                                     static_cast<const float4 *>(c->rec), c->partials, c->clock,
                                     rec, sch, c->has_inertial, c->block, P.total_blocks,
                                     c->stream));
            if (perm) c->cur = 1 - c->cur;
        } else {
            // one launch per species: each launch runs one (scheme, kind)
            // body and spreads that species over all XCDs
            for (int s = 0; s < P.nspecies; ++s) {
                const SpeciesDev &d = P.sp[s];
                if (d.block_end <= d.block_begin) continue;
                StepParams Q = P;
                Q.block_base = d.block_begin;
                Q.launch_blocks = d.block_end - d.block_begin;
                HIP_TRY(c, launch_step32(Q, c->s32[c->cur], c->s32[perm ? 1 - c->cur : c->cur],
                                         perm, static_cast<const float4 *>(c->rec), c->partials,
                                         c->clock, rec, d.scheme, d.inertial != 0, c->block,
                                         Q.launch_blocks, c->stream));
            }
            if (perm) c->cur = 1 - c->cur;
        }
        if (c->time_kernels) {
            HIP_TRY(c, mark(c, e1));
            (perm ? c->ev_perm : (rec ? c->ev_stat : c->ev_step)).emplace_back(e0, e1);
        }
        if (rec) {
            if (c->time_kernels) HIP_TRY(c, mark(c, e0));
            HIP_TRY(c, launch_finalize(P, c->partials, c->clock, c->records, c->rec_cap,
                                       c->cfg.t0, c->block, c->stream));
            if (c->time_kernels) {
                HIP_TRY(c, mark(c, e1));
                c->ev_fin.emplace_back(e0, e1);
            }
            c->nrec += 1;
        }
        c->t += dt;
        c->steps += 1;
    }
    return LPT_OK;
}

// Steps in chunks of c->graph_chunk, each captured once into a hipGraph and
// replayed.  A chunk's kernel parameters depend only on the step number
// modulo the ping-pong/statistics/sort period, the current state buffer, the
// chunk length, dt and stats_every, which together key the cache; any
// reallocation of a buffer a graph holds clears it.  The host bookkeeping
// (time, step count, records, state buffer) advances exactly as for eager
// launches.  The step and sort paths hold no memset and no allocation, so
// they capture cleanly; the sort workspace is allocated before capture.
lpt_status run_graph_chunks_on(lpt_ctx *c, int64_t nsteps, double dt, int32_t stats_every)
{
    if (c->sort_interval > 0) {
        const lpt_status s = ensure_sort_work(c);
        if (s != LPT_OK) return s;
    }
    auto lcm = [](int64_t a, int64_t b) {
        int64_t x = a, y = b;
        while (y) {
            const int64_t t = x % y;
            x = y;
            y = t;
        }
        return a / x * b;
    };
    int64_t period = 2;
    if (c->sort_interval > 0) period = lcm(period, c->sort_interval);
    if (stats_every > 0) period = lcm(period, stats_every);
    uint64_t dt_bits;
    std::memcpy(&dt_bits, &dt, sizeof dt_bits);
    while (nsteps > 0) {
        const int64_t len = std::min<int64_t>(c->graph_chunk, nsteps);
        // the first re-sort may use another key than the later ones
        const auto key = std::make_tuple(c->steps % period, c->cur, len, dt_bits, stats_every,
                                         c->epoch, c->sorted_once);
        auto it = c->graphs.find(key);
        hipGraphExec_t exec = nullptr;
        if (it == c->graphs.end()) {
            HIP_TRY(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
            const lpt_status s = run_steps(c, len, dt, stats_every, false, true);
            hipGraph_t g = nullptr;
            const hipError_t e = hipStreamEndCapture(c->stream, &g);
            if (s != LPT_OK) {
                if (g) (void)hipGraphDestroy(g);
                return s;
            }
            HIP_TRY(c, e);
            const hipError_t ei = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            HIP_TRY(c, ei);
            c->graphs.emplace(key, exec);
        } else {
            exec = it->second;
            const lpt_status s = run_steps(c, len, dt, stats_every, false, false);
            if (s != LPT_OK) return s;
        }
        HIP_TRY(c, hipGraphLaunch(exec, c->stream));
        nsteps -= len;
    }
    return LPT_OK;
}

// Graph chunks need a capturable stream: a context on the null stream
// captures and replays on a blocking stream of its own, which stays ordered
// with the null stream.
lpt_status run_graph_chunks(lpt_ctx *c, int64_t nsteps, double dt, int32_t stats_every)
{
    if (c->stream) return run_graph_chunks_on(c, nsteps, dt, stats_every);
    if (!c->own_stream) HIP_TRY(c, hipStreamCreate(&c->own_stream));
    c->stream = c->own_stream;
    const lpt_status s = run_graph_chunks_on(c, nsteps, dt, stats_every);
    c->stream = nullptr;
    return s;
}

}  // namespace

lpt_status lpt_step(lpt_ctx *c, int64_t nsteps, double dt, int32_t stats_every)
{
    if (!c) return LPT_E_ARG;
    lpt_status s = check_steps(c, nsteps, dt, stats_every);
    if (s != LPT_OK || nsteps == 0) return s;
    HIP_TRY(c, hipSetDevice(c->device));
    s = grow_records(c, nsteps, stats_every);
    if (s == LPT_OK) s = ensure_order(c);
    if (s != LPT_OK) return s;
    c->ck_valid = false;
    if (c->graph_chunk <= 0 || c->time_mode != LPT_TIME_PINGPONG || c->time_kernels)
        return run_steps(c, nsteps, dt, stats_every, false);
    return run_graph_chunks(c, nsteps, dt, stats_every);
}

lpt_status lpt_time_steps(lpt_ctx *c, int64_t nsteps, double dt, int32_t stats_every,
                          double *ms)
{
    if (!c) return LPT_E_ARG;
    if (!ms) return fail(c, LPT_E_ARG, "ms must not be NULL");
    lpt_status s = check_steps(c, nsteps, dt, stats_every);
    if (s != LPT_OK) return s;
    HIP_TRY(c, hipSetDevice(c->device));
    s = grow_records(c, nsteps, stats_every);   // outside the timed interval
    if (s == LPT_OK) s = ensure_order(c);
    if (s != LPT_OK) return s;
    if (c->sort_interval > 0) {
        s = ensure_sort_work(c);
        if (s != LPT_OK) return s;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(c, hipEventCreate(&e0));
    hipError_t e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        (void)hipEventDestroy(e0);
        HIP_TRY(c, e);
    }
    // a null-stream context replays graphs on its own blocking stream, which
    // the null stream waits for, so the events bracket the work either way
    e = hipEventRecord(e0, c->stream);
    if (e == hipSuccess) {
        s = lpt_step(c, nsteps, dt, stats_every);
        if (s == LPT_OK) e = hipEventRecord(e1, c->stream);
    }
    float t = 0.f;
    if (e == hipSuccess && s == LPT_OK) e = hipEventSynchronize(e1);
    if (e == hipSuccess && s == LPT_OK) e = hipEventElapsedTime(&t, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (s != LPT_OK) return s;
    HIP_TRY(c, e);
    *ms = t;
    return LPT_OK;
}

lpt_status lpt_forward_checkpointed(lpt_ctx *c, int64_t nsteps, double dt, int32_t ckpt_every)
{
    if (!c) return LPT_E_ARG;
    if (c->precision != LPT_FP64)
        return fail(c, LPT_E_STATE, "derivatives need an LPT_FP64 context");
    for (const SpeciesHost &h : c->sp)
        if (h.kind == LPT_INERTIAL && h.st > 0.0)
            return fail(c, LPT_E_STATE, "derivatives are implemented for tracers only");
    if (nsteps < 1) return fail(c, LPT_E_ARG, "nsteps must be >= 1");
    if (ckpt_every < 1) return fail(c, LPT_E_ARG, "ckpt_every must be >= 1");
    lpt_status s = check_steps(c, nsteps, dt, 0);
    if (s != LPT_OK) return s;
    HIP_TRY(c, hipSetDevice(c->device));
    s = ensure_order(c);
    if (s != LPT_OK) return s;
    const int64_t nseg = (nsteps + ckpt_every - 1) / ckpt_every;
    const size_t need = (size_t)nseg * (size_t)c->np * sizeof(double2);
    if (need > c->ck_bytes) {
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        dfree(c->ck);
        c->ck_bytes = 0;
        void *q = nullptr;
        if (hipMalloc(&q, need) != hipSuccess) {
            (void)hipGetLastError();
            return fail(c, LPT_E_NOMEM, "checkpoint buffer allocation failed");
        }
        c->ck = static_cast<double2 *>(q);
        c->ck_bytes = need;
    }
    // with re-sorting enabled, every segment starts from cell order, so both
    // sweeps touch the grid coherently per block all along the run
    const bool sorted = c->sort_interval > 0 && c->np > 1;
    if (sorted) {
        const size_t pb = (size_t)(nseg - 1) * (size_t)c->np * sizeof(uint32_t);
        const size_t ib = (size_t)c->np * sizeof(uint32_t);
        if (pb > c->ck_perm_bytes || ib > c->ck_id0_bytes) {
            HIP_TRY(c, hipStreamSynchronize(c->stream));
            dfree(c->ck_perm);
            dfree(c->ck_id0);
            c->ck_perm_bytes = c->ck_id0_bytes = 0;
            void *q = nullptr, *r = nullptr;
            if (hipMalloc(&q, std::max<size_t>(pb, 4)) != hipSuccess ||
                hipMalloc(&r, ib) != hipSuccess) {
                (void)hipGetLastError();
                if (q) (void)hipFree(q);
                return fail(c, LPT_E_NOMEM, "checkpoint permutation allocation failed");
            }
            c->ck_perm = static_cast<uint32_t *>(q);
            c->ck_id0 = static_cast<uint32_t *>(r);
            c->ck_perm_bytes = std::max<size_t>(pb, 4);
            c->ck_id0_bytes = ib;
        }
    }
    c->ck_every = ckpt_every;
    c->ck_nsteps = nsteps;
    c->ck_w.clear();
    c->ck_dt = dt;
    c->ck_step0 = c->steps;
    c->ck_t0 = c->t;
    c->ck_valid = false;
    c->ck_sorted = sorted;
    s = run_steps(c, nsteps, dt, 0, true);
    if (s != LPT_OK) return s;
    c->ck_valid = true;
    return LPT_OK;
}

namespace {

// Reverse sweep over the last checkpointed run: per segment, newest first,
// rebuild the segment's per-step positions from its checkpoint, then take
// the adjoint kernel back through them.
lpt_status reverse_sweep(lpt_ctx *c, int nl, double2 *&lam, double2 *&lam_spare, void *gU,
                         bool det)
{
    const int64_t E = c->ck_every, N = c->ck_nsteps, np = c->np;
    const int64_t tape_len = std::min(E, N);
    double2 *tape = nullptr;
    HIP_TRY(c, dalloc(tape, (size_t)(tape_len * np)));
    StepParams P = make_params(c);
    set_dt(P, c->ck_dt);
    // The sweep's LDS boxes (field tile, gradient accumulators) take the full
    // displacement bound as their halo, so that a block's stage points stay
    // inside them (an oversized box is trimmed by the kernels); a point
    // outside costs global gathers and, in the adjoint, global atomics.
    P.halo_scale = 1.0f;
    const Rec64 *rec = static_cast<const Rec64 *>(c->rec);
    hipError_t e = hipSuccess;
    for (int64_t seg = (N - 1) / E; seg >= 0 && e == hipSuccess; --seg) {
        const int64_t k0 = seg * E, len = std::min(E, N - k0);
        e = hipMemcpyAsync(tape, c->ck + seg * np, (size_t)np * sizeof(double2),
                           hipMemcpyDeviceToDevice, c->stream);
        for (int64_t s = 1; s < len && e == hipSuccess; ++s) {
            const StepWeights &w = c->ck_w[(size_t)(k0 + s - 1)];
            for (int q = 0; q < 4; ++q) {
                P.wa[q] = w.wa[q];
                P.wb[q] = w.wb[q];
                P.smode[q] = slot_mode(w.wa[q], w.wb[q]);
            }
            e = launch_recompute64(P, rec, tape + (s - 1) * np, tape + s * np, c->has_cubic,
                                   c->block, c->stream);
        }
        for (int64_t s = len - 1; s >= 0 && e == hipSuccess; --s) {
            const StepWeights &w = c->ck_w[(size_t)(k0 + s)];
            for (int q = 0; q < 4; ++q) {
                P.wa[q] = w.wa[q];
                P.wb[q] = w.wb[q];
                P.smode[q] = slot_mode(w.wa[q], w.wb[q]);
            }
            e = launch_adjoint64(P, rec, tape + s * np, lam, nl, gU, det, c->has_cubic,
                                 c->block, c->stream);
        }
        // back to the previous segment's slot order: the slot that segment
        // seg's sort filled from slot perm[i] gives its adjoint back there
        if (c->ck_sorted && seg > 0 && e == hipSuccess) {
            e = launch_unpermute_adjoint(c->ck_perm + (seg - 1) * np, np, nl, lam, lam_spare,
                                         c->stream);
            std::swap(lam, lam_spare);
        }
    }
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    dfree(tape);
    HIP_TRY(c, e);
    return LPT_OK;
}

lpt_status check_adjoint(lpt_ctx *c)
{
    if (!c->ck_valid || c->steps != c->ck_step0 + c->ck_nsteps)
        return fail(c, LPT_E_STATE,
                    "call lpt_forward_checkpointed first (and take no other step after it)");
    return LPT_OK;
}

}  // namespace

lpt_status lpt_adjoint(lpt_ctx *c, const double *gx_T, const double *gy_T, double *gx_0,
                       double *gy_0, double *gU, int32_t on_device)
{
    if (!c) return LPT_E_ARG;
    if (!gx_T || !gy_T) return fail(c, LPT_E_ARG, "gx_T and gy_T must not be NULL");
    lpt_status s = check_adjoint(c);
    if (s != LPT_OK) return s;
    HIP_TRY(c, hipSetDevice(c->device));
    const int64_t np = c->np, nn4 = 4 * (int64_t)c->n * c->n;
    Staged st(c->stream);
    const double *dgx = nullptr, *dgy = nullptr;
    s = stage_in(c, st, gx_T, np, on_device, dgx);
    if (s == LPT_OK) s = stage_in(c, st, gy_T, np, on_device, dgy);
    if (s != LPT_OK) return s;
    double2 *lam = nullptr, *spare = nullptr;
    HIP_TRY(c, dalloc(lam, (size_t)np));
    st.bufs.push_back(reinterpret_cast<double *>(lam));
    if (c->ck_sorted) {
        HIP_TRY(c, dalloc(spare, (size_t)np));
        st.bufs.push_back(reinterpret_cast<double *>(spare));
    }
    double *dU = nullptr;
    if (gU) {
        if (on_device) {
            dU = gU;
        } else {
            HIP_TRY(c, dalloc(dU, (size_t)nn4));
            st.bufs.push_back(dU);
        }
        if (!c->det_grad) HIP_TRY(c, hipMemsetAsync(dU, 0, (size_t)nn4 * sizeof(double), c->stream));
    }
    // deterministic mode: the sweep sums fixed-point pairs in a context-owned
    // accumulator (two 64-bit words per gradient entry), converted at the end
    void *acc = dU;
    if (gU && c->det_grad) {
        if (c->det_acc_words < 2 * nn4) {
            HIP_TRY(c, hipStreamSynchronize(c->stream));
            dfree(c->det_acc);
            c->det_acc_words = 0;
            HIP_TRY(c, dalloc(c->det_acc, (size_t)(2 * nn4)));
            c->det_acc_words = 2 * nn4;
        }
        HIP_TRY(c, launch_zero_words(c->det_acc, 2 * nn4, c->stream));
        acc = c->det_acc;
    }
    // seeded in the final slot order; the sweep ends in the first segment's
    const uint32_t *id = c->s64[c->cur].id;
    HIP_TRY(c, launch_seed_adjoint(id, np, 1, dgx, dgy, lam, c->stream));
    s = reverse_sweep(c, 1, lam, spare, acc, gU && c->det_grad);
    if (s != LPT_OK) return s;
    if (c->ck_sorted) id = c->ck_id0;
    if (gU && c->det_grad) HIP_TRY(c, launch_fixed_to_double(c->det_acc, nn4, dU, c->stream));
    double *ox = gx_0, *oy = gy_0;
    if (!on_device) {
        if (gx_0) {
            HIP_TRY(c, dalloc(ox, (size_t)np));
            st.bufs.push_back(ox);
        }
        if (gy_0) {
            HIP_TRY(c, dalloc(oy, (size_t)np));
            st.bufs.push_back(oy);
        }
    }
    HIP_TRY(c, launch_gather_adjoint(id, np, 1, lam, ox, oy, nullptr, nullptr, 0.0, c->stream));
    if (!on_device) {
        if (gx_0)
            HIP_TRY(c, hipMemcpyAsync(gx_0, ox, (size_t)np * sizeof(double),
                                      hipMemcpyDeviceToHost, c->stream));
        if (gy_0)
            HIP_TRY(c, hipMemcpyAsync(gy_0, oy, (size_t)np * sizeof(double),
                                      hipMemcpyDeviceToHost, c->stream));
        if (gU)
            HIP_TRY(c, hipMemcpyAsync(gU, dU, (size_t)nn4 * sizeof(double),
                                      hipMemcpyDeviceToHost, c->stream));
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return LPT_OK;
}

namespace {
// Jacobian sweep of the last checkpointed run: F (4 np doubles) and/or the
// FTLE sigma (np doubles) over the run's duration, in id order.
lpt_status jacobian_sweep(lpt_ctx *c, double *F, double *sigma, int32_t on_device)
{
    lpt_status s = check_adjoint(c);
    if (s != LPT_OK) return s;
    HIP_TRY(c, hipSetDevice(c->device));
    const int64_t np = c->np;
    Staged st(c->stream);
    double2 *lam = nullptr, *spare = nullptr;
    HIP_TRY(c, dalloc(lam, (size_t)(2 * np)));
    st.bufs.push_back(reinterpret_cast<double *>(lam));
    if (c->ck_sorted) {
        HIP_TRY(c, dalloc(spare, (size_t)(2 * np)));
        st.bufs.push_back(reinterpret_cast<double *>(spare));
    }
    const uint32_t *id = c->s64[c->cur].id;
    HIP_TRY(c, launch_seed_adjoint(id, np, 2, nullptr, nullptr, lam, c->stream));
    s = reverse_sweep(c, 2, lam, spare, nullptr, false);
    if (s != LPT_OK) return s;
    if (c->ck_sorted) id = c->ck_id0;
    double *dF = F, *dS = sigma;
    if (!on_device) {
        if (F) {
            HIP_TRY(c, dalloc(dF, (size_t)(4 * np)));
            st.bufs.push_back(dF);
        }
        if (sigma) {
            HIP_TRY(c, dalloc(dS, (size_t)np));
            st.bufs.push_back(dS);
        }
    }
    const double T = (double)c->ck_nsteps * c->ck_dt;
    HIP_TRY(c, launch_gather_adjoint(id, np, 2, lam, nullptr, nullptr, dF, dS, T, c->stream));
    if (!on_device) {
        if (F)
            HIP_TRY(c, hipMemcpyAsync(F, dF, (size_t)(4 * np) * sizeof(double),
                                      hipMemcpyDeviceToHost, c->stream));
        if (sigma)
            HIP_TRY(c, hipMemcpyAsync(sigma, dS, (size_t)np * sizeof(double),
                                      hipMemcpyDeviceToHost, c->stream));
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return LPT_OK;
}
}  // namespace

lpt_status lpt_jacobian(lpt_ctx *c, double *F, int32_t on_device)
{
    if (!c) return LPT_E_ARG;
    if (!F) return fail(c, LPT_E_ARG, "F must not be NULL");
    return jacobian_sweep(c, F, nullptr, on_device);
}

lpt_status lpt_ftle(lpt_ctx *c, double *sigma, double *F, int32_t on_device)
{
    if (!c) return LPT_E_ARG;
    if (!sigma) return fail(c, LPT_E_ARG, "sigma must not be NULL");
    return jacobian_sweep(c, F, sigma, on_device);
}

lpt_status lpt_sort(lpt_ctx *c)
{
    if (!c) return LPT_E_ARG;
    if (c->sp.empty()) return fail(c, LPT_E_STATE, "no species");
    HIP_TRY(c, hipSetDevice(c->device));
    return do_sort(c);
}

namespace {
lpt_status readout(lpt_ctx *c, int32_t sid, double *xw, double *yw, double *xu, double *yu,
                   double *vx, double *vy, int32_t on_device)
{
    const SpeciesHost &s = c->sp[sid];
    HIP_TRY(c, hipSetDevice(c->device));
    double *outs[6] = {xw, yw, xu, yu, vx, vy};
    double *dev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    Staged st(c->stream);
    for (int k = 0; k < 6; ++k) {
        if (!outs[k]) continue;
        if (on_device) {
            dev[k] = outs[k];
        } else {
            HIP_TRY(c, dalloc(dev[k], (size_t)s.count));
            st.bufs.push_back(dev[k]);
        }
    }
    if (c->precision == LPT_FP64)
        HIP_TRY(c, launch_readout64(c->s64[c->cur], c->x0, s.offset, s.count, c->L, dev[0], dev[1],
                                    dev[2], dev[3], dev[4], dev[5], c->stream));
    else
        HIP_TRY(c, launch_readout32(make_params(c), c->s32[c->cur], s.offset, s.count, dev[0],
                                    dev[1], dev[2], dev[3], dev[4], dev[5], c->stream));
    if (!on_device) {
        for (int k = 0; k < 6; ++k)
            if (outs[k])
                HIP_TRY(c, hipMemcpyAsync(outs[k], dev[k], (size_t)s.count * sizeof(double),
                                          hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
    }
    return LPT_OK;
}
}  // namespace

lpt_status lpt_get_positions(lpt_ctx *c, int32_t sid, double *xw, double *yw, double *xu,
                             double *yu, int32_t on_device)
{
    if (!c) return LPT_E_ARG;
    if (sid < 0 || sid >= (int32_t)c->sp.size()) return fail(c, LPT_E_ARG, "unknown species");
    return readout(c, sid, xw, yw, xu, yu, nullptr, nullptr, on_device);
}

lpt_status lpt_get_velocities(lpt_ctx *c, int32_t sid, double *vx, double *vy, int32_t on_device)
{
    if (!c) return LPT_E_ARG;
    if (sid < 0 || sid >= (int32_t)c->sp.size()) return fail(c, LPT_E_ARG, "unknown species");
    const SpeciesHost &s = c->sp[sid];
    if (!(s.kind == LPT_INERTIAL && s.st > 0.0))
        return fail(c, LPT_E_STATE, "species carries no particle velocity (tracer or St = 0)");
    return readout(c, sid, nullptr, nullptr, nullptr, nullptr, vx, vy, on_device);
}

lpt_status lpt_get_stats(lpt_ctx *c, int32_t sid, lpt_stat *out, int64_t cap, int64_t *n_written)
{
    if (!c) return LPT_E_ARG;
    if (sid < 0 || sid >= (int32_t)c->sp.size()) return fail(c, LPT_E_ARG, "unknown species");
    if (cap < 0 || (cap > 0 && !out)) return fail(c, LPT_E_ARG, "bad output buffer");
    HIP_TRY(c, hipSetDevice(c->device));
    const int64_t m = std::min(cap, c->nrec);
    if (m > 0) {
        HIP_TRY(c, hipMemcpyAsync(out, c->records + (int64_t)sid * c->rec_cap * 8,
                                  (size_t)m * sizeof(lpt_stat), hipMemcpyDeviceToHost,
                                  c->stream));
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (n_written) *n_written = m;
    return LPT_OK;
}

lpt_status lpt_get_order(lpt_ctx *c, int32_t sid, int32_t *ids, int32_t on_device)
{
    if (!c) return LPT_E_ARG;
    if (sid < 0 || sid >= (int32_t)c->sp.size()) return fail(c, LPT_E_ARG, "unknown species");
    if (!ids) return fail(c, LPT_E_ARG, "ids must not be NULL");
    HIP_TRY(c, hipSetDevice(c->device));
    const SpeciesHost &s = c->sp[sid];
    const uint32_t *id = c->precision == LPT_FP64 ? c->s64[c->cur].id : c->s32[c->cur].id;
    int32_t *d = ids;
    if (!on_device) HIP_TRY(c, dalloc(d, (size_t)s.count));
    hipError_t e = launch_order(id, s.offset, s.count, d, c->stream);
    if (e == hipSuccess && !on_device)
        e = hipMemcpyAsync(ids, d, (size_t)s.count * sizeof(int32_t), hipMemcpyDeviceToHost,
                           c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (!on_device) (void)hipFree(d);
    HIP_TRY(c, e);
    return LPT_OK;
}

lpt_status lpt_get_timing(lpt_ctx *c, lpt_timing *out, int32_t reset)
{
    if (!c) return LPT_E_ARG;
    if (!out) return fail(c, LPT_E_ARG, "out must not be NULL");
    if (!c->time_kernels) return fail(c, LPT_E_STATE, "context created without LPT_FLAG_TIME_KERNELS");
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    lpt_timing t{};
    for (const auto &p : c->ev_step) {
        float ms = 0.f;
        HIP_TRY(c, hipEventElapsedTime(&ms, p.first, p.second));
        t.step_kernel_ms += ms;
        t.step_launches += 1;
    }
    for (const auto &p : c->ev_sort) {
        float ms = 0.f;
        HIP_TRY(c, hipEventElapsedTime(&ms, p.first, p.second));
        t.sort_ms += ms;
        t.sorts += 1;
    }
    for (const auto &p : c->ev_perm) {
        float ms = 0.f;
        HIP_TRY(c, hipEventElapsedTime(&ms, p.first, p.second));
        t.perm_step_ms += ms;
        t.perm_steps += 1;
    }
    for (const auto &p : c->ev_stat) {
        float ms = 0.f;
        HIP_TRY(c, hipEventElapsedTime(&ms, p.first, p.second));
        t.stats_step_ms += ms;
        t.stats_steps += 1;
    }
    for (const auto &p : c->ev_fin) {
        float ms = 0.f;
        HIP_TRY(c, hipEventElapsedTime(&ms, p.first, p.second));
        t.finalize_ms += ms;
    }
    *out = t;
    if (reset) {
        c->ev_step.clear();
        c->ev_sort.clear();
        c->ev_perm.clear();
        c->ev_stat.clear();
        c->ev_fin.clear();
        c->ev_used = 0;
    }
    return LPT_OK;
}

lpt_status lpt_get_time(lpt_ctx *c, int64_t *steps, double *t)
{
    if (!c) return LPT_E_ARG;
    if (steps) *steps = c->steps;
    if (t) *t = c->t;
    return LPT_OK;
}

lpt_status lpt_interp(lpt_ctx *c, lpt_scheme scheme, int64_t npts, const double *x, const double *y,
                      double w_a, double w_b, double *u, double *v, int32_t on_device)
{
    if (!c) return LPT_E_ARG;
    if (scheme < LPT_BILINEAR || scheme > LPT_BSPLINE) return fail(c, LPT_E_ARG, "unknown scheme");
    if (npts < 0) return fail(c, LPT_E_ARG, "npts must be >= 0");
    if (npts > 0 && (!x || !y || !u || !v)) return fail(c, LPT_E_ARG, "NULL array");
    if (!is_finite(w_a) || !is_finite(w_b)) return fail(c, LPT_E_ARG, "weights must be finite");
    if (npts == 0) return LPT_OK;
    HIP_TRY(c, hipSetDevice(c->device));
    Staged st(c->stream);
    const double *dx = nullptr, *dy = nullptr;
    lpt_status s = stage_in(c, st, x, npts, on_device, dx);
    if (s == LPT_OK) s = stage_in(c, st, y, npts, on_device, dy);
    if (s != LPT_OK) return s;
    double *du = u, *dv = v;
    if (!on_device) {
        HIP_TRY(c, dalloc(du, (size_t)npts));
        st.bufs.push_back(du);
        HIP_TRY(c, dalloc(dv, (size_t)npts));
        st.bufs.push_back(dv);
    }
    const StepParams P = make_params(c);
    if (c->precision == LPT_FP64)
        HIP_TRY(c, launch_interp64(P, static_cast<const Rec64 *>(c->rec), scheme, npts, dx, dy,
                                   w_a, w_b, du, dv, c->stream));
    else
        HIP_TRY(c, launch_interp32(P, static_cast<const float4 *>(c->rec), scheme, npts, dx, dy,
                                   w_a, w_b, du, dv, c->stream));
    if (!on_device) {
        HIP_TRY(c, hipMemcpyAsync(u, du, (size_t)npts * sizeof(double), hipMemcpyDeviceToHost,
                                  c->stream));
        HIP_TRY(c, hipMemcpyAsync(v, dv, (size_t)npts * sizeof(double), hipMemcpyDeviceToHost,
                                  c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
    }
    return LPT_OK;
}

lpt_status lpt_radix_sort(lpt_ctx *c, int64_t npts, int32_t key_bits, const uint32_t *keys_in,
                          uint32_t *keys_out, uint32_t *perm)
{
    if (!c) return LPT_E_ARG;
    if (npts < 0 || npts > (int64_t)0x7FFFFFFF) return fail(c, LPT_E_ARG, "bad npts");
    if (key_bits < 1 || key_bits > 32) return fail(c, LPT_E_ARG, "key_bits must be in [1, 32]");
    if (npts > 0 && !keys_in) return fail(c, LPT_E_ARG, "keys_in must not be NULL");
    if (npts == 0) return LPT_OK;
    HIP_TRY(c, hipSetDevice(c->device));
    SortWork w{};
    lpt_status s = LPT_OK;
    auto release = [&]() {
        (void)hipStreamSynchronize(c->stream);
        dfree(w.keys[0]); dfree(w.keys[1]); dfree(w.vals[0]); dfree(w.vals[1]);
        dfree(w.hist); dfree(w.scan_tmp);
    };
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = dalloc(w.keys[0], npts);
    if (e == hipSuccess) e = dalloc(w.keys[1], npts);
    if (e == hipSuccess) e = dalloc(w.vals[0], npts);
    if (e == hipSuccess) e = dalloc(w.vals[1], npts);
    if (e == hipSuccess) e = dalloc(w.hist, (size_t)sort_hist_entries(npts));
    if (e == hipSuccess) e = dalloc(w.scan_tmp, (size_t)sort_scan_blocks(npts));
    if (e == hipSuccess)
        e = hipMemcpyAsync(w.keys[0], keys_in, (size_t)npts * 4, hipMemcpyDeviceToDevice, c->stream);
    // a single key is its own sorted order (the sort then launches nothing)
    if (e == hipSuccess && npts == 1) e = hipMemsetAsync(w.vals[0], 0, sizeof(uint32_t), c->stream);
    int res = 0;
    if (e == hipSuccess) e = radix_sort(w, npts, key_bits, false, false, &res, c->stream);
    if (e == hipSuccess && keys_out)
        e = hipMemcpyAsync(keys_out, w.keys[res], (size_t)npts * 4, hipMemcpyDeviceToDevice,
                           c->stream);
    if (e == hipSuccess && perm)
        e = hipMemcpyAsync(perm, w.vals[res], (size_t)npts * 4, hipMemcpyDeviceToDevice, c->stream);
    release();
    if (e != hipSuccess) s = fail(c, LPT_E_HIP, std::string("radix sort: ") + hipGetErrorString(e));
    return s;
}

lpt_status lpt_radix_sort_static(lpt_ctx *c, int64_t npts, int32_t key_bits,
                                 const uint32_t *keys_in, uint32_t *keys_out, uint32_t *perm)
{
    if (!c) return LPT_E_ARG;
    if (npts < 0) return fail(c, LPT_E_ARG, "bad npts");
    if (npts > kStaticSortMax)
        return fail(c, LPT_E_ARG,
                    "npts exceeds the fixed scratch of lpt_radix_sort_static (at most " +
                        std::to_string((long long)kStaticSortMax) + " keys)");
    if (key_bits < 1 || key_bits > 32) return fail(c, LPT_E_ARG, "key_bits must be in [1, 32]");
    if (npts > 0 && !keys_in) return fail(c, LPT_E_ARG, "keys_in must not be NULL");
    if (npts == 0) return LPT_OK;
    HIP_TRY(c, hipSetDevice(c->device));
    if (!c->static_sort) return fail(c, LPT_E_STATE, "no fixed scratch on this device");
    uint32_t *base = c->static_sort;
    if (npts == 1) {   // a single key is its own sorted order
        if (keys_out)
            HIP_TRY(c, hipMemcpyAsync(keys_out, keys_in, sizeof(uint32_t),
                                      hipMemcpyDeviceToDevice, c->stream));
        if (perm) HIP_TRY(c, launch_fill_u32(perm, 1, 0u, c->stream));
        return LPT_OK;
    }
    SortWork w{};
    w.keys[0] = base;
    w.keys[1] = base + kStaticSortMax;
    w.vals[0] = base + 2 * kStaticSortMax;
    w.vals[1] = base + 3 * kStaticSortMax;
    w.hist = base + 4 * kStaticSortMax;
    w.scan_tmp = w.hist + kStaticSortHist;
    w.capacity = kStaticSortMax;
    HIP_TRY(c, hipMemcpyAsync(w.keys[0], keys_in, (size_t)npts * 4, hipMemcpyDeviceToDevice,
                              c->stream));
    int res = 0;
    HIP_TRY(c, radix_sort(w, npts, key_bits, false, false, &res, c->stream));
    if (keys_out)
        HIP_TRY(c, hipMemcpyAsync(keys_out, w.keys[res], (size_t)npts * 4,
                                  hipMemcpyDeviceToDevice, c->stream));
    if (perm)
        HIP_TRY(c, hipMemcpyAsync(perm, w.vals[res], (size_t)npts * 4, hipMemcpyDeviceToDevice,
                                  c->stream));
    return LPT_OK;
}

// ---- checkpoint / resume ---------------------------------------------------
}  // extern "C"

namespace {

struct StateHeader {
    char magic[8];
    uint32_t version;
    int32_t n, precision, nspecies;
    int64_t np, steps, nrec;
    double t;
    int32_t time_mode, has_vel;
    int32_t sorted_once, pad_;   // whether the first re-sort has happened
    DevClock clock;
};

struct StateSpecies {
    int32_t kind, scheme;
    double st;
    int64_t count;
    int32_t vel_from_field, pad_;
};

const char kStateMagic[8] = {'L', 'P', 'T', 'S', 'T', 'A', 'T', 'E'};

// Byte sizes of the per-particle arrays, in blob order.
std::vector<size_t> state_arrays(const lpt_ctx *c)
{
    const size_t np = (size_t)c->np;
    std::vector<size_t> a;
    if (c->precision == LPT_FP64) {
        a = {np * sizeof(double2), np * sizeof(double2)};
        if (c->has_inertial) a.push_back(np * sizeof(double2));
    } else {
        a = {np * sizeof(int2), np * sizeof(float2)};
        if (c->has_inertial) a.push_back(np * sizeof(float2));
    }
    a.push_back(np * sizeof(uint32_t));                    // id (slot -> particle)
    a.push_back(np * sizeof(double2));                     // x0 (by particle)
    if (c->has_inertial) a.push_back(np * sizeof(double2));  // v0 (by particle)
    return a;
}

std::vector<void *> state_ptrs(lpt_ctx *c, int k)
{
    std::vector<void *> p;
    if (c->precision == LPT_FP64) {
        p = {c->s64[k].pos, c->s64[k].disp};
        if (c->has_inertial) p.push_back(c->s64[k].vel);
        p.push_back(c->s64[k].id);
    } else {
        p = {c->s32[k].uc, c->s32[k].off};
        if (c->has_inertial) p.push_back(c->s32[k].vel);
        p.push_back(c->s32[k].id);
    }
    p.push_back(c->x0);
    if (c->has_inertial) p.push_back(c->v0);
    return p;
}

size_t state_size(const lpt_ctx *c)
{
    size_t s = sizeof(StateHeader) + c->sp.size() * sizeof(StateSpecies);
    for (size_t b : state_arrays(c)) s += b;
    return s + c->sp.size() * (size_t)c->nrec * 8 * sizeof(double);
}

}  // namespace

extern "C" {

lpt_status lpt_get_state(lpt_ctx *c, void *blob, size_t cap, size_t *size)
{
    if (!c) return LPT_E_ARG;
    const size_t need = state_size(c);
    if (size) *size = need;
    if (!blob) return LPT_OK;
    if (cap < need) return fail(c, LPT_E_ARG, "state buffer too small");
    if (c->sp.empty()) return fail(c, LPT_E_STATE, "no species");
    HIP_TRY(c, hipSetDevice(c->device));
    const int o = c->cur;
    char *out = static_cast<char *>(blob);
    StateHeader h{};
    std::memcpy(h.magic, kStateMagic, 8);
    h.version = 2;   // 2: FP32-split state as unwrapped cells + offsets
    h.n = c->n;
    h.precision = c->precision;
    h.nspecies = (int32_t)c->sp.size();
    h.np = c->np;
    h.steps = c->steps;
    h.nrec = c->nrec;
    h.t = c->t;
    h.time_mode = c->time_mode;
    h.has_vel = c->has_inertial ? 1 : 0;
    h.sorted_once = c->sorted_once ? 1 : 0;
    HIP_TRY(c, hipMemcpyAsync(&h.clock, c->clock, sizeof(DevClock), hipMemcpyDeviceToHost,
                              c->stream));
    size_t off = sizeof(StateHeader);
    for (const SpeciesHost &sh : c->sp) {
        StateSpecies ss{sh.kind, sh.scheme, sh.st, sh.count, sh.vel_from_field ? 1 : 0, 0};
        std::memcpy(out + off, &ss, sizeof ss);
        off += sizeof ss;
    }
    const std::vector<size_t> sizes = state_arrays(c);
    const std::vector<void *> src = state_ptrs(c, o);
    for (size_t a = 0; a < sizes.size(); ++a) {
        HIP_TRY(c, hipMemcpyAsync(out + off, src[a], sizes[a], hipMemcpyDeviceToHost, c->stream));
        off += sizes[a];
    }
    const size_t rb = (size_t)c->nrec * 8 * sizeof(double);
    for (size_t sidx = 0; sidx < c->sp.size(); ++sidx) {
        if (rb)
            HIP_TRY(c, hipMemcpyAsync(out + off, c->records + sidx * c->rec_cap * 8, rb,
                                      hipMemcpyDeviceToHost, c->stream));
        off += rb;
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    std::memcpy(out, &h, sizeof h);
    return LPT_OK;
}

lpt_status lpt_set_state(lpt_ctx *c, const void *blob, size_t size)
{
    if (!c) return LPT_E_ARG;
    if (!blob || size < sizeof(StateHeader)) return fail(c, LPT_E_ARG, "state blob too small");
    const char *in = static_cast<const char *>(blob);
    StateHeader h;
    std::memcpy(&h, in, sizeof h);
    if (std::memcmp(h.magic, kStateMagic, 8) != 0 || h.version != 2)
        return fail(c, LPT_E_ARG, "not an lpt state blob");
    if (h.n != c->n || h.precision != c->precision || h.nspecies != (int32_t)c->sp.size() ||
        h.np != c->np || h.has_vel != (c->has_inertial ? 1 : 0))
        return fail(c, LPT_E_ARG, "state blob does not match this context (grid, precision or "
                                  "species)");
    size_t off = sizeof(StateHeader);
    if (size < off + c->sp.size() * sizeof(StateSpecies))
        return fail(c, LPT_E_ARG, "state blob truncated");
    for (const SpeciesHost &sh : c->sp) {
        StateSpecies ss;
        std::memcpy(&ss, in + off, sizeof ss);
        off += sizeof ss;
        if (ss.kind != sh.kind || ss.scheme != sh.scheme || ss.st != sh.st || ss.count != sh.count)
            return fail(c, LPT_E_ARG, "state blob species differ from this context's");
    }
    if (h.nrec < 0 || h.steps < 0) return fail(c, LPT_E_ARG, "corrupt state blob");
    const size_t need = sizeof(StateHeader) + c->sp.size() * sizeof(StateSpecies) +
                        [&] {
                            size_t b = 0;
                            for (size_t x : state_arrays(c)) b += x;
                            return b;
                        }() +
                        c->sp.size() * (size_t)h.nrec * 8 * sizeof(double);
    if (size < need) return fail(c, LPT_E_ARG, "state blob truncated");
    HIP_TRY(c, hipSetDevice(c->device));
    // statistics capacity first (the only step that may fail for lack of memory)
    if (h.nrec > c->rec_cap) {
        const int64_t ns = (int64_t)c->sp.size();
        double *nr = nullptr;
        if (dalloc(nr, (size_t)(ns * (h.nrec + 64) * 8)) != hipSuccess) {
            (void)hipGetLastError();
            return fail(c, LPT_E_NOMEM, "statistics records allocation failed");
        }
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        dfree(c->records);
        c->records = nr;
        c->rec_cap = h.nrec + 64;
    }
    const std::vector<size_t> sizes = state_arrays(c);
    const std::vector<void *> dst = state_ptrs(c, c->cur);
    // the blob's initial positions replace the species' own: record steps
    // read them from now on instead of drawing them again
    for (SpeciesHost &sh : c->sp) sh.x0_drawn = false;
    for (size_t a = 0; a < sizes.size(); ++a) {
        HIP_TRY(c, hipMemcpyAsync(dst[a], in + off, sizes[a], hipMemcpyHostToDevice, c->stream));
        off += sizes[a];
    }
    const size_t rb = (size_t)h.nrec * 8 * sizeof(double);
    for (size_t sidx = 0; sidx < c->sp.size(); ++sidx) {
        if (rb)
            HIP_TRY(c, hipMemcpyAsync(c->records + sidx * c->rec_cap * 8, in + off, rb,
                                      hipMemcpyHostToDevice, c->stream));
        off += rb;
    }
    HIP_TRY(c, hipMemcpyAsync(c->clock, &h.clock, sizeof(DevClock), hipMemcpyHostToDevice,
                              c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->steps = h.steps;
    c->t = h.t;
    c->nrec = h.nrec;
    c->time_mode = h.time_mode;
    c->sorted_once = h.sorted_once != 0;
    c->ck_valid = false;
    invalidate_graphs(c);
    return LPT_OK;
}

lpt_status lpt_get_tuning(lpt_ctx *c, lpt_tuning *out)
{
    if (!c) return LPT_E_ARG;
    if (!out) return fail(c, LPT_E_ARG, "out must not be NULL");
    out->block_size = c->block;
    out->tile_records = c->tile_auto ? 0 : (c->tile_cap > 0 ? c->tile_cap : -1);
    out->sort_interval = c->sort_interval;
    out->persistent = c->persistent;
    out->graph_chunk = c->graph_chunk;
    out->halo_scale = c->halo_scale;
    out->max_workgroups = c->max_wg;
    out->fused = c->fused;
    out->sort_cells = c->sort_cells;
    out->rows = c->rows;
    return LPT_OK;
}

lpt_status lpt_set_tuning(lpt_ctx *c, const lpt_tuning *t)
{
    if (!c) return LPT_E_ARG;
    if (!t) return fail(c, LPT_E_ARG, "tuning must not be NULL");
    const int32_t block = t->block_size == 0 ? 256 : t->block_size;
    if (block != 64 && block != 128 && block != 256 && block != 512)
        return fail(c, LPT_E_ARG, "block_size must be 64, 128, 256 or 512");
    const size_t rec_size = c->precision == LPT_FP64 ? sizeof(Rec64) : sizeof(float4);
    int32_t tile = t->tile_records;
    const int32_t tile_auto = tile == 0;
    if (tile == 0) tile = kTileRecordsDefault;
    else if (tile == -1) tile = 0;
    else if (tile < 16 || (size_t)tile > kTileBytesMax / rec_size)
        return fail(c, LPT_E_ARG, "tile_records out of range");
    if (t->sort_interval < 0) return fail(c, LPT_E_ARG, "sort_interval must be >= 0");
    if (t->persistent != 0 && t->persistent != 1) return fail(c, LPT_E_ARG, "persistent is 0 or 1");
    if (t->graph_chunk < 0) return fail(c, LPT_E_ARG, "graph_chunk must be >= 0");
    const float halo = t->halo_scale == 0.0f ? kHaloScaleDefault : t->halo_scale;
    if (!(halo > 0.0f && halo <= 4.0f)) return fail(c, LPT_E_ARG, "halo_scale must be in (0, 4]");
    if (t->max_workgroups < 0) return fail(c, LPT_E_ARG, "max_workgroups must be >= 0");
    if (t->fused < 0 || t->fused > 2) return fail(c, LPT_E_ARG, "fused is 0, 1 or 2");
    if (t->sort_cells < 0 || t->sort_cells > 2) return fail(c, LPT_E_ARG, "sort_cells is 0, 1 or 2");
    const int32_t rows = t->rows == 0 ? 1 : t->rows;
    if (rows != 1 && rows != 2) return fail(c, LPT_E_ARG, "rows is 1 or 2");
    if (block / rows < 64) return fail(c, LPT_E_ARG, "block_size / rows must be at least 64");
    if (key_width(c->n, c->sort_tile, t->sort_cells == 1, (int)c->sp.size()) > 32)
        return fail(c, LPT_E_ARG, "sort key wider than 32 bits with sort_cells; raise sort_tile");
    HIP_TRY(c, hipSetDevice(c->device));
    const bool block_changed = block != c->block;
    if (block_changed) {
        // the statistics partials hold one slot per wave of every logical block
        const int32_t old = c->block;
        c->block = block;
        const StepParams P = make_params(c);
        const int64_t need = stat_partials_doubles(P, block);
        if (need > c->partial_cap) {
            double *np = nullptr;
            if (dalloc(np, (size_t)need) != hipSuccess) {
                c->block = old;
                (void)hipGetLastError();
                return fail(c, LPT_E_NOMEM, "statistics partials allocation failed");
            }
            HIP_TRY(c, hipStreamSynchronize(c->stream));
            dfree(c->partials);
            c->partials = np;
            c->partial_cap = need;
        }
    }
    c->tile_cap = tile;
    c->tile_auto = tile_auto;
    c->sort_interval = t->sort_interval;
    c->persistent = t->persistent;
    c->graph_chunk = t->graph_chunk;
    c->halo_scale = halo;
    c->max_wg = t->max_workgroups;
    if (t->fused != c->fused || block_changed) c->order_ok = false;
    c->fused = t->fused;
    c->sort_cells = t->sort_cells;
    c->rows = rows;
    invalidate_graphs(c);
    return LPT_OK;
}

lpt_status lpt_bw_probe(lpt_ctx *c, int64_t bytes, int32_t iters, double *copy_gbps,
                        double *triad_gbps)
{
    if (!c) return LPT_E_ARG;
    bytes &= ~(int64_t)15;
    if (bytes <= 0 || iters < 1) return fail(c, LPT_E_ARG, "bytes and iters must be positive");
    HIP_TRY(c, hipSetDevice(c->device));
    void *a = nullptr, *b = nullptr, *d = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMalloc(&a, bytes);
    if (e == hipSuccess) e = hipMalloc(&b, bytes);
    if (e == hipSuccess) e = hipMalloc(&d, bytes);
    if (e == hipSuccess) e = hipMemsetAsync(a, 0, bytes, c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(b, 0, bytes, c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(d, 0, bytes, c->stream);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    float ms = 0.f;
    // copy: one warm-up pass, then iters timed passes
    if (e == hipSuccess) e = launch_copy(a, b, bytes, c->stream);
    if (e == hipSuccess) e = hipEventRecord(e0, c->stream);
    for (int32_t k = 0; k < iters && e == hipSuccess; ++k) e = launch_copy(a, b, bytes, c->stream);
    if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e == hipSuccess && copy_gbps) *copy_gbps = 2.0 * bytes * iters / (ms * 1e-3) / 1e9;
    if (e == hipSuccess) e = launch_triad(a, b, d, bytes, c->stream);
    if (e == hipSuccess) e = hipEventRecord(e0, c->stream);
    for (int32_t k = 0; k < iters && e == hipSuccess; ++k) e = launch_triad(a, b, d, bytes, c->stream);
    if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e == hipSuccess && triad_gbps) *triad_gbps = 3.0 * bytes * iters / (ms * 1e-3) / 1e9;
    (void)hipStreamSynchronize(c->stream);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (a) (void)hipFree(a);
    if (b) (void)hipFree(b);
    if (d) (void)hipFree(d);
    HIP_TRY(c, e);
    return LPT_OK;
}

}  // extern "C"
