// lbm_batch.hip -- batched plates: arena, tables, graphs (include/lbm_solid.h).
//
// A batch holds up to max_plates plates of any sizes in one device arena
// carved from the caller's workspace. Plates are admitted while the arena
// (first fit) and the tile table have room, advance together through one
// persistent launch per time step, and are retired when done. lbm_batch_step
// enqueues a chunk of K steps as a HIP graph of K launches (captured once per
// K); the plate and tile tables are rewritten between chunks from pinned
// host buffers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <new>
#include <queue>
#include <string>
#include <vector>

#include "batch_kernel.hpp"
#include "host_common.hpp"

using namespace lbm;

namespace {

constexpr int kBatchBlock = 256;
constexpr int kSegRowsMin = 4;  // shortest segment when few plates run
// The planner tries segment heights from kSegRowsMin up to twice this (the
// two-step halo is twice as deep).
constexpr int seg_rows_max(int spl) { return spl == 2 ? 128 : 64; }

struct Slot {
    bool live = false;
    int nx = 0, ny = 0;
    Units U{};
    double tau = 1.0;
    double body[2] = {0, 0};
    int bc_lo = 0, bc_hi = 0;
    double val_lo[2] = {0, 0}, val_hi[2] = {0, 0};
    size_t arena_off = 0;
    StateLayout L{};
    Shape shape{};
    int parity = 0;
    int64_t done = 0, target = 0;
    double f_scale = 1.0;
    int sr = 0;
    unsigned long long seed = 0;
};

struct BatchLayout {
    size_t plates, tiles, ntiles, flags, staging, staging_bytes, partials, diag, arena, total;
};

BatchLayout batch_layout(int max_plates, int max_tiles, size_t arena_bytes)
{
    BatchLayout B{};
    size_t off = 0;
    B.plates = off;
    off = align_up(off + (size_t)max_plates * sizeof(PlateDesc));
    B.tiles = off;
    off = align_up(off + (size_t)max_tiles * sizeof(TileDesc));
    B.ntiles = off;
    off = align_up(off + sizeof(int));
    B.flags = off;
    off = align_up(off + (size_t)max_plates * sizeof(unsigned));
    B.staging = off;
    B.staging_bytes = kStagingCap;
    off = align_up(off + B.staging_bytes);
    B.partials = off;
    off = align_up(off + kMaxDiagBlocks * 8 * sizeof(double));
    B.diag = off;
    off = align_up(off + 64 * sizeof(double));
    B.arena = off;
    off = align_up(off + arena_bytes);
    B.total = off;
    return B;
}

Shape batch_shape(int nx, int ny, lbm_precision p, lbm_scheme s, int seg_rows, int spl)
{
    return make_shape(nx, ny, p, s, kBatchBlock, std::max(1, (ny + seg_rows / 2) / seg_rows), spl);
}

// Tile-table entries a plate may need (at the shortest segments, either
// number of steps per launch).
int max_plate_tiles(int nx, int ny, lbm_precision p, lbm_scheme s)
{
    int n = 0;
    for (int spl = 1; spl <= max_steps_per_launch(p, s); ++spl) {
        const Shape sh = batch_shape(nx, ny, p, s, kSegRowsMin, spl);
        n = std::max(n, sh.n_strips * sh.n_segs);
    }
    return n;
}

}  // namespace

struct lbm_batch {
    int max_plates = 0, max_tiles = 0;
    lbm_precision prec = LBM_FP16_STORE;
    lbm_scheme scheme = LBM_SCHEME_PC;
    bool walled = false;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    hipStream_t stream = nullptr;
    hipStream_t capture = nullptr;  // own stream for graph capture (the caller's may be the null stream)
    BatchLayout B{};
    size_t arena_bytes = 0;
    std::map<size_t, size_t> free_list;  // offset -> bytes
    std::vector<Slot> slots;
    PlateDesc *h_plates[2] = {nullptr, nullptr};
    TileDesc *h_tiles[2] = {nullptr, nullptr};
    int *h_ntiles[2] = {nullptr, nullptr};
    hipEvent_t ev[2] = {nullptr, nullptr};
    bool ev_used[2] = {false, false};
    int buf = 0;
    std::vector<int> running;  // slots in the uploaded tile table
    bool tables_valid = false;
    std::map<long long, hipGraphExec_t> graphs;  // key: chunk steps * 2 + (steps per launch - 1)
    int spl = 1;              // time steps per launch
    int grid_for[3] = {0, 0, 0};  // persistent grid of the one- and two-step kernels
    int grid = 0;
    int tiles_used = 0;
    std::string err;

    PlateDesc *d_plates() const { return reinterpret_cast<PlateDesc *>(ws + B.plates); }
    TileDesc *d_tiles() const { return reinterpret_cast<TileDesc *>(ws + B.tiles); }
    int *d_ntiles() const { return reinterpret_cast<int *>(ws + B.ntiles); }
    unsigned *d_flags() const { return reinterpret_cast<unsigned *>(ws + B.flags); }
    char *arena() const { return ws + B.arena; }

    PlateIO io(int s) const
    {
        const Slot &sl = slots[s];
        PlateIO p{};
        p.nx = sl.nx;
        p.ny = sl.ny;
        p.prec = prec;
        p.U = sl.U;
        p.bc_lo = sl.bc_lo;
        p.bc_hi = sl.bc_hi;
        for (int a = 0; a < 2; ++a) {
            p.val_lo[a] = sl.val_lo[a];
            p.val_hi[a] = sl.val_hi[a];
        }
        char *base = arena() + sl.arena_off;
        p.f = base + sl.L.f[sl.parity];
        p.u = base + sl.L.u[sl.parity];
        p.j = base + sl.L.j[sl.parity];
        p.f_other = base + sl.L.f[sl.parity ^ 1];
        p.f_scale = sl.f_scale;
        p.staging = reinterpret_cast<double *>(ws + B.staging);
        p.staging_bytes = B.staging_bytes;
        p.partials = reinterpret_cast<double *>(ws + B.partials);
        p.diag_out = reinterpret_cast<double *>(ws + B.diag);
        p.stream = stream;
        return p;
    }
};

namespace {

thread_local std::string g_batch_create_error;

lbm_status bfail(lbm_batch *b, lbm_status s, const std::string &msg)
{
    if (b)
        b->err = msg;
    else
        g_batch_create_error = msg;
    return s;
}

lbm_status bhip(lbm_batch *b, hipError_t e, const char *what)
{
    return bfail(b, LBM_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define BHIP_TRY(b, call)                                 \
    do {                                                  \
        hipError_t e_ = (call);                           \
        if (e_ != hipSuccess) return bhip(b, e_, #call);  \
    } while (0)

// first fit in the arena, 256-byte granules
bool arena_alloc(lbm_batch *b, size_t bytes, size_t *off)
{
    bytes = align_up(bytes);
    for (auto it = b->free_list.begin(); it != b->free_list.end(); ++it) {
        if (it->second >= bytes) {
            *off = it->first;
            const size_t rest = it->second - bytes, roff = it->first + bytes;
            b->free_list.erase(it);
            if (rest) b->free_list[roff] = rest;
            return true;
        }
    }
    return false;
}

void arena_free(lbm_batch *b, size_t off, size_t bytes)
{
    bytes = align_up(bytes);
    auto it = b->free_list.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != b->free_list.end() && it->first + it->second == nx->first) {
        it->second += nx->second;
        b->free_list.erase(nx);
    }
    if (it != b->free_list.begin()) {
        auto pv = std::prev(it);
        if (pv->first + pv->second == it->first) {
            pv->second += it->second;
            b->free_list.erase(it);
        }
    }
}

template <class PR, bool PC, bool W>
const void *batch_kernel_ptr(int spl)
{
    // (deviation storage has no two-step kernel)
    if constexpr (PC && !FStore<typename PR::TF>::kDeviation) {
        if (spl == 2) return reinterpret_cast<const void *>(&batch_step2_kernel<PR, kBatchBlock, W>);
    }
    return reinterpret_cast<const void *>(&batch_step_kernel<PR, kBatchBlock, PC, W>);
}

template <class PR>
const void *batch_kernel_for(bool pc, bool walled, int spl)
{
    if (pc) return walled ? batch_kernel_ptr<PR, true, true>(spl) : batch_kernel_ptr<PR, true, false>(spl);
    return walled ? batch_kernel_ptr<PR, false, true>(spl) : batch_kernel_ptr<PR, false, false>(spl);
}

const void *batch_kernel(lbm_precision p, bool pc, bool walled, int spl)
{
    switch (p) {
    case LBM_FP64: return batch_kernel_for<PrecF64>(pc, walled, spl);
    case LBM_FP32: return batch_kernel_for<PrecF32>(pc, walled, spl);
    case LBM_FP16_STORE: return batch_kernel_for<PrecF16>(pc, walled, spl);
    case LBM_FP32_U64: return batch_kernel_for<PrecF32U64>(pc, walled, spl);
    default: return batch_kernel_for<PrecBF16>(pc, walled, spl);
    }
}

PlateDesc describe(const lbm_batch *b, int s, int nsteps)
{
    const Slot &sl = b->slots[s];
    PlateDesc d{};
    char *base = b->arena() + sl.arena_off;
    for (int c = 0; c < 2; ++c) {
        d.f[c] = base + sl.L.f[c];
        d.u[c] = base + sl.L.u[c];
        d.j[c] = base + sl.L.j[c];
    }
    d.nx = sl.nx;
    d.ny = sl.ny;
    d.plane = (long long)sl.nx * sl.ny;
    StepParams sp{};
    fill_physics(sp, sl.U, sl.tau, sl.body, sl.bc_lo, sl.val_lo, sl.bc_hi, sl.val_hi);
    d.omega = sp.omega;
    d.lam = sp.lam;
    d.mu = sp.mu;
    d.bx = sp.bx;
    d.by = sp.by;
    d.bc_lo = sp.bc_lo;
    d.bc_hi = sp.bc_hi;
    for (int a = 0; a < 2; ++a) {
        d.val_lo[a] = sp.val_lo[a];
        d.val_hi[a] = sp.val_hi[a];
    }
    d.f_scale = sl.f_scale;
    d.f_inv_scale = 1.0 / sl.f_scale;
    d.strip_w = sl.shape.strip_w;
    d.n_strips = sl.shape.n_strips;
    d.n_segs = sl.shape.n_segs;
    d.halo_a = sl.shape.halo_a;
    d.step0 = sl.done;
    d.parity0 = sl.parity;
    d.nsteps = nsteps;
    d.flag = b->d_flags() + s;
    d.sr = sl.sr;
    d.seed = sl.seed;
    return d;
}

// Graph of the launches that advance a chunk of K steps: K one-step
// launches, or (K + 1) / 2 two-step launches.
hipError_t get_graph(lbm_batch *b, int K, hipGraphExec_t *out)
{
    const long long key = 2LL * K + (b->spl - 1);
    auto it = b->graphs.find(key);
    if (it != b->graphs.end()) {
        *out = it->second;
        return hipSuccess;
    }
    const void *fn = batch_kernel(b->prec, b->scheme == LBM_SCHEME_PC, b->walled, b->spl);
    const int launches = b->spl == 2 ? (K + 1) / 2 : K;
    // captured on the batch's own stream, launched on the caller's
    hipError_t e = hipStreamBeginCapture(b->capture, hipStreamCaptureModeRelaxed);
    if (e) return e;
    const PlateDesc *plates = b->d_plates();
    const TileDesc *tiles = b->d_tiles();
    const int *nt = b->d_ntiles();
    for (int k = 0; k < launches && e == hipSuccess; ++k) {
        void *args[] = {(void *)&plates, (void *)&tiles, (void *)&nt, (void *)&k};
        e = hipLaunchKernel(fn, dim3(b->grid), dim3(kBatchBlock), args, 0, b->capture);
    }
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(b->capture, &g);
    if (e) {
        if (g) (void)hipGraphDestroy(g);
        return e;
    }
    if (e2) return e2;
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e) return e;
    b->graphs[key] = ex;
    *out = ex;
    return hipSuccess;
}

}  // namespace

extern "C" {

size_t lbm_batch_plate_bytes(int nx, int ny, lbm_precision p)
{
    if (nx < 5 || ny < 5 || !valid_precision(p)) return 0;
    return state_layout(nx, ny, p).bytes;
}

int lbm_batch_plate_tiles(int nx, int ny, lbm_precision p, lbm_scheme s)
{
    if (nx < 5 || ny < 5 || !valid_precision(p)) return 0;
    return max_plate_tiles(nx, ny, p, s);
}

size_t lbm_batch_workspace_bytes(int max_plates, int max_tiles, size_t arena_bytes)
{
    if (max_plates < 1 || max_tiles < 1) return 0;
    return batch_layout(max_plates, max_tiles, arena_bytes).total;
}

lbm_status lbm_batch_create(int max_plates, int max_tiles, lbm_precision p, lbm_scheme s, int walled,
                            void *dev_workspace, size_t ws_bytes, void *hip_stream, lbm_batch **out)
{
    if (!out) return bfail(nullptr, LBM_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (max_plates < 1 || max_tiles < 1) return bfail(nullptr, LBM_ERR_ARG, "max_plates and max_tiles must be >= 1");
    if (!valid_precision(p)) return bfail(nullptr, LBM_ERR_ARG, "unknown precision");
    if (s != LBM_SCHEME_PC && s != LBM_SCHEME_EXPLICIT) return bfail(nullptr, LBM_ERR_ARG, "unknown scheme");
    if (!dev_workspace || reinterpret_cast<uintptr_t>(dev_workspace) % kAlign)
        return bfail(nullptr, LBM_ERR_ARG, "workspace NULL or not 256-byte aligned");
    const BatchLayout B0 = batch_layout(max_plates, max_tiles, 0);
    if (ws_bytes < B0.total + kAlign) return bfail(nullptr, LBM_ERR_NOMEM, "workspace leaves no arena");
    lbm_batch *b = new (std::nothrow) lbm_batch();
    if (!b) return bfail(nullptr, LBM_ERR_NOMEM, "host allocation failed");
    b->max_plates = max_plates;
    b->max_tiles = max_tiles;
    b->prec = p;
    b->scheme = s;
    b->walled = walled != 0;
    b->ws = static_cast<char *>(dev_workspace);
    b->ws_bytes = ws_bytes;
    b->stream = static_cast<hipStream_t>(hip_stream);
    b->arena_bytes = (ws_bytes - B0.total) / kAlign * kAlign;
    b->B = batch_layout(max_plates, max_tiles, b->arena_bytes);
    b->free_list[0] = b->arena_bytes;
    b->slots.resize(max_plates);
    hipError_t e = hipSuccess;
    for (int i = 0; i < 2 && e == hipSuccess; ++i) {
        e = hipHostMalloc((void **)&b->h_plates[i], sizeof(PlateDesc) * max_plates, hipHostMallocDefault);
        if (!e) e = hipHostMalloc((void **)&b->h_tiles[i], sizeof(TileDesc) * max_tiles, hipHostMallocDefault);
        if (!e) e = hipHostMalloc((void **)&b->h_ntiles[i], sizeof(int), hipHostMallocDefault);
        if (!e) e = hipEventCreateWithFlags(&b->ev[i], hipEventDisableTiming);
    }
    if (!e) e = hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking);
    int dev = 0, cus = 0;
    if (!e) e = hipGetDevice(&dev);
    if (!e) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    int per_cu[3] = {0, 0, 0};
    for (int k = 1; k <= max_steps_per_launch(p, s) && !e; ++k) {
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu[k], batch_kernel(p, s == LBM_SCHEME_PC, b->walled, k),
                                                         kBatchBlock, 0);
        b->grid_for[k] = std::max(1, cus * std::max(1, per_cu[k]));
    }
    if (e) {
        lbm_batch_destroy(b);
        return bfail(nullptr, LBM_ERR_HIP, std::string("batch set-up: ") + hipGetErrorString(e));
    }
    // Two steps per launch by default with the predictor-corrector when the
    // two-step kernel keeps at least two waves per SIMD (two 256-thread blocks
    // per CU); with fewer it cannot hide its latency and one step is faster
    // (FP16 storage: 23.0k against 33.9k MLUPS on 256 uneven plates). FP64
    // moves 208 B per update, so halving the passes wins even at one wave
    // per SIMD (22.7k against 17.1k MLUPS on the same plates).
    b->spl = (max_steps_per_launch(p, s) == 2 && (per_cu[2] >= 2 || p == LBM_FP64)) ? 2 : 1;
    b->grid = b->grid_for[b->spl];
    // zero the plate flags and the tile count
    e = hipMemsetAsync(b->d_flags(), 0, sizeof(unsigned) * max_plates, b->stream);
    if (!e) e = hipMemsetAsync(b->d_ntiles(), 0, sizeof(int), b->stream);
    if (!e) e = hipStreamSynchronize(b->stream);
    if (e) {
        lbm_batch_destroy(b);
        return bfail(nullptr, LBM_ERR_HIP, std::string("batch set-up: ") + hipGetErrorString(e));
    }
    *out = b;
    return LBM_OK;
}

lbm_status lbm_batch_add(lbm_batch *b, const lbm_plate_desc *d, const double *u0, const double *v0, int64_t nsteps,
                         int *slot)
{
    if (!b) return LBM_ERR_ARG;
    if (!d || !u0 || !v0 || !slot) return bfail(b, LBM_ERR_ARG, "NULL argument");
    if (d->nx < 5 || d->ny < 5) return bfail(b, LBM_ERR_ARG, "nx and ny must be >= 5");
    if ((long long)d->nx * d->ny > (1LL << 29)) return bfail(b, LBM_ERR_UNSUPPORTED, "more than 2^29 sites");
    if (!(d->dx > 0) || !(d->rho0 > 0) || !(d->mu > 0) || !(d->lambda + d->mu > 0) || !(d->tau_over_dt > 0.5))
        return bfail(b, LBM_ERR_ARG, "invalid spacing or material");
    if (nsteps < 0) return bfail(b, LBM_ERR_ARG, "nsteps < 0");
    const bool pw = d->bc_ymin != LBM_BC_PERIODIC;
    if ((d->bc_ymin == LBM_BC_PERIODIC) != (d->bc_ymax == LBM_BC_PERIODIC))
        return bfail(b, LBM_ERR_ARG, "periodic y edges come in pairs");
    if (d->bc_ymin < LBM_BC_PERIODIC || d->bc_ymin > LBM_BC_NEUMANN_T || d->bc_ymax < LBM_BC_PERIODIC ||
        d->bc_ymax > LBM_BC_NEUMANN_T)
        return bfail(b, LBM_ERR_ARG, "unknown boundary rule");
    if (pw != b->walled) return bfail(b, LBM_ERR_UNSUPPORTED, "plate edges do not match the batch (walled or periodic)");
    if (d->rounding != LBM_ROUND_NEAREST && d->rounding != LBM_ROUND_STOCHASTIC)
        return bfail(b, LBM_ERR_ARG, "unknown rounding");
    if (d->rounding == LBM_ROUND_STOCHASTIC && b->prec != LBM_FP16_STORE && b->prec != LBM_BF16_STORE)
        return bfail(b, LBM_ERR_UNSUPPORTED, "stochastic rounding needs 16-bit population storage");
    int s = -1;
    for (int i = 0; i < b->max_plates; ++i)
        if (!b->slots[i].live) {
            s = i;
            break;
        }
    if (s < 0) return bfail(b, LBM_ERR_NOMEM, "no free plate slot");
    const Shape sh = batch_shape(d->nx, d->ny, b->prec, b->scheme, seg_rows_max(b->spl), b->spl);
    const int tmax = max_plate_tiles(d->nx, d->ny, b->prec, b->scheme);
    if (b->tiles_used + tmax > b->max_tiles) return bfail(b, LBM_ERR_NOMEM, "tile table full");
    const StateLayout L = state_layout(d->nx, d->ny, b->prec);
    size_t off = 0;
    if (!arena_alloc(b, L.bytes, &off)) return bfail(b, LBM_ERR_NOMEM, "arena full");
    Slot &sl = b->slots[s];
    sl = Slot{};
    sl.nx = d->nx;
    sl.ny = d->ny;
    sl.U = Units{d->dx, d->rho0, d->lambda, d->mu};
    sl.tau = d->tau_over_dt;
    sl.sr = d->rounding == LBM_ROUND_STOCHASTIC;
    sl.seed = d->seed;
    sl.body[0] = d->body[0];
    sl.body[1] = d->body[1];
    sl.bc_lo = d->bc_ymin;
    sl.bc_hi = d->bc_ymax;
    for (int a = 0; a < 2; ++a) {
        sl.val_lo[a] = d->val_ymin[a];
        sl.val_hi[a] = d->val_ymax[a];
    }
    sl.arena_off = off;
    sl.L = L;
    sl.shape = sh;
    sl.parity = 0;
    sl.done = 0;
    sl.target = nsteps;
    double scale = 1.0;
    bool nonfinite = false;
    hipError_t e = hipMemsetAsync(b->d_flags() + s, 0, sizeof(unsigned), b->stream);
    if (!e) {
        const int bc4[4] = {LBM_BC_PERIODIC, LBM_BC_PERIODIC, sl.bc_lo, sl.bc_hi};
        const double val4[4][2] = {{0, 0}, {0, 0}, {sl.val_lo[0], sl.val_lo[1]}, {sl.val_hi[0], sl.val_hi[1]}};
        e = plate_start(b->io(s), u0, v0, load_population_bound(sl.U, sl.nx, sl.ny, bc4, val4, sl.body), &scale,
                        &nonfinite);
    }
    if (e || nonfinite) {
        arena_free(b, off, L.bytes);
        if (e) return bhip(b, e, "start-up");
        return bfail(b, LBM_ERR_ARG, "initial fields not finite");
    }
    sl.f_scale = scale;
    sl.live = true;
    b->tiles_used += tmax;
    b->tables_valid = false;
    *slot = s;
    return LBM_OK;
}

lbm_status lbm_batch_step(lbm_batch *b, int64_t nsteps)
{
    if (!b) return LBM_ERR_ARG;
    if (nsteps < 0) return bfail(b, LBM_ERR_ARG, "nsteps < 0");
    int64_t kmax = 0;
    std::vector<int> run;
    for (int i = 0; i < b->max_plates; ++i) {
        const Slot &sl = b->slots[i];
        if (sl.live && sl.target > sl.done) {
            run.push_back(i);
            kmax = std::max(kmax, sl.target - sl.done);
        }
    }
    const int64_t K64 = std::min<int64_t>(nsteps, kmax);
    if (K64 <= 0) return LBM_OK;
    if (K64 > (1 << 20)) return bfail(b, LBM_ERR_ARG, "chunk too long (at most 2^20 steps per call)");
    const int K = (int)K64;
    // rewrite the tables in the pinned buffer not read by an earlier copy still in flight
    const int w = b->buf;
    if (b->ev_used[w]) BHIP_TRY(b, hipEventSynchronize(b->ev[w]));
    const bool tiles_changed = !b->tables_valid || run != b->running;
    std::vector<TileDesc> plan;
    if (tiles_changed) {
        // Segment height and placement for the running set. Block g of the
        // persistent grid takes entries g, g + G, g + 2G, ... of the table, and
        // a tile costs its rows plus the pipeline's fill. Each candidate height
        // (kSegRowsMin up to twice seg_rows_max) splits the strips into
        // tiles, which are packed longest first onto the least loaded block;
        // the height whose busiest block has the least work is kept (the
        // larger one on a tie: fewer halo rows). Short segments win when few
        // plates run, long ones when many do.
        const int G = b->grid;
        const int fill = (b->scheme == LBM_SCHEME_PC ? 11 : 7) * b->spl;
        long long best = -1;
        int best_rows = kSegRowsMin;
        for (int rows = kSegRowsMin; rows <= 2 * seg_rows_max(b->spl); rows *= 2) {
            std::vector<long long> cost;
            for (int i : run) {
                const Shape sh = batch_shape(b->slots[i].nx, b->slots[i].ny, b->prec, b->scheme, rows, b->spl);
                const int ny = b->slots[i].ny;
                for (int st = 0; st < sh.n_strips; ++st)
                    for (int sg = 0; sg < sh.n_segs; ++sg)
                        cost.push_back((long long)(sg + 1) * ny / sh.n_segs - (long long)sg * ny / sh.n_segs + fill);
            }
            std::sort(cost.begin(), cost.end(), std::greater<long long>());
            std::priority_queue<long long, std::vector<long long>, std::greater<long long>> load;
            for (int g = 0; g < G; ++g) load.push(0);
            long long top = 0;
            for (long long c : cost) {
                const long long l = load.top() + c;
                load.pop();
                load.push(l);
                top = std::max(top, l);
            }
            if (best < 0 || top <= best) {
                best = top;
                best_rows = rows;
            }
        }
        for (int i : run)
            b->slots[i].shape = batch_shape(b->slots[i].nx, b->slots[i].ny, b->prec, b->scheme, best_rows, b->spl);
        // Pack the chosen tiles: longest first, onto the least loaded block.
        // A plate's tiles are listed segment by segment and equally loaded
        // blocks are taken XCD by XCD (blocks are dealt round-robin to the 8
        // XCDs), so horizontal neighbours tend to run at the same time on
        // one XCD and share their halo columns in its L2.
        std::vector<std::pair<int, TileDesc>> tl;
        for (int i : run) {
            const Shape &sh = b->slots[i].shape;
            const int ny = b->slots[i].ny;
            for (int sg = 0; sg < sh.n_segs; ++sg)
                for (int st = 0; st < sh.n_strips; ++st)
                    tl.push_back({(int)((long long)(sg + 1) * ny / sh.n_segs - (long long)sg * ny / sh.n_segs),
                                  TileDesc{i, st, sg, 0}});
        }
        std::stable_sort(tl.begin(), tl.end(), [](const auto &a, const auto &c) { return a.first > c.first; });
        std::vector<std::vector<int>> bins(G);  // tiles of each block of the persistent grid
        const int per_xcd = (G + 7) / 8;
        auto rank = [&](int g) { return (g & 7) * per_xcd + (g >> 3); };  // XCD-major order of block g
        std::priority_queue<std::pair<long long, int>, std::vector<std::pair<long long, int>>,
                            std::greater<std::pair<long long, int>>>
            load;  // (work, rank)
        std::vector<int> block_of(8 * per_xcd, -1);
        for (int g = 0; g < G; ++g) {
            block_of[rank(g)] = g;
            load.push({0, rank(g)});
        }
        for (int t = 0; t < (int)tl.size(); ++t) {
            auto [l, r] = load.top();
            load.pop();
            bins[block_of[r]].push_back(t);
            load.push({l + tl[t].first + fill, r});
        }
        size_t depth = 0;
        for (const auto &bn : bins) depth = std::max(depth, bn.size());
        if (depth * (size_t)G <= (size_t)b->max_tiles) {
            // block g's k-th tile at entry g + kG; empty entries elsewhere
            plan.assign(depth * (size_t)G, TileDesc{-1, 0, 0, 0});
            for (int g = 0; g < G; ++g)
                for (size_t q = 0; q < bins[g].size(); ++q) plan[g + q * (size_t)G] = tl[bins[g][q]].second;
        } else {
            // the packed table would not fit: tiles in plan order, dealt by the stride
            for (const auto &e : tl) plan.push_back(e.second);
        }
    }
    int max_slot = 0;
    for (int i : run) max_slot = std::max(max_slot, i + 1);
    std::memset(b->h_plates[w], 0, sizeof(PlateDesc) * max_slot);
    for (int i : run) b->h_plates[w][i] = describe(b, i, (int)std::min<int64_t>(K, b->slots[i].target - b->slots[i].done));
    int nt = 0;
    if (tiles_changed) {
        nt = (int)plan.size();
        std::memcpy(b->h_tiles[w], plan.data(), sizeof(TileDesc) * plan.size());
        *b->h_ntiles[w] = nt;
    }
    BHIP_TRY(b, hipMemcpyAsync(b->d_plates(), b->h_plates[w], sizeof(PlateDesc) * max_slot, hipMemcpyHostToDevice,
                               b->stream));
    if (tiles_changed) {
        BHIP_TRY(b, hipMemcpyAsync(b->d_tiles(), b->h_tiles[w], sizeof(TileDesc) * nt, hipMemcpyHostToDevice,
                                   b->stream));
        BHIP_TRY(b, hipMemcpyAsync(b->d_ntiles(), b->h_ntiles[w], sizeof(int), hipMemcpyHostToDevice, b->stream));
        b->running = run;
        b->tables_valid = true;
    }
    BHIP_TRY(b, hipEventRecord(b->ev[w], b->stream));
    b->ev_used[w] = true;
    b->buf ^= 1;
    hipGraphExec_t ex = nullptr;
    BHIP_TRY(b, get_graph(b, K, &ex));
    BHIP_TRY(b, hipGraphLaunch(ex, b->stream));
    for (int i : run) {
        Slot &sl = b->slots[i];
        const int64_t n = std::min<int64_t>(K, sl.target - sl.done);
        sl.done += n;
        // each launch writes the other copy once, whatever it advanced
        sl.parity ^= (int)((b->spl == 2 ? (n + 1) / 2 : n) & 1);
    }
    return LBM_OK;
}

lbm_status lbm_batch_set_steps_per_launch(lbm_batch *b, int k)
{
    if (!b) return LBM_ERR_ARG;
    if (k != 1 && k != 2) return bfail(b, LBM_ERR_ARG, "steps per launch must be 1 or 2");
    if (k == 2 && b->scheme != LBM_SCHEME_PC)
        return bfail(b, LBM_ERR_UNSUPPORTED, "two steps per launch need the predictor-corrector scheme");
    if (k == 2 && max_steps_per_launch(b->prec, b->scheme) < 2)
        return bfail(b, LBM_ERR_UNSUPPORTED, "16-bit population storage runs one step per launch");
    if (k != b->spl) {
        // the plates' shapes carry the halo of the kernel: re-plan the tiles
        BHIP_TRY(b, hipStreamSynchronize(b->stream));
        b->spl = k;
        b->grid = b->grid_for[k];
        b->tables_valid = false;
        b->running.clear();
    }
    return LBM_OK;
}

lbm_status lbm_batch_get_steps_per_launch(const lbm_batch *b, int *k)
{
    if (!b || !k) return LBM_ERR_ARG;
    *k = b->spl;
    return LBM_OK;
}

lbm_status lbm_batch_query(lbm_batch *b, int slot, int64_t *steps_done, int64_t *steps_left, int *unstable)
{
    if (!b) return LBM_ERR_ARG;
    if (slot < 0 || slot >= b->max_plates || !b->slots[slot].live) return bfail(b, LBM_ERR_ARG, "no such plate");
    unsigned flag = 0;
    BHIP_TRY(b, hipMemcpyAsync(&flag, b->d_flags() + slot, sizeof(unsigned), hipMemcpyDeviceToHost, b->stream));
    BHIP_TRY(b, hipStreamSynchronize(b->stream));
    const Slot &sl = b->slots[slot];
    if (steps_done) *steps_done = sl.done;
    if (steps_left) *steps_left = sl.target - sl.done;
    if (unstable) *unstable = flag != 0;
    return LBM_OK;
}

lbm_status lbm_batch_read(lbm_batch *b, int slot, double *u, double *v, double *P, lbm_diagnostics *d)
{
    if (!b) return LBM_ERR_ARG;
    if (slot < 0 || slot >= b->max_plates || !b->slots[slot].live) return bfail(b, LBM_ERR_ARG, "no such plate");
    const Slot &sl = b->slots[slot];
    double out[7] = {0, 0, 0, 0, 0, 0, 0};
    const hipError_t e = plate_read(b->io(slot), (double)sl.done, u, v, P, d ? out : nullptr);
    if (e) return bhip(b, e, "read-out");
    unsigned flag = 0;
    BHIP_TRY(b, hipMemcpyAsync(&flag, b->d_flags() + slot, sizeof(unsigned), hipMemcpyDeviceToHost, b->stream));
    BHIP_TRY(b, hipStreamSynchronize(b->stream));
    if (d) {
        d->momentum[0] = out[0];
        d->momentum[1] = out[1];
        d->mass_moment = out[2];
        d->energy = out[3];
        d->min_J = out[4];
        d->max_strain = out[5];
        d->unstable = (out[6] != 0.0 || flag != 0) ? 1 : 0;
        d->reserved = 0;
        d->steps = sl.done;
    }
    if (flag) return bfail(b, LBM_ERR_UNSTABLE, "J <= 0 or a non-finite value appeared");
    return LBM_OK;
}

lbm_status lbm_batch_read_derived(lbm_batch *b, int slot, double *sigma, double *E, double *W)
{
    if (!b) return LBM_ERR_ARG;
    if (slot < 0 || slot >= b->max_plates || !b->slots[slot].live) return bfail(b, LBM_ERR_ARG, "no such plate");
    const hipError_t e = plate_read_derived(b->io(slot), (double)b->slots[slot].done, sigma, E, W);
    if (e) return bhip(b, e, "read-out");
    return LBM_OK;
}

lbm_status lbm_batch_sample(lbm_batch *b, int slot, int n, const int *x, const int *y, double *out)
{
    if (!b) return LBM_ERR_ARG;
    if (slot < 0 || slot >= b->max_plates || !b->slots[slot].live) return bfail(b, LBM_ERR_ARG, "no such plate");
    if (n < 0 || (n > 0 && (!x || !y || !out))) return bfail(b, LBM_ERR_ARG, "invalid node list");
    const Slot &sl = b->slots[slot];
    const PlateIO io = b->io(slot);
    if (n > sample_capacity(io)) return bfail(b, LBM_ERR_ARG, "too many nodes for one call");
    for (int k = 0; k < n; ++k)
        if (x[k] < 0 || x[k] >= sl.nx || y[k] < 0 || y[k] >= sl.ny) return bfail(b, LBM_ERR_ARG, "node outside the plate");
    const hipError_t e = plate_sample(io, (double)sl.done, n, x, y, out);
    if (e) return bhip(b, e, "sample");
    return LBM_OK;
}

lbm_status lbm_batch_retire(lbm_batch *b, int slot)
{
    if (!b) return LBM_ERR_ARG;
    if (slot < 0 || slot >= b->max_plates || !b->slots[slot].live) return bfail(b, LBM_ERR_ARG, "no such plate");
    // work already enqueued may still use the plate's memory
    BHIP_TRY(b, hipStreamSynchronize(b->stream));
    Slot &sl = b->slots[slot];
    arena_free(b, sl.arena_off, sl.L.bytes);
    b->tiles_used -= max_plate_tiles(sl.nx, sl.ny, b->prec, b->scheme);
    sl.live = false;
    b->tables_valid = false;
    return LBM_OK;
}

lbm_status lbm_batch_info(const lbm_batch *b, int *live_plates, size_t *arena_free, size_t *arena_largest_free)
{
    if (!b) return LBM_ERR_ARG;
    int n = 0;
    for (const Slot &s : b->slots) n += s.live;
    size_t tot = 0, big = 0;
    for (const auto &kv : b->free_list) {
        tot += kv.second;
        big = std::max(big, kv.second);
    }
    if (live_plates) *live_plates = n;
    if (arena_free) *arena_free = tot;
    if (arena_largest_free) *arena_largest_free = big;
    return LBM_OK;
}

void lbm_batch_destroy(lbm_batch *b)
{
    if (!b) return;
    (void)hipStreamSynchronize(b->stream);
    for (auto &kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
    if (b->capture) (void)hipStreamDestroy(b->capture);
    for (int i = 0; i < 2; ++i) {
        if (b->h_plates[i]) (void)hipHostFree(b->h_plates[i]);
        if (b->h_tiles[i]) (void)hipHostFree(b->h_tiles[i]);
        if (b->h_ntiles[i]) (void)hipHostFree(b->h_ntiles[i]);
        if (b->ev[i]) (void)hipEventDestroy(b->ev[i]);
    }
    delete b;
}

const char *lbm_batch_last_error(const lbm_batch *b) { return b ? b->err.c_str() : g_batch_create_error.c_str(); }

}  // extern "C"
