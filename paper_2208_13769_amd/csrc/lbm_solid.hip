// lbm_solid.hip -- single-plate host runtime and C ABI (include/lbm_solid.h).
//
// A handle owns no device memory: the caller's workspace is carved into two
// copies of the state (ping-pong), a read-out staging area, reduction
// scratch and a flag word. lbm_step only enqueues kernels on the caller's
// stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "general_kernels.hpp"
#include "host_common.hpp"

using namespace lbm;

namespace {

struct Layout {
    StateLayout state;
    size_t staging, staging_bytes;
    size_t partials, small, total;
    size_t scratch, total_walled;  // scratch of the general step (walls on the x edges)
    size_t mask;                   // material mask [ny][nx] bytes, after the scratch
    size_t tiles;                  // tile table of the general step (TILE_* bytes), after the mask
    size_t flist;                  // fused-kernel tiles of the general step (3 ints each), after the tiles
    size_t tlist;                  // the 2D tiles the general step launches (int each), after the fused list
    // paired steps: the two-step fused list, the 2D tiles of the first step
    // (the rest widened by one tile) and of the second (the rest), and a
    // third copy of the state for the first step's output
    size_t flist2, tlist_a, tlist_b;
    size_t mid_f, mid_u, mid_j;
};

size_t general_scratch(int nx, int ny, lbm_precision p)
{
    switch (p) {
    case LBM_FP64: return general_scratch_bytes<PrecF64>(nx, ny);
    case LBM_FP32: return general_scratch_bytes<PrecF32>(nx, ny);
    case LBM_FP16_STORE: return general_scratch_bytes<PrecF16>(nx, ny);
    case LBM_FP32_U64: return general_scratch_bytes<PrecF32U64>(nx, ny);
    default: return general_scratch_bytes<PrecBF16>(nx, ny);
    }
}

Layout make_layout(int nx, int ny, lbm_precision p)
{
    Layout L{};
    L.state = state_layout(nx, ny, p);
    size_t off = L.state.bytes;
    L.staging = off;
    L.staging_bytes = staging_bytes_for(nx, ny);
    off = align_up(off + L.staging_bytes);
    L.partials = off;
    off = align_up(off + kMaxDiagBlocks * 8 * sizeof(double));
    L.small = off;  // flag word + final diagnostics
    off = align_up(off + 64 * sizeof(double));
    L.total = off;
    L.scratch = off;
    L.mask = align_up(off + general_scratch(nx, ny, p));
    L.tiles = align_up(L.mask + (size_t)nx * ny);
    L.flist = align_up(L.tiles + max_tiles(nx, ny));
    L.tlist = align_up(L.flist + 3 * sizeof(int) * max_tiles(nx, ny));
    L.flist2 = align_up(L.tlist + sizeof(int) * max_tiles(nx, ny));
    L.tlist_a = align_up(L.flist2 + 3 * sizeof(int) * max_tiles(nx, ny));
    L.tlist_b = align_up(L.tlist_a + sizeof(int) * max_tiles(nx, ny));
    const ElemSizes es = elem_sizes(p);
    const size_t n = (size_t)nx * ny;
    L.mid_f = align_up(L.tlist_b + sizeof(int) * max_tiles(nx, ny));
    L.mid_u = align_up(L.mid_f + 9 * n * es.f);
    L.mid_j = align_up(L.mid_u + 2 * n * es.u);
    L.total_walled = align_up(L.mid_j + 2 * n * es.j);
    return L;
}

}  // namespace

// Device scratch of lbm_read_diagnostics_noalloc: the per-block partial sums
// of the diagnostics kernel (kMaxDiagBlocks blocks, 8 doubles each) and the
// folded values (8 doubles). Each GPU holds its own copy until the process
// ends; every call on a GPU shares it.
constexpr size_t kNoAllocDiagDoubles = (size_t)kMaxDiagBlocks * 8 + 8;
static __device__ __align__(256) double scratch[kNoAllocDiagDoubles];

struct lbm_solver {
    int nx = 0, ny = 0;
    int device = 0;  // the device current at lbm_create
    double dx = 1.0;
    lbm_precision prec = LBM_FP64;
    lbm_scheme scheme = LBM_SCHEME_PC;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    hipStream_t stream = nullptr;
    Layout L{};
    int cur = 0;  // copy holding the current state
    bool material = false, fields = false;
    double rho0 = 1, lam = 0, mu = 0, tau = 1;
    double body[2] = {0, 0};
    int bc[4] = {LBM_BC_PERIODIC, LBM_BC_PERIODIC, LBM_BC_PERIODIC, LBM_BC_PERIODIC};
    double bcval[4][2] = {};
    // Momentum walls move with velocity j* / rho0: the wall of edge e is at
    // uwb[e] + j*_L n at step n (lattice units). Changing j* at step n moves
    // uwb so that the displacement stays continuous.
    double uwb[4][2] = {};
    double f_scale = 1.0;
    int64_t steps = 0;
    Shape shape{};
    int spl = 1;  // time steps per launch (1, or 2 with the predictor-corrector)
    int sr = 0;   // stochastic rounding of 16-bit populations
    unsigned long long seed = 0;
    bool force_general = false;  // run the general step even without x walls
    bool has_mask = false;       // holes (lbm_set_mask)
    std::vector<unsigned char> mask_host;  // host copy of the mask (1 material, 0 hole)
    bool tables_dirty = true;    // the general step's tile table and fused list need rebuilding
    bool tables_built = false;   // the tile table in the workspace is valid
    int n_flist = 0;             // entries of the fused list
    int n_tlist = 0;             // entries of the 2D tile list
    int n_flist2 = 0, n_tlist_a = 0, n_tlist_b = 0;  // paired steps (n_flist2 = 0: none)
    Shape fshape2{};             // the two-step fused list's launch shape
    Shape fshape{};              // the fused list's launch shape (256 threads, one step)
    // The 2D tiles run on a second stream beside the fused share (forked
    // from and joined back into the handle's stream each step or pair);
    // created on first use, default priority.
    hipStream_t aux = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    ~lbm_solver()
    {
        if (aux) (void)hipStreamSynchronize(aux);
        if (fork) (void)hipEventDestroy(fork);
        if (join) (void)hipEventDestroy(join);
        if (aux) (void)hipStreamDestroy(aux);
    }

    bool general() const
    {
        return force_general || has_mask || bc[LBM_EDGE_XMIN] != LBM_BC_PERIODIC || scheme == LBM_SCHEME_EXTRAP;
    }
    const unsigned char *mask_ptr() const
    {
        return has_mask ? reinterpret_cast<const unsigned char *>(ws + L.mask) : nullptr;
    }
    const unsigned char *tiles_ptr() const
    {
        return tables_built ? reinterpret_cast<const unsigned char *>(ws + L.tiles) : nullptr;
    }
    std::string err;

    void *fptr(int c) const { return ws + L.state.f[c]; }
    void *uptr(int c) const { return ws + L.state.u[c]; }
    void *jptr(int c) const { return ws + L.state.j[c]; }
    unsigned *flag() const { return reinterpret_cast<unsigned *>(ws + L.small); }
    Units units() const { return Units{dx, rho0, lam, mu}; }

    // lattice velocity of edge e's wall (zero unless a momentum wall)
    double wall_speed(int e, int a) const
    {
        return bc[e] == LBM_BC_DIRICHLET_J && material ? bcval[e][a] / units().momentum() : 0.0;
    }
    double load_bound() const { return load_population_bound(units(), nx, ny, bc, bcval, body); }
    // 16-bit storage: lower the population scale (rescaling the stored
    // populations on the stream) when the loads now set could drive the
    // populations beyond the headroom of the current scale
    hipError_t refit_scale()
    {
        if (!fields || (prec != LBM_FP16_STORE && prec != LBM_BF16_STORE)) return hipSuccess;
        const double need = load_bound();
        if (!(need * f_scale > kScaledHeadroom)) return hipSuccess;
        const double ns = population_scale(need);
        const hipError_t e = plate_rescale(prec, fptr(cur), (size_t)nx * ny, ns / f_scale, stream);
        if (e == hipSuccess) f_scale = ns;
        return e;
    }
    // set edge e's rule and value, keeping its wall displacement continuous
    // at the current step
    void set_edge(int e, int kind, double v0, double v1)
    {
        const double n = (double)steps;
        const double now[2] = {uwb[e][0] + wall_speed(e, 0) * n, uwb[e][1] + wall_speed(e, 1) * n};
        bc[e] = kind;
        bcval[e][0] = v0;
        bcval[e][1] = v1;
        for (int a = 0; a < 2; ++a) uwb[e][a] = now[a] - wall_speed(e, a) * n;
    }

    PlateIO io() const
    {
        PlateIO p{};
        p.nx = nx;
        p.ny = ny;
        p.prec = prec;
        p.U = units();
        p.bc_lo = bc[LBM_EDGE_YMIN];
        p.bc_hi = bc[LBM_EDGE_YMAX];
        p.bc_left = bc[LBM_EDGE_XMIN];
        p.bc_right = bc[LBM_EDGE_XMAX];
        for (int a = 0; a < 2; ++a) {
            p.val_lo[a] = bcval[LBM_EDGE_YMIN][a];
            p.val_hi[a] = bcval[LBM_EDGE_YMAX][a];
            p.val_left[a] = bcval[LBM_EDGE_XMIN][a];
            p.val_right[a] = bcval[LBM_EDGE_XMAX][a];
            p.uwb_lo[a] = uwb[LBM_EDGE_YMIN][a];
            p.uwb_hi[a] = uwb[LBM_EDGE_YMAX][a];
            p.uwb_left[a] = uwb[LBM_EDGE_XMIN][a];
            p.uwb_right[a] = uwb[LBM_EDGE_XMAX][a];
        }
        p.f = fptr(cur);
        p.u = uptr(cur);
        p.j = jptr(cur);
        p.f_other = fptr(cur ^ 1);
        p.f_scale = f_scale;
        p.staging = reinterpret_cast<double *>(ws + L.staging);
        p.staging_bytes = L.staging_bytes;
        p.partials = reinterpret_cast<double *>(ws + L.partials);
        p.diag_out = reinterpret_cast<double *>(ws + L.small + 64);
        p.mask = mask_ptr();
        p.stream = stream;
        return p;
    }
};

namespace {

thread_local std::string g_create_error;

lbm_status fail(lbm_solver *h, lbm_status s, const std::string &msg)
{
    if (h)
        h->err = msg;
    else
        g_create_error = msg;
    return s;
}

lbm_status hip_fail(lbm_solver *h, hipError_t e, const char *what)
{
    return fail(h, LBM_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(h, call)                                     \
    do {                                                     \
        hipError_t e_ = (call);                              \
        if (e_ != hipSuccess) return hip_fail(h, e_, #call); \
    } while (0)

int resident_blocks(const lbm_solver *h, int block, int spl, int walled_form = -1)
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    const bool pc = h->scheme == LBM_SCHEME_PC;
    // the kernel form of the handle's y edges, unless one is asked for
    const bool walled = walled_form >= 0 ? walled_form != 0 : h->bc[LBM_EDGE_YMIN] != LBM_BC_PERIODIC;
    int per_cu = 0;
    switch (h->prec) {
    case LBM_FP64: per_cu = Kernels<PrecF64>::resident_per_cu(block, spl, pc, walled); break;
    case LBM_FP32: per_cu = Kernels<PrecF32>::resident_per_cu(block, spl, pc, walled); break;
    case LBM_FP16_STORE: per_cu = Kernels<PrecF16>::resident_per_cu(block, spl, pc, walled); break;
    case LBM_FP32_U64: per_cu = Kernels<PrecF32U64>::resident_per_cu(block, spl, pc, walled); break;
    default: per_cu = Kernels<PrecBF16>::resident_per_cu(block, spl, pc, walled); break;
    }
    return per_cu * cus;
}

// whether two steps per launch fit the LDS with this block size, for the
// handle's precision and y boundaries
bool two_step_fits(const lbm_solver *h, int block)
{
    const bool walled = h->bc[LBM_EDGE_YMIN] != LBM_BC_PERIODIC;
    switch (h->prec) {
    case LBM_FP64: return Kernels<PrecF64>::step2_ok(block, walled);
    case LBM_FP32: return Kernels<PrecF32>::step2_ok(block, walled);
    case LBM_FP16_STORE: return Kernels<PrecF16>::step2_ok(block, walled);
    case LBM_FP32_U64: return Kernels<PrecF32U64>::step2_ok(block, walled);
    default: return Kernels<PrecBF16>::step2_ok(block, walled);
    }
}

// a two-step tiling whose block no longer fits (the y edges stopped being
// periodic) runs with 256 threads
void refit_two_step(lbm_solver *h)
{
    if (h->spl == 2 && !two_step_fits(h, h->shape.block))
        h->shape = make_shape(h->nx, h->ny, h->prec, h->scheme, 256, h->shape.n_segs, 2);
}

void plan_launch(lbm_solver *h)
{
    const int halo = stencil_halo(h->prec, h->scheme, h->spl);
    // narrowest block whose strip covers the width, else 256 threads
    int block = 256;
    if (h->nx <= 64 - 2 * halo)
        block = 64;
    else if (h->nx <= 128 - 2 * halo)
        block = 128;
    const Shape probe = make_shape(h->nx, h->ny, h->prec, h->scheme, block, 1, h->spl);
    const int resident = std::max(resident_blocks(h, block, h->spl), probe.n_strips);
    // A block marches its rows one after another, so on a small plate the
    // step takes as long as the longest march: use the shortest segments (1,
    // 2, 4 or 8 rows) whose recomputed halo rows keep the launch within one
    // wave of resident blocks and about 1.5 M thread-rows (measured on 64^2
    // to 512^2 plates: 1.6-2.5 times faster than 16-row segments).
    for (int rows = 1; rows <= 8; rows *= 2) {
        const long long segs = (h->ny + rows - 1) / rows;
        const long long work = (long long)probe.n_strips * segs * (rows + 2 * halo + 1) * block;
        if (probe.n_strips * segs <= resident && work <= 1500000) {
            h->shape = make_shape(h->nx, h->ny, h->prec, h->scheme, block, (int)segs, h->spl);
            return;
        }
    }
    // otherwise as many segments as fit one wave of resident blocks (the last
    // wave of a longer grid would run part-empty), each of at least 16 rows
    int n_segs = resident / probe.n_strips;
    n_segs = std::max(1, std::min(n_segs, h->ny / 16));
    h->shape = make_shape(h->nx, h->ny, h->prec, h->scheme, block, n_segs, h->spl);
}

}  // namespace

extern "C" {

size_t lbm_workspace_bytes(int nx, int ny, lbm_precision p)
{
    if (nx < 5 || ny < 5 || !valid_precision(p)) return 0;
    return make_layout(nx, ny, p).total;
}

size_t lbm_workspace_bytes_walled(int nx, int ny, lbm_precision p)
{
    if (nx < 5 || ny < 5 || !valid_precision(p)) return 0;
    return make_layout(nx, ny, p).total_walled;
}

lbm_status lbm_create(int nx, int ny, double dx, lbm_precision p, lbm_scheme s, void *dev_workspace,
                      size_t ws_bytes, void *hip_stream, lbm_solver **out)
{
    if (!out) return fail(nullptr, LBM_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (nx < 5 || ny < 5) return fail(nullptr, LBM_ERR_ARG, "nx and ny must be >= 5");
    if (!(dx > 0.0) || !std::isfinite(dx)) return fail(nullptr, LBM_ERR_ARG, "dx must be positive");
    if (!valid_precision(p)) return fail(nullptr, LBM_ERR_ARG, "unknown precision");
    if (s != LBM_SCHEME_PC && s != LBM_SCHEME_EXPLICIT && s != LBM_SCHEME_EXTRAP)
        return fail(nullptr, LBM_ERR_ARG, "unknown scheme");
    if (!dev_workspace) return fail(nullptr, LBM_ERR_ARG, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(dev_workspace) % kAlign)
        return fail(nullptr, LBM_ERR_ARG, "workspace not 256-byte aligned");
    if ((long long)nx * ny > (1LL << 29)) return fail(nullptr, LBM_ERR_UNSUPPORTED, "more than 2^29 sites");
    const Layout L = make_layout(nx, ny, p);
    if (ws_bytes < L.total) return fail(nullptr, LBM_ERR_NOMEM, "workspace smaller than lbm_workspace_bytes()");
    if (s == LBM_SCHEME_EXTRAP && ws_bytes < L.total_walled)
        return fail(nullptr, LBM_ERR_NOMEM, "the extrapolation scheme needs lbm_workspace_bytes_walled() bytes");
    lbm_solver *h = new (std::nothrow) lbm_solver();
    if (!h) return fail(nullptr, LBM_ERR_NOMEM, "host allocation failed");
    h->nx = nx;
    h->ny = ny;
    h->dx = dx;
    h->prec = p;
    h->scheme = s;
    h->ws = static_cast<char *>(dev_workspace);
    h->ws_bytes = ws_bytes;
    h->stream = static_cast<hipStream_t>(hip_stream);
    h->L = L;
    if (hipGetDevice(&h->device) != hipSuccess) h->device = 0;
    plan_launch(h);
    *out = h;
    return LBM_OK;
}

lbm_status lbm_set_material(lbm_solver *h, double rho0, double lambda, double mu, double tau_over_dt)
{
    if (!h) return LBM_ERR_ARG;
    if (!(rho0 > 0) || !std::isfinite(rho0)) return fail(h, LBM_ERR_ARG, "rho0 must be positive");
    if (!(mu > 0) || !std::isfinite(mu)) return fail(h, LBM_ERR_ARG, "mu must be positive");
    if (!(lambda + mu > 0) || !std::isfinite(lambda)) return fail(h, LBM_ERR_ARG, "lambda + mu must be positive");
    if (!(tau_over_dt > 0.5) || !std::isfinite(tau_over_dt)) return fail(h, LBM_ERR_ARG, "tau/dt must exceed 1/2");
    if (h->fields) return fail(h, LBM_ERR_STATE, "set the material before the fields");
    h->rho0 = rho0;
    h->lam = lambda;
    h->mu = mu;
    h->tau = tau_over_dt;
    h->material = true;
    return LBM_OK;
}

lbm_status lbm_set_body_force(lbm_solver *h, const double b[2])
{
    if (!h) return LBM_ERR_ARG;
    if (!b) return fail(h, LBM_ERR_ARG, "NULL argument");
    if (!std::isfinite(b[0]) || !std::isfinite(b[1])) return fail(h, LBM_ERR_ARG, "body force not finite");
    h->body[0] = b[0];
    h->body[1] = b[1];
    HIP_TRY(h, h->refit_scale());
    return LBM_OK;
}

lbm_status lbm_set_boundary(lbm_solver *h, lbm_edge e, lbm_bc bc, const double value[2])
{
    if (!h) return LBM_ERR_ARG;
    if (e < LBM_EDGE_XMIN || e > LBM_EDGE_YMAX) return fail(h, LBM_ERR_ARG, "unknown edge");
    if (bc < LBM_BC_PERIODIC || bc > LBM_BC_NEUMANN_T) return fail(h, LBM_ERR_ARG, "unknown boundary rule");
    if ((e == LBM_EDGE_XMIN || e == LBM_EDGE_XMAX) && bc != LBM_BC_PERIODIC && h->ws_bytes < h->L.total_walled)
        return fail(h, LBM_ERR_NOMEM, "walls on the x edges need a workspace of lbm_workspace_bytes_walled() bytes");
    if (bc != LBM_BC_PERIODIC && (!value || !std::isfinite(value[0]) || !std::isfinite(value[1])))
        return fail(h, LBM_ERR_ARG, "boundary value missing or not finite");
    const int other = e == LBM_EDGE_YMIN ? LBM_EDGE_YMAX
                      : e == LBM_EDGE_YMAX ? LBM_EDGE_YMIN
                      : e == LBM_EDGE_XMIN ? LBM_EDGE_XMAX
                                           : LBM_EDGE_XMIN;
    if (h->has_mask && (h->bc[e] == LBM_BC_PERIODIC) != (bc == LBM_BC_PERIODIC))
        return fail(h, LBM_ERR_STATE, "a mask was checked against the edges: make edges periodic or not before it");
    if (bc == LBM_BC_PERIODIC && h->bc[other] != LBM_BC_PERIODIC) {
        // periodic edges come in pairs
        h->set_edge(other, LBM_BC_PERIODIC, 0.0, 0.0);
    }
    if (bc != LBM_BC_PERIODIC && h->bc[other] == LBM_BC_PERIODIC) {
        // the opposite edge stops being periodic: it becomes a wall at rest until set
        h->set_edge(other, LBM_BC_DIRICHLET_J, 0.0, 0.0);
    }
    if ((h->bc[e] == LBM_BC_PERIODIC) != (bc == LBM_BC_PERIODIC)) h->tables_dirty = true;
    h->set_edge(e, bc, bc == LBM_BC_PERIODIC ? 0.0 : value[0], bc == LBM_BC_PERIODIC ? 0.0 : value[1]);
    refit_two_step(h);
    HIP_TRY(h, h->refit_scale());
    return LBM_OK;
}

lbm_status lbm_set_tiling(lbm_solver *h, int block, int n_segs)
{
    if (!h) return LBM_ERR_ARG;
    if (block != 64 && block != 128 && block != 256 && block != 512)
        return fail(h, LBM_ERR_ARG, "block must be 64, 128, 256 or 512");
    if (n_segs < 1 || n_segs > h->ny) return fail(h, LBM_ERR_ARG, "n_segs must be in [1, ny]");
    if ((long long)h->nx * n_segs > (1LL << 30)) return fail(h, LBM_ERR_ARG, "too many blocks");
    if (h->spl == 2 && !two_step_fits(h, block))
        return fail(h, LBM_ERR_UNSUPPORTED, "two steps per launch with this block size exceed the LDS");
    h->shape = make_shape(h->nx, h->ny, h->prec, h->scheme, block, n_segs, h->spl);
    return LBM_OK;
}

lbm_status lbm_set_steps_per_launch(lbm_solver *h, int k)
{
    if (!h) return LBM_ERR_ARG;
    if (k != 1 && k != 2) return fail(h, LBM_ERR_ARG, "steps per launch must be 1 or 2");
    if (k == 2 && h->scheme != LBM_SCHEME_PC)
        return fail(h, LBM_ERR_UNSUPPORTED, "two steps per launch need the predictor-corrector scheme");
    if (k == 2 && max_steps_per_launch(h->prec, h->scheme) < 2)
        return fail(h, LBM_ERR_UNSUPPORTED, "16-bit population storage runs one step per launch");
    h->spl = k;
    const int block = k == 2 && !two_step_fits(h, h->shape.block) ? 256 : h->shape.block;
    h->shape = make_shape(h->nx, h->ny, h->prec, h->scheme, block, h->shape.n_segs, k);
    return LBM_OK;
}

lbm_status lbm_resident_blocks(const lbm_solver *h, int block, int steps_per_launch, int *blocks)
{
    if (!h || !blocks) return LBM_ERR_ARG;
    *blocks = 0;
    if (block != 64 && block != 128 && block != 256 && block != 512) return LBM_OK;
    if (steps_per_launch != 1 && steps_per_launch != 2) return LBM_OK;
    if (steps_per_launch == 2 && h->scheme != LBM_SCHEME_PC) return LBM_OK;
    *blocks = resident_blocks(h, block, steps_per_launch);
    return LBM_OK;
}

lbm_status lbm_set_mask(lbm_solver *h, const unsigned char *solid)
{
    if (!h) return LBM_ERR_ARG;
    if (h->fields) return fail(h, LBM_ERR_STATE, "set the mask before the fields");
    if (!solid) {
        h->has_mask = false;
        h->mask_host.clear();
        h->tables_dirty = true;
        return LBM_OK;
    }
    if (h->ws_bytes < h->L.total_walled)
        return fail(h, LBM_ERR_NOMEM, "holes need a workspace of lbm_workspace_bytes_walled() bytes");
    const int nx = h->nx, ny = h->ny;
    const bool perx = h->bc[LBM_EDGE_XMIN] == LBM_BC_PERIODIC, pery = h->bc[LBM_EDGE_YMIN] == LBM_BC_PERIODIC;
    auto hole = [&](int x, int y) {
        if (y < 0 || y >= ny) {
            if (!pery) return false;
            y = (y % ny + ny) % ny;
        }
        if (x < 0 || x >= nx) {
            if (!perx) return false;
            x = (x % nx + nx) % nx;
        }
        return solid[(size_t)y * nx + x] == 0;
    };
    bool any_material = false;
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            if (hole(x, y)) {
                if (((y == 0 || y == ny - 1) && !pery) || ((x == 0 || x == nx - 1) && !perx))
                    return fail(h, LBM_ERR_ARG, "a hole touches a wall edge");
                continue;
            }
            any_material = true;
            if ((hole(x - 1, y) && hole(x + 1, y)) || (hole(x, y - 1) && hole(x, y + 1)))
                return fail(h, LBM_ERR_ARG, "material one node thick between holes");
        }
    if (!any_material) return fail(h, LBM_ERR_ARG, "no material node");
    std::vector<unsigned char> dev(solid, solid + (size_t)nx * ny);
    for (auto &m : dev) m = m ? 1 : 0;
    HIP_TRY(h, hipMemcpyAsync(h->ws + h->L.mask, dev.data(), (size_t)nx * ny, hipMemcpyHostToDevice, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    h->mask_host.swap(dev);
    h->has_mask = true;
    h->tables_dirty = true;
    return LBM_OK;
}

lbm_status lbm_set_general_path(lbm_solver *h, int on)
{
    if (!h) return LBM_ERR_ARG;
    // (holes, x walls and the extrapolation scheme already hold the walled
    // workspace; the general step of any other plate needs no more)
    h->force_general = on != 0;
    return LBM_OK;
}

lbm_status lbm_set_rounding(lbm_solver *h, lbm_rounding r, uint64_t seed)
{
    if (!h) return LBM_ERR_ARG;
    if (r != LBM_ROUND_NEAREST && r != LBM_ROUND_STOCHASTIC) return fail(h, LBM_ERR_ARG, "unknown rounding");
    if (r == LBM_ROUND_STOCHASTIC && h->prec != LBM_FP16_STORE && h->prec != LBM_BF16_STORE)
        return fail(h, LBM_ERR_UNSUPPORTED, "stochastic rounding needs 16-bit population storage");
    h->sr = r == LBM_ROUND_STOCHASTIC;
    h->seed = seed;
    return LBM_OK;
}

lbm_status lbm_get_steps_per_launch(const lbm_solver *h, int *k)
{
    if (!h || !k) return LBM_ERR_ARG;
    *k = h->spl;
    return LBM_OK;
}

lbm_status lbm_get_tiling(const lbm_solver *h, int *block, int *n_segs)
{
    if (!h || !block || !n_segs) return LBM_ERR_ARG;
    *block = h->shape.block;
    *n_segs = h->shape.n_segs;
    return LBM_OK;
}

lbm_status lbm_get_dt(const lbm_solver *h, double *dt)
{
    if (!h || !dt) return LBM_ERR_ARG;
    if (!h->material) return LBM_ERR_STATE;
    *dt = h->units().dt();
    return LBM_OK;
}

lbm_status lbm_set_fields(lbm_solver *h, const double *u0, const double *v0)
{
    if (!h) return LBM_ERR_ARG;
    if (!u0 || !v0) return fail(h, LBM_ERR_ARG, "u0 or v0 is NULL");
    if (!h->material) return fail(h, LBM_ERR_STATE, "set the material before the fields");
    h->cur = 0;
    for (auto &w : h->uwb) w[0] = w[1] = 0.0;  // every wall starts undisplaced
    double scale = 1.0;
    bool nonfinite = false;
    const hipError_t e = plate_start(h->io(), u0, v0, h->load_bound(), &scale, &nonfinite);
    if (e != hipSuccess) return hip_fail(h, e, "start-up");
    if (nonfinite) return fail(h, LBM_ERR_ARG, "initial fields not finite");
    h->f_scale = scale;
    if (h->scheme == LBM_SCHEME_EXTRAP)  // j one step back: j(0) before the first step
        HIP_TRY(h, hipMemcpyAsync(h->jptr(1), h->jptr(0), 2 * (size_t)h->nx * h->ny * elem_sizes(h->prec).j,
                                  hipMemcpyDeviceToDevice, h->stream));
    HIP_TRY(h, hipMemsetAsync(h->flag(), 0, sizeof(unsigned), h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    h->steps = 0;
    h->fields = true;
    return LBM_OK;
}

namespace {

// The general step's tables, built on the host when the mask or the edges
// change. The tile table marks each 2D tile whose window holds a hole node,
// that holds a material node, and that the fused kernel computes instead.
// The fused list: on a plate with x walls or holes, the tiles of the fused
// step kernel (256-thread strips, row runs aligned to the 2D tiles' rows)
// whose outputs lie farther than the stencil's reach from every wall and
// hole. There the fused kernel's periodic arithmetic is the general rules'
// arithmetic, and it runs those sites at the fused kernel's rate.
hipError_t build_general_tables(lbm_solver *h)
{
    const int nx = h->nx, ny = h->ny;
    const bool perx = h->bc[LBM_EDGE_XMIN] == LBM_BC_PERIODIC, pery = h->bc[LBM_EDGE_YMIN] == LBM_BC_PERIODIC;
    const bool pc = h->scheme != LBM_SCHEME_EXPLICIT;
    int tw = 0, th = 0, ru = 0;
    switch (h->prec) {
    case LBM_FP64: tile_shape<PrecF64>(pc, tw, th, ru); break;
    case LBM_FP32: tile_shape<PrecF32>(pc, tw, th, ru); break;
    case LBM_FP16_STORE: tile_shape<PrecF16>(pc, tw, th, ru); break;
    case LBM_FP32_U64: tile_shape<PrecF32U64>(pc, tw, th, ru); break;
    default: tile_shape<PrecBF16>(pc, tw, th, ru); break;
    }
    const int mg = stencil_halo(h->prec, h->scheme, 1);
    // hole counts of boxes: per-row prefix sums over the rows and columns
    // within max(ru, mg) of the plate (wrapped across periodic edges; beyond
    // a wall there are no holes)
    const int e = std::max(ru, mg);
    const int W = nx + 2 * e, Hh = ny + 2 * e;
    std::vector<uint32_t> pre;
    const bool any_mask = h->has_mask;
    if (any_mask) {
        pre.assign((size_t)Hh * (W + 1), 0u);
        const unsigned char *m = h->mask_host.data();
        for (int r = 0; r < Hh; ++r) {
            int y = r - e;
            bool row_in = true;
            if (y < 0 || y >= ny) {
                if (pery) y = ((y % ny) + ny) % ny;
                else row_in = false;
            }
            uint32_t *pr = pre.data() + (size_t)r * (W + 1);
            for (int c = 0; c < W; ++c) {
                int x = c - e;
                bool in = row_in;
                if (x < 0 || x >= nx) {
                    if (perx) x = ((x % nx) + nx) % nx;
                    else in = false;
                }
                pr[c + 1] = pr[c] + ((in && m[(size_t)y * nx + x] == 0) ? 1u : 0u);
            }
        }
    }
    // holes in [x0, x1) x [y0, y1), plate coordinates within e of the plate
    auto holes_in = [&](int x0, int x1, int y0, int y1) -> bool {
        if (!any_mask) return false;
        x0 = std::max(x0, -e) + e, x1 = std::min(x1, nx + e) + e;
        y0 = std::max(y0, -e) + e, y1 = std::min(y1, ny + e) + e;
        for (int r = y0; r < y1; ++r) {
            const uint32_t *pr = pre.data() + (size_t)r * (W + 1);
            if (pr[x1] != pr[x0]) return true;
        }
        return false;
    };
    const int nbx = (nx + tw - 1) / tw, nby = (ny + th - 1) / th;
    std::vector<unsigned char> tiles((size_t)nbx * nby, 0);
    for (int ty = 0; ty < nby; ++ty)
        for (int tx = 0; tx < nbx; ++tx) {
            const int x0 = tx * tw, y0 = ty * th;
            const int x1 = std::min(nx, x0 + tw), y1 = std::min(ny, y0 + th);
            unsigned char f = 0;
            // material: fewer hole nodes than nodes in the tile
            if (!any_mask) {
                f = TILE_MATERIAL;
            } else {
                uint32_t n = 0;
                for (int r = y0 + e; r < y1 + e; ++r) {
                    const uint32_t *pr = pre.data() + (size_t)r * (W + 1);
                    n += pr[x1 + e] - pr[x0 + e];
                }
                if (n < (uint32_t)((x1 - x0) * (y1 - y0))) f = TILE_MATERIAL;
            }
            if (holes_in(x0 - ru, x0 + tw + ru, y0 - ru, y0 + th + ru)) f |= TILE_HOLES;
            tiles[(size_t)ty * nbx + tx] = f;
        }
    // fused-kernel entries of a launch of spl steps: (strip, row run) pairs
    // whose outputs lie farther than the launch's stencil reach from x walls
    // and holes; `mark` receives the 2D tiles they cover
    auto fused_list = [&](int spl, int runs, Shape &fs, std::vector<unsigned char> &mark) {
        std::vector<int> list;
        mark.assign(tiles.size(), 0);
        if (h->scheme == LBM_SCHEME_EXTRAP || !(any_mask || !perx)) return list;
        fs = make_shape(nx, ny, h->prec, h->scheme, 256, 1, spl);
        const int reach = stencil_halo(h->prec, h->scheme, spl);
        // row runs of at most seg_rows rows: about `runs` per strip
        const int seg_rows = std::max(th, (ny / runs) / th * th);
        // a strip's columns start on a 2D tile's column (strips are a
        // multiple of 32 columns wide, or the whole plate)
        if (!(fs.n_strips == 1 || fs.strip_w % tw == 0)) return list;
        // with x walls the strips start at the first tile column beyond the
        // reach from the wall and end at the last one before the far wall,
        // so the 2D tiles keep one tile column at each wall, not a strip
        int n_st = fs.n_strips;
        if (!perx) {
            fs.x_lo = (reach + tw - 1) / tw * tw;
            fs.x_end = (nx - reach) / tw * tw;
            n_st = fs.x_end > fs.x_lo ? (fs.x_end - fs.x_lo + fs.strip_w - 1) / fs.strip_w : 0;
        }
        const int xe = fs.x_end > 0 ? fs.x_end : nx;
        // likewise the row runs stay a tile row clear of y walls: no output
        // of the fused share then depends on a wall rule or a ghost row, and
        // it runs the fused kernel's periodic form (fewer registers and LDS
        // bytes than the walled one), leaving the rows at y walls to the tiles
        const int ylo = pery ? 0 : (reach + th - 1) / th * th;
        const int yend = pery ? ny : (ny - reach) / th * th;
        for (int st = 0; st < n_st; ++st) {
            const int x0 = fs.x_lo + st * fs.strip_w, x1 = std::min(xe, x0 + fs.strip_w);
            if (!perx && (x0 - reach < 0 || x1 + reach > nx)) continue;
            int run0 = -1;
            for (int ty = 0; ty <= nby; ++ty) {
                const bool clean = ty < nby && ty * th >= ylo && std::min(ny, ty * th + th) <= yend &&
                                   !holes_in(x0 - reach, x1 + reach, ty * th - reach,
                                             std::min(ny, ty * th + th) + reach);
                if (clean && run0 < 0) run0 = ty;
                if (!clean && run0 >= 0) {
                    const int ya = run0 * th, yb = std::min(ny, ty * th);
                    for (int a = ya; a < yb; a += seg_rows) {
                        list.push_back(st);
                        list.push_back(a);
                        list.push_back(std::min(yb, a + seg_rows));
                    }
                    for (int t = run0; t < ty; ++t)
                        for (int tx = x0 / tw; tx < (x1 + tw - 1) / tw; ++tx) mark[(size_t)t * nbx + tx] = 1;
                    run0 = -1;
                }
            }
        }
        return list;
    };
    // The fused grid is sized to one wave of resident blocks of its periodic
    // form: from 26 row runs per strip (as the default plan's segments of a
    // periodic plate) down until the list fits; a block that waits for a
    // second wave would double the share's time.
    auto fused_fit = [&](int spl, Shape &fs, std::vector<unsigned char> &mark) {
        const int slots = resident_blocks(h, 256, spl, 0);
        int runs = 26;
        for (;;) {
            std::vector<int> list = fused_list(spl, runs, fs, mark);
            const int n = (int)(list.size() / 3);
            if (slots <= 0 || n <= slots || runs == 1) return list;
            runs = std::max(1, std::min(runs - 1, (int)((long long)runs * slots / n)));
        }
    };
    std::vector<unsigned char> mark1, mark2;
    const std::vector<int> list = fused_fit(1, h->fshape, mark1);
    for (size_t t = 0; t < tiles.size(); ++t)
        if (mark1[t]) tiles[t] |= TILE_FUSED;
    // the 2D tiles to launch: those with material that the fused kernel does
    // not compute, in row-major order (the kernel deals them to the XCDs in
    // equal runs)
    std::vector<int> tl;
    for (size_t t = 0; t < tiles.size(); ++t)
        if ((tiles[t] & TILE_MATERIAL) && !(tiles[t] & TILE_FUSED)) tl.push_back((int)t);
    // Paired steps: the two-step fused kernel over the strips clear of walls
    // and holes by two steps' reach; the 2D tiles advance the rest in two
    // launches, the first over the rest widened by one tile (at least the
    // one-step reach in each direction) into a third state copy, the second
    // from it over the rest.
    // The fused share runs the periodic form, whose two-step block leaves
    // room for a second one on a compute unit. On the 4096² plate with a
    // hole, paired steps take 0.576 ms per step in FP64, 0.329 in FP32 and
    // 0.429 in FP32 with a double displacement, against 0.534 one step at a
    // time in the last (16-bit storage has no two-step kernel).
    std::vector<int> list2, tla, tlb;
    bool pair = false;
    if (h->scheme == LBM_SCHEME_PC && th >= mg && tw >= mg) {
        if (h->prec == LBM_FP64) pair = Kernels<PrecF64>::step2_ok(256, false);
        if (h->prec == LBM_FP32) pair = Kernels<PrecF32>::step2_ok(256, false);
        if (h->prec == LBM_FP32_U64) pair = Kernels<PrecF32U64>::step2_ok(256, false);
    }
    if (pair) {
        list2 = fused_fit(2, h->fshape2, mark2);
        std::vector<unsigned char> rest(tiles.size(), 0), wide(tiles.size(), 0);
        for (size_t t = 0; t < tiles.size(); ++t) rest[t] = (tiles[t] & TILE_MATERIAL) && !mark2[t];
        // nodes between [a0, a1) and [b0, b1) on a line or a ring of n nodes
        auto gap = [](int a0, int a1, int b0, int b1, int n, bool per) {
            int best = 1 << 30;
            for (int sh = per ? -n : 0; sh <= (per ? n : 0); sh += n ? n : 1) {
                const int c0 = b0 + sh, c1 = b1 + sh;
                const int g = c0 >= a1 ? c0 - a1 + 1 : (a0 >= c1 ? a0 - c1 + 1 : 0);
                best = std::min(best, g);
                if (!per) break;
            }
            return best;
        };
        // the first launch covers every tile with a node within the
        // one-step reach of a rest tile (two tiles around suffice: tiles are
        // at least that reach wide, the ragged last one aside)
        for (int ty = 0; ty < nby; ++ty)
            for (int tx = 0; tx < nbx; ++tx) {
                if (!rest[(size_t)ty * nbx + tx]) continue;
                const int ax0 = tx * tw, ax1 = std::min(nx, ax0 + tw), ay0 = ty * th, ay1 = std::min(ny, ay0 + th);
                for (int dy = -2; dy <= 2; ++dy)
                    for (int dx = -2; dx <= 2; ++dx) {
                        int ux = tx + dx, uy = ty + dy;
                        if (ux < 0 || ux >= nbx) {
                            if (!perx) continue;
                            ux = (ux % nbx + nbx) % nbx;
                        }
                        if (uy < 0 || uy >= nby) {
                            if (!pery) continue;
                            uy = (uy % nby + nby) % nby;
                        }
                        const int bx0 = ux * tw, bx1 = std::min(nx, bx0 + tw);
                        const int by0 = uy * th, by1 = std::min(ny, by0 + th);
                        if (gap(ax0, ax1, bx0, bx1, nx, perx) <= mg && gap(ay0, ay1, by0, by1, ny, pery) <= mg)
                            wide[(size_t)uy * nbx + ux] = 1;
                    }
            }
        for (size_t t = 0; t < tiles.size(); ++t) {
            if (wide[t] && (tiles[t] & TILE_MATERIAL)) tla.push_back((int)t);
            if (rest[t]) tlb.push_back((int)t);
        }
        if (list2.empty()) tla.clear(), tlb.clear();
    }
    hipError_t err = hipMemcpyAsync(h->ws + h->L.tiles, tiles.data(), tiles.size(), hipMemcpyHostToDevice,
                                    h->stream);
    auto up = [&](size_t off, const std::vector<int> &v) {
        if (!err && !v.empty())
            err = hipMemcpyAsync(h->ws + off, v.data(), sizeof(int) * v.size(), hipMemcpyHostToDevice, h->stream);
    };
    up(h->L.flist, list);
    up(h->L.tlist, tl);
    up(h->L.flist2, list2);
    up(h->L.tlist_a, tla);
    up(h->L.tlist_b, tlb);
    if (!err) err = hipStreamSynchronize(h->stream);
    if (err) return err;
    h->n_flist = (int)(list.size() / 3);
    h->n_tlist = (int)tl.size();
    h->n_flist2 = (int)(list2.size() / 3);
    h->n_tlist_a = (int)tla.size();
    h->n_tlist_b = (int)tlb.size();
    h->tables_built = true;
    h->tables_dirty = false;
    return hipSuccess;
}

}  // namespace

lbm_status lbm_step(lbm_solver *h, int64_t nsteps)
{
    if (!h) return LBM_ERR_ARG;
    if (nsteps < 0) return fail(h, LBM_ERR_ARG, "nsteps < 0");
    if (!h->fields) return fail(h, LBM_ERR_STATE, "set the fields before stepping");
    StepParams sp{};
    sp.nx = h->nx;
    sp.ny = h->ny;
    sp.plane = (long long)h->nx * h->ny;
    fill_physics(sp, h->units(), h->tau, h->body, h->bc[LBM_EDGE_YMIN], h->bcval[LBM_EDGE_YMIN],
                 h->bc[LBM_EDGE_YMAX], h->bcval[LBM_EDGE_YMAX]);
    for (int a = 0; a < 2; ++a) {
        sp.uwb_lo[a] = h->uwb[LBM_EDGE_YMIN][a];
        sp.uwb_hi[a] = h->uwb[LBM_EDGE_YMAX][a];
    }
    sp.f_scale = h->f_scale;
    sp.f_inv_scale = 1.0 / h->f_scale;
    sp.strip_w = h->shape.strip_w;
    sp.halo_a = h->shape.halo_a;
    sp.n_strips = h->shape.n_strips;
    sp.n_segs = h->shape.n_segs;
    sp.flag = h->flag();
    sp.sr = h->sr;
    sp.seed = h->seed;
    const int nblocks = h->shape.n_strips * h->shape.n_segs;
    const bool pc = h->scheme == LBM_SCHEME_PC;
    if (h->general()) {
        GenParams gp{};
        gp.nx = h->nx;
        gp.ny = h->ny;
        gp.plane = sp.plane;
        gp.omega = sp.omega;
        gp.lam = sp.lam;
        gp.mu = sp.mu;
        gp.bx = sp.bx;
        gp.by = sp.by;
        const Units U = h->units();
        for (int e = 0; e < 4; ++e) {
            gp.bc[e] = h->bc[e];
            for (int a = 0; a < 2; ++a) {  // j* -> lattice momentum, T* -> lattice stress
                gp.val[e][a] = h->bc[e] == LBM_BC_DIRICHLET_J ? h->bcval[e][a] / U.momentum()
                                                              : h->bcval[e][a] / U.stress();
                gp.uwb[e][a] = h->uwb[e][a];
            }
        }
        gp.f_scale = sp.f_scale;
        gp.f_inv_scale = sp.f_inv_scale;
        gp.sr = sp.sr;
        gp.seed = sp.seed;
        gp.pc = h->scheme == LBM_SCHEME_EXTRAP ? 2 : (pc ? 1 : 0);
        gp.flag = sp.flag;
        gp.mask = h->mask_ptr();
        if (h->tables_dirty && h->ws_bytes >= h->L.total_walled) HIP_TRY(h, build_general_tables(h));
        gp.tiles = h->tiles_ptr();
        // without holes and without a fused share the table marks every
        // tile as material and nothing else: go without it, so that small
        // plates may take the two-row tiles
        if (gp.tiles && !h->has_mask && h->n_flist == 0 && h->n_flist2 == 0) gp.tiles = nullptr;
        gp.tlist = gp.tiles ? reinterpret_cast<const int *>(h->ws + h->L.tlist) : nullptr;
        gp.n_tlist = gp.tiles ? h->n_tlist : 0;
        // the fused kernel's share: the tiles clear of walls and holes (on
        // the handle's stream, the 2D tiles beside it on the aux stream)
        const int nf = gp.tiles ? h->n_flist : 0;
        if ((nf > 0 || (gp.tiles && h->n_flist2 > 0)) && !h->aux) {
            HIP_TRY(h, hipStreamCreateWithFlags(&h->aux, hipStreamNonBlocking));
            HIP_TRY(h, hipEventCreateWithFlags(&h->fork, hipEventDisableTiming));
            HIP_TRY(h, hipEventCreateWithFlags(&h->join, hipEventDisableTiming));
        }
        const int *flist = reinterpret_cast<const int *>(h->ws + h->L.flist);
        StepParams fp = sp;
        fp.strip_w = h->fshape.strip_w;
        fp.halo_a = h->fshape.halo_a;
        fp.n_strips = h->fshape.n_strips;
        fp.x_lo = h->fshape.x_lo;
        fp.x_end = h->fshape.x_end;
        fp.n_segs = 1;
        fp.bc_lo = fp.bc_hi = BC_PERIODIC;  // the fused share is clear of y walls: periodic form
        int64_t k = 0;
        // paired steps: the two-step fused kernel on the handle's stream; on
        // the aux stream the 2D tiles' first step (widened rest) into the
        // third state copy, then their second step (rest) from it. The fused
        // grid is one wave of resident blocks, so it is enqueued first: tile
        // blocks holding compute units when it dispatches would push part of
        // it into a second wave (0.86 against 0.49 ms per pair on the 4096²
        // plate with a hole).
        const int nf2 = gp.tiles ? h->n_flist2 : 0;
        if (nf2 > 0) {
            const int *flist2 = reinterpret_cast<const int *>(h->ws + h->L.flist2);
            StepParams fp2 = sp;
            fp2.strip_w = h->fshape2.strip_w;
            fp2.halo_a = h->fshape2.halo_a;
            fp2.n_strips = h->fshape2.n_strips;
            fp2.x_lo = h->fshape2.x_lo;
            fp2.x_end = h->fshape2.x_end;
            fp2.n_segs = 1;
            fp2.bc_lo = fp2.bc_hi = BC_PERIODIC;
            GenParams ga = gp, gb = gp;
            ga.tlist = reinterpret_cast<const int *>(h->ws + h->L.tlist_a);
            ga.n_tlist = h->n_tlist_a;
            gb.tlist = reinterpret_cast<const int *>(h->ws + h->L.tlist_b);
            gb.n_tlist = h->n_tlist_b;
            ga.f_out = h->ws + h->L.mid_f;
            ga.u_out = h->ws + h->L.mid_u;
            ga.j_out = h->ws + h->L.mid_j;
            gb.f_in = ga.f_out;
            gb.u_in = ga.u_out;
            gb.j_in = ga.j_out;
            for (; k + 2 <= nsteps; k += 2) {
                fp2.f_in = ga.f_in = h->fptr(h->cur);
                fp2.u_in = ga.u_in = h->uptr(h->cur);
                fp2.j_in = ga.j_in = h->jptr(h->cur);
                fp2.f_out = gb.f_out = h->fptr(h->cur ^ 1);
                fp2.u_out = gb.u_out = h->uptr(h->cur ^ 1);
                fp2.j_out = gb.j_out = h->jptr(h->cur ^ 1);
                fp2.step = ga.step = h->steps;
                gb.step = h->steps + 1;
                HIP_TRY(h, hipEventRecord(h->fork, h->stream));
                HIP_TRY(h, hipStreamWaitEvent(h->aux, h->fork, 0));
                HIP_TRY(h, LBM_DISPATCH(h->prec, Kernels<PR>::step2_list(fp2, flist2, nf2, h->stream)));
                HIP_TRY(h, LBM_DISPATCH(h->prec, general_step<PR>(ga, h->ws + h->L.scratch, h->aux)));
                HIP_TRY(h, LBM_DISPATCH(h->prec, general_step<PR>(gb, h->ws + h->L.scratch, h->aux)));
                HIP_TRY(h, hipEventRecord(h->join, h->aux));
                HIP_TRY(h, hipStreamWaitEvent(h->stream, h->join, 0));
                h->cur ^= 1;
                h->steps += 2;
            }
        }
        for (; k < nsteps; ++k) {
            gp.f_in = fp.f_in = h->fptr(h->cur);
            gp.u_in = fp.u_in = h->uptr(h->cur);
            gp.j_in = fp.j_in = h->jptr(h->cur);
            gp.f_out = fp.f_out = h->fptr(h->cur ^ 1);
            gp.u_out = fp.u_out = h->uptr(h->cur ^ 1);
            gp.j_out = fp.j_out = h->jptr(h->cur ^ 1);
            gp.step = fp.step = h->steps;
            if (nf > 0) {
                HIP_TRY(h, hipEventRecord(h->fork, h->stream));
                HIP_TRY(h, hipStreamWaitEvent(h->aux, h->fork, 0));
                HIP_TRY(h, LBM_DISPATCH(h->prec, Kernels<PR>::step_list(fp, flist, nf, pc, h->stream)));
                HIP_TRY(h, LBM_DISPATCH(h->prec, general_step<PR>(gp, h->ws + h->L.scratch, h->aux)));
                HIP_TRY(h, hipEventRecord(h->join, h->aux));
                HIP_TRY(h, hipStreamWaitEvent(h->stream, h->join, 0));
            } else {
                HIP_TRY(h, LBM_DISPATCH(h->prec, general_step<PR>(gp, h->ws + h->L.scratch, h->stream)));
            }
            h->cur ^= 1;
            h->steps += 1;
        }
        return LBM_OK;
    }
    int64_t k = 0;
    if (h->spl == 2) {
        for (; k + 2 <= nsteps; k += 2) {
            sp.f_in = h->fptr(h->cur);
            sp.u_in = h->uptr(h->cur);
            sp.j_in = h->jptr(h->cur);
            sp.f_out = h->fptr(h->cur ^ 1);
            sp.u_out = h->uptr(h->cur ^ 1);
            sp.j_out = h->jptr(h->cur ^ 1);
            sp.step = h->steps;
            HIP_TRY(h, LBM_DISPATCH(h->prec, Kernels<PR>::step2(sp, h->shape.block, nblocks, h->stream)));
            h->cur ^= 1;
            h->steps += 2;
        }
    }
    for (; k < nsteps; ++k) {
        sp.f_in = h->fptr(h->cur);
        sp.u_in = h->uptr(h->cur);
        sp.j_in = h->jptr(h->cur);
        sp.f_out = h->fptr(h->cur ^ 1);
        sp.u_out = h->uptr(h->cur ^ 1);
        sp.j_out = h->jptr(h->cur ^ 1);
        sp.step = h->steps;
        HIP_TRY(h, LBM_DISPATCH(h->prec, Kernels<PR>::step(sp, h->shape.block, nblocks, pc, h->stream)));
        h->cur ^= 1;
        h->steps += 1;
    }
    return LBM_OK;
}

lbm_status lbm_read_fields(lbm_solver *h, double *u, double *v, double *P, lbm_diagnostics *d)
{
    if (!h) return LBM_ERR_ARG;
    if (!h->fields) return fail(h, LBM_ERR_STATE, "no fields set");
    double out[7] = {0, 0, 0, 0, 0, 0, 0};
    const hipError_t e = plate_read(h->io(), (double)h->steps, u, v, P, d ? out : nullptr);
    if (e != hipSuccess) return hip_fail(h, e, "read-out");
    unsigned flag = 0;
    HIP_TRY(h, hipMemcpyAsync(&flag, h->flag(), sizeof(unsigned), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    if (d) {
        d->momentum[0] = out[0];
        d->momentum[1] = out[1];
        d->mass_moment = out[2];
        d->energy = out[3];
        d->min_J = out[4];
        d->max_strain = out[5];
        d->unstable = (out[6] != 0.0 || flag != 0) ? 1 : 0;
        d->reserved = 0;
        d->steps = h->steps;
    }
    if (flag != 0) return fail(h, LBM_ERR_UNSTABLE, "J <= 0 or a non-finite value appeared");
    return LBM_OK;
}

namespace {

// Device address of `scratch` on each device, looked up once per device with
// that device current (the array's name is a host-side stand-in, not the
// device address).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double *g_scratch_ptr[kMaxDevices] = {};

hipError_t device_scratch(int dev, double **out)
{
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = static_cast<double *>(p);
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace

lbm_status lbm_read_diagnostics_noalloc(lbm_solver *h, lbm_diagnostics *d)
{
    if (!h) return LBM_ERR_ARG;
    if (!d) return fail(h, LBM_ERR_ARG, "d is NULL");
    if (!h->fields) return fail(h, LBM_ERR_STATE, "no fields set");
    // the diagnostics grid is capped at kMaxDiagBlocks blocks
    const size_t n = (size_t)h->nx * h->ny;
    const size_t nblocks = std::min<size_t>(kMaxDiagBlocks, (n + 255) / 256);
    if (nblocks * 8 + 8 > kNoAllocDiagDoubles)
        return fail(h, LBM_ERR_UNSUPPORTED, "diagnostics need more scratch than the static array holds");
    int cur = 0;
    HIP_TRY(h, hipGetDevice(&cur));
    if (cur != h->device) HIP_TRY(h, hipSetDevice(h->device));
    double *sp = nullptr;
    hipError_t e = device_scratch(h->device, &sp);
    double out[7] = {0, 0, 0, 0, 0, 0, 0};
    unsigned flag = 0;
    if (e == hipSuccess) {
        PlateIO io = h->io();
        io.partials = sp;
        io.diag_out = sp + (size_t)kMaxDiagBlocks * 8;
        e = plate_read(io, (double)h->steps, nullptr, nullptr, nullptr, out);
    }
    if (e == hipSuccess) e = hipMemcpyAsync(&flag, h->flag(), sizeof(unsigned), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (cur != h->device) {
        const hipError_t e2 = hipSetDevice(cur);
        if (e == hipSuccess) e = e2;
    }
    if (e != hipSuccess) return hip_fail(h, e, "diagnostics");
    d->momentum[0] = out[0];
    d->momentum[1] = out[1];
    d->mass_moment = out[2];
    d->energy = out[3];
    d->min_J = out[4];
    d->max_strain = out[5];
    d->unstable = (out[6] != 0.0 || flag != 0) ? 1 : 0;
    d->reserved = 0;
    d->steps = h->steps;
    if (flag != 0) return fail(h, LBM_ERR_UNSTABLE, "J <= 0 or a non-finite value appeared");
    return LBM_OK;
}

lbm_status lbm_read_derived(lbm_solver *h, double *sigma, double *E, double *W)
{
    if (!h) return LBM_ERR_ARG;
    if (!h->fields) return fail(h, LBM_ERR_STATE, "no fields set");
    const hipError_t e = plate_read_derived(h->io(), (double)h->steps, sigma, E, W);
    if (e != hipSuccess) return hip_fail(h, e, "read-out");
    return LBM_OK;
}

lbm_status lbm_sample(lbm_solver *h, int n, const int *x, const int *y, double *out)
{
    if (!h) return LBM_ERR_ARG;
    if (!h->fields) return fail(h, LBM_ERR_STATE, "no fields set");
    if (n < 0 || (n > 0 && (!x || !y || !out))) return fail(h, LBM_ERR_ARG, "invalid node list");
    const PlateIO io = h->io();
    if (n > sample_capacity(io)) return fail(h, LBM_ERR_ARG, "too many nodes for one call");
    for (int k = 0; k < n; ++k)
        if (x[k] < 0 || x[k] >= h->nx || y[k] < 0 || y[k] >= h->ny) return fail(h, LBM_ERR_ARG, "node outside the plate");
    const hipError_t e = plate_sample(io, (double)h->steps, n, x, y, out);
    if (e != hipSuccess) return hip_fail(h, e, "sample");
    return LBM_OK;
}

void lbm_destroy(lbm_solver *h) { delete h; }

const char *lbm_last_error(const lbm_solver *h) { return h ? h->err.c_str() : g_create_error.c_str(); }

}  // extern "C"
