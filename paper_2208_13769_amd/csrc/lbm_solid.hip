// lbm_solid.hip -- host runtime and C ABI (include/lbm_solid.h).
//
// A handle owns no device memory: the caller's workspace is carved into two
// copies of the state (ping-pong), a read-out staging area, reduction
// scratch and a flag word. lbm_step only enqueues kernels on the caller's
// stream.
#include "../../include/lbm_solid.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "aux_kernels.hpp"
#include "step_kernel.hpp"

using namespace lbm;

namespace {

constexpr size_t kAlign = 256;
constexpr int kMaxDiagBlocks = 1024;
constexpr size_t kStagingCap = size_t(16) << 20;  // bytes of read-out staging at most

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Sizes {
    size_t f, u, j;  // bytes per element
};

Sizes elem_sizes(lbm_precision p)
{
    switch (p) {
    case LBM_FP64: return {8, 8, 8};
    case LBM_FP32: return {4, 4, 4};
    case LBM_FP16_STORE:
    case LBM_BF16_STORE: return {2, 8, 4};
    }
    return {0, 0, 0};
}

struct Layout {
    size_t f[2], u[2], j[2];
    size_t staging, staging_bytes;
    size_t partials, small, total;
};

Layout make_layout(int nx, int ny, lbm_precision p)
{
    Layout L{};
    const Sizes s = elem_sizes(p);
    const size_t n = (size_t)nx * ny;
    size_t off = 0;
    for (int c = 0; c < 2; ++c) {
        L.f[c] = off;
        off = align_up(off + 9 * n * s.f);
        L.u[c] = off;
        off = align_up(off + 2 * n * s.u);
        L.j[c] = off;
        off = align_up(off + 2 * n * s.j);
    }
    L.staging = off;
    L.staging_bytes = std::min(8 * n * sizeof(double), std::max(kStagingCap, 8 * (size_t)nx * sizeof(double)));
    off = align_up(off + L.staging_bytes);
    L.partials = off;
    off = align_up(off + kMaxDiagBlocks * 8 * sizeof(double));
    L.small = off;  // flag word + final diagnostics + max |f|
    off = align_up(off + 64 * sizeof(double));
    L.total = off;
    return L;
}

bool valid_precision(int p) { return p >= LBM_FP64 && p <= LBM_BF16_STORE; }

}  // namespace

struct lbm_solver {
    int nx = 0, ny = 0;
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
    double f_scale = 1.0;
    int64_t steps = 0;
    int block = 256, strip_w = 0, n_strips = 0, n_segs = 0, halo_a = 0;
    std::string err;

    void *fptr(int c) const { return ws + L.f[c]; }
    void *uptr(int c) const { return ws + L.u[c]; }
    void *jptr(int c) const { return ws + L.j[c]; }
    double *staging() const { return reinterpret_cast<double *>(ws + L.staging); }
    double *partials() const { return reinterpret_cast<double *>(ws + L.partials); }
    unsigned *flag() const { return reinterpret_cast<unsigned *>(ws + L.small); }
    double *diag_out() const { return reinterpret_cast<double *>(ws + L.small + 64); }
    double dt() const { return dx / (std::sqrt(3.0) * std::sqrt(mu / rho0)); }
    double c() const { return dx / dt(); }
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

#define HIP_TRY(h, call)                                   \
    do {                                                   \
        hipError_t e_ = (call);                            \
        if (e_ != hipSuccess) return hip_fail(h, e_, #call); \
    } while (0)

FieldParams field_params(const lbm_solver *h, double t_steps)
{
    FieldParams fp{};
    fp.nx = h->nx;
    fp.ny = h->ny;
    fp.plane = (long long)h->nx * h->ny;
    fp.bc_lo = h->bc[LBM_EDGE_YMIN];
    fp.bc_hi = h->bc[LBM_EDGE_YMAX];
    const double jl = 1.0 / (h->rho0 * h->c());
    for (int a = 0; a < 2; ++a) {
        fp.uw_lo[a] = fp.bc_lo == LBM_BC_DIRICHLET_J ? h->bcval[LBM_EDGE_YMIN][a] * jl * t_steps : 0.0;
        fp.uw_hi[a] = fp.bc_hi == LBM_BC_DIRICHLET_J ? h->bcval[LBM_EDGE_YMAX][a] * jl * t_steps : 0.0;
    }
    const double sl = 1.0 / (h->rho0 * h->c() * h->c());
    fp.lam = h->lam * sl;
    fp.mu = h->mu * sl;
    return fp;
}

// ---------------------------------------------------------------- dispatch

template <class PR>
struct Kernels {
    template <int B, bool PC>
    static void step_w(const StepParams &sp, int nblocks, hipStream_t st)
    {
        if (sp.bc_lo != BC_PERIODIC)
            hipLaunchKernelGGL((step_kernel<PR, B, PC, true>), dim3(nblocks), dim3(B), 0, st, sp);
        else
            hipLaunchKernelGGL((step_kernel<PR, B, PC, false>), dim3(nblocks), dim3(B), 0, st, sp);
    }
    template <int B>
    static hipError_t step_b(const StepParams &sp, int nblocks, bool pc, hipStream_t st)
    {
        if (pc)
            step_w<B, true>(sp, nblocks, st);
        else
            step_w<B, false>(sp, nblocks, st);
        return hipGetLastError();
    }
    static hipError_t step(const StepParams &sp, int block, int nblocks, bool pc, hipStream_t st)
    {
        switch (block) {
        case 64: return step_b<64>(sp, nblocks, pc, st);
        case 128: return step_b<128>(sp, nblocks, pc, st);
        case 512: return step_b<512>(sp, nblocks, pc, st);
        default: return step_b<256>(sp, nblocks, pc, st);
        }
    }
    static hipError_t init(const InitParams &ip, int nblocks, hipStream_t st)
    {
        hipLaunchKernelGGL((init_kernel<PR>), dim3(nblocks), dim3(256), 0, st, ip);
        return hipGetLastError();
    }
    static hipError_t readout(const ReadParams &rp, int nblocks, hipStream_t st)
    {
        hipLaunchKernelGGL((readout_kernel<PR>), dim3(nblocks), dim3(256), 0, st, rp);
        return hipGetLastError();
    }
    static hipError_t diag(const DiagParams &dp, int nblocks, hipStream_t st)
    {
        hipLaunchKernelGGL((diag_kernel<PR>), dim3(nblocks), dim3(256), 0, st, dp);
        return hipGetLastError();
    }
};

#define LBM_DISPATCH(prec, expr_with_PR)                         \
    [&]() -> hipError_t {                                        \
        switch (prec) {                                          \
        case LBM_FP64: { using PR = PrecF64; return expr_with_PR; } \
        case LBM_FP32: { using PR = PrecF32; return expr_with_PR; } \
        case LBM_FP16_STORE: { using PR = PrecF16; return expr_with_PR; } \
        default: { using PR = PrecBF16; return expr_with_PR; }   \
        }                                                        \
    }()

int halo_of(const lbm_solver *h) { return h->scheme == LBM_SCHEME_PC ? 5 : 3; }

// Column strips: when the plate is wider than one block's reach, each
// strip's output width is a multiple of 128 bytes of the population type
// (32 floats / doubles, 64 halves), so no cache line is written by two
// blocks; the spare threads of the block extend the halo.
void set_shape(lbm_solver *h, int block, int n_segs)
{
    const int halo = halo_of(h);
    const int wmax = block - 2 * halo;
    const int align = (h->prec == LBM_FP16_STORE || h->prec == LBM_BF16_STORE) ? 64 : 32;
    int strip_w, n_strips, halo_a;
    if (h->nx <= wmax) {
        strip_w = h->nx;
        n_strips = 1;
        halo_a = halo;
    } else {
        strip_w = wmax >= align ? wmax / align * align : wmax;
        n_strips = (h->nx + strip_w - 1) / strip_w;
        halo_a = (block - strip_w) / 2;
    }
    h->block = block;
    h->n_strips = n_strips;
    h->strip_w = strip_w;
    h->halo_a = halo_a;
    h->n_segs = n_segs;
}

void plan_launch(lbm_solver *h)
{
    const int halo = halo_of(h);
    // narrowest block whose strip covers the width, else 256 threads
    int block = 256;
    if (h->nx <= 64 - 2 * halo)
        block = 64;
    else if (h->nx <= 128 - 2 * halo)
        block = 128;
    const int wmax = block - 2 * halo;
    const int n_strips = (h->nx + wmax - 1) / wmax;
    // enough blocks to fill 256 CUs a few times over, segments of >= 16 rows
    const int target = 2048;
    int n_segs = (target + n_strips - 1) / n_strips;
    n_segs = std::max(1, std::min(n_segs, h->ny / 16));
    set_shape(h, block, n_segs);
}

}  // namespace

extern "C" {

size_t lbm_workspace_bytes(int nx, int ny, lbm_precision p)
{
    if (nx < 5 || ny < 5 || !valid_precision(p)) return 0;
    return make_layout(nx, ny, p).total;
}

lbm_status lbm_create(int nx, int ny, double dx, lbm_precision p, lbm_scheme s, void *dev_workspace,
                      size_t ws_bytes, void *hip_stream, lbm_solver **out)
{
    if (!out) return fail(nullptr, LBM_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (nx < 5 || ny < 5) return fail(nullptr, LBM_ERR_ARG, "nx and ny must be >= 5");
    if (!(dx > 0.0) || !std::isfinite(dx)) return fail(nullptr, LBM_ERR_ARG, "dx must be positive");
    if (!valid_precision(p)) return fail(nullptr, LBM_ERR_ARG, "unknown precision");
    if (s != LBM_SCHEME_PC && s != LBM_SCHEME_EXPLICIT) return fail(nullptr, LBM_ERR_ARG, "unknown scheme");
    if (!dev_workspace) return fail(nullptr, LBM_ERR_ARG, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(dev_workspace) % kAlign) return fail(nullptr, LBM_ERR_ARG, "workspace not 256-byte aligned");
    if ((long long)nx * ny > (1LL << 31)) return fail(nullptr, LBM_ERR_UNSUPPORTED, "more than 2^31 sites");
    const Layout L = make_layout(nx, ny, p);
    if (ws_bytes < L.total) return fail(nullptr, LBM_ERR_NOMEM, "workspace smaller than lbm_workspace_bytes()");
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
    h->rho0 = rho0;
    h->lam = lambda;
    h->mu = mu;
    h->tau = tau_over_dt;
    h->material = true;
    return LBM_OK;
}

lbm_status lbm_set_body_force(lbm_solver *h, const double b[2])
{
    if (!h || !b) return fail(h, LBM_ERR_ARG, "NULL argument");
    if (!std::isfinite(b[0]) || !std::isfinite(b[1])) return fail(h, LBM_ERR_ARG, "body force not finite");
    h->body[0] = b[0];
    h->body[1] = b[1];
    return LBM_OK;
}

lbm_status lbm_set_boundary(lbm_solver *h, lbm_edge e, lbm_bc bc, const double value[2])
{
    if (!h) return LBM_ERR_ARG;
    if (e < LBM_EDGE_XMIN || e > LBM_EDGE_YMAX) return fail(h, LBM_ERR_ARG, "unknown edge");
    if (bc < LBM_BC_PERIODIC || bc > LBM_BC_NEUMANN_T) return fail(h, LBM_ERR_ARG, "unknown boundary rule");
    if ((e == LBM_EDGE_XMIN || e == LBM_EDGE_XMAX) && bc != LBM_BC_PERIODIC)
        return fail(h, LBM_ERR_UNSUPPORTED, "x edges are periodic in this build");
    if (bc != LBM_BC_PERIODIC && (!value || !std::isfinite(value[0]) || !std::isfinite(value[1])))
        return fail(h, LBM_ERR_ARG, "boundary value missing or not finite");
    const int other = e == LBM_EDGE_YMIN ? LBM_EDGE_YMAX : e == LBM_EDGE_YMAX ? LBM_EDGE_YMIN : e ^ 1;
    if (bc == LBM_BC_PERIODIC && h->bc[other] != LBM_BC_PERIODIC && (e == LBM_EDGE_YMIN || e == LBM_EDGE_YMAX)) {
        // setting one y edge back to periodic also needs the other one; accept and pair them
        h->bc[other] = LBM_BC_PERIODIC;
    }
    if (bc != LBM_BC_PERIODIC && h->bc[other] == LBM_BC_PERIODIC && (e == LBM_EDGE_YMIN || e == LBM_EDGE_YMAX)) {
        // the opposite edge stops being periodic: it becomes a wall at rest until set
        h->bc[other] = LBM_BC_DIRICHLET_J;
        h->bcval[other][0] = h->bcval[other][1] = 0.0;
    }
    h->bc[e] = bc;
    h->bcval[e][0] = bc == LBM_BC_PERIODIC ? 0.0 : value[0];
    h->bcval[e][1] = bc == LBM_BC_PERIODIC ? 0.0 : value[1];
    return LBM_OK;
}

lbm_status lbm_set_tiling(lbm_solver *h, int block, int n_segs)
{
    if (!h) return LBM_ERR_ARG;
    if (block != 64 && block != 128 && block != 256 && block != 512)
        return fail(h, LBM_ERR_ARG, "block must be 64, 128, 256 or 512");
    if (n_segs < 1 || n_segs > h->ny) return fail(h, LBM_ERR_ARG, "n_segs must be in [1, ny]");
    if ((long long)h->nx * n_segs > (1LL << 30)) return fail(h, LBM_ERR_ARG, "too many blocks");
    set_shape(h, block, n_segs);
    return LBM_OK;
}

lbm_status lbm_get_tiling(const lbm_solver *h, int *block, int *n_segs)
{
    if (!h || !block || !n_segs) return LBM_ERR_ARG;
    *block = h->block;
    *n_segs = h->n_segs;
    return LBM_OK;
}

lbm_status lbm_get_dt(const lbm_solver *h, double *dt)
{
    if (!h || !dt) return LBM_ERR_ARG;
    if (!h->material) return LBM_ERR_STATE;
    *dt = h->dt();
    return LBM_OK;
}

lbm_status lbm_set_fields(lbm_solver *h, const double *u0, const double *v0)
{
    if (!h) return LBM_ERR_ARG;
    if (!u0 || !v0) return fail(h, LBM_ERR_ARG, "u0 or v0 is NULL");
    if (!h->material) return fail(h, LBM_ERR_STATE, "set the material before the fields");
    const size_t n = (size_t)h->nx * h->ny;
    // stage u0, v0 (FP64) in the second state copy, which is at least 32 bytes per site
    double *su = reinterpret_cast<double *>(h->fptr(1));
    double *sv = su + 2 * n;
    HIP_TRY(h, hipMemcpyAsync(su, u0, 2 * n * sizeof(double), hipMemcpyHostToDevice, h->stream));
    HIP_TRY(h, hipMemcpyAsync(sv, v0, 2 * n * sizeof(double), hipMemcpyHostToDevice, h->stream));
    InitParams ip{};
    ip.fp = field_params(h, 0.0);
    ip.u0 = su;
    ip.v0 = sv;
    ip.f = h->fptr(0);
    ip.u = h->uptr(0);
    ip.j = h->jptr(0);
    ip.inv_dx = 1.0 / h->dx;
    ip.v_to_j = h->dt() / h->dx;
    ip.maxf = h->partials();
    const int nblocks = (int)((n + 255) / 256);
    h->f_scale = 1.0;
    if (h->prec == LBM_FP16_STORE || h->prec == LBM_BF16_STORE) {
        // power-of-two scale that puts max |f| near 2^12 (FP16 tops out at 65504)
        if (nblocks > (int)(h->L.staging_bytes / sizeof(double)))
            return fail(h, LBM_ERR_UNSUPPORTED, "plate too large for the start-up reduction");
        ip.mode = 0;
        ip.maxf = h->staging();
        HIP_TRY(h, LBM_DISPATCH(h->prec, Kernels<PR>::init(ip, nblocks, h->stream)));
        std::vector<double> m(nblocks);
        HIP_TRY(h, hipMemcpyAsync(m.data(), ip.maxf, nblocks * sizeof(double), hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(h, hipStreamSynchronize(h->stream));
        double mx = 0.0;
        for (double v : m) mx = std::max(mx, v);
        if (!std::isfinite(mx)) return fail(h, LBM_ERR_ARG, "initial fields not finite");
        if (mx > 0.0) h->f_scale = std::ldexp(1.0, (int)std::floor(std::log2(4096.0 / mx)));
    }
    ip.mode = 1;
    ip.f_scale = h->f_scale;
    HIP_TRY(h, LBM_DISPATCH(h->prec, Kernels<PR>::init(ip, nblocks, h->stream)));
    HIP_TRY(h, hipMemsetAsync(h->flag(), 0, sizeof(unsigned), h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    h->cur = 0;
    h->steps = 0;
    h->fields = true;
    return LBM_OK;
}

lbm_status lbm_step(lbm_solver *h, int64_t nsteps)
{
    if (!h) return LBM_ERR_ARG;
    if (nsteps < 0) return fail(h, LBM_ERR_ARG, "nsteps < 0");
    if (!h->fields) return fail(h, LBM_ERR_STATE, "set the fields before stepping");
    const double c = h->c();
    StepParams sp{};
    sp.nx = h->nx;
    sp.ny = h->ny;
    sp.plane = (long long)h->nx * h->ny;
    sp.omega = 1.0 / h->tau;
    const double sl = 1.0 / (h->rho0 * c * c);
    sp.lam = h->lam * sl;
    sp.mu = h->mu * sl;
    sp.bx = h->body[0] * h->dt() / c;
    sp.by = h->body[1] * h->dt() / c;
    sp.bc_lo = h->bc[LBM_EDGE_YMIN];
    sp.bc_hi = h->bc[LBM_EDGE_YMAX];
    for (int a = 0; a < 2; ++a) {
        const double lo = h->bcval[LBM_EDGE_YMIN][a], hi = h->bcval[LBM_EDGE_YMAX][a];
        // j* -> lattice momentum, T* -> lattice stress
        sp.val_lo[a] = sp.bc_lo == LBM_BC_DIRICHLET_J ? lo / (h->rho0 * c) : lo * sl;
        sp.val_hi[a] = sp.bc_hi == LBM_BC_DIRICHLET_J ? hi / (h->rho0 * c) : hi * sl;
    }
    sp.f_scale = h->f_scale;
    sp.f_inv_scale = 1.0 / h->f_scale;
    sp.strip_w = h->strip_w;
    sp.halo_a = h->halo_a;
    sp.n_strips = h->n_strips;
    sp.n_segs = h->n_segs;
    sp.flag = h->flag();
    const int nblocks = h->n_strips * h->n_segs;
    const bool pc = h->scheme == LBM_SCHEME_PC;
    for (int64_t k = 0; k < nsteps; ++k) {
        sp.f_in = h->fptr(h->cur);
        sp.u_in = h->uptr(h->cur);
        sp.j_in = h->jptr(h->cur);
        sp.f_out = h->fptr(h->cur ^ 1);
        sp.u_out = h->uptr(h->cur ^ 1);
        sp.j_out = h->jptr(h->cur ^ 1);
        sp.step = h->steps;
        HIP_TRY(h, LBM_DISPATCH(h->prec, Kernels<PR>::step(sp, h->block, nblocks, pc, h->stream)));
        h->cur ^= 1;
        h->steps += 1;
    }
    return LBM_OK;
}

lbm_status lbm_read_fields(lbm_solver *h, double *u, double *v, double *P, lbm_diagnostics *d)
{
    if (!h) return LBM_ERR_ARG;
    if (!h->fields) return fail(h, LBM_ERR_STATE, "no fields set");
    const int nx = h->nx, ny = h->ny;
    const size_t n = (size_t)nx * ny;
    const double c = h->c();
    if (u || v || P) {
        ReadParams rp{};
        rp.fp = field_params(h, (double)h->steps);
        rp.u = h->uptr(h->cur);
        rp.j = h->jptr(h->cur);
        rp.out = h->staging();
        rp.dx = h->dx;
        rp.c = c;
        rp.stress = h->rho0 * c * c;
        const int rows_per = (int)std::max<size_t>(1, std::min<size_t>(ny, h->L.staging_bytes / (8 * sizeof(double) * nx)));
        for (int y = 0; y < ny; y += rows_per) {
            const int rows = std::min(rows_per, ny - y);
            rp.y_begin = y;
            rp.rows = rows;
            const size_t cnt = (size_t)rows * nx;
            HIP_TRY(h, LBM_DISPATCH(h->prec, Kernels<PR>::readout(rp, (int)((cnt + 255) / 256), h->stream)));
            double *dst[8] = {u, u ? u + n : nullptr, v, v ? v + n : nullptr,
                              P, P ? P + n : nullptr, P ? P + 2 * n : nullptr, P ? P + 3 * n : nullptr};
            for (int k = 0; k < 8; ++k) {
                if (!dst[k]) continue;
                HIP_TRY(h, hipMemcpyAsync(dst[k] + (size_t)y * nx, rp.out + k * cnt, cnt * sizeof(double),
                                          hipMemcpyDeviceToHost, h->stream));
            }
            HIP_TRY(h, hipStreamSynchronize(h->stream));
        }
    }
    double out[7] = {0, 0, 0, 0, 0, 0, 0};
    if (d) {
        DiagParams dp{};
        dp.fp = field_params(h, (double)h->steps);
        dp.f = h->fptr(h->cur);
        dp.u = h->uptr(h->cur);
        dp.j = h->jptr(h->cur);
        dp.f_inv_scale = 1.0 / h->f_scale;
        dp.rho0 = h->rho0;
        dp.dx = h->dx;
        dp.c = c;
        dp.lam_phys = h->lam;
        dp.mu_phys = h->mu;
        dp.partials = h->partials();
        const int nblocks = (int)std::min<size_t>(kMaxDiagBlocks, (n + 255) / 256);
        HIP_TRY(h, LBM_DISPATCH(h->prec, Kernels<PR>::diag(dp, nblocks, h->stream)));
        hipLaunchKernelGGL(diag_final_kernel, dim3(1), dim3(64), 0, h->stream, h->partials(), nblocks, h->diag_out());
        HIP_TRY(h, hipGetLastError());
        HIP_TRY(h, hipMemcpyAsync(out, h->diag_out(), 7 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    }
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

void lbm_destroy(lbm_solver *h) { delete h; }

const char *lbm_last_error(const lbm_solver *h) { return h ? h->err.c_str() : g_create_error.c_str(); }

}  // extern "C"
