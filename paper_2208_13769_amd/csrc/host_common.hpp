// host_common.hpp -- host-side helpers shared by the single-plate and the
// batched runtimes: state layout, launch shape and unit conversion.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <string>
#include <vector>

#include "../../include/lbm_solid.h"
#include "aux_kernels.hpp"
#include "step_kernel.hpp"

namespace lbm {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct ElemSizes {
    size_t f, u, j;  // bytes per element
};

inline ElemSizes elem_sizes(lbm_precision p)
{
    switch (p) {
    case LBM_FP64: return {8, 8, 8};
    case LBM_FP32: return {4, 4, 4};
    case LBM_FP16_STORE:
    case LBM_BF16_STORE: return {2, 8, 4};
    case LBM_FP32_U64: return {4, 8, 4};
    }
    return {0, 0, 0};
}

inline bool valid_precision(int p) { return p >= LBM_FP64 && p <= LBM_FP32_U64; }

// Offsets of the two state copies (f, u, j) of one plate from its base.
struct StateLayout {
    size_t f[2], u[2], j[2];
    size_t bytes;  // total, 256-byte aligned
};

inline StateLayout state_layout(int nx, int ny, lbm_precision p)
{
    StateLayout L{};
    const ElemSizes s = elem_sizes(p);
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
    L.bytes = off;
    return L;
}

// 16-bit populations are stored as deviations from a reference equilibrium
// (lattice.hpp, ref_eq): the store waits for the new displacement's gradient,
// which needs one more halo row and column per step.
inline bool deviation_storage(lbm_precision p) { return p == LBM_FP16_STORE || p == LBM_BF16_STORE; }

// Most time steps one launch may fuse: two with the predictor-corrector,
// except with deviation storage (no two-step kernel).
inline int max_steps_per_launch(lbm_precision p, lbm_scheme s)
{
    return s == LBM_SCHEME_PC && !deviation_storage(p) ? 2 : 1;
}

// Columns (and rows) of halo a tile recomputes: the stencil reach of the
// steps it fuses.
inline int stencil_halo(lbm_precision p, lbm_scheme s, int steps_per_launch)
{
    return ((s == LBM_SCHEME_PC ? 5 : 3) + (deviation_storage(p) ? 1 : 0)) * steps_per_launch;
}

// Launch shape of one plate: column strips and row segments.
struct Shape {
    int block, strip_w, n_strips, n_segs, halo_a;
    int x_lo = 0, x_end = 0;  // strips over columns [x_lo, x_end) (x_end 0: the whole width)
};

// When the plate is wider than one block's reach, each strip's output width
// is a multiple of 32 columns: whole 128-byte lines of floats (two lines of
// doubles), so no line is written by two blocks; with 16-bit populations two
// blocks may write the two 64-byte halves of a line, which costs less than
// the halo columns a 64-column rule wastes. The spare threads of the block
// extend the halo.
inline Shape make_shape(int nx, int ny, lbm_precision p, lbm_scheme s, int block, int n_segs,
                        int steps_per_launch = 1)
{
    const int halo = stencil_halo(p, s, steps_per_launch);
    const int wmax = block - 2 * halo;
    const int align = 32;
    Shape sh{};
    sh.block = block;
    if (nx <= wmax) {
        sh.strip_w = nx;
        sh.n_strips = 1;
        sh.halo_a = halo;
    } else {
        sh.strip_w = wmax >= align ? wmax / align * align : wmax;
        sh.n_strips = (nx + sh.strip_w - 1) / sh.strip_w;
        sh.halo_a = (block - sh.strip_w) / 2;
    }
    sh.n_segs = std::max(1, std::min(n_segs, ny));
    return sh;
}

// Physical -> lattice units (dX = dt = rho0 = 1, c = dX/dt = sqrt(3 mu / rho0)).
struct Units {
    double dx, rho0, lam, mu;
    double dt() const { return dx / (std::sqrt(3.0) * std::sqrt(mu / rho0)); }
    double c() const { return dx / dt(); }
    double stress() const { return rho0 * c() * c(); }  // P = stress * P_L
    double momentum() const { return rho0 * c(); }     // j = momentum * j_L
};

// Material, body force and wall parameters of a step in lattice units.
inline void fill_physics(StepParams &sp, const Units &U, double tau_over_dt, const double body[2], int bc_lo,
                         const double val_lo[2], int bc_hi, const double val_hi[2])
{
    const double c = U.c(), sl = 1.0 / U.stress();
    sp.omega = 1.0 / tau_over_dt;
    sp.lam = U.lam * sl;
    sp.mu = U.mu * sl;
    sp.bx = body[0] * U.dt() / c;
    sp.by = body[1] * U.dt() / c;
    sp.bc_lo = bc_lo;
    sp.bc_hi = bc_hi;
    for (int a = 0; a < 2; ++a) {
        // j* -> lattice momentum, T* -> lattice stress
        sp.val_lo[a] = bc_lo == LBM_BC_DIRICHLET_J ? val_lo[a] / U.momentum() : val_lo[a] * sl;
        sp.val_hi[a] = bc_hi == LBM_BC_DIRICHLET_J ? val_hi[a] / U.momentum() : val_hi[a] * sl;
    }
}


// ---------------------------------------------------------------- launches

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
    // The two pipelines of a two-step block share one compute unit's 160 KiB
    // of LDS: a 512-thread block fits with 32-bit values only, or with a
    // double displacement on plates periodic in y.
    // (Deviation storage has no two-step kernel.)
    template <int B, bool W>
    static constexpr bool step2_fits()
    {
        return !FStore<typename PR::TF>::kDeviation && 2 * sizeof(TileLds<PR, B, true, W>) <= size_t(160) * 1024;
    }
    template <int B>
    static hipError_t step2_b(const StepParams &sp, int nblocks, hipStream_t st)
    {
        if (sp.bc_lo != BC_PERIODIC) {
            if constexpr (step2_fits<B, true>())
                hipLaunchKernelGGL((step2_kernel<PR, B, true>), dim3(nblocks), dim3(B), 0, st, sp);
            else
                return hipErrorInvalidConfiguration;
        } else {
            if constexpr (step2_fits<B, false>())
                hipLaunchKernelGGL((step2_kernel<PR, B, false>), dim3(nblocks), dim3(B), 0, st, sp);
            else
                return hipErrorInvalidConfiguration;
        }
        return hipGetLastError();
    }
    // blocks of one step-kernel instantiation that a compute unit holds at once
    template <typename K>
    static int per_cu(K kernel, int block)
    {
        int n = 0;
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, block, 0) == hipSuccess ? n : 0;
    }
    template <int B>
    static int resident_b(int spl, bool pc, bool walled)
    {
        if (spl == 2) {
            if (walled) {
                if constexpr (step2_fits<B, true>()) return per_cu(step2_kernel<PR, B, true>, B);
                return 0;
            }
            if constexpr (step2_fits<B, false>()) return per_cu(step2_kernel<PR, B, false>, B);
            return 0;
        }
        if (pc)
            return walled ? per_cu(step_kernel<PR, B, true, true>, B) : per_cu(step_kernel<PR, B, true, false>, B);
        return walled ? per_cu(step_kernel<PR, B, false, true>, B) : per_cu(step_kernel<PR, B, false, false>, B);
    }

    // The entry points below are defined out of the class (not inline), so
    // that each precision is instantiated in one object only.
    static hipError_t step(const StepParams &sp, int block, int nblocks, bool pc, hipStream_t st);
    // one step over a tile list (256 threads per block; sp's shape is the
    // 256-thread shape)
    static hipError_t step_list(const StepParams &sp, const int *list, int n, bool pc, hipStream_t st);
    // two predictor-corrector steps over a tile list (256 threads, the
    // two-step shape); hipErrorInvalidConfiguration where the block's LDS
    // does not fit
    static hipError_t step2_list(const StepParams &sp, const int *list, int n, hipStream_t st);
    // whether a two-step block of this many threads fits the LDS
    static bool step2_ok(int block, bool walled);
    // two predictor-corrector steps per launch
    static hipError_t step2(const StepParams &sp, int block, int nblocks, hipStream_t st);
    static int resident_per_cu(int block, int spl, bool pc, bool walled);
    static hipError_t init(const InitParams &ip, int nblocks, hipStream_t st);
    static hipError_t readout(const ReadParams &rp, int nblocks, hipStream_t st);
    static hipError_t diag(const DiagParams &dp, int nblocks, hipStream_t st);
};

template <class PR>
hipError_t Kernels<PR>::step(const StepParams &sp, int block, int nblocks, bool pc, hipStream_t st)
{
    switch (block) {
    case 64: return step_b<64>(sp, nblocks, pc, st);
    case 128: return step_b<128>(sp, nblocks, pc, st);
    case 512: return step_b<512>(sp, nblocks, pc, st);
    default: return step_b<256>(sp, nblocks, pc, st);
    }
}

template <class PR>
hipError_t Kernels<PR>::step_list(const StepParams &sp, const int *list, int n, bool pc, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const bool w = sp.bc_lo != BC_PERIODIC;
    if (pc) {
        if (w)
            hipLaunchKernelGGL((step_list_kernel<PR, 256, true, true>), dim3(n), dim3(256), 0, st, sp, list, n);
        else
            hipLaunchKernelGGL((step_list_kernel<PR, 256, true, false>), dim3(n), dim3(256), 0, st, sp, list, n);
    } else {
        if (w)
            hipLaunchKernelGGL((step_list_kernel<PR, 256, false, true>), dim3(n), dim3(256), 0, st, sp, list, n);
        else
            hipLaunchKernelGGL((step_list_kernel<PR, 256, false, false>), dim3(n), dim3(256), 0, st, sp, list, n);
    }
    return hipGetLastError();
}

template <class PR>
hipError_t Kernels<PR>::step2_list(const StepParams &sp, const int *list, int n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    if (sp.bc_lo != BC_PERIODIC) {
        if constexpr (step2_fits<256, true>())
            hipLaunchKernelGGL((step2_list_kernel<PR, 256, true>), dim3(n), dim3(256), 0, st, sp, list, n);
        else
            return hipErrorInvalidConfiguration;
    } else {
        if constexpr (step2_fits<256, false>())
            hipLaunchKernelGGL((step2_list_kernel<PR, 256, false>), dim3(n), dim3(256), 0, st, sp, list, n);
        else
            return hipErrorInvalidConfiguration;
    }
    return hipGetLastError();
}

template <class PR>
bool Kernels<PR>::step2_ok(int block, bool walled)
{
    switch (block) {
    case 64: return walled ? step2_fits<64, true>() : step2_fits<64, false>();
    case 128: return walled ? step2_fits<128, true>() : step2_fits<128, false>();
    case 256: return walled ? step2_fits<256, true>() : step2_fits<256, false>();
    case 512: return walled ? step2_fits<512, true>() : step2_fits<512, false>();
    default: return false;
    }
}

template <class PR>
hipError_t Kernels<PR>::step2(const StepParams &sp, int block, int nblocks, hipStream_t st)
{
    switch (block) {
    case 64: return step2_b<64>(sp, nblocks, st);
    case 128: return step2_b<128>(sp, nblocks, st);
    case 256: return step2_b<256>(sp, nblocks, st);
    case 512: return step2_b<512>(sp, nblocks, st);
    default: return hipErrorInvalidConfiguration;
    }
}

template <class PR>
int Kernels<PR>::resident_per_cu(int block, int spl, bool pc, bool walled)
{
    switch (block) {
    case 64: return resident_b<64>(spl, pc, walled);
    case 128: return resident_b<128>(spl, pc, walled);
    case 256: return resident_b<256>(spl, pc, walled);
    default: return resident_b<512>(spl, pc, walled);
    }
}

template <class PR>
hipError_t Kernels<PR>::init(const InitParams &ip, int nblocks, hipStream_t st)
{
    hipLaunchKernelGGL((init_kernel<PR>), dim3(nblocks), dim3(256), 0, st, ip);
    return hipGetLastError();
}

template <class PR>
hipError_t Kernels<PR>::readout(const ReadParams &rp, int nblocks, hipStream_t st)
{
    hipLaunchKernelGGL((readout_kernel<PR>), dim3(nblocks), dim3(256), 0, st, rp);
    return hipGetLastError();
}

template <class PR>
hipError_t Kernels<PR>::diag(const DiagParams &dp, int nblocks, hipStream_t st)
{
    hipLaunchKernelGGL((diag_kernel<PR>), dim3(nblocks), dim3(256), 0, st, dp);
    return hipGetLastError();
}

// Each precision's kernels and launch helpers are compiled in an object of
// their own (instantiate.hip), so the precisions build in parallel.
extern template struct Kernels<PrecF64>;
extern template struct Kernels<PrecF32>;
extern template struct Kernels<PrecF32U64>;
extern template struct Kernels<PrecF16>;
extern template struct Kernels<PrecBF16>;

#define LBM_DISPATCH(prec, expr_with_PR)                                  \
    [&]() -> hipError_t {                                                 \
        switch (prec) {                                                   \
        case LBM_FP64: { using PR = PrecF64; return expr_with_PR; }        \
        case LBM_FP32: { using PR = PrecF32; return expr_with_PR; }        \
        case LBM_FP16_STORE: { using PR = PrecF16; return expr_with_PR; }  \
        case LBM_FP32_U64: { using PR = PrecF32U64; return expr_with_PR; } \
        default: { using PR = PrecBF16; return expr_with_PR; }            \
        }                                                                 \
    }()

constexpr int kMaxDiagBlocks = 1024;
constexpr size_t kStagingCap = size_t(16) << 20;  // bytes of read-out staging at most

inline size_t staging_bytes_for(int nx, int ny)
{
    // 8 doubles per site, at most 16 MiB (one row at least), at least 64 KiB
    const size_t want = std::min(8 * (size_t)nx * ny * sizeof(double), std::max(kStagingCap, 9 * (size_t)nx * sizeof(double)));
    return std::max(want, size_t(64) << 10);
}

// Everything needed to start, read and diagnose one plate's state.
struct PlateIO {
    int nx, ny;
    lbm_precision prec;
    Units U;
    int bc_lo, bc_hi;           // y edges
    double val_lo[2], val_hi[2];
    int bc_left, bc_right;      // x edges (periodic unless set)
    double val_left[2], val_right[2];
    // momentum walls: displacement uwb + j* n at step n, lattice units
    double uwb_lo[2], uwb_hi[2], uwb_left[2], uwb_right[2];
    const unsigned char *mask;  // device [ny][nx] material mask, or nullptr
    void *f, *u, *j;            // current state copy
    void *f_other;              // the other copy (staging for start-up)
    double f_scale;
    double *staging;            // read-out staging
    size_t staging_bytes;
    double *partials;           // kMaxDiagBlocks * 8 doubles
    double *diag_out;           // 8 doubles
    hipStream_t stream;
};

// Geometry/material view used by the start-up, read-out and diagnostics
// kernels at step t_steps (a momentum wall is at uwb + j* t).
inline FieldParams field_params(const PlateIO &io, double t_steps)
{
    const Units &U = io.U;
    FieldParams fp{};
    fp.nx = io.nx;
    fp.ny = io.ny;
    fp.plane = (long long)io.nx * io.ny;
    fp.bc_lo = io.bc_lo;
    fp.bc_hi = io.bc_hi;
    fp.bc_left = io.bc_left;
    fp.bc_right = io.bc_right;
    auto uw = [&](int bc, double v, double base) {
        return bc == LBM_BC_DIRICHLET_J ? base + v / U.momentum() * t_steps : 0.0;
    };
    for (int a = 0; a < 2; ++a) {
        fp.uw_lo[a] = uw(io.bc_lo, io.val_lo[a], io.uwb_lo[a]);
        fp.uw_hi[a] = uw(io.bc_hi, io.val_hi[a], io.uwb_hi[a]);
        fp.uw_left[a] = uw(io.bc_left, io.val_left[a], io.uwb_left[a]);
        fp.uw_right[a] = uw(io.bc_right, io.val_right[a], io.uwb_right[a]);
    }
    fp.lam = U.lam / U.stress();
    fp.mu = U.mu / U.stress();
    fp.mask = io.mask;
    return fp;
}

// Largest population magnitude (lattice units) that a plate's loads drive,
// with a margin: a traction T* enters the wall populations and the stresses
// near the wall through the boundary Poisson stress (about |T*|); a wall
// momentum j* through 6 w_i e_i . j* and the stress of the wave it launches
// (about |j*|); a body force builds stresses of about |rho0 b| times the
// plate's extent. (A body force on a plate without walls accelerates it
// without bound; no scale covers that.) val: j* or T* of the edges in
// physical units, body: b per unit mass.
inline double load_population_bound(const Units &U, int nx, int ny, const int bc[4], const double val[4][2],
                                    const double body[2])
{
    double m = 0.0;
    for (int e = 0; e < 4; ++e)
        for (int a = 0; a < 2; ++a) {
            if (bc[e] == LBM_BC_NEUMANN_T) m = std::max(m, 2.0 * std::fabs(val[e][a]) / U.stress());
            if (bc[e] == LBM_BC_DIRICHLET_J) m = std::max(m, 2.0 * std::fabs(val[e][a]) / U.momentum());
        }
    const double bl = std::hypot(body[0], body[1]) * U.dt() / U.c();  // rho0 b per step, lattice units
    return std::max(m, 2.0 * bl * std::max(nx, ny));
}

// Power-of-two scale of 16-bit populations that puts a largest magnitude mx
// near 2^12 (binary16 tops out at 65504); the exponent stays within +-60 so
// the scale and its inverse are normal floats. 1 for mx = 0.
inline double population_scale(double mx)
{
    if (!(mx > 0.0)) return 1.0;
    return std::ldexp(1.0, std::max(-60, std::min(60, (int)std::floor(std::log2(4096.0 / mx)))));
}

// Largest scaled magnitude a 16-bit plate may reach before its scale is
// lowered: 16 times the start target, 4 times below the binary16 maximum.
constexpr double kScaledHeadroom = 16384.0;

// Lower a 16-bit plate's population scale to new_scale (a power of two below
// the current one) by rescaling the stored populations f of its current
// state copy on the stream. Returns the error of the launch.
inline hipError_t plate_rescale(lbm_precision prec, void *f, size_t sites, double factor, hipStream_t st)
{
    const long long n = 9 * (long long)sites;
    const int nb = (int)((n + 255) / 256);
    if (prec == LBM_FP16_STORE)
        hipLaunchKernelGGL(rescale_kernel<__half>, dim3(nb), dim3(256), 0, st, static_cast<__half *>(f), n,
                           (float)factor);
    else if (prec == LBM_BF16_STORE)
        hipLaunchKernelGGL(rescale_kernel<__hip_bfloat16>, dim3(nb), dim3(256), 0, st,
                           static_cast<__hip_bfloat16 *>(f), n, (float)factor);
    return hipGetLastError();
}

// f = f^eq of the start fields (u0, v0 host arrays). For 16-bit storage the
// population scale is chosen here (returned in *scale) from the largest start
// population and load_bound (load_population_bound of the plate's loads);
// *nonfinite is set if the start populations are not finite. Synchronises.
inline hipError_t plate_start(const PlateIO &io, const double *u0, const double *v0, double load_bound,
                              double *scale, bool *nonfinite)
{
    *nonfinite = false;
    const size_t n = (size_t)io.nx * io.ny;
    // the start fields themselves, every value (a NaN would slip through the
    // max |f| reduction below, and FP32/FP64 storage has no such pass)
    for (size_t i = 0; i < 2 * n; ++i)
        if (!std::isfinite(u0[i]) || !std::isfinite(v0[i])) {
            *nonfinite = true;
            return hipSuccess;
        }
    double *su = static_cast<double *>(io.f_other);  // the other copy holds >= 32 bytes per site
    double *sv = su + 2 * n;
    hipError_t e;
    if ((e = hipMemcpyAsync(su, u0, 2 * n * sizeof(double), hipMemcpyHostToDevice, io.stream))) return e;
    if ((e = hipMemcpyAsync(sv, v0, 2 * n * sizeof(double), hipMemcpyHostToDevice, io.stream))) return e;
    InitParams ip{};
    ip.fp = field_params(io, 0.0);
    ip.u0 = su;
    ip.v0 = sv;
    ip.f = io.f;
    ip.u = io.u;
    ip.j = io.j;
    ip.inv_dx = 1.0 / io.U.dx;
    ip.v_to_j = io.U.dt() / io.U.dx;
    const int nblocks = (int)((n + 255) / 256);
    *scale = 1.0;
    if (io.prec == LBM_FP16_STORE || io.prec == LBM_BF16_STORE) {
        // power-of-two scale that puts max |f| near 2^12 (FP16 tops out at 65504)
        if ((size_t)nblocks * sizeof(double) > io.staging_bytes) return hipErrorOutOfMemory;
        ip.mode = 0;
        ip.maxf = io.staging;
        if ((e = LBM_DISPATCH(io.prec, Kernels<PR>::init(ip, nblocks, io.stream)))) return e;
        std::vector<double> m(nblocks);
        if ((e = hipMemcpyAsync(m.data(), ip.maxf, nblocks * sizeof(double), hipMemcpyDeviceToHost, io.stream)))
            return e;
        if ((e = hipStreamSynchronize(io.stream))) return e;
        double mx = 0.0;
        for (double v : m) mx = std::max(mx, v);
        if (!std::isfinite(mx)) {
            *nonfinite = true;
            return hipSuccess;
        }
        *scale = population_scale(std::max(mx, load_bound));
    }
    ip.mode = 1;
    ip.f_scale = *scale;
    if ((e = LBM_DISPATCH(io.prec, Kernels<PR>::init(ip, nblocks, io.stream)))) return e;
    return hipStreamSynchronize(io.stream);
}

// u, v, P (any may be NULL) and diagnostics (out7 may be NULL) of a plate
// after t_steps steps. Synchronises.
// Values of read-out kind `what` (1: u, v, P; 2: sigma, E, W) of every site,
// copied into the host planes dst[0 .. nv-1] ([ny][nx] each, NULL skips a
// plane) through the staging area in row chunks. Synchronises.
inline hipError_t plate_rows(const PlateIO &io, double t_steps, int what, double *const *dst, int nv)
{
    const int nx = io.nx, ny = io.ny;
    ReadParams rp{};
    rp.fp = field_params(io, t_steps);
    rp.u = io.u;
    rp.j = io.j;
    rp.out = io.staging;
    rp.nodes = nullptr;
    rp.what = what;
    rp.dx = io.U.dx;
    rp.c = io.U.c();
    rp.stress = io.U.stress();
    const int rows_per =
        (int)std::max<size_t>(1, std::min<size_t>(ny, io.staging_bytes / (nv * sizeof(double) * nx)));
    hipError_t e;
    for (int y = 0; y < ny; y += rows_per) {
        const int rows = std::min(rows_per, ny - y);
        rp.y_begin = y;
        rp.count = rows * nx;
        const size_t cnt = (size_t)rows * nx;
        if ((e = LBM_DISPATCH(io.prec, Kernels<PR>::readout(rp, (int)((cnt + 255) / 256), io.stream)))) return e;
        for (int k = 0; k < nv; ++k) {
            if (!dst[k]) continue;
            if ((e = hipMemcpyAsync(dst[k] + (size_t)y * nx, rp.out + k * cnt, cnt * sizeof(double),
                                    hipMemcpyDeviceToHost, io.stream)))
                return e;
        }
        if ((e = hipStreamSynchronize(io.stream))) return e;
    }
    return hipSuccess;
}

// Nodes one sample call can read through the staging area.
inline int sample_capacity(const PlateIO &io)
{
    return (int)std::min<size_t>(1 << 20, (io.staging_bytes - 256) / (17 * sizeof(double) + sizeof(int)));
}

// u, v, P, sigma, E, W (17 values) at the nodes (x[k], y[k]) into out[n][17].
// The caller has checked the nodes and n <= sample_capacity(io). Synchronises.
inline hipError_t plate_sample(const PlateIO &io, double t_steps, int n, const int *xs, const int *ys, double *out)
{
    if (n == 0) return hipSuccess;
    std::vector<int> idx(n);
    for (int k = 0; k < n; ++k) idx[k] = ys[k] * io.nx + xs[k];
    int *d_idx = reinterpret_cast<int *>(io.staging);
    double *vals = io.staging + align_up((size_t)n * sizeof(int)) / sizeof(double);
    hipError_t e;
    if ((e = hipMemcpyAsync(d_idx, idx.data(), n * sizeof(int), hipMemcpyHostToDevice, io.stream))) return e;
    ReadParams rp{};
    rp.fp = field_params(io, t_steps);
    rp.u = io.u;
    rp.j = io.j;
    rp.out = vals;
    rp.nodes = d_idx;
    rp.count = n;
    rp.what = 3;
    rp.dx = io.U.dx;
    rp.c = io.U.c();
    rp.stress = io.U.stress();
    if ((e = LBM_DISPATCH(io.prec, Kernels<PR>::readout(rp, (n + 255) / 256, io.stream)))) return e;
    std::vector<double> tmp((size_t)17 * n);
    if ((e = hipMemcpyAsync(tmp.data(), vals, tmp.size() * sizeof(double), hipMemcpyDeviceToHost, io.stream)))
        return e;
    if ((e = hipStreamSynchronize(io.stream))) return e;
    for (int k = 0; k < n; ++k)
        for (int c = 0; c < 17; ++c) out[(size_t)k * 17 + c] = tmp[(size_t)c * n + k];
    return hipSuccess;
}

inline hipError_t plate_read(const PlateIO &io, double t_steps, double *u, double *v, double *P, double *out7)
{
    const size_t n = (size_t)io.nx * io.ny;
    hipError_t e;
    if (u || v || P) {
        double *dst[8] = {u, u ? u + n : nullptr, v, v ? v + n : nullptr,
                          P, P ? P + n : nullptr, P ? P + 2 * n : nullptr, P ? P + 3 * n : nullptr};
        if ((e = plate_rows(io, t_steps, 1, dst, 8))) return e;
    }
    if (out7) {
        DiagParams dp{};
        dp.fp = field_params(io, t_steps);
        dp.f = io.f;
        dp.u = io.u;
        dp.j = io.j;
        dp.f_inv_scale = 1.0 / io.f_scale;
        dp.rho0 = io.U.rho0;
        dp.dx = io.U.dx;
        dp.c = io.U.c();
        dp.lam_phys = io.U.lam;
        dp.mu_phys = io.U.mu;
        dp.partials = io.partials;
        const int nblocks = (int)std::min<size_t>(kMaxDiagBlocks, (n + 255) / 256);
        if ((e = LBM_DISPATCH(io.prec, Kernels<PR>::diag(dp, nblocks, io.stream)))) return e;
        hipLaunchKernelGGL(diag_final_kernel, dim3(1), dim3(64), 0, io.stream, io.partials, nblocks, io.diag_out);
        if ((e = hipGetLastError())) return e;
        if ((e = hipMemcpyAsync(out7, io.diag_out, 7 * sizeof(double), hipMemcpyDeviceToHost, io.stream))) return e;
        if ((e = hipStreamSynchronize(io.stream))) return e;
    }
    return hipSuccess;
}

// sigma [4][ny][nx], E [4][ny][nx], W [ny][nx]; any may be NULL. Synchronises.
inline hipError_t plate_read_derived(const PlateIO &io, double t_steps, double *sig, double *E, double *W)
{
    if (!sig && !E && !W) return hipSuccess;
    const size_t n = (size_t)io.nx * io.ny;
    double *dst[9] = {sig, sig ? sig + n : nullptr, sig ? sig + 2 * n : nullptr, sig ? sig + 3 * n : nullptr,
                      E,   E ? E + n : nullptr,     E ? E + 2 * n : nullptr,     E ? E + 3 * n : nullptr, W};
    return plate_rows(io, t_steps, 2, dst, 9);
}

}  // namespace lbm
