// aux_kernels.hpp -- start-up, read-out and diagnostics kernels.
//
// These run once per set_fields / read call, not per step; they favour
// plain per-site code over tiling.
#pragma once

#include "lattice.hpp"

namespace lbm {

struct FieldParams {
    int nx, ny;
    long long plane;
    int bc_lo, bc_hi;           // y edges
    double uw_lo[2], uw_hi[2];  // wall displacement of momentum walls (lattice units)
    int bc_left, bc_right;      // x edges
    double uw_left[2], uw_right[2];
    double lam, mu;             // lattice units
    const unsigned char *mask;  // [ny][nx]: material (1) or hole (0), Sec. 7.2; nullptr: no holes
};

// Node (x, y) lies in a hole; coordinates beyond a periodic edge wrap,
// beyond a wall they are in no hole.
__device__ inline bool in_hole(const FieldParams &p, int x, int y)
{
    if (!p.mask) return false;
    if (y < 0 || y >= p.ny) {
        if (p.bc_lo != BC_PERIODIC) return false;
        y = (y % p.ny + p.ny) % p.ny;
    }
    if (x < 0 || x >= p.nx) {
        if (p.bc_left != BC_PERIODIC) return false;
        x = (x % p.nx + p.nx) % p.nx;
    }
    return (p.mask[(size_t)y * p.nx + x] & 1) == 0;
}

// Displacement of node (x, y), 0 <= x < nx, in lattice units, with the
// ghost-row rules of the y walls for y = -1 and y = ny.
template <class TU>
__device__ inline double u_row(const TU *u, const FieldParams &p, int a, int x, int y)
{
    const size_t pl = (size_t)p.plane;
    if (p.bc_lo == BC_PERIODIC) {
        y = (y % p.ny + p.ny) % p.ny;
        return (double)u[a * pl + (size_t)y * p.nx + x];
    }
    if (y >= 0 && y < p.ny) return (double)u[a * pl + (size_t)y * p.nx + x];
    if (y < 0) {
        const double u0 = (double)u[a * pl + x], u1 = (double)u[a * pl + (size_t)p.nx + x];
        (void)u1;
        if (p.bc_lo == BC_NEUMANN) return u0;
        return 2.0 * p.uw_lo[a] - u0;
    }
    const double v0 = (double)u[a * pl + (size_t)(p.ny - 1) * p.nx + x];
    const double v1 = (double)u[a * pl + (size_t)(p.ny - 2) * p.nx + x];
    (void)v1;
    if (p.bc_hi == BC_NEUMANN) return v0;
    return 2.0 * p.uw_hi[a] - v0;
}

// Displacement at (x, y), -1 <= x <= nx, -1 <= y <= ny: beyond an x wall the
// ghost column is extrapolated across the wall from the row value of the
// nearest column (ghost rows included), as the y walls do for rows.
template <class TU>
__device__ inline double u_at(const TU *u, const FieldParams &p, int a, int x, int y)
{
    if (x >= 0 && x < p.nx) return u_row(u, p, a, x, y);
    if (p.bc_left == BC_PERIODIC) return u_row(u, p, a, (x % p.nx + p.nx) % p.nx, y);
    const bool left = x < 0;
    const int kind = left ? p.bc_left : p.bc_right;
    const double u0 = u_row(u, p, a, left ? 0 : p.nx - 1, y);
    if (kind == BC_NEUMANN) return u0;
    return 2.0 * (left ? p.uw_left[a] : p.uw_right[a]) - u0;
}

// Central-difference gradient at (x, y); a hole neighbour takes the node's
// own displacement (the constant ghost of a traction-free wall).
template <class TU>
__device__ inline void grad_at(const TU *u, const FieldParams &p, int x, int y, double H[4])
{
    const bool hxp = in_hole(p, x + 1, y), hxm = in_hole(p, x - 1, y);
    const bool hyp = in_hole(p, x, y + 1), hym = in_hole(p, x, y - 1);
    for (int a = 0; a < 2; ++a) {
        const double c = (hxp || hxm || hyp || hym) ? u_at(u, p, a, x, y) : 0.0;
        const double xp = hxp ? c : u_at(u, p, a, x + 1, y), xm = hxm ? c : u_at(u, p, a, x - 1, y);
        const double yp = hyp ? c : u_at(u, p, a, x, y + 1), ym = hym ? c : u_at(u, p, a, x, y - 1);
        H[2 * a + 0] = 0.5 * (xp - xm);
        H[2 * a + 1] = 0.5 * (yp - ym);
    }
}

// ---------------------------------------------------------------- start-up

struct InitParams {
    FieldParams fp;
    const double *u0;   // staged host input, physical units, [2][ny][nx]
    const double *v0;
    void *f, *u, *j;    // state (storage types of the precision)
    double inv_dx;      // u_L = u / dX
    double v_to_j;      // j_L = v dt / dX
    double f_scale;
    double *maxf;       // per-block max |f| (mode 0)
    int mode;           // 0: reduce max |f| only, 1: write the state
};

// f = f^eq(r0, j0, Pbar(H(u0))) with r0 = -div u0, j0 = rho0 v0
// (Algorithm 1, initialisation; eqs. (15), (18), (20)), lattice units. With
// deviation storage the stored value is f minus ref_eq of the stored state,
// which the start state equals up to rounding (the same moments).
template <class PR>
__global__ void __launch_bounds__(256) init_kernel(const InitParams p)
{
    using TF = typename PR::TF;
    using TU = typename PR::TU;
    using TJ = typename PR::TJ;
    using TC = typename PR::TC;
    __shared__ double red[256];
    const FieldParams &fp = p.fp;
    const size_t pl = (size_t)fp.plane;
    const long long n = (long long)fp.nx * fp.ny;
    const long long s = (long long)blockIdx.x * 256 + threadIdx.x;
    double m = 0.0;
    if (s < n) {
        const int y = (int)(s / fp.nx), x = (int)(s - (long long)y * fp.nx);
        const bool hole = in_hole(fp, x, y);
        // u0 in lattice units; the staged array has the same layout as u.
        // The ghost rules apply with the walls at rest (t = 0).
        FieldParams rest = fp;
        rest.uw_lo[0] = rest.uw_lo[1] = rest.uw_hi[0] = rest.uw_hi[1] = 0.0;
        rest.uw_left[0] = rest.uw_left[1] = rest.uw_right[0] = rest.uw_right[1] = 0.0;
        double H[4];
        grad_at(p.u0, rest, x, y, H);
        for (int c = 0; c < 4; ++c) H[c] *= p.inv_dx;
        const double mu = fp.mu;
        const double tr = H[0] + H[3];
        const double r = -tr;
        const double Pxx = -mu * (2.0 * H[0] + tr), Pyy = -mu * (2.0 * H[3] + tr);
        const double Pxy = -mu * (H[1] + H[2]);
        const double jx = hole ? 0.0 : p.v0[s] * p.v_to_j, jy = hole ? 0.0 : p.v0[pl + s] * p.v_to_j;
        const double axx = Pxx - r / 3.0, ayy = Pyy - r / 3.0, trA = axx + ayy;
        const double q[9] = {-trA / 3.0,
                             axx - trA / 3.0,
                             ayy - trA / 3.0,
                             axx - trA / 3.0,
                             ayy - trA / 3.0,
                             2.0 * (trA / 3.0 + Pxy),
                             2.0 * (trA / 3.0 - Pxy),
                             2.0 * (trA / 3.0 + Pxy),
                             2.0 * (trA / 3.0 - Pxy)};
        const int ex[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
        const int ey[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
        const double w[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
        TC fr[9] = {};
        if constexpr (FStore<TF>::kDeviation) {
            if (!hole) {
                const TC Hc[4] = {TC(H[0]), TC(H[1]), TC(H[2]), TC(H[3])};
                ref_eq(Hc, TC(TJ(jx)), TC(TJ(jy)), fr);
            }
        }
        for (int i = 0; i < 9; ++i) {
            const double fi = hole ? 0.0 : w[i] * (r + 3.0 * (ex[i] * jx + ey[i] * jy) + 4.5 * q[i]);
            m = fmax(m, fabs(fi));
            if (p.mode == 1)
                FStore<TF>::store(static_cast<TF *>(p.f), i * pl + s, TC(fi - (double)fr[i]), TC(p.f_scale));
        }
        if (p.mode == 1) {
            TU *u = static_cast<TU *>(p.u);
            TJ *j = static_cast<TJ *>(p.j);
            u[s] = hole ? TU(0) : TU(p.u0[s] * p.inv_dx);
            u[pl + s] = hole ? TU(0) : TU(p.u0[pl + s] * p.inv_dx);
            j[s] = TJ(jx);
            j[pl + s] = TJ(jy);
        }
    }
    if (p.mode == 0) {
        red[threadIdx.x] = m;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
            __syncthreads();
        }
        if (threadIdx.x == 0) p.maxf[blockIdx.x] = red[0];
    }
}

// Multiply the n stored 16-bit populations at f by a power of two (lowering
// the per-plate scale when a new load needs more headroom). Exact unless a
// value drops below the format's normal range.
template <class TF>
__global__ void __launch_bounds__(256) rescale_kernel(TF *f, long long n, float factor)
{
    const long long s = (long long)blockIdx.x * 256 + threadIdx.x;
    if (s < n) f[s] = FStore<TF>::conv(FStore<TF>::cvt(f[s], 1.0f) * factor, 1.0f);
}

// ---------------------------------------------------------------- read-out

struct ReadParams {
    FieldParams fp;
    const void *u, *j;
    double *out;        // staging: [values][count]
    int y_begin;        // first row of a row read (nodes == nullptr)
    const int *nodes;   // or: site indices y * nx + x of the nodes sampled
    int count;          // sites read: rows * nx, or the number of nodes
    int what;           // bit 0: u (2), v (2), P (4); bit 1: sigma (4), E (4), W (1)
    double dx;          // u = dX u_L
    double c;           // v = c j_L
    double stress;      // P, sigma, W = rho0 c^2 (lattice value)
};

// Read-out of fields at sites, in physical units, from the central-difference
// gradient H(u) (Sec. 5):
//   P     first Piola-Kirchhoff stress (eq. (27));
//   sigma Cauchy stress, in the left Cauchy-Green form of the neo-Hooke law,
//         sigma = (mu / J)(F F^T - I) + lam (J^2 - 1) / (2 J) I;
//   E     Green-Lagrange strain (F^T F - I) / 2;
//   W     strain-energy density of eq. (27).
template <class PR>
__global__ void __launch_bounds__(256) readout_kernel(const ReadParams p)
{
    using TU = typename PR::TU;
    using TJ = typename PR::TJ;
    const FieldParams &fp = p.fp;
    const size_t pl = (size_t)fp.plane;
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= p.count) return;
    int x, y;
    if (p.nodes) {
        const int g = p.nodes[s];
        y = g / fp.nx;
        x = g - y * fp.nx;
    } else {
        const int yl = s / fp.nx;
        x = s - yl * fp.nx;
        y = p.y_begin + yl;
    }
    const TU *u = static_cast<const TU *>(p.u);
    const TJ *j = static_cast<const TJ *>(p.j);
    const size_t g = (size_t)y * fp.nx + x;
    const size_t cp = (size_t)p.count;
    if (in_hole(fp, x, y)) {  // no material: every value reads as zero
        const int nv = ((p.what & 1) ? 8 : 0) + ((p.what & 2) ? 9 : 0);
        for (int k = 0; k < nv; ++k) p.out[k * cp + s] = 0.0;
        return;
    }
    double H[4];
    grad_at(u, fp, x, y, H);
    int k = 0;
    if (p.what & 1) {
        double P[4];
        piola<double>(H, fp.lam, fp.mu, P);
        p.out[k++ * cp + s] = (double)u[g] * p.dx;
        p.out[k++ * cp + s] = (double)u[pl + g] * p.dx;
        p.out[k++ * cp + s] = (double)j[g] * p.c;
        p.out[k++ * cp + s] = (double)j[pl + g] * p.c;
        for (int c = 0; c < 4; ++c) p.out[k++ * cp + s] = P[c] * p.stress;
    }
    if (p.what & 2) {
        const double F11 = 1.0 + H[0], F12 = H[1], F21 = H[2], F22 = 1.0 + H[3];
        const double J = F11 * F22 - F12 * F21;
        // left Cauchy-Green B = F F^T and right C = F^T F
        const double B11 = F11 * F11 + F12 * F12, B12 = F11 * F21 + F12 * F22, B22 = F21 * F21 + F22 * F22;
        const double C11 = F11 * F11 + F21 * F21, C12 = F11 * F12 + F21 * F22, C22 = F12 * F12 + F22 * F22;
        const double a = fp.mu / J, d = fp.lam * (J * J - 1.0) / (2.0 * J);
        const double sg[4] = {a * (B11 - 1.0) + d, a * B12, a * B12, a * (B22 - 1.0) + d};
        for (int c = 0; c < 4; ++c) p.out[k++ * cp + s] = sg[c] * p.stress;
        p.out[k++ * cp + s] = 0.5 * (C11 - 1.0);
        p.out[k++ * cp + s] = 0.5 * C12;
        p.out[k++ * cp + s] = 0.5 * C12;
        p.out[k++ * cp + s] = 0.5 * (C22 - 1.0);
        const double lj = log(J);
        const double W = 0.5 * fp.mu * (C11 + C22 - 2.0) + 0.25 * fp.lam * (J * J - 1.0) - 0.5 * fp.lam * lj - fp.mu * lj;
        p.out[k++ * cp + s] = W * p.stress;
    }
}

// ---------------------------------------------------------------- diagnostics

struct DiagParams {
    FieldParams fp;
    const void *f, *u, *j;
    double f_inv_scale;
    double rho0, dx, c, lam_phys, mu_phys;
    double *partials;   // [gridDim.x][8]
};

// Per-block partial sums in FP64 with a fixed tree; blocks cover fixed site
// ranges, so the result does not depend on scheduling.
template <class PR>
__global__ void __launch_bounds__(256) diag_kernel(const DiagParams p)
{
    using TF = typename PR::TF;
    using TU = typename PR::TU;
    using TJ = typename PR::TJ;
    __shared__ double red[7][256];
    const FieldParams &fp = p.fp;
    const size_t pl = (size_t)fp.plane;
    const long long n = (long long)fp.nx * fp.ny;
    double acc[7] = {0, 0, 0, 0, 1e300, 0, 0};  // jx, jy, r, energy, minJ, maxE, bad
    const TF *f = static_cast<const TF *>(p.f);
    const TU *u = static_cast<const TU *>(p.u);
    const TJ *j = static_cast<const TJ *>(p.j);
    for (long long s = (long long)blockIdx.x * 256 + threadIdx.x; s < n; s += (long long)gridDim.x * 256) {
        const int y = (int)(s / fp.nx), x = (int)(s - (long long)y * fp.nx);
        if (in_hole(fp, x, y)) continue;
        double H[4];
        grad_at(u, fp, x, y, H);
        double r = 0.0;
        for (int i = 0; i < 9; ++i) r += (double)FStore<TF>::load(f, i * pl + s, (typename PR::TC)p.f_inv_scale);
        if constexpr (FStore<TF>::kDeviation) {
            // the stored deviations plus the reference equilibrium's zeroth
            // moment, sum_i ref_eq_i = -tr H
            using TC = typename PR::TC;
            const TC Hc[4] = {TC(H[0]), TC(H[1]), TC(H[2]), TC(H[3])};
            TC fr[9];
            ref_eq(Hc, TC(j[s]), TC(j[pl + s]), fr);
            for (int i = 0; i < 9; ++i) r += (double)fr[i];
        }
        const double F11 = 1.0 + H[0], F12 = H[1], F21 = H[2], F22 = 1.0 + H[3];
        const double J = F11 * F22 - F12 * F21;
        const double E11 = 0.5 * (F11 * F11 + F21 * F21 - 1.0);
        const double E12 = 0.5 * (F11 * F12 + F21 * F22);
        const double E22 = 0.5 * (F12 * F12 + F22 * F22 - 1.0);
        const double mean = 0.5 * (E11 + E22);
        const double dev = sqrt(0.25 * (E11 - E22) * (E11 - E22) + E12 * E12);
        const double En = fmax(fabs(mean + dev), fabs(mean - dev));
        const double jx = (double)j[s] * p.rho0 * p.c, jy = (double)j[pl + s] * p.rho0 * p.c;
        const double ux = (double)u[s], uy = (double)u[pl + s];
        acc[0] += jx;
        acc[1] += jy;
        acc[2] += r * p.rho0;
        const bool ok = (J > 0.0) && isfinite(jx) && isfinite(jy) && isfinite(ux) && isfinite(uy);
        if (ok) {
            const double IC = F11 * F11 + F12 * F12 + F21 * F21 + F22 * F22;
            const double W = 0.5 * p.mu_phys * (IC - 2.0) + 0.25 * p.lam_phys * (J * J - 1.0) -
                             0.5 * p.lam_phys * log(J) - p.mu_phys * log(J);
            acc[3] += ((jx * jx + jy * jy) / (2.0 * p.rho0) + W) * p.dx * p.dx;
        } else {
            acc[6] = 1.0;
        }
        acc[4] = fmin(acc[4], J);
        acc[5] = fmax(acc[5], En);
    }
    for (int k = 0; k < 7; ++k) red[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            for (int k = 0; k < 4; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
            red[4][threadIdx.x] = fmin(red[4][threadIdx.x], red[4][threadIdx.x + w]);
            red[5][threadIdx.x] = fmax(red[5][threadIdx.x], red[5][threadIdx.x + w]);
            red[6][threadIdx.x] = fmax(red[6][threadIdx.x], red[6][threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x < 7) p.partials[blockIdx.x * 8 + threadIdx.x] = red[threadIdx.x][0];
}

// Second stage: one block folds the per-block partials in index order.
static __global__ void __launch_bounds__(64) diag_final_kernel(const double *partials, int nblocks, double *out)
{
    if (threadIdx.x != 0) return;
    double acc[7] = {0, 0, 0, 0, 1e300, 0, 0};
    for (int b = 0; b < nblocks; ++b) {
        for (int k = 0; k < 4; ++k) acc[k] += partials[b * 8 + k];
        acc[4] = fmin(acc[4], partials[b * 8 + 4]);
        acc[5] = fmax(acc[5], partials[b * 8 + 5]);
        acc[6] = fmax(acc[6], partials[b * 8 + 6]);
    }
    for (int k = 0; k < 7; ++k) out[k] = acc[k];
}

}  // namespace lbm
