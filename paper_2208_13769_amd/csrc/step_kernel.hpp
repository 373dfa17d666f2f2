// step_kernel.hpp -- one fused time step of the Lagrangian solid LBM.
//
// One launch advances a plate from state n (f, u, j) to state n+1 by the
// steps of Algorithm 1 (Sec. 5), all in registers and LDS:
//   a1 stress sum K = P(H) + Pbar(H) from central differences of u (eqs. (10), (15), (27))
//   a2 source 1S = rho0 b + div K (eq. (23))
//   a3 r = sum f, Pi = sum e e f (the populations' own second moment)
//   a4-a6 equilibrium (20), forcing (22) and BGK collision (4)
//   a7 pull streaming (5), a8 bounce-back (25) / anti-bounce-back (26) at y walls
//   a9 moments with half source (6); predictor-corrector source at t + dt
//   a10 trapezoidal displacement update (24)
//
// Work decomposition ("y-march"): a block of BLOCK threads owns a strip of
// columns, one column per thread, and walks up a segment of rows. Each
// dependency in y is carried by the thread's own register rings; each
// dependency in x goes through LDS, double buffered, so every row costs one
// barrier. The stages of one iteration work on different rows:
//   A  load u_n at row R                       (LDS: u)
//   B  K at row R-1                            (LDS: K_a1)
//   C  S_n at row R-2, load f_n, j_n, collide  (LDS: f^col with e_x != 0)
//   D  pull row R-4 -> f_{n+1}, jf; u^p        (LDS: u^p)        [PC]
//   E  K^p at row R-5                          (LDS: K^p_a1)     [PC]
//   F  S^p at row R-6, j_{n+1}, u_{n+1}                          [PC]
// The explicit scheme (source at t in the moment step, as printed in
// Algorithm 1) finishes at stage D with S_n. Each stage reads the LDS rows
// its neighbours wrote in the previous iteration, so the halo in x is 5
// columns (PC) or 3 (explicit) and the segment is extended by the same
// pipeline depth in y; halo work is recomputed, never exchanged.
// Within an iteration the global loads for stages A and C are issued first
// and stages D, E, F (which only need earlier rows) run before A, B, C, so
// the loads are in flight while D-F compute.
//
// Walls (y edges only) lie half a spacing outside the node rows 0 and ny-1.
// Ghost displacement rows for the finite differences: momentum wall -- the
// quadratic through the wall displacement u_w = j* t / rho0 and the two
// nearest rows; traction wall -- the nearest row repeated. Rows above the
// top wall follow from rows already walked; the ghost row below the bottom
// wall is folded into the source of row 0 when that row is reached.
#pragma once

#include "lattice.hpp"

namespace lbm {

struct StepParams {
    const void *f_in;
    void *f_out;
    const void *u_in;
    void *u_out;
    const void *j_in;
    void *j_out;
    int nx, ny;
    long long plane;        // elements per component plane
    double omega;           // dt / tau
    double lam, mu;         // lattice units
    double bx, by;          // rho0 b in lattice units (source per step)
    int bc_lo, bc_hi;       // rule of the y edges (BC_*)
    double val_lo[2], val_hi[2];  // j* or T* in lattice units
    double f_scale, f_inv_scale;  // 16-bit population scaling (1 otherwise)
    int strip_w, n_strips, n_segs;
    int halo_a;             // threads left of the first output column (>= the stencil halo)
    unsigned int *flag;     // set to 1 on J <= 0 or a non-finite value
    long long step;         // index n of the input state
};

template <class TC>
__device__ __forceinline__ void collide(const TC f[9], TC jx, TC jy, TC Sx, TC Sy, TC omega,
                                        TC fc[9], TC &r_out, TC &pxx_out)
{
    const TC r = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
    const TC dsum = (f[5] + f[6]) + (f[7] + f[8]);
    const TC pxx = (f[1] + f[3]) + dsum;
    const TC pyy = (f[2] + f[4]) + dsum;
    const TC pxy = (f[5] - f[6]) + (f[7] - f[8]);
    const TC third = TC(1) / TC(3);
    // A = Pi - r/3 I, Q_i = A : (e_i e_i - I/3)
    const TC axx = pxx - r * third, ayy = pyy - r * third;
    const TC trA = axx + ayy;
    const TC q0 = -trA * third;
    const TC q13 = axx + q0;
    const TC q24 = ayy + q0;
    const TC q57 = TC(2) * (trA * third + pxy);
    const TC q68 = TC(2) * (trA * third - pxy);
    // f^col_i = (1 - w) f_i + w_i (w (r + 9/2 Q_i) + 3 e_i . g), g = w j + (1 - w/2) S
    const TC om1 = TC(1) - omega;
    const TC hs = TC(1) - TC(0.5) * omega;
    const TC gx = omega * jx + hs * Sx, gy = omega * jy + hs * Sy;
    const TC wr = omega * r, w45 = TC(4.5) * omega;
    const TC gx3 = TC(3) * gx, gy3 = TC(3) * gy;
    const TC w0 = TC(4) / TC(9), w1 = TC(1) / TC(9), w5 = TC(1) / TC(36);
    fc[0] = om1 * f[0] + w0 * (wr + w45 * q0);
    const TC b13 = wr + w45 * q13, b24 = wr + w45 * q24;
    fc[1] = om1 * f[1] + w1 * (b13 + gx3);
    fc[3] = om1 * f[3] + w1 * (b13 - gx3);
    fc[2] = om1 * f[2] + w1 * (b24 + gy3);
    fc[4] = om1 * f[4] + w1 * (b24 - gy3);
    const TC b57 = wr + w45 * q57, b68 = wr + w45 * q68;
    fc[5] = om1 * f[5] + w5 * (b57 + (gx3 + gy3));
    fc[7] = om1 * f[7] + w5 * (b57 - (gx3 + gy3));
    fc[6] = om1 * f[6] + w5 * (b68 + (gy3 - gx3));
    fc[8] = om1 * f[8] + w5 * (b68 - (gy3 - gx3));
    r_out = r;
    pxx_out = pxx;
}

// Populations entering a wall node through the wall (Sec. 6). top: outgoing
// e_y = +1 links (2, 5, 6) return as (4, 7, 8); bottom: (4, 7, 8) -> (2, 5, 6).
// Momentum wall, eq. (25): f_ibar = fc_i - 6 w_i e_i . j*.
// Traction wall, eq. (26): f_ibar = -fc_i + 2 w_i (r_bd + 9/2 A* : (e_i e_i - I/3)),
// A* = Pbar* - r_bd/3 I, with Pbar*_12 = Pbar*_21 = -s T*_1 + K_12,
// Pbar*_22 = -s T*_2 + K_22, Pbar*_11 = Pi_11 (outward normal (0, s)).
template <class TC>
__device__ __forceinline__ void wall_populations(bool top, int kind, const TC fc[9], const double val[2],
                                                 TC r, TC pxx, TC k12, TC k22, TC out[3])
{
    const int i0 = top ? 2 : 4, i1 = top ? 5 : 7, i2 = top ? 6 : 8;
    if (kind == BC_DIRICHLET) {
        const TC jx = TC(val[0]), jy = TC(val[1]);
        const TC sy = top ? TC(1) : TC(-1);  // e_y of the outgoing links
        out[0] = fc[i0] - TC(6.0 / 9.0) * (sy * jy);
        // i1: e = (sy, sy) for top (1,1) / bottom (-1,-1); i2: (-1, 1) top / (1, -1) bottom
        out[1] = fc[i1] - TC(6.0 / 36.0) * (sy * jx + sy * jy);
        out[2] = fc[i2] - TC(6.0 / 36.0) * (-sy * jx + sy * jy);
    } else {
        const TC s = top ? TC(1) : TC(-1);
        const TC p12 = -s * TC(val[0]) + k12;
        const TC p22 = -s * TC(val[1]) + k22;
        const TC third = TC(1) / TC(3);
        const TC axx = pxx - r * third, ayy = p22 - r * third;
        const TC trA = axx + ayy;
        const TC q2 = ayy - trA * third;
        const TC q5 = TC(2) * (trA * third + p12);
        const TC q6 = TC(2) * (trA * third - p12);
        out[0] = -fc[i0] + TC(2.0 / 9.0) * (r + TC(4.5) * q2);
        out[1] = -fc[i1] + TC(2.0 / 36.0) * (r + TC(4.5) * q5);
        out[2] = -fc[i2] + TC(2.0 / 36.0) * (r + TC(4.5) * q6);
    }
}

// One tile (column strip `strip`, row segment `seg`) of one plate for one
// time step. Called by every thread of a block; ends with a barrier.
template <class PR, int BLOCK, bool PC, bool WALLED>
__device__ __forceinline__ void step_tile(const StepParams &p, const int strip, const int seg)
{
    using TF = typename PR::TF;
    using TU = typename PR::TU;
    using TJ = typename PR::TJ;
    using TC = typename PR::TC;
    using FS = FStore<TF>;
    constexpr int HX = PC ? 5 : 3;
    constexpr int NU = PC ? 6 : 4;   // rows of u_n kept: R .. R-NU+1
    constexpr int NJ = PC ? 4 : 2;   // rows of j_n kept: R-2 .. R-NJ-1

    __shared__ TU s_u[2][2][BLOCK];
    __shared__ TC s_k[2][2][BLOCK];
    __shared__ TC s_f[2][6][BLOCK];
    __shared__ TU s_up[PC ? 2 : 1][2][BLOCK];
    __shared__ TC s_kp[PC ? 2 : 1][2][BLOCK];
    __shared__ TC s_wall[WALLED ? 2 : 1][3][BLOCK];

    const TF *__restrict__ fin = static_cast<const TF *>(p.f_in);
    TF *__restrict__ fout = static_cast<TF *>(p.f_out);
    const TU *__restrict__ uin = static_cast<const TU *>(p.u_in);
    TU *__restrict__ uout = static_cast<TU *>(p.u_out);
    const TJ *__restrict__ jin = static_cast<const TJ *>(p.j_in);
    TJ *__restrict__ jout = static_cast<TJ *>(p.j_out);

    const int t = threadIdx.x;
    const int tl = t > 0 ? t - 1 : 0;
    const int tr = t < BLOCK - 1 ? t + 1 : BLOCK - 1;
    const int nx = p.nx, ny = p.ny;
    const size_t plane = (size_t)p.plane;

    // Output strips start on multiples of strip_w, which the host keeps a
    // multiple of the 128-byte line, so row writes cover whole lines; the
    // threads outside [halo_a, halo_a + strip_w) only feed the halo.
    const int x0 = strip * p.strip_w;
    const int xc = x0 - p.halo_a + t;
    int gx = xc % nx;
    if (gx < 0) gx += nx;
    const bool out_col = (t >= p.halo_a) && (t < p.halo_a + p.strip_w) && (xc < nx);
    const int y0 = (int)((long long)seg * ny / p.n_segs);
    const int y1 = (int)((long long)(seg + 1) * ny / p.n_segs);

    constexpr bool walled = WALLED;
    const int bc_lo = p.bc_lo, bc_hi = p.bc_hi;
    const TC omega = TC(p.omega), lam = TC(p.lam), mu = TC(p.mu);
    const TC bx = TC(p.bx), by = TC(p.by);
    const TC f_scale = TC(p.f_scale), f_inv = TC(p.f_inv_scale);
    // wall displacement u_w = j* t (lattice units) at t = n and t = n+1
    const double tn = (double)p.step;
    const TU uw_lo_n[2] = {TU(p.val_lo[0] * tn), TU(p.val_lo[1] * tn)};
    const TU uw_hi_n[2] = {TU(p.val_hi[0] * tn), TU(p.val_hi[1] * tn)};
    const TU uw_lo_p[2] = {TU(p.val_lo[0] * (tn + 1)), TU(p.val_lo[1] * (tn + 1))};
    const TU uw_hi_p[2] = {TU(p.val_hi[0] * (tn + 1)), TU(p.val_hi[1] * (tn + 1))};

    auto is_node = [&](int r) { return !walled || (r >= 0 && r < ny); };
    // row for a load: wrapped (periodic) or clamped into the plate (walls)
    auto rowc = [&](int r) {
        if (!walled) {
            r %= ny;
            if (r < 0) r += ny;
            return r;
        }
        return r < 0 ? 0 : (r >= ny ? ny - 1 : r);
    };
    auto rowi = [&](int r) {
        if (!walled) {
            r %= ny;
            if (r < 0) r += ny;
        }
        return r;
    };
    // ghost rows above the top wall from the two rows below it
    auto ghost_hi = [&](int which, TU a, TU b, TU uw) -> TU {
        if (bc_hi == BC_NEUMANN) return a;
        return which == 0 ? TU(8.0 / 3.0) * uw - TU(2) * a + b / TU(3) : TU(8) * uw - TU(9) * a + TU(2) * b;
    };
    // first ghost row below the bottom wall from rows 0 and 1
    auto ghost_lo = [&](TU a, TU b, TU uw) -> TU {
        if (bc_lo == BC_NEUMANN) return a;
        return TU(8.0 / 3.0) * uw - TU(2) * a + b / TU(3);
    };
    // stress sum in the ghost row below the bottom wall, from rows 0 and 1:
    // own values u0, u1 and x-derivatives hx0, hx1 (du_x/dx, du_y/dx)
    auto ghost_lo_K = [&](const TU u0[2], const TU u1[2], const TC hx0[2], const TC hx1[2], const TU uw[2],
                          TC &k12, TC &k22) {
        TC H[4], K[4];
        if (bc_lo == BC_NEUMANN) {
            H[0] = hx0[0];
            H[2] = hx0[1];
            H[1] = TC(0);
            H[3] = TC(0);
        } else {
            H[0] = TC(-2) * hx0[0] + hx1[0] / TC(3);
            H[2] = TC(-2) * hx0[1] + hx1[1] / TC(3);
            H[1] = TC(TU(5) * u0[0] - u1[0] - TU(4) * uw[0]);
            H[3] = TC(TU(5) * u0[1] - u1[1] - TU(4) * uw[1]);
        }
        stress_sum(H, lam, mu, K);
        k12 = K[1];
        k22 = K[3];
    };

    // register rings: index k holds row (current stage row) - k
    TU uR[NU][2];
    TC kA2[3][2];
    TC sN[2][2];
    TC jN[NJ][2];
    TC hxCur[2] = {0, 0}, hxPrev[2] = {0, 0};
    TC o0[2] = {0, 0}, o2[3] = {0, 0, 0}, o4 = 0;
    TC n1 = 0, n3 = 0, n5[2] = {0, 0}, n6[2] = {0, 0};
    TC jfR[3][2];
    TU upR[3][2];
    TC kpA2[3][2];
    TC hxpCur[2] = {0, 0}, hxpPrev[2] = {0, 0};
#pragma unroll
    for (int k = 0; k < NU; ++k) uR[k][0] = uR[k][1] = TU(0);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        kA2[k][0] = kA2[k][1] = TC(0);
        jfR[k][0] = jfR[k][1] = kpA2[k][0] = kpA2[k][1] = TC(0);
        upR[k][0] = upR[k][1] = TU(0);
    }
#pragma unroll
    for (int k = 0; k < NJ; ++k) jN[k][0] = jN[k][1] = TC(0);
    sN[0][0] = sN[0][1] = sN[1][0] = sN[1][1] = TC(0);

    bool bad = false;
    const int n_iter = (y1 - y0) + (PC ? 11 : 7);
    const int Rstart = y0 - HX;


    for (int it = 0; it < n_iter; ++it) {
        const int R = Rstart + it;
        const int b = it & 1, pb = b ^ 1;

        // Loads of this iteration (u_n at row R for stage A, f_n and j_n at
        // row R-2 for stage C) are issued first; stages D-F, which only use
        // earlier rows, run while they are in flight. Rows beyond a wall are
        // clamped to a valid address and their values discarded.
        const int rA = R, rC = R - 2;
        const bool nodeA = is_node(rA), nodeC = is_node(rC);
        const size_t oA = (size_t)rowc(rA) * nx + gx;
        const size_t oC = (size_t)rowc(rC) * nx + gx;
        const TU la0 = uin[oA], la1 = uin[plane + oA];
        TF lf[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) lf[i] = fin[i * plane + oC];
        const TJ lj0 = jin[oC], lj1 = jin[plane + oC];

        // ---------------- stage D: pull row R-4, moments
        // (rings not yet advanced this iteration: uR[k] = row R-1-k,
        //  sN[k] = row R-3-k, jN[k] = row R-3-k)
        const int rD = R - 4;
        {
            const TC a1 = s_f[pb][0][tl], a3 = s_f[pb][1][tr], a5 = s_f[pb][2][tl];
            const TC a6 = s_f[pb][3][tr], a7 = s_f[pb][4][tr], a8 = s_f[pb][5][tl];
            TC fn[9];
            fn[0] = o0[1];
            fn[1] = n1;
            fn[2] = o2[2];
            fn[3] = n3;
            fn[4] = o4;
            fn[5] = n5[1];
            fn[6] = n6[1];
            fn[7] = a7;
            fn[8] = a8;
            if (walled && rD == 0) {
                fn[2] = s_wall[0][0][t];
                fn[5] = s_wall[0][1][t];
                fn[6] = s_wall[0][2][t];
            }
            if (walled && rD == ny - 1) {
                fn[4] = s_wall[1][0][t];
                fn[7] = s_wall[1][1][t];
                fn[8] = s_wall[1][2][t];
            }
            n5[1] = n5[0];
            n5[0] = a5;
            n6[1] = n6[0];
            n6[0] = a6;
            n1 = a1;
            n3 = a3;

            const bool nodeD = is_node(rD);
            const TC jfx = ((fn[1] - fn[3]) + (fn[5] - fn[6])) + (fn[8] - fn[7]);
            const TC jfy = ((fn[2] - fn[4]) + (fn[5] + fn[6])) - (fn[7] + fn[8]);
            if (nodeD && out_col && rD >= y0 && rD < y1) {
                const size_t o = (size_t)rowi(rD) * nx + gx;
#pragma unroll
                for (int i = 0; i < 9; ++i) FS::store(fout, i * plane + o, fn[i], f_scale);
            }
            if constexpr (PC) {
                const TC jpx = jfx + TC(0.5) * sN[1][0];
                const TC jpy = jfy + TC(0.5) * sN[1][1];
                TU upx, upy;
                if (nodeD) {
                    upx = uR[3][0] + TU(TC(0.5) * (jpx + jN[1][0]));
                    upy = uR[3][1] + TU(TC(0.5) * (jpy + jN[1][1]));
                } else if (rD == ny && bc_hi != BC_PERIODIC) {
                    upx = ghost_hi(0, upR[0][0], upR[1][0], uw_hi_p[0]);
                    upy = ghost_hi(0, upR[0][1], upR[1][1], uw_hi_p[1]);
                } else if (rD == ny + 1 && bc_hi != BC_PERIODIC) {
                    upx = ghost_hi(1, upR[1][0], upR[2][0], uw_hi_p[0]);
                    upy = ghost_hi(1, upR[1][1], upR[2][1], uw_hi_p[1]);
                } else {
                    upx = upy = TU(0);
                }
#pragma unroll
                for (int k = 2; k > 0; --k) {
                    upR[k][0] = upR[k - 1][0];
                    upR[k][1] = upR[k - 1][1];
                    jfR[k][0] = jfR[k - 1][0];
                    jfR[k][1] = jfR[k - 1][1];
                }
                upR[0][0] = upx;
                upR[0][1] = upy;
                jfR[0][0] = jfx;
                jfR[0][1] = jfy;
                s_up[b][0][t] = upx;
                s_up[b][1][t] = upy;
            } else {
                // explicit: the source at t also serves the moment step
                if (nodeD && out_col && rD >= y0 && rD < y1) {
                    const TC jx = jfx + TC(0.5) * sN[1][0];
                    const TC jy = jfy + TC(0.5) * sN[1][1];
                    const TU ux = uR[3][0] + TU(TC(0.5) * (jx + jN[1][0]));
                    const TU uy = uR[3][1] + TU(TC(0.5) * (jy + jN[1][1]));
                    const size_t o = (size_t)rowi(rD) * nx + gx;
                    uout[o] = ux;
                    uout[plane + o] = uy;
                    jout[o] = TJ(jx);
                    jout[plane + o] = TJ(jy);
                    if (!isfinite((double)ux) || !isfinite((double)uy) || !isfinite((double)jx) ||
                        !isfinite((double)jy))
                        bad = true;
                }
            }
        }

        if constexpr (PC) {
            // ---------------- stage E: K^p at row R-5
            {
                TC H[4], K[4];
                H[0] = TC((s_up[pb][0][tr] - s_up[pb][0][tl]) * TU(0.5));
                H[2] = TC((s_up[pb][1][tr] - s_up[pb][1][tl]) * TU(0.5));
                TU um0 = upR[2][0], um1 = upR[2][1];
                if (walled && R - 5 == 0) {
                    um0 = ghost_lo(upR[1][0], upR[0][0], uw_lo_p[0]);
                    um1 = ghost_lo(upR[1][1], upR[0][1], uw_lo_p[1]);
                }
                H[1] = TC((upR[0][0] - um0) * TU(0.5));
                H[3] = TC((upR[0][1] - um1) * TU(0.5));
                stress_sum(H, lam, mu, K);
                s_kp[b][0][t] = K[0];
                s_kp[b][1][t] = K[2];
#pragma unroll
                for (int k = 2; k > 0; --k) {
                    kpA2[k][0] = kpA2[k - 1][0];
                    kpA2[k][1] = kpA2[k - 1][1];
                }
                kpA2[0][0] = K[1];
                kpA2[0][1] = K[3];
                hxpPrev[0] = hxpCur[0];
                hxpPrev[1] = hxpCur[1];
                hxpCur[0] = H[0];
                hxpCur[1] = H[2];
            }
            // ---------------- stage F: S^p at row R-6, new j and u
            const int rF = R - 6;
            if (is_node(rF) && out_col && rF >= y0 && rF < y1) {
                TC k12d = kpA2[2][0], k22d = kpA2[2][1];
                if (walled && rF == 0) ghost_lo_K(upR[2], upR[1], hxpPrev, hxpCur, uw_lo_p, k12d, k22d);
                const TC Sx = bx + TC(0.5) * (s_kp[pb][0][tr] - s_kp[pb][0][tl]) + TC(0.5) * (kpA2[0][0] - k12d);
                const TC Sy = by + TC(0.5) * (s_kp[pb][1][tr] - s_kp[pb][1][tl]) + TC(0.5) * (kpA2[0][1] - k22d);
                const TC jx = jfR[2][0] + TC(0.5) * Sx;
                const TC jy = jfR[2][1] + TC(0.5) * Sy;
                const TU ux = uR[5][0] + TU(TC(0.5) * (jx + jN[3][0]));
                const TU uy = uR[5][1] + TU(TC(0.5) * (jy + jN[3][1]));
                const size_t o = (size_t)rowi(rF) * nx + gx;
                uout[o] = ux;
                uout[plane + o] = uy;
                jout[o] = TJ(jx);
                jout[plane + o] = TJ(jy);
                if (!isfinite((double)ux) || !isfinite((double)uy) || !isfinite((double)jx) || !isfinite((double)jy))
                    bad = true;
            }
        }

        // ---------------- stage A: u_n at row R
#pragma unroll
        for (int k = NU - 1; k > 0; --k) {
            uR[k][0] = uR[k - 1][0];
            uR[k][1] = uR[k - 1][1];
        }
        if (nodeA) {
            uR[0][0] = la0;
            uR[0][1] = la1;
        } else if (R == ny && bc_hi != BC_PERIODIC) {
            uR[0][0] = ghost_hi(0, uR[1][0], uR[2][0], uw_hi_n[0]);
            uR[0][1] = ghost_hi(0, uR[1][1], uR[2][1], uw_hi_n[1]);
        } else if (R == ny + 1 && bc_hi != BC_PERIODIC) {
            uR[0][0] = ghost_hi(1, uR[2][0], uR[3][0], uw_hi_n[0]);
            uR[0][1] = ghost_hi(1, uR[2][1], uR[3][1], uw_hi_n[1]);
        } else {
            uR[0][0] = uR[0][1] = TU(0);
        }
        s_u[b][0][t] = uR[0][0];
        s_u[b][1][t] = uR[0][1];

        // ---------------- stage B: K at row R-1
        {
            TC H[4], K[4];
            H[0] = TC((s_u[pb][0][tr] - s_u[pb][0][tl]) * TU(0.5));
            H[2] = TC((s_u[pb][1][tr] - s_u[pb][1][tl]) * TU(0.5));
            const int rB = R - 1;
            TU um0 = uR[2][0], um1 = uR[2][1];
            if (walled && rB == 0) {
                um0 = ghost_lo(uR[1][0], uR[0][0], uw_lo_n[0]);
                um1 = ghost_lo(uR[1][1], uR[0][1], uw_lo_n[1]);
            }
            H[1] = TC((uR[0][0] - um0) * TU(0.5));
            H[3] = TC((uR[0][1] - um1) * TU(0.5));
            const TC J = stress_sum(H, lam, mu, K);
            if (out_col && rB >= y0 && rB < y1 && !(J > TC(0))) bad = true;
            s_k[b][0][t] = K[0];
            s_k[b][1][t] = K[2];
#pragma unroll
            for (int k = 2; k > 0; --k) {
                kA2[k][0] = kA2[k - 1][0];
                kA2[k][1] = kA2[k - 1][1];
            }
            kA2[0][0] = K[1];
            kA2[0][1] = K[3];
            hxPrev[0] = hxCur[0];
            hxPrev[1] = hxCur[1];
            hxCur[0] = H[0];
            hxCur[1] = H[2];
        }

        // ---------------- stage C: S_n at row R-2, collision
        {
            TC fc[9];
            TC k12d = kA2[2][0], k22d = kA2[2][1];
            if (walled && rC == 0) ghost_lo_K(uR[2], uR[1], hxPrev, hxCur, uw_lo_n, k12d, k22d);
            const TC Sx = bx + TC(0.5) * (s_k[pb][0][tr] - s_k[pb][0][tl]) + TC(0.5) * (kA2[0][0] - k12d);
            const TC Sy = by + TC(0.5) * (s_k[pb][1][tr] - s_k[pb][1][tl]) + TC(0.5) * (kA2[0][1] - k22d);
            sN[1][0] = sN[0][0];
            sN[1][1] = sN[0][1];
            sN[0][0] = Sx;
            sN[0][1] = Sy;
#pragma unroll
            for (int k = NJ - 1; k > 0; --k) {
                jN[k][0] = jN[k - 1][0];
                jN[k][1] = jN[k - 1][1];
            }
            if (nodeC) {
                TC f[9];
#pragma unroll
                for (int i = 0; i < 9; ++i) f[i] = FS::cvt(lf[i], f_inv);
                const TC jx = TC(lj0), jy = TC(lj1);
                jN[0][0] = jx;
                jN[0][1] = jy;
                TC r, pxx;
                collide(f, jx, jy, Sx, Sy, omega, fc, r, pxx);
                if (walled && rC == 0) {
                    TC w[3];
                    wall_populations(false, bc_lo, fc, p.val_lo, r, pxx, kA2[1][0], kA2[1][1], w);
                    s_wall[0][0][t] = w[0];
                    s_wall[0][1][t] = w[1];
                    s_wall[0][2][t] = w[2];
                }
                if (walled && rC == ny - 1) {
                    TC w[3];
                    wall_populations(true, bc_hi, fc, p.val_hi, r, pxx, kA2[1][0], kA2[1][1], w);
                    s_wall[1][0][t] = w[0];
                    s_wall[1][1][t] = w[1];
                    s_wall[1][2][t] = w[2];
                }
            } else {
#pragma unroll
                for (int i = 0; i < 9; ++i) fc[i] = TC(0);
                jN[0][0] = jN[0][1] = TC(0);
            }
            s_f[b][0][t] = fc[1];
            s_f[b][1][t] = fc[3];
            s_f[b][2][t] = fc[5];
            s_f[b][3][t] = fc[6];
            s_f[b][4][t] = fc[7];
            s_f[b][5][t] = fc[8];
            // own-column collision rings of the pull
            o2[2] = o2[1];
            o2[1] = o2[0];
            o2[0] = fc[2];
            o0[1] = o0[0];
            o0[0] = fc[0];
            o4 = fc[4];
        }
        __syncthreads();
    }
    if (bad) p.flag[0] = 1u;
}

// Single-plate step: one block per tile. Blocks are dealt round-robin to the
// 8 XCDs; the remap gives each XCD a run of consecutive tiles, which are
// vertical neighbours sharing their halo rows in that XCD's L2.
template <class PR, int BLOCK, bool PC, bool WALLED>
__global__ void __launch_bounds__(BLOCK) step_kernel(const StepParams p)
{
    const int nb = p.n_strips * p.n_segs;
    const int bid = blockIdx.x;
    const int xq = nb >> 3, xr = nb & 7;
    const int xcd = bid & 7, loc = bid >> 3;
    const int logical = xcd * xq + min(xcd, xr) + loc;
    const int strip = logical / p.n_segs;
    const int seg = logical - strip * p.n_segs;
    step_tile<PR, BLOCK, PC, WALLED>(p, strip, seg);
}

}  // namespace lbm
