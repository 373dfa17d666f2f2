// general_kernels.hpp -- one time step of a plate with walls on any edge, holes
// (Sec. 6, Sec. 7.2) or the j-extrapolation variant (end of Sec. 5), as one
// launch of 2D tiles.
//
// A block owns a TW x TH tile of output sites and works on a window around
// it in LDS. The stages of the step shrink the window one ring at a time,
// each reading only what the previous stage left in LDS:
//   u_n (ring RU, loaded with the ghost values beyond walls)
//   -> K = P + Pbar of u_n (ring RK)
//   -> source S_n, populations f_n, BGK collision f_col (ring RF)
//   -> pull streaming with the wall and hole rules, moments, predictor
//      u^p (ring RS)
//   -> K of u^p (ring RP) -> corrector j_{n+1}, u_{n+1} (ring RC).
// With 16-bit storage the new populations are stored as deviations from the
// reference equilibrium of the new state, whose gradient needs u_{n+1} one
// ring beyond the tile (RC = 1). The explicit scheme ends at the streaming
// ring. Every ring beyond the tile is recomputed by the neighbouring blocks
// as well: no stage waits for another block, so one launch is one step.
//
// The rules are those of the per-site formulation of the method:
// - a ghost node beyond a wall takes the value of the node next to the wall
//   (traction wall) or the straight line through the wall displacement (a
//   momentum wall: 2 uw - a, then 4 uw - 3 a); beyond two walls (a corner)
//   the x wall's rule applies to the y wall's ghost;
// - in a central difference a hole neighbour takes the node's own value;
// - the stress sum at a hole neighbour across axis n, as a material node
//   sees it, is K of that node's gradient with the derivatives along n set
//   to zero (reading Q23). Each node computes it from its own gradient, so a
//   hole one node wide, seen from both sides, needs nothing stored;
// - a link whose source lies beyond a wall or in a hole takes the wall's
//   bounce-back (eq. (25)) or anti-bounce-back (eq. (26)) rule.
#pragma once

#include "step_kernel.hpp"

namespace lbm {

enum : int { EDGE_XMIN = 0, EDGE_XMAX = 1, EDGE_YMIN = 2, EDGE_YMAX = 3 };

struct GenParams {
    const void *f_in, *u_in, *j_in;  // state n
    void *f_out, *u_out, *j_out;     // state n + 1
    const void *j_prev;              // j_{n-1} (j-extrapolation only)
    int nx, ny;
    long long plane;
    double omega, lam, mu, bx, by;  // lattice units
    int bc[4];                      // rule of each edge (BC_*), EDGE_* order
    double val[4][2];               // j* or T* of each edge, lattice units
    double uwb[4][2];               // momentum walls: displacement uwb + j* n at step n
    double f_scale, f_inv_scale;
    long long step;                 // index n of the input state
    int sr;
    unsigned long long seed;
    int pc;  // explicit (0), predictor-corrector (1), j extrapolated for the predictor (2)
    unsigned *flag;
    const unsigned char *mask;   // [ny][nx]: 1 material, 0 hole; nullptr: no holes
    const unsigned char *tiles;  // TILE_* bits of each tile (row-major); nullptr: no holes
    const int *tlist;            // the tiles to launch (row-major indices); nullptr: every tile
    int n_tlist;
};

// D2Q9 of this implementation (see lattice.hpp)
__device__ constexpr int kGx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__device__ constexpr int kGy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
__device__ constexpr int kGopp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

template <class TC>
__device__ __forceinline__ TC gweight(int i)
{
    return i == 0 ? TC(4.0 / 9.0) : (i < 5 ? TC(1.0 / 9.0) : TC(1.0 / 36.0));
}

// Ghost value k = 1 or 2 spacings beyond a wall from the node next to it
// (a): at a momentum wall the straight line through the wall displacement
// uw and a (2 uw - a, then 4 uw - 3 a), at a traction wall the value a.
template <class TU>
__device__ __forceinline__ TU gen_ghost(int kind, TU uw, TU a, int k)
{
    if (kind == BC_NEUMANN) return a;
    return k == 1 ? TU(2) * uw - a : TU(4) * uw - TU(3) * a;
}

// momentum-wall displacement of edge e at step t (lattice units)
template <class TU>
__device__ __forceinline__ TU gen_uw(const GenParams &p, int e, int a, double t)
{
    return TU(p.uwb[e][a] + p.val[e][a] * t);
}

// Threads of a tile's block.
constexpr int kTileBlock = 512;

// Tile shape and the rings (distance from the tile) of the stages.
// MODE 0: explicit; 1: predictor-corrector (also with j extrapolated).
template <class PR, int MODE, bool SMALL = false>
struct TileCfg {
    using TU = typename PR::TU;
    using TC = typename PR::TC;
    static constexpr bool DEV = FStore<typename PR::TF>::kDeviation;
    static constexpr int BLOCK = kTileBlock;
    static constexpr int TW = 32;
    // Rows per tile: LDS within 80 KB, so two blocks share a CU, and few
    // enough sites per thread on the streaming ring (at most two) and, with
    // deviation storage, on the collision ring (at most two) that the
    // registers holding them are not spilled (16-bit storage with eight rows:
    // 80 VGPRs, 72.6 KB; 0.385 against 0.415 ms per step with four rows on
    // the 4096² plate with a hole). SMALL: two rows, so that every stage's
    // ring fits one round of the block's threads, for plates whose tiles fit
    // one per compute unit (the step is then bound by the tile's latency,
    // not by the chip's throughput).
    static constexpr int TH = SMALL ? 2 : (sizeof(TC) == 8 ? 6 : 8);
    static constexpr int RC = DEV ? 1 : 0;          // corrector (PC) or update (explicit)
    static constexpr int RS = MODE ? RC + 2 : RC;   // streaming, predictor
    static constexpr int RP = MODE ? RC + 1 : 0;    // K of u^p
    static constexpr int RF = RS + 1;               // collision
    static constexpr int RK = RS + 2;               // K of u_n
    static constexpr int RU = RS + 3;               // u_n
    static constexpr int W(int r) { return TW + 2 * r; }
    static constexpr int H(int r) { return TH + 2 * r; }
    static constexpr int N(int r) { return W(r) * H(r); }
};

template <class PR, int MODE, bool SMALL = false>
struct TileLdsG {
    using C = TileCfg<PR, MODE, SMALL>;
    static_assert(C::N(C::RS) <= 2 * C::BLOCK && C::N(C::RC) <= 2 * C::BLOCK,
                  "two sites per thread at most on the streaming and corrector rings");
    using TU = typename PR::TU;
    using TC = typename PR::TC;
    TU u[2][C::N(C::RU)];
    TC k[4][C::N(C::RK)];
    TC fc[9][C::N(C::RF)];
    TC jc[2][MODE || C::DEV ? C::N(C::RC) : 1];  // jf, then j_{n+1}, at the corrector ring
    TC jn[2][C::N(C::RF)];                       // j_n on the collision ring
    TU un[2][MODE ? C::N(C::RC) : 1];            // u_n at the corrector ring
    TC fn[9][C::DEV ? C::TW * C::TH : 1];        // new populations of the tile (deviation storage)
    unsigned char kind[C::N(C::RU)];
};

enum : unsigned char { SITE_NODE = 1, SITE_HOLE = 2, SITE_GHOST = 4 };

// Bits of a tile's entry in the tile table (built on the host): the window
// holds a hole node; the tile holds a material node; the fused step kernel
// computes the tile (it lies clear of walls and holes).
enum : unsigned char { TILE_HOLES = 1, TILE_MATERIAL = 2, TILE_FUSED = 4 };

template <class PR, int MODE, bool SMALL = false>
struct TileStep {
    using C = TileCfg<PR, MODE, SMALL>;
    using TF = typename PR::TF;
    using TU = typename PR::TU;
    using TJ = typename PR::TJ;
    using TC = typename PR::TC;
    using FS = FStore<TF>;
    using Lds = TileLdsG<PR, MODE, SMALL>;

    const GenParams &p;
    Lds &L;
    const int x0, y0;
    const bool perx, pery;
    const TC lam, mu, omega;
    // From the tile table (all set without a mask): the window holds a hole
    // node, so the hole rules are tested; the tile holds a material node (a
    // tile wholly inside a hole computes nothing: its sites only get the
    // zero state of hole nodes).
    const bool holes, active;

    __device__ TileStep(const GenParams &p_, Lds &l, int x0_, int y0_, unsigned char tf)
        : p(p_), L(l), x0(x0_), y0(y0_), perx(p_.bc[EDGE_XMIN] == BC_PERIODIC),
          pery(p_.bc[EDGE_YMIN] == BC_PERIODIC), lam(TC(p_.lam)), mu(TC(p_.mu)), omega(TC(p_.omega)),
          holes((tf & TILE_HOLES) != 0), active((tf & TILE_MATERIAL) != 0)
    {
    }

    // index of tile-relative (dx, dy) in an array over ring r
    template <int R>
    __device__ __forceinline__ static int at(int dx, int dy)
    {
        return (dy + R) * C::W(R) + (dx + R);
    }

    // Plate coordinates of tile-relative (dx, dy): wrapped across periodic
    // edges; bx, by: spacings beyond a wall (0 inside the plate).
    __device__ __forceinline__ void coords(int dx, int dy, int &x, int &y, int &bx, int &by) const
    {
        x = x0 + dx;
        y = y0 + dy;
        bx = by = 0;
        if (x < 0 || x >= p.nx) {
            if (perx) {
                x %= p.nx;
                if (x < 0) x += p.nx;
            } else {
                bx = x < 0 ? -x : x - (p.nx - 1);
            }
        }
        if (y < 0 || y >= p.ny) {
            if (pery) {
                y %= p.ny;
                if (y < 0) y += p.ny;
            } else {
                by = y < 0 ? -y : y - (p.ny - 1);
            }
        }
    }

    __device__ __forceinline__ unsigned char kind(int dx, int dy) const { return L.kind[at<C::RU>(dx, dy)]; }
    __device__ __forceinline__ bool hole(int dx, int dy) const { return kind(dx, dy) & SITE_HOLE; }
    __device__ __forceinline__ TU uval(int a, int dx, int dy) const { return L.u[a][at<C::RU>(dx, dy)]; }
    __device__ __forceinline__ TC kval(int c, int dx, int dy) const { return L.k[c][at<C::RK>(dx, dy)]; }

    // Ghost value at (dx, dy), bx and by spacings beyond the walls, from the
    // value a of the node next to the wall(s); step t.
    __device__ __forceinline__ TU ghost(int aidx, int dx, int dy, int bx, int by, TU a, double t) const
    {
        if (by) {
            const int e = y0 + dy < 0 ? EDGE_YMIN : EDGE_YMAX;
            a = gen_ghost<TU>(p.bc[e], gen_uw<TU>(p, e, aidx, t), a, by);
        }
        if (bx) {
            const int e = x0 + dx < 0 ? EDGE_XMIN : EDGE_XMAX;
            a = gen_ghost<TU>(p.bc[e], gen_uw<TU>(p, e, aidx, t), a, bx);
        }
        return a;
    }

    // tile-relative position of the node next to the wall(s) for a ghost
    __device__ __forceinline__ void edge_of(int dx, int dy, int bx, int by, int &ex, int &ey) const
    {
        ex = dx + (bx ? (x0 + dx < 0 ? bx : -bx) : 0);
        ey = dy + (by ? (y0 + dy < 0 ? by : -by) : 0);
    }

    // central-difference gradient of the displacement in LDS at (dx, dy); a
    // hole neighbour takes the node's own value
    __device__ __forceinline__ void grad(int dx, int dy, TC H[4]) const
    {
        const bool m = holes;
        const bool hxp = m && hole(dx + 1, dy), hxm = m && hole(dx - 1, dy);
        const bool hyp = m && hole(dx, dy + 1), hym = m && hole(dx, dy - 1);
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            const TU c = uval(a, dx, dy);
            const TU xp = hxp ? c : uval(a, dx + 1, dy), xm = hxm ? c : uval(a, dx - 1, dy);
            const TU yp = hyp ? c : uval(a, dx, dy + 1), ym = hym ? c : uval(a, dx, dy - 1);
            H[2 * a + 0] = TC((xp - xm) * TU(0.5));
            H[2 * a + 1] = TC((yp - ym) * TU(0.5));
        }
    }

    // K at the hole neighbour across axis n as node (dx, dy) sees it
    __device__ __forceinline__ void k_hole(const TC H[4], int n, TC K[4]) const
    {
        TC Hn[4] = {H[0], H[1], H[2], H[3]};
        Hn[n] = TC(0);
        Hn[2 + n] = TC(0);
        stress_sum(Hn, lam, mu, K);
    }

    // Source S = rho0 b + div K at node (dx, dy) (eq. (23)) from the K in
    // LDS; across a hole the node's own hole K.
    __device__ __forceinline__ void source(int dx, int dy, TC S[2]) const
    {
        TC kxp[4], kxm[4], kyp[4], kym[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            kxp[c] = kval(c, dx + 1, dy);
            kxm[c] = kval(c, dx - 1, dy);
            kyp[c] = kval(c, dx, dy + 1);
            kym[c] = kval(c, dx, dy - 1);
        }
        if (holes) {
            const bool hxp = hole(dx + 1, dy), hxm = hole(dx - 1, dy);
            const bool hyp = hole(dx, dy + 1), hym = hole(dx, dy - 1);
            if (hxp || hxm || hyp || hym) {
                TC H[4], kh[4];
                grad(dx, dy, H);
                if (hxp || hxm) {
                    k_hole(H, 0, kh);
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        if (hxp) kxp[c] = kh[c];
                        if (hxm) kxm[c] = kh[c];
                    }
                }
                if (hyp || hym) {
                    k_hole(H, 1, kh);
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        if (hyp) kyp[c] = kh[c];
                        if (hym) kym[c] = kh[c];
                    }
                }
            }
        }
        S[0] = TC(p.bx) + TC(0.5) * (kxp[0] - kxm[0]) + TC(0.5) * (kyp[1] - kym[1]);
        S[1] = TC(p.by) + TC(0.5) * (kxp[2] - kxm[2]) + TC(0.5) * (kyp[3] - kym[3]);
    }

    // populations of state n at node (dx, dy), site s (with deviation
    // storage plus the reference equilibrium of the stored state)
    __device__ __forceinline__ void load_f(int dx, int dy, size_t s, TC jn0, TC jn1, TC f[9]) const
    {
        const size_t pl = (size_t)p.plane;
        const TF *fin = static_cast<const TF *>(p.f_in);
#pragma unroll
        for (int i = 0; i < 9; ++i) f[i] = FS::load(fin, i * pl + s, TC(p.f_inv_scale));
        if constexpr (FS::kDeviation) {
            TC H[4], fr[9];
            grad(dx, dy, H);
            ref_eq(H, jn0, jn1, fr);
#pragma unroll
            for (int i = 0; i < 9; ++i) f[i] = fr[i] + f[i];
        }
    }

    // Value the wall returns into direction opp(o) at node (dx, dy) for the
    // link o that leaves through the wall(s); sx, sy: outward signs of the
    // walls crossed. Bounce-back with the wall momentum (eq. (25)) if a
    // crossed wall is a momentum wall (the mean j* if both are); otherwise
    // anti-bounce-back (eq. (26)) with r_bd and Pbar* at the node: each
    // traction wall's column of Pbar* is -s T* + K n, K at the wall the mean
    // of the node's and the one beyond the wall (a ghost node, or the hole K
    // the node sees); a tangential entry keeps the populations' second
    // moment, and at a corner the off-diagonal entry is the mean of both
    // walls' values. m: r, Pxx, Pyy, Pxy of the node's populations.
    __device__ __forceinline__ TC wall(int dx, int dy, int o, int sx, int sy, TC fco, bool hole_wall, const TC m[4],
                                       const TC H[4]) const
    {
        const int ex = sx < 0 ? EDGE_XMIN : EDGE_XMAX, ey = sy < 0 ? EDGE_YMIN : EDGE_YMAX;
        const bool ddx = !hole_wall && sx != 0 && p.bc[ex] == BC_DIRICHLET;
        const bool ddy = !hole_wall && sy != 0 && p.bc[ey] == BC_DIRICHLET;
        const TC w = gweight<TC>(o);
        const TC cx = TC(kGx[o]), cy = TC(kGy[o]);
        if (ddx || ddy) {
            TC jx, jy;
            if (ddx && ddy) {
                jx = TC(0.5 * (p.val[ex][0] + p.val[ey][0]));
                jy = TC(0.5 * (p.val[ex][1] + p.val[ey][1]));
            } else {
                const int e = ddx ? ex : ey;
                jx = TC(p.val[e][0]);
                jy = TC(p.val[e][1]);
            }
            return fco - TC(6) * w * (cx * jx + cy * jy);
        }
        const double tx0 = hole_wall ? 0.0 : p.val[ex][0], tx1 = hole_wall ? 0.0 : p.val[ex][1];
        const double ty0 = hole_wall ? 0.0 : p.val[ey][0], ty1 = hole_wall ? 0.0 : p.val[ey][1];
        const TC r = m[0];
        TC Pxx = m[1], Pyy = m[2], Pxy = m[3];
        TC qx0 = 0, qx1 = 0, qy0 = 0, qy1 = 0;
        if (sx) {
            TC kb0, kb2;
            if (holes && hole(dx + sx, dy)) {
                TC kh[4];
                k_hole(H, 0, kh);
                kb0 = kh[0];
                kb2 = kh[2];
            } else {
                kb0 = kval(0, dx + sx, dy);
                kb2 = kval(2, dx + sx, dy);
            }
            const TC sg = TC(sx);
            qx0 = -sg * TC(tx0) + TC(0.5) * (kval(0, dx, dy) + kb0);
            qx1 = -sg * TC(tx1) + TC(0.5) * (kval(2, dx, dy) + kb2);
        }
        if (sy) {
            TC kb1, kb3;
            if (holes && hole(dx, dy + sy)) {
                TC kh[4];
                k_hole(H, 1, kh);
                kb1 = kh[1];
                kb3 = kh[3];
            } else {
                kb1 = kval(1, dx, dy + sy);
                kb3 = kval(3, dx, dy + sy);
            }
            const TC sg = TC(sy);
            qy0 = -sg * TC(ty0) + TC(0.5) * (kval(1, dx, dy) + kb1);
            qy1 = -sg * TC(ty1) + TC(0.5) * (kval(3, dx, dy) + kb3);
        }
        if (sx && sy) {
            Pxx = qx0;
            Pyy = qy1;
            Pxy = TC(0.5) * (qx1 + qy0);
        } else if (sy) {
            Pxy = qy0;
            Pyy = qy1;
        } else {
            Pxx = qx0;
            Pxy = qx1;
        }
        const TC third = TC(1) / TC(3);
        const TC axx = Pxx - r * third, ayy = Pyy - r * third;
        const TC q = axx * cx * cx + TC(2) * Pxy * cx * cy + ayy * cy * cy - (axx + ayy) * third;
        return -fco + TC(2) * w * (r + TC(4.5) * q);
    }

    // Pull streaming (eq. (5)) at node (dx, dy), site s: a link whose source
    // lies beyond a wall or in a hole takes the wall's rule.
    __device__ __forceinline__ void stream(int dx, int dy, size_t s, TC jn0, TC jn1, TC fn[9]) const
    {
        constexpr int R = C::RF;
        const int xn = x0 + dx, yn = y0 + dy;  // unwrapped: a source beyond a wall leaves [0, n)
        bool any = false;
        int cross[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const int sx = dx - kGx[i], sy = dy - kGy[i];
            int c = 0;
            if (i && holes && hole(sx, sy)) {
                c = 4;
            } else {
                const bool bx = !perx && (xn - kGx[i] < 0 || xn - kGx[i] >= p.nx);
                const bool by = !pery && (yn - kGy[i] < 0 || yn - kGy[i] >= p.ny);
                c = (bx ? 1 : 0) | (by ? 2 : 0);
            }
            cross[i] = c;
            any |= c != 0;
            fn[i] = L.fc[i][at<R>(sx, sy)];
        }
        if (!any) return;
        TC f[9], H[4], m[4];
        load_f(dx, dy, s, jn0, jn1, f);
        grad(dx, dy, H);
        m[0] = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
        const TC dsum = (f[5] + f[6]) + (f[7] + f[8]);
        m[1] = (f[1] + f[3]) + dsum;
        m[2] = (f[2] + f[4]) + dsum;
        m[3] = (f[5] - f[6]) + (f[7] - f[8]);
#pragma unroll
        for (int i = 1; i < 9; ++i) {
            if (!cross[i]) continue;
            const int o = kGopp[i];  // the link that left through the wall
            const TC fco = L.fc[o][at<R>(dx, dy)];
            if (cross[i] == 4) {
                // the wall its axis step enters, or both for the diagonal
                // through a hole corner
                const bool hx = kGx[o] && hole(dx + kGx[o], dy), hy = kGy[o] && hole(dx, dy + kGy[o]);
                const bool both = !hx && !hy;
                fn[i] = wall(dx, dy, o, (hx || both) ? kGx[o] : 0, (hy || both) ? kGy[o] : 0, fco, true, m, H);
            } else {
                fn[i] = wall(dx, dy, o, (cross[i] & 1) ? kGx[o] : 0, (cross[i] & 2) ? kGy[o] : 0, fco, false, m, H);
            }
        }
    }

    // Fill the ghost nodes of ring R in L.u from the nodes next to the walls
    // (step t). The caller has written the plate's nodes and synchronised.
    template <int R>
    __device__ __forceinline__ void ghost_fill(double t)
    {
        if ((perx && pery) || !active) return;
        constexpr int NR = C::N(R), PR_ = (NR + C::BLOCK - 1) / C::BLOCK;
#pragma unroll
        for (int q = 0; q < PR_; ++q) {
            const int w = threadIdx.x + q * C::BLOCK;
            if (w >= NR) continue;
            const int dy = w / C::W(R) - R, dx = w % C::W(R) - R;
            int x, y, bx, by;
            coords(dx, dy, x, y, bx, by);
            if (!(bx | by) || bx > 2 || by > 2) continue;
            int ex, ey;
            edge_of(dx, dy, bx, by, ex, ey);
#pragma unroll
            for (int a = 0; a < 2; ++a) L.u[a][at<C::RU>(dx, dy)] = ghost(a, dx, dy, bx, by, uval(a, ex, ey), t);
        }
    }

    // K = P + Pbar (eqs. (15), (27)) of the displacement in LDS on ring R;
    // flag: J <= 0 at a node of the tile (u_n only)
    template <int R>
    __device__ __forceinline__ void stress(bool flag)
    {
        constexpr int NR = C::N(R), PR_ = (NR + C::BLOCK - 1) / C::BLOCK;
        bool bad = false;
#pragma unroll
        for (int q = 0; q < PR_; ++q) {
            const int w = threadIdx.x + q * C::BLOCK;
            if (w >= NR || !active) continue;
            const int dy = w / C::W(R) - R, dx = w % C::W(R) - R;
            const unsigned char kd = kind(dx, dy);
            if (kd & SITE_HOLE) continue;
            TC H[4], K[4];
            grad(dx, dy, H);
            const TC J = stress_sum(H, lam, mu, K);
#pragma unroll
            for (int c = 0; c < 4; ++c) L.k[c][at<C::RK>(dx, dy)] = K[c];
            if (flag && (kd & SITE_NODE) && dx >= 0 && dx < C::TW && dy >= 0 && dy < C::TH &&
                x0 + dx < p.nx && y0 + dy < p.ny && !(J > TC(0)))
                bad = true;
        }
        if (bad) p.flag[0] = 1u;
    }

    __device__ __forceinline__ bool in_tile(int dx, int dy) const
    {
        return dx >= 0 && dx < C::TW && dy >= 0 && dy < C::TH && x0 + dx < p.nx && y0 + dy < p.ny;
    }

    __device__ __forceinline__ void run()
    {
        const size_t pl = (size_t)p.plane;
        const double tn = (double)p.step, tn1 = (double)(p.step + 1);
        const TF *fin = static_cast<const TF *>(p.f_in);
        const TU *uin = static_cast<const TU *>(p.u_in);
        const TJ *jin = static_cast<const TJ *>(p.j_in);
        TU *uout = static_cast<TU *>(p.u_out);
        TJ *jout = static_cast<TJ *>(p.j_out);
        const bool sr = FS::kStochastic && p.sr;
        const uint32_t key = sr ? sr_key(p.seed, p.step + 1) : 0u;
        const TC inv = TC(p.f_inv_scale);
        bool bad = false;

        // Every load of the state is issued here, before the first barrier
        // waits for all of them at once: f_n and j_n of the collision ring
        // into registers, u_n (or the edge value a ghost is made from) and
        // the mask on the u ring.
        constexpr int NF = C::N(C::RF), PF = (NF + C::BLOCK - 1) / C::BLOCK;
        constexpr int NU = C::N(C::RU), PU = (NU + C::BLOCK - 1) / C::BLOCK;
        TF fr[PF][9];
        TJ jr[PF][2];
#pragma unroll
        for (int q = 0; q < PF; ++q) {
#pragma unroll
            for (int i = 0; i < 9; ++i) fr[q][i] = TF(0);
            jr[q][0] = jr[q][1] = TJ(0);
            const int w = threadIdx.x + q * C::BLOCK;
            if (w >= NF) continue;
            const int dy = w / C::W(C::RF) - C::RF, dx = w % C::W(C::RF) - C::RF;
            int x, y, bx, by;
            coords(dx, dy, x, y, bx, by);
            if (bx | by) continue;
            const size_t s = (size_t)y * p.nx + x;
#pragma unroll
            for (int i = 0; i < 9; ++i) fr[q][i] = fin[i * pl + s];
            jr[q][0] = jin[s];
            jr[q][1] = jin[pl + s];
        }
        TU ur[PU][2];
        unsigned char mr[PU];
#pragma unroll
        for (int q = 0; q < PU; ++q) {
            ur[q][0] = ur[q][1] = TU(0);
            mr[q] = 1;
            const int w = threadIdx.x + q * C::BLOCK;
            if (w >= NU) continue;
            const int dy = w / C::W(C::RU) - C::RU, dx = w % C::W(C::RU) - C::RU;
            int x, y, bx, by;
            coords(dx, dy, x, y, bx, by);
            if (bx > 2 || by > 2) continue;
            const int xe = x < 0 ? 0 : (x >= p.nx ? p.nx - 1 : x);
            const int ye = y < 0 ? 0 : (y >= p.ny ? p.ny - 1 : y);
            const size_t s = (size_t)ye * p.nx + xe;
            ur[q][0] = uin[s];
            ur[q][1] = uin[pl + s];
            if (p.mask && !(bx | by)) mr[q] = p.mask[s];
        }
#pragma unroll
        for (int q = 0; q < PU; ++q) {
            const int w = threadIdx.x + q * C::BLOCK;
            if (w >= NU) continue;
            const int dy = w / C::W(C::RU) - C::RU, dx = w % C::W(C::RU) - C::RU;
            int x, y, bx, by;
            coords(dx, dy, x, y, bx, by);
            unsigned char kd = SITE_GHOST;
            TU v0 = ur[q][0], v1 = ur[q][1];
            if (!(bx | by)) {
                kd = (mr[q] & 1) ? SITE_NODE : SITE_HOLE;
            } else if (bx <= 2 && by <= 2) {
                v0 = ghost(0, dx, dy, bx, by, v0, tn);
                v1 = ghost(1, dx, dy, bx, by, v1, tn);
            }
            L.kind[w] = kd;
            L.u[0][w] = v0;
            L.u[1][w] = v1;
        }
        __syncthreads();

        stress<C::RK>(true);
        __syncthreads();

        // source, populations and collision on the collision ring
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            const int w = threadIdx.x + q * C::BLOCK;
            if (w >= NF) continue;
            const int dy = w / C::W(C::RF) - C::RF, dx = w % C::W(C::RF) - C::RF;
            if (!active || !(kind(dx, dy) & SITE_NODE)) continue;
            const TC jn0 = TC(jr[q][0]), jn1 = TC(jr[q][1]);
            TC S[2], f[9], fc[9], r, pxx;
            source(dx, dy, S);
#pragma unroll
            for (int i = 0; i < 9; ++i) f[i] = FS::cvt(fr[q][i], inv);
            if constexpr (FS::kDeviation) {
                TC H[4], fq[9];
                grad(dx, dy, H);
                ref_eq(H, jn0, jn1, fq);
#pragma unroll
                for (int i = 0; i < 9; ++i) f[i] = fq[i] + f[i];
            }
            collide(f, jn0, jn1, S[0], S[1], omega, fc, r, pxx);
#pragma unroll
            for (int i = 0; i < 9; ++i) L.fc[i][w] = fc[i];
            L.jn[0][w] = jn0;
            L.jn[1][w] = jn1;
        }
        __syncthreads();

        // streaming and moments on the streaming ring: the predictor u^p
        // (PC) or the new state (explicit), held in registers until the
        // ring's reads of L.u are over
        constexpr int NS = C::N(C::RS), PS = (NS + C::BLOCK - 1) / C::BLOCK;
        TU un[PS][2];
#pragma unroll
        for (int q = 0; q < PS; ++q) {
            un[q][0] = un[q][1] = TU(0);
            const int w = threadIdx.x + q * C::BLOCK;
            if (w >= NS) continue;
            const int dy = w / C::W(C::RS) - C::RS, dx = w % C::W(C::RS) - C::RS;
            const unsigned char kd = kind(dx, dy);
            int x, y, bx, by;
            coords(dx, dy, x, y, bx, by);
            const size_t s = (size_t)y * p.nx + x;
            if (!active || !(kd & SITE_NODE)) {
                if ((kd & SITE_HOLE) && MODE == 0 && in_tile(dx, dy)) {
                    uout[s] = uout[pl + s] = TU(0);
                    jout[s] = jout[pl + s] = TJ(0);
                }
                continue;
            }
            const TC jn0 = L.jn[0][at<C::RF>(dx, dy)], jn1 = L.jn[1][at<C::RF>(dx, dy)];
            TC fn[9], S[2];
            stream(dx, dy, s, jn0, jn1, fn);
            if (in_tile(dx, dy)) {
                if constexpr (C::DEV) {
#pragma unroll
                    for (int i = 0; i < 9; ++i) L.fn[i][dy * C::TW + dx] = fn[i];
                } else {
                    store_site<FS>(static_cast<TF *>(p.f_out), pl, (uint32_t)s, fn, TC(p.f_scale), sr, key);
                }
            }
            const TC jfx = ((fn[1] - fn[3]) + (fn[5] - fn[6])) + (fn[8] - fn[7]);
            const TC jfy = ((fn[2] - fn[4]) + (fn[5] + fn[6])) - (fn[7] + fn[8]);
            source(dx, dy, S);
            const TU u0 = uval(0, dx, dy), u1 = uval(1, dx, dy);
            if constexpr (MODE) {
                if (dx >= -C::RC && dx < C::TW + C::RC && dy >= -C::RC && dy < C::TH + C::RC) {
                    const int c = at<C::RC>(dx, dy);
                    L.jc[0][c] = jfx;
                    L.jc[1][c] = jfy;
                    L.un[0][c] = u0;
                    L.un[1][c] = u1;
                }
                TC jpx = jfx + TC(0.5) * S[0], jpy = jfy + TC(0.5) * S[1];
                if (p.pc == 2) {
                    const TJ *jold = static_cast<const TJ *>(p.j_prev);
                    jpx = TC(2) * jn0 - TC(jold[s]);
                    jpy = TC(2) * jn1 - TC(jold[pl + s]);
                }
                un[q][0] = u0 + TU(TC(0.5) * (jpx + jn0));
                un[q][1] = u1 + TU(TC(0.5) * (jpy + jn1));
            } else {
                const TC j0 = jfx + TC(0.5) * S[0], j1 = jfy + TC(0.5) * S[1];
                un[q][0] = u0 + TU(TC(0.5) * (j0 + jn0));
                un[q][1] = u1 + TU(TC(0.5) * (j1 + jn1));
                if constexpr (C::DEV) {
                    L.jc[0][at<C::RC>(dx, dy)] = j0;
                    L.jc[1][at<C::RC>(dx, dy)] = j1;
                }
                if (in_tile(dx, dy)) {
                    uout[s] = un[q][0];
                    uout[pl + s] = un[q][1];
                    jout[s] = TJ(j0);
                    jout[pl + s] = TJ(j1);
                    if (!isfinite((double)un[q][0]) || !isfinite((double)un[q][1]) || !isfinite((double)j0) ||
                        !isfinite((double)j1))
                        bad = true;
                }
            }
        }
        __syncthreads();

        if constexpr (MODE) {
            // K of u^p on its ring, then the corrector
#pragma unroll
            for (int q = 0; q < PS; ++q) {
                const int w = threadIdx.x + q * C::BLOCK;
                if (w < NS) {
                    const int dy = w / C::W(C::RS) - C::RS, dx = w % C::W(C::RS) - C::RS;
                    L.u[0][at<C::RU>(dx, dy)] = un[q][0];
                    L.u[1][at<C::RU>(dx, dy)] = un[q][1];
                }
            }
            __syncthreads();
            if (!(perx && pery)) {  // ghost sites exist only beyond a wall (uniform)
                ghost_fill<C::RS>(tn1);
                __syncthreads();
            }
            stress<C::RP>(false);
            __syncthreads();

            constexpr int NC = C::N(C::RC), PC_ = (NC + C::BLOCK - 1) / C::BLOCK;
#pragma unroll
            for (int q = 0; q < PC_; ++q) {
                const int w = threadIdx.x + q * C::BLOCK;
                if (w >= NC) continue;
                const int dy = w / C::W(C::RC) - C::RC, dx = w % C::W(C::RC) - C::RC;
                const unsigned char kd = kind(dx, dy);
                int x, y, bx, by;
                coords(dx, dy, x, y, bx, by);
                const size_t s = (size_t)y * p.nx + x;
                if (!active || !(kd & SITE_NODE)) {
                    if ((kd & SITE_HOLE) && in_tile(dx, dy)) {
                        uout[s] = uout[pl + s] = TU(0);
                        jout[s] = jout[pl + s] = TJ(0);
                    }
                    continue;
                }
                TC Sp[2];
                source(dx, dy, Sp);
                const int f = at<C::RF>(dx, dy);
                const TC jn0 = L.jn[0][f], jn1 = L.jn[1][f];
                const TC j0 = L.jc[0][w] + TC(0.5) * Sp[0], j1 = L.jc[1][w] + TC(0.5) * Sp[1];
                const TU u0 = L.un[0][w] + TU(TC(0.5) * (j0 + jn0));
                const TU u1 = L.un[1][w] + TU(TC(0.5) * (j1 + jn1));
                if constexpr (C::DEV) {
                    // u_{n+1} and j_{n+1} in place of this site's u_n and jf
                    L.un[0][w] = u0;
                    L.un[1][w] = u1;
                    L.jc[0][w] = j0;
                    L.jc[1][w] = j1;
                }
                if (in_tile(dx, dy)) {
                    uout[s] = u0;
                    uout[pl + s] = u1;
                    jout[s] = TJ(j0);
                    jout[pl + s] = TJ(j1);
                    if (!isfinite((double)u0) || !isfinite((double)u1) || !isfinite((double)j0) ||
                        !isfinite((double)j1))
                        bad = true;
                }
            }
            if constexpr (C::DEV) {
                __syncthreads();
                for (int w = threadIdx.x; w < NC; w += C::BLOCK) {
                    const int dy = w / C::W(C::RC) - C::RC, dx = w % C::W(C::RC) - C::RC;
                    if (kind(dx, dy) & SITE_NODE) {
                        L.u[0][at<C::RU>(dx, dy)] = L.un[0][w];
                        L.u[1][at<C::RU>(dx, dy)] = L.un[1][w];
                    }
                }
            }
        } else if constexpr (C::DEV) {
            // explicit: the new state of the update ring is in registers
#pragma unroll
            for (int q = 0; q < PS; ++q) {
                const int w = threadIdx.x + q * C::BLOCK;
                if (w < NS) {
                    const int dy = w / C::W(C::RS) - C::RS, dx = w % C::W(C::RS) - C::RS;
                    L.u[0][at<C::RU>(dx, dy)] = un[q][0];
                    L.u[1][at<C::RU>(dx, dy)] = un[q][1];
                }
            }
        }

        if constexpr (C::DEV) {
            // store the new populations' deviation from the reference
            // equilibrium of the new state (the gradient of u_{n+1} and
            // j_{n+1}), as the next step's loads rebuild it
            __syncthreads();
            if (!(perx && pery)) {
                ghost_fill<C::RC>(tn1);
                __syncthreads();
            }
            for (int w = threadIdx.x; w < C::TW * C::TH; w += C::BLOCK) {
                const int dy = w / C::TW, dx = w % C::TW;
                if (!in_tile(dx, dy) || !(kind(dx, dy) & SITE_NODE)) continue;
                int x, y, bx, by;
                coords(dx, dy, x, y, bx, by);
                const size_t s = (size_t)y * p.nx + x;
                TC H[4], fq[9], dv[9];
                grad(dx, dy, H);
                const int c = at<C::RC>(dx, dy);
                ref_eq(H, TC(TJ(L.jc[0][c])), TC(TJ(L.jc[1][c])), fq);
#pragma unroll
                for (int i = 0; i < 9; ++i) dv[i] = L.fn[i][w] - fq[i];
                store_site<FS>(static_cast<TF *>(p.f_out), pl, (uint32_t)s, dv, TC(p.f_scale), sr, key);
            }
        }
        if (bad) p.flag[0] = 1u;
    }
};

// One block per tile. Blocks are dealt round-robin to the 8 XCDs; the remap
// gives each XCD a run of consecutive tiles, row by row of tiles, so the
// windows of horizontal neighbours overlap in one L2. (Column by column,
// which puts vertical neighbours one after another, measured 10 % slower.)
template <class PR, int MODE, bool SMALL = false>
__global__ void __launch_bounds__(kTileBlock) tile_step_kernel(const GenParams p, const int nbx, const int nb)
{
    using C = TileCfg<PR, MODE, SMALL>;
    __shared__ TileLdsG<PR, MODE, SMALL> lds;
    const int bid = blockIdx.x;
    const int xq = nb >> 3, xr = nb & 7;
    const int xcd = bid & 7, loc = bid >> 3;
    const int logical = xcd * xq + min(xcd, xr) + loc;
    const int tile = p.tlist ? p.tlist[logical] : logical;
    const int ty = tile / nbx, tx = tile - ty * nbx;
    const unsigned char tf = p.tiles ? p.tiles[tile] : (unsigned char)TILE_MATERIAL;
    // (without a list the fused kernel computes a TILE_FUSED tile; nothing
    // reads the state of hole nodes, so a tile without material has nothing
    // to do)
    if ((!p.tlist && (tf & TILE_FUSED)) || !(tf & TILE_MATERIAL)) return;
    TileStep<PR, MODE, SMALL> t(p, lds, tx * C::TW, ty * C::TH, tf);
    t.run();
}

// Tile width, height and the u ring (the window's margin) of the general
// step of a precision and scheme (pc: predictor-corrector or extrapolation),
// for the host's tile table.
template <class PR>
inline void tile_shape(bool pc, int &tw, int &th, int &ru)
{
    if (pc) {
        using C = TileCfg<PR, 1>;
        tw = C::TW, th = C::TH, ru = C::RU;
    } else {
        using C = TileCfg<PR, 0>;
        tw = C::TW, th = C::TH, ru = C::RU;
    }
}

// Upper bound of the tile table's entries for an nx x ny plate.
inline size_t max_tiles(int nx, int ny) { return (size_t)((nx + 31) / 32) * (size_t)((ny + 3) / 4); }

// Scratch bytes of the general step for an nx x ny plate: j_{n-1} of the
// extrapolation variant.
template <class PR>
inline size_t general_scratch_bytes(int nx, int ny)
{
    return ((size_t)2 * nx * ny * sizeof(typename PR::TJ) + 255) / 256 * 256;
}

// Compute units of the current device (queried once: the library's devices
// are alike).
inline int device_cus()
{
    static const int n = [] {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            return 0;
        return cus;
    }();
    return n;
}

// One launch of the 2D tiles: without a tile table (no mask, no fused
// share), plates whose two-row tiles fit one per compute unit take those
// (64 x 64 FP64: 6.8 against 7.9 us per step; 128 x 128: 7.1 against 8.2),
// the rest the default tiles.
template <class PR, int MODE>
void launch_tiles(const GenParams &p, hipStream_t st)
{
    if (!p.tiles) {
        using S = TileCfg<PR, MODE, true>;
        const int nbx = (p.nx + S::TW - 1) / S::TW;
        const int nb = nbx * ((p.ny + S::TH - 1) / S::TH);
        if (nb <= device_cus()) {
            hipLaunchKernelGGL((tile_step_kernel<PR, MODE, true>), dim3(nb), dim3(S::BLOCK), 0, st, p, nbx, nb);
            return;
        }
    }
    using C = TileCfg<PR, MODE>;
    const int nbx = (p.nx + C::TW - 1) / C::TW;
    const int nb = p.tlist ? p.n_tlist : nbx * ((p.ny + C::TH - 1) / C::TH);
    if (nb > 0) hipLaunchKernelGGL((tile_step_kernel<PR, MODE>), dim3(nb), dim3(C::BLOCK), 0, st, p, nbx, nb);
}

// Enqueue one time step on the stream; scratch is general_scratch_bytes<PR>
// bytes, 256-byte aligned.
template <class PR>
hipError_t general_step(GenParams p, char *scratch, hipStream_t st)
{
    if (p.pc == 2) {
        // j_{n-1} sits in the output buffer of j, which the tiles overwrite
        // while their neighbours still read it: keep a copy
        const size_t bytes = (size_t)2 * p.nx * p.ny * sizeof(typename PR::TJ);
        const hipError_t e = hipMemcpyAsync(scratch, p.j_out, bytes, hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return e;
        p.j_prev = scratch;
    }
    if (p.pc)
        launch_tiles<PR, 1>(p, st);
    else
        launch_tiles<PR, 0>(p, st);
    return hipGetLastError();
}

// Each precision's kernels are compiled in an object of their own
// (instantiate.hip).
extern template hipError_t general_step<PrecF64>(GenParams, char *, hipStream_t);
extern template hipError_t general_step<PrecF32>(GenParams, char *, hipStream_t);
extern template hipError_t general_step<PrecF32U64>(GenParams, char *, hipStream_t);
extern template hipError_t general_step<PrecF16>(GenParams, char *, hipStream_t);
extern template hipError_t general_step<PrecBF16>(GenParams, char *, hipStream_t);

}  // namespace lbm
