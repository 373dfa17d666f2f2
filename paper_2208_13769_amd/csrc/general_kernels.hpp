// general_kernels.hpp -- the time step as plain per-site passes, for plates
// with walls on the x edges and corners (Sec. 6), holes (Sec. 7.2) and the
// j-extrapolation variant (end of Sec. 5).
//
// The fused step kernel marches rows with a register/LDS pipeline whose x
// halo is periodic; walls on the x edges need ghost columns and wall rules
// in every stage, which that pipeline cannot hold without extra barriers.
// These kernels do one time step as per-site passes over full fields
// instead (one thread per site; the stress and streaming passes in two
// launches each, interior nodes and a list of edge nodes):
//   1. K = P + Pbar on the lattice and one ring of ghost nodes, from u_n and
//      its ghost values (stress_pass);
//   2. source S_n (central divergence of K), moments, equilibrium and BGK
//      collision into f_col (collide_pass);
//   3. pull streaming; a link whose source lies beyond a wall takes the
//      wall's rule instead; moments jf of the new populations and the
//      predictor u^p (stream_pass);
//   4. K of u^p at t + dt (stress_pass again), then S^p, j_{n+1} and
//      u_{n+1} (update_pass). The explicit scheme stops after pass 3.
// With deviation storage (16-bit populations) pass 3 keeps the new
// populations in scratch and a last pass (store_pass) stores their
// deviation from the reference equilibrium of the new state; the passes that
// load populations add the reference of the input state back.
// In the extrapolation variant (end of Sec. 5) u^p takes 2 j_n - j_{n-1}
// for j at t + dt; j_{n-1} is still in the output buffer of j, which pass 3
// reads at its own site before pass 4b overwrites it.
// Holes (Sec. 7.2): a mask marks nodes outside the material. A link from a
// material node into a hole crosses a traction-free wall half-way; the wall
// is the one its axis step enters, both for the diagonal that meets a hole
// corner. In the differences a hole neighbour takes the node's own
// displacement, and K there is K of the node's gradient with the
// derivatives along that axis set to zero. Holes are at least two nodes
// wide, so a hole node has at most one material neighbour per axis: the
// stress pass stores that K in the hole node's own slot (columns of the x
// neighbour's K in entries 0 and 2, of the y neighbour's in 1 and 3, the
// entries the divergence reads), and the source needs no special case.
// Hole nodes carry no state: no pass reads it (the read-outs report zeros
// there), so only the hole nodes on a border are visited at all.
// Same lattice units, arithmetic and storage rounding as the fused kernel.
#pragma once

#include "step_kernel.hpp"

namespace lbm {

enum : int { EDGE_XMIN = 0, EDGE_XMAX = 1, EDGE_YMIN = 2, EDGE_YMAX = 3 };

struct GenParams {
    const void *f_in, *u_in, *j_in;  // state n
    void *f_out, *u_out, *j_out;     // state n + 1
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
    void *K;     // scratch [4][ny + 2][k_pitch(nx)] TC: stress sum with one ghost ring
    void *fcol;  // scratch [9][ny][nx] TC: post-collision populations
    void *S;     // scratch [2][ny][nx] TC: source S_n
    void *jf;    // scratch [2][ny][nx] TC: first moment of the new populations
    void *up;    // scratch [2][ny][nx] TU: predictor displacement
    void *fnew;  // scratch [9][ny][nx] TC: new populations (deviation storage only)
    unsigned *flag;
    const unsigned char *mask;  // [ny][nx] bit 0: material (1) or hole (0); bit 1: interior; nullptr: no holes
    const int *edge_k;          // ring indices (y + 1)(nx + 2) + x + 1 of the stress pass's edge nodes
    const int *edge_f;          // lattice indices of the stream pass's edge nodes
    int n_edge_k, n_edge_f;
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
// (b, the node after a, is used by neither rule.)
template <class TU>
__device__ __forceinline__ TU gen_ghost(int kind, TU uw, TU a, TU b, int k)
{
    (void)b;
    if (kind == BC_NEUMANN) return a;
    return k == 1 ? TU(2) * uw - a : TU(4) * uw - TU(3) * a;
}

// momentum-wall displacement of edge e at step t (lattice units)
template <class TU>
__device__ __forceinline__ TU gen_uw(const GenParams &p, int e, int a, double t)
{
    return TU(p.uwb[e][a] + p.val[e][a] * t);
}

// u of column x (0 <= x < nx) at row y (-2 <= y <= ny + 1): ghost rows of
// the y walls, or the periodic image
template <class TU>
__device__ __forceinline__ TU gen_u_row(const TU *u, const GenParams &p, int a, int x, int y, double t)
{
    const size_t pl = (size_t)p.plane;
    if (y >= 0 && y < p.ny) return u[a * pl + (size_t)y * p.nx + x];
    if (p.bc[EDGE_YMIN] == BC_PERIODIC) {
        y = (y % p.ny + p.ny) % p.ny;
        return u[a * pl + (size_t)y * p.nx + x];
    }
    const bool lo = y < 0;
    const int e = lo ? EDGE_YMIN : EDGE_YMAX;
    const int k = lo ? -y : y - (p.ny - 1);
    const TU u0 = u[a * pl + (size_t)(lo ? 0 : p.ny - 1) * p.nx + x];
    const TU u1 = u[a * pl + (size_t)(lo ? 1 : p.ny - 2) * p.nx + x];
    return gen_ghost<TU>(p.bc[e], gen_uw<TU>(p, e, a, t), u0, u1, k);
}

// u at (x, y) within two spacings of the lattice: ghost columns of the x
// walls are extrapolated across the wall from the rows' values (ghost rows
// included), so corner ghosts come from the ghost rows
template <class TU>
__device__ __forceinline__ TU gen_u(const TU *u, const GenParams &p, int a, int x, int y, double t)
{
    if (x >= 0 && x < p.nx) return gen_u_row(u, p, a, x, y, t);
    if (p.bc[EDGE_XMIN] == BC_PERIODIC) return gen_u_row(u, p, a, (x % p.nx + p.nx) % p.nx, y, t);
    const bool lo = x < 0;
    const int e = lo ? EDGE_XMIN : EDGE_XMAX;
    const int k = lo ? -x : x - (p.nx - 1);
    const TU u0 = gen_u_row(u, p, a, lo ? 0 : p.nx - 1, y, t);
    const TU u1 = gen_u_row(u, p, a, lo ? 1 : p.nx - 2, y, t);
    return gen_ghost<TU>(p.bc[e], gen_uw<TU>(p, e, a, t), u0, u1, k);
}

// node (x, y) lies in a hole; coordinates beyond a periodic edge wrap,
// beyond a wall they are in no hole
__device__ __forceinline__ bool g_hole(const GenParams &p, int x, int y)
{
    if (!p.mask) return false;
    if (y < 0 || y >= p.ny) {
        if (p.bc[EDGE_YMIN] != BC_PERIODIC) return false;
        y = (y % p.ny + p.ny) % p.ny;
    }
    if (x < 0 || x >= p.nx) {
        if (p.bc[EDGE_XMIN] != BC_PERIODIC) return false;
        x = (x % p.nx + p.nx) % p.nx;
    }
    return (p.mask[(size_t)y * p.nx + x] & 1) == 0;
}

// central-difference gradient of u at (x, y) (lattice or ghost ring); a hole
// neighbour takes the node's own value
template <class PR>
__device__ __forceinline__ void gen_grad(const GenParams &p, const typename PR::TU *u, int x, int y, double t,
                                         typename PR::TC H[4])
{
    using TU = typename PR::TU;
    using TC = typename PR::TC;
    const bool hxp = g_hole(p, x + 1, y), hxm = g_hole(p, x - 1, y);
    const bool hyp = g_hole(p, x, y + 1), hym = g_hole(p, x, y - 1);
    for (int a = 0; a < 2; ++a) {
        const TU c = (hxp || hxm || hyp || hym) ? gen_u(u, p, a, x, y, t) : TU(0);
        const TU xp = hxp ? c : gen_u(u, p, a, x + 1, y, t), xm = hxm ? c : gen_u(u, p, a, x - 1, y, t);
        const TU yp = hyp ? c : gen_u(u, p, a, x, y + 1, t), ym = hym ? c : gen_u(u, p, a, x, y - 1, t);
        H[2 * a + 0] = TC((xp - xm) * TU(0.5));
        H[2 * a + 1] = TC((yp - ym) * TU(0.5));
    }
}

// The populations of state n at node (x, y), site s: the stored values or,
// with deviation storage, the stored deviations plus the reference
// equilibrium of the stored state (gradient at step n, stored momentum).
template <class PR>
__device__ __forceinline__ void gen_load_f(const GenParams &p, int x, int y, size_t s, typename PR::TC f[9])
{
    using TF = typename PR::TF;
    using TU = typename PR::TU;
    using TJ = typename PR::TJ;
    using TC = typename PR::TC;
    using FS = FStore<TF>;
    const size_t pl = (size_t)p.plane;
    const TF *fin = static_cast<const TF *>(p.f_in);
    for (int i = 0; i < 9; ++i) f[i] = FS::load(fin, i * pl + s, TC(p.f_inv_scale));
    if constexpr (FS::kDeviation) {
        TC H[4], fr[9];
        gen_grad<PR>(p, static_cast<const TU *>(p.u_in), x, y, (double)p.step, H);
        const TJ *jin = static_cast<const TJ *>(p.j_in);
        ref_eq(H, TC(jin[s]), TC(jin[pl + s]), fr);
        for (int i = 0; i < 9; ++i) f[i] = fr[i] + f[i];
    }
}

// (x, y) and its eight neighbours are lattice nodes of the material (no
// ghost value, no wall, no hole): the common case, taken without branches
__device__ __forceinline__ bool g_inner(const GenParams &p, int x, int y)
{
    if (x < 1 || x > p.nx - 2 || y < 1 || y > p.ny - 2) return false;
    // bit 1 of the mask: the host marked the node interior
    return !p.mask || (p.mask[(size_t)y * p.nx + x] & 2) != 0;
}

// Row pitch of K: column x sits at x + 32, so the lattice columns of every
// row start on a 128-byte line and a wave's store covers whole lines.
__host__ __device__ __forceinline__ size_t k_pitch(int nx) { return ((size_t)nx + 33 + 31) / 32 * 32; }

__device__ __forceinline__ size_t k_index(const GenParams &p, int c, int x, int y)
{
    return ((size_t)c * (p.ny + 2) + (size_t)(y + 1)) * k_pitch(p.nx) + (size_t)(x + 32);
}

// K at the hole neighbour of (x, y) across axis n: K of the node's gradient
// with the derivatives along n set to zero
template <class PR>
__device__ __forceinline__ void gen_k_hole(const GenParams &p, int x, int y, int which, int n,
                                           typename PR::TC K[4])
{
    using TU = typename PR::TU;
    using TC = typename PR::TC;
    TC H[4];
    gen_grad<PR>(p, static_cast<const TU *>(which ? p.up : p.u_in), x, y, (double)(p.step + which), H);
    H[n] = TC(0);
    H[2 + n] = TC(0);
    stress_sum(H, TC(p.lam), TC(p.mu), K);
}

// Pass 1 / 4a: K = P + Pbar from central differences of u (eqs. (10), (15),
// (27)) on the lattice and its ring of ghost nodes. `which`: 0 = u_n at step
// n, 1 = the predictor u^p at step n + 1. Sets the flag where J <= 0.
// EDGE: the launch over the listed nodes with a ghost, wall or hole in
// their stencil; the other launch takes the interior nodes (no branches), so
// neither carries the registers of the other's path.
template <class PR, bool EDGE>
__global__ void __launch_bounds__(256) stress_pass(const GenParams p, const int which)
{
    using TU = typename PR::TU;
    using TC = typename PR::TC;
    const TU *u = static_cast<const TU *>(which ? p.up : p.u_in);
    TC *Kp = static_cast<TC *>(p.K);
    if (!EDGE) {
        // lattice rows of ceil(nx / 256) blocks each: the row index is the
        // same for the whole block (no per-thread division)
        const int nbx = (p.nx + 255) / 256;
        const int y = (int)blockIdx.x / nbx;
        const int x = ((int)blockIdx.x - y * nbx) * 256 + (int)threadIdx.x;
        if (x < 1 || x > p.nx - 2 || y < 1 || y > p.ny - 2) return;
        // the four neighbours lie in the lattice: load them before the mask
        // test so that both loads are in flight together (a hole node's u is
        // read for nothing; measured faster all the same)
        const size_t pl = (size_t)p.plane, o = (size_t)y * p.nx + x;
        TU v[2][4];
        for (int a = 0; a < 2; ++a) {
            const TU *ua = u + a * pl + o;
            v[a][0] = ua[1];
            v[a][1] = ua[-1];
            v[a][2] = ua[p.nx];
            v[a][3] = ua[-(ptrdiff_t)p.nx];
        }
        if (!g_inner(p, x, y)) return;
        TC H[4], K[4];
        for (int a = 0; a < 2; ++a) {
            H[2 * a + 0] = TC((v[a][0] - v[a][1]) * TU(0.5));
            H[2 * a + 1] = TC((v[a][2] - v[a][3]) * TU(0.5));
        }
        const TC J = stress_sum(H, TC(p.lam), TC(p.mu), K);
        for (int c = 0; c < 4; ++c) Kp[k_index(p, c, x, y)] = K[c];
        if (which == 0 && !(J > TC(0))) p.flag[0] = 1u;
        return;
    }
    const int w = p.nx + 2;
    const int tid = blockIdx.x * 256 + threadIdx.x;
    if (tid >= p.n_edge_k) return;
    const int s = p.edge_k[tid];
    const int y = s / w - 1, x = s % w - 1;
    const double t = (double)(p.step + which);
    if (g_hole(p, x, y)) {
        // K seen from the material neighbour across each axis (zero if none)
        TC kx[4] = {TC(0), TC(0), TC(0), TC(0)}, ky[4] = {TC(0), TC(0), TC(0), TC(0)};
        const int sx = !g_hole(p, x - 1, y) ? -1 : (!g_hole(p, x + 1, y) ? 1 : 0);
        const int sy = !g_hole(p, x, y - 1) ? -1 : (!g_hole(p, x, y + 1) ? 1 : 0);
        if (sx) gen_k_hole<PR>(p, x + sx, y, which, 0, kx);
        if (sy) gen_k_hole<PR>(p, x, y + sy, which, 1, ky);
        Kp[k_index(p, 0, x, y)] = kx[0];
        Kp[k_index(p, 2, x, y)] = kx[2];
        Kp[k_index(p, 1, x, y)] = ky[1];
        Kp[k_index(p, 3, x, y)] = ky[3];
        return;
    }
    TC H[4], K[4];
    gen_grad<PR>(p, u, x, y, t, H);
    const TC J = stress_sum(H, TC(p.lam), TC(p.mu), K);
    for (int c = 0; c < 4; ++c) Kp[k_index(p, c, x, y)] = K[c];
    if (which == 0 && x >= 0 && x < p.nx && y >= 0 && y < p.ny && !(J > TC(0))) p.flag[0] = 1u;
}

// central divergence of K at node (x, y) plus the body force (eq. (23))
template <class PR>
__device__ __forceinline__ void gen_source(const GenParams &p, int x, int y, typename PR::TC S[2])
{
    using TC = typename PR::TC;
    const TC *K = static_cast<const TC *>(p.K);
    TC kxp[4], kxm[4], kyp[4], kym[4];
    for (int c = 0; c < 4; ++c) {
        kxp[c] = K[k_index(p, c, x + 1, y)];
        kxm[c] = K[k_index(p, c, x - 1, y)];
        kyp[c] = K[k_index(p, c, x, y + 1)];
        kym[c] = K[k_index(p, c, x, y - 1)];
    }
    S[0] = TC(p.bx) + TC(0.5) * (kxp[0] - kxm[0]) + TC(0.5) * (kyp[1] - kym[1]);
    S[1] = TC(p.by) + TC(0.5) * (kxp[2] - kxm[2]) + TC(0.5) * (kyp[3] - kym[3]);
}

// Pass 2: source, moments, equilibrium (20), forcing (22) and BGK collision (4)
template <class PR>
__global__ void __launch_bounds__(256) collide_pass(const GenParams p)
{
    using TJ = typename PR::TJ;
    using TC = typename PR::TC;
    const int n = p.nx * p.ny;
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= n) return;
    const int y = s / p.nx, x = s - y * p.nx;
    if (g_hole(p, x, y)) return;
    const size_t pl = (size_t)p.plane;
    const TJ *jin = static_cast<const TJ *>(p.j_in);
    TC S[2], f[9], fc[9], r, pxx;
    gen_source<PR>(p, x, y, S);
    gen_load_f<PR>(p, x, y, (size_t)s, f);
    collide(f, TC(jin[s]), TC(jin[pl + s]), S[0], S[1], TC(p.omega), fc, r, pxx);
    TC *fcol = static_cast<TC *>(p.fcol);
    for (int i = 0; i < 9; ++i) fcol[i * pl + s] = fc[i];
    TC *Sp = static_cast<TC *>(p.S);
    Sp[s] = S[0];
    Sp[pl + s] = S[1];
}

// Value the wall returns into direction opp(o) at node (x, y) for the link o
// that leaves through the wall(s): sx, sy are the outward signs of the x
// and y walls it crosses (0 = none). Bounce-back with the wall momentum
// (eq. (25)) if a crossed wall is a momentum wall (the mean j* if both are);
// otherwise anti-bounce-back (eq. (26)) with r_bd and Pbar* at the node:
// each traction wall's transform gives its normal column, -s T* + K N; a
// tangential entry keeps the populations' second moment; at a corner the
// off-diagonal entry is the mean of both walls' values.
// hole: the walls are those of a hole (traction-free), not of the edges.
template <class PR>
__device__ __forceinline__ typename PR::TC gen_wall(const GenParams &p, int x, int y, int o, int sx, int sy,
                                                    typename PR::TC fco, bool hole)
{
    using TC = typename PR::TC;
    const int ex = sx < 0 ? EDGE_XMIN : EDGE_XMAX, ey = sy < 0 ? EDGE_YMIN : EDGE_YMAX;
    const bool dx = !hole && sx != 0 && p.bc[ex] == BC_DIRICHLET;
    const bool dy = !hole && sy != 0 && p.bc[ey] == BC_DIRICHLET;
    const double tx0 = hole ? 0.0 : p.val[ex][0], tx1 = hole ? 0.0 : p.val[ex][1];
    const double ty0 = hole ? 0.0 : p.val[ey][0], ty1 = hole ? 0.0 : p.val[ey][1];
    const TC w = gweight<TC>(o);
    const TC cx = TC(kGx[o]), cy = TC(kGy[o]);
    if (dx || dy) {
        TC jx, jy;
        if (dx && dy) {
            jx = TC(0.5 * (p.val[ex][0] + p.val[ey][0]));
            jy = TC(0.5 * (p.val[ex][1] + p.val[ey][1]));
        } else {
            const int e = dx ? ex : ey;
            jx = TC(p.val[e][0]);
            jy = TC(p.val[e][1]);
        }
        return fco - TC(6) * w * (cx * jx + cy * jy);
    }
    // populations' moments r and Pi at the node (state n)
    const size_t s = (size_t)y * p.nx + x;
    TC f[9];
    gen_load_f<PR>(p, x, y, s, f);
    const TC r = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
    const TC dsum = (f[5] + f[6]) + (f[7] + f[8]);
    TC Pxx = (f[1] + f[3]) + dsum, Pyy = (f[2] + f[4]) + dsum, Pxy = (f[5] - f[6]) + (f[7] - f[8]);
    const TC *K = static_cast<const TC *>(p.K);
    TC qx0 = 0, qx1 = 0, qy0 = 0, qy1 = 0;
    // K at a wall: the mean of the node and the neighbour beyond the wall (a
    // ghost node, or a hole node holding the K its material neighbour sees)
    if (sx) {  // x wall: column x of Pbar*, q_a = -s T_a + K_ax
        const TC sg = TC(sx);
        qx0 = -sg * TC(tx0) + TC(0.5) * (K[k_index(p, 0, x, y)] + K[k_index(p, 0, x + sx, y)]);
        qx1 = -sg * TC(tx1) + TC(0.5) * (K[k_index(p, 2, x, y)] + K[k_index(p, 2, x + sx, y)]);
    }
    if (sy) {  // y wall: column y, q_a = -s T_a + K_ay
        const TC sg = TC(sy);
        qy0 = -sg * TC(ty0) + TC(0.5) * (K[k_index(p, 1, x, y)] + K[k_index(p, 1, x, y + sy)]);
        qy1 = -sg * TC(ty1) + TC(0.5) * (K[k_index(p, 3, x, y)] + K[k_index(p, 3, x, y + sy)]);
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
    // A = Pbar* - r/3 I; A : (e e - I/3)
    const TC third = TC(1) / TC(3);
    const TC axx = Pxx - r * third, ayy = Pyy - r * third;
    const TC q = axx * cx * cx + TC(2) * Pxy * cx * cy + ayy * cy * cy - (axx + ayy) * third;
    return -fco + TC(2) * w * (r + TC(4.5) * q);
}

// Pull of the nine populations of a node next to an edge or a hole: a link
// whose source lies beyond a wall, or in a hole, takes the wall's rule.
template <class PR>
__device__ __forceinline__ void stream_edge(const GenParams &p, int x, int y, int s, bool perx, bool pery,
                                         typename PR::TC fn[9])
{
    using TC = typename PR::TC;
    const size_t pl = (size_t)p.plane;
    const TC *fcol = static_cast<const TC *>(p.fcol);
    for (int i = 0; i < 9; ++i) {
        int sxp = x - kGx[i], syp = y - kGy[i];
        if (i && g_hole(p, sxp, syp)) {
            // the link o = opp(i) enters a hole: the wall its axis step
            // enters, or both for the diagonal through a hole corner
            const int o = kGopp[i];
            const bool hx = kGx[o] && g_hole(p, x + kGx[o], y), hy = kGy[o] && g_hole(p, x, y + kGy[o]);
            const bool both = !hx && !hy;
            fn[i] = gen_wall<PR>(p, x, y, o, (hx || both) ? kGx[o] : 0, (hy || both) ? kGy[o] : 0,
                                 fcol[o * pl + s], true);
            continue;
        }
        bool cx = sxp < 0 || sxp >= p.nx, cy = syp < 0 || syp >= p.ny;
        if (cx && perx) {
            sxp = (sxp + p.nx) % p.nx;
            cx = false;
        }
        if (cy && pery) {
            syp = (syp + p.ny) % p.ny;
            cy = false;
        }
        if (!cx && !cy) {
            fn[i] = fcol[i * pl + (size_t)syp * p.nx + sxp];
        } else {
            const int o = kGopp[i];  // the link that left through the wall
            fn[i] = gen_wall<PR>(p, x, y, o, cx ? kGx[o] : 0, cy ? kGy[o] : 0, fcol[o * pl + s], false);
        }
    }
}

// Pass 3: pull streaming (5) with the wall rules (Sec. 6), storage of the
// new populations, their first moment jf and the predictor u^p (PC), or the
// new j and u directly (explicit).
template <class PR, bool EDGE>
__global__ void __launch_bounds__(256) stream_pass(const GenParams p)
{
    using TF = typename PR::TF;
    using TU = typename PR::TU;
    using TJ = typename PR::TJ;
    using TC = typename PR::TC;
    using FS = FStore<TF>;
    const int tid = blockIdx.x * 256 + threadIdx.x;
    if (tid >= (EDGE ? p.n_edge_f : p.nx * p.ny)) return;
    const int s = EDGE ? p.edge_f[tid] : tid;
    const int y = s / p.nx, x = s - y * p.nx;
    const size_t pl = (size_t)p.plane;
    if (!EDGE && !g_inner(p, x, y)) return;  // (hole nodes are in no launch: their state is never read)
    const TC *fcol = static_cast<const TC *>(p.fcol);
    const bool perx = p.bc[EDGE_XMIN] == BC_PERIODIC, pery = p.bc[EDGE_YMIN] == BC_PERIODIC;
    TC fn[9];
    if (!EDGE) {
        for (int i = 0; i < 9; ++i) fn[i] = fcol[i * pl + (size_t)(s - kGy[i] * p.nx - kGx[i])];
    } else {
        stream_edge<PR>(p, x, y, s, perx, pery, fn);
    }
    if constexpr (FS::kDeviation) {
        // stored by store_pass once the new state's gradient is known
        TC *fnw = static_cast<TC *>(p.fnew);
        for (int i = 0; i < 9; ++i) fnw[i * pl + s] = fn[i];
    } else {
        const bool sr = FS::kStochastic && p.sr;
        const uint32_t key = sr ? sr_key(p.seed, p.step + 1) : 0u;
        store_site<FS>(static_cast<TF *>(p.f_out), pl, (uint32_t)s, fn, TC(p.f_scale), sr, key);
    }
    const TC jfx = ((fn[1] - fn[3]) + (fn[5] - fn[6])) + (fn[8] - fn[7]);
    const TC jfy = ((fn[2] - fn[4]) + (fn[5] + fn[6])) - (fn[7] + fn[8]);
    const TC *S = static_cast<const TC *>(p.S);
    const TU *u = static_cast<const TU *>(p.u_in);
    const TJ *jin = static_cast<const TJ *>(p.j_in);
    const TC jn0 = TC(jin[s]), jn1 = TC(jin[pl + s]);
    if (p.pc) {
        TC *jf = static_cast<TC *>(p.jf);
        jf[s] = jfx;
        jf[pl + s] = jfy;
        TC jpx = jfx + TC(0.5) * S[s], jpy = jfy + TC(0.5) * S[pl + s];
        if (p.pc == 2) {
            const TJ *jold = static_cast<const TJ *>(p.j_out);
            jpx = TC(2) * jn0 - TC(jold[s]);
            jpy = TC(2) * jn1 - TC(jold[pl + s]);
        }
        TU *up = static_cast<TU *>(p.up);
        up[s] = u[s] + TU(TC(0.5) * (jpx + jn0));
        up[pl + s] = u[pl + s] + TU(TC(0.5) * (jpy + jn1));
    } else {
        const TC j0 = jfx + TC(0.5) * S[s], j1 = jfy + TC(0.5) * S[pl + s];
        const TU u0 = u[s] + TU(TC(0.5) * (j0 + jn0)), u1 = u[pl + s] + TU(TC(0.5) * (j1 + jn1));
        static_cast<TU *>(p.u_out)[s] = u0;
        static_cast<TU *>(p.u_out)[pl + s] = u1;
        static_cast<TJ *>(p.j_out)[s] = TJ(j0);
        static_cast<TJ *>(p.j_out)[pl + s] = TJ(j1);
        if (!isfinite((double)u0) || !isfinite((double)u1) || !isfinite((double)j0) || !isfinite((double)j1))
            p.flag[0] = 1u;
    }
}

// Pass 4b (PC): S^p from K(u^p), j_{n+1} = jf + S^p / 2 and the trapezoidal
// displacement update (eq. (24)).
template <class PR>
__global__ void __launch_bounds__(256) update_pass(const GenParams p)
{
    using TU = typename PR::TU;
    using TJ = typename PR::TJ;
    using TC = typename PR::TC;
    const int n = p.nx * p.ny;
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= n) return;
    const int y = s / p.nx, x = s - y * p.nx;
    const size_t pl = (size_t)p.plane;
    if (g_hole(p, x, y)) {
        static_cast<TU *>(p.u_out)[s] = static_cast<TU *>(p.u_out)[pl + s] = TU(0);
        static_cast<TJ *>(p.j_out)[s] = static_cast<TJ *>(p.j_out)[pl + s] = TJ(0);
        return;
    }
    TC Sp[2];
    gen_source<PR>(p, x, y, Sp);
    const TC *jf = static_cast<const TC *>(p.jf);
    const TU *u = static_cast<const TU *>(p.u_in);
    const TJ *jin = static_cast<const TJ *>(p.j_in);
    const TC j0 = jf[s] + TC(0.5) * Sp[0], j1 = jf[pl + s] + TC(0.5) * Sp[1];
    const TU u0 = u[s] + TU(TC(0.5) * (j0 + TC(jin[s]))), u1 = u[pl + s] + TU(TC(0.5) * (j1 + TC(jin[pl + s])));
    static_cast<TU *>(p.u_out)[s] = u0;
    static_cast<TU *>(p.u_out)[pl + s] = u1;
    static_cast<TJ *>(p.j_out)[s] = TJ(j0);
    static_cast<TJ *>(p.j_out)[pl + s] = TJ(j1);
    if (!isfinite((double)u0) || !isfinite((double)u1) || !isfinite((double)j0) || !isfinite((double)j1))
        p.flag[0] = 1u;
}

// Last pass with deviation storage: the new populations minus the reference
// equilibrium of the new state (the gradient of u_{n+1} at step n + 1 and
// j_{n+1}, as the next step's loads rebuild it), rounded to the storage type.
template <class PR>
__global__ void __launch_bounds__(256) store_pass(const GenParams p)
{
    using TF = typename PR::TF;
    using TU = typename PR::TU;
    using TJ = typename PR::TJ;
    using TC = typename PR::TC;
    using FS = FStore<TF>;
    const int n = p.nx * p.ny;
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= n) return;
    const int y = s / p.nx, x = s - y * p.nx;
    if (g_hole(p, x, y)) return;
    const size_t pl = (size_t)p.plane;
    TC H[4], fr[9], dv[9];
    gen_grad<PR>(p, static_cast<const TU *>(p.u_out), x, y, (double)(p.step + 1), H);
    const TJ *jo = static_cast<const TJ *>(p.j_out);
    ref_eq(H, TC(jo[s]), TC(jo[pl + s]), fr);
    const TC *fnw = static_cast<const TC *>(p.fnew);
    for (int i = 0; i < 9; ++i) dv[i] = fnw[i * pl + s] - fr[i];
    const bool sr = FS::kStochastic && p.sr;
    const uint32_t key = sr ? sr_key(p.seed, p.step + 1) : 0u;
    store_site<FS>(static_cast<TF *>(p.f_out), pl, (uint32_t)s, dv, TC(p.f_scale), sr, key);
}

// Scratch bytes of the passes for an nx x ny plate.
template <class PR>
inline size_t general_scratch_bytes(int nx, int ny)
{
    using TU = typename PR::TU;
    using TC = typename PR::TC;
    const size_t n = (size_t)nx * ny, ne = k_pitch(nx) * (ny + 2);
    auto al = [](size_t v) { return (v + 255) / 256 * 256; };
    const size_t fnew = FStore<typename PR::TF>::kDeviation ? al(9 * n * sizeof(TC)) : 0;
    return al(4 * ne * sizeof(TC)) + al(9 * n * sizeof(TC)) + al(2 * n * sizeof(TC)) + al(2 * n * sizeof(TC)) +
           al(2 * n * sizeof(TU)) + fnew;
}

// Enqueue one time step of the passes on the stream; scratch is
// general_scratch_bytes<PR>(nx, ny) bytes, 256-byte aligned.
template <class PR>
hipError_t general_step(GenParams p, char *scratch, hipStream_t st)
{
    using TC = typename PR::TC;
    const size_t n = (size_t)p.nx * p.ny, ne = k_pitch(p.nx) * (p.ny + 2);
    auto al = [](size_t v) { return (v + 255) / 256 * 256; };
    size_t off = 0;
    p.K = scratch + off;
    off += al(4 * ne * sizeof(TC));
    p.fcol = scratch + off;
    off += al(9 * n * sizeof(TC));
    p.S = scratch + off;
    off += al(2 * n * sizeof(TC));
    p.jf = scratch + off;
    off += al(2 * n * sizeof(TC));
    p.up = scratch + off;
    off += al(2 * n * sizeof(typename PR::TU));
    p.fnew = scratch + off;
    const int nb = (int)((n + 255) / 256), nbi = (p.nx + 255) / 256 * p.ny;
    const int nbk = (p.n_edge_k + 255) / 256, nbf = (p.n_edge_f + 255) / 256;
    hipLaunchKernelGGL((stress_pass<PR, false>), dim3(nbi), dim3(256), 0, st, p, 0);
    if (nbk) hipLaunchKernelGGL((stress_pass<PR, true>), dim3(nbk), dim3(256), 0, st, p, 0);
    hipLaunchKernelGGL((collide_pass<PR>), dim3(nb), dim3(256), 0, st, p);
    hipLaunchKernelGGL((stream_pass<PR, false>), dim3(nb), dim3(256), 0, st, p);
    if (nbf) hipLaunchKernelGGL((stream_pass<PR, true>), dim3(nbf), dim3(256), 0, st, p);
    if (p.pc) {
        hipLaunchKernelGGL((stress_pass<PR, false>), dim3(nbi), dim3(256), 0, st, p, 1);
        if (nbk) hipLaunchKernelGGL((stress_pass<PR, true>), dim3(nbk), dim3(256), 0, st, p, 1);
        hipLaunchKernelGGL((update_pass<PR>), dim3(nb), dim3(256), 0, st, p);
    }
    if constexpr (FStore<typename PR::TF>::kDeviation) hipLaunchKernelGGL((store_pass<PR>), dim3(nb), dim3(256), 0, st, p);
    return hipGetLastError();
}

// Each precision's passes are compiled in an object of their own
// (instantiate.hip).
extern template hipError_t general_step<PrecF64>(GenParams, char *, hipStream_t);
extern template hipError_t general_step<PrecF32>(GenParams, char *, hipStream_t);
extern template hipError_t general_step<PrecF32U64>(GenParams, char *, hipStream_t);
extern template hipError_t general_step<PrecF16>(GenParams, char *, hipStream_t);
extern template hipError_t general_step<PrecBF16>(GenParams, char *, hipStream_t);

}  // namespace lbm
