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
// Deviation storage (16-bit populations): the populations are stored as
// their deviation from the reference equilibrium ref_eq of the state they
// belong to. A step adds ref_eq of its input state back when it loads a row
// (the gradient comes from stage B, kept one more row), and holds the new
// populations back until the new displacement's gradient at their row is
// known (RefGrad, the next step's stages A and B run on this step's output),
// three rows later with the predictor-corrector, one with the explicit
// source; that needs one more halo row and column.
//
// Walls (y edges only) lie half a spacing outside the node rows 0 and ny-1.
// Ghost displacement rows for the finite differences: momentum wall -- the
// straight line through the wall displacement u_w and the nearest row (the
// wall moves with j* / rho0, so u_w is the integral of the values of j* in
// effect); traction wall -- the nearest row repeated. Rows above the
// top wall follow from rows already walked; the ghost row below the bottom
// wall is folded into the source of row 0 when that row is reached.
#pragma once

#include <type_traits>

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
    // momentum walls: displacement uwb + j* n at step n (lattice units); uwb
    // carries the displacement accumulated under earlier values of j*
    double uwb_lo[2], uwb_hi[2];
    double f_scale, f_inv_scale;  // 16-bit population scaling (1 otherwise)
    int strip_w, n_strips, n_segs;
    int halo_a;             // threads left of the first output column (>= the stencil halo)
    int x_lo, x_end;        // strips cover columns [x_lo, x_end) (x_end 0: the plate's width)
    unsigned int *flag;     // set to 1 on J <= 0 or a non-finite value
    long long step;         // index n of the input state
    int sr;                 // 16-bit populations: 1 = stochastic rounding, 0 = to nearest
    unsigned long long seed;  // key of the stochastic rounding
};

// Element e of an array through a uniform base pointer and a 32-bit byte
// offset: the global load/store form with the base in scalar registers and
// one vector register per address (plates have at most 2^29 sites, so the
// byte offset of an element of any plane fits in 32 bits).
template <class T>
__device__ __forceinline__ T gload(const T *__restrict__ base, uint32_t e)
{
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + e * (uint32_t)sizeof(T));
}
template <class T>
__device__ __forceinline__ void gstore(T *__restrict__ base, uint32_t e, T v)
{
    *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + e * (uint32_t)sizeof(T)) = v;
}

// A row offset the optimiser may not rewrite: an empty asm statement (no
// instruction, no memory access) passes it through a vector register. Without
// it, loop strength reduction turns the affine row offsets into 64-bit
// pointer induction variables, one register pair per plane, instead of one
// 32-bit offset shared by all planes.
__device__ __forceinline__ uint32_t row_offset(uint32_t e)
{
    asm("" : "+v"(e));
    return e;
}

// Store the nine populations of site o (plane-major), rounded to the storage
// type to nearest or, for 16-bit storage with sr set, stochastically with the
// bits of (key, o).
template <class FS, class TF, class TC>
__device__ __forceinline__ void store_site(TF *__restrict__ f, size_t plane, uint32_t o, const TC fn[9], TC scale,
                                           bool sr, uint32_t key)
{
    if constexpr (FS::kStochastic) {
        if (sr) {
#pragma unroll
            for (int q = 0; q < 5; ++q) {
                const uint32_t r = sr_bits(key, o, q);
                gstore(f + (size_t)(2 * q) * plane, o, FS::conv_sr(fn[2 * q], scale, r));
                if (q < 4) gstore(f + (size_t)(2 * q + 1) * plane, o, FS::conv_sr(fn[2 * q + 1], scale, r >> 16));
            }
            return;
        }
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) gstore(f + (size_t)i * plane, o, FS::conv(fn[i], scale));
}

// The values store_site would write for site o, read back.
template <class FS, class TC>
__device__ __forceinline__ void roundtrip_site(uint32_t o, const TC fn[9], TC scale, TC inv, bool sr, uint32_t key,
                                               TC out[9])
{
    if constexpr (FS::kStochastic) {
        if (sr) {
#pragma unroll
            for (int q = 0; q < 5; ++q) {
                const uint32_t r = sr_bits(key, o, q);
                out[2 * q] = FS::roundtrip_sr(fn[2 * q], scale, inv, r);
                if (q < 4) out[2 * q + 1] = FS::roundtrip_sr(fn[2 * q + 1], scale, inv, r >> 16);
            }
            return;
        }
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) out[i] = FS::roundtrip(fn[i], scale, inv);
}

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
// Pbar*_22 = -s T*_2 + K_22, Pbar*_11 = Pi_11 (outward normal (0, s)); k12
// and k22 are K at the wall (the caller passes the mean of the node row and
// the ghost row).
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

// Momentum-wall displacement at step tn + dn (lattice units): base plus j*
// times the step index. One expression, shared by every stage that needs it,
// so that all of them give the same value for a state.
__device__ __forceinline__ double wall_disp(double base, double jstar, double tn, int dn)
{
    return base + jstar * (tn + dn);
}

// Ghost displacement rows (Sec. 6, reading Q11): rows above the top wall
// from the two rows below it (which = 0: the first ghost row, 1: the
// second), and the first ghost row below the bottom wall from rows 0 and 1;
// a momentum wall takes the straight line through its displacement uw and
// the nearest row a (2 uw - a one spacing beyond, 4 uw - 3 a two spacings
// beyond), a traction wall repeats the nearest row. (b, the row after a, is
// used by neither rule.)
template <class TU>
__device__ __forceinline__ TU ghost_hi_u(int bc, int which, TU a, TU b, TU uw)
{
    (void)b;
    if (bc == BC_NEUMANN) return a;
    return which == 0 ? TU(2) * uw - a : TU(4) * uw - TU(3) * a;
}
template <class TU>
__device__ __forceinline__ TU ghost_lo_u(int bc, TU a, TU b, TU uw)
{
    (void)b;
    if (bc == BC_NEUMANN) return a;
    return TU(2) * uw - a;
}

// LDS of one pipeline (one time step in flight): double-buffered rows of the
// values whose x-neighbours are needed, the wall populations and, with
// deviation storage, the output displacement rows of RefGrad.
template <class TU, class TC, int BLOCK, bool PC, bool WALLED, bool DEV = false>
struct PipeLds {
    TU u[2][2][BLOCK];
    TC k[2][2][BLOCK];
    TC f[2][6][BLOCK];
    TU up[PC ? 2 : 1][2][BLOCK];
    TC kp[PC ? 2 : 1][2][BLOCK];
    TC wall[WALLED ? 2 : 1][3][BLOCK];
    TU ref[DEV ? 2 : 1][2][DEV ? BLOCK : 1];
};

// Register ring of L rows of N values for a row loop unrolled by U = 4
// (phases 0..3). Logical row k (0 = newest) is a fixed register at each phase, so a
// push renames instead of moving: rows 0..H-1 (H = 4, 2 or 1, a divisor of
// the unroll) rotate through H registers, and the remaining L - H rows (at
// most 2, again a divisor) form a second rotating part fed by one move per
// push. at<P, K> is row K after the push of phase P (P - 1 before it).
template <int A, int M>
struct PMod {
    static constexpr int v = ((A % M) + M) % M;
};

template <class T, int L, int N, int U = 4>
struct Ring {
    static_assert(U == 4, "rotating rings need the 4-phase unroll");
    static constexpr int H = L >= 4 ? 4 : (L >= 2 ? 2 : 1);
    static constexpr int TL = L - H;
    static constexpr int TS = TL > 0 ? TL : 1;
    static_assert(TL <= 2, "ring too long for the 4-phase unroll");
    T h[H][N];
    T tail[TS][N];

    __device__ __forceinline__ void zero()
    {
#pragma unroll
        for (int k = 0; k < H; ++k)
#pragma unroll
            for (int c = 0; c < N; ++c) h[k][c] = T(0);
#pragma unroll
        for (int k = 0; k < TS; ++k)
#pragma unroll
            for (int c = 0; c < N; ++c) tail[k][c] = T(0);
    }
    template <int P, int K>
    __device__ __forceinline__ T &at(int c)
    {
        static_assert(K >= 0 && K < L, "ring row out of range");
        if constexpr (K < H)
            return h[PMod<P - K, H>::v][c];
        else
            return tail[PMod<P - (K - H), TS>::v][c];
    }
    template <int P>
    __device__ __forceinline__ void push(int c, T v)
    {
        if constexpr (TL > 0) tail[PMod<P, TS>::v][c] = h[PMod<P, H>::v][c];
        h[PMod<P, H>::v][c] = v;
    }
};

// Without unrolling (U = 1) a push shifts the ring by one row and the phase
// is ignored: row k is always register k.
template <class T, int L, int N>
struct Ring<T, L, N, 1> {
    T h[L][N];
    __device__ __forceinline__ void zero()
    {
#pragma unroll
        for (int k = 0; k < L; ++k)
#pragma unroll
            for (int c = 0; c < N; ++c) h[k][c] = T(0);
    }
    template <int P, int K>
    __device__ __forceinline__ T &at(int c)
    {
        static_assert(K >= 0 && K < L, "ring row out of range");
        return h[K][c];
    }
    template <int P>
    __device__ __forceinline__ void push(int c, T v)
    {
#pragma unroll
        for (int k = L - 1; k > 0; --k) h[k][c] = h[k - 1][c];
        h[0][c] = v;
    }
};

// The y-march pipeline of one time step (state n -> n+1) for one column per
// thread. `def` runs stages D, E, F (they use only rows of earlier
// iterations) and hands out f_{n+1} at row R-4 and (PC) u_{n+1}, j_{n+1} at
// row R-6; `abc` takes u_n at row R and f_n, j_n at row R-2 and runs stages
// A, B, C. Both are instantiated per phase PH of the 4-way unrolled row loop
// (iteration index = PH mod 4) or, with U = 1, not unrolled (PH = 0 and
// shifting rings); b is the LDS buffer of the iteration (its index & 1).
template <class PR, int BLOCK, bool PC, bool WALLED, int U = 4>
struct Pipe {
    using TF = typename PR::TF;
    using TU = typename PR::TU;
    using TJ = typename PR::TJ;
    using TC = typename PR::TC;
    static constexpr bool DEV = FStore<TF>::kDeviation;
    using Lds = PipeLds<TU, TC, BLOCK, PC, WALLED, DEV>;
    static constexpr int NU = PC ? 6 : 4;  // rows of u_n kept
    static constexpr int NJ = PC ? 4 : 2;  // rows of j_n kept

    Lds &L;
    const int t, tl, tr, ny, y0, y1;
    const bool out_col;
    const int bc_lo, bc_hi;
    const TC omega, lam, mu, bx, by;
    const double *val_lo, *val_hi;
    const double *uwb_lo, *uwb_hi;
    const double tn;  // step index n of the input state

    // rings (row k = k rows before the stage's current row)
    Ring<TU, NU, 2, U> uR;   // u_n, rows R .. R-NU+1 (pushed in abc)
    Ring<TC, 3, 2, U> kA2;   // K12, K22 of rows R-1 .. R-3 (abc)
    Ring<TC, 2, 2, U> sN;    // source S_n of rows R-2, R-3 (abc)
    Ring<TC, NJ, 2, U> jN;   // j_n of rows R-2 .. (abc)
    Ring<TC, 2, 2, U> hx;    // du_x/dx, du_y/dx of rows R-1, R-2 (abc)
    Ring<TC, 2, 2, U> hy;    // du_x/dy, du_y/dy of rows R-1, R-2 (abc; deviation storage)
    Ring<TC, 2, 1, U> o0;    // own f^col_0 of rows R-2, R-3 (abc)
    Ring<TC, 3, 1, U> o2;    // own f^col_2 of rows R-2 .. R-4 (abc)
    TC o4;                // own f^col_4 of row R-2 (abc)
    TC n1, n3;            // pulled f_1, f_3 of row R-3 (def)
    Ring<TC, 2, 1, U> n5, n6;  // pulled f_5, f_6 of rows R-3, R-4 (def)
    Ring<TC, 3, 2, U> jfR;   // first moment of f_{n+1}, rows R-4 .. R-6 (def)
    Ring<TU, 3, 2, U> upR;   // u^p, rows R-4 .. R-6 (def)
    Ring<TC, 3, 2, U> kpA2;  // K^p_12, K^p_22 of rows R-5 .. R-7 (def)
    Ring<TC, 2, 2, U> hxp;   // du^p/dx of rows R-5, R-6 (def)
    bool bad;

    __device__ __forceinline__ Pipe(Lds &lds, const StepParams &p, long long step, int t_, int y0_, int y1_,
                                    bool out_col_)
        : L(lds), t(t_), tl(t_ > 0 ? t_ - 1 : 0), tr(t_ < BLOCK - 1 ? t_ + 1 : BLOCK - 1), ny(p.ny), y0(y0_),
          y1(y1_), out_col(out_col_), bc_lo(p.bc_lo), bc_hi(p.bc_hi), omega(TC(p.omega)), lam(TC(p.lam)),
          mu(TC(p.mu)), bx(TC(p.bx)), by(TC(p.by)), val_lo(p.val_lo), val_hi(p.val_hi), uwb_lo(p.uwb_lo),
          uwb_hi(p.uwb_hi), tn((double)step),
          bad(false)
    {
        uR.zero();
        kA2.zero();
        sN.zero();
        jN.zero();
        hx.zero();
        hy.zero();
        o0.zero();
        o2.zero();
        o4 = n1 = n3 = TC(0);
        n5.zero();
        n6.zero();
        jfR.zero();
        upR.zero();
        kpA2.zero();
        hxp.zero();
    }

    __device__ __forceinline__ bool is_node(int r) const { return !WALLED || (r >= 0 && r < ny); }

    // momentum-wall displacement (lattice units) at step n + dn
    __device__ __forceinline__ TU uw_lo(int a, int dn) const { return TU(wall_disp(uwb_lo[a], val_lo[a], tn, dn)); }
    __device__ __forceinline__ TU uw_hi(int a, int dn) const { return TU(wall_disp(uwb_hi[a], val_hi[a], tn, dn)); }

    // ghost rows above the top wall from the two rows below it
    __device__ __forceinline__ TU ghost_hi(int which, TU a, TU b, TU uw) const
    {
        return ghost_hi_u(bc_hi, which, a, b, uw);
    }
    // first ghost row below the bottom wall from rows 0 and 1
    __device__ __forceinline__ TU ghost_lo(TU a, TU b, TU uw) const { return ghost_lo_u(bc_lo, a, b, uw); }
    // stress sum in the ghost row below the bottom wall, from rows 0 and 1:
    // own values u0, u1 and x-derivatives hx0, hx1 (du_x/dx, du_y/dx)
    __device__ __forceinline__ void ghost_lo_K(const TU u0[2], const TU u1[2], const TC hx0[2], const TC hx1[2],
                                               const TU uw[2], TC &k12, TC &k22) const
    {
        TC H[4], K[4];
        if (bc_lo == BC_NEUMANN) {
            H[0] = hx0[0];
            H[2] = hx0[1];
            H[1] = TC(0);
            H[3] = TC(0);
        } else {
            // ghost rows 2 uw - u0 and 4 uw - 3 u0: the x-derivatives change
            // sign, and the central y-difference at row -1 is 2 (u0 - uw)
            (void)u1;
            (void)hx1;
            H[0] = -hx0[0];
            H[2] = -hx0[1];
            H[1] = TC(TU(2) * (u0[0] - uw[0]));
            H[3] = TC(TU(2) * (u0[1] - uw[1]));
        }
        stress_sum(H, lam, mu, K);
        k12 = K[1];
        k22 = K[3];
    }

    // ---------------- stages D, E, F. Before this iteration's pushes (phase
    // Q = PH - 1): uR row k = R-1-k, sN row k = R-3-k, jN row k = R-3-k.
    // fn: f_{n+1} at row R-4. PC: unew, jnew at row R-6 (meaningful when
    // that row is a node). Explicit: unew, jnew at row R-4.
    template <int PH>
    __device__ __forceinline__ void def(const int R, const int b, TC fn[9], TU unew[2], TC jnew[2])
    {
        constexpr int Q = PH - 1;
        const int pb = b ^ 1;
        const int rD = R - 4;
        {
            const TC a1 = L.f[pb][0][tl], a3 = L.f[pb][1][tr], a5 = L.f[pb][2][tl];
            const TC a6 = L.f[pb][3][tr], a7 = L.f[pb][4][tr], a8 = L.f[pb][5][tl];
            fn[0] = o0.template at<Q, 1>(0);
            fn[1] = n1;
            fn[2] = o2.template at<Q, 2>(0);
            fn[3] = n3;
            fn[4] = o4;
            fn[5] = n5.template at<Q, 1>(0);
            fn[6] = n6.template at<Q, 1>(0);
            fn[7] = a7;
            fn[8] = a8;
            if (WALLED && rD == 0) {
                fn[2] = L.wall[0][0][t];
                fn[5] = L.wall[0][1][t];
                fn[6] = L.wall[0][2][t];
            }
            if (WALLED && rD == ny - 1) {
                fn[4] = L.wall[WALLED ? 1 : 0][0][t];
                fn[7] = L.wall[WALLED ? 1 : 0][1][t];
                fn[8] = L.wall[WALLED ? 1 : 0][2][t];
            }
            n5.template push<PH>(0, a5);
            n6.template push<PH>(0, a6);
            n1 = a1;
            n3 = a3;

            const bool nodeD = is_node(rD);
            const TC jfx = ((fn[1] - fn[3]) + (fn[5] - fn[6])) + (fn[8] - fn[7]);
            const TC jfy = ((fn[2] - fn[4]) + (fn[5] + fn[6])) - (fn[7] + fn[8]);
            if constexpr (PC) {
                const TC jpx = jfx + TC(0.5) * sN.template at<Q, 1>(0);
                const TC jpy = jfy + TC(0.5) * sN.template at<Q, 1>(1);
                TU upx, upy;
                if (nodeD) {
                    upx = uR.template at<Q, 3>(0) + TU(TC(0.5) * (jpx + jN.template at<Q, 1>(0)));
                    upy = uR.template at<Q, 3>(1) + TU(TC(0.5) * (jpy + jN.template at<Q, 1>(1)));
                } else if (rD == ny && bc_hi != BC_PERIODIC) {
                    upx = ghost_hi(0, upR.template at<Q, 0>(0), upR.template at<Q, 1>(0), uw_hi(0, 1));
                    upy = ghost_hi(0, upR.template at<Q, 0>(1), upR.template at<Q, 1>(1), uw_hi(1, 1));
                } else if (rD == ny + 1 && bc_hi != BC_PERIODIC) {
                    upx = ghost_hi(1, upR.template at<Q, 1>(0), upR.template at<Q, 2>(0), uw_hi(0, 1));
                    upy = ghost_hi(1, upR.template at<Q, 1>(1), upR.template at<Q, 2>(1), uw_hi(1, 1));
                } else {
                    upx = upy = TU(0);
                }
                upR.template push<PH>(0, upx);
                upR.template push<PH>(1, upy);
                jfR.template push<PH>(0, jfx);
                jfR.template push<PH>(1, jfy);
                L.up[b][0][t] = upx;
                L.up[b][1][t] = upy;
            } else {
                // explicit: the source at t also serves the moment step
                jnew[0] = jfx + TC(0.5) * sN.template at<Q, 1>(0);
                jnew[1] = jfy + TC(0.5) * sN.template at<Q, 1>(1);
                unew[0] = uR.template at<Q, 3>(0) + TU(TC(0.5) * (jnew[0] + jN.template at<Q, 1>(0)));
                unew[1] = uR.template at<Q, 3>(1) + TU(TC(0.5) * (jnew[1] + jN.template at<Q, 1>(1)));
            }
        }

        if constexpr (PC) {
            // ---------------- stage E: K^p at row R-5
            {
                TC H[4], K[4];
                H[0] = TC((L.up[pb][0][tr] - L.up[pb][0][tl]) * TU(0.5));
                H[2] = TC((L.up[pb][1][tr] - L.up[pb][1][tl]) * TU(0.5));
                TU um0 = upR.template at<PH, 2>(0), um1 = upR.template at<PH, 2>(1);
                if (WALLED && R - 5 == 0) {
                    um0 = ghost_lo(upR.template at<PH, 1>(0), upR.template at<PH, 0>(0), uw_lo(0, 1));
                    um1 = ghost_lo(upR.template at<PH, 1>(1), upR.template at<PH, 0>(1), uw_lo(1, 1));
                }
                H[1] = TC((upR.template at<PH, 0>(0) - um0) * TU(0.5));
                H[3] = TC((upR.template at<PH, 0>(1) - um1) * TU(0.5));
                stress_sum(H, lam, mu, K);
                L.kp[b][0][t] = K[0];
                L.kp[b][1][t] = K[2];
                kpA2.template push<PH>(0, K[1]);
                kpA2.template push<PH>(1, K[3]);
                hxp.template push<PH>(0, H[0]);
                hxp.template push<PH>(1, H[2]);
            }
            // ---------------- stage F: S^p at row R-6, new j and u
            const int rF = R - 6;
            if (is_node(rF)) {
                TC k12d = kpA2.template at<PH, 2>(0), k22d = kpA2.template at<PH, 2>(1);
                if (WALLED && rF == 0) {
                    const TU u0[2] = {upR.template at<PH, 2>(0), upR.template at<PH, 2>(1)};
                    const TU u1[2] = {upR.template at<PH, 1>(0), upR.template at<PH, 1>(1)};
                    const TC h0[2] = {hxp.template at<PH, 1>(0), hxp.template at<PH, 1>(1)};
                    const TC h1[2] = {hxp.template at<PH, 0>(0), hxp.template at<PH, 0>(1)};
                    const TU uw[2] = {uw_lo(0, 1), uw_lo(1, 1)};
                    ghost_lo_K(u0, u1, h0, h1, uw, k12d, k22d);
                }
                const TC Sx = bx + TC(0.5) * (L.kp[pb][0][tr] - L.kp[pb][0][tl]) +
                              TC(0.5) * (kpA2.template at<PH, 0>(0) - k12d);
                const TC Sy = by + TC(0.5) * (L.kp[pb][1][tr] - L.kp[pb][1][tl]) +
                              TC(0.5) * (kpA2.template at<PH, 0>(1) - k22d);
                jnew[0] = jfR.template at<PH, 2>(0) + TC(0.5) * Sx;
                jnew[1] = jfR.template at<PH, 2>(1) + TC(0.5) * Sy;
                unew[0] = uR.template at<Q, (PC ? 5 : 0)>(0) + TU(TC(0.5) * (jnew[0] + jN.template at<Q, (PC ? 3 : 0)>(0)));
                unew[1] = uR.template at<Q, (PC ? 5 : 0)>(1) + TU(TC(0.5) * (jnew[1] + jN.template at<Q, (PC ? 3 : 0)>(1)));
            } else {
                jnew[0] = jnew[1] = TC(0);
                unew[0] = unew[1] = TU(0);
            }
        }
    }

    // ---------------- stages A, B, C with this iteration's inputs
    template <int PH>
    __device__ __forceinline__ void abc(const int R, const int b, const bool nodeA, const TU ua0, const TU ua1,
                                        const bool nodeC, const TC f[9], const TC jx, const TC jy)
    {
        constexpr int Q = PH - 1;
        const int pb = b ^ 1;
        // stage A: u_n at row R
        TU un0, un1;
        if (nodeA) {
            un0 = ua0;
            un1 = ua1;
        } else if (R == ny && bc_hi != BC_PERIODIC) {
            un0 = ghost_hi(0, uR.template at<Q, 0>(0), uR.template at<Q, 1>(0), uw_hi(0, 0));
            un1 = ghost_hi(0, uR.template at<Q, 0>(1), uR.template at<Q, 1>(1), uw_hi(1, 0));
        } else if (R == ny + 1 && bc_hi != BC_PERIODIC) {
            un0 = ghost_hi(1, uR.template at<Q, 1>(0), uR.template at<Q, 2>(0), uw_hi(0, 0));
            un1 = ghost_hi(1, uR.template at<Q, 1>(1), uR.template at<Q, 2>(1), uw_hi(1, 0));
        } else {
            un0 = un1 = TU(0);
        }
        uR.template push<PH>(0, un0);
        uR.template push<PH>(1, un1);
        L.u[b][0][t] = un0;
        L.u[b][1][t] = un1;

        // stage B: K at row R-1
        {
            TC H[4], K[4];
            H[0] = TC((L.u[pb][0][tr] - L.u[pb][0][tl]) * TU(0.5));
            H[2] = TC((L.u[pb][1][tr] - L.u[pb][1][tl]) * TU(0.5));
            const int rB = R - 1;
            TU um0 = uR.template at<PH, 2>(0), um1 = uR.template at<PH, 2>(1);
            if (WALLED && rB == 0) {
                um0 = ghost_lo(uR.template at<PH, 1>(0), uR.template at<PH, 0>(0), uw_lo(0, 0));
                um1 = ghost_lo(uR.template at<PH, 1>(1), uR.template at<PH, 0>(1), uw_lo(1, 0));
            }
            H[1] = TC((uR.template at<PH, 0>(0) - um0) * TU(0.5));
            H[3] = TC((uR.template at<PH, 0>(1) - um1) * TU(0.5));
            const TC J = stress_sum(H, lam, mu, K);
            if (out_col && rB >= y0 && rB < y1 && !(J > TC(0))) bad = true;
            L.k[b][0][t] = K[0];
            L.k[b][1][t] = K[2];
            kA2.template push<PH>(0, K[1]);
            kA2.template push<PH>(1, K[3]);
            hx.template push<PH>(0, H[0]);
            hx.template push<PH>(1, H[2]);
            if constexpr (DEV) {
                hy.template push<PH>(0, H[1]);
                hy.template push<PH>(1, H[3]);
            }
        }

        // stage C: S_n at row R-2, collision
        const int rC = R - 2;
        TC fc[9];
        TC k12d = kA2.template at<PH, 2>(0), k22d = kA2.template at<PH, 2>(1);
        if (WALLED && rC == 0) {
            const TU u0[2] = {uR.template at<PH, 2>(0), uR.template at<PH, 2>(1)};
            const TU u1[2] = {uR.template at<PH, 1>(0), uR.template at<PH, 1>(1)};
            const TC h0[2] = {hx.template at<PH, 1>(0), hx.template at<PH, 1>(1)};
            const TC h1[2] = {hx.template at<PH, 0>(0), hx.template at<PH, 0>(1)};
            const TU uw[2] = {uw_lo(0, 0), uw_lo(1, 0)};
            ghost_lo_K(u0, u1, h0, h1, uw, k12d, k22d);
        }
        const TC Sx = bx + TC(0.5) * (L.k[pb][0][tr] - L.k[pb][0][tl]) + TC(0.5) * (kA2.template at<PH, 0>(0) - k12d);
        const TC Sy = by + TC(0.5) * (L.k[pb][1][tr] - L.k[pb][1][tl]) + TC(0.5) * (kA2.template at<PH, 0>(1) - k22d);
        sN.template push<PH>(0, Sx);
        sN.template push<PH>(1, Sy);
        if (nodeC) {
            jN.template push<PH>(0, jx);
            jN.template push<PH>(1, jy);
            // the populations: with deviation storage the loaded deviations
            // plus the reference equilibrium of row R-2 (gradient of stage B)
            TC fl[9];
#pragma unroll
            for (int i = 0; i < 9; ++i) fl[i] = f[i];
            if constexpr (DEV) {
                const TC Hc[4] = {hx.template at<PH, 1>(0), hy.template at<PH, 1>(0), hx.template at<PH, 1>(1),
                                  hy.template at<PH, 1>(1)};
                TC fr[9];
                ref_eq(Hc, jx, jy, fr);
#pragma unroll
                for (int i = 0; i < 9; ++i) fl[i] = fr[i] + f[i];
            }
            TC r, pxx;
            collide(fl, jx, jy, Sx, Sy, omega, fc, r, pxx);
            // K at a wall: the mean of the node row and the ghost row beyond it
            if (WALLED && rC == 0) {
                TC w[3];
                wall_populations(false, bc_lo, fc, val_lo, r, pxx, TC(0.5) * (kA2.template at<PH, 1>(0) + k12d),
                                 TC(0.5) * (kA2.template at<PH, 1>(1) + k22d), w);
                L.wall[0][0][t] = w[0];
                L.wall[0][1][t] = w[1];
                L.wall[0][2][t] = w[2];
            }
            if (WALLED && rC == ny - 1) {
                TC w[3];
                wall_populations(true, bc_hi, fc, val_hi, r, pxx,
                                 TC(0.5) * (kA2.template at<PH, 1>(0) + kA2.template at<PH, 0>(0)),
                                 TC(0.5) * (kA2.template at<PH, 1>(1) + kA2.template at<PH, 0>(1)), w);
                L.wall[WALLED ? 1 : 0][0][t] = w[0];
                L.wall[WALLED ? 1 : 0][1][t] = w[1];
                L.wall[WALLED ? 1 : 0][2][t] = w[2];
            }
        } else {
#pragma unroll
            for (int i = 0; i < 9; ++i) fc[i] = TC(0);
            jN.template push<PH>(0, TC(0));
            jN.template push<PH>(1, TC(0));
        }
        L.f[b][0][t] = fc[1];
        L.f[b][1][t] = fc[3];
        L.f[b][2][t] = fc[5];
        L.f[b][3][t] = fc[6];
        L.f[b][4][t] = fc[7];
        L.f[b][5][t] = fc[8];
        // own-column collision rings of the pull
        o2.template push<PH>(0, fc[2]);
        o0.template push<PH>(0, fc[0]);
        o4 = fc[4];
    }
};

// The gradient of the displacement a step writes, for the reference
// equilibrium of deviation storage: row A's new displacement arrives at one
// iteration (every column of the block at once), goes to LDS and to a ring,
// and the central differences at row A - 1 take that row's x-neighbours from
// LDS (written one iteration earlier) and rows A and A - 2, with the ghost
// rows of the y walls. These are the next step's stages A and B on the same
// values, in the same expressions, so the reference that step rebuilds when
// it loads the row equals the one subtracted before the store, bit for bit.
// `state` is the step index of the displacement (the output state).
template <class TU, class TC, int BLOCK, bool WALLED, int U>
struct RefGrad {
    TU *const L;  // LDS [2 buffers][2 components][BLOCK]
    const int t, tl, tr, ny, bc_lo, bc_hi;
    TU uwl[2], uwh[2];
    Ring<TU, 3, 2, U> uq;  // rows A, A-1, A-2 after the push

    __device__ __forceinline__ TU &at(int b, int c, int x) const { return L[(b * 2 + c) * BLOCK + x]; }

    __device__ __forceinline__ RefGrad(TU *lds, const StepParams &p, long long state, int t_)
        : L(lds), t(t_), tl(t_ > 0 ? t_ - 1 : 0), tr(t_ < BLOCK - 1 ? t_ + 1 : BLOCK - 1), ny(p.ny),
          bc_lo(p.bc_lo), bc_hi(p.bc_hi)
    {
        const double tn = (double)state;
        for (int a = 0; a < 2; ++a) {
            uwl[a] = TU(wall_disp(p.uwb_lo[a], p.val_lo[a], tn, 0));
            uwh[a] = TU(wall_disp(p.uwb_hi[a], p.val_hi[a], tn, 0));
        }
        uq.zero();
    }

    // Row A's displacement (a node's value; the ghost row above the top wall
    // from the rows below it); returns the gradient at row A - 1.
    template <int PH>
    __device__ __forceinline__ void push(int A, int b, bool nodeA, TU a0, TU a1, TC H[4])
    {
        constexpr int Q = PH - 1;
        const int pb = b ^ 1;
        TU v0, v1;
        if (nodeA) {
            v0 = a0;
            v1 = a1;
        } else if (A == ny && bc_hi != BC_PERIODIC) {
            v0 = ghost_hi_u(bc_hi, 0, uq.template at<Q, 0>(0), uq.template at<Q, 1>(0), uwh[0]);
            v1 = ghost_hi_u(bc_hi, 0, uq.template at<Q, 0>(1), uq.template at<Q, 1>(1), uwh[1]);
        } else {
            v0 = v1 = TU(0);
        }
        uq.template push<PH>(0, v0);
        uq.template push<PH>(1, v1);
        at(b, 0, t) = v0;
        at(b, 1, t) = v1;
        H[0] = TC((at(pb, 0, tr) - at(pb, 0, tl)) * TU(0.5));
        H[2] = TC((at(pb, 1, tr) - at(pb, 1, tl)) * TU(0.5));
        TU um0 = uq.template at<PH, 2>(0), um1 = uq.template at<PH, 2>(1);
        if (WALLED && A - 1 == 0) {
            um0 = ghost_lo_u(bc_lo, uq.template at<PH, 1>(0), uq.template at<PH, 0>(0), uwl[0]);
            um1 = ghost_lo_u(bc_lo, uq.template at<PH, 1>(1), uq.template at<PH, 0>(1), uwl[1]);
        }
        H[1] = TC((uq.template at<PH, 0>(0) - um0) * TU(0.5));
        H[3] = TC((uq.template at<PH, 0>(1) - um1) * TU(0.5));
    }
};

// Column/row geometry of one tile. Output strips start on multiples of
// strip_w, which the host keeps a multiple of 32 columns, so row writes cover
// whole lines (half lines with 16-bit populations); the threads outside
// [halo_a, halo_a + strip_w) only feed the halo.
struct TileGeom {
    int gx, y0, y1;
    bool out_col;
};

__device__ __forceinline__ TileGeom tile_geom(const StepParams &p, int strip, int seg)
{
    TileGeom g;
    const int t = threadIdx.x;
    const int x0 = p.x_lo + strip * p.strip_w;
    const int xc = x0 - p.halo_a + t;
    g.gx = xc % p.nx;
    if (g.gx < 0) g.gx += p.nx;
    g.out_col = (t >= p.halo_a) && (t < p.halo_a + p.strip_w) && (xc < (p.x_end > 0 ? p.x_end : p.nx));
    g.y0 = (int)((long long)seg * p.ny / p.n_segs);
    g.y1 = (int)((long long)(seg + 1) * p.ny / p.n_segs);
    return g;
}

// row of a load: wrapped (periodic) or clamped into the plate (walls)
template <bool WALLED>
__device__ __forceinline__ int row_load(int r, int ny)
{
    if (!WALLED) {
        r %= ny;
        return r < 0 ? r + ny : r;
    }
    return r < 0 ? 0 : (r >= ny ? ny - 1 : r);
}

// row of a store (the caller has checked that r is a node)
template <bool WALLED>
__device__ __forceinline__ int row_store(int r, int ny)
{
    if (!WALLED) {
        r %= ny;
        return r < 0 ? r + ny : r;
    }
    return r;
}

// LDS of one pipeline (one time step of one tile)
template <class PR, int BLOCK, bool PC, bool WALLED>
using TileLds = typename Pipe<PR, BLOCK, PC, WALLED>::Lds;

template <int V>
using Phase = std::integral_constant<int, V>;

// One tile (column strip `strip`, row segment `seg`) of one plate for one
// time step. Called by every thread of a block; ends with a barrier. The row
// loop is unrolled by four so the register rings rotate by renaming; the row
// count is rounded up to a multiple of four, and the extra rows lie past the
// segment's last output row, where nothing is stored or checked.
template <class PR, int BLOCK, bool PC, bool WALLED>
__device__ __forceinline__ void step_tile(const StepParams &p, const int strip, const int seg,
                                          TileLds<PR, BLOCK, PC, WALLED> &lds, const int yr0 = -1,
                                          const int yr1 = 0)
{
    using TF = typename PR::TF;
    using TU = typename PR::TU;
    using TJ = typename PR::TJ;
    using TC = typename PR::TC;
    using FS = FStore<TF>;
    using P = Pipe<PR, BLOCK, PC, WALLED>;
    constexpr int HX = PC ? 5 : 3;

    const TF *__restrict__ fin = static_cast<const TF *>(p.f_in);
    TF *__restrict__ fout = static_cast<TF *>(p.f_out);
    const TU *__restrict__ uin = static_cast<const TU *>(p.u_in);
    TU *__restrict__ uout = static_cast<TU *>(p.u_out);
    const TJ *__restrict__ jin = static_cast<const TJ *>(p.j_in);
    TJ *__restrict__ jout = static_cast<TJ *>(p.j_out);
    const int nx = p.nx, ny = p.ny;
    const size_t plane = (size_t)p.plane;
    const TC f_scale = TC(p.f_scale), f_inv = TC(p.f_inv_scale);
    TileGeom g = tile_geom(p, strip, seg);
    if (yr0 >= 0) {  // an explicit row range in place of segment seg
        g.y0 = yr0;
        g.y1 = yr1;
    }
    P pipe(lds, p, p.step, (int)threadIdx.x, g.y0, g.y1, g.out_col);
    const bool sr = FS::kStochastic && p.sr;
    const uint32_t key = sr ? sr_key(p.seed, p.step + 1) : 0u;

    // Deviation storage: the new populations of row rF - 1 are stored when
    // RefGrad has the gradient of the new displacement there (rF: the row
    // whose u_{n+1} and j_{n+1} this iteration produces); they wait FD rows.
    constexpr bool DEV = FS::kDeviation;
    constexpr int FD = PC ? 3 : 1;
    RefGrad<TU, TC, BLOCK, WALLED, 4> rg(&lds.ref[0][0][0], p, p.step + 1, (int)threadIdx.x);
    Ring<TC, FD, 9> fdl;  // f_{n+1} of rows rF .. rF - FD + 1 (PC) before the push
    Ring<TC, 1, 2> jdl;   // j_{n+1} of row rF - 1 before the push
    if constexpr (DEV) {
        fdl.zero();
        jdl.zero();
    }

    auto row = [&](auto phase, const int R) {
        constexpr int PH = decltype(phase)::value;
        // Loads of this iteration (u_n at row R, f_n and j_n at row R-2) are
        // issued first; stages D-F, which only use earlier rows, run while
        // they are in flight. Rows beyond a wall are clamped to a valid
        // address and their values discarded.
        const uint32_t oA = row_offset((uint32_t)row_load<WALLED>(R, ny) * (uint32_t)nx + (uint32_t)g.gx);
        const uint32_t oC = row_offset((uint32_t)row_load<WALLED>(R - 2, ny) * (uint32_t)nx + (uint32_t)g.gx);
        const TU la0 = gload(uin, oA), la1 = gload(uin + plane, oA);
        TF lf[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) lf[i] = gload(fin + (size_t)i * plane, oC);
        const TJ lj0 = gload(jin, oC), lj1 = gload(jin + plane, oC);

        TC fn[9], jnew[2];
        TU unew[2];
        pipe.template def<PH>(R, PH & 1, fn, unew, jnew);
        const int rD = R - 4, rF = PC ? R - 6 : R - 4;
        if constexpr (!DEV) {
            if (pipe.is_node(rD) && g.out_col && rD >= g.y0 && rD < g.y1) {
                const uint32_t o = row_offset((uint32_t)row_store<WALLED>(rD, ny) * (uint32_t)nx + (uint32_t)g.gx);
                store_site<FS>(fout, plane, o, fn, f_scale, sr, key);
            }
        } else {
            TC H1[4];
            rg.template push<PH>(rF, PH & 1, pipe.is_node(rF), unew[0], unew[1], H1);
            const int rS = rF - 1;
            if (pipe.is_node(rS) && g.out_col && rS >= g.y0 && rS < g.y1) {
                TC fr[9], dv[9];
                ref_eq(H1, jdl.template at<PH - 1, 0>(0), jdl.template at<PH - 1, 0>(1), fr);
#pragma unroll
                for (int i = 0; i < 9; ++i) dv[i] = fdl.template at<PH - 1, FD - 1>(i) - fr[i];
                const uint32_t o = row_offset((uint32_t)row_store<WALLED>(rS, ny) * (uint32_t)nx + (uint32_t)g.gx);
                store_site<FS>(fout, plane, o, dv, f_scale, sr, key);
            }
#pragma unroll
            for (int i = 0; i < 9; ++i) fdl.template push<PH>(i, fn[i]);
            jdl.template push<PH>(0, TC(TJ(jnew[0])));
            jdl.template push<PH>(1, TC(TJ(jnew[1])));
        }
        if (pipe.is_node(rF) && g.out_col && rF >= g.y0 && rF < g.y1) {
            const uint32_t o = row_offset((uint32_t)row_store<WALLED>(rF, ny) * (uint32_t)nx + (uint32_t)g.gx);
            gstore(uout, o, unew[0]);
            gstore(uout + plane, o, unew[1]);
            gstore(jout, o, TJ(jnew[0]));
            gstore(jout + plane, o, TJ(jnew[1]));
            if (!isfinite((double)unew[0]) || !isfinite((double)unew[1]) || !isfinite((double)jnew[0]) ||
                !isfinite((double)jnew[1]))
                pipe.bad = true;
        }

        TC f[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) f[i] = FS::cvt(lf[i], f_inv);
        pipe.template abc<PH>(R, PH & 1, pipe.is_node(R), la0, la1, pipe.is_node(R - 2), f, TC(lj0), TC(lj1));
        __syncthreads();
    };

    // deviation storage: one more halo row below and the store delay above
    const int n_iter = (g.y1 - g.y0) + (PC ? 11 : 7) + (DEV ? 2 : 0);
    const int Rstart = g.y0 - HX - (DEV ? 1 : 0);
    for (int it = 0; it < n_iter; it += 4) {
        const int R = Rstart + it;
        row(Phase<0>{}, R);
        row(Phase<1>{}, R + 1);
        row(Phase<2>{}, R + 2);
        row(Phase<3>{}, R + 3);
    }
    if (pipe.bad) p.flag[0] = 1u;
}

// Delay line that hands the first step's populations f_{n+1} (rows R-4 ..
// R-7) to the second step, holding each value as the storage type would:
// 32/64-bit storage keeps the values, 16-bit storage keeps the stored bit
// patterns two to a word (20 registers instead of 36). A 4-row ring: the
// oldest row is read before the push of the same phase.
template <class FS, class TC, int U, bool PACKED = FS::kStochastic>
struct FDelay {
    Ring<TC, 4, 9, U> v;
    __device__ __forceinline__ FDelay() { v.zero(); }
    template <int PH>
    __device__ __forceinline__ void push(uint32_t o, const TC fn[9], TC scale, TC inv, bool sr, uint32_t key)
    {
        TC rt[9];
        roundtrip_site<FS>(o, fn, scale, inv, sr, key, rt);
#pragma unroll
        for (int i = 0; i < 9; ++i) v.template push<PH>(i, rt[i]);
    }
    template <int PH>
    __device__ __forceinline__ void oldest(TC out[9], TC)
    {
#pragma unroll
        for (int i = 0; i < 9; ++i) out[i] = v.template at<PH - 1, 3>(i);
    }
};

template <class FS, class TC, int U>
struct FDelay<FS, TC, U, true> {
    Ring<uint32_t, 4, 5, U> w;
    __device__ __forceinline__ FDelay() { w.zero(); }
    template <int PH>
    __device__ __forceinline__ void push(uint32_t o, const TC fn[9], TC scale, TC, bool sr, uint32_t key)
    {
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            uint32_t lo, hi = 0u;
            if (sr) {
                const uint32_t r = sr_bits(key, o, q);
                lo = FS::bits_sr(fn[2 * q], scale, r);
                if (q < 4) hi = FS::bits_sr(fn[2 * q + 1], scale, r >> 16);
            } else {
                lo = FS::bits(fn[2 * q], scale);
                if (q < 4) hi = FS::bits(fn[2 * q + 1], scale);
            }
            w.template push<PH>(q, lo | (hi << 16));
        }
    }
    template <int PH>
    __device__ __forceinline__ void oldest(TC out[9], TC inv)
    {
#pragma unroll
        for (int i = 0; i < 9; ++i)
            out[i] = FS::from_bits((w.template at<PH - 1, 3>(i >> 1) >> (16 * (i & 1))) & 0xffffu, inv);
    }
};

// Two time steps of one tile in one pass (predictor-corrector only): a second
// pipeline takes the first one's outputs six rows behind it -- u_{n+1} at
// its row R2 = R - 6 as it is produced, f_{n+1} and j_{n+1} at row R2 - 2
// from short delay rings -- so the state is read and written once per two
// steps. Needs a halo of 10 columns and 10 rows; the halo work of the first
// step is recomputed, never exchanged. The values handed over pass through
// the storage precision, so the result equals two single steps bitwise.
// Row-loop unroll of the two-step tile: 4, except with float arithmetic on a
// double-precision displacement (FP32_U64), whose double rings leave no
// registers for the values an unrolled schedule keeps live: unrolled by four
// or by two (rings rotating in register pairs) it needs 283-290 registers,
// one wave per SIMD, and runs 0.307 ms per step on the 4096^2 plate (0.409
// with two waves forced, spilling 26 registers) against 0.250 for the
// shifting loop at two waves.
template <class PR>
constexpr int step2_unroll()
{
    return (sizeof(typename PR::TU) == 8 && sizeof(typename PR::TC) == 4) ? 1 : 4;
}

template <class PR, int BLOCK, bool WALLED>
__device__ __forceinline__ void step2_tile(const StepParams &p, const int strip, const int seg,
                                           TileLds<PR, BLOCK, true, WALLED> &lds1,
                                           TileLds<PR, BLOCK, true, WALLED> &lds2, const int yr0 = -1,
                                           const int yr1 = 0)
{
    using TF = typename PR::TF;
    using TU = typename PR::TU;
    using TJ = typename PR::TJ;
    using TC = typename PR::TC;
    using FS = FStore<TF>;
    constexpr int U = step2_unroll<PR>();
    using P = Pipe<PR, BLOCK, true, WALLED, U>;

    const TF *__restrict__ fin = static_cast<const TF *>(p.f_in);
    TF *__restrict__ fout = static_cast<TF *>(p.f_out);
    const TU *__restrict__ uin = static_cast<const TU *>(p.u_in);
    TU *__restrict__ uout = static_cast<TU *>(p.u_out);
    const TJ *__restrict__ jin = static_cast<const TJ *>(p.j_in);
    TJ *__restrict__ jout = static_cast<TJ *>(p.j_out);
    const int nx = p.nx, ny = p.ny;
    const size_t plane = (size_t)p.plane;
    const TC f_scale = TC(p.f_scale), f_inv = TC(p.f_inv_scale);
    TileGeom g = tile_geom(p, strip, seg);
    if (yr0 >= 0) {  // an explicit row range in place of segment seg
        g.y0 = yr0;
        g.y1 = yr1;
    }
    P p1(lds1, p, p.step, (int)threadIdx.x, g.y0, g.y1, g.out_col);
    P p2(lds2, p, p.step + 1, (int)threadIdx.x, g.y0, g.y1, g.out_col);
    const bool sr = FS::kStochastic && p.sr;
    const uint32_t key1 = sr ? sr_key(p.seed, p.step + 1) : 0u;
    const uint32_t key2 = sr ? sr_key(p.seed, p.step + 2) : 0u;

    // f_{n+1} of rows R-4 .. R-7 and j_{n+1} of rows R-6, R-7
    FDelay<FS, TC, U> fd;
    Ring<TC, 2, 2, U> jd;
    jd.zero();

    auto row = [&](auto phase, const int R, const int b) {
        constexpr int PH = decltype(phase)::value;
        const uint32_t oA = row_offset((uint32_t)row_load<WALLED>(R, ny) * (uint32_t)nx + (uint32_t)g.gx);
        const uint32_t oC = row_offset((uint32_t)row_load<WALLED>(R - 2, ny) * (uint32_t)nx + (uint32_t)g.gx);
        const TU la0 = gload(uin, oA), la1 = gload(uin + plane, oA);
        TF lf[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) lf[i] = gload(fin + (size_t)i * plane, oC);
        const TJ lj0 = gload(jin, oC), lj1 = gload(jin + plane, oC);

        // first step: f_{n+1} at row R-4, u_{n+1} and j_{n+1} at row R-6
        TC fn1[9], j1[2];
        TU u1[2];
        p1.template def<PH>(R, b, fn1, u1, j1);

        // second step at row R2 = R - 6
        const int R2 = R - 6;
        TC fn2[9], j2[2];
        TU u2[2];
        p2.template def<PH>(R2, b, fn2, u2, j2);
        const int rD = R2 - 4, rF = R2 - 6;
        if (p2.is_node(rD) && g.out_col && rD >= g.y0 && rD < g.y1) {
            const uint32_t o = row_offset((uint32_t)row_store<WALLED>(rD, ny) * (uint32_t)nx + (uint32_t)g.gx);
            store_site<FS>(fout, plane, o, fn2, f_scale, sr, key2);
        }
        if (p2.is_node(rF) && g.out_col && rF >= g.y0 && rF < g.y1) {
            const uint32_t o = row_offset((uint32_t)row_store<WALLED>(rF, ny) * (uint32_t)nx + (uint32_t)g.gx);
            gstore(uout, o, u2[0]);
            gstore(uout + plane, o, u2[1]);
            gstore(jout, o, TJ(j2[0]));
            gstore(jout + plane, o, TJ(j2[1]));
            if (!isfinite((double)u2[0]) || !isfinite((double)u2[1]) || !isfinite((double)j2[0]) ||
                !isfinite((double)j2[1]))
                p2.bad = true;
        }
        // inputs of the second step: u_{n+1}(R2) now, f and j_{n+1}(R2 - 2) delayed
        {
            TC f2[9];
            fd.template oldest<PH>(f2, f_inv);
            p2.template abc<PH>(R2, b, p2.is_node(R2), u1[0], u1[1], p2.is_node(R2 - 2), f2,
                                jd.template at<PH - 1, 1>(0), jd.template at<PH - 1, 1>(1));
        }
        // (the site the first step's row R-4 value belongs to, as a store would index it)
        fd.template push<PH>((uint32_t)row_load<WALLED>(R - 4, ny) * (uint32_t)nx + (uint32_t)g.gx, fn1, f_scale,
                             f_inv, sr, key1);
        jd.template push<PH>(0, TC(TJ(j1[0])));
        jd.template push<PH>(1, TC(TJ(j1[1])));

        // first step's own inputs
        TC f[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) f[i] = FS::cvt(lf[i], f_inv);
        p1.template abc<PH>(R, b, p1.is_node(R), la0, la1, p1.is_node(R - 2), f, TC(lj0), TC(lj1));
        __syncthreads();
    };

    const int n_iter = (g.y1 - g.y0) + 22;
    const int Rstart = g.y0 - 10;
    if constexpr (U == 4) {
        for (int it = 0; it < n_iter; it += 4) {
            const int R = Rstart + it;
            row(Phase<0>{}, R, 0);
            row(Phase<1>{}, R + 1, 1);
            row(Phase<2>{}, R + 2, 0);
            row(Phase<3>{}, R + 3, 1);
        }
    } else {
        for (int it = 0; it < n_iter; ++it) row(Phase<0>{}, Rstart + it, it & 1);
    }
    if (p1.bad || p2.bad) p.flag[0] = 1u;
}

// Single-plate step: one block per tile. Blocks are dealt round-robin to the
// 8 XCDs; the remap gives each XCD a run of consecutive tiles, ordered row
// segment by row segment: horizontal neighbours march the same rows at the
// same time, so the halo columns they share are read once into that XCD's
// L2. (Vertical neighbours reach their shared halo rows a whole segment
// apart, long after L2 has dropped them.)
template <class PR, int BLOCK, bool PC, bool WALLED>
__global__ void __launch_bounds__(BLOCK) step_kernel(const StepParams p)
{
    const int nb = p.n_strips * p.n_segs;
    const int bid = blockIdx.x;
    const int xq = nb >> 3, xr = nb & 7;
    const int xcd = bid & 7, loc = bid >> 3;
    const int logical = xcd * xq + min(xcd, xr) + loc;
    const int seg = logical / p.n_strips;
    const int strip = logical - seg * p.n_strips;
    __shared__ TileLds<PR, BLOCK, PC, WALLED> lds;
    step_tile<PR, BLOCK, PC, WALLED>(p, strip, seg, lds);
}

// One step over a list of tiles (strip, first row, end row), three ints per
// entry: the parts of a plate with x walls or holes that lie clear of them,
// next to the general step's 2D tiles for the rest. Blocks map to entries
// as in step_kernel.
template <class PR, int BLOCK, bool PC, bool WALLED>
__global__ void __launch_bounds__(BLOCK) step_list_kernel(const StepParams p, const int *__restrict__ list, const int n)
{
    const int bid = blockIdx.x;
    const int xq = n >> 3, xr = n & 7;
    const int xcd = bid & 7, loc = bid >> 3;
    const int logical = xcd * xq + min(xcd, xr) + loc;
    const int *e = list + 3 * logical;
    __shared__ TileLds<PR, BLOCK, PC, WALLED> lds;
    step_tile<PR, BLOCK, PC, WALLED>(p, e[0], 0, lds, e[1], e[2]);
}

// Two steps over a tile list (strip, first row, end row), as step_list_kernel.
template <class PR, int BLOCK, bool WALLED>
__global__ void __launch_bounds__(BLOCK) step2_list_kernel(const StepParams p, const int *__restrict__ list,
                                                           const int n)
{
    const int bid = blockIdx.x;
    const int xq = n >> 3, xr = n & 7;
    const int xcd = bid & 7, loc = bid >> 3;
    const int logical = xcd * xq + min(xcd, xr) + loc;
    const int *e = list + 3 * logical;
    __shared__ TileLds<PR, BLOCK, true, WALLED> lds[2];
    step2_tile<PR, BLOCK, WALLED>(p, e[0], 0, lds[0], lds[1], e[1], e[2]);
}

// Two steps per launch, one block per tile (same tile order as step_kernel).
template <class PR, int BLOCK, bool WALLED>
__global__ void __launch_bounds__(BLOCK) step2_kernel(const StepParams p)
{
    const int nb = p.n_strips * p.n_segs;
    const int bid = blockIdx.x;
    const int xq = nb >> 3, xr = nb & 7;
    const int xcd = bid & 7, loc = bid >> 3;
    const int logical = xcd * xq + min(xcd, xr) + loc;
    const int seg = logical / p.n_strips;
    const int strip = logical - seg * p.n_strips;
    __shared__ TileLds<PR, BLOCK, true, WALLED> lds[2];
    step2_tile<PR, BLOCK, WALLED>(p, strip, seg, lds[0], lds[1]);
}

}  // namespace lbm
