/*
 * lbm_oracle.c -- plain, slow, FP64 CPU reference of the Lagrangian
 * (reference-configuration) lattice Boltzmann method for nonlinear solids of
 * Faust, Schlueter, Mueller & Mueller (2022).
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library. The HIP product path
 * never calls it, and it shares no code, header or table with that path.
 *
 * It follows Algorithm 1 (Sec. 5) phase by phase, in physical units and with
 * the lattice velocities C_i = (dX/dt) e_i as printed. Each phase is a plain
 * loop over all sites that writes a full field before the next phase starts.
 * Streaming is done by *push* (Sec. 3, eq. (5) read literally).
 *
 * Readings where the paper is silent or ambiguous:
 *  R1  The second-order moment that enters the equilibrium is the
 *      populations' own second moment Pi = sum_i C_i C_i f_i (Sec. 4 and
 *      Sec. 5: the LBM itself evolves Pbar through the third equation of the
 *      chain (19)). The finite-difference Poisson stress Pbar(H) of eq. (15)
 *      is used only inside the source term (23) and in the traction
 *      transform of Sec. 6.
 *  R2  Default time level of the source in the moment step: the
 *      predictor-corrector of the footnote in Sec. 5 (evaluates 1S at
 *      t + dt as the Crank-Nicolson footnote of Sec. 4 asks). The literal
 *      Algorithm 1 level (1S at t) is the "explicit" scheme.
 *  Q3  c_s and C_s are the same: C_s = sqrt(mu/rho0), and dX/dt = sqrt(3) C_s
 *      (the time steps printed in Sec. 7 follow from it).
 *  Q4  The trapezoidal rule (24) carries the factor dt.
 *  Q7  r in the collision is sum_i f_i; at start r0 = -rho0 div u0 (eq. (18)).
 *  Q8  Gradient and divergence are radius-1 central differences; the source
 *      is their composition (radius 2).
 *  Q11 Walls lie half a spacing outside the first and last node rows.
 *      Ghost displacement rows for the finite differences: at a wall with a
 *      momentum (Dirichlet) rule, the straight line through the wall value
 *      and the nearest row (the quadratic through the wall value and the
 *      two nearest rows makes the step grow 1.07 to 1.26 times per step for
 *      lambda/mu between 5.75 and 7 at tau/dt = 0.8); at a traction
 *      (Neumann) wall, constant extrapolation of the nearest row. Of the boundary moments of the
 *      anti-bounce-back rule (26), r_bd and the tangential entry of Pbar*
 *      are taken at the node row next to the wall (zeroth-order
 *      extrapolation; higher orders make the scheme grow without bound near
 *      the wall), and P + Pbar in the traction transform is its value at
 *      the wall, the mean of the node row and the ghost row (the wall lies
 *      midway) -- the same wall value the central divergence at the node
 *      row implies, so the wall passes exactly T*.
 *  Q12 The anti-bounce-back rule uses r_bd in both places (eq. (26)).
 *  Q22 The extrapolation variant (scheme 2, end of Sec. 5): the predictor
 *      displacement for the source at t + dt comes from the trapezoidal
 *      rule with j at t + dt extrapolated linearly from t - dt and t,
 *      2 j(t) - j(t - dt). At the first step j(t - dt) is taken as j(0).
 *
 * Layout: every field is structure-of-arrays, component-major, row-major
 * inside a component: f[i][y][x] with i in the oracle's own D2Q9 order
 * i = 3*(ey+1) + (ex+1), u[a][y][x], j[a][y][x], P[a][b][y][x] (a,b in {x,y}).
 *
 * Every edge is periodic (in pairs), a momentum wall or a traction wall.
 *  Q20 Corners (both edges walls): the diagonal link that leaves a corner
 *      node through both walls takes the rule of the momentum wall if one
 *      of the two is a momentum wall (the mean j* if both are); between two
 *      traction walls it is anti-bounced with a boundary Poisson tensor
 *      whose normal entries come from the two walls' traction transforms
 *      and whose off-diagonal entry is the mean of the two walls' values.
 *      Ghost displacements beyond a corner are extrapolated across the x
 *      wall from the ghost rows.
 *  Q23 Holes (Sec. 7.2): a mask marks lattice nodes outside the material.
 *      Links from a material node to a hole node cross a traction-free wall
 *      half-way between them (the rules of Q11 with T* = 0). The wall of a
 *      hole edge is the one the link's axis step enters: a link whose x
 *      step (y step) lands in the hole crosses the x (y) wall, one whose
 *      axis steps both stay in the material -- the diagonal that meets a
 *      hole corner, at a re-entrant corner of the material -- crosses both
 *      and takes the two-wall rule of Q20. In the central differences at a
 *      material node a hole neighbour's displacement is replaced by the
 *      node's own (zeroth-order ghost, as Q11); the stress sum K at such a
 *      neighbour, needed by the divergence, is K of the node's gradient
 *      with the derivatives along that axis set to zero (what the constant
 *      ghost gives at a straight edge). Hole nodes carry no state.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_PERIODIC 0
#define ORACLE_DIRICHLET_J 1
#define ORACLE_NEUMANN_T 2

typedef struct {
    int nx, ny;
    double dx;          /* lattice spacing dX */
    double rho0;        /* reference density */
    double lam, mu;     /* Lame parameters of the neo-Hooke law (27) */
    double tau_over_dt; /* relaxation time tau / dt */
    double body[2];     /* body force per unit mass b */
    int scheme;         /* 0: predictor-corrector (R2), 1: explicit (Alg. 1),
                           2: j extrapolated to t + dt for the predictor (Q22) */
    int bc_ymin, bc_ymax;        /* ORACLE_* kind of the bottom / top edge */
    double val_ymin[2], val_ymax[2]; /* j* (Dirichlet) or T* (Neumann) */
    int bc_xmin, bc_xmax;        /* ORACLE_* kind of the left / right edge */
    double val_xmin[2], val_xmax[2];
    const unsigned char *solid;  /* [ny][nx]: 1 material, 0 hole (Q23); NULL: all material */
} oracle_params;

/* ---- D2Q9 lattice (Sec. 3): 9 velocities incl. the rest velocity ---- */

static int ex_of(int i) { return i % 3 - 1; }
static int ey_of(int i) { return i / 3 - 1; }
static int opposite(int i) { return 8 - i; }
static double weight(int i)
{
    int n = abs(ex_of(i)) + abs(ey_of(i));
    if (n == 0) return 4.0 / 9.0;
    if (n == 1) return 1.0 / 9.0;
    return 1.0 / 36.0;
}

/* shear-wave speed squared C_s^2 = mu / rho0 (Sec. 4, after eq. (15)) */
static double cs2(const oracle_params *p) { return p->mu / p->rho0; }

/* dt = dX / (sqrt(3) C_s): the lattice speed is sqrt(3) times C_s (Q3) */
double oracle_dt(const oracle_params *p)
{
    return p->dx / (sqrt(3.0) * sqrt(cs2(p)));
}

static double lattice_speed(const oracle_params *p) { return p->dx / oracle_dt(p); }

/* ---- constitutive law (Sec. 7, eq. (27)) ----
 * W = mu/2 (I_C - 2) + lam/4 (J^2 - 1) - lam/2 log J - mu log J, with
 * C = F^T F, F = I + H. Its derivative is the first Piola-Kirchhoff stress
 * P = dW/dF = mu (F - F^-T) + lam/2 (J^2 - 1) F^-T.
 * Tensors are stored row-major: T[0]=T11, T[1]=T12, T[2]=T21, T[3]=T22. */
void oracle_piola(double lam, double mu, const double H[4], double P[4])
{
    double F11 = 1.0 + H[0], F12 = H[1], F21 = H[2], F22 = 1.0 + H[3];
    double J = F11 * F22 - F12 * F21;
    /* F^-1 = [[F22, -F12], [-F21, F11]] / J, so F^-T = [[F22, -F21], [-F12, F11]] / J */
    double FiT11 = F22 / J, FiT12 = -F21 / J, FiT21 = -F12 / J, FiT22 = F11 / J;
    double a = 0.5 * lam * (J * J - 1.0);
    P[0] = mu * (F11 - FiT11) + a * FiT11;
    P[1] = mu * (F12 - FiT12) + a * FiT12;
    P[2] = mu * (F21 - FiT21) + a * FiT21;
    P[3] = mu * (F22 - FiT22) + a * FiT22;
}

double oracle_strain_energy(double lam, double mu, const double H[4])
{
    double F11 = 1.0 + H[0], F12 = H[1], F21 = H[2], F22 = 1.0 + H[3];
    double J = F11 * F22 - F12 * F21;
    double IC = F11 * F11 + F12 * F12 + F21 * F21 + F22 * F22; /* tr(F^T F) */
    return 0.5 * mu * (IC - 2.0) + 0.25 * lam * (J * J - 1.0) - 0.5 * lam * log(J) - mu * log(J);
}

/* Cauchy stress sigma = J^-1 P F^T (Sec. 7, the stress read out at the
 * plate-with-hole points), written out as the product of the two matrices. */
void oracle_cauchy(double lam, double mu, const double H[4], double sig[4])
{
    double P[4];
    oracle_piola(lam, mu, H, P);
    double F[4] = {1.0 + H[0], H[1], H[2], 1.0 + H[3]};
    double J = F[0] * F[3] - F[1] * F[2];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            /* (P F^T)_ab = sum_k P_ak F_bk */
            double s = 0.0;
            for (int k = 0; k < 2; ++k) s += P[2 * a + k] * F[2 * b + k];
            sig[2 * a + b] = s / J;
        }
}

/* Green-Lagrange strain E = (F^T F - I) / 2 */
void oracle_green_lagrange(const double H[4], double E[4])
{
    double F[4] = {1.0 + H[0], H[1], H[2], 1.0 + H[3]};
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            double s = 0.0;
            for (int k = 0; k < 2; ++k) s += F[2 * k + a] * F[2 * k + b]; /* (F^T F)_ab */
            E[2 * a + b] = 0.5 * (s - (a == b ? 1.0 : 0.0));
        }
}

/* Poisson stress Pbar(H) = -mu (H + H^T + tr H I), eq. (15) */
void oracle_poisson(double mu, const double H[4], double Pb[4])
{
    double tr = H[0] + H[3];
    Pb[0] = -mu * (H[0] + H[0] + tr);
    Pb[1] = -mu * (H[1] + H[2]);
    Pb[2] = -mu * (H[2] + H[1]);
    Pb[3] = -mu * (H[3] + H[3] + tr);
}

/* lattice velocity C_i = (dX/dt) e_i */
void oracle_velocity(const oracle_params *p, int i, double C[2])
{
    double c = lattice_speed(p);
    C[0] = c * ex_of(i);
    C[1] = c * ey_of(i);
}

double oracle_weight(int i) { return weight(i); }

/* equilibrium (Sec. 5, eq. (20)):
 * f_i^eq = w_i ( r + C_i.j / C_s^2
 *                + (Pb - r C_s^2 I) : (C_i C_i - C_s^2 I) / (2 C_s^4) ) */
void oracle_equilibrium(const oracle_params *p, double r, const double j[2],
                        const double Pb[4], double feq[9])
{
    double s2 = cs2(p);
    for (int i = 0; i < 9; ++i) {
        double C[2];
        oracle_velocity(p, i, C);
        double A[4] = {Pb[0] - r * s2, Pb[1], Pb[2], Pb[3] - r * s2};
        double B[4] = {C[0] * C[0] - s2, C[0] * C[1], C[1] * C[0], C[1] * C[1] - s2};
        double AB = A[0] * B[0] + A[1] * B[1] + A[2] * B[2] + A[3] * B[3];
        feq[i] = weight(i) * (r + (C[0] * j[0] + C[1] * j[1]) / s2 + AB / (2.0 * s2 * s2));
    }
}

/* source populations (Sec. 5, eq. (22)): psi_i = w_i C_i . 1S / C_s^2 */
void oracle_source_pop(const oracle_params *p, const double S[2], double psi[9])
{
    double s2 = cs2(p);
    for (int i = 0; i < 9; ++i) {
        double C[2];
        oracle_velocity(p, i, C);
        psi[i] = weight(i) * (C[0] * S[0] + C[1] * S[1]) / s2;
    }
}

/* ---- indexing helpers ---- */

static size_t at(const oracle_params *p, int y, int x) { return (size_t)y * p->nx + x; }
static int wrap(int a, int n) { return ((a % n) + n) % n; }
static size_t plane(const oracle_params *p) { return (size_t)p->nx * p->ny; }
/* node (y, x) of the lattice lies in a hole (Q23); coordinates beyond a
 * periodic edge wrap, beyond a wall they are outside every hole */
static int in_hole(const oracle_params *p, int y, int x)
{
    if (!p->solid) return 0;
    if (y < 0 || y >= p->ny) {
        if (p->bc_ymin != ORACLE_PERIODIC) return 0;
        y = ((y % p->ny) + p->ny) % p->ny;
    }
    if (x < 0 || x >= p->nx) {
        if (p->bc_xmin != ORACLE_PERIODIC) return 0;
        x = ((x % p->nx) + p->nx) % p->nx;
    }
    return !p->solid[(size_t)y * p->nx + x];
}

/* Extended grids: the displacement with two ghost rows and columns on every
 * side, (ny + 4) rows of (nx + 4) values, lattice node (y, x) at (y + 2,
 * x + 2); the stress sum with one, (ny + 2) x (nx + 2), node at (y + 1, x + 1). */
static size_t ue_cols(const oracle_params *p) { return (size_t)p->nx + 4; }
static size_t ue_plane(const oracle_params *p) { return ue_cols(p) * ((size_t)p->ny + 4); }
static size_t ue_at(const oracle_params *p, int a, int y, int x)
{
    return (size_t)a * ue_plane(p) + (size_t)(y + 2) * ue_cols(p) + (size_t)(x + 2);
}
static size_t k_cols(const oracle_params *p) { return (size_t)p->nx + 2; }
static size_t k_plane(const oracle_params *p) { return k_cols(p) * ((size_t)p->ny + 2); }
static size_t k_at(const oracle_params *p, int c, int y, int x)
{
    return (size_t)c * k_plane(p) + (size_t)(y + 1) * k_cols(p) + (size_t)(x + 1);
}

/* Ghost value k = 1 or 2 spacings beyond the node u0 next to a wall (Q11):
 * at a momentum wall the straight line through the wall displacement uw
 * (half a spacing beyond u0) and u0, so u(-1) = 2 uw - u0 and
 * u(-2) = 4 uw - 3 u0; at a traction wall the value u0. (u1, the node after
 * u0, is not used by either rule.) */
static double ghost(int kind, double uw, double u0, double u1, int k)
{
    (void)u1;
    if (kind == ORACLE_DIRICHLET_J) return k == 1 ? 2.0 * uw - u0 : 4.0 * uw - 3.0 * u0;
    return u0;
}

/* Wall displacements: wall[e][a] for the edges e = xmin, xmax, ymin, ymax
 * (component a) is the displacement of a momentum wall at the time of the
 * state. Every wall starts at rest (zero displacement) and moves with the
 * velocity j* / rho0 of the value in effect, so one step of length dt moves
 * it by j* dt / rho0 (the wall is a rigid body driven by its prescribed
 * momentum, Sec. 6). */
enum { WALL_XMIN = 0, WALL_XMAX = 1, WALL_YMIN = 2, WALL_YMAX = 3 };

static void advance_walls(const oracle_params *p, const double wall[8], double out[8])
{
    const int kind[4] = {p->bc_xmin, p->bc_xmax, p->bc_ymin, p->bc_ymax};
    const double *val[4] = {p->val_xmin, p->val_xmax, p->val_ymin, p->val_ymax};
    double dt = oracle_dt(p);
    for (int e = 0; e < 4; ++e)
        for (int a = 0; a < 2; ++a)
            out[2 * e + a] = wall[2 * e + a] + (kind[e] == ORACLE_DIRICHLET_J ? val[e][a] * dt / p->rho0 : 0.0);
}

/* Ghost displacements (Q11, Q20) around the lattice, with the momentum
 * walls at the displacements wall[] (see advance_walls). Periodic edges copy
 * the opposite side. */
static void extend_u(const oracle_params *p, const double *u, const double wall[8], double *ue)
{
    int nx = p->nx, ny = p->ny;
    for (int a = 0; a < 2; ++a) {
        const double *ua = u + a * plane(p);
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) ue[ue_at(p, a, y, x)] = ua[at(p, y, x)];
        /* ghost rows of the lattice columns */
        double uwlo = wall[2 * WALL_YMIN + a], uwhi = wall[2 * WALL_YMAX + a];
        for (int x = 0; x < nx; ++x)
            for (int k = 1; k <= 2; ++k) {
                if (p->bc_ymin == ORACLE_PERIODIC) {
                    ue[ue_at(p, a, -k, x)] = ua[at(p, ny - k, x)];
                    ue[ue_at(p, a, ny - 1 + k, x)] = ua[at(p, k - 1, x)];
                } else {
                    ue[ue_at(p, a, -k, x)] = ghost(p->bc_ymin, uwlo, ua[at(p, 0, x)], ua[at(p, 1, x)], k);
                    ue[ue_at(p, a, ny - 1 + k, x)] =
                        ghost(p->bc_ymax, uwhi, ua[at(p, ny - 1, x)], ua[at(p, ny - 2, x)], k);
                }
            }
        /* ghost columns of every extended row (corners included) */
        double uwl = wall[2 * WALL_XMIN + a], uwr = wall[2 * WALL_XMAX + a];
        for (int y = -2; y < ny + 2; ++y)
            for (int k = 1; k <= 2; ++k) {
                if (p->bc_xmin == ORACLE_PERIODIC) {
                    ue[ue_at(p, a, y, -k)] = ue[ue_at(p, a, y, nx - k)];
                    ue[ue_at(p, a, y, nx - 1 + k)] = ue[ue_at(p, a, y, k - 1)];
                } else {
                    ue[ue_at(p, a, y, -k)] = ghost(p->bc_xmin, uwl, ue[ue_at(p, a, y, 0)], ue[ue_at(p, a, y, 1)], k);
                    ue[ue_at(p, a, y, nx - 1 + k)] =
                        ghost(p->bc_xmax, uwr, ue[ue_at(p, a, y, nx - 1)], ue[ue_at(p, a, y, nx - 2)], k);
                }
            }
    }
}

/* displacement gradient H_ab = d_b u_a by central differences (eq. (10),
 * Sec. 5), at lattice node (y, x) with -1 <= y <= ny, -1 <= x <= nx. */
static void grad_u(const oracle_params *p, const double *ue, int y, int x, double H[4])
{
    for (int a = 0; a < 2; ++a) {
        /* a hole neighbour takes the node's own value (Q23) */
        double c = ue[ue_at(p, a, y, x)];
        double xp = in_hole(p, y, x + 1) ? c : ue[ue_at(p, a, y, x + 1)];
        double xm = in_hole(p, y, x - 1) ? c : ue[ue_at(p, a, y, x - 1)];
        double yp = in_hole(p, y + 1, x) ? c : ue[ue_at(p, a, y + 1, x)];
        double ym = in_hole(p, y - 1, x) ? c : ue[ue_at(p, a, y - 1, x)];
        double dudx = (xp - xm) / (2.0 * p->dx);
        double dudy = (yp - ym) / (2.0 * p->dx);
        H[2 * a + 0] = dudx;
        H[2 * a + 1] = dudy;
    }
}

/* K = P(H) + Pbar(H) on the lattice and one ring of ghost nodes */
static void stress_sum(const oracle_params *p, const double *ue, double *K)
{
    int nx = p->nx, ny = p->ny;
#pragma omp parallel for schedule(static)
    for (int y = -1; y <= ny; ++y)
        for (int x = -1; x <= nx; ++x) {
            double H[4], P[4], Pb[4];
            if (in_hole(p, y, x)) {
                for (int c = 0; c < 4; ++c) K[k_at(p, c, y, x)] = 0.0;
                continue;
            }
            grad_u(p, ue, y, x, H);
            oracle_piola(p->lam, p->mu, H, P);
            oracle_poisson(p->mu, H, Pb);
            for (int c = 0; c < 4; ++c) K[k_at(p, c, y, x)] = P[c] + Pb[c];
        }
}

/* K at the hole neighbour of node (y, x) across axis n (Q23): K of the
 * node's gradient with the derivatives along n set to zero */
static void k_hole(const oracle_params *p, const double *ue, int y, int x, int n, double K[4])
{
    double H[4], P[4], Pb[4];
    grad_u(p, ue, y, x, H);
    H[n] = 0.0;
    H[2 + n] = 0.0;
    oracle_piola(p->lam, p->mu, H, P);
    oracle_poisson(p->mu, H, Pb);
    for (int c = 0; c < 4; ++c) K[c] = P[c] + Pb[c];
}

/* 1S_a = rho0 b_a + d_b (P_ab + Pbar_ab), eq. (23), central divergence.
 * Hole nodes get zero. */
static void source_field(const oracle_params *p, const double *ue, const double *K, double *S)
{
    int nx = p->nx, ny = p->ny;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            if (in_hole(p, y, x)) {
                S[at(p, y, x)] = S[plane(p) + at(p, y, x)] = 0.0;
                continue;
            }
            double kxp[4], kxm[4], kyp[4], kym[4];
            for (int c = 0; c < 4; ++c) {
                kxp[c] = K[k_at(p, c, y, x + 1)];
                kxm[c] = K[k_at(p, c, y, x - 1)];
                kyp[c] = K[k_at(p, c, y + 1, x)];
                kym[c] = K[k_at(p, c, y - 1, x)];
            }
            if (in_hole(p, y, x + 1)) k_hole(p, ue, y, x, 0, kxp);
            if (in_hole(p, y, x - 1)) k_hole(p, ue, y, x, 0, kxm);
            if (in_hole(p, y + 1, x)) k_hole(p, ue, y, x, 1, kyp);
            if (in_hole(p, y - 1, x)) k_hole(p, ue, y, x, 1, kym);
            for (int a = 0; a < 2; ++a) {
                /* K_a1 at the x neighbours, K_a2 at the y neighbours */
                double div = (kxp[2 * a + 0] - kxm[2 * a + 0]) / (2.0 * p->dx)
                           + (kyp[2 * a + 1] - kym[2 * a + 1]) / (2.0 * p->dx);
                S[a * plane(p) + at(p, y, x)] = p->rho0 * p->body[a] + div;
            }
        }
}

/* source 1S(u) for the whole lattice, walls at the displacements wall[] */
static void source_of_u(const oracle_params *p, const double *u, const double wall[8], double *S)
{
    double *ue = malloc(sizeof(double) * 2 * ue_plane(p));
    double *K = malloc(sizeof(double) * 4 * k_plane(p));
    extend_u(p, u, wall, ue);
    stress_sum(p, ue, K);
    source_field(p, ue, K, S);
    free(ue);
    free(K);
}

/* zeroth moment r = sum_i f_i and second moment Pi = sum_i C_i C_i f_i */
static void moments_r_pi(const oracle_params *p, const double *f, size_t s, double *r, double Pi[4])
{
    *r = 0.0;
    Pi[0] = Pi[1] = Pi[2] = Pi[3] = 0.0;
    for (int i = 0; i < 9; ++i) {
        double C[2], fi = f[i * plane(p) + s];
        oracle_velocity(p, i, C);
        *r += fi;
        Pi[0] += C[0] * C[0] * fi;
        Pi[1] += C[0] * C[1] * fi;
        Pi[2] += C[1] * C[0] * fi;
        Pi[3] += C[1] * C[1] * fi;
    }
}

/* Traction transform at a wall (Sec. 6) for node (y, x) next to it: the
 * wall normal is axis n (0: x, 1: y) with outward sign s, T the traction.
 * Pbar N = -T* + (P + Pbar) N gives the wall's normal column of the boundary
 * Poisson tensor, q_a = Pbar*_an = (-T_a + K_an s) / s, with K = P + Pbar
 * at the wall: the mean of K at the node and at the neighbour beyond the
 * wall (a ghost node, or a hole node whose K is that of Q23) (reading Q11). */
static void traction_column(const oracle_params *p, const double *K, const double *ue, int y, int x, int n,
                            double s, const double T[2], double q[2])
{
    const int gy = y + (n == 1 ? (int)s : 0), gx = x + (n == 0 ? (int)s : 0);
    double kg[4];
    if (in_hole(p, gy, gx))
        k_hole(p, ue, y, x, n, kg);
    else
        for (int c = 0; c < 4; ++c) kg[c] = K[k_at(p, c, gy, gx)];
    for (int a = 0; a < 2; ++a) {
        const double kw = 0.5 * (K[k_at(p, 2 * a + n, y, x)] + kg[2 * a + n]);
        q[a] = (-T[a] + kw * s) / s;
    }
}

/* Boundary moments r_bd and Pbar* for the anti-bounce-back rule (26) at node
 * (y, x): walls across axis x (sx = -1 or +1, 0 if none) and axis y (sy).
 * In the wall frame the normal row and column take the transformed
 * tractions (the tensor is symmetric); a tangential entry keeps the
 * populations' moment Pi at the node. At a corner the normal entries come
 * from the two walls and the off-diagonal is the mean of both (Q20). */
static void traction_wall_moments(const oracle_params *p, const double *f, const double *K, const double *ue,
                                  int y, int x,
                                  int sx, const double Tx[2], int sy, const double Ty[2],
                                  double *rbd, double Pstar[4])
{
    double r0, Pi0[4], qx[2], qy[2];
    moments_r_pi(p, f, at(p, y, x), &r0, Pi0);
    *rbd = r0;
    Pstar[0] = Pi0[0];
    Pstar[1] = Pi0[1];
    Pstar[2] = Pi0[2];
    Pstar[3] = Pi0[3];
    if (sx && sy) {
        traction_column(p, K, ue, y, x, 0, (double)sx, Tx, qx);
        traction_column(p, K, ue, y, x, 1, (double)sy, Ty, qy);
        Pstar[0] = qx[0];
        Pstar[3] = qy[1];
        Pstar[1] = Pstar[2] = 0.5 * (qx[1] + qy[0]);
    } else if (sy) {
        traction_column(p, K, ue, y, x, 1, (double)sy, Ty, qy);
        Pstar[1] = qy[0];
        Pstar[2] = qy[0];
        Pstar[3] = qy[1];
    } else {
        traction_column(p, K, ue, y, x, 0, (double)sx, Tx, qx);
        Pstar[0] = qx[0];
        Pstar[1] = qx[1];
        Pstar[2] = qx[1];
    }
}

/* anti-bounce-back value (eq. (26)) for outgoing direction i */
static double abb_term(const oracle_params *p, int i, double rbd, const double Pstar[4])
{
    double s2 = cs2(p), C[2];
    oracle_velocity(p, i, C);
    double A[4] = {Pstar[0] - rbd * s2, Pstar[1], Pstar[2], Pstar[3] - rbd * s2};
    double B[4] = {C[0] * C[0] - s2, C[0] * C[1], C[1] * C[0], C[1] * C[1] - s2};
    double AB = A[0] * B[0] + A[1] * B[1] + A[2] * B[2] + A[3] * B[3];
    return 2.0 * weight(i) * (rbd + AB / (2.0 * s2 * s2));
}

/* bounce-back correction (eq. (25)) for outgoing direction i */
static double bb_term(const oracle_params *p, int i, const double jstar[2])
{
    double C[2];
    oracle_velocity(p, i, C);
    return -2.0 / cs2(p) * weight(i) * (C[0] * jstar[0] + C[1] * jstar[1]);
}

/* Periodic edges come in pairs. Hole nodes (Q23) keep off rows and columns
 * next to a wall, and no material node has hole nodes on both sides along
 * one axis (the method gives such a node no gradient along that axis). A
 * hole may be a single node wide. */
static int edges_valid(const oracle_params *p)
{
    if ((p->bc_xmin == ORACLE_PERIODIC) != (p->bc_xmax == ORACLE_PERIODIC) ||
        (p->bc_ymin == ORACLE_PERIODIC) != (p->bc_ymax == ORACLE_PERIODIC))
        return 0;
    if (!p->solid) return 1;
    for (int y = 0; y < p->ny; ++y)
        for (int x = 0; x < p->nx; ++x) {
            int hole = in_hole(p, y, x);
            if (hole && (((y == 0 || y == p->ny - 1) && p->bc_ymin != ORACLE_PERIODIC) ||
                         ((x == 0 || x == p->nx - 1) && p->bc_xmin != ORACLE_PERIODIC)))
                return 0;
            if (!hole && ((in_hole(p, y, x - 1) && in_hole(p, y, x + 1)) ||
                          (in_hole(p, y - 1, x) && in_hole(p, y + 1, x))))
                return 0;
        }
    return 1;
}

/* Initialisation (Algorithm 1): r0 = -rho0 div u0 (eq. (18)), j0 = rho0 v0,
 * Pbar0 = Pbar(H(u0)) (eq. (15)), f = f^eq(r0, j0, Pbar0) (eq. (20)). */
int oracle_init(const oracle_params *p, const double *u0, const double *v0,
                double *f, double *u, double *j)
{
    int nx = p->nx, ny = p->ny;
    if (nx < 5 || ny < 5 || !edges_valid(p)) return -1;
    double *ue = malloc(sizeof(double) * 2 * ue_plane(p));
    static const double rest[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    extend_u(p, u0, rest, ue);
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            size_t s = at(p, y, x);
            double H[4], Pb[4], jj[2], feq[9];
            if (in_hole(p, y, x)) {
                for (int i = 0; i < 9; ++i) f[i * plane(p) + s] = 0.0;
                u[s] = u[plane(p) + s] = j[s] = j[plane(p) + s] = 0.0;
                continue;
            }
            grad_u(p, ue, y, x, H);
            oracle_poisson(p->mu, H, Pb);
            double r = -p->rho0 * (H[0] + H[3]);
            jj[0] = p->rho0 * v0[s];
            jj[1] = p->rho0 * v0[plane(p) + s];
            oracle_equilibrium(p, r, jj, Pb, feq);
            for (int i = 0; i < 9; ++i) f[i * plane(p) + s] = feq[i];
            u[s] = u0[s];
            u[plane(p) + s] = u0[plane(p) + s];
            j[s] = jj[0];
            j[plane(p) + s] = jj[1];
        }
    free(ue);
    return 0;
}

/* One time step of Algorithm 1 with readings R1/R2. wall[] holds the
 * momentum walls' displacements at the time of the state on entry and is
 * advanced with it. */
static void one_step(const oracle_params *p, double *f, double *u, double *j, double *jprev, double wall[8])
{
    int nx = p->nx, ny = p->ny;
    size_t N = plane(p);
    double dt = oracle_dt(p);
    double wall_next[8];
    advance_walls(p, wall, wall_next);
    double omega = 1.0 / p->tau_over_dt; /* dt / tau */
    double *ue = malloc(sizeof(double) * 2 * ue_plane(p));
    double *K = malloc(sizeof(double) * 4 * k_plane(p));
    double *S = malloc(sizeof(double) * 2 * N);
    double *fcol = malloc(sizeof(double) * 9 * N);
    double *fnew = malloc(sizeof(double) * 9 * N);
    double *jf = malloc(sizeof(double) * 2 * N);
    double *Sp = malloc(sizeof(double) * 2 * N);

    /* 1. stress sum K(u_n) and source 1S_n (eq. (23)) */
    extend_u(p, u, wall, ue);
    stress_sum(p, ue, K);
    source_field(p, ue, K, S);

    /* 2. moments of f_n, equilibrium (20), source populations (22), collision (4) */
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            size_t s = at(p, y, x);
            if (in_hole(p, y, x)) {
                for (int i = 0; i < 9; ++i) fcol[i * N + s] = 0.0;
                continue;
            }
            double r, Pi[4], jj[2] = {j[s], j[N + s]}, SS[2] = {S[s], S[N + s]}, feq[9], psi[9];
            moments_r_pi(p, f, s, &r, Pi);
            oracle_equilibrium(p, r, jj, Pi, feq);
            oracle_source_pop(p, SS, psi);
            for (int i = 0; i < 9; ++i) {
                double fi = f[i * N + s];
                fcol[i * N + s] = fi - omega * (fi - feq[i]) + dt * (1.0 - 0.5 * omega) * psi[i];
            }
        }

    /* 3. push streaming (5); links that cross a wall are handled below */
#pragma omp parallel for schedule(static)
    for (int i = 0; i < 9; ++i) {
        int ex = ex_of(i), ey = ey_of(i);
        for (int y = 0; y < ny; ++y) {
            int yt = y + ey;
            if (yt < 0 || yt >= ny) {
                if (p->bc_ymin != ORACLE_PERIODIC) continue;
                yt = wrap(yt, ny);
            }
            for (int x = 0; x < nx; ++x) {
                int xt = x + ex;
                if (xt < 0 || xt >= nx) {
                    if (p->bc_xmin != ORACLE_PERIODIC) continue;
                    xt = wrap(xt, nx);
                }
                if (in_hole(p, y, x) || in_hole(p, yt, xt)) continue;
                fnew[i * N + at(p, yt, xt)] = fcol[i * N + at(p, y, x)];
            }
        }
    }

    /* 4. boundary rules (Sec. 6, eqs. (25), (26)): a link that would leave
     * through a wall returns into the opposite direction at the same node */
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x)
            for (int i = 0; i < 9; ++i) {
                int ex = ex_of(i), ey = ey_of(i);
                int sx = 0, sy = 0; /* walls the link crosses (outward sign) */
                if (in_hole(p, y, x)) continue;
                if ((ex || ey) && in_hole(p, y + ey, x + ex)) {
                    /* a traction-free hole wall (Q23) */
                    static const double zero[2] = {0.0, 0.0};
                    int hx = ex && in_hole(p, y, x + ex), hy = ey && in_hole(p, y + ey, x);
                    if (!hx && !hy) hx = hy = 1; /* the diagonal through a hole corner */
                    double rbd, Pstar[4];
                    traction_wall_moments(p, f, K, ue, y, x, hx ? ex : 0, zero, hy ? ey : 0, zero, &rbd, Pstar);
                    fnew[opposite(i) * N + at(p, y, x)] = -fcol[i * N + at(p, y, x)] + abb_term(p, i, rbd, Pstar);
                    continue;
                }
                if ((x + ex < 0 || x + ex >= nx) && p->bc_xmin != ORACLE_PERIODIC) sx = ex;
                if ((y + ey < 0 || y + ey >= ny) && p->bc_ymin != ORACLE_PERIODIC) sy = ey;
                if (!sx && !sy) continue;
                int kx = sx < 0 ? p->bc_xmin : p->bc_xmax, ky = sy < 0 ? p->bc_ymin : p->bc_ymax;
                const double *vx = sx < 0 ? p->val_xmin : p->val_xmax;
                const double *vy = sy < 0 ? p->val_ymin : p->val_ymax;
                double fc = fcol[i * N + at(p, y, x)], v;
                int dir_x = sx && kx == ORACLE_DIRICHLET_J, dir_y = sy && ky == ORACLE_DIRICHLET_J;
                if (dir_x || dir_y) {
                    double js[2];
                    for (int a = 0; a < 2; ++a)
                        js[a] = (dir_x && dir_y) ? 0.5 * (vx[a] + vy[a]) : (dir_x ? vx[a] : vy[a]);
                    v = fc + bb_term(p, i, js);
                } else {
                    double rbd, Pstar[4];
                    traction_wall_moments(p, f, K, ue, y, x, sx, vx, sy, vy, &rbd, Pstar);
                    v = -fc + abb_term(p, i, rbd, Pstar);
                }
                fnew[opposite(i) * N + at(p, y, x)] = v;
            }

    /* hole nodes carry no populations */
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x)
            if (in_hole(p, y, x))
                for (int i = 0; i < 9; ++i) fnew[i * N + at(p, y, x)] = 0.0;

    /* 5. first moment of the streamed populations, jf = sum_i C_i f_i */
#pragma omp parallel for schedule(static)
    for (size_t s = 0; s < N; ++s) {
        double a0 = 0.0, a1 = 0.0;
        for (int i = 0; i < 9; ++i) {
            double C[2];
            oracle_velocity(p, i, C);
            a0 += C[0] * fnew[i * N + s];
            a1 += C[1] * fnew[i * N + s];
        }
        jf[s] = a0;
        jf[N + s] = a1;
    }

    /* 6. source at the new time level: predictor-corrector (R2), j
     * extrapolated from t - dt and t (Q22), or explicit */
    if (p->scheme == 0 || p->scheme == 2) {
        double *up = malloc(sizeof(double) * 2 * N);
        for (int a = 0; a < 2; ++a)
            for (size_t s = 0; s < N; ++s) {
                double jp = p->scheme == 0 ? jf[a * N + s] + 0.5 * dt * S[a * N + s]
                                           : 2.0 * j[a * N + s] - jprev[a * N + s];
                up[a * N + s] = u[a * N + s] + dt / (2.0 * p->rho0) * (jp + j[a * N + s]);
            }
        source_of_u(p, up, wall_next, Sp);
        free(up);
    } else {
        memcpy(Sp, S, sizeof(double) * 2 * N);
    }

    /* 7. moments with half source (6) and trapezoidal displacement (24) */
    for (int a = 0; a < 2; ++a)
        for (size_t s = 0; s < N; ++s) {
            double jnew = jf[a * N + s] + 0.5 * dt * Sp[a * N + s];
            u[a * N + s] += dt / (2.0 * p->rho0) * (jnew + j[a * N + s]);
            if (jprev) jprev[a * N + s] = j[a * N + s];
            j[a * N + s] = jnew;
        }
    memcpy(f, fnew, sizeof(double) * 9 * N);
    memcpy(wall, wall_next, sizeof(wall_next));

    free(ue);
    free(K);
    free(S);
    free(fcol);
    free(fnew);
    free(jf);
    free(Sp);
}

/* nsteps steps of the predictor-corrector or explicit scheme; wall[8] (see
 * advance_walls) is advanced with the state. */
int oracle_step(const oracle_params *p, double *f, double *u, double *j, double *wall, int nsteps)
{
    if (p->nx < 5 || p->ny < 5 || p->tau_over_dt <= 0.5 || !edges_valid(p) || p->scheme < 0 || p->scheme > 1)
        return -1;
    for (int n = 0; n < nsteps; ++n) one_step(p, f, u, j, NULL, wall);
    return 0;
}

/* any scheme; jprev holds j one step before the state (j itself before the
 * first step) and is advanced with it, as is wall[8] */
int oracle_step_prev(const oracle_params *p, double *f, double *u, double *j, double *jprev, double *wall,
                     int nsteps)
{
    if (p->nx < 5 || p->ny < 5 || p->tau_over_dt <= 0.5 || !edges_valid(p) || p->scheme < 0 || p->scheme > 2)
        return -1;
    for (int n = 0; n < nsteps; ++n) one_step(p, f, u, j, jprev, wall);
    return 0;
}

/* Output fields: v = j / rho0 and the first Piola-Kirchhoff stress P(H(u)),
 * with the walls at the displacements wall[8]. */
int oracle_fields(const oracle_params *p, const double *u, const double *j, const double *wall,
                  double *v, double *P)
{
    int nx = p->nx, ny = p->ny;
    size_t N = plane(p);
    double *ue = malloc(sizeof(double) * 2 * ue_plane(p));
    extend_u(p, u, wall, ue);
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            size_t s = at(p, y, x);
            double H[4], PP[4];
            if (in_hole(p, y, x)) {
                for (int c = 0; c < 4; ++c) P[c * N + s] = 0.0;
                v[s] = v[N + s] = 0.0;
                continue;
            }
            grad_u(p, ue, y, x, H);
            oracle_piola(p->lam, p->mu, H, PP);
            for (int c = 0; c < 4; ++c) P[c * N + s] = PP[c];
            v[s] = j[s] / p->rho0;
            v[N + s] = j[N + s] / p->rho0;
        }
    free(ue);
    return 0;
}

/* Derived fields of the displacement: Cauchy stress sig[a][b][y][x],
 * Green-Lagrange strain E[a][b][y][x] and strain-energy density W[y][x], all
 * from the same central-difference H(u) as the Piola stress of
 * oracle_fields. Any output may be NULL. */
int oracle_derived(const oracle_params *p, const double *u, const double *wall, double *sig, double *E, double *W)
{
    int nx = p->nx, ny = p->ny;
    size_t N = plane(p);
    double *ue = malloc(sizeof(double) * 2 * ue_plane(p));
    extend_u(p, u, wall, ue);
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            size_t s = at(p, y, x);
            double H[4], T[4];
            if (in_hole(p, y, x)) {
                for (int c = 0; c < 4; ++c) {
                    if (sig) sig[c * N + s] = 0.0;
                    if (E) E[c * N + s] = 0.0;
                }
                if (W) W[s] = 0.0;
                continue;
            }
            grad_u(p, ue, y, x, H);
            if (sig) {
                oracle_cauchy(p->lam, p->mu, H, T);
                for (int c = 0; c < 4; ++c) sig[c * N + s] = T[c];
            }
            if (E) {
                oracle_green_lagrange(H, T);
                for (int c = 0; c < 4; ++c) E[c * N + s] = T[c];
            }
            if (W) W[s] = oracle_strain_energy(p->lam, p->mu, H);
        }
    free(ue);
    return 0;
}

/* Diagnostics: out[0..1] = sum of j, out[2] = sum of r, out[3] = energy
 * sum (|j|^2/(2 rho0) + W) dX^2, out[4] = min J, out[5] = max spectral norm of
 * the Green-Lagrange strain E = (F^T F - I)/2, out[6] = 1 if any value is not
 * finite or J <= 0. Sums run in plain row-major order. */
int oracle_diagnostics(const oracle_params *p, const double *f, const double *u,
                       const double *j, const double *wall, double out[7])
{
    int nx = p->nx, ny = p->ny;
    size_t N = plane(p);
    double *ue = malloc(sizeof(double) * 2 * ue_plane(p));
    extend_u(p, u, wall, ue);
    double sj0 = 0, sj1 = 0, sr = 0, en = 0, minJ = INFINITY, maxE = 0;
    int bad = 0;
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            size_t s = at(p, y, x);
            double H[4], r = 0.0;
            if (in_hole(p, y, x)) continue;
            grad_u(p, ue, y, x, H);
            for (int i = 0; i < 9; ++i) r += f[i * N + s];
            double F11 = 1.0 + H[0], F12 = H[1], F21 = H[2], F22 = 1.0 + H[3];
            double J = F11 * F22 - F12 * F21;
            double E11 = 0.5 * (F11 * F11 + F21 * F21 - 1.0);
            double E12 = 0.5 * (F11 * F12 + F21 * F22);
            double E22 = 0.5 * (F12 * F12 + F22 * F22 - 1.0);
            double mean = 0.5 * (E11 + E22), dev = sqrt(0.25 * (E11 - E22) * (E11 - E22) + E12 * E12);
            double En = fmax(fabs(mean + dev), fabs(mean - dev));
            double jj0 = j[s], jj1 = j[N + s];
            sj0 += jj0;
            sj1 += jj1;
            sr += r;
            if (!(J > 0.0) || !isfinite(jj0) || !isfinite(jj1) || !isfinite(u[s]) || !isfinite(u[N + s]))
                bad = 1;
            else
                en += ((jj0 * jj0 + jj1 * jj1) / (2.0 * p->rho0) + oracle_strain_energy(p->lam, p->mu, H)) * p->dx * p->dx;
            if (J < minJ) minJ = J;
            if (En > maxE) maxE = En;
        }
    free(ue);
    out[0] = sj0;
    out[1] = sj1;
    out[2] = sr;
    out[3] = en;
    out[4] = minJ;
    out[5] = maxE;
    out[6] = bad;
    return 0;
}
