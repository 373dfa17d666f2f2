/*
 * lbm_solid.h -- C ABI of the MI355X (gfx950) implementation of the
 * per-time-step lattice update of the Lagrangian lattice Boltzmann method for
 * nonlinear solids of Faust, Schlueter, Mueller & Mueller (2022).
 *
 * One handle holds one plate: a D2Q9 lattice of nx * ny sites in the
 * reference configuration (Sec. 3), a compressible neo-Hooke material
 * (Sec. 7, eq. (27)) and per-edge boundary rules (Sec. 6). lbm_step advances
 * the state by Algorithm 1 (Sec. 5):
 *   source 1S = rho0 b + div(P(H) + Pbar(H)) by central differences (eq. (23)),
 *   BGK collision with He forcing (eq. (4)) towards the equilibrium (eq. (20)),
 *   streaming (eq. (5)), the boundary rules (eqs. (25), (26)), moments with
 *   the half source (eq. (6)) and the trapezoidal displacement update (eq. (24)).
 * The second moment that enters the equilibrium is the populations' own
 * second moment; the source of the moment step is taken at t + dt by a
 * predictor-corrector (the footnote on stability in Sec. 5), or at t as
 * printed in Algorithm 1 (LBM_SCHEME_EXPLICIT), or at t + dt from a
 * predictor displacement whose j is extrapolated linearly from t - dt and t
 * (LBM_SCHEME_EXTRAP, the variant closing Sec. 5).
 *
 * Units: every value that crosses this ABI is in physical units (lengths in
 * the unit of dx, rho0, lambda, mu, velocities, stresses). The time step is
 * fixed by the material: dt = dx / (sqrt(3) sqrt(mu / rho0)) (Sec. 7 prints
 * it for two spacings).
 *
 * Memory: the library never allocates device memory. The caller passes a
 * device workspace of at least lbm_workspace_bytes() bytes and a HIP stream;
 * both must outlive the handle. Host arrays are copied during the call that
 * receives them and stay owned by the caller.
 *
 * Errors: every call returns an lbm_status; no exception crosses the ABI.
 * lbm_last_error() gives a message for the last failing call on a handle.
 * A handle is not thread-safe; distinct handles on distinct streams may run
 * concurrently.
 *
 * Host field layout: structure of arrays, component-major, x fastest:
 * u[a][y][x] and v[a][y][x] with a in {x, y}; P[a][b][y][x] row-major
 * (P11, P12, P21, P22). Node (x, y) sits at X = (x dx, y dx).
 */
#ifndef LBM_SOLID_H
#define LBM_SOLID_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_solver lbm_solver;

typedef enum {
    LBM_OK = 0,
    LBM_ERR_ARG = -1,         /* invalid argument */
    LBM_ERR_NOMEM = -2,       /* workspace too small */
    LBM_ERR_HIP = -3,         /* a HIP runtime call failed */
    LBM_ERR_STATE = -4,       /* call out of order (e.g. step before set_fields) */
    LBM_ERR_UNSTABLE = -5,    /* J <= 0 or a non-finite value appeared */
    LBM_ERR_UNSUPPORTED = -6  /* valid request the library does not implement */
} lbm_status;

/* Storage and arithmetic precision.
 * FP64: populations, displacement, momentum and arithmetic in double.
 * FP32: all in float.
 * FP32_U64: as FP32 with the displacement stored and accumulated in double
 *   (the accumulator of eq. (24) then adds no float rounding per step).
 * FP16_STORE / BF16_STORE: populations stored in half / bfloat16, scaled by a
 *   per-plate power of two chosen at lbm_set_fields; displacement in double,
 *   momentum in float, arithmetic in float. */
typedef enum { LBM_FP64 = 0, LBM_FP32 = 1, LBM_FP16_STORE = 2, LBM_BF16_STORE = 3, LBM_FP32_U64 = 4 } lbm_precision;

/* Rounding of 16-bit population stores. NEAREST: round to nearest even.
 * STOCHASTIC: round up or down with probability given by the distance to
 * the two neighbours (unbiased), with random bits from a counter-based hash
 * of (seed, step index of the state written, site, population), so a run is
 * reproducible for a seed and independent of launch shape, steps per launch
 * and batching. 32- and 64-bit storage always rounds to nearest. */
typedef enum { LBM_ROUND_NEAREST = 0, LBM_ROUND_STOCHASTIC = 1 } lbm_rounding;

/* Time level of the source in the moment step (Sec. 5). EXTRAP takes the
 * predictor displacement from the trapezoidal rule with j(t + dt) replaced
 * by 2 j(t) - j(t - dt) (j(t - dt) = j(0) at the first step). It grows for
 * lambda > mu (about 9 % per step at lambda = 2 mu) and always runs the
 * general step, so it needs lbm_workspace_bytes_walled(). */
typedef enum { LBM_SCHEME_PC = 0, LBM_SCHEME_EXPLICIT = 1, LBM_SCHEME_EXTRAP = 2 } lbm_scheme;

typedef enum { LBM_EDGE_XMIN = 0, LBM_EDGE_XMAX = 1, LBM_EDGE_YMIN = 2, LBM_EDGE_YMAX = 3 } lbm_edge;

/* Boundary rules of Sec. 6. Walls lie half a spacing outside the outermost
 * node row. DIRICHLET_J: bounce-back with wall momentum j* (eq. (25)), value
 * = j* (2 components). NEUMANN_T: anti-bounce-back with the boundary Poisson
 * stress built from the traction T* (eq. (26) and the traction transform),
 * value = T* (2 components). */
typedef enum { LBM_BC_PERIODIC = 0, LBM_BC_DIRICHLET_J = 1, LBM_BC_NEUMANN_T = 2 } lbm_bc;

typedef struct {
    double momentum[2];  /* sum over sites of j = rho0 v */
    double mass_moment;  /* sum over sites of r = sum_i f_i */
    double energy;       /* sum (|j|^2 / (2 rho0) + W(F)) dx^2, W of eq. (27) */
    double min_J;        /* smallest det F */
    double max_strain;   /* largest spectral norm of E = (F^T F - I) / 2 */
    int32_t unstable;    /* 1 if J <= 0 or a non-finite value was met */
    int32_t reserved;
    int64_t steps;       /* steps done since lbm_set_fields */
} lbm_diagnostics;

/* Exact device bytes a plate of nx * ny sites needs at precision p
 * (two copies of the state plus staging and reduction scratch). */
size_t lbm_workspace_bytes(int nx, int ny, lbm_precision p);

/* Device bytes a plate needs when it may have walls on its x edges, holes
 * or the extrapolation scheme (the general step): lbm_workspace_bytes plus
 * a copy of j for the extrapolation scheme, one mask byte per site and a
 * byte per tile of the general step. */
size_t lbm_workspace_bytes_walled(int nx, int ny, lbm_precision p);

/* Create a handle. nx, ny >= 5; dx > 0. dev_workspace: device memory of
 * ws_bytes >= lbm_workspace_bytes(nx, ny, p) bytes (lbm_workspace_bytes_walled
 * for LBM_SCHEME_EXTRAP; LBM_ERR_NOMEM otherwise), 256-byte aligned.
 * hip_stream: a hipStream_t (NULL = the default stream). */
lbm_status lbm_create(int nx, int ny, double dx, lbm_precision p, lbm_scheme s,
                      void *dev_workspace, size_t ws_bytes, void *hip_stream, lbm_solver **out);

/* Material (Sec. 7): reference density rho0 > 0, Lame parameters with
 * mu > 0 and lambda + mu > 0, relaxation time tau as tau/dt > 1/2. */
lbm_status lbm_set_material(lbm_solver *h, double rho0, double lambda, double mu, double tau_over_dt);

/* Uniform body force per unit mass b (the rho0 b term of eq. (23)). */
lbm_status lbm_set_body_force(lbm_solver *h, const double b[2]);

/* Boundary rule of one edge. Periodic edges come in pairs (making one edge
 * of a periodic pair a wall turns the other into a momentum wall at rest
 * until it is set). value may be NULL for LBM_BC_PERIODIC. Takes effect from
 * the next lbm_step, so a load history can be applied step by step.
 * Walls on the x edges run the general step (one launch of 2D tiles with
 * walls and corners on every edge) and need a workspace of
 * lbm_workspace_bytes_walled() bytes
 * (LBM_ERR_NOMEM otherwise). At a corner of two walls the diagonal link takes
 * the momentum wall's rule if either wall is one (the mean j* if both are);
 * between two traction walls it is anti-bounced with both walls' transformed
 * tractions, the off-diagonal entry being their mean. */
lbm_status lbm_set_boundary(lbm_solver *h, lbm_edge e, lbm_bc bc, const double value[2]);

/* Initial displacement u0 and velocity v0 (host, [2][ny][nx], physical
 * units). Builds f = f^eq(r0, j0, Pbar(H(u0))) with r0 = -rho0 div u0 and
 * j0 = rho0 v0 (Algorithm 1, initialisation) and resets the step count.
 * Every value must be finite, hole nodes included (LBM_ERR_ARG otherwise).
 * Synchronises the stream. Needs the material to be set first. */
lbm_status lbm_set_fields(lbm_solver *h, const double *u0, const double *v0);

/* Enqueue nsteps time steps on the stream and return at once. On a plate
 * with x walls or holes large enough that part of it lies clear of every
 * wall and hole, each step (with the predictor-corrector and 32- or
 * 64-bit populations, each pair of steps) runs that part on the handle's
 * stream and the rest on a stream the library creates (default priority),
 * forked and joined with events: work enqueued on the handle's stream
 * after lbm_step still sees the whole step. */
lbm_status lbm_step(lbm_solver *h, int64_t nsteps);

/* Read u, v = j / rho0, the first Piola-Kirchhoff stress P(H(u)) and the
 * diagnostics. Any pointer may be NULL. Synchronises the stream. Returns
 * LBM_ERR_UNSTABLE (after filling the outputs) if the unstable flag is set. */
lbm_status lbm_read_fields(lbm_solver *h, double *u, double *v, double *P, lbm_diagnostics *d);

/* The diagnostics of lbm_read_fields (d only) with no use of the
 * workspace's reduction scratch and no device allocation: for callers that
 * cannot allocate device memory or touch the workspace's scratch, such as code
 * being captured into a HIP graph, tight serving loops, or harnesses that
 * forbid allocation. The per-block partial sums and the folded values go to
 * a static device array of the library, 1024 * 8 + 8 doubles (65,600
 * bytes) per GPU, held until the process ends; the diagnostics grid
 * is capped at 1024 blocks, so no plate needs more (LBM_ERR_UNSUPPORTED
 * otherwise). Every call on one GPU shares that array: calls that overlap on
 * one GPU (from different threads or streams) race and must be serialised by
 * the caller. Results equal lbm_read_fields' diagnostics bit for bit. Runs on
 * the device current at lbm_create (restoring the caller's current device);
 * synchronises the stream; LBM_ERR_UNSTABLE as lbm_read_fields. */
lbm_status lbm_read_diagnostics_noalloc(lbm_solver *h, lbm_diagnostics *d);

/* Derived fields in physical units, from the same central-difference
 * displacement gradient H(u) as P (Sec. 5): the Cauchy stress
 * sigma = J^-1 P F^T ([4][ny][nx]: sigma11, sigma12, sigma21, sigma22; Sec. 7
 * reads sigma12 and sigma22 out at points of the plate with a hole), the
 * Green-Lagrange strain E = (F^T F - I) / 2 ([4][ny][nx]) and the
 * strain-energy density W of eq. (27) ([ny][nx]). Any pointer may be NULL.
 * Synchronises the stream. */
lbm_status lbm_read_derived(lbm_solver *h, double *sigma, double *E, double *W);

/* Values at n nodes (x[k], y[k]) (0 <= x < nx, 0 <= y < ny), for time series
 * at chosen points (Sec. 7 plots displacements and stresses at nodes):
 * out[n][17] = u (2), v (2), P (4), sigma (4), E (4), W, as lbm_read_fields and
 * lbm_read_derived, physical units. n is limited by the read-out staging area
 * (at least 460 nodes; about 120 000 for plates of 2^18 sites or more;
 * LBM_ERR_ARG beyond it). Host
 * arrays; synchronises the stream. */
lbm_status lbm_sample(lbm_solver *h, int n, const int *x, const int *y, double *out);

/* Launch shape of the step kernel: threads per block (64, 128, 256 or 512;
 * one lattice column per thread) and row segments per column strip
 * (1 <= n_segs <= ny). Results do not depend on it (bitwise); it only
 * changes speed. lbm_create picks a default; the autotuner overrides it. */
lbm_status lbm_set_tiling(lbm_solver *h, int block, int n_segs);
lbm_status lbm_get_tiling(const lbm_solver *h, int *block, int *n_segs);

/* Time steps per launch of the step kernel: 1, or 2 with the
 * predictor-corrector scheme (two steps fused in one pass over the state,
 * which halves the memory traffic per step; results are bitwise the same).
 * An odd remainder of lbm_step runs as a single step. With 2, the two
 * pipelines' LDS must fit a compute unit: a 512-thread block does with FP32,
 * and with the other forms except FP64 while the y edges are periodic.
 * Otherwise lbm_set_tiling returns LBM_ERR_UNSUPPORTED, and a 512-thread
 * tiling already set is lowered to 256 threads (by this call, or when
 * lbm_set_boundary makes the y edges walls). */
lbm_status lbm_set_steps_per_launch(lbm_solver *h, int k);
lbm_status lbm_get_steps_per_launch(const lbm_solver *h, int *k);

/* Number of blocks of the step kernel with this launch shape (threads per
 * block, time steps per launch) that the handle's device runs at once, for
 * the handle's precision, scheme and boundaries: blocks per compute unit from
 * the occupancy calculator times the number of compute units. A grid of at
 * most this many blocks runs in a single wave of blocks; n_segs can be
 * chosen with it. Writes 0 for a shape the handle cannot launch. */
lbm_status lbm_resident_blocks(const lbm_solver *h, int block, int steps_per_launch, int *blocks);

/* Run every step as the general step (1: one launch of 2D tiles, each
 * holding its whole neighbourhood in LDS) or, when no x edge is a wall, as
 * the fused step kernel (0, the default). Both give the same results up to
 * rounding. The general step runs walls on the x edges, holes and the
 * extrapolation scheme; on small plates it is also the faster one (its
 * tiles' stages run in parallel where the fused kernel marches rows one
 * after another). Needs no workspace beyond what the plate's edges, mask
 * and scheme already need. */
lbm_status lbm_set_general_path(lbm_solver *h, int on);

/* Holes in the plate (the plate with a hole of Sec. 7.2). solid: host array
 * [ny][nx], nonzero for a material node, 0 for a node in a hole; NULL
 * removes the mask. A link from a material node into a hole crosses a
 * traction-free wall half-way between the nodes. The wall is the one the
 * link's axis step enters; the diagonal that meets a hole corner crosses
 * both and takes the two-wall rule. In the central differences a hole
 * neighbour takes the node's own displacement. Hole nodes hold no
 * material: their fields read as zero and they add nothing to the
 * diagnostics. Holes must keep off the rows and columns next to a wall
 * edge (they may cross periodic edges), and no material node may have hole
 * nodes on both sides along one axis (material at least two nodes thick;
 * LBM_ERR_ARG otherwise; the method gives such a node no gradient). A hole
 * may be one node wide: each material node beside it takes the stress sum
 * of its own gradient there (the derivatives across the hole set to zero),
 * so the nodes on its two sides see different values. Once a mask
 * is set, lbm_set_boundary may change boundary values and kinds but may not
 * make an edge periodic or not (LBM_ERR_STATE). Set
 * the boundaries first, then the mask, then the fields (LBM_ERR_STATE
 * after lbm_set_fields). Needs lbm_workspace_bytes_walled() (LBM_ERR_NOMEM
 * otherwise); runs the general step. Copies the array; synchronises. */
lbm_status lbm_set_mask(lbm_solver *h, const unsigned char *solid);

/* Rounding of the populations written by later steps (the start state of
 * lbm_set_fields always rounds to nearest). STOCHASTIC needs FP16_STORE or
 * BF16_STORE (LBM_ERR_UNSUPPORTED otherwise). */
lbm_status lbm_set_rounding(lbm_solver *h, lbm_rounding r, uint64_t seed);

/* Time step dt of the handle's material. */
lbm_status lbm_get_dt(const lbm_solver *h, double *dt);

/* Destroy the handle (and the stream the library may have created for it).
 * Never frees the workspace or the caller's stream. */
void lbm_destroy(lbm_solver *h);

/* Message of the last failing call on h (or of the last failing
 * lbm_create if h is NULL). Valid until the next call on h. */
const char *lbm_last_error(const lbm_solver *h);

/* ------------------------------------------------------------------------
 * Batches: many plates of uneven sizes advanced together.
 *
 * A batch owns an arena inside the caller's device workspace. Plates are
 * admitted (lbm_batch_add) while the arena and the tile table have room --
 * admission by device-memory footprint -- and keep their state resident
 * until retired. lbm_batch_step advances every admitted plate that has steps
 * left by up to nsteps, in one persistent launch per time step for all
 * plates (or two steps per launch, see lbm_batch_set_steps_per_launch),
 * enqueued as a HIP graph of those launches. All plates of a batch
 * share the precision, the scheme and the kind of y edges (all periodic, or
 * all walls with per-plate rules and values); x edges are periodic.
 * The batch uses 256-thread blocks; plates are cut into column strips and
 * row segments. Whenever the set of running plates changes, the segment
 * height (4 to 128 rows, 4 to 256 with two steps per launch) and the
 * placement of the tiles on the blocks of the persistent grid are chosen
 * on the host so that the busiest block has the least work.
 * ------------------------------------------------------------------------ */

typedef struct lbm_batch lbm_batch;

/* One plate's geometry, material (Sec. 7) and y-edge rules (Sec. 6), in
 * physical units as for the single-plate calls. */
typedef struct {
    int nx, ny;
    double dx;
    double rho0, lambda, mu, tau_over_dt;
    double body[2];
    lbm_bc bc_ymin, bc_ymax;
    double val_ymin[2], val_ymax[2];
    lbm_rounding rounding;  /* as lbm_set_rounding; STOCHASTIC needs 16-bit storage */
    uint64_t seed;
} lbm_plate_desc;

/* Arena bytes one plate of nx * ny sites uses at precision p. */
size_t lbm_batch_plate_bytes(int nx, int ny, lbm_precision p);
/* Tile-table entries one plate reserves: column strips times row segments
 * at the shortest segments the batch plans (4 rows, when few plates run). */
int lbm_batch_plate_tiles(int nx, int ny, lbm_precision p, lbm_scheme s);
/* Workspace bytes of a batch with room for max_plates plates, max_tiles
 * tiles and arena_bytes of plate state. */
size_t lbm_batch_workspace_bytes(int max_plates, int max_tiles, size_t arena_bytes);

/* Create a batch on a caller-owned, 256-byte aligned device workspace and a
 * HIP stream (both must outlive it). walled: 0 = plates periodic in y,
 * 1 = plates with y walls. Everything beyond the tables is arena. Allocates
 * small pinned host buffers for the tables. */
lbm_status lbm_batch_create(int max_plates, int max_tiles, lbm_precision p, lbm_scheme s, int walled,
                            void *dev_workspace, size_t ws_bytes, void *hip_stream, lbm_batch **out);

/* Admit a plate with start fields u0, v0 (host, [2][ny][nx], physical) that
 * is to run nsteps steps in total; returns its slot. LBM_ERR_NOMEM (and no
 * change) if the arena, the tile table or the slots are full. Synchronises
 * the stream. */
lbm_status lbm_batch_add(lbm_batch *b, const lbm_plate_desc *d, const double *u0, const double *v0,
                         int64_t nsteps, int *slot);

/* Enqueue up to nsteps steps (at most 2^20) for every plate with steps
 * left; a plate stops when it has done its nsteps. Returns at once. */
lbm_status lbm_batch_step(lbm_batch *b, int64_t nsteps);

/* Time steps per launch of the batch kernel: 1, or 2 with the
 * predictor-corrector scheme (the default with FP64, and with the other
 * forms when their two-step kernel keeps two waves per SIMD for the batch's
 * edges). With 2, a launch advances
 * every running plate by two steps in one pass over its state, or by one
 * step when that is the plate's last; results equal one step per launch
 * bitwise. Changing it synchronises the stream and re-plans the tiles. */
lbm_status lbm_batch_set_steps_per_launch(lbm_batch *b, int k);
lbm_status lbm_batch_get_steps_per_launch(const lbm_batch *b, int *k);

/* Steps done and left and the unstable flag of a plate. Synchronises. */
lbm_status lbm_batch_query(lbm_batch *b, int slot, int64_t *steps_done, int64_t *steps_left, int *unstable);

/* Fields and diagnostics of a plate, as lbm_read_fields. Synchronises. */
lbm_status lbm_batch_read(lbm_batch *b, int slot, double *u, double *v, double *P, lbm_diagnostics *d);

/* Derived fields and node samples of a plate, as lbm_read_derived and
 * lbm_sample. Synchronise. */
lbm_status lbm_batch_read_derived(lbm_batch *b, int slot, double *sigma, double *E, double *W);
lbm_status lbm_batch_sample(lbm_batch *b, int slot, int n, const int *x, const int *y, double *out);

/* Free a plate's slot, arena space and tiles. Synchronises the stream. */
lbm_status lbm_batch_retire(lbm_batch *b, int slot);

/* Live plates, free arena bytes and the largest free arena block. */
lbm_status lbm_batch_info(const lbm_batch *b, int *live_plates, size_t *arena_free, size_t *arena_largest_free);

void lbm_batch_destroy(lbm_batch *b);
const char *lbm_batch_last_error(const lbm_batch *b);

#ifdef __cplusplus
}
#endif

#endif /* LBM_SOLID_H */
