// batch_kernel.hpp -- one time step of many plates in one launch.
//
// The plates of a batch live in one device arena; a plate table and a tile
// table (plate, strip, segment) sit in device memory. A persistent grid of
// a fixed size walks the tile table with a stride of gridDim.x, so one launch
// (and one captured graph of K launches) serves any mix of plate sizes; the
// host only rewrites the tables between chunks. With one step per launch,
// launch k of a chunk advances plate p iff k < p.nsteps; its input copy is
// (parity0 + k) & 1 and its step index step0 + k. The two-step variant is
// described at its kernel.
#pragma once

#include "step_kernel.hpp"

namespace lbm {

struct PlateDesc {
    void *f[2], *u[2], *j[2];  // the two state copies
    int nx, ny;
    long long plane;
    double omega, lam, mu, bx, by;  // lattice units
    int bc_lo, bc_hi;
    double val_lo[2], val_hi[2];
    double f_scale, f_inv_scale;
    int strip_w, n_strips, n_segs, halo_a;
    long long step0;  // step index of the state at the start of the chunk
    int parity0;      // copy holding that state
    int nsteps;       // steps of this plate in the chunk (0: idle)
    unsigned *flag;   // this plate's unstable flag
    int sr;           // stochastic rounding of 16-bit populations
    unsigned long long seed;
};

// One tile of the persistent grid's table; plate < 0 marks an empty entry
// (a block with fewer tiles than others in a packed table).
struct TileDesc {
    int plate, strip, seg, pad;
};

// Step parameters of plate pd with input copy `in` at step index `step`.
__device__ __forceinline__ StepParams plate_step_params(const PlateDesc &pd, int in, long long step)
{
    StepParams sp;
    sp.f_in = pd.f[in];
    sp.u_in = pd.u[in];
    sp.j_in = pd.j[in];
    sp.f_out = pd.f[in ^ 1];
    sp.u_out = pd.u[in ^ 1];
    sp.j_out = pd.j[in ^ 1];
    sp.nx = pd.nx;
    sp.ny = pd.ny;
    sp.plane = pd.plane;
    sp.omega = pd.omega;
    sp.lam = pd.lam;
    sp.mu = pd.mu;
    sp.bx = pd.bx;
    sp.by = pd.by;
    sp.bc_lo = pd.bc_lo;
    sp.bc_hi = pd.bc_hi;
    sp.val_lo[0] = pd.val_lo[0];
    sp.val_lo[1] = pd.val_lo[1];
    sp.val_hi[0] = pd.val_hi[0];
    sp.val_hi[1] = pd.val_hi[1];
    // a batch plate's wall values never change: its walls are at j* n
    sp.uwb_lo[0] = sp.uwb_lo[1] = sp.uwb_hi[0] = sp.uwb_hi[1] = 0.0;
    sp.f_scale = pd.f_scale;
    sp.f_inv_scale = pd.f_inv_scale;
    sp.strip_w = pd.strip_w;
    sp.n_strips = pd.n_strips;
    sp.n_segs = pd.n_segs;
    sp.halo_a = pd.halo_a;
    sp.x_lo = sp.x_end = 0;  // strips over the whole width
    sp.flag = pd.flag;
    sp.step = step;
    sp.sr = pd.sr;
    sp.seed = pd.seed;
    return sp;
}

template <class PR, int BLOCK, bool PC, bool WALLED>
__global__ void __launch_bounds__(BLOCK)
    batch_step_kernel(const PlateDesc *__restrict__ plates, const TileDesc *__restrict__ tiles,
                      const int *__restrict__ n_tiles, const int k)
{
    __shared__ TileLds<PR, BLOCK, PC, WALLED> lds;
    const int nt = *n_tiles;
    for (int tile = blockIdx.x; tile < nt; tile += gridDim.x) {
        const TileDesc td = tiles[tile];
        if (td.plate < 0) continue;  // empty entry (uniform over the block)
        const PlateDesc &pd = plates[td.plate];
        if (k >= pd.nsteps) continue;  // uniform over the block
        const StepParams sp = plate_step_params(pd, (pd.parity0 + k) & 1, pd.step0 + k);
        step_tile<PR, BLOCK, PC, WALLED>(sp, td.strip, td.seg, lds);
    }
}

// Two steps per launch (predictor-corrector): launch k advances plate p by
// steps 2k and 2k+1 of the chunk, or by step 2k alone when that is its last
// (odd count), in one pass over its state; the plate's shapes carry the
// two-step halo, which also covers a single step. Launch k reads copy
// (parity0 + k) & 1 and writes the other one.
template <class PR, int BLOCK, bool WALLED>
__global__ void __launch_bounds__(BLOCK)
    batch_step2_kernel(const PlateDesc *__restrict__ plates, const TileDesc *__restrict__ tiles,
                       const int *__restrict__ n_tiles, const int k)
{
    __shared__ TileLds<PR, BLOCK, true, WALLED> lds[2];
    const int nt = *n_tiles;
    for (int tile = blockIdx.x; tile < nt; tile += gridDim.x) {
        const TileDesc td = tiles[tile];
        if (td.plate < 0) continue;  // empty entry (uniform over the block)
        const PlateDesc &pd = plates[td.plate];
        const int left = pd.nsteps - 2 * k;
        if (left <= 0) continue;  // uniform over the block
        const StepParams sp = plate_step_params(pd, (pd.parity0 + k) & 1, pd.step0 + 2 * k);
        if (left >= 2)
            step2_tile<PR, BLOCK, WALLED>(sp, td.strip, td.seg, lds[0], lds[1]);
        else
            step_tile<PR, BLOCK, true, WALLED>(sp, td.strip, td.seg, lds[0]);
    }
}

}  // namespace lbm
