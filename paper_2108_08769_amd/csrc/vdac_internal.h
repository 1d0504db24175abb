// vdac_internal.h -- structures shared by the host driver and the HIP kernels of libvdac.
//
// Device memory of one tank (all planes x-fastest, 256-byte aligned):
//   state[3]   three rotating state buffers, 4 planes each: rho, rho*u, rho*v, p.  The current
//              state, the stage-0 state of the running pseudo-iteration and the stage outputs
//              rotate among them (see stage_buffers below), so no state is ever copied.
//   level_n    3 planes (rho, rho*u, rho*v) of real-time level n; level_nm1 the same for BDF2.
//   flags      one byte per cell: which faces are walls (domain wall or solid neighbour) and
//              whether the cell itself is solid.
//   partials   per-workgroup residual partial sums of the last Runge-Kutta stage.
//   status     pseudo-loop control of the tank (iteration count, stop flags, norms).
#pragma once

#include <stddef.h>
#include <stdint.h>

namespace vdac {

enum : uint8_t {
    FLAG_WALL_XM = 1,   // face at x - dx/2 is a wall
    FLAG_WALL_XP = 2,   // face at x + dx/2 is a wall
    FLAG_WALL_YM = 4,
    FLAG_WALL_YP = 8,
    FLAG_SOLID = 16,    // the cell is solid (never updated)
};

// Pseudo-loop control of one tank, in device memory.  Written by begin_step and finalize only.
struct Status {
    int32_t done;        // nonzero: the kernels of this tank return at once
    int32_t iters;       // pseudo-iterations completed in the current real step
    int32_t cur;         // index (0..2) of the state buffer holding the current state
    int32_t diverged;    // nonzero once a non-finite residual or rho <= 0 was seen
    int32_t max_pseudo;  // iteration limit of the current real step
    int32_t pad;
    double tol;          // <= 0: run exactly max_pseudo iterations
    double norms[4];     // residual norms of the last iteration (rho, rho u, rho v, p)
};

// Real-time coefficients of the current real step (Table 1), in device memory so that a captured
// pseudo-iteration graph stays valid from one step to the next.
struct StepParams {
    double inv_dt;          // 1/dt
    double b0, b1, b2;      // BDF coefficients: dQ/dt = (b0 Q^0 + b1 Q^n + b2 Q^{n-1}) / dt
};

// Number of doubles per workgroup in the residual partials: four field sums (or maxima) and the
// count of cells whose updated density is not finite and positive.
constexpr int kPartialWidth = 5;

// Buffer rotation: stage s of a pseudo-iteration whose stage-0 state is in buffer `cur` reads
// Q^{s-1} from `in` and writes Q^s to `out`; neither is `cur` for s >= 2, and no stage writes the
// buffer it or the stage-0 state reads.  The iteration's result lands in next_cur().
struct StageBuffers {
    int in, out;
};
__host__ __device__ inline StageBuffers stage_buffers(int cur, int s)
{
    StageBuffers b;
    b.in = (s == 1) ? cur : (cur + 1 + ((s - 2) & 1)) % 3;
    b.out = (cur + 1 + ((s - 1) & 1)) % 3;
    return b;
}
__host__ __device__ inline int next_cur(int cur, int smax) { return (cur + 1 + ((smax - 1) & 1)) % 3; }

// Everything a stage kernel needs about one tank.
struct TankDev {
    int32_t nx, ny;
    int32_t per_x, per_y;     // periodic in x / y
    double dx, dy;
    double inv_dx, inv_dy;
    double half_dx, half_dy;  // dx/2, dy/2 (face offsets)
    double gx, gy;
    double beta, inv_beta;
    double cfl;
    size_t plane;             // nx*ny
    double *state[3];         // 4 planes each
    double *level_n;          // 3 planes
    double *level_nm1;        // 3 planes (BDF2) or nullptr
    const uint8_t *flags;
    double *partials;         // [n_blocks][kPartialWidth]
    Status *status;
    const StepParams *step;
    int32_t n_fluid;
};

// Scheme settings common to all tanks of a grid.
struct Scheme {
    int32_t smax;
    double alpha[8];
    double k;        // limiter parameter
    int32_t slip;    // free-slip wall ghosts
    int32_t norm_max;
    int32_t bdf2;    // the grid keeps a level n-1 history
};

// Launch wrappers.  All return hipError_t cast to int.  A stage launch with tile (1, 1) runs the
// plain one-thread-per-cell kernel (kernels_f64.hip); tile (-W, L) with W = 1, 2 or 3 runs the
// row-marching kernel (stage_march.hip) on 64-column strips swept in chunks of L rows, compiled
// for W = 3 waves per SIMD (tighter register budget) or 2 otherwise; the supported 2D tiles run
// the tiled kernel (stage_tile.hip).  stage_blocks() is the number of residual partials a stage
// launch writes.
int launch_begin_step(const TankDev &t, const Scheme &sc, double dt, int max_pseudo, double tol,
                      int use_history, void *stream);
int launch_stage(const TankDev &t, const Scheme &sc, int stage, int tile_x, int tile_y,
                 void *stream);
int launch_stage_direct_f64(const TankDev &t, const Scheme &sc, int stage, void *stream);
int launch_stage_tile_f64(const TankDev &t, const Scheme &sc, int stage, int tile_x, int tile_y,
                          void *stream);
int launch_finalize(const TankDev &t, const Scheme &sc, int n_blocks, void *stream);
int launch_stage_march_f64(const TankDev &t, const Scheme &sc, int stage, int chunk, int waves,
                           void *stream);
int march_units(const TankDev &t, int chunk);
int stage_blocks(const TankDev &t, int tile_x, int tile_y);
int direct_blocks(const TankDev &t);
int tile_count(const TankDev &t, int tile_x, int tile_y);
bool tile_supported(int tile_x, int tile_y);

// Tile used when the options leave the choice open.
constexpr int kDefaultTileX = 32, kDefaultTileY = 8;

}  // namespace vdac
