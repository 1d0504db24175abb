// vdac_internal.h -- structures shared by the host driver and the HIP kernels of libvdac.
//
// Device memory of one tank (all planes x-fastest, 256-byte aligned):
//   state[3]   three rotating state buffers, 4 planes each.  FP64 form: rho, rho*u, rho*v, p in
//              FP64.  Mixed form: FP32 deviations rho - rho^n, rho*u - (rho*u)^n,
//              rho*v - (rho*v)^n, p - p^n from real-time level n.  The current state, the
//              stage-0 state of the running pseudo-iteration and the stage outputs rotate among
//              them (see stage_buffers below) without copies; begin_step moves the state into
//              buffer 0 once per real step.
//   level_n    real-time level n in FP64: 3 planes (rho, rho*u, rho*v) in the FP64 form, 4 (and
//              p) in the mixed form; level_nm1 (BDF2, BDF3) and level_nm2 (BDF3) 3 planes each.
// A tank of a batch may be stored reflected about its diagonal (x and y exchanged); the host
// reflects states and norms at the C ABI, and the kernels see an ordinary tank.
//   flags      one byte per cell: which faces are walls (domain wall or solid neighbour) and
//              whether the cell itself is solid.
//   partials   per-work-unit residual partial sums of the last Runge-Kutta stage.
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
    double dtau_global;  // global pseudo-time step: the minimum local step of the current state
};

// Per-launch arguments of a stage kernel that change from one pseudo-iteration m to the next.
//   cur_off   the iteration's stage-0 buffer, cur_of_iter(m): every real step starts from buffer 0
//             (begin_step moves the state there), so the buffers follow from m alone and not from
//             the status, which the deferred finalize (below) rewrites while the launch runs
//   fin       stage 1 only: the launch also runs the finalize of iteration m - 1 (extra waves, one
//             per tank, dispatched first); its stage-1 work for a tank that this finalize stops is
//             discarded, as it goes to a buffer that is neither the result nor read again
//   n_fin     row-marching launches: finalize waves in front of the unit table (a multiple of 8
//             workgroups, so that every unit stays on the XCD the unit table assigns it)
struct IterArgs {
    int32_t cur_off;
    int32_t fin;
    int32_t n_fin;
    int32_t n_tanks;
    int32_t persist;    // host side: launch the row-marching kernel persistently
    int32_t stride;     // row-marching kernel: 0 one unit per wave; > 0 a persistent launch, whose
                        // waves take every stride-th entry of the unit table
    int32_t n_entries;  // row-marching kernel: entries in the unit table
};


// Real-time coefficients of one tank's current real step (Table 1), in device memory so that a
// captured pseudo-iteration graph stays valid from one step to the next.  Each tank has its own:
// its BDF order follows the earlier levels it holds, which set_state and set_history change per
// tank.
enum : int32_t {
    HISTORY_RESET = 0,  // begin_step sets the kept earlier levels to the new level n
    HISTORY_SHIFT = 1,  // begin_step shifts the levels: n-2 <- n-1 <- n
    HISTORY_KEEP = 2,   // the earlier levels were restored (set_history): begin_step keeps them
};
struct StepParams {
    double inv_dt;          // 1/dt (0: pseudo-time only)
    double b0, b1, b2, b3;  // BDF coefficients: dQ/dt = (b0 Q^0 + b1 Q^n + b2 Q^{n-1} + b3 Q^{n-2})/dt
    int32_t history;        // HISTORY_*: what begin_step does with levels n-1 and n-2
    int32_t pad;
};

// Number of doubles per work unit in the residual partials: four field sums (or maxima), the
// count of cells whose updated density is not finite and positive, and the minimum local
// pseudo-time step of the updated state (infinity where not computed).
constexpr int kPartialWidth = 6;

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
// Buffer of the state after m pseudo-iterations of a real step (which starts from buffer 0).
__host__ __device__ inline int cur_of_iter(long long m, int smax)
{
    return (int)((m * (1 + ((smax - 1) & 1))) % 3);
}

// Everything a stage kernel needs about one tank.
struct TankDev {
    int32_t nx, ny;
    int32_t per_x, per_y;     // periodic in x / y
    double dx, dy;
    double inv_dx, inv_dy;
    double half_dx, half_dy;  // dx/2, dy/2 (face offsets)
    double flux_dx, flux_dy;  // 1/(2 dx), 1/(2 dy): the flux functions return twice the face flux
    double gx, gy;
    double beta, inv_beta;
    double cfl;
    size_t plane;             // nx*ny
    void *state[3];           // 4 planes each (double, or float in the mixed form)
    double *level_n;          // 3 planes (4 in the mixed form)
    double *level_nm1;        // 3 planes (BDF2, BDF3) or nullptr
    double *level_nm2;        // 3 planes (BDF3) or nullptr
    const uint8_t *flags;
    double *partials;         // [n_partials][kPartialWidth]
    Status *status;
    const StepParams *step;   // this tank's coefficients of the current real step
    int32_t n_fluid;
    int32_t n_partials;       // residual partials one stage launch writes for this tank
    int32_t n_strips;         // row-marching kernel: 64-column strips across the tank
    int32_t chunk;            // row-marching kernel: rows per work unit
    int32_t open;             // zero-gradient sides: bit 0 x-, 1 x+, 2 y-, 3 y+
};

// One wave's work in the row-marching kernel: rows [chunk*c, chunk*(c+1)) of strip s of a tank,
// with local = c * n_strips + s.  tank < 0 marks padding.
struct MarchUnit {
    int32_t tank;
    int32_t local;
};

// Scheme settings common to all tanks of a grid.
struct Scheme {
    int32_t smax;
    double alpha[8];
    double k;        // limiter parameter
    int32_t slip;    // free-slip wall ghosts
    int32_t norm_max;
    int32_t bdf;     // highest BDF order of the grid (1..3): levels n-1 (, n-2) are kept
    int32_t mixed;   // FP32 deviation storage and FP32 reconstruction / flux
    int32_t general; // a non-default option below is set: the general stage kernel runs
    int32_t flux;    // 0 Osher-Dumbser-Toro, 1 Roe, 2 exact (Bassi)
    int32_t pgrad;   // 0 new method, 1 k-limiter on p, 2 split limiter
    double pk;       // k of the limiter on p
    int32_t global_dtau;  // one pseudo-time step for the whole tank (the minimum local step)
};

// Launch wrappers.  All return hipError_t cast to int.
//
// Per-tank launches: tile (1, 1) runs the plain one-thread-per-cell kernel (FP64 and the default
// scheme only, kernels_f64.hip), the supported 2D tiles the LDS-tiled kernel (stage_tile.hip,
// FP64 or mixed, every option).  Grid-wide
// launches: the row-marching kernel (stage_march.hip) runs every work unit of every tank from
// the device unit table in one launch per stage, with `waves_per_block` table entries per
// workgroup and a register budget of `waves_simd` (2 or 3) waves per SIMD; begin_step and
// finalize cover all tanks in one launch each.
// begin_step: each tank's StepParams (in device memory before the launch) give its BDF
// coefficients and what happens to its earlier levels (HISTORY_*).
int launch_begin_step_all(const TankDev *tanks_dev, int n_tanks, size_t max_plane, const Scheme &sc,
                          int max_pseudo, double tol, void *stream);
int launch_finalize_all(const TankDev *tanks_dev, int n_tanks, const Scheme &sc, void *stream);
// The per-tank stage launches: the plain kernel never finalizes (ia.fin must be 0); the tiled
// kernel runs the finalize of its tank in one extra workgroup when ia.fin is set.
int launch_stage_direct_f64(const TankDev &t, const Scheme &sc, int stage, const IterArgs &ia,
                            void *stream);
int launch_stage_tile(const TankDev &t, const Scheme &sc, int stage, int tile_x, int tile_y,
                      const IterArgs &ia, void *stream);
int launch_stage_march(const TankDev *tanks_dev, const MarchUnit *units, int n_entries,
                       int waves_per_block, const Scheme &sc, int stage, const IterArgs &ia,
                       int waves_simd, void *stream);
int launch_stage_march_general(const TankDev *tanks_dev, const MarchUnit *units, int n_entries,
                               int waves_per_block, const Scheme &sc, int stage, const IterArgs &ia,
                               void *stream);
// Minima over the fluid cells of the current states of tanks first .. first + n_tanks - 1 (device
// table), in two launches: blocks_per_tank per-workgroup minima per tank into
// scratch[n_tanks][blocks_per_tank], then each tank's minimum (fixed order) into
// out[k * out_stride].  kind MIN_REALTIME_DT: the global real-time step of Sec. 2.2.4,
// CFL_t dx dy / (|u| dy + |v| dx) with CFL_t = cfl (infinity at rest); kind MIN_PSEUDO_DTAU: the
// smallest local pseudo-time step of Sec. 2.2.3 (the tank's own CFL_tau; cfl unused).
// blocks_per_tank in 1..kMinBlocksMax; every scratch slot is written before it is read.
enum { MIN_REALTIME_DT = 0, MIN_PSEUDO_DTAU = 1 };
constexpr int kMinBlocksMax = 1024;
int launch_tanks_min(const TankDev *tanks_dev, int first, int n_tanks, int mixed, int kind,
                     double cfl, double *scratch, int blocks_per_tank, double *out, int out_stride,
                     void *stream);
// Conversions between the caller's FP64 conserved state [4][ny][nx] (rho, rho u, rho v, p) in
// device memory and the storage: import sets every state buffer (cur = 0 after it) and the
// real-time levels; q null imports the state at rest (rho = 1, rho u = rho v = p = 0).
int launch_import_f64(const TankDev &t, const double *q, void *stream);
int launch_import_mixed(const TankDev &t, const double *q, void *stream);
int launch_export_mixed(const TankDev &t, int cur, double *q, void *stream);
// Plane-stream bandwidth reference (n_in, n_out) in {(1, 0), (1, 1), (11, 4)}; blocks = 0: one
// element per lane.
int launch_stream_probe(int n_in, int n_out, size_t n, int blocks, const double *in, double *out,
                        void *stream);
int march_strips(int nx);
int direct_blocks(const TankDev &t);
int tile_count(const TankDev &t, int tile_x, int tile_y);
bool tile_supported(int tile_x, int tile_y);

// Tile used when the options leave the choice open.
constexpr int kDefaultTileX = 32, kDefaultTileY = 8;

}  // namespace vdac
