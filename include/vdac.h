/*
 * vdac.h -- C ABI of the MI355X (gfx950) solver for the inviscid variable-density
 * artificial-compressibility equations with dual time stepping, after Leakey, Glenis & Hewett,
 * "Riemann solvers and pressure gradients in Godunov-type schemes for variable density
 * incompressible flows" (arXiv:2108.08769).
 *
 * One call of step_dual_time advances every tank of a grid by one real-time step (Algorithm 1,
 * Sec. 2.2.2): level n <- current state, then explicit Runge-Kutta pseudo-time iterations
 * (eqs. 23-24) until every residual norm is below the tolerance.  Each Runge-Kutta stage runs,
 * on the GPU and per cell: limited MUSCL gradients of rho, u, v (Sec. 2.3.1), the new pressure
 * gradient from the rearranged momentum equation (Sec. 2.3.2), face states, the
 * Osher-Dumbser-Toro flux (Sec. 2.4.3) rotated to each face (Sec. 2.4), the flux divergence,
 * the real-time and body-force sources frozen at stage 0 and the point-implicit update
 * (coefficient of eq. 27), with the local pseudo-time step of Sec. 2.2.3.  Walls are ghost cells
 * with zero-gradient rho and p, mirrored velocity and reversed gravity (Sec. 2.5).
 *
 * Conventions shared by every entry point
 *   - Host state arrays are float64 structure-of-arrays planes [4][ny][nx], x fastest, holding
 *     (rho, rho*u, rho*v, p) -- the pressure itself, not p/beta.
 *   - Every function returns a VDAC_* status and never aborts or throws across the ABI; on
 *     failure last_error() describes the cause (thread-local, valid until the next call).
 *   - A grid is not thread-safe; distinct grids are independent.  All device work is issued on
 *     the stream given to create_grid.  Host buffers are owned by the caller and copied
 *     synchronously: the library keeps no pointer to them.
 */
#ifndef VDAC_H
#define VDAC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vdac_grid vdac_grid; /* opaque, owned by the library */

enum {
    VDAC_OK = 0,
    VDAC_E_INVALID = 1,  /* bad argument, shape or option */
    VDAC_E_NOMEM = 2,    /* device allocation failed or workspace too small */
    VDAC_E_DEVICE = 3,   /* a HIP call failed */
    VDAC_E_DIVERGED = 4  /* non-finite residual or rho <= 0 during stepping */
};

/* Boundary kind per side, in the order x-, x+, y-, y+ (periodic sides must come in pairs):
 * walls (Sec. 2.5), periodic, or zero gradient of every variable (transmissive; its ghosts
 * reflect the interior without changing any sign and keep gravity). */
enum { VDAC_BC_WALL = 0, VDAC_BC_PERIODIC = 1, VDAC_BC_TRANSMISSIVE = 2 };

/* x-split Riemann solver (Sec. 2.4): Osher-Dumbser-Toro (2.4.3), Roe at the Roe average
 * (2.4.2), or the exact solver of Sec. 2.4.1 (Bassi et al.). */
enum { VDAC_FLUX_OSHER = 0, VDAC_FLUX_ROE = 1, VDAC_FLUX_BASSI = 2 };

/* Pressure gradient of the reconstruction (Sec. 2.3.2): the new method (rearranged momentum
 * equation), the k-limiter applied to p, or the split limiter (hydrostatic part removed before
 * limiting, restored after). */
enum { VDAC_PGRAD_NEW = 0, VDAC_PGRAD_LIMITER = 1, VDAC_PGRAD_SPLIT = 2 };

/* Precision of the stage: FP64 throughout, or mixed (the state stored as FP32 deviations from an
 * FP64 level n; reconstruction, Riemann fluxes and the local pseudo-time step in FP32; sources,
 * flux divergence, update and residual norm in FP64).  The state crosses the boundary in FP64
 * either way. */
enum { VDAC_FP64 = 0, VDAC_FP32_MIXED = 1 };
enum { VDAC_NORM_RMS = 0, VDAC_NORM_MAX = 1 };

/* One tank: a rectangle of nx * ny cells of size (lx/nx) x (ly/ny), at most 2^29 cells. */
typedef struct {
    int32_t nx, ny;
    double lx, ly;
    double gx, gy;        /* gravity */
    double beta;          /* artificial compressibility coefficient (Sec. 2.1.1), > 0 */
    int32_t bc[4];        /* VDAC_BC_* for x-, x+, y-, y+ */
    const uint8_t *solid; /* nullable host mask [ny][nx], nonzero = solid cell; copied at
                             create_grid.  Each fluid-solid face acts as a wall.  Solid cells keep
                             the state given to set_state. */
} vdac_tank;

typedef struct {
    int32_t precision;   /* VDAC_FP64 or VDAC_FP32_MIXED */
    int32_t rk_stages;   /* s_max, 1..8 */
    double rk_alpha[8];  /* alpha_1..alpha_smax; alpha_smax must be 1 (Sec. 2.2.2) */
    double cfl_tau;      /* pseudo-time Courant number (Sec. 2.2.3), > 0 */
    double limiter_k;    /* k-limiter: 1 minmod, 2 superbee, in [1, 2] (Sec. 2.3.1) */
    int32_t local_dtau;  /* 1: local pseudo-time steps (Sec. 2.2.3); 0: one global step per
                            tank and pseudo-iteration, the minimum local step */
    int32_t bdf_order;   /* 1 backward Euler, 2 BDF2, 3 BDF3 (Table 1); the first step after
                            set_state is backward Euler, the second at most BDF2 */
    int32_t norm;        /* VDAC_NORM_RMS or VDAC_NORM_MAX over fluid cells */
    int32_t wall_slip;   /* 0: no-slip wall ghosts as in Sec. 2.5; 1: free-slip ghosts */
    int32_t tile_x, tile_y; /* stage-kernel shape: 0 x 0 automatic; 1 x 1 one thread per cell;
                               -W x L row marching over 64-column strips in chunks of L rows,
                               W = 3 for a 3-waves-per-SIMD register budget, 1 or 2 otherwise;
                               32 x 8, 16 x 16 or 64 x 4 two-dimensional LDS tiles (256
                               threads), 3208 x 2, 1616 x 2 for the 32 x 8 and 16 x 16 tiles
                               with 512 threads, and 1608 x 2 for a 16 x 8 tile with 320 threads;
                               tiles take one tank, FP64 or mixed; one thread per cell is FP64
                               with the default scheme only */
    int32_t graph_iters; /* pseudo-iterations captured per HIP graph and replayed on the stream:
                            0 automatic, K > 0 exactly K, -1 launch kernels one by one */
    int32_t flux;        /* VDAC_FLUX_* */
    int32_t pgrad;       /* VDAC_PGRAD_* */
    double p_limiter_k;  /* k of the limiter on p for VDAC_PGRAD_LIMITER / _SPLIT, in [1, 2] */
    int32_t persistent;  /* row-marching kernel: 0 one wave per work unit of the stage launch;
                            1 one persistent launch per stage, only as many workgroups as the
                            chip holds at once, each wave looping over its share of the units
                            (same results bit for bit); ignored by the other kernels */
} vdac_options;
/* Options other than the defaults of flux, pgrad and local_dtau, BDF3 and zero-gradient sides
 * run on the row-marching and tiled stage kernels, not on the one-thread-per-cell kernel (tile
 * 1 x 1); the split limiter is not available with zero-gradient sides. */

/* Fills o with the defaults: FP64, 3 stages alpha = (1/3, 1/2, 1), CFL_tau 0.48, minmod,
 * local dtau, backward Euler, RMS norm, no-slip walls, automatic tiles, automatic graphs, Osher
 * flux, new pressure gradient, one wave per work unit (not persistent). */
void vdac_default_options(vdac_options *o);

/* Device bytes create_grid needs for these tanks and options (0 on invalid arguments). */
size_t workspace_bytes(const vdac_tank *tanks, int32_t n_tanks, const vdac_options *o);

/* Builds a grid of n_tanks independent tanks: the problem statement the paper's tests give (the
 * domain and its cells, gravity, beta, the walls of Sec. 2.5, the scheme of Sec. 2.2-2.4), one
 * tank per problem.  o may be NULL (defaults).  device_workspace, if
 * not NULL, is a device buffer of at least ws_bytes >= workspace_bytes(...) bytes that the
 * library borrows until destroy_grid (the caller keeps it alive); if NULL the library allocates
 * and frees its own.  hip_stream is a hipStream_t (NULL = the null stream).  The initial state
 * of every tank is rho = 1, zero velocity and pressure until set_state is called.
 * In a grid of more than one tank on the row-marching kernel, the library may store a tank
 * reflected about its diagonal (x and y exchanged) when that leaves fewer SIMD lanes idle; the
 * scheme is the same under the reflection, and every call of this interface (set_state,
 * get_state, residual_norm, realtime_dt) takes and returns the caller's orientation. */
int create_grid(const vdac_tank *tanks, int32_t n_tanks, const vdac_options *o,
                void *device_workspace, size_t ws_bytes, void *hip_stream, vdac_grid **out);

/* Sets the state of one tank from a host array q [4][ny][nx] (rho, rho*u, rho*v, p).  Also
 * sets level n to q and discards this tank's earlier real-time levels, so its next step uses
 * backward Euler (Sec. 2.2.2); the other tanks of the grid keep theirs.  rho must be finite and
 * > 0 in every fluid cell, else VDAC_E_INVALID. */
int set_state(vdac_grid *g, int32_t tank, const double *q);

/* One real-time step of size dt > 0 for every tank (Algorithm 1); dt = +infinity switches the
 * real-time term off (pseudo-time only, as in the Riemann problems of Sec. 3.1).
 * Pseudo-iterations stop per tank once every residual norm is below tol; tol <= 0 runs exactly
 * max_pseudo iterations.
 * pseudo_done (nullable, [n_tanks]) receives the iterations each tank ran.  Returns
 * VDAC_E_DIVERGED if any tank produced a non-finite residual or rho <= 0 (that tank stops; its
 * state is the one after the failing iteration). */
int step_dual_time(vdac_grid *g, double dt, int32_t max_pseudo, double tol,
                   int32_t *pseudo_done);

/* Residual norms (rho, rho*u, rho*v, p) of the last pseudo-iteration of one tank: the norm of
 * the last Runge-Kutta stage's bracket of eq. 24 (the pseudo-time derivative dQ/dtau that the
 * convergence test of Algorithm 1 measures), the p row as beta times the p/beta row (= dp/dtau);
 * RMS or maximum over the fluid cells (options.norm). */
int residual_norm(const vdac_grid *g, int32_t tank, double out[4]);

/* Copies one tank's state to the host array q [4][ny][nx]: the conserved variables of Sec. 2.1.2
 * (rho, rho*u, rho*v) and the pressure p itself (not p/beta). */
int get_state(const vdac_grid *g, int32_t tank, double *q);

/* Real-time history of one tank, for an exact restart of a BDF2 or BDF3 run (Table 1: a step of
 * order k needs the states at the k - 1 earlier real times besides the current one).
 * get_history writes to the host array levels [2][3][ny][nx] the states (rho, rho*u, rho*v) at
 * the starts of the last and of the one but last completed real steps (the pressure has no
 * real-time term), and to *count how many of them the next step of this grid would use:
 * min(real steps completed since set_state, bdf_order - 1); levels[1] is written only when
 * *count is 2.  set_history, called after set_state on a grid with the same options and tank,
 * restores them, so that the next step_dual_time continues the run bit for bit: count 0..2 and at
 * most bdf_order - 1, else VDAC_E_INVALID; levels[1] is read only when count is 2.  Host arrays are
 * owned by the caller and copied synchronously.  A later set_state discards the restored levels. */
int get_history(const vdac_grid *g, int32_t tank, double *levels, int32_t *count);
int set_history(vdac_grid *g, int32_t tank, const double *levels, int32_t count);

/* Global real-time step of one tank from its current state (Sec. 2.2.4):
 * *dt = min over fluid cells of cfl_t dx dy / (|u| dy + |v| dx), +infinity at rest. */
int realtime_dt(const vdac_grid *g, int32_t tank, double cfl_t, double *dt);

/* For callers that cannot allocate device memory or synchronise with the host: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  The same global
 * real-time steps as realtime_dt, for tanks first_tank .. first_tank + n_tanks - 1, written to
 * the caller's device array dt_device[n_tanks] (FP64, in the caller's orientation; +infinity
 * for a tank at rest) by kernels queued on the grid's stream; the call returns without waiting
 * for them.  It allocates nothing: the per-workgroup minima go to a fixed device array of the
 * library, 8192 doubles (64 KiB) on each GPU it runs on, held until the process ends.  A tank
 * takes min(256, ceil(nx ny / 256)) of them (the range: the largest tank's count times
 * n_tanks); a range that needs more than 8192 is rejected with VDAC_E_INVALID (split it).
 * Every minimum is written before it is read, so nothing needs clearing between calls.  All
 * calls on one GPU share that array: calls that overlap in time on one GPU (other streams,
 * other threads, other grids) race and must be ordered by the caller.  The current device must
 * be the one create_grid ran on (else VDAC_E_INVALID). */
int realtime_dt_device(const vdac_grid *g, int32_t first_tank, int32_t n_tanks, double cfl_t,
                       double *dt_device);

/* Measurement: while enabled, step_dual_time brackets every replayed graph of pseudo-iterations
 * (or, with graph_iters = -1, the s_max back-to-back Runge-Kutta stage launches of every
 * pseudo-iteration) with a pair of HIP events on the grid's stream and accumulates their elapsed
 * times; enabling resets the totals.  The events add markers between launches and nothing
 * else, so a timed region may keep them on.  A graph's time includes its one finalize launch
 * and, with a tolerance, the kernels of tanks that have stopped (they return at once). */
int stage_timing(vdac_grid *g, int32_t enable);

/* Totals since stage timing was enabled: summed stage-kernel milliseconds, number of stage
 * launches (a launch of the row-marching kernel covers every tank of the grid), and fluid
 * cell-stages those launches updated (pseudo-iterations in which every tank had already stopped
 * count neither time nor cells).  Any output pointer may be NULL. */
int stage_timing_read(const vdac_grid *g, double *kernel_ms, int64_t *launches,
                      double *cell_stages);

/* Autotuner of the stage-kernel shape.  For the tanks and options given (o's tile fields are
 * ignored on input), builds a scratch grid per candidate shape -- row marching with chunks of
 * 1..64 rows (and longer chunks that fill the chip's wave slots a whole number of times) under a
 * 2- and a 3-waves-per-SIMD register budget, and for a single tank also the 2D LDS tiles -- runs
 * one untimed and one timed real step of `iters` pseudo-iterations (1..1000) from the initial
 * rest state, then times the leaders (up to three, within 5% of the fastest) again in three
 * interleaved rounds of three steps each and writes the shape with the least of those
 * stage-kernel times into o->tile_x, o->tile_y.  The result is cached for the life of the
 * process, keyed by precision, scheme and tank shapes, so later calls with the same key return
 * at once.  Allocates and frees device memory and runs on hip_stream; the kernel time does not
 * depend on the state. */
int autotune_tile(const vdac_tank *tanks, int32_t n_tanks, vdac_options *o, void *hip_stream,
                  int32_t iters);

/* Frees the grid (and the device memory it allocated).  NULL is ignored. */
void destroy_grid(vdac_grid *g);

/* Message of the last failing call on this thread ("" if none). */
const char *last_error(void);

#ifdef __cplusplus
}
#endif
#endif
