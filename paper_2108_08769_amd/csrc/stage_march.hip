// stage_march.hip -- the Runge-Kutta stage kernel for gfx950 in its row-marching form.
//
// Each 64-lane wave owns a strip of 64 consecutive columns (lanes 2..61 produce output, lanes
// 0-1 and 62-63 are the halo the reconstruction and the x-faces need) and sweeps a chunk of rows
// upward.  The three rows the limited slopes need stay in registers, x-neighbours come from
// cross-lane shuffles, and the loads of the next row are issued a full row ahead of their use.
// No LDS, no workgroup barrier.  Per row r the wave
//   1. reconstructs row r once per lane: limited slopes (Sec. 2.3.1), the stage-0 sources from
//      Q^0 and level n, the new pressure gradient (Sec. 2.3.2), and the states at the four faces;
//   2. evaluates the x-faces of row r with the Osher-Dumbser-Toro flux (Sec. 2.4.3): lane x takes
//      the face on its right, its right neighbour receives the result for its left face; a lane
//      whose left face is a wall evaluates that face itself from its own ghost (Sec. 2.5);
//   3. evaluates the y-face between rows r-1 and r (rotated, Sec. 2.4); a face with a wall above
//      row r is evaluated with row r's ghost and carried to the next row;
//   4. completes row r-1: flux divergence, frozen sources, point-implicit update (eq. RK2), and
//      on the last stage the residual partial.
// Each face is evaluated once.  Periodic sides wrap indices; cells outside a non-periodic side
// read as non-fluid.
#include <hip/hip_runtime.h>

#include "stage_common.h"

namespace vdac {

namespace {

constexpr int kLanes = 64;
constexpr int kOut = 60;            // output columns per strip (lanes 2..61)
constexpr int kWavesPerBlock = 4;
constexpr int kMinWavesPerSimd = 2;  // register budget: at most 256 VGPRs per lane

__device__ __forceinline__ bool locate_axis(int g, int n, int periodic, int &out)
{
    if (g < 0 || g >= n) {
        if (!periodic) return false;
        while (g < 0) g += n;
        while (g >= n) g -= n;
    }
    out = g;
    return true;
}

__device__ __forceinline__ double from_left(double v) { return __shfl_up(v, 1, kLanes); }
__device__ __forceinline__ double from_right(double v) { return __shfl_down(v, 1, kLanes); }

__device__ __forceinline__ Prim<double> prim_from_left(const Prim<double> &w)
{
    return {from_left(w.r), from_left(w.u), from_left(w.v), from_left(w.p)};
}
__device__ __forceinline__ Prim<double> prim_from_right(const Prim<double> &w)
{
    return {from_right(w.r), from_right(w.u), from_right(w.v), from_right(w.p)};
}

// Loads of one row, issued one step ahead of their use: the stage input is fetched two rows
// ahead (it is the upper neighbour of the next row), the stage-0 state, level n (and level
// n-1) and the flags one row ahead.
struct InputLoad {
    double q[4];     // stage input Q^{s-1}: rho, rho u, rho v, p
};
struct SourceLoad {
    double z[4];     // stage-0 state Q^0: rho, rho u, rho v, p
    double n[3];     // level n
    double m[3];     // level n-1 (BDF2 only)
    uint8_t f;       // cell flags (FLAG_SOLID if outside the tank)
};

__device__ __forceinline__ void load_input(const TankDev &t, const double *qprev, bool have_col,
                                           int gi, int r, InputLoad &L)
{
    int gj;
    if (have_col && locate_axis(r, t.ny, t.per_y, gj)) {
        const size_t c = (size_t)gj * t.nx + gi;
#pragma unroll
        for (int k = 0; k < 4; ++k) L.q[k] = qprev[k * t.plane + c];
    } else {
        L.q[0] = 1.0;
        L.q[1] = L.q[2] = L.q[3] = 0.0;
    }
}

template <bool BDF2>
__device__ __forceinline__ void load_sources(const TankDev &t, const double *q0, bool have_col,
                                             int gi, int r, SourceLoad &L)
{
    int gj;
    L.f = FLAG_SOLID;
    if (have_col && locate_axis(r, t.ny, t.per_y, gj)) {
        const size_t plane = t.plane;
        const size_t c = (size_t)gj * t.nx + gi;
        L.f = t.flags[c];
#pragma unroll
        for (int k = 0; k < 4; ++k) L.z[k] = q0[k * plane + c];
#pragma unroll
        for (int k = 0; k < 3; ++k) L.n[k] = t.level_n[k * plane + c];
        if (BDF2) {
#pragma unroll
            for (int k = 0; k < 3; ++k) L.m[k] = t.level_nm1[k * plane + c];
        }
    } else {
        L.z[0] = 1.0;
        L.z[1] = L.z[2] = L.z[3] = 0.0;
        L.n[0] = 1.0;
        L.n[1] = L.n[2] = 0.0;
        if (BDF2) {
            L.m[0] = 1.0;
            L.m[1] = L.m[2] = 0.0;
        }
    }
}

__device__ __forceinline__ Prim<double> to_prim(const InputLoad &L)
{
    return {L.q[0], L.q[1] / L.q[0], L.q[2] / L.q[0], L.q[3]};
}

template <bool NORM_MAX, bool BDF2>
__global__ void __launch_bounds__(kLanes *kWavesPerBlock, kMinWavesPerSimd)
    stage_march_f64(TankDev t, Scheme sc, int stage, int chunk, int n_strips, int n_units)
{
    const Status *st = t.status;
    if (st->done) return;

    // XCD-aware order: block b runs on XCD b % 8; each XCD gets a contiguous run of units, and
    // consecutive units are neighbouring strips of the same row chunk.
    const int n_blocks = (n_units + kWavesPerBlock - 1) / kWavesPerBlock;
    const int per = (n_blocks + 7) >> 3;
    const int blk = (int)(blockIdx.x & 7u) * per + (int)(blockIdx.x >> 3);
    const int wave = threadIdx.x / kLanes, lane = threadIdx.x % kLanes;
    const int unit = blk * kWavesPerBlock + wave;
    if (blk >= n_blocks || unit >= n_units) return;  // uniform per wave

    const int strip = unit % n_strips, ch = unit / n_strips;
    const int col = strip * kOut - 2 + lane;  // this lane's column (may lie outside the tank)
    int gi = 0;
    const bool have_col = locate_axis(col, t.nx, t.per_x, gi);
    const bool out_lane = lane >= 2 && lane < 2 + kOut && col >= 0 && col < t.nx;
    const int j0 = ch * chunk;
    const int j1 = min(j0 + chunk, t.ny);

    const int cur = st->cur;
    const StageBuffers bufs = stage_buffers(cur, stage);
    const double *qprev = t.state[bufs.in];
    const double *q0 = t.state[cur];
    double *qout = t.state[bufs.out];
    const StepParams sp = *t.step;
    const bool slip = sc.slip != 0;
    const double kl = sc.k;
    const double alpha = sc.alpha[stage - 1];
    const bool last = (stage == sc.smax);
    const size_t plane = t.plane;

    // window of primitives: rows r-1 (lo), r (mid), r+1 (hi)
    InputLoad in_ld;
    SourceLoad src_ld;
    load_input(t, qprev, have_col, gi, j0 - 2, in_ld);
    Prim<double> lo = to_prim(in_ld);
    load_input(t, qprev, have_col, gi, j0 - 1, in_ld);
    Prim<double> mid = to_prim(in_ld);
    load_input(t, qprev, have_col, gi, j0, in_ld);
    Prim<double> hi = to_prim(in_ld);
    load_input(t, qprev, have_col, gi, j0 + 1, in_ld);          // row r+2
    load_sources<BDF2>(t, q0, have_col, gi, j0 - 1, src_ld);    // row r

    // carries from row r-1
    Prim<double> top_state = {1.0, 0.0, 0.0, 0.0};  // its state at the face above it
    double g_wall[4] = {0.0, 0.0, 0.0, 0.0};        // flux above it when that face is a wall
    double rpart[4] = {0.0, 0.0, 0.0, 0.0};         // its residual without the flux above it
    double base[4] = {0.0, 0.0, 0.0, 0.0};          // its stage-0 state
    double fac = 0.0, adt = 0.0;                    // its update factors
    bool fluid_lo = false;
    double part[kPartialWidth] = {0.0, 0.0, 0.0, 0.0, 0.0};

    for (int r = j0 - 1; r <= j1; ++r) {
        // sources of row r (loaded one step ahead), then the next loads
        const uint8_t f = src_ld.f;
        const bool fluid = !(f & FLAG_SOLID);
        double z[4], d[3];
#pragma unroll
        for (int k = 0; k < 4; ++k) z[k] = src_ld.z[k];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            double num = sp.b0 * src_ld.z[k] + sp.b1 * src_ld.n[k];
            if (BDF2) num += sp.b2 * src_ld.m[k];
            d[k] = num * sp.inv_dt;
        }
        const Prim<double> next_hi = to_prim(in_ld);
        load_input(t, qprev, have_col, gi, r + 3, in_ld);
        load_sources<BDF2>(t, q0, have_col, gi, r + 1, src_ld);

        // ---- reconstruction of row r ------------------------------------------------------
        const Prim<double> wl = prim_from_left(mid);
        const Prim<double> wr = prim_from_right(mid);
        CellRec rec;
        rec.w = mid;
        rec.d_r = d[0];
        rec.d_ru = d[1];
        rec.d_rv = d[2];
        rec.rho0 = z[0];
        Prim<double> sxl = mid, sxr = mid, syb = mid, syt = mid;
        if (fluid) {
            const Prim<double> xm = (f & FLAG_WALL_XM) ? mirror(mid, 0, slip) : wl;
            const Prim<double> xp = (f & FLAG_WALL_XP) ? mirror(mid, 0, slip) : wr;
            const Prim<double> ym = (f & FLAG_WALL_YM) ? mirror(mid, 1, slip) : lo;
            const Prim<double> yp = (f & FLAG_WALL_YP) ? mirror(mid, 1, slip) : hi;
            rec.gx = slopes(xm, mid, xp, t.inv_dx, kl);
            rec.gy = slopes(ym, mid, yp, t.inv_dy, kl);
            const double px = gradp_x(mid, rec.gx, rec.gy, rec.d_ru, rec.rho0 * t.gx);
            const double py = gradp_y(mid, rec.gx, rec.gy, rec.d_rv, rec.rho0 * t.gy);
            sxl = {mid.r - rec.gx.r * t.half_dx, mid.u - rec.gx.u * t.half_dx,
                   mid.v - rec.gx.v * t.half_dx, mid.p - px * t.half_dx};
            sxr = {mid.r + rec.gx.r * t.half_dx, mid.u + rec.gx.u * t.half_dx,
                   mid.v + rec.gx.v * t.half_dx, mid.p + px * t.half_dx};
            syb = {mid.r - rec.gy.r * t.half_dy, mid.u - rec.gy.u * t.half_dy,
                   mid.v - rec.gy.v * t.half_dy, mid.p - py * t.half_dy};
            syt = {mid.r + rec.gy.r * t.half_dy, mid.u + rec.gy.u * t.half_dy,
                   mid.v + rec.gy.v * t.half_dy, mid.p + py * t.half_dy};
        }

        // ---- y-face between rows r-1 and r ------------------------------------------------
        double gb[4] = {0.0, 0.0, 0.0, 0.0};
        if (r >= j0) {
            if (fluid) {
                const Prim<double> L = fluid_lo ? top_state : ghost_state(t, rec, 1, -1, slip);
                osher_y(L, syb, t.beta, t.inv_beta, gb);
            } else if (fluid_lo) {
#pragma unroll
                for (int k = 0; k < 4; ++k) gb[k] = g_wall[k];
            }
        }

        // ---- update of row r-1 ------------------------------------------------------------
        if (r - 1 >= j0 && out_lane && fluid_lo) {
            int gj;
            locate_axis(r - 1, t.ny, t.per_y, gj);
            const size_t c = (size_t)gj * t.nx + gi;
            double R4[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) R4[k] = rpart[k] - gb[k] * t.inv_dy;
            const double rn = base[0] + fac * R4[0];
            qout[c] = rn;
            qout[plane + c] = base[1] + fac * R4[1];
            qout[2 * plane + c] = base[2] + fac * R4[2];
            qout[3 * plane + c] = base[3] + t.beta * (adt * R4[3]);
            if (last) {
                const double rp = t.beta * R4[3];
                if (NORM_MAX) {
                    part[0] = combine<true>(part[0], fabs(R4[0]));
                    part[1] = combine<true>(part[1], fabs(R4[1]));
                    part[2] = combine<true>(part[2], fabs(R4[2]));
                    part[3] = combine<true>(part[3], fabs(rp));
                } else {
                    part[0] += R4[0] * R4[0];
                    part[1] += R4[1] * R4[1];
                    part[2] += R4[2] * R4[2];
                    part[3] += rp * rp;
                }
                part[4] += (rn > 0.0 && rn < INFINITY) ? 0.0 : 1.0;
            }
        }

        // ---- x-faces of row r and its partial residual -----------------------------------
        double rp4[4] = {0.0, 0.0, 0.0, 0.0};
        if (r >= j0 && r < j1) {
            const Prim<double> partner = prim_from_right(sxl);  // right neighbour's left state
            double fr[4] = {0.0, 0.0, 0.0, 0.0};
            if (fluid) {
                const Prim<double> R = (f & FLAG_WALL_XP) ? ghost_state(t, rec, 0, +1, slip) : partner;
                osher_x(sxr, R, t.beta, t.inv_beta, fr);
            }
            double fl[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) fl[k] = from_left(fr[k]);
            if (fluid && (f & FLAG_WALL_XM)) {
                const Prim<double> Lg = ghost_state(t, rec, 0, -1, slip);
                osher_x(Lg, sxl, t.beta, t.inv_beta, fl);
            }
            // residual of row r without its upper y-face: -(x-divergence) + lower flux / dy
            // - real-time term + body force
#pragma unroll
            for (int k = 0; k < 4; ++k) rp4[k] = -((fr[k] - fl[k]) * t.inv_dx) + gb[k] * t.inv_dy;
            rp4[0] += -d[0];
            rp4[1] += -d[1] + z[0] * t.gx;
            rp4[2] += -d[2] + z[0] * t.gy;
        }
        // a wall above row r: evaluate that face now, from row r's ghost
        double gw[4] = {0.0, 0.0, 0.0, 0.0};
        if (fluid && (f & FLAG_WALL_YP) && r < j1) {
            const Prim<double> U = ghost_state(t, rec, 1, +1, slip);
            osher_y(syt, U, t.beta, t.inv_beta, gw);
        }

        // ---- carry row r to the next step -------------------------------------------------
        if (fluid && r >= j0 && r < j1) {
            const double dtau = local_dtau(t, t.cfl, z[0], z[1], z[2]);
            adt = alpha * dtau;
            fac = adt / (1.0 + sp.b0 * adt * sp.inv_dt);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            rpart[k] = rp4[k];
            base[k] = z[k];
            g_wall[k] = gw[k];
        }
        top_state = syt;
        fluid_lo = fluid;
        lo = mid;
        mid = hi;
        hi = next_hi;
    }

    if (last) {
        // wave reduction (fixed order) and one partial per strip chunk
#pragma unroll
        for (int k = 0; k < kPartialWidth; ++k) {
            double x = part[k];
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) {
                const double y = __shfl_xor(x, off, kLanes);
                x = (NORM_MAX && k < 4) ? combine<true>(x, y) : x + y;
            }
            if (lane == 0) t.partials[(size_t)unit * kPartialWidth + k] = x;
        }
    }
}

}  // namespace

int march_units(const TankDev &t, int chunk)
{
    const int n_strips = (t.nx + kOut - 1) / kOut;
    const int n_chunks = (t.ny + chunk - 1) / chunk;
    return n_strips * n_chunks;
}

int launch_stage_march_f64(const TankDev &t, const Scheme &sc, int stage, int chunk, void *stream)
{
    const int n_strips = (t.nx + kOut - 1) / kOut;
    const int n_units = march_units(t, chunk);
    const int n_blocks = (n_units + kWavesPerBlock - 1) / kWavesPerBlock;
    const int grid = ((n_blocks + 7) / 8) * 8;
    const dim3 g(grid), b(kLanes * kWavesPerBlock);
    hipStream_t s = (hipStream_t)stream;
    const bool bdf2 = t.level_nm1 != nullptr;
    if (sc.norm_max) {
        if (bdf2) hipLaunchKernelGGL((stage_march_f64<true, true>), g, b, 0, s, t, sc, stage, chunk, n_strips, n_units);
        else hipLaunchKernelGGL((stage_march_f64<true, false>), g, b, 0, s, t, sc, stage, chunk, n_strips, n_units);
    } else {
        if (bdf2) hipLaunchKernelGGL((stage_march_f64<false, true>), g, b, 0, s, t, sc, stage, chunk, n_strips, n_units);
        else hipLaunchKernelGGL((stage_march_f64<false, false>), g, b, 0, s, t, sc, stage, chunk, n_strips, n_units);
    }
    return (int)hipGetLastError();
}

}  // namespace vdac
