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
    double r, m, n, p;   // stage input Q^{s-1}: rho, rho u, rho v, p
};
struct SourceLoad {
    double z0, z1, z2, z3;  // stage-0 state Q^0: rho, rho u, rho v, p
    double n0, n1, n2;      // level n
    double m0, m1, m2;      // level n-1 (BDF2 only)
    uint8_t f;              // cell flags (FLAG_SOLID if outside the tank)
};

__device__ __forceinline__ InputLoad load_input(const TankDev &t, const double *qprev,
                                                bool have_col, int gi, int r)
{
    int gj;
    InputLoad L = {1.0, 0.0, 0.0, 0.0};
    if (have_col && locate_axis(r, t.ny, t.per_y, gj)) {
        const size_t c = (size_t)gj * t.nx + gi;
        L.r = qprev[c];
        L.m = qprev[t.plane + c];
        L.n = qprev[2 * t.plane + c];
        L.p = qprev[3 * t.plane + c];
    }
    return L;
}

template <bool BDF2>
__device__ __forceinline__ SourceLoad load_sources(const TankDev &t, const double *q0,
                                                   bool have_col, int gi, int r)
{
    int gj;
    SourceLoad L = {1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 1.0, 0.0, 0.0, FLAG_SOLID};
    if (have_col && locate_axis(r, t.ny, t.per_y, gj)) {
        const size_t plane = t.plane;
        const size_t c = (size_t)gj * t.nx + gi;
        L.f = t.flags[c];
        L.z0 = q0[c];
        L.z1 = q0[plane + c];
        L.z2 = q0[2 * plane + c];
        L.z3 = q0[3 * plane + c];
        L.n0 = t.level_n[c];
        L.n1 = t.level_n[plane + c];
        L.n2 = t.level_n[2 * plane + c];
        if (BDF2) {
            L.m0 = t.level_nm1[c];
            L.m1 = t.level_nm1[plane + c];
            L.m2 = t.level_nm1[2 * plane + c];
        }
    }
    return L;
}

__device__ __forceinline__ Prim<double> to_prim(const InputLoad &L)
{
    const double ir = rcp_pos(L.r);
    return {L.r, L.m * ir, L.n * ir, L.p};
}

// States of a reconstructed cell at one face: W +- grad W h, with the new pressure gradient.
__device__ __forceinline__ Prim<double> state_at(const Prim<double> &w, const Slope<double> &g,
                                                 double gp, double h)
{
    return {fma(g.r, h, w.r), fma(g.u, h, w.u), fma(g.v, h, w.v), fma(gp, h, w.p)};
}

// WAVES: the register budget as waves per SIMD (2: up to 256 VGPRs per lane, 3: up to 168).
template <bool NORM_MAX, bool BDF2, bool LAST, int WAVES>
__global__ void __launch_bounds__(kLanes *kWavesPerBlock, WAVES)
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
    const size_t plane = t.plane;

    // window of primitives: rows r-1 (lo), r (mid), r+1 (hi); loads for later rows in flight
    Prim<double> lo = to_prim(load_input(t, qprev, have_col, gi, j0 - 2));
    Prim<double> mid = to_prim(load_input(t, qprev, have_col, gi, j0 - 1));
    Prim<double> hi = to_prim(load_input(t, qprev, have_col, gi, j0));
    InputLoad in_ld = load_input(t, qprev, have_col, gi, j0 + 1);           // row r+2
    SourceLoad src_ld = load_sources<BDF2>(t, q0, have_col, gi, j0 - 1);    // row r

    // carries from row r-1:
    //  below      its state at its upper face, or, if that face is a wall, the face's flux
    //  pre/base   its update without the flux above it: non-final stages carry
    //             pre = Q^0 + fac R_partial; the final stage keeps Q^0 and R_partial apart for
    //             the residual norm
    Vec4<double> below = {1.0, 0.0, 0.0, 0.0};
    Vec4<double> pre = zero4<double>();
    Vec4<double> rpart = zero4<double>();
    double fac = 0.0, adt = 0.0;
    bool fluid_lo = false;
    double part0 = 0.0, part1 = 0.0, part2 = 0.0, part3 = 0.0, part4 = 0.0;

    for (int r = j0 - 1; r <= j1; ++r) {
        // sources of row r (loaded one step ahead), then the next loads
        const uint8_t f = src_ld.f;
        const bool fluid = !(f & FLAG_SOLID);
        const Vec4<double> z = {src_ld.z0, src_ld.z1, src_ld.z2, src_ld.z3};
        double num0 = fma(sp.b0, src_ld.z0, sp.b1 * src_ld.n0);
        double num1 = fma(sp.b0, src_ld.z1, sp.b1 * src_ld.n1);
        double num2 = fma(sp.b0, src_ld.z2, sp.b1 * src_ld.n2);
        if (BDF2) {
            num0 = fma(sp.b2, src_ld.m0, num0);
            num1 = fma(sp.b2, src_ld.m1, num1);
            num2 = fma(sp.b2, src_ld.m2, num2);
        }
        const Prim<double> next_hi = to_prim(in_ld);
        in_ld = load_input(t, qprev, have_col, gi, r + 3);
        src_ld = load_sources<BDF2>(t, q0, have_col, gi, r + 1);

        // ---- reconstruction of row r ------------------------------------------------------
        const Prim<double> wl = prim_from_left(mid);
        const Prim<double> wr = prim_from_right(mid);
        CellRec rec;
        rec.w = mid;
        rec.d_r = num0 * sp.inv_dt;
        rec.d_ru = num1 * sp.inv_dt;
        rec.d_rv = num2 * sp.inv_dt;
        rec.rho0 = z.a;
        double px = 0.0, py = 0.0;
        if (fluid) {
            const Prim<double> xm = (f & FLAG_WALL_XM) ? mirror(mid, 0, slip) : wl;
            const Prim<double> xp = (f & FLAG_WALL_XP) ? mirror(mid, 0, slip) : wr;
            const Prim<double> ym = (f & FLAG_WALL_YM) ? mirror(mid, 1, slip) : lo;
            const Prim<double> yp = (f & FLAG_WALL_YP) ? mirror(mid, 1, slip) : hi;
            rec.gx = slopes(xm, mid, xp, t.inv_dx, kl);
            rec.gy = slopes(ym, mid, yp, t.inv_dy, kl);
            px = gradp_x(mid, rec.gx, rec.gy, rec.d_ru, rec.rho0 * t.gx);
            py = gradp_y(mid, rec.gx, rec.gy, rec.d_rv, rec.rho0 * t.gy);
        } else {
            rec.gx = {0.0, 0.0, 0.0};
            rec.gy = {0.0, 0.0, 0.0};
        }

        // ---- y-face between rows r-1 and r ------------------------------------------------
        Vec4<double> gb = zero4<double>();
        if (r >= j0) {
            if (fluid) {
                const Prim<double> L = fluid_lo ? Prim<double>{below.a, below.b, below.c, below.d}
                                                : ghost_state(t, rec, 1, -1, slip);
                gb = osher_y(L, state_at(mid, rec.gy, py, -t.half_dy), t.beta, t.inv_beta);
            } else if (fluid_lo) {
                gb = below;  // evaluated with row r-1's ghost
            }
        }

        // ---- update of row r-1 ------------------------------------------------------------
        if (r - 1 >= j0 && out_lane && fluid_lo) {
            int gj;
            locate_axis(r - 1, t.ny, t.per_y, gj);
            const size_t c = (size_t)gj * t.nx + gi;
            if (LAST) {
                const double R0 = fma(-gb.a, t.inv_dy, rpart.a);
                const double R1 = fma(-gb.b, t.inv_dy, rpart.b);
                const double R2 = fma(-gb.c, t.inv_dy, rpart.c);
                const double R3 = fma(-gb.d, t.inv_dy, rpart.d);
                const double rn = fma(fac, R0, pre.a);
                qout[c] = rn;
                qout[plane + c] = fma(fac, R1, pre.b);
                qout[2 * plane + c] = fma(fac, R2, pre.c);
                qout[3 * plane + c] = fma(t.beta, adt * R3, pre.d);
                const double rp = t.beta * R3;
                if (NORM_MAX) {
                    part0 = combine<true>(part0, fabs(R0));
                    part1 = combine<true>(part1, fabs(R1));
                    part2 = combine<true>(part2, fabs(R2));
                    part3 = combine<true>(part3, fabs(rp));
                } else {
                    part0 = fma(R0, R0, part0);
                    part1 = fma(R1, R1, part1);
                    part2 = fma(R2, R2, part2);
                    part3 = fma(rp, rp, part3);
                }
                part4 += (rn > 0.0 && rn < INFINITY) ? 0.0 : 1.0;
            } else {
                // fac and adt already carry 1/dy here
                qout[c] = fma(-fac, gb.a, pre.a);
                qout[plane + c] = fma(-fac, gb.b, pre.b);
                qout[2 * plane + c] = fma(-fac, gb.c, pre.c);
                qout[3 * plane + c] = fma(-adt, gb.d, pre.d);
            }
        }

        // ---- x-faces of row r and its residual without the upper y-face ------------------
        Vec4<double> rp4 = zero4<double>();
        if (r >= j0 && r < j1) {
            const Prim<double> sxl = state_at(mid, rec.gx, px, -t.half_dx);
            const Prim<double> partner = prim_from_right(sxl);  // right neighbour's left state
            Vec4<double> fr = zero4<double>();
            if (fluid) {
                const Prim<double> R = (f & FLAG_WALL_XP) ? ghost_state(t, rec, 0, +1, slip) : partner;
                fr = osher_x(state_at(mid, rec.gx, px, t.half_dx), R, t.beta, t.inv_beta);
            }
            Vec4<double> fl = {from_left(fr.a), from_left(fr.b), from_left(fr.c), from_left(fr.d)};
            if (fluid && (f & FLAG_WALL_XM))
                fl = osher_x(ghost_state(t, rec, 0, -1, slip), sxl, t.beta, t.inv_beta);
            // -(x-divergence) + lower flux / dy - real-time term + body force
            rp4.a = fma(gb.a, t.inv_dy, -((fr.a - fl.a) * t.inv_dx)) - rec.d_r;
            rp4.b = fma(gb.b, t.inv_dy, -((fr.b - fl.b) * t.inv_dx)) + fma(z.a, t.gx, -rec.d_ru);
            rp4.c = fma(gb.c, t.inv_dy, -((fr.c - fl.c) * t.inv_dx)) + fma(z.a, t.gy, -rec.d_rv);
            rp4.d = fma(gb.d, t.inv_dy, -((fr.d - fl.d) * t.inv_dx));
        }

        // ---- carries of row r -------------------------------------------------------------
        const Prim<double> syt = state_at(mid, rec.gy, py, t.half_dy);
        if (fluid && (f & FLAG_WALL_YP) && r < j1)  // a wall above row r: that face's flux now
            below = osher_y(syt, ghost_state(t, rec, 1, +1, slip), t.beta, t.inv_beta);
        else
            below = {syt.r, syt.u, syt.v, syt.p};
        if (fluid && r >= j0 && r < j1) {
            const double dtau = local_dtau(t, t.cfl, z.a, z.b, z.c);
            const double ad = alpha * dtau;
            const double fc = ad / (1.0 + sp.b0 * ad * sp.inv_dt);
            if (LAST) {
                pre = z;
                rpart = rp4;
                fac = fc;
                adt = ad;
            } else {
                pre = {fma(fc, rp4.a, z.a), fma(fc, rp4.b, z.b), fma(fc, rp4.c, z.c),
                       fma(t.beta * ad, rp4.d, z.d)};
                fac = fc * t.inv_dy;
                adt = t.beta * ad * t.inv_dy;
            }
        }
        fluid_lo = fluid;
        lo = mid;
        mid = hi;
        hi = next_hi;
    }

    if (LAST) {
        // wave reduction (fixed order) and one partial per strip chunk
        const double part[kPartialWidth] = {part0, part1, part2, part3, part4};
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

int launch_stage_march_f64(const TankDev &t, const Scheme &sc, int stage, int chunk, int waves,
                           void *stream)
{
    const int n_strips = (t.nx + kOut - 1) / kOut;
    const int n_units = march_units(t, chunk);
    const int n_blocks = (n_units + kWavesPerBlock - 1) / kWavesPerBlock;
    const int grid = ((n_blocks + 7) / 8) * 8;
    const dim3 g(grid), b(kLanes * kWavesPerBlock);
    hipStream_t s = (hipStream_t)stream;
    const bool bdf2 = t.level_nm1 != nullptr;
    const bool last = stage == sc.smax;
#define VDAC_MARCH(NM, B2, LS)                                                                       \
    do {                                                                                             \
        if (waves == 3)                                                                              \
            hipLaunchKernelGGL((stage_march_f64<NM, B2, LS, 3>), g, b, 0, s, t, sc, stage, chunk,    \
                               n_strips, n_units);                                                   \
        else                                                                                         \
            hipLaunchKernelGGL((stage_march_f64<NM, B2, LS, 2>), g, b, 0, s, t, sc, stage, chunk,    \
                               n_strips, n_units);                                                   \
    } while (0)
    if (last) {
        if (sc.norm_max) {
            if (bdf2) VDAC_MARCH(true, true, true);
            else VDAC_MARCH(true, false, true);
        } else {
            if (bdf2) VDAC_MARCH(false, true, true);
            else VDAC_MARCH(false, false, true);
        }
    } else {
        if (bdf2) VDAC_MARCH(false, true, false);
        else VDAC_MARCH(false, false, false);
    }
#undef VDAC_MARCH
    return (int)hipGetLastError();
}

}  // namespace vdac
