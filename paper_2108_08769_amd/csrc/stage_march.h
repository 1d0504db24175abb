// stage_march.h -- the Runge-Kutta stage kernel for gfx950 in its row-marching form, for the
// FP64 and the mixed-precision storage, over any number of tanks in one launch.  Instantiated
// by stage_march.hip (the default scheme: Osher-Dumbser-Toro flux, new pressure gradient, walls
// and periodic sides, local pseudo-time steps) and stage_march_gen.hip (GEN: the Roe or exact
// flux, the k-limiter or the split limiter on p, zero-gradient sides and the global
// pseudo-time step chosen at run time).
//
// Work comes from a unit table: entry e of the table is the work of wave e % W of workgroup
// e / W (W waves per workgroup), one chunk of rows of one 64-column strip of one tank.  The host
// orders the table so that workgroup b, which the dispatcher places on XCD b % 8, gets a unit
// next to the other units of that XCD (one L2 per XCD).
//
// Each 64-lane wave owns a strip of 64 consecutive columns (lanes 2..61 produce output, lanes
// 0-1 and 62-63 are the halo the reconstruction and the x-faces need) and sweeps its chunk of
// rows upward.  The three rows the limited slopes need stay in registers, x-neighbours come from
// cross-lane DPP moves, and the loads of the next row are issued a full row ahead of their use.
// No LDS, no workgroup barrier.  Per row r the wave
//   1. reconstructs row r once per lane: limited slopes (Sec. 2.3.1), the stage-0 sources from
//      Q^0 and level n, the new pressure gradient (Sec. 2.3.2), and the states at the four faces;
//   2. evaluates the x-faces of row r with the Osher-Dumbser-Toro flux (Sec. 2.4.3): lane x takes
//      the face on its right, its right neighbour receives the result for its left face; a lane
//      whose left face is a wall evaluates that face itself from its own ghost (Sec. 2.5);
//   3. evaluates the y-face between rows r-1 and r (rotated, Sec. 2.4); a face with a wall above
//      row r is evaluated with row r's ghost and carried to the next row;
//   4. completes row r-1: flux divergence, frozen sources, point-implicit update (eq. 24), and
//      on the last stage the residual partial.
// Each face is evaluated once.  Periodic sides wrap indices; cells outside a non-periodic side
// read as non-fluid.
//
// Mixed form: all four fields are stored as FP32 deviations from the FP64 level n, so the
// absolute state is known to FP64 accuracy up to the FP32 rounding of the (small) deviations.
// The reconstruction and the fluxes run in FP32 on pressures measured from the pressure of the
// face's lower-index cell (the ghost's, equal to the cell's own, on a wall).  The Osher flux
// depends on p only through the p term of the normal momentum flux and through p differences, so
// the shift is exact: the divergence adds back p_i - p_ref of the lower face in FP64.  This keeps
// the hydrostatic pressure differences, which are small against p itself, to FP32 precision of
// the differences.  Sources, divergence, update and norm run in FP64; the update is formed on
// the deviation from level n, then rounded to FP32.
#pragma once

#include <atomic>

#include <hip/hip_runtime.h>

#include "stage_common.h"

namespace vdac {

namespace march {

constexpr int kLanes = 64;
constexpr int kOut = 60;            // output columns per strip (lanes 2..61)
constexpr int kMaxWavesPerBlock = 4;

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

// Neighbour exchange across the wave with DPP moves (wave_shr:1 / wave_shl:1 shift a value one
// lane up / down the whole 64-lane wave in one VALU instruction); the lane without a source
// (lane 0, resp. 63, a halo lane) reads zero.
constexpr int kDppWaveShr1 = 0x138, kDppWaveShl1 = 0x130;

__device__ __forceinline__ float from_left(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), kDppWaveShr1, 0xf, 0xf, true));
}
__device__ __forceinline__ float from_right(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), kDppWaveShl1, 0xf, 0xf, true));
}
__device__ __forceinline__ double from_left(double v)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)b, kDppWaveShr1, 0xf, 0xf, true);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(b >> 32), kDppWaveShr1, 0xf, 0xf, true);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ double from_right(double v)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)b, kDppWaveShl1, 0xf, 0xf, true);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(b >> 32), kDppWaveShl1, 0xf, 0xf, true);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

template <typename T>
__device__ __forceinline__ Prim<T> prim_from_left(const Prim<T> &w)
{
    return {from_left(w.r), from_left(w.u), from_left(w.v), from_left(w.p)};
}
template <typename T>
__device__ __forceinline__ Prim<T> prim_from_right(const Prim<T> &w)
{
    return {from_right(w.r), from_right(w.u), from_right(w.v), from_right(w.p)};
}

template <typename T, typename U>
__device__ __forceinline__ Vec4<T> cast4(const Vec4<U> &a)
{
    return {(T)a.a, (T)a.b, (T)a.c, (T)a.d};
}

// Loads and stores at a 32-bit byte offset from a wave-uniform base in the global address space:
// the base stays in scalar registers and one vector register holds the offset, shared by every
// plane of a row (a plane holds fewer than 2^29 cells, so its byte offsets fit 32 bits).
template <typename T>
__device__ __forceinline__ T gld(const T *base, uint32_t off)
{
    using GC = __attribute__((address_space(1))) const char;
    using GT = __attribute__((address_space(1))) const T;
    return *(GT *)((GC *)base + off);
}
template <typename T>
__device__ __forceinline__ void gst(T *base, uint32_t off, T v)
{
    using GC = __attribute__((address_space(1))) char;
    using GT = __attribute__((address_space(1))) T;
    *(GT *)((GC *)base + off) = v;
}

// Byte offsets of this lane's column within a row: in the state's element type, in FP64 (the
// real-time levels) and in bytes (the flags).
struct LaneOff {
    uint32_t s, d, f;
};

// Loads of one row, issued one step ahead of their use: the stage input is fetched two rows
// ahead (it is the upper neighbour of the next row), the stage-0 state, level n (and level
// n-1) and the flags one row ahead.
template <class P>
struct InputLoad {
    typename P::Store r, m, n, p;  // stage input Q^{s-1} (mixed: deviations from level n)
    double lr, lm, ln, lp;         // level n of rho, rho u, rho v, p (mixed form only)
};
template <class P>
struct SourceLoad {
    typename P::Store z0, z1, z2, z3;  // stage-0 state Q^0 (mixed: deviations from level n)
    double n0, n1, n2;                 // level n (FP64 form only)
    double m0, m1, m2;                 // level n-1 (BDF2, BDF3)
    double k0, k1, k2;                 // level n-2 (BDF3)
    uint8_t f;                         // cell flags (FLAG_SOLID if outside the tank)
};

// Row of a load: row r itself, wrapped across a periodic side, or (outside a non-periodic side)
// the nearest row of the tank.  The cells outside the tank are not fluid (their flag reads
// FLAG_SOLID), and every use of their values is guarded by that flag or by the wall flags of
// their fluid neighbours, which take ghosts instead; loading a real cell there keeps the loads
// unconditional and the values finite.  r is wave-uniform, and so is the result.
__device__ __forceinline__ int load_row(const TankDev &t, int r, bool &inside)
{
    int gj;
    inside = locate_axis(r, t.ny, t.per_y, gj);
    return uni(inside ? gj : (r < 0 ? 0 : t.ny - 1));
}

template <class P>
__device__ __forceinline__ InputLoad<P> load_input(const TankDev &t,
                                                   const typename P::Store *__restrict__ qprev,
                                                   const LaneOff &lo, int r)
{
    using S = typename P::Store;
    bool inside;
    const uint32_t row = (uint32_t)load_row(t, r, inside) * (uint32_t)t.nx;
    const uint32_t os = row * (uint32_t)sizeof(S) + lo.s;
    const size_t plane = t.plane;
    InputLoad<P> L;
    L.r = gld(qprev, os);
    L.m = gld(qprev + plane, os);
    L.n = gld(qprev + 2 * plane, os);
    L.p = gld(qprev + 3 * plane, os);
    if (P::kMixed) {
        const uint32_t od = row * 8u + lo.d;
        L.lr = gld(t.level_n, od);
        L.lm = gld(t.level_n + plane, od);
        L.ln = gld(t.level_n + 2 * plane, od);
        L.lp = gld(t.level_n + 3 * plane, od);
    } else {
        L.lr = L.lm = L.ln = L.lp = 0.0;
    }
    return L;
}

// Z = false leaves out Q^0 (stage 1 of the FP64 form takes it from the input rows instead).
template <class P, int BDF, bool Z = true>
__device__ __forceinline__ SourceLoad<P> load_sources(const TankDev &t,
                                                      const typename P::Store *__restrict__ q0,
                                                      bool have_col, const LaneOff &lo, int r)
{
    using S = typename P::Store;
    bool inside;
    const uint32_t row = (uint32_t)load_row(t, r, inside) * (uint32_t)t.nx;
    const uint32_t os = row * (uint32_t)sizeof(S) + lo.s, od = row * 8u + lo.d;
    const size_t plane = t.plane;
    SourceLoad<P> L;
    const uint8_t f = gld(t.flags, row + lo.f);
    L.f = (have_col && inside) ? f : (uint8_t)FLAG_SOLID;
    if constexpr (Z) {
        L.z0 = gld(q0, os);
        L.z1 = gld(q0 + plane, os);
        L.z2 = gld(q0 + 2 * plane, os);
        L.z3 = gld(q0 + 3 * plane, os);
    } else {
        L.z0 = L.z1 = L.z2 = L.z3 = 0;
    }
    if (!P::kMixed) {  // the mixed form takes level n from the input row (it carries it)
        L.n0 = gld((const double *)t.level_n, od);
        L.n1 = gld((const double *)t.level_n + plane, od);
        L.n2 = gld((const double *)t.level_n + 2 * plane, od);
    } else {
        L.n0 = L.n1 = L.n2 = 0.0;
    }
    if (BDF >= 2) {
        L.m0 = gld((const double *)t.level_nm1, od);
        L.m1 = gld((const double *)t.level_nm1 + plane, od);
        L.m2 = gld((const double *)t.level_nm1 + 2 * plane, od);
    } else {
        L.m0 = L.m1 = L.m2 = 0.0;
    }
    if (BDF >= 3) {
        L.k0 = gld((const double *)t.level_nm2, od);
        L.k1 = gld((const double *)t.level_nm2 + plane, od);
        L.k2 = gld((const double *)t.level_nm2 + 2 * plane, od);
    } else {
        L.k0 = L.k1 = L.k2 = 0.0;
    }
    return L;
}

// Primitives of a loaded cell in the reconstruction precision.  In the mixed form p is left at
// zero: the face pressures come from the FP64 pressure (abs_p) through differences.
template <class P>
__device__ __forceinline__ Prim<typename P::Real> to_prim(const InputLoad<P> &L)
{
    if constexpr (P::kMixed) {
        const float r = (float)(L.lr + (double)L.r);
        const float m = (float)(L.lm + (double)L.m);
        const float n = (float)(L.ln + (double)L.n);
        const float ir = rcp_pos(r);
        return {r, m * ir, n * ir, 0.0f};
    } else {
        const double ir = rcp_pos(L.r);
        return {L.r, L.m * ir, L.n * ir, L.p};
    }
}

// Absolute pressure of a loaded cell in FP64.
template <class P>
__device__ __forceinline__ double abs_p(const InputLoad<P> &L)
{
    return P::kMixed ? L.lp + (double)L.p : (double)L.p;
}

// WAVES: the register budget as waves per SIMD (2: up to 256 VGPRs per lane, 3: up to 168).
// BDF: the highest real-time order of the grid (levels n-1, n-2 read); GEN: general options.
// FIRST (FP64 form, stage 1 of more than one): Q^{s-1} is Q^0, so Q^0 of a row is taken from
// the input rows the window already holds (the same values) instead of being read again.
template <class P, bool NORM_MAX, int BDF, bool LAST, int WAVES, bool GEN, bool FIRST = false>
__global__ void __launch_bounds__(kLanes *kMaxWavesPerBlock, WAVES)
    stage_march(const TankDev *__restrict__ tanks, const MarchUnit *__restrict__ units, Scheme sc,
                int stage, IterArgs ia)
{
    using R = typename P::Real;
    using S = typename P::Store;

    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kLanes);
    const int lane = threadIdx.x % kLanes;
    int entry = blockIdx.x * (blockDim.x / kLanes) + wave;
    if (ia.fin) {  // the waves in front of the unit table finalize the previous iteration
        if (entry < ia.n_fin) {
            if (entry < ia.n_tanks) finalize_wave(load_tank(tanks + entry), sc, lane);
            return;
        }
        entry -= ia.n_fin;
    }
    // one unit per wave, or, in a persistent launch (stride > 0), every stride-th entry of the
    // unit table from this wave's own: the loop ends for every wave once its entries run out
    const int step = ia.stride > 0 ? ia.stride : 1;
    const int end = ia.stride > 0 ? ia.n_entries : entry + 1;
    for (; entry < end; entry += step) {
        const MarchUnit un = units[entry];
        if (un.tank < 0) continue;  // padding (uniform per wave)
        const TankDev t = load_tank(tanks + un.tank);
        const Status *st = t.status;
        // the buffers follow from the iteration (IterArgs); the stop flag is tested once the first
        // rows' loads are in flight, so that its latency overlaps theirs
        const int stopped = st->done;

        const int strip = un.local % t.n_strips, ch = un.local / t.n_strips;
        const int col = strip * kOut - 2 + lane;  // this lane's column (may lie outside the tank)
        int gi = 0;
        const bool have_col = locate_axis(col, t.nx, t.per_x, gi);
        if (!have_col) gi = col < 0 ? 0 : t.nx - 1;  // loads take the nearest column (see load_row)
        const bool out_lane = lane >= 2 && lane < 2 + kOut && col >= 0 && col < t.nx;
        const int j0 = ch * t.chunk;
        const int j1 = min(j0 + t.chunk, t.ny);
        const LaneOff lof = {(uint32_t)gi * (uint32_t)sizeof(S), (uint32_t)gi * 8u, (uint32_t)gi};

        const int cur = ia.cur_off;
        const StageBuffers bufs = stage_buffers(cur, stage);
        const S *__restrict__ qprev = (const S *)state_buf(tanks + un.tank, bufs.in);
        const S *__restrict__ q0 = (const S *)state_buf(tanks + un.tank, cur);
        S *__restrict__ qout = (S *)state_buf(tanks + un.tank, bufs.out);
        const StepParams sp = *t.step;
        const bool slip = sc.slip != 0;
        const R kl = (R)sc.k;
        const double alpha = sc.alpha[stage - 1];
        const double a_dtau = alpha * (t.cfl * (t.dx * t.dy));  // alpha_s CFL dx dy
        const double fdx = t.flux_dx, fdy = t.flux_dy;  // 1/(2h): the fluxes come doubled
        const double kappa = sp.b0 * a_dtau * sp.inv_dt;
        const size_t plane = t.plane;
        const R hx = (R)t.half_dx, hy = (R)t.half_dy;
        const R beta = (R)t.beta, inv_beta = (R)t.inv_beta;
        // general options: zero-gradient faces of this lane's column, global pseudo-time step
        const bool open_xm = GEN && col == 0 && (t.open & 1);
        const bool open_xp = GEN && col == t.nx - 1 && (t.open & 2);
        const double dtau_glob = GEN ? st->dtau_global : 0.0;
        const bool use_glob = GEN && sc.global_dtau != 0;

        // window of primitives: rows r-1 (lo), r (mid), r+1 (hi); loads for later rows in flight
        // (plo, pmid, phi: their absolute pressures in FP64)
        // (mixed form: lvl_mid, lvl_hi carry level n of rho, rho u, rho v of rows r and r+1, which
        // the input loads fetched, so that the sources need not fetch it again)
        static_assert(!FIRST || (!P::kMixed && !LAST), "FIRST is the FP64 form's stage 1");
        Prim<R> lo, mid, hi;
        double plo, pmid, phi;
        double mlo = 0.0, mmid = 0.0, mhi = 0.0, nlo = 0.0, nmid = 0.0, nhi = 0.0;  // FIRST: rho u, rho v
        Vec4<double> lvl_mid = zero4<double>(), lvl_hi = zero4<double>();
        {
            const InputLoad<P> a = load_input<P>(t, qprev, lof, j0 - 2);
            const InputLoad<P> b = load_input<P>(t, qprev, lof, j0 - 1);
            const InputLoad<P> c = load_input<P>(t, qprev, lof, j0);
            lo = to_prim(a);
            mid = to_prim(b);
            hi = to_prim(c);
            plo = abs_p(a);
            pmid = abs_p(b);
            phi = abs_p(c);
            if constexpr (FIRST) {
                mlo = a.m; mmid = b.m; mhi = c.m;
                nlo = a.n; nmid = b.n; nhi = c.n;
            }
            if constexpr (P::kMixed) {
                lvl_mid = {b.lr, b.lm, b.ln, 0.0};
                lvl_hi = {c.lr, c.lm, c.ln, 0.0};
            }
        }
        InputLoad<P> in_ld = load_input<P>(t, qprev, lof, j0 + 1);              // row r+2
        SourceLoad<P> src_ld = load_sources<P, BDF, !FIRST>(t, q0, have_col, lof, j0 - 1); // row r
        if (stopped) continue;

        // carries from row r-1:
        //  below      its state at its upper face, or, if that face is a wall, the face's flux
        //  pre        its update without the flux above it: non-final stages carry
        //             pre = Q^0 + fac R_partial; the final stage keeps Q^0 and R_partial apart for
        //             the residual norm (mixed form: deviations from level n in place of Q)
        //  lvl        final stage, mixed form: its level-n density (for the positivity check); the
        //             general kernel also keeps rho u, rho v of level n (lvl_m, lvl_n) for the
        //             pseudo-time step of the updated state
        Vec4<R> below = {R(1), R(0), R(0), R(0)};
        Vec4<double> pre = zero4<double>();
        Vec4<double> rpart = zero4<double>();
        double fac = 0.0, adt = 0.0, lvl = 0.0, lvl_m = 0.0, lvl_n = 0.0;
        bool fluid_lo = false;
        double part0 = 0.0, part1 = 0.0, part2 = 0.0, part3 = 0.0, part4 = 0.0, part5 = INFINITY;

        // One row step (row r's reconstruction, its faces, and the update of row r-1).  The window
        // (primitives, FP64 pressures and, mixed form, level n of rows r-1, r, r+1) comes in by
        // reference; the step writes row r+2 into the slots of row r-1, so that consecutive steps
        // rotate the slots' roles instead of copying them.
        auto row_step = [&](int r, Prim<R> &lo, Prim<R> &mid, Prim<R> &hi, double &plo, double &pmid,
                            double &phi, Vec4<double> &lvl_lo, Vec4<double> &lvl_mid,
                            Vec4<double> &lvl_hi) __attribute__((always_inline)) {
            (void)lvl_hi;
            // sources of row r (loaded one step ahead), then the next loads
            const uint8_t f = src_ld.f;
            const bool fluid = !(f & FLAG_SOLID);
            // z: the base of the update (Q^0, or its deviation and p^0); a0..a2: absolute Q^0
            const Vec4<double> z = FIRST ? Vec4<double>{(double)mid.r, mmid, nmid, pmid}
                                         : Vec4<double>{(double)src_ld.z0, (double)src_ld.z1,
                                                        (double)src_ld.z2, (double)src_ld.z3};
            double a0, a1, a2, num0, num1, num2;
            double lvl_r;  // level-n density of row r
            if constexpr (P::kMixed) {
                // (B0 Q^0 + B1 Q^n + B2 Q^{n-1}) = B0 (Q^0 - Q^n) + B2 (Q^{n-1} - Q^n): B0+B1+B2 = 0
                a0 = lvl_mid.a + z.a;
                a1 = lvl_mid.b + z.b;
                a2 = lvl_mid.c + z.c;
                num0 = sp.b0 * z.a;
                num1 = sp.b0 * z.b;
                num2 = sp.b0 * z.c;
                if (BDF >= 2) {
                    num0 = fma(sp.b2, src_ld.m0 - lvl_mid.a, num0);
                    num1 = fma(sp.b2, src_ld.m1 - lvl_mid.b, num1);
                    num2 = fma(sp.b2, src_ld.m2 - lvl_mid.c, num2);
                }
                if (BDF >= 3) {
                    num0 = fma(sp.b3, src_ld.k0 - lvl_mid.a, num0);
                    num1 = fma(sp.b3, src_ld.k1 - lvl_mid.b, num1);
                    num2 = fma(sp.b3, src_ld.k2 - lvl_mid.c, num2);
                }
                lvl_r = lvl_mid.a;
            } else {
                a0 = z.a;
                a1 = z.b;
                a2 = z.c;
                num0 = fma(sp.b0, z.a, sp.b1 * src_ld.n0);
                num1 = fma(sp.b0, z.b, sp.b1 * src_ld.n1);
                num2 = fma(sp.b0, z.c, sp.b1 * src_ld.n2);
                if (BDF >= 2) {
                    num0 = fma(sp.b2, src_ld.m0, num0);
                    num1 = fma(sp.b2, src_ld.m1, num1);
                    num2 = fma(sp.b2, src_ld.m2, num2);
                }
                if (BDF >= 3) {
                    num0 = fma(sp.b3, src_ld.k0, num0);
                    num1 = fma(sp.b3, src_ld.k1, num1);
                    num2 = fma(sp.b3, src_ld.k2, num2);
                }
                lvl_r = src_ld.n0;
            }
            const double d_r = num0 * sp.inv_dt, d_ru = num1 * sp.inv_dt, d_rv = num2 * sp.inv_dt;
            const Prim<R> next_hi = to_prim(in_ld);
            const double next_phi = abs_p(in_ld);
            const double next_m = FIRST ? (double)in_ld.m : 0.0, next_n = FIRST ? (double)in_ld.n : 0.0;
            const Vec4<double> next_lvl = {in_ld.lr, in_ld.lm, in_ld.ln, 0.0};
            // the chunk reconstructs rows up to j1 from inputs up to row j1 + 1: past those rows the
            // loads repeat the last needed row (a cache hit), with no branch around them
            in_ld = load_input<P>(t, qprev, lof, min(r + 3, j1 + 1));
            src_ld = load_sources<P, BDF, !FIRST>(t, q0, have_col, lof, min(r + 1, j1));

            // ---- reconstruction of row r ------------------------------------------------------
            const Prim<R> wl = prim_from_left(mid);
            const Prim<R> wr = prim_from_right(mid);
            CellRecT<R> rec;
            rec.w = mid;
            rec.d_r = (R)d_r;
            rec.d_ru = (R)d_ru;
            rec.d_rv = (R)d_rv;
            rec.rho0 = (R)a0;
            // zero-gradient faces of row r (general kernel)
            const bool open_ym = GEN && r == 0 && (t.open & 4);
            const bool open_yp = GEN && r == t.ny - 1 && (t.open & 8);
            const double pright = GEN ? from_right(pmid) : 0.0;  // shuffles: every lane takes part
            const double pleft_g = GEN ? from_left(pmid) : 0.0;
            // every lane reconstructs (no branch): the values of a lane that holds no fluid cell are
            // finite and never used, since its fluid neighbours see a wall there and take ghosts
            R px, py;
            {
                const Prim<R> xm = (f & FLAG_WALL_XM) ? (open_xm ? mid : mirror(mid, 0, slip)) : wl;
                const Prim<R> xp = (f & FLAG_WALL_XP) ? (open_xp ? mid : mirror(mid, 0, slip)) : wr;
                const Prim<R> ym = (f & FLAG_WALL_YM) ? (open_ym ? mid : mirror(mid, 1, slip)) : lo;
                const Prim<R> yp = (f & FLAG_WALL_YP) ? (open_yp ? mid : mirror(mid, 1, slip)) : hi;
                rec.gx = slopes(xm, mid, xp, (R)t.inv_dx, kl);
                rec.gy = slopes(ym, mid, yp, (R)t.inv_dy, kl);
                if (GEN && sc.pgrad != 0) {
                    // across a wall or zero-gradient face the stencil sees the cell's own p and rho
                    const double dpr_x = (f & FLAG_WALL_XP) ? 0.0 : pright - pmid;
                    const double dpl_x = (f & FLAG_WALL_XM) ? 0.0 : pmid - pleft_g;
                    const double dpr_y = (f & FLAG_WALL_YP) ? 0.0 : phi - pmid;
                    const double dpl_y = (f & FLAG_WALL_YM) ? 0.0 : pmid - plo;
                    px = (R)pgrad_limited(sc.pgrad, sc.pk, dpr_x, dpl_x, t.inv_dx, (double)xm.r,
                                          (double)mid.r, (double)xp.r, t.gx);
                    py = (R)pgrad_limited(sc.pgrad, sc.pk, dpr_y, dpl_y, t.inv_dy, (double)ym.r,
                                          (double)mid.r, (double)yp.r, t.gy);
                } else {
                    px = cell_gradp_x(t, rec);
                    py = cell_gradp_y(t, rec);
                }
            }
            // pressure each face state is expressed from: the absolute p (FP64 form), or p minus
            // the pressure of the face's lower-index cell (mixed form); sx, sy add that reference
            // back at the lower faces in FP64
            R pb_own = mid.p, pb_xl = mid.p, pb_yb = mid.p;
            double sx = 0.0, sy = 0.0;
            if constexpr (P::kMixed) {
                const double pleft = from_left(pmid);  // a shuffle: every lane takes part
                sx = (f & FLAG_WALL_XM) ? 0.0 : pmid - pleft;
                sy = (f & FLAG_WALL_YM) ? 0.0 : pmid - plo;
                pb_own = R(0);
                pb_xl = (R)sx;
                pb_yb = (R)sy;
            }

            // ---- y-face between rows r-1 and r ------------------------------------------------
            // (a fluid row r-1 below a cell without fluid carries the face's flux, evaluated with its
            // ghost, in below; the value of gb where neither is fluid is never used)
            Vec4<R> gb = below;
            if (r >= j0 && fluid) {
                Prim<R> L = Prim<R>{below.a, below.b, below.c, below.d};
                if (!fluid_lo)
                    L = GEN ? ghost_state_gen(t, sc, rec, 1, -1, open_ym, py, pb_own)
                            : ghost_state(t, rec, 1, -1, slip, pb_own);
                const Prim<R> Rs = state_at(mid, rec.gy, py, -hy, pb_yb);
                gb = GEN ? flux_y(sc.flux, L, Rs, beta, inv_beta) : osher_y(L, Rs, beta, inv_beta);
            }
            const Vec4<double> gbd = cast4<double>(gb);

            // ---- update of row r-1 ------------------------------------------------------------
            if (r - 1 >= j0 && out_lane && fluid_lo) {
                int gj;
                locate_axis(r - 1, t.ny, t.per_y, gj);
                const uint32_t os = (uint32_t)uni(gj) * (uint32_t)t.nx * (uint32_t)sizeof(S) + lof.s;
                if (LAST) {
                    const double R0 = fma(-gbd.a, fdy, rpart.a);
                    const double R1 = fma(-gbd.b, fdy, rpart.b);
                    const double R2 = fma(-gbd.c, fdy, rpart.c);
                    const double R3 = fma(-gbd.d, fdy, rpart.d);
                    const double rn = fma(fac, R0, pre.a);
                    gst(qout, os, (S)rn);
                    gst(qout + plane, os, (S)fma(fac, R1, pre.b));
                    gst(qout + 2 * plane, os, (S)fma(fac, R2, pre.c));
                    gst(qout + 3 * plane, os, (S)fma(t.beta, adt * R3, pre.d));
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
                    const double rho_new = P::kMixed ? lvl + rn : rn;
                    part4 += (rho_new > 0.0 && rho_new < INFINITY) ? 0.0 : 1.0;
                    if (GEN && sc.global_dtau) {
                        // pseudo-time step of the updated state: the next iteration's stage 0
                        const double m_new = fma(fac, R1, pre.b) + (P::kMixed ? lvl_m : 0.0);
                        const double n_new = fma(fac, R2, pre.c) + (P::kMixed ? lvl_n : 0.0);
                        if (rho_new > 0.0) part5 = fmin(part5, local_dtau(t, t.cfl, rho_new, m_new, n_new));
                    }
                } else {
                    // fac and adt already carry 1/(2 dy) here
                    gst(qout, os, (S)fma(-fac, gbd.a, pre.a));
                    gst(qout + plane, os, (S)fma(-fac, gbd.b, pre.b));
                    gst(qout + 2 * plane, os, (S)fma(-fac, gbd.c, pre.c));
                    gst(qout + 3 * plane, os, (S)fma(-adt, gbd.d, pre.d));
                }
            }

            // ---- x-faces of row r, its residual without the upper y-face, its carries ----------
            if (r >= j0 && r < j1) {
                // every lane evaluates its right face (no branch); a lane without fluid produces a
                // value that no fluid neighbour reads (that neighbour has a wall there)
                const Prim<R> sxl = state_at(mid, rec.gx, px, -hx, pb_xl);
                Prim<R> Rs = prim_from_right(sxl);  // right neighbour's left state
                if (f & FLAG_WALL_XP)
                    Rs = GEN ? ghost_state_gen(t, sc, rec, 0, +1, open_xp, px, pb_own)
                             : ghost_state(t, rec, 0, +1, slip, pb_own);
                const Prim<R> Ls = state_at(mid, rec.gx, px, hx, pb_own);
                const Vec4<R> fr = GEN ? flux_x(sc.flux, Ls, Rs, beta, inv_beta) : osher_x(Ls, Rs, beta, inv_beta);
                Vec4<R> fl = {from_left(fr.a), from_left(fr.b), from_left(fr.c), from_left(fr.d)};
                if (fluid && (f & FLAG_WALL_XM)) {
                    const Prim<R> Lg = GEN ? ghost_state_gen(t, sc, rec, 0, -1, open_xm, px, pb_own)
                                           : ghost_state(t, rec, 0, -1, slip, pb_own);
                    fl = GEN ? flux_x(sc.flux, Lg, sxl, beta, inv_beta) : osher_x(Lg, sxl, beta, inv_beta);
                }
                const Vec4<double> frd = cast4<double>(fr), fld = cast4<double>(fl);
                // -(x-divergence) + lower flux / dy - real-time term + body force
                Vec4<double> rp4;
                rp4.a = fma(gbd.a, fdy, -((frd.a - fld.a) * fdx)) - d_r;
                rp4.b = fma(gbd.b, fdy, -((frd.b - fld.b) * fdx)) + fma(a0, t.gx, -d_ru);
                rp4.c = fma(gbd.c, fdy, -((frd.c - fld.c) * fdx)) + fma(a0, t.gy, -d_rv);
                rp4.d = fma(gbd.d, fdy, -((frd.d - fld.d) * fdx));
                if constexpr (P::kMixed) {
                    rp4.b = fma(-sx, t.inv_dx, rp4.b);
                    rp4.c = fma(-sy, t.inv_dy, rp4.c);
                }
                // carries of row r (read by the update of row r in the next step, fluid lanes only)
                double ad, fc;
                if (use_glob) {
                    ad = alpha * dtau_glob;
                    fc = ad * rcp_pos(fma(sp.b0 * ad, sp.inv_dt, 1.0));
                } else if (P::kMixed) {
                    dtau_factors_f32(t, (float)a_dtau, (float)kappa, a0, a1, a2, ad, fc);
                } else {
                    dtau_factors(t, a_dtau, kappa, a0, a1, a2, ad, fc);
                }
                if (LAST) {
                    pre = z;
                    rpart = rp4;
                    fac = fc;
                    adt = ad;
                    lvl = lvl_r;
                    if (GEN && P::kMixed) {
                        lvl_m = lvl_mid.b;
                        lvl_n = lvl_mid.c;
                    }
                } else {
                    pre = {fma(fc, rp4.a, z.a), fma(fc, rp4.b, z.b), fma(fc, rp4.c, z.c),
                           fma(t.beta * ad, rp4.d, z.d)};
                    fac = fc * fdy;
                    adt = t.beta * ad * fdy;
                }
            }
            const Prim<R> syt = state_at(mid, rec.gy, py, hy, pb_own);
            below = {syt.r, syt.u, syt.v, syt.p};
            if (fluid && (f & FLAG_WALL_YP) && r < j1)  // a wall above row r: that face's flux now
                below = GEN ? flux_y(sc.flux, syt, ghost_state_gen(t, sc, rec, 1, +1, open_yp, py, pb_own),
                                     beta, inv_beta)
                            : osher_y(syt, ghost_state(t, rec, 1, +1, slip, pb_own), beta, inv_beta);
            fluid_lo = fluid;
            lo = next_hi;
            plo = next_phi;
            if constexpr (FIRST) {
                mlo = next_m;
                nlo = next_n;
            }
            if constexpr (P::kMixed) lvl_lo = next_lvl;
        };

        // rows j0-1 .. j1.  Mixed form (bound by its arithmetic): three steps per trip with the
        // slots' roles rotated, then the last 0..2 rows.  FP64 (bound by memory; the larger loop
        // body measured slower): one step per trip.  A single step moves the roles back into place.
        Vec4<double> lvl_lo = zero4<double>();
        int r = j0 - 1;
        if constexpr (P::kMixed) {
            for (; r + 2 <= j1; r += 3) {
                row_step(r, lo, mid, hi, plo, pmid, phi, lvl_lo, lvl_mid, lvl_hi);
                row_step(r + 1, mid, hi, lo, pmid, phi, plo, lvl_mid, lvl_hi, lvl_lo);
                row_step(r + 2, hi, lo, mid, phi, plo, pmid, lvl_hi, lvl_lo, lvl_mid);
            }
        }
        for (; r <= j1; ++r) {
            row_step(r, lo, mid, hi, plo, pmid, phi, lvl_lo, lvl_mid, lvl_hi);
            const Prim<R> w = lo;
            lo = mid;
            mid = hi;
            hi = w;
            const double pw = plo;
            plo = pmid;
            pmid = phi;
            phi = pw;
            if constexpr (FIRST) {
                const double mw = mlo, nw = nlo;
                mlo = mmid;
                mmid = mhi;
                mhi = mw;
                nlo = nmid;
                nmid = nhi;
                nhi = nw;
            }
            if constexpr (P::kMixed) {
                const Vec4<double> lw = lvl_lo;
                lvl_lo = lvl_mid;
                lvl_mid = lvl_hi;
                lvl_hi = lw;
            }
        }

        if (LAST) {
            // wave reduction (fixed order, in VALU) and one partial per unit
            const double part[kPartialWidth] = {part0, part1, part2, part3, part4, part5};
            auto sum = [](double a, double b) { return a + b; };
            auto mx = [](double a, double b) { return combine<true>(a, b); };
            auto mn = [](double a, double b) { return fmin(a, b); };
#pragma unroll
            for (int k = 0; k < kPartialWidth; ++k) {
                const double x = (k == 5) ? wave_reduce_to_lane63(part[k], INFINITY, mn)
                                          : ((NORM_MAX && k < 4) ? wave_reduce_to_lane63(part[k], 0.0, mx)
                                                                 : wave_reduce_to_lane63(part[k], 0.0, sum));
                if (lane == kLanes - 1) t.partials[(size_t)un.local * kPartialWidth + k] = x;
            }
        }
    }
}

// Workgroups of `threads` threads of kernel `kern` that the whole chip holds at once (its own
// occupancy per CU times the CUs), rounded down to a multiple of 8; cached in `cache` once known
// (0 while unknown: the launch then goes out one wave per unit).
inline int resident_workgroups(const void *kern, int threads, std::atomic<int> &cache)
{
    const int known = cache.load(std::memory_order_relaxed);
    if (known > 0) return known;
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, threads, 0) != hipSuccess)
        return 0;
    const int r = per_cu * cus / 8 * 8;
    cache.store(r, std::memory_order_relaxed);
    return r;
}

// Persistent launch of a stage over the unit table: the finalize workgroups in front as they are,
// then only `resident` workgroups for the units, each wave taking every stride-th entry.  A
// multiple of 8 keeps workgroup b and every entry it takes (b + k x resident workgroups in the
// table) on the same XCD, b mod 8.
inline void persist_grid(dim3 &g, IterArgs &a, unsigned threads, int resident)
{
    const int wpb = (int)threads / kLanes;
    const int fin_blocks = a.n_fin / wpb;
    const int unit_blocks = (int)g.x - fin_blocks;
    if (resident >= 8 && unit_blocks > resident) {
        g.x = (unsigned)(fin_blocks + resident);
        a.stride = resident * wpb;
    }
}

template <class P, bool NM, int BDF, bool LS, bool GEN, bool FIRST = false>
void launch_t(const TankDev *tanks, const MarchUnit *units, dim3 g, dim3 b, int waves_simd,
              const Scheme &sc, int stage, const IterArgs &ia, hipStream_t s)
{
    IterArgs a = ia;
    if constexpr (!GEN) {
        if (waves_simd == 3) {
            static std::atomic<int> resident3{0};  // this kernel's, once known
            const auto k = stage_march<P, NM, BDF, LS, 3, GEN, FIRST>;
            if (a.persist) persist_grid(g, a, b.x, resident_workgroups((const void *)k, b.x, resident3));
            hipLaunchKernelGGL(k, g, b, 0, s, tanks, units, sc, stage, a);
            return;
        }
    }
    static std::atomic<int> resident2{0};
    const auto k = stage_march<P, NM, BDF, LS, 2, GEN, FIRST>;
    if (a.persist) persist_grid(g, a, b.x, resident_workgroups((const void *)k, b.x, resident2));
    hipLaunchKernelGGL(k, g, b, 0, s, tanks, units, sc, stage, a);
}

template <class P, int BDF, bool GEN>
void launch_b(const TankDev *tanks, const MarchUnit *units, dim3 g, dim3 b, int waves_simd,
              const Scheme &sc, int stage, const IterArgs &ia, hipStream_t s)
{
    if (stage == sc.smax) {
        if (sc.norm_max) launch_t<P, true, BDF, true, GEN>(tanks, units, g, b, waves_simd, sc, stage, ia, s);
        else launch_t<P, false, BDF, true, GEN>(tanks, units, g, b, waves_simd, sc, stage, ia, s);
    } else {
        if constexpr (!P::kMixed && !GEN) {
            if (stage == 1) {
                launch_t<P, false, BDF, false, GEN, true>(tanks, units, g, b, waves_simd, sc, stage,
                                                          ia, s);
                return;
            }
        }
        launch_t<P, false, BDF, false, GEN>(tanks, units, g, b, waves_simd, sc, stage, ia, s);
    }
}

// One stage over the unit table, for the scheme's precision and BDF order.
// ia.fin (stage 1 only) puts workgroups in front of the unit table whose waves finalize the
// previous iteration, one tank each: ceil(n_tanks / waves_per_block) rounded up to a multiple of 8.
// ia.persist launches only the workgroups the chip holds at once (by the launched kernel's own
// occupancy), each wave looping over its share of the table (one persistent launch per stage).
template <bool GEN>
int launch(const TankDev *tanks, const MarchUnit *units, int n_entries, int waves_per_block,
           const Scheme &sc, int stage, const IterArgs &ia_in, int waves_simd, void *stream)
{
    if (waves_per_block < 1 || waves_per_block > kMaxWavesPerBlock || n_entries % waves_per_block)
        return (int)hipErrorInvalidValue;
    // the finalize waves read the partials of the previous iteration's last stage: stage 1 must
    // not be that stage, as its units write the partials in the same launch
    if (ia_in.fin && (stage != 1 || stage == sc.smax || ia_in.n_tanks < 1)) return (int)hipErrorInvalidValue;
    IterArgs ia = ia_in;
    const int fin_blocks = ia.fin ? ((ia.n_tanks + 8 * waves_per_block - 1) / (8 * waves_per_block)) * 8 : 0;
    ia.n_fin = fin_blocks * waves_per_block;
    ia.stride = 0;  // one wave per unit unless the launch below goes out persistent
    ia.n_entries = n_entries;
    const dim3 g(n_entries / waves_per_block + fin_blocks), b(kLanes * waves_per_block);
    hipStream_t s = (hipStream_t)stream;
    if (sc.mixed) {
        if (sc.bdf >= 3) launch_b<PrecMixed, 3, GEN>(tanks, units, g, b, waves_simd, sc, stage, ia, s);
        else if (sc.bdf == 2) launch_b<PrecMixed, 2, GEN>(tanks, units, g, b, waves_simd, sc, stage, ia, s);
        else launch_b<PrecMixed, 1, GEN>(tanks, units, g, b, waves_simd, sc, stage, ia, s);
    } else {
        if (sc.bdf >= 3) launch_b<PrecF64, 3, GEN>(tanks, units, g, b, waves_simd, sc, stage, ia, s);
        else if (sc.bdf == 2) launch_b<PrecF64, 2, GEN>(tanks, units, g, b, waves_simd, sc, stage, ia, s);
        else launch_b<PrecF64, 1, GEN>(tanks, units, g, b, waves_simd, sc, stage, ia, s);
    }
    return (int)hipGetLastError();
}

}  // namespace march

}  // namespace vdac
