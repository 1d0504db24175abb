// stage_tile.hip -- the Runge-Kutta stage kernel for gfx950 in its tiled form, FP64 or mixed
// precision (the policies of stage_common.h).
//
// One workgroup of 256, 320 or 512 threads updates one TX x TY tile of cells of a single tank in four
// phases separated by workgroup barriers:
//   1. the stage input Q^{s-1} of the tile and a two-cell halo is loaded once from memory and
//      kept in LDS as primitives (rho, u, v in the reconstruction precision, p in FP64), with the
//      cell flags of the tile and a one-cell ring;
//   2. every fluid cell of the tile and of the ring is reconstructed once: limited slopes of
//      rho, u, v (Sec. 2.3.1), the stage-0 sources from Q^0 and level n, and the new pressure
//      gradient (Sec. 2.3.2).  The cell writes its own state at each of its faces that belong to
//      the tile into that face's LDS slot; across a wall face (domain wall or solid neighbour) it
//      also writes the ghost's state into the opposite slot (Sec. 2.5).  Each slot therefore has
//      exactly one writer;
//   3. every face of the tile is evaluated once with the Osher-Dumbser-Toro flux (Sec. 2.4.3);
//      the flux overwrites the face's left/lower state slot;
//   4. each tile cell forms the flux divergence in FP64, adds the frozen sources and applies the
//      point-implicit update (eq. 24), and the last stage accumulates the residual.
// Mixed form: the state is stored as FP32 deviations from the FP64 level n; reconstruction and
// fluxes run in FP32 with every face pressure expressed from the pressure of the face's
// lower-index cell, and that reference (an FP64 difference) is added back in the divergence.
// Periodic sides are handled by wrapping halo indices; cells outside a non-periodic side read
// as non-fluid.
// GEN (the general options): the Roe or exact flux in place of Osher's (Sec. 2.4), the k-limiter
// or split limiter on p in place of the new pressure gradient (Sec. 2.3.2), zero-gradient sides
// (Sec. 3.1), one pseudo-time step per tank (the minimum local step, from the previous iteration's
// last stage), and BDF3 (Table 1).
#include <hip/hip_runtime.h>

#include "stage_common.h"

namespace vdac {

namespace {

// Index along one axis of a tile-relative position: wraps across a periodic side, or reports
// the position outside the tank.
__device__ __forceinline__ bool locate(int g, int n, int periodic, int &out)
{
    if (g < 0 || g >= n) {
        if (!periodic) return false;
        while (g < 0) g += n;
        while (g >= n) g -= n;
    }
    out = g;
    return true;
}

// Tile position of the pidx-th cell that phase 2 reconstructs: the tile cells first, then the
// ring around the tile without its corners (below, above, left, right).
template <int TX, int TY>
__device__ __forceinline__ void ring_position(int pidx, int &i, int &j)
{
    constexpr int NC = TX * TY;
    if (pidx < NC) {
        i = pidx % TX;
        j = pidx / TX;
        return;
    }
    const int q = pidx - NC;
    if (q < TX) {
        i = q;
        j = -1;
    } else if (q < 2 * TX) {
        i = q - TX;
        j = TY;
    } else if (q < 2 * TX + TY) {
        i = -1;
        j = q - 2 * TX;
    } else {
        i = TX;
        j = q - 2 * TX - TY;
    }
}

// Stage-0 data of one cell: Q^0 (rho, rho u, rho v; the mixed form keeps its deviation from
// level n), level n, level n-1 and level n-2.
struct SourceData {
    double z0, z1, z2, n0, n1, n2, m0, m1, m2, k0, k1, k2;
};

// Level n (and n-1 with BDF2, n-2 with BDF3) of cell c; these do not depend on the pseudo-loop
// status.
__device__ __forceinline__ void load_levels(const TankDev &t, size_t c, bool bdf2, bool bdf3,
                                            SourceData &s)
{
    const size_t plane = t.plane;
    s.n0 = t.level_n[c];
    s.n1 = t.level_n[plane + c];
    s.n2 = t.level_n[2 * plane + c];
    if (bdf2) {
        s.m0 = t.level_nm1[c];
        s.m1 = t.level_nm1[plane + c];
        s.m2 = t.level_nm1[2 * plane + c];
    } else {
        s.m0 = s.m1 = s.m2 = 0.0;
    }
    if (bdf3) {
        s.k0 = t.level_nm2[c];
        s.k1 = t.level_nm2[plane + c];
        s.k2 = t.level_nm2[2 * plane + c];
    } else {
        s.k0 = s.k1 = s.k2 = 0.0;
    }
}

template <class P>
__device__ __forceinline__ SourceData load_source(const TankDev &t, const typename P::Store *q0,
                                                  size_t c, bool bdf2, bool bdf3)
{
    const size_t plane = t.plane;
    SourceData s;
    s.z0 = (double)q0[c];
    s.z1 = (double)q0[plane + c];
    s.z2 = (double)q0[2 * plane + c];
    load_levels(t, c, bdf2, bdf3, s);
    return s;
}

// Stage-0 quantities of a cell from its SourceData: absolute Q^0 (a0 .. a2) and the real-time
// numerators B0 Q^0 + B1 Q^n + B2 Q^{n-1} + B3 Q^{n-2} (Table 1).  The mixed form uses
// B0 + B1 + B2 + B3 = 0: B0 (Q^0 - Q^n) + B2 (Q^{n-1} - Q^n) + B3 (Q^{n-2} - Q^n), with
// Q^0 - Q^n its stored deviation.
template <class P>
__device__ __forceinline__ void stage0_terms(const SourceData &sd, const StepParams &sp, bool bdf2,
                                             bool bdf3, double a[3], double num[3])
{
    const double z[3] = {sd.z0, sd.z1, sd.z2}, n[3] = {sd.n0, sd.n1, sd.n2},
                 m[3] = {sd.m0, sd.m1, sd.m2}, k2[3] = {sd.k0, sd.k1, sd.k2};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if constexpr (P::kMixed) {
            a[k] = n[k] + z[k];
            num[k] = sp.b0 * z[k];
            if (bdf2) num[k] = fma(sp.b2, m[k] - n[k], num[k]);
            if (bdf3) num[k] = fma(sp.b3, k2[k] - n[k], num[k]);
        } else {
            a[k] = z[k];
            num[k] = fma(sp.b0, z[k], sp.b1 * n[k]);
            if (bdf2) num[k] = fma(sp.b2, m[k], num[k]);
            if (bdf3) num[k] = fma(sp.b3, k2[k], num[k]);
        }
    }
}

// Residual partial of one tile in a fixed order (deterministic): each wave holding tile cells
// combines its lanes with the DPP tree (in VALU), then lane k of wave 0 combines the waves'
// results for value k and stores it.
template <bool NORM_MAX, int NC>
__device__ __forceinline__ void tile_reduce_store(double part[kPartialWidth], double *out)
{
    static_assert(NC % 64 == 0, "tile cells fill whole waves");
    __shared__ double red[NC / 64][kPartialWidth];
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    if (tid < NC) {
        auto sum = [](double a, double b) { return a + b; };
        auto mx = [](double a, double b) { return combine<true>(a, b); };
        auto mn = [](double a, double b) { return fmin(a, b); };
#pragma unroll
        for (int k = 0; k < kPartialWidth; ++k) {
            const double x = (k == 5) ? wave_reduce_to_lane63(part[k], INFINITY, mn)
                                      : ((NORM_MAX && k < 4) ? wave_reduce_to_lane63(part[k], 0.0, mx)
                                                             : wave_reduce_to_lane63(part[k], 0.0, sum));
            if (lane == 63) red[wave][k] = x;
        }
    }
    __syncthreads();
    if (tid < kPartialWidth) {
        const int k = tid;
        double x = red[0][k];
#pragma unroll
        for (int w = 1; w < NC / 64; ++w)
            x = (k == 5) ? fmin(x, red[w][k]) : ((NORM_MAX && k < 4) ? combine<true>(x, red[w][k]) : x + red[w][k]);
        out[k] = x;
    }
}

// Primitives of the stored cell c of a state buffer in the reconstruction precision, and its
// absolute pressure in FP64 (mixed form: level n plus the FP32 deviation).
template <class P>
__device__ __forceinline__ void load_cell(const TankDev &t, const typename P::Store *q, size_t c,
                                          Prim<typename P::Real> &w, double &p)
{
    const size_t plane = t.plane;
    if constexpr (P::kMixed) {
        const float r = (float)(t.level_n[c] + (double)q[c]);
        const float m = (float)(t.level_n[plane + c] + (double)q[plane + c]);
        const float n = (float)(t.level_n[2 * plane + c] + (double)q[2 * plane + c]);
        const float ir = rcp_pos(r);
        w = {r, m * ir, n * ir, 0.0f};
        p = t.level_n[3 * plane + c] + (double)q[3 * plane + c];
    } else {
        w = load_prim(q, plane, c);
        p = w.p;
    }
}

// NT threads per tile: 256 (one per tile cell) or 512 (every phase finishes in at most two
// rounds, which shortens the critical path of small grids).
// Whether the last wave of an NT-thread workgroup is idle in phases 1 and 2 (no primitive, flag
// or phase-2 position falls to it), so that it can run the deferred finalize there.
template <int TX, int TY, int NT>
__host__ __device__ constexpr bool fin_in_block()
{
    return NT == 512 && (TX + 4) * (TY + 4) <= NT - 64 && (TX + 2) * (TY + 2) <= NT - 64 &&
           TX * TY + 2 * (TX + TY) <= NT - 64;
}

// Launch bounds: NT threads, and for the mixed form's 16 x 8 tile of the default scheme a register
// budget that fits four workgroups (five waves per SIMD; the FP64 form reaches 96 VGPRs, five
// waves, without the bound, and spills with it).  GEN: the general options (file comment).
template <class P, int TX, int TY, int NT, bool NORM_MAX, bool GEN>
__global__ void __launch_bounds__(NT, (TX * TY == 128 && !GEN && P::kMixed ? 5 : 1))
    stage_tile(TankDev t, Scheme sc, int stage, int tiles_x, int n_tiles, IterArgs ia)
{
    using R = typename P::Real;
    using S = typename P::Store;
    constexpr int RX = TX + 4, RY = TY + 4, NR2 = RX * RY;  // primitives: tile + 2-cell halo
    constexpr int SX = TX + 2, SY = TY + 2, NR1 = SX * SY;  // flags: tile + 1-cell ring
    constexpr int NC = TX * TY;
    static_assert(NC <= NT, "at most one tile cell per thread");
    constexpr int NRING = 2 * (TX + TY);                    // ring positions without corners
    constexpr int NPOS = NC + NRING;
    constexpr int NFX = (TX + 1) * TY, NFY = TX * (TY + 1);

    __shared__ R sW[3][NR2];      // rho, u, v
    __shared__ double sP[NR2];    // absolute pressure
    __shared__ uint8_t sF[NR1];
    __shared__ R sXL[4][NFX], sXR[4][NFX];  // x-face states (then fluxes in sXL)
    __shared__ R sYL[4][NFY], sYU[4][NFY];  // y-face states (then fluxes in sYL)

    // The finalize of the previous iteration (stage-1 launches with ia.fin set): where the last
    // wave has no work in phases 1 and 2 (512 threads), that wave of workgroup 0 runs it between
    // the first two barriers; otherwise 8 workgroups go in front of the tiles (8 keeps each tile
    // on the same XCD as in the other stages), the first of which runs it, dispatched before any
    // tile so that it does not trail the launch.
    constexpr bool kFinInBlock = fin_in_block<TX, TY, NT>();
    int bid = (int)blockIdx.x;
    if (ia.fin && !kFinInBlock) {
        if (bid < 8) {
            if (bid == 0 && threadIdx.x < 64) finalize_wave(t, sc, threadIdx.x);
            return;
        }
        bid -= 8;
    }
    // XCD-aware tile order: the hardware hands block b to XCD b % 8; each XCD gets a contiguous
    // run of tiles so that neighbouring tiles, which share halo cells, share an L2.
    const int per = (n_tiles + 7) >> 3;
    const int tile = (bid & 7) * per + (bid >> 3);
    if (tile >= n_tiles) return;
    const int x0 = (tile % tiles_x) * TX;
    const int y0 = (tile / tiles_x) * TY;
    const int tid = threadIdx.x;
    const size_t plane = t.plane;
    const bool slip = sc.slip != 0;
    const R k = (R)sc.k;

    // ---- phase 1: every global load of the stage is issued here --------------------------
    // The cell flags and the real-time levels of this thread's first phase-2 cell go first.
    constexpr int NFL = (NR1 + NT - 1) / NT;
    uint8_t fl[NFL];
#pragma unroll
    for (int q = 0; q < NFL; ++q) {
        const int r = tid + q * NT;
        const int ri = r % SX, rj = r / SX;
        int gi, gj;
        fl[q] = FLAG_SOLID;  // outside a non-periodic side: not a fluid cell
        if (r < NR1 && locate(x0 - 1 + ri, t.nx, t.per_x, gi) && locate(y0 - 1 + rj, t.ny, t.per_y, gj))
            fl[q] = t.flags[(size_t)gj * t.nx + gi];
    }
    const StepParams sp = *t.step;
    const bool bdf2 = sp.b2 != 0.0;
    const bool bdf3 = GEN && sp.b3 != 0.0;
    SourceData src0 = {P::kMixed ? 0.0 : 1.0, 0.0, 0.0, 1.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    size_t own_c = ~(size_t)0;  // this thread's first phase-2 cell, if inside the tank
    if (tid < NPOS) {
        int i, j, gi, gj;
        ring_position<TX, TY>(tid, i, j);
        if (locate(x0 + i, t.nx, t.per_x, gi) && locate(y0 + j, t.ny, t.per_y, gj)) {
            own_c = (size_t)gj * t.nx + gi;
            load_levels(t, own_c, bdf2, bdf3, src0);
        }
    }

    // the buffers follow from the iteration (IterArgs); the stop flag is tested once the loads
    // below are in flight, so that its latency overlaps theirs
    const int stopped = t.status->done;
    const double dtau_glob = (GEN && sc.global_dtau) ? t.status->dtau_global : 0.0;
    const int cur = ia.cur_off;
    const StageBuffers bufs = stage_buffers(cur, stage);
    const S *qprev = (const S *)t.state[bufs.in];
    const S *q0 = (const S *)t.state[cur];
    S *qout = (S *)t.state[bufs.out];

    for (int r = tid; r < NR2; r += NT) {
        const int ri = r % RX, rj = r / RX;
        int gi, gj;
        Prim<R> w = {R(1), R(0), R(0), R(0)};
        double p = 0.0;
        if (locate(x0 - 2 + ri, t.nx, t.per_x, gi) && locate(y0 - 2 + rj, t.ny, t.per_y, gj))
            load_cell<P>(t, qprev, (size_t)gj * t.nx + gi, w, p);
        sW[0][r] = w.r;
        sW[1][r] = w.u;
        sW[2][r] = w.v;
        sP[r] = p;
    }
    // Q^0 of this thread's first phase-2 cell (and its pressure, or pressure deviation, for the
    // tile cell's update)
    double own_p0 = 0.0;
    if (own_c != ~(size_t)0) {
        src0.z0 = (double)q0[own_c];
        src0.z1 = (double)q0[plane + own_c];
        src0.z2 = (double)q0[2 * plane + own_c];
        if (tid < NC) own_p0 = (double)q0[3 * plane + own_c];
    }
    if (stopped) return;
#pragma unroll
    for (int q = 0; q < NFL; ++q)
        if (tid + q * NT < NR1) sF[tid + q * NT] = fl[q];
    __syncthreads();
    if constexpr (kFinInBlock) {
        if (ia.fin && bid == 0 && tid >= NT - 64) finalize_wave(t, sc, tid - (NT - 64));
    }

    // ---- phase 2: reconstruction of the tile and ring cells --------------------------------
    // The tile cell of this thread keeps its stage-0 data for phase 4 (mixed form: also the
    // references sx, sy of its left and lower faces, and its level-n density).
    double own_a[3] = {1.0, 0.0, 0.0}, own_z[3] = {0.0, 0.0, 0.0}, own_d[3] = {0.0, 0.0, 0.0};
    double own_sx = 0.0, own_sy = 0.0, own_lvl = 0.0, own_lvl_m = 0.0, own_lvl_n = 0.0;

    for (int pidx = tid; pidx < NPOS; pidx += NT) {
        int i, j;
        ring_position<TX, TY>(pidx, i, j);
        const uint8_t f = sF[(j + 1) * SX + (i + 1)];
        if (f & FLAG_SOLID) continue;
        const int r = (j + 2) * RX + (i + 2);
        CellRecT<R> rec;
        rec.w = {sW[0][r], sW[1][r], sW[2][r], P::kMixed ? R(0) : (R)sP[r]};
        // zero-gradient sides (general options): the cell's faces on the tank's open sides
        const bool open_xm = GEN && x0 + i == 0 && (t.open & 1);
        const bool open_xp = GEN && x0 + i == t.nx - 1 && (t.open & 2);
        const bool open_ym = GEN && y0 + j == 0 && (t.open & 4);
        const bool open_yp = GEN && y0 + j == t.ny - 1 && (t.open & 8);
        // a wall face shows the cell its own mirror image (Sec. 2.5), a zero-gradient face the
        // cell itself
        const Prim<R> xm = (f & FLAG_WALL_XM) ? (open_xm ? rec.w : mirror(rec.w, 0, slip))
                                              : Prim<R>{sW[0][r - 1], sW[1][r - 1], sW[2][r - 1], R(0)};
        const Prim<R> xp = (f & FLAG_WALL_XP) ? (open_xp ? rec.w : mirror(rec.w, 0, slip))
                                              : Prim<R>{sW[0][r + 1], sW[1][r + 1], sW[2][r + 1], R(0)};
        const Prim<R> ym = (f & FLAG_WALL_YM) ? (open_ym ? rec.w : mirror(rec.w, 1, slip))
                                              : Prim<R>{sW[0][r - RX], sW[1][r - RX], sW[2][r - RX], R(0)};
        const Prim<R> yp = (f & FLAG_WALL_YP) ? (open_yp ? rec.w : mirror(rec.w, 1, slip))
                                              : Prim<R>{sW[0][r + RX], sW[1][r + RX], sW[2][r + RX], R(0)};
        rec.gx = slopes(xm, rec.w, xp, (R)t.inv_dx, k);
        rec.gy = slopes(ym, rec.w, yp, (R)t.inv_dy, k);

        // stage-0 sources: real-time term and rho^0
        SourceData sd = src0;
        if (pidx != tid) {  // later rounds (256-thread tiles) load here
            int gi, gj;
            locate(x0 + i, t.nx, t.per_x, gi);
            locate(y0 + j, t.ny, t.per_y, gj);
            sd = load_source<P>(t, q0, (size_t)gj * t.nx + gi, bdf2, bdf3);
        }
        double a[3], num[3];
        stage0_terms<P>(sd, sp, bdf2, bdf3, a, num);
        const double d_r = num[0] * sp.inv_dt, d_ru = num[1] * sp.inv_dt, d_rv = num[2] * sp.inv_dt;
        rec.d_r = (R)d_r;
        rec.d_ru = (R)d_ru;
        rec.d_rv = (R)d_rv;
        rec.rho0 = (R)a[0];
        // pressure each face state is expressed from: the cell's own p (FP64 form), or p minus
        // the pressure of the face's lower-index cell (mixed form; sx, sy go back in in phase 4)
        double sx = 0.0, sy = 0.0;
        R pb_own = rec.w.p, pb_xl = rec.w.p, pb_yb = rec.w.p;
        if constexpr (P::kMixed) {
            sx = (f & FLAG_WALL_XM) ? 0.0 : sP[r] - sP[r - 1];
            sy = (f & FLAG_WALL_YM) ? 0.0 : sP[r] - sP[r - RX];
            pb_own = R(0);
            pb_xl = (R)sx;
            pb_yb = (R)sy;
        }
        if (pidx < NC) {
            own_a[0] = a[0];
            own_a[1] = a[1];
            own_a[2] = a[2];
            own_z[0] = sd.z0;
            own_z[1] = sd.z1;
            own_z[2] = sd.z2;
            own_d[0] = d_r;
            own_d[1] = d_ru;
            own_d[2] = d_rv;
            own_sx = sx;
            own_sy = sy;
            own_lvl = sd.n0;
            own_lvl_m = sd.n1;
            own_lvl_n = sd.n2;
        }

        // the cell's pressure gradient: the new method, or (general options) the k-limiter or
        // split limiter on p, whose stencil sees the cell's own p across a wall or open face
        R px = R(0), py = R(0);
        FaceStatesT<R> fs;
        if constexpr (GEN) {
            if (sc.pgrad != 0) {
                const double pm = sP[r];
                const double dpr_x = (f & FLAG_WALL_XP) ? 0.0 : sP[r + 1] - pm;
                const double dpl_x = (f & FLAG_WALL_XM) ? 0.0 : pm - sP[r - 1];
                const double dpr_y = (f & FLAG_WALL_YP) ? 0.0 : sP[r + RX] - pm;
                const double dpl_y = (f & FLAG_WALL_YM) ? 0.0 : pm - sP[r - RX];
                px = (R)pgrad_limited(sc.pgrad, sc.pk, dpr_x, dpl_x, t.inv_dx, (double)xm.r,
                                      (double)rec.w.r, (double)xp.r, t.gx);
                py = (R)pgrad_limited(sc.pgrad, sc.pk, dpr_y, dpl_y, t.inv_dy, (double)ym.r,
                                      (double)rec.w.r, (double)yp.r, t.gy);
            } else {
                px = cell_gradp_x(t, rec);
                py = cell_gradp_y(t, rec);
            }
            const R hx = (R)t.half_dx, hy = (R)t.half_dy;
            fs.xl = state_at(rec.w, rec.gx, px, -hx, pb_xl);
            fs.xr = state_at(rec.w, rec.gx, px, hx, pb_own);
            fs.yb = state_at(rec.w, rec.gy, py, -hy, pb_yb);
            fs.yt = state_at(rec.w, rec.gy, py, hy, pb_own);
        } else {
            fs = face_states<R>(t, rec, pb_xl, pb_own, pb_yb, pb_own);
        }
        const bool row_in = (j >= 0 && j < TY), col_in = (i >= 0 && i < TX);
        if (row_in) {
            if (i >= 0) {  // left face i of the tile's x-faces
                const int fi = j * (TX + 1) + i;
                const Prim<R> s = fs.xl;
                sXR[0][fi] = s.r; sXR[1][fi] = s.u; sXR[2][fi] = s.v; sXR[3][fi] = s.p;
                if (f & FLAG_WALL_XM) {
                    const Prim<R> gs = GEN ? ghost_state_gen<R>(t, sc, rec, 0, -1, open_xm, px, pb_own)
                                           : ghost_state<R>(t, rec, 0, -1, slip, pb_own);
                    sXL[0][fi] = gs.r; sXL[1][fi] = gs.u; sXL[2][fi] = gs.v; sXL[3][fi] = gs.p;
                }
            }
            if (i < TX) {  // right face i + 1
                const int fi = j * (TX + 1) + i + 1;
                const Prim<R> s = fs.xr;
                sXL[0][fi] = s.r; sXL[1][fi] = s.u; sXL[2][fi] = s.v; sXL[3][fi] = s.p;
                if (f & FLAG_WALL_XP) {
                    const Prim<R> gs = GEN ? ghost_state_gen<R>(t, sc, rec, 0, +1, open_xp, px, pb_own)
                                           : ghost_state<R>(t, rec, 0, +1, slip, pb_own);
                    sXR[0][fi] = gs.r; sXR[1][fi] = gs.u; sXR[2][fi] = gs.v; sXR[3][fi] = gs.p;
                }
            }
        }
        if (col_in) {
            if (j >= 0) {  // lower face j of the tile's y-faces
                const int fi = j * TX + i;
                const Prim<R> s = fs.yb;
                sYU[0][fi] = s.r; sYU[1][fi] = s.u; sYU[2][fi] = s.v; sYU[3][fi] = s.p;
                if (f & FLAG_WALL_YM) {
                    const Prim<R> gs = GEN ? ghost_state_gen<R>(t, sc, rec, 1, -1, open_ym, py, pb_own)
                                           : ghost_state<R>(t, rec, 1, -1, slip, pb_own);
                    sYL[0][fi] = gs.r; sYL[1][fi] = gs.u; sYL[2][fi] = gs.v; sYL[3][fi] = gs.p;
                }
            }
            if (j < TY) {  // upper face j + 1
                const int fi = (j + 1) * TX + i;
                const Prim<R> s = fs.yt;
                sYL[0][fi] = s.r; sYL[1][fi] = s.u; sYL[2][fi] = s.v; sYL[3][fi] = s.p;
                if (f & FLAG_WALL_YP) {
                    const Prim<R> gs = GEN ? ghost_state_gen<R>(t, sc, rec, 1, +1, open_yp, py, pb_own)
                                           : ghost_state<R>(t, rec, 1, +1, slip, pb_own);
                    sYU[0][fi] = gs.r; sYU[1][fi] = gs.u; sYU[2][fi] = gs.v; sYU[3][fi] = gs.p;
                }
            }
        }
    }
    __syncthreads();

    // ---- phase 3: one flux per face (Osher's, or with the general options Roe's or the exact) -
    const R beta = (R)t.beta, inv_beta = (R)t.inv_beta;
    for (int fidx = tid; fidx < NFX + NFY; fidx += NT) {
        if (fidx < NFX) {
            const int fi = fidx % (TX + 1), j = fidx / (TX + 1);
            const uint8_t fl_ = sF[(j + 1) * SX + fi], fr = sF[(j + 1) * SX + fi + 1];
            if ((fl_ & FLAG_SOLID) && (fr & FLAG_SOLID)) continue;
            const Prim<R> L = {sXL[0][fidx], sXL[1][fidx], sXL[2][fidx], sXL[3][fidx]};
            const Prim<R> Rt = {sXR[0][fidx], sXR[1][fidx], sXR[2][fidx], sXR[3][fidx]};
            const Vec4<R> F = GEN ? flux_x(sc.flux, L, Rt, beta, inv_beta) : osher_x(L, Rt, beta, inv_beta);
            sXL[0][fidx] = F.a; sXL[1][fidx] = F.b; sXL[2][fidx] = F.c; sXL[3][fidx] = F.d;
        } else {
            const int q = fidx - NFX;
            const int i = q % TX, g = q / TX;
            const uint8_t fb = sF[g * SX + i + 1], fu = sF[(g + 1) * SX + i + 1];
            if ((fb & FLAG_SOLID) && (fu & FLAG_SOLID)) continue;
            const Prim<R> L = {sYL[0][q], sYL[1][q], sYL[2][q], sYL[3][q]};
            const Prim<R> U = {sYU[0][q], sYU[1][q], sYU[2][q], sYU[3][q]};
            const Vec4<R> F = GEN ? flux_y(sc.flux, L, U, beta, inv_beta) : osher_y(L, U, beta, inv_beta);
            sYL[0][q] = F.a; sYL[1][q] = F.b; sYL[2][q] = F.c; sYL[3][q] = F.d;
        }
    }
    __syncthreads();

    // ---- phase 4: divergence, sources and the point-implicit update ------------------------
    const double alpha = sc.alpha[stage - 1];
    const bool last = (stage == sc.smax);
    double part[kPartialWidth] = {0.0, 0.0, 0.0, 0.0, 0.0, INFINITY};
    constexpr size_t kNoCell = ~(size_t)0;
    size_t out_c = kNoCell;  // this thread's updated cell, if any, and its new state
    double out[4] = {0.0, 0.0, 0.0, 0.0};
    if (tid < NC) {
        const int i = tid % TX, j = tid / TX;
        const int gi = x0 + i, gj = y0 + j;
        const uint8_t f = sF[(j + 1) * SX + (i + 1)];
        if (gi < t.nx && gj < t.ny && !(f & FLAG_SOLID)) {
            const size_t c = (size_t)gj * t.nx + gi;
            const int xm = j * (TX + 1) + i, ym = j * TX + i;
            double R4[4];
            const double fdx = t.flux_dx, fdy = t.flux_dy;  // 1/(2h): the faces hold twice the flux
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const double div = ((double)sXL[m][xm + 1] - (double)sXL[m][xm]) * fdx
                                   + ((double)sYL[m][ym + TX] - (double)sYL[m][ym]) * fdy;
                R4[m] = -div;
            }
            if constexpr (P::kMixed) {  // the face pressures' references
                R4[1] = fma(-own_sx, t.inv_dx, R4[1]);
                R4[2] = fma(-own_sy, t.inv_dy, R4[2]);
            }
            const double r0 = own_a[0];
            R4[0] += -own_d[0];
            R4[1] += -own_d[1] + r0 * t.gx;
            R4[2] += -own_d[2] + r0 * t.gy;
            const double dtau = (GEN && sc.global_dtau) ? dtau_glob
                                : (P::kMixed ? local_dtau_f32(t, t.cfl, r0, own_a[1], own_a[2])
                                             : local_dtau(t, t.cfl, r0, own_a[1], own_a[2]));
            const double ad = alpha * dtau;
            const double api = 1.0 + sp.b0 * ad * sp.inv_dt;
            const double fac = ad * rcp_pos(api);
            out_c = c;
            out[0] = own_z[0] + fac * R4[0];
            out[1] = own_z[1] + fac * R4[1];
            out[2] = own_z[2] + fac * R4[2];
            out[3] = own_p0 + t.beta * (ad * R4[3]);
            if (last) {
                const double rp = t.beta * R4[3];
                if (NORM_MAX) {
                    part[0] = fabs(R4[0]);
                    part[1] = fabs(R4[1]);
                    part[2] = fabs(R4[2]);
                    part[3] = fabs(rp);
                } else {
                    part[0] = R4[0] * R4[0];
                    part[1] = R4[1] * R4[1];
                    part[2] = R4[2] * R4[2];
                    part[3] = rp * rp;
                }
                const double rho_new = P::kMixed ? own_lvl + out[0] : out[0];
                part[4] = (rho_new > 0.0 && rho_new < INFINITY) ? 0.0 : 1.0;
                if (GEN && sc.global_dtau && rho_new > 0.0) {
                    // pseudo-time step of the updated state: the next iteration's stage 0
                    const double m_new = out[1] + (P::kMixed ? own_lvl_m : 0.0);
                    const double n_new = out[2] + (P::kMixed ? own_lvl_n : 0.0);
                    part[5] = local_dtau(t, t.cfl, rho_new, m_new, n_new);
                }
            }
        }
    }
    // the residual is reduced before the state is stored: the workgroup barrier of the reduction
    // would otherwise wait for the stores to complete
    if (last) tile_reduce_store<NORM_MAX, NC>(part, t.partials + (size_t)tile * kPartialWidth);
    if (out_c != kNoCell) {
        qout[out_c] = (S)out[0];
        qout[plane + out_c] = (S)out[1];
        qout[2 * plane + out_c] = (S)out[2];
        qout[3 * plane + out_c] = (S)out[3];
    }
}

template <class P, int TX, int TY, int NT, bool GEN>
int launch_tile(const TankDev &t, const Scheme &sc, int stage, const IterArgs &ia, void *stream)
{
    const int tiles_x = (t.nx + TX - 1) / TX, tiles_y = (t.ny + TY - 1) / TY;
    const int n_tiles = tiles_x * tiles_y;
    const int blocks = ((n_tiles + 7) / 8) * 8 + (ia.fin && !fin_in_block<TX, TY, NT>() ? 8 : 0);
    if (sc.norm_max)
        hipLaunchKernelGGL((stage_tile<P, TX, TY, NT, true, GEN>), dim3(blocks), dim3(NT), 0,
                           (hipStream_t)stream, t, sc, stage, tiles_x, n_tiles, ia);
    else
        hipLaunchKernelGGL((stage_tile<P, TX, TY, NT, false, GEN>), dim3(blocks), dim3(NT), 0,
                           (hipStream_t)stream, t, sc, stage, tiles_x, n_tiles, ia);
    return (int)hipGetLastError();
}

template <class P, bool GEN>
int launch_tile_p(const TankDev &t, const Scheme &sc, int stage, int tile_x, int tile_y,
                  const IterArgs &ia, void *stream)
{
    if (tile_x == 32 && tile_y == 8) return launch_tile<P, 32, 8, 256, GEN>(t, sc, stage, ia, stream);
    if (tile_x == 16 && tile_y == 16) return launch_tile<P, 16, 16, 256, GEN>(t, sc, stage, ia, stream);
    if (tile_x == 64 && tile_y == 4) return launch_tile<P, 64, 4, 256, GEN>(t, sc, stage, ia, stream);
    if (tile_x == 3208 && tile_y == 2) return launch_tile<P, 32, 8, 512, GEN>(t, sc, stage, ia, stream);
    if (tile_x == 1616 && tile_y == 2) return launch_tile<P, 16, 16, 512, GEN>(t, sc, stage, ia, stream);
    if (tile_x == 1608 && tile_y == 2) return launch_tile<P, 16, 8, 320, GEN>(t, sc, stage, ia, stream);
    return (int)hipErrorInvalidValue;
}

}  // namespace

// 32 x 8, 16 x 16 and 64 x 4 tiles run with 256 threads; 3208 and 1616 name the 32 x 8 and
// 16 x 16 tiles run with 512 threads, 1608 the 16 x 8 tile with 320 threads (tile_y 2 for all
// three).
bool tile_supported(int tile_x, int tile_y)
{
    return (tile_x == 32 && tile_y == 8) || (tile_x == 16 && tile_y == 16) ||
           (tile_x == 64 && tile_y == 4) || (tile_x == 3208 && tile_y == 2) ||
           (tile_x == 1616 && tile_y == 2) || (tile_x == 1608 && tile_y == 2);
}

int tile_count(const TankDev &t, int tile_x, int tile_y)
{
    if (tile_x == 3208) tile_x = 32, tile_y = 8;
    if (tile_x == 1616) tile_x = 16, tile_y = 16;
    if (tile_x == 1608) tile_x = 16, tile_y = 8;
    return ((t.nx + tile_x - 1) / tile_x) * ((t.ny + tile_y - 1) / tile_y);
}

int launch_stage_tile(const TankDev &t, const Scheme &sc, int stage, int tile_x, int tile_y,
                      const IterArgs &ia, void *stream)
{
    // the finalize reads the partials of the previous iteration's last stage, which stage 1 would
    // overwrite in the same launch if it were the last stage
    if (ia.fin && (stage != 1 || stage == sc.smax)) return (int)hipErrorInvalidValue;
    // the general options and BDF3 run in the GEN instances
    if (sc.general || sc.bdf > 2)
        return sc.mixed ? launch_tile_p<PrecMixed, true>(t, sc, stage, tile_x, tile_y, ia, stream)
                        : launch_tile_p<PrecF64, true>(t, sc, stage, tile_x, tile_y, ia, stream);
    return sc.mixed ? launch_tile_p<PrecMixed, false>(t, sc, stage, tile_x, tile_y, ia, stream)
                    : launch_tile_p<PrecF64, false>(t, sc, stage, tile_x, tile_y, ia, stream);
}

}  // namespace vdac
