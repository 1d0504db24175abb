// stage_tile.hip -- the Runge-Kutta stage kernel for gfx950 in its tiled form.
//
// One 256-thread workgroup updates one TX x TY tile of cells in four phases separated by
// workgroup barriers:
//   1. the stage input Q^{s-1} of the tile and a two-cell halo is loaded once from memory and
//      kept in LDS as primitives (rho, u, v, p), with the cell flags of the tile and a one-cell
//      ring;
//   2. every fluid cell of the tile and of the ring is reconstructed once: limited slopes of
//      rho, u, v (Sec. 2.3.1), the stage-0 sources from Q^0 and level n, and the new pressure
//      gradient (Sec. 2.3.2).  The cell writes its own state at each of its faces that belong to
//      the tile into that face's LDS slot; across a wall face (domain wall or solid neighbour) it
//      also writes the ghost's state into the opposite slot (Sec. 2.5).  Each slot therefore has
//      exactly one writer;
//   3. every face of the tile is evaluated once with the Osher-Dumbser-Toro flux (Sec. 2.4.3);
//      the flux overwrites the face's left/lower state slot;
//   4. each tile cell forms the flux divergence, adds the frozen sources and applies the
//      point-implicit update (eq. RK2), and the last stage accumulates the residual.
// Periodic sides are handled by wrapping halo indices; cells outside a non-periodic side read
// as non-fluid.
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

// Stage-0 data of one cell: Q^0 (rho, rho u, rho v), level n and level n-1.
struct SourceData {
    double z0, z1, z2, n0, n1, n2, m0, m1, m2;
};

// Level n (and n-1 with BDF2) of cell c; these do not depend on the pseudo-loop status.
__device__ __forceinline__ void load_levels(const TankDev &t, size_t c, bool bdf2, SourceData &s)
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
}

__device__ __forceinline__ SourceData load_source(const TankDev &t, const double *q0, size_t c,
                                                  bool bdf2)
{
    const size_t plane = t.plane;
    SourceData s;
    s.z0 = q0[c];
    s.z1 = q0[plane + c];
    s.z2 = q0[2 * plane + c];
    load_levels(t, c, bdf2, s);
    return s;
}

// Residual partial of one tile in a fixed order (deterministic): each tile cell's six values go
// to LDS, then value k is combined by lanes 8k .. 8k+7 of wave 0, each over NC/8 cells, and a DPP
// tree within those 8 lanes combines them; lane 8k+7 stores value k.  Only wave 0 works after the
// barrier, and no lane exchange goes through LDS.
template <bool NORM_MAX, int NC>
__device__ __forceinline__ void tile_reduce_store(const double part[kPartialWidth], double *scratch,
                                                  double *out)
{
    static_assert(NC % 8 == 0, "eight lanes per value");
    const int tid = threadIdx.x;
    if (tid < NC)
#pragma unroll
        for (int k = 0; k < kPartialWidth; ++k) scratch[k * NC + tid] = part[k];
    __syncthreads();
    if (tid < 8 * kPartialWidth) {
        const int k = tid >> 3, l = tid & 7;
        const bool mn = k == 5;               // minimum pseudo-time step
        const bool mx = NORM_MAX && k < 4;    // maximum norm
        const double id = mn ? INFINITY : 0.0;
        auto op = [&](double a, double b) { return mn ? fmin(a, b) : (mx ? combine<true>(a, b) : a + b); };
        double x = scratch[k * NC + l];
#pragma unroll
        for (int j = 1; j < NC / 8; ++j) x = op(x, scratch[k * NC + l + 8 * j]);
        // row shifts stay within rows of 16 lanes; lane 8k+7 only ever combines lanes 8k .. 8k+7
        x = op(x, dpp_row_shr<1>(id, x));
        x = op(x, dpp_row_shr<2>(id, x));
        x = op(x, dpp_row_shr<4>(id, x));
        if (l == 7) out[k] = x;
    }
}

// NT threads per tile: 256 (one per tile cell) or 512 (every phase finishes in at most two
// rounds, which shortens the critical path of small grids).
template <int TX, int TY, int NT, bool NORM_MAX>
__global__ void __launch_bounds__(NT) stage_tile_f64(TankDev t, Scheme sc, int stage, int tiles_x,
                                                     int n_tiles, IterArgs ia)
{
    constexpr int RX = TX + 4, RY = TY + 4, NR2 = RX * RY;  // primitives: tile + 2-cell halo
    constexpr int SX = TX + 2, SY = TY + 2, NR1 = SX * SY;  // flags: tile + 1-cell ring
    constexpr int NC = TX * TY;
    static_assert(NC <= NT, "at most one tile cell per thread");
    static_assert(kPartialWidth * NC <= 4 * NR2, "the residual reduction reuses the primitives' LDS");
    constexpr int NRING = 2 * (TX + TY);                    // ring positions without corners
    constexpr int NPOS = NC + NRING;
    constexpr int NFX = (TX + 1) * TY, NFY = TX * (TY + 1);

    __shared__ double sW[4][NR2];
    __shared__ uint8_t sF[NR1];
    __shared__ double sXL[4][NFX], sXR[4][NFX];  // x-face states (then fluxes in sXL)
    __shared__ double sYL[4][NFY], sYU[4][NFY];  // y-face states (then fluxes in sYL)

    // A stage-1 launch with ia.fin set puts 8 workgroups in front of the tiles (8 keeps each
    // tile on the same XCD as in the other stages); the first finalizes the previous iteration,
    // dispatched before any tile so that it does not trail the launch.
    int bid = (int)blockIdx.x;
    if (ia.fin) {
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
    const double k = sc.k;

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
    SourceData src0 = {1.0, 0.0, 0.0, 1.0, 0.0, 0.0, 1.0, 0.0, 0.0};
    size_t own_c = ~(size_t)0;  // this thread's first phase-2 cell, if inside the tank
    if (tid < NPOS) {
        int i, j, gi, gj;
        ring_position<TX, TY>(tid, i, j);
        if (locate(x0 + i, t.nx, t.per_x, gi) && locate(y0 + j, t.ny, t.per_y, gj)) {
            own_c = (size_t)gj * t.nx + gi;
            load_levels(t, own_c, bdf2, src0);
        }
    }

    // the buffers follow from the iteration (IterArgs); the stop flag is tested once the loads
    // below are in flight, so that its latency overlaps theirs
    const int stopped = t.status->done;
    const int cur = ia.cur_off;
    const StageBuffers bufs = stage_buffers(cur, stage);
    const double *qprev = (const double *)t.state[bufs.in];
    const double *q0 = (const double *)t.state[cur];
    double *qout = (double *)t.state[bufs.out];

    for (int r = tid; r < NR2; r += NT) {
        const int ri = r % RX, rj = r / RX;
        int gi, gj;
        Prim<double> w = {1.0, 0.0, 0.0, 0.0};
        if (locate(x0 - 2 + ri, t.nx, t.per_x, gi) && locate(y0 - 2 + rj, t.ny, t.per_y, gj))
            w = load_prim(qprev, plane, (size_t)gj * t.nx + gi);
        sW[0][r] = w.r;
        sW[1][r] = w.u;
        sW[2][r] = w.v;
        sW[3][r] = w.p;
    }
    // Q^0 of this thread's first phase-2 cell (and its pressure for the tile cell's update)
    double own_p0 = 0.0;
    if (own_c != ~(size_t)0) {
        src0.z0 = q0[own_c];
        src0.z1 = q0[plane + own_c];
        src0.z2 = q0[2 * plane + own_c];
        if (tid < NC) own_p0 = q0[3 * plane + own_c];
    }
    if (stopped) return;
#pragma unroll
    for (int q = 0; q < NFL; ++q)
        if (tid + q * NT < NR1) sF[tid + q * NT] = fl[q];
    __syncthreads();

    // ---- phase 2: reconstruction of the tile and ring cells --------------------------------
    // The tile cell of this thread keeps its stage-0 data for phase 4.
    double own_q0[3] = {1.0, 0.0, 0.0}, own_d[3] = {0.0, 0.0, 0.0};

    for (int pidx = tid; pidx < NPOS; pidx += NT) {
        int i, j;
        ring_position<TX, TY>(pidx, i, j);
        const uint8_t f = sF[(j + 1) * SX + (i + 1)];
        if (f & FLAG_SOLID) continue;
        const int r = (j + 2) * RX + (i + 2);
        CellRec rec;
        rec.w = {sW[0][r], sW[1][r], sW[2][r], sW[3][r]};
        // a wall face shows the cell its own mirror image (Sec. 2.5)
        const Prim<double> xm = (f & FLAG_WALL_XM) ? mirror(rec.w, 0, slip)
                                                   : Prim<double>{sW[0][r - 1], sW[1][r - 1], sW[2][r - 1], 0.0};
        const Prim<double> xp = (f & FLAG_WALL_XP) ? mirror(rec.w, 0, slip)
                                                   : Prim<double>{sW[0][r + 1], sW[1][r + 1], sW[2][r + 1], 0.0};
        const Prim<double> ym = (f & FLAG_WALL_YM) ? mirror(rec.w, 1, slip)
                                                   : Prim<double>{sW[0][r - RX], sW[1][r - RX], sW[2][r - RX], 0.0};
        const Prim<double> yp = (f & FLAG_WALL_YP) ? mirror(rec.w, 1, slip)
                                                   : Prim<double>{sW[0][r + RX], sW[1][r + RX], sW[2][r + RX], 0.0};
        rec.gx = slopes(xm, rec.w, xp, t.inv_dx, k);
        rec.gy = slopes(ym, rec.w, yp, t.inv_dy, k);

        // stage-0 sources: real-time term (B0 Q^0 + B1 Q^n + B2 Q^{n-1})/dt and rho^0
        SourceData sd = src0;
        if (pidx != tid) {  // later rounds (256-thread tiles) load here
            int gi, gj;
            locate(x0 + i, t.nx, t.per_x, gi);
            locate(y0 + j, t.ny, t.per_y, gj);
            sd = load_source(t, q0, (size_t)gj * t.nx + gi, bdf2);
        }
        double num0 = fma(sp.b0, sd.z0, sp.b1 * sd.n0);
        double num1 = fma(sp.b0, sd.z1, sp.b1 * sd.n1);
        double num2 = fma(sp.b0, sd.z2, sp.b1 * sd.n2);
        if (bdf2) {
            num0 = fma(sp.b2, sd.m0, num0);
            num1 = fma(sp.b2, sd.m1, num1);
            num2 = fma(sp.b2, sd.m2, num2);
        }
        rec.d_r = num0 * sp.inv_dt;
        rec.d_ru = num1 * sp.inv_dt;
        rec.d_rv = num2 * sp.inv_dt;
        rec.rho0 = sd.z0;
        if (pidx < NC) {
            own_q0[0] = sd.z0;
            own_q0[1] = sd.z1;
            own_q0[2] = sd.z2;
            own_d[0] = rec.d_r;
            own_d[1] = rec.d_ru;
            own_d[2] = rec.d_rv;
        }

        const FaceStates fs = face_states(t, rec);
        const bool row_in = (j >= 0 && j < TY), col_in = (i >= 0 && i < TX);
        if (row_in) {
            if (i >= 0) {  // left face i of the tile's x-faces
                const int fi = j * (TX + 1) + i;
                const Prim<double> s = fs.xl;
                sXR[0][fi] = s.r; sXR[1][fi] = s.u; sXR[2][fi] = s.v; sXR[3][fi] = s.p;
                if (f & FLAG_WALL_XM) {
                    const Prim<double> gs = ghost_state(t, rec, 0, -1, slip);
                    sXL[0][fi] = gs.r; sXL[1][fi] = gs.u; sXL[2][fi] = gs.v; sXL[3][fi] = gs.p;
                }
            }
            if (i < TX) {  // right face i + 1
                const int fi = j * (TX + 1) + i + 1;
                const Prim<double> s = fs.xr;
                sXL[0][fi] = s.r; sXL[1][fi] = s.u; sXL[2][fi] = s.v; sXL[3][fi] = s.p;
                if (f & FLAG_WALL_XP) {
                    const Prim<double> gs = ghost_state(t, rec, 0, +1, slip);
                    sXR[0][fi] = gs.r; sXR[1][fi] = gs.u; sXR[2][fi] = gs.v; sXR[3][fi] = gs.p;
                }
            }
        }
        if (col_in) {
            if (j >= 0) {  // lower face j of the tile's y-faces
                const int fi = j * TX + i;
                const Prim<double> s = fs.yb;
                sYU[0][fi] = s.r; sYU[1][fi] = s.u; sYU[2][fi] = s.v; sYU[3][fi] = s.p;
                if (f & FLAG_WALL_YM) {
                    const Prim<double> gs = ghost_state(t, rec, 1, -1, slip);
                    sYL[0][fi] = gs.r; sYL[1][fi] = gs.u; sYL[2][fi] = gs.v; sYL[3][fi] = gs.p;
                }
            }
            if (j < TY) {  // upper face j + 1
                const int fi = (j + 1) * TX + i;
                const Prim<double> s = fs.yt;
                sYL[0][fi] = s.r; sYL[1][fi] = s.u; sYL[2][fi] = s.v; sYL[3][fi] = s.p;
                if (f & FLAG_WALL_YP) {
                    const Prim<double> gs = ghost_state(t, rec, 1, +1, slip);
                    sYU[0][fi] = gs.r; sYU[1][fi] = gs.u; sYU[2][fi] = gs.v; sYU[3][fi] = gs.p;
                }
            }
        }
    }
    __syncthreads();

    // ---- phase 3: one Osher flux per face --------------------------------------------------
    for (int fidx = tid; fidx < NFX + NFY; fidx += NT) {
        if (fidx < NFX) {
            const int fi = fidx % (TX + 1), j = fidx / (TX + 1);
            const uint8_t fl = sF[(j + 1) * SX + fi], fr = sF[(j + 1) * SX + fi + 1];
            if ((fl & FLAG_SOLID) && (fr & FLAG_SOLID)) continue;
            const Prim<double> L = {sXL[0][fidx], sXL[1][fidx], sXL[2][fidx], sXL[3][fidx]};
            const Prim<double> R = {sXR[0][fidx], sXR[1][fidx], sXR[2][fidx], sXR[3][fidx]};
            const Vec4<double> F = osher_x(L, R, t.beta, t.inv_beta);
            sXL[0][fidx] = F.a; sXL[1][fidx] = F.b; sXL[2][fidx] = F.c; sXL[3][fidx] = F.d;
        } else {
            const int q = fidx - NFX;
            const int i = q % TX, g = q / TX;
            const uint8_t fl = sF[g * SX + i + 1], fu = sF[(g + 1) * SX + i + 1];
            if ((fl & FLAG_SOLID) && (fu & FLAG_SOLID)) continue;
            const Prim<double> L = {sYL[0][q], sYL[1][q], sYL[2][q], sYL[3][q]};
            const Prim<double> U = {sYU[0][q], sYU[1][q], sYU[2][q], sYU[3][q]};
            const Vec4<double> F = osher_y(L, U, t.beta, t.inv_beta);
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
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const double div = (sXL[m][xm + 1] - sXL[m][xm]) * t.inv_dx
                                   + (sYL[m][ym + TX] - sYL[m][ym]) * t.inv_dy;
                R4[m] = -div;
            }
            const double r0 = own_q0[0], m0 = own_q0[1], n0 = own_q0[2];
            R4[0] += -own_d[0];
            R4[1] += -own_d[1] + r0 * t.gx;
            R4[2] += -own_d[2] + r0 * t.gy;
            const double dtau = local_dtau(t, t.cfl, r0, m0, n0);
            const double ad = alpha * dtau;
            const double api = 1.0 + sp.b0 * ad * sp.inv_dt;
            const double fac = ad * rcp_pos(api);
            out_c = c;
            out[0] = r0 + fac * R4[0];
            out[1] = m0 + fac * R4[1];
            out[2] = n0 + fac * R4[2];
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
                part[4] = (out[0] > 0.0 && out[0] < INFINITY) ? 0.0 : 1.0;
            }
        }
    }
    // the residual is reduced before the state is stored: the workgroup barrier of the reduction
    // would otherwise wait for the stores to complete
    if (last) tile_reduce_store<NORM_MAX, NC>(part, &sW[0][0], t.partials + (size_t)tile * kPartialWidth);
    if (out_c != kNoCell) {
        qout[out_c] = out[0];
        qout[plane + out_c] = out[1];
        qout[2 * plane + out_c] = out[2];
        qout[3 * plane + out_c] = out[3];
    }
}

template <int TX, int TY, int NT>
int launch_tile(const TankDev &t, const Scheme &sc, int stage, const IterArgs &ia, void *stream)
{
    const int tiles_x = (t.nx + TX - 1) / TX, tiles_y = (t.ny + TY - 1) / TY;
    const int n_tiles = tiles_x * tiles_y;
    const int blocks = ((n_tiles + 7) / 8) * 8 + (ia.fin ? 8 : 0);
    if (sc.norm_max)
        hipLaunchKernelGGL((stage_tile_f64<TX, TY, NT, true>), dim3(blocks), dim3(NT), 0,
                           (hipStream_t)stream, t, sc, stage, tiles_x, n_tiles, ia);
    else
        hipLaunchKernelGGL((stage_tile_f64<TX, TY, NT, false>), dim3(blocks), dim3(NT), 0,
                           (hipStream_t)stream, t, sc, stage, tiles_x, n_tiles, ia);
    return (int)hipGetLastError();
}

}  // namespace

// 32 x 8, 16 x 16 and 64 x 4 tiles run with 256 threads; 3208 and 1616 name the 32 x 8 and
// 16 x 16 tiles run with 512 threads.
bool tile_supported(int tile_x, int tile_y)
{
    return (tile_x == 32 && tile_y == 8) || (tile_x == 16 && tile_y == 16) ||
           (tile_x == 64 && tile_y == 4) || (tile_x == 3208 && tile_y == 2) ||
           (tile_x == 1616 && tile_y == 2);
}

int tile_count(const TankDev &t, int tile_x, int tile_y)
{
    if (tile_x == 3208) tile_x = 32, tile_y = 8;
    if (tile_x == 1616) tile_x = 16, tile_y = 16;
    return ((t.nx + tile_x - 1) / tile_x) * ((t.ny + tile_y - 1) / tile_y);
}

int launch_stage_tile_f64(const TankDev &t, const Scheme &sc, int stage, int tile_x, int tile_y,
                          const IterArgs &ia, void *stream)
{
    if (ia.fin && stage != 1) return (int)hipErrorInvalidValue;
    if (tile_x == 32 && tile_y == 8) return launch_tile<32, 8, 256>(t, sc, stage, ia, stream);
    if (tile_x == 16 && tile_y == 16) return launch_tile<16, 16, 256>(t, sc, stage, ia, stream);
    if (tile_x == 64 && tile_y == 4) return launch_tile<64, 4, 256>(t, sc, stage, ia, stream);
    if (tile_x == 3208 && tile_y == 2) return launch_tile<32, 8, 512>(t, sc, stage, ia, stream);
    if (tile_x == 1616 && tile_y == 2) return launch_tile<16, 16, 512>(t, sc, stage, ia, stream);
    return (int)hipErrorInvalidValue;
}

}  // namespace vdac
