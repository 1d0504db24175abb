// kernels_f64.hip -- kernels of one real-time step on gfx950 other than the row-marching stage:
// begin-of-step bookkeeping and the deterministic residual finalize (all tanks in one launch each),
// the conversions of the mixed-precision storage, the tank-wide minima (real-time step bound,
// smallest pseudo-time step), and the plain FP64 stage kernel.
//
// stage_direct_f64 is the plain form of a stage: one thread per cell, which reconstructs itself
// and its four neighbours and evaluates all four of its faces.  Every face is therefore computed
// twice across the grid (once per side, with identical operands in identical order, so both
// sides agree bit for bit and the scheme stays conservative).
#include <hip/hip_runtime.h>

#include "stage_common.h"

namespace vdac {

namespace {

__device__ __forceinline__ void reconstruct(const TankDev &t, const Scheme &sc,
                                            const StepParams &sp, const double *qprev,
                                            const double *q0, int i, int j, CellRec &rec)
{
    const size_t plane = t.plane;
    const size_t c = (size_t)j * t.nx + i;
    const uint8_t f = t.flags[c];
    const bool slip = sc.slip != 0;
    rec.w = load_prim(qprev, plane, c);
    // a wall face shows the cell its own mirror image (Sec. 2.5)
    Prim<double> xm = (f & FLAG_WALL_XM) ? mirror(rec.w, 0, slip)
                                         : load_prim(qprev, plane, (size_t)j * t.nx + wrap(i - 1, t.nx));
    Prim<double> xp = (f & FLAG_WALL_XP) ? mirror(rec.w, 0, slip)
                                         : load_prim(qprev, plane, (size_t)j * t.nx + wrap(i + 1, t.nx));
    Prim<double> ym = (f & FLAG_WALL_YM) ? mirror(rec.w, 1, slip)
                                         : load_prim(qprev, plane, (size_t)wrap(j - 1, t.ny) * t.nx + i);
    Prim<double> yp = (f & FLAG_WALL_YP) ? mirror(rec.w, 1, slip)
                                         : load_prim(qprev, plane, (size_t)wrap(j + 1, t.ny) * t.nx + i);
    rec.gx = slopes(xm, rec.w, xp, t.inv_dx, sc.k);
    rec.gy = slopes(ym, rec.w, yp, t.inv_dy, sc.k);
    // real-time term (B0 Q^0 + B1 Q^n + B2 Q^{n-1})/dt on rho, rho u, rho v (eq. 26)
    const double *qn = t.level_n;
    double num[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        num[k] = sp.b0 * q0[k * plane + c] + sp.b1 * qn[k * plane + c];
        if (sp.b2 != 0.0) num[k] += sp.b2 * t.level_nm1[k * plane + c];
    }
    rec.d_r = num[0] * sp.inv_dt;
    rec.d_ru = num[1] * sp.inv_dt;
    rec.d_rv = num[2] * sp.inv_dt;
    rec.rho0 = q0[c];
}

constexpr int kDirectTX = 16, kDirectTY = 16;

template <bool NORM_MAX>
__global__ void __launch_bounds__(kDirectTX *kDirectTY)
    stage_direct_f64(TankDev t, Scheme sc, int stage, IterArgs ia)
{
    const Status *st = t.status;
    if (st->done) return;
    const int cur = ia.cur_off;
    const StageBuffers b = stage_buffers(cur, stage);
    const double *qprev = (const double *)t.state[b.in];
    const double *q0 = (const double *)t.state[cur];
    double *qout = (double *)t.state[b.out];
    const StepParams sp = *t.step;
    const double alpha = sc.alpha[stage - 1];
    const bool last = (stage == sc.smax);
    const bool slip = sc.slip != 0;
    const size_t plane = t.plane;

    const int i = blockIdx.x * kDirectTX + threadIdx.x;
    const int j = blockIdx.y * kDirectTY + threadIdx.y;
    double part[kPartialWidth] = {0.0, 0.0, 0.0, 0.0, 0.0, INFINITY};
    constexpr size_t kNoCell = ~(size_t)0;
    size_t out_c = kNoCell;  // this thread's updated cell, if any, and its new state
    double out[4] = {0.0, 0.0, 0.0, 0.0};

    if (i < t.nx && j < t.ny) {
        const size_t c = (size_t)j * t.nx + i;
        const uint8_t f = t.flags[c];
        if (!(f & FLAG_SOLID)) {
            CellRec me;
            reconstruct(t, sc, sp, qprev, q0, i, j, me);
            Vec4<double> Fxm, Fxp, Fym, Fyp;
            {
                Prim<double> L, R;
                R = own_state(t, me, 0, -1);
                if (f & FLAG_WALL_XM) {
                    L = ghost_state(t, me, 0, -1, slip);
                } else {
                    CellRec nb;
                    reconstruct(t, sc, sp, qprev, q0, wrap(i - 1, t.nx), j, nb);
                    L = own_state(t, nb, 0, +1);
                }
                Fxm = osher_x(L, R, t.beta, t.inv_beta);
                L = own_state(t, me, 0, +1);
                if (f & FLAG_WALL_XP) {
                    R = ghost_state(t, me, 0, +1, slip);
                } else {
                    CellRec nb;
                    reconstruct(t, sc, sp, qprev, q0, wrap(i + 1, t.nx), j, nb);
                    R = own_state(t, nb, 0, -1);
                }
                Fxp = osher_x(L, R, t.beta, t.inv_beta);
                R = own_state(t, me, 1, -1);
                if (f & FLAG_WALL_YM) {
                    L = ghost_state(t, me, 1, -1, slip);
                } else {
                    CellRec nb;
                    reconstruct(t, sc, sp, qprev, q0, i, wrap(j - 1, t.ny), nb);
                    L = own_state(t, nb, 1, +1);
                }
                Fym = osher_y(L, R, t.beta, t.inv_beta);
                L = own_state(t, me, 1, +1);
                if (f & FLAG_WALL_YP) {
                    R = ghost_state(t, me, 1, +1, slip);
                } else {
                    CellRec nb;
                    reconstruct(t, sc, sp, qprev, q0, i, wrap(j + 1, t.ny), nb);
                    R = own_state(t, nb, 1, -1);
                }
                Fyp = osher_y(L, R, t.beta, t.inv_beta);
            }
            // bracket of eq. 24 and the point-implicit update (coefficient of eq. 27)
            const double r0 = q0[c], m0 = q0[plane + c], n0 = q0[2 * plane + c];
            const double p0 = q0[3 * plane + c];
            const double dtau = local_dtau(t, t.cfl, r0, m0, n0);
            const double src[3] = {-me.d_r, -me.d_ru + r0 * t.gx, -me.d_rv + r0 * t.gy};
            const double base[3] = {r0, m0, n0};
            const double ad = alpha * dtau;
            const double api = 1.0 + sp.b0 * ad * sp.inv_dt;
            double R4[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                // 1/(2h): the flux functions return twice the face flux
                const double div = (Fxp[k] - Fxm[k]) * t.flux_dx + (Fyp[k] - Fym[k]) * t.flux_dy;
                R4[k] = -div + (k < 3 ? src[k] : 0.0);
            }
            const double fac = ad * rcp_pos(api);
            out_c = c;
#pragma unroll
            for (int k = 0; k < 3; ++k) out[k] = base[k] + fac * R4[k];
            out[3] = p0 + t.beta * (ad * R4[3]);
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
    if (last) {
        const int blk = blockIdx.x + blockIdx.y * gridDim.x;
        block_reduce<NORM_MAX, kDirectTX * kDirectTY>(part);
        if (threadIdx.x == 0 && threadIdx.y == 0)
            for (int k = 0; k < kPartialWidth; ++k) t.partials[(size_t)blk * kPartialWidth + k] = part[k];
    }
    if (out_c != kNoCell)
#pragma unroll
        for (int k = 0; k < 4; ++k) qout[k * plane + out_c] = out[k];
}

// The finalize of every tank in its own launch (one wave per tank; see finalize_wave).
__global__ void __launch_bounds__(64) finalize_kernel(const TankDev *__restrict__ tanks, Scheme sc)
{
    finalize_wave(load_tank(tanks + blockIdx.x), sc, threadIdx.x);
}

// Start of a real-time step (Algorithm 1) for tank blockIdx.y, by the tank's StepParams (which
// the host has stored before the launch): with HISTORY_SHIFT the real-time levels shift
// (n-2 <- n-1 <- n), with HISTORY_RESET the kept earlier levels are set to the new level n, with
// HISTORY_KEEP they stay as restored; then level n <- current state and a fresh pseudo-loop
// status.  In the mixed form the new level n is level n plus the current deviation, which then
// becomes zero.  The current state moves to buffer 0, where every step's pseudo-loop starts (the
// status keeps naming the old buffer, which still holds it, until the first finalize).
__global__ void __launch_bounds__(256)
    begin_step_kernel(const TankDev *__restrict__ tanks, int max_pseudo, double tol, int mixed)
{
    const TankDev &t = tanks[blockIdx.y];
    Status *st = t.status;
    const int cur = st->cur;
    const int history = t.step->history;
    const size_t plane = t.plane;
    for (size_t c = (size_t)blockIdx.x * 256 + threadIdx.x; c < plane;
         c += (size_t)gridDim.x * 256) {
        float *d = (float *)t.state[cur];
        const double *q = (const double *)t.state[cur];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const size_t e = k * plane + c;
            if (k == 3 && !mixed) {  // the FP64 form keeps no level-n pressure
                if (cur != 0) ((double *)t.state[0])[e] = q[e];
                break;
            }
            const double old = t.level_n[e];
            const double nw = mixed ? old + (double)d[e] : q[e];
            if (k < 3 && history != HISTORY_KEEP) {
                const bool shift = history == HISTORY_SHIFT;
                if (t.level_nm2) t.level_nm2[e] = shift ? t.level_nm1[e] : nw;
                if (t.level_nm1) t.level_nm1[e] = shift ? old : nw;
            }
            t.level_n[e] = nw;
            // the step starts from buffer 0: the state moves there (mixed: zero deviations)
            if (mixed) {
                d[e] = 0.0f;
                if (cur != 0) ((float *)t.state[0])[e] = 0.0f;
            } else if (cur != 0) {
                ((double *)t.state[0])[e] = nw;
            }
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->iters = 0;
        st->diverged = 0;
        st->max_pseudo = max_pseudo;
        st->tol = tol;
        st->done = (max_pseudo <= 0) ? 1 : 0;
    }
}

// Mixed form: the caller's FP64 state q [4][plane] (rho, rho u, rho v, p) becomes level n (and
// n-1, n-2 for the first three fields) and zero deviations in all three state buffers.
// FP64 form: every state buffer and the real-time levels n, n-1, n-2 (rho, rho u, rho v) of a
// tank from q [4][plane] in device memory, which may be state buffer 0 itself (each thread reads
// a cell before it writes it), or, q null, the state at rest (rho = 1, rho u = rho v = p = 0).
__global__ void __launch_bounds__(256) import_f64_kernel(TankDev t, const double *q)
{
    const size_t plane = t.plane;
    for (size_t c = (size_t)blockIdx.x * 256 + threadIdx.x; c < plane;
         c += (size_t)gridDim.x * 256) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const double v = q ? q[k * plane + c] : (k == 0 ? 1.0 : 0.0);
#pragma unroll
            for (int b = 0; b < 3; ++b) ((double *)t.state[b])[k * plane + c] = v;
            if (k < 3) {
                t.level_n[k * plane + c] = v;
                if (t.level_nm1) t.level_nm1[k * plane + c] = v;
                if (t.level_nm2) t.level_nm2[k * plane + c] = v;
            }
        }
    }
}

// q null: the state at rest (rho = 1, rho u = rho v = p = 0).
__global__ void __launch_bounds__(256) import_mixed_kernel(TankDev t, const double *__restrict__ q)
{
    const size_t plane = t.plane;
    for (size_t c = (size_t)blockIdx.x * 256 + threadIdx.x; c < plane;
         c += (size_t)gridDim.x * 256) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const double v = q ? q[k * plane + c] : (k == 0 ? 1.0 : 0.0);
            t.level_n[k * plane + c] = v;
            if (k < 3 && t.level_nm1) t.level_nm1[k * plane + c] = v;
            if (k < 3 && t.level_nm2) t.level_nm2[k * plane + c] = v;
        }
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            float *d = (float *)t.state[b];
#pragma unroll
            for (int k = 0; k < 4; ++k) d[k * plane + c] = 0.0f;
        }
    }
}

// Mixed form: q [4][plane] <- level n + deviation of buffer cur, in FP64.
__global__ void __launch_bounds__(256)
    export_mixed_kernel(TankDev t, int cur, double *__restrict__ q)
{
    const size_t plane = t.plane;
    const float *d = (const float *)t.state[cur];
    for (size_t c = (size_t)blockIdx.x * 256 + threadIdx.x; c < plane;
         c += (size_t)gridDim.x * 256) {
#pragma unroll
        for (int k = 0; k < 4; ++k) q[k * plane + c] = t.level_n[k * plane + c] + (double)d[k * plane + c];
    }
}

// Per-workgroup minima over the fluid cells of the current state of tank first + blockIdx.y into
// scratch[blockIdx.y * gridDim.x + blockIdx.x]: kind MIN_REALTIME_DT, the global real-time step of
// Sec. 2.2.4, CFL_t dx dy / (|u| dy + |v| dx) (infinity at rest); kind MIN_PSEUDO_DTAU, the local
// pseudo-time step of Sec. 2.2.3 (the function the stage kernels use, so that the minimum is the
// one the last stage reduces).  Every workgroup writes its slot (infinity if it has no cell).
__global__ void __launch_bounds__(256)
    tanks_min_kernel(const TankDev *__restrict__ tanks, int first, int mixed, int kind, double cfl,
                     double *__restrict__ scratch)
{
    const TankDev &t = tanks[first + blockIdx.y];
    const Status *st = t.status;
    const int cur = st->cur;
    const size_t plane = t.plane;
    double m = INFINITY;
    for (size_t c = (size_t)blockIdx.x * 256 + threadIdx.x; c < plane;
         c += (size_t)gridDim.x * 256) {
        if (t.flags[c] & FLAG_SOLID) continue;
        double r, mu, mv;
        if (mixed) {
            const float *d = (const float *)t.state[cur];
            r = t.level_n[c] + (double)d[c];
            mu = t.level_n[plane + c] + (double)d[plane + c];
            mv = t.level_n[2 * plane + c] + (double)d[2 * plane + c];
        } else {
            const double *q = (const double *)t.state[cur];
            r = q[c];
            mu = q[plane + c];
            mv = q[2 * plane + c];
        }
        if (kind == MIN_PSEUDO_DTAU) {
            m = fmin(m, local_dtau(t, t.cfl, r, mu, mv));
        } else {
            const double lam = (fabs(mu) * t.dy + fabs(mv) * t.dx) / r;
            m = fmin(m, cfl * (t.dx * t.dy) / lam);
        }
    }
    m = wave_reduce_to_lane63(m, INFINITY, [](double a, double b) { return fmin(a, b); });
    __shared__ double red[4];
    if ((threadIdx.x & 63) == 63) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0)
        scratch[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = fmin(fmin(red[0], red[1]), fmin(red[2], red[3]));
}

// out[blockIdx.x * out_stride] = the minimum of scratch[blockIdx.x * n .. + n) (one workgroup per
// tank; each thread strides over its row, then the tree).
__global__ void __launch_bounds__(256) min_rows_kernel(const double *__restrict__ scratch, int n,
                                                       double *__restrict__ out, int out_stride)
{
    const double *row = scratch + (size_t)blockIdx.x * n;
    double m = INFINITY;
    for (int i = threadIdx.x; i < n; i += 256) m = fmin(m, row[i]);
    m = wave_reduce_to_lane63(m, INFINITY, [](double a, double b) { return fmin(a, b); });
    __shared__ double red[4];
    if ((threadIdx.x & 63) == 63) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0)
        out[(size_t)blockIdx.x * out_stride] = fmin(fmin(red[0], red[1]), fmin(red[2], red[3]));
}

unsigned cell_blocks(size_t plane)
{
    size_t blocks = (plane + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    return (unsigned)blocks;
}

}  // namespace

int direct_blocks(const TankDev &t)
{
    return ((t.nx + kDirectTX - 1) / kDirectTX) * ((t.ny + kDirectTY - 1) / kDirectTY);
}

int launch_begin_step_all(const TankDev *tanks_dev, int n_tanks, size_t max_plane, const Scheme &sc,
                          int max_pseudo, double tol, void *stream)
{
    const dim3 grid(cell_blocks(max_plane), (unsigned)n_tanks);
    hipLaunchKernelGGL(begin_step_kernel, grid, dim3(256), 0, (hipStream_t)stream, tanks_dev,
                       max_pseudo, tol, sc.mixed);
    return (int)hipGetLastError();
}

int launch_tanks_min(const TankDev *tanks_dev, int first, int n_tanks, int mixed, int kind,
                     double cfl, double *scratch, int blocks_per_tank, double *out, int out_stride,
                     void *stream)
{
    if (n_tanks < 1 || blocks_per_tank < 1 || blocks_per_tank > kMinBlocksMax || !scratch || !out)
        return (int)hipErrorInvalidValue;
    hipLaunchKernelGGL(tanks_min_kernel, dim3((unsigned)blocks_per_tank, (unsigned)n_tanks), dim3(256),
                       0, (hipStream_t)stream, tanks_dev, first, mixed, kind, cfl, scratch);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return (int)e;
    hipLaunchKernelGGL(min_rows_kernel, dim3((unsigned)n_tanks), dim3(256), 0, (hipStream_t)stream,
                       (const double *)scratch, blocks_per_tank, out, out_stride);
    return (int)hipGetLastError();
}

int launch_import_f64(const TankDev &t, const double *q, void *stream)
{
    hipLaunchKernelGGL(import_f64_kernel, dim3(cell_blocks(t.plane)), dim3(256), 0,
                       (hipStream_t)stream, t, q);
    return (int)hipGetLastError();
}

int launch_import_mixed(const TankDev &t, const double *q, void *stream)
{
    hipLaunchKernelGGL(import_mixed_kernel, dim3(cell_blocks(t.plane)), dim3(256), 0,
                       (hipStream_t)stream, t, q);
    return (int)hipGetLastError();
}

int launch_export_mixed(const TankDev &t, int cur, double *q, void *stream)
{
    hipLaunchKernelGGL(export_mixed_kernel, dim3(cell_blocks(t.plane)), dim3(256), 0,
                       (hipStream_t)stream, t, cur, q);
    return (int)hipGetLastError();
}

int launch_stage_direct_f64(const TankDev &t, const Scheme &sc, int stage, const IterArgs &ia,
                            void *stream)
{
    if (ia.fin) return (int)hipErrorInvalidValue;
    dim3 grid((t.nx + kDirectTX - 1) / kDirectTX, (t.ny + kDirectTY - 1) / kDirectTY);
    dim3 block(kDirectTX, kDirectTY);
    if (sc.norm_max)
        hipLaunchKernelGGL(stage_direct_f64<true>, grid, block, 0, (hipStream_t)stream, t, sc, stage, ia);
    else
        hipLaunchKernelGGL(stage_direct_f64<false>, grid, block, 0, (hipStream_t)stream, t, sc, stage, ia);
    return (int)hipGetLastError();
}

int launch_finalize_all(const TankDev *tanks_dev, int n_tanks, const Scheme &sc, void *stream)
{
    hipLaunchKernelGGL(finalize_kernel, dim3((unsigned)n_tanks), dim3(64), 0, (hipStream_t)stream,
                       tanks_dev, sc);
    return (int)hipGetLastError();
}

}  // namespace vdac
