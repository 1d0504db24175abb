// stage_common.h -- device helpers shared by the stage kernels: periodic index wrap, loads of
// the state as primitives, the local pseudo-time step and the residual workgroup reduction.
#pragma once

#include <hip/hip_runtime.h>

#include "vdac_device.h"
#include "vdac_internal.h"

namespace vdac {

// Wave-uniform copies (readfirstlane) of values every lane of a wave holds alike, so that they
// live in scalar registers.
__device__ __forceinline__ uint32_t uni(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); }
__device__ __forceinline__ int32_t uni(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t uni(uint64_t v)
{
    return ((uint64_t)uni((uint32_t)(v >> 32)) << 32) | uni((uint32_t)v);
}
__device__ __forceinline__ double uni(double v) { return __builtin_bit_cast(double, uni(__builtin_bit_cast(uint64_t, v))); }
template <typename T>
__device__ __forceinline__ T *uni(T *p)
{
    return (T *)uni((uint64_t)(uintptr_t)p);
}

// The descriptor of a tank read from the device table into scalar registers, field by field (a
// struct copy would go through private memory); the state buffers come from state_buf.
__device__ __forceinline__ TankDev load_tank(const TankDev *__restrict__ p)
{
    TankDev t;
    t.nx = uni(p->nx);
    t.ny = uni(p->ny);
    t.per_x = uni(p->per_x);
    t.per_y = uni(p->per_y);
    t.dx = uni(p->dx);
    t.dy = uni(p->dy);
    t.inv_dx = uni(p->inv_dx);
    t.inv_dy = uni(p->inv_dy);
    t.half_dx = uni(p->half_dx);
    t.half_dy = uni(p->half_dy);
    t.flux_dx = uni(p->flux_dx);
    t.flux_dy = uni(p->flux_dy);
    t.gx = uni(p->gx);
    t.gy = uni(p->gy);
    t.beta = uni(p->beta);
    t.inv_beta = uni(p->inv_beta);
    t.cfl = uni(p->cfl);
    t.plane = (size_t)uni((uint64_t)p->plane);
    t.state[0] = t.state[1] = t.state[2] = nullptr;  // see state_buf
    t.level_n = uni(p->level_n);
    t.level_nm1 = uni(p->level_nm1);
    t.level_nm2 = uni(p->level_nm2);
    t.flags = uni(p->flags);
    t.partials = uni(p->partials);
    t.status = uni(p->status);
    t.step = uni(p->step);
    t.n_fluid = uni(p->n_fluid);
    t.n_partials = uni(p->n_partials);
    t.n_strips = uni(p->n_strips);
    t.chunk = uni(p->chunk);
    t.open = uni(p->open);
    return t;
}

// State buffer b (0..2) of a tank, read from the device table (indexing the array of a local
// copy would force the copy into private memory).
__device__ __forceinline__ void *state_buf(const TankDev *__restrict__ p, int b)
{
    return uni(p->state[b]);
}

__device__ __forceinline__ int wrap(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

__device__ __forceinline__ Prim<double> load_prim(const double *q, size_t plane, size_t c)
{
    Prim<double> w;
    w.r = q[c];
    const double ir = rcp_pos(w.r);
    w.u = q[plane + c] * ir;
    w.v = q[2 * plane + c] * ir;
    w.p = q[3 * plane + c];
    return w;
}

// Pseudo-time step of Sec. 2.2.3 in 2D: CFL dx dy / ((|u| + c_x) dy/2 + (|v| + c_y) dx/2).
__device__ __forceinline__ double local_dtau(const TankDev &t, double cfl, double rho, double m,
                                             double n)
{
    const double ir = rcp_pos(rho);
    const double u = m * ir, v = n * ir;
    const double fb = 4.0 * t.beta * ir;
    const double cx2 = fma(u, u, fb), cy2 = fma(v, v, fb);
    const double cx = cx2 * rsqrt_pos(cx2);
    const double cy = cy2 * rsqrt_pos(cy2);
    const double lx = 0.5 * (fabs(u) + cx) * t.dy;
    const double ly = 0.5 * (fabs(v) + cy) * t.dx;
    return cfl * (t.dx * t.dy) * rcp_pos(lx + ly);
}

// The pseudo-time step scaled by alpha_s, ad = alpha_s dtau, and the point-implicit factor
// fc = ad / (1 + B0 ad / dt) (eq. 27) of a cell with stage-0 state (rho, m, n), in FP64 with two
// reciprocal-square-root estimates and one reciprocal.  With u = m/rho, c_x = sqrt(u^2 + 4 beta/rho)
// = sqrt(m^2 + 4 beta rho)/rho, so the denominator of Sec. 2.2.3 is D'/rho with
//   D' = (|m| + sqrt(m^2 + 4 beta rho)) dy/2 + (|n| + sqrt(n^2 + 4 beta rho)) dx/2,
// and ad = a rho / D', fc = a rho / (D' + kappa rho) with a = alpha_s CFL dx dy and
// kappa = B0 a / dt; both reciprocals come from one of their product.
__device__ __forceinline__ void dtau_factors(const TankDev &t, double a, double kappa, double rho,
                                             double m, double n, double &ad, double &fc)
{
    const double fb = 4.0 * t.beta * rho;
    const double sx2 = fma(m, m, fb), sy2 = fma(n, n, fb);
    const double sx = sx2 * rsqrt_pos(sx2), sy = sy2 * rsqrt_pos(sy2);
    const double d = 0.5 * fma(fabs(m) + sx, t.dy, (fabs(n) + sy) * t.dx);
    const double e = fma(kappa, rho, d);
    const double ip = rcp_pos(d * e);
    const double ar = a * rho;
    ad = ar * (e * ip);
    fc = ar * (d * ip);
}

// The same step in FP32 with the hardware reciprocal and reciprocal-square-root estimates, for
// the mixed form: the step only scales the pseudo-time update (the converged state does not
// depend on it), so it needs no more precision than the fluxes it multiplies.
__device__ __forceinline__ double local_dtau_f32(const TankDev &t, double cfl, double rho, double m,
                                                 double n)
{
    const float ir = rcp_pos((float)rho);
    const float u = (float)m * ir, v = (float)n * ir;
    const float fb = 4.0f * (float)t.beta * ir;
    const float cx2 = fmaf(u, u, fb), cy2 = fmaf(v, v, fb);
    const float cx = cx2 * rsqrt_pos(cx2);
    const float cy = cy2 * rsqrt_pos(cy2);
    const float lx = 0.5f * (fabsf(u) + cx) * (float)t.dy;
    const float ly = 0.5f * (fabsf(v) + cy) * (float)t.dx;
    return (double)((float)(cfl * (t.dx * t.dy)) * rcp_pos(lx + ly));
}

// dtau_factors in FP32 with the hardware estimates, for the mixed form, whose pseudo-time step is
// an FP32 step size (it scales the update; the converged state does not depend on it).
__device__ __forceinline__ void dtau_factors_f32(const TankDev &t, float a, float kappa, double rho_d,
                                                 double m_d, double n_d, double &ad, double &fc)
{
    const float rho = (float)rho_d, m = (float)m_d, n = (float)n_d;
    const float fb = 4.0f * (float)t.beta * rho;
    const float sx2 = fmaf(m, m, fb), sy2 = fmaf(n, n, fb);
    const float sx = sx2 * rsqrt_pos(sx2), sy = sy2 * rsqrt_pos(sy2);
    const float d = 0.5f * fmaf(fabsf(m) + sx, (float)t.dy, (fabsf(n) + sy) * (float)t.dx);
    const float e = fmaf(kappa, rho, d);
    const float ip = rcp_pos(d * e);
    const float ar = a * rho;
    ad = (double)(ar * (e * ip));
    fc = (double)(ar * (d * ip));
}

template <bool NORM_MAX>
__device__ __forceinline__ double combine(double a, double b)
{
    return NORM_MAX ? (a > b || a != a ? a : b) : a + b;
}

// DPP move of a double (gfx9 data-parallel primitives, in VALU: no LDS traffic).  Lanes whose
// source lies outside the pattern, and rows outside ROW_MASK, keep `old`.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_f64(double old, double x)
{
    const uint64_t o = __builtin_bit_cast(uint64_t, old), b = __builtin_bit_cast(uint64_t, x);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)o, (int)(uint32_t)b, CTRL,
                                                              ROW_MASK, 0xf, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)(o >> 32), (int)(uint32_t)(b >> 32),
                                                              CTRL, ROW_MASK, 0xf, false);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Row shift: lane i of each row of 16 lanes receives x from lane i - N of the same row.
template <int N>
__device__ __forceinline__ double dpp_row_shr(double old, double x)
{
    static_assert(N >= 1 && N <= 15, "row_shr takes 1..15");
    return dpp_f64<0x110 | N, 0xf>(old, x);
}

// Fixed-order reduction over the 64 lanes of a wave with the associative op (identity id): a tree
// within each row of 16 lanes, then the rows combined by broadcasts of lanes 15 and 31.  The
// result is complete in lane 63 only.
template <class Op>
__device__ __forceinline__ double wave_reduce_to_lane63(double x, double id, Op op)
{
    x = op(x, dpp_row_shr<1>(id, x));
    x = op(x, dpp_row_shr<2>(id, x));
    x = op(x, dpp_row_shr<4>(id, x));
    x = op(x, dpp_row_shr<8>(id, x));        // lane 15 of each row: the row
    x = op(x, dpp_f64<0x142, 0xa>(id, x));   // row_bcast:15 -> lane 31: rows 0-1, lane 63: rows 2-3
    x = op(x, dpp_f64<0x143, 0xc>(id, x));   // row_bcast:31 -> lane 63: all rows
    return x;
}

// Workgroup reduction of the residual partials (fixed order: deterministic): sums or maxima of the
// four fields, the sum of bad cells, the minimum pseudo-time step.  The totals end up in every lane
// of wave 0 (each wave's tree in VALU, then the waves' results through LDS).
template <bool NORM_MAX, int NT>
__device__ __forceinline__ void block_reduce(double v[kPartialWidth])
{
    auto sum = [](double a, double b) { return a + b; };
    auto mx = [](double a, double b) { return combine<true>(a, b); };
    auto mn = [](double a, double b) { return fmin(a, b); };
#pragma unroll
    for (int k = 0; k < kPartialWidth; ++k)
        v[k] = (k == 5) ? wave_reduce_to_lane63(v[k], INFINITY, mn)
                        : ((NORM_MAX && k < 4) ? wave_reduce_to_lane63(v[k], 0.0, mx)
                                               : wave_reduce_to_lane63(v[k], 0.0, sum));
    __shared__ double red[NT / 64][kPartialWidth];
    const int tid = threadIdx.x + threadIdx.y * blockDim.x;
    const int wave = tid >> 6, lane = tid & 63;
    if (lane == 63)
        for (int k = 0; k < kPartialWidth; ++k) red[wave][k] = v[k];
    __syncthreads();
    if (wave == 0) {
        for (int k = 0; k < kPartialWidth; ++k) {
            double x = red[0][k];
            for (int w = 1; w < NT / 64; ++w)
                x = (k == 5) ? fmin(x, red[w][k])
                             : ((NORM_MAX && k < 4) ? combine<true>(x, red[w][k]) : x + red[w][k]);
            v[k] = x;
        }
    }
}

// Deterministic second pass of the residual and the pseudo-loop control of tank t (Algorithm 1),
// by one whole wave: the tank's partials combined in a fixed order (lane-strided, then the wave
// tree), then the norms, the stop flags, the buffer rotation and the global pseudo-time step
// stored.  A stopped tank is left alone.
__device__ __forceinline__ void finalize_wave(const TankDev &t, const Scheme &sc, int lane)
{
    Status *st = t.status;
    const int n = t.n_partials;
    const bool nm = sc.norm_max != 0;
    // the partials are read before the stop flag is known (one memory round trip fewer)
    double acc[kPartialWidth] = {0.0, 0.0, 0.0, 0.0, 0.0, INFINITY};
    constexpr int kBatch = 4;  // partials per lane whose loads are in flight together
    for (int b0 = 0; b0 < n; b0 += kBatch * 64) {
        double x[kBatch][kPartialWidth];
#pragma unroll
        for (int q = 0; q < kBatch; ++q) {
            const int b = min(b0 + q * 64 + lane, n - 1);
#pragma unroll
            for (int k = 0; k < kPartialWidth; ++k) x[q][k] = t.partials[(size_t)b * kPartialWidth + k];
        }
#pragma unroll
        for (int q = 0; q < kBatch; ++q) {
            if (b0 + q * 64 + lane >= n) continue;
#pragma unroll
            for (int k = 0; k < kPartialWidth; ++k)
                acc[k] = (k == 5) ? fmin(acc[k], x[q][k])
                                  : ((nm && k < 4) ? combine<true>(acc[k], x[q][k]) : acc[k] + x[q][k]);
        }
    }
    auto sum = [](double a, double b) { return a + b; };
    auto mx = [](double a, double b) { return combine<true>(a, b); };
    auto mn = [](double a, double b) { return fmin(a, b); };
#pragma unroll
    for (int k = 0; k < kPartialWidth; ++k)
        acc[k] = (k == 5) ? wave_reduce_to_lane63(acc[k], INFINITY, mn)
                          : ((nm && k < 4) ? wave_reduce_to_lane63(acc[k], 0.0, mx)
                                           : wave_reduce_to_lane63(acc[k], 0.0, sum));
    if (st->done) return;
    if (lane == 63) {
        const double tol = st->tol;
        bool finite = true, below = true;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const double nk = nm ? acc[k] : sqrt(acc[k] / (double)(t.n_fluid > 0 ? t.n_fluid : 1));
            if (!(nk < INFINITY)) finite = false;  // NaN or Inf
            if (!(nk < tol)) below = false;
            st->norms[k] = nk;
        }
        const int iters = st->iters + 1;
        const bool bad = !finite || acc[4] > 0.0;
        st->iters = iters;
        st->cur = cur_of_iter(iters, sc.smax);
        if (bad) st->diverged = 1;
        const bool converged = tol > 0.0 && below;
        st->done = (bad || converged || iters >= st->max_pseudo) ? 1 : 0;
        if (acc[5] < INFINITY) st->dtau_global = acc[5];  // reduced only when global
    }
}

// ------------------------------------------------------------------------------------------
// Precision policies.  FP64: the state is stored as (rho, rho u, rho v, p) in FP64 and every step
// runs in FP64.  Mixed: the state is stored in FP32 as the deviation from real-time level n
// (rho - rho^n, rho u - (rho u)^n, rho v - (rho v)^n) plus the absolute pressure, level n (and
// n-1) stay in FP64; reconstruction and Riemann fluxes run in FP32 on pressures taken relative to
// the face's left (lower) cell, and the divergence, sources, update and norm run in FP64.
// ------------------------------------------------------------------------------------------
struct PrecF64 {
    using Real = double;   // reconstruction and flux arithmetic
    using Store = double;  // state storage
    static constexpr bool kMixed = false;
};
struct PrecMixed {
    using Real = float;
    using Store = float;
    static constexpr bool kMixed = true;
};

// Absolute state (rho, rho u, rho v, p) of cell c of a state buffer.
template <class P>
__device__ __forceinline__ void load_state(const TankDev &t, const void *buf, size_t c, double &r,
                                           double &m, double &n, double &p)
{
    const size_t plane = t.plane;
    const typename P::Store *q = (const typename P::Store *)buf;
    if (P::kMixed) {
        r = t.level_n[c] + (double)q[c];
        m = t.level_n[plane + c] + (double)q[plane + c];
        n = t.level_n[2 * plane + c] + (double)q[2 * plane + c];
    } else {
        r = (double)q[c];
        m = (double)q[plane + c];
        n = (double)q[2 * plane + c];
    }
    p = (double)q[3 * plane + c];
}

// Primitives of cell c of a state buffer in the reconstruction precision.
template <class P>
__device__ __forceinline__ Prim<typename P::Real> load_prim_p(const TankDev &t, const void *buf,
                                                              size_t c)
{
    using R = typename P::Real;
    double r, m, n, p;
    load_state<P>(t, buf, c, r, m, n, p);
    const double ir = rcp_pos(r);
    return {(R)r, (R)(m * ir), (R)(n * ir), (R)p};
}

// Stores the absolute state (rho, rho u, rho v, p) of cell c; the mixed form stores deviations
// from level n given in ln0..ln2.
template <class P>
__device__ __forceinline__ void store_state(const TankDev &t, void *buf, size_t c, double r, double m,
                                            double n, double p, double ln0, double ln1, double ln2)
{
    const size_t plane = t.plane;
    typename P::Store *q = (typename P::Store *)buf;
    if (P::kMixed) {
        q[c] = (float)(r - ln0);
        q[plane + c] = (float)(m - ln1);
        q[2 * plane + c] = (float)(n - ln2);
    } else {
        q[c] = r;
        q[plane + c] = m;
        q[2 * plane + c] = n;
    }
    q[3 * plane + c] = (typename P::Store)p;
}

// A fluid cell as the reconstruction sees it: W, limited slopes along x and y, and the stage-0
// sources (real-time term of rho u, rho v and rho^0 for the body force).
template <typename R>
struct CellRecT {
    Prim<R> w;
    Slope<R> gx, gy;
    R d_r, d_ru, d_rv, rho0;
};
using CellRec = CellRecT<double>;

// State of a reconstructed cell at one face: W +- grad W h, with the new pressure gradient gp
// for p; pbase is the pressure the state is expressed from (the cell's own pressure for the
// absolute form, its difference to the face's reference pressure for the compensated form).
template <typename R>
__device__ __forceinline__ Prim<R> state_at(const Prim<R> &w, const Slope<R> &g, R gp, R h, R pbase)
{
    return {fma(g.r, h, w.r), fma(g.u, h, w.u), fma(g.v, h, w.v), fma(gp, h, pbase)};
}

// New pressure gradient of a reconstructed cell (Sec. 2.3.2).
template <typename R>
__device__ __forceinline__ R cell_gradp_x(const TankDev &t, const CellRecT<R> &c)
{
    return gradp_x(c.w, c.gx, c.gy, c.d_ru, c.rho0 * (R)t.gx);
}
template <typename R>
__device__ __forceinline__ R cell_gradp_y(const TankDev &t, const CellRecT<R> &c)
{
    return gradp_y(c.w, c.gx, c.gy, c.d_rv, c.rho0 * (R)t.gy);
}

// States of a reconstructed cell at its four faces (left, right, lower, upper), with the
// pressure gradient evaluated once and p expressed from pbase.
template <typename R>
struct FaceStatesT {
    Prim<R> xl, xr, yb, yt;
};
using FaceStates = FaceStatesT<double>;

template <typename R>
__device__ __forceinline__ FaceStatesT<R> face_states(const TankDev &t, const CellRecT<R> &c,
                                                      R pb_xl, R pb_xr, R pb_yb, R pb_yt)
{
    const R px = cell_gradp_x(t, c);
    const R py = cell_gradp_y(t, c);
    const R hx = (R)t.half_dx, hy = (R)t.half_dy;
    FaceStatesT<R> s;
    s.xl = state_at(c.w, c.gx, px, -hx, pb_xl);
    s.xr = state_at(c.w, c.gx, px, hx, pb_xr);
    s.yb = state_at(c.w, c.gy, py, -hy, pb_yb);
    s.yt = state_at(c.w, c.gy, py, hy, pb_yt);
    return s;
}

__device__ __forceinline__ FaceStates face_states(const TankDev &t, const CellRec &c)
{
    return face_states<double>(t, c, c.w.p, c.w.p, c.w.p, c.w.p);
}

// State of a reconstructed cell at its face on side sd (+1 / -1) of axis (0 = x, 1 = y):
// W + grad W . (x_f - x_i), with the new pressure gradient for p.
__device__ __forceinline__ Prim<double> own_state(const TankDev &t, const CellRec &c, int axis,
                                                  int sd)
{
    if (axis == 0) {
        const double h = sd > 0 ? t.half_dx : -t.half_dx;
        return state_at(c.w, c.gx, cell_gradp_x(t, c), h, c.w.p);
    }
    const double h = sd > 0 ? t.half_dy : -t.half_dy;
    return state_at(c.w, c.gy, cell_gradp_y(t, c), h, c.w.p);
}

// State of the wall ghost on side sd of axis, at the face it shares with cell c.  The ghost
// mirrors c and its stencil mirrors c's stencil, so (limiter symmetric and odd) its slope normal
// to the wall equals c's and its tangential slopes are c's with the mirror's signs; its sources
// are mirrored and gravity is reversed in it (Sec. 2.5).  Its pressure equals c's; pbase is that
// pressure in the form the face uses.
template <typename R>
__device__ __forceinline__ Prim<R> ghost_state(const TankDev &t, const CellRecT<R> &c, int axis,
                                               int sd, bool slip, R pbase)
{
    const R su = (!slip || axis == 0) ? R(-1) : R(1);  // mirror sign of u
    const R sv = (!slip || axis == 1) ? R(-1) : R(1);  // mirror sign of v
    const Prim<R> w = {c.w.r, su * c.w.u, sv * c.w.v, c.w.p};
    if (axis == 0) {
        const Slope<R> gx = c.gx;
        const Slope<R> gy = {c.gy.r, su * c.gy.u, sv * c.gy.v};
        const R px = gradp_x(w, gx, gy, su * c.d_ru, -(c.rho0 * (R)t.gx));
        const R h = sd > 0 ? -(R)t.half_dx : (R)t.half_dx;  // ghost's face toward c
        return state_at(w, gx, px, h, pbase);
    }
    const Slope<R> gy = c.gy;
    const Slope<R> gx = {c.gx.r, su * c.gx.u, sv * c.gx.v};
    const R py = gradp_y(w, gx, gy, sv * c.d_rv, -(c.rho0 * (R)t.gy));
    const R h = sd > 0 ? -(R)t.half_dy : (R)t.half_dy;
    return state_at(w, gy, py, h, pbase);
}

__device__ __forceinline__ Prim<double> ghost_state(const TankDev &t, const CellRec &c, int axis,
                                                    int sd, bool slip)
{
    return ghost_state<double>(t, c, axis, sd, slip, c.w.p);
}

// Pressure gradient along one axis by the k-limiter on p (pgrad 1) or the split limiter
// (pgrad 2, Sec. 2.3.2): from the pressure differences dpr = p_{i+1} - p_i, dpl = p_i - p_{i-1}
// (FP64), the densities of the stencil and the gravity component g along the axis.
__device__ __forceinline__ double pgrad_limited(int pgrad, double pk, double dpr, double dpl,
                                               double inv_h, double rl, double rc, double rr,
                                               double g)
{
    if (pgrad == 1) return limiter(dpr * inv_h, dpl * inv_h, pk);
    const double kr = fma(dpr, inv_h, -0.5 * (rc + rr) * g);
    const double kl = fma(dpl, inv_h, -0.5 * (rl + rc) * g);
    return fma(rc, g, limiter(kr, kl, pk));
}

// Ghost of a reconstructed cell for the general kernel: across a wall (open = false) or a
// zero-gradient side (open = true: no velocity sign change, gravity kept, sources kept).  Its
// normal p-slope: the new method evaluates the rearranged momentum equation in the ghost; the
// k-limiter on p gives zero at such a face on both sides; the split limiter gives minus the
// cell's (the wall ghost's stencil is the cell's reflected, with gravity reversed).
template <typename R>
__device__ __forceinline__ Prim<R> ghost_state_gen(const TankDev &t, const Scheme &sc,
                                                   const CellRecT<R> &c, int axis, int sd,
                                                   bool open, R p_own_slope, R pbase)
{
    const bool slip = sc.slip != 0;
    const R su = (open || (slip && axis == 1)) ? R(1) : R(-1);
    const R sv = (open || (slip && axis == 0)) ? R(1) : R(-1);
    const R gs = open ? R(1) : R(-1);
    const Prim<R> w = {c.w.r, su * c.w.u, sv * c.w.v, c.w.p};
    if (axis == 0) {
        const Slope<R> gx = c.gx;
        const Slope<R> gy = {c.gy.r, su * c.gy.u, sv * c.gy.v};
        const R px = sc.pgrad == 0 ? gradp_x(w, gx, gy, su * c.d_ru, gs * (c.rho0 * (R)t.gx))
                                   : (sc.pgrad == 1 ? p_own_slope : -p_own_slope);
        const R h = sd > 0 ? -(R)t.half_dx : (R)t.half_dx;
        return state_at(w, gx, px, h, pbase);
    }
    const Slope<R> gy = c.gy;
    const Slope<R> gx = {c.gx.r, su * c.gx.u, sv * c.gx.v};
    const R py = sc.pgrad == 0 ? gradp_y(w, gx, gy, sv * c.d_rv, gs * (c.rho0 * (R)t.gy))
                               : (sc.pgrad == 1 ? p_own_slope : -p_own_slope);
    const R h = sd > 0 ? -(R)t.half_dy : (R)t.half_dy;
    return state_at(w, gy, py, h, pbase);
}

}  // namespace vdac
