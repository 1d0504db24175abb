// stage_common.h -- device helpers shared by the stage kernels: periodic index wrap, loads of
// the state as primitives, the local pseudo-time step and the residual workgroup reduction.
#pragma once

#include <hip/hip_runtime.h>

#include "vdac_device.h"
#include "vdac_internal.h"

namespace vdac {

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

template <bool NORM_MAX>
__device__ __forceinline__ double combine(double a, double b)
{
    return NORM_MAX ? (a > b || a != a ? a : b) : a + b;
}

// Workgroup reduction of the residual partials (fixed order: deterministic).
template <bool NORM_MAX, int NT>
__device__ __forceinline__ void block_reduce_store(double v[kPartialWidth], double *out)
{
#pragma unroll
    for (int k = 0; k < kPartialWidth; ++k) {
        double x = v[k];
        const bool mx = NORM_MAX && k < 4;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            const double y = __shfl_xor(x, off, 64);
            x = mx ? combine<true>(x, y) : x + y;
        }
        v[k] = x;
    }
    __shared__ double red[NT / 64][kPartialWidth];
    const int tid = threadIdx.x + threadIdx.y * blockDim.x;
    const int wave = tid >> 6, lane = tid & 63;
    if (lane == 0)
        for (int k = 0; k < kPartialWidth; ++k) red[wave][k] = v[k];
    __syncthreads();
    if (tid == 0) {
        for (int k = 0; k < kPartialWidth; ++k) {
            double x = red[0][k];
            for (int w = 1; w < NT / 64; ++w)
                x = (NORM_MAX && k < 4) ? combine<true>(x, red[w][k]) : x + red[w][k];
            out[k] = x;
        }
    }
}

// A fluid cell as the reconstruction sees it: W, limited slopes along x and y, and the stage-0
// sources (real-time term of rho, rho u, rho v and rho^0 for the body force).
struct CellRec {
    Prim<double> w;
    Slope<double> gx, gy;
    double d_r, d_ru, d_rv, rho0;
};

// States of a reconstructed cell at its four faces (left, right, lower, upper):
// W + grad W . (x_f - x_i), with the new pressure gradient for p, evaluated once.
struct FaceStates {
    Prim<double> xl, xr, yb, yt;
};

__device__ __forceinline__ FaceStates face_states(const TankDev &t, const CellRec &c)
{
    const double px = gradp_x(c.w, c.gx, c.gy, c.d_ru, c.rho0 * t.gx);
    const double py = gradp_y(c.w, c.gx, c.gy, c.d_rv, c.rho0 * t.gy);
    const double hx = t.half_dx, hy = t.half_dy;
    FaceStates s;
    s.xl = {fma(-c.gx.r, hx, c.w.r), fma(-c.gx.u, hx, c.w.u), fma(-c.gx.v, hx, c.w.v), fma(-px, hx, c.w.p)};
    s.xr = {fma(c.gx.r, hx, c.w.r), fma(c.gx.u, hx, c.w.u), fma(c.gx.v, hx, c.w.v), fma(px, hx, c.w.p)};
    s.yb = {fma(-c.gy.r, hy, c.w.r), fma(-c.gy.u, hy, c.w.u), fma(-c.gy.v, hy, c.w.v), fma(-py, hy, c.w.p)};
    s.yt = {fma(c.gy.r, hy, c.w.r), fma(c.gy.u, hy, c.w.u), fma(c.gy.v, hy, c.w.v), fma(py, hy, c.w.p)};
    return s;
}

// State of a reconstructed cell at its face on side sd (+1 / -1) of axis (0 = x, 1 = y):
// W + grad W . (x_f - x_i), with the new pressure gradient for p.
__device__ __forceinline__ Prim<double> own_state(const TankDev &t, const CellRec &c, int axis,
                                                  int sd)
{
    Prim<double> s;
    if (axis == 0) {
        const double h = sd > 0 ? t.half_dx : -t.half_dx;
        const double px = gradp_x(c.w, c.gx, c.gy, c.d_ru, c.rho0 * t.gx);
        s.r = c.w.r + c.gx.r * h;
        s.u = c.w.u + c.gx.u * h;
        s.v = c.w.v + c.gx.v * h;
        s.p = c.w.p + px * h;
    } else {
        const double h = sd > 0 ? t.half_dy : -t.half_dy;
        const double py = gradp_y(c.w, c.gx, c.gy, c.d_rv, c.rho0 * t.gy);
        s.r = c.w.r + c.gy.r * h;
        s.u = c.w.u + c.gy.u * h;
        s.v = c.w.v + c.gy.v * h;
        s.p = c.w.p + py * h;
    }
    return s;
}

// State of the wall ghost on side sd of axis, at the face it shares with cell c.  The ghost
// mirrors c and its stencil mirrors c's stencil, so (limiter symmetric and odd) its slope normal
// to the wall equals c's and its tangential slopes are c's with the mirror's signs; its sources
// are mirrored and gravity is reversed in it (Sec. 2.5).
__device__ __forceinline__ Prim<double> ghost_state(const TankDev &t, const CellRec &c, int axis,
                                                    int sd, bool slip)
{
    const double su = (!slip || axis == 0) ? -1.0 : 1.0;  // mirror sign of u
    const double sv = (!slip || axis == 1) ? -1.0 : 1.0;  // mirror sign of v
    Prim<double> w = {c.w.r, su * c.w.u, sv * c.w.v, c.w.p};
    Prim<double> s;
    if (axis == 0) {
        Slope<double> gx = c.gx;
        Slope<double> gy = {c.gy.r, su * c.gy.u, sv * c.gy.v};
        const double px = gradp_x(w, gx, gy, su * c.d_ru, -(c.rho0 * t.gx));
        const double h = sd > 0 ? -t.half_dx : t.half_dx;  // ghost's face toward c
        s.r = w.r + gx.r * h;
        s.u = w.u + gx.u * h;
        s.v = w.v + gx.v * h;
        s.p = w.p + px * h;
    } else {
        Slope<double> gy = c.gy;
        Slope<double> gx = {c.gx.r, su * c.gx.u, sv * c.gx.v};
        const double py = gradp_y(w, gx, gy, sv * c.d_rv, -(c.rho0 * t.gy));
        const double h = sd > 0 ? -t.half_dy : t.half_dy;
        s.r = w.r + gy.r * h;
        s.u = w.u + gy.u * h;
        s.v = w.v + gy.v * h;
        s.p = w.p + py * h;
    }
    return s;
}

}  // namespace vdac
