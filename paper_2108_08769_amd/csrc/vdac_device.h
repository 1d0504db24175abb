// vdac_device.h -- per-point pieces of the scheme as device functions, templated on the
// arithmetic type T (double for the FP64 path, float for the reconstruction and flux of the
// mixed path).
//
// Face states carry primitives W = (rho, u, v, p); fluxes are returned for the conserved
// vector (rho, rho u, rho v, p/beta) of the compact form (Sec. 2.1.2).
#pragma once

#include <hip/hip_runtime.h>

namespace vdac {

template <typename T>
struct Prim {
    T r, u, v, p;
};

// Four components of a flux or a residual: rho, rho u, rho v, p/beta.
template <typename T>
struct Vec4 {
    T a, b, c, d;
    __device__ __forceinline__ T operator[](int k) const
    {
        return k == 0 ? a : (k == 1 ? b : (k == 2 ? c : d));
    }
};

template <typename T>
__device__ __forceinline__ Vec4<T> zero4()
{
    return {T(0), T(0), T(0), T(0)};
}

// Derivatives of rho, u, v along one axis.
template <typename T>
struct Slope {
    T r, u, v;
};

// Reciprocal and reciprocal square root of a positive, finite, normal FP64 argument: the
// hardware estimates (v_rcp_f64, v_rsq_f64, relative error about 5e-8) refined by one
// third-order step, which leaves an error of about one unit in the last place:
//   1/x      = y (1 + e + e^2 + ...),             e = 1 - x y,
//   1/sqrt x = y (1 + e/2 + 3 e^2/8 + ...),       e = 1 - x y^2.
// Used where an IEEE division or square root would cost about ten instructions more.
__device__ __forceinline__ double rcp_pos(double x)
{
    const double y = __builtin_amdgcn_rcp(x);
    const double e = fma(-x, y, 1.0);
    return fma(y, fma(e, e, e), y);
}

__device__ __forceinline__ double rsqrt_pos(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-x * y, y, 1.0);
    return fma(y, e * fma(e, 0.375, 0.5), y);
}

__device__ __forceinline__ float rcp_pos(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float rsqrt_pos(float x) { return __builtin_amdgcn_rsqf(x); }

// k-limiter G(a, b) = s max(0, min(k|b|, s a), min(|b|, k s a)), s = sgn(b), sgn(0) = 0
// (Sec. 2.3.1).  k = 1 is minmod, k = 2 superbee.
template <typename T>
__device__ __forceinline__ T limiter(T a, T b, T k)
{
    T s = (b > T(0)) ? T(1) : ((b < T(0)) ? T(-1) : T(0));
    T ab = fabs(b);
    T sa = s * a;
    T t1 = fmin(k * ab, sa);
    T t2 = fmin(ab, k * sa);
    return s * fmax(T(0), fmax(t1, t2));
}

// k = 1: minmod(a, b) = sgn(b) min(|a|, |b|) when a and b share a sign, else 0 -- the same value
// as limiter(a, b, 1) (up to the sign of a zero result).  It is the median of a, b and 0: the
// smaller of the two when both are positive, the larger when both are negative, else zero.  In
// FP32 that is one median instruction; in FP64, max(min(a, b), min(max(a, b), 0)).
__device__ __forceinline__ float minmod(float a, float b) { return __builtin_amdgcn_fmed3f(a, b, 0.0f); }
__device__ __forceinline__ double minmod(double a, double b)
{
    return fmax(fmin(a, b), fmin(fmax(a, b), 0.0));
}

// Limited one-sided slopes of rho, u, v at a cell from its two neighbours along one axis:
// G((W_{i+1} - W_i)/h, (W_i - W_{i-1})/h).  With minmod the scale 1/h > 0 is applied after the
// limiter: rounding is monotonic, so minmod(a/h, b/h) and minmod(a, b)/h are the same number.
template <typename T>
__device__ __forceinline__ Slope<T> slopes(const Prim<T> &m, const Prim<T> &c, const Prim<T> &p,
                                           T inv_h, T k)
{
    Slope<T> g;
    if (k == T(1)) {
        g.r = minmod(p.r - c.r, c.r - m.r) * inv_h;
        g.u = minmod(p.u - c.u, c.u - m.u) * inv_h;
        g.v = minmod(p.v - c.v, c.v - m.v) * inv_h;
    } else {
        g.r = limiter((p.r - c.r) * inv_h, (c.r - m.r) * inv_h, k);
        g.u = limiter((p.u - c.u) * inv_h, (c.u - m.u) * inv_h, k);
        g.v = limiter((p.v - c.v) * inv_h, (c.v - m.v) * inv_h, k);
    }
    return g;
}

// Mirror image across a wall whose normal lies along `axis` (0 = x, 1 = y): rho and p keep
// their value (zero gradient); the velocity is negated, both components for no-slip walls and the
// normal one only for free slip (Sec. 2.5).
template <typename T>
__device__ __forceinline__ Prim<T> mirror(Prim<T> w, int axis, bool slip)
{
    if (!slip || axis == 0) w.u = -w.u;
    if (!slip || axis == 1) w.v = -w.v;
    return w;
}

// New pressure gradient (Sec. 2.3.2): the rearranged x-momentum equation
//   dp/dx = -d(rho u)/dt - d(rho u^2)/dx - d(rho u v)/dy + rho g_x
// with the products expanded by the product rule and every derivative taken from the limited
// slopes; d(rho u)/dt is the frozen real-time source and rho g_x the frozen body force.  The
// y-component exchanges the roles of x and y.
template <typename T>
__device__ __forceinline__ T gradp_x(const Prim<T> &w, const Slope<T> &gx, const Slope<T> &gy,
                                     T d_ru, T body_x)
{
    return -d_ru - (w.u * w.u * gx.r + T(2) * w.r * w.u * gx.u)
           - (w.u * w.v * gy.r + w.r * w.u * gy.v + w.r * w.v * gy.u) + body_x;
}

template <typename T>
__device__ __forceinline__ T gradp_y(const Prim<T> &w, const Slope<T> &gx, const Slope<T> &gy,
                                     T d_rv, T body_y)
{
    return -d_rv - (w.u * w.v * gx.r + w.r * w.u * gx.v + w.r * w.v * gx.u)
           - (w.v * w.v * gy.r + T(2) * w.r * w.v * gy.v) + body_y;
}

// Osher-Dumbser-Toro flux for the x-split problem (Sec. 2.4.3):
//   F = (F(Q_L) + F(Q_R))/2 - (1/2) sum_j (w_j/2) |A(Q_j)| (Q_R - Q_L),
// Q_j = Q_L + t_j (Q_R - Q_L) on the straight path in conserved variables, t_j = (1 + xi_j)/2 with
// the three-point Gauss-Legendre nodes xi = (-sqrt(3/5), 0, sqrt(3/5)), w = (5, 8, 5)/9.
//
// |A| = R |Lambda| L of Sec. 2.1.3 is applied in closed form: with lambda_{1,2} = u,
// lambda_4 = (u + c)/2 > 0 > lambda_5 = (u - c)/2 and sum_k r_k l_k^T = I,
//   |A| dQ = |u| dQ + (lambda_4 - |u|)(l_4 . dQ) r_4 + (-lambda_5 - |u|)(l_5 . dQ) r_5,
// where, with a = (d(rho u) - u d(rho))/beta and dq = d(p/beta),
//   l_4 . dQ =  (rho/c)(lambda_4 a + dq),   l_5 . dQ = -(rho/c)(lambda_5 a + dq),
//   r_4 = (lambda_4, u lambda_4 + beta/rho, v lambda_4, -lambda_5/rho),
//   r_5 = (lambda_5, u lambda_5 + beta/rho, v lambda_5, -lambda_4/rho).
// Accumulator of sum_j w_j |A(Q_j)| dQ / 2 in the closed form below, one point at a time.
template <typename T>
struct AbsAAcc {
    T sau, a0, a1u, a1b, a2, a3;
};

// Adds the point (rho, u, v), 1/rho = ir, with half weight wj (and wjb = wj / beta) to acc, for
// the jump (dr, dm, dp) in (rho, rho u, p):
//   |A| dQ = |u| dQ + (lambda_4 - |u|)(l_4 . dQ) r_4 + (-lambda_5 - |u|)(l_5 . dQ) r_5,
// where, with a = (d(rho u) - u d(rho))/beta and dq = d(p/beta),
//   l_4 . dQ =  (rho/c)(lambda_4 a + dq),   l_5 . dQ = -(rho/c)(lambda_5 a + dq),
//   r_4 = (lambda_4, u lambda_4 + beta/rho, v lambda_4, -lambda_5/rho),
//   r_5 = (lambda_5, u lambda_5 + beta/rho, v lambda_5, -lambda_4/rho).
// With a' = beta a, dp = beta dq and g = w/(2 beta c), the weighted terms are rho g K4 r_4 and
// rho g K5 r_5 with K4 = (lambda_4 - |u|)(lambda_4 a' + dp), K5 = (lambda_5 + |u|)(lambda_5 a' + dp).
// Their components 0, 1 (its u part) and 2 share s = K4 lambda_4 + K5 lambda_5 times rho g, u rho g
// = m g and v rho g = n g; components 1 (its beta/rho part, kept apart as a1b) and 3 carry 1/rho,
// which cancels rho: g (K4 + K5) and -g (K4 lambda_5 + K5 lambda_4).  So neither v nor rho g
// itself is formed.
template <typename T>
__device__ __forceinline__ void absA_point(AbsAAcc<T> &acc, T rho, T ir, T m, T n, T wj, T wjb,
                                           T four_beta, T dr, T dm, T dp)
{
    const T u = m * ir;
    const T c2 = fma(u, u, four_beta * ir);
    const T y = rsqrt_pos(c2);          // 1/c
    const T hc = T(0.5) * (c2 * y);     // c/2
    const T g = wjb * y;                // w / (2 beta c)
    const T l4 = fma(T(0.5), u, hc), l5 = fma(T(0.5), u, -hc);
    const T au = fabs(u);
    acc.sau = fma(wj, au, acc.sau);
    const T a = fma(-u, dr, dm);
    const T K4 = (l4 - au) * fma(l4, a, dp);
    const T K5 = (l5 + au) * fma(l5, a, dp);
    const T sg = g * fma(K4, l4, K5 * l5);
    acc.a0 = fma(rho, sg, acc.a0);
    acc.a1u = fma(m, sg, acc.a1u);
    acc.a1b = fma(g, K4 + K5, acc.a1b);
    acc.a2 = fma(n, sg, acc.a2);
    acc.a3 = fma(-g, fma(K4, l5, K5 * l4), acc.a3);
}

// Reciprocals of the densities at the three Gauss points.  FP64: one refined reciprocal of their
// product and five multiplications (a reciprocal issues at a quarter of the rate of a
// multiplication); the densities lie between rho_L and rho_R, so the product stays finite and
// normal for densities between 1e-100 and 1e100.  FP32: the hardware estimate of each.
__device__ __forceinline__ void gauss_reciprocals(const double rho[3], double ir[3])
{
    const double p01 = rho[0] * rho[1];
    const double ip = rcp_pos(p01 * rho[2]);
    const double i01 = ip * rho[2];  // 1/(rho0 rho1)
    ir[2] = ip * p01;
    ir[0] = i01 * rho[1];
    ir[1] = i01 * rho[0];
}
__device__ __forceinline__ void gauss_reciprocals(const float rho[3], float ir[3])
{
    ir[0] = rcp_pos(rho[0]);
    ir[1] = rcp_pos(rho[1]);
    ir[2] = rcp_pos(rho[2]);
}

// The face flux functions below return TWICE the face flux, 2F: the factor 1/2 goes into the
// 1/h of the flux divergence, where a power of two scales every result exactly (the divergence
// comes out bit for bit as with F).  Here 2F = F(Q_L) + F(Q_R) - acc with
// acc = sum_j (w_j/2) |A_j| dQ.
template <typename T>
__device__ __forceinline__ Vec4<T> upwind_flux(const Prim<T> &L, const Prim<T> &R, T mL, T mR,
                                               T dr, T dm, T dn, T dp, T beta, T inv_beta,
                                               const AbsAAcc<T> &acc)
{
    const T a1 = fma(beta, acc.a1b, acc.a1u);
    Vec4<T> F;
    F.a = mL + mR - fma(acc.sau, dr, acc.a0);
    F.b = fma(mL, L.u, L.p) + fma(mR, R.u, R.p) - fma(acc.sau, dm, a1);
    F.c = mL * L.v + mR * R.v - fma(acc.sau, dn, acc.a2);
    F.d = L.u + R.u - fma(acc.sau, dp * inv_beta, acc.a3);
    return F;
}

template <typename T>
__device__ __forceinline__ Vec4<T> osher_x(const Prim<T> &L, const Prim<T> &R, T beta, T inv_beta)
{
    const T mL = L.r * L.u, nL = L.r * L.v;
    const T mR = R.r * R.u, nR = R.r * R.v;
    const T dr = R.r - L.r, dm = mR - mL, dn = nR - nL;
    const T dp = R.p - L.p;
    const T four_beta = T(4) * beta;

    // Gauss-Legendre nodes on [0, 1], half weights, and half weights over beta
    const T t0 = T(0.11270166537925831148207346002176);  // (1 - sqrt(3/5))/2
    const T t2 = T(0.88729833462074168851792653997824);  // (1 + sqrt(3/5))/2
    const T w0 = T(5.0) / T(18.0), w1 = T(8.0) / T(18.0);
    const T w0b = w0 * inv_beta, w1b = w1 * inv_beta;

    AbsAAcc<T> acc = {T(0), T(0), T(0), T(0), T(0), T(0)};
    T rho[3], m[3], n[3], ir[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const T t = (j == 0) ? t0 : ((j == 1) ? T(0.5) : t2);
        rho[j] = fma(dr, t, L.r);
        m[j] = fma(dm, t, mL);
        n[j] = fma(dn, t, nL);
    }
    gauss_reciprocals(rho, ir);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const T wj = (j == 1) ? w1 : w0;
        const T wjb = (j == 1) ? w1b : w0b;
        absA_point(acc, rho[j], ir[j], m[j], n[j], wj, wjb, four_beta, dr, dm, dp);
    }
    return upwind_flux(L, R, mL, mR, dr, dm, dn, dp, beta, inv_beta, acc);
}

// Roe flux (Sec. 2.4.2): |A| at the Roe average rho~ = sqrt(rho_L rho_R),
// u~ = (sqrt(rho_L) u_L + sqrt(rho_R) u_R)/(sqrt(rho_L) + sqrt(rho_R)), v~ alike, applied to the
// jump with weight 1 (p does not enter the eigenstructure).
template <typename T>
__device__ __forceinline__ Vec4<T> roe_x(const Prim<T> &L, const Prim<T> &R, T beta, T inv_beta)
{
    const T mL = L.r * L.u, nL = L.r * L.v;
    const T mR = R.r * R.u, nR = R.r * R.v;
    const T dr = R.r - L.r, dm = mR - mL, dn = nR - nL;
    const T dp = R.p - L.p;
    const T sl = L.r * rsqrt_pos(L.r), sr = R.r * rsqrt_pos(R.r);  // square roots
    const T iw = rcp_pos(sl + sr);
    const T rho = sl * sr;
    const T ut = fma(sl, L.u, sr * R.u) * iw;
    const T vt = fma(sl, L.v, sr * R.v) * iw;
    AbsAAcc<T> acc = {T(0), T(0), T(0), T(0), T(0), T(0)};
    absA_point(acc, rho, rcp_pos(rho), rho * ut, rho * vt, T(1), inv_beta, T(4) * beta, dr, dm, dp);
    return upwind_flux(L, R, mL, mR, dr, dm, dn, dp, beta, inv_beta, acc);
}

// Exact (Bassi) flux (Sec. 2.4.1): acoustic speeds S_L = lambda_5,L < 0 < S_R = lambda_4,R, so
// x/tau = 0 lies in the star region, on the contact's left if u* > 0:
//   u* = (p_R - p_L + rho_R u_R lambda_5,R - rho_L u_L lambda_4,L)/(rho_R lambda_5,R - rho_L lambda_4,L),
//   p* = p_R + rho_R lambda_5,R (u_R - u*),
//   rho*_L = rho_L lambda_4,L/(u* - lambda_5,L),  rho*_R = rho_R lambda_5,R/(u* - lambda_4,R),
// and the tangential velocity of the side; the flux is the physical flux of that state.
template <typename T>
__device__ __forceinline__ Vec4<T> bassi_x(const Prim<T> &L, const Prim<T> &R, T beta, T inv_beta)
{
    const T four_beta = T(4) * beta;
    const T cl2 = fma(L.u, L.u, four_beta * rcp_pos(L.r));
    const T cr2 = fma(R.u, R.u, four_beta * rcp_pos(R.r));
    const T hcl = T(0.5) * (cl2 * rsqrt_pos(cl2)), hcr = T(0.5) * (cr2 * rsqrt_pos(cr2));
    const T l4l = fma(T(0.5), L.u, hcl), l5l = fma(T(0.5), L.u, -hcl);
    const T l4r = fma(T(0.5), R.u, hcr), l5r = fma(T(0.5), R.u, -hcr);
    const T rl4 = L.r * l4l, rr5 = R.r * l5r;
    const T us = (R.p - L.p + fma(rr5, R.u, -(rl4 * L.u))) / (rr5 - rl4);
    const T ps = fma(rr5, R.u - us, R.p);
    const bool left = us > T(0);
    const T rs = left ? rl4 / (us - l5l) : rr5 / (us - l4r);
    const T vs = left ? L.v : R.v;
    const T ms2 = T(2) * (rs * us);  // twice the flux, as the other solvers return it
    (void)inv_beta;
    return {ms2, fma(ms2, us, T(2) * ps), ms2 * vs, T(2) * us};
}

// Face flux with normal +y: Algorithm 2 gives t1 = (1, 0, 0) for n = (0, 1, 0), so the rotated
// problem is the x-split one with u and v exchanged, and R^T exchanges the momentum components of
// the result back (Sec. 2.4).
template <typename T>
__device__ __forceinline__ Vec4<T> osher_y(const Prim<T> &L, const Prim<T> &R, T beta, T inv_beta)
{
    const Prim<T> Ls = {L.r, L.v, L.u, L.p};
    const Prim<T> Rs = {R.r, R.v, R.u, R.p};
    const Vec4<T> G = osher_x(Ls, Rs, beta, inv_beta);
    return {G.a, G.c, G.b, G.d};
}

// x-split flux chosen at run time: 0 Osher-Dumbser-Toro, 1 Roe, 2 exact (Bassi); the y-face form
// exchanges u and v as above.
template <typename T>
__device__ __forceinline__ Vec4<T> flux_x(int kind, const Prim<T> &L, const Prim<T> &R, T beta,
                                          T inv_beta)
{
    if (kind == 1) return roe_x(L, R, beta, inv_beta);
    if (kind == 2) return bassi_x(L, R, beta, inv_beta);
    return osher_x(L, R, beta, inv_beta);
}

template <typename T>
__device__ __forceinline__ Vec4<T> flux_y(int kind, const Prim<T> &L, const Prim<T> &R, T beta,
                                          T inv_beta)
{
    const Prim<T> Ls = {L.r, L.v, L.u, L.p};
    const Prim<T> Rs = {R.r, R.v, R.u, R.p};
    const Vec4<T> G = flux_x(kind, Ls, Rs, beta, inv_beta);
    return {G.a, G.c, G.b, G.d};
}

}  // namespace vdac
