/*
 * vdac_oracle.c -- plain serial FP64 reference ("oracle") for the dual-time Godunov scheme of
 * Leakey, Glenis & Hewett (arXiv:2108.08769): 2D Cartesian cell-centred finite volumes for the
 * inviscid variable-density artificial-compressibility equations, explicit Runge-Kutta pseudo-time
 * stepping with a point-implicit real-time term, MUSCL reconstruction with the k-limiter, the
 * paper's new pressure gradient, the Osher-Dumbser-Toro flux and ghost-cell walls with reversed
 * gravity.
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the benchmark's CPU-baseline
 * leg; never by the product path.  It shares no code with the GPU library.
 *
 * Built serial for the tests.  A second build with -fopenmp (for the all-cores CPU baseline only)
 * runs the row loops of a stage on all host threads; every cell's arithmetic is the same, and the
 * only reduction inside them is a minimum, so that build's results are bit for bit the serial
 * ones.
 *
 * Written for a reader holding the paper: every step follows the definition it cites, in the
 * paper's order and notation, with no blocking, fusion or reordering.  Build with
 * -O2 -ffp-contract=off (no fused multiply-add, no fast-math).
 *
 * Readings of the paper taken here where it is silent, garbled or ambiguous:
 *   R1  Slopes use the true one-sided differences (W_{i+1}-W_i)/dx; the face sits at +-dx/2 from
 *       the centre (Sec. 2.3.1 prints dx/2 in the denominator, which would double every slope).
 *   R2  W_L = W_i + grad(W_i).(x_f - x_i): the gradient dots the position offset (the printed
 *       "(W_f - W_i)" is read as the displacement).
 *   R3  Reconstructed primitives are W = (rho, u, v, p); p uses the new gradient of Sec. 2.3.2.
 *   R4  sgn(0) = 0 in the limiter, so G(a, 0) = 0.
 *   R5  alpha_PI = 1 + B0*alpha_s*dtau/dt scales the components that carry a real-time term
 *       (I_C = 1); the p/beta component has none and uses 1 (this is what solving the real-time
 *       term point-implicitly gives; both readings share the converged state).
 *   R6  The real-time term, the body force and dtau are evaluated once per pseudo-iteration from
 *       the stage-0 state (Algorithm 1 computes them before the Runge-Kutta loop).
 *   R7  The new pressure gradient takes rho, u, v and their limited gradients from the stage
 *       being evaluated, and the stored stage-0 sources: the real-time term of rho*u (rho*v) and
 *       the body force rho^0 g.  The y-component is the x formula with x and y exchanged.
 *   R8  Walls use two mirrored ghost layers: the ghost at distance d copies the interior cell at
 *       distance d-1 with rho and p unchanged (zero gradient) and both velocity components
 *       negated (no-slip); corner ghosts receive both reflections; gravity is reversed in wall
 *       ghosts when their pressure gradient is formed (Sec. 2.5).  The ghost's real-time term is
 *       mirrored like its state.  The paper expects the tangential sign to have no effect without
 *       viscosity; with the new pressure gradient it does (the ghost's cross terms change sign
 *       relative to the cell's, so the face pressures differ at the wall and some mass crosses
 *       it).  A free-slip option (normal component only negated) is kept beside the default.
 *   R9  Solid (obstacle) cells are not in the paper.  Each fluid-solid face is a wall: the ghost
 *       across it mirrors the fluid cell, and the ghost's stencil mirrors the fluid cell's
 *       stencil as the fluid cell sees it.  For domain walls this rule yields exactly the ghost
 *       layers of R8, so one construction serves both.  Solid cells keep their state.
 *   R10 The residual is the bracket of the last Runge-Kutta stage, per field, with the p row
 *       reported as beta*R_(p/beta) (= dp/dtau).  Norm: RMS over fluid cells (or max norm).
 *       Converged when every field is below the tolerance.
 *   R11 The y-direction spectral radius uses c_y = sqrt(v^2 + 4 beta/rho).
 *   R12 Gauss-Legendre on [0,1]: the integral of |A| dQ is (1/2) sum_j w_j |A(Q_j)| (Q_R - Q_L).
 *   R13 Zero-gradient (transmissive) sides: the ghosts mirror the interior like wall ghosts but
 *       keep every variable's sign, and gravity is not reversed in them; the normal derivative of
 *       every variable then vanishes at the boundary face.
 *   R14 The pressure-gradient variants of Sec. 2.3.2 use the same stencils as rho, u, v: the
 *       k-limiter applied to p, or the split limiter whose hydrostatic parts use the stencil's
 *       densities and the gravity of the cell (reversed in wall ghosts).
 *   R15 Roe averages of rho, u, v only: p does not enter the eigenstructure (Sec. 2.4.2).
 *   R16 BDF order: the smallest of the order asked for and the real-time levels available
 *       (the first step is backward Euler, the second at most BDF2; Table 1).
 */
#include "vdac_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#define ORC_PRAGMA(x) _Pragma(#x)
#define ORC_ROWS _Pragma("omp parallel for schedule(static)")
#define ORC_ROWS_MIN(v) ORC_PRAGMA(omp parallel for schedule(static) reduction(min : v))
#else
#define ORC_ROWS
#define ORC_ROWS_MIN(v)
#endif

/* ------------------------------------------------------------------------------------------ */
/* Single-point pieces                                                                        */
/* ------------------------------------------------------------------------------------------ */

static double max2(double a, double b) { return a > b ? a : b; }
static double min2(double a, double b) { return a < b ? a : b; }

/* Sec. 2.3.1: G(a,b) = s max(0, min(k|b|, s a), min(|b|, k s a)), s = sgn(b) (R4). */
double orc_limiter(double a, double b, double k)
{
    double s = (b > 0.0) ? 1.0 : ((b < 0.0) ? -1.0 : 0.0);
    double t1 = min2(k * fabs(b), s * a);
    double t2 = min2(fabs(b), k * s * a);
    return s * max2(0.0, max2(t1, t2));
}

/* Sec. 2.1.2: F_x,inv = (rho u, rho u^2 + p, rho u v, u), with p = beta * Q[3]. */
void orc_flux_phys(const double q[4], double beta, double f[4])
{
    double u = q[1] / q[0];
    double v = q[2] / q[0];
    double p = beta * q[3];
    f[0] = q[1];
    f[1] = q[1] * u + p;
    f[2] = q[1] * v;
    f[3] = u;
}

/* Sec. 2.1.3: eigenvalues lambda_{1,2} = u, lambda_{4,5} = (u +- c)/2, c = sqrt(u^2 + 4 beta/rho),
 * and the right/left eigenvector matrices R_x, L_x as printed, with the w row and column
 * removed (2D). */
void orc_eigen(const double q[4], double beta, double R[16], double L[16], double lam[4])
{
    double rho = q[0];
    double u = q[1] / rho;
    double v = q[2] / rho;
    double c = sqrt(u * u + 4.0 * beta / rho);
    double l4 = 0.5 * (u + c);
    double l5 = 0.5 * (u - c);

    double Rm[16] = {
        1.0, 0.0, l4,                    l5,
        u,   0.0, u * l4 + beta / rho,   u * l5 + beta / rho,
        0.0, 1.0, v * l4,                v * l5,
        0.0, 0.0, -l5 / rho,             -l4 / rho,
    };
    double Lm[16] = {
        1.0 + u * u * rho / beta,          -rho * u / beta,               0.0, -rho,
        u * u * v * rho / beta,            -u * v * rho / beta,           1.0, -rho * v,
        -u * l4 * rho / (beta * c),        l4 * rho / (beta * c),         0.0, rho / c,
        u * l5 * rho / (beta * c),         -l5 * rho / (beta * c),        0.0, -rho / c,
    };
    memcpy(R, Rm, sizeof Rm);
    memcpy(L, Lm, sizeof Lm);
    lam[0] = u;
    lam[1] = u;
    lam[2] = l4;
    lam[3] = l5;
}

/* |A_x| = R_x |Lambda_x| L_x (Sec. 2.1.3, used in Sec. 2.4.3). */
void orc_abs_jacobian(const double q[4], double beta, double absA[16])
{
    double R[16], L[16], lam[4];
    orc_eigen(q, beta, R, L, lam);
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) {
            double s = 0.0;
            for (int k = 0; k < 4; ++k) s += R[r * 4 + k] * fabs(lam[k]) * L[k * 4 + c];
            absA[r * 4 + c] = s;
        }
}

/* Sec. 2.4.3: F = (F(Q_R) + F(Q_L) - int_{Q_L}^{Q_R} |A| dQ) / 2, the integral along the straight
 * line Q_j = Q_L + (Q_R - Q_L)(xi_j + 1)/2 by three-point Gauss-Legendre (R12). */
void orc_osher_x(const double ql[4], const double qr[4], double beta, double f[4])
{
    const double xi[3] = {-sqrt(3.0 / 5.0), 0.0, sqrt(3.0 / 5.0)};
    const double w[3] = {5.0 / 9.0, 8.0 / 9.0, 5.0 / 9.0};
    double fl[4], fr[4], dq[4], integral[4] = {0.0, 0.0, 0.0, 0.0};

    orc_flux_phys(ql, beta, fl);
    orc_flux_phys(qr, beta, fr);
    for (int k = 0; k < 4; ++k) dq[k] = qr[k] - ql[k];

    for (int j = 0; j < 3; ++j) {
        double qj[4], A[16];
        double t = 0.5 * (xi[j] + 1.0);
        for (int k = 0; k < 4; ++k) qj[k] = ql[k] + dq[k] * t;
        orc_abs_jacobian(qj, beta, A);
        for (int r = 0; r < 4; ++r) {
            double s = 0.0;
            for (int c = 0; c < 4; ++c) s += A[r * 4 + c] * dq[c];
            integral[r] += 0.5 * w[j] * s;
        }
    }
    for (int k = 0; k < 4; ++k) f[k] = 0.5 * (fr[k] + fl[k] - integral[k]);
}

/* Sec. 2.4.2: F = (F(Q_R) + F(Q_L) - |A~| (Q_R - Q_L)) / 2 with |A~| = R |Lambda| L at the Roe
 * average rho~ = sqrt(rho_L rho_R), u~ = (sqrt(rho_L) u_L + sqrt(rho_R) u_R)/(sqrt(rho_L) +
 * sqrt(rho_R)), v~ alike (R15). */
void orc_roe_x(const double ql[4], const double qr[4], double beta, double f[4])
{
    double rl = ql[0], rr = qr[0];
    double ul = ql[1] / rl, ur = qr[1] / rr;
    double vl = ql[2] / rl, vr = qr[2] / rr;
    double sl = sqrt(rl), sr = sqrt(rr);
    double rt = sqrt(rl * rr);
    double ut = (sl * ul + sr * ur) / (sl + sr);
    double vt = (sl * vl + sr * vr) / (sl + sr);
    double qt[4] = {rt, rt * ut, rt * vt, 0.0};
    double A[16], fl[4], fr[4];
    orc_abs_jacobian(qt, beta, A);
    orc_flux_phys(ql, beta, fl);
    orc_flux_phys(qr, beta, fr);
    for (int r = 0; r < 4; ++r) {
        double s = 0.0;
        for (int c = 0; c < 4; ++c) s += A[r * 4 + c] * (qr[c] - ql[c]);
        f[r] = 0.5 * (fr[r] + fl[r] - s);
    }
}

/* Sec. 2.4.1: acoustic speeds S_L = (u_L - c_L)/2 = lambda_5,L and S_R = (u_R + c_R)/2 =
 * lambda_4,R; the star velocity, pressure and densities as printed. */
void orc_bassi_star(const double ql[4], const double qr[4], double beta, double star[6])
{
    double rl = ql[0], rr = qr[0];
    double ul = ql[1] / rl, ur = qr[1] / rr;
    double pl = beta * ql[3], pr = beta * qr[3];
    double cl = sqrt(ul * ul + 4.0 * beta / rl);
    double cr = sqrt(ur * ur + 4.0 * beta / rr);
    double l4l = 0.5 * (ul + cl), l5l = 0.5 * (ul - cl);
    double l4r = 0.5 * (ur + cr), l5r = 0.5 * (ur - cr);
    double us = (pr - pl + rr * ur * l5r - rl * ul * l4l) / (rr * l5r - rl * l4l);
    double ps = pr + rr * l5r * (ur - us);
    star[0] = l5l;
    star[1] = l4r;
    star[2] = us;
    star[3] = ps;
    star[4] = rl * l4l / (us - l5l);
    star[5] = rr * l5r / (us - l4r);
}

/* Sec. 2.4.1: the tangential velocity changes only across the contact; the exact solution at
 * xi = x/tau is Q_L left of the acoustic fan, Q_R right of it, and inside it the left or right
 * star state by the side of the contact.  (If the contact leaves the fan, the solver's
 * assumption fails; the sampler still returns Q_L and Q_R outside the fan.) */
void orc_exact_sample(const double ql[4], const double qr[4], double beta, double xi, double q[4])
{
    double st[6];
    orc_bassi_star(ql, qr, beta, st);
    if (xi < st[0]) {
        for (int k = 0; k < 4; ++k) q[k] = ql[k];
    } else if (xi >= st[1]) {
        for (int k = 0; k < 4; ++k) q[k] = qr[k];
    } else if (xi < st[2]) {
        double v = ql[2] / ql[0];
        q[0] = st[4];
        q[1] = st[4] * st[2];
        q[2] = st[4] * v;
        q[3] = st[3] / beta;
    } else {
        double v = qr[2] / qr[0];
        q[0] = st[5];
        q[1] = st[5] * st[2];
        q[2] = st[5] * v;
        q[3] = st[3] / beta;
    }
}

void orc_bassi_x(const double ql[4], const double qr[4], double beta, double f[4])
{
    double q[4];
    orc_exact_sample(ql, qr, beta, 0.0, q);
    orc_flux_phys(q, beta, f);
}

/* Sec. 2.4: rotate to an x-split problem with R(n), built from n by Algorithm 2, then rotate the
 * flux back with R^T.  In 2D the state is (rho, rho u, rho v, p/beta) and only n and t1 enter. */
void orc_face_flux_kind(const double qa[4], const double qb[4], double nx, double ny, double beta,
                        int kind, double f[4])
{
    double t1x, t1y;
    if (nx == 0.0) {
        t1x = 1.0;
        t1y = 0.0;
    } else if (ny == 0.0) {
        t1x = 0.0;
        t1y = 1.0;
    } else {
        double h = sqrt(nx * nx + ny * ny);
        t1x = ny / h;
        t1y = -nx / h;
    }
    double Rm[16] = {
        1.0, 0.0, 0.0, 0.0,
        0.0, nx,  ny,  0.0,
        0.0, t1x, t1y, 0.0,
        0.0, 0.0, 0.0, 1.0,
    };
    double ql[4], qr[4], fx[4];
    for (int r = 0; r < 4; ++r) {
        ql[r] = 0.0;
        qr[r] = 0.0;
        for (int c = 0; c < 4; ++c) {
            ql[r] += Rm[r * 4 + c] * qa[c];
            qr[r] += Rm[r * 4 + c] * qb[c];
        }
    }
    if (kind == ORC_FLUX_ROE)
        orc_roe_x(ql, qr, beta, fx);
    else if (kind == ORC_FLUX_BASSI)
        orc_bassi_x(ql, qr, beta, fx);
    else
        orc_osher_x(ql, qr, beta, fx);
    for (int r = 0; r < 4; ++r) {
        f[r] = 0.0;
        for (int c = 0; c < 4; ++c) f[r] += Rm[c * 4 + r] * fx[c];
    }
}

void orc_face_flux(const double qa[4], const double qb[4], double nx, double ny, double beta,
                   double f[4])
{
    orc_face_flux_kind(qa, qb, nx, ny, beta, ORC_FLUX_OSHER, f);
}

/* ------------------------------------------------------------------------------------------ */
/* Grid                                                                                       */
/* ------------------------------------------------------------------------------------------ */

typedef struct {
    double r, u, v, p; /* primitive W */
} prim;

/* A cell or a ghost as the reconstruction sees it: W, limited gradients of rho, u, v and the new
 * pressure gradient. */
typedef struct {
    prim w;
    double gx[3], gy[3]; /* d/dx and d/dy of rho, u, v */
    double px, py;       /* new pressure gradient */
} entity;

typedef struct {
    const orc_problem *pb;
    int nx, ny;
    size_t n;
    double dx, dy;
} geom;

static size_t at(const geom *g, int i, int j) { return (size_t)j * (size_t)g->nx + (size_t)i; }

static int is_solid(const geom *g, int i, int j)
{
    return g->pb->solid != NULL && g->pb->solid[at(g, i, j)] != 0;
}

/* R8: mirror image across a wall whose normal lies along axis (0 = x, 1 = y): rho, p kept; with
 * no-slip both velocity components are negated, with free slip only the normal one. */
static int g_slip; /* set per call from the problem (single-threaded oracle) */

static prim mirror_axis(prim w, int axis)
{
    if (!g_slip || axis == 0) w.u = -w.u;
    if (!g_slip || axis == 1) w.v = -w.v;
    return w;
}

/* What lies across the face of cell (i,j) in direction (di,dj): a fluid cell (after periodic
 * wrapping; its index in *idx), a wall (domain wall or solid cell) or a zero-gradient side. */
enum { SIDE_FLUID = 0, SIDE_WALL = 1, SIDE_OPEN = 2 };

static int side_of(const geom *g, int s)
{
    return g->pb->bc[s] == ORC_BC_TRANSMISSIVE ? SIDE_OPEN : SIDE_WALL;
}

static int neighbour_kind(const geom *g, int i, int j, int di, int dj, size_t *idx)
{
    int ni = i + di, nj = j + dj;
    if (ni < 0) {
        if (g->pb->bc[0] != ORC_BC_PERIODIC) return side_of(g, 0);
        ni += g->nx;
    }
    if (ni >= g->nx) {
        if (g->pb->bc[1] != ORC_BC_PERIODIC) return side_of(g, 1);
        ni -= g->nx;
    }
    if (nj < 0) {
        if (g->pb->bc[2] != ORC_BC_PERIODIC) return side_of(g, 2);
        nj += g->ny;
    }
    if (nj >= g->ny) {
        if (g->pb->bc[3] != ORC_BC_PERIODIC) return side_of(g, 3);
        nj -= g->ny;
    }
    if (is_solid(g, ni, nj)) return SIDE_WALL;
    *idx = at(g, ni, nj);
    return SIDE_FLUID;
}

static int neighbour(const geom *g, int i, int j, int di, int dj, size_t *idx)
{
    return neighbour_kind(g, i, j, di, dj, idx) == SIDE_FLUID;
}

/* Image across a wall (R8) or a zero-gradient side (R13). */
static prim reflect(prim w, int axis, int kind)
{
    return kind == SIDE_WALL ? mirror_axis(w, axis) : w;
}

/* The value fluid cell (i,j) sees at its neighbour (i+di, j+dj): the neighbour's W, or across a
 * wall or zero-gradient side the ghost, which reflects cell (i,j) itself (R8, R9, R13). */
static prim seen(const geom *g, const prim *W, int i, int j, int di, int dj)
{
    size_t nb;
    int kind = neighbour_kind(g, i, j, di, dj, &nb);
    if (kind == SIDE_FLUID) return W[nb];
    return reflect(W[at(g, i, j)], di != 0 ? 0 : 1, kind);
}

/* Limited gradients of rho, u, v from a five-point stencil (Sec. 2.3.1, R1). */
static void stencil_gradient(const geom *g, prim c, prim xm, prim xp, prim ym, prim yp,
                             double gx[3], double gy[3])
{
    double k = g->pb->k, dx = g->dx, dy = g->dy;
    gx[0] = orc_limiter((xp.r - c.r) / dx, (c.r - xm.r) / dx, k);
    gx[1] = orc_limiter((xp.u - c.u) / dx, (c.u - xm.u) / dx, k);
    gx[2] = orc_limiter((xp.v - c.v) / dx, (c.v - xm.v) / dx, k);
    gy[0] = orc_limiter((yp.r - c.r) / dy, (c.r - ym.r) / dy, k);
    gy[1] = orc_limiter((yp.u - c.u) / dy, (c.u - ym.u) / dy, k);
    gy[2] = orc_limiter((yp.v - c.v) / dy, (c.v - ym.v) / dy, k);
}

/* Sec. 2.3.2, new method: dp/dx = -d(rho u)/dt - d(rho u^2)/dx - d(rho u v)/dy + rho g_x with the
 * products expanded by the product rule and the derivatives taken from the limited gradients;
 * dp/dy by exchanging x and y (R7). */
static void new_pressure_gradient(prim w, const double gx[3], const double gy[3], double d_ru,
                                  double d_rv, double rho0, double grav_x, double grav_y,
                                  double *px, double *py)
{
    double r = w.r, u = w.u, v = w.v;
    double rx = gx[0], ux = gx[1], vx = gx[2];
    double ry = gy[0], uy = gy[1], vy = gy[2];
    *px = -d_ru - (u * u * rx + 2.0 * r * u * ux) - (u * v * ry + r * u * vy + r * v * uy)
          + rho0 * grav_x;
    *py = -d_rv - (u * v * rx + r * u * vx + r * v * ux) - (v * v * ry + 2.0 * r * v * vy)
          + rho0 * grav_y;
}

/* Pressure gradient of an entity with the stencil (xm, xp, ym, yp) around c, by the method the
 * problem asks for (Sec. 2.3.2, R14); grav is the gravity at the entity (reversed in wall
 * ghosts). */
static void pressure_gradient(const geom *g, prim c, prim xm, prim xp, prim ym, prim yp,
                              const double gx[3], const double gy[3], double d_ru, double d_rv,
                              double rho0, double grav_x, double grav_y, double *px, double *py)
{
    const orc_problem *pb = g->pb;
    double dx = g->dx, dy = g->dy;
    if (pb->pgrad == ORC_PGRAD_LIMITER) {
        *px = orc_limiter((xp.p - c.p) / dx, (c.p - xm.p) / dx, pb->pk);
        *py = orc_limiter((yp.p - c.p) / dy, (c.p - ym.p) / dy, pb->pk);
    } else if (pb->pgrad == ORC_PGRAD_SPLIT) {
        /* one-sided dynamic gradients minus the hydrostatic ones (rho_{i-1} + rho_i) g/2 and
           (rho_i + rho_{i+1}) g/2 give the kinematic gradients; limit them, add rho_i g */
        double kxr = (xp.p - c.p) / dx - 0.5 * (c.r + xp.r) * grav_x;
        double kxl = (c.p - xm.p) / dx - 0.5 * (xm.r + c.r) * grav_x;
        double kyr = (yp.p - c.p) / dy - 0.5 * (c.r + yp.r) * grav_y;
        double kyl = (c.p - ym.p) / dy - 0.5 * (ym.r + c.r) * grav_y;
        *px = c.r * grav_x + orc_limiter(kxr, kxl, pb->pk);
        *py = c.r * grav_y + orc_limiter(kyr, kyl, pb->pk);
    } else {
        new_pressure_gradient(c, gx, gy, d_ru, d_rv, rho0, grav_x, grav_y, px, py);
    }
}

/* Per-cell stage-0 data of one pseudo-iteration (R6). */
typedef struct {
    double *D;    /* [3][n] real-time term I_C dQ/dt for rho, rho u, rho v */
    double *rho0; /* [n] */
    double *dtau; /* [n] */
    double B0;    /* leading BDF coefficient (Table 1), for alpha_PI */
} frozen;

/* The ghost across the face of fluid cell (i,j) in direction (di,dj) (R8, R9, R13). */
static void ghost_entity(const geom *g, const prim *W, const frozen *fz, int i, int j, int di,
                         int dj, entity *e)
{
    size_t a = at(g, i, j), nb;
    int axis = (di != 0) ? 0 : 1;
    int kind = neighbour_kind(g, i, j, di, dj, &nb);
    prim wa = W[a];
    prim c = reflect(wa, axis, kind);
    prim far = reflect(seen(g, W, i, j, -di, -dj), axis, kind); /* outer neighbour: image of a - d */
    prim xm, xp, ym, yp;
    if (di != 0) {
        ym = reflect(seen(g, W, i, j, 0, -1), axis, kind);
        yp = reflect(seen(g, W, i, j, 0, +1), axis, kind);
        if (di > 0) {
            xm = wa;
            xp = far;
        } else {
            xm = far;
            xp = wa;
        }
    } else {
        xm = reflect(seen(g, W, i, j, -1, 0), axis, kind);
        xp = reflect(seen(g, W, i, j, +1, 0), axis, kind);
        if (dj > 0) {
            ym = wa;
            yp = far;
        } else {
            ym = far;
            yp = wa;
        }
    }
    e->w = c;
    stencil_gradient(g, c, xm, xp, ym, yp, e->gx, e->gy);
    /* a wall ghost's sources are mirrored like its state and gravity is reversed in it; a
       zero-gradient ghost keeps both */
    double d_ru = fz->D[1 * g->n + a], d_rv = fz->D[2 * g->n + a];
    double sg = 1.0;
    if (kind == SIDE_WALL) {
        if (!g_slip || axis == 0) d_ru = -d_ru;
        if (!g_slip || axis == 1) d_rv = -d_rv;
        sg = -1.0;
    }
    pressure_gradient(g, c, xm, xp, ym, yp, e->gx, e->gy, d_ru, d_rv, fz->rho0[a],
                      sg * g->pb->gx, sg * g->pb->gy, &e->px, &e->py);
}

/* Reconstructed conserved state of entity e at its face in direction (di,dj): W + grad.(x_f-x_e)
 * (Sec. 2.3.1 with R1-R3), then Q = (rho, rho u, rho v, p/beta). */
static void face_state(const geom *g, const entity *e, int di, int dj, double q[4])
{
    double r, u, v, p;
    if (di != 0) {
        double h = 0.5 * g->dx * (double)di;
        r = e->w.r + e->gx[0] * h;
        u = e->w.u + e->gx[1] * h;
        v = e->w.v + e->gx[2] * h;
        p = e->w.p + e->px * h;
    } else {
        double h = 0.5 * g->dy * (double)dj;
        r = e->w.r + e->gy[0] * h;
        u = e->w.u + e->gy[1] * h;
        v = e->w.v + e->gy[2] * h;
        p = e->w.p + e->py * h;
    }
    q[0] = r;
    q[1] = r * u;
    q[2] = r * v;
    q[3] = p / g->pb->beta;
}

/* Local pseudo-time step (Sec. 2.2.3): dtau = CFL |Omega| / (Lx + Ly), Lx = (|u| + c_x) dS_x / 2,
 * dS_x = dy, dS_y = dx in 2D (R11). */
static double local_dtau(const geom *g, double rho, double u, double v)
{
    double beta = g->pb->beta;
    double cx = sqrt(u * u + 4.0 * beta / rho);
    double cy = sqrt(v * v + 4.0 * beta / rho);
    double lx = 0.5 * (fabs(u) + cx) * g->dy;
    double ly = 0.5 * (fabs(v) + cy) * g->dx;
    return g->pb->cfl * (g->dx * g->dy) / (lx + ly);
}

static int valid_problem(const orc_problem *pb)
{
    if (pb == NULL || pb->nx < 1 || pb->ny < 1) return 0;
    if (!(pb->lx > 0.0) || !(pb->ly > 0.0) || !(pb->beta > 0.0)) return 0;
    if (pb->stages < 1 || pb->stages > 8) return 0;
    if (!(pb->cfl > 0.0) || !(pb->k >= 1.0 && pb->k <= 2.0)) return 0;
    if (pb->bdf < 1 || pb->bdf > 3) return 0;
    if (pb->wall_slip != 0 && pb->wall_slip != 1) return 0;
    if (pb->flux < ORC_FLUX_OSHER || pb->flux > ORC_FLUX_BASSI) return 0;
    if (pb->pgrad < ORC_PGRAD_NEW || pb->pgrad > ORC_PGRAD_SPLIT) return 0;
    if (pb->pgrad != ORC_PGRAD_NEW && !(pb->pk >= 1.0 && pb->pk <= 2.0)) return 0;
    for (int s = 0; s < 4; ++s)
        if (pb->bc[s] != ORC_BC_WALL && pb->bc[s] != ORC_BC_PERIODIC &&
            pb->bc[s] != ORC_BC_TRANSMISSIVE)
            return 0;
    if ((pb->bc[0] == ORC_BC_PERIODIC) != (pb->bc[1] == ORC_BC_PERIODIC)) return 0;
    if ((pb->bc[2] == ORC_BC_PERIODIC) != (pb->bc[3] == ORC_BC_PERIODIC)) return 0;
    return 1;
}

/* Stage-0 data (Algorithm 1 before the Runge-Kutta loop): real-time term
 * (B0 Q^0 + B1 Q^n + B2 Q^{n-1} + B3 Q^{n-2})/dt on the I_C = 1 components (Table 1, R16),
 * rho^0 for the body force, and the pseudo-time step.  Q arrays are internal-form [4][n]. */
static void freeze_sources(const geom *g, const double *Q0, const double *Qn, const double *Qnm1,
                           const double *Qnm2, double dt, frozen *fz)
{
    size_t n = g->n;
    int order = 1;
    if (g->pb->bdf >= 2 && Qnm1 != NULL) order = 2;
    if (g->pb->bdf >= 3 && Qnm1 != NULL && Qnm2 != NULL) order = 3;
    double B[4] = {1.0, -1.0, 0.0, 0.0};
    if (order == 2) {
        B[0] = 1.5;
        B[1] = -2.0;
        B[2] = 0.5;
    } else if (order == 3) {
        B[0] = 11.0 / 6.0;
        B[1] = -3.0;
        B[2] = 1.5;
        B[3] = -1.0 / 3.0;
    }
    double dmin = INFINITY;
    ORC_ROWS_MIN(dmin)
    for (int j = 0; j < g->ny; ++j)
        for (int i = 0; i < g->nx; ++i) {
            size_t c = at(g, i, j);
            if (is_solid(g, i, j)) continue;
            for (int k = 0; k < 3; ++k) {
                double d = 0.0;
                if (dt > 0.0) {
                    double num = B[0] * Q0[k * n + c] + B[1] * Qn[k * n + c];
                    if (order >= 2) num += B[2] * Qnm1[k * n + c];
                    if (order >= 3) num += B[3] * Qnm2[k * n + c];
                    d = num / dt;
                }
                fz->D[k * n + c] = d;
            }
            fz->rho0[c] = Q0[c];
            fz->dtau[c] = local_dtau(g, Q0[c], Q0[n + c] / Q0[c], Q0[2 * n + c] / Q0[c]);
            if (fz->dtau[c] < dmin) dmin = fz->dtau[c];
        }
    if (!g->pb->local_dtau)
        for (size_t c = 0; c < n; ++c) fz->dtau[c] = dmin;
    fz->B0 = B[0];
}

/* Entity of fluid cell (i,j) and of its neighbours, for the face in direction (di,dj). */
static void side_entities(const geom *g, const prim *W, const entity *E, const frozen *fz, int i,
                          int j, int di, int dj, const entity **out_nb, entity *ghost)
{
    size_t nb;
    if (neighbour(g, i, j, di, dj, &nb)) {
        *out_nb = &E[nb];
    } else {
        ghost_entity(g, W, fz, i, j, di, dj, ghost);
        *out_nb = ghost;
    }
}

/* One Runge-Kutta stage (eq. 24) on internal-form arrays.  R (nullable) receives the bracket
 * [4][n] with the p row as beta*R_(p/beta). */
static void stage_internal(const geom *g, const double *Qprev, const double *Q0, const frozen *fz,
                           double dt, int s, double *Qout, double *R, orc_detail *det)
{
    const orc_problem *pb = g->pb;
    size_t n = g->n;
    int nx = g->nx, ny = g->ny;
    prim *W = (prim *)calloc(n, sizeof(prim));
    entity *E = (entity *)calloc(n, sizeof(entity));
    double *Fx = (double *)calloc(4 * (size_t)ny * (size_t)(nx + 1), sizeof(double));
    double *Fy = (double *)calloc(4 * (size_t)(ny + 1) * (size_t)nx, sizeof(double));
    size_t nfx = (size_t)ny * (size_t)(nx + 1), nfy = (size_t)(ny + 1) * (size_t)nx;

    /* primitives of the stage input */
    ORC_ROWS
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            size_t c = at(g, i, j);
            if (is_solid(g, i, j)) continue;
            W[c].r = Qprev[c];
            W[c].u = Qprev[n + c] / Qprev[c];
            W[c].v = Qprev[2 * n + c] / Qprev[c];
            W[c].p = pb->beta * Qprev[3 * n + c];
        }

    /* limited gradients and the new pressure gradient of every fluid cell */
    ORC_ROWS
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            size_t c = at(g, i, j);
            if (is_solid(g, i, j)) continue;
            prim xm = seen(g, W, i, j, -1, 0), xp = seen(g, W, i, j, +1, 0);
            prim ym = seen(g, W, i, j, 0, -1), yp = seen(g, W, i, j, 0, +1);
            E[c].w = W[c];
            stencil_gradient(g, W[c], xm, xp, ym, yp, E[c].gx, E[c].gy);
            pressure_gradient(g, W[c], xm, xp, ym, yp, E[c].gx, E[c].gy, fz->D[n + c],
                              fz->D[2 * n + c], fz->rho0[c], pb->gx, pb->gy, &E[c].px, &E[c].py);
        }

    /* x-faces: face i is the left face of cell i, between cells i-1 and i */
    ORC_ROWS
    for (int j = 0; j < ny; ++j)
        for (int f = 0; f <= nx; ++f) {
            int il = f - 1, ir = f;
            int per = (pb->bc[0] == ORC_BC_PERIODIC);
            if (per && f == nx) continue; /* same face as f = 0 */
            if (per && il < 0) il += nx;
            int lf = (il >= 0 && !is_solid(g, il, j));
            int rf = (ir < nx && !is_solid(g, ir, j));
            double qa[4], qb[4], flux[4] = {0.0, 0.0, 0.0, 0.0};
            entity ghost;
            const entity *ea, *eb;
            if (lf) {
                ea = &E[at(g, il, j)];
                side_entities(g, W, E, fz, il, j, +1, 0, &eb, &ghost);
            } else if (rf) {
                eb = &E[at(g, ir, j)];
                side_entities(g, W, E, fz, ir, j, -1, 0, &ea, &ghost);
            }
            if (lf || rf) {
                face_state(g, ea, +1, 0, qa);
                face_state(g, eb, -1, 0, qb);
                orc_face_flux_kind(qa, qb, 1.0, 0.0, pb->beta, pb->flux, flux);
            }
            for (int k = 0; k < 4; ++k) {
                Fx[k * nfx + (size_t)j * (nx + 1) + f] = flux[k];
                if (per && f == 0) Fx[k * nfx + (size_t)j * (nx + 1) + nx] = flux[k];
            }
        }

    /* y-faces: face j is the lower face of cell row j, between rows j-1 and j */
    ORC_ROWS
    for (int f = 0; f <= ny; ++f)
        for (int i = 0; i < nx; ++i) {
            int jl = f - 1, jr = f;
            int per = (pb->bc[2] == ORC_BC_PERIODIC);
            if (per && f == ny) continue;
            if (per && jl < 0) jl += ny;
            int lf = (jl >= 0 && !is_solid(g, i, jl));
            int rf = (jr < ny && !is_solid(g, i, jr));
            double qa[4], qb[4], flux[4] = {0.0, 0.0, 0.0, 0.0};
            entity ghost;
            const entity *ea, *eb;
            if (lf) {
                ea = &E[at(g, i, jl)];
                side_entities(g, W, E, fz, i, jl, 0, +1, &eb, &ghost);
            } else if (rf) {
                eb = &E[at(g, i, jr)];
                side_entities(g, W, E, fz, i, jr, 0, -1, &ea, &ghost);
            }
            if (lf || rf) {
                face_state(g, ea, 0, +1, qa);
                face_state(g, eb, 0, -1, qb);
                orc_face_flux_kind(qa, qb, 0.0, 1.0, pb->beta, pb->flux, flux);
            }
            for (int k = 0; k < 4; ++k) {
                Fy[k * nfy + (size_t)f * nx + i] = flux[k];
                if (per && f == 0) Fy[k * nfy + (size_t)ny * nx + i] = flux[k];
            }
        }

    /* bracket of eq. 24 and the update */
    double alpha = pb->alpha[s - 1];
    ORC_ROWS
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            size_t c = at(g, i, j);
            if (is_solid(g, i, j)) {
                for (int k = 0; k < 4; ++k) Qout[k * n + c] = Qprev[k * n + c];
                continue;
            }
            double body[4] = {0.0, fz->rho0[c] * pb->gx, fz->rho0[c] * pb->gy, 0.0};
            double Dk[4] = {fz->D[c], fz->D[n + c], fz->D[2 * n + c], 0.0};
            double dtau = fz->dtau[c];
            for (int k = 0; k < 4; ++k) {
                double divx = (Fx[k * nfx + (size_t)j * (nx + 1) + i + 1]
                               - Fx[k * nfx + (size_t)j * (nx + 1) + i]) / g->dx;
                double divy = (Fy[k * nfy + (size_t)(j + 1) * nx + i]
                               - Fy[k * nfy + (size_t)j * nx + i]) / g->dy;
                double bracket = -(divx + divy) - Dk[k] + body[k];
                double apI = 1.0;
                if (k < 3 && dt > 0.0) apI = 1.0 + fz->B0 * alpha * dtau / dt;
                Qout[k * n + c] = Q0[k * n + c] + (alpha * dtau / apI) * bracket;
                if (R) R[k * n + c] = (k == 3) ? pb->beta * bracket : bracket;
            }
        }

    if (det) {
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t c = at(g, i, j);
                if (is_solid(g, i, j)) continue;
                if (det->prim) {
                    det->prim[c] = W[c].r;
                    det->prim[n + c] = W[c].u;
                    det->prim[2 * n + c] = W[c].v;
                    det->prim[3 * n + c] = W[c].p;
                }
                if (det->grad) {
                    for (int k = 0; k < 3; ++k) {
                        det->grad[k * n + c] = E[c].gx[k];
                        det->grad[(4 + k) * n + c] = E[c].gy[k];
                    }
                    det->grad[3 * n + c] = E[c].px;
                    det->grad[7 * n + c] = E[c].py;
                }
                if (det->dtau) det->dtau[c] = fz->dtau[c];
            }
        if (det->fx) memcpy(det->fx, Fx, 4 * nfx * sizeof(double));
        if (det->fy) memcpy(det->fy, Fy, 4 * nfy * sizeof(double));
    }

    free(W);
    free(E);
    free(Fx);
    free(Fy);
}

/* ------------------------------------------------------------------------------------------ */
/* Public stage and step                                                                      */
/* ------------------------------------------------------------------------------------------ */

static void to_internal(const geom *g, const double *q, double *Q)
{
    size_t n = g->n;
    memcpy(Q, q, 3 * n * sizeof(double));
    for (size_t c = 0; c < n; ++c) Q[3 * n + c] = q[3 * n + c] / g->pb->beta;
}

static void to_external(const geom *g, const double *Q, double *q)
{
    size_t n = g->n;
    memcpy(q, Q, 3 * n * sizeof(double));
    for (size_t c = 0; c < n; ++c) q[3 * n + c] = g->pb->beta * Q[3 * n + c];
}

static void make_geom(const orc_problem *pb, geom *g)
{
    g_slip = (pb->wall_slip != 0);
    g->pb = pb;
    g->nx = pb->nx;
    g->ny = pb->ny;
    g->n = (size_t)pb->nx * (size_t)pb->ny;
    g->dx = pb->lx / pb->nx;
    g->dy = pb->ly / pb->ny;
}

int orc_stage(const orc_problem *pb, const double *qprev, const double *q0, const double *qn,
              const double *qnm1, const double *qnm2, double dt, int stage, double *qout,
              orc_detail *detail)
{
    if (!valid_problem(pb) || stage < 1 || stage > pb->stages) return -1;
    if (!qprev || !q0 || !qn || !qout) return -1;
    geom g;
    make_geom(pb, &g);
    size_t n = g.n;
    double *Qp = (double *)malloc(4 * n * sizeof(double));
    double *Q0 = (double *)malloc(4 * n * sizeof(double));
    double *Qn = (double *)malloc(4 * n * sizeof(double));
    double *Qm = qnm1 ? (double *)malloc(4 * n * sizeof(double)) : NULL;
    double *Qm2 = qnm2 ? (double *)malloc(4 * n * sizeof(double)) : NULL;
    double *Qo = (double *)malloc(4 * n * sizeof(double));
    double *R = (double *)calloc(4 * n, sizeof(double));
    frozen fz;
    fz.D = (double *)calloc(3 * n, sizeof(double));
    fz.rho0 = (double *)calloc(n, sizeof(double));
    fz.dtau = (double *)calloc(n, sizeof(double));
    to_internal(&g, qprev, Qp);
    to_internal(&g, q0, Q0);
    to_internal(&g, qn, Qn);
    if (Qm) to_internal(&g, qnm1, Qm);
    if (Qm2) to_internal(&g, qnm2, Qm2);
    freeze_sources(&g, Q0, Qn, Qm, Qm2, dt, &fz);
    stage_internal(&g, Qp, Q0, &fz, dt, stage, Qo, R, detail);
    to_external(&g, Qo, qout);
    if (detail && detail->resid) memcpy(detail->resid, R, 4 * n * sizeof(double));
    free(Qp);
    free(Q0);
    free(Qn);
    free(Qm);
    free(Qm2);
    free(Qo);
    free(R);
    free(fz.D);
    free(fz.rho0);
    free(fz.dtau);
    return 0;
}

/* Residual norms of the last stage's bracket over fluid cells (R10). */
static void residual_norms(const geom *g, const double *R, int norm_kind, double res[4])
{
    size_t n = g->n, count = 0;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int j = 0; j < g->ny; ++j)
        for (int i = 0; i < g->nx; ++i) {
            size_t c = at(g, i, j);
            if (is_solid(g, i, j)) continue;
            ++count;
            for (int k = 0; k < 4; ++k) {
                double r = R[k * n + c];
                if (norm_kind == 1) {
                    double a = fabs(r);
                    if (!(a <= acc[k])) acc[k] = a; /* NaN propagates */
                } else {
                    acc[k] += r * r;
                }
            }
        }
    for (int k = 0; k < 4; ++k)
        res[k] = (norm_kind == 1) ? acc[k] : sqrt(acc[k] / (double)(count ? count : 1));
}

int orc_step(const orc_problem *pb, double *q, const double *qnm1, const double *qnm2, double dt,
             int max_pseudo, double tol, int norm_kind, int *iters, double res[4])
{
    if (!valid_problem(pb) || q == NULL || max_pseudo < 0 || (norm_kind != 0 && norm_kind != 1))
        return -1;
    if (pb->alpha[pb->stages - 1] != 1.0) return -1;
    geom g;
    make_geom(pb, &g);
    size_t n = g.n;
    double *Q = (double *)malloc(4 * n * sizeof(double));
    double *Qn = (double *)malloc(4 * n * sizeof(double));
    double *Qm = qnm1 ? (double *)malloc(4 * n * sizeof(double)) : NULL;
    double *Qm2 = qnm2 ? (double *)malloc(4 * n * sizeof(double)) : NULL;
    double *Q0 = (double *)malloc(4 * n * sizeof(double));
    double *Qa = (double *)malloc(4 * n * sizeof(double));
    double *Qb = (double *)malloc(4 * n * sizeof(double));
    double *R = (double *)calloc(4 * n, sizeof(double));
    frozen fz;
    fz.D = (double *)calloc(3 * n, sizeof(double));
    fz.rho0 = (double *)calloc(n, sizeof(double));
    fz.dtau = (double *)calloc(n, sizeof(double));
    double norms[4] = {0.0, 0.0, 0.0, 0.0};
    int status = 0, m = 0;

    to_internal(&g, q, Q);
    if (Qm) to_internal(&g, qnm1, Qm);
    if (Qm2) to_internal(&g, qnm2, Qm2);
    memcpy(Qn, Q, 4 * n * sizeof(double)); /* Algorithm 1: Q^n <- Q */

    for (m = 0; m < max_pseudo;) {
        memcpy(Q0, Q, 4 * n * sizeof(double)); /* Q^m <- Q (eq. 23) */
        freeze_sources(&g, Q0, Qn, Qm, Qm2, dt, &fz);
        const double *prev = Q0;
        for (int s = 1; s <= pb->stages; ++s) {
            double *out = (s % 2) ? Qa : Qb;
            stage_internal(&g, prev, Q0, &fz, dt, s, out, (s == pb->stages) ? R : NULL, NULL);
            prev = out;
        }
        memcpy(Q, prev, 4 * n * sizeof(double));
        ++m;
        residual_norms(&g, R, norm_kind, norms);
        int bad = 0;
        for (int k = 0; k < 4; ++k)
            if (!isfinite(norms[k])) bad = 1;
        for (size_t c = 0; c < n && !bad; ++c)
            if (!(pb->solid && pb->solid[c]) && !(Q[c] > 0.0)) bad = 1;
        if (bad) {
            status = -2;
            break;
        }
        if (tol > 0.0 && norms[0] < tol && norms[1] < tol && norms[2] < tol && norms[3] < tol)
            break;
    }

    to_external(&g, Q, q);
    if (iters) *iters = m;
    if (res)
        for (int k = 0; k < 4; ++k) res[k] = norms[k];
    free(Q);
    free(Qn);
    free(Qm);
    free(Qm2);
    free(Q0);
    free(Qa);
    free(Qb);
    free(R);
    free(fz.D);
    free(fz.rho0);
    free(fz.dtau);
    return status;
}

/* Threads the row loops run on: 1 in the serial build. */
int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Sec. 2.2.4: dt = min over fluid cells of CFL_t |Omega| / (|u| dS_x + |v| dS_y), dS_x = dy and
 * dS_y = dx in 2D. */
double orc_realtime_dt(const orc_problem *pb, const double *q, double cfl_t)
{
    if (!valid_problem(pb) || q == NULL) return NAN;
    geom g;
    make_geom(pb, &g);
    size_t n = g.n;
    double dt = INFINITY;
    for (int j = 0; j < g.ny; ++j)
        for (int i = 0; i < g.nx; ++i) {
            size_t c = at(&g, i, j);
            if (is_solid(&g, i, j)) continue;
            double u = q[n + c] / q[c], v = q[2 * n + c] / q[c];
            double lam = fabs(u) * g.dy + fabs(v) * g.dx;
            double d = cfl_t * (g.dx * g.dy) / lam; /* +infinity at rest */
            if (d < dt) dt = d;
        }
    return dt;
}
