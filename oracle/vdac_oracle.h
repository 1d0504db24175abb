/*
 * vdac_oracle.h -- plain serial FP64 reference ("oracle") for the dual-time Godunov scheme of
 * Leakey, Glenis & Hewett, "Riemann solvers and pressure gradients in Godunov-type schemes for
 * variable density incompressible flows" (arXiv:2108.08769).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists so that the tests, the smoke check and the
 * CPU-baseline leg of the benchmark have something slow and obviously correct to compare the
 * GPU library against.  It shares no code, header or constant with the GPU library, and the
 * product path never calls it.
 *
 * Conventions
 *   - Arrays of cell data are structure-of-arrays planes, [field][ny][nx], x fastest.
 *   - At this interface the state is (rho, rho*u, rho*v, p) with the pressure itself; inside,
 *     the conserved vector of the compact form (Sec. 2.1.2) is Q = (rho, rho*u, rho*v, p/beta).
 *   - Single-point helpers (limiter, eigenstructure, fluxes) take Q in the internal form.
 */
#ifndef VDAC_ORACLE_H
#define VDAC_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_BC_WALL = 0, ORC_BC_PERIODIC = 1 };

typedef struct {
    int nx, ny;                 /* cells in x and y */
    double lx, ly;              /* domain extent; dx = lx/nx, dy = ly/ny */
    double gx, gy;              /* gravity */
    double beta;                /* artificial compressibility coefficient */
    int bc[4];                  /* sides x-, x+, y-, y+ : ORC_BC_WALL or ORC_BC_PERIODIC */
    const unsigned char *solid; /* nullable, [ny][nx]; nonzero = solid (obstacle) cell */
    int stages;                 /* Runge-Kutta stages s_max, 1..8 */
    double alpha[8];            /* RK coefficients alpha_1..alpha_smax */
    double cfl;                 /* pseudo-time Courant number CFL_tau */
    double k;                   /* k-limiter parameter: 1 minmod, 2 superbee */
    int local_dtau;             /* 1: local pseudo-time step per cell; 0: global minimum */
    int bdf;                    /* real-time derivative: 1 backward Euler, 2 BDF2 */
    int wall_slip;              /* 0: no-slip wall ghosts (both velocity components negated, as
                                   the paper states); 1: free-slip (normal component only) */
} orc_problem;

/* k-limiter G(a, b) of Sec. 2.3.1. */
double orc_limiter(double a, double b, double k);

/* Physical x-flux F_x,inv(Q) of Sec. 2.1.2 (2D: the w row dropped). */
void orc_flux_phys(const double q[4], double beta, double f[4]);

/* Eigenstructure of A_x (Sec. 2.1.3) in 2D: R (columns r1, r2, r4, r5), L (rows), and
 * lambda = (u, u, (u+c)/2, (u-c)/2).  Matrices are row-major 4x4. */
void orc_eigen(const double q[4], double beta, double R[16], double L[16], double lam[4]);

/* |A_x| = R |Lambda| L, row-major 4x4. */
void orc_abs_jacobian(const double q[4], double beta, double absA[16]);

/* Osher-Dumbser-Toro x-split flux (Sec. 2.4.3), three-point Gauss-Legendre on the straight
 * path in conserved variables. */
void orc_osher_x(const double ql[4], const double qr[4], double beta, double f[4]);

/* Flux through a face with unit normal (nx, ny) pointing from cell a into cell b: the states
 * are rotated with R(n) built by Algorithm 2, the x-split flux is taken, and R^T rotates back
 * (Sec. 2.4). */
void orc_face_flux(const double qa[4], const double qb[4], double nx, double ny, double beta,
                   double f[4]);

/* Intermediate results of one Runge-Kutta stage, for tests on tiny grids.  Every pointer is
 * nullable; sizes are given per member.  Fluid cells only; the rest are left untouched. */
typedef struct {
    double *prim;   /* [4][ny][nx]  W = (rho, u, v, p) of the stage input */
    double *grad;   /* [8][ny][nx]  rho_x, u_x, v_x, p_x, rho_y, u_y, v_y, p_y (p: new method) */
    double *fx;     /* [4][ny][nx+1] x-face fluxes (face i is the left face of cell i) */
    double *fy;     /* [4][ny+1][nx] y-face fluxes (face j is the lower face of cell j) */
    double *resid;  /* [4][ny][nx]  bracket of the update; p row reported as beta*R_(p/beta) */
    double *dtau;   /* [ny][nx]     pseudo-time step */
} orc_detail;

/* One Runge-Kutta stage s (1-based) of one pseudo-iteration.
 * qprev = Q^{s-1}, q0 = Q^0, qn = level n, qnm1 = level n-1 (BDF2 only, else nullable); all
 * [4][ny][nx] in the (rho, rho*u, rho*v, p) form.  qout receives Q^s in the same form.
 * dt <= 0 switches the real-time term off (pseudo-time only, alpha_PI = 1).
 * Returns 0, or -1 on invalid arguments. */
int orc_stage(const orc_problem *pb, const double *qprev, const double *q0, const double *qn,
              const double *qnm1, double dt, int stage, double *qout, orc_detail *detail);

/* One real-time step (Algorithm 1): level n <- q, then pseudo-iterations until every
 * residual norm is below tol (tol <= 0: exactly max_pseudo iterations).
 * q [4][ny][nx] is updated in place.  qnm1 is level n-1 for BDF2 (nullable: backward Euler).
 * norm_kind 0: RMS over fluid cells, 1: max norm.  iters and res (rho, rho*u, rho*v, p) are
 * nullable outputs.  Returns 0, -1 on invalid arguments, -2 if the iteration diverged
 * (non-finite residual or rho <= 0; q then holds the state after the failing iteration). */
int orc_step(const orc_problem *pb, double *q, const double *qnm1, double dt, int max_pseudo,
             double tol, int norm_kind, int *iters, double res[4]);

#ifdef __cplusplus
}
#endif
#endif
