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

enum { ORC_BC_WALL = 0, ORC_BC_PERIODIC = 1, ORC_BC_TRANSMISSIVE = 2 };
enum { ORC_FLUX_OSHER = 0, ORC_FLUX_ROE = 1, ORC_FLUX_BASSI = 2 };
enum { ORC_PGRAD_NEW = 0, ORC_PGRAD_LIMITER = 1, ORC_PGRAD_SPLIT = 2 };

typedef struct {
    int nx, ny;                 /* cells in x and y */
    double lx, ly;              /* domain extent; dx = lx/nx, dy = ly/ny */
    double gx, gy;              /* gravity */
    double beta;                /* artificial compressibility coefficient */
    int bc[4];                  /* sides x-, x+, y-, y+ : ORC_BC_WALL, ORC_BC_PERIODIC or
                                   ORC_BC_TRANSMISSIVE (zero gradient of every variable) */
    const unsigned char *solid; /* nullable, [ny][nx]; nonzero = solid (obstacle) cell */
    int stages;                 /* Runge-Kutta stages s_max, 1..8 */
    double alpha[8];            /* RK coefficients alpha_1..alpha_smax */
    double cfl;                 /* pseudo-time Courant number CFL_tau */
    double k;                   /* k-limiter parameter: 1 minmod, 2 superbee */
    int local_dtau;             /* 1: local pseudo-time step per cell; 0: global minimum */
    int bdf;                    /* real-time derivative: 1 backward Euler, 2 BDF2, 3 BDF3 */
    int wall_slip;              /* 0: no-slip wall ghosts (both velocity components negated, as
                                   the paper states); 1: free-slip (normal component only) */
    int flux;                   /* ORC_FLUX_OSHER, ORC_FLUX_ROE or ORC_FLUX_BASSI (Sec. 2.4) */
    int pgrad;                  /* ORC_PGRAD_NEW (Sec. 2.3.2), ORC_PGRAD_LIMITER (the k-limiter
                                   applied to p) or ORC_PGRAD_SPLIT (hydrostatic/kinematic split) */
    double pk;                  /* k of the limiter on p for ORC_PGRAD_LIMITER and _SPLIT */
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

/* Roe flux (Sec. 2.4.2): F = (F(Q_L) + F(Q_R) - |A(Q~)| (Q_R - Q_L))/2 at the Roe average Q~ of
 * rho, u, v. */
void orc_roe_x(const double ql[4], const double qr[4], double beta, double f[4]);

/* Exact Riemann solution of the x-split pseudo-time system (Sec. 2.4.1): star[6] receives the
 * acoustic wave speeds S_L, S_R, the star velocity and pressure u*, p* and the star densities
 * rho*L, rho*R. */
void orc_bassi_star(const double ql[4], const double qr[4], double beta, double star[6]);

/* The exact solution sampled at xi = x/tau: Q_L left of S_L, the left star state up to u*, the
 * right star state up to S_R, Q_R beyond. */
void orc_exact_sample(const double ql[4], const double qr[4], double beta, double xi, double q[4]);

/* Bassi flux: the physical flux of the exact solution at xi = 0. */
void orc_bassi_x(const double ql[4], const double qr[4], double beta, double f[4]);

/* Flux through a face with unit normal (nx, ny) pointing from cell a into cell b: the states
 * are rotated with R(n) built by Algorithm 2, the x-split flux is taken, and R^T rotates back
 * (Sec. 2.4). */
void orc_face_flux(const double qa[4], const double qb[4], double nx, double ny, double beta,
                   double f[4]);

/* The same with the x-split solver chosen by kind (ORC_FLUX_*). */
void orc_face_flux_kind(const double qa[4], const double qb[4], double nx, double ny, double beta,
                        int kind, double f[4]);

/* Global real-time step (Sec. 2.2.4): min over fluid cells of CFL_t |Omega| / (|u| dy + |v| dx)
 * for the state q [4][ny][nx] (rho, rho*u, rho*v, p); +infinity if the fluid is at rest. */
double orc_realtime_dt(const orc_problem *pb, const double *q, double cfl_t);

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
 * qprev = Q^{s-1}, q0 = Q^0, qn = level n, qnm1 = level n-1 and qnm2 = level n-2 (nullable; the
 * BDF order used is the smallest of pb->bdf and the levels given); all [4][ny][nx] in the
 * (rho, rho*u, rho*v, p) form.  qout receives Q^s in the same form.
 * dt <= 0 switches the real-time term off (pseudo-time only, alpha_PI = 1).
 * Returns 0, or -1 on invalid arguments. */
int orc_stage(const orc_problem *pb, const double *qprev, const double *q0, const double *qn,
              const double *qnm1, const double *qnm2, double dt, int stage, double *qout,
              orc_detail *detail);

/* One real-time step (Algorithm 1): level n <- q, then pseudo-iterations until every
 * residual norm is below tol (tol <= 0: exactly max_pseudo iterations).
 * q [4][ny][nx] is updated in place.  qnm1, qnm2 are levels n-1, n-2 (nullable; BDF order as in
 * orc_stage).  dt <= 0: pseudo-time only.
 * norm_kind 0: RMS over fluid cells, 1: max norm.  iters and res (rho, rho*u, rho*v, p) are
 * nullable outputs.  Returns 0, -1 on invalid arguments, -2 if the iteration diverged
 * (non-finite residual or rho <= 0; q then holds the state after the failing iteration). */
int orc_step(const orc_problem *pb, double *q, const double *qnm1, const double *qnm2, double dt,
             int max_pseudo, double tol, int norm_kind, int *iters, double res[4]);

/* Threads the row loops run on: 1 in the serial build, the OpenMP thread count in the build
 * made with -fopenmp (used only to time the oracle on all host cores). */
int orc_threads(void);

#ifdef __cplusplus
}
#endif
#endif
