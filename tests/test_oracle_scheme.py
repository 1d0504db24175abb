"""Pins of the oracle's full stage and real-time step against what the paper and the
mathematics fix: an independent high-precision evaluation on tiny grids, closed forms,
conservation, symmetry, exact discrete equilibria and the paper's own test settings."""
import csv
import os

import numpy as np
import pytest

import oracle
from paper_2108_08769_amd import workloads as wl
import brute_force_stage as bf

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
W, P = oracle.BC_WALL, oracle.BC_PERIODIC


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def problem(nx, ny, lx=1.0, ly=1.0, **kw):
    return oracle.Problem(nx, ny, lx, ly, **kw)


def hydro_profile(rho_col, g, h, p_top=0.0):
    """Exact discrete hydrostatic pressure along gravity: p_{j+1} - p_j = g h (rho_j + rho_{j+1})/2
    (the face pressures p_j + rho_j g h/2 from both sides then agree)."""
    p = np.zeros(len(rho_col))
    for j in range(len(rho_col) - 1):
        p[j + 1] = p[j] + g * h * (rho_col[j] + rho_col[j + 1]) / 2
    return p + p_top


# ---------------------------------------------------------------------------------------------
# One stage against an independent high-precision evaluation (explicit ghost arrays, eig |A|)
# ---------------------------------------------------------------------------------------------

@pytest.mark.parametrize("nx,ny,bc,k,seed,slip", [
    (3, 3, (W, W, W, W), 1.0, 1, False), (3, 3, (W, W, W, W), 2.0, 2, False),
    (4, 3, (P, P, W, W), 1.0, 3, False), (3, 4, (W, W, P, P), 2.0, 4, False),
    (2, 2, (W, W, W, W), 1.0, 5, False), (3, 3, (W, W, W, W), 1.0, 6, True),
    (4, 3, (P, P, W, W), 2.0, 7, True)])
def test_stage_against_brute_force(nx, ny, bc, k, seed, slip):
    lx, ly, gx, gy, beta, dt = 1.5, 0.9, 0.7, -9.81, 1100.0, 1e-3
    qp = wl.random_state(nx, ny, seed)
    q0 = wl.random_state(nx, ny, seed + 100)
    qn = wl.random_state(nx, ny, seed + 200)
    for s, alpha in ((1, 1.0 / 3.0), (3, 1.0)):
        pb = problem(nx, ny, lx, ly, gx=gx, gy=gy, beta=beta, bc=bc, k=k, wall_slip=slip)
        out, det = oracle.stage(pb, qp, q0, qn, dt, s)
        ref = bf.stage(nx, ny, lx, ly, gx, gy, beta, bc, qp, q0, qn, dt, alpha, 0.48, k, slip=slip)
        for key in ("prim", "grad", "fx", "fy", "resid", "dtau"):
            assert rel(det[key], ref[key]) < 1e-14, key
        assert rel(out, ref["qout"]) < 1e-14


# ---------------------------------------------------------------------------------------------
# Closed forms
# ---------------------------------------------------------------------------------------------

def test_free_stream_is_exact():
    """g = 0 and a uniform moving state on a periodic grid: every face sees the same state, so
    F(Q, Q) = F(Q) cancels exactly and the residual is exactly zero."""
    q = np.zeros((4, 5, 6))
    q[0], q[1], q[2], q[3] = 3.0, 3.0 * 0.7, 3.0 * -0.4, 12.5
    pb = problem(6, 5, gx=0.0, gy=0.0, beta=50.0, bc=(P, P, P, P))
    out, det = oracle.stage(pb, q, q, q, 1e-2, 1)
    assert np.all(det["resid"] == 0.0)
    q2, it, res, rc = oracle.step(pb, q, 1e-2, 5)
    assert rc == 0 and it == 5 and np.all(res == 0.0)
    np.testing.assert_array_equal(q2, q)


def uniform_dtau(rho, u, v, beta, cfl, dx, dy):
    cx, cy = np.sqrt(u * u + 4 * beta / rho), np.sqrt(v * v + 4 * beta / rho)
    return cfl * dx * dy / (0.5 * (abs(u) + cx) * dy + 0.5 * (abs(v) + cy) * dx)


def read_bdf_table():
    with open(os.path.join(GOLDEN, "bdf_coefficients_table1.csv")) as fh:
        rows = {r["scheme"]: r for r in csv.DictReader(l for l in fh if not l.startswith("#"))}
    return {k: [float(v[c]) if v[c] else 0.0 for c in ("B0", "B1", "B2", "B3")]
            for k, v in rows.items()}


def test_bdf_table_is_textbook():
    """Table 1 rows are the backward differentiation formulae: sum_s B_s (-s)^m = m (i.e. 0 for
    m = 0, 1 for m = 1, 0 above) for m up to the order, so polynomials of that degree are
    differentiated exactly."""
    for name, order in (("backward_euler", 1), ("bdf2", 2), ("bdf3", 3)):
        B = read_bdf_table()[name]
        for m in range(order + 1):
            moment = sum(b * (-s) ** m for s, b in enumerate(B))
            assert abs(moment - (1.0 if m == 1 else 0.0)) < 1e-15, (name, m)


@pytest.mark.parametrize("bdf", [1, 2])
def test_uniform_relaxation_closed_form(bdf):
    """A spatially uniform state on a fully periodic grid has zero flux divergence (all faces
    alike), so each pseudo-iteration solves dQ/dtau = -I_C dQ/dt + rho^0 g point-implicitly:
    Q^{m+1} = Q^m + dtau/alpha_PI (-(B0 Q^m + B1 Q^n + B2 Q^{n-1})/dt + rho^m g),
    alpha_PI = 1 + B0 dtau/dt on rho, rho u, rho v and 1 on p/beta (eqs. 24, 26,
    27; Table 1), with the local dtau of Sec. 2.2.3.  Two iterations, so that Q^0
    differs from Q^n and every coefficient enters."""
    B0, B1, B2, _ = read_bdf_table()["backward_euler" if bdf == 1 else "bdf2"]
    nx, ny, lx, ly, beta, gx, gy, dt, cfl = 4, 3, 2.0, 1.5, 700.0, 1.3, -9.81, 2e-3, 0.48

    def uni(rho, u, v, p):
        q = np.zeros((4, ny, nx))
        q[0], q[1], q[2], q[3] = rho, rho * u, rho * v, p
        return q

    q = uni(2.5, 0.4, -0.1, 7.0)
    qnm1 = uni(2.2, -0.2, 0.25, 6.0)
    pb = problem(nx, ny, lx, ly, gx=gx, gy=gy, beta=beta, bc=(P, P, P, P), bdf=bdf, cfl=cfl)
    out, it, res, rc = oracle.step(pb, q, dt, 2, qnm1=qnm1 if bdf == 2 else None)
    assert rc == 0 and it == 2
    dx, dy = lx / nx, ly / ny
    Qn = np.array([2.5, 2.5 * 0.4, 2.5 * -0.1, 7.0 / beta])   # Algorithm 1: Q^n <- Q
    Qnm1 = np.array([2.2, 2.2 * -0.2, 2.2 * 0.25, 6.0 / beta])
    Q = Qn.copy()
    for _ in range(2):
        rho, u, v = Q[0], Q[1] / Q[0], Q[2] / Q[0]
        cx, cy = np.sqrt(u * u + 4 * beta / rho), np.sqrt(v * v + 4 * beta / rho)
        dtau = cfl * dx * dy / (0.5 * (abs(u) + cx) * dy + 0.5 * (abs(v) + cy) * dx)
        D = (B0 * Q + B1 * Qn + (B2 * Qnm1 if bdf == 2 else 0.0)) / dt
        D[3] = 0.0
        body = np.array([0.0, rho * gx, rho * gy, 0.0])
        apI = np.array([1 + B0 * dtau / dt] * 3 + [1.0])
        Q = Q + dtau / apI * (-D + body)
    got = np.array([out[0, 0, 0], out[1, 0, 0], out[2, 0, 0], out[3, 0, 0] / beta])
    np.testing.assert_allclose(got, Q, rtol=1e-13, atol=0)
    assert np.all(out == out[:, :1, :1])


# ---------------------------------------------------------------------------------------------
# Well-balance of the new pressure gradient (Sec. 2.3.2, 2.5)
# ---------------------------------------------------------------------------------------------

def hydrostatic_state(nx, ny, ly, g, solid=None):
    dy = ly / ny
    yc = (np.arange(ny) + 0.5) * dy
    rho = np.where(yc < 0.5 * ly, 1000.0, 1.0)
    p = hydro_profile(rho, g, dy, p_top=123.0)
    q = np.zeros((4, ny, nx))
    q[0] = rho[:, None]
    q[3] = p[:, None]
    return q


@pytest.mark.parametrize("with_obstacle", [False, True])
def test_hydrostatic_equilibrium_is_exact(with_obstacle):
    """u = v = 0 with the exact discrete hydrostatic pressure: the new gradient reduces to
    rho g, minmod zeroes the density slope at the interface, the reversed-gravity wall ghosts
    reproduce the wall pressure, so the residual vanishes to rounding and the state stays put.
    Solid obstacle faces act as walls and keep the balance."""
    nx = ny = 64
    g = -9.81
    solid = None
    if with_obstacle:
        solid = np.zeros((ny, nx), np.uint8)
        solid[0:12, 40:46] = 1            # block on the floor
        solid[20:26, 10:20] = 1           # block in the water
        solid[44:50, 30:33] = 1           # block in the air
    q = hydrostatic_state(nx, ny, 1.0, g)
    pb = problem(nx, ny, gy=g, beta=1000.0, solid=solid)
    out, det = oracle.stage(pb, q, q, q, 1e-3, 1)
    fl = np.ones((ny, nx), bool) if solid is None else solid == 0
    scale = 1000.0 * abs(g)
    for k in range(4):
        assert np.abs(det["resid"][k][fl]).max() <= 1e-12 * scale, k
    q2, it, res, rc = oracle.step(pb, q, 1e-3, 60)
    assert rc == 0
    assert np.abs(q2[1:3] / q2[0]).max() <= 1e-12
    assert rel(q2[3], q[3]) <= 1e-13
    assert rel(q2[0], q[0]) <= 1e-13


def test_paper_hydrostatic_column_converges():
    """Sec. 3.2 (1D hydrostatic): 20 x 1 cells, walls, g = (9.81, 0), beta = 2000, three stages,
    CFL 0.98, local pseudo-time steps, one step of dt = 0.05 until the residuals fall below
    1e-5, starting from u = 0, p = 0.  The new gradient must converge to the hydrostatic
    solution with no spurious velocity."""
    nx, ny, lx = 20, 1, 1.0
    xc = (np.arange(nx) + 0.5) / nx
    rho = np.where(xc > 0.5, 1000.0, 1.0)       # gravity along +x: water on the +x side
    q = np.zeros((4, ny, nx))
    q[0] = rho
    pb = problem(nx, ny, lx, lx / nx, gx=9.81, gy=0.0, beta=2000.0, cfl=0.98)
    q2, it, res, rc = oracle.step(pb, q, 0.05, 20000, tol=1e-5)
    assert rc == 0 and it < 20000 and np.all(res < 1e-5)
    pe = hydro_profile(rho, 9.81, lx / nx)
    p = q2[3, 0]
    assert np.abs((p - p.mean()) - (pe - pe.mean())).max() <= 1e-8 * np.abs(pe).max()
    assert np.abs(q2[1] / q2[0]).max() <= 1e-8


def test_cfl_independence_of_converged_state():
    """At the incompressible limit the pseudo-time path does not matter: the converged state does
    not depend on CFL_tau."""
    nx, ny = 4, 12
    q = np.zeros((4, ny, nx))
    yc = (np.arange(ny) + 0.5) / ny
    q[0] = np.where(yc < 0.4, 1000.0, 1.0)[:, None]
    outs = []
    for cfl in (0.48, 0.3):
        pb = problem(nx, ny, 1.0, 1.0, gy=-9.81, beta=1000.0, cfl=cfl)
        q2, it, res, rc = oracle.step(pb, q, 1e-2, 50000, tol=1e-9)
        assert rc == 0 and it < 50000
        outs.append(q2)
    p0, p1 = outs[0][3] - outs[0][3].mean(), outs[1][3] - outs[1][3].mean()
    assert np.abs(p0 - p1).max() <= 1e-8 * np.abs(p0).max()
    assert np.abs(outs[0][1:3]).max() <= 1e-8 and np.abs(outs[1][1:3]).max() <= 1e-8


# ---------------------------------------------------------------------------------------------
# Conservation and symmetry
# ---------------------------------------------------------------------------------------------

def dam_state(nx, ny, lx, ly, double=False):
    xc = (np.arange(nx) + 0.5) * lx / nx
    yc = (np.arange(ny) + 0.5) * ly / ny
    water = (xc[None, :] < 1.0) & (yc[:, None] < 1.0)
    if double:
        water |= (xc[None, :] > lx - 1.0) & (yc[:, None] < 1.0)
    q = np.zeros((4, ny, nx))
    q[0] = np.where(water, 1000.0, 1.0)
    return q


def developed_dam(nx, ny, lx, ly, dt, slip):
    pb = problem(nx, ny, lx, ly, gy=-9.81, beta=1100.0, wall_slip=slip)
    q = dam_state(nx, ny, lx, ly)
    qa, _, _, _ = oracle.step(pb, q, dt, 3)           # a developed, non-trivial state
    qb, _, _, _ = oracle.step(pb, qa, dt, 2)
    return pb, qa, qb


@pytest.mark.parametrize("slip", [False, True])
def test_flux_divergence_telescopes(slip):
    """Each face flux enters its two cells with opposite signs (eq. 22), so summed
    over the tank the divergence reduces to the boundary fluxes:
    sum_i R_i |Omega| = -sum_i D_i |Omega| + sum_i B_i |Omega| - (net outward boundary flux)."""
    nx, ny, lx, ly, dt = 16, 8, 4.0, 2.0, 1e-3
    dx, dy = lx / nx, ly / ny
    pb, qa, qb = developed_dam(nx, ny, lx, ly, dt, slip)
    out, det = oracle.stage(pb, qb, qb, qa, dt, 2)
    for k in range(4):
        fx, fy = det["fx"][k], det["fy"][k]
        outflow = (fx[:, nx].sum() - fx[:, 0].sum()) * dy + (fy[ny, :].sum() - fy[0, :].sum()) * dx
        D = (qb[k] - qa[k]) / dt if k < 3 else 0.0 * qb[k]
        body = qb[0] * (-9.81) if k == 2 else 0.0 * qb[0]
        R = det["resid"][k] / (1100.0 if k == 3 else 1.0)
        lhs = R.sum() * dx * dy
        rhs = (-D.sum() + body.sum()) * dx * dy - outflow
        scale = (np.abs(R).sum() + np.abs(D).sum() + np.abs(body).sum()) * dx * dy
        assert abs(lhs - rhs) <= 1e-13 * scale, k


def test_wall_mass_flux():
    """With free-slip ghosts the wall is a true mirror: no mass and no p/beta flux cross it and a
    closed tank keeps sum R_rho = -sum D_rho to rounding.  With the paper's no-slip ghosts the
    new pressure gradient's cross terms change sign between cell and ghost, so the face
    pressures differ and a small mass flux crosses the wall where the flow runs along it."""
    nx, ny, lx, ly, dt = 16, 8, 4.0, 2.0, 1e-3
    for slip in (True, False):
        pb, qa, qb = developed_dam(nx, ny, lx, ly, dt, slip)
        out, det = oracle.stage(pb, qb, qb, qa, dt, 2)
        fx, fy = det["fx"], det["fy"]
        wall = max(np.abs(fx[0, :, 0]).max(), np.abs(fx[0, :, nx]).max(),
                   np.abs(fy[0, 0, :]).max(), np.abs(fy[0, ny, :]).max())
        scale = np.abs(fx[0]).max()
        if slip:
            assert wall <= 1e-14 * scale
            wall_p = max(np.abs(fx[3, :, 0]).max(), np.abs(fy[3, 0, :]).max())
            assert wall_p <= 1e-14 * np.abs(fx[3]).max()
            D = (qb[0] - qa[0]) / dt
            sc = np.abs(det["resid"][0]).sum() + np.abs(D).sum()
            assert abs(det["resid"][0].sum() + D.sum()) <= 1e-13 * sc
        else:
            assert wall > 1e-6 * scale


@pytest.mark.parametrize("slip", [False, True])
def test_mass_conserved_pseudo_time_only_global_step(slip):
    """The paper's Riemann-problem settings (Sec. 3.1: no gravity, no real-time term, one global
    pseudo-time step) with Table 2's RP2 states in a closed tank: total mass changes only by
    rounding.  The flow is one-dimensional, so even no-slip walls carry no cross terms."""
    with open(os.path.join(GOLDEN, "riemann_problems_table2.csv")) as fh:
        rp = [r for r in csv.DictReader(l for l in fh if not l.startswith("#"))][1]
    rp = {k: float(v) for k, v in rp.items()}
    nx, ny, lx, ly = 40, 2, 1.0, 0.05
    xc = (np.arange(nx) + 0.5) / nx
    left = xc < 0.5
    q = np.zeros((4, ny, nx))
    q[0] = np.where(left, rp["rho_L"], rp["rho_R"])
    q[1] = q[0] * np.where(left, rp["u_L"], rp["u_R"])
    q[3] = np.where(left, rp["p_L"], rp["p_R"])
    pb = problem(nx, ny, lx, ly, gx=0.0, gy=0.0, beta=rp["beta"], local_dtau=False,
                 wall_slip=slip)
    q2, it, res, rc = oracle.step(pb, q, 0.0, 30)
    assert rc == 0 and it == 30
    assert abs(q2[0].sum() - q[0].sum()) <= 1e-14 * q[0].sum()
    assert np.abs(q2[1]).max() > 1.0                  # the waves did move


def test_global_pseudo_step_is_minimum_of_local():
    nx, ny, lx, ly = 8, 6, 4.0, 2.0
    q = wl.random_state(nx, ny, 11)
    loc = problem(nx, ny, lx, ly, beta=300.0)
    glo = problem(nx, ny, lx, ly, beta=300.0, local_dtau=False)
    _, dl = oracle.stage(loc, q, q, q, 1e-3, 1)
    _, dg = oracle.stage(glo, q, q, q, 1e-3, 1)
    assert np.all(dg["dtau"] == dl["dtau"].min())


@pytest.mark.parametrize("obstacle", [False, True])
def test_mirror_symmetry(obstacle):
    """A setup symmetric about x = L/2 (double dam break) stays symmetric: rho, v, p even and u
    odd, with no-slip walls, reversed-gravity ghosts and (optionally) a symmetric obstacle."""
    nx, ny, lx, ly = 24, 10, 4.0, 2.0
    solid = None
    if obstacle:
        solid = np.zeros((ny, nx), np.uint8)
        solid[0:3, 10:14] = 1
        solid[6:8, 3:5] = 1
        solid[6:8, nx - 5:nx - 3] = 1
    pb = problem(nx, ny, lx, ly, gy=-9.81, beta=1100.0, solid=solid)
    q = dam_state(nx, ny, lx, ly, double=True)
    for _ in range(2):
        q, it, res, rc = oracle.step(pb, q, 1e-3, 15)
        assert rc == 0
    m = q[:, :, ::-1]
    for k, sign in ((0, 1), (1, -1), (2, 1), (3, 1)):
        assert np.abs(q[k] - sign * m[k]).max() <= 1e-12 * np.abs(q[k]).max(), k
    assert np.abs(q[1]).max() > 1e-3                   # the flow did develop


def test_periodic_translation_is_bitwise():
    nx, ny, lx, ly = 16, 12, 1.0, 2.0
    q = wl.random_state(nx, ny, 21, rho_range=(1.0, 3.0), vel=0.05, p_scale=1.0)
    pb = problem(nx, ny, lx, ly, gy=-1.0, beta=100.0, bc=(P, P, W, W))
    a, _, _, rca = oracle.step(pb, q, 1e-3, 4)
    b, _, _, rcb = oracle.step(pb, np.roll(q, 5, axis=2), 1e-3, 4)
    assert rca == 0 and rcb == 0
    np.testing.assert_array_equal(np.roll(a, 5, axis=2), b)


def test_transpose_symmetry():
    """Exchanging x and y (with u and v, gravity components and boundary kinds) transposes the
    result, to rounding (only the order of some additions changes)."""
    nx, ny, lx, ly = 10, 7, 2.0, 1.4
    q = wl.random_state(nx, ny, 31, rho_range=(1.0, 3.0), vel=0.3, p_scale=5.0)
    pb = problem(nx, ny, lx, ly, gx=1.5, gy=-9.81, beta=500.0, bc=(P, P, W, W))
    qt = np.stack([q[0].T, q[2].T, q[1].T, q[3].T])
    pbt = problem(ny, nx, ly, lx, gx=-9.81, gy=1.5, beta=500.0, bc=(W, W, P, P))
    a, _, _, rca = oracle.step(pb, q, 1e-3, 3)
    b, _, _, rcb = oracle.step(pbt, qt, 1e-3, 3)
    assert rca == 0 and rcb == 0
    at = np.stack([a[0].T, a[2].T, a[1].T, a[3].T])
    for k in range(4):
        assert rel(b[k], at[k]) <= 1e-12, k


# ---------------------------------------------------------------------------------------------
# Solid cells (not in the paper: each fluid-solid face is a wall)
# ---------------------------------------------------------------------------------------------

def test_solid_border_equals_smaller_tank_bitwise():
    """Solid columns along the right side and solid rows along the top turn the remaining fluid
    into a smaller walled tank: the result equals that tank's, bit for bit."""
    nx, ny, dx = 14, 9, 0.25
    big = dam_state(nx, ny, nx * dx, ny * dx)
    solid = np.zeros((ny, nx), np.uint8)
    solid[:, 11:] = 1
    solid[7:, :] = 1
    pb = problem(nx, ny, nx * dx, ny * dx, gy=-9.81, beta=1100.0, solid=solid)
    small = np.ascontiguousarray(big[:, :7, :11])
    pbs = problem(11, 7, 11 * dx, 7 * dx, gy=-9.81, beta=1100.0)
    a, _, _, rca = oracle.step(pb, big, 1e-3, 6)
    b, _, _, rcb = oracle.step(pbs, small, 1e-3, 6)
    assert rca == 0 and rcb == 0
    np.testing.assert_array_equal(a[:, :7, :11], b)
    np.testing.assert_array_equal(a[:, solid == 1], big[:, solid == 1])


def test_solid_wall_splits_into_independent_tanks():
    nx, ny, dx = 15, 6, 0.25
    q = wl.random_state(nx, ny, 41, rho_range=(1.0, 3.0), vel=0.2, p_scale=5.0)
    solid = np.zeros((ny, nx), np.uint8)
    solid[:, 6] = 1
    pb = problem(nx, ny, nx * dx, ny * dx, gy=-9.81, beta=900.0, solid=solid)
    a, _, _, rc = oracle.step(pb, q, 1e-3, 3)
    left = np.ascontiguousarray(q[:, :, :6])
    right = np.ascontiguousarray(q[:, :, 7:])
    bl, _, _, rcl = oracle.step(problem(6, ny, 6 * dx, ny * dx, gy=-9.81, beta=900.0), left, 1e-3, 3)
    br, _, _, rcr = oracle.step(problem(8, ny, 8 * dx, ny * dx, gy=-9.81, beta=900.0), right, 1e-3, 3)
    assert rc == 0 and rcl == 0 and rcr == 0
    np.testing.assert_array_equal(a[:, :, :6], bl)
    np.testing.assert_array_equal(a[:, :, 7:], br)


# ---------------------------------------------------------------------------------------------
# Errors
# ---------------------------------------------------------------------------------------------

def test_divergence_and_invalid_arguments():
    nx, ny = 6, 5
    q = dam_state(nx, ny, 3.0, 2.5)
    q[1, 2, 2] = np.nan
    pb = problem(nx, ny, 3.0, 2.5, gy=-9.81, beta=1100.0)
    _, it, res, rc = oracle.step(pb, q, 1e-3, 5)
    assert rc == -2 and it == 1
    q = dam_state(nx, ny, 3.0, 2.5)
    with pytest.raises(ValueError):
        oracle.step(problem(nx, ny, 3.0, 2.5, bc=(P, W, W, W)), q, 1e-3, 1)
    with pytest.raises(ValueError):
        oracle.step(problem(nx, ny, 3.0, 2.5, alpha=(0.3, 0.5, 0.9)), q, 1e-3, 1)
