"""Pins of the oracle's single-point pieces against what the paper and the mathematics fix.

Limiter (Sec. 2.3.1), physical flux and Jacobian (Sec. 2.1.2-2.1.3), eigenstructure, the
Osher-Dumbser-Toro flux (Sec. 2.4.3) and the face rotation (Sec. 2.4, Algorithm 2).
"""
import csv
import os

import numpy as np
import pytest
import scipy.integrate

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def riemann_table():
    rows = []
    with open(os.path.join(GOLDEN, "riemann_problems_table2.csv")) as fh:
        for r in csv.DictReader(line for line in fh if not line.startswith("#")):
            rows.append({k: float(v) for k, v in r.items()})
    return rows


def q_of(rho, u, v, p, beta):
    return np.array([rho, rho * u, rho * v, p / beta])


# ---------------------------------------------------------------------------------------------
# k-limiter: k = 1 is textbook minmod, k = 2 textbook superbee (Sec. 2.3.1)
# ---------------------------------------------------------------------------------------------

def textbook_minmod(a, b):
    if a * b <= 0:
        return 0.0
    return np.sign(a) * min(abs(a), abs(b))


def textbook_superbee(a, b):
    # Roe's superbee in slope form: maxmod(minmod(2a, b), minmod(a, 2b))
    s1, s2 = textbook_minmod(2 * a, b), textbook_minmod(a, 2 * b)
    return s1 if abs(s1) >= abs(s2) else s2


VALUES = [-3.0, -2.0, -1.5, -1.0, -0.25, 0.0, 0.25, 0.5, 1.0, 1.75, 2.0, 4.0]


@pytest.mark.parametrize("a", VALUES)
@pytest.mark.parametrize("b", VALUES)
def test_limiter_truth_tables(a, b):
    assert oracle.limiter(a, b, 1.0) == textbook_minmod(a, b)
    assert oracle.limiter(a, b, 2.0) == textbook_superbee(a, b)


def test_limiter_symmetry_oddness_and_zero():
    rng = np.random.default_rng(0)
    for a, b in rng.normal(size=(500, 2)) * 10:
        for k in (1.0, 1.5, 2.0):
            g = oracle.limiter(a, b, k)
            assert g == oracle.limiter(b, a, k)
            assert -g == oracle.limiter(-a, -b, k)
            assert oracle.limiter(a, 0.0, k) == 0.0
            assert oracle.limiter(0.0, b, k) == 0.0
            # TVD region: between 0 and k*min and never beyond max(|a|,|b|)
            assert abs(g) <= max(abs(a), abs(b)) + 0.0


# ---------------------------------------------------------------------------------------------
# Physical flux, Jacobian and eigenstructure (Sec. 2.1.2, 2.1.3)
# ---------------------------------------------------------------------------------------------

def test_physical_flux_hand_values():
    beta = 4.0
    # rho = 2, u = 3, v = 5, p = 7: F = (rho u, rho u^2 + p, rho u v, u) = (6, 25, 30, 3)
    f = oracle.flux_phys(q_of(2.0, 3.0, 5.0, 7.0, beta), beta)
    np.testing.assert_array_equal(f, [6.0, 25.0, 30.0, 3.0])


def flux_complex(q, beta):
    """F_x,inv of Sec. 2.1.2 on a complex state (for complex-step differentiation)."""
    rho, m, n, s = q
    u = m / rho
    return np.array([m, m * u + beta * s, m * n / rho, u])


def jacobian_complex_step(q, beta, h=1e-30):
    J = np.zeros((4, 4))
    for k in range(4):
        qc = q.astype(complex)
        qc[k] += 1j * h
        J[:, k] = flux_complex(qc, beta).imag / h
    return J


def jacobian_printed(q, beta):
    """A_x as printed in Sec. 2.1.3, with the w row and column removed."""
    rho, u, v = q[0], q[1] / q[0], q[2] / q[0]
    return np.array([[0.0, 1.0, 0.0, 0.0],
                     [-u * u, 2 * u, 0.0, beta],
                     [-u * v, v, u, 0.0],
                     [-u / rho, 1.0 / rho, 0.0, 0.0]])


STATES = [(1000.0, 0.3, -0.2, 5.0, 1100.0), (1.0, 1.0, 0.0, 0.1, 0.81), (0.00125, 1.0, 0.5, 0.1, 1.0),
          (1.4, 0.0, 0.0, 1.0, 1.0), (3.0, -2.5, 1.5, -40.0, 100.0), (1.0, 60.0, -3.0, 0.0, 1100.0)]


@pytest.mark.parametrize("rho,u,v,p,beta", STATES)
def test_printed_jacobian_is_flux_derivative(rho, u, v, p, beta):
    q = q_of(rho, u, v, p, beta)
    np.testing.assert_allclose(jacobian_printed(q, beta), jacobian_complex_step(q, beta),
                               rtol=1e-13, atol=1e-13 * (1 + u * u))


@pytest.mark.parametrize("rho,u,v,p,beta", STATES)
def test_eigenstructure(rho, u, v, p, beta):
    q = q_of(rho, u, v, p, beta)
    R, L, lam = oracle.eigen(q, beta)
    A = jacobian_complex_step(q, beta)
    scale = np.abs(R).max() * np.abs(L).max()
    assert np.abs(L @ R - np.eye(4)).max() <= 1e-14 * scale
    assert np.abs(A @ R - R @ np.diag(lam)).max() <= 1e-13 * np.abs(A).max() * np.abs(R).max()
    np.testing.assert_allclose(np.sort(lam), np.sort(np.linalg.eigvals(A).real), rtol=1e-12,
                               atol=1e-14)
    # lambda_4 > 0 > lambda_5 always (c > |u|), and u = l4 + l5
    assert lam[2] > 0 > lam[3]


@pytest.mark.parametrize("rho,u,v,p,beta", STATES)
def test_abs_jacobian_vs_numpy_eig(rho, u, v, p, beta):
    q = q_of(rho, u, v, p, beta)
    A = jacobian_complex_step(q, beta)
    w, V = np.linalg.eig(A)
    ref = (V @ np.diag(np.abs(w)) @ np.linalg.inv(V)).real
    got = oracle.abs_jacobian(q, beta)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


# ---------------------------------------------------------------------------------------------
# Osher-Dumbser-Toro flux (Sec. 2.4.3)
# ---------------------------------------------------------------------------------------------

def test_osher_consistency_bitwise():
    rng = np.random.default_rng(1)
    for _ in range(200):
        beta = float(rng.uniform(0.5, 2000))
        q = q_of(float(rng.uniform(0.01, 1000)), *rng.normal(size=2), float(rng.normal() * 100), beta)
        np.testing.assert_array_equal(oracle.osher_x(q, q, beta), oracle.flux_phys(q, beta))


def test_osher_stationary_contact_rp3():
    """RP3 of Table 2 is a stationary contact: u = 0 and equal pressures on both sides, so the
    exact flux is (0, p, 0, 0) and a contact-capturing solver must return it."""
    rp = riemann_table()[2]
    beta = rp["beta"]
    ql = q_of(rp["rho_L"], rp["u_L"], 0.0, rp["p_L"], beta)
    qr = q_of(rp["rho_R"], rp["u_R"], 0.0, rp["p_R"], beta)
    np.testing.assert_array_equal(oracle.osher_x(ql, qr, beta), [0.0, rp["p_L"], 0.0, 0.0])


def test_osher_constant_path_matrix():
    """With u = v = 0 and equal density on both sides only p/beta varies along the path, |A|
    depends on (rho, u, v) only and is constant, so the flux is exactly
    (F_L + F_R)/2 - |A| (Q_R - Q_L)/2 whatever the quadrature (weights sum to 2)."""
    for rho, beta, pl, pr in [(1000.0, 1100.0, 5.0, -3.0), (1.0, 1000.0, 1000.0, 0.01)]:
        ql, qr = q_of(rho, 0.0, 0.0, pl, beta), q_of(rho, 0.0, 0.0, pr, beta)
        A = jacobian_complex_step(ql, beta)
        w, V = np.linalg.eig(A)
        absA = (V @ np.diag(np.abs(w)) @ np.linalg.inv(V)).real
        ref = 0.5 * (oracle.flux_phys(ql, beta) + oracle.flux_phys(qr, beta)) - 0.5 * absA @ (qr - ql)
        got = oracle.osher_x(ql, qr, beta)
        np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


def abs_A_numpy(q, beta):
    A = jacobian_complex_step(q, beta)
    w, V = np.linalg.eig(A)
    return (V @ np.diag(np.abs(w)) @ np.linalg.inv(V)).real


def test_osher_three_point_rule_against_independent_evaluation():
    """The same path integral evaluated with numpy's Gauss-Legendre nodes and weights and an
    eigendecomposition-based |A|: agrees to rounding on the Table 2 states and random ones."""
    xg, wg = np.polynomial.legendre.leggauss(3)
    cases = []
    for rp in riemann_table():
        beta = rp["beta"]
        cases.append((q_of(rp["rho_L"], rp["u_L"], 0.0, rp["p_L"], beta),
                      q_of(rp["rho_R"], rp["u_R"], 0.0, rp["p_R"], beta), beta))
    rng = np.random.default_rng(2)
    for _ in range(30):
        beta = float(rng.uniform(1, 2000))
        cases.append((q_of(float(rng.uniform(1, 1000)), *rng.normal(size=2), float(rng.normal()) * 10, beta),
                      q_of(float(rng.uniform(1, 1000)), *rng.normal(size=2), float(rng.normal()) * 10, beta), beta))
    for ql, qr, beta in cases:
        dq = qr - ql
        integral = sum(0.5 * wj * abs_A_numpy(ql + dq * 0.5 * (xj + 1), beta) @ dq
                       for xj, wj in zip(xg, wg))
        ref = 0.5 * (oracle.flux_phys(ql, beta) + oracle.flux_phys(qr, beta) - integral)
        got = oracle.osher_x(ql, qr, beta)
        scale = np.abs(oracle.flux_phys(ql, beta)).max() + np.abs(oracle.flux_phys(qr, beta)).max() \
            + np.abs(integral).max()
        assert np.abs(got - ref).max() <= 2e-13 * scale, (ql, qr, beta, got, ref)


def test_osher_gauss_rule_is_sixth_order():
    """Three-point Gauss-Legendre is exact to degree 5.  The integrand |A(Q_L + s dQ)| dQ carries
    one factor of the jump and each s-derivative another, so against an adaptive quadrature of
    the exact path integral the error falls about 2^7 = 128 times when the jump is halved."""
    beta = 1100.0
    qc = q_of(500.0, 0.4, -0.3, 20.0, beta)
    dqdir = np.array([400.0, 150.0, -100.0, 0.02])
    errs = []
    for h in (0.25, 0.125):
        ql, qr = qc - 0.5 * h * dqdir, qc + 0.5 * h * dqdir
        dq = qr - ql
        exact, _ = scipy.integrate.quad_vec(lambda s: abs_A_numpy(ql + dq * s, beta) @ dq, 0.0, 1.0,
                                            epsabs=1e-15, epsrel=1e-14)
        ref = 0.5 * (oracle.flux_phys(ql, beta) + oracle.flux_phys(qr, beta) - exact)
        errs.append(np.abs(oracle.osher_x(ql, qr, beta) - ref).max())
    ratio = errs[0] / errs[1]
    assert 90.0 < ratio < 180.0, (errs, ratio)


def test_wall_mirror_flux():
    """Across a wall the ghost mirrors the cell (velocity negated): no mass and no p/beta
    (velocity) flux crosses it."""
    rng = np.random.default_rng(3)
    for _ in range(100):
        beta = float(rng.uniform(1, 2000))
        rho, u, v = float(rng.uniform(1, 1000)), *rng.normal(size=2)
        p = float(rng.normal() * 100)
        ql = q_of(rho, u, v, p, beta)
        qr = q_of(rho, -u, -v, p, beta)
        f = oracle.osher_x(ql, qr, beta)
        assert abs(f[0]) <= 1e-13 * rho * max(abs(u), 1e-3) * 10
        assert abs(f[3]) <= 1e-13 * max(abs(u), 1e-3) * 10


def test_face_rotation():
    """Algorithm 2: for n = (1,0) the rotation is the identity; for n = (0,1) the y-flux of a
    uniform state is G = (rho v, rho u v, rho v^2 + p, v) (Sec. 2.1.2)."""
    beta = 7.0
    rng = np.random.default_rng(4)
    for _ in range(50):
        qa = q_of(float(rng.uniform(1, 10)), *rng.normal(size=2), float(rng.normal()), beta)
        qb = q_of(float(rng.uniform(1, 10)), *rng.normal(size=2), float(rng.normal()), beta)
        np.testing.assert_array_equal(oracle.face_flux(qa, qb, (1.0, 0.0), beta),
                                      oracle.osher_x(qa, qb, beta))
        rho, u, v, p = qa[0], qa[1] / qa[0], qa[2] / qa[0], qa[3] * beta
        G = np.array([rho * v, rho * u * v, rho * v * v + p, v])
        np.testing.assert_allclose(oracle.face_flux(qa, qa, (0.0, 1.0), beta), G, rtol=1e-14,
                                   atol=1e-14 * np.abs(G).max())
        # y-face flux is the x-flux of the (u, v)-swapped states, swapped back
        sw = [0, 2, 1, 3]
        np.testing.assert_array_equal(oracle.face_flux(qa, qb, (0.0, 1.0), beta),
                                      oracle.osher_x(qa[sw], qb[sw], beta)[sw])
