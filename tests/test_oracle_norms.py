"""Pins of the oracle's residual norm and its pseudo-loop control (Algorithm 1's convergence test,
read as in DESIGN R10: the residual of an iteration is the bracket of its last Runge-Kutta stage,
the pressure row reported as dp/dtau = beta R_(p/beta); the norm is the RMS, or the maximum, over
the fluid cells; the loop stops at the first iteration whose four norms are all below tol, and
diverges at the first iteration that leaves a fluid density <= 0 or a non-finite residual).

The norms are recomputed here from the update equation instead of from the bracket the oracle
returns: the last stage has alpha = 1, so its update (eq. 24) is
    Q^3 - Q^0 = dtau R / alpha_PI   (rho, rho u, rho v; alpha_PI = 1 + B0 dtau / dt, eq. 27)
    p^3 - p^0 = beta dtau R_(p/beta)   (the p/beta row has no real-time term, alpha_PI = 1),
so R follows from the states before and after one iteration and the frozen local step.  A norm
that counted the solid cells, dropped beta from the pressure row, used the first stage's bracket
or missed alpha_PI fails the comparison.  The stop and divergence iterations are pinned against
one-iteration calls chained by hand in pseudo-time only (dt = 0: no real-time level, so a run of
m iterations is m runs of one), each checked with numpy.
"""
import numpy as np
import pytest

import oracle
from paper_2108_08769_amd import workloads as wl


def obstacle_tank(rho_range=(1.0, 3.0), vel=0.3, p_scale=10.0, cfl=0.48, seed=5):
    nx, ny = 12, 10
    q = wl.random_state(nx, ny, seed=seed, rho_range=rho_range, vel=vel, p_scale=p_scale)
    solid = np.zeros((ny, nx), np.uint8)
    solid[4:6, 5:8] = 1
    pb = oracle.Problem(nx, ny, 1.2, 1.0, gx=0.3, gy=-9.81, beta=1000.0, bc=(0, 0, 0, 0),
                        solid=solid, cfl=cfl)
    return pb, q, solid


def residual_from_update(pb, q0, q1, dt):
    """R per field from one iteration's states (the last stage, alpha = 1), with dtau the frozen
    local step the oracle's stage reports."""
    _, det = oracle.stage(pb, q0, q0, q0, dt, 1)
    dtau = det["dtau"]
    api = 1.0 + dtau / dt if dt > 0 else np.ones_like(dtau)  # backward Euler: B0 = 1
    R = np.zeros_like(q0)
    fluid = dtau > 0  # solid cells have no step
    for k in range(3):
        R[k][fluid] = (q1[k] - q0[k])[fluid] * api[fluid] / dtau[fluid]
    R[3][fluid] = (q1[3] - q0[3])[fluid] / dtau[fluid]  # = beta R_(p/beta) = dp/dtau
    return R


@pytest.mark.parametrize("dt", [0.0, 2e-3])
@pytest.mark.parametrize("norm", [0, 1])
def test_norms_are_the_last_stage_bracket_over_fluid_cells(norm, dt):
    pb, q, solid = obstacle_tank()
    q1, it, res, rc = oracle.step(pb, q, dt, 1, 0.0, norm=norm)
    assert rc == 0 and it == 1
    R = residual_from_update(pb, q, q1, dt)
    fluid = solid == 0
    if norm == 0:
        expect = np.sqrt(np.array([np.mean(R[k][fluid] ** 2) for k in range(4)]))
        wrong_count = np.sqrt(np.array([np.sum(R[k][fluid] ** 2) / R[k].size for k in range(4)]))
        assert np.all(np.abs(wrong_count / expect - 1.0) > 1e-3)
    else:
        expect = np.array([np.abs(R[k][fluid]).max() for k in range(4)])
    np.testing.assert_allclose(res, expect, rtol=1e-9)
    # the pressure row is dp/dtau: without beta it would be 1000 times smaller
    assert abs(res[3] / (expect[3] / pb.beta) - pb.beta) < 1e-6 * pb.beta
    # the first stage's bracket is a different residual (the norm is not taken there)
    _, det1 = oracle.stage(pb, q, q, q, dt, 1)
    first = np.sqrt(np.array([np.mean(det1["resid"][k][fluid] ** 2) for k in range(4)]))
    if norm == 0:
        assert np.all(np.abs(first / expect - 1.0) > 1e-3)


def chain(pb, q, n, tol_check=None):
    """n one-iteration calls in pseudo-time only; returns the states and norms after each, and
    the first iteration (1-based) whose state has a fluid density <= 0 or non-finite values or
    whose norms are not finite (None if there is none)."""
    states, norms, bad_at = [q], [], None
    fluid = pb.solid == 0 if pb.solid is not None else np.ones((pb.ny, pb.nx), bool)
    for m in range(1, n + 1):
        qm, it, res, rc = oracle.step(pb, states[-1], 0.0, 1, 0.0)
        assert it == 1
        states.append(qm)
        norms.append(res)
        bad = (not np.all(np.isfinite(res)) or not np.all(np.isfinite(qm[:, fluid]))
               or np.any(qm[0][fluid] <= 0.0))
        if bad:
            bad_at = m
            break
    return states, norms, bad_at


def test_tolerance_stops_at_the_first_iteration_below_it():
    pb, q, _ = obstacle_tank(cfl=0.9)
    states, norms, bad_at = chain(pb, q, 60)
    assert bad_at is None
    peak = np.array([n.max() for n in norms])
    # a tolerance between the largest norm of iteration m* and the largest of every earlier one
    m_star = next(m for m in range(10, 60) if peak[m] < peak[:m].min() * (1 - 1e-6))
    tol = peak[m_star] * (1 + 1e-9)
    assert np.all(peak[:m_star] > tol)
    q_end, it, res, rc = oracle.step(pb, q, 0.0, 60, tol)
    assert rc == 0 and it == m_star + 1
    np.testing.assert_allclose(res, norms[m_star], rtol=1e-11)
    np.testing.assert_allclose(q_end, states[m_star + 1], rtol=1e-11, atol=1e-11)
    # every field must be below tol: with one field left above, the loop runs on
    tol_one = np.sort(norms[m_star])[-2] * (1 + 1e-9)  # below the largest norm of m*
    _, it2, _, _ = oracle.step(pb, q, 0.0, m_star + 1, tol_one)
    assert it2 == m_star + 1 and np.max(norms[m_star]) > tol_one


@pytest.mark.parametrize("rho_range,vel,seed,kind", [((1.0, 3.0), 0.3, 5, "rho"),
                                                     ((1.0, 30.0), 0.5, 5, "nan")])
def test_divergence_stops_at_the_failing_iteration(rho_range, vel, seed, kind):
    pb, q, solid = obstacle_tank(rho_range=rho_range, vel=vel, cfl=2.0, seed=seed)
    states, norms, bad_at = chain(pb, q, 40)
    assert bad_at is not None and bad_at > 1
    fluid = solid == 0
    if kind == "rho":  # finite norms, a density at or below zero
        assert np.all(np.isfinite(norms[-1])) and np.any(states[-1][0][fluid] <= 0.0)
    else:
        assert not np.all(np.isfinite(norms[-1]))
    q_end, it, res, rc = oracle.step(pb, q, 0.0, 40, 0.0)
    assert rc == -2 and it == bad_at
    # the state is the one after the failing iteration
    ok = np.isfinite(states[-1]) & np.isfinite(q_end)
    np.testing.assert_allclose(q_end[ok], states[-1][ok], rtol=1e-9, atol=1e-9)
    np.testing.assert_array_equal(np.isfinite(q_end), np.isfinite(states[-1]))
