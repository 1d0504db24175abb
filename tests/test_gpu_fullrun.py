"""Whole runs against the oracle, error against step (opt-in: VDAC_FULL_RUNS=1, or a number of
steps N > 1 to run only the first N of each, rounded down to a multiple of 50).

The other parity files hold the full-size configurations over their first real steps and
smaller tanks over 20; these run the 512 x 256 dam break for its 500 real steps (up to 100
pseudo-iterations each to 1e-6) and the 256 x 1024 Rayleigh-Taylor tank for its first 200, in
the shape the autotuner picks, beside the OpenMP build of the oracle, and compare the states
every 50 steps.  The oracle takes about an hour of host time for the dam break and as long for
the Rayleigh-Taylor steps, so the tests run only when asked for.

Bars: FP64 as in the other parity files (1e-12 of each field's physical scale, and plain
max |a - b| / max |b| where max |b| is at least 1e-3 of the scale), equal iteration counts at
every step; the mixed form against the same oracle states within its own bar (rho 1e-6, rho u
and rho v 1e-5, p 1e-4 of the scales).
"""
import os

import numpy as np
import pytest

import oracle
from paper_2108_08769_amd import vdac
from paper_2108_08769_amd import workloads as wl
from parity import field_errors, field_scales, oracle_problem, plain_errors

FULL = os.environ.get("VDAC_FULL_RUNS", "")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not FULL.isdigit() or int(FULL) < 1,
                                 reason="whole runs take about an hour of oracle time each; "
                                        "set VDAC_FULL_RUNS=1 (or a step count)")]

FP64_BAR = 1e-12
MIXED_BAR = np.array([1e-6, 1e-5, 1e-5, 1e-4])


def gpu_run(wk, precision, steps, every):
    t = wk.tanks[0]
    tanks = [dict(nx=t.nx, ny=t.ny, lx=t.lx, ly=t.ly, gx=t.gx, gy=t.gy, beta=t.beta, bc=t.bc)]
    opts = vdac.autotune(tanks, vdac.make_options(precision=precision), iters=5)
    grid = vdac.Grid(tanks, opts)
    its, states = [], {}
    try:
        grid.set_state(0, t.q)
        for s in range(1, steps + 1):
            rc, done = grid.step(wk.dt, wk.max_pseudo, wk.tol, check=False)
            assert rc == 0, (s, rc)
            its.append(int(done[0]))
            if s % every == 0:
                states[s] = grid.get_state(0)
    finally:
        grid.close()
    return np.array(its), states


@pytest.mark.parametrize("name,steps", [("dam_break", 500), ("rayleigh_taylor", 200)])
def test_whole_run_against_oracle(name, steps):
    every = 50
    if int(FULL) > 1:
        steps = max(every, min(steps, int(FULL)) // every * every)
    wk = getattr(wl, name)(precision="f64")
    t = wk.tanks[0]
    sc = field_scales(t)
    g_its, g_states = gpu_run(wk, "f64", steps, every)
    m_its, m_states = gpu_run(wk, "mixed", steps, every)
    pb = oracle_problem(t, wk)
    q = t.q.copy()
    for s in range(1, steps + 1):
        q, it, _, rc = oracle.step(pb, q, wk.dt, wk.max_pseudo, wk.tol, 0, omp=True)
        assert rc == 0 and it == g_its[s - 1], (s, rc, it, g_its[s - 1])
        if s % every:
            continue
        err = field_errors(g_states[s], q, None, sc)
        plain = plain_errors(g_states[s], q, None, sc)
        held = ~np.isnan(plain)
        merr = field_errors(m_states[s], q, None, sc)
        print(f"[fullrun] {wk.name} step {s}: FP64 scaled {err.max():.2e} plain "
              f"{np.nanmax(plain) if held.any() else 0.0:.2e}; mixed scaled {merr}", flush=True)
        assert err.max() <= FP64_BAR, (s, err)
        assert np.all(plain[held] <= FP64_BAR), (s, plain)
        assert np.all(merr <= MIXED_BAR), (s, merr)
    np.testing.assert_array_equal(m_its, g_its)
