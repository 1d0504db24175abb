"""The -fopenmp build of the oracle (used only to time it on all host cores) gives the serial
build's results bit for bit: its parallel loops run each cell's arithmetic unchanged and reduce
only by a minimum."""
import numpy as np
import pytest

import oracle
from paper_2108_08769_amd import workloads as wl
from parity import oracle_problem


@pytest.mark.parametrize("case", ["dam_bdf2", "obstacle_global_dtau", "periodic_roe"])
def test_openmp_build_equals_serial(case):
    if case == "dam_bdf2":
        wk, steps, kw = wl.dam_break(nx=96, ny=48), 2, {}
        wk.bdf = 2
    elif case == "obstacle_global_dtau":
        wk, steps, kw = wl.obstacle_dam_break(n=64), 2, {}
        wk.local_dtau = False
    else:
        wk, steps, kw = wl.rayleigh_taylor(nx=32, ny=96, precision="f64"), 1, {"flux": oracle.FLUX_ROE}
    t = wk.tanks[0]
    pb = oracle_problem(t, wk, **kw)
    out = {}
    for omp in (False, True):
        q, prev, norms = t.q.copy(), None, None
        for _ in range(steps):
            qn, it, norms, rc = oracle.step(pb, q, wk.dt, 6, 0.0, 0, qnm1=prev if wk.bdf >= 2 else None,
                                            omp=omp)
            assert rc == 0 and it == 6
            prev, q = q, qn
        out[omp] = (q, norms)
    assert oracle.threads(True) >= 1 and oracle.threads(False) == 1
    np.testing.assert_array_equal(out[True][0], out[False][0])
    np.testing.assert_array_equal(out[True][1], out[False][1])
