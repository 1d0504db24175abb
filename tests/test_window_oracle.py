"""The window argument the full-size GPU parity tests rest on, checked on the CPU with the oracle
alone: after real steps totalling N pseudo-iterations, a cell's state computed from a window of
the initial state of radius 2 s_max N + 1 around it (cut sides as walls, the domain's own walls
where the window reaches them) equals the cell's state from the whole tank."""
import numpy as np

import oracle
from paper_2108_08769_amd import workloads as wl
from parity import oracle_problem


def window_state(wk, t, i, j, radius, pseudo, steps):
    i0, i1 = max(0, i - radius), min(t.nx, i + radius + 1)
    j0, j1 = max(0, j - radius), min(t.ny, j + radius + 1)
    dx, dy = t.lx / t.nx, t.ly / t.ny
    q = np.ascontiguousarray(t.q[:, j0:j1, i0:i1])
    solid = np.ascontiguousarray(t.solid[j0:j1, i0:i1])
    wt = wl.Tank(i1 - i0, j1 - j0, (i1 - i0) * dx, (j1 - j0) * dy, q, gx=t.gx, gy=t.gy,
                 beta=t.beta, solid=solid)
    pb = oracle_problem(wt, wk)
    out = q
    for _ in range(steps):
        out, it, _, rc = oracle.step(pb, out, wk.dt, pseudo, 0.0, 0)
        assert rc == 0 and it == pseudo
    return out[:, j - j0, i - i0]


def test_window_of_radius_2_smax_N_plus_1_reproduces_the_whole_tank():
    pseudo, steps = 2, 2
    wk = wl.obstacle_dam_break(n=128)
    t = wk.tanks[0]
    pb = oracle_problem(t, wk)
    full = t.q
    for _ in range(steps):
        full, it, _, rc = oracle.step(pb, full, wk.dt, pseudo, 0.0, 0)
        assert rc == 0 and it == pseudo
    radius = 2 * wk.stages * pseudo * steps + 1
    rng = np.random.default_rng(5)
    pts = [(0, 0), (127, 127), (80, 0), (79, 9), (87, 10), (32, 40), (31, 64), (16, 63)]
    pts += [tuple(int(v) for v in p) for p in rng.integers(0, 128, size=(12, 2))]
    scale = np.array([1000.0, 1000.0 * np.sqrt(9.81 * 4), 1000.0 * np.sqrt(9.81 * 4), 1000.0 * 9.81 * 4])
    worst = 0.0
    for i, j in pts:
        if t.solid[j, i]:
            continue
        err = np.abs(window_state(wk, t, i, j, radius, pseudo, steps) - full[:, j, i]) / scale
        worst = max(worst, float(err.max()))
        assert np.all(err <= 1e-14), ((i, j), err)
    # a window much shorter than the reach changes the result next to the dam front and the
    # layer interface, where the state varies (the comparison above has teeth)
    short = [np.abs(window_state(wk, t, i, j, 2, pseudo, steps) - full[:, j, i]).max()
             for i, j in [(34, 20), (29, 20), (20, 66)]]
    assert min(short) > 0.0, short


def test_window_reproduces_the_whole_tank_after_20_iterations():
    """The reach the 4096^2 GPU check uses: two real steps of 10 pseudo-iterations (radius 121),
    on a 256^2 obstacle tank; windows run on the oracle's -fopenmp build (bitwise the serial
    one's results)."""
    pseudo, steps = 10, 2
    wk = wl.obstacle_dam_break(n=256)
    t = wk.tanks[0]
    pb = oracle_problem(t, wk)
    full = t.q
    for _ in range(steps):
        full, it, _, rc = oracle.step(pb, full, wk.dt, pseudo, 0.0, 0, omp=True)
        assert rc == 0 and it == pseudo
    radius = 2 * wk.stages * pseudo * steps + 1
    scale = np.array([1000.0, 1000.0 * np.sqrt(9.81 * 4), 1000.0 * np.sqrt(9.81 * 4), 1000.0 * 9.81 * 4])
    for i, j in [(64, 128), (159, 18), (255, 255), (200, 100), (127, 60)]:
        assert not t.solid[j, i]
        i0, i1 = max(0, i - radius), min(t.nx, i + radius + 1)
        j0, j1 = max(0, j - radius), min(t.ny, j + radius + 1)
        dx, dy = t.lx / t.nx, t.ly / t.ny
        q = np.ascontiguousarray(t.q[:, j0:j1, i0:i1])
        solid = np.ascontiguousarray(t.solid[j0:j1, i0:i1])
        wt = wl.Tank(i1 - i0, j1 - j0, (i1 - i0) * dx, (j1 - j0) * dy, q, gx=t.gx, gy=t.gy,
                     beta=t.beta, solid=solid)
        wpb = oracle_problem(wt, wk)
        out = q
        for _ in range(steps):
            out, it, _, rc = oracle.step(wpb, out, wk.dt, pseudo, 0.0, 0, omp=True)
            assert rc == 0
        err = np.abs(out[:, j - j0, i - i0] - full[:, j, i]) / scale
        assert np.all(err <= 1e-14), ((i, j), err)
