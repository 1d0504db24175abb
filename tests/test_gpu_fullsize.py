"""Parity at the full sizes of the large benchmark workloads, in the launch configuration that
bench.py times (the autotuned stage-kernel shape), on outputs the oracle can compute.

* 64 x 64 hydrostatic tank (the first benchmark configuration) in full: 10 real steps of exactly
  200 pseudo-iterations, every step compared (the error is printed against the step).
* 4096 x 4096 obstacle dam break.  After real steps totalling N pseudo-iterations a cell's state
  depends only on the initial state within 2 cells per stage (a face's states need the slopes of
  the two cells beside it, and each slope its two neighbours; the real-time levels are the
  cell's own), so within R = 2 s_max N cells.  The oracle runs a window of the initial state of
  radius R + 1 around each sampled cell, clipped at the domain, where the domain's own walls
  apply.  The window's cut sides are walls in the oracle, which can reach at most R cells inward,
  so the window's centre cell is exact.  Samples: the obstacle's corners and top, the dam front,
  the layer interface, the four walls and corners, and seeded interior cells.
* 512-tank sloshing ensemble.  The whole batched launch runs; the oracle runs a sample of whole
  tanks (the smallest, the largest and seeded ones).
* A tank of exactly 2^29 cells, the largest a grid takes, with the same window check.

FP64 bar: |gpu - oracle| <= 1e-12 x the field's physical scale (as in the other parity tests).
Mixed form: the mixed bar (rho 1e-6, rho u and rho v 1e-5, p 1e-4 of the same scales).
"""
import numpy as np
import pytest

import oracle
from paper_2108_08769_amd import vdac
from paper_2108_08769_amd import workloads as wl
from parity import gpu_options, oracle_problem, field_errors, field_scales

pytestmark = pytest.mark.gpu

FP64_BAR = np.array([1e-12, 1e-12, 1e-12, 1e-12])
MIXED_BAR = np.array([1e-6, 1e-5, 1e-5, 1e-4])


def tank_dict(t):
    return dict(nx=t.nx, ny=t.ny, lx=t.lx, ly=t.ly, gx=t.gx, gy=t.gy, beta=t.beta, bc=t.bc,
                solid=t.solid)


def run_tuned(wk, precision, pseudo, steps=1):
    """`steps` real steps of `pseudo` pseudo-iterations of every tank, in one grid, with the shape
    the autotuner picks (as bench.py does); returns the states, the iteration counts of the last
    step and the shape."""
    tanks = [tank_dict(t) for t in wk.tanks]
    opts = vdac.autotune(tanks, gpu_options(wk, precision), iters=5)
    shape = (opts.tile_x, opts.tile_y)
    print(f"[fullsize] {wk.name} {precision}: autotuned shape {shape}", flush=True)
    grid = vdac.Grid(tanks, opts)
    try:
        for i, t in enumerate(wk.tanks):
            grid.set_state(i, t.q)
        for _ in range(steps):
            rc, done = grid.step(wk.dt, pseudo, 0.0, check=False)
            assert rc == 0
        states = [grid.get_state(i) for i in range(len(wk.tanks))]
    finally:
        grid.close()
    return states, np.asarray(done), shape


def obstacle_samples(t, n_random=10, seed=21):
    n = t.nx
    at = lambda x: min(n - 1, int(x / t.lx * n))  # cell containing coordinate x
    pts = [(at(2.5) - 1, 0), (at(2.5) - 1, at(0.3)), (at(2.7) + 1, 2), (at(2.6), at(0.3) + 1),
           (at(1.0), 5), (at(1.0) - 1, at(1.0)), (at(0.5), at(2.0)), (at(0.5), at(2.0) - 1),
           (0, 0), (n - 1, 0), (0, n - 1), (n - 1, n - 1), (0, n // 2), (n - 1, n // 3),
           (n // 2, 0), (n // 3, n - 1)]
    rng = np.random.default_rng(seed)
    pts += [(int(i), int(j)) for i, j in rng.integers(0, n, size=(n_random, 2))]
    return [(i, j) for i, j in pts if not t.solid[j, i]]


def window_oracle(wk, t, i, j, radius, pseudo, steps=1):
    """The oracle's state at cell (i, j) after `steps` real steps, from a window of the initial
    state (the -fopenmp build of the oracle, which gives the serial build's results bit for
    bit)."""
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
        out, it, _, rc = oracle.step(pb, out, wk.dt, pseudo, 0.0, 0, omp=True)
        assert rc == 0 and it == pseudo
    return out[:, j - j0, i - i0]


def test_hydrostatic_64_in_full_every_step():
    """The first benchmark configuration in full: 10 real steps of exactly 200 pseudo-iterations
    in the autotuned shape, each step's state against the oracle's."""
    wk = wl.hydrostatic()
    t = wk.tanks[0]
    tanks = [tank_dict(t)]
    opts = vdac.autotune(tanks, gpu_options(wk, "f64"), iters=5)
    print(f"[fullsize] {wk.name}: autotuned shape {(opts.tile_x, opts.tile_y)}", flush=True)
    pb = oracle_problem(t, wk)
    grid = vdac.Grid(tanks, opts)
    try:
        grid.set_state(0, t.q)
        ref = t.q
        for step in range(wk.steps):
            rc, done = grid.step(wk.dt, wk.max_pseudo, 0.0, check=False)
            ref, it, _, orc = oracle.step(pb, ref, wk.dt, wk.max_pseudo, 0.0, 0)
            assert rc == 0 and orc == 0 and int(done[0]) == it == wk.max_pseudo
            err = field_errors(grid.get_state(0), ref, None, field_scales(t))
            print(f"[fullsize] hydrostatic step {step + 1}: field errors {err}", flush=True)
            assert np.all(err <= FP64_BAR), (step, err)
    finally:
        grid.close()


@pytest.mark.parametrize("precision", ["f64", "mixed"])
def test_obstacle_4096_sampled_windows(precision):
    """Two real steps of 10 pseudo-iterations (N = 20, window radius 2 s_max N + 1 = 121) on
    the whole 4096^2 tank, 36 sampled cells against the oracle's windows.  Besides the scaled
    error per cell, the plain max |gpu - oracle| / max |oracle| over the sampled cells is held to
    the bar for every field whose sampled max |oracle| is at least 1e-3 of its scale."""
    pseudo, steps = 10, 2
    wk = wl.obstacle_dam_break(n=4096, precision=precision)
    t = wk.tanks[0]
    states, done, _ = run_tuned(wk, precision, pseudo, steps)
    assert int(done[0]) == pseudo
    got = states[0]
    np.testing.assert_array_equal(got[:, t.solid == 1], t.q[:, t.solid == 1])
    radius = 2 * wk.stages * pseudo * steps + 1
    scales = field_scales(t)
    bar = FP64_BAR if precision == "f64" else MIXED_BAR
    worst = np.zeros(4)
    samples = obstacle_samples(t, n_random=20)
    g_s, o_s = [], []
    for i, j in samples:
        ref = window_oracle(wk, t, i, j, radius, pseudo, steps)
        g_s.append(got[:, j, i])
        o_s.append(ref)
        err = np.abs(got[:, j, i] - ref) / scales
        worst = np.maximum(worst, err)
        assert np.all(err <= bar), ((i, j), err, got[:, j, i], ref)
    g_s, o_s = np.array(g_s), np.array(o_s)
    omax = np.abs(o_s).max(axis=0)
    plain = np.abs(g_s - o_s).max(axis=0) / np.where(omax > 0, omax, 1.0)
    held = omax >= 1e-3 * scales
    print(f"[fullsize] obstacle 4096 {precision}: {len(samples)} cells after {steps * pseudo} "
          f"pseudo-iterations, worst scaled error per field {worst}, plain max|a-b|/max|b| "
          f"{plain} (held for fields {np.flatnonzero(held).tolist()})", flush=True)
    if precision == "f64":
        assert np.all(plain[held] <= FP64_BAR[held]), plain


@pytest.mark.parametrize("precision", ["f64", "mixed"])
def test_ensemble_512_sampled_tanks(precision):
    pseudo = 5
    wk = wl.sloshing_ensemble(precision=precision)
    states, done, _ = run_tuned(wk, precision, pseudo)
    assert np.all(done == pseudo)
    cells = np.array([t.nx * t.ny for t in wk.tanks])
    order = np.argsort(cells, kind="stable")
    rng = np.random.default_rng(8)
    picks = sorted(set(order[:2].tolist() + order[-2:].tolist()
                       + rng.choice(len(wk.tanks), 4, replace=False).tolist()))
    bar = FP64_BAR if precision == "f64" else MIXED_BAR
    worst = np.zeros(4)
    for k in picks:
        t = wk.tanks[k]
        pb = oracle_problem(t, wk)
        ref, it, _, rc = oracle.step(pb, t.q, wk.dt, pseudo, 0.0, 0)
        assert rc == 0 and it == pseudo
        err = field_errors(states[k], ref, None, field_scales(t))
        worst = np.maximum(worst, err)
        assert np.all(err <= bar), (k, t.nx, t.ny, err)
    print(f"[fullsize] ensemble {precision}: tanks {picks}, worst field error {worst}", flush=True)


@pytest.mark.parametrize("precision", ["f64", "mixed"])
def test_largest_tank_2_29_cells(precision):
    """A tank of exactly 2^29 cells, the limit that the row-marching kernel's 32-bit plane offsets
    set (8-byte elements: the last cell of a plane starts at byte 2^32 - 8): a dam break of
    16384 x 32768 square cells with an obstacle next to the far corner, one real step of 2
    pseudo-iterations in the benchmark's shape (-2 x 32), sampled cells against the oracle's
    windows, the far corner, the last row and column and the obstacle's sides among them.  The
    grid takes 61 GiB (mixed: 57 GiB) of device memory and the host 35 GB."""
    nx, ny, pseudo = 16384, 32768, 2
    assert nx * ny == 1 << 29
    h = 1.0 / 4096
    q = np.zeros((4, ny, nx))
    q[0] = 1.0
    q[0, :int(2.0 / h), :int(1.0 / h)] = 1000.0
    solid = np.zeros((ny, nx), np.uint8)
    solid[ny - 24:ny - 12, nx - 40:nx - 28] = 1
    t = wl.Tank(nx, ny, nx * h, ny * h, q, gy=-9.81, beta=1100.0, solid=solid)
    wk = wl.Workload("dam_break_16384x32768", [t], dt=2e-5, steps=1, max_pseudo=pseudo)
    print(f"[fullsize] {wk.name} {precision}: {nx * ny} cells, shape (-2, 32)", flush=True)
    grid = vdac.Grid([tank_dict(t)], gpu_options(wk, precision, tile=(-2, 32)))
    try:
        grid.set_state(0, q)
        rc, done = grid.step(wk.dt, pseudo, 0.0, check=False)
        assert rc == 0 and int(done[0]) == pseudo
        got = grid.get_state(0)
    finally:
        grid.close()
    np.testing.assert_array_equal(got[:, solid == 1], q[:, solid == 1])
    samples = [(nx - 1, ny - 1), (nx - 2, ny - 1), (nx - 1, ny - 2), (0, ny - 1), (nx - 1, 0),
               (nx // 2, ny - 1), (nx - 1, ny // 2), (nx - 41, ny - 18), (nx - 27, ny - 13),
               (nx - 34, ny - 25), (nx - 34, ny - 11), (4095, 100), (4096, 100), (100, 8191),
               (100, 8192), (nx // 2, ny // 2)]
    rng = np.random.default_rng(29)
    samples += [(int(rng.integers(0, nx)), int(rng.integers(0, ny))) for _ in range(8)]
    radius = 2 * wk.stages * pseudo + 1
    # the tank starts at rest with rho_max 1000: its scales from a one-cell stand-in (field_scales
    # on the whole state would take 17 GB of temporaries)
    q1 = np.array([1000.0, 0.0, 0.0, 0.0]).reshape(4, 1, 1)
    scales = field_scales(wl.Tank(1, 1, t.lx, t.ly, q1, gy=t.gy, beta=t.beta))
    bar = FP64_BAR if precision == "f64" else MIXED_BAR
    worst = np.zeros(4)
    for i, j in samples:
        ref = window_oracle(wk, t, i, j, radius, pseudo)
        err = np.abs(got[:, j, i] - ref) / scales
        worst = np.maximum(worst, err)
        assert np.all(err <= bar), ((i, j), err, got[:, j, i], ref)
    print(f"[fullsize] {wk.name} {precision}: {len(samples)} cells, worst scaled error per field "
          f"{worst}", flush=True)
