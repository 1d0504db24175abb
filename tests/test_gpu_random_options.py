"""Seeded random combinations of every option on random small batches, GPU against the oracle.

The other parity files take each option alone, or one fixed combination, on fixed tanks; here
each seed draws all of them together, so that an interaction (an open side beside an obstacle
under the Roe flux and a global step, a periodic pair in a BDF3 batch, wall slip with the
k-limiter on p on a ragged LDS tile) meets the oracle too:

* one to three tanks of 3..70 x 3..45 cells with square or stretched cells, gravity tilted at
  random, beta in [400, 3000];
* sides per axis: a periodic pair, or each side a wall or zero-gradient;
* with probability 0.4 a rectangular obstacle of solid cells;
* a two-layer state with its interface and heavy block placed at random, density ratio 1.2..1000,
  small random velocities and a random pressure offset;
* flux (Osher, Roe, exact), pressure gradient (new, k-limiter, split limiter where no side is
  open) with k in [1, 2], MUSCL k in [1, 2], wall slip, RMS or max norm, 1..4 Runge-Kutta stages
  with their coefficients, CFL 0.3..0.9, local or global pseudo-time steps, BDF order 1..3, HIP
  graphs of 0, 3 or all pseudo-iterations;
* the kernel: row marching with 1..3 waves per workgroup and chunks of 1..80 rows, every LDS
  tile shape, or the autotuner's pick;
* 1..4 real steps of dt in {5e-4, 1e-3, 2e-3} with 3..12 pseudo-iterations each.

Bar as in the other parity files: per field max |gpu - oracle| / max(max |oracle|, physical
scale) <= 1e-12 and the same for the plain relative error of every field above 1e-3 of its
scale, equal iteration counts, equal residual norms to rtol 1e-7.  A combination can diverge
(seed 26: a periodic 7 x 17 tank under a global pseudo-time step at CFL 0.87 reaches rho <= 0
in the first pseudo-iteration of its first BDF2 step); then the GPU must report the divergence
in the same steps and stop at the same iteration as the oracle, and the batch's other tanks
still meet the bar.  Measured worst: 9.1e-16.

The mixed form takes the first 40 combinations against the oracle at its own bars; measured
worst per field 2.7e-9 (rho), 1.7e-9 (rho u), 2.3e-9 (rho v), 6.6e-8 (p).
"""
import numpy as np
import pytest

from paper_2108_08769_amd import workloads as wl
from parity import field_errors, field_scales, plain_errors, run_gpu, run_oracle

pytestmark = pytest.mark.gpu

TOL = 1e-12
DIVERGED = 4
W, P, O = 0, 1, 2
TILES = [(32, 8), (16, 16), (64, 4), (3208, 2), (1616, 2), (1608, 2)]
RK = {1: (1.0,), 2: (0.5, 1.0), 3: (1.0 / 3.0, 0.5, 1.0), 4: (0.25, 1.0 / 3.0, 0.5, 1.0)}


def sides(rng):
    if rng.random() < 0.25:
        return (P, P)
    return tuple(O if rng.random() < 0.3 else W for _ in range(2))


def tank(rng):
    nx, ny = int(rng.integers(3, 71)), int(rng.integers(3, 46))
    h = rng.uniform(0.02, 0.1)
    lx, ly = nx * h, ny * h * (1.0 if rng.random() < 0.5 else rng.uniform(0.5, 2.0))
    bx, by = sides(rng), sides(rng)
    ang = rng.uniform(-0.4, 0.4)
    g = 9.81 * rng.uniform(0.5, 1.0)
    xc = (np.arange(nx) + 0.5) * lx / nx
    yc = (np.arange(ny) + 0.5) * ly / ny
    ratio = float(rng.choice([1.2, 3.0, 50.0, 1000.0]))
    heavy = yc[:, None] < rng.uniform(0.1, 0.6) * ly
    heavy = heavy | ((xc[None, :] < rng.uniform(0.1, 0.5) * lx) & (yc[:, None] < rng.uniform(0.3, 0.9) * ly))
    q = np.zeros((4, ny, nx))
    q[0] = np.where(heavy, ratio, 1.0) * rng.uniform(0.9, 1.1)
    q[1] = q[0] * rng.uniform(-0.05, 0.05, size=(ny, nx))
    q[2] = q[0] * rng.uniform(-0.05, 0.05, size=(ny, nx))
    q[3] = rng.uniform(-10.0, 10.0)
    solid = None
    if rng.random() < 0.4 and nx >= 4 and ny >= 4:
        i0, j0 = int(rng.integers(0, nx - 1)), int(rng.integers(0, ny - 1))
        i1, j1 = i0 + int(rng.integers(1, max(2, nx // 3))), j0 + int(rng.integers(1, max(2, ny // 3)))
        solid = np.zeros((ny, nx), np.uint8)
        solid[j0:j1, i0:i1] = 1
        if solid.all():
            solid = None
    return wl.Tank(nx, ny, lx, ly, q, gx=g * np.sin(ang), gy=-g * np.cos(ang),
                   beta=rng.uniform(400.0, 3000.0), bc=bx + by, solid=solid)


def draw(seed):
    """(workload, keyword options of run_gpu and run_oracle, kernel shape) of one seed."""
    rng = np.random.default_rng(7000 + seed)
    tanks = [tank(rng) for _ in range(int(rng.choice([1, 1, 2, 3])))]
    stages = int(rng.integers(1, 5))
    wk = wl.Workload(f"random_options_{seed}", tanks, dt=float(rng.choice([5e-4, 1e-3, 2e-3])),
                     steps=int(rng.integers(1, 5)), max_pseudo=int(rng.integers(3, 13)),
                     stages=stages, alpha=RK[stages], cfl=float(rng.uniform(0.3, 0.9)),
                     k=float(rng.choice([1.0, rng.uniform(1.0, 2.0), 2.0])),
                     local_dtau=bool(rng.random() < 0.6), bdf=int(rng.integers(1, 4)))
    any_open = any(O in t.bc for t in tanks)
    pgrad = int(rng.integers(0, 2 if any_open else 3))
    kw = dict(flux=int(rng.integers(0, 3)), pgrad=pgrad,
              pk=float(rng.choice([1.0, rng.uniform(1.0, 2.0), 2.0])) if pgrad else 1.0,
              wall_slip=bool(rng.random() < 0.3), norm=int(rng.integers(0, 2)),
              graph_iters=int(rng.choice([0, 3, -1])))
    r = rng.random()
    if r < 0.45:
        tile = (-int(rng.integers(1, 4)), int(rng.integers(1, 81)))
    elif r < 0.9:
        tile = TILES[int(rng.integers(0, len(TILES)))]
    else:
        tile = (0, 0)
    return wk, kw, tile


@pytest.mark.parametrize("seed", range(1, 61))
def test_random_option_combination_against_oracle(seed):
    wk, kw, tile = draw(seed)
    desc = [(t.nx, t.ny, t.bc, t.solid is not None) for t in wk.tanks]
    print(f"[random-options] seed {seed}: tanks {desc} tile {tile} stages {wk.stages} "
          f"cfl {wk.cfl:.2f} k {wk.k:.2f} local {wk.local_dtau} bdf {wk.bdf} dt {wk.dt} "
          f"steps {wk.steps} pseudo {wk.max_pseudo} {kw}", flush=True)
    g = run_gpu(wk, wk.steps, wk.max_pseudo, tile=tile, **kw)
    o = run_oracle(wk, wk.steps, wk.max_pseudo, **kw)
    # a tank that diverges (non-finite residual or rho <= 0) stops at the failing iteration on
    # both sides: the step reports it, and the iteration counts still agree
    o_bad = np.array(o[3]).reshape(len(wk.tanks), wk.steps).T != 0     # [steps, tanks]
    np.testing.assert_array_equal(np.array(g[3]), np.where(o_bad.any(axis=1), DIVERGED, 0))
    np.testing.assert_array_equal(g[1], o[1])
    worst = 0.0
    for i, (t, a, b) in enumerate(zip(wk.tanks, g[0], o[0])):
        if o_bad[:, i].any():
            print(f"[random-options]   tank {i} diverges at steps "
                  f"{np.flatnonzero(o_bad[:, i]).tolist()} on both sides", flush=True)
            continue
        sc = field_scales(t)
        err = field_errors(a, b, t.solid, sc)
        worst = max(worst, err.max())
        assert np.all(err <= TOL), (t.nx, t.ny, err)
        plain = plain_errors(a, b, t.solid, sc)
        held = ~np.isnan(plain)
        assert np.all(plain[held] <= TOL), (t.nx, t.ny, plain)
        np.testing.assert_allclose(g[2][i], o[2][i], rtol=1e-7,
                                   atol=max(1e-12, 1e-14 * np.abs(o[2][i]).max()))
    print(f"[random-options]   worst field error {worst:.3e}", flush=True)


MIXED_BAR = np.array([1e-6, 1e-5, 1e-5, 1e-4])


@pytest.mark.parametrize("seed", range(1, 41))
def test_random_option_combination_mixed_against_oracle(seed):
    """The mixed form on the same combinations against the oracle: per field max |gpu - oracle|
    over max(max |oracle|, physical scale) within the mixed bars (rho 1e-6, rho u and rho v 1e-5,
    p 1e-4), equal iteration counts (the combination that diverges is left to the FP64 test:
    whether a near-zero density crosses zero is a rounding decision)."""
    wk, kw, tile = draw(seed)
    o = run_oracle(wk, wk.steps, wk.max_pseudo, **kw)
    if any(c != 0 for c in o[3]):
        pytest.skip("the oracle diverges on this combination")
    m = run_gpu(wk, wk.steps, wk.max_pseudo, tile=tile, precision="mixed", **kw)
    assert all(c == 0 for c in m[3]), m[3]
    np.testing.assert_array_equal(m[1], o[1])
    worst = np.zeros(4)
    for t, a, b in zip(wk.tanks, m[0], o[0]):
        err = field_errors(a, b, t.solid, field_scales(t))
        worst = np.maximum(worst, err)
        assert np.all(err <= MIXED_BAR), (t.nx, t.ny, err)
    print(f"[random-options-mixed] seed {seed}: worst per field {worst}", flush=True)
