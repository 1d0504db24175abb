"""Properties of the scheme that hold at any size, checked on every cell of the full 4096 x 4096
tank in the stage-kernel shapes bench.py times (the row-marching kernel, 2 waves per SIMD, chunks
of 32 rows in FP64 and 16 in the mixed form) and in the LDS-tiled kernel.  The sampled windows of
the full-size parity file hold a few dozen cells to the oracle; these hold all of them to what the
paper's scheme fixes.

* Mass conservation (Sec. 2.1: the continuity equation in conservation form; the flux of a face
  leaves one cell and enters its neighbour).  With free-slip walls the wall ghost is a true
  mirror, so no mass crosses a wall; in a closed tank under one global pseudo-time step the flux
  divergence then sums to zero, and the real-time term sums to zero as long as the total mass
  equals that of level n, so every stage keeps the total mass to rounding.  (With the paper's
  no-slip ghosts the new pressure gradient's cross terms keep their sign in the ghost, so the
  two face pressures of a wall differ where the flow runs along it and a little mass crosses:
  3e-11 of a small sloshing tank's mass over 20 pseudo-iterations, in the oracle as on the GPU.
  The checks therefore take free slip.)  A face whose flux the two units beside it (a strip's
  halo lanes, a chunk's halo rows, a tile's ring) evaluated differently would show here.
* Mirror symmetry.  A double dam break symmetric about x = L/2 stays symmetric: rho, rho v and p
  even, rho u odd.  The 60-column strips and the tiles are not laid out symmetrically (4096 =
  68 x 60 + 16), so mirror cells sit at different places in their strips and tiles.
* Transpose symmetry.  A tank symmetric about its diagonal (state, obstacle and gravity) stays
  symmetric, although the kernels take the x and y faces by different code.
* Translation along a periodic axis, on the full 256 x 1024 Rayleigh-Taylor tank: bit for bit.
* Free stream: a uniform state in a tank periodic on both axes, without gravity, stays the same
  bit for bit with zero residual norms.
* Hydrostatic balance (Sec. 2.3.2): the exact discrete two-layer hydrostatic state stays at rest
  around the benchmark's obstacle; measured momenta 1.2e-13 (FP64) and 7.5e-12 (mixed), pressure
  changes 3.7e-16 and 1.0e-14 of its largest value.
* The steady state does not depend on the pseudo-time CFL number: the 64 x 64 two-layer tank run
  to residuals below 1e-9 with CFL_tau 0.48 and 0.3 (69k and 111k pseudo-iterations) ends in the
  same pressure to 2.5e-15 with momenta of 4.7e-10.

FP64 bars: total mass to 1e-13 relative; mirror and transpose differences to 1e-12 of each
field's physical scale.  The mixed form stores the state as FP32 deviations from level n,
rounded on every stage, and takes its fluxes in FP32, whose Gauss-point sums run in opposite
orders on mirror faces: mass to 1e-12, mirror and transpose differences to 1e-9 of the scales.
Measured (3 real steps of 10 pseudo-iterations, each option set): mass within 2.3e-15 in
every form; mirror differences about 1e-19 of the scales (FP64) and at most 2.2e-11 (mixed);
transpose differences at most 2.3e-16 (FP64 row marching, whose x and y sums run in different
orders) and 1.6e-11 (mixed row marching), none at all in the tiles.

The mass, mirror and transpose checks each run with the Osher flux and the new pressure gradient
(BDF1), the Roe flux with BDF2, the exact flux with the k-limiter on p (k = 2), and the split
limiter (k = 1.5) with BDF3, so the general kernels meet the full size too.
"""
import functools

import numpy as np
import pytest

from paper_2108_08769_amd import vdac
from paper_2108_08769_amd import workloads as wl
from parity import field_scales, gpu_options

pytestmark = pytest.mark.gpu

SHAPES = {("f64", "march"): (-2, 32), ("mixed", "march"): (-2, 16),
          ("f64", "tile"): (3208, 2), ("mixed", "tile"): (1608, 2)}


# option sets of the general kernels (flux 0 Osher, 1 Roe, 2 exact; pgrad 0 new, 1 k-limiter
# on p, 2 split limiter), with the BDF order of the run
OPTIONS = {
    "osher": (dict(), 1),
    "roe_bdf2": (dict(flux=1), 2),
    "exact_plimiter": (dict(flux=2, pgrad=1, pk=2.0), 1),
    "split_bdf3": (dict(pgrad=2, pk=1.5), 3),
}


def run(wk, precision, shape, steps, pseudo, with_norms=False, **kw):
    t = wk.tanks[0]
    tank = dict(nx=t.nx, ny=t.ny, lx=t.lx, ly=t.ly, gx=t.gx, gy=t.gy, beta=t.beta, bc=t.bc,
                solid=t.solid)
    grid = vdac.Grid([tank], gpu_options(wk, precision, tile=shape, **kw))
    try:
        grid.set_state(0, t.q)
        for _ in range(steps):
            rc, done = grid.step(wk.dt, pseudo, 0.0, check=False)
            assert rc == 0 and int(done[0]) == pseudo, (rc, done)
        if with_norms:
            return grid.get_state(0), np.asarray(grid.residual_norm(0))
        return grid.get_state(0)
    finally:
        grid.close()


@pytest.mark.parametrize("options", list(OPTIONS))
@pytest.mark.parametrize("kernel", ["march", "tile"])
@pytest.mark.parametrize("precision", ["f64", "mixed"])
def test_mass_conserved_on_the_full_tank(precision, kernel, options):
    """Also with the Roe and exact fluxes, the limiters on p and BDF2 and BDF3 (Table 1: the
    real-time coefficients sum to zero, and every level holds the same total mass)."""
    kw, bdf = OPTIONS[options]
    wk = wl.obstacle_dam_break(precision=precision)
    wk.local_dtau = False
    wk.bdf = bdf
    t = wk.tanks[0]
    fluid = t.solid == 0
    shape = SHAPES[(precision, kernel)]
    print(f"[invariants] mass: {wk.name} {precision} shape {shape} {options}, global pseudo-time "
          f"step, free-slip walls, 3 steps x 10 pseudo-iterations", flush=True)
    q = run(wk, precision, shape, steps=3, pseudo=10, wall_slip=True, **kw)
    m0 = float(np.sum(t.q[0][fluid], dtype=np.float64))
    m1 = float(np.sum(q[0][fluid], dtype=np.float64))
    moved = float(np.abs(q[0] - t.q[0])[fluid].max())
    rel = abs(m1 - m0) / m0
    print(f"[invariants]   total mass {m0:.17e} -> {m1:.17e}: relative change {rel:.2e} "
          f"(largest density change of a cell {moved:.3e})", flush=True)
    assert moved > 1e-6          # the state did move
    assert rel <= (1e-13 if precision == "f64" else 1e-12), rel


def double_dam_break(n=4096):
    """Water (rho = 1000) at x < 1 and x > 3, y < 2 on a 4 x 4 tank, air (rho = 1) elsewhere, at
    rest with p = 0, walls, gravity -9.81 in y, beta = 1100, dt = 2e-5."""
    xc = (np.arange(n) + 0.5) * 4.0 / n
    yc = (np.arange(n) + 0.5) * 4.0 / n
    # mirror cells get bitwise mirror states: decide the columns on the left half and reflect
    left = xc[: n // 2] < 1.0
    water_x = np.concatenate([left, left[::-1]])
    q = np.zeros((4, n, n))
    q[0] = np.where(water_x[None, :] & (yc[:, None] < 2.0), 1000.0, 1.0)
    t = wl.Tank(n, n, 4.0, 4.0, q, gy=-9.81, beta=1100.0)
    return wl.Workload(f"double_dam_break_{n}x{n}", [t], dt=2e-5, steps=1, max_pseudo=1)


@pytest.mark.parametrize("options", list(OPTIONS))
@pytest.mark.parametrize("kernel", ["march", "tile"])
@pytest.mark.parametrize("precision", ["f64", "mixed"])
def test_mirror_symmetry_on_the_full_tank(precision, kernel, options):
    kw, bdf = OPTIONS[options]
    wk = double_dam_break()
    wk.bdf = bdf
    t = wk.tanks[0]
    shape = SHAPES[(precision, kernel)]
    print(f"[invariants] mirror: {wk.name} {precision} shape {shape} {options}, 3 steps x 10 "
          f"pseudo-iterations", flush=True)
    q = run(wk, precision, shape, steps=3, pseudo=10, **kw)
    m = q[:, :, ::-1].copy()
    m[1] = -m[1]
    sc = field_scales(t)
    err = np.array([np.abs(q[k] - m[k]).max() / sc[k] for k in range(4)])
    moved = np.abs(q[1]).max() / sc[1]
    print(f"[invariants]   mirror differences / scale: rho {err[0]:.2e} rho_u {err[1]:.2e} "
          f"rho_v {err[2]:.2e} p {err[3]:.2e} (max |rho u| / scale {moved:.2e})", flush=True)
    assert moved > 1e-6
    assert np.all(err <= (1e-12 if precision == "f64" else 1e-9)), err


@functools.lru_cache(maxsize=1)
def corner_state(n=4096):
    c = (np.arange(n) + 0.5) * 4.0 / n
    x, y = c[None, :], c[:, None]
    water = ((x < 2.0) & (y < 1.0)) | ((x < 1.0) & (y < 2.0))
    q = np.zeros((4, n, n))
    q[0] = np.where(water, 1000.0, 1.0)
    solid = ((x > 2.5) & (x < 2.7) & (y > 2.5) & (y < 2.7)).astype(np.uint8)
    assert np.array_equal(q[0], q[0].T) and np.array_equal(solid, solid.T)
    q.flags.writeable = False
    solid.flags.writeable = False
    return q, solid


def transposed(a, block=256):
    """a.T as a contiguous array, copied in square blocks (a strided whole-array transpose of a
    4096 x 4096 plane is several times slower)."""
    out = np.empty((a.shape[1], a.shape[0]), a.dtype)
    for i in range(0, a.shape[0], block):
        for j in range(0, a.shape[1], block):
            out[j:j + block, i:i + block] = a[i:i + block, j:j + block].T
    return out


def corner_dam_break(n=4096):
    """A tank symmetric about its diagonal: water (rho = 1000) in the L-shaped region x < 2, y < 1
    or x < 1, y < 2 of a 4 x 4 tank, a square obstacle on the diagonal (2.5 < x, y < 2.7),
    gravity of 9.81 along the diagonal towards the corner (0, 0), beta = 1100, dt = 2e-5."""
    q, solid = corner_state(n)
    g = -9.81 / np.sqrt(2.0)
    t = wl.Tank(n, n, 4.0, 4.0, q, gx=g, gy=g, beta=1100.0, solid=solid)
    return wl.Workload(f"corner_dam_break_{n}x{n}", [t], dt=2e-5, steps=1, max_pseudo=1)


@pytest.mark.parametrize("options", list(OPTIONS))
@pytest.mark.parametrize("kernel", ["march", "tile"])
@pytest.mark.parametrize("precision", ["f64", "mixed"])
def test_transpose_symmetry_on_the_full_tank(precision, kernel, options):
    """The scheme is the same with x and y exchanged (per-axis slopes and limiters, the flux
    rotated to each face, the pressure gradient's x and y forms, the symmetric pseudo-time step),
    so a tank symmetric about its diagonal stays symmetric: rho and p equal their transposes and
    rho u that of rho v.  The row-marching kernel takes the x faces across the lanes of a wave
    and the y faces down its march, and the tiles are 32 x 8, so this holds the two code paths
    of every cell against each other."""
    kw, bdf = OPTIONS[options]
    wk = corner_dam_break()
    wk.bdf = bdf
    t = wk.tanks[0]
    shape = SHAPES[(precision, kernel)]
    print(f"[invariants] transpose: {wk.name} {precision} shape {shape} {options}, 3 steps x 10 "
          f"pseudo-iterations", flush=True)
    q = run(wk, precision, shape, steps=3, pseudo=10, **kw)
    sc = field_scales(t)
    # solid cells come back as they went in, which is symmetric, so every cell is compared
    qt = [transposed(q[k]) for k in range(4)]
    pairs = [(q[0], qt[0]), (q[1], qt[2]), (q[2], qt[1]), (q[3], qt[3])]
    err = np.array([np.abs(a - b).max() / sc[k] for k, (a, b) in enumerate(pairs)])
    moved = max(np.abs(q[1]).max(), np.abs(q[2]).max()) / sc[1]
    print(f"[invariants]   transpose differences / scale: rho {err[0]:.2e} rho_u {err[1]:.2e} "
          f"rho_v {err[2]:.2e} p {err[3]:.2e} (max |rho u|, |rho v| / scale {moved:.2e})",
          flush=True)
    assert moved > 1e-6
    assert np.all(err <= (1e-12 if precision == "f64" else 1e-9)), err


RT_SHAPES = {("f64", "march"): (-2, 6), ("mixed", "march"): (-2, 3),
             ("f64", "tile"): (3208, 2), ("mixed", "tile"): (1608, 2)}


@pytest.mark.parametrize("kernel", ["march", "tile"])
@pytest.mark.parametrize("precision", ["f64", "mixed"])
def test_periodic_translation_on_the_full_tank(precision, kernel):
    """Translation along a periodic axis: the 256 x 1024 Rayleigh-Taylor tank (periodic in x) with
    its initial state shifted by k columns gives the shifted result, bit for bit.  With local
    pseudo-time steps every cell's arithmetic depends only on its neighbourhood, not on where it
    sits in its strip (256 = 4 x 60 + 16 columns), chunk or tile, nor on the wrap across the
    periodic sides; shifts of 17 and 61 columns move every cell to another lane and strip."""
    wk = wl.rayleigh_taylor(precision=precision)
    t = wk.tanks[0]
    shape = RT_SHAPES[(precision, kernel)]
    print(f"[invariants] translation: {wk.name} {precision} shape {shape}, 3 steps x 10 "
          f"pseudo-iterations", flush=True)
    base = run(wk, precision, shape, steps=3, pseudo=10)
    q0 = t.q
    for k in (17, 61):
        t.q = np.ascontiguousarray(np.roll(q0, k, axis=2))
        shifted = run(wk, precision, shape, steps=3, pseudo=10)
        diff = np.abs(np.roll(base, k, axis=2) - shifted).max()
        print(f"[invariants]   shift {k}: max difference {diff:.3e}", flush=True)
        np.testing.assert_array_equal(np.roll(base, k, axis=2), shifted)
    t.q = q0


@pytest.mark.parametrize("kernel", ["march", "tile"])
@pytest.mark.parametrize("precision", ["f64", "mixed"])
def test_free_stream_on_the_full_tank(precision, kernel):
    """A uniform state moving obliquely through a tank periodic on both axes, without gravity,
    is a steady state: every face flux is F(Q, Q) on both sides of every cell, the gradients and
    the real-time term vanish, so the state stays the same bit for bit and the residual norms
    are exactly zero."""
    n = 4096
    q = np.zeros((4, n, n))
    q[0], q[1], q[2], q[3] = 2.0, 2.0 * 0.3, 2.0 * -0.2, 5.0
    t = wl.Tank(n, n, 4.0, 4.0, q, gx=0.0, gy=0.0, beta=1100.0, bc=(1, 1, 1, 1))
    wk = wl.Workload(f"free_stream_{n}x{n}", [t], dt=2e-5, steps=1, max_pseudo=1)
    shape = SHAPES[(precision, kernel)]
    print(f"[invariants] free stream: {wk.name} {precision} shape {shape}", flush=True)
    out, norms = run(wk, precision, shape, steps=2, pseudo=10, with_norms=True)
    print(f"[invariants]   max change {np.abs(out - q).max():.3e}, norms {norms}", flush=True)
    np.testing.assert_array_equal(out, q)
    np.testing.assert_array_equal(norms, np.zeros(4))


def hydrostatic_obstacle(n=4096):
    """The exact discrete hydrostatic state of a two-layer tank on 4 x 4 (water below y = 2, on a
    face; p_{j+1} - p_j = g dy (rho_j + rho_{j+1}) / 2 plus a constant) with the benchmark's
    obstacle in the water (2.5 < x < 2.7, y < 0.3), at rest, beta = 1100, dt = 2e-5."""
    dy = 4.0 / n
    yc = (np.arange(n) + 0.5) * dy
    rho = np.where(yc < 2.0, 1000.0, 1.0)
    p = np.concatenate([[0.0], np.cumsum(-9.81 * dy * (rho[:-1] + rho[1:]) / 2)])
    q = np.zeros((4, n, n))
    q[0] = rho[:, None]
    q[3] = (p + 50.0)[:, None]
    xc = (np.arange(n) + 0.5) * 4.0 / n
    solid = ((xc[None, :] > 2.5) & (xc[None, :] < 2.7) & (yc[:, None] < 0.3)).astype(np.uint8)
    t = wl.Tank(n, n, 4.0, 4.0, q, gy=-9.81, beta=1100.0, solid=solid)
    return wl.Workload(f"hydrostatic_obstacle_{n}x{n}", [t], dt=2e-5, steps=1, max_pseudo=1)


@pytest.mark.parametrize("kernel", ["march", "tile"])
@pytest.mark.parametrize("precision", ["f64", "mixed"])
def test_hydrostatic_balance_on_the_full_tank(precision, kernel):
    """Sec. 2.3.2: the new pressure gradient (rho g at rest, with reversed gravity in the wall
    ghosts of Sec. 2.5) makes the two face pressures of every face agree exactly for the discrete
    hydrostatic profile, so a two-layer tank at rest stays at rest, around an obstacle too: on
    every fluid cell of the 4096 x 4096 tank the momenta stay below 1e-9 and the pressure moves
    by at most 1e-12 of its largest value."""
    wk = hydrostatic_obstacle()
    t = wk.tanks[0]
    fluid = t.solid == 0
    shape = SHAPES[(precision, kernel)]
    print(f"[invariants] hydrostatic: {wk.name} {precision} shape {shape}", flush=True)
    out, norms = run(wk, precision, shape, steps=2, pseudo=20, with_norms=True)
    mom = np.abs(out[1:3][:, fluid]).max()
    dp = np.abs(out[3] - t.q[3])[fluid].max() / np.abs(t.q[3]).max()
    print(f"[invariants]   max |rho u|, |rho v| {mom:.3e}, pressure change {dp:.3e} of max |p|, "
          f"norms {norms}", flush=True)
    assert mom <= 1e-9 and dp <= 1e-12, (mom, dp)


@pytest.mark.parametrize("precision", ["f64", "mixed"])
def test_mass_conserved_in_every_tank_of_the_ensemble(precision):
    """The batched launch on the full 512-tank sloshing ensemble (uneven closed tanks, some
    stored reflected about their diagonal), in the shape bench.py times (row marching, 2 waves
    per SIMD, chunks of 16 rows), under a global pseudo-time step with free-slip walls: every
    tank keeps its own total mass, so no unit of the batch reads or writes another tank's cells
    or mixes their steps.  FP64: 1e-13 relative.  The mixed form rounds every cell's deviation
    from level n to FP32 on each of the 30 stages of a step, by at most 2^-24 of it; the
    deviation within a step is about the step's own change, which in these small tanks reaches a
    few density units at the moving interface, so each tank is held to 30 x 2^-24 x (sum over
    its steps and cells of |that step's density change|) / its mass (worst case 7e-10, measured
    9e-12)."""
    from parity import stored_transposed_in_batch
    wk = wl.sloshing_ensemble(precision=precision)
    wk.local_dtau = False
    tanks = [dict(nx=t.nx, ny=t.ny, lx=t.lx, ly=t.ly, gx=t.gx, gy=t.gy, beta=t.beta, bc=t.bc)
             for t in wk.tanks]
    n_reflected = sum(stored_transposed_in_batch(t) for t in wk.tanks)
    print(f"[invariants] ensemble mass: {len(wk.tanks)} tanks ({n_reflected} stored reflected), "
          f"{precision}, shape (-2, 16), global pseudo-time step, free-slip walls, 2 steps x 10",
          flush=True)
    grid = vdac.Grid(tanks, gpu_options(wk, precision, tile=(-2, 16), wall_slip=True))
    n = len(wk.tanks)
    change = np.zeros(n)   # sum over steps of sum over cells of |the step's density change|
    try:
        for i, t in enumerate(wk.tanks):
            grid.set_state(i, t.q)
        prev = [t.q[0] for t in wk.tanks]
        for _ in range(2):
            rc, done = grid.step(wk.dt, 10, 0.0, check=False)
            assert rc == 0 and np.all(np.asarray(done) == 10), rc
            states = [grid.get_state(i) for i in range(n)]
            for i in range(n):
                change[i] += np.abs(states[i][0] - prev[i]).sum()
                prev[i] = states[i][0]
    finally:
        grid.close()
    mass0 = np.array([t.q[0].sum() for t in wk.tanks])
    mass1 = np.array([q[0].sum() for q in states])
    rel = np.abs(mass1 - mass0) / mass0
    if precision == "f64":
        bar = np.full(n, 1e-13)
    else:
        bar = np.maximum(1e-13, 30 * 2.0 ** -24 * change / mass0)
    worst = int(np.argmax(rel / bar))
    print(f"[invariants]   worst relative mass change {rel.max():.2e} (tank {int(rel.argmax())}); "
          f"largest share of its bar {rel[worst] / bar[worst]:.3f} (tank {worst}, bar "
          f"{bar[worst]:.2e})", flush=True)
    assert change.max() > 1e-6
    assert np.all(rel <= bar), (worst, rel[worst], bar[worst])


@pytest.mark.parametrize("kernel", ["march", "tile"])
def test_steady_state_independent_of_the_pseudo_time_cfl(kernel):
    """At the incompressible limit the pseudo-time path does not matter (Algorithm 1 iterates
    to the state whose pseudo-time derivative vanishes): the 64 x 64 two-layer tank of the first
    benchmark configuration, from p = 0, run to residual norms below 1e-9 with CFL_tau 0.48 and
    0.3 (local steps, one real step of 1e-2), reaches the same state: p minus its mean (local
    steps do not keep the total p) to 1e-8 of its size, momenta below 1e-8."""
    from paper_2108_08769_amd import workloads as wl2
    shape = (-2, 1) if kernel == "march" else (32, 8)
    outs, its = [], []
    for cfl in (0.48, 0.3):
        wk = wl2.hydrostatic()
        wk.cfl = cfl
        t = wk.tanks[0]
        tank = dict(nx=t.nx, ny=t.ny, lx=t.lx, ly=t.ly, gx=t.gx, gy=t.gy, beta=t.beta, bc=t.bc)
        grid = vdac.Grid([tank], gpu_options(wk, "f64", tile=shape))
        try:
            grid.set_state(0, t.q)
            rc, done = grid.step(1e-2, 200000, 1e-9, check=False)
            assert rc == 0 and int(done[0]) < 200000, (rc, done)
            outs.append(grid.get_state(0))
            its.append(int(done[0]))
        finally:
            grid.close()
    p0 = outs[0][3] - outs[0][3].mean()
    p1 = outs[1][3] - outs[1][3].mean()
    dp = np.abs(p0 - p1).max() / np.abs(p0).max()
    mom = max(np.abs(o[1:3]).max() for o in outs)
    print(f"[invariants] steady state, {kernel}: {its} iterations (CFL 0.48, 0.3), p difference "
          f"{dp:.2e} of max |p - mean|, momenta {mom:.2e}", flush=True)
    assert dp <= 1e-8 and mom <= 1e-8, (dp, mom)
