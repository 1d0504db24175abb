"""GPU path of the further options against the oracle, through the C ABI: the Roe and exact
(Bassi) fluxes, the k-limiter and split limiter on p, zero-gradient sides with the
pseudo-time-only mode and global pseudo-time steps (the Riemann problems of Table 2), BDF3, and
the global real-time step; the mixed form of each against FP64; each in the row-marching kernel
and in every LDS tile shape.

Bars as in the other parity files: FP64 per field max |gpu - oracle| / max(max |oracle|,
physical scale) <= 1e-12 with equal iteration counts; mixed against FP64 normwise <= 1e-6 (rho),
1e-5 (rho u; rho v against its physical scale), 1e-4 (p).
"""
import csv
import math
import os

import numpy as np
import pytest

from paper_2108_08769_amd import vdac
from paper_2108_08769_amd import workloads as wl
from parity import (run_gpu, run_oracle, field_errors, field_scales, plain_errors, reflect,
                    stored_transposed_in_batch, unreflect_state)

pytestmark = pytest.mark.gpu

TOL = 1e-12
W, P, O = 0, 1, 2
OSHER, ROE, BASSI = 0, 1, 2
NEW, LIMITER, SPLIT = 0, 1, 2
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def check(wk, steps, pseudo, bar=TOL, scales=None, **kw):
    print(f"[next] {wk.name} steps={steps} pseudo={pseudo} {kw}", flush=True)
    g = run_gpu(wk, steps, pseudo, **kw)
    o = run_oracle(wk, steps, pseudo, **kw)
    assert all(c == 0 for c in g[3]) and all(c == 0 for c in o[3]), (g[3], o[3])
    np.testing.assert_array_equal(g[1], o[1])
    worst = 0.0
    for t, a, b in zip(wk.tanks, g[0], o[0]):
        sc = field_scales(t) if scales is None else scales
        err = field_errors(a, b, t.solid, sc)
        worst = max(worst, err.max())
        assert np.all(err <= bar), (t.nx, t.ny, err)
        plain = plain_errors(a, b, t.solid, sc)
        ok = ~np.isnan(plain)
        assert np.all(plain[ok] <= bar), (t.nx, t.ny, plain)
    for a, b in zip(g[2], o[2]):
        # norms agree to rtol 1e-7 above the rounding floor of the flux divergence: the kernel
        # sums face fluxes scaled by 1/h, so a field whose fluxes cancel (v = 0 in a 1D problem)
        # keeps the rounding error of p/h, about 1e-16 of the largest residual
        np.testing.assert_allclose(a, b, rtol=1e-7, atol=max(1e-12, 1e-14 * np.abs(b).max()))
    print(f"[next]   worst field error {worst:.3e}", flush=True)


def check_mixed(wk, steps, pseudo, **kw):
    print(f"[next-mixed] {wk.name} steps={steps} pseudo={pseudo} {kw}", flush=True)
    m = run_gpu(wk, steps, pseudo, precision="mixed", **kw)
    d = run_gpu(wk, steps, pseudo, precision="f64", **kw)
    assert all(c == 0 for c in m[3]) and all(c == 0 for c in d[3])
    np.testing.assert_array_equal(m[1], d[1])
    for t, a, b in zip(wk.tanks, m[0], d[0]):
        mask = np.ones(a.shape[1:], bool) if t.solid is None else t.solid == 0
        nw = [np.abs(a[k][mask] - b[k][mask]).max() / max(np.abs(b[k][mask]).max(), 1e-300)
              for k in range(4)]
        sc = field_errors(a, b, t.solid, field_scales(t))
        print(f"[next-mixed]   normwise rho {nw[0]:.2e} rho_u {nw[1]:.2e} rho_v(scaled) "
              f"{sc[2]:.2e} p {nw[3]:.2e}", flush=True)
        assert nw[0] <= 1e-6 and nw[1] <= 1e-5 and sc[2] <= 1e-5 and nw[3] <= 1e-4, (nw, sc)


def dam(nx, ny, bc=(W, W, W, W), dt=1e-3, lx=4.0, ly=2.0, **wkargs):
    xc = (np.arange(nx) + 0.5) * lx / nx
    yc = (np.arange(ny) + 0.5) * ly / ny
    rho = np.where((xc[None, :] < 1.0) & (yc[:, None] < 1.0), 1000.0, 1.0)
    q = np.zeros((4, ny, nx))
    q[0] = rho
    return wl.Workload(f"dam_{nx}x{ny}", [wl.Tank(nx, ny, lx, ly, q, gy=-9.81, beta=1100.0, bc=bc)],
                       dt=dt, steps=1, max_pseudo=1, **wkargs)


def obstacle(n=48):
    wk = wl.obstacle_dam_break(n=n)
    wk.dt = 1e-3
    return wk


# ---- fluxes and pressure gradients ------------------------------------------------------------

@pytest.mark.parametrize("flux", [ROE, BASSI])
def test_riemann_solvers(flux):
    check(dam(37, 23), steps=3, pseudo=20, flux=flux)
    check(wl.rayleigh_taylor(nx=32, ny=72, precision="f64"), steps=2, pseudo=10, flux=flux)


@pytest.mark.parametrize("pgrad,pk", [(LIMITER, 1.0), (LIMITER, 2.0), (SPLIT, 1.0), (SPLIT, 2.0)])
def test_pressure_gradient_variants(pgrad, pk):
    check(dam(37, 23), steps=3, pseudo=20, pgrad=pgrad, pk=pk)
    check(obstacle(), steps=2, pseudo=10, pgrad=pgrad, pk=pk)


def test_split_limiter_is_well_balanced_on_gpu():
    """The exact discrete hydrostatic state is a steady state of the split limiter."""
    ny, nx = 40, 8
    dy = 1.0 / ny
    yc = (np.arange(ny) + 0.5) * dy
    rho = np.where(yc < 0.5, 1000.0, 1.0)
    p = np.zeros(ny)
    for j in range(ny - 1):
        p[j + 1] = p[j] - 9.81 * dy * (rho[j] + rho[j + 1]) / 2
    q = np.zeros((4, ny, nx))
    q[0], q[3] = rho[:, None], (p + 50.0)[:, None]
    wk = wl.Workload("hydro_split", [wl.Tank(nx, ny, 0.2, 1.0, q, gy=-9.81, beta=1000.0)], dt=1e-3,
                     steps=1, max_pseudo=1)
    states, _, norms, codes = run_gpu(wk, 2, 30, pgrad=SPLIT, pk=2.0)
    assert codes == [0, 0]
    assert np.abs(states[0][1:3]).max() <= 1e-9 and norms[0].max() <= 1e-8


# ---- zero-gradient sides, global pseudo-time steps, pseudo-time only --------------------------

def table2():
    with open(os.path.join(GOLDEN, "riemann_problems_table2.csv")) as f:
        rows = [r for r in csv.reader(line for line in f if not line.startswith("#"))]
    return [dict(zip(rows[0], map(float, r))) for r in rows[1:]]


def rp_workload(rp, nx):
    """Sec. 3.1 setup: nx x 1 square cells on [0, 1], jump at x = 1/2, zero-gradient sides, no
    gravity, global pseudo-time steps at CFL 0.98, no real-time term (dt = +infinity)."""
    dx = 1.0 / nx
    x = (np.arange(nx) + 0.5) * dx
    left = x < 0.5
    q = np.zeros((4, 1, nx))
    q[0, 0] = np.where(left, rp["rho_L"], rp["rho_R"])
    q[1, 0] = q[0, 0] * np.where(left, rp["u_L"], rp["u_R"])
    q[3, 0] = np.where(left, rp["p_L"], rp["p_R"])
    t = wl.Tank(nx, 1, 1.0, dx, q, gx=0.0, gy=0.0, beta=rp["beta"], bc=(O, O, O, O))
    return wl.Workload(f"rp_{int(rp['rp'])}_{nx}", [t], dt=math.inf, steps=1, max_pseudo=1,
                       cfl=0.98, local_dtau=False)


@pytest.mark.parametrize("flux", [OSHER, ROE, BASSI])
@pytest.mark.parametrize("rp_index", [0, 1, 2, 3, 4])
def test_riemann_problems_of_table2(rp_index, flux):
    rp = table2()[rp_index]
    wk = rp_workload(rp, 100)
    t = wk.tanks[0]
    scales = np.array([np.abs(t.q[0]).max(), np.abs(t.q[0]).max() * 10.0,
                       np.abs(t.q[0]).max() * 10.0, np.abs(t.q[3]).max()])
    check(wk, steps=1, pseudo=25, scales=scales, flux=flux, pgrad=LIMITER, pk=1.0)


def test_zero_gradient_sides_on_a_dam_break():
    check(dam(37, 23, bc=(O, O, W, W)), steps=3, pseudo=20)
    check(dam(41, 19, bc=(W, O, W, O)), steps=2, pseudo=15, pgrad=LIMITER, pk=2.0, flux=ROE)


def test_global_pseudo_time_step():
    wk = dam(37, 23, local_dtau=False)
    check(wk, steps=3, pseudo=20)


def test_pseudo_time_only_with_walls():
    """Pseudo-time only (dt = +infinity) on the two-layer tank relaxing from p = 0 (a dam break
    without the real-time term diverges, on the GPU and in the oracle alike)."""
    wk = wl.hydrostatic(16, 16)
    wk.dt = math.inf
    check(wk, steps=2, pseudo=20)


# ---- BDF3 and the real-time step ---------------------------------------------------------------

def test_bdf3():
    """Five steps: backward Euler, BDF2, then BDF3 (Table 1), as in the oracle."""
    wk = dam(37, 23, bdf=3)
    check(wk, steps=5, pseudo=10)


def test_realtime_dt_matches_oracle():
    import oracle
    from parity import oracle_problem
    wk = dam(37, 23)
    tanks = [dict(nx=t.nx, ny=t.ny, lx=t.lx, ly=t.ly, gx=t.gx, gy=t.gy, beta=t.beta, bc=t.bc)
             for t in wk.tanks]
    for prec in ("f64", "mixed"):
        grid = vdac.Grid(tanks, vdac.make_options(precision=prec))
        try:
            grid.set_state(0, wk.tanks[0].q)
            assert grid.realtime_dt(0, 0.45) == math.inf       # at rest
            for _ in range(3):
                grid.step(wk.dt, 20)
            q = grid.get_state(0)
            got = grid.realtime_dt(0, 0.45)
        finally:
            grid.close()
        ref = oracle.realtime_dt(oracle_problem(wk.tanks[0], wk), q, 0.45)
        print(f"[next] realtime dt {prec}: {got:.6e} (oracle on the same state {ref:.6e})", flush=True)
        assert got == pytest.approx(ref, rel=1e-14)


# ---- the mixed form, graphs and batches of the general kernel ---------------------------------

CASES = ["roe", "bassi", "limiter", "split", "open", "global", "bdf3", "combined"]


def case_options(case):
    """(flux/pgrad keywords, workload keywords, sides) of one general-option case; "combined"
    puts zero-gradient sides, the Roe flux, the k-limiter on p and the global step together."""
    kw, wkargs, bc = {}, {}, (W, W, W, W)
    if case == "roe":
        kw["flux"] = ROE
    elif case == "bassi":
        kw["flux"] = BASSI
    elif case == "limiter":
        kw.update(pgrad=LIMITER, pk=1.0)
    elif case == "split":
        kw.update(pgrad=SPLIT, pk=2.0)
    elif case == "open":
        bc = (O, O, W, W)
    elif case == "global":
        wkargs["local_dtau"] = False
    elif case == "bdf3":
        wkargs["bdf"] = 3
    elif case == "combined":
        kw.update(flux=ROE, pgrad=LIMITER, pk=2.0)
        wkargs["local_dtau"] = False
        bc = (W, O, W, O)
    return kw, wkargs, bc


@pytest.mark.parametrize("case", CASES[:-1])
def test_mixed_general_options(case):
    kw, wkargs, bc = case_options(case)
    check_mixed(dam(96, 48, bc=bc, **wkargs), steps=4, pseudo=20, tile=(-2, 8), **kw)


# every LDS tile shape: 256-thread 32 x 8, 16 x 16, 64 x 4; 512-thread 32 x 8, 16 x 16; 320-thread 16 x 8
TILE_SHAPES = [(32, 8), (16, 16), (64, 4), (3208, 2), (1616, 2), (1608, 2)]


@pytest.mark.parametrize("tile", TILE_SHAPES)
@pytest.mark.parametrize("case", CASES)
def test_general_options_on_tiles(case, tile):
    """Each general option in the LDS-tiled kernel, on a tank whose sides are not multiples of
    any tile, against the oracle (four real steps: BDF3 from the third)."""
    kw, wkargs, bc = case_options(case)
    check(dam(37, 23, bc=bc, **wkargs), steps=4, pseudo=12, tile=tile, **kw)


@pytest.mark.parametrize("tile", [(64, 4), (3208, 2), (1608, 2)])
@pytest.mark.parametrize("flux", [OSHER, BASSI])
@pytest.mark.parametrize("rp_index", [0, 1, 2, 3, 4])
def test_riemann_problem_on_tiles(rp_index, flux, tile):
    """The Riemann problems of Table 2 (a tank one cell tall: zero-gradient sides, global step,
    no real-time term) in the tiled kernel against the oracle."""
    rp = table2()[rp_index]
    wk = rp_workload(rp, 100)
    t = wk.tanks[0]
    scales = np.array([np.abs(t.q[0]).max(), np.abs(t.q[0]).max() * 10.0,
                       np.abs(t.q[0]).max() * 10.0, np.abs(t.q[3]).max()])
    check(wk, steps=1, pseudo=25, scales=scales, flux=flux, pgrad=LIMITER, pk=1.0, tile=tile)


@pytest.mark.parametrize("tile", [(3208, 2), (1608, 2)])
@pytest.mark.parametrize("case", CASES)
def test_mixed_general_options_on_tiles(case, tile):
    kw, wkargs, bc = case_options(case)
    check_mixed(dam(96, 48, bc=bc, **wkargs), steps=4, pseudo=20, tile=tile, **kw)


@pytest.mark.parametrize("tile", [(-2, 8), (3208, 2)], ids=["march", "tile"])
def test_general_kernel_graph_replay_matches_eager(tile):
    wk = dam(70, 40, bc=(O, W, W, W), local_dtau=False)
    a = run_gpu(wk, 3, 12, flux=BASSI, pgrad=LIMITER, graph_iters=0, tile=tile)
    b = run_gpu(wk, 3, 12, flux=BASSI, pgrad=LIMITER, graph_iters=-1, tile=tile)
    for x, y in zip(a[0], b[0]):
        np.testing.assert_array_equal(x, y)
    np.testing.assert_array_equal(a[2], b[2])


def test_general_kernel_batch_equals_single_tanks():
    """Tanks with different side kinds in one grid (one launch per stage) come out bit for bit
    as in grids of their own."""
    tanks = [dam(37, 23, bc=(O, O, W, W)).tanks[0], dam(45, 17).tanks[0],
             dam(29, 31, bc=(W, O, O, W)).tanks[0]]
    wk = wl.Workload("mixed_sides", tanks, dt=1e-3, steps=1, max_pseudo=1)
    batch = run_gpu(wk, 2, 8, flux=ROE, pgrad=LIMITER, tile=(-2, 8))
    for i, t in enumerate(tanks):
        # the batch stores the 29 x 31 tank with x and y exchanged: compare with its reflection
        tr = stored_transposed_in_batch(t)
        one = wl.Workload("one", [reflect(t) if tr else t], dt=1e-3, steps=1, max_pseudo=1)
        single = run_gpu(one, 2, 8, flux=ROE, pgrad=LIMITER, tile=(-2, 8))
        got = unreflect_state(single[0][0]) if tr else single[0][0]
        np.testing.assert_array_equal(batch[0][i], got, err_msg=f"tank {i} (transposed {tr})")
    assert [stored_transposed_in_batch(t) for t in tanks] == [False, False, True]


def test_pressure_gradient_comparison_of_sec_3_3_1():
    """The first real step of the 20 x 20 dam break of Sec. 3.3.1 (Osher, minmod on rho, u, v,
    three stages, CFL 0.48, local steps, dt = 0.01, beta = 1100; water at x < 0.4, y < 0.8 of the
    unit square; 3000 pseudo-iterations) with the new pressure gradient and the split limiter
    with superbee and with minmod: each against the oracle at the FP64 bar, and the paper's
    ordering of how much the water beside the free surface is compressed (the new method least,
    the split minmod limiter most) on the GPU."""
    n = 20
    xc = (np.arange(n) + 0.5) / n
    q = np.zeros((4, n, n))
    q[0] = np.where((xc[None, :] < 0.4) & (xc[:, None] < 0.8), 1000.0, 1.0)
    comp = {}
    for name, pgrad, pk in [("new", NEW, 1.0), ("split-superbee", SPLIT, 2.0),
                            ("split-minmod", SPLIT, 1.0)]:
        wk = wl.Workload(f"sec331_{name}", [wl.Tank(n, n, 1.0, 1.0, q, gy=-9.81, beta=1100.0)],
                         dt=0.01, steps=1, max_pseudo=1)
        check(wk, steps=1, pseudo=3000, pgrad=pgrad, pk=pk)
        states = run_gpu(wk, 1, 3000, pgrad=pgrad, pk=pk)[0]
        comp[name] = states[0][0, 0, 7] - 1000.0     # lowest row, the cell left of x = 0.4
    print(f"[next] Sec. 3.3.1 compression of the water beside the surface: {comp}", flush=True)
    assert 0.0 < comp["new"] < comp["split-superbee"] < comp["split-minmod"], comp


@pytest.mark.parametrize("method", ["new", "split-minmod", "split-superbee", "minmod", "superbee"])
def test_hydrostatic_comparison_of_sec_3_2(method):
    """Sec. 3.2: a 20-cell column (gravity 9.81 along x, water on the +x half, beta = 2000, local
    pseudo-time steps at CFL 0.98, one real step of dt = 0.05 from rest with p = 0,
    pseudo-iterations until every residual norm is below 1e-5).  The GPU stops at the oracle's iteration with the
    oracle's state; the new gradient and the split limiters end at rest (|u| < 1e-8), the
    k-limiter applied to p (minmod, superbee) leaves spurious speeds (|u| > 1e-6)."""
    pgrad, pk = {"new": (NEW, 1.0), "split-minmod": (SPLIT, 1.0), "split-superbee": (SPLIT, 2.0),
                 "minmod": (LIMITER, 1.0), "superbee": (LIMITER, 2.0)}[method]
    nx = 20
    xc = (np.arange(nx) + 0.5) / nx
    q = np.zeros((4, 1, nx))
    q[0] = np.where(xc > 0.5, 1000.0, 1.0)
    wk = wl.Workload(f"sec32_{method}", [wl.Tank(nx, 1, 1.0, 1.0 / nx, q, gx=9.81, gy=0.0,
                                                  beta=2000.0)],
                     dt=0.05, steps=1, max_pseudo=1, cfl=0.98)
    g = run_gpu(wk, 1, 20000, tol=1e-5, pgrad=pgrad, pk=pk)
    o = run_oracle(wk, 1, 20000, tol=1e-5, pgrad=pgrad, pk=pk)
    assert g[3] == [0] and o[3] == [0], (g[3], o[3])
    np.testing.assert_array_equal(g[1], o[1])
    t = wk.tanks[0]
    err = field_errors(g[0][0], o[0][0], None, field_scales(t))
    umax = np.abs(g[0][0][1] / g[0][0][0]).max()
    print(f"[next] Sec. 3.2 {method}: {int(g[1][0, 0])} pseudo-iterations, max |u| {umax:.3e}, "
          f"field errors {err}", flush=True)
    assert np.all(err <= TOL), err
    if method in ("new", "split-minmod", "split-superbee"):
        assert umax < 1e-8
    else:
        assert umax > 1e-6
