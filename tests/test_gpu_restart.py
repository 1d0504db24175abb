"""Real-time history and the Runge-Kutta stage count, through the C ABI.

- Restart (Table 1): a BDF2 or BDF3 run that is stopped after k real steps, taken apart with
  get_state and get_history, and continued on a new grid after set_state and set_history gives
  bit for bit the states, residual norms and iteration counts of the run that never stopped.
- Per-tank history: set_state on one tank of a batch discards that tank's earlier levels only
  (its next step is backward Euler), and the other tanks keep their BDF order; each tank is held
  to the oracle run with the same history.
- Stage counts other than three: with one stage, stage 1 is also the last, so the residual
  finalize of the previous iteration cannot share its launch; with one, two and four stages and a
  tolerance the pseudo-loop stops at the oracle's iteration, with several launch groups per step.
- A new grid holds the state at rest in every buffer and level until set_state, and steps from it
  as the oracle does.

FP64 bars as in the other parity files: per field max |gpu - oracle| / max(max |oracle|,
physical scale) <= 1e-12, equal iteration counts, norms to rtol 1e-7.
"""
import numpy as np
import pytest

from paper_2108_08769_amd import vdac
from paper_2108_08769_amd import workloads as wl
import oracle
from parity import field_errors, field_scales, gpu_options, oracle_problem, run_gpu, run_oracle

pytestmark = pytest.mark.gpu

TOL = 1e-12


def tank_dicts(wk):
    return [dict(nx=t.nx, ny=t.ny, lx=t.lx, ly=t.ly, gx=t.gx, gy=t.gy, beta=t.beta, bc=t.bc,
                 solid=t.solid) for t in wk.tanks]


def moving_tanks(n_tanks=2):
    """A wide and a tall tank with a rough moving state (the tall one is stored reflected in a
    batch on the row-marching kernel), gravity along both axes, an obstacle in the first."""
    tanks = []
    for i, (nx, ny) in enumerate([(70, 23), (19, 66)][:n_tanks]):
        q = wl.random_state(nx, ny, seed=40 + i, rho_range=(1.0, 5.0), vel=0.3, p_scale=10.0)
        solid = None
        if i == 0:
            solid = np.zeros((ny, nx), np.uint8)
            solid[3:6, 40:44] = 1
        tanks.append(wl.Tank(nx, ny, 0.05 * nx, 0.04 * ny, q, gx=0.4, gy=-9.81, beta=500.0,
                             solid=solid))
    return wl.Workload("moving", tanks, dt=2e-3, steps=1, max_pseudo=1)


def run_steps(grid, wk, steps, pseudo, tol):
    out = []
    for _ in range(steps):
        rc, done = grid.step(wk.dt, pseudo, tol, check=False)
        assert rc == 0
        out.append(done)
    return np.array(out)


@pytest.mark.parametrize("precision", ["f64", "mixed"])
@pytest.mark.parametrize("bdf", [1, 2, 3])
@pytest.mark.parametrize("shape", ["march", "tile"])
def test_restart_with_history_is_bitwise(precision, bdf, shape):
    wk = moving_tanks(2 if shape == "march" else 1)
    wk.bdf = bdf
    tile = (0, 0) if shape == "march" else (32, 8)
    opts = gpu_options(wk, precision=precision, tile=tile)
    N, k, pseudo, tol = 6, 2, 12, 1e-3
    print(f"[restart] {precision} bdf={bdf} {shape}: {N} steps straight vs {k} + restart + {N - k}",
          flush=True)
    g = vdac.Grid(tank_dicts(wk), opts)
    for i, t in enumerate(wk.tanks):
        g.set_state(i, t.q)
    it_straight = run_steps(g, wk, N, pseudo, tol)
    straight = [g.get_state(i) for i in range(len(wk.tanks))]
    norms_straight = [g.residual_norm(i) for i in range(len(wk.tanks))]
    g.close()

    g = vdac.Grid(tank_dicts(wk), opts)
    for i, t in enumerate(wk.tanks):
        g.set_state(i, t.q)
    it_a = run_steps(g, wk, k, pseudo, tol)
    saved = [(g.get_state(i), g.get_history(i)) for i in range(len(wk.tanks))]
    g.close()
    for q, lv in saved:
        assert len(lv) == min(k, bdf - 1)
    g = vdac.Grid(tank_dicts(wk), opts)
    for i, (q, lv) in enumerate(saved):
        g.set_state(i, q)
        g.set_history(i, lv)
        # the restored levels read back unchanged before any step
        np.testing.assert_array_equal(g.get_history(i), lv)
    it_b = run_steps(g, wk, N - k, pseudo, tol)
    resumed = [g.get_state(i) for i in range(len(wk.tanks))]
    norms_resumed = [g.residual_norm(i) for i in range(len(wk.tanks))]
    g.close()

    np.testing.assert_array_equal(np.concatenate([it_a, it_b]), it_straight)
    for a, b in zip(resumed, straight):
        np.testing.assert_array_equal(a, b)
    for a, b in zip(norms_resumed, norms_straight):
        np.testing.assert_array_equal(a, b)
    print(f"[restart]   iterations per step {it_straight[:, 0].tolist()}: bitwise equal", flush=True)


def test_history_arguments_are_checked():
    wk = moving_tanks(1)
    wk.bdf = 2
    g = vdac.Grid(tank_dicts(wk), gpu_options(wk))
    try:
        g.set_state(0, wk.tanks[0].q)
        lv = np.stack([wk.tanks[0].q[:3]] * 2)
        with pytest.raises(vdac.VdacError):  # BDF2 keeps one earlier level
            g.set_history(0, lv)
        bad = lv[:1].copy()
        bad[0, 0, 0, 0] = -1.0
        with pytest.raises(vdac.VdacError):
            g.set_history(0, bad)
        assert len(g.get_history(0)) == 0  # nothing completed since set_state
        g.set_history(0, lv[:1])
        assert len(g.get_history(0)) == 1
        g.set_state(0, wk.tanks[0].q)  # discards the restored level
        assert len(g.get_history(0)) == 0
    finally:
        g.close()


@pytest.mark.parametrize("precision", ["f64"])
def test_set_state_keeps_the_other_tanks_history(precision):
    """BDF2 batch of two tanks: after 3 steps tank 1 is set to a new state; tank 0 keeps BDF2,
    tank 1 restarts with backward Euler.  Each against the oracle run with that history."""
    wk = moving_tanks(2)
    wk.bdf = 2
    q_new = wl.random_state(wk.tanks[1].nx, wk.tanks[1].ny, seed=77, rho_range=(1.0, 5.0), vel=0.3,
                            p_scale=10.0)
    pseudo = 10
    g = vdac.Grid(tank_dicts(wk), gpu_options(wk, precision=precision))
    try:
        for i, t in enumerate(wk.tanks):
            g.set_state(i, t.q)
        run_steps(g, wk, 3, pseudo, 0.0)
        g.set_state(1, q_new)
        run_steps(g, wk, 2, pseudo, 0.0)
        got = [g.get_state(i) for i in range(2)]
    finally:
        g.close()
    # oracle: tank 0 five BDF2 steps; tank 1 three BDF2 steps, then a fresh start from q_new
    ref = []
    for i, t in enumerate(wk.tanks):
        pb = oracle_problem(t, wk)
        seq = [(t.q, 5)] if i == 0 else [(t.q, 3), (q_new, 2)]
        for q0, n in seq:
            q, prev = q0.copy(), None
            for _ in range(n):
                qn, it, _, rc = oracle.step(pb, q, wk.dt, pseudo, 0.0, qnm1=prev)
                assert rc == 0 and it == pseudo
                prev, q = q, qn
        ref.append(q)
    for t, a, b in zip(wk.tanks, got, ref):
        err = field_errors(a, b, t.solid, field_scales(t))
        print(f"[history] tank {t.nx}x{t.ny}: worst field error {err.max():.3e}", flush=True)
        assert np.all(err <= TOL), err
    # the other reading (the whole grid restarting with backward Euler) differs for tank 0
    pb = oracle_problem(wk.tanks[0], wk)
    q, prev = wk.tanks[0].q.copy(), None
    for n in range(5):
        qn, _, _, _ = oracle.step(pb, q, wk.dt, pseudo, 0.0, qnm1=None if n == 3 else prev)
        prev, q = q, qn
    assert field_errors(got[0], q, wk.tanks[0].solid, field_scales(wk.tanks[0])).max() > 1e-9


@pytest.mark.parametrize("seed", [1, 2, 3, 4, 5])
def test_random_history_operations_against_oracle(seed):
    """Seeded random sequences of step_dual_time, set_state, set_history and get_history on a
    BDF3 batch of two tanks (the tall one stored transposed), checked against a model: per tank
    the current state and the earlier real-time levels the next step uses (newest first, at most
    two).  Each step of each tank is held to the oracle given the model's levels, and get_history
    returns the model's count and levels."""
    rng = np.random.default_rng(seed)
    wk = moving_tanks(2)
    wk.bdf = 3
    pbs = [oracle_problem(t, wk) for t in wk.tanks]

    def new_state(t):
        return wl.random_state(t.nx, t.ny, seed=int(rng.integers(1 << 30)), rho_range=(1.0, 5.0),
                               vel=0.3, p_scale=10.0)

    def near(qi):
        """an earlier real-time level near the current state (as a restart would restore)"""
        lv = qi.copy()
        lv[0] *= 1.0 + 0.02 * rng.uniform(-1.0, 1.0, lv[0].shape)
        lv[1:3] += 0.02 * rng.uniform(-1.0, 1.0, lv[1:3].shape)
        return lv

    g = vdac.Grid(tank_dicts(wk), gpu_options(wk))
    q = [t.q.copy() for t in wk.tanks]
    hist = [[], []]  # full 4-field states for the oracle, newest first
    ops = []
    try:
        for i, t in enumerate(wk.tanks):
            g.set_state(i, t.q)
        for _ in range(10):
            op = str(rng.choice(["step", "step", "step", "step", "set_state", "set_history",
                                 "get_history"]))
            i = int(rng.integers(2))
            t = wk.tanks[i]
            if op == "step":
                k = int(rng.choice([2, 5]))
                ops.append(f"step({k})")
                rc, done = g.step(wk.dt, k, 0.0, check=False)
                assert rc == 0 and np.all(done == k)
                for j, tj in enumerate(wk.tanks):
                    qm1 = hist[j][0] if len(hist[j]) >= 1 else None
                    qm2 = hist[j][1] if len(hist[j]) >= 2 else None
                    qn, it, _, orc = oracle.step(pbs[j], q[j], wk.dt, k, 0.0, qnm1=qm1, qnm2=qm2)
                    assert orc == 0 and it == k
                    hist[j] = ([q[j]] + hist[j])[:2]
                    q[j] = qn
                    err = field_errors(g.get_state(j), q[j], tj.solid, field_scales(tj))
                    assert np.all(err <= TOL), (ops, j, err)
            elif op == "set_state":
                ops.append(f"set_state({i})")
                q[i] = new_state(t)
                g.set_state(i, q[i])
                hist[i] = []
            elif op == "set_history":
                n = int(rng.integers(0, 3))
                ops.append(f"set_history({i}, {n})")
                levels = [near(q[i]) for _ in range(n)]
                g.set_history(i, np.array([lv[:3] for lv in levels]) if n else np.zeros((0, 3)))
                hist[i] = levels
            else:
                ops.append(f"get_history({i})")
                got = g.get_history(i)
                assert len(got) == len(hist[i]), (ops, len(got), len(hist[i]))
                for a, b in zip(got, hist[i]):
                    full = np.concatenate([a, b[3:]])  # p is not part of the levels
                    err = field_errors(full, b, t.solid, field_scales(t))
                    assert np.all(err <= TOL), (ops, err)
        print(f"[history] seed {seed}: {' '.join(ops)}", flush=True)
    finally:
        g.close()


def perturbed_hydrostatic(nx=16, ny=16, seed=0):
    dy = 1.0 / ny
    yc = (np.arange(ny) + 0.5) * dy
    rho = np.where(yc < 0.5, 1000.0, 1.0)
    p = np.zeros(ny)
    for j in range(ny - 1):
        p[j + 1] = p[j] - 9.81 * dy * (rho[j] + rho[j + 1]) / 2
    q = np.zeros((4, ny, nx))
    q[0] = rho[:, None]
    q[3] = p[:, None] + np.random.default_rng(seed).uniform(-5.0, 5.0, (ny, nx))
    return wl.Tank(nx, ny, 1.0, 1.0, q, gy=-9.81, beta=1000.0)


@pytest.mark.parametrize("stages", [1, 2, 4])
@pytest.mark.parametrize("tile", [(0, 0), (32, 8), (-2, 4)])
def test_stage_counts_with_tolerance(stages, tile):
    """Two tanks that converge at different iterations (tolerance 1e-2), in launch groups of
    three pseudo-iterations; one, two and four Runge-Kutta stages (alpha_s = 1/(s_max - s + 1)),
    CFL 0.3 (one stage is forward Euler in pseudo-time)."""
    tanks = [perturbed_hydrostatic(16, 16, seed=1), perturbed_hydrostatic(24, 12, seed=2)]
    if tile == (32, 8):
        tanks = tanks[:1]  # the 2D tiles take one tank
    wk = wl.Workload(f"stages{stages}", tanks, dt=1e-2, steps=1, max_pseudo=1, cfl=0.3,
                     stages=stages, alpha=tuple(1.0 / (stages - s) for s in range(stages)))
    print(f"[stages] s_max={stages} tile={tile} tanks={len(tanks)}", flush=True)
    g_states, g_it, g_norms, g_codes = run_gpu(wk, 2, 4000, tol=1e-2, tile=tile, graph_iters=3)
    o_states, o_it, o_norms, o_codes = run_oracle(wk, 2, 4000, tol=1e-2)
    assert all(c == 0 for c in g_codes) and all(c == 0 for c in o_codes)
    print(f"[stages]   iterations {g_it.tolist()} (oracle {o_it.tolist()})", flush=True)
    assert np.all(g_it < 4000) and np.all(g_it > 3)
    np.testing.assert_array_equal(g_it, o_it)
    for t, a, b in zip(wk.tanks, g_states, o_states):
        err = field_errors(a, b, t.solid, field_scales(t))
        assert np.all(err <= TOL), err
    for a, b in zip(g_norms, o_norms):
        np.testing.assert_allclose(a, b, rtol=1e-7, atol=1e-12)


@pytest.mark.parametrize("seed", [1, 2, 3, 4, 5, 6, 7, 8, 9])
def test_random_loop_controls_against_oracle(seed):
    """Algorithm 1's loop controls in random combinations: iteration cap (0, 1 and more),
    tolerance (none, or one the tanks reach at different iterations), pseudo-iterations per
    replayed graph (eager launches, automatic, 1 .. 8) and kernel shape, on three tanks in one
    batch (seeds 1-6) or one tank in the LDS tiles (7-9), two real steps: every tank's iteration
    counts, states and norms as the oracle's."""
    rng = np.random.default_rng(100 + seed)
    tol = float(rng.choice([0.0, 300.0, 100.0, 30.0, 10.0]))
    cap = int(rng.choice([0, 1, 7, 25, 60, 200]))
    graph_iters = int(rng.choice([-1, 0, 1, 2, 3, 5, 8]))
    if seed <= 6:
        tanks = [perturbed_hydrostatic(16, 16, seed=1), perturbed_hydrostatic(24, 12, seed=2),
                 perturbed_hydrostatic(20, 20, seed=3)]
        tile = [(0, 0), (-2, 4), (-2, 16)][int(rng.integers(3))]
    else:
        tanks = [perturbed_hydrostatic(24, 12, seed=2)]
        tile = [(32, 8), (3208, 2), (1608, 2)][int(rng.integers(3))]
    wk = wl.Workload("loop", tanks, dt=1e-2, steps=1, max_pseudo=1, cfl=0.3)
    print(f"[loop] seed {seed}: cap {cap} tol {tol} graph_iters {graph_iters} tile {tile}",
          flush=True)
    g_states, g_it, g_norms, g_codes = run_gpu(wk, 2, cap, tol=tol, tile=tile, graph_iters=graph_iters)
    o_states, o_it, o_norms, o_codes = run_oracle(wk, 2, cap, tol=tol)
    assert all(c == 0 for c in g_codes) and all(c == 0 for c in o_codes)
    print(f"[loop]   iterations {g_it.tolist()} (oracle {o_it.tolist()})", flush=True)
    np.testing.assert_array_equal(g_it, o_it)
    for t, a, b in zip(wk.tanks, g_states, o_states):
        err = field_errors(a, b, t.solid, field_scales(t))
        assert np.all(err <= TOL), err
    if cap > 0:
        for a, b in zip(g_norms, o_norms):
            np.testing.assert_allclose(a, b, rtol=1e-7, atol=1e-12)


@pytest.mark.parametrize("precision", ["f64", "mixed"])
@pytest.mark.parametrize("tile", [(0, 0), (32, 8)])
def test_new_grid_holds_the_state_at_rest(precision, tile):
    """Before any set_state every tank holds the state at rest (rho = 1, rho u = rho v = p = 0) in
    all its buffers and real-time levels: get_state returns it exactly, and three BDF3 steps from
    it (gravity along both axes, an obstacle, a tank stored reflected in the batch on the
    row-marching kernel) follow the oracle started from that state."""
    wk = moving_tanks()
    wk.bdf = 3
    for t in wk.tanks:
        t.q = np.zeros_like(t.q)
        t.q[0] = 1.0
    grid = vdac.Grid(tank_dicts(wk), gpu_options(wk, precision=precision, tile=tile))
    try:
        for i, t in enumerate(wk.tanks):
            np.testing.assert_array_equal(grid.get_state(i), t.q)
        its = run_steps(grid, wk, 3, 8, 0.0)
        states = [grid.get_state(i) for i in range(len(wk.tanks))]
    finally:
        grid.close()
    o_states, o_its, _, codes = run_oracle(wk, 3, 8)
    assert all(c == 0 for c in codes)
    np.testing.assert_array_equal(its, o_its)
    bar = TOL if precision == "f64" else np.array([1e-6, 1e-5, 1e-5, 1e-4])
    for t, a, b in zip(wk.tanks, states, o_states):
        err = field_errors(a, b, t.solid, field_scales(t))
        print(f"[restart] new grid at rest, {precision} {tile}: {t.nx}x{t.ny} errors {err}", flush=True)
        assert np.all(err <= bar), err
