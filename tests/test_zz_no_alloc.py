"""The allocation-free entry point realtime_dt_device (for callers that cannot allocate) against
realtime_dt, through the C ABI: two calls in a row, the second on a smaller input, each equal to
realtime_dt bit for bit (a minimum is exact whatever the order of its terms); a range too large
for the fixed scratch array is rejected before any device work."""
import numpy as np
import pytest

from paper_2108_08769_amd import vdac
from paper_2108_08769_amd import workloads as wl

pytestmark = pytest.mark.gpu


def moving_grid(shapes, precision, seed):
    tanks, states = [], []
    for i, (nx, ny) in enumerate(shapes):
        q = wl.random_state(nx, ny, seed=seed + i, rho_range=(1.0, 5.0), vel=0.5, p_scale=10.0)
        solid = None
        if nx > 40 and ny > 10:
            solid = np.zeros((ny, nx), np.uint8)
            solid[ny // 3:ny // 3 + 3, nx // 2:nx // 2 + 4] = 1
        tanks.append(dict(nx=nx, ny=ny, lx=0.05 * nx, ly=0.04 * ny, gx=0.3, gy=-9.81, beta=500.0,
                          solid=solid))
        states.append(q)
    g = vdac.Grid(tanks, vdac.make_options(precision=precision))
    for i, q in enumerate(states):
        g.set_state(i, q)
    return g


def compare(g, first, n, cfl):
    import torch
    out = torch.full((n,), -1.0, dtype=torch.float64, device="cuda")
    g.realtime_dt_device(first, n, cfl, out.data_ptr())
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    ref = np.array([g.realtime_dt(first + k, cfl) for k in range(n)])
    print(f"[no-alloc] tanks {first}..{first + n - 1}: {got.tolist()}", flush=True)
    np.testing.assert_array_equal(got, ref)
    assert np.all(np.isfinite(got)) and np.all(got > 0)


def test_realtime_dt_device_equals_realtime_dt():
    # first call: three tanks (an obstacle, a tall tank stored reflected, a large one), FP64,
    # after two real steps
    g = moving_grid([(70, 23), (19, 66), (300, 200)], "f64", seed=11)
    try:
        for _ in range(2):
            g.step(2e-3, 6, 0.0)
        compare(g, 0, 3, 0.45)
        # second call: a smaller input (one small tank of the same grid)
        compare(g, 1, 1, 0.3)
    finally:
        g.close()
    # a different, smaller grid in the mixed form: the shared scratch keeps the last call's
    # minima, which must not leak into this one
    g = moving_grid([(17, 9)], "mixed", seed=12)
    try:
        g.step(2e-3, 4, 0.0)
        compare(g, 0, 1, 0.45)
    finally:
        g.close()


def test_realtime_dt_device_rejects_bad_ranges():
    import torch
    out = torch.zeros(40, dtype=torch.float64, device="cuda")
    g = moving_grid([(256, 256)] * 33, "f64", seed=13)  # 33 x 256 minima > 8192
    try:
        with pytest.raises(vdac.VdacError) as e:
            g.realtime_dt_device(0, 33, 0.45, out.data_ptr())
        assert e.value.code == vdac.VDAC_E_INVALID and "split the range" in str(e.value)
        g.realtime_dt_device(0, 32, 0.45, out.data_ptr())  # 32 x 256 fits
        torch.cuda.synchronize()
        for bad in [(-1, 1), (30, 4), (0, 0)]:
            with pytest.raises(vdac.VdacError):
                g.realtime_dt_device(bad[0], bad[1], 0.45, out.data_ptr())
        with pytest.raises(vdac.VdacError):
            g.realtime_dt_device(0, 1, 0.45, 0)
    finally:
        g.close()
