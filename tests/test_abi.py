"""The C-ABI library loads, exports every entry point its header declares, and rejects bad
arguments before any device work (no GPU needed)."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_2108_08769_amd import vdac

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions(header="vdac.h"):
    text = open(os.path.join(ROOT, "include", header)).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b([a-z_][a-z0-9_]*)\s*\(", text, re.M)
    return sorted(set(n for n in names if n not in ("sizeof",)))


def all_headers():
    return sorted(f for f in os.listdir(os.path.join(ROOT, "include")) if f.endswith(".h"))


def test_header_lists_the_boundary():
    assert set(vdac.EXPORTS) == set(declared_functions())
    assert declared_functions("vdac_probe.h") == ["vdac_march_probe", "vdac_stream_probe"]


@pytest.mark.parametrize("header", all_headers())
def test_library_exports_every_declared_symbol(header):
    lib = vdac.lib()
    names = declared_functions(header)
    assert names
    for name in names:
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", vdac.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    for name in names:
        assert name in exported, name


def test_library_exports_no_other_c_symbols():
    """The unmangled (C-linkage) functions the library exports are exactly those its headers
    declare: no helper leaks into the boundary."""
    out = subprocess.run(["nm", "-D", "--defined-only", vdac.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    c_names = {n for n in exported if not n.startswith("_Z")}
    declared = set()
    for h in all_headers():
        declared |= set(declared_functions(h))
    assert c_names == declared, (sorted(c_names - declared), sorted(declared - c_names))


@pytest.mark.parametrize("n_in,n_out,n,blocks,null", [(2, 1, 10, 0, False), (11, 3, 10, 0, False),
                                                      (1, 1, 0, 0, False), (1, 1, 10, -1, False),
                                                      (1, 1, 10, 0, True)])
def test_stream_probe_rejects_bad_arguments(n_in, n_out, n, blocks, null):
    """Argument checks run before any device call."""
    buf = ctypes.create_string_buffer(64)
    ptr = None if null else ctypes.addressof(buf)
    with pytest.raises(vdac.VdacError) as e:
        vdac.stream_probe(n_in, n_out, n, blocks, ptr or 0, ptr or 0)
    assert e.value.code == vdac.VDAC_E_INVALID


@pytest.mark.parametrize("nx,ny,chunk,null", [(0, 10, 4, False), (10, 0, 4, False), (10, 10, 0, False),
                                               (1 << 15, 1 << 15, 4, False), (10, 10, 4, True)])
def test_march_probe_rejects_bad_arguments(nx, ny, chunk, null):
    """Argument checks run before any device call."""
    buf = ctypes.create_string_buffer(64)
    ptr = None if null else ctypes.addressof(buf)
    with pytest.raises(vdac.VdacError) as e:
        vdac.march_probe(nx, ny, chunk, ptr or 0, ptr or 0)
    assert e.value.code == vdac.VDAC_E_INVALID


def test_default_options():
    o = vdac.default_options()
    assert o.precision == vdac.FP64 and o.rk_stages == 3
    assert list(o.rk_alpha)[:3] == [1.0 / 3.0, 0.5, 1.0]
    assert o.cfl_tau == 0.48 and o.limiter_k == 1.0 and o.local_dtau == 1
    assert o.bdf_order == 1 and o.norm == vdac.NORM_RMS and o.wall_slip == 0


def test_workspace_bytes():
    o = vdac.default_options()
    t, _ = vdac.make_tank(64, 32, 2.0, 1.0)
    n = vdac.workspace_bytes([t], o)
    plane = 64 * 32 * 8
    assert n >= 3 * 4 * plane + 3 * plane + 64 * 32
    t2, _ = vdac.make_tank(16, 16, 1.0, 1.0)
    both = vdac.workspace_bytes([t, t2], o)
    assert n < both <= n + vdac.workspace_bytes([t2], o)
    bad, _ = vdac.make_tank(0, 32, 2.0, 1.0)
    assert vdac.workspace_bytes([bad], o) == 0


def _create(tanks, opt):
    arr = (vdac.Tank * len(tanks))(*tanks)
    h = ctypes.c_void_p()
    rc = vdac.lib().create_grid(arr, len(tanks), ctypes.byref(opt), None, 0, None, ctypes.byref(h))
    return rc, vdac.lib().last_error().decode()


@pytest.mark.parametrize("change,needle", [
    (lambda t, o: setattr(t, "nx", 0), "nx and ny"),
    (lambda t, o: setattr(t, "beta", -1.0), "beta"),
    (lambda t, o: setattr(t, "lx", float("nan")), "lx and ly"),
    (lambda t, o: t.bc.__setitem__(0, 1), "pairs"),
    (lambda t, o: t.bc.__setitem__(2, 7), "bc[2]"),
    (lambda t, o: setattr(o, "rk_stages", 0), "rk_stages"),
    (lambda t, o: o.rk_alpha.__setitem__(2, 0.9), "last Runge-Kutta"),
    (lambda t, o: setattr(o, "cfl_tau", 0.0), "cfl_tau"),
    (lambda t, o: setattr(o, "limiter_k", 3.0), "limiter_k"),
    (lambda t, o: setattr(o, "bdf_order", 4), "bdf_order"),
    (lambda t, o: setattr(o, "norm", 5), "norm"),
    (lambda t, o: setattr(o, "local_dtau", 2), "local"),
    (lambda t, o: setattr(o, "flux", 3), "flux"),
    (lambda t, o: setattr(o, "pgrad", 3), "pgrad"),
    (lambda t, o: setattr(o, "persistent", 2), "persistent"),
    (lambda t, o: (setattr(o, "pgrad", 1), setattr(o, "p_limiter_k", 3.0)), "p_limiter_k"),
    (lambda t, o: (setattr(o, "flux", 1), setattr(o, "tile_x", 1), setattr(o, "tile_y", 1)),
     "one-thread-per-cell"),
    (lambda t, o: (setattr(o, "bdf_order", 3), setattr(o, "tile_x", 1), setattr(o, "tile_y", 1)),
     "one-thread-per-cell"),
    (lambda t, o: (t.bc.__setitem__(3, 2), setattr(o, "tile_x", 1), setattr(o, "tile_y", 1)),
     "one-thread-per-cell"),
    (lambda t, o: (t.bc.__setitem__(0, 2), setattr(o, "pgrad", 2)), "split"),
    (lambda t, o: (setattr(t, "nx", 16385), setattr(t, "ny", 32768)), "2^29"),
])
def test_create_grid_rejects_bad_arguments(change, needle):
    t, _ = vdac.make_tank(8, 8, 1.0, 1.0)
    o = vdac.default_options()
    change(t, o)
    rc, msg = _create([t], o)
    assert rc == vdac.VDAC_E_INVALID
    assert needle in msg


def test_null_handles_are_rejected():
    L = vdac.lib()
    q = (ctypes.c_double * 4)()
    assert L.set_state(None, 0, q) == vdac.VDAC_E_INVALID
    assert L.step_dual_time(None, 1e-3, 1, 0.0, None) == vdac.VDAC_E_INVALID
    assert L.get_state(None, 0, q) == vdac.VDAC_E_INVALID
    assert L.residual_norm(None, 0, q) == vdac.VDAC_E_INVALID
    L.destroy_grid(None)


@pytest.mark.parametrize("offset,short,code,needle", [(0, 1, vdac.VDAC_E_NOMEM, "smaller than"),
                                                      (8, 0, vdac.VDAC_E_INVALID, "aligned")])
def test_create_grid_checks_a_borrowed_workspace(offset, short, code, needle):
    """A caller's workspace that is smaller than workspace_bytes, or not 256-byte aligned, is
    rejected before any device call (the pointer is never dereferenced)."""
    o = vdac.default_options()
    t, _ = vdac.make_tank(40, 24, 2.0, 1.0)
    need = vdac.workspace_bytes([t], o)
    arr = (vdac.Tank * 1)(t)
    h = ctypes.c_void_p()
    fake = 0x10000000 + offset  # never touched
    rc = vdac.lib().create_grid(arr, 1, ctypes.byref(o), ctypes.c_void_p(fake), need - short, None,
                                ctypes.byref(h))
    assert rc == code and needle in vdac.lib().last_error().decode()
    assert not h.value


def test_workspace_at_the_tank_size_limit():
    """2^29 cells is the largest tank (the row-marching kernel's 32-bit plane offsets): the
    workspace of one is sized, one more row is refused."""
    o = vdac.default_options()
    t, _ = vdac.make_tank(16384, 32768, 4.0, 8.0)
    assert vdac.workspace_bytes([t], o) > 4 * 8 * (1 << 29)
    t, _ = vdac.make_tank(16384, 32769, 4.0, 8.0)
    assert vdac.workspace_bytes([t], o) == 0


# ---- argument validation as a property: workspace_bytes and create_grid agree ----------------

from hypothesis import HealthCheck, event, given, settings, strategies as st  # noqa: E402

_TANK_OK = {
    "nx": st.integers(1, 40), "ny": st.integers(1, 40), "lx": st.floats(0.1, 5.0),
    "ly": st.floats(0.1, 5.0), "gx": st.floats(-10.0, 10.0), "gy": st.floats(-10.0, 10.0),
    "beta": st.floats(1.0, 2000.0),
    "bc": st.sampled_from([(0, 0, 0, 0), (1, 1, 0, 0), (0, 0, 1, 1), (2, 0, 0, 2), (1, 1, 2, 2),
                           (0, 2, 1, 1)]),
}
_TANK_BAD = {
    "nx": st.sampled_from([-1, 0, 16385]), "ny": st.sampled_from([-1, 0, 32769]),
    "lx": st.sampled_from([0.0, -1.0, float("nan"), float("inf")]),
    "ly": st.sampled_from([0.0, -1.0, float("nan"), float("inf")]),
    "gx": st.sampled_from([float("nan"), float("inf")]),
    "gy": st.sampled_from([float("nan"), float("-inf")]),
    "beta": st.sampled_from([0.0, -5.0, float("nan"), float("inf")]),
    "bc": st.sampled_from([(1, 0, 0, 0), (0, 0, 0, 1), (3, 0, 0, 0), (0, -1, 0, 0)]),
}
_OPT_OK = {
    "precision": st.integers(0, 1), "rk_stages": st.integers(1, 8), "last_alpha": st.just(1.0),
    "cfl_tau": st.floats(0.1, 1.0), "limiter_k": st.floats(1.0, 2.0), "local_dtau": st.integers(0, 1),
    "bdf_order": st.integers(1, 3), "norm": st.integers(0, 1), "wall_slip": st.integers(0, 1),
    "graph_iters": st.integers(-1, 20),
    "tile": st.sampled_from([(0, 0), (1, 1), (32, 8), (16, 16), (64, 4), (3208, 2), (1616, 2),
                             (1608, 2), (-2, 16), (-3, 5), (-1, 1)]),
    "flux": st.integers(0, 2), "pgrad": st.integers(0, 2), "p_limiter_k": st.floats(1.0, 2.0),
    "persistent": st.integers(0, 1),
}
_OPT_BAD = {
    "precision": st.sampled_from([-1, 2]), "rk_stages": st.sampled_from([0, 9]),
    "last_alpha": st.just(0.9), "cfl_tau": st.sampled_from([0.0, -1.0, float("nan")]),
    "limiter_k": st.sampled_from([0.5, 2.5]), "local_dtau": st.just(2),
    "bdf_order": st.sampled_from([0, 4]), "norm": st.just(2), "wall_slip": st.just(2),
    "graph_iters": st.sampled_from([-2, 1001]),
    "tile": st.sampled_from([(-4, 8), (32, 9), (0, 5), (-2, 0)]),
    "flux": st.sampled_from([-1, 3]), "pgrad": st.sampled_from([-1, 3]),
    "p_limiter_k": st.sampled_from([0.5, 2.5]), "persistent": st.sampled_from([-1, 2]),
}


@st.composite
def _arguments(draw):
    """A valid set of tanks and options, and in half of the draws one field made invalid."""
    tanks = [draw(st.fixed_dictionaries(_TANK_OK)) for _ in range(draw(st.integers(1, 3)))]
    opt = draw(st.fixed_dictionaries(_OPT_OK))
    if draw(st.booleans()):
        if draw(st.booleans()):
            t = draw(st.sampled_from(tanks))
            key = draw(st.sampled_from(sorted(_TANK_BAD)))
            t[key] = draw(_TANK_BAD[key])
        else:
            key = draw(st.sampled_from(sorted(_OPT_BAD)))
            opt[key] = draw(_OPT_BAD[key])
    return tanks, opt


@settings(max_examples=400, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(args=_arguments())
def test_workspace_bytes_and_create_grid_agree(args):
    """workspace_bytes returns 0 exactly for the arguments create_grid rejects as invalid, and
    neither crashes on any of them; valid arguments get past validation (on a machine without a
    GPU create_grid then fails at its first allocation)."""
    tanks, opt = args
    structs = [vdac.make_tank(t["nx"], t["ny"], t["lx"], t["ly"], t["gx"], t["gy"], t["beta"],
                              t["bc"])[0] for t in tanks]
    o = vdac.default_options()
    o.precision, o.rk_stages = opt["precision"], opt["rk_stages"]
    for i in range(8):
        o.rk_alpha[i] = 0.5 if i < opt["rk_stages"] - 1 else (opt["last_alpha"] if i < opt["rk_stages"] else 0.0)
    o.cfl_tau, o.limiter_k, o.local_dtau = opt["cfl_tau"], opt["limiter_k"], opt["local_dtau"]
    o.bdf_order, o.norm, o.wall_slip = opt["bdf_order"], opt["norm"], opt["wall_slip"]
    o.graph_iters, o.tile_x, o.tile_y = opt["graph_iters"], opt["tile"][0], opt["tile"][1]
    o.flux, o.pgrad, o.p_limiter_k = opt["flux"], opt["pgrad"], opt["p_limiter_k"]
    o.persistent = opt["persistent"]
    ws = vdac.workspace_bytes(structs, o)
    arr = (vdac.Tank * len(structs))(*structs)
    h = ctypes.c_void_p()
    rc = vdac.lib().create_grid(arr, len(structs), ctypes.byref(o), None, 0, None, ctypes.byref(h))
    if rc == vdac.VDAC_OK:
        vdac.lib().destroy_grid(h)
    event("valid" if ws else "invalid")
    if ws == 0:
        assert rc == vdac.VDAC_E_INVALID, (rc, vdac.lib().last_error())
    else:
        assert rc in (vdac.VDAC_OK, vdac.VDAC_E_NOMEM, vdac.VDAC_E_DEVICE), (rc, vdac.lib().last_error())
