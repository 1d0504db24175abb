"""Thin Python binding of libvdac's C ABI (include/vdac.h).

Argument marshalling only: every step of the solver runs in the HIP library.  PyTorch provides
the device workspace (a uint8 tensor) and the stream (torch's current stream); nothing here
computes.  The binding refuses to run if the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libvdac.so")

VDAC_OK, VDAC_E_INVALID, VDAC_E_NOMEM, VDAC_E_DEVICE, VDAC_E_DIVERGED = range(5)
BC_WALL, BC_PERIODIC, BC_TRANSMISSIVE = 0, 1, 2
FLUX_OSHER, FLUX_ROE, FLUX_BASSI = 0, 1, 2
PGRAD_NEW, PGRAD_LIMITER, PGRAD_SPLIT = 0, 1, 2
FP64, FP32_MIXED = 0, 1
NORM_RMS, NORM_MAX = 0, 1

EXPORTS = ("vdac_default_options", "workspace_bytes", "create_grid", "set_state",
           "step_dual_time", "residual_norm", "get_state", "get_history", "set_history",
           "stage_timing", "stage_timing_read", "autotune_tile", "realtime_dt",
           "realtime_dt_device", "destroy_grid", "last_error")


class VdacError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"vdac error {code}: {message}")
        self.code = code


class Tank(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("lx", ctypes.c_double), ("ly", ctypes.c_double),
        ("gx", ctypes.c_double), ("gy", ctypes.c_double),
        ("beta", ctypes.c_double),
        ("bc", ctypes.c_int32 * 4),
        ("solid", ctypes.POINTER(ctypes.c_uint8)),
    ]


class Options(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int32),
        ("rk_stages", ctypes.c_int32),
        ("rk_alpha", ctypes.c_double * 8),
        ("cfl_tau", ctypes.c_double),
        ("limiter_k", ctypes.c_double),
        ("local_dtau", ctypes.c_int32),
        ("bdf_order", ctypes.c_int32),
        ("norm", ctypes.c_int32),
        ("wall_slip", ctypes.c_int32),
        ("tile_x", ctypes.c_int32),
        ("tile_y", ctypes.c_int32),
        ("graph_iters", ctypes.c_int32),
        ("flux", ctypes.c_int32),
        ("pgrad", ctypes.c_int32),
        ("p_limiter_k", ctypes.c_double),
        ("persistent", ctypes.c_int32),
    ]


_lib = None


def lib():
    """Load libvdac.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        # PyTorch ships its own HIP runtime (soname libamdhip64.so.7).  Loading torch first lets
        # the dynamic loader resolve libvdac's libamdhip64.so.7 to that same runtime; loading
        # libvdac first would put a second HIP runtime into the process, and the one torch does
        # not own then sees no device.
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2108_08769_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        vp = ctypes.c_void_p
        L.vdac_default_options.argtypes = [ctypes.POINTER(Options)]
        L.vdac_default_options.restype = None
        L.workspace_bytes.argtypes = [ctypes.POINTER(Tank), ctypes.c_int32, ctypes.POINTER(Options)]
        L.workspace_bytes.restype = ctypes.c_size_t
        L.create_grid.argtypes = [ctypes.POINTER(Tank), ctypes.c_int32, ctypes.POINTER(Options), vp,
                                  ctypes.c_size_t, vp, ctypes.POINTER(vp)]
        L.create_grid.restype = ctypes.c_int
        L.set_state.argtypes = [vp, ctypes.c_int32, dp]
        L.set_state.restype = ctypes.c_int
        L.step_dual_time.argtypes = [vp, ctypes.c_double, ctypes.c_int32, ctypes.c_double,
                                     ctypes.POINTER(ctypes.c_int32)]
        L.step_dual_time.restype = ctypes.c_int
        L.residual_norm.argtypes = [vp, ctypes.c_int32, dp]
        L.residual_norm.restype = ctypes.c_int
        L.get_state.argtypes = [vp, ctypes.c_int32, dp]
        L.get_state.restype = ctypes.c_int
        L.get_history.argtypes = [vp, ctypes.c_int32, dp, ctypes.POINTER(ctypes.c_int32)]
        L.get_history.restype = ctypes.c_int
        L.set_history.argtypes = [vp, ctypes.c_int32, dp, ctypes.c_int32]
        L.set_history.restype = ctypes.c_int
        L.stage_timing.argtypes = [vp, ctypes.c_int32]
        L.stage_timing.restype = ctypes.c_int
        L.stage_timing_read.argtypes = [vp, dp, ctypes.POINTER(ctypes.c_int64), dp]
        L.stage_timing_read.restype = ctypes.c_int
        L.autotune_tile.argtypes = [ctypes.POINTER(Tank), ctypes.c_int32, ctypes.POINTER(Options),
                                    vp, ctypes.c_int32]
        L.autotune_tile.restype = ctypes.c_int
        L.realtime_dt.argtypes = [vp, ctypes.c_int32, ctypes.c_double, dp]
        L.realtime_dt.restype = ctypes.c_int
        L.realtime_dt_device.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_double, vp]
        L.realtime_dt_device.restype = ctypes.c_int
        L.destroy_grid.argtypes = [vp]
        L.destroy_grid.restype = None
        L.last_error.argtypes = []
        L.last_error.restype = ctypes.c_char_p
        L.vdac_stream_probe.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64,
                                        ctypes.c_int32, vp, vp, vp]
        L.vdac_stream_probe.restype = ctypes.c_int
        L.vdac_march_probe.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp, vp, vp]
        L.vdac_march_probe.restype = ctypes.c_int
        _lib = L
    return _lib


def _check(rc: int):
    if rc != VDAC_OK:
        raise VdacError(rc, lib().last_error().decode())


def stream_probe(n_in: int, n_out: int, n: int, blocks: int, in_ptr: int, out_ptr: int,
                 stream: int = 0):
    """One pass of the plane-stream bandwidth reference (include/vdac_probe.h) on `stream`."""
    _check(lib().vdac_stream_probe(n_in, n_out, n, blocks, in_ptr, out_ptr, stream or None))


def march_probe(nx: int, ny: int, chunk: int, in_ptr: int, out_ptr: int, stream: int = 0):
    """One pass of the row-marching bandwidth reference (include/vdac_probe.h) on `stream`."""
    rc = lib().vdac_march_probe(nx, ny, chunk, in_ptr, out_ptr, stream or None)
    if rc != VDAC_OK:
        raise VdacError(rc, "march probe: bad size or pointer, or the launch failed")


def default_options() -> Options:
    o = Options()
    lib().vdac_default_options(ctypes.byref(o))
    return o


def make_options(precision="f64", stages=3, alpha=(1.0 / 3.0, 0.5, 1.0), cfl=0.48, k=1.0,
                 bdf=1, norm=NORM_RMS, wall_slip=False, tile=(0, 0), graph_iters=0, flux=0,
                 pgrad=0, pk=1.0, local_dtau=True, persistent=False) -> Options:
    o = default_options()
    o.precision = {"f64": FP64, "mixed": FP32_MIXED}[precision] if isinstance(precision, str) \
        else int(precision)
    o.rk_stages = int(stages)
    for i in range(8):
        o.rk_alpha[i] = float(alpha[i]) if i < len(alpha) else 0.0
    o.cfl_tau = float(cfl)
    o.limiter_k = float(k)
    o.bdf_order = int(bdf)
    o.norm = int(norm)
    o.wall_slip = int(bool(wall_slip))
    o.tile_x, o.tile_y = int(tile[0]), int(tile[1])
    o.graph_iters = int(graph_iters)
    o.flux, o.pgrad, o.p_limiter_k = int(flux), int(pgrad), float(pk)
    o.local_dtau = int(bool(local_dtau))
    o.persistent = int(bool(persistent))
    return o


def make_tank(nx, ny, lx, ly, gx=0.0, gy=-9.81, beta=1000.0, bc=(0, 0, 0, 0), solid=None):
    t = Tank()
    t.nx, t.ny, t.lx, t.ly = int(nx), int(ny), float(lx), float(ly)
    t.gx, t.gy, t.beta = float(gx), float(gy), float(beta)
    for i in range(4):
        t.bc[i] = int(bc[i])
    keep = None
    if solid is not None:
        keep = np.ascontiguousarray(solid, dtype=np.uint8)
        assert keep.shape == (ny, nx)
        t.solid = keep.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    return t, keep


def workspace_bytes(tanks, options: Options | None = None) -> int:
    arr = (Tank * len(tanks))(*tanks)
    return int(lib().workspace_bytes(arr, len(tanks), ctypes.byref(options) if options else None))


def autotune(tanks, options: Options, iters: int = 5, device="cuda", stream=None) -> Options:
    """Runs the library's tile autotuner for these tanks and options and returns a copy of the
    options with the fastest stage-kernel shape filled in."""
    import torch  # stream only
    structs, keep = [], []
    for t in tanks:
        if isinstance(t, Tank):
            structs.append(t)
        else:
            s, k = make_tank(**t)
            structs.append(s)
            keep.append(k)
    arr = (Tank * len(structs))(*structs)
    out = Options()
    ctypes.pointer(out)[0] = options
    st = stream if stream is not None else torch.cuda.current_stream(device)
    _check(lib().autotune_tile(arr, len(structs), ctypes.byref(out), ctypes.c_void_p(st.cuda_stream),
                               int(iters)))
    return out


class Grid:
    """A set of independent tanks on the GPU (one create_grid)."""

    def __init__(self, tanks, options: Options | None = None, device="cuda", stream=None,
                 own_workspace=False):
        import torch  # device memory and stream only
        self._lib = lib()
        self.n_tanks = len(tanks)
        self._shapes = []
        structs, self._keep = [], []
        for t in tanks:
            if isinstance(t, Tank):
                structs.append(t)
                self._shapes.append((t.ny, t.nx))
            else:
                s, keep = make_tank(**t)
                structs.append(s)
                self._keep.append(keep)
                self._shapes.append((s.ny, s.nx))
        arr = (Tank * len(structs))(*structs)
        opt = options if options is not None else default_options()
        self.options = opt
        need = int(self._lib.workspace_bytes(arr, len(structs), ctypes.byref(opt)))
        if need == 0:
            # let create_grid report the reason
            ws_ptr, need = None, 0
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        if own_workspace or need == 0:
            self.workspace = None
            ws_ptr = None
        else:
            self.workspace = torch.empty(need + 256, dtype=torch.uint8, device=device)
            base = self.workspace.data_ptr()
            ws_ptr = (base + 255) & ~255
        handle = ctypes.c_void_p()
        rc = self._lib.create_grid(arr, len(structs), ctypes.byref(opt), ws_ptr,
                                   ctypes.c_size_t(need), ctypes.c_void_p(self.stream.cuda_stream),
                                   ctypes.byref(handle))
        _check(rc)
        self._h = handle

    def close(self):
        if getattr(self, "_h", None):
            self._lib.destroy_grid(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_state(self, tank: int, q: np.ndarray):
        ny, nx = self._shapes[tank]
        q = np.ascontiguousarray(q, dtype=np.float64)
        assert q.shape == (4, ny, nx)
        _check(self._lib.set_state(self._h, tank, q.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))

    def step(self, dt: float, max_pseudo: int, tol: float = 0.0, check: bool = True):
        done = (ctypes.c_int32 * self.n_tanks)()
        rc = self._lib.step_dual_time(self._h, float(dt), int(max_pseudo), float(tol), done)
        if check:
            _check(rc)
        return rc, np.array(done[:], dtype=np.int64)

    def residual_norm(self, tank: int = 0) -> np.ndarray:
        out = np.zeros(4)
        _check(self._lib.residual_norm(self._h, tank, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out

    def stage_timing(self, enable: bool = True):
        _check(self._lib.stage_timing(self._h, int(bool(enable))))

    def stage_timing_read(self):
        """(summed stage-kernel ms, stage launches, fluid cell-stages) since timing was enabled."""
        ms, n, cs = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
        _check(self._lib.stage_timing_read(self._h, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(cs)))
        return ms.value, n.value, cs.value

    def realtime_dt(self, tank: int = 0, cfl_t: float = 0.45) -> float:
        """Global real-time step of one tank from its current state (Sec. 2.2.4)."""
        dt = ctypes.c_double()
        _check(self._lib.realtime_dt(self._h, tank, float(cfl_t), ctypes.byref(dt)))
        return dt.value

    def realtime_dt_device(self, first_tank: int, n_tanks: int, cfl_t: float, out_ptr: int):
        """Queues the global real-time steps of n_tanks tanks into the device array at out_ptr
        (n_tanks doubles) on the grid's stream; allocates nothing and does not wait."""
        _check(self._lib.realtime_dt_device(self._h, int(first_tank), int(n_tanks), float(cfl_t),
                                            ctypes.c_void_p(out_ptr)))

    def get_state(self, tank: int = 0) -> np.ndarray:
        ny, nx = self._shapes[tank]
        q = np.zeros((4, ny, nx))
        _check(self._lib.get_state(self._h, tank, q.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return q

    def get_history(self, tank: int = 0) -> np.ndarray:
        """The earlier real-time levels [count, 3, ny, nx] (rho, rho u, rho v) the next step would
        use (Table 1), newest first."""
        ny, nx = self._shapes[tank]
        lv = np.zeros((2, 3, ny, nx))
        n = ctypes.c_int32()
        _check(self._lib.get_history(self._h, tank, lv.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                     ctypes.byref(n)))
        return lv[:n.value].copy()

    def set_history(self, tank: int, levels: np.ndarray):
        """Restores earlier real-time levels [count, 3, ny, nx] after set_state."""
        ny, nx = self._shapes[tank]
        lv = np.zeros((2, 3, ny, nx))
        n = int(len(levels))
        if n:
            lv[:n] = np.asarray(levels, dtype=np.float64)
        _check(self._lib.set_history(self._h, tank, lv.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                     n))
