"""Python access to the plain serial FP64 oracle (``vdac_oracle.c``).

TEST INFRASTRUCTURE ONLY.  Imported by ``tests/``, by ``__graft_entry__.smoke()`` and by the
CPU-baseline leg of ``bench.py``; never by the product package.  It shares no code with the GPU
library: it has its own C source, its own header and this ctypes wrapper.

Arrays at this interface are float64 numpy arrays ``[4, ny, nx]`` holding (rho, rho*u, rho*v, p)
with the pressure itself.  Single-point helpers take the internal conserved vector
Q = (rho, rho*u, rho*v, p/beta) of the paper's compact form (Sec. 2.1.2).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vdac_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_LIB_OMP = os.path.join(_HERE, "liboracle_omp.so")

BC_WALL = 0
BC_PERIODIC = 1
BC_TRANSMISSIVE = 2
FLUX_OSHER, FLUX_ROE, FLUX_BASSI = 0, 1, 2
PGRAD_NEW, PGRAD_LIMITER, PGRAD_SPLIT = 0, 1, 2


def build() -> str:
    """Compile the oracle (plain C99, -O2, no contraction, no fast-math), serial, and the same
    source with -fopenmp (its row loops on all host threads; used only to time the oracle)."""
    for lib_path, extra in ((_LIB, []), (_LIB_OMP, ["-fopenmp"])):
        tmp = lib_path + ".tmp"
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99", "-Wall", *extra,
               "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, lib_path)
    return _LIB


class _Problem(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int),
        ("lx", ctypes.c_double), ("ly", ctypes.c_double),
        ("gx", ctypes.c_double), ("gy", ctypes.c_double),
        ("beta", ctypes.c_double),
        ("bc", ctypes.c_int * 4),
        ("solid", ctypes.POINTER(ctypes.c_ubyte)),
        ("stages", ctypes.c_int),
        ("alpha", ctypes.c_double * 8),
        ("cfl", ctypes.c_double),
        ("k", ctypes.c_double),
        ("local_dtau", ctypes.c_int),
        ("bdf", ctypes.c_int),
        ("wall_slip", ctypes.c_int),
        ("flux", ctypes.c_int),
        ("pgrad", ctypes.c_int),
        ("pk", ctypes.c_double),
    ]


class _Detail(ctypes.Structure):
    _fields_ = [(name, ctypes.POINTER(ctypes.c_double))
                for name in ("prim", "grad", "fx", "fy", "resid", "dtau")]


_libs = {}


def lib(omp: bool = False):
    """The serial oracle, or (omp=True) the same source built with -fopenmp."""
    path = _LIB_OMP if omp else _LIB
    if path not in _libs:
        if not os.path.exists(path):
            build()
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        L.orc_limiter.restype = ctypes.c_double
        L.orc_limiter.argtypes = [ctypes.c_double] * 3
        for name in ("orc_flux_phys",):
            getattr(L, name).argtypes = [dp, ctypes.c_double, dp]
        L.orc_eigen.argtypes = [dp, ctypes.c_double, dp, dp, dp]
        L.orc_abs_jacobian.argtypes = [dp, ctypes.c_double, dp]
        L.orc_osher_x.argtypes = [dp, dp, ctypes.c_double, dp]
        L.orc_roe_x.argtypes = [dp, dp, ctypes.c_double, dp]
        L.orc_bassi_x.argtypes = [dp, dp, ctypes.c_double, dp]
        L.orc_bassi_star.argtypes = [dp, dp, ctypes.c_double, dp]
        L.orc_exact_sample.argtypes = [dp, dp, ctypes.c_double, ctypes.c_double, dp]
        L.orc_face_flux.argtypes = [dp, dp, ctypes.c_double, ctypes.c_double, ctypes.c_double, dp]
        L.orc_face_flux_kind.argtypes = [dp, dp, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_int, dp]
        L.orc_realtime_dt.restype = ctypes.c_double
        L.orc_realtime_dt.argtypes = [ctypes.POINTER(_Problem), dp, ctypes.c_double]
        L.orc_stage.restype = ctypes.c_int
        L.orc_stage.argtypes = [ctypes.POINTER(_Problem), dp, dp, dp, dp, dp, ctypes.c_double,
                                ctypes.c_int, dp, ctypes.POINTER(_Detail)]
        L.orc_step.restype = ctypes.c_int
        L.orc_step.argtypes = [ctypes.POINTER(_Problem), dp, dp, dp, ctypes.c_double, ctypes.c_int,
                               ctypes.c_double, ctypes.c_int, ctypes.POINTER(ctypes.c_int), dp]
        L.orc_threads.restype = ctypes.c_int
        L.orc_threads.argtypes = []
        _libs[path] = L
    return _libs[path]


def threads(omp: bool = False) -> int:
    """Host threads the oracle's row loops run on (1 for the serial build)."""
    return int(lib(omp).orc_threads())


def _ptr(a: np.ndarray | None):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


@dataclass
class Problem:
    """Grid, physics and pseudo-time settings of one tank."""
    nx: int
    ny: int
    lx: float
    ly: float
    gx: float = 0.0
    gy: float = -9.81
    beta: float = 1000.0
    bc: tuple = (BC_WALL, BC_WALL, BC_WALL, BC_WALL)
    solid: np.ndarray | None = None
    stages: int = 3
    alpha: tuple = (1.0 / 3.0, 0.5, 1.0)
    cfl: float = 0.48
    k: float = 1.0
    local_dtau: bool = True
    bdf: int = 1
    wall_slip: bool = False
    flux: int = FLUX_OSHER
    pgrad: int = PGRAD_NEW
    pk: float = 1.0
    _keep: list = field(default_factory=list, repr=False)

    def c_struct(self) -> _Problem:
        p = _Problem()
        p.nx, p.ny, p.lx, p.ly = self.nx, self.ny, self.lx, self.ly
        p.gx, p.gy, p.beta = self.gx, self.gy, self.beta
        for i in range(4):
            p.bc[i] = int(self.bc[i])
        if self.solid is not None:
            s = np.ascontiguousarray(self.solid, dtype=np.uint8)
            assert s.shape == (self.ny, self.nx)
            self._keep = [s]
            p.solid = s.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte))
        p.stages = self.stages
        for i, a in enumerate(self.alpha):
            p.alpha[i] = a
        p.cfl, p.k = self.cfl, self.k
        p.local_dtau = int(bool(self.local_dtau))
        p.bdf = self.bdf
        p.wall_slip = int(bool(self.wall_slip))
        p.flux, p.pgrad, p.pk = int(self.flux), int(self.pgrad), float(self.pk)
        return p


def limiter(a: float, b: float, k: float) -> float:
    return lib().orc_limiter(a, b, k)


def flux_phys(q, beta):
    q = np.ascontiguousarray(q, dtype=np.float64)
    f = np.zeros(4)
    lib().orc_flux_phys(_ptr(q), beta, _ptr(f))
    return f


def eigen(q, beta):
    q = np.ascontiguousarray(q, dtype=np.float64)
    R, L, lam = np.zeros(16), np.zeros(16), np.zeros(4)
    lib().orc_eigen(_ptr(q), beta, _ptr(R), _ptr(L), _ptr(lam))
    return R.reshape(4, 4), L.reshape(4, 4), lam


def abs_jacobian(q, beta):
    q = np.ascontiguousarray(q, dtype=np.float64)
    A = np.zeros(16)
    lib().orc_abs_jacobian(_ptr(q), beta, _ptr(A))
    return A.reshape(4, 4)


def osher_x(ql, qr, beta):
    ql = np.ascontiguousarray(ql, dtype=np.float64)
    qr = np.ascontiguousarray(qr, dtype=np.float64)
    f = np.zeros(4)
    lib().orc_osher_x(_ptr(ql), _ptr(qr), beta, _ptr(f))
    return f


def _flux2(name, ql, qr, beta):
    ql = np.ascontiguousarray(ql, dtype=np.float64)
    qr = np.ascontiguousarray(qr, dtype=np.float64)
    f = np.zeros(4)
    getattr(lib(), name)(_ptr(ql), _ptr(qr), beta, _ptr(f))
    return f


def roe_x(ql, qr, beta):
    return _flux2("orc_roe_x", ql, qr, beta)


def bassi_x(ql, qr, beta):
    return _flux2("orc_bassi_x", ql, qr, beta)


def bassi_star(ql, qr, beta):
    """(S_L, S_R, u*, p*, rho*L, rho*R) of the exact Riemann solution."""
    ql = np.ascontiguousarray(ql, dtype=np.float64)
    qr = np.ascontiguousarray(qr, dtype=np.float64)
    st = np.zeros(6)
    lib().orc_bassi_star(_ptr(ql), _ptr(qr), beta, _ptr(st))
    return st


def exact_sample(ql, qr, beta, xi):
    ql = np.ascontiguousarray(ql, dtype=np.float64)
    qr = np.ascontiguousarray(qr, dtype=np.float64)
    q = np.zeros(4)
    lib().orc_exact_sample(_ptr(ql), _ptr(qr), beta, float(xi), _ptr(q))
    return q


def face_flux(qa, qb, normal, beta, kind=FLUX_OSHER):
    qa = np.ascontiguousarray(qa, dtype=np.float64)
    qb = np.ascontiguousarray(qb, dtype=np.float64)
    f = np.zeros(4)
    lib().orc_face_flux_kind(_ptr(qa), _ptr(qb), float(normal[0]), float(normal[1]), beta,
                             int(kind), _ptr(f))
    return f


def realtime_dt(pb: Problem, q, cfl_t: float) -> float:
    q = np.ascontiguousarray(q, dtype=np.float64)
    st = pb.c_struct()
    return lib().orc_realtime_dt(ctypes.byref(st), _ptr(q), float(cfl_t))


def stage(pb: Problem, qprev, q0, qn, dt, s, qnm1=None, qnm2=None):
    """One Runge-Kutta stage; returns (q_out, detail dict)."""
    ny, nx = pb.ny, pb.nx
    arrs = [np.ascontiguousarray(a, dtype=np.float64) if a is not None else None
            for a in (qprev, q0, qn, qnm1, qnm2)]
    out = np.zeros((4, ny, nx))
    det = {"prim": np.zeros((4, ny, nx)), "grad": np.zeros((8, ny, nx)),
           "fx": np.zeros((4, ny, nx + 1)), "fy": np.zeros((4, ny + 1, nx)),
           "resid": np.zeros((4, ny, nx)), "dtau": np.zeros((ny, nx))}
    d = _Detail(*[_ptr(det[k]) for k in ("prim", "grad", "fx", "fy", "resid", "dtau")])
    st = pb.c_struct()
    rc = lib().orc_stage(ctypes.byref(st), _ptr(arrs[0]), _ptr(arrs[1]), _ptr(arrs[2]),
                         _ptr(arrs[3]), _ptr(arrs[4]), dt, s, _ptr(out), ctypes.byref(d))
    if rc != 0:
        raise ValueError(f"orc_stage returned {rc}")
    return out, det


def step(pb: Problem, q, dt, max_pseudo, tol=0.0, norm=0, qnm1=None, qnm2=None, omp=False):
    """One real-time step.  Returns (q_new, iterations, norms[4], status).  omp=True runs the
    -fopenmp build of the same source (same results; for timing on all host threads)."""
    q = np.array(q, dtype=np.float64, order="C", copy=True)
    assert q.shape == (4, pb.ny, pb.nx)
    qm = None if qnm1 is None else np.ascontiguousarray(qnm1, dtype=np.float64)
    qm2 = None if qnm2 is None else np.ascontiguousarray(qnm2, dtype=np.float64)
    it = ctypes.c_int(0)
    res = np.zeros(4)
    st = pb.c_struct()
    rc = lib(omp).orc_step(ctypes.byref(st), _ptr(q), _ptr(qm), _ptr(qm2), dt, int(max_pseudo),
                           float(tol), int(norm), ctypes.byref(it), _ptr(res))
    if rc == -1:
        raise ValueError("orc_step: invalid arguments")
    return q, it.value, res, rc
