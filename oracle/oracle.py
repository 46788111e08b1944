"""Python binding of the FP64 CPU oracle (oracle/biot_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg.  The product path never imports this module.

Populations are exchanged as component planes: f is (9, ny, nx), g is (8, ny, nx)
(D2Q9 order of Table 1; D2Q8 order 10, 01, -10, 0-1, 11, -11, -1-1, 1-1).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

from paper_2409_11382_amd.problem import Problem

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "biot_oracle.c")
_LIB = os.path.join(_HERE, "libbiot_oracle.so")

OR_OK, OR_ERR_ARG, OR_ERR_DIVERGED, OR_ERR_STATE = 0, -1, -4, -6


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, OpenMP over rows)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-Wall", "-Wno-unused-variable", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Problem(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("dx", C.c_double), ("dt", C.c_double),
                ("lambda_", C.c_double), ("mu", C.c_double), ("c0", C.c_double),
                ("alpha", C.c_double), ("kappa", C.POINTER(C.c_double)),
                ("kappa_uniform", C.c_double), ("r", C.c_double), ("levels", C.c_int32),
                ("K", C.c_int32), ("gamma", C.c_double), ("ne_fixed", C.c_int32),
                ("ne_tol", C.c_double), ("ne_max", C.c_int32),
                ("el_type", C.c_int32 * 4), ("flow_type", C.POINTER(C.c_int8) * 4),
                ("el_value", C.POINTER(C.c_double) * 4), ("p_value", C.POINTER(C.c_double) * 4),
                ("pressure_gradient", C.c_int32), ("cycle", C.c_int32),
                ("fstar_literal", C.c_int32), ("coarse_sweeps", C.c_int32), ("lag", C.c_int32)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = C.CDLL(_LIB)
        vp, dp, ip = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int)
        lib.or_create.restype = vp
        lib.or_create.argtypes = [C.POINTER(_Problem), ip]
        lib.or_destroy.argtypes = [vp]
        lib.or_set_loads.argtypes = [vp, dp, dp, C.c_int]
        lib.or_step.argtypes = [vp, C.c_int]
        lib.or_set_threads.argtypes = [vp, C.c_int]
        lib.or_set_history.argtypes = [vp, C.c_int]
        lib.or_get_history.argtypes = [vp, ip, dp, C.c_int]
        lib.or_set_ne_schedule.argtypes = [vp, ip, C.c_int]
        lib.or_get_fields.argtypes = [vp, dp, dp, dp, ip]
        lib.or_get_state.argtypes = [vp, dp, dp, dp, dp, ip]
        lib.or_set_state.argtypes = [vp, dp, dp, dp, dp, C.c_int]
        lib.or_explicit_force.argtypes = [vp, dp]
        lib.or_apply_elastic.argtypes = [vp, C.c_int, dp, dp, dp, dp]
        lib.or_mg_cycle.argtypes = [vp, C.c_int, dp, dp, dp]
        lib.or_level_shape.argtypes = [vp, C.c_int, ip, ip]
        lib.or_flow_step.argtypes = [vp, dp]
        lib.or_default_levels.argtypes = [C.c_int, C.c_int]
        lib.or_coarsest_visits.restype = C.c_long
        lib.or_coarsest_visits.argtypes = [vp]
        _lib = lib
    return _lib


def _dptr(a):
    if a is None:
        return C.cast(None, C.POINTER(C.c_double))
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(C.c_double))


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"oracle {what} failed with status {code}")
        self.code = code


class Oracle:
    """FP64 reference solver for one Problem."""

    def __init__(self, p: Problem, threads: int = 1, history: int = 0):
        lib = _load()
        self.p = p
        self._keep = []
        pb = _Problem()
        pb.nx, pb.ny, pb.dx, pb.dt = p.nx, p.ny, p.dx, p.dt
        pb.lambda_, pb.mu, pb.c0, pb.alpha = p.lam, p.mu, p.c0, p.alpha
        if np.isscalar(p.kappa):
            pb.kappa = C.cast(None, C.POINTER(C.c_double))
            pb.kappa_uniform = float(p.kappa)
        else:
            k = np.ascontiguousarray(p.kappa, dtype=np.float64).reshape(-1)
            self._keep.append(k)
            pb.kappa = _dptr(k)
            pb.kappa_uniform = 0.0
        pb.r, pb.levels, pb.K, pb.gamma = p.r, p.levels, p.K, p.gamma
        pb.ne_fixed, pb.ne_tol, pb.ne_max = p.ne_fixed, p.ne_tol, p.ne_max
        pb.pressure_gradient = int(getattr(p, "pressure_gradient", 0))
        pb.cycle = int(getattr(p, "cycle", 0))
        pb.fstar_literal = int(getattr(p, "fstar_literal", 0))
        pb.coarse_sweeps = int(getattr(p, "coarse_sweeps", 0))
        pb.lag = int(getattr(p, "lag", 0))
        for s in range(4):
            side = p.sides[s]
            fl = np.ascontiguousarray(side.flow, dtype=np.int8)
            ev = np.ascontiguousarray(side.el_value, dtype=np.float64).reshape(-1)
            pv = np.ascontiguousarray(side.p_value, dtype=np.float64)
            self._keep += [fl, ev, pv]
            pb.el_type[s] = int(side.el)
            pb.flow_type[s] = fl.ctypes.data_as(C.POINTER(C.c_int8))
            pb.el_value[s] = _dptr(ev)
            pb.p_value[s] = _dptr(pv)
        err = C.c_int(0)
        h = lib.or_create(C.byref(pb), C.byref(err))
        if not h:
            raise OracleError(err.value, "create")
        self._h = C.c_void_p(h)
        self._lib = lib
        lib.or_set_threads(self._h, int(threads))
        self.history = history
        if history:
            lib.or_set_history(self._h, int(history))
        self._sched = None
        self.set_loads(p.body_f, p.source_s, reinit=True)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.or_destroy(h)
            self._h = None

    # ------------------------------------------------------------ driving
    def set_loads(self, body_f=None, source_s=None, reinit=False):
        bf = None if body_f is None else np.ascontiguousarray(body_f, dtype=np.float64).reshape(-1)
        ss = None if source_s is None else np.ascontiguousarray(source_s, dtype=np.float64).reshape(-1)
        self._lib.or_set_loads(self._h, _dptr(bf), _dptr(ss), int(reinit))

    def set_threads(self, threads: int):
        self._lib.or_set_threads(self._h, int(threads))

    def step(self, n: int = 1):
        rc = self._lib.or_step(self._h, int(n))
        if rc != OR_OK:
            raise OracleError(rc, "step")

    def set_ne_schedule(self, ne):
        self._sched = np.ascontiguousarray(ne, dtype=np.int32)
        self._lib.or_set_ne_schedule(self._h, self._sched.ctypes.data_as(C.POINTER(C.c_int)),
                                     len(self._sched))

    def get_history(self):
        cap = max(self.history, 1)
        ne = np.zeros(cap, dtype=np.int32)
        ratio = np.zeros(cap)
        m = self._lib.or_get_history(self._h, ne.ctypes.data_as(C.POINTER(C.c_int)), _dptr(ratio), cap)
        return ne[:m], ratio[:m]

    def fields(self):
        p = self.p
        eta = np.zeros((2, p.ny, p.nx))
        pr = np.zeros((p.ny, p.nx))
        sig = np.zeros((3, p.ny, p.nx))
        st = C.c_int(0)
        rc = self._lib.or_get_fields(self._h, _dptr(eta), _dptr(pr), _dptr(sig), C.byref(st))
        return dict(eta=eta, p=pr, sigma=sig, step=st.value, status=rc)

    def get_state(self):
        p = self.p
        f = np.zeros((9, p.ny, p.nx))
        g = np.zeros((8, p.ny, p.nx))
        d1 = np.zeros((p.ny, p.nx))
        d2 = np.zeros((p.ny, p.nx))
        st = C.c_int(0)
        self._lib.or_get_state(self._h, _dptr(f), _dptr(g), _dptr(d1), _dptr(d2), C.byref(st))
        return dict(f=f, g=g, D1=d1, D2=d2, step=st.value)

    def set_state(self, f=None, g=None, D1=None, D2=None, step=0):
        arr = [None if a is None else np.ascontiguousarray(a, dtype=np.float64) for a in (f, g, D1, D2)]
        self._lib.or_set_state(self._h, *[_dptr(a) for a in arr], int(step))

    # ------------------------------------------------------ single operations
    def level_shape(self, l):
        nx, ny = C.c_int(0), C.c_int(0)
        L = self._lib.or_level_shape(self._h, int(l), C.byref(nx), C.byref(ny))
        if L < 0:
            raise OracleError(L, "level_shape")
        return nx.value, ny.value

    @property
    def levels(self):
        nx, ny = C.c_int(0), C.c_int(0)
        return self._lib.or_level_shape(self._h, 1, C.byref(nx), C.byref(ny))

    def explicit_force(self):
        p = self.p
        Ft = np.zeros((2, p.ny, p.nx))
        self._lib.or_explicit_force(self._h, _dptr(Ft))
        return Ft

    def apply_elastic(self, level, g, r=None, Ft=None):
        g = np.ascontiguousarray(g, dtype=np.float64)
        out = np.zeros_like(g)
        r = None if r is None else np.ascontiguousarray(r, dtype=np.float64)
        Ft = None if Ft is None else np.ascontiguousarray(Ft, dtype=np.float64)
        rc = self._lib.or_apply_elastic(self._h, int(level), _dptr(g), _dptr(r), _dptr(Ft), _dptr(out))
        if rc != OR_OK:
            raise OracleError(rc, "apply_elastic")
        return out

    def mg_cycle(self, level, g, r=None, Ft=None):
        g = np.array(g, dtype=np.float64, copy=True, order="C")
        r = None if r is None else np.ascontiguousarray(r, dtype=np.float64)
        Ft = None if Ft is None else np.ascontiguousarray(Ft, dtype=np.float64)
        rc = self._lib.or_mg_cycle(self._h, int(level), _dptr(g), _dptr(r), _dptr(Ft))
        if rc != OR_OK:
            raise OracleError(rc, "mg_cycle")
        return g

    def coarsest_visits(self):
        """Coarsest-level solves since creation (2K sweeps each)."""
        return int(self._lib.or_coarsest_visits(self._h))

    def flow_step(self, s_lat):
        s = np.ascontiguousarray(s_lat, dtype=np.float64)
        self._lib.or_flow_step(self._h, _dptr(s))


def default_levels(nx, ny):
    return _load().or_default_levels(int(nx), int(ny))


def run(p: Problem, nsteps: int, loads=None, threads: int = 1, history: int = 0,
        every: int = 0, callback=None):
    """Run the oracle for nsteps; ``loads(t)`` (optional) returns (f, s) at time t
    and is applied before every step; ``callback(k, oracle)`` is called after
    every ``every`` steps."""
    o = Oracle(p, threads=threads, history=history or nsteps)
    if loads is not None:
        f0, s0 = loads(0.0)
        o.set_loads(f0, s0, reinit=True)
    for k in range(nsteps):
        if loads is not None and k > 0:
            f, s = loads(k * p.dt)
            o.set_loads(f, s)
        o.step(1)
        if callback is not None and every and (k + 1) % every == 0:
            callback(k + 1, o)
    return o
