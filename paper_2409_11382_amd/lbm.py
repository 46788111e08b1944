"""ctypes binding of libbiotlbm.so (include/biotlbm.h).

Argument marshalling only: every step of the method runs in the HIP library.
PyTorch provides the device workspace and the stream.  The library must have
been built (``python -m paper_2409_11382_amd.build`` or ``__graft_entry__.build``);
there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from .problem import PREC_NAMES, Problem

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbiotlbm.so")

BP_OK, BP_ERR_ARG, BP_ERR_SHAPE, BP_ERR_DEVICE = 0, -1, -2, -3
BP_ERR_DIVERGED, BP_ERR_WORKSPACE, BP_ERR_STATE = -4, -5, -6


class BiotError(RuntimeError):
    def __init__(self, code: int, what: str, msg: str):
        super().__init__(f"{what} failed ({code}): {msg}")
        self.code = code


class _Side(C.Structure):
    _fields_ = [("el", C.c_int32), ("flow_uniform", C.c_int32), ("flow_type", C.POINTER(C.c_int8)),
                ("el_value", C.POINTER(C.c_double)), ("p_value", C.POINTER(C.c_double))]


class _Problem(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("dx", C.c_double), ("dt", C.c_double),
                ("lambda_", C.c_double), ("mu", C.c_double), ("c0", C.c_double), ("alpha", C.c_double),
                ("kappa", C.POINTER(C.c_double)), ("kappa_uniform", C.c_double),
                ("body_f", C.POINTER(C.c_double)), ("source_s", C.POINTER(C.c_double)),
                ("r", C.c_double), ("levels", C.c_int32), ("K", C.c_int32), ("gamma", C.c_double),
                ("ne_fixed", C.c_int32), ("ne_tol", C.c_double), ("ne_max", C.c_int32),
                ("side", _Side * 4), ("prec", C.c_int32), ("pressure_gradient", C.c_int32),
                ("cycle", C.c_int32), ("fstar_literal", C.c_int32), ("coarse_sweeps", C.c_int32),
                ("lag", C.c_int32)]


class _Tuning(C.Structure):
    _fields_ = [("quad_max_cells", C.c_int64), ("tall_max_cells", C.c_int64),
                ("fuse_res_max_cells", C.c_int64), ("quad_res_narrow_max_cells", C.c_int64),
                ("ms_per_step", C.c_double)]


def _tuning_dict(t):
    return {k: getattr(t, k) for k, _ in _Tuning._fields_}


def _tuning_struct(d):
    t = _Tuning()
    for k, _ in _Tuning._fields_:
        if k in d:
            setattr(t, k, d[k])
    return t


class _Stats(C.Structure):
    _fields_ = [("step", C.c_int32), ("last_ne", C.c_int32), ("total_cycles", C.c_int64),
                ("last_ratio", C.c_double), ("levels", C.c_int32), ("diverged", C.c_int32),
                ("adaptive_steps", C.c_int32), ("steps_at_cap", C.c_int32),
                ("max_ratio", C.c_double), ("mean_ratio", C.c_double)]


class _KernelStat(C.Structure):
    _fields_ = [("name", C.c_char * 48), ("depth", C.c_int32), ("launches", C.c_int32),
                ("us_per_step", C.c_double), ("bytes_per_step", C.c_double)]


_lib = None


def load_library():
    """Load libbiotlbm.so; raises if it has not been built.

    PyTorch is imported first: the library and PyTorch's bundled HIP runtime
    share the soname libamdhip64.so.7, so whichever loads first is the one HIP
    runtime of the process, and it must be the runtime PyTorch was built with
    (the workspaces and streams come from PyTorch)."""
    global _lib
    if _lib is None:
        import torch  # noqa: F401  (see above)

        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2409_11382_amd/build.py")
        lib = C.CDLL(LIB_PATH)
        vp, dp, i32 = C.c_void_p, C.POINTER(C.c_double), C.c_int32
        st = C.c_int
        for name, args in {
            "bp_workspace_bytes": [C.POINTER(_Problem), C.POINTER(C.c_size_t)],
            "bp_create": [C.POINTER(_Problem), vp, C.c_size_t, vp, C.POINTER(vp)],
            "bp_create_static": [C.POINTER(_Problem), vp, C.POINTER(vp)],
            "bp_step": [vp, i32],
            "bp_set_loads": [vp, dp, dp, i32],
            "bp_get_fields": [vp, dp, dp, dp, C.POINTER(i32)],
            "bp_get_state": [vp, dp, dp, dp, dp, C.POINTER(i32)],
            "bp_set_state": [vp, dp, dp, dp, dp, i32],
            "bp_apply_elastic": [vp, i32, dp, dp, dp, dp],
            "bp_mg_cycle": [vp, i32, dp, dp, dp],
            "bp_explicit_force": [vp, dp],
            "bp_level_shape": [vp, i32, C.POINTER(i32), C.POINTER(i32)],
            "bp_stats": [vp, C.POINTER(_Stats)],
            "bp_time_kernel": [vp, i32, i32, dp, dp],
            "bp_profile_step": [vp, i32, C.POINTER(_KernelStat), i32, C.POINTER(i32)],
            "bp_batch_profile_step": [vp, i32, C.POINTER(_KernelStat), i32, C.POINTER(i32)],
            "bp_get_tuning": [vp, C.POINTER(_Tuning)],
            "bp_set_tuning": [vp, C.POINTER(_Tuning)],
            "bp_autotune": [vp, i32, C.POINTER(_Tuning)],
            "bp_batch_get_tuning": [vp, C.POINTER(_Tuning)],
            "bp_batch_set_tuning": [vp, C.POINTER(_Tuning)],
            "bp_batch_autotune": [vp, i32, C.POINTER(_Tuning)],
            "bp_device_copy": [vp, vp, C.c_size_t, vp],
            "bp_destroy": [vp],
            "bp_batch_workspace_bytes": [C.POINTER(_Problem), i32, C.POINTER(C.c_size_t)],
            "bp_batch_create": [C.POINTER(_Problem), i32, vp, C.c_size_t, vp, C.POINTER(vp)],
            "bp_batch_step": [vp, i32],
            "bp_batch_get_fields": [vp, i32, dp, dp, dp, C.POINTER(i32)],
            "bp_batch_destroy": [vp],
            "bp_server_request_bytes": [C.POINTER(_Problem), C.POINTER(C.c_size_t)],
            "bp_server_create": [vp, C.c_size_t, vp, i32, i32, i32, i32, C.POINTER(vp)],
            "bp_server_submit": [vp, C.POINTER(_Problem), i32, C.POINTER(C.c_int64)],
            "bp_server_advance": [vp, i32, C.POINTER(i32), C.POINTER(i32)],
            "bp_server_poll": [vp, C.c_int64, C.POINTER(i32), C.POINTER(i32)],
            "bp_server_result": [vp, C.c_int64, dp, dp, dp],
            "bp_server_stats": [vp, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t), C.POINTER(i32), C.POINTER(i32)],
            "bp_server_destroy": [vp],
        }.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = st
        lib.bp_last_error.restype = C.c_char_p
        lib.bp_last_error.argtypes = []
        _lib = lib
    return _lib


def _check(rc, what):
    if rc != BP_OK:
        raise BiotError(rc, what, _lib.bp_last_error().decode())


def _dptr(a):
    if a is None:
        return C.cast(None, C.POINTER(C.c_double))
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"], "expected C-contiguous float64"
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def marshal_problem(p: Problem, prec="fp64"):
    """Build the bp_problem struct; returns (struct, keep-alive list)."""
    keep = []
    pb = _Problem()
    pb.nx, pb.ny, pb.dx, pb.dt = p.nx, p.ny, p.dx, p.dt
    pb.lambda_, pb.mu, pb.c0, pb.alpha = p.lam, p.mu, p.c0, p.alpha
    if np.isscalar(p.kappa):
        pb.kappa = _dptr(None)
        pb.kappa_uniform = float(p.kappa)
    else:
        k = _f64(p.kappa).reshape(-1)
        keep.append(k)
        pb.kappa = _dptr(k)
    for name in ("body_f", "source_s"):
        a = getattr(p, name)
        if a is None:
            setattr(pb, name, _dptr(None))
        else:
            a = _f64(a).reshape(-1)
            keep.append(a)
            setattr(pb, name, _dptr(a))
    pb.r, pb.levels, pb.K, pb.gamma = p.r, p.levels, p.K, p.gamma
    pb.ne_fixed, pb.ne_tol, pb.ne_max = p.ne_fixed, p.ne_tol, p.ne_max
    for s in range(4):
        side = p.sides[s]
        fl = np.ascontiguousarray(side.flow, dtype=np.int8)
        ev = _f64(side.el_value).reshape(-1)
        pv = _f64(side.p_value)
        keep += [fl, ev, pv]
        pb.side[s].el = int(side.el)
        pb.side[s].flow_uniform = int(fl[0]) if len(fl) else 0
        pb.side[s].flow_type = fl.ctypes.data_as(C.POINTER(C.c_int8))
        pb.side[s].el_value = _dptr(ev)
        pb.side[s].p_value = _dptr(pv)
    pb.prec = PREC_NAMES[prec] if isinstance(prec, str) else int(prec)
    pb.pressure_gradient = int(p.pressure_gradient)
    pb.cycle = int(p.cycle)
    pb.fstar_literal = int(p.fstar_literal)
    pb.coarse_sweeps = int(p.coarse_sweeps)
    pb.lag = int(p.lag)
    return pb, keep


def workspace_bytes(p: Problem, prec="fp64") -> int:
    lib = load_library()
    pb, _keep = marshal_problem(p, prec)
    n = C.c_size_t(0)
    _check(lib.bp_workspace_bytes(C.byref(pb), C.byref(n)), "bp_workspace_bytes")
    return n.value


class Solver:
    """One problem resident on a GPU.  Method names follow biotlbm.h."""

    def __init__(self, p: Problem, prec="fp64", device="cuda:0", stream=None, static_workspace=False):
        """static_workspace: bp_create_static (the library's static device
        array as the workspace; nothing is allocated) instead of bp_create on
        a workspace from PyTorch."""
        import torch

        lib = load_library()
        self.p = p
        self.prec = prec
        self.device = torch.device(device)
        pb, keep = marshal_problem(p, prec)
        n = C.c_size_t(0)
        _check(lib.bp_workspace_bytes(C.byref(pb), C.byref(n)), "bp_workspace_bytes")
        self.ws_bytes = n.value
        # a stream of its own (default priority): the library replays each time
        # step as one captured HIP graph, which the legacy null stream cannot hold
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        h = C.c_void_p(0)
        if static_workspace:
            self.ws = None
            with torch.cuda.device(self.device):
                _check(lib.bp_create_static(C.byref(pb), C.c_void_p(self.stream.cuda_stream), C.byref(h)),
                       "bp_create_static")
        else:
            self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
            self.ws.record_stream(self.stream)
            _check(lib.bp_create(C.byref(pb), C.c_void_p(self.ws.data_ptr()), self.ws_bytes,
                                 C.c_void_p(self.stream.cuda_stream), C.byref(h)), "bp_create")
        del keep
        self._h = h
        self._lib = lib

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.bp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # --------------------------------------------------------------- driving
    def step(self, n=1):
        _check(self._lib.bp_step(self._h, int(n)), "bp_step")

    def set_loads(self, body_f=None, source_s=None, reinit=False):
        bf, ss = _f64(body_f), _f64(source_s)
        _check(self._lib.bp_set_loads(self._h, _dptr(None if bf is None else bf.reshape(-1)),
                                      _dptr(None if ss is None else ss.reshape(-1)), int(reinit)),
               "bp_set_loads")

    def fields(self):
        p = self.p
        eta = np.zeros((2, p.ny, p.nx))
        pr = np.zeros((p.ny, p.nx))
        sig = np.zeros((3, p.ny, p.nx))
        st = C.c_int32(0)
        _check(self._lib.bp_get_fields(self._h, _dptr(eta), _dptr(pr), _dptr(sig), C.byref(st)),
               "bp_get_fields")
        return dict(eta=eta, p=pr, sigma=sig, step=st.value)

    def get_state(self):
        p = self.p
        f = np.zeros((9, p.ny, p.nx))
        g = np.zeros((8, p.ny, p.nx))
        d1 = np.zeros((p.ny, p.nx))
        d2 = np.zeros((p.ny, p.nx))
        st = C.c_int32(0)
        _check(self._lib.bp_get_state(self._h, _dptr(f), _dptr(g), _dptr(d1), _dptr(d2), C.byref(st)),
               "bp_get_state")
        return dict(f=f, g=g, D1=d1, D2=d2, step=st.value)

    def set_state(self, f=None, g=None, D1=None, D2=None, step=0):
        arr = [_f64(a) for a in (f, g, D1, D2)]
        _check(self._lib.bp_set_state(self._h, *[_dptr(a) for a in arr], int(step)), "bp_set_state")

    # ------------------------------------------------------ single operations
    def level_shape(self, level):
        nx, ny = C.c_int32(0), C.c_int32(0)
        _check(self._lib.bp_level_shape(self._h, int(level), C.byref(nx), C.byref(ny)), "bp_level_shape")
        return nx.value, ny.value

    def apply_elastic(self, level, g, r=None, Ft=None):
        g = _f64(g)
        out = np.zeros_like(g)
        _check(self._lib.bp_apply_elastic(self._h, int(level), _dptr(g), _dptr(_f64(r)), _dptr(_f64(Ft)),
                                          _dptr(out)), "bp_apply_elastic")
        return out

    def mg_cycle(self, level, g, r=None, Ft=None):
        g = np.array(g, dtype=np.float64, copy=True, order="C")
        _check(self._lib.bp_mg_cycle(self._h, int(level), _dptr(g), _dptr(_f64(r)), _dptr(_f64(Ft))),
               "bp_mg_cycle")
        return g

    def explicit_force(self):
        Ft = np.zeros((2, self.p.ny, self.p.nx))
        _check(self._lib.bp_explicit_force(self._h, _dptr(Ft)), "bp_explicit_force")
        return Ft

    def stats(self):
        st = _Stats()
        _check(self._lib.bp_stats(self._h, C.byref(st)), "bp_stats")
        return {k: getattr(st, k) for k, _ in _Stats._fields_}

    def autotune(self, steps=4):
        """Choose the launch-shape bounds by timing (before the first step;
        the state is re-initialised).  Returns the chosen bounds."""
        t = _Tuning()
        _check(self._lib.bp_autotune(self._h, int(steps), C.byref(t)), "bp_autotune")
        return _tuning_dict(t)

    def tuning(self):
        t = _Tuning()
        _check(self._lib.bp_get_tuning(self._h, C.byref(t)), "bp_get_tuning")
        return _tuning_dict(t)

    def set_tuning(self, bounds):
        cur = self.tuning()
        cur.update(bounds)
        t = _tuning_struct(cur)
        _check(self._lib.bp_set_tuning(self._h, C.byref(t)), "bp_set_tuning")

    def profile_step(self, steps=5, cap=256):
        """bp_profile_step: per kernel variant and depth, launches, device
        microseconds and algorithmic bytes per step (runs `steps` steps)."""
        rows = (_KernelStat * cap)()
        n = C.c_int32(0)
        _check(self._lib.bp_profile_step(self._h, int(steps), rows, int(cap), C.byref(n)), "bp_profile_step")
        return [{"name": rows[k].name.decode(), "depth": rows[k].depth, "launches": rows[k].launches,
                 "us_per_step": rows[k].us_per_step, "bytes_per_step": rows[k].bytes_per_step}
                for k in range(min(n.value, cap))]

    def time_kernel(self, which, iters=20):
        us, by = C.c_double(0), C.c_double(0)
        _check(self._lib.bp_time_kernel(self._h, int(which), int(iters), C.byref(us), C.byref(by)),
               "bp_time_kernel")
        return us.value, by.value


def device_copy(dst_ptr: int, src_ptr: int, nbytes: int, stream_ptr: int):
    lib = load_library()
    _check(lib.bp_device_copy(C.c_void_p(dst_ptr), C.c_void_p(src_ptr), nbytes, C.c_void_p(stream_ptr)),
           "bp_device_copy")


class Batch:
    """Many independent problems advanced together (one launch per multigrid
    depth and phase covers all of them).  Method names follow biotlbm.h."""

    def __init__(self, problems, prec="fp32_shifted", device="cuda:0", stream=None):
        import torch

        lib = load_library()
        self.problems = list(problems)
        n = len(self.problems)
        arr = (_Problem * n)()
        keep = []
        for i, p in enumerate(self.problems):
            pb, k = marshal_problem(p, prec)
            arr[i] = pb
            keep.append(k)
        nbytes = C.c_size_t(0)
        _check(lib.bp_batch_workspace_bytes(arr, n, C.byref(nbytes)), "bp_batch_workspace_bytes")
        self.ws_bytes = nbytes.value
        self.device = torch.device(device)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        # a stream of its own (default priority): the library replays each time
        # step as one captured HIP graph, which the legacy null stream cannot hold
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        self.ws.record_stream(self.stream)
        h = C.c_void_p(0)
        _check(lib.bp_batch_create(arr, n, C.c_void_p(self.ws.data_ptr()), self.ws_bytes,
                                   C.c_void_p(self.stream.cuda_stream), C.byref(h)), "bp_batch_create")
        del keep
        self._h = h
        self._lib = lib

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.bp_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __len__(self):
        return len(self.problems)

    def step(self, n=1):
        _check(self._lib.bp_batch_step(self._h, int(n)), "bp_batch_step")

    def profile_step(self, steps=3, cap=256):
        """bp_batch_profile_step (see Solver.profile_step)."""
        rows = (_KernelStat * cap)()
        n = C.c_int32(0)
        _check(self._lib.bp_batch_profile_step(self._h, int(steps), rows, int(cap), C.byref(n)),
               "bp_batch_profile_step")
        return [{"name": rows[k].name.decode(), "depth": rows[k].depth, "launches": rows[k].launches,
                 "us_per_step": rows[k].us_per_step, "bytes_per_step": rows[k].bytes_per_step}
                for k in range(min(n.value, cap))]

    def autotune(self, steps=2):
        """Choose the launch-shape bounds by timing (before the first step;
        the problems are re-initialised).  Returns the chosen bounds."""
        t = _Tuning()
        _check(self._lib.bp_batch_autotune(self._h, int(steps), C.byref(t)), "bp_batch_autotune")
        return _tuning_dict(t)

    def tuning(self):
        t = _Tuning()
        _check(self._lib.bp_batch_get_tuning(self._h, C.byref(t)), "bp_batch_get_tuning")
        return _tuning_dict(t)

    def set_tuning(self, bounds):
        cur = self.tuning()
        cur.update(bounds)
        t = _tuning_struct(cur)
        _check(self._lib.bp_batch_set_tuning(self._h, C.byref(t)), "bp_batch_set_tuning")

    def fields(self, i):
        p = self.problems[i]
        eta = np.zeros((2, p.ny, p.nx))
        pr = np.zeros((p.ny, p.nx))
        sig = np.zeros((3, p.ny, p.nx))
        st = C.c_int32(0)
        _check(self._lib.bp_batch_get_fields(self._h, int(i), _dptr(eta), _dptr(pr), _dptr(sig), C.byref(st)),
               "bp_batch_get_fields")
        return dict(eta=eta, p=pr, sigma=sig, step=st.value)


REQ_QUEUED, REQ_RUNNING, REQ_DONE, REQ_FAILED = 0, 1, 2, 3


def request_bytes(p: Problem, prec="fp32_shifted") -> int:
    """Device bytes a request occupies in a server's pool (host-only)."""
    lib = load_library()
    pb, _keep = marshal_problem(p, prec)
    n = C.c_size_t(0)
    _check(lib.bp_server_request_bytes(C.byref(pb), C.byref(n)), "bp_server_request_bytes")
    return n.value


class Server:
    """Continuous batching of solve requests on one GPU (bp_server_*): queued
    requests are admitted by pool memory as earlier ones finish, and all
    admitted requests advance together.  Method names follow biotlbm.h."""

    def __init__(self, ws_bytes: int, prec="fp32_shifted", K=4, ne_fixed=3, max_slots=512, device="cuda:0",
                 stream=None):
        import torch

        lib = load_library()
        self.prec = prec
        self.K, self.ne_fixed = K, ne_fixed
        self.device = torch.device(device)
        self.ws_bytes = int(ws_bytes) // 256 * 256
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        self.ws.record_stream(self.stream)
        h = C.c_void_p(0)
        _check(lib.bp_server_create(C.c_void_p(self.ws.data_ptr()), self.ws_bytes, C.c_void_p(self.stream.cuda_stream),
                                    PREC_NAMES[prec], int(K), int(ne_fixed), int(max_slots), C.byref(h)),
               "bp_server_create")
        self._h = h
        self._lib = lib
        self._shape = {}

    def submit(self, p: Problem, nsteps: int) -> int:
        p = p.replace(K=self.K, ne_fixed=self.ne_fixed)
        pb, keep = marshal_problem(p, self.prec)
        t = C.c_int64(0)
        _check(self._lib.bp_server_submit(self._h, C.byref(pb), int(nsteps), C.byref(t)), "bp_server_submit")
        del keep
        self._shape[t.value] = (p.nx, p.ny)
        return t.value

    def advance(self, nsteps=1):
        a, q = C.c_int32(0), C.c_int32(0)
        _check(self._lib.bp_server_advance(self._h, int(nsteps), C.byref(a), C.byref(q)), "bp_server_advance")
        return a.value, q.value

    def poll(self, ticket: int):
        st, n = C.c_int32(0), C.c_int32(0)
        _check(self._lib.bp_server_poll(self._h, int(ticket), C.byref(st), C.byref(n)), "bp_server_poll")
        return st.value, n.value

    def result(self, ticket: int):
        nx, ny = self._shape[ticket]
        eta = np.zeros((2, ny, nx))
        p = np.zeros((ny, nx))
        sig = np.zeros((3, ny, nx))
        rc = self._lib.bp_server_result(self._h, int(ticket), _dptr(eta), _dptr(p), _dptr(sig))
        if rc != BP_ERR_STATE:  # the library forgets the ticket unless it is still running
            self._shape.pop(ticket, None)
        _check(rc, "bp_server_result")
        return {"eta": eta, "p": p, "sigma": sig}

    def stats(self):
        pool, free = C.c_size_t(0), C.c_size_t(0)
        a, q = C.c_int32(0), C.c_int32(0)
        _check(self._lib.bp_server_stats(self._h, C.byref(pool), C.byref(free), C.byref(a), C.byref(q)),
               "bp_server_stats")
        return {"pool_bytes": pool.value, "free_bytes": free.value, "active": a.value, "queued": q.value}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.bp_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
