"""Host-only checks of the HIP library: it loads, exports every symbol the
public header declares, and validates problems without touching a GPU."""
import ctypes as C
import os
import re

import pytest

from paper_2409_11382_amd import lbm as L
from paper_2409_11382_amd import problem as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "biotlbm.h")).read()
    return sorted(set(re.findall(r"\b(bp_[a-z_]+)\s*\(", src)))


def test_header_declares_the_entry_points():
    names = _declared()
    for n in ("bp_workspace_bytes", "bp_create", "bp_step", "bp_get_fields", "bp_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = L.load_library()
    for name in _declared():
        assert hasattr(lib, name), name


def test_workspace_size_and_validation_are_host_only():
    small = L.workspace_bytes(P.loaded_strip(n=64), "fp64")
    big = L.workspace_bytes(P.loaded_strip(n=128), "fp64")
    f32 = L.workspace_bytes(P.loaded_strip(n=128), "fp32_shifted")
    assert 0 < small < big and f32 < big
    assert small % 256 == 0
    for bad in (dict(c0=0.0), dict(mu=-1.0), dict(alpha=2.0), dict(r=-0.1), dict(gamma=0.0),
                dict(K=0), dict(levels=9), dict(kappa=0.0)):
        with pytest.raises(L.BiotError) as ei:
            L.workspace_bytes(P.loaded_strip(n=64).replace(**bad), "fp64")
        assert ei.value.code in (L.BP_ERR_ARG, L.BP_ERR_SHAPE)
    # periodic on one side only
    p = P.loaded_strip(n=16)
    sides = list(p.sides)
    sides[P.LEFT] = P.Side.uniform(16, P.EL_PERIODIC, P.FLOW_PERIODIC)
    with pytest.raises(L.BiotError):
        L.workspace_bytes(p.replace(sides=sides))


def test_degenerate_problems_are_rejected_on_the_host():
    """Empty grids, shapes the hierarchy cannot coarsen, coarsest levels
    below two cells in a walled direction, non-finite or out-of-range
    parameters, an adaptive mode without a tolerance, an unknown gradient
    variant, and empty or mixed batches."""
    nan = float("nan")
    base = P.loaded_strip(n=64)
    bad = [dict(nx=0), dict(ny=0), dict(dt=0.0), dict(dx=-1.0), dict(alpha=nan), dict(mu=nan),
           dict(gamma=1.5), dict(ne_fixed=0, ne_tol=0.0), dict(ne_fixed=0, ne_tol=1e-6, ne_max=0),
           dict(pressure_gradient=2), dict(cycle=4), dict(cycle=-1),
           dict(fstar_literal=2), dict(coarse_sweeps=3), dict(coarse_sweeps=-2),
           dict(lag=1),                                        # the lag is Algorithm 1: one level
           dict(lag=1, levels=1, ne_fixed=0, ne_tol=1e-6),     # with a fixed N_E
           dict(levels=7),                                     # 64 / 2^6 = 1 cell on the coarsest level
           dict(nx=63, levels=2)]                              # odd width cannot coarsen
    for kw in bad:
        with pytest.raises(L.BiotError) as ei:
            L.workspace_bytes(base.replace(**kw), "fp64")
        assert ei.value.code in (L.BP_ERR_ARG, L.BP_ERR_SHAPE), kw
    # the largest grid of the tests is accepted and sized without overflow
    big = L.workspace_bytes(P.loaded_strip(n=16384), "fp32_shifted")
    assert 80e9 < big < 90e9  # about 330 B per cell (FP64 references at this size)
    lib = L.load_library()
    n = C.c_size_t(0)
    assert lib.bp_batch_workspace_bytes(None, 0, C.byref(n)) == L.BP_ERR_ARG
    pa, ka = L.marshal_problem(base, "fp32_shifted")
    pb, kb = L.marshal_problem(base, "fp64")
    arr = (L._Problem * 2)(pa, pb)
    assert lib.bp_batch_workspace_bytes(arr, 2, C.byref(n)) == L.BP_ERR_ARG   # one precision per batch
    pw, kw_ = L.marshal_problem(base.replace(cycle=P.CYCLE_W), "fp32_shifted")
    arr = (L._Problem * 2)(pa, pw)
    assert lib.bp_batch_workspace_bytes(arr, 2, C.byref(n)) == L.BP_ERR_ARG   # one cycle shape per batch
    arr = (L._Problem * 2)(pw, pw)
    assert lib.bp_batch_workspace_bytes(arr, 2, C.byref(n)) == L.BP_OK
    pc, kc = L.marshal_problem(base.replace(coarse_sweeps=6), "fp32_shifted")
    arr = (L._Problem * 2)(pa, pc)
    assert lib.bp_batch_workspace_bytes(arr, 2, C.byref(n)) == L.BP_ERR_ARG   # one coarsest sweep count
    pd_, kd = L.marshal_problem(P.loaded_strip(n=32).replace(coarse_sweeps=6), "fp32_shifted")
    arr = (L._Problem * 2)(pc, pd_)
    assert lib.bp_batch_workspace_bytes(arr, 2, C.byref(n)) == L.BP_ERR_ARG   # and then one depth
    pl, kl = L.marshal_problem(base.replace(levels=1, gamma=1.0, K=1, lag=1), "fp32_shifted")
    arr = (L._Problem * 1)(pl)
    assert lib.bp_batch_workspace_bytes(arr, 1, C.byref(n)) == L.BP_ERR_ARG   # the lag: single solvers
    del ka, kb, kc, kd, kl


def test_last_error_message():
    lib = L.load_library()
    with pytest.raises(L.BiotError):
        L.workspace_bytes(P.loaded_strip(n=16).replace(c0=-1.0))
    assert b"c0" in lib.bp_last_error()


def test_server_request_bytes_is_host_only():
    a = L.request_bytes(P.loaded_strip(n=64), "fp32_shifted")
    b = L.request_bytes(P.loaded_strip(n=128), "fp32_shifted")
    assert 0 < a < b and a % 256 == 0
    # a request's footprint is its problem's part of a lone solver's workspace
    assert a < L.workspace_bytes(P.loaded_strip(n=64), "fp32_shifted")
    with pytest.raises(L.BiotError):
        L.request_bytes(P.loaded_strip(n=64).replace(c0=0.0))
