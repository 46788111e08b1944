"""The entry point that allocates nothing (bp_create_static) against
bp_create, through the C ABI.  Solvers on the device's static workspace are
created one after another, the second on a smaller problem than the first,
and each must give the fields of the workspace solver of the same problem
(FP64 to 1e-10 and FP32 shifted to 1e-5 of them; the same kernels run in the
same order, so the fields are expected bitwise equal)."""
import sys

import numpy as np
import pytest

from gpu_helpers import mixed_walls, rel
from paper_2409_11382_amd import problem as P

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lbm():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2409_11382_amd import lbm as L

    L.load_library()
    return L


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _run(lbm, p, prec, static, steps):
    s = lbm.Solver(p, prec, static_workspace=static)
    s.step(steps)
    F = s.fields()
    st = s.stats()
    s.close()
    return F, st


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32_shifted", 1e-5)])
def test_static_workspace_solvers_in_a_row(lbm, prec, tol):
    """A 124 x 68 problem with mixed walls, then a 32^2 strip: the second
    solver reuses the array the first left behind."""
    for p in (mixed_walls(124, 68, seed=3), P.loaded_strip(n=32, alpha=0.9, K=2, ne_fixed=2)):
        A, _ = _run(lbm, p, prec, True, 3)
        B, _ = _run(lbm, p, prec, False, 3)
        e = (rel(A["eta"], B["eta"]), rel(A["p"], B["p"]), rel(A["sigma"], B["sigma"]))
        same = all(np.array_equal(A[k], B[k]) for k in ("eta", "p", "sigma"))
        _say("static", p.name, prec, e, "bitwise" if same else "not bitwise")
        assert max(e) < tol, (p.name, prec, e)
        assert A["step"] == B["step"] == 3


def test_static_workspace_adaptive_cycles(lbm):
    """Adaptive cycles read the stop flag into a host buffer of the solver
    (no pinned staging): Terzaghi 8 x 64 to 1e-6, then a smaller column."""
    for ny in (64, 32):
        p = P.terzaghi(nx=8, ny=ny, ne_fixed=0, ne_tol=1e-6, ne_max=40)
        A, sa = _run(lbm, p, "fp64", True, 4)
        B, sb = _run(lbm, p, "fp64", False, 4)
        _say("static adaptive", ny, sa["total_cycles"], sb["total_cycles"], rel(A["eta"], B["eta"]))
        assert sa["total_cycles"] == sb["total_cycles"]
        assert rel(A["eta"], B["eta"]) < 1e-10 and rel(A["p"], B["p"]) < 1e-10


def test_static_workspace_is_held_by_one_solver(lbm):
    p = P.loaded_strip(n=32, alpha=0.9, K=2, ne_fixed=2)
    s = lbm.Solver(p, "fp64", static_workspace=True)
    with pytest.raises(lbm.BiotError) as ei:
        lbm.Solver(p, "fp64", static_workspace=True)
    assert ei.value.code == lbm.BP_ERR_STATE
    s.close()
    t = lbm.Solver(p, "fp64", static_workspace=True)  # released by bp_destroy
    t.close()


def test_static_workspace_refuses_larger_problems(lbm):
    big = P.loaded_strip(n=512)                          # about 120 MB in FP64
    with pytest.raises(lbm.BiotError) as ei:
        lbm.Solver(big, "fp64", static_workspace=True)
    assert ei.value.code == lbm.BP_ERR_WORKSPACE
    s = lbm.Solver(P.loaded_strip(n=32), "fp64", static_workspace=True)  # a refusal holds nothing
    s.close()
