"""GPU parity of the W- and F-cycles (textbook shapes of the multigrid cycle
that the paper names as future work) against the oracle, through the C ABI:
time steps with fixed and adaptive cycle counts, one cycle from a given
iterate, a batch, and the server's refusal."""
import sys

import numpy as np
import pytest

from conftest import oracle_threads
from gpu_helpers import mixed_walls, problems_small, rel
from oracle.oracle import Oracle
from paper_2409_11382_amd import problem as P

pytestmark = pytest.mark.gpu

STEP_TOL = 1e-10
SHAPES = [P.CYCLE_W, P.CYCLE_F]


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


@pytest.mark.parametrize("cyc", SHAPES)
@pytest.mark.parametrize("name", ["mixed_124x68", "strip_130x72", "periodic_64", "terzaghi_8x128"])
def test_time_steps_match_oracle(lbm, name, cyc):
    """Four coupled steps with a fixed cycle count: FP64 to 1e-10, FP32
    shifted to 1e-5 of the oracle."""
    p = problems_small()[name].replace(cycle=cyc)
    o = Oracle(p, threads=oracle_threads())
    o.step(4)
    B = o.fields()
    for prec, tol in (("fp64", STEP_TOL), ("fp32_shifted", 1e-5)):
        s = lbm.Solver(p, prec)
        s.step(4)
        A = s.fields()
        s.close()
        e = (rel(A["eta"], B["eta"]), rel(A["p"], B["p"]), rel(A["sigma"], B["sigma"]))
        _say("cycle", cyc, name, prec, e)
        assert e[0] < tol and e[1] < tol, (name, prec, e)


@pytest.mark.parametrize("cyc", SHAPES)
def test_one_cycle_from_a_given_iterate(lbm, cyc):
    """bp_mg_cycle on the finest level (with the explicit force) and on the
    level below (with a random right-hand side) against the oracle's cycle."""
    p = mixed_walls(124, 68, seed=3).replace(cycle=cyc, K=2)
    s = lbm.Solver(p, "fp64")
    o = Oracle(p, threads=oracle_threads())
    f, g, d1, d2 = P.random_state(p, 11, scale=1e-2)
    o.set_state(f, g, d1, d2, step=5)
    s.set_state(f, g, d1, d2, step=5)
    Ft = o.explicit_force()
    L = o.levels
    ga, gb = s.mg_cycle(L, g, None, Ft), o.mg_cycle(L, g, None, Ft)
    e1 = np.abs(ga - gb).max() / np.abs(gb).max()
    nx, ny = o.level_shape(L - 1)
    rng = np.random.default_rng(4)
    gc, rc = rng.standard_normal((8, ny, nx)) * 0.1, rng.standard_normal((8, ny, nx)) * 0.1
    ha, hb = s.mg_cycle(L - 1, gc, rc, None), o.mg_cycle(L - 1, gc, rc, None)
    e2 = np.abs(ha - hb).max() / np.abs(hb).max()
    s.close()
    _say("one cycle", cyc, L, e1, e2)
    assert e1 < 1e-12 and e2 < 1e-12


@pytest.mark.parametrize("cyc", SHAPES)
def test_adaptive_cycle_counts_follow_oracle(lbm, cyc):
    """Adaptive mode (stop at ||g - S(g)|| <= 1e-6 ||g||): the device-side
    stopping test takes the oracle's cycle counts, and the fields agree."""
    p = P.terzaghi(nx=8, ny=32, ne_fixed=0, ne_tol=1e-6, ne_max=40).replace(cycle=cyc)
    s = lbm.Solver(p, "fp64")
    ne = []
    for _ in range(6):
        s.step(1)
        ne.append(s.stats()["last_ne"])
    o = Oracle(p, threads=1, history=6)
    o.step(6)
    ne_o, _ = o.get_history()
    _say("adaptive", cyc, "gpu", ne, "oracle", list(ne_o))
    assert ne == list(ne_o)
    assert rel(s.fields()["eta"], o.fields()["eta"]) < STEP_TOL
    s.close()


@pytest.mark.parametrize("cyc", SHAPES)
def test_adaptive_shapes_on_the_tile_schedule(lbm, cyc):
    """Adaptive W- and F-cycles on a problem too large for one workgroup
    (124 x 68: the tile kernels on the finest depths, the shaped coarse tail
    below, continued visits included), in FP64 and FP32 shifted storage,
    against the oracle replaying the GPU's cycle counts."""
    p = mixed_walls(124, 68, seed=3).replace(ne_fixed=0, ne_tol=1e-6, ne_max=20, K=3, cycle=cyc)
    for prec, tol in (("fp64", STEP_TOL), ("fp32_shifted", 1e-5)):
        s = lbm.Solver(p, prec)
        ne = []
        for _ in range(4):
            s.step(1)
            ne.append(s.stats()["last_ne"])
        A = s.fields()
        s.close()
        o = Oracle(p, threads=oracle_threads(), history=4)
        o.set_ne_schedule(np.array(ne, dtype=np.int32))
        o.step(4)
        B = o.fields()
        e = (rel(A["eta"], B["eta"]), rel(A["p"], B["p"]), rel(A["sigma"], B["sigma"]))
        _say("adaptive tile", cyc, prec, ne, e)
        assert e[0] < tol and e[1] < tol, (prec, ne, e)


def test_batch_of_w_cycles_equals_alone(lbm):
    """A batch of W-cycle problems of different sizes: each problem matches its
    lone solve (to rounding: the launch variants follow the cells a depth
    covers in all)."""
    probs = [mixed_walls(124, 68, seed=3).replace(cycle=P.CYCLE_W, ne_fixed=2, K=2),
             P.loaded_strip(n=64, alpha=0.9, ne_fixed=2, K=2).replace(cycle=P.CYCLE_W)]
    b = lbm.Batch(probs, "fp64")
    b.step(3)
    for i, p in enumerate(probs):
        s = lbm.Solver(p, "fp64")
        s.step(3)
        A, B = s.fields(), b.fields(i)
        s.close()
        d = (rel(B["eta"], A["eta"]), rel(B["p"], A["p"]))
        _say("batch W", i, d)
        assert max(d) < 1e-12, (i, d)
    b.close()


def test_server_refuses_other_shapes(lbm):
    srv = lbm.Server(64 << 20, prec="fp32_shifted", K=4, ne_fixed=3, max_slots=4)
    with pytest.raises(lbm.BiotError):
        srv.submit(P.loaded_strip(n=32).replace(cycle=P.CYCLE_W), 2)
    srv.close()
