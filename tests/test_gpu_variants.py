"""GPU parity of the switchable variants against the oracle, through the C
ABI: full multigrid as the first cycle of a step, the self-dependence constant
as printed, the coarsest level's own sweep count, Algorithm 1 with the lag of
eq. source:implicit; and the divergence handling of batches and the server
(the coupled scheme's own instability, Sec. 4.1, not a fault)."""
import sys

import numpy as np
import pytest

from conftest import oracle_threads
from gpu_helpers import mixed_walls, problems_small, rel
from oracle.oracle import Oracle
from paper_2409_11382_amd import problem as P

pytestmark = pytest.mark.gpu

STEP_TOL = 1e-10


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


def _steps_match(lbm, p, nsteps, precs=(("fp64", STEP_TOL), ("fp32_shifted", 1e-5)), label=""):
    o = Oracle(p, threads=oracle_threads())
    o.step(nsteps)
    B = o.fields()
    for prec, tol in precs:
        s = lbm.Solver(p, prec)
        s.step(nsteps)
        A = s.fields()
        s.close()
        e = (rel(A["eta"], B["eta"]), rel(A["p"], B["p"]), rel(A["sigma"], B["sigma"]))
        _say(label, p.name, prec, e)
        assert e[0] < tol and e[1] < tol, (label, p.name, prec, e)


# --------------------------------------------------------- full multigrid
@pytest.mark.parametrize("name", ["mixed_124x68", "strip_130x72", "periodic_64", "terzaghi_8x128"])
def test_full_multigrid_steps_match_oracle(lbm, name):
    p = problems_small()[name].replace(cycle=P.CYCLE_FMG)
    _steps_match(lbm, p, 4, label="fmg")


def test_full_multigrid_deep_hierarchy(lbm):
    """256^2 strip (8 levels; the coarse tail's levels run on the tile kernels
    inside the FMG correction), three cycles per step."""
    p = P.loaded_strip(n=256, alpha=1.0, ne_fixed=3).replace(cycle=P.CYCLE_FMG)
    _steps_match(lbm, p, 2, label="fmg deep")


def test_full_multigrid_one_cycle_from_a_given_iterate(lbm):
    p = mixed_walls(124, 68, seed=3).replace(cycle=P.CYCLE_FMG, K=2)
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
    _say("fmg one cycle", L, e1, e2)
    assert e1 < 1e-12 and e2 < 1e-12


@pytest.mark.parametrize("prec", ["fp64", "fp32_shifted"])
def test_full_multigrid_adaptive_counts_follow_oracle(lbm, prec):
    """Adaptive mode with the FMG first cycle (on the tile schedule: the
    whole-problem tail runs V-, W- and F-cycles only): the GPU's cycle counts
    replayed by the oracle give the same fields."""
    p = P.terzaghi(nx=8, ny=64, ne_fixed=0, ne_tol=1e-6, ne_max=40).replace(cycle=P.CYCLE_FMG)
    s = lbm.Solver(p, prec)
    ne = []
    for _ in range(5):
        s.step(1)
        ne.append(s.stats()["last_ne"])
    A = s.fields()
    s.close()
    o = Oracle(p, threads=1, history=5)
    o.set_ne_schedule(np.array(ne, dtype=np.int32))
    o.step(5)
    tol = STEP_TOL if prec == "fp64" else 1e-5
    e = rel(A["eta"], o.fields()["eta"])
    _say("fmg adaptive", prec, ne, e)
    assert e < tol
    if prec == "fp64":
        a = Oracle(p, threads=1, history=5)
        a.step(5)
        assert list(a.get_history()[0]) == ne


def test_full_multigrid_batch_equals_alone(lbm):
    probs = [mixed_walls(124, 68, seed=3).replace(cycle=P.CYCLE_FMG, ne_fixed=2, K=2),
             P.loaded_strip(n=64, alpha=0.9, ne_fixed=2, K=2).replace(cycle=P.CYCLE_FMG)]
    b = lbm.Batch(probs, "fp64")
    b.step(3)
    for i, p in enumerate(probs):
        s = lbm.Solver(p, "fp64")
        s.step(3)
        A, B = s.fields(), b.fields(i)
        s.close()
        d = (rel(B["eta"], A["eta"]), rel(B["p"], A["p"]))
        _say("batch fmg", i, d)
        assert max(d) < 1e-12, (i, d)
    b.close()


# ------------------------------------------- literal self-dependence constant
@pytest.mark.parametrize("name", ["mixed_124x68", "periodic_64"])
def test_literal_constant_steps_match_oracle(lbm, name):
    p = problems_small()[name].replace(fstar_literal=1)
    _steps_match(lbm, p, 4, label="fstar literal")


# ------------------------------------------------ coarsest-level sweeps
def test_coarse_sweeps_in_the_coarse_tail(lbm):
    """Terzaghi 8 x 128 (3 levels, the 2 x 32 coarsest level in the
    one-workgroup tail): fixed cycles and adaptive cycles to 1e-8 with 512
    coarsest sweeps; the GPU's cycle counts are the oracle's own."""
    p = P.terzaghi(ne_fixed=3, ne_tol=0.0).replace(coarse_sweeps=64)
    _steps_match(lbm, p, 3, precs=(("fp64", STEP_TOL),), label="coarse sweeps tail")
    q = P.terzaghi(ne_tol=1e-8, ne_max=50).replace(coarse_sweeps=512)
    s = lbm.Solver(q, "fp64")
    ne = []
    for _ in range(4):
        s.step(1)
        ne.append(s.stats()["last_ne"])
    st = s.stats()
    A = s.fields()
    s.close()
    o = Oracle(q, threads=1, history=4)
    o.step(4)
    ne_o, ratio_o = o.get_history()
    _say("coarse sweeps adaptive", ne, list(ne_o), st)
    assert ne == list(ne_o) and max(ne) <= 25
    assert st["steps_at_cap"] == 0 and st["max_ratio"] <= 1e-8
    assert rel(A["eta"], o.fields()["eta"]) < STEP_TOL


def test_coarse_sweeps_on_the_tile_kernels(lbm):
    """256^2 strip with 3 levels: the 64^2 coarsest level is swept by the tile
    kernels, 10 sweeps in place of 2K = 8; one cycle on the coarsest level
    alone as well."""
    p = P.loaded_strip(n=256, alpha=1.0, ne_fixed=2, levels=3).replace(coarse_sweeps=10)
    _steps_match(lbm, p, 2, label="coarse sweeps tiles")
    s = lbm.Solver(p, "fp64")
    o = Oracle(p, threads=oracle_threads())
    nx, ny = o.level_shape(1)
    rng = np.random.default_rng(6)
    gc, rc = rng.standard_normal((8, ny, nx)) * 0.1, rng.standard_normal((8, ny, nx)) * 0.1
    ha, hb = s.mg_cycle(1, gc, rc, None), o.mg_cycle(1, gc, rc, None)
    s.close()
    assert np.abs(ha - hb).max() < 1e-12 * np.abs(hb).max()


def test_adaptive_statistics_report_the_cap(lbm):
    """The paper's 2K coarsest sweeps on Terzaghi 8 x 128: every step stops at
    N_E,max above the tolerance, and bp_stats says so."""
    p = P.terzaghi(ne_tol=1e-8, ne_max=50)
    s = lbm.Solver(p, "fp64")
    s.step(3)
    st = s.stats()
    s.close()
    o = Oracle(p, threads=1, history=3)
    o.step(3)
    _ne, ratio = o.get_history()
    _say("stats", st, ratio)
    assert st["adaptive_steps"] == 3 and st["steps_at_cap"] == 3
    assert abs(st["max_ratio"] - ratio.max()) < 1e-6 * ratio.max()
    assert abs(st["mean_ratio"] - ratio.mean()) < 1e-6 * ratio.mean()


# ------------------------------------------------ Algorithm 1 with the lag
def _alg1(n=64, lag=1):
    M = P.Manufactured(n, alpha=0.9, r=0.5, K=1, ne_fixed=4, levels=1)
    f, s = M.loads(0.3)
    return M.problem.replace(gamma=1.0, lag=lag, body_f=f, source_s=s, name=f"alg1_lag{lag}_{n}")


@pytest.mark.parametrize("lag", [1, 0])
def test_algorithm1_steps_match_oracle(lbm, lag):
    """Plain pseudo-time stepping (one level, gamma = 1, eight applications
    per step), with and without the lag, on the periodic problem and on the
    mixed walls."""
    _steps_match(lbm, _alg1(64, lag), 3, label="alg1")
    q = mixed_walls(124, 68, seed=3).replace(levels=1, gamma=1.0, K=1, ne_fixed=3, lag=lag)
    _steps_match(lbm, q, 3, label="alg1 walls")


def test_algorithm1_lagged_cycle_from_a_given_iterate(lbm):
    p = _alg1(64, 1).replace(K=2)
    s = lbm.Solver(p, "fp64")
    o = Oracle(p, threads=oracle_threads())
    f, g, d1, d2 = P.random_state(p, 12, scale=1e-2)
    o.set_state(f, g, d1, d2, step=2)
    s.set_state(f, g, d1, d2, step=2)
    Ft = o.explicit_force()
    ga, gb = s.mg_cycle(1, g, None, Ft), o.mg_cycle(1, g, None, Ft)
    s.close()
    assert np.abs(ga - gb).max() < 1e-12 * np.abs(gb).max()


# ------------------------------------------------------------ divergence
def _diverging():
    """Sec. 4.1: the explicit coupling (r = 0) with MG(4,2) is unstable at
    alpha = 0.9; with the loads frozen at t = 1/2 the norm of the elastic
    populations passes 1e8 times its first value after about 50 steps."""
    M = P.Manufactured(32, alpha=0.9, r=0.0, K=2, ne_fixed=4)
    f, s = M.loads(0.5)
    return M.problem.replace(body_f=f, source_s=s, name="diverging")


def test_batch_evicts_a_diverging_member(lbm):
    stable = P.loaded_strip(n=32, alpha=0.9, K=2, ne_fixed=4)
    probs = [_diverging(), stable]
    b = lbm.Batch(probs, "fp64")
    b.step(80)
    with pytest.raises(lbm.BiotError) as ei:
        b.fields(0)
    assert ei.value.code == lbm.BP_ERR_DIVERGED
    A = b.fields(1)
    b.close()
    s = lbm.Solver(stable, "fp64")
    s.step(80)
    B = s.fields()
    s.close()
    _say("evicted; neighbour", rel(A["eta"], B["eta"]))
    assert np.array_equal(A["eta"], B["eta"]) and np.array_equal(A["p"], B["p"])


def test_server_fails_a_diverging_request_early(lbm):
    srv = lbm.Server(256 << 20, prec="fp64", K=2, ne_fixed=4, max_slots=4)
    stable = P.loaded_strip(n=32, alpha=0.9, K=2, ne_fixed=4)
    tb = srv.submit(_diverging(), 400)
    ts = srv.submit(stable, 100)
    states = None
    for _ in range(30):
        srv.advance(8)
        states = (srv.poll(tb), srv.poll(ts))
        if states[0][0] == 3 and states[1][0] == 2:
            break
    _say("server states", states)
    assert states[0][0] == 3 and states[0][1] < 400      # failed before its step count
    with pytest.raises(lbm.BiotError) as ei:
        srv.result(tb)
    assert ei.value.code == lbm.BP_ERR_DIVERGED
    A = srv.result(ts)
    srv.close()
    s = lbm.Solver(stable, "fp64")
    s.step(100)
    B = s.fields()
    s.close()
    assert np.array_equal(A["eta"], B["eta"]) and np.array_equal(A["p"], B["p"])


def test_lone_solver_reports_divergence(lbm):
    s = lbm.Solver(_diverging(), "fp64")
    s.step(80)
    with pytest.raises(lbm.BiotError) as ei:
        s.fields()
    assert ei.value.code == lbm.BP_ERR_DIVERGED
    assert s.stats()["diverged"] == 1
    s.close()


# ---------------------------------------------------------------- schedules
@pytest.mark.parametrize("prec", ["fp64", "fp32_shifted"])
def test_merged_coarse_tails_equal_the_tails_at_their_own_depths(lbm, prec, monkeypatch):
    """A batch whose problems' coarse tails start at three depths runs them in
    one launch where the V-cycle turns; with BIOT_NO_MERGE_TAIL=1 each depth
    launches its own.  Independent problems, the same kernels: bitwise equal."""
    probs = [P.loaded_strip(n=64, alpha=0.7, ne_fixed=3), P.loaded_strip(n=128, nu=0.4, ne_fixed=3),
             P.loaded_strip(n=256, alpha=0.5, ne_fixed=3)]
    out = []
    for merge in (True, False):
        if merge:
            monkeypatch.delenv("BIOT_NO_MERGE_TAIL", raising=False)
        else:
            monkeypatch.setenv("BIOT_NO_MERGE_TAIL", "1")
        _say("merged tails" if merge else "tails per depth", prec)
        b = lbm.Batch(probs, prec)
        b.step(4)
        out.append([b.fields(i) for i in range(len(probs))])
        b.close()
    for A, B in zip(*out):
        assert np.array_equal(A["eta"], B["eta"]) and np.array_equal(A["p"], B["p"])


@pytest.mark.parametrize("prec", ["fp64", "fp32_shifted"])
def test_fixed_steps_in_one_call_equal_steps_one_at_a_time(lbm, prec):
    """A call of at least four fixed-cycle steps replays a graph of four
    steps (then single steps for the rest); steps taken one call at a time
    replay the one-step graph.  The same launches in the same order: bitwise
    equal fields, step numbers and cycle counts after 4 + 4 + 3 steps."""
    p = P.loaded_strip(n=128, alpha=1.0, ne_fixed=3, K=4)
    a, b = lbm.Solver(p, prec), lbm.Solver(p, prec)
    a.step(11)
    for _ in range(11):
        b.step(1)
    A, B = a.fields(), b.fields()
    sa, sb = a.stats(), b.stats()
    _say("four-step graph", prec, sa["step"], sa["total_cycles"], sb["step"], sb["total_cycles"])
    assert sa["step"] == sb["step"] == 11 and sa["total_cycles"] == sb["total_cycles"] == 33
    assert np.array_equal(A["eta"], B["eta"]) and np.array_equal(A["p"], B["p"])
    assert np.array_equal(A["sigma"], B["sigma"])
    a.close()
    b.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32_shifted"])
@pytest.mark.parametrize("tol", [1e-6, 1e-10])
def test_adaptive_steps_in_one_call_equal_steps_one_at_a_time(lbm, prec, tol):
    """Within one bp_step call the adaptive schedule enqueues the flow step and
    the next step's first cycle before it reads the stopping test, gated on a
    normal stop; steps taken one call at a time read first.  Same launches in
    the same order on the device: bitwise equal fields and the same cycle
    counts, including steps whose count differs from the one before."""
    p = P.loaded_strip(n=64, alpha=1.0, ne_fixed=0, ne_tol=tol, ne_max=20)
    a, b = lbm.Solver(p, prec), lbm.Solver(p, prec)
    a.step(8)
    ne = []
    for _ in range(8):
        b.step(1)
        ne.append(b.stats()["last_ne"])
    A, B = a.fields(), b.fields()
    sa, sb = a.stats(), b.stats()
    _say("pipelined", prec, tol, ne, sa["total_cycles"], sb["total_cycles"])
    assert sa["total_cycles"] == sb["total_cycles"] and sa["last_ne"] == sb["last_ne"]
    assert np.array_equal(A["eta"], B["eta"]) and np.array_equal(A["p"], B["p"])
    a.close()
    b.close()
    # the finest level of 64^2 runs four applications per launch, the first
    # with the restriction: its test sums that launch's partials; the counts
    # are the oracle's own decisions
    if prec == "fp64":
        o = Oracle(p, threads=oracle_threads(), history=8)
        o.step(8)
        ne_o, _ = o.get_history()
        assert ne == list(ne_o), (ne, list(ne_o))
        assert rel(A["eta"], o.fields()["eta"]) < STEP_TOL and rel(A["p"], o.fields()["p"]) < STEP_TOL


def test_adaptive_test_on_four_application_launches_follows_oracle(lbm):
    """A finest level swept four applications at a time, the first launch
    with the restriction in its 64 x 32 region (above 128^2 cells): the
    stopping test sums that launch's partials, and the counts are the
    oracle's own decisions at 1e-10 on the fields."""
    p = mixed_walls(200, 152, seed=7).replace(K=4, ne_fixed=0, ne_tol=1e-6, ne_max=20)
    s = lbm.Solver(p, "fp64")
    ne = []
    for _ in range(4):
        s.step(1)
        ne.append(s.stats()["last_ne"])
    o = Oracle(p, threads=oracle_threads(), history=4)
    o.step(4)
    ne_o, _ = o.get_history()
    _say("four-application adaptive", ne, list(ne_o))
    assert ne == list(ne_o)
    A, B = s.fields(), o.fields()
    assert rel(A["eta"], B["eta"]) < STEP_TOL and rel(A["p"], B["p"]) < STEP_TOL
    s.close()
