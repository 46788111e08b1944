"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle.

Bars: single operations 1e-13 relative, whole FP64 steps 1e-10 relative
(element-wise over all cells), FP32 paths 1e-5 relative L2 for eta and p.
"""
import sys

import numpy as np
import pytest

from conftest import oracle_threads
from gpu_helpers import mixed_walls, problems_small, rel, tail_level
from oracle.oracle import Oracle
from paper_2409_11382_amd import problem as P

pytestmark = pytest.mark.gpu

OP_TOL = 1e-13
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


def _rand_state(p, seed):
    f, g, d1, d2 = P.random_state(p, seed, scale=1e-2)
    return f, g, d1, d2


@pytest.mark.parametrize("name", list(problems_small().keys()))
def test_apply_elastic_every_level(lbm, name):
    p = problems_small()[name]
    _say("apply_elastic", name, p.nx, p.ny)
    s = lbm.Solver(p, "fp64")
    o = Oracle(p, threads=oracle_threads())
    L = o.levels
    rng = np.random.default_rng(7)
    for level in range(L, 0, -1):
        nx, ny = o.level_shape(level)
        assert s.level_shape(level) == (nx, ny)
        g = rng.standard_normal((8, ny, nx))
        if level == L:
            Ft = rng.standard_normal((2, ny, nx)) * 0.1
            a = s.apply_elastic(level, g, None, Ft)
            b = o.apply_elastic(level, g, None, Ft)
        else:
            r = rng.standard_normal((8, ny, nx)) * 0.1
            a = s.apply_elastic(level, g, r, None)
            b = o.apply_elastic(level, g, r, None)
        err = np.abs(a - b).max() / np.abs(b).max()
        _say("  level", level, (nx, ny), "max rel", err)
        assert err < OP_TOL


@pytest.mark.parametrize("name", list(problems_small().keys()))
def test_vcycle_and_force(lbm, name):
    p = problems_small()[name]
    _say("vcycle", name)
    s = lbm.Solver(p, "fp64")
    o = Oracle(p, threads=oracle_threads())
    f, g, d1, d2 = _rand_state(p, 11)
    o.set_state(f, g, d1, d2, step=5)
    s.set_state(f, g, d1, d2, step=5)
    Fa, Fb = s.explicit_force(), o.explicit_force()
    _say("  force rel", rel(Fa, Fb))
    assert np.abs(Fa - Fb).max() <= OP_TOL * np.abs(Fb).max()
    L = o.levels
    ga = s.mg_cycle(L, g, None, Fb)
    gb = o.mg_cycle(L, g, None, Fb)
    err = np.abs(ga - gb).max() / np.abs(gb).max()
    _say("  vcycle max rel", err)
    assert err < 1e-12


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("name", ["terzaghi_8x128", "mixed_124x68", "periodic_64"])
def test_tail_cycle(lbm, name, prec):
    """The coarse levels that one workgroup runs per problem: a V-cycle from a
    zero iterate on the tail's top level against the oracle's cycle."""
    p = problems_small()[name]
    s = lbm.Solver(p, prec)
    o = Oracle(p, threads=oracle_threads())
    shapes = [s.level_shape(l) for l in range(1, o.levels + 1)]
    lt = tail_level(shapes, prec)
    _say("tail", name, prec, "top level", lt, shapes[lt - 1] if lt else None)
    assert lt >= 1
    nx, ny = shapes[lt - 1]
    rng = np.random.default_rng(23)
    r = rng.standard_normal((8, ny, nx)) * 0.1
    g0 = np.zeros((8, ny, nx))
    ga = s.mg_cycle(lt, g0.copy(), r, None)
    gb = o.mg_cycle(lt, g0.copy(), r, None)
    err = np.abs(ga - gb).max() / np.abs(gb).max()
    _say("  tail cycle max rel", err)
    assert err < (1e-12 if prec == "fp64" else 2e-5)


def _compare_steps(lbm, p, nsteps, prec="fp64", loads=None, tol=STEP_TOL, check_every=None):
    s = lbm.Solver(p, prec)
    o = Oracle(p, threads=oracle_threads())
    if loads is not None:
        f0, s0 = loads(0.0)
        o.set_loads(f0, s0, reinit=True)
        s.set_loads(f0, s0, reinit=True)
    worst = 0.0
    for k in range(nsteps):
        if loads is not None and k > 0:
            fk, sk = loads(k * p.dt)
            o.set_loads(fk, sk)
            s.set_loads(fk, sk)
        o.step(1)
        s.step(1)
        if check_every and (k + 1) % check_every == 0 or k == nsteps - 1:
            A, B = s.fields(), o.fields()
            e = max(rel(A["eta"], B["eta"]), rel(A["p"], B["p"]), rel(A["sigma"], B["sigma"]))
            worst = max(worst, e)
            assert e < tol, (k, rel(A["eta"], B["eta"]), rel(A["p"], B["p"]), rel(A["sigma"], B["sigma"]))
    return worst, s, o


@pytest.mark.parametrize("name", list(problems_small().keys()))
def test_fp64_steps_match_oracle(lbm, name):
    p = problems_small()[name]
    _say("fp64 steps", name)
    worst, s, o = _compare_steps(lbm, p, 6, check_every=2)
    A, B = s.fields(), o.fields()
    # element-wise bar on every cell as well
    scale = np.abs(B["eta"]).max()
    assert np.abs(A["eta"] - B["eta"]).max() <= STEP_TOL * scale
    assert np.abs(A["p"] - B["p"]).max() <= STEP_TOL * np.abs(B["p"]).max()
    _say("  worst rel", worst)


@pytest.mark.parametrize("r,alpha", [(0.5, 1.0), (0.0, 0.5), (1.0, 0.7)])
def test_manufactured_time_dependent_loads(lbm, r, alpha):
    """Sec. 4.1's periodic problem with its time-dependent body force and
    source, for the centred, explicit and implicit couplings (each at a
    coupling strength the section reports stable)."""
    M = P.Manufactured(32, alpha=alpha, r=r, K=2, ne_fixed=3)
    worst, _, _ = _compare_steps(lbm, M.problem, 12, loads=M.loads, check_every=3)
    _say("manufactured r", r, "worst rel", worst)


@pytest.mark.parametrize("alpha", [0.8, 1.0])
def test_terzaghi_paper_parameters(lbm, alpha):
    """Sec. 4.2's Terzaghi parameters (E = 1, nu = 0.8, p0 = 1) with MG(3,4)."""
    p = P.terzaghi_paper(alpha, 64, nx=8, K=4)
    worst, _, _ = _compare_steps(lbm, p, 10, check_every=5)
    _say("terzaghi paper alpha", alpha, "worst rel", worst)


@pytest.mark.parametrize("prec,tol", [("fp64", STEP_TOL), ("fp32_shifted", 1e-5)])
def test_plain_pseudo_time_stepping(lbm, prec, tol):
    """Algorithm 1 (no multigrid): one level, gamma = 1, 16 plain elastic steps
    per time step."""
    p = P.loaded_strip(n=64, alpha=0.8, ne_fixed=8).replace(levels=1, gamma=1.0, K=1)
    worst, _, _ = _compare_steps(lbm, p, 4, prec=prec, tol=tol)
    _say("plain pseudo-time", prec, worst)


def test_central_pressure_gradient_variant(lbm):
    """Eq. pressure:gradient:alternative in the explicit force: the periodic
    manufactured problem with time-dependent loads, and a walled problem (the
    gradient's ghost values reflect at walls) in FP64 and FP32 shifted."""
    M = P.Manufactured(32, alpha=1.0, r=0.5, K=2, ne_fixed=3)
    pm = M.problem.replace(pressure_gradient=P.GRAD_CENTRAL)
    worst, _, _ = _compare_steps(lbm, pm, 9, loads=M.loads, check_every=3)
    _say("central gradient, periodic", worst)
    pw = mixed_walls(124, 68, seed=4).replace(pressure_gradient=P.GRAD_CENTRAL, ne_fixed=3, K=4)
    worst, _, _ = _compare_steps(lbm, pw, 6, check_every=3)
    _say("central gradient, walls fp64", worst)
    ps = P.loaded_strip(n=128, alpha=1.0, ne_fixed=3).replace(pressure_gradient=P.GRAD_CENTRAL)
    worst, _, _ = _compare_steps(lbm, ps, 20, prec="fp32_shifted", tol=1e-5)
    _say("central gradient, strip fp32 shifted", worst)


def _adaptive_run(lbm, p, prec, nsteps):
    s = lbm.Solver(p, prec)
    ne = []
    for _ in range(nsteps):
        s.step(1)
        ne.append(s.stats()["last_ne"])
    F = s.fields()
    s.close()
    return ne, F


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("cyc", [P.CYCLE_V, P.CYCLE_W])
def test_whole_problem_tail_in_adaptive_cycles(lbm, monkeypatch, prec, cyc):
    """A problem whose finest level fits one workgroup (32 x 32) runs every
    adaptive cycle after the stopping test as one launch: the finest level's
    sweeps with the explicit force and the wall data of Dirichlet, traction
    and symmetry walls, then the coarse levels.  Against the tile schedule
    (BIOT_NO_FULL_TAIL=1) and, in FP64, the oracle replaying the cycle counts."""
    n = 32
    yy, xx = np.mgrid[0:n, 0:n] / n
    body = np.stack([0.3 * np.sin(2 * np.pi * yy), 0.2 * np.cos(np.pi * xx)])
    p = mixed_walls(n, n, seed=5).replace(ne_fixed=0, ne_tol=1e-7, ne_max=30, K=3, cycle=cyc, body_f=body)
    ne, A = _adaptive_run(lbm, p, prec, 5)
    monkeypatch.setenv("BIOT_NO_FULL_TAIL", "1")
    ne_t, B = _adaptive_run(lbm, p, prec, 5)
    d = (rel(A["eta"], B["eta"]), rel(A["p"], B["p"]), rel(A["sigma"], B["sigma"]))
    _say("whole-problem tail", prec, cyc, ne, ne_t, d)
    if prec == "fp64":
        assert ne == ne_t and max(d) < 1e-12, (ne, ne_t, d)
        o = Oracle(p, threads=oracle_threads(), history=5)
        o.set_ne_schedule(np.array(ne, dtype=np.int32))
        o.step(5)
        C = o.fields()
        e = (rel(A["eta"], C["eta"]), rel(A["p"], C["p"]), rel(A["sigma"], C["sigma"]))
        _say("  vs oracle", e)
        assert max(e) < STEP_TOL, e
    else:
        assert max(d) < 1e-4, d


def test_adaptive_cycles_shifted_and_large(lbm):
    """The adaptive schedule where the finest level of 512^2 runs single
    applications after the measuring sweep and the coarser depths fused
    launches (the oracle replays the GPU's counts), and in shifted storage:
    FP64 shifted takes the plain FP64 counts and fields, FP32 shifted stays
    within 1e-5 of the oracle replaying its counts."""
    p = P.loaded_strip(n=512, alpha=1.0, ne_fixed=0, ne_tol=1e-6, ne_max=20)
    ne, A = _adaptive_run(lbm, p, "fp64", 2)
    _say("adaptive 512 fp64 N_E", ne)
    o = Oracle(p, threads=oracle_threads(), history=2)
    o.set_ne_schedule(np.array(ne, dtype=np.int32))
    o.step(2)
    B = o.fields()
    assert rel(A["eta"], B["eta"]) < STEP_TOL and rel(A["p"], B["p"]) < STEP_TOL
    q = mixed_walls(124, 68, seed=3).replace(ne_fixed=0, ne_tol=1e-7, ne_max=30)
    n64, F64 = _adaptive_run(lbm, q, "fp64", 6)
    n64s, F64s = _adaptive_run(lbm, q, "fp64_shifted", 6)
    _say("adaptive mixed N_E fp64", n64, "fp64 shifted", n64s)
    assert n64 == n64s
    assert rel(F64s["eta"], F64["eta"]) < 1e-12 and rel(F64s["p"], F64["p"]) < 1e-12
    n32, F32 = _adaptive_run(lbm, q, "fp32_shifted", 6)
    o = Oracle(q, threads=oracle_threads(), history=6)
    o.set_ne_schedule(np.array(n32, dtype=np.int32))
    o.step(6)
    C = o.fields()
    e = (rel(F32["eta"], C["eta"]), rel(F32["p"], C["p"]))
    _say("adaptive mixed fp32 shifted N_E", n32, e)
    assert max(e) < 1e-5


def test_adaptive_cycles_follow_oracle(lbm):
    """Configuration 1 (Terzaghi 8x128, tolerance 1e-8, at most 50 cycles): the
    GPU's V-cycle counts are replayed by the oracle; the oracle's own adaptive
    decisions agree except at near-ties of the residual ratio."""
    p = P.terzaghi(ne_fixed=0, ne_tol=1e-8, ne_max=50)
    nsteps = 12
    s = lbm.Solver(p, "fp64")
    ne = []
    for _ in range(nsteps):
        s.step(1)
        ne.append(s.stats()["last_ne"])
    _say("gpu N_E", ne)
    o = Oracle(p.replace(ne_fixed=0), threads=oracle_threads(), history=nsteps)
    o.set_ne_schedule(np.array(ne, dtype=np.int32))
    o.step(nsteps)
    A, B = s.fields(), o.fields()
    assert rel(A["eta"], B["eta"]) < STEP_TOL and rel(A["p"], B["p"]) < STEP_TOL
    # a tighter tolerance that the cycles do reach
    p2 = P.terzaghi(nx=8, ny=32, ne_fixed=0, ne_tol=1e-6, ne_max=40)
    s2 = lbm.Solver(p2, "fp64")
    ne2 = []
    for _ in range(8):
        s2.step(1)
        ne2.append(s2.stats()["last_ne"])
    o2 = Oracle(p2, threads=1, history=8)
    o2.step(8)
    ne_o, ratio_o = o2.get_history()
    _say("gpu", ne2, "oracle", list(ne_o))
    assert ne2 == list(ne_o)
    assert rel(s2.fields()["eta"], o2.fields()["eta"]) < STEP_TOL


def test_zero_load_is_exactly_zero_on_gpu(lbm):
    for prec in ("fp64", "fp32", "fp32_shifted"):
        p = P.loaded_strip(n=64, load=0.0, ne_fixed=2)
        s = lbm.Solver(p, prec)
        s.step(4)
        F = s.fields()
        assert not np.any(F["eta"]) and not np.any(F["p"]) and not np.any(F["sigma"]), prec


def test_shifted_fp64_equals_plain_fp64(lbm):
    p = mixed_walls(124, 68, seed=5)
    a = lbm.Solver(p, "fp64")
    b = lbm.Solver(p, "fp64_shifted")
    a.step(8)
    b.step(8)
    A, B = a.fields(), b.fields()
    _say("shift rel", rel(B["eta"], A["eta"]), rel(B["p"], A["p"]))
    assert rel(B["eta"], A["eta"]) < 1e-13 and rel(B["p"], A["p"]) < 1e-12


def test_fp32_shifted_with_fp64_references(lbm, monkeypatch):
    """FP32 shifted storage with its references in FP64 (the library's choice
    on grids above 4096^2 cells; forced here) on mixed boundaries and with
    the re-bases between cycles, against the oracle."""
    monkeypatch.setenv("BIOT_REF64", "1")
    p = mixed_walls(124, 68, seed=7).replace(ne_fixed=3, K=4)
    s = lbm.Solver(p, "fp32_shifted")
    s.step(6)
    A = s.fields()
    s.close()
    o = Oracle(p, threads=oracle_threads())
    o.step(6)
    B = o.fields()
    e = (rel(A["eta"], B["eta"]), rel(A["p"], B["p"]), rel(A["sigma"], B["sigma"]))
    _say("fp32 shifted, FP64 references", e)
    assert max(e) < 1e-5


def test_batch_mixed_reference_precisions(lbm, monkeypatch):
    """One batch whose FP32 shifted problems keep their references in
    different precisions (FP64 above a cell count, lowered here to 96^2): its
    launches read either precision per problem.  Every problem matches the
    oracle and, to rounding, the same problem run alone."""
    monkeypatch.setenv("BIOT_REF64_CELLS", str(96 * 96))
    probs = [mixed_walls(124, 68, seed=7).replace(ne_fixed=3, K=4),   # FP32 references
             mixed_walls(128, 96, seed=3).replace(ne_fixed=3, K=4),   # FP64 references
             P.loaded_strip(n=64, alpha=1.0, ne_fixed=3)]             # FP32 references
    b = lbm.Batch(probs, "fp32_shifted")
    b.step(6)
    for i, p in enumerate(probs):
        B = b.fields(i)
        s = lbm.Solver(p, "fp32_shifted")
        s.step(6)
        A = s.fields()
        s.close()
        o = Oracle(p, threads=oracle_threads())
        o.step(6)
        C = o.fields()
        d = (rel(B["eta"], A["eta"]), rel(B["p"], A["p"]))
        e = (rel(B["eta"], C["eta"]), rel(B["p"], C["p"]), rel(B["sigma"], C["sigma"]))
        _say("mixed references", i, p.nx, p.ny, d, e)
        assert max(d) < 1e-6 and max(e) < 1e-5, (i, d, e)


@pytest.mark.parametrize("K,ne", [(3, 4), (2, 2), (4, 5)])
def test_shifted_rebase_schedules(lbm, K, ne):
    """Shifted storage re-bases between V-cycles inside the cycle's last
    finest-level launch for an even number of boundaries and with the
    re-basing kernel for the rest: odd K (that launch is a pair after a single
    application), even and odd N_E.  FP64 shifted equals plain FP64 to
    rounding; FP32 shifted stays within 1e-5."""
    p = mixed_walls(124, 68, seed=5).replace(K=K, ne_fixed=ne)
    F = {}
    for prec in ("fp64", "fp64_shifted", "fp32_shifted"):
        s = lbm.Solver(p, prec)
        s.step(4)
        F[prec] = s.fields()
        s.close()
    A = F["fp64"]
    d64 = (rel(F["fp64_shifted"]["eta"], A["eta"]), rel(F["fp64_shifted"]["p"], A["p"]))
    d32 = (rel(F["fp32_shifted"]["eta"], A["eta"]), rel(F["fp32_shifted"]["p"], A["p"]))
    _say("rebase schedule K", K, "N_E", ne, d64, d32)
    assert max(d64) < 1e-12 and max(d32) < 1e-5


@pytest.mark.parametrize("prec,tol", [("fp32_shifted", 1e-5), ("fp32", 1e-2)])
def test_fp32_paths_against_fp64_oracle(lbm, prec, tol):
    """FP32 with shifted storage must stay within 1e-5 of the FP64 oracle.  Plain
    FP32 is the ablation: the stress moments cancel against the displacement
    equilibrium and lose about log10(N) digits; it is only bounded here."""
    p = P.loaded_strip(n=128, alpha=1.0, ne_fixed=3)
    nsteps = 40
    s = lbm.Solver(p, prec)
    o = Oracle(p, threads=oracle_threads())
    s.step(nsteps)
    o.step(nsteps)
    A, B = s.fields(), o.fields()
    e_eta, e_p = rel(A["eta"], B["eta"]), rel(A["p"], B["p"])
    _say(prec, "rel eta", e_eta, "rel p", e_p)
    assert e_eta < tol and e_p < tol


def test_determinism_and_mirror_symmetry(lbm):
    p = P.loaded_strip(n=256, alpha=1.0, ne_fixed=3)
    a = lbm.Solver(p, "fp64")
    b = lbm.Solver(p, "fp64")
    a.step(5)
    b.step(5)
    A, B = a.fields(), b.fields()
    assert np.array_equal(A["eta"], B["eta"]) and np.array_equal(A["p"], B["p"])
    assert np.abs(A["eta"][0] + A["eta"][0][:, ::-1]).max() < 1e-10 * np.abs(A["eta"]).max()
    assert np.abs(A["p"] - A["p"][:, ::-1]).max() < 1e-10 * np.abs(A["p"]).max()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32_shifted", 1e-4)])
def test_layered_permeability_steady_state(lbm, prec, tol):
    """Heterogeneous permeability: the GPU's steady flow through random
    horizontal layers is the continuum's series-resistance solution (one flux
    through every layer), to rounding in FP64.  In FP32 the fixed point of the
    iteration carries about eps_32 / (1 - rho) of rounding, with 1 / (1 - rho)
    ~ N^2 / (pi^2 k_min) ~ 1e3 for 32 rows and a lattice diffusivity of 0.1:
    the bar is 1e-4 (measured 1e-5)."""
    from oracle import analytic as An

    p = P.layered_column()
    s = lbm.Solver(p, prec)
    s.step(16000)
    F = s.fields()["p"]
    s.close()
    pc = An.layered_steady_pressure(p.kappa[:, 0], p.dx)
    e = np.abs(F - pc[:, None]).max()
    _say("layered steady state", prec, e)
    assert e < tol


def test_checkpoint_resume_is_bitwise(lbm):
    p = P.loaded_strip(n=64, alpha=0.8, ne_fixed=3)
    a = lbm.Solver(p, "fp64")
    a.step(6)
    st = a.get_state()
    a.step(4)
    b = lbm.Solver(p, "fp64")
    b.set_state(st["f"], st["g"], st["D1"], st["D2"], step=st["step"])
    b.step(4)
    A, B = a.fields(), b.fields()
    assert np.array_equal(A["eta"], B["eta"]) and np.array_equal(A["p"], B["p"])


@pytest.mark.parametrize("ref64", ["0", "1"])
@pytest.mark.parametrize("nsteps", [5, 6])
def test_checkpoint_shifted_storage(lbm, monkeypatch, ref64, nsteps):
    """FP32 shifted storage, FP32 and FP64 references, a checkpoint after an
    odd and an even number of steps (the pressure reference alternates
    between two buffers by step parity).  A restored state is split into
    references and offsets in FP64, so the round trip keeps what FP32 full
    populations would round away: on a state with a displacement and
    pressure of 1e3 (equilibria of ~300) it returns g and f within 1e-6 (FP32
    full populations would lose ~2e-5).  A run resumed from a checkpoint
    follows the uninterrupted run to rounding."""
    monkeypatch.setenv("BIOT_REF64", ref64)
    p = P.loaded_strip(n=64, alpha=0.8, ne_fixed=3)
    a = lbm.Solver(p, "fp32_shifted")
    a.step(nsteps)
    st = a.get_state()
    a.step(4)
    b = lbm.Solver(p, "fp32_shifted")
    b.set_state(st["f"], st["g"], st["D1"], st["D2"], step=st["step"])
    b.step(4)
    A, B = a.fields(), b.fields()
    d = (rel(B["eta"], A["eta"]), rel(B["p"], A["p"]))
    # a large rigid displacement and pressure offset on top of the state
    E, P0 = 1e3, 1e3
    w8 = np.array([1 / 3, 1 / 3, 1 / 3, 1 / 3, 1 / 12, 1 / 12, 1 / 12, 1 / 12])
    c8 = np.array([[1, 0], [0, 1], [-1, 0], [0, -1], [1, 1], [-1, 1], [-1, -1], [1, -1]])
    w9 = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    g = st["g"] + (w8 * (c8[:, 0] * E + c8[:, 1] * E))[:, None, None]
    f = st["f"] + (w9 * P0)[:, None, None]
    b.set_state(f, g, st["D1"], st["D2"], step=st["step"])
    rt = b.get_state()
    eg, ef = np.abs(rt["g"] - g).max(), np.abs(rt["f"] - f).max()
    _say("checkpoint shifted ref64", ref64, "steps", nsteps, d, "round trip", eg, ef)
    assert max(d) < 1e-6, d
    assert eg < 1e-6 and ef < 1e-6, (eg, ef)
    a.close()
    b.close()


def test_full_size_loaded_strip_512(lbm):
    """The benchmarked workload (loaded strip 512 x 512, alpha = 1, MG(3,4)) at
    its real size for a few steps, FP64 against the oracle, plus the FP32
    shifted path's error."""
    p = P.loaded_strip(n=512, alpha=1.0, ne_fixed=3)
    nsteps = 3
    o = Oracle(p, threads=oracle_threads())
    o.step(nsteps)
    B = o.fields()
    for prec, tol in (("fp64", STEP_TOL), ("fp32_shifted", 1e-5)):
        s = lbm.Solver(p, prec)
        s.step(nsteps)
        A = s.fields()
        e = (rel(A["eta"], B["eta"]), rel(A["p"], B["p"]), rel(A["sigma"], B["sigma"]))
        _say("512", prec, e)
        assert e[0] < tol and e[1] < tol


@pytest.mark.parametrize("shape", [(2, 2, 1), (4, 4, 2), (2, 8, 1), (8, 2, 1), (6, 6, 1)])
def test_smallest_grids_match_oracle(lbm, shape):
    """Grids of a few cells with every boundary type (one level, or two down
    to 2 x 2): every cell is a wall cell and most tiles are mostly empty.
    Three coupled steps against the oracle."""
    nx, ny, levels = shape
    p = mixed_walls(nx, ny, seed=9, levels=levels).replace(kappa=0.7, name=f"tiny_{nx}x{ny}")
    o = Oracle(p, threads=1)
    o.step(3)
    B = o.fields()
    for prec, tol in (("fp64", STEP_TOL), ("fp32_shifted", 1e-5)):
        s = lbm.Solver(p, prec)
        s.step(3)
        A = s.fields()
        s.close()
        e = (rel(A["eta"], B["eta"]), rel(A["p"], B["p"]))
        _say("tiny", shape, prec, e)
        assert e[0] < tol and e[1] < tol, (shape, prec, e)


def test_zero_steps_leave_the_initial_state(lbm):
    """No step: the fields are the initial conditions (zero) at step 0; a
    negative count is refused and leaves the solver usable; two steps after
    that equal two steps of a fresh solver bitwise."""
    p = P.loaded_strip(n=64, ne_fixed=2)
    a, b = lbm.Solver(p, "fp32_shifted"), lbm.Solver(p, "fp32_shifted")
    a.step(0)
    F, st = a.fields(), a.stats()
    assert st["step"] == 0 and st["total_cycles"] == 0
    assert not np.any(F["eta"]) and not np.any(F["p"]) and not np.any(F["sigma"])
    with pytest.raises(lbm.BiotError):
        a.step(-1)
    a.step(2)
    b.step(2)
    A, B = a.fields(), b.fields()
    assert np.array_equal(A["eta"], B["eta"]) and np.array_equal(A["p"], B["p"])
    a.close()
    b.close()


def test_invalid_problems_rejected(lbm):
    base = P.loaded_strip(n=16)
    for bad in (dict(c0=0.0), dict(alpha=1.5), dict(gamma=1.5), dict(levels=6)):
        with pytest.raises(lbm.BiotError):
            lbm.Solver(base.replace(**bad))


def _batch_against_alone(lbm, probs, prec, bitwise):
    b = lbm.Batch(probs, prec)
    b.step(5)
    for i, p in enumerate(probs):
        s = lbm.Solver(p, prec)
        s.step(5)
        A, B = s.fields(), b.fields(i)
        d = (rel(B["eta"], A["eta"]), rel(B["p"], A["p"]))
        _say("batch", i, p.name, d)
        if bitwise:
            assert np.array_equal(A["eta"], B["eta"]) and np.array_equal(A["p"], B["p"]), (i, p.name)
        else:
            assert max(d) < (1e-6 if prec == "fp32_shifted" else 1e-12), (i, p.name, d)
        if prec == "fp64":
            o = Oracle(p, threads=oracle_threads())
            o.step(5)
            assert rel(B["eta"], o.fields()["eta"]) < STEP_TOL


@pytest.mark.parametrize("prec", ["fp64", "fp32_shifted"])
def test_batch_alone_equals_in_mix(lbm, prec):
    """Problems of different sizes, hierarchy depths, parameters and boundary
    types advanced together give bitwise the same fields as each alone: every
    depth of this mix holds at most 128^2 cells in all, as every problem alone
    does, so each keeps its launch variants."""
    probs = [P.loaded_strip(n=64, alpha=0.7, kappa=0.3, ne_fixed=3),
             mixed_walls(100, 60, seed=9).replace(ne_fixed=3, K=4),
             P.terzaghi(nx=16, ny=64, ne_fixed=3),
             P.loaded_strip(n=32, ny=96, alpha=0.5, ne_fixed=3),
             P.loaded_strip(n=32, ny=64, nu=0.4, alpha=1.0, ne_fixed=3)]
    assert sum(p.nx * p.ny for p in probs) <= 128 * 128
    _batch_against_alone(lbm, probs, prec, bitwise=True)


@pytest.mark.parametrize("prec", ["fp64", "fp32_shifted"])
def test_batch_alone_close_in_larger_mix(lbm, prec):
    """A mix whose finest depth holds more than 128^2 cells in all: there the
    four-application launch with the restriction takes its 64-column form, the
    problems alone the 32-column one.  Same arithmetic, separately compiled:
    equal to rounding (FP64 also agrees with the oracle element-wise)."""
    probs = [P.loaded_strip(n=64, alpha=0.7, kappa=0.3, ne_fixed=3),
             P.loaded_strip(n=128, nu=0.4, alpha=1.0, ne_fixed=3),
             mixed_walls(124, 68, seed=9).replace(ne_fixed=3, K=4),
             P.terzaghi(nx=16, ny=64, ne_fixed=3),
             P.loaded_strip(n=32, ny=96, alpha=0.5, ne_fixed=3)]
    assert sum(p.nx * p.ny for p in probs) > 128 * 128
    _batch_against_alone(lbm, probs, prec, bitwise=False)