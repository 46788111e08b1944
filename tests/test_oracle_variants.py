"""Pins of the oracle's switchable variants.

* the self-dependence constant of eq. MG:selfdependence as printed
  (alpha^2/2 for every r) against the default r alpha^2/2;
* the coarsest level's own number of smoothing steps;
* full multigrid (named as future work in the conclusion, not defined there);
* Algorithm 1 with the lag of eq. source:implicit, and the cost scaling of
  plain pseudo-time stepping that Sec. 4.1 reports.

Each test checks a fact that follows from the definition (a special case that
reduces to another pinned operation, a composition by hand from the pinned
single operations, a brute-force solve) or a statement of the paper.
"""
import functools

import numpy as np
import pytest

from conftest import oracle_threads
from oracle import analytic as A
from oracle.oracle import Oracle, OracleError, run
from paper_2409_11382_amd import problem as P

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _loaded_state(p, seed=11, zero_history=False):
    """An oracle on p with a random flow state and divergence history (zero
    history: D^{n-1} = D^{n-2} = 0), and the explicit force of that state."""
    o = Oracle(p, threads=1)
    rng = np.random.default_rng(seed)
    st = o.get_state()
    d1 = np.zeros(st["D1"].shape) if zero_history else rng.standard_normal(st["D1"].shape) * 1e-3
    d2 = np.zeros(st["D2"].shape) if zero_history else rng.standard_normal(st["D2"].shape) * 1e-3
    o.set_state(f=rng.standard_normal(st["f"].shape) * 1e-2, g=st["g"], D1=d1, D2=d2, step=3)
    return o, o.explicit_force()


def _brute_fixed_point(o, level, Ft, r=None):
    """Fixed point g = S(g) of level `level` by a dense solve of the affine map
    assembled column by column from single applications."""
    nx, ny = o.level_shape(level)
    m = 8 * nx * ny
    b = o.apply_elastic(level, np.zeros((8, ny, nx)), r, Ft).reshape(-1)
    Amat = np.zeros((m, m))
    for k in range(m):
        e = np.zeros(m)
        e[k] = 1.0
        Amat[:, k] = o.apply_elastic(level, e.reshape(8, ny, nx), r, Ft).reshape(-1) - b
    return np.linalg.solve(np.eye(m) - Amat, b).reshape(8, ny, nx)


def _restrict(rho):
    n8, ny, nx = rho.shape
    return rho.reshape(8, ny // 2, 2, nx // 2, 2).sum(axis=(2, 4))


def _prolong(e):
    return e.repeat(2, axis=1).repeat(2, axis=2)


# ------------------------------------------------- self-dependence constant
def test_literal_constant_equals_default_for_implicit_coupling():
    """The printed alpha^2/2 is the r = 1 value of r alpha^2/2: at r = 1 both
    readings take the same steps bitwise; at r = 1/2 they differ."""
    p = P.loaded_strip(n=16, alpha=0.9, ne_fixed=2)
    for r, same in ((1.0, True), (0.5, False)):
        a = Oracle(p.replace(r=r))
        b = Oracle(p.replace(r=r, fstar_literal=1))
        a.step(3)
        b.step(3)
        ea, eb = a.fields()["eta"], b.fields()["eta"]
        assert np.array_equal(ea, eb) == same, (r, np.abs(ea - eb).max())


def test_literal_constant_is_the_implicit_one_in_the_elastic_solve():
    """With no divergence history (D^{n-1} = D^{n-2} = 0) the explicit force
    does not depend on r, so the elastic cycle of the literal constant at any
    r is the default cycle at r = 1, bitwise."""
    base = P.loaded_strip(n=16, alpha=0.8, K=2)
    g0 = np.random.default_rng(4).standard_normal((8, 16, 16))
    o1, F1 = _loaded_state(base.replace(r=0.5, fstar_literal=1), zero_history=True)
    o2, F2 = _loaded_state(base.replace(r=1.0), zero_history=True)
    assert np.array_equal(F1, F2)
    L = o1.levels
    assert np.array_equal(o1.mg_cycle(L, g0, None, F1), o2.mg_cycle(L, g0, None, F2))


def test_literal_constant_does_not_reproduce_the_reported_instability():
    """Sec. 4.1 reports that the explicit coupling (r = 0) diverges from
    alpha = 0.6 with MG(4,2).  With the literal constant the explicit scheme
    keeps the full implicit self-dependence and stays stable there, so the
    reported pattern is that of r alpha^2/2 (pinned in test_oracle_pins)."""
    M = P.Manufactured(32, alpha=0.6, r=0.0, K=2, ne_fixed=4)
    p = M.problem.replace(fstar_literal=1)
    nt = int(round(1.0 / p.dt))
    o = run(p, nt, loads=M.loads, threads=oracle_threads())
    err = A.rel_l2(o.fields()["p"], M.p((nt - 1) * p.dt))
    assert err < 0.02, err


def _manufactured_errors(n, **kw):
    M = P.Manufactured(n, alpha=0.5, r=0.5, K=2, ne_fixed=3)
    p = M.problem.replace(**kw)
    nt = int(round(1.0 / p.dt))
    acc = np.zeros(6)

    def cb(k, o):
        t = (k - 1) * p.dt
        F = o.fields()
        for j, (num, ref) in enumerate(((F["p"], M.p(t)), (F["eta"], M.eta(t)), (F["sigma"], M.sigma(t)))):
            acc[2 * j] += np.sum((num - ref) ** 2)
            acc[2 * j + 1] += np.sum(ref ** 2)

    run(p, nt, loads=M.loads, threads=oracle_threads(), every=1, callback=cb)
    return np.sqrt(acc[0::2] / acc[1::2])


def test_literal_constant_changes_the_limit_of_the_centred_scheme():
    """At r = 1/2 the literal constant adds (1 - r) alpha^2/2 grad^c D^n to
    the elastic force, a stiffness the continuum problem does not have: the
    displacement and stress errors of the manufactured solution stay near
    15% under refinement, where the default converges at second order
    (Sec. 4.1)."""
    e16, e32 = (_manufactured_errors(n, fstar_literal=1) for n in (16, 32))
    for j in (1, 2):
        assert e32[j] > 0.1 and e16[j] / e32[j] < 1.5, (e16, e32)


# ------------------------------------------------ coarsest-level sweeps
def test_coarse_sweeps_of_2k_are_the_default():
    p = P.loaded_strip(n=16, alpha=0.9, K=2, ne_fixed=2)
    a, b = Oracle(p), Oracle(p.replace(coarse_sweeps=4))
    a.step(2)
    b.step(2)
    assert np.array_equal(a.fields()["eta"], b.fields()["eta"])


def test_converged_coarsest_level_is_the_two_grid_cycle_with_an_exact_coarse_solve():
    """Two levels, the coarsest smoothed to convergence: the cycle equals K
    fine smoothing steps, the restricted residual, the coarse problem's own
    fixed point (dense solve) prolongated and added, and K more fine steps."""
    n, K = 8, 2
    p = P.loaded_strip(n=n, alpha=0.9).replace(levels=2, K=K, coarse_sweeps=3000)
    o, Ft = _loaded_state(p)
    gam = p.gamma
    g0 = np.random.default_rng(5).standard_normal((8, n, n))

    def smooth(g):
        return (1.0 - gam) * g + gam * o.apply_elastic(2, g, None, Ft)

    g = g0.copy()
    for _ in range(K):
        g = smooth(g)
    rc = _restrict(g - o.apply_elastic(2, g, None, Ft))
    e = _brute_fixed_point(o, 1, None, rc)
    g = g + _prolong(e)
    for _ in range(K):
        g = smooth(g)
    ref = o.mg_cycle(2, g0, None, Ft)
    assert np.abs(ref - g).max() < 1e-11 * np.abs(g).max()


def test_coarse_sweeps_count_on_the_coarsest_level():
    """A cycle on two levels with m coarsest sweeps equals one written out
    with m smoothing steps on level 1."""
    n, K, m = 8, 2, 6
    p = P.loaded_strip(n=n, alpha=0.9).replace(levels=2, K=K, coarse_sweeps=m)
    o, Ft = _loaded_state(p)
    gam = p.gamma
    g0 = np.random.default_rng(7).standard_normal((8, n, n))
    g = g0.copy()
    for _ in range(K):
        g = (1 - gam) * g + gam * o.apply_elastic(2, g, None, Ft)
    rc = _restrict(g - o.apply_elastic(2, g, None, Ft))
    e = np.zeros((8, n // 2, n // 2))
    for _ in range(m):
        e = (1 - gam) * e + gam * o.apply_elastic(1, e, rc, None)
    g = g + _prolong(e)
    for _ in range(K):
        g = (1 - gam) * g + gam * o.apply_elastic(2, g, None, Ft)
    assert np.abs(o.mg_cycle(2, g0, None, Ft) - g).max() < 1e-12 * np.abs(g).max()


def test_terzaghi_column_reaches_its_tolerance_once_the_coarsest_level_is_solved():
    """Terzaghi on 8 x 128 cells with 3 levels, adaptive to 1e-8 (the
    benchmark configuration): the 2 x 32 coarsest level with the 2K = 8 sweeps
    of Algorithm 4 is far from solved, the V-cycle contracts the residual by
    less than 0.9 per cycle and every step stops at N_E,max = 50 above the
    tolerance; with 512 coarsest sweeps every step reaches 1e-8 in at most 25
    cycles."""
    base = P.terzaghi(ne_tol=1e-8, ne_max=50)
    a = Oracle(base, threads=oracle_threads(), history=6)
    a.step(6)
    ne, ratio = a.get_history()
    assert np.all(ne == 50) and np.all(ratio > 1e-6), (ne, ratio)
    b = Oracle(base.replace(coarse_sweeps=512), threads=oracle_threads(), history=6)
    b.step(6)
    ne, ratio = b.get_history()
    assert np.all(ne <= 25) and np.all(ratio <= 1e-8), (ne, ratio)


# --------------------------------------------------------- full multigrid
@pytest.mark.parametrize("levels", [1, 2])
def test_full_multigrid_is_the_v_cycle_on_one_or_two_levels(levels):
    """With at most one coarser level the nested iteration has nothing to
    nest: the coarse correction is the coarsest level's sweeps from zero, as
    in the V-cycle, bitwise."""
    p = P.loaded_strip(n=8, alpha=0.9).replace(levels=levels, K=2)
    g0 = np.random.default_rng(3).standard_normal((8, 8, 8))
    o1, F1 = _loaded_state(p)
    o2, F2 = _loaded_state(p.replace(cycle=P.CYCLE_FMG))
    assert np.array_equal(o1.mg_cycle(levels, g0, None, F1), o2.mg_cycle(levels, g0, None, F2))


def test_three_level_full_multigrid_composed_by_hand():
    """Three levels, written out from the single operations: K smoothing
    steps on the fine iterate, its residual restricted; on level 2 the
    correction from zero by nested iteration: the residual of the zero
    iterate restricted to level 1, 2K sweeps there from zero, prolongated as
    level 2's starting iterate, one two-level V-cycle on level 2; that
    correction prolongated and added, K more fine smoothing steps."""
    n, K = 8, 2
    p = P.loaded_strip(n=n, alpha=0.9).replace(levels=3, K=K, cycle=P.CYCLE_FMG)
    o, Ft = _loaded_state(p)
    gam = p.gamma
    g0 = np.random.default_rng(5).standard_normal((8, n, n))

    def smooth(level, g, r, F):
        return (1.0 - gam) * g + gam * o.apply_elastic(level, g, r, F)

    def coarsest(r1):
        e = np.zeros((8, n // 4, n // 4))
        for _ in range(2 * K):
            e = smooth(1, e, r1, None)
        return e

    def vcycle2(e, r2):
        for _ in range(K):
            e = smooth(2, e, r2, None)
        e = e + _prolong(coarsest(_restrict(e - o.apply_elastic(2, e, r2, None))))
        for _ in range(K):
            e = smooth(2, e, r2, None)
        return e

    g = g0.copy()
    for _ in range(K):
        g = smooth(3, g, None, Ft)
    r2 = _restrict(g - o.apply_elastic(3, g, None, Ft))
    z = np.zeros((8, n // 2, n // 2))
    e2 = _prolong(coarsest(_restrict(z - o.apply_elastic(2, z, r2, None))))
    e2 = vcycle2(e2, r2)
    g = g + _prolong(e2)
    for _ in range(K):
        g = smooth(3, g, None, Ft)
    ref = o.mg_cycle(3, g0, None, Ft)
    assert np.abs(ref - g).max() < 1e-12 * np.abs(g).max()


@pytest.mark.parametrize("levels", [3, 4])
def test_full_multigrid_solves_the_coarsest_level_once_per_coarse_level(levels):
    """The nested iteration ends the correction of every coarse level with a
    V-cycle (the coarsest level with its sweeps), so an FMG cycle on L levels
    reaches the coarsest level L - 1 times."""
    p = P.loaded_strip(n=16, alpha=0.9).replace(levels=levels, K=1, cycle=P.CYCLE_FMG)
    o, Ft = _loaded_state(p)
    before = o.coarsest_visits()
    o.mg_cycle(levels, np.zeros((8, 16, 16)), None, Ft)
    assert o.coarsest_visits() - before == levels - 1


def test_full_multigrid_converges_to_brute_force_fixed_point():
    p = P.loaded_strip(n=8, alpha=0.9).replace(levels=3, K=2, cycle=P.CYCLE_FMG)
    o, Ft = _loaded_state(p)
    gstar = _brute_fixed_point(o, 3, Ft)
    g = np.zeros_like(gstar)
    for _ in range(200):
        g = o.mg_cycle(3, g, None, Ft)
    assert np.abs(g - gstar).max() < 1e-12 * max(1.0, np.abs(gstar).max())


def test_full_multigrid_from_rest_improves_with_the_grid():
    """Nested iteration: one FMG cycle from a zero iterate leaves an algebraic
    error that falls as the grid is refined (8, 16, 32 cells, full hierarchy),
    while one V-cycle's does not, and ends well below the V-cycle's."""
    errs = {P.CYCLE_V: [], P.CYCLE_FMG: []}
    for n in (8, 16, 32):
        p = P.loaded_strip(n=n, alpha=0.0, K=2)
        ov = Oracle(p, threads=oracle_threads())
        Ft = ov.explicit_force()
        L = ov.levels
        gstar = np.zeros((8, n, n))
        for _ in range(150):
            gstar = ov.mg_cycle(L, gstar, None, Ft)
        for cyc in errs:
            o = Oracle(p.replace(cycle=cyc), threads=oracle_threads())
            g = o.mg_cycle(L, np.zeros((8, n, n)), None, Ft)
            errs[cyc].append(np.linalg.norm(g - gstar) / np.linalg.norm(gstar))
    v, f = np.array(errs[P.CYCLE_V]), np.array(errs[P.CYCLE_FMG])
    assert f[0] > f[1] > f[2] and v[2] >= v[0], errs
    assert np.all(f < 0.7 * v) and f[2] < 0.3 * v[2], errs


def test_full_multigrid_step_takes_it_as_the_first_cycle():
    """A time step with N_E = 2 and full multigrid: the elastic state after
    the step is one FMG cycle then one V-cycle from the warm start, with the
    explicit force of the step."""
    p = P.loaded_strip(n=16, alpha=0.9, K=2, ne_fixed=2)
    a = Oracle(p.replace(cycle=P.CYCLE_FMG))
    a.step(2)
    Ft = a.explicit_force()
    g0 = a.get_state()["g"]
    b = Oracle(p.replace(cycle=P.CYCLE_FMG))
    c = Oracle(p)
    b.set_state(**{k: v for k, v in a.get_state().items()})
    c.set_state(**{k: v for k, v in a.get_state().items()})
    L = a.levels
    want = c.mg_cycle(L, b.mg_cycle(L, g0, None, Ft), None, Ft)
    a.step(1)
    assert np.array_equal(a.get_state()["g"], want)


# ------------------------------------------ Algorithm 1 and its lag
def test_lagged_applications_composed_by_hand():
    """Algorithm 1 read with the lag of eq. source:implicit: the first
    pseudo-time step of a time step is the plain one (g(-1) = g(0)); every
    later one collides with the self-force of the previous step's iterate.
    Since S(g; r) = ELASTIC_STEP(g - r, Ft + F_*(g)), the lagged step from g_k
    is S(g_{k-1}; g_{k-1} - g_k)."""
    n = 8
    p = P.Manufactured(n, alpha=0.9, r=0.5, K=2, ne_fixed=1, levels=1).problem.replace(gamma=1.0, lag=1)
    f, s = P.Manufactured(n, alpha=0.9).loads(0.3)
    p = p.replace(body_f=f, source_s=s)
    o, Ft = _loaded_state(p)
    g0 = np.random.default_rng(2).standard_normal((8, n, n))
    g1 = o.apply_elastic(1, g0, None, Ft)
    g2 = o.apply_elastic(1, g0, g0 - g1, Ft)
    g3 = o.apply_elastic(1, g1, g1 - g2, Ft)
    g4 = o.apply_elastic(1, g2, g2 - g3, Ft)
    got = o.mg_cycle(1, g0, None, Ft)       # K = 2: four applications
    assert np.abs(got - g4).max() < 1e-12 * np.abs(g4).max()
    plain, Fp = _loaded_state(p.replace(lag=0))
    assert np.abs(plain.mg_cycle(1, g0, None, Fp) - g4).max() > 1e-6


def test_lagged_pseudo_time_stepping_reaches_the_fixed_point():
    p = P.loaded_strip(n=8, alpha=0.9).replace(levels=1, gamma=1.0, K=1, lag=1)
    o, Ft = _loaded_state(p)
    gstar = _brute_fixed_point(o, 1, Ft)
    g = np.zeros_like(gstar)
    for _ in range(1500):
        g = o.mg_cycle(1, g, None, Ft)
    assert np.abs(g - gstar).max() < 1e-12 * np.abs(gstar).max()


@functools.lru_cache(maxsize=None)
def _converged_errors(n):
    return _manufactured_errors(n, ne_fixed=6)


def _alg1_error_ratio(n, napps, lag):
    """Errors of Algorithm 1 with napps pseudo-time steps per time step on the
    periodic problem of Sec. 4.1 (alpha = 0.5, centred), relative to those of
    the converged elastic solve (MG(6,2)), for p, eta and sigma."""
    e_mg = _converged_errors(n)
    e = _manufactured_errors(n, levels=1, K=1, gamma=1.0, ne_fixed=napps // 2, lag=lag)
    return e / e_mg


def test_plain_pseudo_time_stepping_cost_scales_with_n_squared():
    """Sec. 4.1, Algorithm 1 on the periodic problem with alpha = 0.5 and the
    centred coupling: with N_E pseudo-time steps the error approaches that of
    the converged elastic solve once N_E is well above 0.015 N_x^2 (here 0.04
    N_x^2: within 6%), is dominated by the pseudo-time error well below it
    (0.006 N_x^2: 30% and more above), depends on N_E / N_x^2 rather than on
    N_E / N_x, and N_E = 1.5 N_x still gives almost second order between 16
    and 32 cells."""
    r_above = [_alg1_error_ratio(n, round(0.04 * n * n / 2) * 2, 1) for n in (16, 32)]
    assert all(np.all(r < 1.06) for r in r_above), r_above
    assert np.abs(r_above[0] - r_above[1]).max() < 0.03, r_above     # a function of N_E / N_x^2
    r_below = _alg1_error_ratio(32, 6, 1)
    assert r_below.max() > 1.3, r_below
    e = [_manufactured_errors(n, levels=1, K=1, gamma=1.0, ne_fixed=int(1.5 * n) // 2, lag=1) for n in (16, 32)]
    rates = np.log2(e[0] / e[1])
    assert np.all(rates > 1.8), rates


def test_lag_is_distinguishable_but_does_not_change_the_reported_behaviour():
    """The lagged and the current-iterate self-force are different iterations
    (their results differ beyond rounding) that the cost-scaling study cannot
    tell apart: their error ratios agree to 1% at N_E = 0.006 N_x^2."""
    n = 32
    a = run(P.Manufactured(n, alpha=0.5).problem.replace(levels=1, K=1, gamma=1.0, ne_fixed=3, lag=1), 4,
            loads=P.Manufactured(n, alpha=0.5).loads, threads=oracle_threads())
    b = run(P.Manufactured(n, alpha=0.5).problem.replace(levels=1, K=1, gamma=1.0, ne_fixed=3, lag=0), 4,
            loads=P.Manufactured(n, alpha=0.5).loads, threads=oracle_threads())
    assert A.rel_l2(a.fields()["eta"], b.fields()["eta"]) > 1e-6
    r1, r0 = _alg1_error_ratio(n, 6, 1), _alg1_error_ratio(n, 6, 0)
    assert np.abs(r1 / r0 - 1).max() < 0.01, (r1, r0)


# ------------------------------------------------------------- validation
def test_invalid_variant_parameters_are_rejected():
    base = P.loaded_strip(n=8)
    for bad in (dict(cycle=4), dict(fstar_literal=2), dict(coarse_sweeps=3), dict(coarse_sweeps=-2),
                dict(lag=1),                                   # lag needs one level
                dict(lag=1, levels=1, ne_fixed=0, ne_tol=1e-6)):  # and a fixed N_E
        with pytest.raises(OracleError):
            Oracle(base.replace(**bad))
