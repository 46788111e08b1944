"""Pins of the oracle's W- and F-cycles.

The paper defines the V-cycle (Algorithm 4) and names W- and F-cycles as future
work without defining them.  The oracle takes the textbook recursions: a
W-cycle visits the coarser level twice, the second visit continuing from the
first's coarse iterate with the same coarse right-hand side; an F-cycle makes
an F-visit and then a V-visit.  These tests check the oracle against facts
that follow from those definitions: shapes that must coincide, the number of
coarsest-level solves, a two-level cycle composed by hand from the pinned
single operations, the brute-force fixed point, and the contraction.
"""
import numpy as np
import pytest

from conftest import oracle_threads
from oracle.oracle import Oracle, OracleError
from paper_2409_11382_amd import problem as P

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")

CYCLES = (P.CYCLE_V, P.CYCLE_W, P.CYCLE_F)


def _loaded_state(p, seed=11):
    """An oracle on p with a random flow state and divergence history, and the
    explicit force of that state."""
    o = Oracle(p, threads=1)
    rng = np.random.default_rng(seed)
    st = o.get_state()
    o.set_state(f=rng.standard_normal(st["f"].shape) * 1e-2, g=st["g"],
                D1=rng.standard_normal(st["D1"].shape) * 1e-3,
                D2=rng.standard_normal(st["D2"].shape) * 1e-3, step=3)
    return o, o.explicit_force()


def _cycle(p, cyc, g0, seed=11):
    o, Ft = _loaded_state(p.replace(cycle=cyc), seed)
    return o.mg_cycle(o.levels, g0, None, Ft)


def test_cycle_shapes_coincide_without_recursion():
    """One level (Algorithm 1 and any single-level hierarchy): there is no
    coarser level to visit, so V, W and F are the same 2K sweeps."""
    p = P.loaded_strip(n=8, alpha=0.9).replace(levels=1, K=2)
    g0 = np.random.default_rng(3).standard_normal((8, 8, 8))
    out = [_cycle(p, c, g0) for c in CYCLES]
    assert np.array_equal(out[0], out[1]) and np.array_equal(out[0], out[2])


def test_w_and_f_coincide_on_two_levels():
    """Two levels: W visits the coarsest twice, F visits it once as an F-visit
    and once as a V-visit, which on the coarsest are the same sweeps; V visits
    it once and differs."""
    p = P.loaded_strip(n=8, alpha=0.9).replace(levels=2, K=2)
    g0 = np.random.default_rng(3).standard_normal((8, 8, 8))
    v, w, f = (_cycle(p, c, g0) for c in CYCLES)
    assert np.array_equal(w, f)
    assert np.abs(w - v).max() > 1e-6


@pytest.mark.parametrize("levels", [3, 4])
def test_coarsest_solves_per_cycle(levels):
    """Coarsest-level solves per cycle on L levels: V 1, W 2^(L-1), F L (an
    F-visit of level l makes an F-visit and a V-visit of level l - 1)."""
    p = P.loaded_strip(n=16, alpha=0.9).replace(levels=levels, K=1)
    for cyc, want in ((P.CYCLE_V, 1), (P.CYCLE_W, 2 ** (levels - 1)), (P.CYCLE_F, levels)):
        o, Ft = _loaded_state(p.replace(cycle=cyc))
        before = o.coarsest_visits()
        o.mg_cycle(levels, np.zeros((8, 16, 16)), None, Ft)
        assert o.coarsest_visits() - before == want, (cyc, o.coarsest_visits() - before)


def test_two_level_w_cycle_composed_by_hand():
    """A two-level W-cycle written out from the oracle's single operations:
    K smoothing steps g <- (1 - gamma) g + gamma S(g) on the fine level,
    the residual g - S(g) summed over 2x2 blocks, two coarse visits of 2K
    smoothing steps from zero (the second continuing from the first) with that
    right-hand side, the coarse result added to each fine cell of its block,
    K more fine smoothing steps."""
    n, K = 8, 2
    p = P.loaded_strip(n=n, alpha=0.9).replace(levels=2, K=K, cycle=P.CYCLE_W)
    o, Ft = _loaded_state(p)
    gam = p.gamma
    g0 = np.random.default_rng(5).standard_normal((8, n, n))

    def smooth(level, g, r, F):
        return (1.0 - gam) * g + gam * o.apply_elastic(level, g, r, F)

    g = g0.copy()
    for _ in range(K):
        g = smooth(2, g, None, Ft)
    rho = g - o.apply_elastic(2, g, None, Ft)
    rc = rho.reshape(8, n // 2, 2, n // 2, 2).sum(axis=(2, 4))
    e = np.zeros((8, n // 2, n // 2))
    for _ in range(2 * 2 * K):
        e = smooth(1, e, rc, None)
    g = g + e.repeat(2, axis=1).repeat(2, axis=2)
    for _ in range(K):
        g = smooth(2, g, None, Ft)
    ref = o.mg_cycle(2, g0, None, Ft)
    assert np.abs(ref - g).max() < 1e-12 * np.abs(g).max()


def _brute_fixed_point(o, L, Ft):
    nx, ny = o.level_shape(L)
    m = 8 * nx * ny
    b = o.apply_elastic(L, np.zeros((8, ny, nx)), None, Ft).reshape(-1)
    Amat = np.zeros((m, m))
    for k in range(m):
        e = np.zeros(m)
        e[k] = 1.0
        Amat[:, k] = o.apply_elastic(L, e.reshape(8, ny, nx), None, Ft).reshape(-1) - b
    return np.linalg.solve(np.eye(m) - Amat, b).reshape(8, ny, nx)


@pytest.mark.parametrize("cyc", [P.CYCLE_W, P.CYCLE_F])
def test_cycles_converge_to_brute_force_fixed_point(cyc):
    """Every consistent cycle converges to the fixed point g = S(g) of the
    fine elastic step, found here by a dense linear solve."""
    p = P.loaded_strip(n=8, alpha=0.9).replace(levels=3, K=2, cycle=cyc)
    o, Ft = _loaded_state(p)
    gstar = _brute_fixed_point(o, 3, Ft)
    g = np.zeros_like(gstar)
    for _ in range(300):
        g = o.mg_cycle(3, g, None, Ft)
    assert np.abs(g - gstar).max() < 1e-12 * max(1.0, np.abs(gstar).max())


def test_w_and_f_contract_faster_than_v_independently_of_the_grid():
    """Periodic elasticity: the W- and F-cycles contract the residual at least
    as fast as the V-cycle (they do more coarse work per cycle), W at least as
    fast as F, and all three factors stay bounded as the grid is refined."""
    factors = {c: [] for c in CYCLES}
    for n in (16, 32):
        M = P.Manufactured(n, K=2)
        f, _ = M.loads(1.0)
        base = M.problem.replace(alpha=0.0, body_f=f, source_s=np.zeros((n, n)))
        for c in CYCLES:
            o = Oracle(base.replace(cycle=c), threads=oracle_threads())
            Ft = o.explicit_force()
            L = o.levels
            g = np.random.default_rng(0).standard_normal((8, n, n))
            res = []
            for _ in range(16):
                res.append(np.sqrt(np.sum((g - o.apply_elastic(L, g, None, Ft)) ** 2)))
                g = o.mg_cycle(L, g, None, Ft)
            factors[c].append((res[-1] / res[-6]) ** 0.2)
    v, w, f = (np.array(factors[c]) for c in CYCLES)
    assert np.all(w <= f + 1e-3) and np.all(f < v - 0.02), factors
    assert max(np.ptp(v), np.ptp(w), np.ptp(f)) < 0.03 and v.max() < 0.85, factors


def test_unknown_cycle_shape_is_rejected():
    with pytest.raises(OracleError):
        Oracle(P.loaded_strip(n=8).replace(cycle=4))
