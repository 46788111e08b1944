"""Shared helpers of the GPU parity tests (problem builders and error norms)."""
import numpy as np

from paper_2409_11382_amd import problem as P


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = float(np.sqrt(np.sum(b * b)))
    d = float(np.sqrt(np.sum((a - b) ** 2)))
    return d / nb if nb > 0 else d


def mixed_walls(nx, ny, seed=0, levels=0, alpha=0.8):
    """Dirichlet left, traction right/top, symmetry bottom, random boundary data,
    mixed flow types (Dirichlet / no-flow / symmetry) along the sides."""
    rng = np.random.default_rng(seed)
    lam, mu = P.plane_stress_lame(1.0, 0.3)

    def side(n, el, flows):
        return P.Side(el=el, flow=rng.choice(flows, size=n).astype(np.int8),
                      el_value=rng.standard_normal((n, 2)), p_value=rng.standard_normal(n))

    sides = [side(ny, P.EL_DIRICHLET, [P.FLOW_DIRICHLET, P.FLOW_NOFLOW]),
             side(ny, P.EL_TRACTION, [P.FLOW_NOFLOW, P.FLOW_DIRICHLET]),
             side(nx, P.EL_SYMMETRY, [P.FLOW_SYMMETRY]),
             side(nx, P.EL_TRACTION, [P.FLOW_DIRICHLET, P.FLOW_NOFLOW])]
    h = 1.0 / max(nx, ny)
    kap = P.lognormal_permeability(nx, sigma_log=0.7, corr=6.0, seed=seed + 1, ny=ny)
    return P.Problem(nx=nx, ny=ny, dx=h, dt=h * h / 4, lam=lam, mu=mu, c0=0.1, alpha=alpha,
                     kappa=kap, sides=sides, levels=levels, K=2, ne_fixed=2, name="mixed")


def problems_small():
    """Small problems that span several column tiles and strips with ragged
    tails, covering every boundary type."""
    out = {}
    out["strip_130x72"] = P.loaded_strip(n=130, ny=72, alpha=1.0, K=2, ne_fixed=2)
    out["terzaghi_8x128"] = P.terzaghi(ne_fixed=3, ne_tol=0.0)
    out["mixed_124x68"] = mixed_walls(124, 68, seed=3)
    M = P.Manufactured(64, alpha=0.9, r=0.5, K=2, ne_fixed=2)
    f, s = M.loads(0.2)
    out["periodic_64"] = M.problem.replace(body_f=f, source_s=s)
    return out


def tail_level(shapes, prec):
    """Top level of the multigrid tail that one workgroup runs (0: none): the
    largest coarse level whose cells fit the tail kernel (1024, one cell
    per thread).
    shapes[l - 1] is the (nx, ny) of level l."""
    L = len(shapes)
    for l in range(L - 1, 0, -1):
        nx, ny = shapes[l - 1]
        if nx * ny <= 1024:
            return l
    return 0
