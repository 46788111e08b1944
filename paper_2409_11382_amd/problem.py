"""Problem descriptions and seeded synthetic workloads for the coupled Biot LBM.

This module holds inputs only: grids, dimensional material parameters, boundary
types and boundary data, loads and seeded random fields.  It performs none of
the lattice Boltzmann arithmetic (no scaling to lattice units, no relaxation
rates, no velocity sets); both the FP64 oracle and the HIP library read a
``Problem`` and do their own conversion.

Conventions
-----------
* Fields are row-major ``[y, x]`` with x fastest; vector fields carry the
  component first (``body_f`` is ``(2, ny, nx)``).
* Cell ``(i, j)`` has its centre at ``((i + 1/2) dx, (j + 1/2) dx)``.
* Sides are numbered 0 = left (x = 0), 1 = right, 2 = bottom (y = 0), 3 = top.
  Left/right boundary arrays are indexed by the row j (length ny), bottom/top
  arrays by the column i (length nx).  Boundary data are given at the face
  centre of each boundary cell.
* Everything here is dimensional, in the units of the Biot system (eqs. 1-4 of
  the paper): displacement ``eta``, stress ``sigma``, pressure ``p``, storage
  ``c0``, permeability ``kappa``, body force ``f`` and fluid source ``s``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, Optional, Sequence

import numpy as np

# Boundary type codes (shared numbering with include/biotlbm.h).
FLOW_PERIODIC, FLOW_DIRICHLET, FLOW_NOFLOW, FLOW_SYMMETRY = 0, 1, 2, 3
EL_PERIODIC, EL_DIRICHLET, EL_TRACTION, EL_SYMMETRY = 0, 1, 2, 3
LEFT, RIGHT, BOTTOM, TOP = 0, 1, 2, 3

PREC_FP64, PREC_FP32, PREC_FP32_SHIFTED, PREC_FP64_SHIFTED = 0, 1, 2, 3
PREC_NAMES = {"fp64": PREC_FP64, "fp32": PREC_FP32,
              "fp32_shifted": PREC_FP32_SHIFTED, "fp64_shifted": PREC_FP64_SHIFTED}


# pressure gradient of the explicit force: first moments of the flow
# populations (eq. pressure:gradient) or the central difference of the pressure
# (eq. pressure:gradient:alternative)
GRAD_MOMENTS, GRAD_CENTRAL = 0, 1
# multigrid cycle shape: the V-cycle of Algorithm 4; W- and F-cycles (named as
# future work in the conclusion) in their textbook form; full multigrid (also
# future work there) as the first cycle of every time step, V-cycles after it
CYCLE_V, CYCLE_W, CYCLE_F, CYCLE_FMG = 0, 1, 2, 3


@dataclasses.dataclass
class Side:
    """One side of the rectangular domain.

    ``el`` is uniform along the side; the flow type may vary per boundary cell
    (the loaded strip is impermeable under the load and drained elsewhere).
    ``el_value`` holds eta_D for a Dirichlet side or the traction t = sigma n for
    a traction side, two values per boundary cell; ``p_value`` holds p_D.
    """
    el: int
    flow: np.ndarray          # int8, one code per boundary cell
    el_value: np.ndarray      # float64, (n, 2)
    p_value: np.ndarray       # float64, (n,)

    @staticmethod
    def uniform(n: int, el: int, flow: int, el_value=(0.0, 0.0), p_value=0.0) -> "Side":
        return Side(el=el,
                    flow=np.full(n, flow, dtype=np.int8),
                    el_value=np.tile(np.asarray(el_value, dtype=np.float64), (n, 1)),
                    p_value=np.full(n, float(p_value), dtype=np.float64))


@dataclasses.dataclass
class Problem:
    """A 2D Biot consolidation problem and the method parameters used to solve it."""
    nx: int
    ny: int
    dx: float
    dt: float
    lam: float
    mu: float
    c0: float
    alpha: float
    kappa: object                      # float or (ny, nx) float64 array
    sides: Sequence[Side]
    body_f: Optional[np.ndarray] = None    # (2, ny, nx) or None
    source_s: Optional[np.ndarray] = None  # (ny, nx) or None
    r: float = 0.5
    levels: int = 0                    # 0 => default hierarchy depth
    K: int = 4
    gamma: float = 0.75
    ne_fixed: int = 3                  # > 0: fixed number of V-cycles per step
    ne_tol: float = 0.0                # used when ne_fixed == 0
    ne_max: int = 50
    name: str = ""
    pressure_gradient: int = 0         # GRAD_MOMENTS or GRAD_CENTRAL
    cycle: int = 0                     # CYCLE_V, CYCLE_W, CYCLE_F or CYCLE_FMG
    fstar_literal: int = 0             # 1: self-dependence constant alpha^2/2 for every r
    coarse_sweeps: int = 0             # smoothing steps on the coarsest level (0: 2K)
    lag: int = 0                       # Algorithm 1 (one level): divergence of the previous
                                       # pseudo-time step in the implicit source

    # ---- helpers ---------------------------------------------------------
    @property
    def ncells(self) -> int:
        return self.nx * self.ny

    def kappa_field(self) -> np.ndarray:
        if np.isscalar(self.kappa):
            return np.full((self.ny, self.nx), float(self.kappa))
        return np.asarray(self.kappa, dtype=np.float64).reshape(self.ny, self.nx)

    def default_levels(self) -> int:
        """1 + the number of exact halvings of both dimensions that keep >= 2 cells."""
        L, nx, ny = 1, self.nx, self.ny
        while nx % 2 == 0 and ny % 2 == 0 and nx // 2 >= 2 and ny // 2 >= 2:
            nx //= 2
            ny //= 2
            L += 1
        return L

    def num_levels(self) -> int:
        return self.levels if self.levels > 0 else self.default_levels()

    def cell_centres(self):
        x = (np.arange(self.nx) + 0.5) * self.dx
        y = (np.arange(self.ny) + 0.5) * self.dx
        return np.meshgrid(x, y)  # X[y, x], Y[y, x]

    def replace(self, **kw) -> "Problem":
        return dataclasses.replace(self, **kw)


def plane_stress_lame(E: float, nu: float):
    """Lame coefficients under the plane-stress assumption used throughout the
    paper's experiments (Sec. 4.1, 4.2, 4.3)."""
    return E * nu / (1.0 - nu * nu), E / (2.0 * (1.0 + nu))


def _sides_periodic_x(nx, ny, bottom: Side, top: Side):
    return [Side.uniform(ny, EL_PERIODIC, FLOW_PERIODIC),
            Side.uniform(ny, EL_PERIODIC, FLOW_PERIODIC), bottom, top]


# ---------------------------------------------------------------------------
# Terzaghi consolidation (Sec. 4.2): top drained with a step traction load,
# bottom impermeable and clamped, periodic in x.
# ---------------------------------------------------------------------------
def terzaghi(nx=8, ny=128, lam=1.0, mu=1.0, kappa=1.0, c0=0.1, alpha=1.0, load=1.0,
             dt=None, levels=0, K=4, gamma=0.75, r=0.5, ne_fixed=0, ne_tol=1e-8,
             ne_max=50) -> Problem:
    h = 1.0 / ny
    bottom = Side.uniform(nx, EL_DIRICHLET, FLOW_NOFLOW, (0.0, 0.0), 0.0)
    top = Side.uniform(nx, EL_TRACTION, FLOW_DIRICHLET, (0.0, -load), 0.0)
    return Problem(nx=nx, ny=ny, dx=h, dt=(h * h / 4.0 if dt is None else dt), lam=lam, mu=mu,
                   c0=c0, alpha=alpha, kappa=kappa, sides=_sides_periodic_x(nx, ny, bottom, top),
                   r=r, levels=levels, K=K, gamma=gamma, ne_fixed=ne_fixed, ne_tol=ne_tol,
                   ne_max=ne_max, name=f"terzaghi_{nx}x{ny}")


def layered_column(n=32, nx=4, seed=3, kmin=0.1, kmax=1.0) -> Problem:
    """Flow only (alpha = 0) up an x-periodic column of horizontal layers, one
    log-uniform random permeability in [kmin, kmax] per row, pressure 1 at the
    bottom face and 0 at the top; the elastic field stays zero (clamped
    bottom, traction-free top).  kappa[:, 0] holds the layers."""
    h = 1.0 / n
    kr = 10 ** np.random.default_rng(seed).uniform(np.log10(kmin), np.log10(kmax), n)
    bottom = Side.uniform(nx, EL_DIRICHLET, FLOW_DIRICHLET, (0.0, 0.0), 1.0)
    top = Side.uniform(nx, EL_TRACTION, FLOW_DIRICHLET, (0.0, 0.0), 0.0)
    base = terzaghi(nx=nx, ny=n)
    return base.replace(sides=[base.sides[0], base.sides[1], bottom, top], kappa=kr[:, None] * np.ones((n, nx)),
                        alpha=0.0, c0=1.0, dt=h * h, ne_fixed=1, K=1, levels=2, name=f"layered_{nx}x{n}")


def terzaghi_paper(alpha: float, n: int, nx=None, **kw) -> Problem:
    """Terzaghi parameters of Sec. 4.2: E = 1, nu = 0.8 (plane stress),
    kappa = (lam + 2 mu + alpha^2)/(lam + 2 mu), load = alpha + (lam + 2 mu)/alpha,
    which makes the instantaneous pressure response p0 = 1."""
    lam, mu = plane_stress_lame(1.0, 0.8)
    m = lam + 2 * mu
    kappa = (m + alpha * alpha) / m
    load = alpha + m / alpha
    kw.setdefault("ne_fixed", 3)
    return terzaghi(nx=(n if nx is None else nx), ny=n, lam=lam, mu=mu, kappa=kappa, c0=1.0,
                    alpha=alpha, load=load, **kw)


# ---------------------------------------------------------------------------
# Loaded strip (2D extension of Terzaghi, as in Sec. 4.3 but on a unit square):
# unit load on the central quarter of the top, impermeable under the load and
# drained elsewhere on the top; the other sides are impermeable rollers.
# ---------------------------------------------------------------------------
def loaded_strip(n=512, E=1.0, nu=0.3, kappa=1.0, c0=1.0, alpha=1.0, load=1.0,
                 ny=None, dt=None, levels=0, K=4, gamma=0.75, r=0.5, ne_fixed=3,
                 ne_tol=0.0, ne_max=50, whole_top_drained=False) -> Problem:
    nx = n
    ny = n if ny is None else ny
    h = 1.0 / nx
    lam, mu = plane_stress_lame(E, nu)
    xc = (np.arange(nx) + 0.5) * h
    under = (xc > 3.0 / 8.0) & (xc < 5.0 / 8.0)
    tval = np.zeros((nx, 2))
    tval[under, 1] = -load
    tflow = np.where(under & (not whole_top_drained), FLOW_NOFLOW, FLOW_DIRICHLET).astype(np.int8)
    top = Side(el=EL_TRACTION, flow=tflow, el_value=tval, p_value=np.zeros(nx))
    sym_y = Side.uniform(ny, EL_SYMMETRY, FLOW_SYMMETRY)
    sides = [sym_y, Side.uniform(ny, EL_SYMMETRY, FLOW_SYMMETRY),
             Side.uniform(nx, EL_SYMMETRY, FLOW_SYMMETRY), top]
    if dt is None:
        # lattice diffusion number kappa' dt / h^2 = 1/4 (omega_f = 0.8) at the
        # problem's permeability (the geometric mean 1 for a field): with the
        # first-moment pressure gradient the coupled scheme goes unstable as
        # omega_f approaches 2, which small kappa at a fixed dt would cause
        kbar = float(kappa) if np.isscalar(kappa) else 1.0
        dt = c0 * h * h / (4.0 * kbar)
    return Problem(nx=nx, ny=ny, dx=h, dt=dt, lam=lam, mu=mu,
                   c0=c0, alpha=alpha, kappa=kappa, sides=sides, r=r, levels=levels, K=K,
                   gamma=gamma, ne_fixed=ne_fixed, ne_tol=ne_tol, ne_max=ne_max,
                   name=f"loaded_strip_{nx}x{ny}")


# ---------------------------------------------------------------------------
# Two-dimensional loading problem (Sec. 4.3), dimensional: domain (0, 100)^2,
# final time 2e6, top drained with the traction (0, -1e4 (1 - cos(pi (x1 + 25)
# / 50))), bottom clamped and impermeable, periodic in x1; E = 1e5, nu = 0.9
# (plane stress), c0 = 1e-6, kappa = 1e-9, alpha = 1; N_T = N_x^2 time steps,
# centred coupling with MG(3,4).
# ---------------------------------------------------------------------------
def loading_2d(n=128, steps=None, K=4, ne_fixed=3, r=0.5, levels=0) -> Problem:
    length, t_final = 100.0, 2.0e6
    h = length / n
    nt = n * n if steps is None else steps
    lam, mu = plane_stress_lame(1.0e5, 0.9)
    x1 = (np.arange(n) + 0.5) * h
    tval = np.zeros((n, 2))
    tval[:, 1] = -1.0e4 * (1.0 - np.cos((x1 + 25.0) / 50.0 * math.pi))
    top = Side(el=EL_TRACTION, flow=np.full(n, FLOW_DIRICHLET, dtype=np.int8), el_value=tval,
               p_value=np.zeros(n))
    bottom = Side.uniform(n, EL_DIRICHLET, FLOW_NOFLOW)
    return Problem(nx=n, ny=n, dx=h, dt=t_final / nt, lam=lam, mu=mu, c0=1.0e-6, alpha=1.0, kappa=1.0e-9,
                   sides=_sides_periodic_x(n, n, bottom, top), r=r, levels=levels, K=K, ne_fixed=ne_fixed,
                   name=f"loading_2d_{n}")


def lognormal_permeability(n: int, sigma_log=1.0, corr=32.0, seed=0, ny=None) -> np.ndarray:
    """ln kappa = sigma_log * Z with Z a zero-mean, unit-variance Gaussian random
    field of covariance exp(-r^2/corr^2) (corr in cells), made by FFT filtering of
    white noise from numpy's PCG64 (default_rng(seed)) and normalised
    empirically; geometric mean 1."""
    ny = n if ny is None else ny
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((ny, n))
    ky = np.fft.fftfreq(ny) * 2 * np.pi
    kx = np.fft.fftfreq(n) * 2 * np.pi
    KX, KY = np.meshgrid(kx, ky)
    spec = np.exp(-(KX ** 2 + KY ** 2) * corr * corr / 8.0)  # sqrt of exp(-k^2 l^2/4)
    z = np.real(np.fft.ifft2(np.fft.fft2(w) * spec))
    sd = z.std()
    # a grid too small for the correlation length can come out constant: kappa 1
    z = (z - z.mean()) / sd if sd > 0 else np.zeros_like(z)
    return np.exp(sigma_log * z)


def heterogeneous_strip(n=2048, sigma_log=1.0, corr=32.0, seed=0, levels=6,
                        pressure_gradient=GRAD_CENTRAL, **kw) -> Problem:
    """The loaded strip with a log-normal permeability field (geometric mean 1,
    so dt = h^2/4).  Its cells reach kappa ~ 0.03, where omega_f approaches 2
    and the first-moment pressure gradient makes the coupled scheme unstable;
    the central-difference gradient (eq. pressure:gradient:alternative), which
    Sec. 4.1 reports to delay the onset of instability, stays stable there."""
    kap = lognormal_permeability(n, sigma_log, corr, seed)
    kw.setdefault("alpha", 1.0)
    p = loaded_strip(n=n, kappa=kap, levels=levels, **kw)
    p.name = f"heterogeneous_{n}x{n}"
    p.pressure_gradient = pressure_gradient
    return p


# ---------------------------------------------------------------------------
# Periodic manufactured solution (Sec. 4.1).
# ---------------------------------------------------------------------------
class Manufactured:
    """Closed-form eta, p, sigma and the loads f, s of the periodic problem of
    Sec. 4.1 on the unit square (c0 = 1, E = 0.11, nu = 0.8 plane stress,
    kappa = 1/10).  The loads are time dependent: call ``loads(t)`` before each
    step."""

    def __init__(self, n: int, alpha=0.5, r=0.5, K=2, ne_fixed=3, dt=None, levels=0,
                 lam=None, mu=None, kappa=0.1):
        lam0, mu0 = plane_stress_lame(0.11, 0.8)
        self.lam = lam0 if lam is None else lam
        self.mu = mu0 if mu is None else mu
        self.kappa = kappa
        self.alpha = alpha
        h = 1.0 / n
        self.problem = Problem(
            nx=n, ny=n, dx=h, dt=(h * h if dt is None else dt), lam=self.lam, mu=self.mu,
            c0=1.0, alpha=alpha, kappa=kappa,
            sides=[Side.uniform(n, EL_PERIODIC, FLOW_PERIODIC) for _ in range(4)],
            body_f=np.zeros((2, n, n)), source_s=np.zeros((n, n)), r=r, levels=levels,
            K=K, ne_fixed=ne_fixed, name=f"manufactured_{n}")
        self.X, self.Y = self.problem.cell_centres()

    def _a(self, t):
        return 1.0 - math.exp(-8 * math.pi ** 2 * self.kappa * t)

    def loads(self, t):
        a = self._a(t)
        pi = math.pi
        sx, cx = np.sin(2 * pi * self.X), np.cos(2 * pi * self.X)
        sy, cy = np.sin(2 * pi * self.Y), np.cos(2 * pi * self.Y)
        f = np.zeros((2,) + self.X.shape)
        f[0] = 0.5 * a * 16 * pi ** 2 * self.mu * cx * sy
        s = (-8 * pi ** 3 * self.kappa
             * (16 * self.alpha * math.exp(-8 * pi ** 2 * self.kappa * t)
                + (16 * self.lam + 30 * self.mu) / self.alpha) * sx * sy)
        return f, s

    def eta(self, t):
        a = self._a(t)
        pi = math.pi
        out = np.zeros((2,) + self.X.shape)
        out[0] = 0.5 * a * 9 * np.cos(2 * pi * self.X) * np.sin(2 * pi * self.Y)
        out[1] = 0.5 * a * 7 * np.sin(2 * pi * self.X) * np.cos(2 * pi * self.Y)
        return out

    def p(self, t):
        a = self._a(t)
        pi = math.pi
        return (-(16 * self.lam + 30 * self.mu) * pi / self.alpha * a
                * np.sin(2 * pi * self.X) * np.sin(2 * pi * self.Y))

    def sigma(self, t):
        """(sigma11, sigma12, sigma22) of the manufactured displacement."""
        a = self._a(t)
        pi = math.pi
        ss = np.sin(2 * pi * self.X) * np.sin(2 * pi * self.Y)
        cc = np.cos(2 * pi * self.X) * np.cos(2 * pi * self.Y)
        return np.stack([-(16 * pi * self.lam + 18 * pi * self.mu) * a * ss,
                         16 * pi * self.mu * a * cc,
                         -(16 * pi * self.lam + 14 * pi * self.mu) * a * ss])


# ---------------------------------------------------------------------------
# Batched and served workloads.
# ---------------------------------------------------------------------------
def batch_problems(count=256, seed=1, sizes=(64, 128, 256, 512), ne_fixed=3, K=4):
    """Independent loaded-strip problems with square grids drawn uniformly from
    ``sizes``, nu ~ U[0.2, 0.45], alpha ~ U[0.5, 1], log10 kappa ~ U[-2, 0],
    E = 1, c0 = 1, drawn from default_rng(seed); each with the time step that
    puts its lattice diffusion number at 1/4 (dt = c0 h^2 / (4 kappa))."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(rng.choice(sizes))
        nu = float(rng.uniform(0.2, 0.45))
        alpha = float(rng.uniform(0.5, 1.0))
        kap = float(10.0 ** rng.uniform(-2.0, 0.0))
        out.append(loaded_strip(n=n, nu=nu, alpha=alpha, kappa=kap, ne_fixed=ne_fixed, K=K))
    return out


def serving_requests(rate: float, count: int, seed=2, nmin=128, nmax=1024,
                     steps=(100, 1000)):
    """Poisson arrival stream of loaded-strip solve requests: returns a list of
    (arrival_time_s, Problem, nsteps).  Grid sizes N = 32*round(exp(U[ln nmin,
    ln nmax])/32), steps ~ U{steps}, parameters as in ``batch_problems``."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for _ in range(count):
        t += float(rng.exponential(1.0 / rate))
        n = int(32 * round(math.exp(rng.uniform(math.log(nmin), math.log(nmax))) / 32))
        nsteps = int(rng.integers(steps[0], steps[1] + 1))
        nu = float(rng.uniform(0.2, 0.45))
        alpha = float(rng.uniform(0.5, 1.0))
        kap = float(10.0 ** rng.uniform(-2.0, 0.0))
        out.append((t, loaded_strip(n=n, nu=nu, alpha=alpha, kappa=kap), nsteps))
    return out


def random_state(p: Problem, seed: int, scale=1e-3):
    """Seeded random populations for single-operation parity tests:
    f (9, ny, nx), g (8, ny, nx), D1, D2 (ny, nx)."""
    rng = np.random.default_rng(seed)
    n = p.ncells
    f = rng.standard_normal((9, p.ny, p.nx)) * scale
    g = rng.standard_normal((8, p.ny, p.nx)) * scale
    d1 = rng.standard_normal((p.ny, p.nx)) * scale * p.dx
    d2 = rng.standard_normal((p.ny, p.nx)) * scale * p.dx
    del n
    return f, g, d1, d2


def with_random_boundary_data(p: Problem, seed: int, scale=1.0) -> Problem:
    """Copy of p whose boundary data (eta_D, traction, p_D) are seeded random
    values; types are unchanged."""
    rng = np.random.default_rng(seed)
    sides = []
    for s in p.sides:
        n = len(s.flow)
        sides.append(Side(el=s.el, flow=s.flow.copy(),
                          el_value=rng.standard_normal((n, 2)) * scale,
                          p_value=rng.standard_normal(n) * scale))
    return p.replace(sides=sides)


LoadFn = Callable[[float], tuple]
