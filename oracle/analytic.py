"""Closed-form references used to pin the oracle (test infrastructure only).

* Terzaghi consolidation series (Sec. 4.2): pressure p(t, x2) and surface
  subsidence S(t), written for the dimensional system (c0 kept explicit).
* Steady flow through horizontal layers of different permeability.
* Error norms of Sec. 4: discrete L2(D) and time-space L2(Q).
"""
from __future__ import annotations

import math

import numpy as np


def terzaghi_constants(lam, mu, c0, alpha, kappa, load):
    """Closed-form constants of the Terzaghi solution of Sec. 4.2 for the
    dimensional system: instantaneous pressure p0, consolidation coefficient c_f,
    initial and final subsidence S0, S_inf.  The paper states them for the
    c0-scaled system; here lam' = c0 lam, mu' = c0 mu, kappa' = kappa/c0 and the
    load c0*load are substituted and p is scaled back by 1/c0."""
    m = lam + 2.0 * mu
    denom = c0 * m + alpha * alpha
    return dict(p0=alpha * load / denom, cf=m * kappa / denom,
                S0=load / (m + alpha * alpha / c0), Sinf=load / m)


def terzaghi_p(t, y, p0, cf, terms=4000):
    """Pressure of the Terzaghi problem at height y in (0, 1) (bottom y = 0
    impermeable, top y = 1 drained), t > 0."""
    y = np.asarray(y, dtype=np.float64)
    out = np.zeros_like(y)
    for k in range(terms):
        a = (k + 0.5) * math.pi
        e = math.exp(-a * a * cf * t)
        if e < 1e-300:
            break
        out += 2.0 * (-1) ** k / a * e * np.cos(a * y)
    return p0 * out


def terzaghi_S(t, S0, Sinf, cf, terms=4000):
    """Surface subsidence S(t) = S_inf + (S0 - S_inf) sum 2/a_k^2 exp(-a_k^2 cf t)."""
    acc = 0.0
    for k in range(terms):
        a = (k + 0.5) * math.pi
        e = math.exp(-a * a * cf * t)
        if e < 1e-300:
            break
        acc += 2.0 / (a * a) * e
    return Sinf + (S0 - Sinf) * acc


def l2_space(err, dx):
    """Discrete L2(D) norm: dx * sqrt(sum |e|^2) over all cells (and components)."""
    return dx * math.sqrt(float(np.sum(np.asarray(err, dtype=np.float64) ** 2)))


def rel_l2(a, b):
    """Relative L2 distance ||a - b|| / ||b|| over all entries (b is the reference)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = math.sqrt(float(np.sum(b * b)))
    d = math.sqrt(float(np.sum((a - b) ** 2)))
    return d / nb if nb > 0 else d


def layered_steady_pressure(kappa_rows, h, p_bottom=1.0, p_top=0.0):
    """Steady Darcy flow up a column of horizontal layers (kappa_rows[j] in
    row j of height h), pressure given at the bottom and top faces: the flux
    is the same through every layer, q = (p_bottom - p_top) / sum(h / kappa_j),
    so p falls linearly inside each layer, by q h / kappa_j across layer j.
    Returns p at the row centres."""
    k = np.asarray(kappa_rows, dtype=np.float64)
    res = h / k
    q = (p_bottom - p_top) / res.sum()
    return p_bottom - q * (np.concatenate([[0.0], np.cumsum(res)[:-1]]) + 0.5 * res)
