"""Discretisation of the metallic band (Appendix A).

Test infrastructure only (see the package docstring).

The continuum coupling integral is replaced by a sum over M states with
energies eps_k and weights w_k; the couplings are V_k = V(eps_k) sqrt(w_k)
(Appendix A), and with an energy-independent hybridisation Gamma the
continuum coupling is V = sqrt(Gamma / 2 pi) (Eq. hybridization, Sec. II.A).

Readings:
* Trapezoid: the paper's formula eps_k = a + (k-1)(b-a)/M is a left-endpoint
  grid (it contains a, not b).  It is used literally; the midpoint grid is
  offered as an option.
* Gauss-Legendre: the printed sums run to N in both halves and the printed
  lower-half weight for eps_f at the band centre carries a minus sign.  Both
  are evident typos: each half holds M/2 nodes, and the weight of the lower
  half is (eps_f - a)/2 times the Legendre weight, which is +W/4 times it for
  a band [-W/2, W/2] split at eps_f = 0.  With these readings the weights sum
  to the band width, as any quadrature of a constant must.
"""
from __future__ import annotations

import numpy as np


def trapezoid(M: int, a: float, b: float):
    """eps_k = a + (k-1)(b-a)/M, w_k = (b-a)/M, k = 1..M (Appendix A)."""
    k = np.arange(M, dtype=np.float64)
    eps = a + k * (b - a) / M
    w = np.full(M, (b - a) / M)
    return eps, w


def trapezoid_midpoint(M: int, a: float, b: float):
    """Option: midpoint grid eps_k = a + (k - 1/2)(b-a)/M."""
    k = np.arange(M, dtype=np.float64)
    eps = a + (k + 0.5) * (b - a) / M
    w = np.full(M, (b - a) / M)
    return eps, w


def gauss_legendre(M: int, a: float, b: float, eps_f: float = 0.0):
    """Two-half Gauss-Legendre discretisation split at eps_f (Appendix A,
    Eq. gaussian-quadrature): M/2 Legendre nodes on [a, eps_f] and M/2 on
    [eps_f, b], each affinely mapped from [-1, 1]."""
    if M % 2:
        raise ValueError("Gauss-Legendre split needs an even number of states")
    x, wt = np.polynomial.legendre.leggauss(M // 2)
    lo_e = 0.5 * (eps_f - a) * x + 0.5 * (a + eps_f)
    lo_w = 0.5 * (eps_f - a) * wt
    hi_e = 0.5 * (b - eps_f) * x + 0.5 * (eps_f + b)
    hi_w = 0.5 * (b - eps_f) * wt
    return np.concatenate([lo_e, hi_e]), np.concatenate([lo_w, hi_w])


def discretise(kind: str, M: int, W: float, eps_f: float = 0.0, centre: float = 0.0):
    """Bath on [centre - W/2, centre + W/2]; Gauss-Legendre halves split at eps_f."""
    a, b = centre - 0.5 * W, centre + 0.5 * W
    if kind == "trapezoid":
        return trapezoid(M, a, b)
    if kind == "trapezoid_midpoint":
        return trapezoid_midpoint(M, a, b)
    if kind == "gauss_legendre":
        return gauss_legendre(M, a, b, eps_f)
    raise ValueError(kind)


def two_leads(eps, w):
    """Two leads on one grid, each coupled with half the hybridisation
    (Gamma/2 each, so the total width stays Gamma): every level appears once
    per lead with half its weight.  Levels are listed in ascending energy,
    lead 0 before lead 1 at equal energy.  Returns (eps, w, lead)."""
    eps = np.asarray(eps, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    M = len(eps)
    e2, w2, lead = [], [], []
    for k in range(M):
        for l in (0, 1):
            e2.append(eps[k])
            w2.append(0.5 * w[k])
            lead.append(l)
    return np.array(e2), np.array(w2), np.array(lead, dtype=np.int32)


def couplings(Gamma: float, w):
    """V_k = sqrt(Gamma w_k / (2 pi)) (Eq. hybridization with Appendix A)."""
    return np.sqrt(Gamma * np.asarray(w) / (2.0 * np.pi))
