"""Independent two-state fewest-switches surface hopping (one impurity level,
one bath level, one electron).

Test infrastructure only (see the package docstring).

With M = 1 and N = 1 IESH reduces to Tully's original two-state
fewest-switches algorithm (Sec. II.B states the IESH rates are the
fewest-switches ones).  This module implements that limit from closed forms
only, without any general linear algebra: the 2x2 eigenpairs from the
mixing angle, the coupling from the derivative of the mixing angle, the
propagator from the closed-form exponential of a 2x2 Hermitian matrix, and
the one-dimensional velocity rescaling.  It uses the same step order as
``dynamics.step`` (midpoint propagator) and the same uniform per step.

Gauge: impurity components positive.  For H = [[h, V], [V, e]] with V > 0,
R = sqrt(((h - e)/2)^2 + V^2), the mixing angle theta in (0, pi/2) has
cos 2theta = (h - e)/(2R), sin 2theta = V/R; the lower orbital is
(sin theta, -cos theta), the upper (cos theta, sin theta), and
<lower| d/dx upper> = -theta'.
"""
from __future__ import annotations

import math

import numpy as np


def _pieces(h, dh, e, V, dV):
    mean = 0.5 * (h + e)
    delta = 0.5 * (h - e)
    R = math.sqrt(delta * delta + V * V)
    lam = np.array([mean - R, mean + R])
    theta = 0.5 * math.atan2(V, delta)
    dtheta = (delta * dV - V * 0.5 * dh) / (2.0 * R * R)
    # D[0, 1] = <lower|d upper> = -theta', D[1, 0] = +theta'
    D = np.array([[0.0, -dtheta], [dtheta, 0.0]])
    U = np.array([[math.sin(theta), math.cos(theta)],
                  [-math.cos(theta), math.sin(theta)]])   # columns: lower, upper
    return lam, D, U


def _expm2(A, dt):
    """exp(-i A dt) for a 2x2 Hermitian A in closed form."""
    t = 0.5 * (A[0, 0] + A[1, 1]).real
    B = A - t * np.eye(2)
    # B is traceless Hermitian: B^2 = w^2 I with w^2 = -det(B)
    w = math.sqrt(max(-(B[0, 0] * B[1, 1] - B[0, 1] * B[1, 0]).real, 0.0))
    if w == 0.0:
        U = np.eye(2, dtype=complex)
    else:
        U = math.cos(w * dt) * np.eye(2) - 1j * math.sin(w * dt) / w * B
    return np.exp(-1j * t * dt) * U


def step(model, x, v, c, a, dt, xi, F=None):
    """One step for the two-state problem; model must have M = 1.

    Returns (x, v, c, a, event, F)."""
    m = float(model.mass[0])
    e = float(model.eps[0])

    def pieces(xx):
        X = np.atleast_1d(xx)
        return _pieces(model.h(X), float(model.dh(X)[0]), e, float(model.V(X)[0]),
                       float(model.dV(X)[0, 0]))

    def force(xx, occ):
        _, _, U = pieces(xx)
        X = np.atleast_1d(xx)
        # Hellmann-Feynman: d lambda_a / dx = u_a^T dH u_a
        dh = float(model.dh(X)[0])
        dV = float(model.dV(X)[0, 0])
        u0, u1 = U[0, occ], U[1, occ]
        return -float(model.dU0(X)[0]) - (dh * u0 * u0 + 2.0 * dV * u0 * u1)

    if F is None:
        F = force(x, a)
    v_half = v + 0.5 * dt * F / m
    x_new = x + dt * v_half
    lam_m, D_m, _ = pieces(0.5 * (x + x_new))
    A = np.diag(lam_m).astype(complex) - 1j * v_half * D_m
    c = _expm2(A, dt) @ c
    lam, D, _ = pieces(x_new)
    F_new = force(x_new, a)
    v_new = v_half + 0.5 * dt * F_new / m
    b = 1 - a
    g = max(-2.0 * dt * v_new * D[b, a] * (c[b] * np.conj(c[a])).real / abs(c[a]) ** 2, 0.0)
    event = dict(attempted=g > xi, accepted=False, a=a, b=b, g=g)
    if g > xi:
        dE = lam[b] - lam[a]
        disc = v_new * v_new - 2.0 * dE / m
        if disc >= 0.0:
            v_new = math.copysign(math.sqrt(disc), v_new)
            a = b
            event["accepted"] = True
            F_new = force(x_new, a)
    return x_new, v_new, c, a, event, F_new
