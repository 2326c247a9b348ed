"""Closed forms used to pin the oracle.

Test infrastructure only (see the package docstring).

Impurity occupation in equilibrium.  For an energy-independent
hybridisation Gamma (Eq. hybridization) in the wide-band limit, the impurity
spectral function is the Lorentzian A(e) = (Gamma/2pi) / ((e - h)^2 +
(Gamma/2)^2) (the same broadening that enters the wide-band friction of
Eq. exact-friction), and its Fermi-weighted integral is

    n_d = 1/2 - (1/pi) Im psi(1/2 + (Gamma/2 + i (h - mu)) / (2 pi kT))

with psi the digamma function (sum the Matsubara poles of the Fermi
function).  At kT -> 0 this becomes 1/2 + arctan((mu - h)/(Gamma/2))/pi.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import psi


def impurity_occupation(h, Gamma, mu, kT):
    if kT == 0.0:
        return 0.5 + math.atan((mu - h) / (0.5 * Gamma)) / math.pi
    z = 0.5 + (0.5 * Gamma + 1j * (h - mu)) / (2.0 * math.pi * kT)
    return 0.5 - float(np.imag(psi(z))) / math.pi


def two_level_eigenvalues(h, e, V):
    mean, delta = 0.5 * (h + e), 0.5 * (h - e)
    R = math.sqrt(delta * delta + V * V)
    return mean - R, mean + R


def harmonic_wigner_factor(beta, omega):
    """Q(beta, omega) = beta omega / (2 tanh(beta omega / 2)) (Eq. wigner, hbar = 1)."""
    y = beta * omega
    return y / (2.0 * math.tanh(0.5 * y))
