"""Seeded draws of initial nuclear conditions (inputs, not method arithmetic).

Every function takes a seed and returns plain numpy arrays.  Draw order is
fixed so that a seed reproduces the same arrays on every machine:
``numpy.random.default_rng(seed)`` is consumed first for positions, then for
velocities, then for anything else the function documents.
"""
from __future__ import annotations

import numpy as np


def boltzmann_harmonic(n_traj: int, mass: float, omega: float, kT: float,
                       seed: int, kT_factor: float = 1.0):
    """Classical Boltzmann sample of a harmonic well centred at x = 0.

    The phase-space density of the double-well section (Sec. III.B) is a
    product of Gaussians: x has variance kT'/(m w^2) and v has variance
    kT'/m, with kT' = kT_factor * kT (the paper prepares at 5 kT).
    """
    rng = np.random.default_rng(seed)
    kt = kT * kT_factor
    sx = np.sqrt(kt / (mass * omega * omega))
    sv = np.sqrt(kt / mass)
    x = rng.normal(0.0, sx, size=n_traj)
    v = rng.normal(0.0, sv, size=n_traj)
    return x, v


def wigner_harmonic(n_traj: int, mass: float, omega: float, x_centre: float, kT: float,
                    seed: int):
    """Harmonic Wigner sample about x_centre (Sec. III.C, Eq. wigner): the
    classical Boltzmann Gaussians with kT replaced by Q kT, where
    Q = (beta omega / 2) / tanh(beta omega / 2) (hbar = 1).  x has variance
    Q kT / (m w^2) and v has variance Q kT / m."""
    rng = np.random.default_rng(seed)
    half = 0.5 * omega / kT
    q = half / np.tanh(half)
    sx = np.sqrt(q * kT / (mass * omega * omega))
    sv = np.sqrt(q * kT / mass)
    x = x_centre + rng.normal(0.0, sx, size=n_traj)
    v = rng.normal(0.0, sv, size=n_traj)
    return x, v


def boltzmann_coordinates(n_traj: int, masses, omegas, centres, kT: float, seed: int):
    """Classical Boltzmann sample of independent harmonic coordinates (one
    per column): R_nu ~ N(c_nu, kT / (m_nu w_nu^2)), v_nu ~ N(0, kT / m_nu).
    Positions are drawn first (all trajectories, coordinate-major per
    trajectory), then velocities."""
    rng = np.random.default_rng(seed)
    m = np.asarray(masses, dtype=np.float64)
    w = np.asarray(omegas, dtype=np.float64)
    c = np.asarray(centres, dtype=np.float64)
    x = c[None, :] + rng.normal(size=(n_traj, len(m))) * np.sqrt(kT / (m * w * w))[None, :]
    v = rng.normal(size=(n_traj, len(m))) * np.sqrt(kT / m)[None, :]
    return x, v


def scattering_initial(n_traj: int, mass: float, x_start: float,
                       e_range: tuple, seed: int):
    """Incoming scattering trajectories: x = x_start, moving toward the
    surface with kinetic energy drawn uniformly in e_range (Sec. III.D)."""
    rng = np.random.default_rng(seed)
    e = rng.uniform(e_range[0], e_range[1], size=n_traj)
    x = np.full(n_traj, float(x_start))
    v = -np.sqrt(2.0 * e / mass)
    return x, v, e


def bath_classes(n_traj: int, classes, seed: int):
    """Uniform draw of a bath-size class index per trajectory."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, len(classes), size=n_traj).astype(np.int32)


def fixed_paths(n_traj: int, n_steps: int, dt: float, omega: float, seed: int,
                x_scale: float = 3.0, v_scale: float = 7e-4, amp_scale: float = 3.0):
    """Prescribed nuclear paths x(t) = x0 + v0 t + A sin(omega t + phi).

    Returns positions and analytic velocities on the grid t = 0, dt, ...,
    n_steps*dt, each of shape (n_traj, n_steps + 1).
    """
    rng = np.random.default_rng(seed)
    x0 = rng.normal(0.0, x_scale, size=n_traj)
    v0 = rng.normal(0.0, v_scale, size=n_traj) * 0.1
    amp = rng.uniform(0.0, amp_scale, size=n_traj)
    phi = rng.uniform(0.0, 2 * np.pi, size=n_traj)
    t = np.arange(n_steps + 1) * dt
    x = x0[:, None] + v0[:, None] * t[None, :] + amp[:, None] * np.sin(omega * t[None, :] + phi[:, None])
    v = v0[:, None] + amp[:, None] * omega * np.cos(omega * t[None, :] + phi[:, None])
    return x, v


def uniforms(seed: int, shape):
    rng = np.random.default_rng(seed)
    return rng.random(shape)


def random_orbitals(n: int, n_elec: int, seed: int):
    """A random n x N complex matrix with orthonormal columns (QR of a
    complex Gaussian matrix), for single-step and hop-probability tests."""
    rng = np.random.default_rng(seed)
    z = rng.normal(size=(n, n_elec)) + 1j * rng.normal(size=(n, n_elec))
    q, r = np.linalg.qr(z)
    return q * (np.diag(r) / np.abs(np.diag(r)))[None, :]
