"""Workload descriptions (constants only, atomic units throughout).

Model constants follow the paper: the double-well harmonic diabats of
Sec. III.B and the desorption/scattering model of Sec. III.C
(Eqs. U0, U1, Vk and Table et-parameters).  Sizes, time steps, trajectory
counts and seeds are the synthetic workloads this library is measured on.

Unit conversions use CODATA 2018 values.
"""
from __future__ import annotations

import copy

# CODATA 2018
HARTREE_EV = 27.211386245988
BOHR_ANGSTROM = 0.529177210903
AMU_ME = 1822.888486209          # unified atomic mass unit in electron masses
KB_HARTREE_PER_K = 3.166811563e-6  # Boltzmann constant in Hartree/K
FS_AU = 41.341373335             # 1 fs in atomic time units


def ev(x):
    return x / HARTREE_EV


def angstrom(x):
    return x / BOHR_ANGSTROM


# Double-well model of Sec. III.B (harmonic diabats).  The paper's relaxation
# study uses g = 20.6097; the throughput workloads below use g = 20.
DOUBLE_WELL = dict(kind="harmonic", mass=2000.0, omega=2e-4, g=20.6097, dG=-3.8e-3)

# Desorption / scattering model of Sec. III.C, Table et-parameters, in a.u.
# The scattering workload replaces the Morse depth and range by D = 0.1 Ha and
# a = 1.0 / bohr.
DESORPTION_TABLE = dict(
    De=ev(3.52), x0=angstrom(1.78), a=1.7361 * BOHR_ANGSTROM,
    D1=ev(4.52), D2=ev(0.79), ap=1.379 * BOHR_ANGSTROM,
    Vinf=ev(-1.5), q=0.05, atil=angstrom(0.5), xtil=angstrom(3.5),
    mass=10.54 * AMU_ME, c=ev(-45.7e-3),
)

CONFIGS = {
    # Plain IESH, FP64, small: the parity workload.
    "c1": dict(
        name="harmonic M=20 N=10, 128 trajectories, dt=50",
        model=dict(kind="harmonic", mass=2000.0, omega=2e-4, g=20.0, dG=-3.8e-3,
                   Gamma=0.01, eps_d=0.0),
        bath=dict(kind="trapezoid", M=20, W=0.1),
        n_elec=10, kT=9.5e-4, sample_kT_factor=1.0,
        n_traj=128, n_steps=1000, dt=50.0, seed=0,
    ),
    # Plain IESH at scale: the headline throughput workload.
    "c2": dict(
        name="harmonic M=200 N=100, 4096 trajectories, dt=20",
        model=dict(kind="harmonic", mass=2000.0, omega=2e-4, g=20.0, dG=-3.8e-3,
                   Gamma=0.01, eps_d=0.0),
        bath=dict(kind="trapezoid", M=200, W=0.1),
        n_elec=100, kT=9.5e-4, sample_kT_factor=1.0,
        n_traj=4096, n_steps=20000, dt=20.0, seed=0,
    ),
    # Same as c2 with the Gauss-Legendre two-half discretisation (App. A).
    "c2gl": dict(
        name="harmonic M=200 N=100 Gauss-Legendre bath, 4096 trajectories, dt=20",
        model=dict(kind="harmonic", mass=2000.0, omega=2e-4, g=20.0, dG=-3.8e-3,
                   Gamma=0.01, eps_d=0.0),
        bath=dict(kind="gauss_legendre", M=200, W=0.1),
        n_elec=100, kT=9.5e-4, sample_kT_factor=1.0,
        n_traj=4096, n_steps=20000, dt=20.0, seed=0,
    ),
    # Uneven batched scattering (Morse / repulsive diabats, tanh coupling).
    "c3": dict(
        name="scattering, M in {40,80,160,320}, N=M/2, 16384 trajectories, dt=5",
        model=dict(kind="morse_tanh", De=0.1, x0=DESORPTION_TABLE["x0"], a=1.0,
                   D1=DESORPTION_TABLE["D1"], D2=DESORPTION_TABLE["D2"],
                   ap=DESORPTION_TABLE["ap"], Vinf=DESORPTION_TABLE["Vinf"],
                   q=DESORPTION_TABLE["q"], atil=DESORPTION_TABLE["atil"],
                   xtil=DESORPTION_TABLE["xtil"], mass=DESORPTION_TABLE["mass"],
                   c=DESORPTION_TABLE["c"], Gamma=ev(1.0), eps_d=0.0),
        bath=dict(kind="gauss_legendre", M_classes=[40, 80, 160, 320], W=ev(64.0)),
        kT=0.0, x_start=angstrom(5.0), E_inc=(ev(0.05), ev(1.0)),
        exit_x=15.0, max_steps=20000,
        n_traj=16384, dt=5.0, seed=0,
    ),
    # Desorption (Sec. III.C): the vibronic model of Table et-parameters,
    # Gauss-Legendre bath of 100 states over 64 eV, half filling, 300 K Fermi
    # occupations and a harmonic Wigner sample of the Morse well; a trajectory
    # counts as desorbed once x exceeds 5 Angstrom.
    "desorption": dict(
        name="desorption, Table et-parameters, GL M=100 W=64 eV, N=50, 300 K, 8192 trajectories, dt=5",
        model=dict(kind="morse_tanh", **{k: v for k, v in DESORPTION_TABLE.items()},
                   Gamma=ev(1.0), eps_d=0.0),
        bath=dict(kind="gauss_legendre", M=100, W=ev(64.0)),
        n_elec=50, kT=300.0 * KB_HARTREE_PER_K, x_threshold=angstrom(5.0),
        n_traj=8192, n_steps=2000, dt=5.0, seed=0,
    ),
    # Several nuclear coordinates (six: one surface-normal Morse mode and
    # five internal modes), the library's multi-coordinate model: Morse U0 per
    # coordinate, impurity level linear in the displacements, Gaussian
    # hybridisation Gamma(R); one band of 256 states, half filling, mixed path.
    # Biased two-lead junction: two leads of 128 levels on one trapezoid grid
    # (each coupled with Gamma/2; equal energies, deflated), bias V between
    # the leads' chemical potentials (V in {0, 0.01, 0.02}).
    "c5": dict(
        name="two leads 2x128 (n=257), bias V, six coordinates, Morse U0, Gaussian Gamma(R), "
             "N=128, 8192 trajectories, dt=20",
        model=dict(kind="multi_dof", Gamma=0.01, Delta=0.005, eps_d=0.0,
                   dof=[[2000.0, 0.10, 1.0, 3.0, -0.004, 3.0, 1.5],
                        [2000.0, 0.15, 1.2, 2.0, 0.002, 2.0, 2.0],
                        [4000.0, 0.08, 0.8, 0.0, 0.001, 0.0, 2.5],
                        [4000.0, 0.08, 0.8, 0.0, -0.001, 0.0, 2.5],
                        [8000.0, 0.05, 0.6, 0.0, 0.0005, 0.0, 3.0],
                        [8000.0, 0.05, 0.6, 0.0, -0.0005, 0.0, 3.0]]),
        bath=dict(kind="trapezoid", M=256, W=0.1, leads=2, bias=0.0),
        n_elec=128, kT=9.5e-4, n_traj=8192, n_steps=10000, dt=20.0, seed=0,
        biases=[0.0, 0.01, 0.02],
    ),
    # Adjoint workload: fixed nuclear paths.
    "c4": dict(
        name="adjoint, harmonic M=100 N=50, 1024 fixed paths, 2000 steps, dt=20",
        model=dict(kind="harmonic", mass=2000.0, omega=2e-4, g=20.0, dG=-3.8e-3,
                   Gamma=0.01, eps_d=0.0),
        bath=dict(kind="trapezoid", M=100, W=0.1),
        n_elec=50, kT=9.5e-4, n_traj=1024, n_steps=2000, dt=20.0, ckpt_every=100,
        seed=0,
    ),
    # General (dense) one-electron Hamiltonian, the fallback for H(x) of any
    # structure: the double-well impurity on a band of 95 levels whose levels
    # also couple to their neighbours (a tight-binding chain, hopping t_bath),
    # with an x-dependent impurity coupling V_k(x) = V_k (1 + alpha x); H(x) =
    # H0 + x H1 with a rank-2 H1 (workloads.dense_matrices builds both).
    "dense": dict(
        name="dense H(x) = H0 + x H1, n=96 (impurity + 95-level chain), N=48, 4096 trajectories, dt=20",
        model=dict(kind="dense", mass=2000.0, omega=2e-4, g=20.0, dG=-3.8e-3, Gamma=0.01,
                   t_bath=2.0e-4, alpha=0.02, x_c=0.0),
        bath=dict(kind="cells", M=95, W=0.1),
        n_elec=48, kT=9.5e-4, sample_kT_factor=1.0,
        n_traj=4096, n_steps=2000, dt=20.0, seed=0,
    ),
}


def get_config(name: str) -> dict:
    return copy.deepcopy(CONFIGS[name])


def dense_matrices(cfg: dict, M: int | None = None):
    """H0 and H1 of a dense workload (H(x) = H0 + x H1), as plain input
    arrays: impurity level h(x) = m omega^2 (g^2 - 2 g x)/2 + dG of the
    double well, M bath levels at the cell centres of [-W/2, W/2] (equal
    widths W/M), impurity couplings V_k (1 + alpha x) with
    V_k = sqrt(Gamma (W/M) / (2 pi)), and nearest-neighbour couplings t_bath
    between bath levels."""
    import numpy as np
    m, b = cfg["model"], cfg["bath"]
    M = M if M is not None else b["M"]
    W = b["W"]
    eps = -0.5 * W + (np.arange(M) + 0.5) * (W / M)
    V = np.full(M, np.sqrt(m["Gamma"] * (W / M) / (2.0 * np.pi)))
    k = m["mass"] * m["omega"] ** 2
    n = M + 1
    H0 = np.zeros((n, n))
    H0[0, 0] = 0.5 * k * m["g"] ** 2 + m["dG"]
    H0[0, 1:] = H0[1:, 0] = V
    H0[1:, 1:] = np.diag(eps)
    idx = np.arange(1, M)
    H0[idx, idx + 1] = H0[idx + 1, idx] = m["t_bath"]
    H1 = np.zeros((n, n))
    H1[0, 0] = -k * m["g"]
    H1[0, 1:] = H1[1:, 0] = m["alpha"] * V
    return H0, H1
