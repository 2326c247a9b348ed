"""Newns-Anderson models (Sec. II.A, Sec. III.B, Sec. III.C).

Test infrastructure only (see the package docstring).

The discrete one-electron Hamiltonian (Eq. single_electron_discrete_
electronic_hamiltonian) in the diabatic basis {|d>, |1>, ..., |M>} is the
(M+1) x (M+1) matrix

    H[0, 0] = h(x) = U1(x) - U0(x) (+ eps_d, an optional constant shift)
    H[k, k] = eps_k
    H[0, k] = H[k, 0] = V_k(x)

and the nuclear potential of a configuration s is U0(x) + sum_{k in s}
lambda_k(x) (Eq. classical_hamiltonian).  Positions are arrays of n_dof
coordinates; the models of the paper have n_dof = 1, MultiDof has several.
"""
from __future__ import annotations

import numpy as np

from . import bath as _bath


class Model:
    n_dof = 1
    lead = None  # per bath level 0 or 1 for two leads (else None)

    def __init__(self, eps, w, Gamma, mass):
        self.eps = np.asarray(eps, dtype=np.float64)
        self.w = np.asarray(w, dtype=np.float64)
        self.M = len(self.eps)
        self.n = self.M + 1
        self.Gamma = float(Gamma)
        self.mass = np.atleast_1d(np.asarray(mass, dtype=np.float64))
        self.Vbar = _bath.couplings(self.Gamma, self.w)

    # --- diabatic pieces, overridden by subclasses --------------------------------
    def U0(self, x):
        raise NotImplementedError

    def dU0(self, x):
        raise NotImplementedError

    def h(self, x):
        raise NotImplementedError

    def dh(self, x):
        raise NotImplementedError

    def V(self, x):
        raise NotImplementedError

    def dV(self, x):
        """(M, n_dof) derivative of the couplings."""
        raise NotImplementedError

    # --- dense matrices --------------------------------------------------------------
    def H(self, x):
        x = np.atleast_1d(x)
        H = np.diag(np.concatenate([[self.h(x)], self.eps]))
        V = self.V(x)
        H[0, 1:] = V
        H[1:, 0] = V
        return H

    def dH(self, x):
        """List of n_dof derivative matrices dH/dx_nu."""
        x = np.atleast_1d(x)
        dh = np.atleast_1d(self.dh(x))
        dV = self.dV(x)
        out = []
        for nu in range(self.n_dof):
            d = np.zeros((self.n, self.n))
            d[0, 0] = dh[nu]
            d[0, 1:] = dV[:, nu]
            d[1:, 0] = dV[:, nu]
            out.append(d)
        return out


class Harmonic(Model):
    """Double-well model, Sec. III.B:
    U0 = m w^2 x^2 / 2,  U1 = m w^2 (x - g)^2 / 2 + dG,  V_k constant."""

    def __init__(self, eps, w, Gamma, mass, omega, g, dG, eps_d=0.0):
        super().__init__(eps, w, Gamma, mass)
        self.omega, self.g, self.dG, self.eps_d = float(omega), float(g), float(dG), float(eps_d)
        self.k = self.mass[0] * self.omega ** 2

    def U0(self, x):
        return 0.5 * self.k * x[0] ** 2

    def dU0(self, x):
        return np.array([self.k * x[0]])

    def U1(self, x):
        return 0.5 * self.k * (x[0] - self.g) ** 2 + self.dG

    def h(self, x):
        return self.U1(x) - self.U0(x) + self.eps_d

    def dh(self, x):
        return np.array([-self.k * self.g])

    def V(self, x):
        return self.Vbar.copy()

    def dV(self, x):
        return np.zeros((self.M, 1))


class MorseTanh(Model):
    """Desorption/scattering model, Sec. III.C, Eqs. U0, U1 and Vk:
    U0 = De (exp(-a (x - x0)) - 1)^2 + c
    U1 = D1 exp(-2 a' (x - x0)) - D2 exp(-a' (x - x0)) + Vinf
    V_k(x) = Vbar_k [ (1 - q)/2 (1 - tanh((x - xt)/at)) + q ].

    Reading: as typeset the bracket of Eq. Vk encloses "+ q" inside the
    (1-q)/2 prefactor, which would give ~0.97 Vbar near the surface and
    ~0.02 Vbar far away; the intended form is the one above, which goes from
    Vbar (near) to q Vbar (far).
    """

    def __init__(self, eps, w, Gamma, mass, De, x0, a, D1, D2, ap, Vinf, q, atil, xtil, c,
                 eps_d=0.0):
        super().__init__(eps, w, Gamma, mass)
        self.De, self.x0, self.a, self.c = De, x0, a, c
        self.D1, self.D2, self.ap, self.Vinf = D1, D2, ap, Vinf
        self.q, self.atil, self.xtil, self.eps_d = q, atil, xtil, eps_d

    def U0(self, x):
        e = np.exp(-self.a * (x[0] - self.x0))
        return self.De * (e - 1.0) ** 2 + self.c

    def dU0(self, x):
        e = np.exp(-self.a * (x[0] - self.x0))
        return np.array([-2.0 * self.De * self.a * e * (e - 1.0)])

    def U1(self, x):
        e = np.exp(-self.ap * (x[0] - self.x0))
        return self.D1 * e * e - self.D2 * e + self.Vinf

    def dU1(self, x):
        e = np.exp(-self.ap * (x[0] - self.x0))
        return np.array([-2.0 * self.ap * self.D1 * e * e + self.ap * self.D2 * e])

    def h(self, x):
        return self.U1(x) - self.U0(x) + self.eps_d

    def dh(self, x):
        return self.dU1(x) - self.dU0(x)

    def _f(self, x):
        t = np.tanh((x[0] - self.xtil) / self.atil)
        return 0.5 * (1.0 - self.q) * (1.0 - t) + self.q, t

    def V(self, x):
        f, _ = self._f(x)
        return self.Vbar * f

    def dV(self, x):
        _, t = self._f(x)
        df = -0.5 * (1.0 - self.q) * (1.0 - t * t) / self.atil
        return (self.Vbar * df)[:, None]


class MultiDof(Model):
    """Several coordinates R_1 .. R_D (the library's multi-coordinate model;
    the paper's models are one-dimensional):
        U0(R) = sum_nu D_nu (1 - exp(-a_nu (R_nu - r_nu)))^2
        h(R)  = Delta + eps_d + sum_nu g_nu (R_nu - r_nu)
        V_k(R) = Vbar_k exp(-sum_nu (R_nu - c_nu)^2 / (4 s_nu^2)).
    dof rows: (mass, D, a, r, g, c, s)."""

    def __init__(self, eps, w, Gamma, dof, Delta, eps_d=0.0):
        dof = np.asarray(dof, dtype=np.float64)
        super().__init__(eps, w, Gamma, dof[:, 0])
        self.n_dof = dof.shape[0]
        self.D, self.a, self.r, self.g, self.c, self.s = (dof[:, k] for k in range(1, 7))
        self.Delta, self.eps_d = float(Delta), float(eps_d)

    def U0(self, x):
        e = np.exp(-self.a * (x - self.r))
        return float(np.sum(self.D * (1.0 - e) ** 2))

    def dU0(self, x):
        e = np.exp(-self.a * (x - self.r))
        return 2.0 * self.D * self.a * e * (1.0 - e)

    def h(self, x):
        return self.Delta + self.eps_d + float(np.sum(self.g * (x - self.r)))

    def dh(self, x):
        return self.g.copy()

    def _f(self, x):
        return float(np.exp(-np.sum((x - self.c) ** 2 / (4.0 * self.s ** 2))))

    def V(self, x):
        return self.Vbar * self._f(x)

    def dV(self, x):
        df = -self._f(x) * (x - self.c) / (2.0 * self.s ** 2)  # (n_dof,)
        return self.Vbar[:, None] * df[None, :]


class Dense(Model):
    """A one-electron Hamiltonian of any symmetric structure, affine in one
    nuclear coordinate: H(x) = H0 + x H1, dH/dx = H1 (Eq.
    single_electron_discrete_electronic_hamiltonian for a general H; state 0
    is the impurity |d> for the observables), with the harmonic nuclear
    potential U0 = m omega^2 (x - x_c)^2 / 2."""

    def __init__(self, H0, H1, mass, omega, x_c=0.0):
        H0 = np.asarray(H0, dtype=np.float64)
        H1 = np.asarray(H1, dtype=np.float64)
        self.H0, self.H1 = H0.copy(), H1.copy()
        self.n = H0.shape[0]
        self.M = self.n - 1
        self.eps = np.diag(H0)[1:].copy()
        self.mass = np.atleast_1d(np.asarray(mass, dtype=np.float64))
        self.omega, self.x_c = float(omega), float(x_c)
        self.k = self.mass[0] * self.omega ** 2

    def U0(self, x):
        return 0.5 * self.k * (x[0] - self.x_c) ** 2

    def dU0(self, x):
        return np.array([self.k * (x[0] - self.x_c)])

    def H(self, x):
        return self.H0 + np.atleast_1d(x)[0] * self.H1

    def dH(self, x):
        return [self.H1.copy()]


def from_config(cfg: dict, M: int | None = None):
    """Build a model from a workload description (``workloads.configs``)."""
    mcfg, bcfg = cfg["model"], cfg["bath"]
    M = M if M is not None else bcfg["M"]
    if mcfg["kind"] == "dense":
        from workloads import dense_matrices
        H0, H1 = dense_matrices(cfg, M)
        m = Dense(H0, H1, mcfg["mass"], mcfg["omega"], mcfg.get("x_c", 0.0))
        return m
    # chemical potential mu: the band moves with mu ("shift", wide-band limit)
    # or only the Gauss-Legendre split does ("split")
    mu = bcfg.get("mu", 0.0)
    centre = mu if bcfg.get("placement", "shift") == "shift" else 0.0
    leads = bcfg.get("leads", 1)
    if leads == 2:
        # M levels in all: one grid of M/2 levels shared by the two leads
        eps, w = _bath.discretise(bcfg["kind"], M // 2, bcfg["W"], eps_f=mu, centre=centre)
        eps, w, lead = _bath.two_leads(eps, w)
    else:
        eps, w = _bath.discretise(bcfg["kind"], M, bcfg["W"], eps_f=mu, centre=centre)
        lead = None
    if mcfg["kind"] == "harmonic":
        m = Harmonic(eps, w, mcfg["Gamma"], mcfg["mass"], mcfg["omega"], mcfg["g"],
                     mcfg["dG"], mcfg.get("eps_d", 0.0))
    elif mcfg["kind"] == "multi_dof":
        m = MultiDof(eps, w, mcfg["Gamma"], mcfg["dof"], mcfg["Delta"], mcfg.get("eps_d", 0.0))
    elif mcfg["kind"] == "morse_tanh":
        m = MorseTanh(eps, w, mcfg["Gamma"], mcfg["mass"], mcfg["De"], mcfg["x0"],
                      mcfg["a"], mcfg["D1"], mcfg["D2"], mcfg["ap"], mcfg["Vinf"],
                      mcfg["q"], mcfg["atil"], mcfg["xtil"], mcfg["c"],
                      mcfg.get("eps_d", 0.0))
    else:
        raise ValueError(mcfg["kind"])
    m.lead = lead
    return m
