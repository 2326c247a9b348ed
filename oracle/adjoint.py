"""Gradient of an electronic loss along prescribed nuclear paths (the adjoint
pattern; not in the paper, which has no parameter gradients).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Model: the double-well Newns-Anderson Hamiltonian of Sec. III.B with a
discretised bath (App. A), written directly in its parameters
    theta = [eps_d, Gamma, eps_1 .. eps_M, omega, g, dG]
(the layout of the library's gradient vector):
    h(x) = U1(x) - U0(x) + eps_d = m omega^2 (g^2 - 2 g x) / 2 + dG + eps_d,
    V_k  = sqrt(Gamma w_k / (2 pi))   (the bath weights w_k are fixed),
    H(x) = [[h(x), V^T], [V, diag(eps)]],   dH/dx = h' e0 e0^T, h' = -m omega^2 g.
The nuclear path x_0 .. x_T is prescribed; the electrons follow the IESH
propagator of Sec. II.C with the readings of the dynamics module: over step n
the matrix A = diag(lambda) - i v D is frozen at the midpoint
(x_n + x_{n+1}) / 2 with v = (x_{n+1} - x_n) / dt, and C_{n+1} =
exp(-i A dt) C_n.  The initial orbitals are the unit vectors of the N lowest
adiabatic states at x_0 (occupations n0).

Loss of one path, with term weights (c_P, c_E, c_G, c_F) (default 1, 1, 0, 0):
    L = c_P (1/T) sum_{t=1..T} P(t) + c_E E_exc(T) + c_G (1/T) sum_t G(t) + c_F (1/T) sum_t F(t),
    P(t)    = sum_n |sum_a Q0_a(x_t) C_an(t)|^2          (impurity population),
    E_exc   = sum_a lambda_a(x_T) (rho_aa - n0_a),  rho_aa = sum_n |C_an(T)|^2,
    G(t)    = sum_{a occupied, b not} g_ab(t)          (accumulated hop probability),
    g_ab    = max(-2 dt v_t D_ba(x_t) Re W_b,r(a), 0),  W = C_U S^-1 (Eqs.
              hopping_probability and hopping_rate, determinant-ratio form),
    F(t)    = -dU0/dx(x_t) - h'(x_t) sum_{a occupied} Q0_a(x_t)^2
              (Hellmann-Feynman force, Eq. classical_hamiltonian),
with the occupations n0 held along the path (no hops), v_t = (x_t - x_{t-1})/dt
and D_jk = h' Q0_j Q0_k / (lambda_k - lambda_j) at x_t.

``loss`` evaluates it plainly; ``tangent`` propagates one directional
derivative alongside (forward mode): eigenvalue and eigenvector perturbation
of the dense H, the derivative of the couplings, and the Frechet derivative
of the matrix exponential from the eigendecomposition of A,
    L(X, E) = P (Phi o (P^H E P)) P^H,  Phi_jk = (e^{x_j} - e^{x_k}) / (x_j - x_k).
Pins: central finite differences of ``loss`` for every term; d L / d eps_d =
d L / d dG (both only shift h, in every term); G(t) against the oracle's determinant-ratio hop probabilities and F(t)
against its Hellmann-Feynman force, both computed from the dense model.
"""
from __future__ import annotations

import numpy as np

from .electronic import eig

__all__ = ["Params", "hamiltonian", "loss", "tangent", "n_params", "pack", "unpack"]


class Params:
    def __init__(self, eps_d, Gamma, eps, omega, g, dG, w, mass):
        self.eps_d = float(eps_d)
        self.Gamma = float(Gamma)
        self.eps = np.asarray(eps, dtype=np.float64).copy()
        self.omega = float(omega)
        self.g = float(g)
        self.dG = float(dG)
        self.w = np.asarray(w, dtype=np.float64).copy()
        self.mass = float(mass)


def n_params(M):
    return M + 5


def pack(p: Params):
    return np.concatenate([[p.eps_d, p.Gamma], p.eps, [p.omega, p.g, p.dG]])


def unpack(theta, w, mass):
    M = len(w)
    return Params(theta[0], theta[1], theta[2:2 + M], theta[2 + M], theta[3 + M], theta[4 + M], w, mass)


def hamiltonian(p: Params, x):
    """H(x) and h' (the only x-dependent element is h)."""
    M = len(p.eps)
    H = np.zeros((M + 1, M + 1))
    H[0, 0] = 0.5 * p.mass * p.omega ** 2 * (p.g ** 2 - 2.0 * p.g * x) + p.dG + p.eps_d
    V = np.sqrt(p.Gamma * p.w / (2.0 * np.pi))
    H[0, 1:] = V
    H[1:, 0] = V
    H[1:, 1:] = np.diag(p.eps)
    hp = -p.mass * p.omega ** 2 * p.g
    return H, hp


def hamiltonian_dir(p: Params, d: Params, x):
    """Directional derivative of (H(x), h') along the parameter direction d
    (d holds the parameter increments; w and mass are fixed)."""
    M = len(p.eps)
    dH = np.zeros((M + 1, M + 1))
    m, om, g = p.mass, p.omega, p.g
    dH[0, 0] = (m * om * d.omega * (g ** 2 - 2.0 * g * x) + 0.5 * m * om ** 2 * (2.0 * g - 2.0 * x) * d.g
                + d.dG + d.eps_d)
    V = np.sqrt(p.Gamma * p.w / (2.0 * np.pi))
    dV = 0.5 * V / p.Gamma * d.Gamma
    dH[0, 1:] = dV
    dH[1:, 0] = dV
    dH[1:, 1:] = np.diag(d.eps)
    dhp = -m * (2.0 * om * d.omega * g + om ** 2 * d.g)
    return dH, dhp


def _couplings(lam, Q, hp):
    n = len(lam)
    q0 = Q[0, :]
    G = hp * np.outer(q0, q0)
    diff = lam[None, :] - lam[:, None]
    D = np.zeros((n, n))
    off = ~np.eye(n, dtype=bool)
    D[off] = G[off] / diff[off]
    return D


def _initial(p, x0, N):
    H, _ = hamiltonian(p, x0)
    lam, Q = eig(H)
    n = len(lam)
    C = np.zeros((n, N), dtype=np.complex128)
    for i in range(N):
        C[i, i] = 1.0
    n0 = np.zeros(n)
    n0[:N] = 1.0
    return C, n0


def _hop_sum(C, N, D, v, dt):
    """G = sum of the hop probabilities out of the occupied orbitals 0 .. N-1
    (the N lowest, so r(a) = a) into every other orbital."""
    S, CU = C[:N, :], C[N:, :]
    W = CU @ np.linalg.inv(S)
    y = -2.0 * dt * v * D[N:, :N] * W.real
    return np.sum(np.maximum(y, 0.0))


def _force(p: Params, x, q0, N, hp):
    return -p.mass * p.omega ** 2 * x - hp * np.sum(q0[:N] ** 2)


def loss(p: Params, path, N, dt, terms=(1.0, 1.0, 0.0, 0.0), history=None):
    """Loss of one prescribed path x_0 .. x_T (array of T + 1 positions).

    history: optional list that receives, per step s = 1 .. T, a dict with the
    orbitals C(s) and the population P(s), and at s = T also E_exc (for tests
    that check the forward pass against the dynamics oracle)."""
    cP, cE, cG, cF = terms
    T = len(path) - 1
    C, n0 = _initial(p, path[0], N)
    total = 0.0
    for s in range(T):
        xm = 0.5 * (path[s] + path[s + 1])
        v = (path[s + 1] - path[s]) / dt
        H, hp = hamiltonian(p, xm)
        lam, Q = eig(H)
        D = _couplings(lam, Q, hp)
        A = np.diag(lam).astype(np.complex128) - 1j * v * D
        mu, P = np.linalg.eigh(A)
        C = P @ (np.exp(-1j * mu * dt)[:, None] * (P.conj().T @ C))
        H1, hp1 = hamiltonian(p, path[s + 1])
        lam1, Q1 = eig(H1)
        z = C.T @ Q1[0, :]
        Pt = np.sum(np.abs(z) ** 2)
        total += cP * Pt / T
        if history is not None:
            history.append(dict(C=C.copy(), P=Pt))
        if cG:
            total += cG * _hop_sum(C, N, _couplings(lam1, Q1, hp1), v, dt) / T
        if cF:
            total += cF * _force(p, path[s + 1], Q1[0, :], N, hp1) / T
        if s == T - 1:
            rho = np.sum(np.abs(C) ** 2, axis=1)
            E_exc = np.sum(lam1 * (rho - n0))
            total += cE * E_exc
            if history is not None:
                history[-1]["E_exc"] = E_exc
    return total


def _eig_dir(lam, Q, dH):
    """Directional derivatives of the eigenvalues and of the gauge-fixed
    eigenvectors of a real symmetric matrix with simple spectrum."""
    n = len(lam)
    R = Q.T @ dH @ Q
    dlam = np.diag(R).copy()
    diff = lam[:, None] - lam[None, :]  # [k, j] -> lambda_k - lambda_j
    F = np.zeros((n, n))
    off = ~np.eye(n, dtype=bool)
    F[off] = 1.0 / (-diff[off])          # 1 / (lambda_j - lambda_k) at [k, j]
    dQ = Q @ (F * R)                     # column j: sum_k Q_k R_kj / (lambda_j - lambda_k)
    return dlam, dQ


def _frechet_exp(mu, P, E, dt):
    """Frechet derivative of exp at X = -i A dt (A = P diag(mu) P^H) in the
    direction E."""
    xv = -1j * mu * dt
    ex = np.exp(xv)
    d = xv[:, None] - xv[None, :]
    num = ex[:, None] - ex[None, :]
    Phi = np.empty_like(num)
    small = np.abs(d) < 1e-300
    Phi[~small] = num[~small] / d[~small]
    Phi[small] = np.broadcast_to(ex[:, None], num.shape)[small]
    return P @ (Phi * (P.conj().T @ E @ P)) @ P.conj().T


def _coupling_dir(lam, q0, hp, dlam, dq0, dhp):
    """D and its directional derivative from (lambda, q0, h') and theirs."""
    n = len(lam)
    diff = lam[None, :] - lam[:, None]
    ddiff = dlam[None, :] - dlam[:, None]
    off = ~np.eye(n, dtype=bool)
    G = hp * np.outer(q0, q0)
    dG = dhp * np.outer(q0, q0) + hp * (np.outer(dq0, q0) + np.outer(q0, dq0))
    D = np.zeros((n, n))
    dD = np.zeros((n, n))
    D[off] = G[off] / diff[off]
    dD[off] = (dG[off] - D[off] * ddiff[off]) / diff[off]
    return D, dD


def tangent(p: Params, d: Params, path, N, dt, terms=(1.0, 1.0, 0.0, 0.0)):
    """(loss, directional derivative of the loss along d), forward mode."""
    cP, cE, cG, cF = terms
    T = len(path) - 1
    C, n0 = _initial(p, path[0], N)
    dC = np.zeros_like(C)
    total = 0.0
    dtotal = 0.0
    for s in range(T):
        xm = 0.5 * (path[s] + path[s + 1])
        v = (path[s + 1] - path[s]) / dt
        H, hp = hamiltonian(p, xm)
        dH, dhp = hamiltonian_dir(p, d, xm)
        lam, Q = eig(H)
        dlam, dQ = _eig_dir(lam, Q, dH)
        q0, dq0 = Q[0, :], dQ[0, :]
        n = len(lam)
        diff = lam[None, :] - lam[:, None]
        ddiff = dlam[None, :] - dlam[:, None]
        off = ~np.eye(n, dtype=bool)
        G = hp * np.outer(q0, q0)
        dG = dhp * np.outer(q0, q0) + hp * (np.outer(dq0, q0) + np.outer(q0, dq0))
        D = np.zeros((n, n))
        dD = np.zeros((n, n))
        D[off] = G[off] / diff[off]
        dD[off] = (dG[off] - D[off] * ddiff[off]) / diff[off]
        A = np.diag(lam).astype(np.complex128) - 1j * v * D
        dA = np.diag(dlam).astype(np.complex128) - 1j * v * dD
        mu, P = np.linalg.eigh(A)
        U = P @ np.diag(np.exp(-1j * mu * dt)) @ P.conj().T
        dU = _frechet_exp(mu, P, -1j * dt * dA, dt)
        dC = U @ dC + dU @ C
        C = U @ C
        H1, hp1 = hamiltonian(p, path[s + 1])
        dH1, dhp1 = hamiltonian_dir(p, d, path[s + 1])
        lam1, Q1 = eig(H1)
        dlam1, dQ1 = _eig_dir(lam1, Q1, dH1)
        z = C.T @ Q1[0, :]
        dz = dC.T @ Q1[0, :] + C.T @ dQ1[0, :]
        total += cP * np.sum(np.abs(z) ** 2) / T
        dtotal += cP * 2.0 * np.sum((z.conj() * dz).real) / T
        if cG:
            D1, dD1 = _coupling_dir(lam1, Q1[0, :], hp1, dlam1, dQ1[0, :], dhp1)
            X = np.linalg.inv(C[:N, :])
            W = C[N:, :] @ X
            dW = (dC[N:, :] - W @ dC[:N, :]) @ X
            y = -2.0 * dt * v * D1[N:, :N] * W.real
            dy = -2.0 * dt * v * (dD1[N:, :N] * W.real + D1[N:, :N] * dW.real)
            total += cG * np.sum(np.maximum(y, 0.0)) / T
            dtotal += cG * np.sum(np.where(y > 0.0, dy, 0.0)) / T
        if cF:
            q0 = Q1[0, :N]
            total += cF * _force(p, path[s + 1], Q1[0, :], N, hp1) / T
            dF = (-p.mass * 2.0 * p.omega * d.omega * path[s + 1] - dhp1 * np.sum(q0 ** 2)
                  - hp1 * 2.0 * np.sum(q0 * dQ1[0, :N]))
            dtotal += cF * dF / T
        if s == T - 1:
            rho = np.sum(np.abs(C) ** 2, axis=1)
            drho = 2.0 * np.sum((C.conj() * dC).real, axis=1)
            total += cE * np.sum(lam1 * (rho - n0))
            dtotal += cE * np.sum(dlam1 * (rho - n0) + lam1 * drho)
    return total, dtotal


def gradient(p: Params, path, N, dt, terms=(1.0, 1.0, 0.0, 0.0)):
    """Full gradient by one tangent sweep per parameter (test sizes only)."""
    M = len(p.eps)
    g = np.zeros(n_params(M))
    for i in range(n_params(M)):
        e = np.zeros(n_params(M))
        e[i] = 1.0
        d = unpack(e, p.w, p.mass)
        g[i] = tangent(p, d, path, N, dt, terms)[1]
    return g
