"""Electronic structure and surface hopping pieces of IESH (Sec. II.B, II.C).

Test infrastructure only (see the package docstring).

Conventions (ħ = 1, atomic units):

* Adiabatic orbitals: columns of Q from a dense ``eigh`` of the one-electron
  Hamiltonian, eigenvalues ascending.  The eigenvector phase is silent in
  the paper; the gauge used here makes the impurity component Q[0, j]
  positive (for an orbital with Q[0, j] = 0, the first nonzero component).
* Nonadiabatic coupling: D[j, k] = <j | d/dx k> = G[j, k] / (lambda_k -
  lambda_j) with G = Q^T (dH/dx) Q, D[j, j] = 0.  This is the negative of the
  paper's d_jk, whose definition has the denominator lambda_j - lambda_k;
  the time-dependent Schrodinger equation of Sec. II.B is consistent with its
  own d_jk, and in the notation here it reads
      i dc/dt = A c,  A = diag(lambda) - i v.D.
  Reading: the matrix form of the propagator printed in Sec. II.C places
  -i v d_jk at A[j, k], which is the transpose of what the Schrodinger
  equation it rewrites implies and flips the sign of the coupling.  The form
  used here follows the Schrodinger equation; the diabatic-consistency test
  fixes it from first principles.
* Hopping rate (Eqs. hopping_probability, hopping_rate): the rate from
  configuration K to J is -2 Re(A_KJ) v.<J|d/dx K> / A_KK with
  A_KJ = <K|psi><psi|J>, which is Tully's fewest-switches flux.  Reading:
  the printed rate multiplies Re(A*_kj) by the paper's d_jk = <k|d/dx j>,
  the opposite sign; the many-body flux test fixes the sign.  For J = K with
  orbital a (row r of the overlap matrix) replaced by b, the determinant
  lemma gives <J|psi>/<K|psi> = W[b, r], W = C S^-1, S = C[s, :], so

      g(a -> b) = max(-2 dt (v.D[b, a]) Re W[b, r], 0).

  The brute-force routines below evaluate the printed determinant formula
  literally instead, for tests.
"""
from __future__ import annotations

import itertools

import numpy as np


# --------------------------------------------------------------------------- eigen
def eig(H):
    """Eigenvalues ascending and gauge-fixed eigenvectors (columns)."""
    lam, Q = np.linalg.eigh(H)
    for j in range(Q.shape[1]):
        col = Q[:, j]
        nz = np.flatnonzero(np.abs(col) > 0)
        if col[nz[0]] < 0:
            Q[:, j] = -col
    return lam, Q


def coupling_matrices(lam, Q, dH_list):
    """G^(nu) = Q^T dH^(nu) Q and D^(nu)[j, k] = G[j, k] / (lambda_k - lambda_j).

    Reading: two states of equal energy (to rounding, 1e-12 of the largest
    |lambda|) get D = 0.  The paper's couplings assume distinct energies;
    equal energies arise only for repeated bath levels (two leads on one
    grid), whose extra eigenstates have no impurity part and a fixed
    direction, so that their coupling to every state vanishes."""
    Gs, Ds = [], []
    n = len(lam)
    diff = lam[None, :] - lam[:, None]          # [j, k] -> lambda_k - lambda_j
    off = ~np.eye(n, dtype=bool) & (np.abs(diff) > 1e-12 * np.max(np.abs(lam)))
    for dH in dH_list:
        G = Q.T @ dH @ Q
        D = np.zeros_like(G)
        D[off] = G[off] / diff[off]
        Gs.append(G)
        Ds.append(D)
    return Gs, Ds


def forces(model, x, s, lam=None, Q=None):
    """Hellmann-Feynman force of Eq. classical_hamiltonian:
    F_nu = -dU0/dx_nu - sum_{a in s} G^(nu)[a, a]."""
    x = np.atleast_1d(x)
    if lam is None:
        lam, Q = eig(model.H(x))
    F = -model.dU0(x).astype(np.float64)
    for nu, dH in enumerate(model.dH(x)):
        G = Q.T @ dH @ Q
        F[nu] -= np.sum(np.diag(G)[np.asarray(s)])
    return F


def potential_energy(model, x, s, lam=None):
    x = np.atleast_1d(x)
    if lam is None:
        lam, _ = eig(model.H(x))
    return model.U0(x) + np.sum(lam[np.asarray(s)])


# ---------------------------------------------------------------------- propagation
def propagator_matrix(lam, Ds, v):
    """A = diag(lambda) - i sum_nu v_nu D^(nu) (Hermitian; Sec. II.C with the
    sign fixed as described in the module docstring)."""
    vD = sum(vn * D for vn, D in zip(np.atleast_1d(v), Ds))
    return np.diag(lam).astype(np.complex128) - 1j * vD


def propagate(C, A, dt):
    """C(t + dt) = exp(-i A dt) C(t) through the eigendecomposition of the
    Hermitian A (Eqs. exponential_integrator, fast_exponential_integrator)."""
    mu, P = np.linalg.eigh(A)
    return P @ (np.exp(-1j * mu * dt)[:, None] * (P.conj().T @ C))


def lowdin(C):
    """Symmetric (Loewdin) orthonormalisation C (C^H C)^{-1/2}, the FP64
    correction that the mixed-precision pattern applies to its FP32 orbitals
    every L steps; the inverse square root is taken from the eigenpairs of the
    Hermitian overlap matrix."""
    w, V = np.linalg.eigh(C.conj().T @ C)
    return C @ (V @ np.diag(1.0 / np.sqrt(w)) @ V.conj().T)


# ------------------------------------------------------------------------- hopping
def vdot_D(Ds, v):
    return sum(vn * D for vn, D in zip(np.atleast_1d(v), Ds))


def hop_probabilities(C, s, vD, dt):
    """g[r, b]: probability that the electron in occupied orbital s[r] hops to
    orbital b during dt (zero when b is occupied).  Determinant-ratio form
    of Eqs. hopping_probability and hopping_rate; returns (g, W, detS)."""
    s = np.asarray(s)
    n, N = C.shape
    S = C[s, :]
    # W = C S^-1, solved as S^T W^T = C^T.
    W = np.linalg.solve(S.T, C.T).T
    occ = np.zeros(n, dtype=bool)
    occ[s] = True
    g = np.zeros((N, n))
    for r, a in enumerate(s):
        raw = -2.0 * dt * vD[:, a] * W[:, r].real
        raw[occ] = 0.0
        g[r] = np.maximum(raw, 0.0)
    return g, W, np.linalg.det(S)


def hop_rates_raw(C, s, vD, dt):
    """Like hop_probabilities but without the max(., 0) clip."""
    s = np.asarray(s)
    n, N = C.shape
    W = np.linalg.solve(C[s, :].T, C.T).T
    occ = np.zeros(n, dtype=bool)
    occ[s] = True
    g = np.zeros((N, n))
    for r, a in enumerate(s):
        raw = -2.0 * dt * vD[:, a] * W[:, r].real
        raw[occ] = 0.0
        g[r] = raw
    return g


def _perm_sign(seq):
    seq = list(seq)
    sign = 1
    for i in range(len(seq)):
        for j in range(i + 1, len(seq)):
            if seq[i] > seq[j]:
                sign = -sign
    return sign


def hop_probabilities_bruteforce(C, s, vD, dt):
    """Literal evaluation of Eqs. hopping_probability / hopping_rate with
    <k|psi> = det(S) over sorted configurations and the many-body coupling of
    two determinants that differ in one orbital (Slater-Condon:
    <J|d/dx K> = sign * <b|d/dx a>, sign from sorting J)."""
    s = sorted(int(a) for a in s)
    n, N = C.shape
    g = np.zeros((N, n))
    ck = np.linalg.det(C[s, :])
    Akk = abs(ck) ** 2
    for r, a in enumerate(s):
        for b in range(n):
            if b in s:
                continue
            j_unsorted = list(s)
            j_unsorted[r] = b
            sign = _perm_sign(j_unsorted)
            J = sorted(j_unsorted)
            cj = np.linalg.det(C[J, :])
            Akj = ck * np.conj(cj)
            dJK = sign * vD[b, a]
            g[r, b] = max(-2.0 * Akj.real * dJK * dt / Akk, 0.0)
    return g


def manybody_nac_fd(model, x, K, J, h=1e-5):
    """<J|d/dx K> for N-electron Slater determinants built from sorted orbital
    sets, by central differences of determinant overlaps
    <J(x)|K(x')> = det(Q(x)[:, J]^T Q(x')[:, K]) (one nuclear coordinate)."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    _, Q0 = eig(model.H(x))
    _, Qp = eig(model.H(x + h))
    _, Qm = eig(model.H(x - h))
    op = np.linalg.det(Q0[:, J].T @ Qp[:, K])
    om = np.linalg.det(Q0[:, J].T @ Qm[:, K])
    return (op - om) / (2 * h)


def all_configurations(n, N):
    return [list(c) for c in itertools.combinations(range(n), N)]


# ----------------------------------------------------------------------- selection
def select_hop(g, xi):
    """Pick a hop by comparing cumulative probabilities with one uniform xi.

    Canonical order (the paper only says the probabilities are sampled with
    one uniform number): rows r ascending (occupied orbitals in ascending
    order), then targets b ascending.  The cumulative sum is formed in two
    levels so that it is reproducible in parallel: row totals P_r =
    sum_b g[r, b] (b ascending), then the running sum over rows; the hop is in
    the first row whose running sum exceeds xi, and within that row at the
    first b whose running sum (started from the previous rows' total)
    exceeds xi.  No hop when the grand total does not exceed xi.

    Returns (r, b, margin) or (None, None, margin); margin is the smallest
    distance between xi and any running sum formed, for near-tie bookkeeping.
    """
    N, n = g.shape
    row = np.zeros(N)
    for r in range(N):
        acc = 0.0
        for b in range(n):
            acc += g[r, b]
        row[r] = acc
    cum = 0.0
    margin = np.inf
    for r in range(N):
        prev = cum
        cum = cum + row[r]
        margin = min(margin, abs(cum - xi))
        if cum > xi:
            acc = prev
            for b in range(n):
                if g[r, b] == 0.0:
                    continue
                acc = acc + g[r, b]
                margin = min(margin, abs(acc - xi))
                if acc > xi:
                    return r, b, margin
            # rounding: the row total exceeded xi but the in-row running sum
            # did not; take the last positive entry of the row.
            nz = np.flatnonzero(g[r] > 0)
            return r, int(nz[-1]), 0.0
    return None, None, margin


def rescale(v, mass, d, dE):
    """Momentum change along d (one component per nuclear coordinate) that
    conserves total energy after a hop with electronic energy change dE
    (Sec. II.B).  Solves sum (p - gamma d)^2 / 2m = sum p^2 / 2m - dE and takes
    the root of smaller |gamma|.  Returns (v_new, accepted); a frustrated hop
    (negative discriminant) leaves v unchanged."""
    v = np.atleast_1d(np.asarray(v, dtype=np.float64))
    mass = np.atleast_1d(mass)
    d = np.atleast_1d(np.asarray(d, dtype=np.float64))
    a = np.sum(d * d / (2.0 * mass))
    b = np.sum(v * d)
    disc = b * b - 4.0 * a * dE
    if a == 0.0 or disc < 0.0:
        return v.copy(), False
    root = np.sqrt(disc)
    q = b + (root if b >= 0 else -root)
    gamma = 2.0 * dE / q if q != 0.0 else 0.0
    return v - gamma * d / mass, True
