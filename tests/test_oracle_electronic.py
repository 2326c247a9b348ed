"""Oracle pins: couplings, forces, propagation, hop probabilities (CPU only)."""
import math

import numpy as np
import pytest
from scipy.linalg import expm

from oracle import bath, models, closed_forms, fssh2
from oracle import electronic as el
from oracle import dynamics as dyn
from workloads import configs as wc
from workloads.sampling import random_orbitals


def small_model(M=6, Gamma=0.02, W=0.1, kind="trapezoid_midpoint"):
    eps, w = bath.discretise(kind, M, W)
    return models.Harmonic(eps, w, Gamma, 2000.0, 2e-4, 20.0, -3.8e-3)


def morse_model(M=8):
    cfg = wc.get_config("c3")
    return models.from_config(cfg, M=M)


# ------------------------------------------------------------------ couplings
@pytest.mark.parametrize("which", ["harmonic", "morse"])
def test_nac_matches_fd_of_eigenvectors(which):
    """D[j, k] = <j|d/dx k> equals the central difference of gauge-fixed
    eigenvectors, and is antisymmetric."""
    m = small_model() if which == "harmonic" else morse_model()
    xs = [-3.0, 4.0, 9.0] if which == "harmonic" else [3.0, 4.5, 7.0]
    h = 1e-6
    for x in xs:
        X = np.array([x])
        lam, Q = el.eig(m.H(X))
        _, Ds = el.coupling_matrices(lam, Q, m.dH(X))
        _, Qp = el.eig(m.H(X + h))
        _, Qm = el.eig(m.H(X - h))
        fd = Q.T @ (Qp - Qm) / (2 * h)
        scale = np.max(np.abs(Ds[0]))
        assert np.max(np.abs(Ds[0] - fd)) < 1e-6 * scale
        assert np.max(np.abs(Ds[0] + Ds[0].T)) < 1e-14 * scale


@pytest.mark.parametrize("which", ["harmonic", "morse"])
def test_hellmann_feynman_force(which):
    """F = -dU0/dx - sum_{a in s} G_aa equals -dE_pot/dx by central difference
    (Eq. classical_hamiltonian)."""
    m = small_model() if which == "harmonic" else morse_model()
    xs = [-3.0, 4.0] if which == "harmonic" else [3.2, 6.0]
    for x in xs:
        for s in ([0, 1, 2], [1, 3, 5], [0, 4, 6]):
            X = np.array([x])
            F = el.forces(m, X, s)
            h = 1e-5
            fd = -(el.potential_energy(m, X + h, s) - el.potential_energy(m, X - h, s)) / (2 * h)
            assert abs(F[0] - fd) < 1e-7 * max(1e-4, abs(F[0]))


# ---------------------------------------------------------------- propagation
def test_propagation_unitary_and_matches_expm():
    m = small_model(M=9)
    X = np.array([2.0])
    lam, Q = el.eig(m.H(X))
    _, Ds = el.coupling_matrices(lam, Q, m.dH(X))
    C = random_orbitals(m.n, 4, seed=3)
    A = el.propagator_matrix(lam, Ds, [0.01])
    assert np.max(np.abs(A - A.conj().T)) < 1e-18
    for dt in (1.0, 50.0, 400.0):
        C1 = el.propagate(C, A, dt)
        assert np.max(np.abs(C1.conj().T @ C1 - np.eye(4))) < 1e-13
        assert np.max(np.abs(C1 - expm(-1j * A * dt) @ C)) < 1e-12


def test_zero_velocity_gives_phases_and_no_hops():
    m = small_model(M=9)
    X = np.array([1.0])
    lam, Q = el.eig(m.H(X))
    _, Ds = el.coupling_matrices(lam, Q, m.dH(X))
    C = random_orbitals(m.n, 4, seed=5)
    A = el.propagator_matrix(lam, Ds, [0.0])
    C1 = el.propagate(C, A, 30.0)
    assert np.max(np.abs(C1 - np.exp(-1j * lam * 30.0)[:, None] * C)) < 1e-13
    g, _, _ = el.hop_probabilities(C1, [0, 2, 5, 7], el.vdot_D(Ds, [0.0]), 30.0)
    assert np.all(g == 0.0)


def _diabatic_reference(m, path, T, c_ad0, n_fine=40000):
    """Exact-in-the-limit diabatic propagation of one orbital along x(t):
    midpoint exponential of H(x) with a very fine step, then projected on the
    adiabatic basis at the end point."""
    dt = T / n_fine
    _, Q0 = el.eig(m.H(np.array([path(0.0)])))
    c = Q0 @ c_ad0
    for k in range(n_fine):
        H = m.H(np.array([path((k + 0.5) * dt)]))
        w, P = np.linalg.eigh(H)
        c = P @ (np.exp(-1j * w * dt) * (P.T @ c))
    _, QT = el.eig(m.H(np.array([path(T)])))
    return QT.T @ c


def _adiabatic(m, path, T, c0, nsteps, sign=+1.0):
    dt = T / nsteps
    c = c0.astype(complex)
    for k in range(nsteps):
        xa, xb = path(k * dt), path((k + 1) * dt)
        xm = np.array([0.5 * (xa + xb)])
        lam, Q = el.eig(m.H(xm))
        _, Ds = el.coupling_matrices(lam, Q, m.dH(xm))
        A = np.diag(lam) - 1j * sign * ((xb - xa) / dt) * Ds[0]
        w, P = np.linalg.eigh(A)
        c = P @ (np.exp(-1j * w * dt) * (P.conj().T @ c))
    return c


def test_diabatic_consistency_fixes_propagator_sign_and_order():
    """The adiabatic exponential integrator with A = diag(lambda) - i v D,
    frozen at the step midpoint, converges at second order to the exact
    diabatic propagation; the transposed (sign-flipped) form does not
    converge at all."""
    m = small_model(M=5, Gamma=0.02)
    path = lambda t: -8.0 + 0.012 * t + 1.5 * math.sin(0.004 * t)
    T = 1500.0
    c0 = np.zeros(m.n, dtype=complex)
    c0[2] = 1.0
    ref = _diabatic_reference(m, path, T, c0)
    errs = [np.linalg.norm(_adiabatic(m, path, T, c0, n) - ref) for n in (50, 100, 200)]
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5
    assert errs[2] < 1e-3
    bad = [np.linalg.norm(_adiabatic(m, path, T, c0, n, sign=-1.0) - ref) for n in (100, 200)]
    assert min(bad) > 100 * errs[2]


# ---------------------------------------------------------------- hop probabilities
def _random_state(seed, M=6, N=3, x=2.0, v=0.02):
    m = small_model(M=M, Gamma=0.03)
    X = np.array([x])
    lam, Q = el.eig(m.H(X))
    _, Ds = el.coupling_matrices(lam, Q, m.dH(X))
    C = random_orbitals(m.n, N, seed=seed)
    return m, X, lam, Q, Ds, C, np.array([v])


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_ratio_formula_equals_bruteforce_determinants(seed):
    m, X, lam, Q, Ds, C, v = _random_state(seed)
    vD = el.vdot_D(Ds, v)
    rng = np.random.default_rng(seed)
    for _ in range(4):
        s = np.sort(rng.choice(m.n, 3, replace=False))
        g, _, _ = el.hop_probabilities(C, s, vD, 10.0)
        gb = el.hop_probabilities_bruteforce(C, s, vD, 10.0)
        assert np.max(np.abs(g - gb)) < 1e-13 * max(1.0, np.max(gb))
        assert np.any(g > 0)


@pytest.mark.parametrize("eps_rot", [0.05, 0.15, 0.3])
def test_no_hop_bound_is_an_upper_bound_of_the_total(eps_rot):
    """The bound that lets a step skip the ratios (Eq. hopping-estimate, with
    Cauchy-Schwarz over the occupied orbitals):
        sum g <= 2 dt sum_{b unocc} ||C[b, :]|| (sum_r |vD[b, s_r]|^2)^(1/2) / s_min,
        s_min^2 = 1 - ||C_U||_F^2 <= sigma_min(S)^2,
    checked against the oracle's determinant-ratio probabilities on orthonormal
    orbitals rotated away from the occupied unit vectors (larger rotations,
    larger C_U); the l2 form never exceeds the l1 form sum_r |vD|."""
    m, X, lam, Q, Ds, _, v = _random_state(0)
    rs = np.random.default_rng(7)
    N, dt = 3, 10.0
    checked = 0
    for trial in range(20):
        K = rs.normal(size=(m.n, m.n)) + 1j * rs.normal(size=(m.n, m.n))
        U = expm(1j * eps_rot * (K + K.conj().T) / 2)
        s = np.sort(rs.choice(m.n, N, replace=False))
        C = U[:, s]
        vD = el.vdot_D(Ds, v * (1.0 + 5.0 * trial))
        g, _, _ = el.hop_probabilities(C, s, vD, dt)
        unocc = np.setdiff1d(np.arange(m.n), s)
        rn = np.linalg.norm(C[unocc, :], axis=1)
        smin2 = 1.0 - np.sum(rn ** 2)
        if smin2 <= 0.0:
            continue
        assert np.linalg.svd(C[s, :], compute_uv=False)[-1] ** 2 >= smin2 - 1e-12
        l2 = np.sqrt(np.sum(vD[np.ix_(unocc, s)] ** 2, axis=1))
        l1 = np.sum(np.abs(vD[np.ix_(unocc, s)]), axis=1)
        bound = 2.0 * dt * np.sum(rn * l2) / np.sqrt(smin2)
        assert np.sum(g) <= bound * (1 + 1e-12)
        assert bound <= 2.0 * dt * np.sum(rn * l1) / np.sqrt(smin2) * (1 + 1e-15)
        checked += 1
    assert checked >= 5


def test_ratio_formula_equals_literal_manybody_fd():
    """Same as above but with the many-body coupling <J|d/dx K> taken by
    finite differences of N-electron determinant overlaps, with no
    Slater-Condon shortcut."""
    m, X, lam, Q, Ds, C, v = _random_state(7, M=5, N=2)
    vD = el.vdot_D(Ds, v)
    dt = 10.0
    for K in ([0, 3], [1, 2], [2, 5]):
        g, _, _ = el.hop_probabilities(C, K, vD, dt)
        cK = np.linalg.det(C[K, :])
        for r, a in enumerate(K):
            for b in range(m.n):
                if b in K:
                    continue
                J = sorted([c for c in K if c != a] + [b])
                dJK = el.manybody_nac_fd(m, X, K, J, h=1e-5) * v[0]
                cJ = np.linalg.det(C[J, :])
                lit = max(-2.0 * (cK * np.conj(cJ)).real * dJK * dt / abs(cK) ** 2, 0.0)
                assert abs(lit - g[r, b]) < 1e-6 * max(1e-3, abs(lit))


def test_manybody_flux_fixes_hop_sign():
    """d|<J|psi>|^2/dt = sum over single excitations K -> J of the
    pairwise rates P_K g_raw(K, a->b)/dt, for every configuration J."""
    m, X, lam, Q, Ds, C, v = _random_state(11, M=5, N=3, v=0.03)
    A = el.propagator_matrix(lam, Ds, v)
    vD = el.vdot_D(Ds, v)
    n, N = C.shape
    configs = el.all_configurations(n, N)
    h = 1e-3
    Cp = expm(-1j * A * h) @ C
    Cm = expm(1j * A * h) @ C
    P = {tuple(J): abs(np.linalg.det(C[J, :])) ** 2 for J in configs}
    worst, scale = 0.0, 0.0
    flux = {tuple(J): 0.0 for J in configs}
    for K in configs:
        raw = el.hop_rates_raw(C, K, vD, 1.0)
        for r, a in enumerate(K):
            for b in range(n):
                if b in K:
                    continue
                J = tuple(sorted([c for c in K if c != a] + [b]))
                flux[J] += P[tuple(K)] * raw[r, b]
    for J in configs:
        dP = (abs(np.linalg.det(Cp[J, :])) ** 2 - abs(np.linalg.det(Cm[J, :])) ** 2) / (2 * h)
        worst = max(worst, abs(dP - flux[tuple(J)]))
        scale = max(scale, abs(dP))
    assert scale > 1e-4
    assert worst < 1e-6 * scale
    # the opposite sign convention violates the identity
    worst_flipped = max(abs((abs(np.linalg.det(Cp[J, :])) ** 2 - abs(np.linalg.det(Cm[J, :])) ** 2) / (2 * h)
                            + flux[tuple(J)]) for J in configs)
    assert worst_flipped > 0.5 * scale


def test_single_electron_reduces_to_fewest_switches():
    m, X, lam, Q, Ds, C, v = _random_state(4, M=6, N=1)
    vD = el.vdot_D(Ds, v)
    c = C[:, 0]
    for a in range(m.n):
        g, _, _ = el.hop_probabilities(C, [a], vD, 5.0)
        for b in range(m.n):
            ref = 0.0 if b == a else max(-2 * 5.0 * vD[b, a] * (c[b] * np.conj(c[a])).real / abs(c[a]) ** 2, 0.0)
            assert abs(g[0, b] - ref) < 1e-13 * max(1.0, abs(ref))


def test_two_state_limit_equals_tully_fssh():
    """M = 1, N = 1: the general oracle and the closed-form two-state FSSH
    code produce the same trajectory, hop for hop, with the same uniforms."""
    # weak coupling (V = 5e-4) so that the crossing near x = 10 is strongly
    # nonadiabatic and hops happen
    eps, w = np.array([0.0]), np.array([0.05])
    m = models.Harmonic(eps, w, 2 * math.pi * 2.5e-7 / 0.05, 2000.0, 2e-4, 20.0, -3.8e-3)
    from oracle import rng
    total_hops = 0
    for traj, (x0, v0) in enumerate([(-12.0, 0.006), (-20.0, 0.009), (25.0, -0.008)]):
        st = dyn.State([x0], [v0], np.array([[1.0], [0.0]], dtype=complex), [0])
        x, v, c, a = x0, v0, np.array([1.0, 0.0], dtype=complex), 0
        F = None
        F2 = None
        n_hops = 0
        for k in range(1500):
            xi = rng.uniform(0, traj, k)
            st, ev, F = dyn.step(m, st, 10.0, xi, F)
            x, v, c, a, ev2, F2 = fssh2.step(m, x, v, c, a, 10.0, xi, F2)
            assert ev["accepted"] == ev2["accepted"]
            if ev["attempted"]:
                assert ev2["attempted"]
            n_hops += ev["accepted"]
            assert int(st.s[0]) == a
            assert abs(st.x[0] - x) < 1e-9 * max(1.0, abs(x))
            assert abs(st.v[0] - v) < 1e-9 * max(1e-3, abs(v))
            assert np.max(np.abs(st.C[:, 0] - c)) < 1e-9
        total_hops += n_hops
    assert total_hops >= 2


# --------------------------------------------------------------- selection, rescale
def test_selection_canonical_order():
    g = np.array([[0.0, 0.1, 0.2], [0.3, 0.0, 0.05]])
    assert el.select_hop(g, 0.05)[:2] == (0, 1)
    assert el.select_hop(g, 0.15)[:2] == (0, 2)
    assert el.select_hop(g, 0.35)[:2] == (1, 0)
    assert el.select_hop(g, 0.62)[:2] == (1, 2)
    assert el.select_hop(g, 0.66)[:2] == (None, None)
    assert el.select_hop(np.zeros((2, 3)), 0.0)[:2] == (None, None)


def _sequential_selection(g, xi):
    """The plain rule (one uniform, Sec. II.B): one running sum over every
    pair in the canonical order (rows ascending, then targets ascending); the
    first pair whose running sum exceeds xi."""
    acc = 0.0
    for r in range(g.shape[0]):
        for b in range(g.shape[1]):
            acc += g[r, b]
            if g[r, b] > 0.0 and acc > xi:
                return r, b
    return None, None


def test_two_level_selection_equals_the_sequential_cumulative_sum():
    """The two-level running sum of select_hop (row totals, then within the
    row) picks the same pair as the plain sequential cumulative sum wherever
    no running sum of either order lies within rounding of xi."""
    rs = np.random.default_rng(11)
    compared = hops = 0
    for trial in range(3000):
        N, n = rs.integers(1, 9), rs.integers(2, 30)
        g = rs.exponential(size=(N, n)) * (rs.random((N, n)) < 0.4)
        g *= rs.uniform(0.05, 1.5) / max(g.sum(), 1e-300)
        xi = rs.random() if trial % 3 else rs.uniform(0.0, 1.2 * g.sum())
        r, b, margin = el.select_hop(g, xi)
        flat = np.cumsum(g.ravel())
        if margin < 1e-12 or np.min(np.abs(flat - xi)) < 1e-12:
            continue
        compared += 1
        hops += r is not None
        assert (r, b) == _sequential_selection(g, xi), trial
    assert compared > 2900 and 500 < hops < compared


def test_rescale_conserves_energy_and_frustration():
    mass = np.array([2000.0, 100.0])
    v = np.array([0.01, -0.02])
    d = np.array([0.3, 1.7])
    for dE in (1e-3, -2e-2, 0.0):
        v2, ok = el.rescale(v, mass, d, dE)
        assert ok
        assert abs(0.5 * np.sum(mass * v2 ** 2) - (0.5 * np.sum(mass * v ** 2) - dE)) < 1e-15
        # the new momentum differs from the old along d
        dp = mass * (v2 - v)
        assert abs(dp[0] * d[1] - dp[1] * d[0]) < 1e-14
    v2, ok = el.rescale(v, mass, d, 1.0)
    assert not ok and np.all(v2 == v)
    # 1D closed form
    v1, ok = el.rescale([0.004], [2000.0], [5.0], 0.01)
    assert ok and abs(v1[0] - math.sqrt(0.004 ** 2 - 2 * 0.01 / 2000.0)) < 1e-16
    v1, ok = el.rescale([-0.004], [2000.0], [-3.0], -0.01)
    assert ok and abs(v1[0] + math.sqrt(0.004 ** 2 + 2 * 0.01 / 2000.0)) < 1e-16


# ------------------------------------------------------------------- equilibrium
@pytest.mark.parametrize("h0", [-0.01, 0.004, 0.015])
def test_equilibrium_impurity_occupation_closed_form(h0):
    """n_d = sum_a f(lambda_a - mu) |Q[0, a]|^2 of the discretised model
    approaches the Lorentzian-broadened Fermi integral (digamma closed form)
    for a band much wider than Gamma and level spacing well below kT."""
    Gamma, W, M, kT = 0.01, 1.0, 2000, 0.004
    eps, w = bath.trapezoid_midpoint(M, -W / 2, W / 2)
    V = bath.couplings(Gamma, w)
    H = np.diag(np.concatenate([[h0], eps]))
    H[0, 1:] = V
    H[1:, 0] = V
    lam, Q = el.eig(H)
    nd = np.sum(dyn.fermi(lam, 0.0, kT) * Q[0] ** 2)
    ref = closed_forms.impurity_occupation(h0, Gamma, 0.0, kT)
    # finite band: spectral weight 2 Gamma / (pi W) lies outside the band
    assert abs(nd - ref) < 2 * Gamma / (math.pi * W)
    # a wrong hybridisation normalisation (missing 2 pi) is far off
    ref_bad = closed_forms.impurity_occupation(h0, Gamma / (2 * math.pi), 0.0, kT)
    assert abs(nd - ref_bad) > 5 * abs(nd - ref)


def test_digamma_closed_form_limits():
    assert abs(closed_forms.impurity_occupation(0.0, 0.01, 0.0, 1e-3) - 0.5) < 1e-15
    for h in (-0.02, 0.003, 0.05):
        t0 = closed_forms.impurity_occupation(h, 0.01, 0.0, 0.0)
        tsmall = closed_forms.impurity_occupation(h, 0.01, 0.0, 1e-7)
        assert abs(t0 - tsmall) < 1e-7


def test_lowdin_is_the_polar_factor():
    """C (C^H C)^{-1/2} equals the unitary polar factor U V^H of the SVD
    C = U S V^H (an independent closed form), is orthonormal, commutes with a
    unitary acting from the left, and leaves orthonormal orbitals unchanged."""
    rs = np.random.default_rng(5)
    n, N = 17, 6
    C = rs.normal(size=(n, N)) + 1j * rs.normal(size=(n, N))
    L = el.lowdin(C)
    U, _, Vh = np.linalg.svd(C, full_matrices=False)
    assert np.allclose(L, U @ Vh, atol=1e-12)
    assert np.allclose(L.conj().T @ L, np.eye(N), atol=1e-12)
    Q, _ = np.linalg.qr(rs.normal(size=(n, n)) + 1j * rs.normal(size=(n, n)))
    assert np.allclose(el.lowdin(Q @ C), Q @ L, atol=1e-12)
    assert np.allclose(el.lowdin(L), L, atol=1e-12)
