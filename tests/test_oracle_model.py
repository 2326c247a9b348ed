"""Oracle pins: bath discretisation, model constants, eigen-solve (CPU only)."""
import json
import math
import os

import numpy as np
import pytest
from scipy.optimize import brentq

from oracle import bath, models, closed_forms
from oracle import electronic as el
from workloads import configs as wc

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _paper():
    with open(os.path.join(GOLDEN, "paper_values.json")) as f:
        return json.load(f)


# ----------------------------------------------------------------- discretisation
@pytest.mark.parametrize("M", [1, 7, 20, 200])
def test_trapezoid_grid(M):
    W = 0.1
    eps, w = bath.trapezoid(M, -W / 2, W / 2)
    assert eps[0] == -W / 2
    assert np.allclose(np.diff(eps), W / M, rtol=0, atol=1e-15)
    assert math.isclose(w.sum(), W, rel_tol=1e-14)
    assert eps[-1] < W / 2


@pytest.mark.parametrize("M", [2, 8, 40, 200])
def test_gauss_legendre_weights_sum_and_exactness(M):
    """Each half integrates polynomials up to degree M-1 exactly: check the
    moments against the closed form of int eps^p over both halves."""
    W = 0.1
    a, b = -W / 2, W / 2
    eps, w = bath.gauss_legendre(M, a, b, 0.0)
    assert np.all(w > 0)
    assert np.all(np.diff(eps) > 0)
    assert math.isclose(w.sum(), W, rel_tol=1e-13)
    half = M // 2
    lo, hi = slice(0, half), slice(half, M)
    for p in range(0, M):
        exact_lo = (0.0 ** (p + 1) - a ** (p + 1)) / (p + 1)
        exact_hi = (b ** (p + 1) - 0.0 ** (p + 1)) / (p + 1)
        scale = (W / 2) ** (p + 1)
        assert abs(np.sum(w[lo] * eps[lo] ** p) - exact_lo) <= 1e-13 * scale
        assert abs(np.sum(w[hi] * eps[hi] ** p) - exact_hi) <= 1e-13 * scale


def test_gauss_legendre_offcentre_split():
    eps, w = bath.gauss_legendre(10, -1.0, 3.0, 0.5)
    assert math.isclose(w[:5].sum(), 1.5, rel_tol=1e-14)
    assert math.isclose(w[5:].sum(), 2.5, rel_tol=1e-14)
    assert eps[4] < 0.5 < eps[5]


@pytest.mark.parametrize("kind", ["trapezoid_midpoint", "gauss_legendre"])
def test_discrete_hybridisation_function(kind):
    """Lambda(E) = sum_k V_k^2/(E - eps_k) approaches the continuum
    (Gamma/2pi) ln((E - a)/(E - b)) for E outside the band (Appendix A)."""
    Gamma, W, E = 0.01, 0.1, 0.08
    exact = Gamma / (2 * math.pi) * math.log((E + W / 2) / (E - W / 2))
    errs = []
    for M in (20, 80, 320):
        eps, w = bath.discretise(kind, M, W)
        V = bath.couplings(Gamma, w)
        errs.append(abs(np.sum(V ** 2 / (E - eps)) - exact))
    assert errs[-1] < 1e-3 * abs(exact)
    assert errs[2] < errs[0]


def test_coupling_sum_rule():
    for kind in ("trapezoid", "gauss_legendre"):
        eps, w = bath.discretise(kind, 40, 0.1)
        V = bath.couplings(0.0064, w)
        assert math.isclose(np.sum(V ** 2), 0.0064 * 0.1 / (2 * math.pi), rel_tol=1e-13)


# ----------------------------------------------------------------- model constants
def test_double_well_constants_match_paper():
    p = _paper()["double_well"]
    dw = wc.DOUBLE_WELL
    assert dw["mass"] == p["mass"] and dw["omega"] == p["omega"]
    assert dw["g"] == p["g"] and dw["dG"] == p["dG"]
    assert wc.get_config("c1")["kT"] == p["kT"]


def test_desorption_unit_conversions_and_classical_ratio():
    """kT/(hbar omega) at 300 K for 1 u and 10.54 u and Q(beta, omega), printed
    in Sec. III.C, from the Table et-parameters Morse constants."""
    p = _paper()
    t = p["desorption_table"]
    De = wc.ev(t["De_eV"])
    a = t["a_per_A"] * wc.BOHR_ANGSTROM
    kT = 300.0 * wc.KB_HARTREE_PER_K
    for mass_u, key in ((1.0, "kT_over_hbar_omega_1u_300K"), (10.54, "kT_over_hbar_omega_10p54u_300K")):
        m = mass_u * wc.AMU_ME
        omega = math.sqrt(2 * De * a * a / m)      # U0''(x0) = 2 De a^2
        ratio = kT / omega
        assert abs(ratio - p[key]["value"]) <= p[key]["unit_last_place"]
    m = 10.54 * wc.AMU_ME
    omega = math.sqrt(2 * De * a * a / m)
    Q = closed_forms.harmonic_wigner_factor(1.0 / kT, omega)
    assert abs(Q - p["wigner_Q_10p54u_300K"]["value"]) <= p["wigner_Q_10p54u_300K"]["unit_last_place"]


def test_crossing_barrier():
    """The U0/U1 crossing lies 1.83 eV above the far-field U1 level
    (Fig. scattering caption)."""
    p = _paper()
    t = wc.DESORPTION_TABLE
    eps, w = bath.discretise("gauss_legendre", 4, 1.0)
    m = models.MorseTanh(eps, w, 0.0, t["mass"], t["De"], t["x0"], t["a"], t["D1"], t["D2"],
                         t["ap"], t["Vinf"], t["q"], t["atil"], t["xtil"], t["c"])
    f = lambda x: m.U0(np.array([x])) - m.U1(np.array([x]))
    xc = brentq(f, 2.0, 10.0)
    barrier_ev = (m.U0(np.array([xc])) - t["Vinf"]) * wc.HARTREE_EV
    assert abs(barrier_ev - p["crossing_barrier_eV"]["value"]) <= p["crossing_barrier_eV"]["unit_last_place"]


def test_model_derivatives_fd():
    cfg3 = wc.get_config("c3")
    for cfg, xs in ((wc.get_config("c1"), [-3.0, 0.0, 7.5]), (cfg3, [3.0, 5.0, 9.0])):
        m = models.from_config(cfg, M=8) if cfg is cfg3 else models.from_config(cfg)
        h = 1e-6
        for x in xs:
            X = np.array([x])
            assert abs(m.dU0(X)[0] - (m.U0(X + h) - m.U0(X - h)) / (2 * h)) < 1e-7 * max(1, abs(m.dU0(X)[0]))
            assert abs(m.dh(X)[0] - (m.h(X + h) - m.h(X - h)) / (2 * h)) < 1e-7 * max(1e-3, abs(m.dh(X)[0]))
            dV = (m.V(X + h) - m.V(X - h)) / (2 * h)
            assert np.allclose(m.dV(X)[:, 0], dV, atol=1e-9)


# ------------------------------------------------------------------- eigen-solve
def test_eig_two_level_closed_form():
    eps, w = np.array([0.01]), np.array([0.1])
    m = models.Harmonic(eps, w, 0.02, 2000.0, 2e-4, 20.0, -3.8e-3)
    for x in (-5.0, 0.0, 3.0, 12.0):
        X = np.array([x])
        lam, Q = el.eig(m.H(X))
        ref = closed_forms.two_level_eigenvalues(m.h(X), 0.01, m.V(X)[0])
        assert np.allclose(lam, ref, rtol=0, atol=1e-16)
        assert np.all(Q[0] > 0)


@pytest.mark.parametrize("cfg_name,M", [("c1", 20), ("c2gl", 40), ("c3", 40)])
def test_eig_arrowhead_identities(cfg_name, M):
    """Dense eigh of the arrowhead Hamiltonian satisfies: reconstruction,
    strict interlacing with the bath levels, the secular equation
    lambda - h - sum V^2/(lambda - eps) = 0, the Loewner identity
    V_k^2 = -prod_j (eps_k - lambda_j) / prod_{l != k} (eps_k - eps_l), and the
    eigenvector form u_j ~ (1, V_k/(lambda_j - eps_k))."""
    cfg = wc.get_config(cfg_name)
    m = models.from_config(cfg, M=M)
    xs = [-4.0, 0.5, 6.0] if cfg_name != "c3" else [2.5, 4.0, 9.0]
    for x in xs:
        X = np.array([x])
        H = m.H(X)
        lam, Q = el.eig(H)
        assert np.max(np.abs(Q @ np.diag(lam) @ Q.T - H)) < 1e-15 * 50
        eps, V, h = m.eps, m.V(X), m.h(X)
        # interlacing lambda_0 < eps_1 < lambda_1 < ... < eps_M < lambda_M
        assert np.all(lam[:-1] < eps) and np.all(eps < lam[1:])
        for j in range(len(lam)):
            terms = V ** 2 / (lam[j] - eps)
            f = lam[j] - h - terms.sum()
            fprime = 1.0 + np.sum(V ** 2 / (lam[j] - eps) ** 2)
            # the Newton correction f/f' is at rounding level of the spectrum
            assert abs(f / fprime) < 1e-14 * np.max(np.abs(lam))
        for k in range(M):
            num = np.prod((eps[k] - lam) / np.where(np.arange(M + 1) == 0, 1.0, 1.0))
            den = np.prod(np.delete(eps[k] - eps, k))
            # pair factors to stay in range: log form
            lv = np.sum(np.log(np.abs(eps[k] - lam))) - np.sum(np.log(np.abs(np.delete(eps[k] - eps, k))))
            # eigh's absolute eigenvalue error ~ eps*|H| propagates through
            # every factor (eps_k - lambda_j)
            tol = 20 * np.finfo(float).eps * np.max(np.abs(lam)) * np.sum(1.0 / np.abs(eps[k] - lam))
            assert abs(math.exp(lv) / V[k] ** 2 - 1.0) < max(tol, 1e-13)
            assert np.sign(num / den) == -1.0
        for j in range(len(lam)):
            u = np.concatenate([[1.0], V / (lam[j] - eps)])
            u /= np.linalg.norm(u)
            assert np.max(np.abs(u - Q[:, j])) < 1e-9


def test_wigner_sample_has_the_quantum_corrected_widths():
    """The desorption workload's harmonic Wigner sample (Eq. wigner): variances
    Q kT / (m w^2) and Q kT / m with Q from the closed form, w the harmonic
    frequency of U0 at its minimum (second derivative from the oracle model by
    central differences), Q = 1.9 at 300 K as printed."""
    from workloads import get_config
    from workloads.sampling import wigner_harmonic
    cfg = get_config("desorption")
    m = models.from_config(cfg, M=4)
    x0 = cfg["model"]["x0"]
    h = 1e-4
    k2 = (m.U0(np.array([x0 + h])) - 2 * m.U0(np.array([x0])) + m.U0(np.array([x0 - h]))) / h ** 2
    omega = float(np.sqrt(k2 / m.mass[0]))
    kT = cfg["kT"]
    Q = closed_forms.harmonic_wigner_factor(1.0 / kT, omega)
    assert abs(Q - _paper()["wigner_Q_10p54u_300K"]["value"]) <= 0.05
    n = 400000
    x, v = wigner_harmonic(n, m.mass[0], omega, x0, kT, seed=3)
    var_x = Q * kT / (m.mass[0] * omega ** 2)
    var_v = Q * kT / m.mass[0]
    # sample variance: relative standard error sqrt(2/n) = 0.22%
    assert abs(np.var(x) / var_x - 1.0) < 0.01
    assert abs(np.var(v) / var_v - 1.0) < 0.01
    assert abs(np.mean(x) - x0) < 4.0 * np.sqrt(var_x / n)


def test_multi_coordinate_model_derivatives_and_forces():
    """The six-coordinate model: dU0, dh and dV against central differences
    of U0, h and V in every coordinate, and the Hellmann-Feynman force of an
    occupied set against central differences of E_pot."""
    from workloads import get_config
    cfg = get_config("c5")
    m = models.from_config(cfg, M=12)
    assert m.n_dof == 6
    rs = np.random.default_rng(3)
    for _ in range(3):
        R = np.array(cfg["model"]["dof"])[:, 3] + rs.normal(0.0, 0.3, size=6)
        hs = 1e-5
        s = np.arange(6)
        F = el.forces(m, R, s)
        for nu in range(6):
            e = np.zeros(6)
            e[nu] = hs
            fd_u0 = (m.U0(R + e) - m.U0(R - e)) / (2 * hs)
            fd_h = (m.h(R + e) - m.h(R - e)) / (2 * hs)
            fd_v = (m.V(R + e) - m.V(R - e)) / (2 * hs)
            assert abs(m.dU0(R)[nu] - fd_u0) < 1e-8 * max(1.0, abs(fd_u0))
            assert abs(m.dh(R)[nu] - fd_h) < 1e-9
            assert np.max(np.abs(m.dV(R)[:, nu] - fd_v)) < 1e-9
            fd_e = (el.potential_energy(m, R + e, s) - el.potential_energy(m, R - e, s)) / (2 * hs)
            assert abs(F[nu] + fd_e) < 1e-7 * max(1.0, abs(fd_e)), (nu, F[nu], fd_e)


def test_vector_rescaling_conserves_energy_along_the_coupling():
    """Several coordinates: the rescaled velocity changes the momentum along
    d only (p' - p parallel to d) and lowers the kinetic energy by exactly dE;
    an unaffordable dE is frustrated (v unchanged)."""
    rs = np.random.default_rng(6)
    m = np.array([2000.0, 2000.0, 4000.0, 4000.0, 8000.0, 8000.0])
    for _ in range(20):
        v = rs.normal(0.0, 2e-3, size=6)
        d = rs.normal(0.0, 1.0, size=6)
        ke = 0.5 * np.sum(m * v * v)
        dE = rs.uniform(-0.5, 0.9) * ke
        v2, ok = el.rescale(v, m, d, dE)
        dp = m * (v2 - v)
        if ok:
            assert abs(0.5 * np.sum(m * v2 * v2) - (ke - dE)) < 1e-12 * ke
            cross = dp - d * (dp @ d) / (d @ d)
            assert np.max(np.abs(cross)) < 1e-12 * max(np.max(np.abs(dp)), 1e-30)
        else:
            assert np.array_equal(v2, v)


# ------------------------------------------------------------- dense model kind
def test_dense_model_with_rank_one_h1_is_the_double_well():
    """H0 = the double-well H at x = 0 and H1 = h' e0 e0^T give exactly the
    double-well model (Sec. III.B): equal H(x), dH/dx, U0, forces and one
    oracle step from the same state."""
    from oracle import bath, dynamics as dyn, rng
    from oracle import electronic as el
    from workloads.sampling import random_orbitals
    eps, w = bath.discretise("trapezoid", 12, 0.1)
    harm = models.Harmonic(eps, w, 0.01, 2000.0, 2e-4, 20.0, -3.8e-3)
    H0 = harm.H(np.array([0.0]))
    H1 = harm.dH(np.array([0.0]))[0]
    dense = models.Dense(H0, H1, 2000.0, 2e-4)
    for x in (-6.0, 0.0, 3.5, 11.0):
        X = np.array([x])
        assert np.max(np.abs(dense.H(X) - harm.H(X))) <= 1e-15
        assert np.array_equal(dense.dH(X)[0], harm.dH(X)[0])
        assert dense.U0(X) == harm.U0(X) and dense.dU0(X)[0] == harm.dU0(X)[0]
    st = dyn.State([2.0], [1e-3], random_orbitals(13, 6, seed=4), [0, 2, 3, 5, 7, 9])
    for k in range(3):
        xi = rng.uniform(0, 0, k)
        a, ea, _ = dyn.step(harm, st, 20.0, xi)
        b, eb, _ = dyn.step(dense, st, 20.0, xi)
        assert np.max(np.abs(a.C - b.C)) <= 1e-12 and abs(a.x[0] - b.x[0]) <= 1e-12
        assert list(a.s) == list(b.s)
        st = a


def test_dense_workload_couplings_and_forces_against_finite_differences():
    """The dense workload's H(x) (impurity plus a tight-binding chain, x-dependent
    impurity couplings): D = <j|d/dx k> against central differences of
    gauge-fixed eigenvectors, the Hellmann-Feynman force against differences of
    E_pot; every orbital keeps a clear impurity component (the gauge
    Q[0, j] > 0 is continuous)."""
    from oracle import electronic as el
    from workloads import get_config
    m = models.from_config(get_config("dense"), M=30)
    h = 1e-6
    for x in (-4.0, 2.0, 9.0):
        X = np.array([x])
        H = m.H(X)
        off = H - np.diag(np.diag(H))
        assert np.count_nonzero(off[1:, 1:]) > 0          # not an arrowhead
        lam, Q = el.eig(H)
        assert np.min(np.abs(Q[0])) > 1e-4
        _, Ds = el.coupling_matrices(lam, Q, m.dH(X))
        _, Qp = el.eig(m.H(X + h))
        _, Qm = el.eig(m.H(X - h))
        fd = Q.T @ (Qp - Qm) / (2 * h)
        assert np.max(np.abs(Ds[0] - fd)) < 1e-6 * np.max(np.abs(Ds[0]))
        for s in ([0, 1, 2, 3], [2, 5, 9, 20]):
            F = el.forces(m, X, s)[0]
            fdF = -(el.potential_energy(m, X + 1e-5, s) - el.potential_energy(m, X - 1e-5, s)) / 2e-5
            assert abs(F - fdF) < 1e-7 * max(1e-4, abs(F))
