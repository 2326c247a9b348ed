"""Pins of the oracle's tangent-linear gradient of the path loss (CPU)."""
import numpy as np
import pytest

from oracle import adjoint as adj
from oracle import bath
from workloads import get_config
from workloads.sampling import fixed_paths


def _case(M=8, N=4, T=12, seed=3):
    cfg = get_config("c4")
    m = cfg["model"]
    eps, w = bath.discretise(cfg["bath"]["kind"], M, cfg["bath"]["W"])
    p = adj.Params(0.0, m["Gamma"], eps, m["omega"], m["g"], m["dG"], w, m["mass"])
    x, _ = fixed_paths(2, T, cfg["dt"], m["omega"], seed=seed)
    return p, x[1], N, cfg["dt"]


def test_tangent_matches_central_differences():
    p, path, N, dt = _case()
    theta = adj.pack(p)
    scale = np.abs(theta).copy()
    scale[scale == 0] = 1e-3
    for i in range(len(theta)):
        e = np.zeros_like(theta)
        e[i] = 1.0
        _, dl = adj.tangent(p, adj.unpack(e, p.w, p.mass), path, N, dt)
        h = 1e-6 * scale[i]
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (adj.loss(adj.unpack(tp, p.w, p.mass), path, N, dt)
              - adj.loss(adj.unpack(tm, p.w, p.mass), path, N, dt)) / (2 * h)
        assert abs(dl - fd) <= 1e-5 * max(abs(fd), 1e-8 / scale[i]) + 1e-9, (i, dl, fd)


def test_eps_d_and_dG_enter_alike():
    """Along prescribed paths eps_d and dG both only shift h."""
    p, path, N, dt = _case(T=8)
    g = adj.gradient(p, path, N, dt)
    M = len(p.eps)
    assert abs(g[0] - g[4 + M]) <= 1e-10 * max(abs(g[0]), 1e-12)


def test_tangent_is_linear_in_the_direction():
    p, path, N, dt = _case(T=6)
    rs = np.random.default_rng(0)
    d1 = rs.normal(size=adj.n_params(len(p.eps))) * 1e-3
    d2 = rs.normal(size=adj.n_params(len(p.eps))) * 1e-3
    f = lambda d: adj.tangent(p, adj.unpack(d, p.w, p.mass), path, N, dt)[1]
    assert np.isclose(f(d1 + 2 * d2), f(d1) + 2 * f(d2), rtol=1e-9, atol=1e-15)


def test_loss_with_no_coupling_motion_is_the_initial_population():
    """A path at rest: v = 0 makes A diagonal; the orbitals only pick up
    phases, so P(t) stays the initial impurity population and E_exc = 0."""
    p, _, N, dt = _case(T=5)
    path = np.full(6, 1.3)
    H, _ = adj.hamiltonian(p, 1.3)
    from oracle.electronic import eig
    lam, Q = eig(H)
    P0 = np.sum(Q[0, :N] ** 2)
    assert np.isclose(adj.loss(p, path, N, dt), P0, rtol=1e-12, atol=1e-15)


TERMS = (0.7, 0.3, 1.5, 2.0)


def test_every_loss_term_matches_central_differences():
    p, path, N, dt = _case(T=10, seed=4)
    theta = adj.pack(p)
    scale = np.abs(theta).copy()
    scale[scale == 0] = 1e-3
    g = adj.gradient(p, path, N, dt, TERMS)
    for i in range(len(theta)):
        h = 1e-6 * scale[i]
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (adj.loss(adj.unpack(tp, p.w, p.mass), path, N, dt, TERMS)
              - adj.loss(adj.unpack(tm, p.w, p.mass), path, N, dt, TERMS)) / (2 * h)
        assert abs(g[i] - fd) <= 1e-5 * max(abs(fd), 1e-8 / scale[i]) + 1e-9, (i, g[i], fd)


def test_eps_d_and_dG_enter_alike_in_every_term():
    p, path, N, dt = _case(T=6, seed=9)
    g = adj.gradient(p, path, N, dt, TERMS)
    M = len(p.eps)
    assert abs(g[0] - g[4 + M]) <= 1e-10 * max(abs(g[0]), 1e-12)


def _dense_model(p):
    from oracle.models import Harmonic
    return Harmonic(p.eps, p.w, p.Gamma, p.mass, p.omega, p.g, p.dG, eps_d=p.eps_d)


def test_hop_term_is_the_sum_of_the_determinant_ratio_probabilities():
    """G(t) equals the total of the hop probabilities of the dynamics'
    determinant-ratio evaluation on the dense model (itself pinned by brute
    force determinants), for random orbitals and both signs of v."""
    from oracle import electronic as el
    from workloads.sampling import random_orbitals
    p, _, N, dt = _case(M=10, N=5)
    m = _dense_model(p)
    for seed, x, v in ((1, 2.5, 3e-4), (2, -4.0, -5e-4), (3, 0.7, 1e-3)):
        lam, Q = el.eig(m.H(np.array([x])))
        _, Ds = el.coupling_matrices(lam, Q, m.dH(np.array([x])))
        C = random_orbitals(len(lam), N, seed=seed)
        ref = el.hop_probabilities(C, np.arange(N), v * Ds[0], dt)[0].sum()
        H, hp = adj.hamiltonian(p, x)
        lam2, Q2 = el.eig(H)
        got = adj._hop_sum(C, N, adj._couplings(lam2, Q2, hp), v, dt)
        assert ref > 0
        assert abs(got - ref) <= 1e-12 * ref


def test_force_term_is_the_hellmann_feynman_force():
    from oracle import electronic as el
    p, _, N, dt = _case(M=12, N=6)
    m = _dense_model(p)
    for x in (-3.0, 0.5, 6.0):
        ref = el.forces(m, np.array([x]), np.arange(N))[0]
        H, hp = adj.hamiltonian(p, x)
        lam, Q = el.eig(H)
        assert abs(adj._force(p, x, Q[0, :], N, hp) - ref) <= 1e-12 * abs(ref)


def _forward_by_the_dynamics_oracle(p, path, N, dt, v_sign=1.0):
    """The adjoint loss's forward pass rebuilt from the dynamics oracle on the
    dense double-well model: couplings from el.coupling_matrices (dense
    Q^T dH Q), the midpoint propagator through el.propagator_matrix and
    el.propagate, and the population from dynamics.observables with the
    occupations held at the N lowest orbitals.  E_exc comes from the energy of
    the diabatic orbitals Psi = Q C: tr(Psi^H H Psi) minus the energy of the
    held configuration."""
    from oracle import dynamics as dyn
    from oracle import electronic as el
    m = _dense_model(p)
    lam0, _ = el.eig(m.H(np.array([path[0]])))
    n = len(lam0)
    C = np.eye(n, N, dtype=np.complex128)
    out = []
    for s in range(len(path) - 1):
        x0, x1 = np.array([path[s]]), np.array([path[s + 1]])
        xm = 0.5 * (x0 + x1)
        v = v_sign * (x1 - x0) / dt
        lam, Q = el.eig(m.H(xm))
        _, Ds = el.coupling_matrices(lam, Q, m.dH(xm))
        C = el.propagate(C, el.propagator_matrix(lam, Ds, v), dt)
        st = dyn.State(x1, v, C, np.arange(N))
        obs = dyn.observables(m, st)
        lam1, Q1 = el.eig(m.H(x1))
        Psi = Q1 @ C
        E_exc = float(np.real(np.trace(Psi.conj().T @ m.H(x1) @ Psi))) - float(np.sum(lam1[:N]))
        out.append(dict(C=C.copy(), P=obs["Pd_wf"], E_exc=E_exc))
    return out


def test_adjoint_forward_on_a_moving_path_matches_the_dynamics_oracle():
    """Pin of the adjoint loss's forward pass (Sec. II.C, Eqs.
    exponential_integrator and fast_exponential_integrator, midpoint reading):
    along moving paths (one of the workload's seeded paths and a fast sweep
    through the level crossings), its orbitals C(t), population P(t) and
    final excitation energy agree with the dynamics oracle to 1e-12.  The
    same comparison with the velocity's sign flipped must fail in C, P and
    E_exc, so that a sign error shared by loss and tangent cannot pass."""
    p, seeded, N, dt = _case(M=10, N=5, T=20, seed=5)
    k = np.arange(21)
    fast = 1.0 + 1e-2 * dt * k + 0.5 * np.sin(0.3 * k)
    for path in (seeded, fast):
        assert np.max(np.abs(np.diff(path))) > 1e-3       # the nuclei do move
        hist = []
        L = adj.loss(p, path, N, dt, history=hist)
        ref = _forward_by_the_dynamics_oracle(p, path, N, dt)
        assert len(hist) == len(ref) == len(path) - 1
        for t, (a, b) in enumerate(zip(hist, ref)):
            assert np.max(np.abs(a["C"] - b["C"])) <= 1e-12, t
            assert abs(a["P"] - b["P"]) <= 1e-12, t
        assert abs(hist[-1]["E_exc"] - ref[-1]["E_exc"]) <= 1e-12 * max(1e-3, abs(ref[-1]["E_exc"]))
        T = len(path) - 1
        assert abs(L - (sum(r["P"] for r in ref) / T + ref[-1]["E_exc"])) <= 1e-12
        # the orbitals do mix along the path (the comparison is not vacuous)
        assert np.max(np.abs(ref[-1]["C"][N:, :])) > 1e-4
        flipped = _forward_by_the_dynamics_oracle(p, path, N, dt, v_sign=-1.0)
        assert max(np.max(np.abs(a["C"] - b["C"])) for a, b in zip(hist, flipped)) > 1e-6
        assert max(abs(a["P"] - b["P"]) for a, b in zip(hist, flipped)) > 1e-6
    assert hist[-1]["E_exc"] > 1e-6
    assert abs(flipped[-1]["E_exc"] - hist[-1]["E_exc"]) > 1e-9
