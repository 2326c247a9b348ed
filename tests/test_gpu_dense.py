"""Parity of the dense model kind (IESH_MODEL_DENSE, H(x) = H0 + x H1 of any
symmetric structure: the LDS-staged Jacobi eigen-solve and the matrix-core
projection G = Q^T H1 Q) with the FP64 oracle's dense model.

Tolerances as in test_gpu_parity: energies and impurity components 1e-10
relative, hop probabilities 1e-10 of the trajectory's largest, positions and
velocities 1e-10 relative, orbitals 1e-9 absolute (FP64); the mixed path at
1e-5; occupations and hop events bit-exact outside near-ties.
"""
import numpy as np
import pytest

from oracle import dynamics as dyn, electronic as el, models, rng
from workloads import boltzmann_harmonic, dense_matrices, get_config
from workloads.sampling import random_orbitals

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2212_00518_amd import _lib
    _lib.lib()  # fails loudly when the library is missing


def _cfg(M, N=None):
    cfg = get_config("dense")
    cfg["bath"]["M"] = M
    cfg["n_elec"] = N if N is not None else (M + 1) // 2
    return cfg


def _ensemble(cfg, T, precision="fp64", **kw):
    from paper_2212_00518_amd import from_config
    return from_config(cfg, n_traj=T, precision=precision, **kw)


def _states(m, N, T, seed, xs, v_scale):
    rs = np.random.default_rng(seed)
    out = []
    for t in range(T):
        C = random_orbitals(m.n, N, seed=seed * 1000 + t)
        s = np.sort(rs.choice(m.n, N, replace=False))
        out.append(dyn.State([xs[t]], [v_scale * rs.normal()], C, s))
    return out


def _upload(ens, states):
    from paper_2212_00518_amd import pack_states
    ens.set_state(*pack_states([(s.x, s.v, s.C, s.s) for s in states], ens.n_max, ens.N_max))


@pytest.mark.parametrize("M", [1, 16, 30, 47, 95])
def test_dense_energies_amplitudes_and_hop_probabilities(M):
    """n = 2 .. 96 (n_pad 16 .. 96, odd and even n): eigenvalues and impurity
    components against the oracle's dense eigh, and the hop probabilities of
    random orbitals against the oracle's determinant-ratio evaluation."""
    cfg = _cfg(M)
    m = models.from_config(cfg, M=M)
    N = cfg["n_elec"]
    T = 6
    xs = np.linspace(-8.0, 20.0, T)
    states = _states(m, N, T, seed=M + 3, xs=xs, v_scale=0.003)
    ens = _ensemble(cfg, T)
    _upload(ens, states)
    lam, q0 = ens.adiabatic()
    g = ens.hop_probs()
    assert np.all(ens.status() == 0)
    for t, st in enumerate(states):
        lr, Q = el.eig(m.H(st.x))
        scale = np.max(np.abs(lr))
        assert np.max(np.abs(lam[t, :m.n] - lr)) <= 1e-10 * scale, t
        assert np.max(np.abs(q0[t, :m.n] - Q[0]) / np.abs(Q[0])) <= 1e-10, t
        ref = dyn.hop_probs(m, st, cfg["dt"])
        gt = g[t, :N * m.n].reshape(N, m.n)
        gmax = np.max(ref)
        print(f"M={M} traj {t}: max |dg| / max g = {np.max(np.abs(gt - ref)) / max(gmax, 1e-300):.2e}",
              flush=True)
        if gmax == 0.0:
            assert np.all(gt == 0.0)
        else:
            assert np.max(np.abs(gt - ref)) <= 1e-10 * gmax, t
    ens.close()


def _compare_step(cfg, m, states, precision, tol):
    from paper_2212_00518_amd import unpack_C
    T, N = len(states), len(states[0].s)
    ens = _ensemble(cfg, T, precision=precision)
    _upload(ens, states)
    ens.step()
    x, v, Cf, occ = ens.get_state()
    evs, _ = ens.events()
    compared = 0
    for t in range(T):
        ref, ev, _ = dyn.step(m, states[t], cfg["dt"], rng.uniform(cfg["seed"], t, 0))
        assert abs(x[t] - ref.x[0]) <= tol * max(1.0, abs(ref.x[0])), t
        assert np.max(np.abs(unpack_C(Cf, t, m.n, N, ens.n_max, ens.N_max) - ref.C)) <= 10 * tol, t
        if ev["attempted"] and ev["margin"] < (1e-7 if precision == "fp64" else 1e-4) * ev["g_total"]:
            continue
        assert abs(v[t] - ref.v[0]) <= tol * max(1e-3, abs(ref.v[0])), t
        assert list(occ[t, :N]) == list(ref.s), t
        mine = [(e["a"], e["b"], e["accepted"]) for e in evs if e["traj"] == t]
        assert mine == ([(ev["a"], ev["b"], ev["accepted"])] if ev["attempted"] else []), t
        compared += 1
    ens.close()
    return compared


@pytest.mark.parametrize("M,N,precision,tol", [(16, 8, "fp64", 1e-10), (47, 20, "fp64", 1e-10),
                                               (95, 48, "fp64", 1e-10), (95, 48, "mixed", 1e-5),
                                               (30, 15, "mixed", 1e-5)])
def test_dense_single_step_random_orbitals(M, N, precision, tol):
    """One step from random orbitals (hops likely): positions, velocities,
    orbitals, occupations and hop events against the oracle."""
    cfg = _cfg(M, N)
    m = models.from_config(cfg, M=M)
    T = 6
    states = _states(m, N, T, seed=11 + M, xs=np.linspace(-6.0, 18.0, T), v_scale=0.02)
    assert _compare_step(cfg, m, states, precision, tol) >= T - (1 if precision == "fp64" else 2)


@pytest.mark.parametrize("M,cap", [(95, 0), (31, 0), (95, 1)])
def test_dense_thirty_step_trajectories_match_the_oracle(M, cap):
    """30 graph-replayed FP64 steps from random orbitals (hops occur): every
    trajectory's states and hop events against the oracle's run.  The warm
    eigen-solves are perturbative refinements; cap = 1 (eig_max_iter) stops
    each after one update, so every warm solve falls back to cold Jacobi
    sweeps."""
    from paper_2212_00518_amd import unpack_C
    cfg = _cfg(M)
    m = models.from_config(cfg, M=M)
    N, T, steps = cfg["n_elec"], 12, 30
    states = _states(m, N, T, seed=70 + M, xs=np.linspace(-6.0, 18.0, T), v_scale=0.005)
    ens = _ensemble(cfg, T, eig_max_iter=cap)
    _upload(ens, states)
    ens.run(steps)
    x, v, Cf, occ = ens.get_state()
    evs, _ = ens.events()
    status = ens.status()
    ens.close()
    assert np.all(status == 0)
    compared = hops = 0
    for t in range(T):
        ref, ref_ev, _ = dyn.run(m, states[t], cfg["dt"], steps, cfg["seed"], t)
        if any(e["margin"] < 1e-7 * max(e["g_total"], 1e-300) for e in ref_ev):
            continue
        mine = [(e["step"], e["a"], e["b"], e["accepted"]) for e in evs if e["traj"] == t]
        assert mine == [(e["step"], e["a"], e["b"], e["accepted"]) for e in ref_ev], t
        hops += sum(e["accepted"] for e in ref_ev)
        assert abs(x[t] - ref.x[0]) <= 1e-9 * max(1.0, abs(ref.x[0])), t
        assert abs(v[t] - ref.v[0]) <= 1e-9 * max(1e-3, abs(ref.v[0])), t
        assert np.max(np.abs(unpack_C(Cf, t, m.n, N, ens.n_max, ens.N_max) - ref.C)) <= 1e-9, t
        assert list(occ[t, :N]) == list(ref.s), t
        compared += 1
    print(f"M={M} cap={cap}: compared {compared} of {T}, hops {hops}", flush=True)
    assert compared >= T - 1 and hops >= 5


def test_dense_three_hundred_steps_cross_the_cold_solve():
    """300 FP64 steps at n = 16: the warm eigen-solves refine the carried
    basis for 255 steps, step 256 solves cold, and the states and hop events
    still match the oracle's run (no drift of the carried basis)."""
    from paper_2212_00518_amd import unpack_C
    M = 15
    cfg = _cfg(M, N=8)
    m = models.from_config(cfg, M=M)
    N, T, steps = cfg["n_elec"], 8, 300
    states = _states(m, N, T, seed=91, xs=np.linspace(-4.0, 14.0, T), v_scale=0.004)
    ens = _ensemble(cfg, T)
    _upload(ens, states)
    ens.run(steps)
    x, v, Cf, occ = ens.get_state()
    evs, _ = ens.events()
    status = ens.status()
    ens.close()
    assert np.all(status == 0)
    compared = 0
    for t in range(T):
        ref, ref_ev, _ = dyn.run(m, states[t], cfg["dt"], steps, cfg["seed"], t)
        if any(e["margin"] < 1e-7 * max(e["g_total"], 1e-300) for e in ref_ev):
            continue
        mine = [(e["step"], e["a"], e["b"], e["accepted"]) for e in evs if e["traj"] == t]
        assert mine == [(e["step"], e["a"], e["b"], e["accepted"]) for e in ref_ev], t
        assert abs(x[t] - ref.x[0]) <= 1e-8 * max(1.0, abs(ref.x[0])), t
        assert abs(v[t] - ref.v[0]) <= 1e-8 * max(1e-3, abs(ref.v[0])), t
        assert np.max(np.abs(unpack_C(Cf, t, m.n, N, ens.n_max, ens.N_max) - ref.C)) <= 1e-8, t
        assert list(occ[t, :N]) == list(ref.s), t
        compared += 1
    print(f"compared {compared} of {T}", flush=True)
    assert compared >= T - 1


def test_dense_thermal_initialisation_matches_the_oracle():
    """iesh_init_thermal on the dense kind: Fermi occupations at kT over the
    dense eigenvalues (same rule and uniforms as the oracle) and unit-vector
    orbitals."""
    from paper_2212_00518_amd import unpack_C
    cfg = _cfg(95)
    m = models.from_config(cfg)
    N, T = cfg["n_elec"], 32
    x0, v0 = boltzmann_harmonic(T, cfg["model"]["mass"], cfg["model"]["omega"], cfg["kT"], seed=3)
    ens = _ensemble(cfg, T)
    ens.init_thermal(x0, v0)
    x, v, Cf, occ = ens.get_state()
    ens.close()
    changed = 0
    for t in range(T):
        ref = dyn.initial_state(m, x0[t], v0[t], N, cfg["kT"], cfg["seed"], t)
        assert list(occ[t, :N]) == list(ref.s), t
        assert np.array_equal(unpack_C(Cf, t, m.n, N, ens.n_max, ens.N_max), ref.C)
        changed += list(ref.s) != list(range(N))
    assert changed > 0  # the sampling does move electrons above the lowest N


def test_dense_kind_with_a_rank_one_h1_is_the_double_well():
    """H0 and H1 of the double well (rank-one H1): the dense path takes the
    same 20 steps as the arrowhead path of the harmonic model (states within
    1e-10, events identical)."""
    from paper_2212_00518_amd import _lib, from_config, pack_states
    cfg = get_config("c1")
    M, N, T = 30, 15, 8
    cfg["bath"]["M"] = M
    cfg["n_elec"] = N
    harm = models.from_config(cfg, M=M)
    H0 = harm.H(np.array([0.0]))
    H1 = harm.dH(np.array([0.0]))[0]
    states = _states(harm, N, T, seed=5, xs=np.linspace(-6.0, 18.0, T), v_scale=0.004)
    d = _lib.dense_model_desc(H0, H1, cfg["model"]["mass"], cfg["model"]["omega"], N)
    run = dict(n_traj=T, precision="fp64", dt=cfg["dt"], kT=cfg["kT"], seed=cfg["seed"])
    out = []
    for ens in (_lib.Ensemble([d], run), from_config(cfg, n_traj=T, M=M, n_elec=N)):
        ens.set_state(*pack_states([(s.x, s.v, s.C, s.s) for s in states], ens.n_max, ens.N_max))
        ens.run(20)
        out.append((ens.get_state(), [(e["step"], e["traj"], e["a"], e["b"], e["accepted"])
                                      for e in ens.events()[0]]))
        ens.close()
    (sd, ed), (sh, eh) = out
    assert ed == eh and len(ed) > 0
    assert np.max(np.abs(sd[0] - sh[0])) <= 1e-10 * np.max(np.abs(sh[0]))
    assert np.max(np.abs(sd[2] - sh[2])) <= 1e-9
    assert np.array_equal(sd[3], sh[3])


def test_dense_error_paths():
    from paper_2212_00518_amd import _lib
    run = dict(n_traj=2, precision="fp64", dt=20.0, kT=1e-3)
    H0, H1 = dense_matrices(_cfg(96), 96)            # n = 97: above the LDS limit
    with pytest.raises(_lib.IeshError, match="IESH_DENSE_MAX_N"):
        _lib.Ensemble([_lib.dense_model_desc(H0, H1, 2000.0, 2e-4, 40)], run)
    H0, H1 = dense_matrices(_cfg(20), 20)
    bad = H0.copy()
    bad[3, 5] += 1e-3
    with pytest.raises(_lib.IeshError, match="not symmetric"):
        _lib.Ensemble([_lib.dense_model_desc(bad, H1, 2000.0, 2e-4, 10)], run)
    d = _lib.dense_model_desc(H0, H1, 2000.0, 2e-4, 10)
    d.dense = None
    with pytest.raises(_lib.IeshError, match="matrices"):
        _lib.Ensemble([d], run)
    ens = _lib.Ensemble([_lib.dense_model_desc(H0, H1, 2000.0, 2e-4, 10)], run)
    with pytest.raises(_lib.IeshError, match="harmonic"):
        ens.adjoint_forward(np.zeros((2, 3)), 1)
    ens.close()
