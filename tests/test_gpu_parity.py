"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Tolerances (FP64 path): energies and impurity amplitudes 1e-10 relative;
hop probabilities 1e-10 relative to the largest probability of the
trajectory; positions and velocities 1e-10 relative; orbital coefficients
1e-10 absolute (orbitals have unit norm); occupations and hop events
bit-exact except at near-ties (|cumulative sum - xi| within the tolerance).
Mixed path: the same at 1e-5.
"""
import math

import numpy as np
import pytest

from oracle import models, dynamics as dyn, electronic as el, rng
from workloads import get_config, boltzmann_harmonic
from workloads.sampling import random_orbitals, uniforms

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2212_00518_amd import _lib
    _lib.lib()  # fails loudly when the library is missing


def make_cfg(name, M=None, N=None, **model_over):
    cfg = get_config(name)
    if M is not None:
        cfg["bath"]["M"] = M
    if N is not None:
        cfg["n_elec"] = N
    elif M is not None:
        cfg["n_elec"] = max(1, M // 2)
    cfg["model"].update(model_over)
    if name == "c3":
        cfg.setdefault("n_elec", cfg["bath"]["M"] // 2)
        cfg["dt"] = 5.0
    return cfg


def ensemble(cfg, T, precision="fp64", **kw):
    from paper_2212_00518_amd import from_config
    return from_config(cfg, n_traj=T, precision=precision, **kw)


def random_states(m, N, T, seed, xs, v_scale):
    rs = np.random.default_rng(seed)
    out = []
    for t in range(T):
        C = random_orbitals(m.n, N, seed=seed * 1000 + t)
        s = np.sort(rs.choice(m.n, N, replace=False))
        out.append(dyn.State([xs[t]], [v_scale * rs.normal()], C, s))
    return out


def upload(ens, states):
    from paper_2212_00518_amd import pack_states
    ens.set_state(*pack_states([(s.x, s.v, s.C, s.s) for s in states], ens.n_max, ens.N_max))


# --------------------------------------------------------------------- eigen
@pytest.mark.parametrize("name,M,xs", [
    ("c1", 20, np.linspace(-12, 30, 8)),
    ("c1", 2, np.linspace(-5, 25, 4)),
    ("c1", 3, np.linspace(-5, 25, 4)),
    ("c1", 64, np.linspace(-5, 25, 4)),
    ("c1", 65, np.linspace(-5, 25, 4)),
    ("c2", 200, np.linspace(-10, 25, 6)),
    ("c2gl", 200, np.linspace(-10, 25, 6)),
    ("c1", 1, np.linspace(-5, 25, 4)),
    ("c1", 5, np.linspace(-5, 25, 4)),
    ("c3", 40, np.linspace(2.0, 14.0, 6)),
    ("c3", 160, np.linspace(2.0, 14.0, 6)),
    ("c2", 222, np.linspace(-10, 25, 3)),
    ("c3", 320, np.linspace(2.0, 14.0, 4)),
    ("c1", 335, np.linspace(-10, 25, 3)),
])
def test_adiabatic_energies_and_amplitudes(name, M, xs):
    cfg = make_cfg(name, M=M)
    m = models.from_config(cfg, M=M)
    N = cfg["n_elec"]
    T = len(xs)
    states = [dyn.State([x], [0.0], np.eye(m.n, N, dtype=complex), np.arange(N)) for x in xs]
    ens = ensemble(cfg, T)
    upload(ens, states)
    lam, q0 = ens.adiabatic()
    assert np.all(ens.status() == 0)
    for t, x in enumerate(xs):
        lr, Q = el.eig(m.H(np.array([x])))
        scale = np.max(np.abs(lr))
        assert np.max(np.abs(lam[t, : m.n] - lr)) <= 1e-10 * scale
        assert np.max(np.abs(q0[t, : m.n] - Q[0]) / np.abs(Q[0])) <= 1e-10
    ens.close()


# --------------------------------------------------------------- hop probabilities
@pytest.mark.parametrize("name,M,N", [
    ("c1", 20, 10), ("c1", 1, 1), ("c1", 6, 1), ("c1", 37, 13), ("c1", 63, 31),
    ("c2", 200, 100), ("c2gl", 200, 100), ("c3", 80, 40), ("c2", 222, 111), ("c1", 127, 127),
    ("c3", 160, 80), ("c3", 320, 160), ("c1", 300, 40), ("c1", 335, 168), ("c1", 250, 120),
])
def test_hop_probabilities(name, M, N):
    cfg = make_cfg(name, M=M, N=N)
    m = models.from_config(cfg, M=M)
    T = 4
    xs = np.linspace(2.0, 12.0, T) if name == "c3" else np.linspace(-6, 16, T)
    vs = 0.01 if name == "c3" else 0.002
    states = random_states(m, N, T, seed=M + N, xs=xs, v_scale=vs)
    ens = ensemble(cfg, T)
    upload(ens, states)
    g = ens.hop_probs()
    for t in range(T):
        ref = dyn.hop_probs(m, states[t], cfg["dt"])
        gt = g[t, : N * m.n].reshape(N, m.n)
        gmax = np.max(ref)
        if gmax == 0.0:  # every rate of this state is negative
            assert np.all(gt == 0.0)
            continue
        assert np.max(np.abs(gt - ref)) <= 1e-10 * gmax, (t, np.max(np.abs(gt - ref)) / gmax)
    ens.close()


# ---------------------------------------------------------------------- one step
def _compare_step(cfg, m, states, precision="fp64", tol=1e-10, step0=0):
    T = len(states)
    N = len(states[0].s)
    ens = ensemble(cfg, T, precision=precision)
    upload(ens, states)
    if step0:
        ens.set_step(step0)
    ens.step()
    x, v, Cf, occ = ens.get_state()
    from paper_2212_00518_amd import unpack_C
    evs, _ = ens.events()
    n_checked = 0
    for t in range(T):
        xi = rng.uniform(cfg["seed"], t, step0)
        ref, ev, _ = dyn.step(m, states[t], cfg["dt"], xi)
        near_tie = ev["attempted"] and ev["margin"] < 1e3 * tol * max(ev["g_total"], 1e-300)
        assert abs(x[t] - ref.x[0]) <= tol * max(1.0, abs(ref.x[0]))
        Cg = unpack_C(Cf, t, m.n, N, ens.n_max, ens.N_max)
        assert np.max(np.abs(Cg - ref.C)) <= tol * 10
        if near_tie:
            continue
        assert list(occ[t, :N]) == list(ref.s), t
        assert abs(v[t] - ref.v[0]) <= tol * max(1e-3, abs(ref.v[0])), (t, v[t], ref.v[0])
        mine = [e for e in evs if e["traj"] == t]
        if ev["attempted"]:
            assert len(mine) == 1 and (mine[0]["a"], mine[0]["b"]) == (ev["a"], ev["b"])
            assert mine[0]["accepted"] == ev["accepted"]
        else:
            assert not mine
        n_checked += 1
    ens.close()
    return n_checked


@pytest.mark.parametrize("name,M,N,vscale", [
    ("c1", 20, 10, 0.002), ("c1", 37, 13, 0.004), ("c2", 200, 100, 0.002),
    ("c2gl", 200, 100, 0.002), ("c3", 40, 20, 0.01), ("c1", 1, 1, 0.003),
    ("c3", 320, 160, 0.01), ("c1", 300, 40, 0.003),
])
def test_single_step_random_orbitals(name, M, N, vscale):
    """Random orthonormal orbitals make hops likely within one step."""
    cfg = make_cfg(name, M=M, N=N)
    m = models.from_config(cfg, M=M)
    T = 6
    xs = np.linspace(2.5, 10.0, T) if name == "c3" else np.linspace(-5, 15, T)
    states = random_states(m, N, T, seed=7 + M, xs=xs, v_scale=vscale)
    assert _compare_step(cfg, m, states) >= T - 1


@pytest.mark.parametrize("M,N", [(1, 1), (15, 7), (16, 8), (47, 20)])
def test_single_step_mixed_ring_edges(M, N):
    """Mixed path at the edges of the propagation's fragment ring: n = 2 and
    n = 16 have exactly as many k-blocks as the ring is deep (it wraps to the
    next Chebyshev term after every block), n = 17 is one row past that, and
    n = 48 spans several ring turns per term."""
    cfg = make_cfg("c1", M=M, N=N)
    m = models.from_config(cfg, M=M)
    T = 6
    states = random_states(m, N, T, seed=11 + M, xs=np.linspace(-5, 15, T), v_scale=0.003)
    assert _compare_step(cfg, m, states, precision="mixed", tol=1e-5) >= T - 1


def test_step_counter_drives_the_hop_uniform():
    cfg = make_cfg("c1", M=20, N=10)
    m = models.from_config(cfg)
    states = random_states(m, 10, 5, seed=3, xs=np.linspace(-4, 8, 5), v_scale=0.003)
    assert _compare_step(cfg, m, states, step0=123456789) >= 4


# ------------------------------------------------------------------ trajectories
def _hot_c1(T, Gamma=0.001, fac=200.0):
    cfg = make_cfg("c1", Gamma=Gamma)
    m = models.from_config(cfg)
    x0, v0 = boltzmann_harmonic(T, 2000.0, 2e-4, cfg["kT"], seed=11, kT_factor=fac)
    states = [dyn.initial_state(m, x0[t], v0[t], cfg["n_elec"], cfg["kT"], cfg["seed"], t)
              for t in range(T)]
    return cfg, m, states


def test_trajectory_parity_with_hops():
    """32 trajectories x 300 steps through iesh_run (graph replay): identical
    hop events and final states, trajectories cut at their first near-tie."""
    T, steps = 32, 300
    cfg, m, states = _hot_c1(T)
    ens = ensemble(cfg, T)
    upload(ens, states)
    ens.run(steps)
    x, v, Cf, occ = ens.get_state()
    evs, n_ev = ens.events()
    from paper_2212_00518_amd import unpack_C
    hops = 0
    compared = 0
    for t in range(T):
        ref, ref_ev, _ = dyn.run(m, states[t], cfg["dt"], steps, cfg["seed"], t)
        mine = [e for e in evs if e["traj"] == t]
        tie = any(e["margin"] < 1e-7 * max(e["g_total"], 1e-300) for e in ref_ev)
        if tie:
            continue
        assert [(e["step"], e["a"], e["b"], e["accepted"]) for e in mine] == \
               [(e["step"], e["a"], e["b"], e["accepted"]) for e in ref_ev], t
        hops += sum(e["accepted"] for e in ref_ev)
        assert list(occ[t, : cfg["n_elec"]]) == list(ref.s)
        assert abs(x[t] - ref.x[0]) <= 1e-8 * max(1.0, abs(ref.x[0]))
        assert abs(v[t] - ref.v[0]) <= 1e-8 * max(1e-3, abs(ref.v[0]))
        Cg = unpack_C(Cf, t, m.n, cfg["n_elec"], ens.n_max, ens.N_max)
        assert np.max(np.abs(Cg - ref.C)) <= 1e-8
        compared += 1
    assert compared >= T - 2
    assert hops >= 5
    ens.close()


def test_observables_records():
    T, steps, rec = 8, 60, 20
    cfg, m, states = _hot_c1(T)
    from paper_2212_00518_amd import from_config
    ens = from_config(cfg, n_traj=T, record_every=rec)
    upload(ens, states)
    obs = ens.run(steps, record=True)
    assert obs.shape == (steps // rec, T, 5)
    for t in range(T):
        _, _, records = dyn.run(m, states[t], cfg["dt"], steps, cfg["seed"], t, record_every=rec)
        for q, r in enumerate(records):
            for i, key in enumerate(("Pd_surf", "Pd_wf", "Ekin", "Epot", "Etot")):
                assert abs(obs[q, t, i] - r[key]) <= 1e-9 * max(1e-6, abs(r[key])), (q, t, key)
    ens.close()


def test_run_is_bitwise_deterministic():
    T = 16
    cfg, m, states = _hot_c1(T)
    outs = []
    for _ in range(2):
        ens = ensemble(cfg, T)
        upload(ens, states)
        ens.run(100)
        outs.append(ens.get_state())
        ens.close()
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


def test_resume_from_a_saved_state_continues_the_run():
    """Checkpoint / resume: the state saved after 60 steps and uploaded into a
    new context with the step counter restored continues like the
    uninterrupted run: identical hop events and occupations, and states equal
    to rounding (the uninterrupted run starts each eigen-solve from the
    previous one's roots, the resumed run its first one from scratch, so the
    roots agree to the last bits, not bit for bit), FP64 and mixed."""
    T = 16
    cfg, m, states = _hot_c1(T)
    for prec in ("fp64", "mixed"):
        full = ensemble(cfg, T, precision=prec)
        upload(full, states)
        full.run(120)
        ref = full.get_state()
        ref_ev = [e for e in full.events(cap=1 << 16)[0] if e["step"] >= 60]
        full.close()
        first = ensemble(cfg, T, precision=prec)
        upload(first, states)
        first.run(60)
        saved = first.get_state()
        first.close()
        second = ensemble(cfg, T, precision=prec)
        second.set_state(*saved)
        second.set_step(60)
        second.run(60)
        got = second.get_state()
        got_ev = second.events(cap=1 << 16)[0]
        second.close()
        tol = 1e-10 if prec == "fp64" else 1e-5
        assert np.max(np.abs(ref[0] - got[0]) / np.maximum(1.0, np.abs(ref[0]))) <= tol, prec
        assert np.max(np.abs(ref[1] - got[1]) / np.maximum(1e-3, np.abs(ref[1]))) <= tol, prec
        assert np.max(np.abs(ref[2] - got[2])) <= 10 * tol, prec
        assert np.array_equal(ref[3], got[3]), prec
        key = lambda e: (e["step"], e["traj"], e["a"], e["b"], e["accepted"])
        assert sorted(map(key, ref_ev)) == sorted(map(key, got_ev)), prec
        assert len(ref_ev) > 0


def test_thermal_initialisation_matches_oracle():
    cfg = make_cfg("c1")
    T = 64
    m = models.from_config(cfg)
    x0, v0 = boltzmann_harmonic(T, 2000.0, 2e-4, cfg["kT"], seed=0)
    ens = ensemble(cfg, T)
    ens.init_thermal(x0, v0)
    x, v, Cf, occ = ens.get_state()
    from paper_2212_00518_amd import unpack_C
    for t in range(T):
        ref = dyn.initial_state(m, x0[t], v0[t], cfg["n_elec"], cfg["kT"], cfg["seed"], t)
        assert list(occ[t, : cfg["n_elec"]]) == list(ref.s)
        assert np.array_equal(unpack_C(Cf, t, m.n, cfg["n_elec"], ens.n_max, ens.N_max), ref.C)
    ens.close()


# ---------------------------------------------------------------------- edge cases
def test_uncoupled_model_is_a_pure_phase_and_never_hops():
    """With g = 0 the impurity level does not depend on x, so every
    coupling vanishes: each step multiplies C by exp(-i lambda dt)."""
    cfg = make_cfg("c1", M=20, N=10, g=0.0)
    m = models.from_config(cfg)
    T = 4
    states = random_states(m, 10, T, seed=5, xs=np.linspace(-3, 3, T), v_scale=0.003)
    ens = ensemble(cfg, T)
    upload(ens, states)
    ens.run(3)
    x, v, Cf, occ = ens.get_state()
    from paper_2212_00518_amd import unpack_C
    lam, _ = el.eig(m.H(np.array([0.0])))
    for t in range(T):
        Cg = unpack_C(Cf, t, m.n, 10, ens.n_max, ens.N_max)
        ref = np.exp(-3j * lam * cfg["dt"])[:, None] * states[t].C
        assert np.max(np.abs(Cg - ref)) <= 1e-12
        assert list(occ[t, :10]) == list(states[t].s)
    assert ens.events()[1] == 0
    ens.close()


def test_singular_overlap_sets_status_and_skips_hop():
    cfg = make_cfg("c1", M=20, N=10)
    m = models.from_config(cfg)
    states = random_states(m, 10, 2, seed=9, xs=np.array([1.0, 2.0]), v_scale=0.003)
    a = states[0].s[3]
    states[0].C[a, :] = 0.0  # an occupied row of S vanishes: det S = 0
    ens = ensemble(cfg, 2)
    upload(ens, states)
    g = ens.hop_probs(0, 1)
    assert np.all(g == 0.0)
    from paper_2212_00518_amd import _lib
    assert ens.status()[0] & _lib.TRAJ_SINGULAR_S
    ens.close()


# ----------------------------------------------------------------------- mixed
@pytest.mark.parametrize("name,M,N", [("c1", 20, 10), ("c2", 200, 100),
                                      ("c2", 230, 115),   # 15 row tiles: slab width capped by tiles per wave
                                      ("c3", 320, 160)])
def test_mixed_precision_single_step(name, M, N):
    cfg = make_cfg(name, M=M, N=N)
    m = models.from_config(cfg, M=M)
    T = 4
    xs = np.linspace(2.5, 10.0, T) if name == "c3" else np.linspace(-4, 10, T)
    states = random_states(m, N, T, seed=17, xs=xs, v_scale=0.01 if name == "c3" else 0.002)
    assert _compare_step(cfg, m, states, precision="mixed", tol=1e-5) >= T - 1


@pytest.mark.parametrize("name,M,N", [("c1", 20, 10), ("c2", 200, 100), ("c3", 320, 160),
                                      ("c2gl", 200, 100)])
def test_mixed_hop_probabilities(name, M, N):
    """Mixed path (Eqs. hopping_probability and hopping_rate): the orbitals
    are held in FP32, the overlap inverse and the ratios in FP64.  From the
    same FP64 orbitals the probabilities agree with the FP64 oracle to
    1e-5 of the trajectory's largest probability."""
    cfg = make_cfg(name, M=M, N=N)
    m = models.from_config(cfg, M=M)
    T = 4
    xs = np.linspace(2.0, 12.0, T) if name == "c3" else np.linspace(-6, 16, T)
    vs = 0.01 if name == "c3" else 0.002
    states = random_states(m, N, T, seed=M + N, xs=xs, v_scale=vs)
    ens = ensemble(cfg, T, precision="mixed")
    upload(ens, states)
    g = ens.hop_probs()
    for t in range(T):
        ref = dyn.hop_probs(m, states[t], cfg["dt"])
        gt = g[t, : N * m.n].reshape(N, m.n)
        gmax = np.max(ref)
        assert gmax > 0.0
        err = np.max(np.abs(gt - ref)) / gmax
        print(f"{name} M={M} traj {t}: max |dg| / max g = {err:.2e}", flush=True)
        assert err <= 1e-5, (t, err)
    ens.close()


@pytest.mark.parametrize("name,M,N,steps", [("c1", 20, 10, 30), ("c2", 200, 100, 6),
                                            ("c3", 160, 80, 6)])
def test_mixed_propagation_against_the_oracle(name, M, N, steps):
    """Mixed path over several steps (FP32 propagation with FP32
    accumulation on the matrix cores): orbitals, hop probabilities and the
    impurity population P_d^wf against the FP64 oracle run from the same
    inputs, at 1e-5; hop events bit-exact outside near-ties.  Near-tie
    window of the mixed path: 1e-4 of the hop-probability total, a hundred
    times the relative error of its running sums (the probabilities agree
    to about 1e-6 of their largest, test_mixed_hop_probabilities)."""
    cfg = make_cfg(name, M=M, N=N)
    m = models.from_config(cfg, M=M)
    T = 6
    xs = np.linspace(2.5, 10.0, T) if name == "c3" else np.linspace(-4, 10, T)
    states = random_states(m, N, T, seed=31 + M, xs=xs, v_scale=0.01 if name == "c3" else 0.002)
    ens = ensemble(cfg, T, precision="mixed", record_every=1)
    upload(ens, states)
    obs = ens.run(steps, record=True)
    x, v, Cf, occ = ens.get_state()
    g = ens.hop_probs()
    evs, _ = ens.events()
    from paper_2212_00518_amd import unpack_C
    compared = 0
    for t in range(T):
        ref, ref_ev, recs = dyn.run(m, states[t], cfg["dt"], steps, cfg["seed"], t, record_every=1)
        if any(e["margin"] < 1e-4 * max(e["g_total"], 1e-300) for e in ref_ev):
            continue
        mine = [(e["step"], e["a"], e["b"], e["accepted"]) for e in evs if e["traj"] == t]
        assert mine == [(e["step"], e["a"], e["b"], e["accepted"]) for e in ref_ev], t
        Cg = unpack_C(Cf, t, m.n, N, ens.n_max, ens.N_max)
        dC = np.max(np.abs(Cg - ref.C))
        dP = max(abs(obs[q, t, 1] - r["Pd_wf"]) for q, r in enumerate(recs))
        gref = dyn.hop_probs(m, ref, cfg["dt"])
        gt = g[t, : N * m.n].reshape(N, m.n)
        dg = np.max(np.abs(gt - gref)) / max(np.max(gref), 1e-300)
        print(f"{name} M={M} traj {t}: |dC| {dC:.2e}  |dPd_wf| {dP:.2e}  |dg|/max g {dg:.2e}",
              flush=True)
        assert dC <= 1e-5 and dP <= 1e-5 and dg <= 1e-5, (t, dC, dP, dg)
        assert abs(x[t] - ref.x[0]) <= 1e-9 * max(1.0, abs(ref.x[0]))
        compared += 1
    assert compared >= T - 2
    ens.close()


def test_mixed_observables_records():
    """Observable records of the mixed path against the FP64 oracle's records
    at 1e-5 (energies relative, populations absolute)."""
    T, steps, rec = 8, 60, 20
    cfg, m, states = _hot_c1(T)
    from paper_2212_00518_amd import from_config
    ens = from_config(cfg, n_traj=T, precision="mixed", record_every=rec)
    upload(ens, states)
    obs = ens.run(steps, record=True)
    compared = 0
    for t in range(T):
        _, ref_ev, records = dyn.run(m, states[t], cfg["dt"], steps, cfg["seed"], t, record_every=rec)
        if any(e["margin"] < 1e-4 * max(e["g_total"], 1e-300) for e in ref_ev):
            continue
        for q, r in enumerate(records):
            for i, key in enumerate(("Pd_surf", "Pd_wf", "Ekin", "Epot", "Etot")):
                scale = 1.0 if key.startswith("Pd") else max(1e-6, abs(r[key]))
                assert abs(obs[q, t, i] - r[key]) <= 1e-5 * scale, (q, t, key)
        compared += 1
    assert compared >= T - 2
    ens.close()


@pytest.mark.parametrize("name,M,N", [("c1", 20, 10), ("c2", 200, 100), ("c1", 70, 40)])
def test_lowdin_step_restores_orthonormality(name, M, N):
    """Mixed path with the FP64 Loewdin correction after every step, from
    orbitals that are off orthonormal by about 1e-4.  Loewdin commutes with
    the unitary propagation, and the determinant ratios are invariant under
    C -> C R, so the result must equal lowdin(oracle step) and the occupations
    and events the oracle's; the overlap defect must drop to FP32 rounding."""
    cfg = make_cfg(name, M=M, N=N)
    m = models.from_config(cfg, M=M)
    T = 4
    states = random_states(m, N, T, seed=23 + M, xs=np.linspace(-4, 10, T), v_scale=0.002)
    rs = np.random.default_rng(99)
    for st in states:
        st.C = st.C + 1e-4 * (rs.normal(size=st.C.shape) + 1j * rs.normal(size=st.C.shape))
    from paper_2212_00518_amd import from_config, pack_states, unpack_C
    ens = from_config(cfg, n_traj=T, precision="mixed", lowdin_every=1)
    ens.set_state(*pack_states([(s.x, s.v, s.C, s.s) for s in states], ens.n_max, ens.N_max))
    ens.step()
    x, v, Cf, occ = ens.get_state()
    for t in range(T):
        ref, ev, _ = dyn.step(m, states[t], cfg["dt"], rng.uniform(cfg["seed"], t, 0))
        defect_before = np.max(np.abs(ref.C.conj().T @ ref.C - np.eye(N)))
        assert defect_before > 1e-5
        expect = el.lowdin(ref.C)
        Cg = unpack_C(Cf, t, m.n, N, ens.n_max, ens.N_max)
        assert np.max(np.abs(Cg - expect)) <= 2e-5, t
        assert np.max(np.abs(Cg.conj().T @ Cg - np.eye(N))) <= 2e-6, t
        near_tie = ev["attempted"] and ev["margin"] < 1e-2 * max(ev["g_total"], 1e-300)
        if not near_tie:
            assert list(occ[t, :N]) == list(ref.s), t
    ens.close()


# ------------------------------------------------------------------ compaction
def _two_class_run(compact_every, steps=200, T=96, **extra):
    from paper_2212_00518_amd import _lib
    cfg = get_config("c1")
    descs = []
    for M in (20, 30):
        eps, w = _lib.discretize(cfg["bath"]["kind"], M, cfg["bath"]["W"])
        descs.append(_lib.model_desc(cfg["model"], eps, w, M // 2))
    tm = np.arange(T) % 2
    run = dict(n_traj=T, precision="fp64", dt=cfg["dt"], kT=cfg["kT"], seed=11,
               record_every=10, exit_enabled=1, exit_x=2.0, compact_every=compact_every)
    run.update(extra)
    ens = _lib.Ensemble(descs, run, traj_model=tm)
    x0, v0 = boltzmann_harmonic(T, cfg["model"]["mass"], cfg["model"]["omega"], cfg["kT"], seed=5)
    x0 = x0 - 2.0  # start below the exit distance; trajectories cross it at scattered times
    ens.init_thermal(x0, v0)
    obs = ens.run(steps, record=True)
    state = ens.get_state()
    status = ens.status()
    evs, _ = ens.events(cap=1 << 16)
    info = [ens.class_info(k) for k in (0, 1)]
    clock = ens.clock()
    ens.close()
    return obs, state, status, evs, info, clock


def test_compaction_is_invisible_in_the_results():
    """Moving exited trajectories behind the active ones (every 10 steps) and
    visiting only the active slots changes nothing a caller can see: states,
    statuses, observable records and hop events are bitwise those of the same
    run without compaction, for two bath-size classes in one context."""
    ref = _two_class_run(0)
    got = _two_class_run(10)
    exited = int(np.sum(ref[2] & 1))
    assert 10 <= exited <= 90, exited  # the test exercises partial exits
    for a, b in zip(ref[1], got[1]):
        assert np.array_equal(a, b)
    assert np.array_equal(ref[2], got[2])
    assert np.array_equal(ref[0], got[0], equal_nan=True)
    key = lambda e: (e["step"], e["traj"], e["a"], e["b"], e["accepted"])
    assert sorted(map(key, ref[3])) == sorted(map(key, got[3]))
    live = sum(i["live"] for i in got[4])
    assert live < 96 and live >= 96 - exited
    assert all(i["live"] == i["n_traj"] for i in ref[4])


# ------------------------------------------------------------------ desorption
def test_desorption_exit_and_total_probability_match_the_oracle():
    """Desorption workload (Table et-parameters, Gauss-Legendre bath, 300 K
    Fermi occupations) with the 5 Angstrom threshold: trajectories started
    just inside it, half moving out; the GPU freezes each at the end of the
    step that takes it past the threshold.  P_total(t) after every 100 steps
    and the frozen states equal the oracle's step-by-step run (trajectories
    with a near-tie hop decision are left out)."""
    from paper_2212_00518_amd import _lib
    cfg = make_cfg("desorption", M=20, N=10)
    m = models.from_config(cfg, M=20)
    T, steps, chunk = 12, 400, 100
    xth = cfg["x_threshold"]
    rs = np.random.default_rng(4)
    x0 = xth - rs.uniform(0.5, 1.2, size=T)
    e_kin = rs.uniform(ev_to_ha(0.1), ev_to_ha(0.5), size=T)
    v0 = np.sqrt(2.0 * e_kin / m.mass[0]) * np.where(np.arange(T) % 2 == 0, 1.0, -1.0)
    states = [dyn.initial_state(m, x0[t], v0[t], 10, cfg["kT"], cfg["seed"], t) for t in range(T)]
    eps, w = _lib.discretize(cfg["bath"]["kind"], 20, cfg["bath"]["W"])
    desc = _lib.model_desc(cfg["model"], eps, w, 10)
    ens = _lib.Ensemble([desc], dict(n_traj=T, precision="fp64", dt=cfg["dt"], kT=cfg["kT"],
                                     seed=cfg["seed"], exit_enabled=1, exit_x=xth))
    upload(ens, states)
    p_gpu = []
    for _ in range(steps // chunk):
        ens.run(chunk)
        p_gpu.append(int(np.sum(ens.status() & _lib.TRAJ_EXITED)))
    x, v, Cf, occ = ens.get_state()
    ens.close()
    exit_step = np.full(T, steps + 1)
    compared = 0
    for t in range(T):
        st = states[t]
        F = None
        tie = False
        for k in range(steps):
            st, ev, F = dyn.step(m, st, cfg["dt"], rng.uniform(cfg["seed"], t, k), F)
            tie |= ev["attempted"] and ev["margin"] < 1e-7 * max(ev["g_total"], 1e-300)
            if st.x[0] > xth:
                exit_step[t] = k + 1
                break
        if tie:
            continue
        assert abs(x[t] - st.x[0]) <= 1e-8 * abs(st.x[0]), t
        assert abs(v[t] - st.v[0]) <= 1e-8 * max(1e-4, abs(st.v[0])), t
        assert list(occ[t, :10]) == list(st.s), t
        compared += 1
    p_ref = [int(np.sum(exit_step <= (q + 1) * chunk)) for q in range(steps // chunk)]
    print("P_total counts", p_gpu, p_ref, "compared", compared, flush=True)
    assert p_gpu == p_ref
    assert compared >= T - 2
    assert 0 < p_ref[-1] < T


def ev_to_ha(e):
    return e / 27.211386245988


@pytest.mark.parametrize("mu_ev,placement", [(0.5, "shift"), (-0.5, "split")])
def test_single_step_with_the_band_placed_for_a_chemical_potential(mu_ev, placement):
    """Desorption model with the chemical potential moved off the band centre
    (the band or only its Gauss-Legendre split follows mu; the electrons fill
    the bath states below mu): one step from random orbitals matches."""
    from paper_2212_00518_amd import bath_levels
    cfg = make_cfg("desorption", M=20)
    cfg["bath"]["mu"] = ev_to_ha(mu_ev)
    cfg["bath"]["placement"] = placement
    _, _, _, N = bath_levels(cfg["bath"], 20)
    assert N == 10
    cfg["n_elec"] = N
    m = models.from_config(cfg, M=20)
    T = 6
    states = random_states(m, N, T, seed=31, xs=np.linspace(3.4, 6.0, T), v_scale=0.002)
    assert _compare_step(cfg, m, states) >= T - 1


# ------------------------------------------------------ electronic sub-steps
def _substep_ensemble(cfg, T, S, precision="fp64"):
    from paper_2212_00518_amd import _lib, bath_levels
    eps, w, _, _ = bath_levels(cfg["bath"], cfg["bath"]["M"])
    desc = _lib.model_desc(cfg["model"], eps, w, cfg["n_elec"])
    return _lib.Ensemble([desc], dict(n_traj=T, precision=precision, dt=cfg["dt"], kT=cfg["kT"],
                                      seed=cfg["seed"], elec_substeps=S,
                                      lowdin_every=100 if precision == "mixed" else 0))


@pytest.mark.parametrize("S,precision,tol", [(4, "fp64", 1e-10), (3, "fp64", 1e-10), (2, "mixed", 1e-5)])
def test_electronic_substeps_match_the_oracle(S, precision, tol):
    """Sub-stepped propagation (S propagators along the drift per nuclear
    step) over 30 steps of the graph-replayed run: states and hop events
    equal the oracle's step(substeps=S) run, trajectories with a near-tie
    hop decision left out."""
    from paper_2212_00518_amd import unpack_C
    T, steps = 8, 30
    cfg, m, states = _hot_c1(T)
    ens = _substep_ensemble(cfg, T, S, precision)
    upload(ens, states)
    ens.run(steps)
    x, v, Cf, occ = ens.get_state()
    evs, _ = ens.events()
    n_max, N_max = ens.n_max, ens.N_max
    ens.close()
    compared = 0
    for t in range(T):
        ref, ref_ev, _ = dyn.run(m, states[t], cfg["dt"], steps, cfg["seed"], t, substeps=S)
        if any(e["margin"] < 1e3 * tol * max(e["g_total"], 1e-300) for e in ref_ev):
            continue
        mine = [e for e in evs if e["traj"] == t]
        assert [(e["step"], e["a"], e["b"], e["accepted"]) for e in mine] == \
               [(e["step"], e["a"], e["b"], e["accepted"]) for e in ref_ev], t
        assert abs(x[t] - ref.x[0]) <= tol * max(1.0, abs(ref.x[0])), t
        assert abs(v[t] - ref.v[0]) <= tol * max(1e-3, abs(ref.v[0])), t
        Cg = unpack_C(Cf, t, m.n, cfg["n_elec"], n_max, N_max)
        assert np.max(np.abs(Cg - ref.C)) <= 10 * tol, t
        assert list(occ[t, :cfg["n_elec"]]) == list(ref.s), t
        compared += 1
    assert compared >= T - 2


def test_one_substep_is_the_plain_step():
    """elec_substeps = 1 and the default give bitwise the same run."""
    T = 8
    cfg, m, states = _hot_c1(T)
    out = []
    for S in (0, 1):
        ens = _substep_ensemble(cfg, T, S)
        upload(ens, states)
        ens.run(40)
        out.append(ens.get_state())
        ens.close()
    for a, b in zip(*out):
        assert np.array_equal(a, b)


# ------------------------------------------------------ several coordinates
def _multi_states(m, N, T, seed, v_scale=2e-3):
    rs = np.random.default_rng(seed)
    R0 = m.r
    out = []
    for t in range(T):
        C = random_orbitals(m.n, N, seed=seed * 100 + t)
        s = np.sort(rs.choice(m.n, N, replace=False))
        out.append(dyn.State(R0 + rs.normal(0.0, 0.2, size=m.n_dof),
                             rs.normal(0.0, v_scale, size=m.n_dof) * np.sqrt(2000.0 / m.mass), C, s))
    return out


@pytest.mark.parametrize("leads", [1, 2])
def test_multi_coordinate_energies_and_hop_probabilities(leads):
    cfg = make_cfg("c5", M=30, N=15)
    cfg["bath"]["leads"] = leads
    m = models.from_config(cfg, M=30)
    T = 6
    states = _multi_states(m, 15, T, seed=3)
    ens = ensemble(cfg, T)
    assert ens.n_dof == 6
    upload(ens, states)
    lam, q0 = ens.adiabatic()
    g = ens.hop_probs()
    x, v, _, _ = ens.get_state()
    for t in range(T):
        assert np.array_equal(x[t], states[t].x) and np.array_equal(v[t], states[t].v)
        lr, Q = el.eig(m.H(states[t].x))
        assert np.max(np.abs(lam[t, :m.n] - lr)) <= 1e-10 * np.max(np.abs(lr))
        assert np.max(np.abs(q0[t, :m.n] - Q[0])) <= 1e-10
        gr = dyn.hop_probs(m, states[t], cfg["dt"])
        gg = g[t].reshape(ens.N_max, ens.n_max)[:15, :m.n]
        assert np.max(np.abs(gg - gr)) <= 1e-10 * max(np.max(gr), 1e-300), t
    ens.close()


@pytest.mark.parametrize("leads", [1, 2])
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("mixed", 1e-5)])
def test_multi_coordinate_steps_match_the_oracle(precision, tol, leads):
    """Six coordinates, 40 graph-replayed steps from random orbitals (hops
    likely): per-coordinate positions and velocities, orbitals, occupations
    and hop events equal the oracle's, trajectories with a near-tie left out.
    Two leads: every bath energy appears twice (deflated eigen-solve)."""
    from paper_2212_00518_amd import unpack_C
    cfg = make_cfg("c5", M=24, N=12)
    cfg["bath"]["leads"] = leads
    m = models.from_config(cfg, M=24)
    T = 8
    # mixed: fewer, slower steps (hop attempts whose margin is within the FP32
    # tolerance of a boundary are left out, and random orbitals give many)
    steps, vs = (40, 4e-3) if precision == "fp64" else (10, 1e-3)
    states = _multi_states(m, 12, T, seed=9, v_scale=vs)
    ens = ensemble(cfg, T, precision=precision)
    upload(ens, states)
    ens.run(steps)
    x, v, Cf, occ = ens.get_state()
    evs, _ = ens.events()
    n_max, N_max = ens.n_max, ens.N_max
    ens.close()
    compared, hops = 0, 0
    for t in range(T):
        ref, ref_ev, _ = dyn.run(m, states[t], cfg["dt"], steps, cfg["seed"], t)
        if any(e["margin"] < 1e3 * tol * max(e["g_total"], 1e-300) for e in ref_ev):
            continue
        mine = [e for e in evs if e["traj"] == t]
        assert [(e["step"], e["a"], e["b"], e["accepted"]) for e in mine] == \
               [(e["step"], e["a"], e["b"], e["accepted"]) for e in ref_ev], t
        hops += sum(e["accepted"] for e in ref_ev)
        assert np.max(np.abs(x[t] - ref.x)) <= tol * max(1.0, np.max(np.abs(ref.x))), t
        assert np.max(np.abs(v[t] - ref.v)) <= tol * max(1e-3, np.max(np.abs(ref.v))), t
        Cg = unpack_C(Cf, t, m.n, 12, n_max, N_max)
        assert np.max(np.abs(Cg - ref.C)) <= 10 * tol, t
        assert list(occ[t, :12]) == list(ref.s), t
        compared += 1
    print("compared", compared, "accepted hops", hops, flush=True)
    assert compared >= (T - 2 if precision == "fp64" else T // 2)
    if precision == "fp64":
        assert hops >= 2


# ------------------------------------------------------- repeated bath energies
def _repeated_bath(M_grid, g, W=0.1):
    """g levels at each energy of a trapezoid grid of M_grid levels, each with
    1/g of the weight (plain input data)."""
    e = -0.5 * W + np.arange(M_grid) * (W / (M_grid - 1))
    w = np.full(M_grid, W / M_grid)
    return np.repeat(e, g), np.repeat(w / g, g)


def _steps_vs_oracle(m, ens, states, steps, dt, seed, tol, N):
    from paper_2212_00518_amd import unpack_C
    upload(ens, states)
    ens.run(steps)
    x, v, Cf, occ = ens.get_state()
    evs, _ = ens.events()
    n_max, N_max = ens.n_max, ens.N_max
    compared, hops = 0, 0
    for t in range(len(states)):
        ref, ref_ev, _ = dyn.run(m, states[t], dt, steps, seed, t)
        if any(e["margin"] < 1e3 * tol * max(e["g_total"], 1e-300) for e in ref_ev):
            continue
        mine = [e for e in evs if e["traj"] == t]
        assert [(e["step"], e["a"], e["b"], e["accepted"]) for e in mine] == \
               [(e["step"], e["a"], e["b"], e["accepted"]) for e in ref_ev], t
        hops += sum(e["accepted"] for e in ref_ev)
        xt, vt = np.atleast_1d(x[t]), np.atleast_1d(v[t])
        assert np.max(np.abs(xt - ref.x)) <= tol * max(1.0, np.max(np.abs(ref.x))), t
        assert np.max(np.abs(vt - ref.v)) <= tol * max(1e-3, np.max(np.abs(ref.v))), t
        Cg = unpack_C(Cf, t, m.n, N, n_max, N_max)
        assert np.all(np.isfinite(Cg))
        assert np.max(np.abs(Cg - ref.C)) <= 10 * tol, t
        assert list(occ[t, :N]) == list(ref.s), t
        compared += 1
    return compared, hops


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("mixed", 1e-5)])
def test_two_lead_double_well_steps_match_the_oracle(precision, tol):
    """The double-well model on two leads of 20 levels (every energy twice):
    graph-replayed steps from random orbitals against the oracle's dense
    eigen-decomposition."""
    cfg = make_cfg("c2", M=40, N=20)
    cfg["bath"]["leads"] = 2
    m = models.from_config(cfg, M=40)
    T = 8
    xs = np.linspace(-8.0, 24.0, T)
    states = random_states(m, 20, T, seed=31, xs=xs, v_scale=1e-2)
    ens = ensemble(cfg, T, precision=precision)
    steps = 30 if precision == "fp64" else 8
    compared, hops = _steps_vs_oracle(m, ens, states, steps, cfg["dt"], cfg["seed"], tol, 20)
    ens.close()
    print("compared", compared, "accepted hops", hops, flush=True)
    assert compared >= (T - 2 if precision == "fp64" else T // 2)
    if precision == "fp64":
        assert hops >= 2


@pytest.mark.parametrize("g", [2, 3])
def test_repeated_levels_energies_amplitudes_and_hops(g):
    """g equal levels per energy: the deflated eigen-solve gives every
    eigenvalue of the dense matrix (g - 1 of them exactly at each bath
    energy, with impurity amplitude 0), the hop probabilities of the oracle,
    and steps equal to the oracle's (FP64)."""
    from paper_2212_00518_amd import _lib
    c1 = get_config("c1")
    eps, w = _repeated_bath(12, g)
    N = len(eps) // 2
    mc = c1["model"]
    m = models.Harmonic(eps, w, mc["Gamma"], mc["mass"], mc["omega"], mc["g"], mc["dG"],
                        mc.get("eps_d", 0.0))
    T = 6
    desc = _lib.model_desc(mc, eps, w, N)
    run = dict(n_traj=T, precision="fp64", dt=c1["dt"], kT=0.0, seed=3)
    ens = _lib.Ensemble([desc], run)
    states = random_states(m, N, T, seed=17, xs=np.linspace(-6.0, 26.0, T), v_scale=4e-3)
    upload(ens, states)
    lam, q0 = ens.adiabatic()
    gp = ens.hop_probs()
    for t in range(T):
        lr, Q = el.eig(m.H(states[t].x))
        assert np.max(np.abs(lam[t, :m.n] - lr)) <= 1e-10 * np.max(np.abs(lr))
        assert np.max(np.abs(np.abs(q0[t, :m.n]) - np.abs(Q[0]))) <= 1e-10
        at_grid = np.isin(lam[t, :m.n], eps)
        assert at_grid.sum() == 12 * (g - 1)
        assert np.all(q0[t, :m.n][at_grid] == 0.0)
        gr = dyn.hop_probs(m, states[t], c1["dt"])
        gg = gp[t].reshape(ens.N_max, ens.n_max)[:N, :m.n]
        assert np.all(np.isfinite(gg))
        assert np.max(np.abs(gg - gr)) <= 1e-10 * max(np.max(gr), 1e-300), t
    compared, hops = _steps_vs_oracle(m, ens, states, 20, c1["dt"], 3, 1e-10, N)
    ens.close()
    print("g", g, "compared", compared, "accepted hops", hops, flush=True)
    assert compared >= T - 2


@pytest.mark.parametrize("bias", [0.0, 0.01, 0.02])
def test_biased_initial_occupations_match_the_oracle(bias):
    """Two leads at mu +- V/2: the occupations drawn by iesh_init_thermal equal
    the oracle's (same Philox uniforms, FP64 probabilities)."""
    from workloads.sampling import boltzmann_coordinates
    cfg = make_cfg("c5", M=40, N=20)
    cfg["bath"]["bias"] = bias
    m = models.from_config(cfg, M=40)
    T = 16
    dof = np.array(cfg["model"]["dof"])
    om = dof[:, 2] * np.sqrt(2.0 * dof[:, 1] / dof[:, 0])
    x0, v0 = boltzmann_coordinates(T, dof[:, 0], om, dof[:, 3], cfg["kT"], seed=4)
    ens = ensemble(cfg, T)
    ens.init_thermal(x0, v0)
    _, _, _, occ = ens.get_state()
    ens.close()
    for t in range(T):
        ref = dyn.initial_state(m, x0[t], v0[t], 20, cfg["kT"], cfg["seed"], t, bias=bias)
        assert list(occ[t, :20]) == list(ref.s), t


def test_two_lead_error_paths():
    from paper_2212_00518_amd import _lib
    cfg = make_cfg("c2", M=20, N=10)
    cfg["bath"]["bias"] = 0.01     # one lead: a bias has no leads to act on
    with pytest.raises(_lib.IeshError):
        ensemble(cfg, 2)
    cfg = make_cfg("c5", M=20, N=10)
    cfg["bath"]["bias"] = 0.01
    cfg["kT"] = 0.0                # a bias needs a temperature
    with pytest.raises(_lib.IeshError):
        ensemble(cfg, 2)
    c1 = get_config("c1")
    eps, w = _repeated_bath(6, 2)
    bad = np.tile(np.array([0, 2], dtype=np.int32), 6)
    with pytest.raises(_lib.IeshError):
        _lib.Ensemble([_lib.model_desc(c1["model"], eps, w, 6, bad)],
                      dict(n_traj=2, precision="fp64", dt=c1["dt"]))
    with pytest.raises(_lib.IeshError):  # not ascending
        _lib.Ensemble([_lib.model_desc(c1["model"], eps[::-1].copy(), w, 6)],
                      dict(n_traj=2, precision="fp64", dt=c1["dt"]))
    ens = _lib.Ensemble([_lib.model_desc(c1["model"], eps, w, 6)],
                        dict(n_traj=2, precision="fp64", dt=c1["dt"]))
    with pytest.raises(_lib.IeshError, match="distinct"):
        ens.adjoint_forward(np.zeros((2, 4)), 2)
    ens.close()


def test_records_of_frozen_trajectories_are_nan_in_every_call():
    """A trajectory frozen before a record falls due takes no step: its
    record is NaN, in the call in which it froze and in later calls (no
    values left over from an earlier call or buffer), while the records of
    the trajectories still running are the observables."""
    from paper_2212_00518_amd import _lib
    cfg = get_config("c1")
    T = 64
    eps, w = _lib.discretize(cfg["bath"]["kind"], 20, cfg["bath"]["W"])
    run = dict(n_traj=T, precision="fp64", dt=cfg["dt"], kT=cfg["kT"], seed=3, record_every=10,
               exit_enabled=1, exit_x=2.0)
    ens = _lib.Ensemble([_lib.model_desc(cfg["model"], eps, w, 10)], run)
    x0, v0 = boltzmann_harmonic(T, cfg["model"]["mass"], cfg["model"]["omega"], cfg["kT"], seed=5)
    ens.init_thermal(x0 - 2.0, v0)
    first = ens.run(60, record=True)
    st1 = ens.status()
    second = ens.run(120, record=True)   # a larger buffer: reallocated
    st2 = ens.status()
    third = ens.run(60, record=True)     # the same buffer again
    st3 = ens.status()
    ens.close()
    frozen = [(st & _lib.TRAJ_EXITED) > 0 for st in (st1, st2, st3)]
    assert 5 <= frozen[0].sum() < frozen[1].sum() < frozen[2].sum() < T - 5, [f.sum() for f in frozen]
    # frozen before the call: NaN throughout it
    assert np.all(np.isnan(second[:, frozen[0], :]))
    assert np.all(np.isnan(third[:, frozen[1], :]))
    # still running at the end of a call: every record of the call is finite
    for rec, fr in zip((first, second, third), frozen):
        assert np.all(np.isfinite(rec[:, ~fr, :]))


def test_no_hop_bound_with_a_long_loewdin_period_is_exact():
    """Mixed path with a Loewdin step only every 400 steps, over 2000 steps:
    the measured orthonormality defect sets the no-hop bound's allowance, and
    the run with the bound is bit-identical to the run with the determinant
    ratios at every step; no measured defect exceeded its allowance.  Without
    Loewdin steps (lowdin_every = 0) the defect is never measured and every
    step evaluates the ratios."""
    cfg = make_cfg("c2", M=40, N=20)
    m = models.from_config(cfg, M=40)
    T = 24
    states = random_states(m, 20, T, seed=43, xs=np.linspace(-8.0, 24.0, T), v_scale=1e-2)
    for t in range(1, T, 2):
        states[t] = dyn.State(states[t].x, states[t].v, np.eye(m.n, 20, dtype=np.complex128),
                              np.arange(20))
    out = []
    for off in (0, 1):
        ens = ensemble(cfg, T, precision="mixed", hop_filter_off=off, lowdin_every=400)
        upload(ens, states)
        ens.run(2000)
        st = ens.get_state()
        evs, _ = ens.events(cap=1 << 18)
        hop_evals = ens.hop_evals()
        d, dmax, viol = ens.defect()
        ens.close()
        out.append((st, [(e["step"], e["traj"], e["a"], e["b"], e["accepted"]) for e in evs],
                    hop_evals, dmax, viol))
    (s0, e0, h0, d0, v0), (s1, e1, h1, d1, v1) = out
    for a, b in zip(s0, s1):
        assert np.array_equal(a, b)
    assert e0 == e1
    print("events", len(e0), "exact evaluations", h0, "->", h1, "max defect", d0, flush=True)
    assert len(e0) > 0 and h1 == T * 2000 and 0 < h0 < h1
    assert 0.0 < d0 < 1e-3 and d0 == d1 and v0 == 0
    ens = ensemble(cfg, T, precision="mixed", lowdin_every=0)
    upload(ens, states)
    ens.timing(True)
    ens.run(50)
    assert ens.hop_evals() == T * 50
    assert ens.defect()[1] == 0.0
    ens.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_exact_hop_filter_does_not_change_the_dynamics(precision):
    """hop_filter_off = 1 evaluates the determinant ratios at every step; the
    no-hop bound is exact, so positions, velocities, orbitals, occupations and
    hop events are bit-identical with and without it."""
    cfg = make_cfg("c2", M=40, N=20)
    m = models.from_config(cfg, M=40)
    T = 24
    # even trajectories: random orbitals (hops happen; the bound never rules a
    # step out); odd ones: the lowest orbitals as unit vectors (the bound rules
    # out most steps)
    states = random_states(m, 20, T, seed=41, xs=np.linspace(-8.0, 24.0, T), v_scale=1e-2)
    for t in range(1, T, 2):
        states[t] = dyn.State(states[t].x, states[t].v, np.eye(m.n, 20, dtype=np.complex128),
                              np.arange(20))
    out = []
    for off in (0, 1):
        ens = ensemble(cfg, T, precision=precision, hop_filter_off=off)
        upload(ens, states)
        ens.run(200)
        st = ens.get_state()
        evs, _ = ens.events()
        hop_evals = ens.hop_evals()
        ens.close()
        out.append((st, [(e["step"], e["traj"], e["a"], e["b"], e["accepted"]) for e in evs], hop_evals))
    (s0, e0, h0), (s1, e1, h1) = out
    for a, b in zip(s0, s1):
        assert np.array_equal(a, b)
    assert e0 == e1
    print("events", len(e0), "exact evaluations", h0, "->", h1, flush=True)
    assert len(e0) > 0
    assert h1 == T * 200 and 0 < h0 < h1


def test_exit_on_a_chosen_coordinate():
    """exit_dof = 2: a trajectory is frozen as soon as coordinate 2 passes
    exit_x, and never otherwise."""
    from paper_2212_00518_amd import _lib
    cfg = make_cfg("c5", M=12, N=6)
    cfg["bath"]["leads"] = 1
    m = models.from_config(cfg, M=12)
    T = 32
    rs = np.random.default_rng(12)
    states = [dyn.State(m.r + rs.normal(0.0, 0.05, size=6), rs.normal(0.0, 2e-3, size=6),
                        np.eye(m.n, 6, dtype=np.complex128), np.arange(6)) for _ in range(T)]
    exit_x = 0.2  # about 19 of 32 pass it within 60 steps (oracle run)
    ens = ensemble(cfg, T, exit_enabled=1, exit_x=exit_x, exit_dof=2)
    upload(ens, states)
    ens.run(60)
    x, _, _, _ = ens.get_state()
    status = ens.status()
    ens.close()
    gone = (status & _lib.TRAJ_EXITED) > 0
    print("exited", int(gone.sum()), "of", T, flush=True)
    assert 0 < gone.sum() < T
    assert np.all(x[gone, 2] > exit_x)
    assert np.all(x[~gone, 2] <= exit_x)



# ------------------------------------------------------------ adaptive step
def _oracle_adaptive(m, st, dt0, steps, seed, traj, g_max, levels):
    """The oracle's adaptive run, step by step, keeping every step's total and
    the margin of each step-size decision."""
    F = el.forces(m, st.x, st.s)
    dt, time, evs, dmargin = dt0, 0.0, [], 1e300
    for k in range(steps):
        st, ev, F = dyn.step(m, st, dt, rng.uniform(seed, traj, k), F)
        ev["step"] = k
        if ev["attempted"]:
            evs.append(ev)
        time += dt
        for q in range(levels + 1):
            dmargin = min(dmargin, abs(ev["g_total"] * (dt0 / 2 ** q) / dt - g_max) / g_max)
        dt = dyn.next_dt(ev["g_total"], dt, dt0, g_max, levels)
    return st, evs, time, dt, dmargin


@pytest.mark.parametrize("filter_off", [0, 1])
def test_adaptive_step_matches_the_oracle(filter_off):
    """dt_levels = 4, hop_gmax = 0.02 on random orbitals (large hop
    probabilities): per-trajectory steps, clocks, states and hop events equal
    the oracle's adaptive run (decisions within 1e-9 of a threshold left out)."""
    from paper_2212_00518_amd import unpack_C
    cfg = make_cfg("c1", M=12, N=6)
    m = models.from_config(cfg, M=12)
    T, steps, g_max, levels = 10, 40, 0.02, 4
    states = random_states(m, 6, T, seed=23, xs=np.linspace(-4.0, 20.0, T), v_scale=1.5e-2)
    ens = ensemble(cfg, T, dt_levels=levels, hop_gmax=g_max, hop_filter_off=filter_off)
    upload(ens, states)
    ens.run(steps)
    x, v, Cf, occ = ens.get_state()
    evs, _ = ens.events()
    time, dtn = ens.clock()
    n_max, N_max = ens.n_max, ens.N_max
    ens.close()
    compared, reduced = 0, 0
    for t in range(T):
        ref, ref_ev, rtime, rdt, dmargin = _oracle_adaptive(m, states[t], cfg["dt"], steps,
                                                            cfg["seed"], t, g_max, levels)
        if dmargin < 1e-9 or any(e["margin"] < 1e-7 * max(e["g_total"], 1e-300) for e in ref_ev):
            continue
        mine = [e for e in evs if e["traj"] == t]
        assert [(e["step"], e["a"], e["b"], e["accepted"]) for e in mine] == \
               [(e["step"], e["a"], e["b"], e["accepted"]) for e in ref_ev], t
        assert time[t] == rtime and dtn[t] == rdt, (t, time[t], rtime, dtn[t], rdt)
        assert abs(x[t] - ref.x[0]) <= 1e-10 * max(1.0, abs(ref.x[0])), t
        assert abs(v[t] - ref.v[0]) <= 1e-10 * max(1e-3, abs(ref.v[0])), t
        assert np.max(np.abs(unpack_C(Cf, t, m.n, 6, n_max, N_max) - ref.C)) <= 1e-9, t
        assert list(occ[t, :6]) == list(ref.s), t
        compared += 1
        reduced += rtime < steps * cfg["dt"]
    print("compared", compared, "with reduced steps", reduced, flush=True)
    assert compared >= T - 2 and reduced >= 3


def test_fixed_step_clock_counts_steps():
    cfg = make_cfg("c1", M=12, N=6)
    T = 4
    x0, v0 = boltzmann_harmonic(T, cfg["model"]["mass"], cfg["model"]["omega"], cfg["kT"], seed=1)
    ens = ensemble(cfg, T)
    ens.init_thermal(x0, v0)
    ens.run(17)
    time, dtn = ens.clock()
    ens.close()
    assert np.all(time == 17 * cfg["dt"]) and np.all(dtn == cfg["dt"])


def test_adaptive_step_with_compaction_is_invisible_in_the_results():
    """The step clocks move with their trajectories: an adaptive run (a tiny
    threshold, so steps shrink near the crossing) with compaction every 10
    steps equals the same run without it, clocks included."""
    extra = dict(dt_levels=3, hop_gmax=1e-7)
    ref = _two_class_run(0, **extra)
    got = _two_class_run(10, **extra)
    for a, b in zip(ref[1], got[1]):
        assert np.array_equal(a, b)
    assert np.array_equal(ref[2], got[2])
    assert np.array_equal(ref[5][0], got[5][0]) and np.array_equal(ref[5][1], got[5][1])
    steps_taken = ref[5][0] / get_config("c1")["dt"]
    print("exited", int(np.sum(ref[2] & 1)), "min time in steps", steps_taken.min(), flush=True)
    assert np.any(ref[5][1] < get_config("c1")["dt"])  # some next steps are reduced
    assert int(np.sum(ref[2] & 1)) >= 10


def test_adaptive_step_error_paths():
    from paper_2212_00518_amd import _lib
    cfg = make_cfg("c1", M=12, N=6)
    with pytest.raises(_lib.IeshError):
        ensemble(cfg, 2, dt_levels=2)            # no threshold
    with pytest.raises(_lib.IeshError):
        ensemble(cfg, 2, dt_levels=31, hop_gmax=0.1)


def test_hop_total_above_one_is_not_clipped():
    """Large velocities: several trajectories have a hop-probability total
    above one.  The probabilities are the oracle's (no clipping), and one step
    selects the same hop as the oracle (with a total above one a uniform
    below one always finds a pair)."""
    cfg = make_cfg("c1", M=20, N=10)
    m = models.from_config(cfg, M=20)
    T = 8
    states = random_states(m, 10, T, seed=71, xs=np.linspace(8.0, 14.0, T), v_scale=0.1)
    ens = ensemble(cfg, T)
    upload(ens, states)
    g = ens.hop_probs()
    above = 0
    for t in range(T):
        gr = dyn.hop_probs(m, states[t], cfg["dt"])
        gg = g[t].reshape(ens.N_max, ens.n_max)[:10, :m.n]
        assert np.max(np.abs(gg - gr)) <= 1e-10 * np.max(gr), t
        above += gr.sum() > 1.0
    assert above >= 3
    ens.set_step(7)
    ens.step()
    evs, _ = ens.events()
    _, _, _, occ = ens.get_state()
    ens.close()
    for t in range(T):
        st, ev, _ = dyn.step(m, states[t], cfg["dt"], rng.uniform(cfg["seed"], t, 7))
        if ev["margin"] < 1e-7 * ev["g_total"]:
            continue
        mine = [e for e in evs if e["traj"] == t]
        if ev["g_total"] > 1.0:
            assert ev["attempted"]
        assert [(e["a"], e["b"], e["accepted"]) for e in mine] == \
               ([(ev["a"], ev["b"], ev["accepted"])] if ev["attempted"] else []), t
        assert list(occ[t, :10]) == list(st.s), t


def test_a_model_without_trajectories_changes_nothing():
    """Two models in one context with every trajectory on the second: the
    empty class is skipped and the run equals the one-model context bit for
    bit; zero steps are a no-op."""
    from paper_2212_00518_amd import _lib
    cfg = get_config("c1")
    T = 12
    descs = []
    for M in (30, 20):
        eps, w = _lib.discretize(cfg["bath"]["kind"], M, cfg["bath"]["W"])
        descs.append(_lib.model_desc(cfg["model"], eps, w, M // 2))
    run = dict(n_traj=T, precision="fp64", dt=cfg["dt"], kT=cfg["kT"], seed=2)
    x0, v0 = boltzmann_harmonic(T, cfg["model"]["mass"], cfg["model"]["omega"], cfg["kT"], seed=9)
    out = []
    for models_, tm in ((descs, np.ones(T, dtype=np.int32)), (descs[1:], None)):
        ens = _lib.Ensemble(models_, run, traj_model=tm)
        ens.init_thermal(x0, v0)
        before = ens.get_state()
        ens.run(0)
        after = ens.get_state()
        for a, b in zip(before, after):
            assert np.array_equal(a, b)
        ens.run(40)
        out.append((ens.get_state(), ens.n_max, ens.N_max))
        ens.close()
    from paper_2212_00518_amd import unpack_C
    (s0, n0, N0), (s1, n1, N1) = out
    assert np.array_equal(s0[0], s1[0]) and np.array_equal(s0[1], s1[1])
    assert np.array_equal(s0[3][:, :10], s1[3][:, :10])
    for t in range(T):
        assert np.array_equal(unpack_C(s0[2], t, 21, 10, n0, N0), unpack_C(s1[2], t, 21, 10, n1, N1))


@pytest.mark.parametrize("bias", [0.01, 0.02])
def test_biased_occupations_with_offset_lead_grids(bias):
    """Two leads on grids offset by half a spacing (no equal energies, no
    deflation): the lead weights of every orbital come from the coupling
    formula alone; the sampled occupations equal the oracle's."""
    from paper_2212_00518_amd import _lib
    from workloads.sampling import boltzmann_coordinates
    cfg = make_cfg("c5", M=40, N=20)
    W, M1 = 0.1, 20
    e1 = -0.5 * W + np.arange(M1) * (W / (M1 - 1))
    w1 = np.full(M1, W / M1)
    eps = np.concatenate([e1, e1 + 0.5 * W / (M1 - 1)])
    w = np.concatenate([0.5 * w1, 0.5 * w1])
    lead = np.repeat(np.array([0, 1], dtype=np.int32), M1)
    order = np.argsort(eps, kind="stable")
    eps, w, lead = eps[order], w[order], lead[order]
    mc = cfg["model"]
    m = models.MultiDof(eps, w, mc["Gamma"], mc["dof"], mc["Delta"], mc.get("eps_d", 0.0))
    m.lead = lead
    T = 12
    dof = np.array(mc["dof"])
    om = dof[:, 2] * np.sqrt(2.0 * dof[:, 1] / dof[:, 0])
    x0, v0 = boltzmann_coordinates(T, dof[:, 0], om, dof[:, 3], cfg["kT"], seed=8)
    ens = _lib.Ensemble([_lib.model_desc(mc, eps, w, 20, lead)],
                        dict(n_traj=T, precision="fp64", dt=cfg["dt"], kT=cfg["kT"], seed=cfg["seed"],
                             bias=bias))
    ens.init_thermal(x0, v0)
    _, _, _, occ = ens.get_state()
    ens.close()
    for t in range(T):
        ref = dyn.initial_state(m, x0[t], v0[t], 20, cfg["kT"], cfg["seed"], t, bias=bias)
        assert list(occ[t, :20]) == list(ref.s), t


# ------------------------------------------------------------- failure states
def test_nonconvergence_hook_freezes_every_trajectory():
    """eig_max_iter = 1 (a host-set cap on the secular iterations): the roots
    do not converge, every trajectory is marked NONCONV at initialisation and
    stays frozen through later steps."""
    from paper_2212_00518_amd import _lib
    cfg = make_cfg("c1", M=20, N=10)
    T = 4
    x0, v0 = boltzmann_harmonic(T, cfg["model"]["mass"], cfg["model"]["omega"], cfg["kT"], seed=3)
    ens = ensemble(cfg, T, eig_max_iter=1)
    ens.init_thermal(x0, v0)
    s0 = ens.status()
    before = ens.get_state()
    ens.run(3)
    after = ens.get_state()
    s1 = ens.status()
    ens.close()
    assert np.all(s0 & _lib.TRAJ_NONCONV) and np.array_equal(s0, s1)
    for a, b in zip(before, after):
        assert np.array_equal(a, b)


def test_nonfinite_input_freezes_only_that_trajectory():
    """A NaN position and an infinite velocity: those two trajectories are
    frozen with NONFINITE (and NONCONV from the failed solve); the others run
    exactly as in an ensemble without the bad inputs."""
    from paper_2212_00518_amd import _lib, unpack_C
    cfg = make_cfg("c1", M=20, N=10)
    m = models.from_config(cfg, M=20)
    T = 6
    states = random_states(m, 10, T, seed=13, xs=np.linspace(-4.0, 20.0, T), v_scale=4e-3)
    bad = [s.copy() for s in states]
    bad[2] = dyn.State([np.nan], bad[2].v, bad[2].C, bad[2].s)
    bad[4] = dyn.State(bad[4].x, [np.inf], bad[4].C, bad[4].s)
    out = []
    for sts in (states, bad):
        ens = ensemble(cfg, T)
        upload(ens, sts)
        ens.run(5)
        out.append((ens.get_state(), ens.status(), ens.events()[0], ens.n_max, ens.N_max))
        ens.close()
    (g, sg, eg, n_max, N_max), (b, sb, eb, _, _) = out
    assert sb[2] & (_lib.TRAJ_NONFINITE | _lib.TRAJ_NONCONV)
    assert sb[4] & _lib.TRAJ_NONFINITE
    for t in (0, 1, 3, 5):
        assert sg[t] == 0 and sb[t] == 0
        assert b[0][t] == g[0][t] and b[1][t] == g[1][t]
        assert np.array_equal(unpack_C(b[2], t, m.n, 10, n_max, N_max), unpack_C(g[2], t, m.n, 10, n_max, N_max))
        assert np.array_equal(b[3][t], g[3][t])
    key = lambda e: (e["step"], e["traj"], e["a"], e["b"], e["accepted"])
    assert [key(e) for e in eb if e["traj"] not in (2, 4)] == [key(e) for e in eg if e["traj"] not in (2, 4)]


def test_frustrated_hops_match_the_oracle():
    """Small velocities and mixed orbitals: selected upward hops that the
    kinetic energy cannot pay for are frustrated (velocity unchanged), event
    for event as in the oracle."""
    cfg = make_cfg("c1", M=20, N=10)
    m = models.from_config(cfg, M=20)
    T = 8
    states = random_states(m, 10, T, seed=5, xs=np.linspace(-4.0, 20.0, T), v_scale=1e-3)
    ens = ensemble(cfg, T)
    compared, hops = _steps_vs_oracle(m, ens, states, 40, cfg["dt"], cfg["seed"], 1e-10, 10)
    evs, _ = ens.events()
    ens.close()
    frustrated = sum(1 for e in evs if not e["accepted"])
    print("compared", compared, "accepted", hops, "frustrated", frustrated, flush=True)
    assert compared >= T - 1 and frustrated >= 2
