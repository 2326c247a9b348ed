"""Oracle pins: whole steps, energy conservation, initial occupations, RNG."""
import itertools
import math
import os

import numpy as np

from oracle import models, rng
from oracle import electronic as el
from oracle import dynamics as dyn
from workloads import get_config, boltzmann_harmonic

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_philox_known_answers():
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        rows = [l.split() for l in f if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for row in rows:
        vals = [int(t, 16) for t in row]
        assert rng.philox4x32_10(vals[0:4], vals[4:6]) == tuple(vals[6:10])


def test_uniform_range_and_moments():
    u = np.array([rng.uniform(123, t, k) for t in range(20) for k in range(500)])
    assert np.all((u >= 0) & (u < 1))
    assert abs(u.mean() - 0.5) < 0.01
    assert abs(u.var() - 1 / 12) < 0.005
    assert len(np.unique(u)) == len(u)


def _c1_like(M=20, N=10):
    cfg = get_config("c1")
    cfg["bath"]["M"] = M
    cfg["n_elec"] = N
    return cfg, models.from_config(cfg)


def test_energy_conserved_between_and_across_hops():
    """Velocity Verlet changes E_tot by a small amount per step, and a step
    with an accepted hop changes it by no more than an ordinary step, although
    the electronic energy jumps by lambda_b - lambda_a (rescaling, Sec. II.B)."""
    cfg, m = _c1_like(M=12, N=6)
    cfg["model"]["Gamma"] = 0.001          # sharp avoided crossings: hops happen
    m = models.from_config(cfg)
    x, v = boltzmann_harmonic(6, 2000.0, 2e-4, cfg["kT"], seed=1, kT_factor=200.0)
    hop_dE, step_dE, jumps = [], [], []
    for t in range(6):
        st = dyn.initial_state(m, x[t], v[t], 6, cfg["kT"], 0, t)
        E = dyn.observables(m, st)["Etot"]
        F = None
        for k in range(400):
            st, ev, F = dyn.step(m, st, 50.0, rng.uniform(5, t, k), F)
            ob = dyn.observables(m, st)
            (hop_dE if ev["accepted"] else step_dE).append(abs(ob["Etot"] - E))
            E = ob["Etot"]
            if ev["accepted"]:
                lam, _ = el.eig(m.H(st.x))
                jumps.append(abs(lam[ev["b"]] - lam[ev["a"]]))
        assert dyn.observables(m, st)["ortho"] < 1e-12
    assert len(hop_dE) >= 5
    assert max(step_dE) < 1e-5 and max(hop_dE) < 1e-5
    assert min(jumps) > 100 * max(hop_dE)


def test_run_is_deterministic():
    cfg, m = _c1_like(M=8, N=4)
    st0 = dyn.initial_state(m, 1.0, 0.002, 4, cfg["kT"], 0, 0)
    a = dyn.run(m, st0.copy(), 50.0, 100, 3, 0)
    b = dyn.run(m, st0.copy(), 50.0, 100, 3, 0)
    assert np.array_equal(a[0].C, b[0].C) and np.array_equal(a[0].x, b[0].x)
    assert [e["step"] for e in a[1]] == [e["step"] for e in b[1]]


def test_fermi_occupations_follow_canonical_distribution():
    """Accepted draws of the fixed-N Fermi sampler are distributed as
    P(s) ~ prod_{a in s} exp(-lambda_a / kT) (exact enumeration, tiny n)."""
    lam = np.array([-0.02, -0.006, -0.001, 0.002, 0.007, 0.015])
    kT, N = 0.006, 3
    counts = {}
    n_draw = 4000
    for t in range(n_draw):
        s, used = dyn.fermi_occupations(lam, N, kT, seed=77, traj=t)
        assert used >= 1
        counts[tuple(s)] = counts.get(tuple(s), 0) + 1
    configs = list(itertools.combinations(range(6), N))
    wts = np.array([math.exp(-sum(lam[list(c)]) / kT) for c in configs])
    p = wts / wts.sum()
    obs = np.array([counts.get(c, 0) for c in configs]) / n_draw
    # chi-square style bound, generous: 4 sigma per cell
    sig = np.sqrt(p * (1 - p) / n_draw)
    assert np.all(np.abs(obs - p) < 4 * sig + 1e-3)


def test_zero_temperature_occupations_are_lowest():
    lam = np.linspace(-1, 1, 9)
    s, used = dyn.fermi_occupations(lam, 4, 0.0, seed=0, traj=0)
    assert list(s) == [0, 1, 2, 3] and used == 0


def test_observables_consistency():
    cfg, m = _c1_like(M=10, N=5)
    st = dyn.initial_state(m, 2.0, 0.001, 5, 0.0, 0, 0)
    ob = dyn.observables(m, st)
    # with unit-vector orbitals the two impurity estimators coincide
    assert abs(ob["Pd_surf"] - ob["Pd_wf"]) < 1e-15
    assert ob["ortho"] < 1e-15


def _substep_case():
    from oracle import models
    from workloads import get_config
    from workloads.sampling import random_orbitals
    cfg = get_config("c1")
    m = models.from_config(cfg, M=12)
    C = random_orbitals(m.n, 6, seed=2)
    st = dyn.State([3.0], [0.004], C, np.arange(6))
    return m, st, cfg["dt"]


def test_substeps_are_exact_for_frozen_nuclei():
    """v = 0 and no force: A is constant, so S sub-steps of dt/S reproduce
    the single step to rounding."""
    m, st, dt = _substep_case()
    st0 = dyn.State(st.x, [0.0], st.C, st.s)
    F0 = np.zeros(1)
    one, _, _ = dyn.step(m, st0, dt, 0.999, F0.copy(), substeps=1)
    five, _, _ = dyn.step(m, st0, dt, 0.999, F0.copy(), substeps=5)
    assert np.max(np.abs(one.C - five.C)) < 1e-13


def test_substeps_converge_at_second_order():
    """Moving nuclei: the sub-stepped orbitals converge to the time-ordered
    propagation along the drift with error ~ 1/S^2 (midpoint rule)."""
    m, st, dt = _substep_case()
    ref, _, _ = dyn.step(m, st, 4 * dt, 0.999, None, substeps=256)
    err = []
    for S in (4, 8, 16):
        out, _, _ = dyn.step(m, st, 4 * dt, 0.999, None, substeps=S)
        err.append(np.max(np.abs(out.C - ref.C)))
    assert err[0] > 1e-9
    for a, b in zip(err, err[1:]):
        assert 3.2 < a / b < 4.8, err
