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


def test_hop_probabilities_are_proportional_to_the_step():
    """The premise of the adaptive step: for fixed orbitals, occupations,
    couplings and velocity the hop probabilities scale with dt."""
    from workloads.sampling import random_orbitals
    cfg, m = _c1_like(M=12, N=6)
    rs = np.random.default_rng(2)
    st = dyn.State([3.0], [4e-3], random_orbitals(m.n, 6, seed=5), np.sort(rs.choice(m.n, 6, replace=False)))
    g1 = dyn.hop_probs(m, st, 1.0)
    assert g1.sum() > 0
    for dt in (0.25, 7.0, 50.0):
        assert np.allclose(dyn.hop_probs(m, st, dt), dt * g1, rtol=1e-14, atol=0)


def test_next_dt_rule():
    dt0 = 40.0
    assert dyn.next_dt(0.0, dt0, dt0, 0.05, 3) == dt0
    # the largest dt0 / 2^k whose rescaled total fits
    assert dyn.next_dt(0.08, dt0, dt0, 0.05, 3) == dt0 / 2
    assert dyn.next_dt(0.3, dt0, dt0, 0.05, 3) == dt0 / 8
    assert dyn.next_dt(0.3, dt0, dt0, 0.05, 2) == dt0 / 4     # floor at levels
    # from a reduced step the rule can grow back in one step
    assert dyn.next_dt(0.02, dt0 / 4, dt0, 0.05, 3) == dt0 / 2   # 0.08 at dt0, 0.04 at dt0/2
    assert dyn.next_dt(0.001, dt0 / 4, dt0, 0.05, 3) == dt0
    # monotone in the total
    got = [dyn.next_dt(g, dt0, dt0, 0.05, 5) for g in np.linspace(0.0, 2.0, 41)]
    assert all(a >= b for a, b in zip(got, got[1:]))


def test_adaptive_run_reduces_to_the_fixed_step():
    """A threshold no step reaches keeps dt fixed: the run is the fixed-step
    run bit for bit, and the clock reads n_steps * dt."""
    from workloads.sampling import random_orbitals
    cfg, m = _c1_like(M=12, N=6)
    st0 = dyn.State([2.0], [6e-3], random_orbitals(m.n, 6, seed=9), np.arange(6))
    a, ea, _ = dyn.run(m, st0, cfg["dt"], 25, 0, 3)
    b, eb, _ = dyn.run(m, st0, cfg["dt"], 25, 0, 3, adapt=(1e300, 4))
    assert np.array_equal(a.x, b.x) and np.array_equal(a.v, b.v) and np.array_equal(a.C, b.C)
    assert np.array_equal(a.s, b.s)
    assert [e["b"] for e in ea] == [e["b"] for e in eb]
    assert b.time == 25 * cfg["dt"] and b.dt == cfg["dt"]


def test_adaptive_run_keeps_the_per_step_total_near_the_threshold():
    """With strong mixing the adapted steps are smaller, the clock is the sum
    of the steps taken, and no step after the first exceeds the threshold by
    more than the one-step change of the probabilities (here a factor 3)."""
    from workloads.sampling import random_orbitals
    cfg, m = _c1_like(M=12, N=6)
    st0 = dyn.State([4.0], [1.5e-2], random_orbitals(m.n, 6, seed=11), np.arange(6))
    g_max, levels = 0.02, 4
    steps = []
    F = el.forces(m, st0.x, st0.s)
    st, dt_cur, time = st0, cfg["dt"], 0.0
    for k in range(40):
        st, ev, F = dyn.step(m, st, dt_cur, rng.uniform(0, 1, k), F)
        steps.append((dt_cur, ev["g_total"]))
        time += dt_cur
        dt_cur = dyn.next_dt(ev["g_total"], dt_cur, cfg["dt"], g_max, levels)
    fin, _, _ = dyn.run(m, st0, cfg["dt"], 40, 0, 1, adapt=(g_max, levels))
    assert fin.time == time and np.array_equal(fin.x, st.x)
    assert min(d for d, _ in steps) < cfg["dt"]
    for d, g in steps[1:]:
        assert g <= 3.0 * g_max or d == cfg["dt"] / 2 ** levels
