"""Parity at the measured sizes, in the launch configuration the benchmark
times (whole ensembles, autotuned propagation slabs, graph-replayed steps):
a few sampled trajectories against the oracle's own step-by-step run, and
properties that hold for every trajectory (energy conservation over the
steps, orthonormal orbitals, sorted distinct occupations).

Tolerances as in test_gpu_parity: FP64 1e-10 relative for positions and
velocities, 1e-9 absolute for orbital coefficients; mixed 1e-5 and 1e-4.
"""
import numpy as np
import pytest

from oracle import models, dynamics as dyn
from workloads import get_config, boltzmann_harmonic
from workloads.sampling import bath_classes, boltzmann_coordinates, scattering_initial

pytestmark = pytest.mark.gpu

TOL = {"fp64": (1e-10, 1e-9), "mixed": (1e-5, 1e-4)}


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2212_00518_amd import _lib
    _lib.lib()  # fails loudly when the library is missing


def _compare(m, st0, N, steps, dt, seed, t, got, precision, n_max, N_max, bias=0.0):
    """Oracle run of trajectory t from st0 against the GPU's state `got`."""
    from paper_2212_00518_amd import unpack_C
    tx, tc = TOL[precision]
    ref, ref_ev, _ = dyn.run(m, st0, dt, steps, seed, t)
    if any(e["margin"] < 1e3 * tx * max(e["g_total"], 1e-300) for e in ref_ev):
        return False  # a near-tie hop decision: not comparable
    x, v, Cf, occ = got
    xt, vt = np.atleast_1d(x[t]), np.atleast_1d(v[t])
    assert np.max(np.abs(xt - ref.x)) <= tx * max(1.0, np.max(np.abs(ref.x))), t
    assert np.max(np.abs(vt - ref.v)) <= tx * max(1e-3, np.max(np.abs(ref.v))), t
    assert np.max(np.abs(unpack_C(Cf, t, m.n, N, n_max, N_max) - ref.C)) <= tc, t
    assert list(occ[t, :N]) == list(ref.s), t
    return True


def _orthonormal(Cf, ts, n, N, n_max, N_max, tol):
    from paper_2212_00518_amd import unpack_C
    for t in ts:
        C = unpack_C(Cf, t, n, N, n_max, N_max)
        assert np.max(np.abs(C.conj().T @ C - np.eye(N))) <= tol, t


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_double_well_4096_trajectories_m200(precision):
    """The headline workload: M = 200, N = 100, 4096 Boltzmann/Fermi-sampled
    trajectories, five graph-replayed steps."""
    from paper_2212_00518_amd import from_config
    cfg = get_config("c2")
    T, steps, N = cfg["n_traj"], 5, cfg["n_elec"]
    x0, v0 = boltzmann_harmonic(T, cfg["model"]["mass"], cfg["model"]["omega"], cfg["kT"],
                                seed=cfg["seed"], kT_factor=cfg.get("sample_kT_factor", 1.0))
    ens = from_config(cfg, n_traj=T, precision=precision, lowdin_every=100, record_every=1)
    ens.init_thermal(x0, v0)
    obs = ens.run(steps, record=True)
    got = ens.get_state()
    status = ens.status()
    n_max, N_max = ens.n_max, ens.N_max
    ens.close()
    assert np.all(status == 0)
    # every trajectory: energy kept over the steps, occupations sorted and distinct
    e = obs[:, :, 4]
    assert np.max(np.abs(e[-1] - e[0]) / np.abs(e[0])) <= 1e-7
    occ = got[3][:, :N]
    assert np.all(np.diff(occ, axis=1) > 0) and occ.min() >= 0 and occ.max() <= 200
    _orthonormal(got[2], range(0, T, 64), 201, N, n_max, N_max, 1e-12 if precision == "fp64" else 1e-5)
    m = models.from_config(cfg)
    compared = 0
    for t in (0, 1234, 2047, 4095):
        st0 = dyn.initial_state(m, x0[t], v0[t], N, cfg["kT"], cfg["seed"], t)
        compared += _compare(m, st0, N, steps, cfg["dt"], cfg["seed"], t, got, precision, n_max, N_max)
    assert compared >= 3


def test_two_lead_junction_8192_trajectories():
    """Two leads of 128 levels (n = 257, N = 128), bias 0.02, six
    coordinates, 8192 trajectories on the mixed path, three steps; the
    biased initial occupations of the sampled trajectories are the oracle's."""
    from paper_2212_00518_amd import from_config
    cfg = get_config("c5")
    cfg["bath"]["bias"] = 0.02
    T, steps, N = cfg["n_traj"], 3, cfg["n_elec"]
    dof = np.array(cfg["model"]["dof"])
    om = dof[:, 2] * np.sqrt(2.0 * dof[:, 1] / dof[:, 0])
    x0, v0 = boltzmann_coordinates(T, dof[:, 0], om, dof[:, 3], cfg["kT"], seed=cfg["seed"])
    ens = from_config(cfg, n_traj=T, precision="mixed", lowdin_every=100)
    ens.init_thermal(x0, v0)
    init_occ = ens.get_state()[3][:, :N].copy()
    ens.run(steps)
    got = ens.get_state()
    status = ens.status()
    n_max, N_max = ens.n_max, ens.N_max
    ens.close()
    assert np.all(status == 0)
    assert np.all(np.diff(got[3][:, :N], axis=1) > 0)
    _orthonormal(got[2], range(0, T, 512), 257, N, n_max, N_max, 1e-5)
    m = models.from_config(cfg)
    compared = 0
    for t in (0, 4097, 8191):
        st0 = dyn.initial_state(m, x0[t], v0[t], N, cfg["kT"], cfg["seed"], t, bias=0.02)
        assert list(init_occ[t]) == list(st0.s), t
        compared += _compare(m, st0, N, steps, cfg["dt"], cfg["seed"], t, got, "mixed", n_max, N_max)
    assert compared >= 2


def test_scattering_16384_trajectories_in_four_bath_classes():
    """The batched workload as the benchmark runs it: 16384 trajectories in
    the classes M = 40, 80, 160, 320 (N = M/2), mixed path, compaction every
    100 steps, exit at 15 bohr; three steps, two sampled trajectories per
    class against the oracle."""
    from paper_2212_00518_amd import _lib
    cfg = get_config("c3")
    T, steps = cfg["n_traj"], 3
    classes = cfg["bath"]["M_classes"]
    cls = bath_classes(T, classes, seed=cfg["seed"])
    descs = []
    for M in classes:
        eps, w = _lib.discretize(cfg["bath"]["kind"], M, cfg["bath"]["W"])
        descs.append(_lib.model_desc(cfg["model"], eps, w, M // 2))
    x0, v0, _ = scattering_initial(T, cfg["model"]["mass"], cfg["x_start"], cfg["E_inc"],
                                   seed=cfg["seed"] + 1)
    run = dict(n_traj=T, precision="mixed", dt=cfg["dt"], kT=0.0, seed=cfg["seed"],
               lowdin_every=100, exit_enabled=1, exit_x=cfg["exit_x"],
               max_steps=cfg["max_steps"], compact_every=100)
    ens = _lib.Ensemble(descs, run, traj_model=cls)
    ens.init_thermal(x0, v0)
    ens.run(steps)
    got = ens.get_state()
    status = ens.status()
    n_max, N_max = ens.n_max, ens.N_max
    ens.close()
    assert np.all(status == 0)
    compared = 0
    for k, M in enumerate(classes):
        m = models.from_config(cfg, M=M)
        for t in np.flatnonzero(cls == k)[:2]:
            st0 = dyn.initial_state(m, x0[t], v0[t], M // 2, 0.0, cfg["seed"], int(t))
            compared += _compare(m, st0, M // 2, steps, cfg["dt"], cfg["seed"], int(t), got, "mixed",
                                 n_max, N_max)
    assert compared >= 6


@pytest.mark.parametrize("name,T,steps", [("c1", 128, 1000), ("c2", 16, 300)])
def test_double_well_trajectories_against_the_oracle(name, T, steps):
    """Whole trajectories: the small double-well workload in full (128
    Boltzmann/Fermi-sampled trajectories x 1000 graph-replayed FP64 steps)
    and the first 16 trajectories of the M = 200 workload over 300 steps;
    every trajectory against the oracle's own run (one process per trajectory
    on the host cores).  Over hundreds of steps the two propagators' rounding
    drifts apart, so positions, velocities and orbitals are compared at 1e-8."""
    import multiprocessing as mp
    import os
    from paper_2212_00518_amd import from_config, unpack_C
    cfg = get_config(name)
    N = cfg["n_elec"]
    x0, v0 = boltzmann_harmonic(T, cfg["model"]["mass"], cfg["model"]["omega"], cfg["kT"],
                                seed=cfg["seed"], kT_factor=cfg.get("sample_kT_factor", 1.0))
    ens = from_config(cfg, n_traj=T, precision="fp64")
    ens.init_thermal(x0, v0)
    ens.run(steps)
    x, v, Cf, occ = ens.get_state()
    evs, _ = ens.events()
    status = ens.status()
    n_max, N_max = ens.n_max, ens.N_max
    ens.close()
    assert np.all(status == 0)
    m = models.from_config(cfg)
    starts = [dyn.initial_state(m, x0[t], v0[t], N, cfg["kT"], cfg["seed"], t) for t in range(T)]
    saved = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS")}
    os.environ["OMP_NUM_THREADS"] = os.environ["OPENBLAS_NUM_THREADS"] = "1"
    try:
        with mp.get_context("spawn").Pool(min(16, os.cpu_count() or 1)) as pool:
            refs = pool.starmap(dyn.run, [(m, starts[t], cfg["dt"], steps, cfg["seed"], t)
                                          for t in range(T)])
    finally:
        for k, val in saved.items():
            if val is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = val
    compared = 0
    for t, (ref, ref_ev, _) in enumerate(refs):
        if any(e["margin"] < 1e-7 * max(e["g_total"], 1e-300) for e in ref_ev):
            continue
        mine = [e for e in evs if e["traj"] == t]
        assert [(e["step"], e["a"], e["b"], e["accepted"]) for e in mine] == \
               [(e["step"], e["a"], e["b"], e["accepted"]) for e in ref_ev], t
        assert abs(x[t] - ref.x[0]) <= 1e-8 * max(1.0, abs(ref.x[0])), t
        assert abs(v[t] - ref.v[0]) <= 1e-8 * max(1e-3, abs(ref.v[0])), t
        assert np.max(np.abs(unpack_C(Cf, t, m.n, N, n_max, N_max) - ref.C)) <= 1e-8, t
        assert list(occ[t, :N]) == list(ref.s), t
        compared += 1
    print("compared", compared, "of", T, flush=True)
    assert compared >= T - 2


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_steady_state_step_after_1000_steps_m200(precision):
    """The headline workload in its steady state: 4096 trajectories at
    M = 200 pre-rolled for 1000 graph-replayed steps (orbitals mixed, the
    exact determinant ratios needed on a fifth of the trajectory-steps), then
    one more step of the whole ensemble.  From each of the 8 most mixed
    sampled states (largest weight of the orbitals outside the occupied
    set) the oracle takes the same step: positions, velocities, orbitals,
    occupations and hop events must agree, and so must the hop
    probabilities of the new state (iesh_hop_probs, the exact ratios).
    Near-tie windows: 1e-7 (FP64) and 1e-4 (mixed) of the hop total."""
    from oracle import rng
    from paper_2212_00518_amd import from_config, unpack_C
    cfg = get_config("c2")
    T, N, pre = cfg["n_traj"], cfg["n_elec"], 1000
    tx, tc = TOL[precision]
    tie = 1e-7 if precision == "fp64" else 1e-4
    x0, v0 = boltzmann_harmonic(T, cfg["model"]["mass"], cfg["model"]["omega"], cfg["kT"],
                                seed=cfg["seed"], kT_factor=cfg.get("sample_kT_factor", 1.0))
    ens = from_config(cfg, n_traj=T, precision=precision, lowdin_every=100)
    ens.init_thermal(x0, v0)
    ens.run(pre)
    x, v, Cf, occ = ens.get_state()
    n_max, N_max = ens.n_max, ens.N_max
    n = cfg["bath"]["M"] + 1
    # weight of every trajectory's orbitals on its unoccupied states
    C3 = Cf.reshape(T, N_max, n_max)[:, :N, :n]
    w_occ = np.take_along_axis(np.sum(np.abs(C3) ** 2, axis=1), occ[:, :N].astype(np.int64), axis=1)
    mixing = N - np.sum(w_occ, axis=1)
    sample = np.argsort(mixing)[-8:]
    print(f"{precision}: mixing of the sampled states {mixing[sample]}", flush=True)
    ens.clear_events()
    ens.timing(True)
    ens.step()
    full_evals = ens.hop_evals()
    ens.timing(False)
    after = ens.get_state()
    evs, _ = ens.events()
    status = ens.status()
    g = {int(t): ens.hop_probs(int(t), 1)[0] for t in sample}
    ens.close()
    assert np.all(status == 0)
    assert full_evals > 0.05 * T, full_evals  # the exact-ratio kernel runs at its real rate
    m = models.from_config(cfg)
    compared = 0
    for t in map(int, sample):
        st = dyn.State([x[t]], [v[t]], unpack_C(Cf, t, n, N, n_max, N_max), occ[t, :N])
        ref, ev, _ = dyn.step(m, st, cfg["dt"], rng.uniform(cfg["seed"], t, pre))
        gref = dyn.hop_probs(m, ref, cfg["dt"])
        gt = g[t][: N * n].reshape(N, n)
        assert np.max(np.abs(gt - gref)) <= tx * np.max(gref), t
        if ev["attempted"] and ev["margin"] < tie * ev["g_total"]:
            continue
        xa, va, Ca, occa = after
        assert abs(xa[t] - ref.x[0]) <= tx * max(1.0, abs(ref.x[0])), t
        assert abs(va[t] - ref.v[0]) <= tx * max(1e-3, abs(ref.v[0])), t
        assert np.max(np.abs(unpack_C(Ca, t, n, N, n_max, N_max) - ref.C)) <= tc, t
        assert list(occa[t, :N]) == list(ref.s), t
        mine = [(e["a"], e["b"], e["accepted"]) for e in evs if e["traj"] == t]
        assert mine == ([(ev["a"], ev["b"], ev["accepted"])] if ev["attempted"] else []), t
        compared += 1
    assert compared >= 6


def test_scattering_2000_steps_with_exits_and_device_compaction():
    """The batched scattering workload as the benchmark runs it, long enough
    for real exits: 16384 trajectories in the classes M = 40, 80, 160, 320,
    forced lifetimes (step caps log-uniform in [200, 20000]), 2000 steps with
    compaction on the device every 100 steps.  Per class, the trajectory with
    the earliest cap is run by the oracle for its capped length (frozen at the
    cap, then moved behind the active slots), and trajectories that left
    through the exit plane (x > 15 bohr) are checked against the oracle's
    exit step; the live-slot counts equal the trajectories still active."""
    import multiprocessing as mp
    import os
    from paper_2212_00518_amd import _lib, unpack_C
    cfg = get_config("c3")
    T, steps = cfg["n_traj"], 2000
    classes = cfg["bath"]["M_classes"]
    cls = bath_classes(T, classes, seed=cfg["seed"])
    descs = []
    for M in classes:
        eps, w = _lib.discretize(cfg["bath"]["kind"], M, cfg["bath"]["W"])
        descs.append(_lib.model_desc(cfg["model"], eps, w, M // 2))
    x0, v0, _ = scattering_initial(T, cfg["model"]["mass"], cfg["x_start"], cfg["E_inc"],
                                   seed=cfg["seed"] + 1)
    run = dict(n_traj=T, precision="mixed", dt=cfg["dt"], kT=0.0, seed=cfg["seed"],
               lowdin_every=100, exit_enabled=1, exit_x=cfg["exit_x"],
               max_steps=cfg["max_steps"], compact_every=100)
    caps = np.exp(np.random.default_rng(cfg["seed"] + 2).uniform(np.log(200.0), np.log(20000.0),
                                                                   size=T)).astype(np.int64)
    ens = _lib.Ensemble(descs, run, traj_model=cls)
    ens.init_thermal(x0, v0)
    ens.set_step_caps(caps)
    for k in range(steps // 500):
        ens.run(500)
        print(f"step {500 * (k + 1)}: live {[ens.class_info(c)['live'] for c in range(4)]}", flush=True)
    status = ens.status()
    live = [ens.class_info(c)["live"] for c in range(4)]
    clock, _ = ens.clock()
    x, v, Cf, occ = ens.get_state()
    n_max, N_max = ens.n_max, ens.N_max
    ens.close()
    taken = np.rint(clock / cfg["dt"]).astype(np.int64)
    active = [int(np.sum((cls == k) & ((status & 0x1b) == 0))) for k in range(4)]
    assert live == active, (live, active)
    exited = (status & _lib.TRAJ_EXITED) > 0
    capped = (status & _lib.TRAJ_STEPCAP) > 0
    print(f"exited {exited.sum()}, capped {capped.sum()}", flush=True)
    assert capped.sum() > 2000 and exited.sum() > 0
    # oracle runs: the earliest-capped trajectory of every class, and up to two
    # exited trajectories of the two smallest classes
    jobs = []
    for k, M in enumerate(classes):
        members = np.flatnonzero(cls == k)
        t = int(members[np.argmin(caps[members])])
        jobs.append((k, t, int(caps[t])))
        if k < 2:
            for t in np.flatnonzero((cls == k) & exited)[:2]:
                jobs.append((k, int(t), steps))
    models_ = [models.from_config(cfg, M=M) for M in classes]
    starts = [dyn.initial_state(models_[k], x0[t], v0[t], classes[k] // 2, 0.0, cfg["seed"], t)
              for k, t, _ in jobs]
    saved = {q: os.environ.get(q) for q in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS")}
    os.environ["OMP_NUM_THREADS"] = os.environ["OPENBLAS_NUM_THREADS"] = "1"
    try:
        with mp.get_context("spawn").Pool(min(16, len(jobs))) as pool:
            refs = pool.starmap(dyn.run_to_exit, [(models_[k], st, cfg["dt"], n, cfg["seed"], t,
                                                   cfg["exit_x"]) for (k, t, n), st in zip(jobs, starts)])
    finally:
        for q, val in saved.items():
            if val is None:
                os.environ.pop(q, None)
            else:
                os.environ[q] = val
    compared = 0
    for (k, t, n), (ref, n_taken, ref_ev) in zip(jobs, refs):
        M = classes[k]
        print(f"M={M} traj {t}: oracle steps {n_taken}, GPU steps {taken[t]} (cap {caps[t]}), "
              f"exited {bool(exited[t])}", flush=True)
        if any(e["margin"] < 1e-4 * e["g_total"] for e in ref_ev):
            continue            # a near-tie hop decision: not comparable
        assert taken[t] == n_taken, t
        if n == steps:          # left through the exit plane
            assert exited[t] and n_taken < steps, t
        else:                   # frozen at its cap
            assert capped[t] and n_taken == n, t
        assert abs(x[t] - ref.x[0]) <= 1e-6 * max(1.0, abs(ref.x[0])), t
        assert list(occ[t, :M // 2]) == list(ref.s), t
        assert np.max(np.abs(unpack_C(Cf, t, M + 1, M // 2, n_max, N_max) - ref.C)) <= 1e-3, t
        compared += 1
    assert compared >= len(jobs) - 2
