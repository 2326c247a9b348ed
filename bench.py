#!/usr/bin/env python
"""Throughput of the IESH ensemble step on one MI355X.

Workload: plain IESH on the double-well Newns-Anderson model with M = 200
bath levels (n = 201 one-electron states) and N = 100 electrons, 4096
trajectories, dt = 20 a.u., Boltzmann-sampled positions and velocities and
Fermi-sampled occupations (synthetic inputs, seed 0).  One step is the
whole per-timestep update of every trajectory.  The timed steps follow a
warm-up of 1000 steps by default: from a thermal start the orbitals are
still unit vectors and the exact no-hop bound skips nearly every
determinant-ratio evaluation, so early steps are cheaper than the steady
state.  The 100 timed steps span one period of the Loewdin correction of
the mixed path.

Both precisions are timed: the mixed path (FP32 MFMA propagation, FP64
eigen-solve / overlap inverse / rescaling, FP64 Loewdin every 100 steps)
gives the headline value; the FP64 path is reported beside it with the
deviation of the mixed path from it.  The JSON line also carries the
roofline of the dominant kernel (the orbital propagation) and the CPU
oracle timed on the host cores on a bounded sample of the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"fp64": 78.6, "mixed": 157.3}  # MI355X dense MFMA FP64 / FP32
HBM_PEAK_GBS = 8000.0
STEADY_WARMUP, STEADY_STEPS = 1000, 100


def algorithmic_prop_flops(n, N, sum_terms):
    # K applications of the real n x n coupling matrix to [Re C | Im C]
    # (n x 2N) per trajectory-step: 2 * n * n * 2N flops each.
    return 4.0 * n * n * N * sum_terms


def traffic_from_profile(path_md, kernel_src):
    """HBM bytes per launch from a committed counter summary, if it was taken
    on the current kernel source."""
    if not os.path.exists(path_md):
        return None
    text = open(path_md).read()
    m = re.search(r"```json\n(.*?)\n```", text, re.S)
    if not m:
        return None
    d = json.loads(m.group(1))
    sha = hashlib.sha256(open(kernel_src, "rb").read()).hexdigest()
    if d.get("kernel_source_sha256") != sha:
        return None
    return d.get("hbm_bytes_per_launch")


def time_path(cfg, precision, T, steps, warmup, x0, v0, substeps=1, keep_sample=0, lowdin_every=100,
              **run_options):
    import torch
    from paper_2212_00518_amd import from_config

    ens = from_config(cfg, n_traj=T, precision=precision, lowdin_every=lowdin_every,
                      elec_substeps=substeps, **run_options)
    ens.init_thermal(x0, v0)
    ens.run(warmup)
    ens.sync()
    ens.timing(True)  # per-kernel HIP events; clears the work counters
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ens.run(steps)
    ens.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tm = ens.timing_read()
    sum_terms, traj_steps = ens.work()
    hop_evals = ens.hop_evals()
    status = ens.status()
    clock_time, _ = ens.clock()
    ens.timing(False)
    defect = ens.defect_max() if precision == "mixed" else None
    sample = state_sample(ens, cfg, keep_sample) if keep_sample else None
    ens.close()
    n, N = cfg["bath"]["M"] + 1, cfg["n_elec"]
    flops = algorithmic_prop_flops(n, N, sum_terms)
    prop_ms, prop_launches = tm["prop"]
    return dict(
        wall_s=wall, traj_steps=traj_steps, value=traj_steps / wall, ms_per_step=1e3 * wall / steps,
        kernels_ms={k: round(v[0] / max(v[1], 1), 4) for k, v in tm.items() if v[1]},
        kernels_share={k: round(v[0] / (1e3 * wall), 4) for k, v in tm.items() if v[1]},
        prop_flops_per_launch=flops / max(prop_launches, 1),
        prop_ms_per_launch=prop_ms / max(prop_launches, 1),
        prop_tflops=flops / (prop_ms * 1e-3) / 1e12 if prop_ms > 0 else 0.0,
        mean_cheb_terms=sum_terms / max(traj_steps, 1),
        exact_hop_fraction=hop_evals / max(traj_steps, 1),
        frozen=int((status != 0).sum()),
        mean_dt=float(clock_time.sum()) / max(warmup + steps, 1) / T,
        lowdin_launches=tm["lowdin"][1],
        lowdin_steps_in_window=sum(1 for k in range(warmup, warmup + steps) if (k + 1) % lowdin_every == 0)
        if precision == "mixed" and lowdin_every > 0 else 0,
        max_orthonormality_defect=defect,
        sample=sample,
    )


def state_sample(ens, cfg, count):
    """States of `count` trajectories taken from a running ensemble: the most
    mixed half (largest orbital weight outside the occupied set, where the
    exact determinant ratios run) and an evenly spaced half."""
    import numpy as np
    from paper_2212_00518_amd import unpack_C
    x, v, Cf, occ = ens.get_state()
    T, N, n = len(x), cfg["n_elec"], cfg["bath"]["M"] + 1
    C3 = Cf.reshape(T, ens.N_max, ens.n_max)[:, :N, :n]
    w_occ = np.take_along_axis(np.sum(np.abs(C3) ** 2, axis=1), occ[:, :N].astype(np.int64), axis=1)
    mixing = N - np.sum(w_occ, axis=1)
    picks = list(np.argsort(mixing)[::-1][: count // 2])
    for t in np.linspace(0, T - 1, count - len(picks)).astype(int):
        if t not in picks:
            picks.append(int(t))
    step = ens.get_step()
    return dict(step=step, traj=[int(t) for t in picks],
                states=[(float(x[t]), float(v[t]), unpack_C(Cf, t, n, N, ens.n_max, ens.N_max),
                         occ[t, :N].copy()) for t in picks])


def error_vs_oracle(cfg, sample, precision, steps=20):
    """Error of a GPU path against the FP64 oracle from the same inputs: the
    sampled steady-state states are uploaded into a small ensemble, which
    runs `steps` steps (from the sample's step, so the hop uniforms are those
    of the running ensemble's step count); the oracle runs the same steps
    from the same states.  Reports, over the trajectories whose hop events
    agree (decisions within the near-tie window excluded), the largest
    deviation of the hop probabilities (iesh_hop_probs at the end, relative to
    the trajectory's largest), of the impurity population P_d^wf (every
    step), of the orbitals and of the total energy (relative)."""
    import numpy as np
    from oracle import models, dynamics as dyn
    from paper_2212_00518_amd import from_config, pack_states, unpack_C

    m = models.from_config(cfg)
    N, n = cfg["n_elec"], cfg["bath"]["M"] + 1
    states = sample["states"]
    T = len(states)
    ens = from_config(cfg, n_traj=T, precision=precision, lowdin_every=100, record_every=1)
    ens.set_state(*pack_states(states, ens.n_max, ens.N_max))
    ens.set_step(sample["step"])
    obs = ens.run(steps, record=True)
    _, _, Cf, _ = ens.get_state()
    g = ens.hop_probs()
    evs, _ = ens.events()
    n_max, N_max = ens.n_max, ens.N_max
    ens.close()
    tie = 1e-7 if precision == "fp64" else 1e-4
    out = dict(trajectories=T, steps=steps, from_step=sample["step"], compared=0, near_tie_excluded=0,
               max_rel_dg=0.0, max_abs_dPd_wf=0.0, max_abs_dC=0.0, max_rel_dEtot=0.0, hops=0)
    for t, (x, v, C, occ) in enumerate(states):
        st = dyn.State([x], [v], C, occ)
        ref, ref_ev, recs = dyn.run(m, st, cfg["dt"], steps, cfg["seed"], t, step0=sample["step"],
                                    record_every=1)
        if any(e["margin"] < tie * max(e["g_total"], 1e-300) for e in ref_ev):
            out["near_tie_excluded"] += 1
            continue
        mine = [(e["step"], e["a"], e["b"], e["accepted"]) for e in evs if e["traj"] == t]
        if mine != [(e["step"], e["a"], e["b"], e["accepted"]) for e in ref_ev]:
            out.setdefault("event_mismatch", []).append(t)
            continue
        out["compared"] += 1
        out["hops"] += sum(e["accepted"] for e in ref_ev)
        gref = dyn.hop_probs(m, ref, cfg["dt"])
        gt = g[t, : N * n].reshape(N, n)
        out["max_rel_dg"] = max(out["max_rel_dg"], float(np.max(np.abs(gt - gref)) / max(np.max(gref), 1e-300)))
        out["max_abs_dPd_wf"] = max(out["max_abs_dPd_wf"],
                                    max(abs(obs[q, t, 1] - r["Pd_wf"]) for q, r in enumerate(recs)))
        out["max_rel_dEtot"] = max(out["max_rel_dEtot"],
                                   max(abs(obs[q, t, 4] - r["Etot"]) / abs(r["Etot"]) for q, r in enumerate(recs)))
        out["max_abs_dC"] = max(out["max_abs_dC"],
                                float(np.max(np.abs(unpack_C(Cf, t, n, N, n_max, N_max) - ref.C))))
    return out


def _oracle_run_worker(args):
    """One FP64 oracle trajectory from a sampled state (pool worker)."""
    cfg_name, x, v, C, occ, steps, step0, t = args
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):
        from oracle import models, dynamics as dyn
        from workloads import get_config
        cfg = get_config(cfg_name)
        m = models.from_config(cfg)
        ref, ev, recs = dyn.run(m, dyn.State([x], [v], C, occ), cfg["dt"], steps, cfg["seed"], t,
                                step0=step0, record_every=1)
        return ([(e["step"], e["a"], e["b"], e["accepted"]) for e in ev],
                min([e["margin"] / max(e["g_total"], 1e-300) for e in ev], default=1.0),
                [r["Pd_wf"] for r in recs], dyn.hop_probs(m, ref, cfg["dt"]))


def lowdin_sweep(a, periods=(25, 50, 100, 200, 400), n_sample=8, steps=800):
    """Mixed path against the Loewdin period L: throughput of the full
    workload (4096 trajectories, L in the timed window) and the error against
    the FP64 oracle of n_sample steady-state trajectories run for `steps`
    steps (at least two Loewdin steps for every L) from the same states: the
    largest |dP_d^wf| over the steps, the largest hop-probability deviation at
    the end (relative to the trajectory's largest), and the largest
    orthonormality defect the Loewdin steps measured."""
    import multiprocessing as mp
    import numpy as np
    from paper_2212_00518_amd import from_config, pack_states
    from workloads import get_config
    cfg = get_config("c2")
    T = cfg["n_traj"]
    N, n = cfg["n_elec"], cfg["bath"]["M"] + 1
    x0, v0 = initial_sample(cfg, T, cfg["seed"])
    pre = time_path(cfg, "mixed", T, 50, 1000, x0, v0, keep_sample=n_sample)
    sample = pre["sample"]
    print(f"# pre-roll done: step {sample['step']}, {len(sample['traj'])} sampled trajectories", flush=True)
    os.environ["OMP_NUM_THREADS"] = "1"
    ctx = mp.get_context("spawn")
    with ctx.Pool(min(16, n_sample)) as pool:
        refs = pool.map(_oracle_run_worker,
                        [("c2", x, v, C, occ, steps, sample["step"], t)
                         for t, (x, v, C, occ) in enumerate(sample["states"])])
    print(f"# oracle runs done ({n_sample} x {steps} steps)", flush=True)
    rows = []
    for L in periods:
        tp = time_path(cfg, "mixed", T, max(100, 2 * L), 1000, x0, v0, lowdin_every=L)
        ens = from_config(cfg, n_traj=n_sample, precision="mixed", lowdin_every=L, record_every=1)
        ens.set_state(*pack_states(sample["states"], ens.n_max, ens.N_max))
        ens.set_step(sample["step"])
        obs = ens.run(steps, record=True)
        g = ens.hop_probs()
        evs, _ = ens.events()
        defect = ens.defect_max()
        ens.close()
        d_pd = d_g = 0.0
        compared = 0
        for t, (ev_ref, rel_margin, pd_ref, g_ref) in enumerate(refs):
            mine = [(e["step"], e["a"], e["b"], e["accepted"]) for e in evs if e["traj"] == t]
            if rel_margin < 1e-4 or mine != ev_ref:
                continue
            compared += 1
            d_pd = max(d_pd, float(np.max(np.abs(obs[:, t, 1] - np.asarray(pd_ref)))))
            gt = g[t, : N * n].reshape(N, n)
            d_g = max(d_g, float(np.max(np.abs(gt - g_ref)) / max(np.max(g_ref), 1e-300)))
        row = dict(L=L, value=round(tp["value"], 1), ms_per_step=round(tp["ms_per_step"], 3),
                   lowdin_ms_per_launch=tp["kernels_ms"].get("lowdin"),
                   lowdin_steps_in_window=tp["lowdin_steps_in_window"],
                   compared=compared, max_abs_dPd_wf=d_pd, max_rel_dg_end=d_g,
                   max_orthonormality_defect=defect)
        rows.append(row)
        print(f"# L={L}: {row}", flush=True)
    print(json.dumps(dict(metric="mixed path against the Loewdin period", config="c2",
                          sample_trajectories=n_sample, steps=steps, from_step=sample["step"],
                          sweep=rows)), flush=True)


def mixed_vs_fp64(cfg, T=64, steps=500):
    """Deviation of the mixed path from the FP64 path on the same inputs."""
    import numpy as np
    from paper_2212_00518_amd import from_config
    from workloads import boltzmann_harmonic

    x0, v0 = boltzmann_harmonic(T, cfg["model"]["mass"], cfg["model"]["omega"], cfg["kT"],
                                seed=cfg["seed"] + 1)
    out = {}
    for prec in ("fp64", "mixed"):
        ens = from_config(cfg, n_traj=T, precision=prec, lowdin_every=100, record_every=steps // 10)
        ens.init_thermal(x0, v0)
        obs = ens.run(steps, record=True)
        evs, _ = ens.events(cap=1 << 18)
        out[prec] = (obs, evs)
        ens.close()
    o64, om = out["fp64"][0], out["mixed"][0]
    ev64 = {}
    for e in out["fp64"][1]:
        ev64.setdefault(e["traj"], []).append((e["step"], e["a"], e["b"], e["accepted"]))
    evm = {}
    for e in out["mixed"][1]:
        evm.setdefault(e["traj"], []).append((e["step"], e["a"], e["b"], e["accepted"]))
    same = sum(1 for t in range(T) if ev64.get(t, []) == evm.get(t, []))
    e0 = o64[0, :, 4]
    return dict(
        trajectories=T, steps=steps,
        max_abs_dPd_wf=float(np.max(np.abs(om[:, :, 1] - o64[:, :, 1]))),
        max_abs_dPd_surf=float(np.max(np.abs(om[:, :, 0] - o64[:, :, 0]))),
        max_rel_dEtot=float(np.max(np.abs(om[:, :, 4] - o64[:, :, 4]) / np.abs(o64[:, :, 4]))),
        fp64_Etot_drift_rel=float(np.max(np.abs(o64[-1, :, 4] - e0) / np.abs(e0))),
        mixed_Etot_drift_rel=float(np.max(np.abs(om[-1, :, 4] - om[0, :, 4]) / np.abs(om[0, :, 4]))),
        identical_event_sequences=same,
        ensemble_mean_dPd_wf=float(abs(om[-1, :, 1].mean() - o64[-1, :, 1].mean())),
    )


def initial_sample(cfg, T, seed):
    """Boltzmann positions and velocities of a workload: the harmonic U0 of
    the double-well models, or every coordinate of the multi-coordinate model
    about its Morse minimum r with the well's harmonic frequency
    a sqrt(2 D / m)."""
    import numpy as np
    from workloads import boltzmann_harmonic
    from workloads.sampling import boltzmann_coordinates
    m = cfg["model"]
    if m["kind"] == "multi_dof":
        dof = np.array(m["dof"])
        om = dof[:, 2] * np.sqrt(2.0 * dof[:, 1] / dof[:, 0])
        return boltzmann_coordinates(T, dof[:, 0], om, dof[:, 3], cfg["kT"], seed=seed)
    return boltzmann_harmonic(T, m["mass"], m["omega"], cfg["kT"], seed=seed,
                              kT_factor=cfg.get("sample_kT_factor", 1.0))


def _cpu_worker(args):
    cfg_name, t, steps = args
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):
        from oracle import models, dynamics as dyn, rng
        from workloads import get_config
        cfg = get_config(cfg_name)
        m = models.from_config(cfg)
        x0, v0 = initial_sample(cfg, t + 1, cfg["seed"])
        st = dyn.initial_state(m, x0[t], v0[t], cfg["n_elec"], cfg["kT"], cfg["seed"], t,
                               bias=cfg["bath"].get("bias", 0.0))
        F = None
        t0 = time.perf_counter()
        for k in range(steps):
            st, _, F = dyn.step(m, st, cfg["dt"], rng.uniform(cfg["seed"], t, k), F)
        return time.perf_counter() - t0


def cpu_baseline(cfg_name, steps_per_worker):
    import multiprocessing as mp
    workers = min(16, os.cpu_count() or 1)
    os.environ["OMP_NUM_THREADS"] = "1"
    os.environ["OPENBLAS_NUM_THREADS"] = "1"
    os.environ["MKL_NUM_THREADS"] = "1"
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(workers) as pool:
        per = pool.map(_cpu_worker, [(cfg_name, t, steps_per_worker) for t in range(workers)])
    wall = time.perf_counter() - t0
    total = workers * steps_per_worker
    return dict(value=total / wall, unit="trajectory-steps/s", cores=workers, kind="oracle",
                cpu_model=cpu_model(),
                sample=f"{workers} trajectories x {steps_per_worker} steps of the same workload, "
                       f"one process per trajectory, one BLAS thread each",
                one_core_s_per_traj_step=sum(per) / total, wall_s=wall)


def cpu_model():
    """CPU model name of the host (from /proc/cpuinfo) and its logical CPU count."""
    name = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    name = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return f"{name} ({os.cpu_count()} logical CPUs on the host)"


def scattering_run(steps, forced_lifetimes, n_traj=None, timed_steps=50, report_progress=True):
    """Uneven batched scattering workload (bath classes M = 40, 80, 160, 320,
    N = M/2, mixed path, compaction every 100 steps on the device): useful
    (active) trajectory-steps/s over `steps` graph-replayed steps, then a
    window of `timed_steps` steps with per-kernel HIP events for the
    propagation roofline (flops from the per-class Chebyshev sums)."""
    import numpy as np
    import torch
    from paper_2212_00518_amd import _lib
    from workloads import get_config
    from workloads.sampling import bath_classes, scattering_initial

    cfg = get_config("c3")
    T = n_traj or cfg["n_traj"]
    classes = cfg["bath"]["M_classes"]
    cls = bath_classes(T, classes, seed=cfg["seed"])
    descs = []
    for M in classes:
        eps, w = _lib.discretize(cfg["bath"]["kind"], M, cfg["bath"]["W"])
        descs.append(_lib.model_desc(cfg["model"], eps, w, M // 2))
    x0, v0, e_inc = scattering_initial(T, cfg["model"]["mass"], cfg["x_start"], cfg["E_inc"],
                                       seed=cfg["seed"] + 1)
    chunk = 100
    run = dict(n_traj=T, precision="mixed", dt=cfg["dt"], kT=0.0, seed=cfg["seed"],
               lowdin_every=100, exit_enabled=1, exit_x=cfg["exit_x"],
               max_steps=cfg["max_steps"], compact_every=chunk)
    t_create = time.perf_counter()
    ens = _lib.Ensemble(descs, run, traj_model=cls)
    t_create = time.perf_counter() - t_create
    ens.init_thermal(x0, v0)
    if forced_lifetimes:
        rng = np.random.default_rng(cfg["seed"] + 2)
        caps = np.exp(rng.uniform(np.log(200.0), np.log(20000.0), size=T)).astype(np.int64)
        ens.set_step_caps(caps)
    info0 = [ens.class_info(k) for k in range(len(classes))]
    ens.timing(True)  # clears the work counters; the steps below replay graphs
    ens.timing(False)
    visited = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        k = min(chunk, steps - done)
        live = sum(ens.class_info(c)["live"] for c in range(len(classes)))
        visited += live * k
        ens.run(k)
        done += k
        if report_progress:
            print(f"# step {done}: live slots {live}", file=sys.stderr, flush=True)
    ens.sync()
    wall = time.perf_counter() - t0
    _, traj_steps = ens.work()
    # propagation roofline over a short window with HIP events on every launch
    ens.timing(True)
    ens.run(timed_steps)
    tm = ens.timing_read()
    flops = 0.0
    for k, M in enumerate(classes):
        kt, _ = ens.class_work(k)
        flops += algorithmic_prop_flops(M + 1, M // 2, kt)
    ens.timing(False)
    status = ens.status()
    info1 = [ens.class_info(k) for k in range(len(classes))]
    _, v_end, _, _ = ens.get_state()
    ens.close()
    prop_ms = tm["prop"][0]
    achieved = flops / (prop_ms * 1e-3) / 1e12 if prop_ms > 0 else 0.0
    return dict(cfg=cfg, T=T, classes=classes, wall=wall, traj_steps=traj_steps, visited=visited,
                status=status, info0=info0, info1=info1, v_end=v_end, e_inc=e_inc, t_create=t_create,
                roofline={"bound": "mfma", "kernel": "k_prop (all classes)", "achieved": round(achieved, 3),
                          "peak": PEAK_TFLOPS["mixed"], "unit": "TFLOP/s",
                          "frac": round(achieved / PEAK_TFLOPS["mixed"], 4), "traffic": None,
                          "window_steps": timed_steps,
                          "prop_ms_per_step": round(prop_ms / timed_steps, 4)},
                kernels_ms_per_step={k: round(v[0] / timed_steps, 4) for k, v in tm.items() if v[1]})


def scattering_bench(a):
    """Uneven batched scattering workload: useful (active) trajectory-steps/s
    with compaction every 100 steps."""
    import numpy as np
    from paper_2212_00518_amd import _lib

    r = scattering_run(a.steps, a.forced_lifetimes, a.n_traj)
    cfg, classes, status, v_end, e_inc = r["cfg"], r["classes"], r["status"], r["v_end"], r["e_inc"]
    # kinetic-energy loss of the trajectories that rebounded past the exit
    # distance: 1 - E_kin(final) / E_inc, by incidence energy (Sec. III.D)
    out = (status & _lib.TRAJ_EXITED) > 0
    loss = 1.0 - 0.5 * cfg["model"]["mass"] * v_end ** 2 / e_inc
    edges = np.linspace(cfg["E_inc"][0], cfg["E_inc"][1], 6)
    ke_loss = []
    for lo, hi in zip(edges[:-1], edges[1:]):
        sel = out & (e_inc >= lo) & (e_inc < hi)
        ke_loss.append({"E_inc_eV": [round(lo * 27.211386, 3), round(hi * 27.211386, 3)],
                        "rebounded": int(sel.sum()),
                        "mean_ke_loss": round(float(loss[sel].mean()), 4) if sel.any() else None})
    line = {
        "metric": "useful trajectory-steps/s (scattering, uneven M, compaction every 100 steps)",
        "value": round(r["traj_steps"] / r["wall"], 2),
        "unit": "trajectory-steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": 0,
        "ms_per_step": round(1e3 * r["wall"] / a.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": cfg["name"], "M_classes": classes, "n_traj": r["T"], "dt": cfg["dt"],
                   "forced_lifetimes": bool(a.forced_lifetimes), "path": "mixed"},
        "roofline": r["roofline"],
        "kernels_ms_per_step": r["kernels_ms_per_step"],
        "active_trajectory_steps": int(r["traj_steps"]),
        "visited_slot_steps": int(r["visited"]),
        "compaction_efficiency": round(r["traj_steps"] / max(r["visited"], 1), 4),
        "frozen_at_end": int((status != 0).sum()),
        "tiles_per_group": {str(M): i["tiles_per_group"] for M, i in zip(classes, r["info0"])},
        "live_slots_at_end": {str(M): i["live"] for M, i in zip(classes, r["info1"])},
        "trajectories_per_class": {str(M): i["n_traj"] for M, i in zip(classes, r["info0"])},
        "context_creation_s": round(r["t_create"], 2),
        "kinetic_energy_loss": ke_loss,
    }
    print(json.dumps(line), flush=True)


def desorption_run(cfg, T, steps):
    """One desorption ensemble: (trajectory-steps, wall s, P_total every 100
    steps, tiles per propagation work-group)."""
    import numpy as np
    import torch
    from paper_2212_00518_amd import _lib, bath_levels
    from workloads.sampling import wigner_harmonic

    m, b = cfg["model"], cfg["bath"]
    # the electrons fill the bath states below mu (half of them when the band follows mu)
    eps, w, _, n_elec = bath_levels(b, b["M"])
    desc = _lib.model_desc(m, eps, w, n_elec)
    omega = m["a"] * np.sqrt(2.0 * m["De"] / m["mass"])  # harmonic frequency of the Morse U0
    x0, v0 = wigner_harmonic(T, m["mass"], omega, m["x0"], cfg["kT"], seed=cfg["seed"] + 1)
    chunk = 100
    run = dict(n_traj=T, precision="mixed", dt=cfg["dt"], kT=cfg["kT"], seed=cfg["seed"],
               lowdin_every=100, exit_enabled=1, exit_x=cfg["x_threshold"], compact_every=chunk)
    ens = _lib.Ensemble([desc], run)
    ens.init_thermal(x0, v0)
    ens.timing(True)
    ens.timing(False)
    p_total = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        k = min(chunk, steps - done)
        ens.run(k)
        done += k
        p_total.append(round(float(np.mean((ens.status() & _lib.TRAJ_EXITED) > 0)), 6))
        print(f"# mu {b.get('mu', 0.0):+.5f} step {done}: P_total {p_total[-1]}", file=sys.stderr,
              flush=True)
    ens.sync()
    wall = time.perf_counter() - t0
    _, traj_steps = ens.work()
    info = ens.class_info(0)
    ens.close()
    return traj_steps, wall, p_total, info["tiles_per_group"], n_elec


def desorption_bench(a):
    """Desorption workload (Sec. III.C): Table et-parameters, Gauss-Legendre
    bath of 100 states over 64 eV, 300 K Fermi occupations, a harmonic Wigner
    sample of the Morse well; P_total(t) is the fraction of trajectories past
    5 Angstrom (frozen on crossing, compaction every 100 steps).  The band
    follows the chemical potential mu (its centre and the Gauss-Legendre split
    sit at mu) and the electrons fill the bath states below it; --mu-sweep
    runs mu = -0.5, 0, +0.5 eV."""
    from workloads import get_config
    from workloads.configs import ev

    cfg = get_config("desorption")
    T = a.n_traj or cfg["n_traj"]
    steps = a.steps if a.steps != 100 else cfg["n_steps"]
    mus = (-0.5, 0.0, 0.5) if a.mu_sweep else (a.mu,)
    total_steps, total_wall, sweep = 0, 0.0, {}
    for mu in mus:
        c = get_config("desorption")
        c["bath"]["mu"] = ev(mu)
        ts, wall, p_total, tiles, n_elec = desorption_run(c, T, steps)
        total_steps += ts
        total_wall += wall
        sweep[f"{mu:+.2f} eV"] = {"p_total_every_100_steps": p_total, "n_elec": n_elec,
                                  "trajectory_steps_per_s": round(ts / wall, 1)}
    b = cfg["bath"]
    m = cfg["model"]
    line = {
        "metric": "trajectory-steps/s (desorption, P_total(t) with x_threshold = 5 Angstrom)",
        "value": round(total_steps / total_wall, 2),
        "unit": "trajectory-steps/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": 0,
        "ms_per_step": round(1e3 * total_wall / (steps * len(mus)), 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": cfg["name"], "M": b["M"], "n_traj": T, "dt": cfg["dt"],
                   "kT": cfg["kT"], "Gamma": m["Gamma"], "path": "mixed",
                   "mu_eV": list(mus), "band": "centred on mu, Gauss-Legendre split at mu"},
        "by_mu": sweep,
        "tiles_per_group": tiles,
    }
    print(json.dumps(line), flush=True)


def two_lead_bench(a):
    """Biased two-lead junction with six nuclear coordinates (two leads of 128
    levels on one grid, n = 257, N = 128, 8192 trajectories, mixed path):
    trajectory-steps/s at each bias V, with the roofline of the propagation
    and the share of the eigen-solve kernel, which carries the six-coordinate
    projection."""
    from workloads import get_config

    cfg = get_config("c5")
    T = a.n_traj or cfg["n_traj"]
    warmup = a.warmup if a.warmup != 1000 else 300
    biases = cfg["biases"] if a.bias is None else [a.bias]
    x0, v0 = initial_sample(cfg, T, cfg["seed"])
    by_bias, total_steps, total_wall, flops, prop_ms = {}, 0, 0.0, 0.0, 0.0
    for V in biases:
        c = get_config("c5")
        c["bath"]["bias"] = V
        r = time_path(c, "mixed", T, a.steps, warmup, x0, v0, a.substeps)
        print(f"# bias {V}: {r['value']:.1f} trajectory-steps/s, {r['ms_per_step']:.2f} ms/step, "
              f"kernels {r['kernels_ms']} ms, propagation {r['prop_tflops']:.2f} TFLOP/s",
              file=sys.stderr, flush=True)
        total_steps += r["traj_steps"]
        total_wall += r["wall_s"]
        flops += r["prop_flops_per_launch"]
        prop_ms += r["prop_ms_per_launch"]
        by_bias[f"{V:g}"] = {"value": round(r["value"], 2), "ms_per_step": round(r["ms_per_step"], 3),
                             "kernels_ms_per_launch": r["kernels_ms"],
                             "kernels_time_share": r["kernels_share"],
                             "mean_chebyshev_terms": round(r["mean_cheb_terms"], 3),
                             "exact_hop_fraction": round(r["exact_hop_fraction"], 4),
                             "frozen": r["frozen"]}
    achieved = flops / (prop_ms * 1e-3) / 1e12 if prop_ms > 0 else 0.0
    n, N = cfg["bath"]["M"] + 1, cfg["n_elec"]
    line = {
        "metric": "trajectory-steps/s (two leads 2x128, six coordinates, bias sweep)",
        "value": round(total_steps / total_wall, 2),
        "unit": "trajectory-steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": warmup,
        "ms_per_step": round(1e3 * total_wall / (a.steps * len(biases)), 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": cfg["name"], "n": n, "N": N, "n_traj": T, "dt": cfg["dt"],
                   "n_dof": len(cfg["model"]["dof"]), "bias": biases, "path": "mixed",
                   "elec_substeps": a.substeps},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK_TFLOPS["mixed"],
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_TFLOPS["mixed"], 4),
                     "traffic": None, "kernel": "k_prop",
                     "ms_per_launch": round(prop_ms / len(biases), 4)},
        "by_bias": by_bias,
    }
    if not a.no_cpu:
        line["cpu_baseline"] = cpu_baseline("c5", a.cpu_steps)
    print(json.dumps(line), flush=True)


def _cpu_adj_worker(args):
    t, steps = args
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):
        from oracle import adjoint as adj, bath
        from workloads import get_config
        from workloads.sampling import fixed_paths
        cfg = get_config("c4")
        m, b = cfg["model"], cfg["bath"]
        eps, w = bath.discretise(b["kind"], b["M"], b["W"])
        p = adj.Params(m.get("eps_d", 0.0), m["Gamma"], eps, m["omega"], m["g"], m["dG"], w, m["mass"])
        x, _ = fixed_paths(t + 1, steps, cfg["dt"], m["omega"], seed=cfg["seed"])
        t0 = time.perf_counter()
        adj.gradient(p, x[t], cfg["n_elec"], cfg["dt"], (1.0, 1.0, 1.0, 1.0))
        return time.perf_counter() - t0


def adjoint_cpu_baseline(steps_per_worker, n_paths):
    """The oracle's loss and tangent-linear gradient (every parameter
    direction) timed on the host cores: one path per process."""
    import multiprocessing as mp
    workers = min(16, os.cpu_count() or 1)
    os.environ["OMP_NUM_THREADS"] = "1"
    os.environ["OPENBLAS_NUM_THREADS"] = "1"
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(workers) as pool:
        per = pool.map(_cpu_adj_worker, [(t, steps_per_worker) for t in range(workers)])
    wall = time.perf_counter() - t0
    path_steps = workers * steps_per_worker
    return dict(value=round(1e3 * n_paths * wall / path_steps, 1), unit="ms/step", cores=workers,
                kind="oracle", cpu_model=cpu_model(),
                sample=f"{workers} paths x {steps_per_worker} steps, one process per path, one BLAS "
                       f"thread each; scaled to {n_paths} paths",
                path_steps_per_s=round(path_steps / wall, 3),
                one_core_s_per_path_step=sum(per) / path_steps)


def peak_probe():
    """Library GEMMs (torch.matmul: hipBLASLt / rocBLAS) on square matrices:
    the FP32 and FP64 matrix-core rates this device reaches in practice."""
    import torch
    out = {}
    for dt, name in ((torch.float32, "fp32"), (torch.float64, "fp64")):
        n = 8192
        a = torch.randn(n, n, device="cuda", dtype=dt)
        b = torch.randn(n, n, device="cuda", dtype=dt)
        for _ in range(3):
            torch.matmul(a, b)
        torch.cuda.synchronize()
        reps = 10
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            torch.matmul(a, b)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[name] = {"n": n, "ms": round(ms, 3), "tflops": round(2.0 * n ** 3 / (ms * 1e-3) / 1e12, 2)}
        del a, b
        # the propagation's product: per trajectory B (n_pad x n_pad) times the
        # real orbital block (n_pad x 2N), 4096 trajectories at n = 201, N = 100
        bt, npad, cols = 4096, 208, 200
        a = torch.randn(bt, npad, npad, device="cuda", dtype=dt)
        b = torch.randn(bt, npad, cols, device="cuda", dtype=dt)
        for _ in range(3):
            torch.bmm(a, b)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            torch.bmm(a, b)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[name + "_batched_208x208x200_x4096"] = {
            "ms": round(ms, 3), "tflops": round(2.0 * bt * npad * npad * cols / (ms * 1e-3) / 1e12, 2)}
        del a, b
    # the dense Jacobi eigen-solver on random symmetric matrices: order 96
    # (in LDS) and order 201 (the double-well size, in a device workspace)
    import ctypes
    import numpy as np
    from paper_2212_00518_amd import _lib
    rs = np.random.default_rng(0)
    L = _lib.lib()
    for bt, n in ((4096, 96), (1024, 201)):
        A = rs.normal(size=(bt, n, n))
        dH = torch.from_numpy(0.5 * (A + np.transpose(A, (0, 2, 1)))).cuda()
        del A
        dlam = torch.zeros((bt, n), dtype=torch.float64, device="cuda")
        dQ = torch.zeros((bt, n, n), dtype=torch.float64, device="cuda")
        dsw = torch.zeros(bt, dtype=torch.int32, device="cuda")
        args = (ctypes.c_void_p(dH.data_ptr()), n, bt, ctypes.c_void_p(dlam.data_ptr()),
                ctypes.c_void_p(dQ.data_ptr()), ctypes.c_void_p(dsw.data_ptr()), _lib.IESH_MEM_DEVICE,
                None)
        L.iesh_eigh_batched(*args)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        L.iesh_eigh_batched(*args)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0)
        sweeps = float(dsw.float().mean())
        # 9 m^3 flops per sweep (rows and columns of A and V for m(m-1)/2 rotations)
        out[f"jacobi_eigh_{n}_x{bt}"] = {
            "ms": round(ms, 3), "matrices_per_s": round(bt / (ms * 1e-3), 1),
            "mean_sweeps": round(sweeps, 2),
            "tflops": round(9.0 * n ** 3 * sweeps * bt / (ms * 1e-3) / 1e12, 3)}
        del dH, dlam, dQ, dsw
    print(json.dumps({"gemm_peak_probe": out, "published_peak_tflops": PEAK_TFLOPS}), flush=True)


def adjoint_flops(n, N, sum_terms):
    """Algorithmic flops of one forward + backward adjoint pass: per
    propagated trajectory-step with K terms, the forward propagation, its
    recomputation, the Chebyshev vectors, the adjoint Clenshaw vectors (each
    4 n^2 N K) and the contraction Im sum_k conj(s_k) t_{k-1}^T (4 n^2 N K)."""
    return 5.0 * algorithmic_prop_flops(n, N, sum_terms)


def adjoint_bench(a, cfg=None, n_steps=None, report=True):
    """Adjoint along 1024 prescribed paths (M = 100, N = 50): forward pass
    with checkpoints every 100 steps, then the checkpointed backward pass.
    The loss carries all four terms (population, excitation energy,
    accumulated hop probability, Hellmann-Feynman force), weights 1."""
    import numpy as np
    import torch
    from paper_2212_00518_amd.adjoint import ensemble_for
    from paper_2212_00518_amd import _lib
    from workloads import get_config
    from workloads.sampling import fixed_paths

    cfg = cfg or get_config("c4")
    T = a.n_traj or cfg["n_traj"]
    n_steps = n_steps or cfg["n_steps"]
    m, b = cfg["model"], cfg["bath"]
    M, N = b["M"], cfg["n_elec"]
    eps, w = _lib.discretize(b["kind"], M, b["W"])
    theta = np.concatenate([[m.get("eps_d", 0.0), m["Gamma"]], eps, [m["omega"], m["g"], m["dG"]]])
    x, _ = fixed_paths(T, n_steps, cfg["dt"], m["omega"], seed=cfg["seed"])
    ens = ensemble_for(theta, w, m["mass"], N, T, cfg["dt"])
    # untimed warm-up pass on a short prefix (allocations, code objects)
    terms = (1.0, 1.0, 1.0, 1.0)
    ens.adjoint_forward(x[:, :11], 5, terms)
    ens.adjoint_backward(np.ones(T))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ens.adjoint_forward(x, cfg["ckpt_every"], terms)
    ens.sync()
    t1 = time.perf_counter()
    g = ens.adjoint_backward(np.full(T, 1.0 / T))
    t2 = time.perf_counter()
    fwd, bwd = t1 - t0, t2 - t1
    # per-kernel breakdown on a shorter prefix with HIP events around every launch
    k_steps = min(n_steps, 200)
    ens.timing(True)
    ens.adjoint_forward(x[:, :k_steps + 1], min(cfg["ckpt_every"], k_steps), terms)
    ens.adjoint_backward(np.full(T, 1.0 / T))
    tm = ens.timing_read()
    sum_terms, traj_steps = ens.work()
    ens.timing(False)
    ens.close()
    n = M + 1
    # every propagated trajectory-step is counted three times by the work
    # counter (forward, recompute, reverse sweep): K per pass is sum / 3
    sum_k = sum_terms / 3.0
    flops = adjoint_flops(n, N, sum_k)
    prop_ms = tm["adj_prop"][0] + tm["adj_phi"][0]
    achieved = 0.8 * flops / (tm["adj_prop"][0] * 1e-3) / 1e12 if tm["adj_prop"][0] > 0 else 0.0
    out = {
        "metric": "adjoint ms/step (forward + backward, all paths)",
        "value": round(1e3 * (fwd + bwd) / n_steps, 4),
        "unit": "ms/step",
        "n_gpus": 1,
        "steps": n_steps,
        "warmup": 10,
        "ms_per_step": round(1e3 * (fwd + bwd) / n_steps, 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": cfg["name"], "M": M, "N": N, "n_paths": T, "dt": cfg["dt"],
                   "ckpt_every": cfg["ckpt_every"], "loss_terms": list(terms)},
        "forward_ms_per_step": round(1e3 * fwd / n_steps, 4),
        "backward_ms_per_step": round(1e3 * bwd / n_steps, 4),
        "backward_over_forward": round(bwd / fwd, 3),
        "path_steps_per_s": round(T * n_steps / (fwd + bwd), 1),
        "roofline": {"bound": "mfma", "kernel": "k_prop (forward, recompute, tap modes)",
                     "achieved": round(achieved, 3), "peak": PEAK_TFLOPS["fp64"], "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_TFLOPS["fp64"], 4), "traffic": None,
                     "mean_chebyshev_terms": round(sum_k / max(traj_steps / 3.0, 1), 3)},
        "kernels_ms_per_step": {k: round(v[0] / k_steps, 4) for k, v in tm.items() if v[1]},
        "contraction_tflops": round(0.2 * flops / (tm["adj_phi"][0] * 1e-3) / 1e12, 3)
        if tm["adj_phi"][0] > 0 else None,
        "grad_norm": float(np.linalg.norm(g.sum(axis=0))),
    }
    if report:
        if not getattr(a, "no_cpu", True):
            out["cpu_baseline"] = adjoint_cpu_baseline(10, T)
        print(json.dumps(out), flush=True)
    return out


def small_workload():
    """The small double-well workload in full (M = 20, N = 10, 128
    trajectories, 1000 FP64 steps, dt = 50): throughput of the graph-replayed
    step loop at a size where launch latency, not arithmetic, sets the pace."""
    import torch
    from paper_2212_00518_amd import from_config
    from workloads import get_config
    cfg = get_config("c1")
    T, steps = cfg["n_traj"], cfg["n_steps"]
    x0, v0 = initial_sample(cfg, T, cfg["seed"])
    ens = from_config(cfg, n_traj=T, precision="fp64")
    ens.init_thermal(x0, v0)
    ens.run(10)
    ens.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ens.run(steps)
    ens.sync()
    wall = time.perf_counter() - t0
    ens.close()
    return {"workload": cfg["name"], "path": "fp64", "steps": steps,
            "value": round(T * steps / wall, 1), "unit": "trajectory-steps/s",
            "ms_per_step": round(1e3 * wall / steps, 4)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=1000)
    ap.add_argument("--config", default="c2")
    ap.add_argument("--n-traj", type=int, default=None)
    ap.add_argument("--precision", default="both", choices=["both", "fp64", "mixed"])
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-error", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=300)
    ap.add_argument("--mu", type=float, default=0.0,
                    help="desorption: chemical potential in eV (the band follows it)")
    ap.add_argument("--mu-sweep", action="store_true",
                    help="desorption: mu = -0.5, 0, +0.5 eV")
    ap.add_argument("--bias", type=float, default=None,
                    help="c5: one bias V (default: the sweep 0, 0.01, 0.02)")
    ap.add_argument("--substeps", type=int, default=1,
                    help="electronic sub-steps per nuclear step (default 1)")
    ap.add_argument("--error-steps", type=int, default=500,
                    help="length of the mixed-vs-FP64 comparison (64 trajectories)")
    ap.add_argument("--dt-levels", type=int, default=0,
                    help="adaptive step: halvings allowed (0: fixed step)")
    ap.add_argument("--hop-gmax", type=float, default=0.0,
                    help="adaptive step: bound on the rescaled hop-probability total per step")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the adjoint ms/step entry of the default line")
    ap.add_argument("--no-steady", action="store_true",
                    help="skip the steady-state window (1000-step pre-roll, 100 timed steps)")
    ap.add_argument("--no-scattering", action="store_true",
                    help="skip the 300-step scattering (uneven batching) entry of the default line")
    ap.add_argument("--no-small", action="store_true",
                    help="skip the small-workload (M = 20, 128 trajectories) throughput entry")
    ap.add_argument("--forced-lifetimes", action="store_true",
                    help="c3: per-trajectory step caps log-uniform in [200, 20000]")
    ap.add_argument("--peak-probe", action="store_true",
                    help="only time library FP32 / FP64 GEMMs (8192^3) for the achievable MFMA rate")
    ap.add_argument("--lowdin-sweep", action="store_true",
                    help="mixed path against the Loewdin period L (throughput and error against the oracle)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy three times (the "
                         "reference dispatch for scaling FETCH_SIZE / WRITE_SIZE counters)")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py measures one GPU: --gpus {a.gpus} is not supported (trajectories are "
              f"independent: shard them by trajectory, one process and one context per GPU)", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if a.peak_probe:
        peak_probe()
        return
    if a.lowdin_sweep:
        lowdin_sweep(a)
        return
    if a.copy_calibration:
        x = torch.ones(256 * 1024 * 1024, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_dispatch": x.numel() * 4, "dispatches": 3}))
        return
    if a.config == "c3":
        scattering_bench(a)
        return
    if a.config == "c4":
        adjoint_bench(a)
        return
    if a.config == "desorption":
        desorption_bench(a)
        return
    if a.config == "c5":
        two_lead_bench(a)
        return
    from workloads import get_config

    cfg = get_config(a.config)
    T = a.n_traj or cfg["n_traj"]
    x0, v0 = initial_sample(cfg, T, cfg["seed"])
    precs = ["fp64", "mixed"] if a.precision == "both" else [a.precision]
    steady_window = a.warmup >= STEADY_WARMUP and a.steps >= STEADY_STEPS
    res, steady = {}, {}
    adapt = dict(dt_levels=a.dt_levels, hop_gmax=a.hop_gmax) if a.dt_levels else {}
    for p in precs:
        res[p] = time_path(cfg, p, T, a.steps, a.warmup, x0, v0, a.substeps,
                           keep_sample=8 if steady_window and not a.no_error else 0, **adapt)
        print(f"# {p}: {res[p]['value']:.1f} trajectory-steps/s, {res[p]['ms_per_step']:.2f} ms/step, "
              f"kernels {res[p]['kernels_ms']} ms, propagation {res[p]['prop_tflops']:.2f} TFLOP/s",
              file=sys.stderr, flush=True)
    if not a.no_steady:
        # the steady state: a 1000-step pre-roll (orbitals mixed, the exact
        # ratios needed on a fifth of the trajectory-steps), then a window of
        # 100 steps that holds one Loewdin step of the mixed path
        for p in precs:
            steady[p] = res[p] if steady_window else time_path(
                cfg, p, T, STEADY_STEPS, STEADY_WARMUP, x0, v0, a.substeps,
                keep_sample=0 if a.no_error else 8, **adapt)
            print(f"# steady {p}: {steady[p]['value']:.1f} trajectory-steps/s, "
                  f"{steady[p]['ms_per_step']:.2f} ms/step, kernels {steady[p]['kernels_ms']} ms",
                  file=sys.stderr, flush=True)
    head = "mixed" if "mixed" in res else "fp64"
    r = res[head]
    src = os.path.join(ROOT, "paper_2212_00518_amd", "csrc", "k_prop.hip")
    traffic = traffic_from_profile(os.path.join(ROOT, "profiles", f"k_prop_{head}_{a.config}_traffic.md"), src)
    achieved = r["prop_tflops"]
    line = {
        # the headline metric on the headline workload; any other workload run
        # through this path names itself
        "metric": ("trajectory-steps/s (M=200,N=100) mixed vs FP64 at stated error; adjoint ms/step"
                   if a.config == "c2" else f"trajectory-steps/s ({cfg['name']})"),
        "value": round(r["value"], 2),
        "unit": "trajectory-steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(r["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if head == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": cfg["name"], "M": cfg["bath"]["M"], "N": cfg["n_elec"],
                   "n_traj": T, "dt": cfg["dt"], "bath": cfg["bath"]["kind"], "path": head,
                   "elec_substeps": a.substeps, "dt_levels": a.dt_levels, "hop_gmax": a.hop_gmax},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK_TFLOPS[head],
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_TFLOPS[head], 4),
                     "traffic": traffic, "kernel": "k_prop",
                     "flops_per_launch": r["prop_flops_per_launch"],
                     "ms_per_launch": round(r["prop_ms_per_launch"], 4),
                     "mean_chebyshev_terms": round(r["mean_cheb_terms"], 3)},
        "kernels_ms_per_launch": r["kernels_ms"],
        "kernels_time_share": r["kernels_share"],
        "exact_hop_fraction": round(r["exact_hop_fraction"], 4),
        "mean_dt": round(r["mean_dt"], 4),
    }
    if "fp64" in res and head != "fp64":
        f = res["fp64"]
        line["fp64"] = {"value": round(f["value"], 2), "ms_per_step": round(f["ms_per_step"], 3),
                        "roofline": {"bound": "mfma", "achieved": round(f["prop_tflops"], 3),
                                     "peak": PEAK_TFLOPS["fp64"], "unit": "TFLOP/s",
                                     "frac": round(f["prop_tflops"] / PEAK_TFLOPS["fp64"], 4),
                                     "ms_per_launch": round(f["prop_ms_per_launch"], 4),
                                     "mean_chebyshev_terms": round(f["mean_cheb_terms"], 3)},
                        "kernels_ms_per_launch": f["kernels_ms"],
                        "exact_hop_fraction": round(f["exact_hop_fraction"], 4)}
        line["mixed_over_fp64"] = round(r["value"] / f["value"], 3)
    if steady:
        line["steady_state"] = {}
        for p, r2 in steady.items():
            line["steady_state"][p] = {
                "value": round(r2["value"], 2), "ms_per_step": round(r2["ms_per_step"], 3),
                "warmup": STEADY_WARMUP if not steady_window else a.warmup,
                "steps": STEADY_STEPS if not steady_window else a.steps,
                "roofline_frac": round(r2["prop_tflops"] / PEAK_TFLOPS[p], 4),
                "prop_ms_per_launch": round(r2["prop_ms_per_launch"], 4),
                "kernels_ms_per_launch": r2["kernels_ms"],
                "kernels_time_share": r2["kernels_share"],
                "exact_hop_fraction": round(r2["exact_hop_fraction"], 4),
                "lowdin_steps_in_window": r2["lowdin_steps_in_window"],
                "max_orthonormality_defect": r2["max_orthonormality_defect"]}
    if not a.no_error:
        # error of each path against the FP64 oracle, from steady-state states
        src = steady if steady else (res if steady_window else {})
        for p, r2 in src.items():
            if r2.get("sample"):
                line[f"{p}_error_vs_oracle"] = error_vs_oracle(cfg, r2["sample"], p)
                print(f"# {p} vs oracle: {line[f'{p}_error_vs_oracle']}", file=sys.stderr, flush=True)
    if not a.no_error and "mixed" in res and "fp64" in res:
        line["mixed_vs_fp64_gpu"] = mixed_vs_fp64(cfg, steps=a.error_steps)
    if not a.no_small and a.config == "c2":
        line["small_workload"] = small_workload()
    if not a.no_scattering and a.config == "c2":
        # the batched scattering workload (four bath-size classes, device-side
        # compaction) over a 300-step prefix with forced lifetimes
        sc = scattering_run(300, True, report_progress=False)
        line["scattering"] = {
            "metric": "useful trajectory-steps/s (scattering, M in {40,80,160,320}, 16384 trajectories)",
            "value": round(sc["traj_steps"] / sc["wall"], 2), "unit": "trajectory-steps/s", "steps": 300,
            "ms_per_step": round(1e3 * sc["wall"] / 300, 3),
            "compaction_efficiency": round(sc["traj_steps"] / max(sc["visited"], 1), 4),
            "live_slots_at_end": {str(M): i["live"] for M, i in zip(sc["classes"], sc["info1"])},
            "roofline": sc["roofline"], "kernels_ms_per_step": sc["kernels_ms_per_step"]}
        print(f"# scattering: {line['scattering']['value']:.1f} useful trajectory-steps/s", file=sys.stderr,
              flush=True)
    if not a.no_adjoint:
        # the adjoint workload's ms/step on a 200-step prefix of its paths
        adj = adjoint_bench(argparse.Namespace(n_traj=None), n_steps=200, report=False)
        line["adjoint"] = {k: adj[k] for k in ("metric", "value", "unit", "steps", "config",
                                               "forward_ms_per_step", "backward_ms_per_step",
                                               "kernels_ms_per_step", "roofline")}
    if not a.no_cpu:
        line["cpu_baseline"] = cpu_baseline(a.config, a.cpu_steps)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
