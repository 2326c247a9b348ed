"""Ensembles from workload descriptions, and state packing helpers."""
from __future__ import annotations

import numpy as np

from . import _lib


def bath_levels(b: dict, M: int):
    """Bath of a workload description from the library (iesh_bath): (eps, w,
    lead, levels below mu).  The band follows the chemical potential mu
    (placement "shift", the default) or keeps [-W/2, W/2] ("split"); with
    ``leads: 2`` the M levels are one grid of M/2 levels shared by two leads;
    lead is None for one lead."""
    return _lib.bath(b["kind"], M, b["W"], mu=b.get("mu", 0.0), placement=b.get("placement", "shift"),
                     n_leads=b.get("leads", 1))


def from_config(cfg: dict, n_traj: int | None = None, precision: str = "fp64", M: int | None = None,
                n_elec: int | None = None, lowdin_every: int = 100, record_every: int = 0,
                stream=None, elec_substeps: int = 1, **run_options):
    """One-class ensemble for a workload description of ``workloads.configs``
    (bath discretised by the library); run_options add iesh_run_desc fields
    (exit_enabled, exit_x, exit_dof, hop_filter_off, ...)."""
    b = cfg["bath"]
    M = M if M is not None else b["M"]
    N = n_elec if n_elec is not None else cfg.get("n_elec", M // 2)
    if cfg["model"]["kind"] == "dense":
        from workloads import dense_matrices
        m = cfg["model"]
        H0, H1 = dense_matrices(cfg, M)
        desc = _lib.dense_model_desc(H0, H1, m["mass"], m["omega"], N, m.get("x_c", 0.0))
    else:
        eps, w, lead, _ = bath_levels(b, M)
        desc = _lib.model_desc(cfg["model"], eps, w, N, lead)
    run = dict(n_traj=n_traj if n_traj is not None else cfg["n_traj"], precision=precision,
               dt=cfg["dt"], kT=cfg.get("kT", 0.0), seed=cfg.get("seed", 0),
               bias=b.get("bias", 0.0),
               lowdin_every=lowdin_every if precision == "mixed" else 0,
               record_every=record_every, elec_substeps=elec_substeps)
    run.update(run_options)
    return _lib.Ensemble([desc], run, stream=stream)


def pack_states(states, n_max: int, N_max: int):
    """states: list of (x, v, C (n x N complex), s (N,)) -> ABI arrays; x and
    v hold one value per coordinate (shape (T,) for one, (T, n_dof) else)."""
    T = len(states)
    nd = np.atleast_1d(states[0][0]).size
    x = np.zeros((T, nd))
    v = np.zeros((T, nd))
    Cc = np.zeros((T, n_max * N_max), dtype=np.complex128)
    occ = np.zeros((T, N_max), dtype=np.int32)
    for t, (xx, vv, CC, ss) in enumerate(states):
        n, N = CC.shape
        x[t] = np.atleast_1d(xx).astype(np.float64)
        v[t] = np.atleast_1d(vv).astype(np.float64)
        Cc[t, : n * N] = np.ascontiguousarray(CC.T).reshape(-1)
        occ[t, :N] = np.asarray(ss, dtype=np.int32)
    if nd == 1:
        x, v = x[:, 0], v[:, 0]
    return x, v, Cc, occ


def unpack_C(Cflat, t: int, n: int, N: int, n_max: int, N_max: int):
    """Orbital matrix (n x N) of trajectory t from the ABI layout."""
    blk = np.asarray(Cflat).reshape(-1)[t * n_max * N_max: t * n_max * N_max + n * N]
    return blk.reshape(N, n).T.copy()
