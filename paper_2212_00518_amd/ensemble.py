"""Ensembles from workload descriptions, and state packing helpers."""
from __future__ import annotations

import numpy as np

from . import _lib


def bath_grid(b: dict, M: int):
    """Bath of a workload description, placed for its chemical potential mu
    (default 0).  Placement "shift" moves the whole band so that its centre
    and the Gauss-Legendre split sit at mu (wide-band limit); "split" keeps
    the band [-W/2, W/2] and splits the Gauss-Legendre halves at mu
    (Sec. II.B, chemical potential; App. A)."""
    mu = b.get("mu", 0.0)
    if b.get("placement", "shift") == "shift":
        return _lib.discretize(b["kind"], M, b["W"], eps_f=mu, centre=mu)
    return _lib.discretize(b["kind"], M, b["W"], eps_f=mu)


def bath_levels(b: dict, M: int):
    """Bath levels of a workload description: (eps, w, lead).  With
    ``leads: 2`` the M levels are one grid of M/2 levels shared by two leads,
    each coupled with half the hybridisation (half of every weight), listed
    in ascending energy with lead 0 first at equal energy; lead is None for
    one lead."""
    if b.get("leads", 1) != 2:
        eps, w = bath_grid(b, M)
        return eps, w, None
    if M % 2:
        raise ValueError("two leads need an even number of bath levels")
    e1, w1 = bath_grid(b, M // 2)
    eps = np.repeat(e1, 2)
    w = np.repeat(0.5 * w1, 2)
    lead = np.tile(np.array([0, 1], dtype=np.int32), M // 2)
    return eps, w, lead


def electrons_below(eps, mu: float) -> int:
    """Electron count that fills the bath states below mu in the lowest
    configuration (Sec. II.B, chemical potential)."""
    return int(np.sum(np.asarray(eps) < mu))


def from_config(cfg: dict, n_traj: int | None = None, precision: str = "fp64", M: int | None = None,
                n_elec: int | None = None, lowdin_every: int = 100, record_every: int = 0,
                stream=None, elec_substeps: int = 1, **run_options):
    """One-class ensemble for a workload description of ``workloads.configs``
    (bath discretised by the library); run_options add iesh_run_desc fields
    (exit_enabled, exit_x, exit_dof, hop_filter_off, ...)."""
    b = cfg["bath"]
    M = M if M is not None else b["M"]
    N = n_elec if n_elec is not None else cfg.get("n_elec", M // 2)
    eps, w, lead = bath_levels(b, M)
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
