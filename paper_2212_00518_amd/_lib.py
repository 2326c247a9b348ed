"""ctypes binding of libiesh (the C ABI declared in include/iesh.h).

Argument marshalling only: every step of the method runs in the HIP library.
Importing this module fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# IESH_LIBRARY may point at another build of the same library (e.g. a tuning
# variant); by default the in-tree build is loaded.
LIB_PATH = os.environ.get("IESH_LIBRARY", os.path.join(HERE, "libiesh.so"))

IESH_OK = 0
IESH_EINVAL, IESH_ENOMEM, IESH_EDEVICE, IESH_ESTATE, IESH_ENOTSUP = -1, -2, -3, -4, -5
IESH_MODEL_HARMONIC = 0
IESH_MODEL_MORSE_TANH = 1
IESH_MODEL_MULTI_DOF = 2
IESH_MODEL_DENSE = 3
IESH_DENSE_MAX_N = 96
IESH_MAX_DOF = 6
IESH_FP64 = 0
IESH_MIXED = 1
IESH_MEM_HOST = 0
IESH_MEM_DEVICE = 1
IESH_BATH_TRAPEZOID = 0
IESH_BATH_TRAPEZOID_MIDPOINT = 1
IESH_BATH_GAUSS_LEGENDRE = 2
IESH_N_OBS = 5
IESH_MAX_STATES = 336
IESH_MAX_ELEC = 168
IESH_EVENT_CAP = 1 << 20

TRAJ_EXITED, TRAJ_NONCONV, TRAJ_SINGULAR_S, TRAJ_NONFINITE, TRAJ_STEPCAP = 1, 2, 4, 8, 16

OBS_NAMES = ("Pd_surf", "Pd_wf", "Ekin", "Epot", "Etot")

# exported symbols (kept in sync with include/iesh.h)
SYMBOLS = (
    "iesh_create", "iesh_destroy", "iesh_discretize", "iesh_set_state", "iesh_get_state",
    "iesh_init_thermal", "iesh_set_step", "iesh_get_step", "iesh_step", "iesh_run",
    "iesh_hop_probs", "iesh_adiabatic", "iesh_traj_status", "iesh_traj_clock", "iesh_events",
    "iesh_clear_events", "iesh_query_sizes", "iesh_sync", "iesh_last_error", "iesh_version",
    "iesh_timing", "iesh_timing_read", "iesh_work", "iesh_hop_evals", "iesh_class_info",
    "iesh_set_step_caps", "iesh_adjoint_forward", "iesh_adjoint_backward", "iesh_eigh_batched",
    "iesh_orthonormality_defect", "iesh_eigh_batched_noalloc", "iesh_bath", "iesh_class_work",
)
TIMERS = ("eig", "prop", "hop", "lowdin", "filter", "adj_prop", "adj_phi", "adj_eig", "adj_hop")


class ModelDesc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_bath", C.c_int32), ("n_elec", C.c_int32),
                ("n_dof", C.c_int32), ("eps", C.POINTER(C.c_double)),
                ("w", C.POINTER(C.c_double)), ("mass", C.c_double), ("Gamma", C.c_double),
                ("params", C.c_double * 16), ("dof", C.POINTER(C.c_double)),
                ("lead", C.POINTER(C.c_int32)), ("dense", C.POINTER(C.c_double))]


class RunDesc(C.Structure):
    _fields_ = [("n_traj", C.c_int32), ("precision", C.c_int32), ("dt", C.c_double),
                ("kT", C.c_double), ("seed", C.c_uint64), ("lowdin_every", C.c_int32),
                ("record_every", C.c_int32), ("exit_enabled", C.c_int32),
                ("compact_every", C.c_int32), ("exit_x", C.c_double), ("max_steps", C.c_int64),
                ("elec_substeps", C.c_int32), ("hop_filter_off", C.c_int32), ("bias", C.c_double),
                ("exit_dof", C.c_int32), ("dt_levels", C.c_int32), ("hop_gmax", C.c_double),
                ("eig_max_iter", C.c_int32), ("reserved3", C.c_int32)]


class BathDesc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("M", C.c_int32), ("n_leads", C.c_int32),
                ("placement", C.c_int32), ("W", C.c_double), ("mu", C.c_double)]


class Event(C.Structure):
    _fields_ = [("step", C.c_int64), ("traj", C.c_int32), ("a", C.c_int32), ("b", C.c_int32),
                ("accepted", C.c_int32), ("margin", C.c_double), ("g_total", C.c_double)]


class Sizes(C.Structure):
    _fields_ = [("n_traj", C.c_int32), ("n_models", C.c_int32), ("n_max", C.c_int32),
                ("N_max", C.c_int32), ("device_bytes", C.c_int64), ("n_dof", C.c_int32),
                ("reserved", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"libiesh.so not found at {LIB_PATH}: build it with "
                "`python -m paper_2212_00518_amd.build_lib` (there is no fallback path)")
        L = C.CDLL(LIB_PATH)
        dp, ip = C.POINTER(C.c_double), C.POINTER(C.c_int32)
        vp = C.c_void_p
        L.iesh_create.argtypes = [C.POINTER(ModelDesc), C.c_int32, ip, C.POINTER(RunDesc), vp,
                                  C.POINTER(vp)]
        L.iesh_destroy.argtypes = [vp]
        L.iesh_discretize.argtypes = [C.c_int32, C.c_int32, C.c_double, C.c_double, C.c_double,
                                      dp, dp]
        L.iesh_bath.argtypes = [C.POINTER(BathDesc), dp, dp, ip, ip]
        L.iesh_set_state.argtypes = [vp, vp, vp, vp, vp, C.c_int32]
        L.iesh_get_state.argtypes = [vp, vp, vp, vp, vp, C.c_int32]
        L.iesh_init_thermal.argtypes = [vp, dp, dp]
        L.iesh_set_step.argtypes = [vp, C.c_int64]
        L.iesh_get_step.argtypes = [vp, C.POINTER(C.c_int64)]
        L.iesh_step.argtypes = [vp]
        L.iesh_run.argtypes = [vp, C.c_int64, dp]
        L.iesh_hop_probs.argtypes = [vp, C.c_int32, C.c_int32, vp, C.c_int32]
        L.iesh_adiabatic.argtypes = [vp, C.c_int32, C.c_int32, dp, dp]
        L.iesh_traj_status.argtypes = [vp, ip]
        L.iesh_traj_clock.argtypes = [vp, dp, dp]
        L.iesh_eigh_batched.argtypes = [vp, C.c_int32, C.c_int32, vp, vp, vp, C.c_int32, vp]
        L.iesh_eigh_batched_noalloc.argtypes = [vp, C.c_int32, C.c_int32, vp, vp, vp, vp]
        L.iesh_events.argtypes = [vp, C.POINTER(Event), C.c_int64, C.POINTER(C.c_int64)]
        L.iesh_clear_events.argtypes = [vp]
        L.iesh_query_sizes.argtypes = [vp, C.POINTER(Sizes)]
        L.iesh_sync.argtypes = [vp]
        L.iesh_last_error.argtypes = [vp]
        L.iesh_last_error.restype = C.c_char_p
        L.iesh_version.argtypes = [ip, ip, ip]
        L.iesh_timing.argtypes = [vp, C.c_int32]
        L.iesh_timing_read.argtypes = [vp, dp, C.POINTER(C.c_int64)]
        L.iesh_work.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.iesh_hop_evals.argtypes = [vp, C.POINTER(C.c_int64)]
        L.iesh_class_work.argtypes = [vp, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.iesh_class_info.argtypes = [vp, C.c_int32, ip]
        L.iesh_set_step_caps.argtypes = [vp, C.POINTER(C.c_int64)]
        L.iesh_adjoint_forward.argtypes = [vp, dp, C.c_int32, C.c_int32, dp, dp]
        L.iesh_adjoint_backward.argtypes = [vp, dp, dp]
        L.iesh_orthonormality_defect.argtypes = [vp, dp, dp, C.POINTER(C.c_int64)]
        _lib = L
    return _lib


class IeshError(RuntimeError):
    pass


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def eigh_batched(H):
    """Eigen-decomposition of a batch of dense symmetric matrices (host
    arrays, shape (batch, n, n) or (n, n)) on the GPU: (lam, Q, sweeps), lam
    ascending, Q[..., :, j] the eigenvector of lam[..., j]."""
    L = lib()
    H = np.ascontiguousarray(H, dtype=np.float64)
    single = H.ndim == 2
    if single:
        H = H[None]
    if H.ndim != 3 or H.shape[1] != H.shape[2]:
        raise ValueError("H: (batch, n, n)")
    b, n = H.shape[0], H.shape[1]
    lam = np.zeros((b, n))
    Q = np.zeros((b, n, n))
    sw = np.zeros(b, dtype=np.int32)
    rc = L.iesh_eigh_batched(_ptr(H), n, b, _ptr(lam), _ptr(Q), _ptr(sw), IESH_MEM_HOST, None)
    if rc != IESH_OK:
        why = L.iesh_last_error(None)
        raise IeshError(f"iesh_eigh_batched failed ({rc}): {why.decode() if why else ''}")
    return (lam[0], Q[0], sw[0]) if single else (lam, Q, sw)


def discretize(kind: str, M: int, W: float, eps_f: float = 0.0, centre: float = 0.0):
    """Bath energies and weights on [centre - W/2, centre + W/2] from the
    library (Appendix A); the Gauss-Legendre halves split at eps_f."""
    k = BATH_KINDS[kind]
    eps = np.zeros(M)
    w = np.zeros(M)
    rc = lib().iesh_discretize(k, M, centre - 0.5 * W, centre + 0.5 * W, eps_f,
                               eps.ctypes.data_as(C.POINTER(C.c_double)),
                               w.ctypes.data_as(C.POINTER(C.c_double)))
    if rc != IESH_OK:
        raise IeshError(f"iesh_discretize failed ({rc})")
    return eps, w


BATH_KINDS = {"trapezoid": IESH_BATH_TRAPEZOID, "trapezoid_midpoint": IESH_BATH_TRAPEZOID_MIDPOINT,
              "gauss_legendre": IESH_BATH_GAUSS_LEGENDRE}
IESH_BAND_CENTRED, IESH_BAND_FIXED = 0, 1


def bath(kind: str, M: int, W: float, mu: float = 0.0, placement: str = "shift", n_leads: int = 1):
    """iesh_bath: (eps, w, lead or None, levels below mu) of a bath of M
    levels over n_leads leads, the band following mu ("shift") or fixed at
    [-W/2, W/2] ("split")."""
    d = BathDesc(BATH_KINDS[kind], int(M), int(n_leads),
                 IESH_BAND_CENTRED if placement == "shift" else IESH_BAND_FIXED, float(W), float(mu))
    eps = np.zeros(M)
    w = np.zeros(M)
    lead = np.zeros(M, dtype=np.int32)
    nb = C.c_int32()
    rc = lib().iesh_bath(C.byref(d), eps.ctypes.data_as(C.POINTER(C.c_double)),
                         w.ctypes.data_as(C.POINTER(C.c_double)),
                         lead.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(nb))
    if rc != IESH_OK:
        raise IeshError(f"iesh_bath failed ({rc})")
    return eps, w, (lead if n_leads == 2 else None), nb.value


def dense_model_desc(H0, H1, mass: float, omega: float, n_elec: int, x_c: float = 0.0):
    """iesh_model_desc of IESH_MODEL_DENSE: H(x) = H0 + x H1 (n x n
    symmetric), U0 = m omega^2 (x - x_c)^2 / 2."""
    H0 = np.ascontiguousarray(H0, dtype=np.float64)
    H1 = np.ascontiguousarray(H1, dtype=np.float64)
    if H0.ndim != 2 or H0.shape[0] != H0.shape[1] or H1.shape != H0.shape:
        raise ValueError("H0, H1: n x n")
    mats = np.ascontiguousarray(np.concatenate([H0.ravel(), H1.ravel()]))
    d = ModelDesc()
    d.kind = IESH_MODEL_DENSE
    d.n_bath = H0.shape[0] - 1
    d.n_elec = int(n_elec)
    d.n_dof = 1
    d.mass = float(mass)
    d.Gamma = 0.0
    p = [0.0] * 16
    p[:2] = [float(omega), float(x_c)]
    d.params[:] = p
    d.dense = mats.ctypes.data_as(C.POINTER(C.c_double))
    d._keep = (mats,)
    return d


def model_desc(model: dict, eps, w, n_elec: int, lead=None):
    """Fill an iesh_model_desc; `model` follows workloads.configs; `lead`
    (optional) labels each bath level 0 or 1 (two leads)."""
    eps = np.ascontiguousarray(eps, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    d = ModelDesc()
    lead_arr = None
    if lead is not None:
        lead_arr = np.ascontiguousarray(lead, dtype=np.int32)
        if lead_arr.shape != eps.shape:
            raise ValueError("lead: one label per bath level")
        d.lead = lead_arr.ctypes.data_as(C.POINTER(C.c_int32))
    d.n_bath = len(eps)
    d.n_elec = int(n_elec)
    d.eps = eps.ctypes.data_as(C.POINTER(C.c_double))
    d.w = w.ctypes.data_as(C.POINTER(C.c_double))
    d.mass = float(model.get("mass", 0.0))
    d.Gamma = float(model["Gamma"])
    p = [0.0] * 16
    dof = None
    d.n_dof = 1
    if model["kind"] == "multi_dof":
        d.kind = IESH_MODEL_MULTI_DOF
        p[:2] = [model["Delta"], model.get("eps_d", 0.0)]
        dof = np.ascontiguousarray(model["dof"], dtype=np.float64)
        if dof.ndim != 2 or dof.shape[1] != 7:
            raise ValueError("dof: rows of (mass, D, a, r, g, c, s)")
        d.n_dof = dof.shape[0]
        d.dof = dof.ctypes.data_as(C.POINTER(C.c_double))
        d.mass = float(dof[0, 0])
    elif model["kind"] == "harmonic":
        d.kind = IESH_MODEL_HARMONIC
        p[:4] = [model["omega"], model["g"], model["dG"], model.get("eps_d", 0.0)]
    elif model["kind"] == "morse_tanh":
        d.kind = IESH_MODEL_MORSE_TANH
        p[:12] = [model[k] for k in ("De", "x0", "a", "D1", "D2", "ap", "Vinf", "q", "atil",
                                     "xtil", "c")] + [model.get("eps_d", 0.0)]
    else:
        raise ValueError(model["kind"])
    d.params[:] = p
    # keep arrays alive with the descriptor
    d._keep = (eps, w, dof, lead_arr)
    return d


class Ensemble:
    """An ensemble of independent IESH trajectories on one GPU."""

    def __init__(self, models, run: dict, traj_model=None, stream=None):
        L = lib()
        self._descs = list(models)
        arr = (ModelDesc * len(self._descs))(*self._descs)
        self._arr = arr
        r = RunDesc()
        r.n_traj = int(run["n_traj"])
        r.precision = IESH_MIXED if run.get("precision", "fp64") == "mixed" else IESH_FP64
        r.dt = float(run["dt"])
        r.kT = float(run.get("kT", 0.0))
        r.seed = int(run.get("seed", 0))
        r.lowdin_every = int(run.get("lowdin_every", 0))
        r.record_every = int(run.get("record_every", 0))
        r.exit_enabled = int(run.get("exit_enabled", 0))
        r.exit_x = float(run.get("exit_x", 0.0))
        r.max_steps = int(run.get("max_steps", 0))
        r.compact_every = int(run.get("compact_every", 0))
        r.elec_substeps = int(run.get("elec_substeps", 1))
        r.bias = float(run.get("bias", 0.0))
        r.hop_filter_off = int(run.get("hop_filter_off", 0))
        r.exit_dof = int(run.get("exit_dof", 0))
        r.dt_levels = int(run.get("dt_levels", 0))
        r.hop_gmax = float(run.get("hop_gmax", 0.0))
        r.eig_max_iter = int(run.get("eig_max_iter", 0))
        self.run_desc = r
        tm = None
        if traj_model is not None:
            self._tm = np.ascontiguousarray(traj_model, dtype=np.int32)
            tm = self._tm.ctypes.data_as(C.POINTER(C.c_int32))
        ctx = C.c_void_p()
        st = C.c_void_p(stream) if stream is not None else None
        rc = L.iesh_create(arr, len(self._descs), tm, C.byref(r), st, C.byref(ctx))
        if rc != IESH_OK:
            why = L.iesh_last_error(None)
            raise IeshError(f"iesh_create failed ({rc}): {why.decode() if why else ''}")
        self.ctx = ctx
        s = Sizes()
        L.iesh_query_sizes(ctx, C.byref(s))
        self.n_traj, self.n_max, self.N_max = s.n_traj, s.n_max, s.N_max
        self.n_dof = max(1, s.n_dof)
        self.device_bytes = s.device_bytes

    def _check(self, rc, what):
        if rc != IESH_OK:
            msg = lib().iesh_last_error(self.ctx)
            raise IeshError(f"{what} failed ({rc}): {msg.decode() if msg else ''}")

    def close(self):
        if getattr(self, "ctx", None):
            lib().iesh_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- state
    def _nuc(self, a):
        """Positions or velocities as the (T * n_dof) block layout of iesh.h."""
        return np.ascontiguousarray(a, dtype=np.float64).reshape(self.n_traj * self.n_dof)

    def _nuc_out(self, a):
        return a if self.n_dof == 1 else a.reshape(self.n_traj, self.n_dof)

    def set_state(self, x, v, Cmat, occ):
        """x, v: (T,) or (T, n_dof), Cmat: (T, N_max, n_max) complex
        (orbital-major, blocks packed as documented in iesh.h), occ:
        (T, N_max) int32."""
        x = self._nuc(x)
        v = self._nuc(v)
        Cc = np.ascontiguousarray(Cmat, dtype=np.complex128)
        occ = np.ascontiguousarray(occ, dtype=np.int32)
        self._check(lib().iesh_set_state(self.ctx, _ptr(x), _ptr(v), _ptr(Cc), _ptr(occ),
                                         IESH_MEM_HOST), "iesh_set_state")

    def get_state(self):
        T = self.n_traj
        x = np.zeros(T * self.n_dof)
        v = np.zeros(T * self.n_dof)
        Cc = np.zeros(T * self.n_max * self.N_max, dtype=np.complex128)
        occ = np.zeros((T, self.N_max), dtype=np.int32)
        self._check(lib().iesh_get_state(self.ctx, _ptr(x), _ptr(v), _ptr(Cc), _ptr(occ),
                                         IESH_MEM_HOST), "iesh_get_state")
        return self._nuc_out(x), self._nuc_out(v), Cc, occ

    def init_thermal(self, x, v):
        x = self._nuc(x)
        v = self._nuc(v)
        self._check(lib().iesh_init_thermal(self.ctx, x.ctypes.data_as(C.POINTER(C.c_double)),
                                            v.ctypes.data_as(C.POINTER(C.c_double))),
                    "iesh_init_thermal")

    def set_step(self, step: int):
        self._check(lib().iesh_set_step(self.ctx, int(step)), "iesh_set_step")

    def get_step(self):
        s = C.c_int64()
        self._check(lib().iesh_get_step(self.ctx, C.byref(s)), "iesh_get_step")
        return s.value

    # ------------------------------------------------------------- dynamics
    def step(self):
        self._check(lib().iesh_step(self.ctx), "iesh_step")

    def run(self, n_steps: int, record: bool = False):
        r = self.run_desc.record_every
        obs = None
        ptr = None
        if record and r > 0:
            obs = np.zeros((n_steps // r, self.n_traj, IESH_N_OBS))
            ptr = obs.ctypes.data_as(C.POINTER(C.c_double))
        self._check(lib().iesh_run(self.ctx, int(n_steps), ptr), "iesh_run")
        return obs

    def sync(self):
        self._check(lib().iesh_sync(self.ctx), "iesh_sync")

    # --------------------------------------------------------------- queries
    def hop_probs(self, traj0: int = 0, ntraj: int | None = None):
        ntraj = self.n_traj - traj0 if ntraj is None else ntraj
        g = np.zeros(ntraj * self.N_max * self.n_max)
        self._check(lib().iesh_hop_probs(self.ctx, traj0, ntraj, _ptr(g), IESH_MEM_HOST),
                    "iesh_hop_probs")
        return g.reshape(ntraj, self.N_max * self.n_max)

    def adiabatic(self, traj0: int = 0, ntraj: int | None = None):
        ntraj = self.n_traj - traj0 if ntraj is None else ntraj
        lam = np.zeros((ntraj, self.n_max))
        q0 = np.zeros((ntraj, self.n_max))
        self._check(lib().iesh_adiabatic(self.ctx, traj0, ntraj,
                                         lam.ctypes.data_as(C.POINTER(C.c_double)),
                                         q0.ctypes.data_as(C.POINTER(C.c_double))),
                    "iesh_adiabatic")
        return lam, q0

    def status(self):
        s = np.zeros(self.n_traj, dtype=np.int32)
        self._check(lib().iesh_traj_status(self.ctx, s.ctypes.data_as(C.POINTER(C.c_int32))),
                    "iesh_traj_status")
        return s

    def clock(self):
        """(elapsed time, next step) per trajectory."""
        t = np.zeros(self.n_traj)
        d = np.zeros(self.n_traj)
        dpt = C.POINTER(C.c_double)
        self._check(lib().iesh_traj_clock(self.ctx, t.ctypes.data_as(dpt), d.ctypes.data_as(dpt)),
                    "iesh_traj_clock")
        return t, d

    def events(self, cap: int = 1 << 16):
        buf = (Event * cap)()
        n = C.c_int64()
        self._check(lib().iesh_events(self.ctx, buf, cap, C.byref(n)), "iesh_events")
        m = min(n.value, cap)
        return [dict(step=buf[i].step, traj=buf[i].traj, a=buf[i].a, b=buf[i].b,
                     accepted=bool(buf[i].accepted), margin=buf[i].margin,
                     g_total=buf[i].g_total) for i in range(m)], n.value

    def timing(self, enable: bool):
        self._check(lib().iesh_timing(self.ctx, 1 if enable else 0), "iesh_timing")

    def timing_read(self):
        ms = np.zeros(len(TIMERS))
        n = np.zeros(len(TIMERS), dtype=np.int64)
        self._check(lib().iesh_timing_read(self.ctx, ms.ctypes.data_as(C.POINTER(C.c_double)),
                                           n.ctypes.data_as(C.POINTER(C.c_int64))),
                    "iesh_timing_read")
        return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(TIMERS)}

    def work(self):
        a, b = C.c_int64(), C.c_int64()
        self._check(lib().iesh_work(self.ctx, C.byref(a), C.byref(b)), "iesh_work")
        return a.value, b.value

    def class_work(self, cls: int):
        """(Chebyshev terms summed, trajectory-steps) of one class since
        iesh_timing was last called."""
        a, b = C.c_int64(), C.c_int64()
        self._check(lib().iesh_class_work(self.ctx, int(cls), C.byref(a), C.byref(b)), "iesh_class_work")
        return a.value, b.value

    def set_step_caps(self, caps):
        caps = np.ascontiguousarray(caps, dtype=np.int64)
        if caps.shape != (self.n_traj,):
            raise ValueError("one cap per trajectory")
        self._check(lib().iesh_set_step_caps(self.ctx, caps.ctypes.data_as(C.POINTER(C.c_int64))),
                    "iesh_set_step_caps")

    def class_info(self, cls: int = 0):
        """(n_traj, live slots, n, N, tiles per propagation work-group,
        work-groups per trajectory, n_pad) of one bath-size class."""
        info = np.zeros(8, dtype=np.int32)
        self._check(lib().iesh_class_info(self.ctx, int(cls), info.ctypes.data_as(C.POINTER(C.c_int32))),
                    "iesh_class_info")
        keys = ("n_traj", "live", "n", "N", "tiles_per_group", "groups_per_traj", "n_pad")
        return dict(zip(keys, (int(v) for v in info[:7])))

    def adjoint_forward(self, path, ckpt_every: int = 100, terms=(1.0, 1.0, 0.0, 0.0)):
        """Losses of the prescribed paths (n_traj, n_steps + 1) with term
        weights (c_P, c_E, c_G, c_F); keeps what the backward pass needs."""
        path = np.ascontiguousarray(path, dtype=np.float64)
        if path.ndim != 2 or path.shape[0] != self.n_traj or path.shape[1] < 2:
            raise ValueError("path must be (n_traj, n_steps + 1) with n_steps >= 1")
        tw = np.ascontiguousarray(terms, dtype=np.float64)
        if tw.shape != (4,):
            raise ValueError("terms: four weights (c_P, c_E, c_G, c_F)")
        loss = np.zeros(self.n_traj)
        self._check(lib().iesh_adjoint_forward(self.ctx, path.ctypes.data_as(C.POINTER(C.c_double)),
                                               path.shape[1] - 1, int(ckpt_every),
                                               tw.ctypes.data_as(C.POINTER(C.c_double)),
                                               loss.ctypes.data_as(C.POINTER(C.c_double))),
                    "iesh_adjoint_forward")
        return loss

    def adjoint_backward(self, dloss):
        """Rows w_t dL_t/dtheta, (n_traj, n_max + 4), layout
        [eps_d, Gamma, eps_1 .. eps_M, omega, g, dG] per row."""
        w = np.ascontiguousarray(dloss, dtype=np.float64)
        if w.shape != (self.n_traj,):
            raise ValueError("one weight per trajectory")
        g = np.zeros((self.n_traj, self.n_max + 4))
        self._check(lib().iesh_adjoint_backward(self.ctx, w.ctypes.data_as(C.POINTER(C.c_double)),
                                                g.ctypes.data_as(C.POINTER(C.c_double))),
                    "iesh_adjoint_backward")
        return g

    def hop_evals(self):
        n = C.c_int64()
        self._check(lib().iesh_hop_evals(self.ctx, C.byref(n)), "iesh_hop_evals")
        return n.value

    def clear_events(self):
        self._check(lib().iesh_clear_events(self.ctx), "iesh_clear_events")

    def defect(self):
        """(per-trajectory defect before the last Loewdin correction, largest
        measured, measurements above the no-hop bound's allowance)."""
        d = np.zeros(self.n_traj)
        mx = C.c_double()
        nv = C.c_int64()
        self._check(lib().iesh_orthonormality_defect(self.ctx, d.ctypes.data_as(C.POINTER(C.c_double)),
                                                     C.byref(mx), C.byref(nv)),
                    "iesh_orthonormality_defect")
        return d, mx.value, nv.value

    def defect_max(self):
        _, mx, nv = self.defect()
        return {"max": mx, "violations": nv}
