"""One IESH time step, trajectories and observables (Sec. II.B, II.C).

Test infrastructure only (see the package docstring).

Step order.  The paper integrates the nuclei with velocity Verlet and the
orbitals with the exponential integrator of Eq. exponential_integrator but
does not say at which nuclear geometry the propagator matrix is frozen over
the step.  Reading used here: the midpoint.  With F_n the force at (x_n, s_n):

  1. v_half = v_n + dt/2 F_n / m
  2. x_new  = x_n + dt v_half
  3. A = diag(lambda(x_mid)) - i v_half . D(x_mid), x_mid = (x_n + x_new)/2
     (v_half is exactly (x_new - x_n)/dt)
  4. C_new = exp(-i A dt) C_n
  5. eigen-solve at x_new, F_new = F(x_new, s_n)
  6. v_new = v_half + dt/2 F_new / m
  7. hop probabilities from (C_new, s_n, D(x_new), v_new); one uniform xi
     selects a hop (electronic.select_hop)
  8. accepted hop: v rescaled along D[b, a] (electronic.rescale), s updated,
     force recomputed at x_new with the new s.  Frustrated hop: nothing
     changes (no velocity reversal).

The energy change of a hop is lambda_b(x_new) - lambda_a(x_new).

Electronic sub-steps (Sec. II.C, the paragraph after Eq.
fast_exponential_integrator): with S > 1 the orbital propagation of step 4
is split into S sub-steps of dt/S; sub-step j freezes A at the geometry
x_n + (j + 1/2)/S (x_new - x_n) along the drift, with the same velocity
v_half, solving the eigenproblem there rather than interpolating lambda and D
between the nuclear steps.  S = 1 is the midpoint rule above.
"""
from __future__ import annotations

import numpy as np

from . import electronic as el
from . import rng as _rng


class State:
    def __init__(self, x, v, C, s):
        self.x = np.atleast_1d(np.asarray(x, dtype=np.float64)).copy()
        self.v = np.atleast_1d(np.asarray(v, dtype=np.float64)).copy()
        self.C = np.asarray(C, dtype=np.complex128).copy()
        self.s = np.sort(np.asarray(s, dtype=np.int64))

    def copy(self):
        return State(self.x, self.v, self.C, self.s)


def step(model, st: State, dt: float, xi: float, F=None, substeps: int = 1):
    """Advance one step; returns (new_state, event, F_new).

    event: dict(hop=bool, attempted=bool, r, a, b, accepted, margin, g_total).
    """
    m = model.mass
    x, v, C, s = st.x, st.v, st.C, st.s
    if F is None:
        F = el.forces(model, x, s)
    v_half = v + 0.5 * dt * F / m
    x_new = x + dt * v_half
    x_mid = 0.5 * (x + x_new)

    if substeps == 1:
        lam_m, Q_m = el.eig(model.H(x_mid))
        _, Ds_m = el.coupling_matrices(lam_m, Q_m, model.dH(x_mid))
        A = el.propagator_matrix(lam_m, Ds_m, v_half)
        C_new = el.propagate(C, A, dt)
    else:
        C_new = C
        for j in range(substeps):
            x_j = x + ((j + 0.5) / substeps) * (x_new - x)
            lam_j, Q_j = el.eig(model.H(x_j))
            _, Ds_j = el.coupling_matrices(lam_j, Q_j, model.dH(x_j))
            C_new = el.propagate(C_new, el.propagator_matrix(lam_j, Ds_j, v_half), dt / substeps)

    lam, Q = el.eig(model.H(x_new))
    Gs, Ds = el.coupling_matrices(lam, Q, model.dH(x_new))
    F_new = -model.dU0(x_new).astype(np.float64)
    for nu, G in enumerate(Gs):
        F_new[nu] -= np.sum(np.diag(G)[s])
    v_new = v_half + 0.5 * dt * F_new / m

    vD = el.vdot_D(Ds, v_new)
    g, _, _ = el.hop_probabilities(C_new, s, vD, dt)
    r, b, margin = el.select_hop(g, xi)
    event = dict(attempted=r is not None, accepted=False, r=r, a=None, b=b,
                 margin=margin, g_total=float(g.sum()))
    s_new = s.copy()
    if r is not None:
        a = int(s[r])
        event["a"] = a
        d = np.array([D[b, a] for D in Ds])
        v_try, ok = el.rescale(v_new, m, d, lam[b] - lam[a])
        if ok:
            event["accepted"] = True
            v_new = v_try
            s_new[r] = b
            s_new = np.sort(s_new)
            F_new = -model.dU0(x_new).astype(np.float64)
            for nu, G in enumerate(Gs):
                F_new[nu] -= np.sum(np.diag(G)[s_new])
    return State(x_new, v_new, C_new, s_new), event, F_new


def hop_probs(model, st: State, dt: float):
    """Hop probabilities at the current state (no sampling): D and lambda at
    st.x, velocity st.v, orbitals st.C, occupations st.s."""
    lam, Q = el.eig(model.H(st.x))
    _, Ds = el.coupling_matrices(lam, Q, model.dH(st.x))
    g, _, _ = el.hop_probabilities(st.C, st.s, el.vdot_D(Ds, st.v), dt)
    return g


def observables(model, st: State):
    """Per-trajectory observables at the current state.

    P_d^surf = sum_{a in s} |Q[0, a]|^2   (impurity content of the occupied
               adiabatic orbitals: the surface-hopping estimator)
    P_d^wf   = sum_n |sum_a Q[0, a] C[a, n]|^2   (impurity occupation of the
               Slater determinant of the propagated orbitals)
    E_kin, E_pot = U0 + sum_{a in s} lambda_a (Eq. classical_hamiltonian),
    E_tot, and the orthonormality defect max |C^H C - I|.
    """
    lam, Q = el.eig(model.H(st.x))
    q0 = Q[0]
    Ekin = 0.5 * np.sum(model.mass * st.v ** 2)
    Epot = model.U0(st.x) + np.sum(lam[st.s])
    amp = q0 @ st.C
    N = st.C.shape[1]
    return dict(
        Pd_surf=float(np.sum(q0[st.s] ** 2)),
        Pd_wf=float(np.sum(np.abs(amp) ** 2)),
        Ekin=float(Ekin), Epot=float(Epot), Etot=float(Ekin + Epot),
        ortho=float(np.max(np.abs(st.C.conj().T @ st.C - np.eye(N)))),
    )


def occupation_probabilities(lam, mu, kT, q0=None, w0=None, bias=0.0):
    """Occupation probability of each orbital at chemical potential mu.

    Without a bias, the Fermi function f(lambda - mu).  With a bias V between
    two leads (Sec. III.C models a bias as a shift of the chemical
    potential; the paper does not say how two leads at different chemical
    potentials fill the orbitals).  Reading: lead 0 sits at mu + V/2, lead 1
    at mu - V/2 and the impurity at mu, and an orbital's probability is the
    mix of the three Fermi functions weighted by its squared components on
    the impurity (q0^2), on lead 0 (w0) and on lead 1 (1 - q0^2 - w0)."""
    if bias == 0.0:
        return fermi(lam, mu, kT)
    q2 = np.asarray(q0) ** 2
    w0 = np.asarray(w0)
    w1 = 1.0 - q2 - w0
    return (q2 * fermi(lam, mu, kT) + w0 * fermi(lam, mu + 0.5 * bias, kT)
            + w1 * fermi(lam, mu - 0.5 * bias, kT))


def lead_weights(Q, lead):
    """Squared weight of every orbital (column of Q) on the levels of lead 0."""
    rows = 1 + np.flatnonzero(np.asarray(lead) == 0)
    return np.sum(Q[rows, :] ** 2, axis=0)


def fermi_occupations(lam, n_elec, kT, seed, traj, max_attempts=4096, q0=None, w0=None,
                      bias=0.0):
    """Occupied set s for the initial state: N electrons at temperature kT
    (Sec. III.C initialises electrons from a Fermi-Dirac distribution; the
    paper does not fix the electron-number constraint).  Reading: the
    chemical potential mu is found by bisection so that sum_a f_a = N with
    f_a = 1/(1 + exp((lambda_a - mu)/kT)); attempt t draws one uniform per
    level from stream 1 at counter t*n + a, occupies level a when u_a < f_a,
    and is accepted when exactly N levels are occupied.  kT = 0, or no
    acceptance within max_attempts, gives the lowest N levels.  With a bias
    (two leads) f_a is occupation_probabilities(...) with the orbitals'
    impurity amplitudes q0 and lead-0 weights w0, and the bisection bracket
    is widened by |bias|.

    Returns (s, attempts_used); attempts_used = 0 means the lowest-N rule.
    """
    n = len(lam)
    if kT <= 0.0:
        return np.arange(n_elec), 0
    lo = lam[0] - 50.0 * kT - 1.0 - abs(bias)
    hi = lam[-1] + 50.0 * kT + 1.0 + abs(bias)
    for _ in range(200):
        mu = 0.5 * (lo + hi)
        f = occupation_probabilities(lam, mu, kT, q0, w0, bias)
        if f.sum() > n_elec:
            hi = mu
        else:
            lo = mu
    mu = 0.5 * (lo + hi)
    f = occupation_probabilities(lam, mu, kT, q0, w0, bias)
    for t in range(max_attempts):
        u = np.array([_rng.uniform(seed, traj, t * n + a, stream=1) for a in range(n)])
        occ = u < f
        if occ.sum() == n_elec:
            return np.flatnonzero(occ), t + 1
    return np.arange(n_elec), 0


def fermi(e, mu, kT):
    z = (np.asarray(e) - mu) / kT
    out = np.empty_like(z)
    pos = z > 0
    ez = np.exp(-z[pos])
    out[pos] = ez / (1.0 + ez)
    out[~pos] = 1.0 / (1.0 + np.exp(z[~pos]))
    return out


def initial_state(model, x0, v0, n_elec, kT, seed, traj, bias=0.0):
    """Initial state: occupations from fermi_occupations at x0 and orbitals
    that are the occupied adiabatic unit vectors (Sec. III.C: the
    coefficients match the discrete populations).  A bias needs a two-lead
    model (model.lead)."""
    lam, Q = el.eig(model.H(np.atleast_1d(x0)))
    if bias != 0.0:
        s, _ = fermi_occupations(lam, n_elec, kT, seed, traj, q0=Q[0], w0=lead_weights(Q, model.lead),
                                 bias=bias)
    else:
        s, _ = fermi_occupations(lam, n_elec, kT, seed, traj)
    C = np.zeros((model.n, n_elec), dtype=np.complex128)
    for i, a in enumerate(s):
        C[a, i] = 1.0
    return State(x0, v0, C, s)


def next_dt(g_total, dt_cur, dt0, g_max, levels):
    """Time step of the next step from the hop probabilities of this one.

    Sec. II.C (the paragraph after Eq. fast_exponential_integrator) limits
    the nuclear step by the size of the hopping probabilities, and the
    outlook proposes adapting it to them; the paper gives no rule.  Reading:
    the probabilities are proportional to the step, so the next step is the
    largest dt0 / 2^k (k = 0 .. levels) for which this step's total,
    rescaled to it, stays at or below g_max: g_total * (dt0 / 2^k) / dt_cur
    <= g_max; the smallest step when none does."""
    dtn = dt0
    k = 0
    while k < levels and g_total * (dtn / dt_cur) > g_max:
        dtn = 0.5 * dtn
        k += 1
    return dtn


def run_to_exit(model, st: State, dt: float, n_max: int, seed: int, traj: int, exit_x: float,
                exit_dof: int = 0):
    """Run until the step that takes coordinate exit_dof past exit_x (the
    trajectory leaves and is frozen there, as a scattering trajectory that has
    rebounded, Sec. III.D), at most n_max steps.  Returns (state, steps taken,
    events)."""
    F = el.forces(model, st.x, st.s)
    events = []
    for k in range(n_max):
        st, ev, F = step(model, st, dt, _rng.uniform(seed, traj, k), F)
        ev["step"] = k
        if ev["attempted"]:
            events.append(ev)
        if st.x[exit_dof] > exit_x:
            return st, k + 1, events
    return st, n_max, events


def run(model, st: State, dt: float, n_steps: int, seed: int, traj: int, step0: int = 0,
        record_every: int = 0, substeps: int = 1, adapt=None):
    """Run n_steps; the hop uniform of step k (0-based, counted from step0) is
    rng.uniform(seed, traj, step0 + k).  Returns (state, events, records).

    adapt = (g_max, levels) makes the step adaptive (next_dt, starting from
    dt); every event records the step's dt, and the returned state carries
    the elapsed time and the next step's dt (attributes time, dt)."""
    F = el.forces(model, st.x, st.s)
    events, records = [], []
    dt_cur, time = dt, 0.0
    for k in range(n_steps):
        xi = _rng.uniform(seed, traj, step0 + k)
        st, ev, F = step(model, st, dt_cur, xi, F, substeps)
        ev["step"] = step0 + k
        ev["dt"] = dt_cur
        time += dt_cur
        if adapt is not None:
            dt_cur = next_dt(ev["g_total"], dt_cur, dt, adapt[0], adapt[1])
        if ev["attempted"]:
            events.append(ev)
        if record_every and (k + 1) % record_every == 0:
            records.append(observables(model, st))
    st.time, st.dt = time, dt_cur
    return st, events, records
