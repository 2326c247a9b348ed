"""Pins of the oracle's two-lead bath (equal bath energies) and of the biased
initial occupations, against closed forms that do not reuse the oracle's
own formulas.

* Two leads on one grid, each with Gamma/2, are one lead with Gamma plus one
  decoupled level per grid energy: the spectrum is the one-lead spectrum
  joined with the grid energies, the extra eigenstates have no impurity part,
  and their nonadiabatic couplings vanish.
* By the symmetry between the leads every orbital sits half on each lead.
* When the impurity decouples (Gamma -> 0) the biased occupation
  probabilities put, at every grid energy, the two leads' own Fermi fillings
  (at mu + V/2 and mu - V/2) on the two orbitals of that energy.
"""
import numpy as np
import pytest

from oracle import bath, dynamics as dyn, electronic as el, models
from workloads import get_config


def _two_lead(name="c5", M=20, **over):
    cfg = get_config(name)
    cfg["bath"]["M"] = M
    cfg["bath"]["leads"] = 2
    cfg["n_elec"] = M // 2
    cfg["model"].update(over)
    return cfg


def _one_lead_of(cfg):
    one = get_config("c5")
    one["bath"] = dict(cfg["bath"])
    one["bath"]["M"] = cfg["bath"]["M"] // 2
    one["bath"]["leads"] = 1
    one["model"] = dict(cfg["model"])
    return one


@pytest.mark.parametrize("name", ["c5", "c2"])
def test_two_lead_spectrum_is_one_lead_plus_the_grid(name):
    cfg = _two_lead(name, M=24)
    m2 = models.from_config(cfg)
    m1 = models.from_config(_one_lead_of(cfg))
    assert m2.n == 25 and m1.n == 13
    assert list(m2.lead) == [0, 1] * 12
    assert np.array_equal(m2.eps[0::2], m2.eps[1::2])
    rs = np.random.default_rng(1)
    for _ in range(3):
        x = np.atleast_1d(np.array(cfg["model"]["dof"])[:, 3] + rs.normal(0.0, 0.2, size=6)
                          if name == "c5" else rs.normal(0.0, 8.0))
        lam2, Q2 = el.eig(m2.H(x))
        lam1, Q1 = el.eig(m1.H(x))
        ref = np.sort(np.concatenate([lam1, m1.eps]))
        assert np.max(np.abs(lam2 - ref)) < 1e-13
        # states at a grid energy have no impurity part; the others carry the
        # one-lead impurity amplitudes
        at_grid = np.array([np.min(np.abs(m1.eps - l)) < 1e-13 for l in lam2])
        assert at_grid.sum() == 12
        assert np.max(np.abs(Q2[0, at_grid])) < 1e-13
        assert np.max(np.abs(np.sort(Q2[0, ~at_grid] ** 2) - np.sort(Q1[0] ** 2))) < 1e-13
        # their nonadiabatic couplings vanish in every coordinate
        _, Ds = el.coupling_matrices(lam2, Q2, m2.dH(x))
        scale = max(np.max(np.abs(D)) for D in Ds)
        for D in Ds:
            assert np.max(np.abs(D[at_grid, :])) < 1e-10 * scale
            assert np.max(np.abs(D[:, at_grid])) < 1e-10 * scale


def test_every_orbital_sits_half_on_each_lead():
    cfg = _two_lead("c5", M=16)
    m = models.from_config(cfg)
    x = np.array(cfg["model"]["dof"])[:, 3] + 0.1
    lam, Q = el.eig(m.H(x))
    w0 = dyn.lead_weights(Q, m.lead)
    w1 = np.sum(Q[1 + np.flatnonzero(m.lead == 1), :] ** 2, axis=0)
    assert np.max(np.abs(w0 - w1)) < 1e-13
    assert np.max(np.abs(w0 + w1 + Q[0] ** 2 - 1.0)) < 1e-13


@pytest.mark.parametrize("V", [0.01, 0.02])
def test_decoupled_impurity_gives_each_lead_its_own_fermi_filling(V):
    """Gamma -> 0: each grid energy holds a bonding and an antibonding
    orbital, both half on each lead; their summed occupation probability is
    f(e - mu - V/2) + f(e - mu + V/2), the two leads' fillings."""
    cfg = _two_lead("c2", M=40, Gamma=1e-12)
    m = models.from_config(cfg)
    x = np.array([-30.0])  # impurity level far above the band
    lam, Q = el.eig(m.H(x))
    kT, mu = 2e-3, 0.004
    f = dyn.occupation_probabilities(lam, mu, kT, Q[0], dyn.lead_weights(Q, m.lead), V)
    grid = m.eps[0::2]
    for k, e in enumerate(grid):
        near = np.flatnonzero(np.abs(lam - e) < 1e-9)
        assert len(near) == 2
        fl = 1.0 / (1.0 + np.exp((e - mu - 0.5 * V) / kT))
        fr = 1.0 / (1.0 + np.exp((e - mu + 0.5 * V) / kT))
        assert abs(f[near].sum() - (fl + fr)) < 1e-9, (k, e)


def test_biased_sampling_keeps_n_and_reduces_to_the_unbiased_rule():
    cfg = _two_lead("c5", M=40)
    m = models.from_config(cfg)
    x = np.array(cfg["model"]["dof"])[:, 3]
    lam, Q = el.eig(m.H(x))
    N, kT = 20, cfg["kT"]
    w0 = dyn.lead_weights(Q, m.lead)
    for V in (0.01, 0.02):
        for t in range(5):
            s, used = dyn.fermi_occupations(lam, N, kT, 0, t, q0=Q[0], w0=w0, bias=V)
            assert used > 0 and len(s) == N and len(set(s.tolist())) == N
    # an infinitesimal bias samples as no bias (the probabilities agree to
    # rounding, so the same uniforms accept the same sets)
    for t in range(5):
        s0, _ = dyn.fermi_occupations(lam, N, kT, 0, t)
        s1, _ = dyn.fermi_occupations(lam, N, kT, 0, t, q0=Q[0], w0=w0, bias=1e-300)
        assert np.array_equal(s0, s1)


def test_an_orbital_on_lead_0_fills_up_to_mu_plus_half_the_bias():
    """Convention of the sign of V: an orbital entirely on lead 0 is filled
    with the Fermi function of mu + V/2, one on lead 1 with mu - V/2."""
    lam = np.array([0.0])
    kT, mu, V = 1e-3, -0.004, 0.01
    f0 = dyn.occupation_probabilities(lam, mu, kT, np.zeros(1), np.ones(1), V)
    f1 = dyn.occupation_probabilities(lam, mu, kT, np.zeros(1), np.zeros(1), V)
    assert abs(f0[0] - 1.0 / (1.0 + np.exp(-(mu + 0.5 * V) / kT))) < 1e-15
    assert abs(f1[0] - 1.0 / (1.0 + np.exp(-(mu - 0.5 * V) / kT))) < 1e-15
    assert f0[0] > 0.5 > f1[0]


def test_two_leads_layout_of_the_grid():
    e, w = bath.discretise("trapezoid", 5, 0.1)
    e2, w2, lead = bath.two_leads(e, w)
    assert np.array_equal(e2, np.repeat(e, 2))
    assert np.array_equal(w2, np.repeat(0.5 * w, 2))
    assert np.array_equal(lead, np.tile([0, 1], 5))
    # the couplings of a pair add up to the one-lead coupling
    V1 = bath.couplings(0.01, w)
    V2 = bath.couplings(0.01, w2)
    assert np.allclose(V2[0::2] ** 2 + V2[1::2] ** 2, V1 ** 2, rtol=1e-15, atol=0)
