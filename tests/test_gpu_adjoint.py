"""Parity of the GPU adjoint (iesh_adjoint_forward / iesh_adjoint_backward)
with the oracle's path loss and its tangent-linear gradient.

Tolerances (FP64): loss 1e-10 relative; gradient 1e-8 relative to the
largest gradient entry of the path (the GPU differentiates the truncated
Chebyshev series with its centre and radius held fixed, the oracle the
exact exponential; both errors are far below this).
"""
import numpy as np
import pytest

from oracle import adjoint as adj
from workloads import get_config
from workloads.sampling import fixed_paths

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2212_00518_amd import _lib
    _lib.lib()  # fails loudly when the library is missing


def _model(M, eps_d=0.0):
    """The double-well model of the adjoint workload on an evenly spaced
    band of width W (plain input data: cell centres, equal weights)."""
    cfg = get_config("c4")
    m = cfg["model"]
    W = cfg["bath"]["W"]
    eps = -0.5 * W + (np.arange(M) + 0.5) * (W / M)
    w = np.full(M, W / M)
    p = adj.Params(eps_d, m["Gamma"], eps, m["omega"], m["g"], m["dG"], w, m["mass"])
    return p, cfg["dt"]


def _ensemble(p, N, T, dt):
    from paper_2212_00518_amd.adjoint import ensemble_for
    return ensemble_for(adj.pack(p), p.w, p.mass, N, T, dt)


def _paths(p, T, n_steps, dt, seed):
    x, _ = fixed_paths(T, n_steps, dt, p.omega, seed=seed)
    return x


def _check_grad(g_gpu, g_ref, what, atol=0.0):
    scale = np.max(np.abs(g_ref))
    err = np.max(np.abs(g_gpu - g_ref))
    assert err <= 1e-8 * scale + atol, (what, err, scale, np.argmax(np.abs(g_gpu - g_ref)))


@pytest.mark.parametrize("M,N,n_steps,ckpt", [
    (8, 4, 12, 5),     # ragged last segment
    (20, 10, 30, 7),
    (35, 17, 16, 16),  # one segment, n not a multiple of 16
    (1, 1, 6, 2),      # one bath level
])
def test_loss_and_gradient_match_the_oracle(M, N, n_steps, ckpt):
    p, dt = _model(M)
    T = 3
    x = _paths(p, T, n_steps, dt, seed=M)
    ens = _ensemble(p, N, T, dt)
    loss = ens.adjoint_forward(x, ckpt)
    w = np.array([1.0, -0.5, 2.0])
    rows = ens.adjoint_backward(w)
    npar = adj.n_params(M)
    assert np.all(rows[:, npar:] == 0.0)
    for t in range(T):
        ref = adj.loss(p, x[t], N, dt)
        assert abs(loss[t] - ref) <= 1e-10 * abs(ref), (t, loss[t], ref)
        g = adj.gradient(p, x[t], N, dt)
        print(f"M={M} N={N} steps={n_steps} path {t}: loss {loss[t]:.12g}", flush=True)
        _check_grad(rows[t, :npar], w[t] * g, f"path {t}")


TERMS = (0.7, 0.3, 1.5, 2.0)


@pytest.mark.parametrize("M,N,n_steps,ckpt", [
    (8, 4, 12, 5),
    (20, 10, 20, 6),
    (1, 1, 6, 4),
    (40, 9, 10, 10),   # few electrons, many unoccupied states
])
def test_each_loss_term_matches_the_oracle(M, N, n_steps, ckpt):
    """Every loss term alone (population, excitation, accumulated hop
    probability through the N x N inverse, Hellmann-Feynman force; their
    magnitudes differ by orders), then all four together, each against the
    oracle at its own scale."""
    p, dt = _model(M)
    T = 3
    x = _paths(p, T, n_steps, dt, seed=100 + M)
    ens = _ensemble(p, N, T, dt)
    w = np.array([1.0, 2.0, -0.5])
    npar = adj.n_params(M)
    for terms in ((1.0, 0, 0, 0), (0, 1.0, 0, 0), (0, 0, 1.0, 0), (0, 0, 0, 1.0), TERMS):
        loss = ens.adjoint_forward(x, ckpt, terms)
        rows = ens.adjoint_backward(w)
        for t in range(T):
            ref = adj.loss(p, x[t], N, dt, terms)
            print(f"M={M} N={N} terms={terms} path {t}: loss {loss[t]:.6e} oracle {ref:.6e}", flush=True)
            # E_exc alone is a small difference of unit populations weighted by
            # energies of order 0.05: an absolute floor of 1e-13 covers rounding
            assert abs(loss[t] - ref) <= 1e-10 * abs(ref) + 1e-13, (terms, t, loss[t], ref)
            # E_exc alone: its cotangent rho - n0 carries the populations'
            # rounding (~1e-15 after the propagation) into derivatives of the
            # energies of size up to ~1e2 (d lambda / d omega), so 1e-12 absolute
            atol = 1e-12 if terms == (0, 1.0, 0, 0) else 0.0
            _check_grad(rows[t, :npar], w[t] * adj.gradient(p, x[t], N, dt, terms), f"{terms} path {t}",
                        atol)


def test_hop_term_alone_is_nonzero_and_matches():
    p, dt = _model(12)
    N, T, n_steps = 6, 2, 15
    x = _paths(p, T, n_steps, dt, seed=77)
    ens = _ensemble(p, N, T, dt)
    only = (0.0, 0.0, 1.0, 0.0)
    loss = ens.adjoint_forward(x, 4, only)
    rows = ens.adjoint_backward(np.ones(T))
    for t in range(T):
        ref = adj.loss(p, x[t], N, dt, only)
        assert ref > 0.0
        assert abs(loss[t] - ref) <= 1e-10 * ref
        _check_grad(rows[t, :adj.n_params(12)], adj.gradient(p, x[t], N, dt, only), f"path {t}")


def test_hop_term_with_the_inverse_outside_lds():
    """N = 95 electrons: the N x N inverse of the hop term does not fit the
    work-group's LDS and is kept in the trajectory's scratch block."""
    p, dt = _model(191)
    N, T, n_steps = 95, 1, 3
    x = _paths(p, T, n_steps, dt, seed=5)
    ens = _ensemble(p, N, T, dt)
    only = (0.0, 0.0, 1.0, 0.0)
    loss = ens.adjoint_forward(x, 2, only)
    rows = ens.adjoint_backward(np.ones(T))
    ref = adj.loss(p, x[0], N, dt, only)
    assert ref > 0.0
    assert abs(loss[0] - ref) <= 1e-10 * ref
    _check_grad(rows[0, :adj.n_params(191)], adj.gradient(p, x[0], N, dt, only), "N = 95")


def test_full_size_model_on_short_paths():
    """The workload's model size (M = 100, N = 50) on two short paths."""
    p, dt = _model(100)
    N, T, n_steps = 50, 2, 4
    x = _paths(p, T, n_steps, dt, seed=11)
    ens = _ensemble(p, N, T, dt)
    loss = ens.adjoint_forward(x, 3)
    rows = ens.adjoint_backward(np.ones(T))
    for t in range(T):
        ref = adj.loss(p, x[t], N, dt)
        assert abs(loss[t] - ref) <= 1e-10 * abs(ref)
        _check_grad(rows[t, :adj.n_params(100)], adj.gradient(p, x[t], N, dt), f"path {t}")


def test_checkpoint_spacing_does_not_change_the_result():
    p, dt = _model(12)
    N, T, n_steps = 6, 4, 40
    x = _paths(p, T, n_steps, dt, seed=5)
    ens = _ensemble(p, N, T, dt)
    out = []
    for ckpt in (1, 9, 40):
        loss = ens.adjoint_forward(x, ckpt)
        rows = ens.adjoint_backward(np.ones(T))
        out.append((loss, rows))
    for loss, rows in out[1:]:
        assert np.array_equal(loss, out[0][0])
        assert np.array_equal(rows, out[0][1])


def test_backward_is_linear_in_the_weights_and_repeatable():
    p, dt = _model(10)
    N, T, n_steps = 5, 3, 10
    x = _paths(p, T, n_steps, dt, seed=8)
    ens = _ensemble(p, N, T, dt)
    ens.adjoint_forward(x, 4)
    g1 = ens.adjoint_backward(np.ones(T))
    g2 = ens.adjoint_backward(np.array([2.0, 0.0, -1.0]))
    g1b = ens.adjoint_backward(np.ones(T))
    assert np.array_equal(g1, g1b)
    np.testing.assert_allclose(g2, g1 * np.array([2.0, 0.0, -1.0])[:, None], rtol=1e-14, atol=0)


def test_autograd_function_sums_the_rows():
    import torch
    from paper_2212_00518_amd.adjoint import path_loss
    p, dt = _model(8)
    N, T, n_steps = 4, 3, 8
    x = _paths(p, T, n_steps, dt, seed=2)
    theta = torch.tensor(adj.pack(p), dtype=torch.float64, requires_grad=True)
    L = path_loss(theta, x, p.w, p.mass, N, dt, ckpt_every=3)
    (L * torch.tensor([1.0, 2.0, 3.0], dtype=torch.float64)).sum().backward()
    ref = sum(c * adj.gradient(p, x[t], N, dt) for t, c in enumerate((1.0, 2.0, 3.0)))
    _check_grad(theta.grad.numpy(), ref, "autograd")
    for t in range(T):
        assert abs(L[t].item() - adj.loss(p, x[t], N, dt)) <= 1e-10 * abs(L[t].item())


def test_error_paths():
    from paper_2212_00518_amd import _lib, from_config
    p, dt = _model(6)
    ens = _ensemble(p, 3, 2, dt)
    with pytest.raises(_lib.IeshError, match="forward must come first"):
        ens.adjoint_backward(np.ones(2))
    x = _paths(p, 2, 4, dt, seed=1)
    bad = x.copy()
    bad[1, 2] = np.nan
    with pytest.raises(_lib.IeshError, match="non-finite"):
        ens.adjoint_forward(bad, 2)
    with pytest.raises(_lib.IeshError, match="ckpt_every"):
        ens.adjoint_forward(x, 0)
    cfg = get_config("c4")
    cfg["bath"]["M"] = 6
    cfg["n_elec"] = 3
    mixed = from_config(cfg, n_traj=2, precision="mixed")
    with pytest.raises(_lib.IeshError, match="FP64"):
        mixed.adjoint_forward(x, 2)
    c3 = get_config("c3")
    c3["bath"]["M"] = 6
    c3["n_elec"] = 3
    morse = from_config(c3, n_traj=2, precision="fp64")
    with pytest.raises(_lib.IeshError, match="harmonic"):
        morse.adjoint_forward(x, 2)


def test_gradient_matches_central_differences_of_the_gpu_loss():
    """Central differences (h = 1e-6 relative) of the GPU's own loss (all four
    terms) agree with its adjoint gradient to 1e-6 of the largest entry."""
    p, dt = _model(8)
    N, T, n_steps = 4, 2, 12
    x = _paths(p, T, n_steps, dt, seed=21)
    theta = adj.pack(p)
    ens = _ensemble(p, N, T, dt)
    ens.adjoint_forward(x, 5, TERMS)
    g = ens.adjoint_backward(np.ones(T))[:, :len(theta)]
    fd = np.zeros_like(g)
    from paper_2212_00518_amd.adjoint import ensemble_for
    for i in range(len(theta)):
        h = 1e-6 * max(abs(theta[i]), 1e-3)
        vals = []
        for sgn in (1.0, -1.0):
            th = theta.copy()
            th[i] += sgn * h
            e = ensemble_for(th, p.w, p.mass, N, T, dt)
            vals.append(e.adjoint_forward(x, 5, TERMS))
            e.close()
        fd[:, i] = (vals[0] - vals[1]) / (2 * h)
    for t in range(T):
        scale = np.max(np.abs(g[t]))
        err = np.abs(g[t] - fd[t])
        assert np.all(err <= 1e-6 * scale + 1e-6 * np.abs(fd[t])), (t, np.max(err), scale)


def test_full_ensemble_of_1024_paths_sampled():
    """The adjoint workload's ensemble size (1024 paths, M = 100, N = 50, all
    four loss terms) on a short prefix; two sampled paths against the oracle,
    every path's loss finite."""
    p, dt = _model(100)
    N, T, n_steps = 50, 1024, 4
    x = _paths(p, T, n_steps, dt, seed=3)
    ens = _ensemble(p, N, T, dt)
    loss = ens.adjoint_forward(x, 3, TERMS)
    w = np.linspace(0.5, 1.5, T)
    rows = ens.adjoint_backward(w)
    assert np.all(np.isfinite(loss)) and np.all(np.isfinite(rows))
    npar = adj.n_params(100)
    for t in (0, 1023):
        ref = adj.loss(p, x[t], N, dt, TERMS)
        assert abs(loss[t] - ref) <= 1e-10 * abs(ref), (t, loss[t], ref)
        _check_grad(rows[t, :npar], w[t] * adj.gradient(p, x[t], N, dt, TERMS), f"path {t}")


def test_workload_length_path_against_the_tangent_in_four_directions():
    """One path of the adjoint workload's length and model size (M = 100,
    N = 50, 2000 steps, checkpoints every 100, all four loss terms): the GPU
    loss against the oracle's loss (1e-9 relative) and the GPU gradient,
    projected on four parameter directions (eps_d, Gamma, omega and a dense
    random direction over every parameter), against the oracle's
    tangent-linear derivative in those directions (1e-7 of the projection's
    scale sum_i |g_i d_i|).  The oracle runs one process per direction."""
    import multiprocessing as mp
    import os
    p, dt = _model(100)
    N, n_steps, ckpt = 50, 2000, 100
    x = _paths(p, 1, n_steps, dt, seed=2024)
    ens = _ensemble(p, N, 1, dt)
    loss = ens.adjoint_forward(x, ckpt, TERMS)
    g = ens.adjoint_backward(np.ones(1))[0, :adj.n_params(100)]
    ens.close()
    theta = adj.pack(p)
    npar = len(theta)
    dirs = []
    for i in (0, 1, 2 + 100):   # eps_d, Gamma, omega
        e = np.zeros(npar)
        e[i] = 1.0
        dirs.append(e)
    rs = np.random.default_rng(7)
    dirs.append(rs.normal(size=npar) * np.maximum(np.abs(theta), 1e-3))
    saved = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS")}
    os.environ["OMP_NUM_THREADS"] = os.environ["OPENBLAS_NUM_THREADS"] = "1"
    try:
        with mp.get_context("spawn").Pool(len(dirs)) as pool:
            refs = pool.starmap(adj.tangent, [(p, adj.unpack(d, p.w, p.mass), x[0], N, dt, TERMS)
                                              for d in dirs])
    finally:
        for k, val in saved.items():
            if val is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = val
    ref_loss = refs[0][0]
    print(f"loss {loss[0]:.15e} oracle {ref_loss:.15e}", flush=True)
    assert abs(loss[0] - ref_loss) <= 1e-9 * abs(ref_loss)
    for d, (_, tan) in zip(dirs, refs):
        proj = float(g @ d)
        scale = float(np.sum(np.abs(g * d)))
        print(f"direction {np.flatnonzero(d)[:3]}: gpu {proj:.12e} tangent {tan:.12e} scale {scale:.3e}",
              flush=True)
        assert abs(proj - tan) <= 1e-7 * scale, (proj, tan, scale)
