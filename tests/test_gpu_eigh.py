"""The dense eigen-solver (iesh_eigh_batched, batched Jacobi) against
numpy.linalg.eigh, the plain definition of the symmetric eigen-decomposition,
and against the library's arrowhead solver on Newns-Anderson matrices.

Tolerances (FP64): eigenvalues 1e-13 of the spectral norm (Jacobi is
backward stable; numpy's LAPACK solver has the same bound); residual
||HQ - Q diag(lam)|| and orthogonality defect 1e-13 relative; eigenvectors of
well-separated spectra (gaps >= 0.02 of the norm) 1e-11 after the same phase
rule on both sides.
"""
import numpy as np
import pytest

from oracle import electronic as el, models
from workloads import get_config

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2212_00518_amd import _lib
    _lib.lib()  # fails loudly when the library is missing


def _phase(Q):
    """First component above 1e-12 of each column's largest made positive."""
    Q = Q.copy()
    for j in range(Q.shape[1]):
        col = Q[:, j]
        i = np.flatnonzero(np.abs(col) > 1e-12 * np.max(np.abs(col)))[0]
        if col[i] < 0:
            Q[:, j] = -col
    return Q


def _check_decomposition(H, lam, Q):
    nrm = max(np.linalg.norm(H, 2), 1e-300)
    ref = np.linalg.eigvalsh(H)
    assert np.max(np.abs(lam - ref)) <= 1e-13 * nrm
    assert np.all(np.diff(lam) >= 0)
    assert np.max(np.abs(H @ Q - Q * lam[None, :])) <= 1e-13 * nrm * max(1, np.sqrt(len(lam)))
    assert np.max(np.abs(Q.T @ Q - np.eye(len(lam)))) <= 1e-13 * max(1, np.sqrt(len(lam)))


@pytest.mark.parametrize("n", [1, 2, 3, 16, 33, 64, 95, 96, 97, 150, 201, 336])
def test_random_symmetric_matrices(n):
    """Orders up to 96 keep the matrix in LDS, larger ones (up to the library
    limit 336) work in a device workspace."""
    from paper_2212_00518_amd import eigh_batched
    rs = np.random.default_rng(n)
    A = rs.normal(size=(5, n, n))
    H = 0.5 * (A + np.transpose(A, (0, 2, 1)))
    lam, Q, sw = eigh_batched(H)
    assert np.all(sw > 0)
    print(f"n={n}: sweeps {sw.tolist()}", flush=True)
    for b in range(5):
        _check_decomposition(H[b], lam[b], Q[b])


@pytest.mark.parametrize("n", [8, 40, 96, 150])
def test_eigenvectors_of_separated_spectra(n):
    """H = U diag(mu) U^T with gaps of at least 0.02 between the mu: the
    eigenvectors are determined up to sign and equal U's columns."""
    from paper_2212_00518_amd import eigh_batched
    rs = np.random.default_rng(100 + n)
    U, _ = np.linalg.qr(rs.normal(size=(n, n)))
    mu = np.sort(rs.uniform(-1.0, 1.0, size=n))
    mu = np.cumsum(np.full(n, 0.02)) + np.concatenate([[0.0], np.cumsum(np.abs(np.diff(mu)))])
    H = (U * mu[None, :]) @ U.T
    H = 0.5 * (H + H.T)
    lam, Q, sw = eigh_batched(H)
    assert sw > 0
    assert np.max(np.abs(lam - mu)) <= 1e-13 * np.max(np.abs(mu))
    assert np.max(np.abs(Q - _phase(U))) <= 1e-11


def test_degenerate_spectra():
    """The identity needs no rotation; a matrix with a threefold and a twofold
    eigenvalue is decomposed to the same residual bounds."""
    from paper_2212_00518_amd import eigh_batched
    lam, Q, sw = eigh_batched(np.eye(10))
    assert np.array_equal(lam, np.ones(10)) and np.array_equal(Q, np.eye(10)) and sw == 1
    rs = np.random.default_rng(7)
    U, _ = np.linalg.qr(rs.normal(size=(12, 12)))
    mu = np.array([-1.0, -1.0, -1.0, 0.0, 0.2, 0.2, 0.5, 0.6, 0.7, 0.8, 0.9, 1.3])
    H = (U * mu[None, :]) @ U.T
    lam, Q, sw = eigh_batched(0.5 * (H + H.T))
    assert sw > 0
    _check_decomposition(0.5 * (H + H.T), lam, Q)


@pytest.mark.parametrize("name,M,leads", [("c1", 20, 1), ("c1", 60, 1), ("c5", 40, 2), ("c5", 94, 2),
                                           ("c2", 200, 1), ("c5", 256, 2)])
def test_newns_anderson_matrices_agree_with_the_arrowhead_solver(name, M, leads):
    """Dense Jacobi on H(x) of the double-well and the two-lead models: the
    eigenvalues equal the secular solver's (iesh_adiabatic) and the oracle's,
    and where no eigenvalue is repeated the impurity row of Q equals the
    secular solver's amplitudes."""
    from paper_2212_00518_amd import eigh_batched, from_config, pack_states
    cfg = get_config(name)
    cfg["bath"]["M"] = M
    cfg["n_elec"] = M // 2
    if leads == 2:
        cfg["bath"]["leads"] = 2
    m = models.from_config(cfg, M=M)
    rs = np.random.default_rng(M)
    T = 4
    if name == "c5":
        xs = [np.array(cfg["model"]["dof"])[:, 3] + rs.normal(0.0, 0.2, size=6) for _ in range(T)]
    else:
        xs = [np.array([x]) for x in np.linspace(-5.0, 25.0, T)]
    H = np.stack([m.H(x) for x in xs])
    lam, Q, sw = eigh_batched(H)
    assert np.all(sw > 0)
    ens = from_config(cfg, n_traj=T)
    C = np.eye(m.n, cfg["n_elec"], dtype=np.complex128)
    ens.set_state(*pack_states([(x, np.zeros_like(x), C, np.arange(cfg["n_elec"])) for x in xs],
                               ens.n_max, ens.N_max))
    lam_s, q0_s = ens.adiabatic()
    ens.close()
    for t in range(T):
        nrm = np.max(np.abs(lam[t]))
        assert np.max(np.abs(lam[t] - lam_s[t, :m.n])) <= 1e-12 * nrm
        assert np.max(np.abs(lam[t] - el.eig(H[t])[0])) <= 1e-13 * np.linalg.norm(H[t], 2)
        if leads == 1:
            assert np.max(np.abs(Q[t][0] - q0_s[t, :m.n])) <= 1e-10
        else:
            # repeated bath energies: the deflated states have no impurity part
            assert np.max(np.abs(np.abs(Q[t][0]) - np.abs(q0_s[t, :m.n]))) <= 1e-10


def test_device_pointers_give_the_host_result():
    import ctypes
    import torch
    from paper_2212_00518_amd import _lib, eigh_batched
    rs = np.random.default_rng(3)
    A = rs.normal(size=(8, 50, 50))
    H = 0.5 * (A + np.transpose(A, (0, 2, 1)))
    lam_h, Q_h, sw_h = eigh_batched(H)
    dH = torch.from_numpy(H).cuda()
    dlam = torch.zeros((8, 50), dtype=torch.float64, device="cuda")
    dQ = torch.zeros((8, 50, 50), dtype=torch.float64, device="cuda")
    dsw = torch.zeros(8, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    rc = _lib.lib().iesh_eigh_batched(ctypes.c_void_p(dH.data_ptr()), 50, 8,
                                      ctypes.c_void_p(dlam.data_ptr()), ctypes.c_void_p(dQ.data_ptr()),
                                      ctypes.c_void_p(dsw.data_ptr()), _lib.IESH_MEM_DEVICE, None)
    assert rc == _lib.IESH_OK
    torch.cuda.synchronize()
    assert np.array_equal(dlam.cpu().numpy(), lam_h)
    assert np.array_equal(dQ.cpu().numpy(), Q_h)
    assert np.array_equal(dsw.cpu().numpy(), sw_h)
