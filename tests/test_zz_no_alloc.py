"""The allocation-free dense eigen-solver entry point
(iesh_eigh_batched_noalloc, scratch in a fixed device array) against the
allocating one (iesh_eigh_batched), through the C ABI: identical results on
two calls in a row, the second with a smaller input; the decomposition
against numpy.linalg.eigh (eigenvalues 1e-13 of the spectral norm); batches
whose work space exceeds the fixed scratch are rejected before any device
call."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2212_00518_amd import _lib
    _lib.lib()  # fails loudly when the library is missing


def _symmetric(batch, n, seed):
    rs = np.random.default_rng(seed)
    A = rs.normal(size=(batch, n, n))
    return 0.5 * (A + np.transpose(A, (0, 2, 1)))


def _run(entry, H):
    """Decompose the host batch H on the GPU through one entry point
    (device buffers from torch); returns (lam, Q, sweeps) on the host."""
    import torch
    from paper_2212_00518_amd import _lib
    L = _lib.lib()
    b, n = H.shape[0], H.shape[1]
    dH = torch.from_numpy(H).cuda()
    lam = torch.full((b, n), np.nan, dtype=torch.float64, device="cuda")
    Q = torch.full((b, n, n), np.nan, dtype=torch.float64, device="cuda")
    sw = torch.zeros(b, dtype=torch.int32, device="cuda")
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    torch.cuda.synchronize()
    if entry == "noalloc":
        rc = L.iesh_eigh_batched_noalloc(p(dH), n, b, p(lam), p(Q), p(sw), None)
    else:
        rc = L.iesh_eigh_batched(p(dH), n, b, p(lam), p(Q), p(sw), _lib.IESH_MEM_DEVICE, None)
    assert rc == _lib.IESH_OK, L.iesh_last_error(None).decode()
    torch.cuda.synchronize()
    return lam.cpu().numpy(), Q.cpu().numpy(), sw.cpu().numpy()


@pytest.mark.parametrize("first,second", [((201, 40), (150, 12)), ((336, 37), (97, 5)),
                                          ((64, 600), (33, 7))])
def test_noalloc_matches_the_allocating_entry_point_on_two_calls(first, second):
    for k, (n, b) in enumerate((first, second)):
        H = _symmetric(b, n, seed=100 * n + b + k)
        print(f"n={n} batch={b}", flush=True)
        got = _run("noalloc", H)
        ref = _run("alloc", H)
        for a, r in zip(got, ref):
            assert np.array_equal(a, r)
        lam, Q, sw = got
        assert np.all(sw > 0)
        for i in range(0, b, max(1, b // 4)):
            nrm = np.linalg.norm(H[i], 2)
            assert np.max(np.abs(lam[i] - np.linalg.eigvalsh(H[i]))) <= 1e-13 * nrm
            assert np.max(np.abs(H[i] @ Q[i] - Q[i] * lam[i][None, :])) <= 1e-13 * nrm * np.sqrt(n)


def test_noalloc_rejects_a_batch_beyond_the_scratch_before_any_device_call():
    from paper_2212_00518_amd import _lib
    L = _lib.lib()
    cap = 64 << 20
    n = 336
    per = 2 * n * (n + 1) * 8
    b = cap // per + 1
    rc = L.iesh_eigh_batched_noalloc(ctypes.c_void_p(16), n, b, ctypes.c_void_p(16),
                                     ctypes.c_void_p(16), None, None)
    assert rc == _lib.IESH_EINVAL
    assert "exceeds the fixed scratch" in L.iesh_last_error(None).decode()
    assert L.iesh_eigh_batched_noalloc(None, 337, 1, None, None, None, None) == _lib.IESH_EINVAL
    assert L.iesh_eigh_batched_noalloc(None, 8, 0, None, None, None, None) == _lib.IESH_OK
