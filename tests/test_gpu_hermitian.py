"""Complex Hermitian variant (gsi_create_hermitian, real embedding on the device) against
the complex float64 oracle and closed forms."""
import numpy as np
import pytest
import scipy.sparse as sps
import torch

from oracle import gsi_oracle as O
from paper_2306_10379_amd import inputs as I

pytestmark = pytest.mark.gpu


def _gsi():
    from paper_2306_10379_amd import gsi
    gsi.load()
    return gsi


def _start(n, p, seed):
    g = np.random.default_rng(seed)
    return g.standard_normal((n, p)) + 1j * g.standard_normal((n, p))


@pytest.mark.parametrize("N,p,which", [(32, 8, -1), (24, 5, 1), (40, 16, -1)])
def test_hermitian_magnetic_lattice_matches_complex_oracle(N, p, which):
    gsi = _gsi()
    H = I.magnetic_lattice(N, flux=0.13, seed=N)
    X0 = _start(N * N, p, N + p)
    print(f"hermitian N={N} p={p} which={which}", flush=True)
    ref = O.rcg_hermitian(H, X0, tol=1e-10, max_iter=20000, which=which)
    w = np.linalg.eigvalsh(H.toarray())
    want = w[:p] if which < 0 else w[::-1][:p]
    with gsi.HermitianSolver(H, X0, p, which=which, tol=1e-10, max_iter=20000) as s:
        status, iters, ritz, X, rho = s.run()
    X = X.cpu().numpy()
    assert status == 0 and ref.converged
    assert np.max(np.abs(ritz - want) / np.abs(want)) <= 1e-9
    assert np.max(np.abs(ritz - ref.theta) / np.abs(want)) <= 1e-9
    assert np.allclose(X.conj().T @ X, np.eye(p), atol=1e-9)
    assert O.principal_angles_complex(X, ref.X).max() <= 1e-6
    # Ritz pairs: each column is an eigenvector to the residual level
    R = H @ X - X * ritz
    assert np.linalg.norm(R, axis=0).max() <= 1e-7 * np.abs(w).max()
    assert abs(iters - ref.iters) <= max(10, ref.iters // 5)


def test_hermitian_magnetic_ring_closed_form():
    gsi = _gsi()
    n, p, theta = 300, 6, 0.37
    S = sps.csr_matrix((np.ones(n), (np.arange(n), (np.arange(n) + 1) % n)), shape=(n, n))
    H = (2.0 * sps.identity(n) - np.exp(1j * theta) * S - np.exp(-1j * theta) * S.T).tocsr()
    lam = np.sort(2.0 - 2.0 * np.cos(2.0 * np.pi * np.arange(n) / n + theta))
    print("hermitian ring", flush=True)
    with gsi.HermitianSolver(H, _start(n, p, 1), p, which=-1, tol=1e-10, max_iter=20000) as s:
        status, iters, ritz, X, rho = s.run()
    assert status == 0
    assert np.allclose(ritz, lam[:p], atol=1e-9)


def test_hermitian_of_a_real_matrix_equals_real_solver():
    gsi = _gsi()
    A = I.laplacian_2d(20)
    p = 6
    X0 = I.start_block(A.n, p, 3)
    print("hermitian real matrix", flush=True)
    with gsi.Solver(A, X0, p, which=-1, tol=1e-10) as s:
        r = s.run()
    with gsi.HermitianSolver(A.to_scipy().astype(np.complex128), X0.astype(np.complex128), p, which=-1,
                             tol=1e-10) as s:
        status, iters, ritz, X, rho = s.run()
    assert status == 0 and r.status == 0
    assert np.allclose(ritz, r.ritz, rtol=1e-10)


def test_hermitian_rejects_p_above_32():
    gsi = _gsi()
    H = I.magnetic_lattice(10, seed=1)
    with pytest.raises(gsi.GsiError):
        gsi.HermitianSolver(H, _start(100, 33, 0), 33)


def test_hermitian_rejects_out_of_range_columns_and_wrong_start_block():
    """A column index of n would land in the other block of the real embedding: the library
    rejects it (GSI_EINVAL) before building the embedding; a start block of the wrong shape
    is caught by the binding."""
    import ctypes
    gsi = _gsi()
    H = sps.csr_matrix(I.magnetic_lattice(6, seed=3))
    H.sort_indices()
    n, p = H.shape[0], 3
    with pytest.raises(ValueError):
        gsi.HermitianSolver(H, _start(n, p + 1, 0), p)
    ci = H.indices.astype(np.int32).copy()
    ci[-1] = n
    rp = torch.as_tensor(H.indptr.astype(np.int32), device="cuda")
    cd = torch.as_tensor(ci, device="cuda")
    vv = torch.as_tensor(np.ascontiguousarray(H.data.astype(np.complex128)).view(np.float64), device="cuda")
    x0 = torch.as_tensor(np.ascontiguousarray(_start(n, p, 1)).view(np.float64), device="cuda")
    L = gsi.load()
    z = gsi.GsiZcsr(n=n, nnz=int(H.nnz), rowptr=rp.data_ptr(), colind=cd.data_ptr(), vals=vv.data_ptr())
    opt = gsi.options(p=p)
    h = ctypes.c_void_p()
    st = L.gsi_create_hermitian(ctypes.byref(h), ctypes.byref(z), ctypes.byref(opt), ctypes.c_void_p(x0.data_ptr()),
                                ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == gsi.GSI_EINVAL and not h.value


@pytest.mark.parametrize("N,p", [(23, 1), (23, 7)])
def test_hermitian_ragged_rows_and_p1(N, p):
    # 2n = 1058 real rows (a partial last tile), p = 1 and an odd p
    gsi = _gsi()
    H = I.magnetic_lattice(N, flux=0.21, seed=3)
    X0 = _start(N * N, p, 11)
    print(f"hermitian ragged N={N} p={p}", flush=True)
    ref = O.rcg_hermitian(H, X0, tol=1e-10, max_iter=20000, which=-1)
    w = np.linalg.eigvalsh(H.toarray())[:p]
    with gsi.HermitianSolver(H, X0, p, which=-1, tol=1e-10, max_iter=20000) as s:
        status, iters, ritz, X, rho = s.run()
    X = X.cpu().numpy()
    assert status == 0 and ref.converged
    assert np.max(np.abs(ritz - w) / np.abs(w)) <= 1e-9
    assert O.principal_angles_complex(X, ref.X).max() <= 1e-6
