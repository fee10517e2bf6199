"""Parity at the benchmark's full size and on the kernel paths it takes (through the C ABI):

* the 3D Laplacian on 128^3 at the clean cut p = 60: Ritz values against the closed-form
  spectrum to 1e-10 relative and principal angles (Sec. 4.2, eq. SVD_for_principal_angles)
  to the closed-form sine eigenvectors within the Davis-Kahan bound;
* the per-iterate step sizes and residuals of RSD (Algorithm 2) and RCG (Algorithm 4) on the
  benchmark workload against the float64 oracle's (tests/golden/c2_histories.json);
* the block SpMM on a 64^3 grid (banded tile order on), CSR and matrix-free, element by
  element against scipy;
* CSR tiles holding more than 2048 nonzeros (the gathers then read the indices and values
  from memory instead of LDS), element by element and in a solve against the oracle.
"""
import json
import os

import numpy as np
import pytest

from oracle import gsi_oracle as O
from paper_2306_10379_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c2_histories.json")


def _gsi():
    from paper_2306_10379_amd import gsi
    gsi.load()
    return gsi


def _device_csr(A):
    dev = torch.device("cuda:0")
    return (torch.as_tensor(A.rowptr.astype(np.int32), device=dev), torch.as_tensor(A.colind, device=dev),
            torch.as_tensor(A.vals, device=dev), A.n)


def laplacian3d_top_modes(N, count):
    """The `count` largest eigenpairs of the 7-point Dirichlet Laplacian on N^3 (closed form):
    eigenvalues mu_a + mu_b + mu_c with mu_k = 4 sin^2(k pi / (2 (N + 1))) and eigenvectors
    s_a(x) s_b(y) s_c(z), s_k(i) = sqrt(2 / (N + 1)) sin(i k pi / (N + 1)), rows x + N y + N^2 z.
    Returns (eigenvalues of the count + 1 largest, the count eigenvectors as an n x count block)."""
    k = np.arange(1, N + 1)
    mu = 4.0 * np.sin(k * np.pi / (2.0 * (N + 1))) ** 2
    top = np.argsort(mu)[::-1][:16]  # indices k - 1 of the largest one-dimensional values
    trip = [(a, b, c) for a in top for b in top for c in top]
    lam = np.array([mu[a] + mu[b] + mu[c] for a, b, c in trip])
    order = np.argsort(lam, kind="stable")[::-1]
    i = np.arange(1, N + 1)
    s = np.sqrt(2.0 / (N + 1)) * np.sin(np.outer(i, k) * np.pi / (N + 1))  # s[:, k-1] = s_k
    Q = np.empty((N ** 3, count))
    for m in range(count):
        a, b, c = trip[order[m]]
        Q[:, m] = np.kron(s[:, c], np.kron(s[:, b], s[:, a]))
    return lam[order[:count + 1]], Q


def test_c2_clean_cut_ritz_and_principal_angles():
    """128^3, p = 60 (lambda_60 > lambda_61: a unique dominant subspace), tol 1e-9, the
    benchmark's launch configuration otherwise."""
    gsi = _gsi()
    N, p, tol = 128, 60, 1e-9
    print("c2 clean cut: building 128^3, p=60", flush=True)
    A = I.laplacian_3d(N)
    lam, Q = laplacian3d_top_modes(N, p)
    delta = lam[p - 1] - lam[p]
    assert delta > 1e-3  # a clean cut
    X0 = torch.as_tensor(I.start_block(A.n, p, 0), device="cuda")
    with gsi.Solver(_device_csr(A), X0, p, tol=tol, max_iter=20000, check_every=50) as s:
        status, iters = s.solve()
        ritz, col_res, rho, _ = s.residuals()
        X = s.get_x().cpu().numpy()
    print(f"c2 clean cut: status {status}, {iters} iterations, rho {rho:.3e}", flush=True)
    assert status == gsi.GSI_OK and rho <= tol
    As = A.to_scipy()
    AX = As @ X
    C = X.T @ AX
    nG = np.linalg.norm(AX - X @ (0.5 * (C + C.T)))
    assert np.max(np.abs(X.T @ X - np.eye(p))) <= 1e-12
    rel = np.abs(ritz - lam[:p]) / lam[:p]
    print(f"c2 clean cut: max Ritz rel err {rel.max():.2e}, ||G||_F {nG:.2e}, gap {delta:.3e}", flush=True)
    assert rel.max() <= 1e-10
    ang = O.principal_angles(X, Q)
    print(f"c2 clean cut: largest principal angle {ang.max():.2e} (bound {10 * nG / delta:.2e})", flush=True)
    assert ang.max() <= 10.0 * nG / delta


@pytest.mark.parametrize("method", ["rsd", "rcg"])
def test_c2_iterates_follow_the_oracle(method):
    """The first iterations on the benchmark workload (3D Laplacian 128^3, p = 64, X0 seed 0)
    take the oracle's step sizes and reach its residuals."""
    gsi = _gsi()
    with open(GOLDEN) as f:
        ref = json.load(f)[method]
    k = ref["iters"]
    print(f"c2 {method}: {k} iterations against the oracle", flush=True)
    A = I.laplacian_3d(128)
    X0 = torch.as_tensor(I.start_block(A.n, 64, 0), device="cuda")
    with gsi.Solver(_device_csr(A), X0, 64, method=method, tol=0.0, max_iter=k, check_every=50) as s:
        status, iters = s.solve()
        h = s.history()
    assert status == gsi.GSI_NOT_CONVERGED and iters == k
    mu, rho = np.asarray(ref["mu"]), np.asarray(ref["rho"])
    err_mu = np.max(np.abs(h["mu"][:k] - mu) / mu)
    err_rho = np.max(np.abs(h["rho"][:k + 1] - rho) / rho)
    print(f"c2 {method}: max rel diff mu {err_mu:.2e}, rho {err_rho:.2e}", flush=True)
    assert err_mu <= 1e-6 and err_rho <= 1e-6
    if method == "rcg":
        beta = np.asarray(ref["beta_pr"])
        assert np.max(np.abs(h["beta_pr"][:k] - beta)) <= 1e-6 * np.max(np.abs(beta))


def test_spmm_64cubed_banded_order_csr_and_stencil():
    """n = 262,144 rows (64 planes of 64 tiles: the banded tile order is on), p = 64 and
    p = 13: the whole product, CSR and matrix-free, against scipy."""
    gsi = _gsi()
    A = I.laplacian_3d(64)
    S = A.to_scipy()
    for p, seed in ((64, 1), (13, 2)):
        print(f"spmm 64^3 p={p}", flush=True)
        W = I.start_block(A.n, p, seed)
        ref = S @ W
        Wd = torch.as_tensor(W, device="cuda")
        with gsi.Solver(_device_csr(A), Wd, p, max_iter=1) as s:
            Zc = s.spmm(Wd).cpu().numpy()
        with gsi.Solver(gsi.Stencil(64, 64, 64, diag=6.0, off=-1.0), Wd, p, max_iter=1) as s:
            Zs = s.spmm(Wd).cpu().numpy()
        scale = np.max(np.abs(ref))
        assert np.max(np.abs(Zc - ref)) <= 1e-13 * scale
        assert np.array_equal(Zc, Zs)  # same terms, same order


def _dense_rows_matrix(n, seed):
    """Symmetric random sparse matrix whose first third of the rows hold ~80 nonzeros (a
    64-row tile there holds > 2048) and the rest ~6, plus a diagonal: both CSR paths in one
    product."""
    g = np.random.default_rng(seed)
    heavy = n // 3
    deg = np.where(np.arange(n) < heavy, 40, 3)
    rows = np.repeat(np.arange(n), deg)
    cols = g.integers(0, n, rows.size)
    vals = g.standard_normal(rows.size) / 8.0
    keep = rows != cols
    rows, cols, vals = rows[keep], cols[keep], vals[keep]
    diag = np.linspace(-1.0, 4.0, n)
    r = np.concatenate([rows, cols, np.arange(n)])
    c = np.concatenate([cols, rows, np.arange(n)])
    v = np.concatenate([vals, vals, diag])
    return I._from_coo(n, r, c, v)


def test_csr_tiles_above_the_lds_capacity():
    gsi = _gsi()
    A = _dense_rows_matrix(3001, 7)
    counts = np.diff(A.rowptr)
    per_tile = np.add.reduceat(counts, np.arange(0, A.n, 64))
    assert per_tile.max() > 2048 and per_tile.min() <= 2048  # both branches taken
    S = A.to_scipy()
    for p, seed in ((64, 3), (30, 4), (5, 5)):
        print(f"unstaged csr p={p}", flush=True)
        W = I.start_block(A.n, p, seed)
        Wd = torch.as_tensor(W, device="cuda")
        with gsi.Solver(A, Wd, p, max_iter=1) as s:
            Z = s.spmm(Wd).cpu().numpy()
        ref = S @ W
        assert np.max(np.abs(Z - ref)) <= 1e-13 * np.max(np.abs(ref))
    # a solve on it: Ritz values and subspace against the oracle
    p = 12
    X0 = I.start_block(A.n, p, 9)
    ref = O.rcg(A, X0, tol=1e-10, max_iter=20000)
    with gsi.Solver(A, X0, p, tol=1e-10, max_iter=20000) as s:
        r = s.run()
        X = s.get_x().cpu().numpy()
    assert r.status == 0
    assert np.max(np.abs(r.ritz - ref.theta) / np.abs(ref.theta)) <= 1e-10
    lam = np.linalg.eigvalsh(A.to_dense())[::-1]
    assert np.max(np.abs(r.ritz - lam[:p]) / np.abs(lam[:p])) <= 1e-10
    assert O.principal_angles(X, ref.X).max() <= 1e-6
