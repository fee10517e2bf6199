"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle."""
import numpy as np
import pytest

from oracle import gsi_oracle as O
from paper_2306_10379_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _gsi():
    from paper_2306_10379_amd import gsi
    gsi.load()
    return gsi


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), device="cuda")


def laplacian_spectrum(*dims):
    lam = np.zeros(1)
    for N in dims:
        k = np.arange(1, N + 1)
        lam = (lam[:, None] + (4.0 * np.sin(k * np.pi / (2.0 * (N + 1))) ** 2)[None, :]).reshape(-1)
    return np.sort(lam)[::-1]


def ragged_sparse(n, seed, p):
    A = I.spiked_sparse(n, 5, p, seed, gap=0.2)
    return A


@pytest.mark.parametrize("n,p,seed", [(1024, 8, 0), (1000, 13, 1), (777, 30, 2), (2049, 64, 3), (130, 1, 4)])
def test_spmm_matches_oracle_operator(n, p, seed):
    gsi = _gsi()
    print(f"spmm n={n} p={p} seed={seed}", flush=True)
    A = I.laplacian_2d(32) if n == 1024 else ragged_sparse(n, seed, max(p, 2))
    W = I.start_block(A.n, p, seed + 10)
    with gsi.Solver(A, W, p, max_iter=1) as s:
        Z = s.spmm(dev(W)).cpu().numpy()
    ref = A.to_scipy() @ W
    assert np.max(np.abs(Z - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))


def _solve_both(A, p, seed, which=1, method="rcg", tol=1e-10, max_iter=20000, **kw):
    gsi = _gsi()
    X0 = I.start_block(A.n, p, seed)
    ref = getattr(O, method)(A, X0, tol=tol, max_iter=max_iter, which=which)
    with gsi.Solver(A, X0, p, which=which, method=method, tol=tol, max_iter=max_iter, **kw) as s:
        r = s.run()
        X = s.get_x().cpu().numpy()
        hist = s.history()
    return ref, r, X, hist


def test_c1_rcg_parity_and_closed_form():
    A = I.laplacian_2d(32)
    lam = laplacian_spectrum(32, 32)[:8]
    for seed in range(3):
        print(f"C1 rcg seed={seed}", flush=True)
        ref, r, X, hist = _solve_both(A, 8, seed)
        assert r.status == 0
        assert np.max(np.abs(r.ritz - ref.theta) / np.abs(ref.theta)) <= 1e-10
        assert np.max(np.abs(r.ritz - lam) / lam) <= 1e-10
        assert O.principal_angles(X, ref.X).max() <= 1e-8
        assert abs(r.iters - ref.iters) <= max(3, ref.iters // 20)
        # the first iterates follow the oracle's: same step sizes
        k = min(20, len(ref.mu))
        assert np.allclose(hist["mu"][:k], ref.mu[:k], rtol=1e-7)


def test_c1_rsd_parity():
    A = I.laplacian_2d(32)
    print("C1 rsd", flush=True)
    ref, r, X, hist = _solve_both(A, 8, 0, method="rsd")
    assert r.status == 0
    assert np.max(np.abs(r.ritz - ref.theta) / np.abs(ref.theta)) <= 1e-10
    assert O.principal_angles(X, ref.X).max() <= 1e-7
    k = min(50, len(ref.mu))
    assert np.allclose(hist["mu"][:k], ref.mu[:k], rtol=1e-7)


def test_recompute_ax_variant_same_iterations():
    A = I.laplacian_2d(32)
    print("C1 rcg(+)", flush=True)
    ref, r, X, hist = _solve_both(A, 8, 1, recompute_ax=True)
    ref2, r2, X2, _ = _solve_both(A, 8, 1)
    assert r.status == 0 and r2.status == 0
    assert abs(r.iters - r2.iters) <= 2
    assert np.allclose(r.ritz, r2.ritz, rtol=1e-12)


@pytest.mark.parametrize("n,p,seed", [(1000, 5, 11), (1333, 13, 12), (777, 30, 13), (4097, 64, 14)])
def test_ragged_shapes_smallest_and_largest(n, p, seed):
    A = I.spiked_sparse(n, 4, p, seed, gap=0.3)
    for which in (1, -1):
        print(f"ragged n={n} p={p} which={which}", flush=True)
        ref, r, X, hist = _solve_both(A, p, seed, which=which, tol=1e-11, max_iter=20000)
        assert ref.converged and r.status == 0
        assert np.max(np.abs(r.ritz - ref.theta) / np.maximum(np.abs(ref.theta), 1e-300)) <= 1e-10
        assert O.principal_angles(X, ref.X).max() <= 1e-7


def test_mixed_precision_reaches_fp64_accuracy():
    A = I.laplacian_2d(32)
    lam = laplacian_spectrum(32, 32)[:8]
    print("C1 mixed", flush=True)
    ref, r, X, hist = _solve_both(A, 8, 0, precision="mixed", switch_tol=1e-5)
    assert r.status == 0
    assert r.counters["low_iters"] > 0
    assert np.max(np.abs(r.ritz - lam) / lam) <= 1e-10
    # both bases lie within Davis-Kahan distance ||G||_F / delta of the exact eigenspace
    delta = laplacian_spectrum(32, 32)[7] - laplacian_spectrum(32, 32)[8]
    nA = 8.0
    bound = (r.rho + ref.rho[-1]) * np.sqrt(8) * nA / delta
    assert O.principal_angles(X, ref.X).max() <= bound
