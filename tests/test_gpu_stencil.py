"""Matrix-free stencil operator (gsi_create_stencil) against the CSR path on the same matrix
and against the float64 oracle. The stencil kernel sums the same terms in the same order as
the CSR kernel, so products, iterates and iteration counts agree exactly."""
import numpy as np
import pytest
import torch

from oracle import gsi_oracle as O
from paper_2306_10379_amd import inputs as I

pytestmark = pytest.mark.gpu


def _gsi():
    from paper_2306_10379_amd import gsi
    gsi.load()
    return gsi


def _csr_of(S):
    """The same operator as a CSR input (from the input generators) and the oracle's matrix."""
    dims = tuple(d for d in (S.nx, S.ny, S.nz))
    A = I._stencil(dims, S.diag, S.off, None if S.diag_vec is None else np.asarray(S.diag_vec, dtype=np.float64))
    M = O.stencil_matrix(S.nx, S.ny, S.nz, S.diag, S.off, S.diag_vec)
    return A, M


# grids with >= 8 rows in y take the plane-marching kernel (tiles of 32 x 8 points, runs of 32
# planes): ragged tiles in x and y, one to three runs of planes, a run of one plane; lines
# (ny < 8) take the row-tile kernel
@pytest.mark.parametrize("dims,p", [((20, 17, 13), 8), ((33, 9, 1), 64), ((70, 1, 1), 5), ((16, 16, 40), 32),
                                    ((45, 23, 70), 64), ((7, 8, 2), 1), ((33, 8, 33), 17), ((40, 5, 3), 30)])
def test_stencil_spmm_equals_csr_spmm_and_operator(dims, p):
    gsi = _gsi()
    nx, ny, nz = dims
    n = nx * ny * nz
    g = np.random.default_rng(n + p)
    S = gsi.Stencil(nx, ny, nz, diag=6.0, off=-1.0, diag_vec=g.standard_normal(n))
    A, M = _csr_of(S)
    X0 = I.start_block(n, p, 1)
    W = torch.as_tensor(g.standard_normal((n, p)), device="cuda")
    print(f"stencil spmm dims={dims} p={p}", flush=True)
    with gsi.Solver(S, X0, p) as s1, gsi.Solver(A, X0, p) as s2:
        for which_sign in (1,):
            Z1 = s1.spmm(W).cpu().numpy()
            Z2 = s2.spmm(W).cpu().numpy()
    assert np.array_equal(Z1, Z2)
    ref = M @ W.cpu().numpy()
    assert np.abs(Z1 - ref).max() <= 1e-13 * np.abs(ref).max()


def test_stencil_solve_identical_to_csr_and_matches_oracle():
    gsi = _gsi()
    N, p = 48, 10
    wells = I.random_wells(5)
    v = wells.sample(N)
    h2 = float(N + 1) ** 2
    S = gsi.Stencil(N, N, 1, diag=4.0 * h2, off=-h2, diag_vec=v)
    A, M = _csr_of(S)
    X0 = I.start_block(N * N, p, 2)
    print("stencil rcg schroedinger 48^2", flush=True)
    ref = O.rcg(M, X0, tol=1e-10, max_iter=20000, which=-1)
    with gsi.Solver(S, X0, p, which=-1, tol=1e-10, max_iter=20000) as s1:
        r1 = s1.run()
        X1 = s1.get_x().cpu().numpy()
    with gsi.Solver(A, X0, p, which=-1, tol=1e-10, max_iter=20000) as s2:
        r2 = s2.run()
        X2 = s2.get_x().cpu().numpy()
    assert r1.status == 0 and r2.status == 0
    assert r1.iters == r2.iters
    assert np.array_equal(X1, X2)
    assert np.max(np.abs(r1.ritz - ref.theta) / np.abs(ref.theta)) <= 1e-10
    assert O.principal_angles(X1, ref.X).max() <= 1e-7


def test_stencil_chebyshev_si_and_tracking_identical_to_csr():
    gsi = _gsi()
    N, p = 24, 6
    S = gsi.Stencil(N, N, 1, diag=4.0, off=-1.0)
    A, M = _csr_of(S)
    lam = np.sort(np.linalg.eigvalsh(M.toarray()))
    X0 = I.start_block(N * N, p, 5)
    lo, hi, top = -lam[-1] * 1.01, -lam[p] * 0.999, -lam[0] * 0.99
    kw = dict(which=-1, method="si", tol=1e-10, max_iter=5000, cheb_degree=6, cheb_lo=lo, cheb_hi=hi, cheb_top=top)
    print("stencil chebyshev si", flush=True)
    with gsi.Solver(S, X0, p, **kw) as s1, gsi.Solver(A, X0, p, **kw) as s2:
        r1, r2 = s1.run(), s2.run()
        assert r1.status == 0 and r1.iters == r2.iters
        assert np.array_equal(s1.get_x().cpu().numpy(), s2.get_x().cpu().numpy())
        assert np.max(np.abs(r1.ritz - lam[:p]) / lam[:p]) <= 1e-10
    # tracking a changing potential: the stencil takes the n diagonal values, the CSR handle
    # the full value array of the same matrix
    print("stencil tracking", flush=True)
    with gsi.Solver(S, X0, p, which=-1, tol=1e-10) as s1, gsi.Solver(A, X0, p, which=-1, tol=1e-10) as s2:
        s1.run(), s2.run()
        for t in range(1, 4):
            v = 0.05 * t * np.sin(np.linspace(0.0, 3.0, N * N))
            S2 = gsi.Stencil(N, N, 1, diag=4.0, off=-1.0, diag_vec=v)
            A2, M2 = _csr_of(S2)
            s1.set_values(v)
            s2.set_values(A2.vals)
            r1, r2 = s1.run(), s2.run()
            assert r1.status == 0 and r1.iters == r2.iters
            assert np.array_equal(s1.get_x().cpu().numpy(), s2.get_x().cpu().numpy())
            w = np.linalg.eigvalsh(M2.toarray())[:p]
            assert np.max(np.abs(r1.ritz - w) / np.abs(w)) <= 1e-9


def test_stencil_mixed_precision_reaches_fp64_accuracy():
    gsi = _gsi()
    N, p = 40, 12
    h2 = float(N + 1) ** 2
    v = I.random_wells(8).sample(N)
    S = gsi.Stencil(N, N, 1, diag=4.0 * h2, off=-h2, diag_vec=v)
    A, M = _csr_of(S)
    X0 = I.start_block(N * N, p, 3)
    print("stencil mixed fp32", flush=True)
    ref = O.rcg(M, X0, tol=1e-10, max_iter=20000, which=-1)
    with gsi.Solver(S, X0, p, which=-1, tol=1e-10, max_iter=20000, precision="mixed", switch_tol=1e-5) as s:
        r = s.run()
        X = s.get_x().cpu().numpy()
    assert r.status == 0
    assert np.max(np.abs(r.ritz - ref.theta) / np.abs(ref.theta)) <= 1e-10
    AX = M @ X
    C = X.T @ AX
    rho = np.linalg.norm(AX - X @ (0.5 * (C + C.T))) / (np.sqrt(p) * O.norm_inf(M))
    assert rho <= 1.05e-10


def test_stencil_rejects_bad_arguments():
    gsi = _gsi()
    X0 = I.start_block(64, 4, 0)
    with pytest.raises(gsi.GsiError):
        gsi.Solver(gsi.Stencil(8, 8, 1, diag=4.0, off=-1.0), X0, 4, precision="bf16")
    with pytest.raises(gsi.GsiError):
        gsi.Solver(gsi.Stencil(8, 8, 1, diag=4.0, off=-1.0, diag_vec=np.full(64, np.inf)), X0, 4)
    with pytest.raises(gsi.GsiError):
        gsi.Solver(gsi.Stencil(0, 8, 1, diag=4.0, off=-1.0), X0, 4)


@pytest.mark.parametrize("kind", ["stencil", "csr"])
def test_automatic_recompute_choice_times_both_and_converges(kind):
    gsi = _gsi()
    N, p = 40, 8
    S = gsi.Stencil(N, N, 1, diag=4.0, off=-1.0)
    A, M = _csr_of(S)
    X0 = I.start_block(N * N, p, 4)
    print(f"auto recompute {kind}", flush=True)
    ref = O.rcg(M, X0, tol=1e-10, max_iter=20000, which=-1)
    with gsi.Solver(S if kind == "stencil" else A, X0, p, which=-1, tol=1e-10, max_iter=20000,
                    recompute_ax="auto") as s:
        r = s.run()
        choice, ms0, ms1 = s.recompute_choice()
    assert r.status == 0
    assert ms0 > 0.0 and ms1 > 0.0
    assert choice == (1 if ms1 < ms0 else 0)
    assert np.max(np.abs(r.ritz - ref.theta) / np.abs(ref.theta)) <= 1e-10
    assert abs(r.iters - ref.iters) <= max(5, ref.iters // 10)


def test_stencil_small_grid_p1_and_tail_tile():
    # a 1D grid of 130 nodes (two full tiles and a 2-row tail) and p = 1
    gsi = _gsi()
    S = gsi.Stencil(130, 1, 1, diag=2.0, off=-1.0)
    A, M = _csr_of(S)
    X0 = I.start_block(130, 1, 0)
    print("stencil 1D p=1", flush=True)
    with gsi.Solver(S, X0, 1, which=-1, tol=1e-10, max_iter=20000) as s1, \
            gsi.Solver(A, X0, 1, which=-1, tol=1e-10, max_iter=20000) as s2:
        r1, r2 = s1.run(), s2.run()
        assert r1.status == 0 and r1.iters == r2.iters
        assert np.array_equal(s1.get_x().cpu().numpy(), s2.get_x().cpu().numpy())
    lam = 2.0 - 2.0 * np.cos(np.pi / 131.0)
    assert abs(r1.ritz[0] - lam) <= 1e-10 * lam
