"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle."""
import ctypes

import numpy as np
import scipy.sparse.linalg
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


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_product_between_steps_does_not_reach_the_iteration(precision):
    """gsi_spmm (gsi_spmm_lowp on a mixed handle) between steps stages its operand in the
    engine's gradient buffer, where the retraction pass may have left the next step's gradient:
    the next step must form the gradient again (and restart the direction) rather than read the
    staged operand. Two solves that make the product with different operands at the same point
    therefore take the same steps bit for bit; each product is A W; both reach the closed-form
    eigenvalues."""
    gsi = _gsi()
    A = I.laplacian_2d(32)
    p = 8
    lam = laplacian_spectrum(32, 32)[:p]
    X0 = I.start_block(A.n, p, 5)
    kw = {"switch_tol": 1e-5} if precision == "mixed" else {}
    runs = []
    for wseed in (6, 7):
        print(f"product between steps: {precision}, operand seed {wseed}", flush=True)
        W = I.start_block(A.n, p, wseed)
        with gsi.Solver(A, X0, p, tol=1e-10, max_iter=5000, precision=precision, **kw) as s:
            s.step(10)
            Z = (s.spmm if precision == "fp64" else s.spmm_lowp)(dev(W)).cpu().numpy()
            status, iters = s.solve()
            hist = s.history()
            c = s.counters()
            ritz = s.residuals()[0]
        ref = A.to_scipy() @ W
        # float64 product to rounding; the float32 one to float32 accumulation of 5 terms
        bound = (1e-13 if precision == "fp64" else 1e-6) * np.max(np.abs(ref))
        assert np.max(np.abs(Z - ref)) <= bound
        assert status == 0
        assert c["restarts"] >= 2  # the first step and the one after the product
        if precision == "mixed":
            assert c["low_iters"] > 10  # the product fell in the float32 phase
        assert np.max(np.abs(ritz - lam) / lam) <= 1e-10
        runs.append((iters, hist))
    (i1, h1), (i2, h2) = runs
    assert i1 == i2
    assert np.array_equal(h1["mu"], h2["mu"]) and np.array_equal(h1["rho"], h2["rho"])


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


@pytest.mark.parametrize("n,p,seed", [(3000, 65, 21), (4000, 96, 22), (5000, 128, 23)])
def test_block_sizes_above_64(n, p, seed):
    """Blocks of 65 to 128 columns (float64 RCG on a CSR matrix): the 8-wave passes at width
    128 with the p x p factors read through the caches, the p x p solves with their matrices in
    the work area, two Get_Mu terms per lane and the Jacobi on 128 players. Ritz values equal
    the oracle's to 1e-10, the bases agree, and the iteration counts match."""
    A = I.spiked_sparse(n, 4, p, seed, gap=0.3)
    print(f"wide block n={n} p={p}", flush=True)
    ref, r, X, hist = _solve_both(A, p, seed, tol=1e-10, max_iter=20000)
    assert ref.converged and r.status == 0
    assert np.max(np.abs(r.ritz - ref.theta) / np.maximum(np.abs(ref.theta), 1e-300)) <= 1e-10
    assert O.principal_angles(X, ref.X).max() <= 1e-7
    assert np.allclose(X.T @ X, np.eye(p), atol=1e-12)
    assert abs(r.iters - ref.iters) <= max(3, ref.iters // 20)
    k = min(20, len(ref.mu))
    assert np.allclose(hist["mu"][:k], ref.mu[:k], rtol=1e-7)


def test_block_size_128_many_tiles_per_workgroup():
    """Width 128 with enough rows that the float64 gradient and direction passes (512
    workgroups) and the Gram pass (1024) give workgroups several tiles, idle workgroups and a
    ragged last tile: the double-buffered tiles and the next-tile loads run, which the smaller
    cases (one tile per workgroup) never reach. 40 iterations against the oracle's: the same
    step sizes, the same basis and Ritz values, orthonormal columns."""
    n, p, seed = 70_000, 128, 26
    ntiles = (n + 63) // 64
    assert ntiles > 1024 and n % 64  # more tiles than Gram workgroups; a ragged last tile
    A = I.spiked_sparse(n, 4, p, seed, gap=0.3)
    print(f"wide block many tiles n={n} p={p}", flush=True)
    ref, r, X, hist = _solve_both(A, p, seed, tol=1e-14, max_iter=40)
    assert r.iters == ref.iters == 40 and len(ref.mu) >= 40
    assert np.allclose(hist["mu"][:40], ref.mu[:40], rtol=1e-7)
    assert O.principal_angles(X, ref.X).max() <= 1e-7
    assert np.allclose(X.T @ X, np.eye(p), atol=1e-12)
    assert np.max(np.abs(r.ritz - ref.theta) / np.maximum(np.abs(ref.theta), 1e-300)) <= 1e-10


def test_block_size_above_64_rsd():
    A = I.spiked_sparse(3000, 4, 100, 24, gap=0.3)
    print("wide block rsd p=100", flush=True)
    ref, r, X, hist = _solve_both(A, 100, 24, method="rsd", tol=1e-9, max_iter=20000)
    assert ref.converged and r.status == 0
    assert np.max(np.abs(r.ritz - ref.theta) / np.maximum(np.abs(ref.theta), 1e-300)) <= 1e-9
    assert O.principal_angles(X, ref.X).max() <= 1e-6


@pytest.mark.parametrize("precision,p,sw", [("mixed", 96, 1e-5), ("bf16", 80, 1e-4)])
def test_block_sizes_above_64_mixed(precision, p, sw):
    """The low-precision engines at width 128 (float32 factors fit LDS there), then the float64
    phase: the basis meets the tolerance recomputed in float64 and the Ritz values equal the
    oracle's."""
    A = I.spiked_sparse(4000, 6, p, 25, gap=0.3)
    print(f"wide block {precision} p={p}", flush=True)
    ref, r, X, hist = _solve_both(A, p, 25, tol=1e-10, max_iter=20000, precision=precision, switch_tol=sw)
    assert ref.converged and r.status == 0
    assert r.counters["low_iters"] > 0
    assert _true_rho(A, X) <= 1.05e-10
    assert np.max(np.abs(r.ritz - ref.theta) / np.maximum(np.abs(ref.theta), 1e-300)) <= 1e-10


def _true_rho(A, X):
    """rho of a basis recomputed from scratch in float64: ||A X - X sym(X^T A X)||_F / (sqrt(p) ||A||_inf)."""
    S = A.to_scipy()
    AX = S @ X
    C = X.T @ AX
    return np.linalg.norm(AX - X @ (0.5 * (C + C.T))) / (np.sqrt(X.shape[1]) * O.norm_inf(S))


def test_mixed_precision_reaches_fp64_accuracy():
    A = I.laplacian_2d(32)
    lam = laplacian_spectrum(32, 32)[:8]
    print("C1 mixed", flush=True)
    ref, r, X, hist = _solve_both(A, 8, 0, precision="mixed", switch_tol=1e-5)
    assert r.status == 0
    assert r.counters["low_iters"] > 0
    # the float64 phase's SpMM reads float32 copies; the residual of the returned basis,
    # recomputed here in float64, meets the tolerance
    assert _true_rho(A, X) <= 1.05e-10
    assert np.max(np.abs(r.ritz - lam) / lam) <= 1e-10
    # both bases lie within Davis-Kahan distance ||G||_F / delta of the exact eigenspace
    delta = laplacian_spectrum(32, 32)[7] - laplacian_spectrum(32, 32)[8]
    nA = 8.0
    bound = (r.rho + ref.rho[-1]) * np.sqrt(8) * nA / delta
    assert O.principal_angles(X, ref.X).max() <= bound


def _schrodinger_batch(count, seed, nmin=8, nmax=24, pmin=2, pmax=12):
    g = I.rng(seed)
    mats, X0s, ps = [], [], []
    for i in range(count):
        N = int(g.integers(nmin, nmax + 1))
        p = int(g.integers(pmin, pmax + 1))
        A = I.schrodinger_2d(N, I.random_wells(seed * 1000 + i))
        mats.append(A)
        ps.append(p)
        X0s.append(I.start_block(A.n, p, seed * 1000 + 500 + i))
    return mats, X0s, ps


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batched_matches_single_problem_oracle(precision):
    """Every problem of a batch with ragged n (tails of 64-row tiles) and p on both sides
    of 16 matches the oracle's Ritz values and subspace; the float32 phase followed by
    float64 refinement reaches the same accuracy as float64 throughout."""
    gsi = _gsi()
    mats, X0s, ps = _schrodinger_batch(12, 5, pmax=30)
    tol = 1e-10
    print(f"batched {precision}: ns={[A.n for A in mats]} ps={ps}", flush=True)
    with gsi.BatchedSolver(mats, X0s, ps, which=-1, precision=precision, tol=tol, max_iter=20000,
                           switch_tol=1e-5) as b:
        st, iters, status = b.solve()
        tb, tsw, te, iters_low, team = b.timeline()
        assert np.all(team == 1)  # every problem is below two tiles per member
        assert np.all(te >= tsw) and np.all(tsw >= tb)
        if precision == "mixed":
            assert np.all(iters_low > 0) and np.all(iters_low <= iters)
        else:
            assert np.all(iters_low == 0)
        pt = b.pass_times()
        assert pt.shape == (len(ps), len(gsi.PASSES)) and np.all(pt >= 0)
        assert np.all(pt.sum(axis=1) <= (te - tb) * 1.001 + 1.0)
        for i, (A, X0, p) in enumerate(zip(mats, X0s, ps)):
            ritz, rho, _ = b.results(i)
            theta = -ritz  # the solver ran on -A: its largest Ritz values are -(smallest of A)
            w = np.linalg.eigh(A.to_dense())[0][:p]
            assert status[i] == 1, (i, status[i], rho)
            assert rho <= tol
            ref = O.rcg(A, X0, tol=tol, which=-1, max_iter=20000)
            assert np.max(np.abs(theta - ref.theta) / np.abs(ref.theta)) <= 1e-10
            assert np.max(np.abs(theta - w) / np.abs(w)) <= 1e-10
            X = b.get_x(i).cpu().numpy()
            delta = np.linalg.eigh(A.to_dense())[0][p] - w[-1]
            nA = O.norm_inf(A.to_scipy())
            bound = (rho + ref.rho[-1]) * np.sqrt(p) * nA / delta
            assert O.principal_angles(X, ref.X).max() <= max(bound, 1e-12)
            if precision == "fp64":
                # float64 blocks follow the oracle's iteration: same iteration count within
                # a few steps (rounding differs, the path is the same)
                assert abs(iters[i] - ref.iters) <= max(5, 0.1 * ref.iters), (i, iters[i], ref.iters)


def test_batched_extreme_block_sizes_and_batch_of_one():
    """The ends of the batched ranges: p = 32 on a 36-row problem (one tile, p close to n),
    p = 1 on 4096 and on 81 rows; solved together and as batches of one, each result
    matches the oracle and the dense eigensolver. An empty batch and p = 33 are rejected."""
    gsi = _gsi()
    cases = [(6, 32, 41), (64, 1, 42), (9, 1, 43)]
    mats = [I.schrodinger_2d(N, I.random_wells(seed)) for N, _, seed in cases]
    ps = [p for _, p, _ in cases]
    X0s = [I.start_block(A.n, p, seed + 100) for A, (_, p, seed) in zip(mats, cases)]
    tol = 1e-10
    refs = [O.rcg(A, X0, tol=tol, which=-1, max_iter=30000) for A, X0 in zip(mats, X0s)]
    for sel in ([0, 1, 2], [0], [1]):
        print(f"batched extremes: problems {sel}", flush=True)
        with gsi.BatchedSolver([mats[i] for i in sel], [X0s[i] for i in sel], [ps[i] for i in sel], which=-1,
                               precision="fp64", tol=tol, max_iter=30000) as b:
            st, iters, status = b.solve()
            assert st == gsi.GSI_OK and np.all(status == 1)
            for j, i in enumerate(sel):
                A, p, ref = mats[i], ps[i], refs[i]
                ritz, rho, _ = b.results(j)
                w = np.linalg.eigh(A.to_dense())[0]
                assert rho <= tol
                assert np.max(np.abs(-ritz - ref.theta) / np.abs(ref.theta)) <= 1e-10
                assert np.max(np.abs(-ritz - w[:p]) / np.abs(w[:p])) <= 1e-10
                bound = (rho + ref.rho[-1]) * np.sqrt(p) * O.norm_inf(A.to_scipy()) / (w[p] - w[p - 1])
                assert O.principal_angles(b.get_x(j).cpu().numpy(), ref.X).max() <= max(bound, 1e-12)
                assert abs(iters[j] - ref.iters) <= max(5, 0.1 * ref.iters)
    with pytest.raises(gsi.GsiError):
        gsi.BatchedSolver([], [], [], which=-1)
    with pytest.raises(gsi.GsiError):
        gsi.BatchedSolver([mats[1]], [I.start_block(mats[1].n, 33, 0)], [33], which=-1)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batched_team_matches_oracle(precision):
    """A problem of 81 row tiles that outlives the small ones recruits the idle workgroups
    (up to 5 members of at least 16 tiles): its result still matches the oracle."""
    gsi = _gsi()
    mats, X0s, ps = _schrodinger_batch(3, 13, nmin=10, nmax=14, pmin=3, pmax=6)
    big = I.schrodinger_2d(72, I.random_wells(13_777, count=(4, 6)))
    mats.insert(0, big)
    ps.insert(0, 12)
    X0s.insert(0, I.start_block(big.n, 12, 13_778))
    tol = 1e-10
    print(f"batched team {precision}: ns={[A.n for A in mats]} ps={ps}", flush=True)
    with gsi.BatchedSolver(mats, X0s, ps, which=-1, precision=precision, tol=tol, max_iter=20000,
                           switch_tol=1e-5) as b:
        st, iters, status = b.solve()
        *_, team = b.timeline()
        print(f"iters {iters} team {team}", flush=True)
        assert team[0] > 1 and np.all(team[1:] == 1)
        assert np.all(status == 1)
        for i, (A, X0, p) in enumerate(zip(mats, X0s, ps)):
            ritz, rho, _ = b.results(i)
            assert rho <= tol
            ref = O.rcg(A, X0, tol=tol, which=-1, max_iter=20000)
            assert np.max(np.abs(-ritz - ref.theta) / np.abs(ref.theta)) <= 1e-10
            w = np.sort(scipy.sparse.linalg.eigsh(A.to_scipy(), k=p + 2, which="SA", tol=1e-13)[0])
            delta = w[p] - w[p - 1]
            nA = O.norm_inf(A.to_scipy())
            bound = (rho + ref.rho[-1]) * np.sqrt(p) * nA / delta
            X = b.get_x(i).cpu().numpy()
            assert O.principal_angles(X, ref.X).max() <= max(bound, 1e-12)


def test_batched_team_wait_limit_abort_and_recovery():
    """A wait limit of 100 ns, set from the host, makes the first team barrier that is not
    met at once end the team: the solve returns GSI_EDEVICE with status 5 for the team's
    problem, while the problems solved by one workgroup finish and repeat their float64
    results bit for bit. With the limit back at 30 s the same handle solves everything,
    the big problem again by a team."""
    gsi = _gsi()
    L = gsi.load()
    mats, X0s, ps = _schrodinger_batch(3, 17, nmin=10, nmax=14, pmin=3, pmax=6)
    big = I.schrodinger_2d(72, I.random_wells(17_777, count=(4, 6)))
    mats.insert(0, big)
    ps.insert(0, 12)
    X0s.insert(0, I.start_block(big.n, 12, 17_778))
    tol = 1e-10
    with gsi.BatchedSolver(mats, X0s, ps, which=-1, precision="fp64", tol=tol, max_iter=20000) as b:
        with pytest.raises(gsi.GsiError):
            b.set_wait_limit(0.0)
        with pytest.raises(gsi.GsiError):
            b.set_wait_limit(7200.0)
        b.set_wait_limit(1e-7)
        iters = (ctypes.c_int32 * len(ps))()
        status = (ctypes.c_int32 * len(ps))()
        print("batched wait limit 1e-7 s", flush=True)
        st = L.gsi_solve_batched(b.h, iters, status)
        status = np.array(status[:])
        print(f"status {st} per problem {status}", flush=True)
        assert st == gsi.GSI_EDEVICE
        assert "team wait" in L.gsi_batched_last_error(b.h).decode()
        assert status[0] == 5 and np.all(status[1:] == 1)
        small = [b.results(i) for i in range(1, len(ps))]
        b.set_wait_limit(30.0)
        print("batched wait limit 30 s", flush=True)
        st, it2, status2 = b.solve()
        *_, team = b.timeline()
        assert st == gsi.GSI_OK and np.all(status2 == 1) and team[0] > 1
        assert np.array_equal(np.array(iters[1:]), it2[1:])
        for i in range(1, len(ps)):
            ritz, rho, _ = b.results(i)
            assert np.array_equal(ritz, small[i - 1][0]) and rho == small[i - 1][1]
        ritz, rho, _ = b.results(0)
        assert rho <= tol
        ref = O.rcg(big, X0s[0], tol=tol, which=-1, max_iter=20000)
        assert np.max(np.abs(-ritz - ref.theta) / np.abs(ref.theta)) <= 1e-10


def test_batched_repeat_solves_from_x0():
    """Each call restarts from the stored X0 and, with fixed-order reductions, repeats the
    float64 result bit for bit."""
    gsi = _gsi()
    mats, X0s, ps = _schrodinger_batch(5, 9, pmax=20)
    with gsi.BatchedSolver(mats, X0s, ps, which=-1, precision="fp64", tol=1e-10, max_iter=20000) as b:
        _, it1, _ = b.solve()
        r1 = [b.results(i)[0] for i in range(len(ps))]
        x1 = [b.get_x(i).cpu().numpy() for i in range(len(ps))]
        _, it2, _ = b.solve()
        assert np.array_equal(it1, it2)
        for i in range(len(ps)):
            assert np.array_equal(r1[i], b.results(i)[0])
            assert np.array_equal(x1[i], b.get_x(i).cpu().numpy())


def test_batched_tile_shapes_change_no_result():
    """Every built tile shape of the batched passes (tiles whose loads are issued together,
    nonzeros gathered together) reproduces the float64 results of the defaults bit for bit
    (the schedule of loads changes, not the arithmetic or its order); shapes may differ
    between problems; unknown codes are refused."""
    gsi = _gsi()
    from paper_2306_10379_amd import tuning
    mats, X0s, ps = _schrodinger_batch(8, 13, pmax=30)
    with gsi.BatchedSolver(mats, X0s, ps, which=-1, precision="fp64", tol=1e-10, max_iter=20000) as b:
        b.set_tuning(1 << 20, 1, 1 << 20)  # no teams: every problem with one workgroup
        _, it0, st0 = b.solve()
        r0 = [b.results(i)[0] for i in range(len(ps))]
        x0 = [b.get_x(i).cpu().numpy() for i in range(len(ps))]
        shapes = [dict(u=1, uu=1, ug=1, ch=4), dict(u=4, uu=2, ug=4, ch=16), dict(u=2, uu=1, ug=2, ch=8)]
        for k in range(len(shapes) + 1):
            if k < len(shapes):
                codes = [tuning.shape_code(**shapes[k])] * len(ps)
            else:  # a different shape per problem
                codes = [tuning.shape_code(**shapes[i % len(shapes)]) for i in range(len(ps))]
            print(f"shapes {codes}", flush=True)
            b.set_shapes(codes)
            _, it, st = b.solve()
            assert np.array_equal(it, it0) and np.array_equal(st, st0)
            for i in range(len(ps)):
                assert np.array_equal(r0[i], b.results(i)[0])
                assert np.array_equal(x0[i], b.get_x(i).cpu().numpy())
        for bad in (3, 3 << 4, 8 << 8, 5 << 12, 1 << 16):
            with pytest.raises(gsi.GsiError):
                b.set_shapes([bad] * len(ps))


def nA_est(A):
    return O.norm_inf(A.to_scipy())


def test_batched_full_schrodinger_batch():
    """The whole 512-problem batch of the benchmark, mixed precision: every problem's basis
    has orthonormal columns, an independently recomputed residual at the tolerance and Ritz
    values equal to the eigenvalues of X^T A X; sampled problems (the two cheapest and one
    solved by a team) match the oracle."""
    gsi = _gsi()
    mats, X0s, ps = I.schrodinger_batch(512, seed=2024)
    tol = 1e-8
    print("full batch: 512 problems, mixed", flush=True)
    with gsi.BatchedSolver(mats, X0s, ps, which=-1, precision="mixed", tol=tol, max_iter=30000,
                           switch_tol=1e-5) as b:
        st, iters, status = b.solve()
        *_, team = b.timeline()
        assert np.all(status == 1)
        print(f"iterations {iters.sum()}, teams {np.bincount(team)}", flush=True)
        for i, (A, p) in enumerate(zip(mats, ps)):
            S = A.to_scipy()
            X = b.get_x(i).cpu().numpy()
            ritz, rho, _ = b.results(i)
            AX = S @ X
            Cx = X.T @ AX
            R = AX - X @ (0.5 * (Cx + Cx.T))
            nA = O.norm_inf(S)
            assert np.linalg.norm(X.T @ X - np.eye(p)) <= 1e-12 * p
            assert np.linalg.norm(R) / (np.sqrt(p) * nA) <= 1.05 * tol + 1e-14, i
            assert np.allclose(np.sort(-ritz), np.linalg.eigvalsh(0.5 * (Cx + Cx.T)), rtol=1e-12, atol=1e-12 * nA)
        # the Ritz values are the p smallest eigenvalues: every problem a team solved plus a
        # stratified sample of the rest (>= 64 in all) against scipy's shift-invert Lanczos,
        # within the quadratic residual bound ||R||_F^2 / (lambda_{p+1} - theta_p)
        teamed = [i for i in range(len(mats)) if team[i] > 1]
        rest = [i for i in range(len(mats)) if team[i] <= 1]
        sample = sorted(set(teamed) | set(rest[::max(1, len(rest) // max(1, 64 - len(teamed)))]))
        print(f"eigsh check: {len(sample)} problems ({len(teamed)} solved by teams)", flush=True)
        assert len(sample) >= 64
        for i in sample:
            A, p = mats[i], ps[i]
            S = A.to_scipy()
            X = b.get_x(i).cpu().numpy()
            ritz, rho, _ = b.results(i)
            theta = np.sort(-ritz)
            d = S.diagonal()
            lower = float(np.min(d - (abs(S).sum(axis=1).A1 - np.abs(d)))) - 1.0  # below the spectrum
            lam = np.sort(scipy.sparse.linalg.eigsh(S.tocsc(), k=p + 1, sigma=lower, which="LM",
                                                    return_eigenvectors=False))
            AX = S @ X
            Cx = X.T @ AX
            nR = np.linalg.norm(AX - X @ (0.5 * (Cx + Cx.T)))
            bound = nR ** 2 / (lam[p] - theta[-1]) + 1e-12 * O.norm_inf(S)
            assert lam[p] - theta[-1] > 0.0, i
            assert np.max(np.abs(theta - lam[:p])) <= bound, (i, np.max(np.abs(theta - lam[:p])), bound)
        cost = np.array([A.n * p for A, p in zip(mats, ps)]) * iters
        teamed = [i for i in np.argsort(cost) if team[i] > 1]
        for i in list(np.argsort(cost)[:2]) + teamed[:1]:
            A, X0, p = mats[i], X0s[i], ps[i]
            print(f"oracle sample {i}: n={A.n} p={p} iters={iters[i]} team={team[i]}", flush=True)
            ref = O.rcg(A, X0, tol=tol, which=-1, max_iter=30000)
            ritz, rho, _ = b.results(i)
            assert np.max(np.abs(-ritz - ref.theta) / np.abs(ref.theta)) <= 1e-9


def _round_bf16(x):
    """float64 -> float32 -> bfloat16 (round to nearest, ties to even), returned as float64."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


@pytest.mark.parametrize("p", [8, 20, 64])
def test_spmm_bf16_matches_rounded_operator(p):
    """The low-precision SpMM of the bfloat16 mode: values and the block rounded to bfloat16,
    products exact in float32, float32 accumulation. Reference: the same roundings in NumPy,
    exact products and sums in float64; bound: float32 accumulation of at most 32 terms."""
    gsi = _gsi()
    A = I.spiked_sparse(3000, 12, max(p, 2), 3)
    W = I.start_block(A.n, p, 4)
    print(f"bf16 spmm n={A.n} nnz={A.nnz} p={p}", flush=True)
    with gsi.Solver(A, W, p, max_iter=1, precision="bf16") as s:
        Z = s.spmm_lowp(dev(W)).cpu().numpy()
    S16 = A.to_scipy().copy()
    S16.data = _round_bf16(S16.data)
    W16 = _round_bf16(W)
    ref = S16 @ W16
    absS = S16.copy()
    absS.data = np.abs(absS.data)
    bound = 32 * 2.0 ** -24 * (absS @ np.abs(W16)) + 1e-30
    assert np.all(np.abs(Z - ref) <= bound)
    # and the rounding is what it claims: far from the float64 product
    assert np.max(np.abs(Z - A.to_scipy() @ W)) > 1e-5 * np.max(np.abs(ref))


def test_mixed_bf16_reaches_fp64_accuracy():
    """Spiked sparse matrix with random columns (the C3 family, small): bfloat16 SpMM phase,
    then float64 refinement to rho <= 1e-10; Ritz values equal the oracle's to 1e-10."""
    A = I.spiked_sparse(6000, 12, 16, 5, gap=2e-2)
    print(f"bf16 mixed n={A.n} nnz={A.nnz} p=16", flush=True)
    ref, r, X, hist = _solve_both(A, 16, 6, precision="bf16", switch_tol=1e-4)
    assert r.status == 0
    assert r.counters["low_iters"] > 0
    assert _true_rho(A, X) <= 1.05e-10
    assert np.max(np.abs(r.ritz - ref.theta) / np.abs(ref.theta)) <= 1e-10
    w = np.sort(scipy.sparse.linalg.eigsh(A.to_scipy(), k=18, which="LA", tol=1e-13)[0])[::-1]
    delta = w[15] - w[16]
    nA = O.norm_inf(A.to_scipy())
    bound = (r.rho + ref.rho[-1]) * np.sqrt(16) * nA / delta
    assert O.principal_angles(X, ref.X).max() <= max(bound, 1e-10)


def test_batched_team_policy_setter_and_results_unchanged():
    """The team policy changes who works on a problem, not what is computed: a batch with a
    team-forming problem gives oracle-equal Ritz values under two policies; invalid policies
    are rejected."""
    gsi = _gsi()
    mats, X0s, ps = _schrodinger_batch(3, 13, nmin=10, nmax=14, pmin=3, pmax=6)
    big = I.schrodinger_2d(72, I.random_wells(13_777, count=(4, 6)))
    mats.insert(0, big)
    ps.insert(0, 12)
    X0s.insert(0, I.start_block(big.n, 12, 13_778))
    ref = O.rcg(big, X0s[0], tol=1e-10, which=-1, max_iter=20000)
    with gsi.BatchedSolver(mats, X0s, ps, which=-1, precision="fp64", tol=1e-10, max_iter=20000) as b:
        with pytest.raises(gsi.GsiError):
            b.set_tuning(2, 4, 32)
        for policy in [(4, 8, 8), (32, 1, 64)]:
            b.set_tuning(*policy)
            _, iters, status = b.solve()
            *_, team = b.timeline()
            print(f"policy {policy}: team {team}", flush=True)
            assert np.all(status == 1)
            assert team[0] <= max(1, min(16, (big.n + 63) // 64 // policy[0]))
            ritz, rho, _ = b.results(0)
            assert np.max(np.abs(-ritz - ref.theta) / np.abs(ref.theta)) <= 1e-10


def test_si_monomial_and_chebyshev_match_oracle():
    # subspace iteration (Algorithm 1) with the monomial filter and with the Chebyshev filter
    # of eq. optimal_poly on the smallest eigenvalues of the 2D Laplacian: the operator solved
    # is -A, whose unwanted eigenvalues lie in [-lambda_n, -lambda_{p+1}]
    gsi = _gsi()
    N, p = 24, 6
    A = I.laplacian_2d(N)
    lam = laplacian_spectrum(N, N)
    X0 = I.start_block(A.n, p, 5)
    # monomial filter on the largest eigenvalues (which = +1)
    print("SI monomial", flush=True)
    ref = O.subspace_iteration(A, X0, tol=1e-9, max_iter=5000, which=1)
    with gsi.Solver(A, X0, p, which=1, method="si", tol=1e-9, max_iter=5000) as s:
        r = s.run()
        X = s.get_x().cpu().numpy()
        hist = s.history()
    assert r.status == 0 and ref.converged
    assert abs(r.iters - ref.iters) <= 1
    k = min(len(hist["rho"]), len(ref.rho))
    assert np.allclose(hist["rho"][:k], ref.rho[:k], rtol=1e-6, atol=1e-14)
    assert np.max(np.abs(r.ritz - lam[:p]) / lam[:p]) <= 1e-10
    assert O.principal_angles(X, ref.X).max() <= 1e-7
    # Chebyshev filters on the smallest eigenvalues (which = -1): the operator is -A, the
    # unwanted interval [-lambda_max, -lambda_{p+1}], normalized just above -lambda_min
    la = np.sort(lam)
    lo, hi, top = -la[-1] * 1.01, -la[p] * 0.999, -la[0] * 0.99
    for d in (1, 2, 8):
        print(f"SI chebyshev degree={d}", flush=True)
        ref = O.chebyshev_si(A, X0, d, lo, hi, top, tol=1e-10, max_iter=5000, which=-1)
        with gsi.Solver(A, X0, p, which=-1, method="si", tol=1e-10, max_iter=5000, cheb_degree=d, cheb_lo=lo,
                        cheb_hi=hi, cheb_top=top) as s:
            r = s.run()
            X = s.get_x().cpu().numpy()
            hist = s.history()
            cnt = s.counters()
        assert r.status == 0 and ref.converged
        assert abs(r.iters - ref.iters) <= 1
        k = min(len(hist["rho"]), len(ref.rho), 30)
        assert np.allclose(hist["rho"][:k], ref.rho[:k], rtol=1e-6, atol=1e-13)
        assert np.max(np.abs(r.ritz - la[:p]) / la[:p]) <= 1e-10
        assert O.principal_angles(X, ref.X).max() <= 1e-7
        assert cnt["spmm"] == 1 + d * r.iters


def test_si_rejects_bad_filter_and_mixed_precision():
    gsi = _gsi()
    A = I.laplacian_2d(16)
    X0 = I.start_block(A.n, 4, 0)
    with pytest.raises(gsi.GsiError):
        gsi.Solver(A, X0, 4, method="si", cheb_degree=4, cheb_lo=1.0, cheb_hi=0.5, cheb_top=2.0)
    with pytest.raises(gsi.GsiError):
        gsi.Solver(A, X0, 4, method="si", precision="mixed")


def test_tracking_sequence_matches_oracle_chain():
    # subspace tracking: each matrix of a slowly varying sequence is solved from the basis of
    # the previous one, through gsi_set_values on one handle; the oracle runs its own chain
    gsi = _gsi()
    N, p, steps = 40, 8, 5
    mats = I.moving_well_sequence(N, steps, seed=4)
    X0 = I.start_block(N * N, p, 9)
    print(f"tracking N={N} p={p} steps={steps}", flush=True)
    ref = O.track(mats, X0, tol=1e-10, max_iter=20000, which=-1)
    iters = []
    with gsi.Solver(mats[0], X0, p, which=-1, tol=1e-10, max_iter=20000) as s:
        for t, A in enumerate(mats):
            if t:
                s.set_values(A.vals)
            r = s.run()
            X = s.get_x().cpu().numpy()
            assert r.status == 0, t
            w = np.linalg.eigvalsh(A.to_dense())[:p]
            assert np.max(np.abs(r.ritz - w) / np.abs(w)) <= 1e-9, t
            assert np.max(np.abs(r.ritz - ref[t].theta) / np.abs(w)) <= 1e-9, t
            assert O.principal_angles(X, ref[t].X).max() <= 1e-6, t
            assert _true_rho(A, X) <= 1.05e-10, t
            iters.append(r.iters)
        # a non-finite value is refused and the handle keeps working on the old values
        bad = np.array(mats[-1].vals)
        bad[7] = np.nan
        with pytest.raises(gsi.GsiError):
            s.set_values(bad)
        s.set_x0(X0)
        r = s.run()
        assert r.status == 0
        assert np.allclose(r.ritz, np.linalg.eigvalsh(mats[-1].to_dense())[:p], rtol=1e-9)
    print("iterations per step", iters, "oracle", [x.iters for x in ref], flush=True)
    assert all(i < iters[0] for i in iters[1:])
    assert all(abs(i - x.iters) <= max(5, x.iters // 5) for i, x in zip(iters, ref))


@pytest.mark.parametrize("n,p,seed", [(1000, 13, 21), (777, 1, 22), (2049, 64, 23)])
def test_si_chebyshev_ragged_shapes(n, p, seed):
    # ragged n (a partial last tile), p not a multiple of 16, p = 1 and p = 64; the filter
    # interval from the dense spectrum of the operator solved (+A, largest eigenvalues)
    gsi = _gsi()
    A = I.spiked_sparse(n, 4, p, seed, gap=0.3)
    lam = np.sort(np.linalg.eigvalsh(A.to_dense()))[::-1]
    lo, hi, top = lam[-1] - 0.01, lam[p] + 1e-3 * abs(lam[p]), lam[0] + 0.01
    X0 = I.start_block(n, p, seed)
    print(f"SI ragged n={n} p={p}", flush=True)
    ref = O.chebyshev_si(A, X0, 10, lo, hi, top, tol=1e-10, max_iter=3000, which=1)
    with gsi.Solver(A, X0, p, which=1, method="si", tol=1e-10, max_iter=3000, cheb_degree=10, cheb_lo=lo,
                    cheb_hi=hi, cheb_top=top) as s:
        r = s.run()
        X = s.get_x().cpu().numpy()
        hist = s.history()
    assert r.status == 0 and ref.converged
    assert abs(r.iters - ref.iters) <= 1
    k = min(len(hist["rho"]), len(ref.rho), 20)
    assert np.allclose(hist["rho"][:k], ref.rho[:k], rtol=1e-6, atol=1e-13)
    assert np.max(np.abs(r.ritz - lam[:p]) / np.abs(lam[:p])) <= 1e-10
    assert O.principal_angles(X, ref.X).max() <= 1e-7


def test_tracking_in_mixed_precision_reaches_fp64_accuracy():
    gsi = _gsi()
    N, p, steps = 32, 6, 3
    mats = I.moving_well_sequence(N, steps, seed=7)
    X0 = I.start_block(N * N, p, 3)
    print("tracking mixed", flush=True)
    with gsi.Solver(mats[0], X0, p, which=-1, tol=1e-10, max_iter=20000, precision="mixed") as s:
        for t, A in enumerate(mats):
            if t:
                s.set_values(A.vals)
            r = s.run()
            X = s.get_x().cpu().numpy()
            assert r.status == 0, t
            w = np.linalg.eigvalsh(A.to_dense())[:p]
            assert np.max(np.abs(r.ritz - w) / np.abs(w)) <= 1e-9, t
            assert _true_rho(A, X) <= 1.05e-10, t


@pytest.mark.parametrize("p", [33, 40, 48, 57])
def test_block_sizes_between_32_and_64(p):
    # p in 33..64 runs in the 64-column kernels with zero padding columns
    gsi = _gsi()
    n = 1500
    A = I.spiked_sparse(n, 4, p, 30 + p, gap=0.3)
    X0 = I.start_block(n, p, p)
    print(f"p={p}", flush=True)
    ref = O.rcg(A, X0, tol=1e-10, max_iter=5000)
    with gsi.Solver(A, X0, p, tol=1e-10, max_iter=5000) as s:
        r = s.run()
        X = s.get_x().cpu().numpy()
    assert r.status == 0
    assert np.max(np.abs(r.ritz - ref.theta) / np.abs(ref.theta)) <= 1e-10
    assert O.principal_angles(X, ref.X).max() <= 1e-7


def test_symmetry_check_on_request():
    gsi = _gsi()
    A = I.spiked_sparse(600, 4, 4, 3, gap=0.3)
    X0 = I.start_block(A.n, 4, 0)
    print("symmetry check", flush=True)
    with gsi.Solver(A, X0, 4, check_symmetric=True) as s:
        assert s.run().status == 0
    B = I.CSR(n=A.n, rowptr=A.rowptr.copy(), colind=A.colind.copy(), vals=A.vals.copy())
    # change one off-diagonal value only on one side
    r = 5
    k = next(k for k in range(B.rowptr[r], B.rowptr[r + 1]) if B.colind[k] != r)
    B.vals[k] += 1e-3
    with pytest.raises(gsi.GsiError):
        gsi.Solver(B, X0, 4, check_symmetric=True)
    # a complex Hermitian matrix passes through its real embedding; a non-Hermitian one fails
    H = I.magnetic_lattice(12, seed=2)
    Z0 = np.random.default_rng(1).standard_normal((144, 3)) + 0j
    with gsi.HermitianSolver(H, Z0, 3, check_symmetric=True) as s:
        assert s.run()[0] == 0
    H2 = H.tolil()
    H2[0, 1] = H2[0, 1] * np.exp(0.1j)
    with pytest.raises(gsi.GsiError):
        gsi.HermitianSolver(H2.tocsr(), Z0, 3, check_symmetric=True)


@pytest.mark.parametrize("precision", ["mixed", "bf16"])
def test_mixed_precision_at_64_columns(precision):
    # p = 50 (64 columns), tol 1e-10: after a bfloat16 phase that stops at rho ~ 2e-4 the
    # float32-input SpMM of the float64 phase stalls near 2e-10; the stall drops it to the
    # float64 SpMM, which reaches the tolerance
    gsi = _gsi()
    n, p = 4097, 50
    A = I.spiked_sparse(n, 4, p, 61, gap=0.3)
    X0 = I.start_block(n, p, 62)
    print(f"mixed {precision} p={p}", flush=True)
    ref = O.rcg(A, X0, tol=1e-10, max_iter=5000)
    with gsi.Solver(A, X0, p, tol=1e-10, max_iter=5000, precision=precision, switch_tol=1e-5) as s:
        r = s.run()
        X = s.get_x().cpu().numpy()
        c = s.counters()
    print(f"  iterations {r.iters} (low {c['low_iters']}), oracle {ref.iters}", flush=True)
    assert r.status == 0
    assert c["low_iters"] > 0 and r.iters > c["low_iters"]
    assert np.max(np.abs(r.ritz - ref.theta) / np.abs(ref.theta)) <= 1e-10
    assert _true_rho(A, X) <= 1.05e-10
    gap = float(np.min(np.abs(ref.theta[-1] - np.sort(np.linalg.eigvalsh(A.to_dense()))[::-1][p])))
    assert O.principal_angles(X, ref.X).max() <= 10 * 1e-10 * O.norm_inf(A.to_scipy()) / gap


def test_solver_options_explicit_grams_restarts_graph_and_timing():
    # explicit C and W Grams in the retraction pass, periodic CG restarts (the k_restart = 75
    # setting of Sec. 6.2), launches without a graph, and the per-pass timing mode
    gsi = _gsi()
    A = I.laplacian_2d(32)
    p = 8
    X0 = I.start_block(A.n, p, 2)
    lam = laplacian_spectrum(32, 32)[:p]
    print("options: explicit_c", flush=True)
    ref = O.rcg(A, X0, tol=1e-10, max_iter=20000)
    with gsi.Solver(A, X0, p, tol=1e-10, explicit_c=True) as s:
        r = s.run()
        X = s.get_x().cpu().numpy()
    assert r.status == 0
    assert np.max(np.abs(r.ritz - lam) / lam) <= 1e-10
    assert O.principal_angles(X, ref.X).max() <= 1e-8
    assert abs(r.iters - ref.iters) <= max(3, ref.iters // 20)
    print("options: k_restart", flush=True)
    ref75 = O.rcg(A, X0, tol=1e-10, max_iter=20000, k_restart=75)
    with gsi.Solver(A, X0, p, tol=1e-10, k_restart=75) as s:
        r = s.run()
        hist = s.history()
        c = s.counters()
    assert r.status == 0
    assert np.max(np.abs(r.ritz - lam) / lam) <= 1e-10
    assert c["restarts"] >= r.iters // 75
    k = min(100, len(ref75.mu))  # past the first periodic restart at k = 75
    assert np.allclose(hist["mu"][:k], ref75.mu[:k], rtol=1e-6)
    print("options: graph off, timing mode", flush=True)
    runs = []
    for graph, timing in ((True, False), (False, False), (True, True)):
        with gsi.Solver(A, X0, p, tol=1e-10, use_graph=graph) as s:
            if timing:
                s.pass_times(1)
            r = s.run()
            runs.append((r.iters, s.get_x().cpu().numpy()))
            if timing:
                pt = s.pass_times(0)
                assert pt["spmm"][1] >= r.iters and pt["grad"][0] > 0.0
    assert runs[0][0] == runs[1][0] == runs[2][0]
    assert np.array_equal(runs[0][1], runs[1][1]) and np.array_equal(runs[0][1], runs[2][1])


def test_degenerate_inputs():
    """Cases the method degenerates on. A = 3 I: every subspace is invariant, the gradient
    vanishes at the start, so the solve stops at iteration 0 with Ritz values 3 and the span
    of X0. Empty rows (every third row of a diagonal matrix stores nothing, spread over
    several tiles and a ragged tail): the dominant subspace is spanned by unit vectors with
    the closed-form eigenvalues. Rank-deficient and zero start blocks are rejected with a
    status (the Cholesky QR of X0 fails), not a crash."""
    gsi = _gsi()
    n, p = 500, 8
    eye = I.CSR(n=n, rowptr=np.arange(n + 1, dtype=np.int32), colind=np.arange(n, dtype=np.int32),
                vals=np.full(n, 3.0))
    X0 = I.start_block(n, p, 31)
    print("degenerate: 3 I", flush=True)
    with gsi.Solver(eye, X0, p, tol=1e-10) as s:
        r = s.run()
        X = s.get_x().cpu().numpy()
    assert r.status == 0 and r.iters == 0
    assert np.max(np.abs(r.ritz - 3.0)) <= 1e-13
    assert O.principal_angles(X, np.linalg.qr(X0)[0]).max() <= 1e-12
    # empty rows
    n = 400
    stored = [r_ for r_ in range(n) if r_ % 3 != 1]
    rowptr = np.zeros(n + 1, dtype=np.int32)
    for r_ in range(n):
        rowptr[r_ + 1] = rowptr[r_] + (1 if r_ % 3 != 1 else 0)
    B = I.CSR(n=n, rowptr=rowptr, colind=np.array(stored, dtype=np.int32),
              vals=np.array([1.0 + r_ / 100.0 for r_ in stored]))
    X0 = I.start_block(n, 6, 32)
    print("degenerate: empty rows", flush=True)
    with gsi.Solver(B, X0, 6, tol=1e-10, max_iter=20000) as s:
        Z = s.spmm(dev(X0)).cpu().numpy()
        r = s.run()
        X = s.get_x().cpu().numpy()
    assert np.array_equal(Z[1::3], np.zeros_like(Z[1::3]))
    assert np.max(np.abs(Z - B.to_scipy() @ X0)) <= 1e-14
    top = sorted(stored)[-6:][::-1]
    assert r.status == 0
    assert np.max(np.abs(r.ritz - np.array([1.0 + t / 100.0 for t in top]))) <= 1e-10 * 5
    E = np.zeros((n, 6))
    E[top, np.arange(6)] = 1.0
    assert O.principal_angles(X, E).max() <= 1e-7
    ref = O.rcg(B, X0, tol=1e-10, max_iter=20000)
    assert abs(r.iters - ref.iters) <= max(5, ref.iters // 10)
    # start blocks without full column rank
    X0 = I.start_block(n, 6, 33)
    X0[:, 5] = X0[:, 2]
    for bad in (X0, np.zeros((n, 6))):
        with pytest.raises(gsi.GsiError) as e:
            gsi.Solver(B, bad, 6)
        assert e.value.status == gsi.GSI_BREAKDOWN


def test_c2_full_size_properties():
    """The benchmark workload at its full size and in the benchmark's launch configuration
    (3D Laplacian 128^3, n = 2,097,152, p = 64, float64, graph launches polled every 50
    iterations, X0 seed 0), solved to rho <= 1e-9 (one decade below the benchmark's 1e-8, so
    that the quadratic Ritz error bound ||G||^2 / delta_eff, delta_eff = lambda_64 - lambda_67
    = 5.96e-4, sits below the stated 1e-10 relative tolerance). Checked on the CPU from what
    the library returns: the Ritz values against the 64 largest eigenvalues of the closed-form
    Dirichlet spectrum to 1e-10 relative, X^T X = I, the float64 residual A X - X (X^T A X)
    recomputed with scipy, the per-column residuals the library reports, and sampled rows of
    the full-size SpMM."""
    gsi = _gsi()
    N, p, tol = 128, 64, 1e-9
    print("c2 full size: building 128^3", flush=True)
    A = I.laplacian_3d(N)
    X0 = I.start_block(A.n, p, 0)
    dev = torch.device("cuda:0")
    rowptr = torch.as_tensor(A.rowptr.astype(np.int32), device=dev)
    colind = torch.as_tensor(A.colind, device=dev)
    vals = torch.as_tensor(A.vals, device=dev)
    X0d = torch.as_tensor(X0, device=dev)
    rows = np.sort(np.random.default_rng(5).choice(A.n, 64, replace=False))
    with gsi.Solver((rowptr, colind, vals, A.n), X0d, p, tol=tol, max_iter=20000, check_every=50) as s:
        Zs = s.spmm(X0d)[torch.as_tensor(rows, device=dev)].cpu().numpy()
        print("c2 full size: solving", flush=True)
        status, iters = s.solve()
        ritz, col_res, rho, _ = s.residuals()
        X = s.get_x().cpu().numpy()
    print(f"c2 full size: status {status}, {iters} iterations, rho {rho:.3e}", flush=True)
    As = A.to_scipy()
    ref = As[rows] @ X0
    assert np.max(np.abs(Zs - ref)) <= 1e-13 * np.max(np.abs(ref))
    assert status == gsi.GSI_OK and rho <= tol
    # the 64 largest sums of three one-dimensional eigenvalues 4 sin^2(k pi / (2 (N + 1)))
    lam1 = np.sort(4.0 * np.sin(np.arange(1, N + 1) * np.pi / (2 * (N + 1))) ** 2)[-p:]
    top = np.sort((lam1[:, None, None] + lam1[None, :, None] + lam1[None, None, :]).ravel())[::-1][:p]
    AX = As @ X
    C = X.T @ AX
    R = AX - X @ C
    nR = np.linalg.norm(R)
    assert np.max(np.abs(X.T @ X - np.eye(p))) <= 1e-12
    assert nR / (np.sqrt(p) * O.norm_inf(As)) <= 1.05 * tol
    # each Ritz value lies within the residual norm of an eigenvalue; the subspace found is
    # the dominant one, so the sorted values pair with the largest eigenvalues
    assert np.max(np.abs(ritz - top)) <= nR, (np.max(np.abs(ritz - top)), nR)
    rel = np.max(np.abs(ritz - top) / top)
    print(f"c2 full size: max Ritz rel err vs closed form {rel:.2e}", flush=True)
    assert rel <= 1e-10
    # C and the column residuals are sums over 2^21 rows: rounding of about eps * 12 * 2^10.5
    # per entry of C, and a few 1e-12 in norms of order 1e-7
    assert np.allclose(np.sort(np.linalg.eigvalsh(0.5 * (C + C.T)))[::-1], ritz, rtol=0, atol=1e-10)
    cr = np.linalg.norm(AX - X * ritz[None, :], axis=0)
    assert np.allclose(cr, col_res, rtol=1e-3, atol=1e-10)


def test_stepping_cap_and_argument_errors():
    gsi = _gsi()
    A = I.laplacian_2d(24)
    p = 6
    X0 = I.start_block(A.n, p, 4)
    print("stepping", flush=True)
    ref = O.rcg(A, X0, tol=1e-10, max_iter=20000)
    # gsi_step in pieces: the iterates follow the same step sizes as one solve
    with gsi.Solver(A, X0, p, tol=1e-10) as s:
        for _ in range(4):
            s.step(10)
        torch.cuda.synchronize()
        c = s.counters()
        hist = s.history()
        assert c["iters"] == 40
        assert np.allclose(hist["mu"][:40], ref.mu[:40], rtol=1e-7)
        r = s.run()
        assert r.status == 0 and abs(r.iters - ref.iters) <= max(3, ref.iters // 20)
    # the iteration cap: not converged, the basis still valid and its residual reported
    with gsi.Solver(A, X0, p, tol=1e-12, max_iter=15) as s:
        status, iters = s.solve()
        ritz, res, rho, phi = s.residuals()
        X = s.get_x().cpu().numpy()
    assert status == gsi.GSI_NOT_CONVERGED and iters == 15
    assert rho > 1e-12 and np.allclose(X.T @ X, np.eye(p), atol=1e-12)
    # steepest descent in mixed precision reaches the float64 answer
    print("rsd mixed", flush=True)
    refs = O.rsd(A, X0, tol=1e-9, max_iter=50000)
    with gsi.Solver(A, X0, p, tol=1e-9, method="rsd", precision="mixed", max_iter=50000) as s:
        r = s.run()
    assert r.status == 0 and np.max(np.abs(r.ritz - refs.theta) / np.abs(refs.theta)) <= 1e-9
    # argument errors come back as statuses with a message, not crashes
    for kw in (dict(p=A.n), dict(p=0), dict(p=4, which=0), dict(p=4, method=7), dict(p=4, precision=9),
               dict(p=129), dict(p=65, explicit_c=1), dict(p=65, method="si"), dict(p=4, tol=-1.0)):
        q = kw.pop("p")
        with pytest.raises(gsi.GsiError):
            gsi.Solver(A, I.start_block(A.n, max(q, 1), 0) if 0 < q <= A.n else X0, q, **kw)
    # the binding checks block sizes against the handle before passing raw pointers on
    with gsi.Solver(A, X0, p) as s:
        for bad in (np.zeros((A.n, p + 1)), np.zeros((A.n - 1, p))):
            with pytest.raises(ValueError):
                s.set_x0(bad)
            with pytest.raises(ValueError):
                s.spmm(dev(bad))
        with pytest.raises(ValueError):
            s.set_values(np.ones(len(A.vals) - 1))
    with pytest.raises(ValueError):
        gsi.Solver(A, np.zeros((A.n, p - 1)), p)


def test_seeded_start_block_drawn_on_the_device():
    """gsi_create with X0 = NULL draws the start block on the device from the option x0_seed
    (SplitMix64 outputs through Box-Muller, as stated in gsi.h); the oracle's own
    implementation of the same definition gives the same block: after the orthonormalization
    both sides apply (two Cholesky QR passes) the bases agree element by element. The C1 solve
    from the drawn block matches the oracle's solve from its block. The grid-stride draw is
    exercised with a block of more entries than one pass of the draw covers."""
    gsi = _gsi()
    A = I.laplacian_2d(32)
    p, seed = 8, 12345
    Xo = O.seeded_start_block(A.n, p, seed)
    print("seeded X0: C1", flush=True)
    with gsi.Solver(A, None, p, x0_seed=seed, tol=1e-10, max_iter=20000) as s:
        X = s.get_x().cpu().numpy()
        assert np.max(np.abs(X - O.cholesky_qr2(Xo))) <= 1e-13
        r = s.run()
    ref = O.rcg(A, Xo, tol=1e-10, max_iter=20000)
    assert r.status == 0
    assert np.max(np.abs(r.ritz - ref.theta) / np.abs(ref.theta)) <= 1e-10
    assert abs(r.iters - ref.iters) <= max(2, ref.iters // 20)
    # 64,000 rows x 13 columns: 832,000 entries, above the 524,288 threads of one draw pass
    B = I.laplacian_3d(40)
    print("seeded X0: 40^3, p=13", flush=True)
    with gsi.Solver(B, None, 13, x0_seed=2**63 + 5, max_iter=1) as s:
        X = s.get_x().cpu().numpy()
    assert np.max(np.abs(X - O.cholesky_qr2(O.seeded_start_block(B.n, 13, 2**63 + 5)))) <= 1e-13
