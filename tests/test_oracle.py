"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix:
closed-form Laplacian spectra, dense-eigensolver brute force, exact identities of the
line search, textbook special cases (polar factor, the p = 1 two-by-two Rayleigh-Ritz),
the convergence lemmas as per-iteration invariants, and the condition numbers the
paper prints for its FD3D matrix."""
import json
import os

import numpy as np
import pytest
import scipy.linalg

from oracle import gsi_oracle as O
from paper_2306_10379_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- closed forms (test side)

def dirichlet_1d(N):
    """Eigenvalues of tridiag(-1, 2, -1) of size N: 4 sin^2(k pi / (2(N+1)))."""
    k = np.arange(1, N + 1)
    return 4.0 * np.sin(k * np.pi / (2.0 * (N + 1))) ** 2


def laplacian_spectrum(*dims):
    lam = np.zeros(1)
    for N in dims:
        lam = (lam[:, None] + dirichlet_1d(N)[None, :]).reshape(-1)
    return np.sort(lam)[::-1]


def dirichlet_vectors_2d(N, count):
    """Closed-form sine eigenvectors of the N x N 5-point Laplacian, largest eigenvalues first."""
    k = np.arange(1, N + 1)
    lam1 = dirichlet_1d(N)
    pairs = sorted(((lam1[i] + lam1[j], i, j) for i in range(N) for j in range(N)), reverse=True)
    x = np.arange(1, N + 1)
    vecs = []
    for _, i, j in pairs[:count]:
        u = np.sin(np.outer(x, [k[i]]) * np.pi / (N + 1))[:, 0]
        v = np.sin(np.outer(x, [k[j]]) * np.pi / (N + 1))[:, 0]
        w = np.outer(v, u).reshape(-1)  # index = x + N*y
        vecs.append(w / np.linalg.norm(w))
    return np.array(vecs).T


def kappa_of(lam_desc, p):
    return (lam_desc[0] - lam_desc[-1]) / (lam_desc[p - 1] - lam_desc[p])


# ---------------------------------------------------------------- generators

def test_generator_laplacian_matches_closed_form():
    for dims in [(5, 6), (4, 3, 5)]:
        A = I.laplacian_2d(*dims) if len(dims) == 2 else I.laplacian_3d(*dims)
        d = A.to_dense()
        assert np.allclose(d, d.T)
        w = np.sort(np.linalg.eigvalsh(d))[::-1]
        assert np.allclose(w, laplacian_spectrum(*dims), atol=1e-12)


def test_fd3d_kappa_reproduces_printed_values():
    g = json.load(open(os.path.join(GOLDEN, "fd3d_kappa.json")))
    lam = laplacian_spectrum(*g["grid"])
    for case in g["cases"]:
        spec = lam if case["type"] == "max" else np.sort(-lam)[::-1]
        kap = kappa_of(spec, case["p"])
        printed = case["kappa_printed"]
        assert float(f"{kap:.2e}") == printed, (case, kap)


# ---------------------------------------------------------------- line-search identities

def _tangent_setup(n=40, p=4, seed=3):
    A = I.random_symmetric_dense(n, seed)
    g = I.rng(seed + 1)
    X = O.orthonormalize(g.standard_normal((n, p)))
    Y = A @ X
    G, C = O.gradient(X, Y)
    Pr = g.standard_normal((n, p))
    P = Pr - X @ (X.T @ Pr)  # a tangent direction
    if np.sum(G * P) < 0:
        P = -P
    return A, X, Y, G, C, P


@pytest.mark.parametrize("use_grad", [True, False])
def test_rational_model_equals_direct_objective(use_grad):
    A, X, Y, G, C, P = _tangent_setup()
    if use_grad:
        P = G
    Z = A @ P
    b, V, al, ga, ze = O.linesearch_diagonals(C, P.T @ P, P.T @ Z, P.T @ Y)
    if use_grad:
        assert np.allclose(ze, b, rtol=1e-12, atol=1e-14)
    for mu in [0.0, 0.01, 0.3, 1.7, 25.0]:
        Xm, _ = O.retraction(X, P, mu, b, V)
        direct = -0.5 * np.trace(Xm.T @ A @ Xm)
        assert abs(O.phi_model(mu, al, b, ga, ze) - direct) < 1e-13 * max(1.0, abs(direct))


def test_retraction_is_polar_factor_and_orthonormal():
    A, X, Y, G, C, P = _tangent_setup(seed=5)
    b, V = np.linalg.eigh(P.T @ P)
    for mu in [0.05, 0.8, 4.0]:
        Xm, _ = O.retraction(X, P, mu, b, V)
        U, s, Wt = np.linalg.svd(X - mu * P, full_matrices=False)
        assert np.allclose(Xm, U @ Wt, atol=1e-14)
        assert np.allclose(Xm.T @ Xm, np.eye(X.shape[1]), atol=1e-14)
        # scipy's polar decomposition as a second textbook routine
        up, _ = scipy.linalg.polar(X - mu * P)
        assert np.allclose(Xm, up, atol=1e-13)


@pytest.mark.parametrize("use_grad", [True, False])
def test_derivative_matches_finite_differences(use_grad):
    A, X, Y, G, C, P = _tangent_setup(seed=7)
    if use_grad:
        P = G
    b, V, al, ga, ze = O.linesearch_diagonals(C, P.T @ P, P.T @ (A @ P), P.T @ Y)
    for mu in [0.02, 0.4, 3.0]:
        h = 1e-6 * max(1.0, mu)
        def direct(m):
            Xm, _ = O.retraction(X, P, m, b, V)
            return -0.5 * np.trace(Xm.T @ A @ Xm)
        fd = (direct(mu + h) - direct(mu - h)) / (2 * h)
        assert abs(O.dphi_model(mu, al, b, ga, ze) - fd) < 1e-7 * max(1.0, abs(fd))


def test_derivative_at_zero_is_minus_gradient_norm_and_trace_zeta():
    A, X, Y, G, C, P = _tangent_setup(seed=9)
    b, V, al, ga, ze = O.linesearch_diagonals(C, G.T @ G, G.T @ (A @ G), G.T @ Y)
    assert abs(O.dphi_model(0.0, al, b, ga, ze) + np.sum(G * G)) < 1e-13 * np.sum(G * G)
    b, V, al, ga, ze = O.linesearch_diagonals(C, P.T @ P, P.T @ (A @ P), P.T @ Y)
    assert abs(np.sum(ze) - np.sum(G * P)) < 1e-12 * abs(np.sum(G * P))


def test_gram_identities_gradient():
    # (AX)^T Pi (AX) = -G^T AX = G^T G  (Sec. 3.1) and X^T G = 0
    A, X, Y, G, C, P = _tangent_setup(seed=11)
    assert np.allclose(-G.T @ Y, G.T @ G, atol=1e-13)
    assert np.allclose(X.T @ G, 0.0, atol=1e-13)
    Xt = X - 0.3 * G
    assert np.allclose(Xt.T @ Xt, np.eye(4) + 0.09 * G.T @ G, atol=1e-13)


def test_branch_roots_stable_equal_naive_and_bracket():
    A, X, Y, G, C, P = _tangent_setup(seed=13)
    b, V, al, ga, ze = O.linesearch_diagonals(C, G.T @ G, G.T @ (A @ G), G.T @ Y)
    xi = O.branch_roots(al, b, ga, b)
    d = ga - al * b
    naive = (d + np.sqrt(d * d + 4 * b ** 3)) / (2 * b * b)  # eq. xii
    assert np.allclose(xi, naive, rtol=1e-12)
    # each root zeroes its own branch numerator
    assert np.allclose(b + d * xi - b * b * xi * xi, 0.0, atol=1e-12 * np.max(np.abs(b)))
    assert O.dphi_model(xi.min(), al, b, ga, b) <= 0.0 <= O.dphi_model(xi.max(), al, b, ga, b)


def test_get_mu_p1_equals_two_by_two_rayleigh_ritz():
    for seed in range(5):
        n = 30
        A = I.random_symmetric_dense(n, 100 + seed)
        g = I.rng(200 + seed)
        x = O.orthonormalize(g.standard_normal((n, 1)))
        G, C = O.gradient(x, A @ x)
        b, V, al, ga, ze = O.linesearch_diagonals(C, G.T @ G, G.T @ (A @ G), G.T @ (A @ x))
        mr = O.get_mu(al, b, ga, ze)
        assert mr.ok
        gn = np.linalg.norm(G)
        Q = np.hstack([x, G / gn])
        w, Z = np.linalg.eigh(Q.T @ A @ Q)
        z = Z[:, -1]
        mu_rr = -(z[1] / gn) / z[0]
        assert abs(mr.mu - mu_rr) < 1e-10 * max(1.0, abs(mu_rr))


def test_get_mu_is_minimiser_on_a_scan():
    A, X, Y, G, C, P = _tangent_setup(n=60, p=6, seed=17)
    # a conjugate-gradient-like direction: G plus a tangent momentum term
    Pcg = G + 0.5 * P * (np.linalg.norm(G) / np.linalg.norm(P))
    for Pd in (G, Pcg):
        b, V, al, ga, ze = O.linesearch_diagonals(C, Pd.T @ Pd, Pd.T @ (A @ Pd), Pd.T @ Y)
        mr = O.get_mu(al, b, ga, ze)
        assert mr.ok and mr.mu > 0
        grid = np.linspace(0, 4 * mr.hi + 1, 4001)
        vals = np.array([O.phi_model(m, al, b, ga, ze) for m in grid])
        assert O.phi_model(mr.mu, al, b, ga, ze) <= vals.min() + 1e-12 * abs(vals.min())


# ---------------------------------------------------------------- whole solves

def test_c1_rcg_matches_closed_form():
    A = I.laplacian_2d(32)
    lam = laplacian_spectrum(32, 32)
    p = 8
    for seed in range(3):
        r = O.rcg(A, I.start_block(A.n, p, seed), tol=1e-10)
        assert r.converged
        assert np.max(np.abs(r.theta - lam[:p]) / lam[:p]) < 1e-12
        # top-8 levels are a clean cut (7.8828 x2 | 7.8477): subspace vs sine eigenvectors
        U = dirichlet_vectors_2d(32, p)
        ang = O.principal_angles(r.X, U)
        delta = lam[p - 1] - lam[p]
        gF = r.rho[-1] * np.sqrt(p) * O.norm_inf(A.to_scipy())
        assert ang.max() <= 10 * gF / delta + 1e-13


def test_c1_rsd_matches_closed_form_and_invariants():
    A = I.laplacian_2d(32)
    lam = laplacian_spectrum(32, 32)
    p = 8
    r = O.rsd(A, I.start_block(A.n, p, 0), tol=1e-10, max_iter=20000)
    assert r.converged
    assert np.max(np.abs(r.theta - lam[:p]) / lam[:p]) < 1e-12
    L = lam[0] - lam[-1]
    phis = np.array(r.phi)
    gF2 = (np.array(r.rho) * np.sqrt(p) * 8.0) ** 2
    dec = phis[:-1] - phis[1:]
    # Lemma 3 (sufficient decrease) with a rounding allowance
    assert np.all(dec >= 0.4 * gF2[:-1] / L - 1e-12)


def test_rcg_vs_rcg_plus_same_iterations():
    A = I.laplacian_2d(32)
    X0 = I.start_block(A.n, 8, 1)
    r1 = O.rcg(A, X0, tol=1e-10)
    r2 = O.rcg(A, X0, tol=1e-10, recompute_ax=True)
    assert abs(r1.iters - r2.iters) <= 1
    assert np.allclose(r1.theta, r2.theta, rtol=1e-12)


@pytest.mark.parametrize("method", ["rcg", "rsd", "si"])
def test_dense_brute_force(method):
    n, p = 80, 5
    spec = np.concatenate([[9.0, 8.5, 8.0, 7.6, 7.3], np.linspace(-3.0, 6.0, n - 5)])
    A = I.random_symmetric_dense(n, 42, spec)
    X0 = I.start_block(n, p, 4)
    if method == "si":
        r = O.subspace_iteration(A, X0, tol=1e-11)
    else:
        r = getattr(O, method)(A, X0, tol=1e-11, max_iter=50000)
    assert r.converged
    w, U = np.linalg.eigh(A)
    assert np.allclose(r.theta, w[::-1][:p], rtol=1e-12, atol=1e-12)
    assert O.principal_angles(r.X, U[:, ::-1][:, :p]).max() < 1e-9


def test_smallest_via_negation():
    A = I.laplacian_2d(12)
    lam = np.sort(laplacian_spectrum(12, 12))
    r = O.rcg(A, I.start_block(A.n, 4, 2), tol=1e-11, which=-1)
    assert r.converged
    # 4 smallest: lambda_1 < lambda_2 = lambda_3 < lambda_4  (cut below lambda_5 is clean)
    assert np.allclose(r.theta, lam[:4], rtol=1e-11)


def test_per_iteration_invariants_rcg():
    A = I.laplacian_2d(20)
    Ad = A.to_scipy()
    p = 6
    lam = laplacian_spectrum(20, 20)
    L = lam[0] - lam[-1]
    X = O.orthonormalize(I.start_block(A.n, p, 3))
    Y = Ad @ X
    G_old = P_old = None
    phis = []
    for k in range(40):
        G, C = O.gradient(X, Y)
        assert np.linalg.norm(X.T @ X - np.eye(p)) < 1e-13 * np.sqrt(p)
        assert np.linalg.norm(X.T @ G) < 1e-12
        assert np.linalg.norm(G, 2) <= L / 2 + 1e-12  # Lemma 2
        phis.append(-0.5 * np.trace(C))
        if k == 0:
            P = O.tangent(X, G)
        else:
            bpr = (np.sum(G * G) - np.sum(G_old * G)) / np.sum(G_old * G_old)
            P = O.tangent(X, G + bpr * P_old)
            if np.sum(G * P) <= 0:
                P = O.tangent(X, G)
        assert np.linalg.norm(X.T @ P) < 1e-12
        Z = Ad @ P
        b, V, al, ga, ze = O.linesearch_diagonals(C, P.T @ P, P.T @ Z, P.T @ Y)
        mr = O.get_mu(al, b, ga, ze)
        X, M = O.retraction(X, P, mr.mu, b, V)
        Y = (Y - mr.mu * Z) @ M
        assert np.linalg.norm(Y - Ad @ X) < 1e-12
        G_old, P_old = G, P
    assert np.all(np.diff(phis) <= 1e-13)


def test_shift_invariance_and_basis_equivariance():
    A = I.laplacian_2d(14)
    Ad = A.to_scipy()
    p = 5
    X0 = I.start_block(A.n, p, 6)
    r0 = O.rcg(Ad, X0, tol=0.0, max_iter=25)
    import scipy.sparse as sp
    r1 = O.rcg(Ad + 3.7 * sp.identity(A.n, format="csr"), X0, tol=0.0, max_iter=25)
    W = np.linalg.qr(I.rng(9).standard_normal((p, p)))[0]
    r2 = O.rcg(Ad, X0 @ W, tol=0.0, max_iter=25)
    assert np.allclose(r0.mu, r1.mu, rtol=1e-8)
    assert np.allclose(r0.mu, r2.mu, rtol=1e-8)
    assert O.subspace_distance(r0.X, r1.X) < 1e-10
    assert O.subspace_distance(r0.X, r2.X) < 1e-10


def test_rate_matches_condition_number_estimate():
    # Sec. 6.2: asymptotic rate of RSD ~ ((kappa-1)/(kappa+1))^2 in the objective error
    A = I.laplacian_2d(32)
    lam = laplacian_spectrum(32, 32)
    p = 8
    kap = kappa_of(lam, p)
    g_sd = ((kap - 1) / (kap + 1)) ** 2
    r = O.rsd(A, I.start_block(A.n, p, 0), tol=1e-10, max_iter=20000)
    phistar = -0.5 * lam[:p].sum()
    err = np.array(r.phi) - phistar
    k = np.arange(len(err))
    sel = (err > 1e-11) & (k > 200)
    slope = np.polyfit(k[sel], np.log(err[sel]), 1)[0]
    assert abs(slope / np.log(g_sd) - 1.0) < 0.5


def test_restart_every_step_is_steepest_descent():
    """A restart sets the direction to the projected gradient (Sec. 5.1), so with a restart
    at every step (k_restart = 1) RCG takes exactly the steps of RSD; a restart period longer
    than the solve changes nothing."""
    A = I.laplacian_2d(10)
    X0 = I.start_block(A.n, 3, 7)
    r1 = O.rcg(A, X0, tol=1e-8, max_iter=5000, k_restart=1)
    rs = O.rsd(A, X0, tol=1e-8, max_iter=5000)
    assert r1.converged and rs.converged
    assert r1.iters == rs.iters and np.array_equal(r1.mu, rs.mu)
    assert all(b == 0.0 for b in r1.beta_pr)
    r0 = O.rcg(A, X0, tol=1e-8, max_iter=5000)
    rl = O.rcg(A, X0, tol=1e-8, max_iter=5000, k_restart=10 ** 6)
    assert r0.iters == rl.iters and np.array_equal(r0.mu, rl.mu)
    assert r0.iters < rs.iters


def test_cholesky_qr2():
    X = I.start_block(500, 7, 3) @ np.diag([1, 10, 100, 1e3, 1e4, 1, 2.0])
    Q = O.cholesky_qr2(X)
    assert np.linalg.norm(Q.T @ Q - np.eye(7)) < 1e-14
    assert O.subspace_distance(Q, O.orthonormalize(X)) < 1e-12
    # columns that are nearly dependent (condition 1e6 after any column scaling): one
    # Cholesky QR pass leaves Q^T Q - I near eps * kappa^2 = 1e-4, the second pass removes it
    g = np.random.default_rng(4)
    U, _ = np.linalg.qr(g.standard_normal((500, 5)))
    W, _ = np.linalg.qr(g.standard_normal((5, 5)))
    X = U @ np.diag([1.0, 1e-2, 1e-3, 1e-5, 1e-6]) @ W
    Q = O.cholesky_qr2(X)
    assert np.linalg.norm(Q.T @ Q - np.eye(5)) < 1e-13
    assert O.subspace_distance(Q, U) < 1e-8


def test_norm_inf_is_the_library_matrix_infinity_norm():
    g = np.random.default_rng(6)
    D = g.standard_normal((30, 20))
    assert np.isclose(O.norm_inf(D), np.linalg.norm(D, np.inf), rtol=1e-15)
    import scipy.sparse as sps
    B = sps.random(200, 150, density=0.05, random_state=7, format="csr")
    B.data -= 0.5
    assert np.isclose(O.norm_inf(B), np.linalg.norm(B.toarray(), np.inf), rtol=1e-15)


def test_rayleigh_ritz_on_an_invariant_subspace():
    """For a basis of an exact invariant subspace (any rotation of dense eigenvectors) the
    Ritz values are those eigenvalues, largest first, and every column residual vanishes."""
    lam = np.array([5.0, 4.0, 3.0, 2.5, 1.0, 0.5, -1.0, -2.0])
    A = I.random_symmetric_dense(8, 9, spectrum=lam)
    w, V = np.linalg.eigh(A)
    Wr, _ = np.linalg.qr(np.random.default_rng(3).standard_normal((3, 3)))
    X = V[:, [7, 5, 6]] @ Wr            # the eigenvalues 5, 3, 4 in a rotated basis
    th, Vr, res = O.rayleigh_ritz(A, X)
    assert np.allclose(th, [5.0, 4.0, 3.0], atol=1e-13)
    assert np.max(res) < 1e-13
    assert np.allclose(A @ Vr, Vr * th, atol=1e-13)


@pytest.mark.parametrize("lo,hi", [(-1.0, 1.0), (-0.5, 1.5)])
def test_chebyshev_filter_is_the_scaled_polynomial(lo, hi):
    """The recurrence equals C_d((t - c)/h) / C_d((top - c)/h) applied to the eigenvalues of a
    dense symmetric matrix (numpy's Chebyshev series evaluation, not the recurrence), for a
    centred unwanted interval and one whose centre c is not 0 (so that the shift by c enters)."""
    import numpy.polynomial.chebyshev as npc
    n, p, d = 60, 4, 9
    lam = np.concatenate([np.linspace(3.0, 2.2, p), np.linspace(hi, lo, n - p)])
    A = I.random_symmetric_dense(n, 3, spectrum=lam)
    X = I.start_block(n, p, 4)
    top = 3.0
    got = O.chebyshev_filter(A, X, A @ X, d, lo, hi, top)
    c, h = 0.5 * (lo + hi), 0.5 * (hi - lo)
    coef = np.zeros(d + 1)
    coef[d] = 1.0
    w, V = np.linalg.eigh(A)
    pw = npc.chebval((w - c) / h, coef) / npc.chebval((top - c) / h, coef)
    ref = V @ (pw[:, None] * (V.T @ X))
    assert np.allclose(got, ref, rtol=1e-10, atol=1e-12 * np.abs(ref).max())


def test_chebyshev_si_matches_brute_force_and_needs_fewer_products():
    """Chebyshev-filtered subspace iteration with the exact unwanted interval converges to
    the dense eigensolver's answer, in fewer matrix products than the monomial filter
    (the acceleration of Sec. 2.3)."""
    A = I.laplacian_2d(16)
    Ad = A.to_dense()
    w = np.sort(np.linalg.eigvalsh(Ad))[::-1]
    p = 6
    X0 = I.start_block(A.n, p, 5)
    r1 = O.subspace_iteration(A, X0, tol=1e-9, max_iter=20000)
    r8 = O.chebyshev_si(A, X0, 8, w[-1], w[p], w[0], tol=1e-9, max_iter=20000)
    assert r8.converged and r1.converged
    assert np.allclose(r8.theta, w[:p], rtol=1e-9)
    assert r8.spmm < 0.5 * r1.spmm
    # degree 1 with the interval is the shifted monomial filter: same subspace as SI on A - cI
    r_shift = O.chebyshev_si(A, X0, 1, w[-1], w[p], w[0], tol=1e-9, max_iter=20000)
    assert r_shift.converged and np.allclose(r_shift.theta, w[:p], rtol=1e-9)


class _CountingMatrix(np.ndarray):
    """A dense matrix that counts the block products A @ X it is asked for."""
    products = 0

    def __matmul__(self, other):
        if isinstance(other, np.ndarray) and other.ndim == 2 and not isinstance(other, _CountingMatrix):
            type(self).products += 1
        return np.asarray(self) @ np.asarray(other)


class _Counted:
    def __init__(self, dense):
        self.M = np.asarray(dense, dtype=np.float64).view(_CountingMatrix)

    def to_scipy(self):
        return self.M


def test_block_product_counts_are_the_products_made():
    """The SpMM counts the subspace iterations report (compared with RCG's per product with A)
    equal the block products an operator that counts its own multiplications sees, apart
    from the one Rayleigh-Ritz product at exit."""
    A = I.laplacian_2d(8).to_dense()
    w = np.sort(np.linalg.eigvalsh(A))[::-1]
    X0 = I.start_block(64, 3, 6)
    for run in (lambda op: O.subspace_iteration(op, X0, tol=1e-8, max_iter=5000),
                lambda op: O.chebyshev_si(op, X0, 5, w[-1], w[3], w[0], tol=1e-8, max_iter=5000),
                lambda op: O.rcg(op, X0, tol=1e-8, max_iter=5000)):
        _CountingMatrix.products = 0
        r = run(_Counted(A))
        assert r.converged and _CountingMatrix.products == r.spmm + 1, (_CountingMatrix.products, r.spmm)


def test_track_restarts_from_previous_subspace():
    # a repeated matrix converges at once from the previous basis, and the tracked subspace
    # of every step is the one dense diagonalization gives (independent of the start)
    mats = I.moving_well_sequence(12, 3, seed=1)
    seq = [mats[0], mats[0], mats[1], mats[2]]
    p = 4  # lambda_4 = 76.5 is well separated from lambda_5 = 93.5
    res = O.track(seq, I.start_block(144, p, 3), tol=1e-10, which=-1)
    assert all(r.converged for r in res)
    assert res[1].iters == 0
    for A, r in zip(seq, res):
        w, V = np.linalg.eigh(A.to_dense())
        assert np.allclose(np.sort(r.theta), w[:p], rtol=1e-10)
        assert O.principal_angles(r.X, V[:, :p]).max() < 1e-7
    # the moving well changes the operator only slightly: tracking costs fewer iterations
    # than the first solve from a random block
    assert res[2].iters < res[0].iters and res[3].iters < res[0].iters


def test_moving_well_sequence_shares_pattern_and_moves():
    mats = I.moving_well_sequence(10, 3, seed=0)
    for A in mats[1:]:
        assert np.array_equal(A.rowptr, mats[0].rowptr) and np.array_equal(A.colind, mats[0].colind)
    d1 = np.abs(mats[1].vals - mats[0].vals).max()
    assert 0.0 < d1 < 0.2 * np.abs(mats[0].vals).max()


def test_stencil_matrix_spectrum_is_the_closed_form():
    # the Dirichlet Laplacian on an nx x ny x nz grid has the eigenvalues
    # sum over dimensions of 4 sin^2(k pi / (2 (N + 1))), k = 1 .. N
    nx, ny, nz = 5, 4, 3
    A = O.stencil_matrix(nx, ny, nz, 6.0, -1.0).toarray()
    lam = np.zeros(1)
    for N in (nx, ny, nz):
        k = np.arange(1, N + 1)
        lam = (lam[:, None] + 4.0 * np.sin(k * np.pi / (2.0 * (N + 1))) ** 2).reshape(-1)
    # the 6 on the diagonal is 2 per dimension
    assert np.allclose(np.sort(np.linalg.eigvalsh(A)), np.sort(lam), atol=1e-12)
    # a potential on the diagonal: the trace grows by its sum, the matrix stays symmetric
    v = np.random.default_rng(0).standard_normal(nx * ny * nz)
    B = O.stencil_matrix(nx, ny, nz, 6.0, -1.0, v).toarray()
    assert np.allclose(B, B.T) and np.isclose(np.trace(B) - np.trace(A), v.sum())
    # 2D with h-scaling: the 5-point operator of the Schroedinger test problems
    N = 6
    C = O.stencil_matrix(N, N, 1, 4.0 * (N + 1) ** 2, -(N + 1) ** 2, v[:N * N])
    assert np.array_equal((C != 0).toarray(), (I.schrodinger_2d(N, None).to_scipy() != 0).toarray())


def _magnetic_ring(n, theta):
    """H = 2I - e^{i theta} S - e^{-i theta} S^T on a ring (S the cyclic shift): Hermitian,
    eigenvalues 2 - 2 cos(2 pi k / n + theta), eigenvectors the Fourier modes."""
    import scipy.sparse as sps
    S = sps.csr_matrix((np.ones(n), (np.arange(n), (np.arange(n) + 1) % n)), shape=(n, n))
    return (2.0 * sps.identity(n) - np.exp(1j * theta) * S - np.exp(-1j * theta) * S.T).tocsr()


def test_hermitian_rcg_magnetic_ring_closed_form():
    n, p, theta = 60, 4, 0.37
    H = _magnetic_ring(n, theta)
    lam = 2.0 - 2.0 * np.cos(2.0 * np.pi * np.arange(n) / n + theta)
    order = np.argsort(lam)
    g = np.random.default_rng(0)
    X0 = g.standard_normal((n, p)) + 1j * g.standard_normal((n, p))
    r = O.rcg_hermitian(H, X0, tol=1e-11, max_iter=5000, which=-1)
    assert r.converged
    assert np.allclose(r.theta, lam[order[:p]], atol=1e-10)
    F = np.exp(2j * np.pi * np.outer(np.arange(n), order[:p]) / n) / np.sqrt(n)
    assert O.principal_angles_complex(r.X, F).max() < 1e-8
    assert np.allclose(r.X.conj().T @ r.X, np.eye(p), atol=1e-12)


def test_hermitian_rcg_on_a_real_matrix_follows_the_real_iteration():
    # a real symmetric matrix with a real start block: the complex variant takes the real
    # steps (same step sizes and Ritz values as the real solver)
    A = I.laplacian_2d(10)
    X0 = I.start_block(100, 4, 2)
    rr = O.rcg(A, X0, tol=1e-10, max_iter=3000)
    rc = O.rcg_hermitian(A.to_scipy().astype(np.complex128), X0.astype(np.complex128), tol=1e-10, max_iter=3000)
    # the same step sizes until rounding differences (complex vs real kernels) grow
    assert np.allclose(rc.mu[:15], rr.mu[:15], rtol=1e-8)
    assert abs(rc.iters - rr.iters) <= 3
    assert np.allclose(rc.theta, rr.theta, rtol=1e-12)


def test_hermitian_rcg_dense_random_matches_library_eigh():
    g = np.random.default_rng(5)
    n, p = 40, 5
    B = g.standard_normal((n, n)) + 1j * g.standard_normal((n, n))
    H = 0.5 * (B + B.conj().T)
    w, V = np.linalg.eigh(H)
    X0 = g.standard_normal((n, p)) + 1j * g.standard_normal((n, p))
    r = O.rcg_hermitian(H, X0, tol=1e-12, max_iter=20000, which=1)
    assert r.converged
    assert np.allclose(r.theta, w[::-1][:p], atol=1e-10)
    assert O.principal_angles_complex(r.X, V[:, ::-1][:, :p]).max() < 1e-8


def test_splitmix64_published_outputs():
    """The first two outputs of SplitMix64 started at state 0, as published with the
    generator (0xe220a8397b1dcdaf, 0x6e789e6aa1b965f4), and a restart from any state continues
    the same stream (outputs are a function of seed + k increments)."""
    out = O.splitmix64(0, np.arange(2))
    assert [int(v) for v in out] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4]
    g = 0x9E3779B97F4A7C15
    assert int(O.splitmix64(5 * g, 0)) == int(O.splitmix64(0, 5))


def test_seeded_start_block_is_standard_normal():
    """Entries of the seeded start block: mean 0, variance 1, the standard normal distribution
    (Kolmogorov-Smirnov), no correlation between neighbouring entries, distinct seeds give
    distinct blocks, and a given seed repeats."""
    import scipy.stats
    X = O.seeded_start_block(50000, 4, 7)
    x = X.ravel()
    assert abs(x.mean()) < 0.01 and abs(x.var() - 1.0) < 0.01
    assert scipy.stats.kstest(x, "norm").pvalue > 1e-3
    assert abs(np.corrcoef(x[:-1], x[1:])[0, 1]) < 0.01
    assert np.array_equal(X, O.seeded_start_block(50000, 4, 7))
    assert not np.allclose(X[:100], O.seeded_start_block(50000, 4, 8)[:100])
    # u1 = ((o >> 11) + 1/2) 2^-53 never reaches 0 or 1: the logarithm stays finite
    assert np.isfinite(X).all()
