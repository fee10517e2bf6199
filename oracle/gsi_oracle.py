"""Plain FP64 CPU oracle for gradient-type subspace iteration
(Alimisis, Saad, Vandereycken: "Gradient-type subspace iteration methods for the
symmetric eigenvalue problem").

TEST INFRASTRUCTURE ONLY. This module is imported by tests, by the package's smoke
check and by the benchmark's CPU-baseline leg, and by nothing else. It shares no code
with the device solver: it uses NumPy/SciPy in float64 and follows the paper's steps
in the paper's order, with library primitives (matrix products, a symmetric
eigensolver, a QR factorization, a bracketing root finder) as single steps.

Notation follows the paper:
  phi(X) = -1/2 Tr(X^T A X)                         (Sec. 2.2, eq. phi)
  G = grad phi(X) = -(A X - X C),  C = X^T A X      (Sec. 3.1, eq. gradPhi)
  X(mu) = (X - mu P) V D_mu^{-1} V^T,  P^T P = V D_beta V^T,
  D_mu = (I + mu^2 D_beta)^{1/2}                    (Sec. 3.1 eq. Ynew; Sec. 5.2 eq. Xnew_P)
  phi(X(mu)) = -1/2 sum_i (alpha_i + 2 zeta_i mu + gamma_i mu^2)/(1 + beta_i mu^2)
                                                    (Sec. 5.2 eq. phi_P; eq. phinew for P = G)
Readings of points the paper leaves open (each is also listed with the tests):
  * stop test: rho = ||G||_F / (sqrt(p) ||A||_inf); the paper's own table uses
    ||G_k||_inf / ||G_0||_inf, which is recorded too;
  * the conjugate-gradient line search diagonalizes P^T P, formed after the new
    direction P (the printed Algorithm 4 lists G^T G before P is formed);
  * beta_PR = 0 at k = 0; restart P <- G when <G, P> <= 0 or every k_restart steps;
  * every direction, restarts and steepest descent included, is formed as
    (I - X X^T)(G + beta_PR P_old), the projected update of Algorithm 4 (the projector
    is the identity on exact tangent vectors and keeps X^T X = I stable in rounding);
  * Get_Mu drops terms with beta_i <= p * eps * max(beta) (P v_i = 0 to rounding), takes
    its bracket between consecutive sorted branch roots of the convex branches
    (zeta_i > 0) around the first sign change of phi' (the minimizer nearest mu = 0:
    near-zero beta_i put roots far out, where phi' can change sign again), widens it if
    no sign change is found, and restarts with P = G when no bracket exists;
  * A X is recomputed explicitly when mu * sqrt(max beta) <= 1e3 * eps (the paper's
    "mu = O(eps_mach)"); RCG(+) recomputes it every iteration.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.optimize
import scipy.sparse as sp

EPS = np.finfo(np.float64).eps


# ----------------------------------------------------------------------------- basics

def as_operator(A):
    """Accept a scipy sparse matrix, a dense ndarray or an object with .to_scipy()."""
    if hasattr(A, "to_scipy"):
        return A.to_scipy()
    return A


def norm_inf(A) -> float:
    """Max absolute row sum of A."""
    if sp.issparse(A):
        return float(abs(A).sum(axis=1).max())
    return float(np.abs(A).sum(axis=1).max())


def phi(A, X) -> float:
    """phi(X) = -1/2 Tr(X^T A X)  (Sec. 2.2, eq. phi)."""
    return -0.5 * float(np.trace(X.T @ (A @ X)))


def orthonormalize(X0: np.ndarray) -> np.ndarray:
    """Orthonormal basis of span(X0) by Householder QR (any orthonormal basis of the
    span gives the same iterates up to a right rotation: Sec. 3, Sec. 3.1)."""
    q, _ = np.linalg.qr(X0)
    return q


def sym(M: np.ndarray) -> np.ndarray:
    return 0.5 * (M + M.T)


def gradient(X: np.ndarray, Y: np.ndarray):
    """Riemannian gradient G = -(AX - XC) with C = X^T A X (Sec. 3.1, eq. gradPhi).
    Y holds A X. Returns (G, C)."""
    C = sym(X.T @ Y)
    G = -(Y - X @ C)
    return G, C


def tangent(X: np.ndarray, D: np.ndarray) -> np.ndarray:
    """Projection (I - X X^T) D onto the tangent space at X (Sec. 3.1, eq. Tang). Every search
    direction goes through it, as the direction update of Algorithm 4 does: the polar
    retraction keeps X^T X = I only if X^T P = 0, and an unprojected G carries
    X^T G = (X^T X - I) C, which the retraction would amplify by about |1 - 2 mu lambda|."""
    return D - X @ (X.T @ D)


def rayleigh_ritz(A, X: np.ndarray):
    """Rayleigh-Ritz on span(X) for orthonormal X (Sec. 2.3, eq. rr1): eigenpairs of
    C = X^T A X, largest first. Returns (theta, ritz_vectors, residual_norms)."""
    AX = A @ X
    C = sym(X.T @ AX)
    w, U = np.linalg.eigh(C)
    w, U = w[::-1], U[:, ::-1]
    V = X @ U
    R = AX @ U - V * w
    return w, V, np.linalg.norm(R, axis=0)


def principal_angles(X: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """Principal angles between span(X) and span(Y), orthonormal X, Y
    (Sec. 4.2, eq. SVD_for_principal_angles), ascending.
    Small angles are taken from the sines (singular values of X - Y Y^T X), which
    resolve them to rounding level; arccos of the cosines alone cannot resolve angles
    below about sqrt(eps)."""
    c = np.sort(np.linalg.svd(Y.T @ X, compute_uv=False))[::-1]
    s = np.sort(np.linalg.svd(X - Y @ (Y.T @ X), compute_uv=False))
    return np.arctan2(s, c)


def subspace_distance(X: np.ndarray, Y: np.ndarray) -> float:
    """dist = ||theta||_2 (Sec. 4.2, eq. distance_with_Log_and_angles)."""
    return float(np.linalg.norm(principal_angles(X, Y)))


# ----------------------------------------------------------------------------- line search

def linesearch_diagonals(C, S, PtZ, PtY):
    """Eigendecomposition P^T P = V D_beta V^T and the diagonals of Sec. 5.2,
    eq. CG_linesearch_D:
        alpha = diag(V^T C V), gamma = diag(V^T (P^T A P) V), zeta = -diag(V^T (P^T A X) V).
    Negative eigenvalues of the computed P^T P (rounding) are set to zero."""
    b, V = np.linalg.eigh(sym(S))
    b = np.maximum(b, 0.0)
    alpha = np.einsum("ki,kl,li->i", V, C, V)
    gamma = np.einsum("ki,kl,li->i", V, sym(PtZ), V)
    zeta = -np.einsum("ki,kl,li->i", V, PtY, V)
    return b, V, alpha, gamma, zeta


def phi_model(mu, alpha, beta, gamma, zeta) -> float:
    """phi(X(mu)) as the rational function of Sec. 5.2, eq. phi_P."""
    return -0.5 * float(np.sum((alpha + 2.0 * zeta * mu + gamma * mu * mu) / (1.0 + beta * mu * mu)))


def dphi_model(mu, alpha, beta, gamma, zeta) -> float:
    """d phi(X(mu)) / d mu, Sec. 5.2, eq. deriv_P (eq. dqnew when zeta = beta)."""
    num = zeta + (gamma - alpha * beta) * mu - beta * zeta * mu * mu
    return -float(np.sum(num / (1.0 + beta * mu * mu) ** 2))


def branch_roots(alpha, beta, gamma, zeta):
    """Positive root xi_i of each branch numerator zeta_i + d_i mu - beta_i zeta_i mu^2,
    d_i = gamma_i - alpha_i beta_i, written without cancellation (Sec. 6.1, eqs. derv1 and
    derv2; eq. xii for zeta = beta). Requires beta_i > 0, zeta_i > 0."""
    d = gamma - alpha * beta
    s = np.sqrt(d * d + 4.0 * beta * zeta * zeta)
    return np.where(d < 0.0, 2.0 * zeta / (np.abs(d) + s), (d + s) / (2.0 * beta * zeta))


@dataclass
class MuResult:
    mu: float
    ok: bool
    evals: int
    lo: float
    hi: float


def get_mu(alpha, beta, gamma, zeta) -> MuResult:
    """Exact line search (Algorithm 3 Get_Mu, extended for P != G as in Sec. 5.2).

    The branch roots xi_i of the convex branches (zeta_i > 0) bound the minimizer
    (Sec. 3.2: phi decreases on [0, xi_min] and increases beyond xi_max). Sorting the
    candidates 0 < xi_(1) <= ... and taking the first one where phi' >= 0, together with
    the candidate before it (where phi' < 0), gives a bracket that holds exactly one sign
    change from - to +: the minimizer closest to mu = 0. A safeguarded root finder
    (Brent's method) then solves phi'(mu) = 0 in it (Sec. 6.1). If phi' < 0 at every
    candidate the bracket is widened by doubling; if phi'(0) >= 0, or there is no convex
    branch, the direction is not usable and ok=False is returned."""
    alpha, beta, gamma, zeta = (np.asarray(v, dtype=np.float64) for v in (alpha, beta, gamma, zeta))
    p = beta.shape[0]
    bmax = float(beta.max()) if p else 0.0
    if not bmax > 0.0:
        return MuResult(0.0, False, 0, 0.0, 0.0)
    act = beta > p * EPS * bmax
    a, b, g, z = alpha[act], beta[act], gamma[act], zeta[act]
    conv = z > 0.0
    if not conv.any():
        return MuResult(0.0, False, 0, 0.0, 0.0)
    evals = [0]

    def f(mu):
        evals[0] += 1
        return dphi_model(mu, a, b, g, z)

    if f(0.0) >= 0.0:
        return MuResult(0.0, False, evals[0], 0.0, 0.0)
    cand = np.sort(branch_roots(a[conv], b[conv], g[conv], z[conv]))
    lo, hi, fhi = 0.0, None, None
    for c in cand:
        fc = f(float(c))
        if fc >= 0.0:
            hi, fhi = float(c), fc
            break
        lo = float(c)
    widen = 0
    while hi is None and widen < 60:
        c = 2.0 * (lo if lo > 0.0 else 1.0)
        fc = f(c)
        if fc >= 0.0:
            hi, fhi = c, fc
        else:
            lo = c
        widen += 1
    if hi is None:
        return MuResult(0.0, False, evals[0], lo, lo)
    if fhi == 0.0:
        return MuResult(hi, True, evals[0], lo, hi)
    mu = scipy.optimize.brentq(f, lo, hi, xtol=1e-300, rtol=4.0 * EPS, maxiter=200)
    return MuResult(float(mu), True, evals[0], lo, hi)


def retraction(X, P, mu, b, V):
    """Polar retraction X(mu) = (X - mu P) V D_mu^{-1} V^T (Sec. 5.2, eq. Xnew_P).
    Returns (X(mu), M) with M = V D_mu^{-1} V^T."""
    M = (V * (1.0 / np.sqrt(1.0 + mu * mu * b))) @ V.T
    return (X - mu * P) @ M, M


# ----------------------------------------------------------------------------- solvers

@dataclass
class SolveResult:
    X: np.ndarray
    theta: np.ndarray          # Ritz values of A (largest first for which=+1, smallest first for -1)
    iters: int
    converged: bool
    rho: list = field(default_factory=list)       # ||G||_F / (sqrt(p) ||A||_inf) per iterate
    gnorm_inf: list = field(default_factory=list) # ||G||_inf per iterate
    phi: list = field(default_factory=list)       # phi(X_k) of the operator the solver runs on
    mu: list = field(default_factory=list)
    beta_pr: list = field(default_factory=list)
    restarts: list = field(default_factory=list)
    brent_evals: list = field(default_factory=list)
    spmm: int = 0


def _finish(A_op, X, which, res: SolveResult) -> SolveResult:
    w, _, _ = rayleigh_ritz(A_op, X)
    res.theta = w if which > 0 else -w
    res.X = X
    return res


def rcg(A, X0, tol: float = 1e-10, max_iter: int = 10000, method: str = "rcg",
        k_restart: int = 0, recompute_ax: bool = False, which: int = 1,
        refresh_threshold: float = 1e3) -> SolveResult:
    """Riemannian steepest descent (method='rsd', Algorithm 2) or Riemannian nonlinear CG
    with Polak-Ribiere directions (method='rcg', Algorithm 4, Sec. 5) with the exact line
    search. AX is updated by the recursion of Sec. 6.1 (eq. save_matvec) unless
    recompute_ax (the RCG(+) variant of Sec. 6.4). which=-1 targets the smallest
    eigenvalues by running on -A (Sec. 2.2)."""
    A = as_operator(A)
    A_op = A if which > 0 else -A
    X = orthonormalize(np.asarray(X0, dtype=np.float64))
    n, p = X.shape
    nA = norm_inf(A)
    Y = A_op @ X
    res = SolveResult(X=X, theta=np.zeros(p), iters=0, converged=False, spmm=1)
    G_old = P_old = None
    k = 0
    while True:
        G, C = gradient(X, Y)
        gg = float(np.sum(G * G))
        rho = np.sqrt(gg) / (np.sqrt(p) * nA)
        res.rho.append(rho)
        res.gnorm_inf.append(float(np.abs(G).sum(axis=1).max()))
        res.phi.append(-0.5 * float(np.trace(C)))
        if rho <= tol:
            res.converged = True
            break
        if k >= max_iter:
            break
        restart = method == "rsd" or k == 0 or (k_restart > 0 and k % k_restart == 0)
        beta_pr = 0.0
        if not restart:
            den = float(np.sum(G_old * G_old))
            beta_pr = (gg - float(np.sum(G_old * G))) / den if den > 0.0 else 0.0
            P = tangent(X, G + beta_pr * P_old)
            if float(np.sum(G * P)) <= 0.0:
                restart, beta_pr = True, 0.0
        if restart:
            P = tangent(X, G)
        Z = A_op @ P
        res.spmm += 1
        while True:
            S = P.T @ P
            b, V, alpha, gamma, zeta = linesearch_diagonals(C, S, P.T @ Z, P.T @ Y)
            mr = get_mu(alpha, b, gamma, zeta)
            if mr.ok or restart:
                break
            P, restart, beta_pr = tangent(X, G), True, 0.0
            Z = A_op @ P
            res.spmm += 1
        if not mr.ok:
            break  # no descent step exists along G (only at G = 0 to rounding)
        mu = mr.mu
        res.mu.append(mu)
        res.beta_pr.append(beta_pr)
        res.restarts.append(bool(restart))
        res.brent_evals.append(mr.evals)
        X, M = retraction(X, P, mu, b, V)
        if recompute_ax or mu * np.sqrt(b.max()) <= refresh_threshold * EPS:
            Y = A_op @ X
            res.spmm += 1
        else:
            Y = (Y - mu * Z) @ M
        G_old, P_old = G, P
        k += 1
    res.iters = k
    return _finish(A_op, X, which, res)


def rsd(A, X0, **kw) -> SolveResult:
    """Riemannian steepest descent with exact line search (Algorithm 2)."""
    return rcg(A, X0, method="rsd", **kw)


def subspace_iteration(A, X0, tol: float = 1e-10, max_iter: int = 100000, which: int = 1) -> SolveResult:
    """Subspace iteration with the monomial filter p(t) = t (Algorithm 1): X_hat = A X,
    QR, Rayleigh-Ritz C = Q^T A Q = U Lambda U^T, X <- Q U; stop on ||(I - XX^T) A X||."""
    A = as_operator(A)
    A_op = A if which > 0 else -A
    X = orthonormalize(np.asarray(X0, dtype=np.float64))
    n, p = X.shape
    nA = norm_inf(A)
    res = SolveResult(X=X, theta=np.zeros(p), iters=0, converged=False)
    k = 0
    while True:
        Y = A_op @ X
        res.spmm += 1
        G, C = gradient(X, Y)
        rho = np.linalg.norm(G) / (np.sqrt(p) * nA)
        res.rho.append(rho)
        res.phi.append(-0.5 * float(np.trace(C)))
        if rho <= tol:
            res.converged = True
            break
        if k >= max_iter:
            break
        Q = orthonormalize(Y)
        AQ = A_op @ Q
        res.spmm += 1
        w, U = np.linalg.eigh(sym(Q.T @ AQ))
        X = Q @ U[:, ::-1]
        k += 1
    res.iters = k
    return _finish(A_op, X, which, res)


def chebyshev_filter(A_op, X: np.ndarray, Y: np.ndarray, degree: int, lo: float, hi: float, top: float) -> np.ndarray:
    """p_d(A) X with p_d(t) = C_d((t - c)/h) / C_d((top - c)/h), c = (lo + hi)/2, h = (hi - lo)/2
    (Sec. 2.3, eq. optimal_poly: the unwanted eigenvalues [lambda_n, lambda_{p+1}] of the
    operator map to [-1, 1]; the division by the value at `top`, an estimate of lambda_1,
    keeps the block bounded). Three-term recurrence of the Chebyshev polynomials with that
    normalization carried step by step (Zhou and Saad 2007); Y = A X is given."""
    c, h = 0.5 * (lo + hi), 0.5 * (hi - lo)
    sigma1 = h / (top - c)
    prev = X
    cur = (sigma1 / h) * (Y - c * X)
    sigma = sigma1
    for _ in range(2, degree + 1):
        sigma_new = 1.0 / (2.0 / sigma1 - sigma)
        nxt = (2.0 * sigma_new / h) * (A_op @ cur - c * cur) - sigma * sigma_new * prev
        prev, cur, sigma = cur, nxt, sigma_new
    return cur


def chebyshev_si(A, X0, degree: int, lo: float, hi: float, top: float, tol: float = 1e-10,
                 max_iter: int = 100000, which: int = 1) -> SolveResult:
    """Subspace iteration with the Chebyshev filter of eq. optimal_poly (Algorithm 1): filter,
    QR, Rayleigh-Ritz C = Q^T A Q = U Lambda U^T, X <- Q U, A X <- (A Q) U; stop on
    ||(I - X X^T) A X||. lo, hi, top refer to the operator solved (-A when which = -1).
    degree 1 is the shifted monomial filter."""
    A = as_operator(A)
    A_op = A if which > 0 else -A
    X = orthonormalize(np.asarray(X0, dtype=np.float64))
    n, p = X.shape
    nA = norm_inf(A)
    res = SolveResult(X=X, theta=np.zeros(p), iters=0, converged=False)
    Y = A_op @ X
    res.spmm += 1
    k = 0
    while True:
        G, C = gradient(X, Y)
        rho = np.linalg.norm(G) / (np.sqrt(p) * nA)
        res.rho.append(rho)
        res.phi.append(-0.5 * float(np.trace(C)))
        if rho <= tol:
            res.converged = True
            break
        if k >= max_iter:
            break
        Xh = chebyshev_filter(A_op, X, Y, degree, lo, hi, top)
        res.spmm += degree - 1
        Q = orthonormalize(Xh)
        AQ = A_op @ Q
        res.spmm += 1
        w, U = np.linalg.eigh(sym(Q.T @ AQ))
        U = U[:, ::-1]
        X = Q @ U
        Y = AQ @ U
        k += 1
    res.iters = k
    return _finish(A_op, X, which, res)


def cholesky_qr2(X: np.ndarray) -> np.ndarray:
    """Two passes of Cholesky QR: R = chol(X^T X), X <- X R^{-1} (used to orthonormalize a
    drifted or warm-started block; the result spans the same space)."""
    for _ in range(2):
        R = np.linalg.cholesky(sym(X.T @ X)).T
        X = np.linalg.solve(R.T, X.T).T
    return X


def track(mats, X0, tol: float = 1e-10, max_iter: int = 10000, which: int = 1, method: str = "rcg"):
    """Subspace tracking over a sequence of matrices A_0, A_1, ... (Sec. 1 and 2.3: related
    eigenproblems solved one after another, each started from the previous converged
    subspace). A_0 starts from X0; A_t from the basis returned for A_{t-1}. Returns the list
    of SolveResults."""
    out = []
    X = np.asarray(X0, dtype=np.float64)
    for A in mats:
        r = rcg(A, X, tol=tol, max_iter=max_iter, method=method, which=which)
        out.append(r)
        X = r.X
    return out


def stencil_matrix(nx: int, ny: int = 1, nz: int = 1, diag: float = 0.0, off: float = -1.0, diag_vec=None):
    """The matrix of a 5- or 7-point stencil operator on an nx x ny x nz grid (lexicographic,
    x fastest): diag + diag_vec[r] on the diagonal, off between grid neighbours. Written out
    entry by entry from that definition (the Sec. 6 test operators: Dirichlet Laplacians and
    -Laplacian + V)."""
    n = nx * ny * nz
    d = np.full(n, float(diag)) + (np.zeros(n) if diag_vec is None else np.asarray(diag_vec, dtype=np.float64))
    rows, cols, vals = [np.arange(n)], [np.arange(n)], [d]
    r = np.arange(n)
    i, j, k = r % nx, (r // nx) % ny, r // (nx * ny)
    for ok, step in ((i < nx - 1, 1), (j < ny - 1, nx), (k < nz - 1, nx * ny)):
        a = r[ok]
        rows += [a, a + step]
        cols += [a + step, a]
        vals += [np.full(a.size, float(off))] * 2
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))


# ----------------------------------------------------------------------------- complex Hermitian

def principal_angles_complex(X: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """Principal angles between the complex column spans of orthonormal X and Y (the
    Sec. 4.2 definition with conjugate transposes), ascending."""
    c = np.sort(np.linalg.svd(Y.conj().T @ X, compute_uv=False))[::-1]
    s = np.sort(np.linalg.svd(X - Y @ (Y.conj().T @ X), compute_uv=False))
    return np.arctan2(s, c)


def rcg_hermitian(A, X0, tol: float = 1e-10, max_iter: int = 10000, method: str = "rcg", which: int = 1,
                  refresh_threshold: float = 1e3) -> SolveResult:
    """The complex Hermitian variant of RSD / RCG with exact line search: the steps of
    Algorithms 2 and 4 with every transpose a conjugate transpose (the extension the paper
    states for Hermitian A), on phi(X) = -1/2 Re Tr(X^H A X) over n x p complex X with
    X^H X = I and the real inner product <U, V> = Re Tr(U^H V) (which makes the Polak-Ribiere
    beta and the descent test real). The line-search model keeps its form with
    alpha = diag(V^H C V), gamma = diag(V^H (P^H A P) V), zeta = -Re diag(V^H (P^H A X) V),
    P^H P = V D_beta V^H; the retraction is (X - mu P) V D_mu^{-1} V^H. rho uses the max
    absolute row sum of the complex entries."""
    A = as_operator(A)
    A_op = A if which > 0 else -A
    X, _ = np.linalg.qr(np.asarray(X0, dtype=np.complex128))
    n, p = X.shape
    nA = norm_inf(A)
    herm = lambda M: 0.5 * (M + M.conj().T)
    tang = lambda D: D - X @ (X.conj().T @ D)
    rip = lambda U, V: float(np.real(np.vdot(U, V)))
    Y = A_op @ X
    res = SolveResult(X=X, theta=np.zeros(p), iters=0, converged=False, spmm=1)
    G_old = P_old = None
    k = 0
    while True:
        C = herm(X.conj().T @ Y)
        G = -(Y - X @ C)
        gg = rip(G, G)
        rho = np.sqrt(gg) / (np.sqrt(p) * nA)
        res.rho.append(rho)
        res.phi.append(-0.5 * float(np.real(np.trace(C))))
        if rho <= tol:
            res.converged = True
            break
        if k >= max_iter:
            break
        restart = method == "rsd" or k == 0
        beta_pr = 0.0
        if not restart:
            den = rip(G_old, G_old)
            beta_pr = (gg - rip(G_old, G)) / den if den > 0.0 else 0.0
            P = tang(G + beta_pr * P_old)
            if rip(G, P) <= 0.0:
                restart, beta_pr = True, 0.0
        if restart:
            P = tang(G)
        Z = A_op @ P
        res.spmm += 1
        while True:
            b, V = np.linalg.eigh(herm(P.conj().T @ P))
            b = np.maximum(b, 0.0)
            VH = V.conj().T
            alpha = np.real(np.diag(VH @ C @ V))
            gamma = np.real(np.diag(VH @ herm(P.conj().T @ Z) @ V))
            zeta = -np.real(np.diag(VH @ (P.conj().T @ Y) @ V))
            mr = get_mu(alpha, b, gamma, zeta)
            if mr.ok or restart:
                break
            P, restart, beta_pr = tang(G), True, 0.0
            Z = A_op @ P
            res.spmm += 1
        if not mr.ok:
            break
        mu = mr.mu
        res.mu.append(mu)
        res.beta_pr.append(beta_pr)
        res.restarts.append(bool(restart))
        M = (V * (1.0 / np.sqrt(1.0 + mu * mu * b))) @ VH
        X = (X - mu * P) @ M
        if mu * np.sqrt(b.max()) <= refresh_threshold * EPS:
            Y = A_op @ X
            res.spmm += 1
        else:
            Y = (Y - mu * Z) @ M
        G_old, P_old = G, P
        k += 1
    res.iters = k
    w, U = np.linalg.eigh(herm(X.conj().T @ (A_op @ X)))
    w, U = w[::-1], U[:, ::-1]
    res.X = X @ U
    res.theta = w if which > 0 else -w
    return res


# ---------------------------------------------------------------- seeded random start block

_GOLDEN = 0x9E3779B97F4A7C15
_M64 = (1 << 64) - 1


def splitmix64(seed: int, k):
    """Output number k (0, 1, ...; scalar or integer array) of SplitMix64 started at state
    `seed` (Steele, Lea and Flood, "Fast splittable pseudorandom number generators", 2014):
    the state advances by the golden-ratio increment before each output, and the output is
    the state passed through the variant-13 mixing function (xor-shift 30, multiply,
    xor-shift 27, multiply, xor-shift 31), all modulo 2^64."""
    k = np.asarray(k, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & _M64) + (k + np.uint64(1)) * np.uint64(_GOLDEN)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def seeded_start_block(n: int, p: int, seed: int) -> np.ndarray:
    """The random start block X0 (n x p, entries i.i.d. N(0,1): the random starts of the
    experiments, Sec. 6) that the library draws on the device when it is given no X0:
    entry e = i p + j takes the first Box-Muller normal (Box and Muller 1958)
    sqrt(-2 ln u1) cos(2 pi u2) of the uniforms u = (floor(o / 2^11) + 1/2) 2^-53 of the
    SplitMix64 outputs o number 2e and 2e + 1. Not orthonormalized (the solver does that)."""
    e = np.arange(n * p, dtype=np.uint64)
    o1 = splitmix64(seed, 2 * e)
    o2 = splitmix64(seed, 2 * e + np.uint64(1))
    u1 = ((o1 >> np.uint64(11)).astype(np.float64) + 0.5) * 2.0 ** -53
    u2 = ((o2 >> np.uint64(11)).astype(np.float64) + 0.5) * 2.0 ** -53
    return (np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)).reshape(n, p)
