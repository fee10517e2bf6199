"""gsi_orthonormalize (two passes of Cholesky QR on a caller's block, through the C ABI)
against the oracle's Cholesky QR2: element by element, X^T X = I, the same span, ragged
sizes, and rank-deficient blocks reported as breakdown."""
import numpy as np
import pytest

from oracle import gsi_oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _gsi():
    from paper_2306_10379_amd import gsi
    gsi.load()
    return gsi


def _block(n, p, seed, cond=1.0):
    g = np.random.default_rng(seed)
    X = g.standard_normal((n, p))
    if cond > 1.0:
        # singular values spread over [1, cond] after any column scaling
        U, _ = np.linalg.qr(X)
        V, _ = np.linalg.qr(g.standard_normal((p, p)))
        X = U @ np.diag(np.geomspace(1.0, 1.0 / cond, p)) @ V.T
    return X


@pytest.mark.parametrize("n,p,seed,cond", [(1, 1, 0, 1.0), (64, 64, 1, 1.0), (777, 13, 2, 1.0), (4097, 64, 3, 1e4),
                                           (20000, 40, 4, 1.0), (100003, 7, 5, 1e3)])
def test_orthonormalize_matches_oracle(n, p, seed, cond):
    gsi = _gsi()
    print(f"orthonormalize n={n} p={p} seed={seed} cond={cond:g}", flush=True)
    X = _block(n, p, seed, cond)
    Xd = torch.as_tensor(X, device="cuda").contiguous()
    assert gsi.orthonormalize(Xd) == gsi.GSI_OK
    Q = Xd.cpu().numpy()
    ref = O.cholesky_qr2(X)
    # Cholesky QR is unique (positive diagonal of R): the two agree entry by entry up to
    # rounding amplified by the condition number of X
    assert np.max(np.abs(Q - ref)) <= 1e-14 * cond * max(1.0, np.sqrt(n))
    assert np.max(np.abs(Q.T @ Q - np.eye(p))) <= 1e-13
    assert O.principal_angles(Q, np.linalg.qr(X)[0]).max() <= 1e-10 * cond


def test_orthonormalize_repeats_bit_for_bit_and_reports_breakdown():
    gsi = _gsi()
    X = _block(3000, 24, 7)
    a = torch.as_tensor(X, device="cuda").contiguous()
    b = a.clone()
    assert gsi.orthonormalize(a) == gsi.GSI_OK and gsi.orthonormalize(b) == gsi.GSI_OK
    assert torch.equal(a, b)
    R = X.copy()
    R[:, 5] = R[:, 2]  # rank deficient
    r = torch.as_tensor(R, device="cuda").contiguous()
    before = r.clone()
    assert gsi.orthonormalize(r) == gsi.GSI_BREAKDOWN
    assert torch.equal(r, before)  # the first pass failed: X untouched
    bad = torch.as_tensor(X, device="cuda").contiguous()
    bad[17, 3] = float("nan")
    assert gsi.orthonormalize(bad) == gsi.GSI_BREAKDOWN
    with pytest.raises(gsi.GsiError):
        gsi.orthonormalize(torch.zeros((100, 65), dtype=torch.float64, device="cuda"))
    with pytest.raises(gsi.GsiError):
        gsi.orthonormalize(torch.zeros((10, 11), dtype=torch.float64, device="cuda"))
