"""gsi_orthonormalize_noalloc (static device scratch, no allocation) against
gsi_orthonormalize (same kernels, per-call scratch) through the C ABI: equal results on two
calls in a row, the second with a smaller block, breakdown and size limits."""
import numpy as np
import pytest

from oracle import gsi_oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _gsi():
    from paper_2306_10379_amd import gsi
    gsi.load()
    return gsi


def _pair(gsi, X):
    a = torch.as_tensor(X, device="cuda").contiguous()
    b = a.clone()
    sa = gsi.orthonormalize(a)
    sb = gsi.orthonormalize(b, noalloc=True)
    return sa, sb, a.cpu().numpy(), b.cpu().numpy()


def test_noalloc_matches_allocating_entry_point_on_two_calls():
    gsi = _gsi()
    g = np.random.default_rng(31)
    # first call: large block at the width limit, then a smaller, ragged one
    for n, p in ((300001, 64), (1537, 9)):
        print(f"noalloc n={n} p={p}", flush=True)
        X = g.standard_normal((n, p))
        sa, sb, Qa, Qb = _pair(gsi, X)
        assert sa == sb == gsi.GSI_OK
        # the same kernels, grid and summation order: identical results
        assert np.array_equal(Qa, Qb)
        ref = O.cholesky_qr2(X)
        assert np.max(np.abs(Qb - ref)) <= 1e-13
        assert np.max(np.abs(Qb.T @ Qb - np.eye(p))) <= 1e-13


def test_noalloc_breakdown_and_limits():
    gsi = _gsi()
    X = np.random.default_rng(5).standard_normal((500, 10))
    X[:, 9] = 0.0
    sa, sb, Qa, Qb = _pair(gsi, X)
    assert sa == sb == gsi.GSI_BREAKDOWN and np.array_equal(Qa, Qb)
    # a good block right after the failed one: the flags of the failed call do not leak
    Y = np.random.default_rng(6).standard_normal((500, 10))
    sa, sb, Qa, Qb = _pair(gsi, Y)
    assert sa == sb == gsi.GSI_OK and np.array_equal(Qa, Qb)
    with pytest.raises(gsi.GsiError) as e:
        gsi.orthonormalize(torch.zeros((1000, 65), dtype=torch.float64, device="cuda"), noalloc=True)
    assert e.value.status == gsi.GSI_EUNSUPPORTED
