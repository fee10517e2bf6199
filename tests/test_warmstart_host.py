"""Host-side data of the warm-start loop (no GPU): the potentials handed to the network are
the ones on the operators' diagonals, and the start blocks are reproducible."""
import numpy as np

from paper_2306_10379_amd import inputs, warmstart


def test_potentials_are_the_operator_diagonals():
    N = 12
    mats, V = warmstart.potential_problems(3, seed=4, N=N, wells=8)
    assert V.shape == (3, N * N)
    h2 = float(N + 1) ** 2
    for A, v in zip(mats, V):
        d = A.to_dense().diagonal()
        assert np.allclose(d, 4.0 * h2 + v, rtol=0, atol=1e-9 * h2)
    # different problems get different wells, the same seed the same ones
    _, V2 = warmstart.potential_problems(3, seed=4, N=N, wells=8)
    assert np.array_equal(V, V2)
    assert not np.allclose(V[0], V[1])


def test_random_starts_are_seeded_and_distinct():
    mats, _ = warmstart.potential_problems(2, seed=1, N=8)
    a = warmstart.random_starts(mats, 4, seed=9)
    b = warmstart.random_starts(mats, 4, seed=9)
    assert all(np.array_equal(x, y) for x, y in zip(a, b))
    assert a[0].shape == (64, 4) and not np.allclose(a[0], a[1])
    assert not np.allclose(a[0], inputs.start_block(64, 4, 9))


def test_chunked_generation_reproduces_the_family():
    """Problems and start blocks built chunk by chunk (start / offset) are those of the whole
    family built at once."""
    mats, V = warmstart.potential_problems(5, seed=3, N=8)
    X0 = warmstart.random_starts(mats, 4, seed=3)
    mats_c, V_c = warmstart.potential_problems(3, seed=3, N=8, start=2)
    X0_c = warmstart.random_starts(mats_c, 4, seed=3, offset=2)
    assert np.array_equal(V_c, V[2:])
    for a, b in zip(mats_c, mats[2:]):
        assert np.array_equal(a.vals, b.vals) and np.array_equal(a.colind, b.colind)
    for a, b in zip(X0_c, X0[2:]):
        assert np.array_equal(a, b)
