"""Host logic of the batched team-policy tuner (no GPU): coordinate descent over the three
knobs with an injected cost, and the JSON table of recorded winners."""
from paper_2306_10379_amd import tuning


class FakeSolver:
    def __init__(self):
        self.policy = None

    def set_tuning(self, a, b, c):
        self.policy = (a, b, c)


def test_coordinate_descent_finds_the_cheapest_policy_along_the_axes():
    # separable cost with its minimum at (32, 2, 64), reachable one axis at a time
    cost = lambda p: abs(p[0] - 32) + 2 * abs(p[1] - 2) + 0.5 * abs(p[2] - 64)
    calls = []

    def timer(solver, policy):
        calls.append(tuple(policy))
        return cost(policy)

    s = FakeSolver()
    best, times = tuning.tune(s, timer=timer)
    assert best == (32, 2, 64)
    assert s.policy == best                      # the solver is left on the winner
    assert len(calls) == len(set(calls))         # no policy timed twice
    assert set(times) == set(calls)


def test_tuning_table_round_trip(tmp_path):
    path = str(tmp_path / "table.json")
    key = tuning.batch_key([100, 200], [4, 8], "mixed")
    s = FakeSolver()
    assert not tuning.apply_cached(s, path, key)
    tuning.record(path, key, (8, 4, 16), {(8, 4, 16): 1.0, (16, 4, 32): 1.5})
    assert tuning.apply_cached(s, path, key)
    assert s.policy == (8, 4, 16)
    assert not tuning.apply_cached(s, path, tuning.batch_key([1], [1], "fp64"))
