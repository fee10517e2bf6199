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


class FakeBatch:
    """ns, ps of a batch; records the shapes and policies it is given."""

    def __init__(self, ns, ps):
        self.ns, self.ps = ns, ps
        self.codes = None
        self.policies = []

    def set_shapes(self, codes):
        self.codes = list(codes)

    def set_tuning(self, a, b, c):
        self.policies.append((a, b, c))


def _fields(code):
    return code & 15, (code >> 4) & 15, (code >> 8) & 15, (code >> 12) & 15


def test_shape_codes_and_group_keys():
    assert tuning.shape_code() == 0
    assert _fields(tuning.shape_code(u=4, uu=2, ug=1, ch=16)) == (4, 2, 1, 15)
    assert tuning.group_key(1024, 4, "fp64") == "n=2^10 PP=16 fp64"
    assert tuning.group_key(2047, 17, "mixed") == "n=2^10 PP=32 mixed"
    assert tuning.group_key(25600, 32, "mixed") == "n=2^14 PP=32 mixed"


def test_shape_tuner_picks_each_groups_cheapest_field_values(tmp_path):
    import numpy as np
    # two groups with different optima: small problems like u=4, ch=4; large ones u=1, ch=16
    ns, ps = [1024, 1100, 20000, 21000], [8, 8, 30, 30]
    want = {"n=2^10 PP=16 mixed": {"u": 4, "uu": 2, "ug": 1, "ch": 4},
            "n=2^14 PP=32 mixed": {"u": 1, "uu": 1, "ug": 4, "ch": 16}}
    keys = [tuning.group_key(n, p, "mixed") for n, p in zip(ns, ps)]
    measured = []

    def measure(solver, passes):
        measured.append(tuple(passes))
        out = []
        for code, k in zip(solver.codes, keys):
            u, uu, ug, ch = _fields(code)
            ch = 16 if ch == 15 else ch
            w = want[k]
            # cost of the field the passes belong to; 0 (the default) costs a little more than any miss
            f = {"grad": ("u", u), "update": ("uu", uu), "gram": ("ug", ug), "spmm": ("ch", ch)}[passes[0]]
            out.append(0.0 if f[1] == w[f[0]] else (5.0 if f[1] == 0 else 1.0 + abs(f[1] - w[f[0]])))
        return np.array(out)

    b = FakeBatch(ns, ps)
    best, costs = tuning.tune_shapes(b, "mixed", measure=measure)
    assert best == want
    assert [tuple(x) for x in measured] == [p for _, c, p in tuning.SHAPE_AXES for _ in (0,) + c]
    # teams are off while measuring, then the default policy is restored
    assert b.policies[0][0] >= 1 << 20 and b.policies[-1] == tuning.DEFAULT
    assert b.codes == [tuning.shape_code(**want[k]) for k in keys]
    path = str(tmp_path / "shapes.json")
    tuning.record_shapes(path, best)
    b2 = FakeBatch(ns + [300], ps + [5])
    assert tuning.apply_shapes(b2, path, "mixed") == 4
    assert b2.codes == [tuning.shape_code(**want[k]) for k in keys] + [0]
