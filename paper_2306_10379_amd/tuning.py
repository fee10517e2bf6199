"""Measured tuning of the batched solve: its team policy and its tile shapes.

Team policy: how few row tiles a recruited workgroup may own (so how large a team can
grow), how many idle workgroups a problem recruits at one check, and how often it checks.
`tune` times whole solves of the caller's batch under candidate policies (coordinate
descent from the current best, one knob at a time), keeps the fastest, and can record the
outcome in a JSON table keyed by the batch's shape and precision, which `apply_cached`
reads back for later batches of the same shape.

Tile shapes (loads in flight per pass, nonzeros per gather batch): `tune_shapes` picks one
per (size band, block width, precision) group from each problem's device pass clocks, and
`record_shapes` / `apply_shapes` keep the table (paper_2306_10379_amd/shape_table.json).
"""
from __future__ import annotations

import json
import os
import time

DEFAULT = (16, 4, 32)  # tiles per member, recruits per check, iterations between checks
AXES = [(0, (8, 32)), (1, (2, 8)), (2, (16, 64))]


def batch_key(ns, ps, precision: str) -> str:
    return f"count={len(ns)} n=[{min(ns)},{max(ns)}] p=[{min(ps)},{max(ps)}] {precision}"


def _time(solver, policy):
    import torch
    solver.set_tuning(*policy)
    solver.tuning_policy = tuple(policy)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    solver.solve()
    return time.perf_counter() - t0


def tune(solver, start=DEFAULT, log=None, timer=None):
    """Returns (best policy, {policy: seconds}); the solver is left on the best policy.
    timer(solver, policy) -> seconds defaults to timing one whole solve."""
    timer = timer or _time
    times = {tuple(start): timer(solver, start)}
    best = tuple(start)
    if log:
        log(f"tuning {best}: {times[best]:.3f} s")
    for axis, values in AXES:
        for v in values:
            cand = list(best)
            cand[axis] = v
            cand = tuple(cand)
            if cand in times:
                continue
            times[cand] = timer(solver, cand)
            if log:
                log(f"tuning {cand}: {times[cand]:.3f} s")
        best = min(times, key=times.get)
    solver.set_tuning(*best)
    return best, times


def record(path: str, key: str, best, times) -> None:
    table = {}
    if os.path.exists(path):
        with open(path) as f:
            table = json.load(f)
    table[key] = {"best": list(best), "seconds": {",".join(map(str, k)): round(v, 4) for k, v in times.items()}}
    with open(path, "w") as f:
        json.dump(table, f, indent=1)


def apply_cached(solver, path: str, key: str) -> bool:
    """Set the recorded best policy for this batch shape, if the table has one."""
    if not os.path.exists(path):
        return False
    with open(path) as f:
        entry = json.load(f).get(key)
    if not entry:
        return False
    solver.set_tuning(*entry["best"])
    return True


# ------------------------------------------------------------------------------- tile shapes
#
# The batched passes' tile shapes are runtime choices per problem (gsi_batched_set_shapes):
# u row tiles whose loads are issued together in the gradient, direction and product passes,
# uu in the retraction pass, ug in the Gram passes, and ch nonzeros gathered together in the
# SpMM. The best choice depends on the problem's size (how many tiles one workgroup sweeps),
# its block width and the precision, so the tuner picks one shape per group
# (power-of-two band of n, block width 16 or 32, precision): coordinate descent over the
# four fields, where every candidate value is measured for all groups by one solve of the
# whole batch (each problem's device clock per pass, per iteration).
SHAPE_AXES = [("u", (1, 2, 4), ("grad", "dir")), ("uu", (1, 2), ("update",)), ("ug", (1, 2, 4), ("gram",)),
              ("ch", (4, 8, 16), ("spmm",))]
SHAPE_FIELDS = ("u", "uu", "ug", "ch")


def shape_code(u: int = 0, uu: int = 0, ug: int = 0, ch: int = 0) -> int:
    """The int32 code of gsi_batched_set_shapes (0 in a field keeps the built default)."""
    return int(u) | (int(uu) << 4) | (int(ug) << 8) | ((15 if ch == 16 else int(ch)) << 12)


def group_key(n: int, p: int, precision: str) -> str:
    band = int(n).bit_length() - 1
    return f"n=2^{band} PP={16 if p <= 16 else 32} {precision}"


def _measure_passes(solver, passes):
    """One solve; per problem, microseconds per iteration of the listed passes."""
    import numpy as np
    from . import gsi
    _, iters, _ = solver.solve()
    us = solver.pass_times()
    cols = [gsi.PASSES.index(p) for p in passes]
    return us[:, cols].sum(axis=1) / np.maximum(iters, 1)


def tune_shapes(solver, precision: str, log=None, measure=None):
    """Pick a tile shape per (n band, block width, precision) group of the solver's batch.
    measure(solver, passes) -> per-problem cost array (default: one solve, device pass clocks
    per iteration). Teams are switched off while measuring (each problem's clock is then one
    workgroup's) and the team policy is restored. Returns ({group: {field: value}}, costs) and
    leaves the solver on the chosen shapes."""
    import numpy as np
    measure = measure or _measure_passes
    keys = [group_key(n, p, precision) for n, p in zip(solver.ns, solver.ps)]
    groups = {}
    for i, k in enumerate(keys):
        groups.setdefault(k, []).append(i)
    best = {k: dict.fromkeys(SHAPE_FIELDS, 0) for k in groups}
    costs = {k: {} for k in groups}
    restore = getattr(solver, "tuning_policy", None) or DEFAULT
    solver.set_tuning(1 << 20, 1, 1 << 20)  # no teams while measuring
    try:
        for field, cands, passes in SHAPE_AXES:
            seen = {k: {} for k in groups}
            for v in (0,) + tuple(cands):
                codes = [shape_code(**{**best[keys[i]], field: v}) for i in range(len(keys))]
                solver.set_shapes(codes)
                c = np.asarray(measure(solver, passes), dtype=np.float64)
                for k, idx in groups.items():
                    seen[k][v] = float(c[idx].sum())
                if log:
                    log(f"shape {field}={v}: " + ", ".join(f"{k}: {seen[k][v]:.1f}" for k in sorted(groups)))
            for k in groups:
                best[k][field] = min(seen[k], key=seen[k].get)
                costs[k][field] = seen[k]
    finally:
        solver.set_tuning(*restore)
    solver.set_shapes([shape_code(**best[k]) for k in keys])
    return best, costs


def record_shapes(path: str, table) -> None:
    """Merge {group: {field: value}} into the JSON table at path."""
    cur = {}
    if os.path.exists(path):
        with open(path) as f:
            cur = json.load(f)
    cur.update({k: {f: int(v[f]) for f in SHAPE_FIELDS} for k, v in table.items()})
    with open(path, "w") as f:
        json.dump(cur, f, indent=1, sort_keys=True)


def apply_shapes(solver, path: str, precision: str) -> int:
    """Set every problem's shape from the table at path (groups it lacks keep the defaults);
    returns the number of problems whose group was found."""
    if not os.path.exists(path):
        return 0
    with open(path) as f:
        table = json.load(f)
    codes, found = [], 0
    for n, p in zip(solver.ns, solver.ps):
        e = table.get(group_key(n, p, precision))
        found += e is not None
        codes.append(shape_code(**e) if e else 0)
    solver.set_shapes(codes)
    return found
