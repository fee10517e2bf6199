"""Measured tuning of the batched solve's team policy.

The batched kernel's per-problem work shapes (64-row tiles, columns per lane, loads in
flight) are fixed at compile time for each block width; what decides the makespan of an
uneven batch is the team policy: how few row tiles a recruited workgroup may own (so how
large a team can grow), how many idle workgroups a problem recruits at one check, and how
often it checks. `tune` times whole solves of the caller's batch under candidate policies
(coordinate descent from the current best, one knob at a time), keeps the fastest, and can
record the outcome in a JSON table keyed by the batch's shape and precision, which
`apply_cached` reads back for later batches of the same shape.
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
