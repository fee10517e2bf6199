"""Learned warm start: training data from the method's own solves, training of the
sine-basis neural operator on the device, and start blocks for new problems.

The solver always iterates to the tolerance from whatever block it is given, so the
network can only change the number of iterations, never the accuracy: the residual test of
the solve is what measures the network's error. A problem whose warm-started solve does not
converge (for instance a rank-deficient network output that the start-block
orthonormalization rejects) is solved again from its random start block, the fallback.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import fno, gsi, inputs


def potential_problems(count: int, seed: int, N: int, wells: int = 8, start: int = 0):
    """Operators start .. start+count-1 of the seeded family H = -Laplacian + V on an N x N
    grid, V a sum of `wells` Gaussian wells (depth U(-20, 0), width U(0.02, 0.2), centre
    U([0,1]^2)); returns (mats, V) with V the potentials at the grid nodes, (count, N*N)."""
    mats, V = [], []
    for i in range(start, start + count):
        W = inputs.random_wells(seed * 100_000 + i, count=wells)
        mats.append(inputs.schrodinger_2d(N, W))
        V.append(W.sample(N))
    return mats, np.stack(V)


def random_starts(mats, p: int, seed: int, offset: int = 0):
    """Seeded random start blocks of problems offset, offset+1, ... (the family's indices)."""
    return [inputs.start_block(A.n, p, seed * 100_000 + 50_000 + offset + i) for i, A in enumerate(mats)]


def solve_batch(mats, p: int, X0s, tol: float, precision: str = "mixed", max_iter: int = 60000):
    """One persistent batched solve of the smallest p eigenpairs of every operator.
    Returns (bases as a list of device float64 n x p tensors, iterations, status, seconds)."""
    import torch
    with gsi.BatchedSolver(mats, X0s, [p] * len(mats), which=-1, precision=precision, tol=tol,
                           max_iter=max_iter, switch_tol=1e-5) as b:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, iters, status = b.solve()
        dt = time.perf_counter() - t0
        X = [b.get_x(i) for i in range(len(mats))]
    return X, iters, status, dt


def chunked(mats, p, X0s, tol, precision="mixed", chunk=None, log=None, max_iter=60000):
    """Batched solves of consecutive groups of `chunk` problems (all at once when None):
    (iterations, status, total seconds)."""
    chunk = chunk or len(mats)
    its, sts, total = [], [], 0.0
    for s0 in range(0, len(mats), chunk):
        _, it, st, dt = solve_batch(mats[s0:s0 + chunk], p, X0s[s0:s0 + chunk], tol, precision, max_iter)
        its.append(it)
        sts.append(st)
        total += dt
        if log:
            log(f"  problems {s0}..{min(len(mats), s0 + chunk) - 1}: {dt:.1f} s, mean iterations {it.mean():.0f}")
    return np.concatenate(its), np.concatenate(sts), total


def train(net: "fno.Net", V, X, epochs: int, batch: int, lr: float, lr_final: float | None = None,
          seed: int = 0, log=None):
    """Minibatch Adam on the mean subspace loss. V: (count, n) float32 device tensor, X:
    (count, n, p) float32 device targets with orthonormal columns. Cosine decay of the
    learning rate from lr to lr_final over the run. Returns the mean loss of each epoch."""
    import torch
    count = V.shape[0]
    steps_per_epoch = max(1, count // batch)
    total = epochs * steps_per_epoch
    lr_final = lr * 0.05 if lr_final is None else lr_final
    g = np.random.default_rng(seed)
    hist, step = [], 0
    for ep in range(epochs):
        order = g.permutation(count)
        losses = []
        for s in range(steps_per_epoch):
            idx = torch.as_tensor(order[s * batch:(s + 1) * batch], device=V.device)
            loss, _ = net.loss_grad(V.index_select(0, idx).contiguous(), X.index_select(0, idx).contiguous(),
                                    want_grad=False)
            rate = lr_final + 0.5 * (lr - lr_final) * (1.0 + math.cos(math.pi * step / max(1, total - 1)))
            net.adam(rate)
            losses.append(float(np.mean(loss)))
            step += 1
        hist.append(float(np.mean(losses)))
        if log:
            log(f"epoch {ep}: mean loss {hist[-1]:.4f}")
    return hist


def mean_loss(net: "fno.Net", V, X, batch: int):
    """Mean subspace loss (sum of squared sines of the principal angles) over a set."""
    out = []
    for s in range(0, V.shape[0], batch):
        loss, _ = net.loss_grad(V[s:s + batch].contiguous(), X[s:s + batch].contiguous(), want_grad=False)
        out.append(loss)
    return float(np.mean(np.concatenate(out)))


def start_blocks(net: "fno.Net", V, batch: int):
    """Network start blocks as float64 (count, n, p) device tensors (orthonormalized by the
    solver when it takes them)."""
    import torch
    return torch.cat([net.forward(V[s:s + batch].contiguous(), f64=True) for s in range(0, V.shape[0], batch)])


def warm_solve(mats, p, Xw, X0_random, tol, precision="mixed", chunk=None, log=None, max_iter=60000):
    """Batched solve from the network's start blocks; problems that do not converge within
    max_iter are solved again from their random start blocks (their iterations add up).
    Returns (iterations, seconds, fallbacks)."""
    iters, status, dt = chunked(mats, p, [x for x in Xw], tol, precision, chunk, log, max_iter)
    bad = [i for i in range(len(mats)) if status[i] != 1]
    if bad:
        it2, st2, dt2 = chunked([mats[i] for i in bad], p, [X0_random[i] for i in bad], tol, precision, chunk, log)
        iters = iters.copy()
        for j, i in enumerate(bad):
            iters[i] += it2[j]
        dt += dt2
    return iters, dt, len(bad)


def prior_blocks(N: int, p: int, count: int):
    """The network's fixed prior (the p lowest Dirichlet modes of the grid Laplacian) as
    start blocks, produced by an untrained network whose output layer is zero."""
    import torch
    net = fno.Net(N=N, modes=1, width=1, layers=0, p=p, max_batch=1, seed=0)
    try:
        Y = net.forward(torch.zeros((1, N * N), dtype=torch.float32, device="cuda"), f64=True)[0]
    finally:
        net.close()
    return [Y for _ in range(count)]


def single_solves(mats, p, X0s, tol, precision="fp64"):
    """Plain single-problem solves one after another: (seconds per solve, iterations)."""
    import torch
    times, its = [], []
    for A, X0 in zip(mats, X0s):
        s = gsi.Solver(A, X0 if not torch.is_tensor(X0) else X0.contiguous(), p, which=-1, precision=precision,
                       tol=tol, max_iter=60000, switch_tol=1e-5)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, it = s.solve()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        its.append(it)
        s.close()
    return np.array(times), np.array(its)


def run_experiment(N=256, p=32, ntrain=512, ntest=64, modes=24, width=20, layers=4, epochs=30, batch=16,
                   lr=3e-3, tol=1e-8, seed=1, nsingle=8, chunk=64, chunk_test=None, compare_prior=True,
                   warm_max_iter=60000, log=None, bf16_weights=False, train_tol=None):
    """Train on the method's own solves and compare start blocks on held-out potentials.

    Training targets: bases of ntrain problems solved from random starts to train_tol
    (default tol; a looser one only has to beat the network's own error, which is orders of
    magnitude above it). Held-out comparison (ntest problems, batched, mixed precision to
    tol): random start, prior start, trained network start (inference time included); plus
    nsingle plain float64 single-problem solves from the random and from the network start.
    bf16_weights: the network's passes read bfloat16 weights (float32 master in Adam)."""
    import torch
    log = log or (lambda s: None)
    chunk_test = chunk_test or ntest
    train_tol = tol if train_tol is None else train_tol
    out = {"grid": N, "p": p, "train": ntrain, "test": ntest, "tol": tol, "train_tol": train_tol,
           "network": {"modes": modes, "width": width, "layers": layers,
                       "weights": "bf16 (fp32 master)" if bf16_weights else "fp32"}}
    # the training problems are built chunk by chunk (operators and start blocks are not kept)
    Vd = torch.empty((ntrain + ntest, N * N), dtype=torch.float32, device="cuda")
    Xd = torch.empty((ntrain, N * N, p), dtype=torch.float32, device="cuda")
    it_tr, st_tr, dt_tr, t_build = [], [], 0.0, 0.0
    for s0 in range(0, ntrain, chunk):
        s1 = min(ntrain, s0 + chunk)
        tb = time.perf_counter()
        mats_c, V_c = potential_problems(s1 - s0, seed, N, start=s0)
        X0_c = random_starts(mats_c, p, seed, offset=s0)
        Vd[s0:s1].copy_(torch.as_tensor(V_c, dtype=torch.float32))
        t_build += time.perf_counter() - tb
        X, it, st, dt = solve_batch(mats_c, p, X0_c, train_tol)
        for i, x in enumerate(X):
            Xd[s0 + i].copy_(x)
        del X, mats_c, X0_c
        it_tr.append(it)
        st_tr.append(st)
        dt_tr += dt
        log(f"training solves {s0}..{s1 - 1}: {dt:.1f} s, mean iterations {it.mean():.0f}")
    it_tr, st_tr = np.concatenate(it_tr), np.concatenate(st_tr)
    tb = time.perf_counter()
    mats_t, V_t = potential_problems(ntest, seed, N, start=ntrain)
    X0_t = random_starts(mats_t, p, seed, offset=ntrain)
    Vd[ntrain:].copy_(torch.as_tensor(V_t, dtype=torch.float32))
    t_build += time.perf_counter() - tb
    mats = [None] * ntrain + mats_t  # indices of the family; training operators are gone
    X0r = [None] * ntrain + X0_t
    prior = prior_blocks(N, p, ntrain + ntest)
    out["build_problems_s"] = round(t_build, 2)
    out["train_solves"] = {"s": round(dt_tr, 2), "iters_mean": float(it_tr.mean()), "converged": int((st_tr == 1).sum()),
                           "tol": train_tol}
    log(f"training solves: {dt_tr:.1f} s, mean iterations {it_tr.mean():.0f}; problems built in {t_build:.1f} s")
    log("held-out problems from random starts")
    Xtd = torch.empty((ntest, N * N, p), dtype=torch.float32, device="cuda")
    it_r, dt_r = [], 0.0
    for s0 in range(ntrain, ntrain + ntest, chunk_test):
        s1 = min(ntrain + ntest, s0 + chunk_test)
        Xt, it, st, dt = solve_batch(mats[s0:s1], p, X0r[s0:s1], tol)
        for i, x in enumerate(Xt):
            Xtd[s0 - ntrain + i].copy_(x)
        del Xt
        it_r.append(it)
        dt_r += dt
        log(f"  problems {s0}..{s1 - 1}: {dt:.1f} s, mean iterations {it.mean():.0f}")
    it_r = np.concatenate(it_r)
    log(f"held-out, random start: {dt_r:.1f} s, mean iterations {it_r.mean():.0f}")
    if compare_prior:
        it_p, dt_p, nfp = warm_solve(mats[ntrain:], p, prior[ntrain:], X0r[ntrain:], tol, chunk=chunk_test, log=log,
                                     max_iter=warm_max_iter)
        log(f"held-out, prior start: {dt_p:.1f} s, mean iterations {it_p.mean():.0f}, fallbacks {nfp}")
    net = fno.Net(N=N, modes=modes, width=width, layers=layers, p=p, max_batch=batch, seed=seed,
                  bf16_weights=bf16_weights)
    out["network"]["params"] = net.count
    loss0 = mean_loss(net, Vd[ntrain:], Xtd, batch)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = train(net, Vd[:ntrain], Xd, epochs, batch, lr, seed=seed)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    loss1 = mean_loss(net, Vd[ntrain:], Xtd, batch)
    log(f"training: {t_train:.1f} s, held-out loss {loss0:.5f} (prior) -> {loss1:.5f} (trained) of {p}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Xw = start_blocks(net, Vd[ntrain:], batch)
    torch.cuda.synchronize()
    t_inf = time.perf_counter() - t0
    it_w, dt_w, nfb = warm_solve(mats[ntrain:], p, Xw, X0r[ntrain:], tol, chunk=chunk_test, log=log,
                                 max_iter=warm_max_iter)
    log(f"held-out, network start: {dt_w:.1f} s (+{t_inf:.3f} s inference), mean iterations {it_w.mean():.0f}, "
        f"fallbacks {nfb}")
    out["training"] = {"s": round(t_train, 2), "epochs": epochs, "batch": batch, "lr": lr,
                       "epoch_loss": [round(h, 6) for h in hist]}
    out["held_out_loss"] = {"prior": loss0, "trained": loss1}
    out["batched_held_out"] = {
        "random": {"s": round(dt_r, 3), "iters_mean": float(it_r.mean())},
        "prior": {"s": round(dt_p, 3), "iters_mean": float(it_p.mean()), "fallbacks": nfp} if compare_prior else None,
        "network": {"s": round(dt_w + t_inf, 3), "iters_mean": float(it_w.mean()), "inference_s": round(t_inf, 4),
                    "fallbacks": nfb}}
    if nsingle > 0:
        sel = list(range(ntrain, ntrain + nsingle))
        t_r, i_r = single_solves([mats[i] for i in sel], p, [X0r[i] for i in sel], tol)
        t_w, i_w = single_solves([mats[i] for i in sel], p, [Xw[i - ntrain] for i in sel], tol)
        out["single_fp64"] = {"problems": nsingle,
                              "random": {"s_per_solve": float(t_r.mean()), "iters_mean": float(i_r.mean())},
                              "network": {"s_per_solve": float(t_w.mean() + t_inf / ntest),
                                          "iters_mean": float(i_w.mean())}}
        log(f"single float64 solves: random {t_r.mean():.3f} s ({i_r.mean():.0f} it), "
            f"network {t_w.mean():.3f} s ({i_w.mean():.0f} it)")
    net.close()
    return out
