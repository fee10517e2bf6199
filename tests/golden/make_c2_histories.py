"""Write c2_histories.json: the per-iterate step sizes mu_k, Polak-Ribiere coefficients and
residual measures rho_k of the float64 oracle on the benchmark workload (3D 7-point Dirichlet
Laplacian on 128^3, p = 64 largest, X0 = start_block(n, 64, seed 0)) for a fixed number of
iterations of Riemannian steepest descent (Algorithm 2) and of Riemannian CG (Algorithm 4).
Calls only the oracle and the seeded input generators; takes ~15 minutes on 8 cores.

    python tests/golden/make_c2_histories.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import gsi_oracle as O  # noqa: E402
from paper_2306_10379_amd import inputs as I  # noqa: E402

N, P, SEED = 128, 64, 0
ITERS = {"rsd": 200, "rcg": 100}


def main():
    A = I.laplacian_3d(N)
    X0 = I.start_block(A.n, P, SEED)
    out = {"workload": f"3D 7-point Dirichlet Laplacian {N}^3, p={P} largest, X0 = start_block(n, {P}, {SEED})",
           "generator": "tests/golden/make_c2_histories.py (float64 oracle)"}
    for method, iters in ITERS.items():
        t0 = time.time()
        r = O.rcg(A, X0, tol=0.0, max_iter=iters, method=method)
        out[method] = {"iters": r.iters, "mu": r.mu, "beta_pr": r.beta_pr, "rho": r.rho,
                       "restarts": [bool(x) for x in r.restarts], "spmm": r.spmm}
        print(f"{method}: {r.iters} iterations in {time.time() - t0:.0f} s, rho {r.rho[-1]:.3e}", flush=True)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_histories.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
