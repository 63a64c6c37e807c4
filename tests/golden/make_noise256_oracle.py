"""Write the oracle's solution of the 256^3 filtered-noise problem at sampled nodes (a stored expected value).

The problem: 6th-order compact scheme (Sec. 2.3, eq. scheme6), N = 256, h = 1/257, k0 = 120, k^2 = k0^2 (1 + 0.2 w)
with w the seeded filtered noise, Gaussian point source, two-point absorbing closure (eq. D_bc). The oracle
assembles A and F (per-offset route), builds its EigT (Sec. 4.1) and solves with its right-preconditioned
GMRES(50) to ||F - A x|| <= 1e-10 ||F|| (Sec. 5.1 rel-res). Only `oracle/` and the seeded input generators run here.

Stored (noise256_oracle_solution.npz, no pickles): `nodes` (flat indices i + N (j + N l)): 32768 seeded random
nodes plus the three axis lines through the centre; `x` the solution there; `x_norm`, `F_norm` the full vectors'
2-norms; `iters`, `relres` of the oracle's solve. Regenerate with
    python tests/golden/make_noise256_oracle.py
It needs about 40 GB of host memory and a few minutes.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import krylov as kr  # noqa: E402
from oracle import operators as op  # noqa: E402
from oracle import precond as pc  # noqa: E402

OUT = os.path.join(HERE, "noise256_oracle_solution.npz")


def sample_nodes(n: int, count: int = 32768, seed: int = 2560) -> np.ndarray:
    rng = np.random.default_rng(seed)
    pts = [rng.choice(n ** 3, count, replace=False)]
    c = n // 2
    a = np.arange(n)
    pts += [a + n * (c + n * c), c + n * (a + n * c), c + n * (c + n * a)]
    return np.unique(np.concatenate(pts)).astype(np.int64)


def main():
    w = synth.workload("noise")
    n, h, k0 = w["n"], w["h"], w["k0"]
    t0 = time.perf_counter()
    A, F = op.problem(w["order"], w["k2"], w["f"], h, k0, route="stencil")
    g = op.gamma_abc(k0, h)
    e = pc.EigT((n, n, n), (h, h, h), k0, (g, g, g))
    print(f"assembly and EigT set-up {time.perf_counter() - t0:.1f} s", flush=True)
    t0 = time.perf_counter()
    x, info = kr.gmres(lambda v: A @ v, e.solve, F, m=w["m"], rtol=1e-10)
    print(f"GMRES({w['m']}): {info['iters']} iterations, relres {info['relres']:.3e}, "
          f"{time.perf_counter() - t0:.1f} s", flush=True)
    assert info["converged"]
    nodes = sample_nodes(n)
    np.savez(OUT, nodes=nodes, x=x[nodes], x_norm=np.linalg.norm(x), F_norm=np.linalg.norm(F),
             iters=info["iters"], relres=info["relres"])
    print(f"wrote {OUT} ({nodes.size} nodes)")


if __name__ == "__main__":
    main()
