"""Writes precision_matern32_n65536_xstar.npy: the direct solution x* = (K + mu I)^{-1} b
of the precision workload (stored dense Matern-3/2 on 65,536 points in [0,1]^3,
ell = 0.1, mu = 1e-5), by the oracle's dense float64 Cholesky solve.

The matrix is formed by the oracle's kernel formula in row blocks into one
n x n float64 array (34 GB) and factored in place by column panels (one LAPACK
call on the whole array would overflow LP64 LAPACK's 32-bit offsets).  Run from the repository
root: python tests/golden/make_precision_xstar.py
"""
import os
import sys
import time

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))

import workloads  # noqa: E402
from oracle import solvers  # noqa: E402
from oracle.operators import kernel_block  # noqa: E402


def main():
    prob = workloads.cfg_precision()
    n = prob.n
    X = prob.pts.T.astype(np.float64)
    A = np.empty((n, n))
    t0 = time.time()
    blk = 2048
    for i0 in range(0, n, blk):
        i1 = min(i0 + blk, n)
        A[i0:i1] = prob.scale * kernel_block(prob.kind, prob.kconst, X[i0:i1], X)
    print(f"matrix formed in {time.time() - t0:.0f} s", flush=True)
    x = solvers.direct_blocked(A, prob.mus[0], prob.b,
                               log=lambda m: print(f"{m} ({time.time() - t0:.0f} s)", flush=True))
    print(f"solved in {time.time() - t0:.0f} s", flush=True)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "precision_matern32_n65536_xstar.npy")
    np.save(out, x)
    print("wrote", out, flush=True)


if __name__ == "__main__":
    main()
