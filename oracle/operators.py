"""The operator of the shifted system (A + mu I) x = b, in float64.

Section 1 (eq. initsys): A is symmetric positive semidefinite and reached only
through matvecs u -> A u (or, for kernels, through its entries).  Kernel ridge
regression (Section 7.2.2, eq. kernel) gives A = K / n with K_ij = kappa(x_i, x_j).

Kernel formulas (the paper names the rbf kernel with a bandwidth but prints no
formula; these are the textbook forms):
  RBF          kappa(x, y) = exp(-kconst * ||x - y||^2),     kconst = 1/(2 sigma^2)
  Matern-3/2   kappa(x, y) = (1 + kconst*r) exp(-kconst*r),  r = ||x - y||, kconst = sqrt(3)/ell

Distances are formed by ``scipy.spatial.distance.cdist`` in float64 (difference
form), so the oracle's operator is the exact kernel of the float32 input points
up to float64 rounding.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
from scipy.spatial.distance import cdist

RBF = 1
MATERN32 = 2


def kernel_block(kind: int, kconst: float, Xr: np.ndarray, Xc: np.ndarray) -> np.ndarray:
    """Kernel values between row points Xr (m, d) and column points Xc (k, d)."""
    if kind == RBF:
        D2 = cdist(Xr, Xc, "sqeuclidean")
        return np.exp(-kconst * D2)
    if kind == MATERN32:
        R = cdist(Xr, Xc, "euclidean")
        t = kconst * R
        return (1.0 + t) * np.exp(-t)
    raise ValueError(kind)


def _default_threads() -> int:
    """ORACLE_THREADS if set, else the CPU count capped by OMP_NUM_THREADS (the host share
    a shared machine grants this process)."""
    if os.environ.get("ORACLE_THREADS"):
        return max(1, int(os.environ["ORACLE_THREADS"]))
    n = os.cpu_count() or 1
    try:
        return max(1, min(n, int(os.environ.get("OMP_NUM_THREADS", n))))
    except ValueError:
        return n


class Operator:
    """A = scale * K(X, X) (kernel) or a stored dense symmetric A, both float64."""

    def __init__(self, dense: np.ndarray | None = None, kind: int = 0, pts=None,
                 kconst: float = 0.0, scale: float = 1.0, threads: int | None = None,
                 block: int = 512):
        self.dense = None if dense is None else np.asarray(dense, dtype=np.float64)
        self.kind = kind
        self.kconst = float(kconst)
        self.scale = float(scale)
        self.block = block
        self.threads = threads or _default_threads()
        if self.dense is not None:
            self.n = self.dense.shape[0]
            self.X = None
        else:
            self.X = np.asarray(pts, dtype=np.float64).T.copy()   # (n, d)
            self.n = self.X.shape[0]

    @classmethod
    def from_problem(cls, prob, dense: bool | None = None, **kw):
        op = cls(kind=prob.kind, pts=prob.pts, kconst=prob.kconst, scale=prob.scale, **kw)
        if dense if dense is not None else prob.dense:
            return cls(dense=op.to_dense(), **kw)
        return op

    def to_dense(self) -> np.ndarray:
        if self.dense is not None:
            return self.dense.copy()
        return self.scale * kernel_block(self.kind, self.kconst, self.X, self.X)

    def _row_blocks(self):
        return [(i, min(i + self.block, self.n)) for i in range(0, self.n, self.block)]

    def matmat(self, U: np.ndarray) -> np.ndarray:
        """A @ U for U of shape (n,) or (n, m)."""
        if self.dense is not None:
            return self.dense @ U
        out = np.empty_like(U, dtype=np.float64)

        def work(rng):
            i0, i1 = rng
            Kb = kernel_block(self.kind, self.kconst, self.X[i0:i1], self.X)
            out[i0:i1] = self.scale * (Kb @ U)

        blocks = self._row_blocks()
        if self.threads > 1 and len(blocks) > 1:
            with ThreadPoolExecutor(self.threads) as ex:
                list(ex.map(work, blocks))
        else:
            for b in blocks:
                work(b)
        return out

    def shifted(self, mu: float):
        """The matvec u -> A_mu u = A u + mu u (Section 1)."""
        return lambda U: self.matmat(U) + mu * U
