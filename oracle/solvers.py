"""Krylov solvers and the direct reference solve (oracle, float64).

* pcg         C-RandRAND PCG with restarts (Algorithm RandRAND_PCG steps 5-11,
              Section 6.2).  Hestenes-Stiefel recurrences in this order per
              iteration: w = A_mu p; alpha = rho / p^T w; x += alpha p;
              r -= alpha w; (stop test on ||r||); z = P r; rho' = r^T z;
              beta = rho'/rho; p = z + beta p.
              Restart after every drop of the residual norm by eta = 1e-2
              (Section 7, experimental setup): the true residual b - A_mu x is
              recomputed, z = P r and p = z.  The relative residual
              ||b - A_mu x|| / ||b|| is the stop test, with the recurrence
              residual inside a restart cycle and the true residual at each
              restart and at the end.
* cg          the same loop with P = I (plain CG, Section 1).
* direct      x* = (A + mu I)^{-1} b by a dense Cholesky solve (LAPACK);
              direct_blocked the same factorisation by column panels in the
              caller's array, for n^2 beyond LP64 LAPACK's 32-bit offsets.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np
import scipy.linalg as sla

OK, NOCONV, BREAKDOWN = 0, 5, 4


@dataclass
class SolveResult:
    x: np.ndarray
    iters: int
    restarts: int
    relres: float
    status: int
    # history[k]: relative residual after k iterations (the recurrence residual
    # inside a cycle, the true residual where a cycle starts and at the end)
    history: List[float] = field(default_factory=list)
    # the true relative residual at the start of every cycle and at the end
    cycle_history: List[float] = field(default_factory=list)


def pcg(Amu: Callable, P: Callable, b: np.ndarray, tol: float, x0: Optional[np.ndarray] = None,
        eta: float = 1e-2, maxit: int = 5000, Amu_true: Optional[Callable] = None) -> SolveResult:
    """C-RandRAND PCG with restarts.

    Amu       working operator used inside the iteration.
    Amu_true  operator used for the residual at each restart (outer iterative
              refinement); defaults to Amu.
    """
    Atrue = Amu_true or Amu
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    nb = float(np.linalg.norm(b))
    if nb == 0.0:
        return SolveResult(np.zeros_like(b), 0, 0, 0.0, OK)
    its = 0
    cycles = 0
    hist: List[float] = []
    cyc: List[float] = []

    def record(k: int, value: float):
        # index k = iterations done; a true residual replaces the recurrence value
        if len(hist) == k + 1:
            hist[k] = value
        else:
            hist.append(value)

    def result(status, relres):
        return SolveResult(x, its, max(cycles - 1, 0), relres, status, hist, cyc)

    while True:
        r = b - Atrue(x)
        rn = float(np.linalg.norm(r))
        record(its, rn / nb)
        cyc.append(rn / nb)
        if rn <= tol * nb:
            return result(OK, rn / nb)
        if its >= maxit:
            return result(NOCONV, rn / nb)
        cycles += 1
        target = max(eta * rn, tol * nb)
        z = P(r)
        p = z.copy()
        rho = float(r @ z)
        if not rho > 0:
            return result(BREAKDOWN, rn / nb)
        while its < maxit:
            w = Amu(p)
            pw = float(p @ w)
            if not pw > 0:
                return result(BREAKDOWN, rn / nb)
            alpha = rho / pw
            x = x + alpha * p
            r = r - alpha * w
            its += 1
            rn = float(np.linalg.norm(r))
            record(its, rn / nb)
            if rn <= target:
                break
            z = P(r)
            rho_new = float(r @ z)
            if not rho_new > 0:
                return result(BREAKDOWN, rn / nb)
            beta = rho_new / rho
            p = z + beta * p
            rho = rho_new


def cg(Amu: Callable, b: np.ndarray, tol: float, **kw) -> SolveResult:
    """Plain unpreconditioned CG: the same loop and stop rule with P = I."""
    return pcg(Amu, lambda r: r.copy(), b, tol, **kw)


def direct(A_dense: np.ndarray, mu: float, b: np.ndarray) -> np.ndarray:
    """x* = (A + mu I)^{-1} b by Cholesky (LAPACK potrf/potrs)."""
    n = A_dense.shape[0]
    c = sla.cho_factor(A_dense + mu * np.eye(n), lower=False)
    return sla.cho_solve(c, b)


def direct_blocked(A_dense: np.ndarray, mu: float, b: np.ndarray, nb: int = 2048,
                   log: Optional[Callable[[str], None]] = None) -> np.ndarray:
    """direct() for a matrix too large for one LAPACK call (an n x n array with
    n^2 >= 2^31 overflows the 32-bit element offsets of LP64 LAPACK): the same
    Cholesky factorisation A + mu I = L L^T, right-looking by column panels of nb
    (LAPACK on each nb x nb diagonal block, triangular solves for the panel below
    it, the trailing lower triangle updated by GEMMs in row chunks), then the two
    triangular solves by the same panels.  Works in the caller's row-major array,
    whose lower triangle holds L afterwards."""
    n = A_dense.shape[0]
    A = A_dense
    A[np.diag_indices_from(A)] += mu
    for k0 in range(0, n, nb):
        k1 = min(k0 + nb, n)
        L11 = np.linalg.cholesky(A[k0:k1, k0:k1])
        A[k0:k1, k0:k1] = L11
        if k1 < n:
            # L21 = A21 L11^{-T}
            A[k1:, k0:k1] = sla.solve_triangular(L11, A[k1:, k0:k1].T, lower=True).T
            L21 = A[k1:, k0:k1]
            for r0 in range(k1, n, nb):
                r1 = min(r0 + nb, n)
                # rows r0..r1 of the trailing block, columns k1..r1 (lower part)
                A[r0:r1, k1:r1] -= L21[r0 - k1:r1 - k1] @ L21[:r1 - k1].T
        if log:
            log(f"panel {k0 // nb + 1} of {(n + nb - 1) // nb}")
    y = np.array(b, dtype=np.float64)
    for k0 in range(0, n, nb):
        k1 = min(k0 + nb, n)
        if k0:
            y[k0:k1] -= A[k0:k1, :k0] @ y[:k0]
        y[k0:k1] = sla.solve_triangular(A[k0:k1, k0:k1], y[k0:k1], lower=True)
    x = y
    for k1 in range(n, 0, -nb):
        k0 = max(k1 - nb, 0)
        if k1 < n:
            x[k0:k1] -= A[k1:, k0:k1].T @ x[k1:]
        x[k0:k1] = sla.solve_triangular(A[k0:k1, k0:k1], x[k0:k1], lower=True, trans="T")
    return x


def relres(Amu_true: Callable, x: np.ndarray, b: np.ndarray) -> float:
    """||b - A_mu x|| / ||b|| with the float64 operator (per column for 2-D input)."""
    r = b - Amu_true(x)
    if b.ndim == 1:
        return float(np.linalg.norm(r) / np.linalg.norm(b))
    return np.linalg.norm(r, axis=0) / np.linalg.norm(b, axis=0)
