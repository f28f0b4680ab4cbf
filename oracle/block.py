"""Block Krylov solvers for several right-hand sides under one shift (oracle, float64).

Test infrastructure: only tests/, the smoke check and the bench's CPU baseline
use this module; the library never does.

Section 7.2.2 solves a block of right-hand sides with block preconditioned
MINRES and reorthogonalises its Krylov basis; a block converges when
max_i ||b_i - A_mu x_i|| / ||b_i|| <= tol.  Both methods here act on the block
Krylov space K_k = span{P R0, (P A_mu) P R0, ..., (P A_mu)^{k-1} P R0} of the
preconditioned operator (P spd, C-RandRAND) and reorthogonalise in full.

* block_minres_cycle  Block Lanczos in the inner product of P: blocks V_j with
      V_i^T P V_j = delta_ij and Z_j = P V_j,
          W = A_mu Z_k - V_{k-1} C_k^T,  M_k = Z_k^T W,  W -= V_k M_k,
          W -= V (Z^T W) over every earlier block (two passes),
          S = W^T P W = C_{k+1}^T C_{k+1} (Cholesky),  V_{k+1} = W C_{k+1}^{-1},
      so that A_mu [Z_1..Z_k] = [V_1..V_{k+1}] T_k with T_k block tridiagonal
      (diagonal M_j, sub-diagonal C_{j+1}, super-diagonal C_j^T).  The iterate
      Y_k = [Z_1..Z_k] F minimises every column of the residual in the norm of P,
      F = argmin ||E_1 C_1 - T_k F||_F with R0 = V_1 C_1: the small
      least-squares problem is solved as it stands at every step (no rotations).
* block_cg_cycle  Block CG with A_mu-orthonormal direction blocks: D_k is
      P R_k made A_mu-orthogonal to every earlier D_j (two passes), then
      normalised by the Cholesky factor of D_k^T A_mu D_k; the update
      Y += D_k (D_k^T R_k), R -= A_mu D_k (D_k^T R_k) is the Galerkin step, so Y_k
      minimises every column's A_mu-norm error over K_k.
* solve_block   restarted driver (Algorithm RandRAND_PCG step 10 with eta): each
      cycle starts from the true residual block, keeps only the columns not yet at
      tol, and runs until every kept column i has ||r_i|| <= max(eta ||r_i^0||,
      tol ||b_i||), or after kmax steps.  Columns are solved in groups of at most
      `group` (in order).

A cycle stops with BREAKDOWN when the block it has to normalise is not
numerically full rank: a Cholesky pivot c_jj with c_jj^2 <= 1e-20 S_jj (the new
column j lies in the span of the others to 1e-10).  A breakdown after the first
step still returns the best iterate over the space built so far.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np

from .solvers import BREAKDOWN, NOCONV, OK

RANK_EPS = 1e-20


@dataclass
class BlockCycle:
    Y: np.ndarray
    its: int
    rn: np.ndarray           # 2-norm of every column of rhs - op(Y)
    status: int
    history: List[np.ndarray] = field(default_factory=list)   # rn after every step


@dataclass
class BlockResult:
    X: np.ndarray
    iters: np.ndarray        # block iterations of every column's group
    restarts: np.ndarray
    relres: np.ndarray       # true relative residual of every column
    status: int
    history: List[float] = field(default_factory=list)        # max_i relres_i per step


def chol_upper(S: np.ndarray) -> Optional[np.ndarray]:
    """Upper C with C^T C = S, or None when S is not numerically positive definite
    (a pivot below the RANK_EPS rule)."""
    S = 0.5 * (S + S.T)
    s = S.shape[0]
    C = np.zeros_like(S)
    for j in range(s):
        piv = S[j, j] - C[:j, j] @ C[:j, j]
        if not piv > RANK_EPS * S[j, j] or not S[j, j] > 0:
            return None
        C[j, j] = np.sqrt(piv)
        for k in range(j + 1, s):
            C[j, k] = (S[j, k] - C[:j, j] @ C[:j, k]) / C[j, j]
    return C


def _cols(R: np.ndarray) -> np.ndarray:
    return np.sqrt(np.sum(R * R, axis=0))


def block_minres_cycle(op: Callable, prec: Callable, R0: np.ndarray, targets: np.ndarray,
                       maxit: int, reorth: bool = True) -> BlockCycle:
    n, s = R0.shape
    W = R0.copy()
    Zt = prec(W)
    C1 = chol_upper(W.T @ Zt)
    if C1 is None:
        return BlockCycle(np.zeros_like(R0), 0, _cols(R0), BREAKDOWN)
    V = [np.linalg.solve(C1.T, W.T).T]          # W C1^{-1}
    Z = [np.linalg.solve(C1.T, Zt.T).T]
    U: List[np.ndarray] = []                       # A_mu Z_j
    T = np.zeros((s * 9, s * 8))                   # grown as the cycle lengthens
    hist: List[np.ndarray] = []
    Cprev = None
    Y = np.zeros_like(R0)
    rn = _cols(R0)
    for k in range(maxit):
        if (k + 2) * s > T.shape[0]:
            T2 = np.zeros((2 * T.shape[0], 2 * T.shape[1]))
            T2[:T.shape[0], :T.shape[1]] = T
            T = T2
        Uk = op(Z[k])
        U.append(Uk)
        W = Uk.copy()
        if k > 0:
            W -= V[k - 1] @ Cprev.T
            T[(k - 1) * s:k * s, k * s:(k + 1) * s] = Cprev.T
        M = Z[k].T @ W
        M = 0.5 * (M + M.T)
        W -= V[k] @ M
        T[k * s:(k + 1) * s, k * s:(k + 1) * s] = M
        if reorth:
            Vall, Zall = np.hstack(V), np.hstack(Z)
            for _ in range(2):
                W -= Vall @ (Zall.T @ W)
        Zt = prec(W)
        C = chol_upper(W.T @ Zt)
        rows = (k + 2) * s if C is not None else (k + 1) * s
        if C is not None:
            T[(k + 1) * s:(k + 2) * s, k * s:(k + 1) * s] = C
        rhs = np.zeros((rows, s))
        rhs[:s] = C1
        F = np.linalg.lstsq(T[:rows, :(k + 1) * s], rhs, rcond=None)[0]
        Y = np.hstack(Z) @ F
        Rk = R0 - np.hstack(U) @ F
        rn = _cols(Rk)
        hist.append(rn)
        if np.all(rn <= targets):
            return BlockCycle(Y, k + 1, rn, OK, hist)
        if C is None:
            return BlockCycle(Y, k + 1, rn, BREAKDOWN, hist)
        V.append(np.linalg.solve(C.T, W.T).T)
        Z.append(np.linalg.solve(C.T, Zt.T).T)
        Cprev = C
    return BlockCycle(Y, maxit, rn, NOCONV, hist)


def block_cg_cycle(op: Callable, prec: Callable, R0: np.ndarray, targets: np.ndarray,
                   maxit: int, reorth: bool = True) -> BlockCycle:
    R = R0.copy()
    Y = np.zeros_like(R0)
    D: List[np.ndarray] = []
    AD: List[np.ndarray] = []
    hist: List[np.ndarray] = []
    rn = _cols(R)
    for k in range(maxit):
        Dk = prec(R)
        passes = 2 if reorth else 1
        for _ in range(passes):
            js = range(len(D)) if reorth else range(max(len(D) - 1, 0), len(D))
            for j in js:
                Dk -= D[j] @ (AD[j].T @ Dk)
        ADk = op(Dk)
        L = chol_upper(Dk.T @ ADk)
        if L is None:
            return BlockCycle(Y, k, rn, BREAKDOWN, hist)
        Dk = np.linalg.solve(L.T, Dk.T).T
        ADk = np.linalg.solve(L.T, ADk.T).T
        a = Dk.T @ R
        Y += Dk @ a
        R -= ADk @ a
        D.append(Dk)
        AD.append(ADk)
        rn = _cols(R)
        hist.append(rn)
        if np.all(rn <= targets):
            return BlockCycle(Y, k + 1, rn, OK, hist)
    return BlockCycle(Y, maxit, rn, NOCONV, hist)


CYCLES = {"minres": block_minres_cycle, "cg": block_cg_cycle}


def _solve_group(Amu, Atrue, prec, B, tol, cycle, eta, maxit, reorth, kmax):
    n, m = B.shape
    X = np.zeros_like(B)
    nb = _cols(B)
    safe = np.where(nb > 0, nb, 1.0)
    its = cycles = 0
    hist: List[float] = []
    while True:
        Rt = B - Atrue(X)
        rel = _cols(Rt) / safe
        rel[nb == 0] = 0.0
        if len(hist) == its + 1:
            hist[its] = float(rel.max())
        else:
            hist.append(float(rel.max()))
        if np.all(rel <= tol):
            return X, its, max(cycles - 1, 0), rel, OK, hist
        if its >= maxit:
            return X, its, max(cycles - 1, 0), rel, NOCONV, hist
        act = np.flatnonzero(rel > tol)
        rn = rel * safe
        targets = np.maximum(eta * rn[act], tol * nb[act])
        cycles += 1
        c = cycle(Amu, prec, Rt[:, act], targets, min(maxit - its, kmax or maxit), reorth)
        X[:, act] += c.Y
        its += c.its
        done = rel.copy()
        for h in c.history:
            done[act] = h / nb[act]
            hist.append(float(done.max()))
        if c.status == BREAKDOWN and c.its == 0:
            Rt = B - Atrue(X)
            rel = _cols(Rt) / safe
            rel[nb == 0] = 0.0
            return X, its, max(cycles - 1, 0), rel, BREAKDOWN, hist


def solve_block(Amu: Callable, prec: Callable, B: np.ndarray, tol: float, method: str = "minres",
                eta: float = 1e-2, maxit: int = 5000, group: int = 32, reorth: bool = True,
                Amu_true: Optional[Callable] = None, kmax: Optional[int] = None) -> BlockResult:
    """Block MINRES or block CG on A_mu X = B (columns in groups of `group`).

    Amu and prec act on n x s blocks; Amu_true (default Amu) gives the residual
    at every restart.  iters counts block iterations (one product with A_mu per
    block of columns).  kmax: steps per cycle (a cycle that reaches it restarts
    from the true residual); None: no limit."""
    cycle = CYCLES[method]
    n, m = B.shape
    X = np.zeros_like(B)
    iters = np.zeros(m, dtype=np.int64)
    restarts = np.zeros(m, dtype=np.int64)
    relres = np.zeros(m)
    status = OK
    hist: List[float] = []
    for g0 in range(0, m, group):
        g1 = min(g0 + group, m)
        Xg, its, rs, rel, st, h = _solve_group(Amu, Amu_true or Amu, prec, B[:, g0:g1], tol, cycle,
                                              eta, maxit, reorth, kmax)
        X[:, g0:g1] = Xg
        iters[g0:g1] = its
        restarts[g0:g1] = rs
        relres[g0:g1] = rel
        if st != OK and status == OK:
            status = st
        hist = h if g0 == 0 else hist
    return BlockResult(X, iters, restarts, relres, status, hist)
