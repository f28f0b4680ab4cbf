"""R-RandRAND, split R-RandRAND and MINRES solvers (oracle, float64).

Test infrastructure: only tests/, the smoke check and the bench's CPU baseline
use this module; the library never does.

* Krylov cycles on an spd operator, started from y = 0:
    cg_cycle      conjugate gradients (Hestenes-Stiefel), plain or preconditioned;
    minres_cycle  preconditioned MINRES (Paige and Saunders, SIAM J. Numer. Anal.
                  12(4), 1975): preconditioned Lanczos, Givens QR of the
                  tridiagonal, three-term update of the search directions.  The
                  2-norm residual rhs - op(y) is carried along (r <- r - phi op(w),
                  with op(w) updated by the same three-term recurrence as w), and a
                  cycle stops when it falls below the cycle's target.
* r_randrand   Algorithm RandRAND_CG (Section 6.1): a Krylov method on the
               right-preconditioned operator B = (I-Pi) A_mu (I-Pi) + tau Pi
               (eq. APdef2), then x = x0 + A_mu^{-1} Pi (tau y - A_mu (I-Pi) y)
               + (I-Pi) y (eq. APdef3), with A_mu^{-1} Pi u = Omega R^{-1} Q^T u
               (eq. projector); restart after every residual drop by eta.
* split_r_randrand  Algorithm RandRAND_CG_split (Section 3.1, split R-RandRAND):
               a Krylov method on E y = (I-Pi) b_c with E u = (I-Pi) A_mu u
               (eq. APdef2_reduced), then x = x0 + A_mu^{-1} Pi (b_c - A_mu y) + y.
* c_randrand_minres  Algorithm RandRAND_PCG with its MINRES branch: preconditioned
               MINRES on A_mu x = b with the C-RandRAND preconditioner.

The projector is the refined one of eq. accurate_proj, Pi = Q T Q^T with
T = 2I - Q^T Q, and A_mu^{-1} Pi u = Omega R^{-1} T Q^T u (the same reading as the
C-RandRAND core).  tau for R-RandRAND is ||E|| (eq. cnd_bound with rho = 1, the
paper's experimental setup), E = (I-Pi) A_mu (I-Pi).

Each outer cycle starts from the true residual b - A_mu x (the float64 operator
Amu_true when given); the cycle's Krylov residual is the residual of the
recovered x in exact arithmetic (right preconditioning and the split identity
b_c - A_mu x = (I-Pi) b_c - E y), so the stopping rule is the same as PCG's.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np
import scipy.linalg as sla

from .solvers import BREAKDOWN, NOCONV, OK, SolveResult


@dataclass
class Cycle:
    y: np.ndarray
    its: int
    rn: float
    status: int
    history: List[float] = field(default_factory=list)


def cg_cycle(op: Callable, rhs: np.ndarray, target: float, maxit: int,
             prec: Optional[Callable] = None) -> Cycle:
    """(P)CG on op(y) = rhs from y = 0 until the recurrence residual is <= target."""
    y = np.zeros_like(rhs)
    r = rhs.copy()
    z = prec(r) if prec else r.copy()
    p = z.copy()
    rho = float(r @ z)
    hist = []
    if not rho > 0:
        return Cycle(y, 0, float(np.linalg.norm(r)), BREAKDOWN, hist)
    its = 0
    rn = float(np.linalg.norm(r))
    while its < maxit:
        w = op(p)
        pw = float(p @ w)
        if not pw > 0:
            return Cycle(y, its, rn, BREAKDOWN, hist)
        alpha = rho / pw
        y = y + alpha * p
        r = r - alpha * w
        its += 1
        rn = float(np.linalg.norm(r))
        hist.append(rn)
        if rn <= target:
            return Cycle(y, its, rn, OK, hist)
        z = prec(r) if prec else r.copy()
        rho_new = float(r @ z)
        if not rho_new > 0:
            return Cycle(y, its, rn, BREAKDOWN, hist)
        p = z + (rho_new / rho) * p
        rho = rho_new
    return Cycle(y, its, rn, NOCONV, hist)


def minres_cycle(op: Callable, rhs: np.ndarray, target: float, maxit: int,
                 prec: Optional[Callable] = None, record_pnorm: bool = False) -> Cycle:
    """Preconditioned MINRES on op(y) = rhs from y = 0 (spd preconditioner prec).

    Lanczos with the preconditioner's inner product: v_k = z_k / beta_k with
    z_k = prec(r_k) and beta_k^2 = r_k^T z_k; T_k is reduced to upper triangular
    form by Givens rotations (cs, sn); the solution and its residual move along
    w_k = (v_k - eps_k w_{k-2} - delta_k w_{k-1}) / gamma_k by phi_k.
    record_pnorm: history holds phibar_k (the preconditioner-norm residual the
    method minimises) instead of the 2-norm residual.
    """
    n = rhs.shape[0]
    y = np.zeros_like(rhs)
    res = rhs.copy()                 # rhs - op(y), tracked
    r1 = rhs.copy()
    z = prec(r1) if prec else r1.copy()
    beta1 = float(r1 @ z)
    hist: List[float] = []
    if not beta1 > 0:
        return Cycle(y, 0, float(np.linalg.norm(res)), BREAKDOWN if beta1 < 0 else OK, hist)
    beta1 = np.sqrt(beta1)
    r2 = r1.copy()
    beta, oldb = beta1, 0.0
    dbar = epsln = 0.0
    phibar = beta1
    cs, sn = -1.0, 0.0
    w = np.zeros(n); w2 = np.zeros(n)
    aw = np.zeros(n); aw2 = np.zeros(n)
    its = 0
    rn = float(np.linalg.norm(res))
    while its < maxit:
        v = z / beta
        av = op(v)
        t = av - (beta / oldb) * r1 if its > 0 else av.copy()
        alfa = float(v @ t)
        t = t - (alfa / beta) * r2
        r1, r2 = r2, t
        z = prec(r2) if prec else r2.copy()
        oldb = beta
        b2 = float(r2 @ z)
        if b2 < 0:
            return Cycle(y, its, rn, BREAKDOWN, hist)
        beta = np.sqrt(b2)
        # apply the previous rotation, then form the new one
        oldeps = epsln
        delta = cs * dbar + sn * alfa
        gbar = sn * dbar - cs * alfa
        epsln = sn * beta
        dbar = -cs * beta
        gamma = float(np.hypot(gbar, beta))
        if gamma == 0.0:
            return Cycle(y, its, rn, BREAKDOWN, hist)
        cs, sn = gbar / gamma, beta / gamma
        phi = cs * phibar
        phibar = sn * phibar
        w1, w2 = w2, w
        w = (v - oldeps * w1 - delta * w2) / gamma
        aw1, aw2 = aw2, aw
        aw = (av - oldeps * aw1 - delta * aw2) / gamma
        y = y + phi * w
        res = res - phi * aw
        its += 1
        rn = float(np.linalg.norm(res))
        hist.append(float(phibar) if record_pnorm else rn)
        if rn <= target:
            return Cycle(y, its, rn, OK, hist)
        if beta == 0.0:
            return Cycle(y, its, rn, OK, hist)
    return Cycle(y, its, rn, NOCONV, hist)


def _cycle(krylov: str):
    if krylov == "cg":
        return cg_cycle
    if krylov == "minres":
        return minres_cycle
    raise ValueError(krylov)


class Projections:
    """Pi = Q T Q^T (eq. accurate_proj), (I-Pi), and A_mu^{-1} Pi = Omega R^{-1} T Q^T."""

    def __init__(self, Q: np.ndarray, T: np.ndarray, R: np.ndarray, Omega: np.ndarray):
        self.Q, self.T, self.R, self.Omega = Q, T, R, Omega

    def pi(self, u):
        return self.Q @ (self.T @ (self.Q.T @ u))

    def comp(self, u):
        return u - self.pi(u)

    def amu_inv_pi(self, u):
        h = sla.solve_triangular(self.R, self.T @ (self.Q.T @ u), lower=False)
        return self.Omega @ h


def _outer(Amu, Atrue, b, tol, eta, maxit, x0, cycle_fn):
    """Restarted driver: true residual, cycle target max(eta ||r||, tol ||b||)."""
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    nb = float(np.linalg.norm(b))
    if nb == 0.0:
        return SolveResult(np.zeros_like(b), 0, 0, 0.0, OK)
    its = cycles = 0
    hist: List[float] = []
    cyc: List[float] = []
    while True:
        rc = b - Atrue(x)
        rn = float(np.linalg.norm(rc))
        if len(hist) == its + 1:
            hist[its] = rn / nb
        else:
            hist.append(rn / nb)
        cyc.append(rn / nb)
        if rn <= tol * nb:
            return SolveResult(x, its, max(cycles - 1, 0), rn / nb, OK, hist, cyc)
        if its >= maxit:
            return SolveResult(x, its, max(cycles - 1, 0), rn / nb, NOCONV, hist, cyc)
        cycles += 1
        target = max(eta * rn, tol * nb)
        dx, c = cycle_fn(rc, target, maxit - its)
        x = x + dx
        its += c.its
        hist.extend(h / nb for h in c.history)
        if c.status == BREAKDOWN:
            return SolveResult(x, its, cycles - 1, c.rn / nb, BREAKDOWN, hist, cyc)


def r_randrand(Amu: Callable, proj: Projections, tau: float, b: np.ndarray, tol: float,
               krylov: str = "cg", eta: float = 1e-2, maxit: int = 5000,
               x0: Optional[np.ndarray] = None, Amu_true: Optional[Callable] = None) -> SolveResult:
    """Algorithm RandRAND_CG (R-RandRAND CG/MINRES) with restarts."""
    def B(u):
        v = proj.comp(u)
        return proj.comp(Amu(v)) + tau * proj.pi(u)

    def cycle(rc, target, left):
        c = _cycle(krylov)(B, rc, target, left)
        u = proj.comp(c.y)
        dx = proj.amu_inv_pi(tau * c.y - Amu(u)) + u
        return dx, c

    return _outer(Amu, Amu_true or Amu, b, tol, eta, maxit, x0, cycle)


def split_r_randrand(Amu: Callable, proj: Projections, b: np.ndarray, tol: float,
                     krylov: str = "cg", eta: float = 1e-2, maxit: int = 5000,
                     x0: Optional[np.ndarray] = None,
                     Amu_true: Optional[Callable] = None) -> SolveResult:
    """Algorithm RandRAND_CG_split (split R-RandRAND CG/MINRES) with restarts.

    b_p = (I-Pi)(I-Pi) b_c (the re-orthogonalised projection of the remark after
    Alg. RandRAND_CG_split's introduction); E u = (I-Pi) A_mu u on range(I-Pi)."""
    def E(u):
        return proj.comp(Amu(u))

    def cycle(rc, target, left):
        bp = proj.comp(proj.comp(rc))
        c = _cycle(krylov)(E, bp, target, left)
        dx = proj.amu_inv_pi(rc - Amu(c.y)) + c.y
        return dx, c

    return _outer(Amu, Amu_true or Amu, b, tol, eta, maxit, x0, cycle)


def c_randrand_minres(Amu: Callable, P: Callable, b: np.ndarray, tol: float, eta: float = 1e-2,
                      maxit: int = 5000, x0: Optional[np.ndarray] = None,
                      Amu_true: Optional[Callable] = None) -> SolveResult:
    """Algorithm RandRAND_PCG, MINRES branch: preconditioned MINRES with restarts."""
    def cycle(rc, target, left):
        c = minres_cycle(Amu, rc, target, left, prec=P)
        return c.y, c

    return _outer(Amu, Amu_true or Amu, b, tol, eta, maxit, x0, cycle)


def minres(Amu: Callable, b: np.ndarray, tol: float, **kw) -> SolveResult:
    """Plain MINRES with the same restarts and stopping rule."""
    return c_randrand_minres(Amu, lambda r: r.copy(), b, tol, **kw)
