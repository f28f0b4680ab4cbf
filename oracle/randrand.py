"""C-RandRAND preconditioner construction in float64 (oracle).

Follows, in order, Algorithm RandRAND_PCG steps 1-4 of the paper (Section 6.2)
with the explicit-basis representation of Section 4.1:

1. sketch            Y_mu = A Omega + mu Omega                      (eq. Rdef, q = 0)
2. orthogonalise     Y_mu = Q R by Cholesky QR (Algorithm chol_qr) or by the
                     sketched/preconditioned Cholesky QR (Algorithm prec_chol_qr)
3. core              G = R^{-T} (Omega^T A_mu Omega) R^{-1}         (eq. g_randrand_explicit)
                     in the spd-safe form G = (R_Omega R^{-1})^T (R_Omega R^{-1}),
                     R_Omega^T R_Omega = Omega^T A_mu Omega          (remark after Alg. RandRAND_PCG)
4. refined projector T = 2I - Q^T Q                                   (eq. accurate_proj)
5. tau               OPT: tau = sqrt(mu ||E|| / lam)  (eq. optimal_rho with F = 1/mu,
                          inserted in eq. c_randrand_tau)
                     RHO: tau = rho ||E|| / lam        (eq. c_randrand_tau)
                     NYS: tau = ||Pi A_mu^{-1} Pi||^{-1} = 1/lambda_max(G) (eq. nys_tau)
                     with ||E|| and lam = lambda_max(Pi A_mu Pi A_mu^{-1} Pi) from power
                     iterations (Section 3.2).
6. apply             P = I - Pi + tau Pi~,  Pi = Q T Q^T,  Pi~ = Q T G T Q^T
                     = I + Q K Q^T with K = tau T G T - T   (eq. g_randrand_explicit,
                     refined with eq. accurate_proj).

Several shifts (Section 5.1): joint basis Q_joint = qr([Omega, A Omega]) and, per
mu, a QR of the 2l x l reduced matrix Q_joint^T A Omega + mu Q_joint^T Omega.

Readings where the paper is silent are listed in the design notes; the main ones:
q = 0; power iterations N_pow = 10 from counter-generated Gaussian starts
(streams seed+2 for ||E||, seed+3 for lam); estimate = ||op(v)|| for unit v;
Cholesky failure ladder alpha in {1e-14, ..., 1e-1} * max_i W_ii (Appendix C);
Algorithm prec_chol_qr returns R = R_chol R_sk (the product order that makes
Y = Q R hold).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np
import scipy.linalg as sla

from . import rng as _rng

OPT, RHO, NYS = 0, 1, 2
SKETCHED_CHOLQR, CHOLQR = 0, 1


class NotSPD(Exception):
    pass


def chol_upper_ladder(W: np.ndarray):
    """Upper Cholesky factor R (R^T R = W); on failure add alpha I (Appendix C ladder).

    Returns (R, alpha_used).
    """
    W = 0.5 * (W + W.T)
    try:
        return sla.cholesky(W, lower=False), 0.0
    except np.linalg.LinAlgError:
        pass
    wn = float(np.max(np.abs(np.diag(W))))
    for e in range(-14, 0):
        alpha = (10.0 ** e) * wn
        try:
            return sla.cholesky(W + alpha * np.eye(W.shape[0]), lower=False), alpha
        except np.linalg.LinAlgError:
            continue
    raise NotSPD("Cholesky ladder exhausted")


def householder_r(S: np.ndarray) -> np.ndarray:
    """R factor of a Householder QR (LAPACK geqrf via numpy), diagonal made positive."""
    R = np.linalg.qr(S, mode="r")
    sgn = np.sign(np.diag(R))
    sgn[sgn == 0] = 1.0
    return sgn[:, None] * R


def householder_qr(S: np.ndarray):
    Q, R = np.linalg.qr(S, mode="reduced")
    sgn = np.sign(np.diag(R))
    sgn[sgn == 0] = 1.0
    return Q * sgn[None, :], sgn[:, None] * R


def tri_inv_upper(R: np.ndarray) -> np.ndarray:
    return sla.solve_triangular(R, np.eye(R.shape[0]), lower=False)


def cholqr(Y: np.ndarray):
    """Algorithm chol_qr: G = Y^T Y, R = chol(G), Q = Y R^{-1}."""
    R, _ = chol_upper_ladder(Y.T @ Y)
    Q = Y @ tri_inv_upper(R)
    return Q, R


def sketched_cholqr(Y: np.ndarray, Theta: np.ndarray):
    """Algorithm prec_chol_qr with the explicit Q of Section 4.1.

    S = Theta Y; R_sk = qr(S); W = Y R_sk^{-1}; G = W^T W; R_chol = chol(G);
    Q = W R_chol^{-1}; R = R_chol R_sk.
    """
    S = np.asarray(Theta @ Y)
    R_sk = householder_r(S)
    W = Y @ tri_inv_upper(R_sk)
    R_c, _ = chol_upper_ladder(W.T @ W)
    Q = W @ tri_inv_upper(R_c)
    return Q, R_c @ R_sk


def power_norm(op: Callable[[np.ndarray], np.ndarray], v0: np.ndarray, iters: int) -> float:
    """Power iteration: v <- op(v)/||op(v)||; returns ||op(v)|| for the last unit v."""
    v = v0 / np.linalg.norm(v0)
    lam = 0.0
    for _ in range(iters):
        w = op(v)
        lam = float(np.linalg.norm(w))
        if lam == 0.0:
            return 0.0
        v = w / lam
    return lam


@dataclass
class Precond:
    """C-RandRAND preconditioner P = I + Qb (Kc) Qb^T for one shift mu.

    For a single shift Qb = Q (n x l) and Kc = K_tau (l x l).  For the joint
    basis Qb = Q_joint (n x 2l) and Kc = Q_red K_tau Q_red^T (2l x 2l).
    """
    mu: float
    Q: Optional[np.ndarray]
    R: Optional[np.ndarray]
    G: Optional[np.ndarray]
    T: Optional[np.ndarray]
    K: Optional[np.ndarray]
    tau: float
    normE: float
    lam: float
    Qb: Optional[np.ndarray] = None
    Kc: Optional[np.ndarray] = None
    extras: dict = field(default_factory=dict)

    def apply(self, r: np.ndarray) -> np.ndarray:
        if self.Qb is None:
            return r.copy()
        return r + self.Qb @ (self.Kc @ (self.Qb.T @ r))

    @property
    def l(self) -> int:
        return 0 if self.Q is None else self.Q.shape[1]

    def dense(self) -> np.ndarray:
        n = self.Qb.shape[0]
        return np.eye(n) + self.Qb @ self.Kc @ self.Qb.T


def _core(Omega, Y_mu, R):
    """G = (R_Omega R^{-1})^T (R_Omega R^{-1}) with R_Omega = chol(Omega^T A_mu Omega)."""
    C = Omega.T @ Y_mu
    R_om, _ = chol_upper_ladder(0.5 * (C + C.T))
    H = R_om @ tri_inv_upper(R)
    return H.T @ H


def _tau(rule, mu, rho, Amu, Q, T, G, seed, n, power_iters):
    """tau and the two power-iteration estimates (||E||, lam) for one shift."""
    def Pi(u):
        return Q @ (T @ (Q.T @ u))

    def Pi_tilde(u):
        return Q @ (T @ (G @ (T @ (Q.T @ u))))

    def E(u):
        v = u - Pi(u)
        w = Amu(v)
        return w - Pi(w)

    def M(u):
        return Pi(Amu(Pi_tilde(u)))

    normE = lam = float("nan")
    if rule == NYS:
        # tau = ||Pi A_mu^{-1} Pi||^{-1}; Pi A_mu^{-1} Pi has the nonzero spectrum of G
        tau = 1.0 / float(np.max(np.linalg.eigvalsh(0.5 * (G + G.T))))
        return tau, normE, lam
    normE = power_norm(E, _rng.gaussian_vector(seed + 2, n), power_iters)
    lam = power_norm(M, _rng.gaussian_vector(seed + 3, n), power_iters)
    if normE == 0.0:
        # range(Q) is the whole space (E = 0): eq. c_randrand_tau would give tau = 0
        # and a singular P; use eq. nys_tau instead
        return 1.0 / float(np.max(np.linalg.eigvalsh(0.5 * (G + G.T)))), normE, lam
    if rule == OPT and mu > 0:
        tau = float(np.sqrt(mu * normE / lam))
    else:
        tau = rho * normE / lam
    return tau, normE, lam


def apply_core(tau, T, G, reorth: bool = False):
    """Core K of P = I + Q K Q^T.

    Default: P = I - Pi + tau Pi~ with the refined Pi = Q T Q^T, Pi~ = Q T G T Q^T
    (eq. g_randrand_explicit with eq. accurate_proj): K = tau T G T - T.
    reorth: the re-orthogonalised C-RandRAND of eq. c_randrand_reorth,
    P = (I-Pi)(I-Pi) + tau (I - (I-Pi)(I-Pi)) A_mu^{-1} Pi with Pi = Q Q^T and
    A_mu^{-1} Pi = Omega R^{-1} Q^T.  Since (I-Pi)(I-Pi) = I - Q T Q^T and
    Q^T Omega R^{-1} = G for Q = A_mu Omega R^{-1}, this is K = tau T G - T (not
    symmetric when Q is not exactly orthonormal)."""
    return tau * (T @ G) - T if reorth else tau * (T @ G @ T) - T


def _finish(mu, Amu, Q, R, C, T, tau_rule, rho, seed, n, power_iters, Qb=None, Qred=None,
            reorth: bool = False):
    """G, tau and the apply core from the basis of one shift (shared tail of build)."""
    R_om, _ = chol_upper_ladder(0.5 * (C + C.T))
    H = R_om @ tri_inv_upper(R)
    G = H.T @ H
    tau, normE, lam = _tau(tau_rule, mu, rho, Amu, Q, T, G, seed, n, power_iters)
    K = apply_core(tau, T, G, reorth)
    if Qb is None:
        return Precond(mu, Q, R, G, T, K, tau, normE, lam, Qb=Q, Kc=K)
    return Precond(mu, Q, R, G, T, K, tau, normE, lam, Qb=Qb, Kc=Qred @ K @ Qred.T,
                   extras={"Qred": Qred})


def test_matrix(op, sketch: str, seed: int, l: int, q: int = 0, omega_bf16: bool = False,
                Omega: Optional[np.ndarray] = None) -> np.ndarray:
    """Omega = A^q X (eq. testmatrix; the sketch is then A_mu Omega = A_mu A^q X).

    X is the generator's Gaussian or SRHT matrix (drawn in bf16 when omega_bf16);
    with q = 1 the product A X is rounded to bf16 as well in that mode, so the bf16
    MFMA sketch sees Omega exactly."""
    X = _rng.omega(sketch, seed, op.n, l, bf16=omega_bf16) if Omega is None else Omega
    if q == 0:
        return X
    if q != 1:
        raise ValueError("q must be 0 or 1")
    AX = op.matmat(X)
    return _rng.round_bf16(AX) if omega_bf16 else AX


def build(op, mus: List[float], l: int, sketch: str = "gaussian", seed: int = 0,
          orth: int = SKETCHED_CHOLQR, tau_rule: int = OPT, rho: float = 1.0,
          power_iters: int = 4, Omega: Optional[np.ndarray] = None,
          omega_bf16: bool = False, q: int = 0, multi: str = "joint",
          reorth: bool = False) -> List[Precond]:
    """Build one C-RandRAND preconditioner per shift (Algorithm RandRAND_PCG steps 1-4).

    omega_bf16: the test matrix is drawn in bfloat16 (as the float32-precision
    kernel path and the mixed-precision dense path do); SRHT entries are unchanged.
    q: power of eq. testmatrix (Omega = A^q X, q in {0, 1}).
    multi (several shifts): "joint" = the joint basis orth([Omega, A Omega]) with a
    reduced QR per shift (Section 5.1); "shifted_chol" = the shifted Cholesky
    technique of Section 5.1 (see build_shifted_cholesky).
    """
    n = op.n
    if l == 0:
        return [Precond(mu, None, None, None, None, None, 1.0, float("nan"), float("nan"))
                for mu in mus]
    Omega = test_matrix(op, sketch, seed, l, q, omega_bf16, Omega)
    if len(mus) == 1:
        mu = mus[0]
        Amu = op.shifted(mu)
        Y = op.matmat(Omega) + mu * Omega
        if orth == SKETCHED_CHOLQR:
            Q, R = sketched_cholqr(Y, _rng.theta(seed, n, l))
        else:
            Q, R = cholqr(Y)
        T = 2.0 * np.eye(l) - Q.T @ Q
        return [_finish(mu, Amu, Q, R, Omega.T @ Y, T, tau_rule, rho, seed, n, power_iters,
                        reorth=reorth)]
    if multi == "shifted_chol":
        return build_shifted_cholesky(op, mus, l, Omega, seed, orth, tau_rule, rho, power_iters)
    if multi != "joint":
        raise ValueError(multi)
    # several shifts sharing one joint basis (Section 5.1)
    AO = op.matmat(Omega)
    Z = np.concatenate([Omega, AO], axis=1)
    if orth == SKETCHED_CHOLQR:
        Qj, _ = sketched_cholqr(Z, _rng.theta(seed, n, 2 * l))
    else:
        Qj, _ = cholqr(Z)
    Zj = Qj.T @ AO
    Oj = Qj.T @ Omega
    OAO = Omega.T @ AO
    OO = Omega.T @ Omega
    QjtQj = Qj.T @ Qj
    out = []
    for mu in mus:
        Amu = op.shifted(mu)
        Qred, R = householder_qr(Zj + mu * Oj)
        Q = Qj @ Qred
        T = 2.0 * np.eye(l) - Qred.T @ QjtQj @ Qred
        out.append(_finish(mu, Amu, Q, R, OAO + mu * OO, T, tau_rule, rho, seed, n, power_iters,
                           Qb=Qj, Qred=Qred))
    return out


@dataclass
class BasislessPrecond:
    """Basis-less C-RandRAND (Section 4.2, Algorithm BL_RandRAND_PCG): Q is never
    formed; Q^T u = R^{-T} (A_mu Omega)^T u and Q d = (A_mu Omega) R^{-1} d, so
    P = I + Y Kr Y^T with Y = A_mu Omega and Kr = R^{-1} K R^{-T}."""
    mu: float
    Y: np.ndarray
    R: np.ndarray
    G: np.ndarray
    T: np.ndarray
    K: np.ndarray
    Kr: np.ndarray
    tau: float
    normE: float
    lam: float

    def apply(self, r: np.ndarray) -> np.ndarray:
        return r + self.Y @ (self.Kr @ (self.Y.T @ r))

    def dense(self) -> np.ndarray:
        return np.eye(self.Y.shape[0]) + self.Y @ self.Kr @ self.Y.T

    @property
    def Q(self) -> np.ndarray:
        return self.Y @ tri_inv_upper(self.R)


def build_basisless(op, mu: float, l: int, sketch: str = "colsample", seed: int = 0,
                    tau_rule: int = OPT, rho: float = 1.0, power_iters: int = 4,
                    reorth: bool = False) -> BasislessPrecond:
    """Algorithm BL_RandRAND_PCG steps 1-3 with the fast Q-less preconditioned Cholesky
    QR (Algorithm prec_chol_qr): S = Theta Y, R_sk = qr(S), the preconditioned Gram
    R_sk^{-T} Y^T Y R_sk^{-1}, R = R_chol R_sk; Q^T Q = R^{-T} Y^T Y R^{-1} gives
    T = 2I - Q^T Q; Omega^T A_mu Omega = Omega^T Y gives G; tau from the same power
    iterations as the explicit build, with Q applied through Y and R."""
    n = op.n
    Omega = _rng.omega(sketch, seed, n, l)
    Y = op.matmat(Omega) + mu * Omega
    S = np.asarray(_rng.theta(seed, n, l) @ Y)
    R_sk = householder_r(S)
    Rski = tri_inv_upper(R_sk)
    GY = Y.T @ Y
    R_c, _ = chol_upper_ladder(Rski.T @ GY @ Rski)
    R = R_c @ R_sk
    Ri = tri_inv_upper(R)
    T = 2.0 * np.eye(l) - Ri.T @ GY @ Ri
    C = Omega.T @ Y
    R_om, _ = chol_upper_ladder(0.5 * (C + C.T))
    H = R_om @ Ri
    G = H.T @ H
    Q = Y @ Ri        # only inside the tau estimates, as the operator Y R^{-1}
    tau, normE, lam = _tau(tau_rule, mu, rho, op.shifted(mu), Q, T, G, seed, n, power_iters)
    K = apply_core(tau, T, G, reorth)
    return BasislessPrecond(mu, Y, R, G, T, K, Ri @ K @ Ri.T, tau, normE, lam)


def build_shifted_cholesky(op, mus: List[float], l: int, Omega: np.ndarray, seed: int = 0,
                           orth: int = SKETCHED_CHOLQR, tau_rule: int = OPT, rho: float = 1.0,
                           power_iters: int = 4, alpha: Optional[float] = None) -> List[Precond]:
    """Several shifts from one orthogonalisation at a fixed shift alpha (Section 5.1,
    shifted Cholesky preconditioning).

    A_alpha Omega = Q_alpha R_alpha (Algorithm prec_chol_qr).  With Om_a = Omega R_alpha^{-1},
    every mu gets R = R_chol R_alpha where R_chol = chol of the preconditioned Gram
        Om_a^T A_alpha^T A_alpha Om_a + 2 (mu - alpha) Om_a^T A_alpha Om_a + (mu - alpha)^2 Om_a^T Om_a
    (A_mu = A_alpha + (mu - alpha) I; the last coefficient is (mu - alpha)^2), whose three
    parts are precomputed once, and the basis Q_mu = A_mu Omega R^{-1}
    = (Q_alpha + (mu - alpha) Om_a) R_chol^{-1}.  The apply basis is Qb = [Q_alpha, Om_a]
    (n x 2l) with the per-shift map M_mu = [I; (mu - alpha) I] R_chol^{-1} (2l x l).
    alpha defaults to the largest shift, so every mu <= alpha as the technique asks.
    """
    n = op.n
    a = max(mus) if alpha is None else float(alpha)
    AO = op.matmat(Omega)
    Ya = AO + a * Omega
    if orth == SKETCHED_CHOLQR:
        Qa, Ra = sketched_cholqr(Ya, _rng.theta(seed, n, l))
    else:
        Qa, Ra = cholqr(Ya)
    Rai = tri_inv_upper(Ra)
    Oma = Omega @ Rai
    W2 = Qa.T @ Qa                       # Om_a^T A_alpha^2 Om_a
    W1 = Rai.T @ (Omega.T @ Ya) @ Rai    # Om_a^T A_alpha Om_a
    W0 = Oma.T @ Oma                     # Om_a^T Om_a
    Qb = np.concatenate([Qa, Oma], axis=1)
    QbtQb = Qb.T @ Qb
    OAO = Omega.T @ AO
    OO = Omega.T @ Omega
    out = []
    for mu in mus:
        s = mu - a
        Rc, _ = chol_upper_ladder(W2 + 2.0 * s * W1 + s * s * W0)
        Rci = tri_inv_upper(Rc)
        M = np.concatenate([Rci, s * Rci], axis=0)
        R = Rc @ Ra
        Q = Qb @ M
        T = 2.0 * np.eye(l) - M.T @ QbtQb @ M
        out.append(_finish(mu, op.shifted(mu), Q, R, OAO + mu * OO, T, tau_rule, rho, seed, n,
                           power_iters, Qb=Qb, Qred=M))
    return out


def ad_threshold(n: int, l_max: int, q: int, mu: float, f: float) -> float:
    """Right-hand side of eq. ad_criterion: f (n / l_max)^(1/(2q+2)) |mu|."""
    return f * (n / l_max) ** (1.0 / (2 * q + 2)) * abs(mu)


def build_adaptive(op, mu: float, l0: int, l_max: int, f: float = 100.0, sketch: str = "gaussian",
                   seed: int = 0, q: int = 0, growth: int = 2, stagnation: float = 0.9, **kw):
    """Adaptive sketch size (Section 5.3, eq. ad_criterion): build with l, and while
    ||E|| = ||(I-Pi) A_mu (I-Pi)|| (the footnote's refinement of ||(I-Pi) A_mu||, the
    build's power-iteration estimate) is above f (n/l_max)^(1/(2q+2)) |mu|, l < l_max and
    the last growth cut ||E|| below `stagnation` times its previous value, grow
    l <- min(growth l, l_max) and build again.  Returns (preconditioner, l, trail of
    (l, ||E||))."""
    thr = ad_threshold(op.n, l_max, q, mu, f)
    l = l0
    trail = []
    prev = None
    while True:
        P = build(op, [mu], l, sketch, seed, q=q, **kw)[0]
        trail.append((l, P.normE))
        if P.normE <= thr or l >= l_max or (prev is not None and P.normE > stagnation * prev):
            return P, l, trail
        prev = P.normE
        l = min(growth * l, l_max)
