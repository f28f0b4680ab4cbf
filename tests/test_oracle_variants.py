"""Pins for the oracle's R-RandRAND, split R-RandRAND and MINRES solvers (CPU only).

* MINRES: the residual after k steps is never above CG's (both minimise over the
  same Krylov space, MINRES in the 2-norm); finite termination in k steps for k
  distinct eigenvalues; preconditioned MINRES minimises ||r||_P over the
  preconditioned Krylov space (brute-force least squares) and its phibar is that
  norm of the true residual.
* R-RandRAND (Section 3.1): B = (I-Pi) A_mu (I-Pi) + tau Pi equals A_mu P for P of
  eq. randrandprecond; Proposition cnd_bound (cond(B) <= rho ||E|| / lambda_min for
  rho^{-1} lambda_min <= tau <= rho ||E||); the diagonal closed form; the recovery
  of eq. APdef3 makes the B-residual the true residual.
* Split R-RandRAND: the effective condition number of E is at most cond(E + tau Pi);
  b - A_mu x = (I-Pi) b - E y for the recovered x.
* Every solver reaches the direct Cholesky solution.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import workloads
from oracle import randrand as rr
from oracle import rng
from oracle import solvers
from oracle import variants as V
from oracle.operators import Operator


def _spd(n, seed, top=12, decay=0.6, tail=1e-3):
    i = np.arange(n)
    eigs = np.where(i < top, 10.0 * decay ** i, tail * (1.0 + (n - i) / n))
    return workloads.synthetic_spectrum_matrix(n, eigs, seed), eigs


def _problem(n=260, l=24, mu=1e-3, seed=3, q_orth=rr.SKETCHED_CHOLQR):
    A, eigs = _spd(n, seed)
    op = Operator(dense=A)
    P = rr.build(op, [mu], l, "gaussian", seed, orth=q_orth, power_iters=200)[0]
    Om = rng.gaussian_matrix(seed, n, l)
    proj = V.Projections(P.Q, P.T, P.R, Om)
    b = np.random.default_rng(seed + 1).standard_normal(n)
    Amu = A + mu * np.eye(n)
    return A, Amu, P, proj, b


def test_minres_residual_not_above_cg():
    A, eigs = _spd(200, 1, top=30, decay=0.8)
    b = np.random.default_rng(2).standard_normal(200)
    op = lambda u: A @ u
    k = 40
    cg = V.cg_cycle(op, b, 0.0, k)
    mr = V.minres_cycle(op, b, 0.0, k)
    h_cg, h_mr = np.array(cg.history), np.array(mr.history)
    assert len(h_cg) == len(h_mr) == k
    assert np.all(h_mr <= h_cg * (1 + 1e-8) + 1e-14)
    # MINRES residuals never increase
    assert np.all(np.diff(h_mr) <= 1e-12 * h_mr[:-1])


def test_minres_finite_termination():
    n, k = 150, 6
    vals = np.repeat(np.linspace(1.0, 9.0, k), n // k + 1)[:n]
    A = workloads.synthetic_spectrum_matrix(n, vals, 4)
    b = np.random.default_rng(1).standard_normal(n)
    c = V.minres_cycle(lambda u: A @ u, b, 1e-10 * np.linalg.norm(b), 50)
    assert c.status == solvers.OK and c.its <= k


def test_pminres_minimises_preconditioner_norm_over_krylov_space():
    # y_k = argmin over span{Pb, (PA)Pb, ...} of ||b - A y||_P  (brute force)
    A, Amu, P, proj, b = _problem(n=120, l=10)
    Pm = P.dense()
    for k in (1, 3, 6):
        c = V.minres_cycle(lambda u: Amu @ u, b, 0.0, k, prec=P.apply)
        K = [Pm @ b]
        for _ in range(k - 1):
            K.append(Pm @ (Amu @ K[-1]))
        Kb, _ = np.linalg.qr(np.array(K).T)
        L = np.linalg.cholesky(Pm)          # ||v||_P = ||L^T v||
        coef, *_ = np.linalg.lstsq(L.T @ Amu @ Kb, L.T @ b, rcond=None)
        y_ref = Kb @ coef
        assert np.linalg.norm(c.y - y_ref) <= 1e-8 * np.linalg.norm(y_ref)


def test_pminres_phibar_is_the_preconditioner_norm_of_the_residual():
    A, Amu, P, proj, b = _problem(n=150, l=12)
    Pm = P.dense()
    c = V.minres_cycle(lambda u: Amu @ u, b, 0.0, 12, prec=P.apply, record_pnorm=True)
    # rerun step by step to get y_k, compare phibar_k with sqrt(r_k^T P r_k)
    for k in (1, 5, 12):
        ck = V.minres_cycle(lambda u: Amu @ u, b, 0.0, k, prec=P.apply)
        r = b - Amu @ ck.y
        assert abs(c.history[k - 1] - np.sqrt(r @ Pm @ r)) <= 1e-9 * np.sqrt(b @ Pm @ b)


def test_r_randrand_operator_is_a_mu_times_p():
    # eq. randrandprecond: P = A_mu^{-1}((I-Pi) A_mu (I-Pi) + tau Pi), B = A_mu P
    A, Amu, P, proj, b = _problem()
    n = A.shape[0]
    tau = P.normE
    Pi = P.Q @ P.T @ P.Q.T
    I = np.eye(n)
    Bdef = (I - Pi) @ Amu @ (I - Pi) + tau * Pi
    Pr = np.linalg.solve(Amu, Bdef)
    u = np.random.default_rng(0).standard_normal(n)
    Bu = proj.comp(Amu @ proj.comp(u)) + tau * proj.pi(u)
    assert np.linalg.norm(Bu - Amu @ (Pr @ u)) <= 1e-10 * np.linalg.norm(Bu)


def test_r_randrand_condition_bound():
    # Proposition cnd_bound with exact ||E|| and rho = 1: cond(A_mu P) <= ||E|| / lambda_min
    A, Amu, P, proj, b = _problem(n=220, l=20)
    n = A.shape[0]
    Q = P.Q
    I = np.eye(n)
    E = (I - Q @ Q.T) @ Amu @ (I - Q @ Q.T)
    nE = np.linalg.norm(E, 2)
    lmin = np.linalg.eigvalsh(Amu).min()
    for rho, tau in ((1.0, nE), (2.0, 0.5 * nE), (3.0, lmin / 2.0)):
        B = E + tau * Q @ Q.T
        ev = np.linalg.eigvalsh(0.5 * (B + B.T))
        assert ev.max() / ev.min() <= rho * nE / lmin * (1 + 1e-8)
    # the estimate the build uses for tau (power iteration) approaches ||E|| from below
    assert P.normE <= nE * (1 + 1e-10) and P.normE >= 0.9 * nE


def test_r_randrand_diagonal_closed_form():
    # A = diag(lambda), Omega = [e_1..e_l]: B = diag(tau (l times), lambda_{l+1}+mu, ...)
    n, l, mu = 50, 6, 0.05
    lam = np.linspace(30.0, 0.5, n)
    op = Operator(dense=np.diag(lam))
    Om = np.eye(n)[:, :l]
    P = rr.build(op, [mu], l, seed=2, Omega=Om, orth=rr.CHOLQR, power_iters=400)[0]
    proj = V.Projections(P.Q, P.T, P.R, Om)
    Amu = np.diag(lam + mu)
    tau = P.normE
    B = np.array([proj.comp(Amu @ proj.comp(e)) + tau * proj.pi(e) for e in np.eye(n)]).T
    expect = np.sort(np.concatenate([np.full(l, tau), lam[l:] + mu]))
    assert np.allclose(np.sort(np.linalg.eigvalsh(0.5 * (B + B.T))), expect, rtol=1e-12)
    assert abs(tau - (lam[l] + mu)) <= 1e-6 * tau


def test_recovery_identities():
    A, Amu, P, proj, b = _problem()
    tau = P.normE
    y = np.random.default_rng(5).standard_normal(b.shape[0])
    # R-RandRAND (eq. APdef3): b - A_mu x = b - B y
    u = proj.comp(y)
    x = proj.amu_inv_pi(tau * y - Amu @ u) + u
    By = proj.comp(Amu @ u) + tau * proj.pi(y)
    assert np.linalg.norm((b - Amu @ x) - (b - By)) <= 1e-9 * np.linalg.norm(b - By)
    # split: b - A_mu x = (I-Pi) b - E y for y in range(I-Pi)
    y = proj.comp(proj.comp(y))
    x = proj.amu_inv_pi(b - Amu @ y) + y
    rhs = proj.comp(b) - proj.comp(Amu @ y)
    assert np.linalg.norm((b - Amu @ x) - rhs) <= 1e-9 * np.linalg.norm(rhs)


def test_split_effective_condition_number():
    A, Amu, P, proj, b = _problem(n=200, l=18)
    n, l = A.shape[0], 18
    Q = P.Q
    I = np.eye(n)
    E = (I - Q @ Q.T) @ Amu @ (I - Q @ Q.T)
    ev = np.sort(np.linalg.eigvalsh(0.5 * (E + E.T)))
    cond_eff = ev[-1] / ev[l]            # largest over the smallest nonzero one
    for tau in (ev[-1], 1.0, ev[l] * 0.1):
        Bt = E + tau * Q @ Q.T
        eb = np.linalg.eigvalsh(0.5 * (Bt + Bt.T))
        assert cond_eff <= eb.max() / eb.min() * (1 + 1e-9)


@pytest.mark.parametrize("krylov", ["cg", "minres"])
@pytest.mark.parametrize("method", ["r", "split"])
def test_r_variants_reach_the_direct_solution(method, krylov):
    A, Amu, P, proj, b = _problem(n=300, l=30, mu=1e-4)
    amu = lambda u: Amu @ u
    if method == "r":
        res = V.r_randrand(amu, proj, P.normE, b, 1e-10, krylov=krylov)
    else:
        res = V.split_r_randrand(amu, proj, b, 1e-10, krylov=krylov)
    assert res.status == solvers.OK and res.relres <= 1e-10
    xs = sla.solve(Amu, b, assume_a="pos")
    cond = np.linalg.cond(Amu)
    assert np.linalg.norm(res.x - xs) <= 10 * 1e-10 * cond * np.linalg.norm(xs)
    plain = solvers.cg(amu, b, 1e-10)
    assert res.iters < plain.iters
    assert len(res.history) == res.iters + 1 and res.history[0] == 1.0


def test_c_randrand_minres_and_plain_minres():
    A, Amu, P, proj, b = _problem(n=300, l=30, mu=1e-4)
    amu = lambda u: Amu @ u
    res = V.c_randrand_minres(amu, P.apply, b, 1e-10)
    assert res.status == solvers.OK and res.relres <= 1e-10
    xs = sla.solve(Amu, b, assume_a="pos")
    assert np.linalg.norm(res.x - xs) <= 1e-10 * np.linalg.cond(Amu) * 10 * np.linalg.norm(xs)
    pcg = solvers.pcg(amu, P.apply, b, 1e-10)
    assert abs(res.iters - pcg.iters) <= max(3, 0.25 * pcg.iters)
    plain = V.minres(amu, b, 1e-10)
    assert plain.status == solvers.OK and plain.iters > res.iters


def test_minres_breakdown_on_indefinite_preconditioner():
    n = 20
    A = np.eye(n)
    b = np.ones(n)
    res = V.c_randrand_minres(lambda u: A @ u, lambda r: -r, b, 1e-8)
    assert res.status == solvers.BREAKDOWN
