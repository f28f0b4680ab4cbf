"""Pins for the oracle's preconditioner construction (CPU only).

Each test checks the oracle against something the paper or the mathematics
fixes independently of the oracle's own formulas:

* orthogonalisation: Q^T Q = I, Q R = Y, R equal to the sign-fixed Householder
  R of LAPACK (uniqueness of the QR with positive diagonal); the sketched
  variant stays orthogonal where plain Cholesky QR cannot (Section 4.2).
* identity eq. invAPi: G = Q^T A_mu^{-1} Q (explicit inverse at small n).
* Nystrom link (Section 1.3): Pi A_mu^{-1} Pi = pinv(Nystrom approximation).
* closed form: A = diag(lambda), Omega = [e_1..e_l] gives Pi = first l
  coordinates, ||E|| = lambda_{l+1} + mu, lam = 1 and the preconditioned
  spectrum {tau (l times), lambda_{l+1}+mu, ..., lambda_n+mu}.
* Proposition cnd_bound2: eigenvalue bracket of P^{1/2} A_mu P^{1/2}.
* Lemma apriori_gen00 (expectation form) for Gaussian Omega.
* scale invariance Omega -> c Omega; joint basis (Section 5.1) equals the
  per-shift basis.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import workloads
from oracle import randrand as rr
from oracle import rng
from oracle.operators import Operator


def _decaying_spd(n, seed, top=20, mu=0.0):
    i = np.arange(n)
    tail = 10.0 * 0.7 ** top * np.maximum(i - top + 1.0, 1.0) ** -0.5
    eigs = np.where(i < top, 10.0 * 0.7 ** i, tail)
    return workloads.synthetic_spectrum_matrix(n, eigs, seed), eigs


def _ill_conditioned(n, l, cond, seed):
    r = np.random.default_rng(seed)
    U, _ = np.linalg.qr(r.standard_normal((n, l)))
    V, _ = np.linalg.qr(r.standard_normal((l, l)))
    s = np.logspace(0, -np.log10(cond), l)
    return (U * s) @ V.T


@pytest.mark.parametrize("method", ["cholqr", "sketched"])
def test_orthogonalisation_unique_qr(method):
    n, l = 400, 30
    Y = _ill_conditioned(n, l, 1e3, 0)
    if method == "cholqr":
        Q, R = rr.cholqr(Y)
    else:
        Q, R = rr.sketched_cholqr(Y, rng.theta(5, n, l))
    assert np.linalg.norm(Q.T @ Q - np.eye(l)) < 1e-10
    assert np.linalg.norm(Q @ R - Y) < 1e-13 * np.linalg.norm(Y)
    assert np.allclose(R, np.triu(R)) and np.all(np.diag(R) > 0)
    Rref = np.linalg.qr(Y, mode="r")
    Rref = np.sign(np.diag(Rref))[:, None] * Rref
    assert np.linalg.norm(R - Rref) < 1e-9 * np.linalg.norm(Rref)


def test_sketched_cholqr_stable_where_cholqr_is_not():
    # orthogonality loss ~ u cond (sketched) versus u cond^2 (plain), Section 4.2
    n, l = 2000, 40
    Y = _ill_conditioned(n, l, 1e10, 1)
    Q, R = rr.sketched_cholqr(Y, rng.theta(9, n, l))
    assert np.linalg.norm(Q.T @ Q - np.eye(l), 2) < 1e-4
    assert np.linalg.norm(Q @ R - Y) < 1e-12 * np.linalg.norm(Y)
    try:
        Qc, _ = rr.cholqr(Y)
        loss = np.linalg.norm(Qc.T @ Qc - np.eye(l), 2)
    except rr.NotSPD:
        loss = np.inf
    assert loss > 1e-3


def test_householder_r_positive():
    S = np.random.default_rng(3).standard_normal((80, 40))
    R = rr.householder_r(S)
    assert np.all(np.diag(R) > 0) and np.allclose(R, np.triu(R))
    assert np.allclose(R.T @ R, S.T @ S, rtol=1e-12, atol=1e-11)


def _small_precond(n=240, l=24, mu=1e-2, seed=4, rule=rr.OPT, orth=rr.SKETCHED_CHOLQR):
    A, eigs = _decaying_spd(n, seed)
    op = Operator(dense=A)
    P = rr.build(op, [mu], l, "gaussian", seed, orth=orth, tau_rule=rule, power_iters=60)[0]
    return A, op, P


def test_core_equals_projected_inverse():
    A, op, P = _small_precond()
    Amu = A + P.mu * np.eye(A.shape[0])
    Ginv = P.Q.T @ np.linalg.inv(Amu) @ P.Q
    assert np.linalg.norm(P.G - Ginv) < 1e-9 * np.linalg.norm(Ginv)
    assert np.linalg.norm(P.T - np.eye(P.l)) < 1e-12


def test_nystrom_link():
    A, op, P = _small_precond(n=200, l=15)
    n = A.shape[0]
    Amu = A + P.mu * np.eye(n)
    Om = rng.gaussian_matrix(4, n, 15)
    Y = Amu @ Om
    nys = Y @ np.linalg.solve(Om.T @ Y, Y.T)
    lhs = P.Q @ P.G @ P.Q.T
    assert np.linalg.norm(lhs - np.linalg.pinv(nys, rcond=1e-10)) < 1e-7 * np.linalg.norm(lhs)


@pytest.mark.parametrize("rule", [rr.OPT, rr.RHO, rr.NYS])
def test_preconditioner_spd(rule):
    A, op, P = _small_precond(rule=rule)
    w = np.linalg.eigvalsh(P.dense())
    assert w.min() > 0
    assert P.tau > 0


def test_closed_form_diagonal():
    n, l, mu = 60, 8, 0.05
    lam = np.linspace(40.0, 0.5, n) ** 1.0
    A = np.diag(lam)
    op = Operator(dense=A)
    Om = np.eye(n)[:, :l]
    P = rr.build(op, [mu], l, seed=2, Omega=Om, orth=rr.CHOLQR, tau_rule=rr.OPT,
                 power_iters=400)[0]
    assert np.allclose(np.abs(P.Q), Om, atol=1e-14)
    normE = lam[l] + mu
    assert abs(P.normE - normE) < 1e-6 * normE
    assert abs(P.lam - 1.0) < 1e-12
    assert abs(P.tau - np.sqrt(mu * P.normE)) < 1e-14
    L = np.linalg.cholesky(P.dense())
    spec = np.sort(np.linalg.eigvalsh(L.T @ (A + mu * np.eye(n)) @ L))
    expect = np.sort(np.concatenate([np.full(l, P.tau), lam[l:] + mu]))
    assert np.allclose(spec, expect, rtol=1e-10)


@pytest.mark.parametrize("rule,rho", [(rr.NYS, 1.0), (rr.RHO, 0.7), (rr.RHO, 2.5)])
def test_closed_form_diagonal_tau_rules(rule, rho):
    # A = diag(lambda) (decreasing), Omega = [e_1 .. e_l]: Q = Omega, R = diag(lambda_i + mu)
    # and G = diag(1 / (lambda_i + mu)), so
    #   eq. nys_tau:         tau = 1 / lambda_max(G) = lambda_l + mu,
    #   eq. c_randrand_tau:  tau = rho ||E|| / lam = rho (lambda_{l+1} + mu)   (lam = 1).
    n, l, mu = 60, 8, 0.05
    lam = np.linspace(40.0, 0.5, n)
    op = Operator(dense=np.diag(lam))
    Om = np.eye(n)[:, :l]
    P = rr.build(op, [mu], l, seed=2, Omega=Om, orth=rr.CHOLQR, tau_rule=rule, rho=rho,
                 power_iters=400)[0]
    assert np.allclose(np.diag(P.G), 1.0 / (lam[:l] + mu), rtol=1e-13)
    if rule == rr.NYS:
        assert abs(P.tau - (lam[l - 1] + mu)) <= 1e-12 * (lam[l - 1] + mu)
    else:
        expect = rho * (lam[l] + mu)
        assert abs(P.tau - expect) <= 1e-6 * expect


def test_cholesky_ladder_alpha_diagonal():
    # W = diag(1, 1, -5e-13): plain Cholesky fails; the ladder adds
    # alpha = 10^e max_i W_ii for e = -14, -13, ...; e = -12 is the first with
    # -5e-13 + alpha > 0, so alpha = 1e-12 and R^T R = W + 1e-12 I.
    W = np.diag([1.0, 1.0, -5e-13])
    R, alpha = rr.chol_upper_ladder(W)
    assert alpha == 1e-12
    assert np.allclose(R.T @ R, W + alpha * np.eye(3), rtol=0, atol=1e-15)


def test_cholesky_ladder_alpha_from_spectrum():
    # A symmetric matrix with a known negative eigenvalue: the first ladder shift
    # that makes it positive definite is determined by lambda_min and max_i W_ii
    # (computed independently here from eigvalsh), and no shift for an spd matrix.
    rg = np.random.default_rng(5)
    U, _ = np.linalg.qr(rg.standard_normal((40, 40)))
    ev = np.logspace(0, -6, 40)
    ev[-1] = -3.7e-9
    W = (U * ev) @ U.T
    W = 0.5 * (W + W.T)
    wn = np.max(np.abs(np.diag(W)))
    lmin = np.min(np.linalg.eigvalsh(W))
    e = next(e for e in range(-14, 0) if lmin + 10.0 ** e * wn > 1e-12 * wn)
    R, alpha = rr.chol_upper_ladder(W)
    assert alpha == 10.0 ** e * wn
    assert np.allclose(R.T @ R, W + alpha * np.eye(40), atol=1e-13)
    R0, a0 = rr.chol_upper_ladder(W + 1e-3 * np.eye(40))
    assert a0 == 0.0


def test_full_rank_sketch_gives_scaled_inverse():
    # l = n: Pi = I and P = tau A_mu^{-1}
    n, mu = 50, 0.1
    A, _ = _decaying_spd(n, 7, top=10)
    op = Operator(dense=A)
    P = rr.build(op, [mu], n, "gaussian", 3, orth=rr.SKETCHED_CHOLQR, tau_rule=rr.NYS)[0]
    Amu = A + mu * np.eye(n)
    assert np.allclose(P.dense(), P.tau * np.linalg.inv(Amu), rtol=1e-6, atol=1e-8 * P.tau)


def test_eigenvalue_bracket_cnd_bound2():
    # Proposition cnd_bound2 with exact ||E||, ||F||, lambda_max(Pi A Pi A^-1 Pi)
    n, l, mu, rho = 200, 20, 1e-2, 0.7
    A, _ = _decaying_spd(n, 11)
    op = Operator(dense=A)
    P = rr.build(op, [mu], l, "gaussian", 8, tau_rule=rr.NYS)[0]
    Amu = A + mu * np.eye(n)
    Pi = P.Q @ P.Q.T
    I = np.eye(n)
    E = (I - Pi) @ Amu @ (I - Pi)
    F = (I - Pi) @ np.linalg.inv(Amu) @ (I - Pi)
    nE, nF = np.linalg.norm(E, 2), np.linalg.norm(F, 2)
    lamhat = np.max(np.real(np.linalg.eigvals(Pi @ Amu @ Pi @ np.linalg.inv(Amu) @ Pi)))
    tau = rho * nE / lamhat
    Pm = I - Pi + tau * P.Q @ P.G @ P.Q.T
    L = np.linalg.cholesky(Pm)
    spec = np.linalg.eigvalsh(L.T @ Amu @ L)
    assert spec.min() >= (nF + 1.0 / tau) ** -1 * (1 - 1e-9)
    assert spec.max() <= (1.0 + rho) * nE * (1 + 1e-9)
    lmin = np.linalg.eigvalsh(Amu).min()
    bound = (1 + rho) * nE / lmin + (1 + 1 / rho) * lamhat
    assert spec.max() / spec.min() <= bound


def test_range_bound_expectation():
    # Lemma apriori_gen00 in expectation: C1 = 2, C2 = sqrt(2) e, l = 2k+2
    n, k, mu = 300, 10, 1e-3
    l = 2 * k + 2
    A, eigs = _decaying_spd(n, 13, top=15)
    Amu = A + mu * np.eye(n)
    sig = np.sort(np.linalg.svd(Amu, compute_uv=False))[::-1]
    sk = sig[k - 1]
    sr = np.sum(sig[k - 1:] ** 2) / sk ** 2
    bound = (2.0 + np.sqrt(2.0) * np.e * np.sqrt(sr / k)) * sk
    errs = []
    for s in range(30):
        Om = rng.gaussian_matrix(100 + s, n, l)
        Q, _ = rr.sketched_cholqr(Amu @ Om, rng.theta(100 + s, n, l))
        errs.append(np.linalg.norm(Amu - Q @ (Q.T @ Amu), 2))
    assert np.mean(errs) <= bound


def test_scale_invariance_of_omega():
    A, _ = _decaying_spd(150, 5)
    op = Operator(dense=A)
    Om = rng.gaussian_matrix(21, 150, 12)
    P1 = rr.build(op, [1e-2], 12, seed=21, Omega=Om, orth=rr.CHOLQR)[0]
    P2 = rr.build(op, [1e-2], 12, seed=21, Omega=3.0 * Om, orth=rr.CHOLQR)[0]
    assert np.allclose(P1.Q, P2.Q, atol=1e-12)
    assert np.allclose(P1.G, P2.G, rtol=1e-10)
    assert abs(P1.tau - P2.tau) < 1e-10 * P1.tau
    assert np.allclose(P2.R, 3.0 * P1.R, rtol=1e-12)


def test_joint_basis_matches_per_shift_basis():
    n, l = 220, 16
    A, _ = _decaying_spd(n, 17)
    op = Operator(dense=A)
    mus = [1e-1, 1e-2, 1e-3]
    joint = rr.build(op, mus, l, "gaussian", 31, power_iters=30)
    for j, mu in enumerate(mus):
        single = rr.build(op, [mu], l, "gaussian", 31, power_iters=30)[0]
        assert np.linalg.norm(joint[j].Q - single.Q) < 1e-8
        assert np.linalg.norm(joint[j].G - single.G) < 1e-7 * np.linalg.norm(single.G)
        assert np.allclose(joint[j].R, single.R, rtol=1e-8, atol=1e-10 * np.abs(single.R).max())
        Pj, Ps = joint[j].dense(), single.dense()
        assert np.linalg.norm(Pj - Ps) / np.linalg.norm(Ps) < 1e-3
