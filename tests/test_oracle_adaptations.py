"""Pins for the oracle's adaptations (Section 5) and the power q = 1 (CPU only).

* q = 1 (eq. testmatrix, Omega = A X): Proposition apriori2 in expectation bounds
  ||(I - Pi) A_mu||; with A diagonal and X = [e_1..e_l], Omega = A X only rescales
  columns, so Q, G, tau equal the q = 0 ones and R picks up the column scales.
* Shifted Cholesky multi-shift (Section 5.1): Q_mu and R equal the direct
  per-shift orthogonalisation of A_mu Omega (unique QR with positive diagonal)
  for every mu <= alpha; the Gram coefficient (mu - alpha)^2 is what makes it hold.
* Adaptive sketch size (eq. ad_criterion): the chosen l is the first of the
  doubling sequence whose exact ||E|| meets the threshold, the threshold follows
  the formula, and the loop stops at l_max or on stagnation.
"""
import numpy as np
import pytest

import workloads
from oracle import randrand as rr
from oracle import rng
from oracle.operators import Operator


def _spd(n, seed, decay=0.85, floor=1e-4):
    i = np.arange(n)
    eigs = np.maximum(10.0 * decay ** i, floor * (1 + (n - i) / n))
    return workloads.synthetic_spectrum_matrix(n, eigs, seed), eigs


def _proj_err(Amu, Q):
    return np.linalg.norm(Amu - Q @ (Q.T @ Amu), 2)


def test_q1_expectation_bound_apriori2():
    n, k, mu = 300, 8, 1e-3
    l = 2 * k + 2
    A, eigs = _spd(n, 21, decay=0.9)
    op = Operator(dense=A)
    Amu = A + mu * np.eye(n)
    lam = np.sort(eigs)[::-1]
    m2 = ((lam + mu) ** 2) * lam ** 2                    # singular values of A_mu^2 A^2
    srk = np.sum(m2[k - 1:]) / m2[k - 1]
    C1, C2 = 2.0, np.sqrt(2.0) * np.e
    bound = mu + np.sqrt(C1 + C2 * np.sqrt(srk / k)) * np.sqrt(lam[k - 1]) * np.sqrt(lam[k - 1] + mu)
    errs0, errs1 = [], []
    for s in range(30):
        for q, errs in ((0, errs0), (1, errs1)):
            Om = rr.test_matrix(op, "gaussian", 50 + s, l, q=q)
            Q, _ = rr.sketched_cholqr(Amu @ Om, rng.theta(50 + s, n, l))
            errs.append(_proj_err(Amu, Q))
    assert np.mean(errs1) <= bound
    # the power iteration captures the range at least as well on average
    assert np.mean(errs1) <= np.mean(errs0)


def test_q1_diagonal_column_scaling():
    n, l, mu = 60, 8, 0.05
    lam = np.linspace(40.0, 0.5, n)
    op = Operator(dense=np.diag(lam))
    X = np.eye(n)[:, :l]
    P0 = rr.build(op, [mu], l, seed=2, Omega=X, orth=rr.CHOLQR, power_iters=300)[0]
    P1 = rr.build(op, [mu], l, seed=2, Omega=X, orth=rr.CHOLQR, power_iters=300, q=1)[0]
    assert np.allclose(P1.Q, P0.Q, atol=1e-13)
    assert np.allclose(P1.G, P0.G, rtol=1e-12)
    assert abs(P1.tau - P0.tau) <= 1e-10 * P0.tau
    assert np.allclose(P1.R, P0.R * lam[None, :l], rtol=1e-12)


@pytest.mark.parametrize("orth", [rr.SKETCHED_CHOLQR, rr.CHOLQR])
def test_shifted_cholesky_equals_direct_per_shift(orth):
    n, l = 240, 16
    A, _ = _spd(n, 7)
    op = Operator(dense=A)
    mus = [1e-1, 1e-2, 1e-3, 0.0]
    Om = rng.gaussian_matrix(13, n, l)
    sc = rr.build(op, mus, l, seed=13, Omega=Om, orth=orth, power_iters=40, multi="shifted_chol")
    for j, mu in enumerate(mus):
        Y = A @ Om + mu * Om
        Q, R = np.linalg.qr(Y)
        sg = np.sign(np.diag(R))
        Q, R = Q * sg, sg[:, None] * R
        assert np.linalg.norm(sc[j].Q - Q) <= 1e-8, mu
        assert np.allclose(sc[j].R, R, rtol=1e-8, atol=1e-10 * np.abs(R).max())
        single = rr.build(op, [mu], l, seed=13, Omega=Om, orth=orth, power_iters=40)[0]
        assert np.linalg.norm(sc[j].G - single.G) <= 1e-7 * np.linalg.norm(single.G)
        Ps, Pc = single.dense(), sc[j].dense()
        assert np.linalg.norm(Pc - Ps) <= 1e-3 * np.linalg.norm(Ps)


def test_shifted_cholesky_needs_the_squared_shift_difference():
    # the coefficient printed in Section 5.1 as (mu^2 + alpha^2) would not give A_mu Omega's R
    n, l, a, mu = 120, 10, 1.0, 0.5
    A, _ = _spd(n, 9)
    Om = rng.gaussian_matrix(3, n, l)
    Ya = A @ Om + a * Om
    Qa, Ra = np.linalg.qr(Ya)
    Rai = np.linalg.inv(Ra)
    Oma = Om @ Rai
    W2, W1, W0 = Qa.T @ Qa, Oma.T @ (A + a * np.eye(n)) @ Oma, Oma.T @ Oma
    G_true = Oma.T @ (A + mu * np.eye(n)) @ (A + mu * np.eye(n)) @ Oma
    good = W2 + 2 * (mu - a) * W1 + (mu - a) ** 2 * W0
    bad = W2 + 2 * (mu - a) * W1 + (mu ** 2 + a ** 2) * W0
    assert np.linalg.norm(good - G_true) <= 1e-10 * np.linalg.norm(G_true)
    assert np.linalg.norm(bad - G_true) > 1e-3 * np.linalg.norm(G_true)


def test_adaptive_sketch_size_matches_exact_criterion():
    n, mu, l0, lmax, f = 400, 1e-3, 8, 128, 30.0
    A, _ = _spd(n, 5, decay=0.93)
    op = Operator(dense=A)
    Amu = A + mu * np.eye(n)
    P, l, trail = rr.build_adaptive(op, mu, l0, lmax, f=f, seed=4, power_iters=200)
    thr = rr.ad_threshold(n, lmax, 0, mu, f)
    assert thr == pytest.approx(f * np.sqrt(n / lmax) * mu)
    # the exact ||E|| (dense) for each l the loop tried, and the first that meets thr
    I = np.eye(n)
    exact = []
    for lt, est in trail:
        Pt = rr.build(op, [mu], lt, "gaussian", 4, power_iters=5)[0]
        E = (I - Pt.Q @ Pt.Q.T) @ Amu @ (I - Pt.Q @ Pt.Q.T)
        exact.append(np.linalg.norm(E, 2))
        assert est <= exact[-1] * (1 + 1e-8) and est >= 0.95 * exact[-1]
    assert [t[0] for t in trail] == [min(l0 * 2 ** i, lmax) for i in range(len(trail))]
    assert exact[-1] <= thr * 1.05 or l == lmax
    assert all(e > thr * 0.95 for e in exact[:-1])
    assert P.l == l


def test_adaptive_sketch_size_limits():
    n, mu = 200, 1e-3
    A, _ = _spd(n, 6)
    op = Operator(dense=A)
    _, l_big, _ = rr.build_adaptive(op, mu, 10, 160, f=1e9, seed=1)
    assert l_big == 10                          # criterion met at once
    _, l_cap, trail = rr.build_adaptive(op, mu, 10, 40, f=1e-9, seed=1, stagnation=1.0)
    assert l_cap == 40 and len(trail) == 3      # 10, 20, 40: stops at l_max
