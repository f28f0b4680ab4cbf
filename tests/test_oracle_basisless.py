"""Pins for the oracle's basis-less C-RandRAND, its column-sampling test matrix and
the re-orthogonalised core (CPU only).

* Column sampling: every column of Omega is +-e_i, the indices are distinct and
  uniform over [0, n) (chi-square over many streams), the signs are fair.
* eq. c_randrand_reorth: for ANY upper-triangular R and Q = A_mu Omega R^{-1} (not
  orthonormal), (I-Pi)(I-Pi) + tau (I - (I-Pi)(I-Pi)) A_mu^{-1} Pi formed densely from
  its definition (Pi = Q Q^T, A_mu^{-1} Pi = Omega R^{-1} Q^T) equals I + Q (tau T G - T) Q^T.
* The basis-less preconditioner (Q applied through A_mu Omega and R) equals the
  explicit one built on the same Omega; with the re-orthogonalised core as well.
* Basis-less PCG reaches the direct solution.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import workloads
from oracle import randrand as rr
from oracle import rng
from oracle import solvers
from oracle.operators import Operator


def test_colsample_structure():
    n, l = 500, 60
    Om = rng.colsample_omega(7, n, l)
    assert np.all(np.sum(Om != 0, axis=0) == 1)
    assert set(np.unique(Om)) <= {-1.0, 0.0, 1.0}
    sgn, idx = rng.colsample_descriptor(7, n, l)
    assert len(set(idx.tolist())) == l and idx.min() >= 0 and idx.max() < n
    assert np.array_equal(Om[idx, np.arange(l)], sgn)
    # uniform indices and fair signs over many streams
    counts = np.zeros(50)
    signs = []
    for s in range(400):
        sg, ix = rng.colsample_descriptor(1000 + s, 50, 10)
        np.add.at(counts, ix, 1)
        signs.append(sg)
    expect = 400 * 10 / 50
    chi2 = np.sum((counts - expect) ** 2 / expect)
    assert chi2 < 90          # 49 dof: p ~ 3e-4 at 90
    assert abs(np.mean(np.concatenate(signs))) < 0.05


def test_reorth_core_equals_definition_for_any_r():
    n, l, mu = 120, 10, 1e-2
    A = workloads.synthetic_spectrum_matrix(n, np.logspace(1, -4, n), 3)
    Amu = A + mu * np.eye(n)
    Om = rng.gaussian_matrix(4, n, l)
    Y = Amu @ Om
    _, R = np.linalg.qr(Y)
    R = R + 1e-3 * np.triu(np.random.default_rng(0).standard_normal((l, l)))   # not the QR factor
    Ri = np.linalg.inv(R)
    Q = Y @ Ri
    I = np.eye(n)
    Pi = Q @ Q.T
    AiPi = Om @ Ri @ Q.T
    tau = 0.37
    P_def = (I - Pi) @ (I - Pi) + tau * (I - (I - Pi) @ (I - Pi)) @ AiPi
    T = 2 * np.eye(l) - Q.T @ Q
    H = sla.cholesky(0.5 * (Om.T @ Y + Y.T @ Om), lower=False) @ Ri
    G = H.T @ H
    P_core = I + Q @ rr.apply_core(tau, T, G, reorth=True) @ Q.T
    assert np.linalg.norm(P_def - P_core) <= 1e-10 * np.linalg.norm(P_def)


@pytest.mark.parametrize("reorth", [False, True])
@pytest.mark.parametrize("sketch", ["colsample", "gaussian"])
def test_basisless_equals_explicit(sketch, reorth):
    p = workloads.cfg_small_dense(n=400, d=8, l=30)
    op = Operator.from_problem(p)
    mu = p.mus[0]
    bl = rr.build_basisless(op, mu, p.l, sketch, 5, reorth=reorth, power_iters=60)
    ex = rr.build(op, [mu], p.l, sketch, 5, reorth=reorth, power_iters=60)[0]
    assert np.linalg.norm(bl.Q - ex.Q) <= 1e-10 * np.linalg.norm(ex.Q)
    assert np.allclose(bl.R, ex.R, rtol=1e-10, atol=1e-12 * np.abs(ex.R).max())
    assert abs(bl.tau - ex.tau) <= 1e-9 * ex.tau
    r = np.random.default_rng(1).standard_normal(p.n)
    assert np.linalg.norm(bl.apply(r) - ex.apply(r)) <= 1e-9 * np.linalg.norm(ex.apply(r))


@pytest.mark.parametrize("reorth", [False, True])
def test_basisless_pcg_reaches_direct_solution(reorth):
    p = workloads.cfg_small_dense(n=500, d=8, l=40)
    op = Operator.from_problem(p)
    mu = p.mus[0]
    bl = rr.build_basisless(op, mu, p.l, "colsample", 2, reorth=reorth)
    res = solvers.pcg(op.shifted(mu), bl.apply, p.b, 1e-10)
    assert res.status == solvers.OK and res.relres <= 1e-10
    xs = solvers.direct(op.dense, mu, p.b)
    cond = np.linalg.cond(op.dense + mu * np.eye(p.n))
    assert np.linalg.norm(res.x - xs) <= 10 * 1e-10 * cond * np.linalg.norm(xs)
