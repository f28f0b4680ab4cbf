"""Pins for the oracle's block MINRES and block CG (CPU only).

* Block MINRES: its iterate minimises every column's residual in the norm of P
  over the block Krylov space of P A_mu (brute force: explicit basis and least
  squares), and that norm never increases.
* Block CG: its iterate is the Galerkin solution over the same space (brute
  force: K (K^T A_mu K)^{-1} K^T R0), so every column's A_mu-norm error never
  increases.
* One column: block MINRES and block CG are preconditioned MINRES and PCG (the
  residual histories of the scalar oracles, themselves pinned elsewhere).
* Several columns: every column does at least as well as its own scalar solve
  after the same number of steps (the block space contains the scalar one).
* Finite termination with few distinct eigenvalues; the driver reaches the direct
  solution for every column; dependent right-hand sides are a breakdown.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import workloads
from oracle import block as B
from oracle import randrand as rr
from oracle import solvers
from oracle import variants as V
from oracle.operators import Operator


def _problem(n=220, l=16, mu=1e-3, seed=3, s=4):
    i = np.arange(n)
    eigs = np.where(i < 14, 10.0 * 0.6 ** i, 1e-3 * (1.0 + (n - i) / n))
    A = workloads.synthetic_spectrum_matrix(n, eigs, seed)
    Amu = A + mu * np.eye(n)
    P = rr.build(Operator(dense=A), [mu], l, "gaussian", seed)[0]
    Rhs = np.random.default_rng(seed + 7).standard_normal((n, s))
    return Amu, P, Rhs


def _krylov_basis(Amu, Pm, R0, k):
    blocks = [Pm @ R0]
    for _ in range(k - 1):
        blocks.append(Pm @ (Amu @ blocks[-1]))
    Kb, _ = np.linalg.qr(np.hstack(blocks))
    return Kb


@pytest.mark.parametrize("k", [1, 2, 4, 7])
def test_block_minres_minimises_p_norm_over_block_krylov_space(k):
    Amu, P, R0 = _problem()
    Pm = P.dense()
    c = B.block_minres_cycle(lambda U: Amu @ U, P.apply, R0, np.zeros(R0.shape[1]), k)
    assert c.its == k
    Kb = _krylov_basis(Amu, Pm, R0, k)
    L = np.linalg.cholesky(Pm)
    for j in range(R0.shape[1]):
        coef = np.linalg.lstsq(L.T @ Amu @ Kb, L.T @ R0[:, j], rcond=None)[0]
        y = Kb @ coef
        assert np.linalg.norm(c.Y[:, j] - y) <= 1e-8 * np.linalg.norm(y)


def test_block_minres_p_norm_monotone():
    Amu, P, R0 = _problem(s=3)
    Pm = P.dense()
    prev = None
    for k in range(1, 9):
        c = B.block_minres_cycle(lambda U: Amu @ U, P.apply, R0, np.zeros(3), k)
        R = R0 - Amu @ c.Y
        pn = np.sqrt(np.einsum("ij,ij->j", R, Pm @ R))
        if prev is not None:
            assert np.all(pn <= prev * (1 + 1e-10))
        prev = pn


@pytest.mark.parametrize("k", [1, 3, 6])
def test_block_cg_is_the_galerkin_solution(k):
    Amu, P, R0 = _problem()
    Pm = P.dense()
    c = B.block_cg_cycle(lambda U: Amu @ U, P.apply, R0, np.zeros(R0.shape[1]), k)
    assert c.its == k
    Kb = _krylov_basis(Amu, Pm, R0, k)
    Y = Kb @ np.linalg.solve(Kb.T @ Amu @ Kb, Kb.T @ R0)
    assert np.linalg.norm(c.Y - Y) <= 1e-8 * np.linalg.norm(Y)
    # residual carried by the recurrence is the true one
    assert np.allclose(c.rn, np.linalg.norm(R0 - Amu @ c.Y, axis=0), rtol=1e-9)


def test_one_column_reduces_to_the_scalar_solvers():
    Amu, P, R0 = _problem(s=1)
    r0 = R0[:, 0]
    k = 12
    bm = B.block_minres_cycle(lambda U: Amu @ U, P.apply, R0, np.zeros(1), k)
    sm = V.minres_cycle(lambda u: Amu @ u, r0, 0.0, k, prec=P.apply)
    assert np.allclose([h[0] for h in bm.history], sm.history, rtol=1e-7)
    bc = B.block_cg_cycle(lambda U: Amu @ U, P.apply, R0, np.zeros(1), k)
    sc = V.cg_cycle(lambda u: Amu @ u, r0, 0.0, k, prec=P.apply)
    assert np.allclose([h[0] for h in bc.history], sc.history, rtol=1e-7)


def test_every_column_at_least_as_good_as_its_scalar_solve():
    Amu, P, R0 = _problem(s=5)
    Pm = P.dense()
    xs = np.linalg.solve(Amu, R0)
    for k in (2, 5, 9):
        bm = B.block_minres_cycle(lambda U: Amu @ U, P.apply, R0, np.zeros(5), k)
        bc = B.block_cg_cycle(lambda U: Amu @ U, P.apply, R0, np.zeros(5), k)
        for j in range(5):
            sm = V.minres_cycle(lambda u: Amu @ u, R0[:, j], 0.0, k, prec=P.apply)
            rb = R0[:, j] - Amu @ bm.Y[:, j]
            rs = R0[:, j] - Amu @ sm.y
            assert rb @ Pm @ rb <= (rs @ Pm @ rs) * (1 + 1e-8)
            sc = V.cg_cycle(lambda u: Amu @ u, R0[:, j], 0.0, k, prec=P.apply)
            eb = xs[:, j] - bc.Y[:, j]
            es = xs[:, j] - sc.y
            assert eb @ Amu @ eb <= (es @ Amu @ es) * (1 + 1e-8)


@pytest.mark.parametrize("method", ["minres", "cg"])
def test_finite_termination(method):
    n, k = 120, 5
    vals = np.repeat(np.linspace(1.0, 5.0, k), n // k + 1)[:n]
    A = workloads.synthetic_spectrum_matrix(n, vals, 2)
    R0 = np.random.default_rng(0).standard_normal((n, 3))
    c = B.CYCLES[method](lambda U: A @ U, lambda U: U.copy(), R0, 1e-10 * np.linalg.norm(R0, axis=0), 20)
    assert c.status == solvers.OK and c.its <= k


@pytest.mark.parametrize("method", ["minres", "cg"])
def test_driver_reaches_the_direct_solution(method):
    Amu, P, Rhs = _problem(n=300, l=24, mu=1e-4, s=6)
    Rhs[:, 2] = 0.0
    res = B.solve_block(lambda U: Amu @ U, P.apply, Rhs, 1e-10, method=method, group=4)
    assert res.status == solvers.OK
    assert np.all(res.relres <= 1e-10) and res.relres[2] == 0.0
    xs = np.linalg.solve(Amu, Rhs)
    cond = np.linalg.cond(Amu)
    assert np.linalg.norm(res.X - xs) <= 10 * 1e-10 * cond * np.linalg.norm(xs)
    assert np.all(res.X[:, 2] == 0.0)
    # groups: the first four columns share a count, the last two theirs
    assert len(set(res.iters[:4])) == 1 and len(set(res.iters[4:])) == 1
    # a group solved alone gives the same result
    alone = B.solve_block(lambda U: Amu @ U, P.apply, Rhs[:, 4:], 1e-10, method=method, group=4)
    assert np.array_equal(alone.X, res.X[:, 4:])
    # the history is the max over columns, ends at the final value and starts at 1
    assert res.history[0] == 1.0 and abs(res.history[-1] - res.relres[:4].max()) < 1e-15
    # block preconditioned MINRES needs fewer block steps than any of its columns alone
    single = [V.c_randrand_minres(lambda u: Amu @ u, P.apply, Rhs[:, j], 1e-10).iters for j in (0, 1, 3)]
    assert res.iters[0] <= min(single)


def test_dependent_columns_break_down():
    Amu, P, Rhs = _problem(s=3)
    Rhs[:, 2] = 2.0 * Rhs[:, 0]
    for method in ("minres", "cg"):
        res = B.solve_block(lambda U: Amu @ U, P.apply, Rhs, 1e-8, method=method)
        assert res.status == solvers.BREAKDOWN


def test_chol_upper_rank_rule():
    S = np.array([[4.0, 2.0], [2.0, 1.0 + 1e-22]])
    assert B.chol_upper(S) is None
    S = np.array([[4.0, 2.0], [2.0, 1.0 + 1e-6]])
    C = B.chol_upper(S)
    assert np.allclose(C.T @ C, S, rtol=1e-14)
    assert np.allclose(C, sla.cholesky(S, lower=False))
