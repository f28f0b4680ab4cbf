"""Pins for the oracle's solvers (CPU only).

* PCG and CG reach the direct Cholesky solution x* = (A + mu I)^{-1} b
  (the plain definition the iteration converges to, Section 1).
* CG on a matrix with k distinct eigenvalues terminates in k iterations
  (textbook finite-termination property) — a dropped or mis-signed term in
  the recurrences breaks it.
* l = n: PCG converges in one iteration (P = tau A_mu^{-1}).
* Failure paths: indefinite operator -> breakdown; maxit -> no convergence
  with a usable iterate.
"""
import numpy as np
import pytest

import workloads
from oracle import randrand as rr
from oracle import solvers
from oracle.operators import Operator


def _kernel_problem(n=600):
    p = workloads.cfg_small_dense(n=n, d=8, l=40)
    op = Operator.from_problem(p)
    return p, op


@pytest.mark.parametrize("orth", [rr.SKETCHED_CHOLQR, rr.CHOLQR])
def test_pcg_matches_direct(orth):
    p, op = _kernel_problem()
    mu = p.mus[0]
    P = rr.build(op, [mu], p.l, p.sketch, p.omega_seed, orth=orth)[0]
    res = solvers.pcg(op.shifted(mu), P.apply, p.b, 1e-10)
    xs = solvers.direct(op.dense, mu, p.b)
    assert res.status == solvers.OK
    assert solvers.relres(op.shifted(mu), res.x, p.b) <= 1e-10
    cond = np.linalg.cond(op.dense + mu * np.eye(p.n))
    assert np.linalg.norm(res.x - xs) / np.linalg.norm(xs) <= 10 * 1e-10 * cond
    cgres = solvers.cg(op.shifted(mu), p.b, 1e-10)
    assert cgres.status == solvers.OK
    assert res.iters < cgres.iters


def test_cg_finite_termination():
    n, k = 200, 7
    vals = np.repeat(np.linspace(1.0, 20.0, k), n // k + 1)[:n]
    A = workloads.synthetic_spectrum_matrix(n, vals, 3)
    b = np.random.default_rng(0).standard_normal(n)
    res = solvers.cg(lambda u: A @ u, b, 1e-10, eta=1e-300)
    assert res.status == solvers.OK
    assert res.iters <= k


def test_full_rank_one_iteration():
    n, mu = 60, 0.1
    p = workloads.cfg_small_dense(n=n, d=8, l=n)
    op = Operator.from_problem(p)
    P = rr.build(op, [mu], n, "gaussian", 5, tau_rule=rr.NYS)[0]
    res = solvers.pcg(op.shifted(mu), P.apply, p.b, 1e-8)
    assert res.status == solvers.OK
    assert res.iters == 1


def test_restart_history_monotone_cycles():
    p, op = _kernel_problem(400)
    mu = p.mus[0]
    P = rr.build(op, [mu], p.l, p.sketch, p.omega_seed)[0]
    res = solvers.pcg(op.shifted(mu), P.apply, p.b, 1e-10, eta=1e-2)
    # one true-residual evaluation per cycle, each at least a factor ~eta lower
    h = np.array(res.cycle_history)
    assert len(h) == res.restarts + 2
    assert np.all(h[1:-1] <= 1.5e-2 * h[:-2])
    # the per-iteration history has one entry per iteration plus the start, and
    # its last entry is the final true residual
    assert len(res.history) == res.iters + 1
    assert res.history[0] == 1.0 and res.history[-1] == res.relres


@pytest.mark.parametrize("precond", [False, True])
def test_history_first_step_closed_form(precond):
    # One (P)CG step from x0 = 0 minimises over span{Pb}: x1 = a P b with
    # a = b^T P b / ((P b)^T A (P b)), so r1 = b - a A P b.  The oracle's history[1]
    # must equal ||r1|| / ||b|| computed directly from that formula.
    p, op = _kernel_problem(300)
    mu = p.mus[0]
    A = op.dense + mu * np.eye(p.n)
    if precond:
        Pc = rr.build(op, [mu], p.l, p.sketch, p.omega_seed)[0]
        Pm = Pc.dense()
        apply = Pc.apply
    else:
        Pm = np.eye(p.n)
        apply = lambda r: r.copy()
    b = p.b
    z = Pm @ b
    a = (b @ z) / (z @ (A @ z))
    r1 = b - a * (A @ z)
    res = solvers.pcg(lambda u: A @ u, apply, b, 1e-10, maxit=3)
    assert abs(res.history[1] - np.linalg.norm(r1) / np.linalg.norm(b)) <= 1e-12


def test_breakdown_on_indefinite():
    n = 30
    b = np.ones(n)
    res = solvers.cg(lambda u: -u, b, 1e-8)
    assert res.status == solvers.BREAKDOWN


def test_maxit_returns_iterate():
    p, op = _kernel_problem(300)
    res = solvers.cg(op.shifted(p.mus[0]), p.b, 1e-12, maxit=3)
    assert res.status == solvers.NOCONV and res.iters == 3
    assert res.relres < 1.0
    # resume from the returned iterate (restart = new x0)
    res2 = solvers.cg(op.shifted(p.mus[0]), p.b, 1e-12, x0=res.x, maxit=10_000)
    assert res2.status == solvers.OK


def test_multi_shift_pcg_all_columns():
    p = workloads.cfg_batched(n=500, d=16, l=40, nrhs=3)
    op = Operator.from_problem(p)
    pcs = rr.build(op, p.mus, p.l, p.sketch, p.omega_seed)
    A = op.to_dense()
    for P, mu in zip(pcs, p.mus):
        for j in range(p.B.shape[1]):
            res = solvers.pcg(op.shifted(mu), P.apply, p.B[:, j], 1e-8)
            assert res.status == solvers.OK
            xs = solvers.direct(A, mu, p.B[:, j])
            assert np.linalg.norm(res.x - xs) / np.linalg.norm(xs) < 1e-8 / mu * 10


def test_direct_blocked_equals_direct():
    rng = np.random.default_rng(0)
    M = rng.standard_normal((300, 300))
    A = M @ M.T / 300
    b = rng.standard_normal(300)
    x = solvers.direct(A, 1e-3, b)
    for nb in (64, 100, 300, 512):
        work = np.ascontiguousarray(A.copy())
        xb = solvers.direct_blocked(work, 1e-3, b, nb=nb)
        assert np.abs(xb - x).max() <= 1e-10 * np.abs(x).max()
        L = np.tril(work)
        assert np.abs(L @ L.T - (A + 1e-3 * np.eye(300))).max() <= 1e-13
