"""Pins for the oracle operators: kernel formulas against scikit-learn's
implementations, blocked/threaded matvec against the dense matrix, symmetry
and positive semidefiniteness of Gram matrices (Section 1: A psd)."""
import numpy as np
from sklearn.gaussian_process.kernels import Matern
from sklearn.metrics.pairwise import rbf_kernel

import workloads
from oracle.operators import MATERN32, RBF, Operator, kernel_block


def test_rbf_matches_sklearn():
    rng = np.random.default_rng(0)
    X = rng.standard_normal((50, 7))
    Y = rng.standard_normal((40, 7))
    g = 0.37
    assert np.allclose(kernel_block(RBF, g, X, Y), rbf_kernel(X, Y, gamma=g), rtol=1e-13, atol=0)


def test_matern32_matches_sklearn():
    rng = np.random.default_rng(1)
    X = rng.random((60, 3))
    ell = 0.1
    k = Matern(length_scale=ell, nu=1.5)(X)
    assert np.allclose(kernel_block(MATERN32, np.sqrt(3) / ell, X, X), k, rtol=1e-12, atol=1e-15)


def test_kernel_matvec_blocks_and_threads():
    p = workloads.cfg_kernel_ridge(n=1500, d=16, l=10)
    op = Operator.from_problem(p, block=97, threads=3)
    A = op.to_dense()
    U = np.random.default_rng(2).standard_normal((p.n, 3))
    assert np.allclose(op.matmat(U), A @ U, rtol=1e-12, atol=1e-14)
    assert np.allclose(op.matmat(U[:, 0]), A @ U[:, 0], rtol=1e-12, atol=1e-14)
    assert np.array_equal(A, A.T)
    w = np.linalg.eigvalsh(A)
    assert w.min() > -1e-12 * w.max()


def test_dense_operator_from_problem():
    p = workloads.cfg_small_dense(n=200, d=8, l=10)
    op = Operator.from_problem(p)
    assert op.dense is not None and op.dense.shape == (200, 200)
    assert np.allclose(np.diag(op.dense), 1.0)
