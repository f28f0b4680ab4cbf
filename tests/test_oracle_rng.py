"""Pins for the oracle's counter-based generator (CPU only).

* SplitMix64 against its published output vectors (tests/golden).
* Box-Muller output against the normal distribution (Kolmogorov-Smirnov,
  moments) — a wrong constant or a swapped word fails these.
* SRHT: Sylvester Hadamard from popcount equals scipy.linalg.hadamard; with
  n = s the SRHT columns are exactly orthogonal (Omega^T Omega = s I), the
  sampled rows are distinct (Section 2, SRHT = S H D).
"""
import os

import numpy as np
import pytest
import scipy.linalg as sla
from scipy import stats

from oracle import rng

GOLD = os.path.join(os.path.dirname(__file__), "golden", "splitmix64_vectors.txt")


def test_splitmix64_published_vectors():
    rows = [l.split() for l in open(GOLD) if l.strip() and not l.startswith("#")]
    assert len(rows) >= 6
    for seed, k, val in rows:
        got = rng.splitmix64_words(int(seed), np.array([int(k)], dtype=np.uint64))[0]
        assert int(got) == int(val)


def test_gaussian_is_standard_normal():
    z = rng.gaussian_vector(12345, 200_000)
    assert abs(z.mean()) < 0.01
    assert abs(z.var() - 1.0) < 0.01
    ks = stats.kstest(z, "norm")
    assert ks.pvalue > 1e-3
    # streams with neighbouring seeds are uncorrelated
    z2 = rng.gaussian_vector(12346, 200_000)
    assert abs(np.corrcoef(z, z2)[0, 1]) < 0.01


def test_gaussian_matrix_counter_layout():
    G = rng.gaussian_matrix(7, 5, 3)
    for c in range(3):
        for i in range(5):
            assert G[i, c] == rng.gaussian(7, np.array([i + c * 5], dtype=np.uint64))[0]


def test_sylvester_hadamard_matches_scipy():
    s = 64
    _, D, _ = rng.srht_descriptor(3, s, 1)
    H = sla.hadamard(s)
    # Omega with all rows sampled, signs removed, is H^T restricted to sampled rows
    Om = rng.srht_omega(3, s, s)
    _, D, rows = rng.srht_descriptor(3, s, s)
    assert np.array_equal(Om / D[:, None], H[rows, :].T.astype(float))


@pytest.mark.parametrize("n,l", [(256, 40), (1024, 1024), (300, 50)])
def test_srht_structure(n, l):
    s, D, rows = rng.srht_descriptor(11, n, l)
    assert s >= n and s & (s - 1) == 0 and s < 2 * n
    assert len(set(rows.tolist())) == l
    assert rows.min() >= 0 and rows.max() < s
    Om = rng.srht_omega(11, n, l)
    assert set(np.unique(Om)) <= {-1.0, 1.0}
    if n == s:
        assert np.array_equal(Om.T @ Om, s * np.eye(l))


def test_srht_signs_balanced():
    _, D, _ = rng.srht_descriptor(5, 100_000, 10)
    assert abs(D.mean()) < 0.02


def test_round_bf16_matches_torch():
    import torch
    x = np.concatenate([rng.gaussian_vector(3, 5000) * 10.0 ** np.arange(-3, 2).repeat(1000),
                        [0.0, 1.0, -1.0, 1.00390625, 1.005859375]])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(rng.round_bf16(x), ref)


@pytest.mark.parametrize("n,k", [(1000, 50), (37, 3), (500, 1), (64, 40)])
def test_theta_sparse_sign_structure(n, k):
    """Theta (2k x n): every column holds exactly zeta = min(8, 2k) entries +-1, one in
    each row block, so Theta^T Theta has zeta on its diagonal (Section 4.2, sparse
    embeddings)."""
    T = rng.theta(11, n, k)
    lsk, zeta, starts = rng.theta_blocks(k)
    assert T.shape == (lsk, n)
    assert zeta == min(8, 2 * k)
    assert starts[0] == 0 and starts[-1] == lsk and all(b > a for a, b in zip(starts, starts[1:]))
    Td = T.toarray()
    assert set(np.unique(Td)) <= {-1.0, 0.0, 1.0}
    for t in range(zeta):
        blk = Td[starts[t]:starts[t + 1]]
        assert np.all(np.count_nonzero(blk, axis=0) == 1)
    assert np.array_equal(np.diag(Td.T @ Td), np.full(n, float(zeta)))


def test_theta_rows_uniform_and_signs_balanced():
    """Within a block every row is equally likely, and the signs are fair."""
    n, k = 200_000, 20
    T = rng.theta(4, n, k).tocoo()
    lsk, zeta, starts = rng.theta_blocks(k)
    counts = np.bincount(T.row, minlength=lsk)
    for t in range(zeta):
        c = counts[starts[t]:starts[t + 1]]
        assert stats.chisquare(c).pvalue > 1e-4
    assert abs(np.mean(T.data)) < 5.0 / np.sqrt(T.nnz)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_theta_is_a_subspace_embedding(seed):
    """eq. epsilon_embedding: for an orthonormal U (n x k) the singular values of
    Theta U / sqrt(zeta) lie in [1 - eps, 1 + eps] with eps < 1, so Theta Y has full
    column rank and cond(Y R_sk^{-1}) stays O(1)."""
    n, k = 4000, 40
    U, _ = np.linalg.qr(np.random.default_rng(seed).standard_normal((n, k)))
    T = rng.theta(seed, n, k)
    sv = np.linalg.svd(np.asarray(T @ U) / np.sqrt(8), compute_uv=False)
    assert sv.min() > 0.15 and sv.max() < 1.85


def test_theta_preserves_inner_products_in_expectation():
    """E[<Theta x, Theta y>] = zeta <x, y>: averaged over independent streams."""
    n, k = 3000, 30
    g = np.random.default_rng(5)
    x = g.standard_normal(n)
    y = x + 0.5 * g.standard_normal(n)
    vals = [float((rng.theta(s, n, k) @ x) @ (rng.theta(s, n, k) @ y)) / 8 for s in range(200)]
    assert abs(np.mean(vals) - x @ y) < 4 * np.std(vals) / np.sqrt(len(vals))
