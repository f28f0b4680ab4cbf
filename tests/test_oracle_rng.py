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
