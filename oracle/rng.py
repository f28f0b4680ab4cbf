"""Counter-based random numbers for the method's random test matrices.

The paper draws Omega = X^T from an oblivious subspace embedding (Section 1.1,
eq. testmatrix; Section 2: Gaussian with iid entries, SRHT = S H D with zero
padding to a power of two) and a second-level sketch Theta (Algorithm
prec_chol_qr, a sparse sign embedding).  It fixes no generator, so both implementations use one
published counter-based generator, implemented independently on each side:

* SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
  generators", OOPSLA 2014): state increments by the odd constant
  GAMMA = 0x9E3779B97F4A7C15 and every state is passed through the 64-bit
  finaliser z ^= z>>30; z *= 0xBF58476D1CE4E5B9; z ^= z>>27;
  z *= 0x94D049BB133111EB; z ^= z>>31.  Word k of the stream with seed s is
  therefore mix(s + (k+1)*GAMMA) mod 2^64, which makes every element
  independently addressable.
* Box-Muller: z = sqrt(-2 ln u1) cos(2 pi u2) with u1 in (0,1], u2 in [0,1)
  taken from the top 53 bits of two consecutive words.

Element e of a Gaussian stream uses words 2e and 2e+1.  Matrices are indexed
column-major (e = row + col * nrows).  The Gaussian scale 1/sqrt(l) of the
paper is dropped: Pi, Omega (A_mu Omega)^+, Q, G and tau are invariant under
Omega -> c Omega.
"""
from __future__ import annotations

import numpy as np

MASK = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15
M1 = 0xBF58476D1CE4E5B9
M2 = 0x94D049BB133111EB


def splitmix64_words(seed: int, k: np.ndarray) -> np.ndarray:
    """Words k (uint64 array of indices) of the SplitMix64 stream started at `seed`."""
    k = np.asarray(k, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & MASK) + (k + np.uint64(1)) * np.uint64(GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(M1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(M2)
        z = z ^ (z >> np.uint64(31))
    return z


def gaussian(seed: int, e: np.ndarray) -> np.ndarray:
    """Standard normal values for element indices e (float64), Box-Muller cosine branch."""
    e = np.asarray(e, dtype=np.uint64)
    w1 = splitmix64_words(seed, np.uint64(2) * e)
    w2 = splitmix64_words(seed, np.uint64(2) * e + np.uint64(1))
    u1 = ((w1 >> np.uint64(11)).astype(np.float64) + 1.0) * 2.0 ** -53
    u2 = (w2 >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


def gaussian_matrix(seed: int, rows: int, cols: int) -> np.ndarray:
    """rows x cols Gaussian matrix, element (i, c) from counter i + c*rows."""
    e = np.arange(rows * cols, dtype=np.uint64)
    return gaussian(seed, e).reshape(cols, rows).T.copy()


def gaussian_vector(seed: int, n: int) -> np.ndarray:
    return gaussian(seed, np.arange(n, dtype=np.uint64))


def srht_descriptor(seed: int, n: int, l: int):
    """SRHT parts (Section 2): padded size s = 2^ceil(log2 n), signs D, sampled rows.

    D_i = +1 if the top bit of word i is 0 else -1 (i < n).
    The l sampled Hadamard rows are distinct, drawn by a partial Fisher-Yates
    shuffle of [0, s): step c swaps position c with c + floor(hi32(w) * (s-c) / 2^32)
    where w is word n + c.
    """
    s = 1
    while s < n:
        s *= 2
    if l > s:
        raise ValueError("l exceeds padded size")
    wsign = splitmix64_words(seed, np.arange(n, dtype=np.uint64))
    D = np.where((wsign >> np.uint64(63)) == 0, 1.0, -1.0)
    perm = np.arange(s, dtype=np.int64)
    wsamp = splitmix64_words(seed, np.arange(n, n + l, dtype=np.uint64))
    for c in range(l):
        span = s - c
        j = c + int(((int(wsamp[c]) >> 32) * span) >> 32)
        perm[c], perm[j] = perm[j], perm[c]
    return s, D, perm[:l].copy()


def srht_omega(seed: int, n: int, l: int) -> np.ndarray:
    """Omega = (S H D)^T restricted to the first n rows (zero padding), scale dropped.

    Omega[i, c] = D_i * H[s_c, i] with Sylvester ordering H[a, b] = (-1)^popcount(a & b).
    """
    s, D, rows = srht_descriptor(seed, n, l)
    i = np.arange(n, dtype=np.int64)[:, None]
    bits = np.bitwise_and(i, rows[None, :])
    par = np.zeros_like(bits)
    b = bits.copy()
    while np.any(b):
        par ^= (b & 1)
        b >>= 1
    H = 1.0 - 2.0 * par
    return D[:, None] * H


def round_bf16(x) -> np.ndarray:
    """Round to bfloat16 (via float32, round-to-nearest-even on the top 16 bits)."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    r = (((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def colsample_descriptor(seed: int, n: int, l: int):
    """Signed uniform column sampling (Section 7.2.2 and the limited-memory kernel
    ridge experiments: Omega = X^T a uniform sampling matrix, so A_mu Omega is a set of
    columns of A_mu).  Column c of Omega is D_{i_c} e_{i_c}: the l distinct indices
    i_c come from a partial Fisher-Yates shuffle of [0, n) (step c swaps position c
    with c + floor(hi32(w) (n - c) / 2^32), w = word n + c of stream `seed`) and the
    signs D_i from the top bit of word i -- the SRHT descriptor's draws with the
    padded size replaced by n.  Returns (signs of the sampled columns, indices)."""
    if l > n:
        raise ValueError("l exceeds n")
    wsign = splitmix64_words(seed, np.arange(n, dtype=np.uint64))
    D = np.where((wsign >> np.uint64(63)) == 0, 1.0, -1.0)
    perm = np.arange(n, dtype=np.int64)
    wsamp = splitmix64_words(seed, np.arange(n, n + l, dtype=np.uint64))
    for c in range(l):
        span = n - c
        j = c + int(((int(wsamp[c]) >> 32) * span) >> 32)
        perm[c], perm[j] = perm[j], perm[c]
    idx = perm[:l].copy()
    return D[idx], idx


def colsample_omega(seed: int, n: int, l: int) -> np.ndarray:
    sgn, idx = colsample_descriptor(seed, n, l)
    Om = np.zeros((n, l))
    Om[idx, np.arange(l)] = sgn
    return Om


def omega(kind: str, seed: int, n: int, l: int, bf16: bool = False) -> np.ndarray:
    """The test matrix; `bf16` draws it in bfloat16 (Gaussian entries rounded once)."""
    if kind == "gaussian":
        g = gaussian_matrix(seed, n, l)
        return round_bf16(g) if bf16 else g
    if kind == "srht":
        return srht_omega(seed, n, l)
    if kind == "colsample":
        return colsample_omega(seed, n, l)
    raise ValueError(kind)


THETA_NNZ = 8   # nonzeros per column of Theta


def theta_blocks(k: int):
    """Row blocks of the sparse sign embedding Theta (2k rows): zeta = min(8, 2k)
    blocks, block t = rows [floor(t 2k / zeta), floor((t+1) 2k / zeta))."""
    lsk = 2 * k
    zeta = min(THETA_NNZ, lsk)
    return lsk, zeta, [t * lsk // zeta for t in range(zeta + 1)]


def theta(seed: int, n: int, k: int):
    """Second-level sketch Theta of Algorithm prec_chol_qr: a sparse sign embedding.

    Section 4.2 asks for a fast transform of small size that embeds range(A_mu Omega)
    (eq. epsilon_embedding) and names sparse embeddings with O(log n) nonzeros per
    column among those that do.  Theta is 2k x n; column i has one entry +-1 in each
    of zeta = min(8, 2k) row blocks (the block construction of a sparse
    Johnson-Lindenstrauss transform, Kane and Nelson 2014).  Word w of stream
    seed+1 at counter i*zeta + t gives, for block t of size b_t starting at row
    r_t, the row r_t + floor(hi32(w) * b_t / 2^32) and the sign -1 if bit 0 of w
    is set.  The scale 1/sqrt(zeta) is dropped: R_sk only preconditions, and
    R = R_chol R_sk is unchanged by it.  Returned as a scipy.sparse CSR matrix.
    """
    import scipy.sparse as sp

    lsk, zeta, starts = theta_blocks(k)
    i = np.arange(n, dtype=np.uint64)
    rows, cols, vals = [], [], []
    for t in range(zeta):
        w = splitmix64_words(seed + 1, i * np.uint64(zeta) + np.uint64(t))
        size = np.uint64(starts[t + 1] - starts[t])
        r = np.uint64(starts[t]) + (((w >> np.uint64(32)) * size) >> np.uint64(32))
        rows.append(r.astype(np.int64))
        cols.append(i.astype(np.int64))
        vals.append(np.where((w & np.uint64(1)) == 0, 1.0, -1.0))
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(lsk, n))
