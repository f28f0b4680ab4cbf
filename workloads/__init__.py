"""Seeded synthetic problem generators shared by the oracle, the tests and the bench.

This module builds *problem data only*: point clouds, kernel constants, right-hand
sides, shift values and serving request streams.  It contains none of the
method's arithmetic (no sketch, no orthogonalisation, no preconditioner, no
solver); the random test matrices the method itself draws (Omega, Theta,
power-iteration starts) are produced separately on each side from a
counter-based generator keyed by a seed.

The problem statement is the shifted system (A + mu I) x = b with A symmetric
positive semidefinite (paper, Section 1, eq. initsys).  Kernel operators follow
the kernel ridge normalisation A = K / n of the kernel-regression experiments
(Section 7.2.2, eq. kernel); the stored dense configurations use A = K.

All draws use ``numpy.random.default_rng(seed)`` in a fixed order, and every
point cloud is rounded to float32 so that the float32 GPU operator and the
float64 oracle see exactly the same inputs.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

RBF = 1
MATERN32 = 2
DENSE = 0


@dataclass
class KernelProblem:
    """A kernel (Gram) operator A = scale * K(X, X) on float32 points.

    pts:    (d, n) float32, structure-of-arrays (coordinate-major).
    kind:   RBF (exp(-kconst * r^2)) or MATERN32 ((1 + kconst*r) exp(-kconst*r)).
    kconst: float32-representable constant: 1/(2 sigma^2) for RBF,
            sqrt(3)/ell for Matern-3/2.
    scale:  1 for a plain Gram matrix, 1/n for kernel ridge normalisation.
    """
    name: str
    kind: int
    pts: np.ndarray
    kconst: float
    scale: float
    mus: List[float]
    l: int
    sketch: str            # "gaussian" | "srht"
    omega_seed: int
    tol: float
    b: Optional[np.ndarray] = None        # (n,) float64
    B: Optional[np.ndarray] = None        # (n, m) float64, column-major semantics
    dense: bool = False                   # materialise A as a stored matrix
    bandwidth: float = float("nan")
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.pts.shape[1])

    @property
    def d(self) -> int:
        return int(self.pts.shape[0])


def _f32(x: float) -> float:
    return float(np.float32(x))


def median_pairwise_distance(pts_dn: np.ndarray, m: int = 2000) -> float:
    """Median Euclidean distance over all pairs among the first m points (float64).

    This is the bandwidth rule of the kernel configurations ("bandwidth = median
    pairwise distance"); using a fixed prefix keeps it cheap and deterministic.
    """
    from scipy.spatial.distance import pdist
    X = np.asarray(pts_dn[:, :m], dtype=np.float64).T
    return float(np.median(pdist(X)))


def gaussian_mixture_points(rng, n: int, d: int, ncomp: int = 10,
                            mean_std: float = 3.0) -> np.ndarray:
    """n points from an equal-weight mixture of ncomp unit-covariance Gaussians.

    Component means are drawn N(0, mean_std^2 I_d).  Returns (d, n) float32.
    """
    means = rng.standard_normal((ncomp, d)) * mean_std
    labels = rng.integers(0, ncomp, size=n)
    X = means[labels] + rng.standard_normal((n, d))
    return np.ascontiguousarray(X.T.astype(np.float32))


def rbf_problem(name, pts, mus, l, sketch, omega_seed, tol, rng, scale_by_n=True,
                bandwidth=None, nrhs=None, dense=False, bw_sample=2000):
    if bandwidth is None:
        bandwidth = median_pairwise_distance(pts, bw_sample)
    kconst = _f32(1.0 / (2.0 * bandwidth * bandwidth))
    n = pts.shape[1]
    p = KernelProblem(name=name, kind=RBF, pts=pts, kconst=kconst,
                      scale=(1.0 / n) if scale_by_n else 1.0, mus=list(mus), l=l,
                      sketch=sketch, omega_seed=omega_seed, tol=tol, dense=dense,
                      bandwidth=float(bandwidth))
    if nrhs is None:
        p.b = rng.standard_normal(n)
    else:
        p.B = rng.standard_normal((n, nrhs))
    return p


# --------------------------------------------------------------------------
# The five workload families.  Each takes optional size overrides so the same
# recipe can be instantiated at sizes a float64 CPU oracle finishes in seconds.
# --------------------------------------------------------------------------

def cfg_small_dense(n: int = 2000, d: int = 8, l: int = 100, seed: int = 1) -> KernelProblem:
    """Plain float64 method, stored dense Gaussian RBF matrix.

    n points x_i ~ N(0, I_d), bandwidth 1 (kconst = 0.5, exact), A = K stored
    dense, mu = 1e-3, l Gaussian test vectors (seed 11), b ~ N(0,1), tol 1e-8.
    """
    rng = np.random.default_rng(seed)
    pts = np.ascontiguousarray(rng.standard_normal((n, d)).T.astype(np.float32))
    return rbf_problem("dense-rbf-fp64", pts, [1e-3], l, "gaussian", 11, 1e-8, rng,
                       scale_by_n=False, bandwidth=1.0, dense=True)


def cfg_kernel_ridge(n: int = 50_000, d: int = 16, l: int = 500, seed: int = 2,
                     mu: float = 1e-4) -> KernelProblem:
    """Matrix-free kernel ridge: n points in d=16 from a 10-component mixture.

    RBF kernel, bandwidth = median pairwise distance, A = K/n, mu = 1e-4,
    l = 500 SRHT test vectors (seed 12), b ~ N(0,1), tol 1e-6.
    """
    rng = np.random.default_rng(seed)
    pts = gaussian_mixture_points(rng, n, d)
    return rbf_problem("kernel-ridge-rbf", pts, [mu], l, "srht", 12, 1e-6, rng)


def cfg_precision(n: int = 65_536, l: int = 1024, seed: int = 3, ell: float = 0.1,
                  mu: float = 1e-5) -> KernelProblem:
    """Precision form: stored dense Matern-3/2 on n uniform points in [0,1]^3.

    A = K (float64 authoritative; the library derives float32/bf16 copies),
    mu = 1e-5, l = 1024 Gaussian test vectors (seed 13), FP64 refinement to 1e-10.
    """
    rng = np.random.default_rng(seed)
    pts = np.ascontiguousarray(rng.random((n, 3)).T.astype(np.float32))
    kconst = _f32(math.sqrt(3.0) / ell)
    p = KernelProblem(name="precision-matern32", kind=MATERN32, pts=pts, kconst=kconst,
                      scale=1.0, mus=[mu], l=l, sketch="gaussian", omega_seed=13,
                      tol=1e-10, dense=True, bandwidth=ell)
    p.b = rng.standard_normal(n)
    return p


def cfg_batched(n: int = 50_000, d: int = 16, l: int = 500, nrhs: int = 256,
                seed: int = 2, mus=(1e-3, 1e-4, 1e-5, 1e-6)) -> KernelProblem:
    """Batched block solve on the kernel-ridge matrix: nrhs RHS x len(mus) shifts.

    Same points and bandwidth as the kernel-ridge workload (same seed and draw
    order), B ~ N(0,1) drawn from a second generator (seed 4), SRHT l = 500
    (seed 14), every RHS under every shift, tol 1e-6 per column.
    """
    rng = np.random.default_rng(seed)
    pts = gaussian_mixture_points(rng, n, d)
    p = rbf_problem("batched-kernel-ridge", pts, list(mus), l, "srht", 14, 1e-6,
                    np.random.default_rng(4), nrhs=nrhs)
    return p


@dataclass
class Request:
    rid: int
    t_arrival: float
    problem: KernelProblem


def serving_stream(num: int = 2200, rate: float = 200.0, seed: int = 5,
                   n_min: int = 1000, n_max: int = 32768, tol: float = 1e-6,
                   d_choices=(4, 8, 16)) -> List[Request]:
    """Poisson stream of independent RBF ridge problems.

    Inter-arrival ~ Exp(rate); n log-uniform in [n_min, n_max]; d uniform in
    d_choices; mu log-uniform in [1e-6, 1e-2]; l = ceil(n/32); 1-8 RHS each;
    points N(0, I_d) rounded to float32; median-rule bandwidth over the first
    400 points of each request (enough for an i.i.d. Gaussian cloud); A = K/n.
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for rid in range(num):
        t += rng.exponential(1.0 / rate)
        n = int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max)))))
        d = int(rng.choice(np.asarray(d_choices)))
        mu = float(math.exp(rng.uniform(math.log(1e-6), math.log(1e-2))))
        nrhs = int(rng.integers(1, 9))
        l = int(math.ceil(n / 32))
        pts = np.ascontiguousarray(rng.standard_normal((n, d)).T.astype(np.float32))
        prob = rbf_problem(f"req{rid}", pts, [mu], l, "gaussian", 1000 + rid, tol, rng,
                           nrhs=nrhs, bw_sample=400)
        out.append(Request(rid=rid, t_arrival=t, problem=prob))
    return out


def synthetic_spectrum_matrix(n: int, eigs: np.ndarray, seed: int) -> np.ndarray:
    """A = U diag(eigs) U^T with U Haar-random orthogonal (dense float64).

    The synthetic-spectrum family of the paper's Section 7.1 (exponential
    top part plus a power-law tail); used for small-n bound checks.
    """
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((n, n))
    U, R = np.linalg.qr(G)
    U = U * np.sign(np.diag(R))
    A = (U * eigs) @ U.T
    return 0.5 * (A + A.T)
