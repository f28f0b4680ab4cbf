"""GPU parity: the HIP path (through the C ABI) against the float64 oracle.

Sizes span several kernel tiles with ragged tails (n not a multiple of 64 or
1024, l not a multiple of 32/64).  Tolerances:
  * random matrices: Gaussian <= 4 ulp-scale (1e-14 relative; log/cos may differ
    in the last bit), SRHT bit-exact;
  * float64 operators / sketch / basis: 1e-12 .. 1e-9 relative (rounding order);
  * float64 solves: relres(x_gpu) <= relres(x_oracle) + 1e-8 with both <= tol,
    iteration counts within max(2, 3%);
  * float32-entry operators: the float32 rounding of each kernel entry bounds
    the matvec error by ~n * 2^-23 * max|A| per row sum (checked at 2e-6 relative).
"""
import os

import numpy as np
import pytest

import workloads
from oracle import randrand as orr
from oracle import rng as orng
from oracle import block as oblk
from oracle import solvers as osol
from oracle.operators import Operator

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

rr = pytest.importorskip("paper_2509_19747_amd")


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.fixture(scope="module")
def dense_small():
    prob = workloads.cfg_small_dense(n=777, d=8, l=45)
    op = Operator.from_problem(prob)
    pts = _cuda(prob.pts)
    kop = rr.kernel_operator(rr.OP_RBF, pts, prob.kconst, prob.scale)
    A = rr.kernel_to_dense(kop, "fp64")
    return prob, op, kop, A


@pytest.mark.parametrize("rows,cols,seed", [(37, 5, 3), (1000, 3, 11), (1, 1, 0)])
def test_gaussian_matrix(rows, cols, seed):
    g = rr.random_matrix("gaussian", seed, rows, cols).cpu().numpy()
    ref = orng.gaussian_matrix(seed, rows, cols)
    assert np.allclose(g, ref, rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("n,l,seed", [(256, 40, 12), (1000, 100, 5), (50_000, 7, 12), (3, 4, 1)])
def test_srht_matrix_bit_exact(n, l, seed):
    g = rr.random_matrix("srht", seed, n, l).cpu().numpy()
    ref = orng.srht_omega(seed, n, l)
    assert np.array_equal(g, ref)


def test_kernel_to_dense_fp64(dense_small):
    prob, op, kop, A = dense_small
    assert np.allclose(A.cpu().numpy(), op.dense, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("kind", [rr.OP_RBF, rr.OP_MATERN32])
@pytest.mark.parametrize("n,d", [(1500, 16), (333, 3), (1025, 4), (1, 2), (7, 32), (33, 9), (257, 17)])
def test_kernel_matvec(kind, n, d):
    rng = np.random.default_rng(n + d)
    pts = rng.standard_normal((d, n)).astype(np.float32)
    kconst, scale, mu = 0.21, 1.0 / n, 1e-3
    op = Operator(kind=kind, pts=pts, kconst=kconst, scale=scale)
    u = rng.standard_normal(n)
    ref = op.matmat(u) + mu * u
    kop = rr.kernel_operator(kind, _cuda(pts), kconst, scale)
    y64 = rr.apply_operator(kop, mu, "fp64", _cuda(u)).cpu().numpy()
    assert np.linalg.norm(y64 - ref) <= 1e-12 * np.linalg.norm(ref)
    y32 = rr.apply_operator(kop, mu, "fp32", _cuda(u)).cpu().numpy()
    assert np.linalg.norm(y32 - ref) <= 2e-6 * np.linalg.norm(ref)


@pytest.mark.parametrize("kind", [rr.OP_RBF, rr.OP_MATERN32])
@pytest.mark.parametrize("n,d,nr", [(5000, 16, 1), (5000, 16, 2), (4100, 5, 3), (3001, 20, 5),
                                    (4500, 8, 8), (2600, 4, 13)])
def test_kernel_matvec_block_multi_tile(kind, n, d, nr):
    # several row blocks with a ragged last block: the symmetric float32 path forms
    # off-diagonal block pairs once and scatters them to rows and columns
    rng = np.random.default_rng(7 * n + d + nr)
    pts = rng.standard_normal((d, n)).astype(np.float32)
    kconst, scale, mu = 0.5 / d, 1.0 / n, 1e-3
    op = Operator(kind=kind, pts=pts, kconst=kconst, scale=scale)
    U = rng.standard_normal((n, nr))
    ref = op.matmat(U) + mu * U
    kop = rr.kernel_operator(kind, _cuda(pts), kconst, scale)
    Y32 = rr.apply_operator_block(kop, mu, "fp32", _cuda(U)).cpu().numpy()
    for q in range(nr):
        assert np.linalg.norm(Y32[:, q] - ref[:, q]) <= 2e-6 * np.linalg.norm(ref[:, q]), q
    Y64 = rr.apply_operator_block(kop, mu, "fp64", _cuda(U)).cpu().numpy()
    assert np.linalg.norm(Y64 - ref) <= 1e-12 * np.linalg.norm(ref)
    # a block product (column blocks of four, two and one) equals the column-by-column
    # products bitwise
    for q in range(nr):
        yq = rr.apply_operator(kop, mu, "fp32", _cuda(U[:, q].copy())).cpu().numpy()
        assert np.array_equal(yq, Y32[:, q]), q


def test_kernel_fp32_matvec_beyond_mfma_slot_bound():
    # n = 600,000 exceeds the MFMA matvec's partial-slot bound, so the float32-mode
    # operator takes the vector-ALU symmetric kernel: sampled rows against the oracle
    from oracle.operators import kernel_block
    n, d = 600_000, 4
    rng = np.random.default_rng(17)
    pts = rng.standard_normal((d, n)).astype(np.float32)
    kconst, scale, mu = 2.0, 1.0 / n, 1e-3
    kop = rr.kernel_operator(rr.OP_RBF, _cuda(pts), kconst, scale)
    u = rng.standard_normal(n)
    y = rr.apply_operator(kop, mu, "fp32", _cuda(u)).cpu().numpy()
    X = pts.T.astype(np.float64)
    rows = np.unique(np.concatenate([rng.integers(0, n, 12), [0, n - 1]]))
    Kr = scale * kernel_block(rr.OP_RBF, kconst, X[rows], X)
    ref = Kr @ u + mu * u[rows]
    bound = np.abs(Kr) @ np.abs(u) + mu * np.abs(u[rows])
    assert np.all(np.abs(y[rows] - ref) <= 2e-6 * bound), np.max(np.abs(y[rows] - ref) / bound)


@pytest.mark.parametrize("kind", [rr.OP_RBF, rr.OP_MATERN32])
def test_kernel_fp32_matvec_large_multi_block_items(kind):
    # n large enough that a work item runs over several column blocks (and row
    # blocks own several runs): sampled rows against the oracle's kernel rows, the
    # two-column block against the single-column product, and exact symmetry of
    # the float32 operator seen through float64 sums (u.Kv = v.Ku to rounding)
    from oracle.operators import kernel_block
    n, d = 40_000, 16
    rng = np.random.default_rng(41 + kind)
    pts = rng.standard_normal((d, n)).astype(np.float32)
    kconst, scale, mu = 0.5 / d, 1.0 / n, 1e-3
    kop = rr.kernel_operator(kind, _cuda(pts), kconst, scale)
    U = rng.standard_normal((n, 2))
    Y = rr.apply_operator_block(kop, mu, "fp32", _cuda(U)).cpu().numpy()
    y0 = rr.apply_operator(kop, mu, "fp32", _cuda(U[:, 0].copy())).cpu().numpy()
    assert np.array_equal(y0, Y[:, 0])
    X = pts.T.astype(np.float64)
    rows = np.unique(np.concatenate([rng.integers(0, n, 48), [0, 255, 256, n - 1, n - 2]]))
    Kr = scale * kernel_block(kind, kconst, X[rows], X)
    ref = Kr @ U + mu * U[rows]
    bound = np.abs(Kr) @ np.abs(U) + mu * np.abs(U[rows])
    assert np.all(np.abs(Y[rows] - ref) <= 2e-6 * bound), np.max(np.abs(Y[rows] - ref) / bound)
    uKv = U[:, 0] @ (Y[:, 1] - mu * U[:, 1])
    vKu = U[:, 1] @ (Y[:, 0] - mu * U[:, 0])
    # an asymmetric float32 operator would leave a gap near 1e-7
    assert abs(uKv - vKu) <= 1e-11 * (np.abs(U[:, 0]) @ np.abs(Y[:, 1] - mu * U[:, 1]))


def test_kernel_fp32_operator_symmetric_multi_tile():
    # float32 entries of different row blocks are formed once: K e_j and K e_i agree
    n, d = 2600, 16
    rng = np.random.default_rng(2)
    pts = rng.standard_normal((d, n)).astype(np.float32)
    kop = rr.kernel_operator(rr.OP_RBF, _cuda(pts), 0.05, 1.0)
    E = torch.eye(n, dtype=torch.float64, device="cuda")
    K = rr.apply_operator_block(kop, 0.0, "fp32", E).cpu().numpy()
    assert np.array_equal(K, K.T)
    ref = Operator(kind=rr.OP_RBF, pts=pts, kconst=0.05, scale=1.0).to_dense()
    # elementwise bound from the arithmetic: the exponent t = -kconst |x_i - x_j|^2 is the
    # float32-class record product (terms g |x_i|^2 / 2, g |x_j|^2 / 2, g x_i.x_j, each
    # split into bf16 pieces to 24 bits, summed over 6 d + 6 products in float32), so
    # |dt| <= (6 d + 6) 2^-24 kconst (|x_i|^2 + |x_j|^2 + 2 |x_i.x_j|); the entry
    # exp(t) then has relative error |dt| plus the exp2's own 2^-22
    X = pts.T.astype(np.float64)
    sq = np.sum(X * X, axis=1)
    mag = sq[:, None] + sq[None, :] + 2.0 * np.abs(X @ X.T)
    bound = ref * ((6 * d + 6) * 2.0 ** -24 * 0.05 * mag + 2.0 ** -22)
    assert np.all(np.abs(K - ref) <= bound), np.max(np.abs(K - ref) / bound)


def test_kernel_fp32_operator_symmetric():
    # float32 entries are formed bitwise-symmetrically: e_i^T K e_j == e_j^T K e_i
    n, d = 300, 16
    rng = np.random.default_rng(1)
    pts = rng.standard_normal((d, n)).astype(np.float32)
    kop = rr.kernel_operator(rr.OP_RBF, _cuda(pts), 0.05, 1.0)
    E = torch.eye(n, dtype=torch.float64, device="cuda")
    cols = torch.stack([rr.apply_operator(kop, 0.0, "fp32", E[j]) for j in range(n)], 1)
    K = cols.cpu().numpy()
    assert np.array_equal(K, K.T)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_dense_matvec(dense_small, prec):
    prob, op, kop, A = dense_small
    u = np.random.default_rng(3).standard_normal(prob.n)
    mu = 0.37
    y = rr.apply_operator(rr.dense_operator(A), mu, prec, _cuda(u)).cpu().numpy()
    ref = op.dense @ u + mu * u
    tol = 1e-13 if prec == "fp64" else 1e-6
    assert np.linalg.norm(y - ref) <= tol * np.linalg.norm(ref)


@pytest.mark.parametrize("n,k", [(3000, 40), (257, 5), (5000, 300), (70, 1), (200, 200)])
def test_theta_apply_matches_oracle_bitwise(n, k):
    """S = Theta Y: each entry sums its hits in increasing column order of Theta,
    as the oracle's CSR product does, and every term is +-Y exactly, so S agrees
    bit for bit; with Y = I the result is Theta itself."""
    Y = np.random.default_rng(n + k).standard_normal((n, k))
    S = rr.theta_apply(7, _cuda(Y)).cpu().numpy()
    assert np.array_equal(S, np.asarray(orng.theta(7, n, k) @ Y))
    if n == k:
        St = rr.theta_apply(7, _cuda(np.eye(n))).cpu().numpy()
        assert np.array_equal(St, orng.theta(7, n, n).toarray())


def test_sketched_cholqr_on_an_ill_conditioned_sketch():
    """Alg. prec_chol_qr keeps Q orthonormal to rounding when cond(Y) ~ 1e10, where
    Cholesky QR of Y^T Y would lose all orthogonality: the sparse Theta must embed
    range(Y) well for R_sk to precondition W = Y R_sk^{-1}."""
    n, l = 600, 48
    g = np.random.default_rng(3)
    U, _ = np.linalg.qr(g.standard_normal((n, n)))
    lam = np.concatenate([np.logspace(0, -11, l), np.full(n - l, 1e-12)])
    A = (U * lam) @ U.T
    A = 0.5 * (A + A.T)
    P = rr.build_precond(rr.dense_operator(_cuda(A)), [1e-12], l=l, sketch="gaussian", seed=5,
                         prec="fp64")
    e = P.export(0)
    Q, R = e["Q"], e["R"]
    Y = A @ orng.gaussian_matrix(5, n, l) + 1e-12 * orng.gaussian_matrix(5, n, l)
    assert np.linalg.cond(Y) > 1e10
    assert np.abs(Q.T @ Q - np.eye(l)).max() < 1e-12
    assert np.linalg.norm(Q @ R - Y) < 1e-12 * np.linalg.norm(Y)


@pytest.mark.parametrize("orth", ["sketched", "cholqr"])
@pytest.mark.parametrize("tau_rule", ["opt", "rho", "nys"])
def test_build_fp64_matches_oracle(dense_small, orth, tau_rule):
    prob, op, kop, A = dense_small
    mu, l = prob.mus[0], prob.l
    P = rr.build_precond(rr.dense_operator(A), [mu], l=l, sketch="gaussian", seed=prob.omega_seed,
                         orth=orth, tau_rule=tau_rule, rho=0.5)
    g = P.export(0)
    o = orr.build(op, [mu], l, "gaussian", prob.omega_seed,
                  orth=orr.SKETCHED_CHOLQR if orth == "sketched" else orr.CHOLQR,
                  tau_rule={"opt": orr.OPT, "rho": orr.RHO, "nys": orr.NYS}[tau_rule], rho=0.5)[0]
    rel = lambda a, b_: np.linalg.norm(a - b_) / np.linalg.norm(b_)
    assert np.allclose(P.omega(), orng.gaussian_matrix(prob.omega_seed, prob.n, l), rtol=1e-14, atol=1e-14)
    assert rel(g["Q"], o.Q) < 1e-10
    assert rel(g["R"], o.R) < 1e-10
    assert rel(g["G"], o.G) < 1e-9
    assert rel(g["T"], o.T) < 1e-12
    if tau_rule == "nys":
        # device Lanczos on the device G versus the exact eigenvalue of the oracle's G
        assert abs(g["tau"] - o.tau) < 1e-9 * o.tau
    else:
        assert abs(g["normE"] - o.normE) < 1e-9 * o.normE
        assert abs(g["lam"] - o.lam) < 1e-9 * o.lam
        assert abs(g["tau"] - o.tau) < 1e-9 * o.tau


def test_build_fp64_wide_basis_matches_oracle():
    """l = 600 (triangular inverses of 600 x 600 factors, Householder panels past
    512 rows of the 1200-row sketch) against the oracle."""
    prob = workloads.cfg_small_dense(n=1400, d=8, l=600)
    op = Operator.from_problem(prob)
    kop = rr.kernel_operator(rr.OP_RBF, _cuda(prob.pts), prob.kconst, prob.scale)
    A = rr.kernel_to_dense(kop, "fp64")
    mu = prob.mus[0]
    P = rr.build_precond(rr.dense_operator(A), [mu], l=prob.l, sketch="gaussian", seed=prob.omega_seed)
    g = P.export(0)
    o = orr.build(op, [mu], prob.l, "gaussian", prob.omega_seed)[0]
    rel = lambda a, b_: np.linalg.norm(a - b_) / np.linalg.norm(b_)
    assert rel(g["Q"], o.Q) < 1e-9
    assert rel(g["R"], o.R) < 1e-9
    assert rel(g["G"], o.G) < 1e-8
    assert abs(g["tau"] - o.tau) < 1e-8 * o.tau


@pytest.mark.parametrize("k,spectrum", [(1, "flat"), (45, "decay"), (300, "cluster"),
                                        (1024, "decay"), (1536, "lowrank")])
def test_lambda_max_matches_eigvalsh(k, spectrum):
    """The NYS rule's lambda_max(G) (eq. nys_tau) against LAPACK's eigvalsh, to rounding:
    decaying, top-clustered (gap 1e-6) and rank-deficient spectra."""
    g = np.random.default_rng(k)
    U, _ = np.linalg.qr(g.standard_normal((k, k)))
    if spectrum == "flat":
        ev = np.full(k, 2.5)
    elif spectrum == "decay":
        ev = np.logspace(2, -8, k)
    elif spectrum == "cluster":
        ev = np.concatenate([[1.0, 1.0 - 1e-6, 1.0 - 2e-6], np.linspace(0.9, 1e-3, k - 3)])
    else:
        ev = np.concatenate([np.logspace(1, -3, 40), np.zeros(k - 40)])
    G = (U * ev) @ U.T
    G = 0.5 * (G + G.T)
    lam, res, steps = rr.binding.lambda_max(_cuda(G), seed=7)
    ref = np.max(np.linalg.eigvalsh(G))
    assert abs(lam - ref) <= 1e-12 * ref, (lam, ref, res, steps)
    assert res <= 1e-13 * ref or steps == k


def test_cholesky_ladder_matches_oracle():
    """The device Cholesky and its shift ladder against the oracle's: same alpha, and
    R^T R = W + alpha I to rounding (no shift for an spd W, one step for a failing pivot)."""
    g = np.random.default_rng(5)
    U, _ = np.linalg.qr(g.standard_normal((40, 40)))
    for ev_min, shift in ((1e-3, 0.0), (-3.7e-9, None)):
        ev = np.logspace(0, -6, 40)
        ev[-1] = ev_min
        W = (U * ev) @ U.T
        W = 0.5 * (W + W.T)
        R, alpha = rr.binding.cholesky_ladder(_cuda(W))
        R = R.cpu().numpy()
        Ro, ao = orr.chol_upper_ladder(W)
        assert alpha == ao
        if shift is not None:
            assert alpha == shift
        assert np.allclose(np.tril(R, -1), 0.0)
        assert np.linalg.norm(R.T @ R - (W + alpha * np.eye(40))) < 1e-13
    W = np.diag([1.0, 1.0, -5e-13])
    R, alpha = rr.binding.cholesky_ladder(_cuda(W))
    assert alpha == 1e-12
    W = -np.eye(4)
    with pytest.raises(rr.RRError):
        rr.binding.cholesky_ladder(_cuda(W))


@pytest.mark.parametrize("n,l", [(300, 64), (320, 65), (600, 200), (800, 300)])
def test_build_fp64_triangular_inverse_widths(n, l):
    """Basis widths at and across the row-slot sizes of the wave-per-column
    triangular inverse (64 rows per register slot: one, two, four and eight slots),
    each against the oracle."""
    prob = workloads.cfg_small_dense(n=n, d=8, l=l)
    op = Operator.from_problem(prob)
    kop = rr.kernel_operator(rr.OP_RBF, _cuda(prob.pts), prob.kconst, prob.scale)
    A = rr.kernel_to_dense(kop, "fp64")
    mu = prob.mus[0]
    P = rr.build_precond(rr.dense_operator(A), [mu], l=prob.l, sketch="gaussian", seed=prob.omega_seed)
    g = P.export(0)
    o = orr.build(op, [mu], prob.l, "gaussian", prob.omega_seed)[0]
    rel = lambda a, b_: np.linalg.norm(a - b_) / np.linalg.norm(b_)
    assert rel(g["Q"], o.Q) < 1e-9
    assert rel(g["R"], o.R) < 1e-9
    assert rel(g["G"], o.G) < 1e-8
    assert abs(g["tau"] - o.tau) < 1e-8 * o.tau
    assert np.abs(g["Q"].T @ g["Q"] - np.eye(l)).max() < 1e-12


@pytest.mark.parametrize("l", [0, 45])
@pytest.mark.parametrize("use_graph", [False, True])
def test_solve_fp64_matches_oracle(dense_small, l, use_graph):
    prob, op, kop, A = dense_small
    mu, tol = prob.mus[0], 1e-10
    P = rr.build_precond(rr.dense_operator(A), [mu], l=l, sketch="gaussian", seed=prob.omega_seed)
    x, info = P.solve(_cuda(prob.b), tol=tol, use_graph=use_graph, check_every=5)
    x = x.cpu().numpy()
    Pr = orr.build(op, [mu], l, "gaussian", prob.omega_seed)[0]
    ref = osol.pcg(op.shifted(mu), Pr.apply, prob.b, tol)
    rel_gpu = osol.relres(op.shifted(mu), x, prob.b)
    assert info["rc"] == rr.RR_OK
    assert rel_gpu <= tol and rel_gpu <= ref.relres + 1e-8
    assert abs(info["iters"] - ref.iters) <= max(2, int(0.03 * ref.iters))
    assert abs(info["relres_fp64"] - rel_gpu) <= 1e-3 * rel_gpu + 1e-15
    xs = osol.direct(op.dense, mu, prob.b)
    cond = np.linalg.cond(op.dense + mu * np.eye(prob.n))
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= 10 * tol * cond


def test_solve_graph_equals_eager_bitwise(dense_small):
    prob, op, kop, A = dense_small
    P = rr.build_precond(rr.dense_operator(A), prob.mus, l=prob.l, seed=prob.omega_seed)
    b = _cuda(prob.b)
    x1, i1 = P.solve(b, tol=1e-9, use_graph=False, check_every=4)
    x2, i2 = P.solve(b, tol=1e-9, use_graph=True, check_every=4)
    x3, i3 = P.solve(b, tol=1e-9, use_graph=True, check_every=4)
    assert torch.equal(x1, x2) and torch.equal(x2, x3)
    assert i1["iters"] == i2["iters"] == i3["iters"]


def test_history_matches_oracle(dense_small):
    # per-iteration relative residuals (recurrence inside a cycle, true residual at
    # each restart) against the oracle's PCG on the same preconditioner, entry by entry
    prob, op, kop, A = dense_small
    mu = prob.mus[0]
    P = rr.build_precond(rr.dense_operator(A), [mu], l=prob.l, seed=prob.omega_seed)
    h = np.full(400, np.nan)
    x, info = P.solve(_cuda(prob.b), tol=1e-10, history=h)
    Pr = orr.build(op, [mu], prob.l, "gaussian", prob.omega_seed)[0]
    ref = osol.pcg(op.shifted(mu), Pr.apply, prob.b, 1e-10)
    href = np.array(ref.history)
    assert len(href) == ref.iters + 1
    k = min(info["iters"], ref.iters, 20)
    assert k >= 10
    assert h[0] == pytest.approx(1.0, rel=1e-14)
    np.testing.assert_allclose(h[: k + 1], href[: k + 1], rtol=1e-7, atol=0)
    assert h[info["iters"]] <= 1e-10 * 1.0001


@pytest.mark.parametrize("kind", [rr.OP_RBF, rr.OP_MATERN32])
def test_kernel_fp64_matvec_large_sampled_rows(kind):
    """The pair-once float64 kernel matvec at n = 40,000 (many row blocks and column
    slices, ragged tail): sampled rows against the oracle's float64 kernel rows."""
    from oracle.operators import kernel_block
    n, d = 40_003, 16
    rng = np.random.default_rng(5 + kind)
    pts = rng.standard_normal((d, n)).astype(np.float32)
    kconst, scale, mu = 0.5 / d, 1.0 / n, 1e-4
    kop = rr.kernel_operator(kind, _cuda(pts), kconst, scale)
    U = rng.standard_normal((n, 2))
    Y = rr.apply_operator_block(kop, mu, "fp64", _cuda(U)).cpu().numpy()
    y0 = rr.apply_operator(kop, mu, "fp64", _cuda(U[:, 0].copy())).cpu().numpy()
    assert np.array_equal(y0, Y[:, 0])
    X = pts.T.astype(np.float64)
    rows = np.unique(np.concatenate([rng.integers(0, n, 40), [0, 1023, 1024, n - 1]]))
    Kr = scale * kernel_block(kind, kconst, X[rows], X)
    ref = Kr @ U + mu * U[rows]
    bound = np.abs(Kr) @ np.abs(U) + mu * np.abs(U[rows])
    assert np.all(np.abs(Y[rows] - ref) <= 1e-13 * bound), np.max(np.abs(Y[rows] - ref) / bound)


def test_operator_delta_norm_matches_dense_difference():
    """||A_fp32 - A||_2 by power iteration against numpy's 2-norm of the difference of
    the two operators formed densely (the float32 one through the library's own
    products with the identity)."""
    n, d = 700, 16
    rng = np.random.default_rng(8)
    pts = rng.standard_normal((d, n)).astype(np.float32)
    kop = rr.kernel_operator(rr.OP_RBF, _cuda(pts), 0.03, 1.0 / n)
    E = torch.eye(n, dtype=torch.float64, device="cuda")
    K32 = rr.apply_operator_block(kop, 0.0, "fp32", E).cpu().numpy()
    K64 = Operator(kind=rr.OP_RBF, pts=pts, kconst=0.03, scale=1.0 / n).to_dense()
    ref = np.linalg.norm(K32 - K64, 2)
    est = rr.binding.operator_delta_norm(kop, "fp32", iters=60)
    assert 0.9 * ref <= est <= ref * (1 + 1e-6)


@pytest.mark.parametrize("kind", [rr.OP_RBF, rr.OP_MATERN32])
def test_kernel_fp32_solve_fp64_refinement_matches_oracle(kind):
    """Outer float64 refinement on a kernel operator (restart residuals with the float64
    pair-once kernel): the float64 relative residual reaches tol = 1e-9, below what the
    float32-class working operator alone can resolve; the iteration count is within
    10 % of the oracle's Alg. RandRAND_PCG run in float64 with the same preconditioner."""
    prob = workloads.cfg_kernel_ridge(n=3000, d=16, l=100)
    mu, tol = prob.mus[0], 1e-9
    kop = rr.kernel_operator(kind, _cuda(prob.pts), prob.kconst, prob.scale)
    op = Operator(kind=kind, pts=prob.pts, kconst=prob.kconst, scale=prob.scale)
    P = rr.build_precond(kop, [mu], l=prob.l, sketch="srht", seed=prob.omega_seed, prec="fp32")
    x, info = P.solve(_cuda(prob.b), tol=tol, fp64_ir=1, maxit=20000)
    x = x.cpu().numpy()
    rel64 = osol.relres(op.shifted(mu), x, prob.b)
    assert info["rc"] == rr.RR_OK
    assert rel64 <= tol * 1.01 and abs(info["relres_fp64"] - rel64) <= 1e-3 * rel64
    Pr = orr.build(op, [mu], prob.l, "srht", prob.omega_seed, omega_bf16=True)[0]
    ref = osol.pcg(op.shifted(mu), Pr.apply, prob.b, tol, maxit=20000)
    assert ref.status == osol.OK
    assert abs(info["iters"] - ref.iters) <= max(3, int(0.1 * ref.iters)), (info["iters"], ref.iters)
    # without refinement the float64 residual is bounded by the S16 bound
    x0, i0 = P.solve(_cuda(prob.b), tol=1e-6, fp64_ir=0, certify=True)
    x0 = x0.cpu().numpy()
    r0 = osol.relres(op.shifted(mu), x0, prob.b)
    dA = rr.binding.operator_delta_norm(kop, "fp32", iters=30)
    assert r0 <= i0["relres_work"] + 1.5 * dA * np.linalg.norm(x0) / np.linalg.norm(prob.b)


@pytest.mark.parametrize("n,l", [(1500, 50), (4000, 120), (9000, 150)])
def test_kernel_fp32_srht_factors_against_oracle(n, l):
    """The float32-mode build with an SRHT test matrix, whose C = Omega^T Y comes from
    Walsh-Hadamard transforms of chunks of Y (one chunk shorter than 4,096 points, one
    full chunk, three chunks with a ragged last one): R, G and tau against the oracle's
    float64 build on the same bf16 Omega, within the float32-class sketch's error (measured
    at 1e-6 for R and 5e-5 for G; a wrong C would put G off by O(1))."""
    prob = workloads.cfg_kernel_ridge(n=n, d=16, l=l)
    mu = prob.mus[0]
    kop = rr.kernel_operator(rr.OP_RBF, _cuda(prob.pts), prob.kconst, prob.scale)
    P = rr.build_precond(kop, [mu], l=l, sketch="srht", seed=prob.omega_seed, prec="fp32")
    g = P.export(0, with_q=False)
    o = orr.build(Operator.from_problem(prob), [mu], l, "srht", prob.omega_seed, omega_bf16=True)[0]
    rel = lambda a, b_: np.linalg.norm(a - b_) / np.linalg.norm(b_)
    assert rel(g["R"], o.R) < 1e-5 and rel(g["G"], o.G) < 1e-3 and abs(g["tau"] - o.tau) < 1e-3 * o.tau


def test_kernel_fp32_solve_with_srht():
    prob = workloads.cfg_kernel_ridge(n=4000, d=16, l=120)
    mu = prob.mus[0]
    op = Operator.from_problem(prob)
    kop = rr.kernel_operator(rr.OP_RBF, _cuda(prob.pts), prob.kconst, prob.scale)
    P = rr.build_precond(kop, [mu], l=prob.l, sketch="srht", seed=prob.omega_seed, prec="fp32")
    assert np.array_equal(P.omega(), orng.srht_omega(prob.omega_seed, prob.n, prob.l))
    x, info = P.solve(_cuda(prob.b), tol=prob.tol)
    x = x.cpu().numpy()
    assert info["rc"] == rr.RR_OK and info["relres_work"] <= prob.tol
    rel64 = osol.relres(op.shifted(mu), x, prob.b)
    # float64 refinement is on by default for a float32 working operator: the final
    # true residual is the float64 one and meets tol
    assert abs(info["relres_fp64"] - rel64) <= 1e-6 * rel64 + 1e-14
    assert rel64 <= prob.tol
    # oracle run of the same algorithm in float64: comparable iteration count
    Pr = orr.build(op, [mu], prob.l, "srht", prob.omega_seed)[0]
    ref = osol.pcg(op.shifted(mu), Pr.apply, prob.b, prob.tol)
    assert abs(info["iters"] - ref.iters) <= max(3, int(0.1 * ref.iters))
    # the tau estimates (float32 entries and sums) agree with the float64 oracle
    # to a few digits
    g = P.export(0, with_q=False)
    for key in ("normE", "lam", "tau"):
        assert abs(g[key] - getattr(Pr, key)) < 1e-3 * getattr(Pr, key), (key, g[key], getattr(Pr, key))
    cg = rr.build_precond(kop, [mu], l=0, prec="fp32").solve(_cuda(prob.b), tol=prob.tol)[1]
    assert cg["iters"] > info["iters"]


def test_joint_basis_multi_shift():
    prob = workloads.cfg_batched(n=1500, d=16, l=50, nrhs=2)
    op = Operator.from_problem(prob)
    kop = rr.kernel_operator(rr.OP_RBF, _cuda(prob.pts), prob.kconst, prob.scale)
    P = rr.build_precond(kop, prob.mus, l=prob.l, sketch="srht", seed=prob.omega_seed, prec="fp64")
    oracle = orr.build(op, prob.mus, prob.l, "srht", prob.omega_seed)
    for j in range(len(prob.mus)):
        g = P.export(j)
        o = oracle[j]
        assert np.linalg.norm(g["Q"] - o.Q) / np.linalg.norm(o.Q) < 1e-9
        assert np.linalg.norm(g["G"] - o.G) / np.linalg.norm(o.G) < 1e-8
        assert abs(g["tau"] - o.tau) < 1e-8 * o.tau
    mus_idx = [j for j in range(len(prob.mus)) for _ in range(prob.B.shape[1])]
    B = np.concatenate([prob.B] * len(prob.mus), axis=1)
    X, infos, st = P.solve_batch(_cuda(B), mus_idx, tol=1e-8)
    X = X.cpu().numpy()
    for c, j in enumerate(mus_idx):
        assert infos[c]["status"] == rr.RR_OK
        assert osol.relres(op.shifted(prob.mus[j]), X[:, c], B[:, c]) <= 1e-8


def test_edge_cases(dense_small):
    prob, op, kop, A = dense_small
    dop = rr.dense_operator(A)
    P = rr.build_precond(dop, prob.mus, l=prob.l, seed=prob.omega_seed)
    # b = 0 -> x = 0
    x, info = P.solve(torch.zeros(prob.n, dtype=torch.float64, device="cuda"))
    assert info["rc"] == rr.RR_OK and float(x.abs().max()) == 0.0
    # NaN in b -> EINVAL before any arithmetic
    bn = _cuda(prob.b).clone()
    bn[5] = float("nan")
    with pytest.raises(rr.RRError) as e:
        P.solve(bn)
    assert e.value.status == rr.RR_EINVAL
    # maxit -> ENOCONV with a usable iterate, then resume from it
    x1, i1 = P.solve(_cuda(prob.b), tol=1e-12, maxit=3, ok=(rr.RR_ENOCONV,))
    assert i1["iters"] == 3 and i1["relres_work"] < 1.0
    x2, i2 = P.solve(_cuda(prob.b), x0=x1, tol=1e-10)
    assert i2["rc"] == rr.RR_OK
    # l = n: one PCG iteration
    small = workloads.cfg_small_dense(n=64, d=8, l=64)
    As = rr.kernel_to_dense(rr.kernel_operator(rr.OP_RBF, _cuda(small.pts), small.kconst, 1.0))
    Pn = rr.build_precond(rr.dense_operator(As), [0.1], l=64, seed=3, tau_rule="nys")
    xn, inn = Pn.solve(_cuda(small.b), tol=1e-8)
    assert inn["iters"] == 1
    # n = 1
    A1 = torch.full((1, 1), 2.0, dtype=torch.float64, device="cuda")
    P1 = rr.build_precond(rr.dense_operator(A1), [0.5], l=1, seed=1)
    x1_, i1_ = P1.solve(torch.tensor([5.0], dtype=torch.float64, device="cuda"), tol=1e-12)
    assert abs(float(x1_[0]) - 2.0) < 1e-12


def test_indefinite_operator_fails_cleanly():
    n = 50
    A = -torch.eye(n, dtype=torch.float64, device="cuda")
    P0 = rr.build_precond(rr.dense_operator(A), [0.0], l=0)
    b = torch.ones(n, dtype=torch.float64, device="cuda")
    x, info = P0.solve(b, ok=(rr.RR_EBREAKDOWN,))
    assert info["rc"] == rr.RR_EBREAKDOWN
    with pytest.raises(rr.RRError) as e:
        rr.build_precond(rr.dense_operator(A), [0.0], l=5, seed=1)
    assert e.value.status in (rr.RR_ENOTSPD,)


def test_deterministic_rerun():
    prob = workloads.cfg_kernel_ridge(n=2500, d=16, l=64)
    kop = rr.kernel_operator(rr.OP_RBF, _cuda(prob.pts), prob.kconst, prob.scale)
    b = _cuda(prob.b)
    xs = []
    for _ in range(2):
        P = rr.build_precond(kop, prob.mus, l=prob.l, sketch="srht", seed=prob.omega_seed, prec="fp32")
        xs.append(P.solve(b, tol=1e-6)[0])
    assert torch.equal(xs[0], xs[1])


@pytest.mark.parametrize("n,l,sketch,prec,d", [
    (3001, 200, "gaussian", "fp32", 16), (1100, 600, "srht", "fp32", 16),
    (700, 37, "gaussian", "fp32", 16), (2600, 130, "srht", "fp32", 5),
    (1500, 513, "gaussian", "fp32", 20), (9000, 64, "srht", "fp32", 16),
    (1100, 600, "srht", "fp64", 16), (257, 70, "gaussian", "fp64", 16)])
def test_kernel_sketch_matches_oracle(n, l, sketch, prec, d):
    # the sketch step alone (Y = A Omega + mu Omega) against the float64 oracle with the
    # same test matrix; float32 mode: bf16 hi/lo split entries -> |dY| <= 2^-15 |A||Omega|.
    # Sizes cover ragged row and column tiles, two column tiles (l > 512), padded
    # point records (d = 5, 20) and split point ranges.
    prob = workloads.cfg_kernel_ridge(n=n, d=d, l=l)
    mu = prob.mus[0]
    op = Operator.from_problem(prob)
    kop = rr.kernel_operator(rr.OP_RBF, _cuda(prob.pts), prob.kconst, prob.scale)
    Y = rr.sketch(kop, mu, l, sketch=sketch, seed=prob.omega_seed, prec=prec).cpu().numpy()
    Om = orng.omega(sketch, prob.omega_seed, n, l, bf16=(prec != "fp64"))
    Yo = op.matmat(Om) + mu * Om
    bound = (np.abs(op.to_dense()) @ np.abs(Om)) * (2.0 ** -15 if prec != "fp64" else 1e-13)
    err = np.abs(Y - Yo)
    worst = np.unravel_index(np.argmax(err / (bound + 1e-300)), err.shape)
    assert np.all(err <= bound + 1e-300), f"worst at {worst}: err {err[worst]:.3e} bound {bound[worst]:.3e}"


@pytest.mark.parametrize("n,l,sketch,d", [(2600, 130, "srht", 5), (1500, 513, "gaussian", 20),
                                          (3001, 64, "gaussian", 16)])
def test_kernel_sketch_matern_matches_oracle(n, l, sketch, d):
    # Matern-3/2 tiles from the augmented records: s from the record product, then
    # (1 + t) exp(-t) with t = kconst sqrt(-2 s); float32 mode, against the oracle
    prob = workloads.cfg_kernel_ridge(n=n, d=d, l=l)
    mu, kconst = prob.mus[0], 0.7
    op = Operator(kind=rr.OP_MATERN32, pts=prob.pts, kconst=kconst, scale=prob.scale)
    kop = rr.kernel_operator(rr.OP_MATERN32, _cuda(prob.pts), kconst, prob.scale)
    Y = rr.sketch(kop, mu, l, sketch=sketch, seed=prob.omega_seed, prec="fp32").cpu().numpy()
    Om = orng.omega(sketch, prob.omega_seed, n, l, bf16=True)
    Yo = op.matmat(Om) + mu * Om
    # the hi/lo split bounds each entry by 2^-15 relative; the Matern entry adds the
    # float32 rounding of its square root and exponential (a few 2^-24)
    bound = (np.abs(op.to_dense()) @ np.abs(Om)) * 2.0 ** -15
    err = np.abs(Y - Yo)
    assert np.all(err <= bound + 1e-300), np.max(err / (bound + 1e-300))


@pytest.mark.parametrize("n,l,sketch", [(3001, 200, "gaussian"), (4000, 520, "srht"), (700, 37, "gaussian")])
def test_kernel_fp32_bf16_sketch_basis(n, l, sketch):
    # float32-mode kernel build: Omega drawn in bf16, sketch on bf16 MFMA with a hi/lo
    # split kernel tile (checked elementwise above).  The device orthogonalisation must
    # be backward stable on its own sketch: Q^T Q = I and Q R = Y to float64 accuracy.
    prob = workloads.cfg_kernel_ridge(n=n, d=16, l=l)
    mu = prob.mus[0]
    op = Operator.from_problem(prob)
    kop = rr.kernel_operator(rr.OP_RBF, _cuda(prob.pts), prob.kconst, prob.scale)
    P = rr.build_precond(kop, [mu], l=l, sketch=sketch, seed=prob.omega_seed, prec="fp32")
    Om = orng.omega(sketch, prob.omega_seed, n, l, bf16=True)
    assert np.array_equal(P.omega(), Om)
    g = P.export(0)
    Y = rr.sketch(kop, mu, l, sketch=sketch, seed=prob.omega_seed, prec="fp32").cpu().numpy()
    Qg = g["Q"]
    assert np.linalg.norm(Qg.T @ Qg - np.eye(l), 2) < 1e-12
    assert np.linalg.norm(Qg @ g["R"] - Y) <= 1e-12 * np.linalg.norm(Y)
    o = orr.build(op, [mu], l, sketch, prob.omega_seed, omega_bf16=True)[0]
    x, info = P.solve(_cuda(prob.b), tol=1e-6)
    assert info["rc"] == rr.RR_OK
    ref = osol.pcg(op.shifted(mu), o.apply, prob.b, 1e-6)
    assert abs(info["iters"] - ref.iters) <= max(3, int(0.1 * ref.iters))


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_batched_multi_shift_matches_single_and_oracle(prec):
    # every RHS under every shift (joint basis), one fused batched solve, compared with
    # the single-column solve of the same column and with the float64 oracle
    prob = workloads.cfg_batched(n=2500, d=16, l=60, nrhs=3)
    op = Operator.from_problem(prob)
    kop = rr.kernel_operator(rr.OP_RBF, _cuda(prob.pts), prob.kconst, prob.scale)
    P = rr.build_precond(kop, prob.mus, l=prob.l, sketch="srht", seed=prob.omega_seed, prec=prec)
    k = prob.B.shape[1]
    mus_idx = [j for j in range(len(prob.mus)) for _ in range(k)]
    B = np.concatenate([prob.B] * len(prob.mus), axis=1)
    tol = 1e-6
    X, infos, st = P.solve_batch(_cuda(B), mus_idx, tol=tol, check_every=4)
    X = X.cpu().numpy()
    assert st == rr.RR_OK
    for c, j in enumerate(mus_idx):
        mu = prob.mus[j]
        assert infos[c]["status"] == rr.RR_OK
        rel64 = osol.relres(op.shifted(mu), X[:, c], B[:, c])
        assert abs(infos[c]["relres_fp64"] - rel64) <= 1e-6 * rel64 + 1e-14
        x1, i1 = P.solve(_cuda(B[:, c]), mu_index=j, tol=tol)
        # rounding order differs (GEMM vs GEMV projections): counts within max(3, 3%)
        assert abs(i1["iters"] - infos[c]["iters"]) <= max(3, int(0.03 * infos[c]["iters"]))
        if prec == "fp64":
            assert rel64 <= tol * 1.0001
        else:
            dA = prob.n * 2.0 ** -23 * prob.scale
            assert rel64 <= tol + dA * np.linalg.norm(X[:, c]) / np.linalg.norm(B[:, c])
        xs = x1.cpu().numpy()
        assert np.linalg.norm(xs - X[:, c]) <= np.linalg.norm(xs) * 1e-3 + 1e-12
    # the same column alone in a batch of one and inside the full batch
    X1, inf1, _ = P.solve_batch(_cuda(B[:, 5:6]), [mus_idx[5]], tol=tol, check_every=4)
    assert inf1[0]["iters"] == infos[5]["iters"]
    assert np.allclose(X1.cpu().numpy()[:, 0], X[:, 5], rtol=0, atol=1e-9 * np.abs(X[:, 5]).max())


def test_batched_graph_replay_and_wide_block():
    # 40 columns take the float64-MFMA kernel product, 5 columns the symmetric
    # few-column matvec; graph replay of the iteration batches must equal eager
    prob = workloads.cfg_batched(n=3000, d=16, l=60, nrhs=40)
    op = Operator.from_problem(prob)
    mu = prob.mus[1]
    kop = rr.kernel_operator(rr.OP_RBF, _cuda(prob.pts), prob.kconst, prob.scale)
    P = rr.build_precond(kop, [mu], l=prob.l, sketch="srht", seed=prob.omega_seed, prec="fp32")
    B = prob.B
    tol = 1e-6
    Xe, ie, st = P.solve_batch(_cuda(B), [0] * 40, tol=tol, check_every=4)
    Xg, ig, sg = P.solve_batch(_cuda(B), [0] * 40, tol=tol, check_every=4, use_graph=True)
    assert st == rr.RR_OK and sg == rr.RR_OK
    assert torch.equal(Xe, Xg)
    assert [i["iters"] for i in ie] == [i["iters"] for i in ig]
    Xe = Xe.cpu().numpy()
    dA = prob.n * 2.0 ** -23 * prob.scale
    for c in range(40):
        rel64 = osol.relres(op.shifted(mu), Xe[:, c], B[:, c])
        assert rel64 <= tol + dA * np.linalg.norm(Xe[:, c]) / np.linalg.norm(B[:, c])
    X5, i5, s5 = P.solve_batch(_cuda(B[:, :5].copy()), [0] * 5, tol=tol, check_every=4)
    assert s5 == rr.RR_OK
    X5 = X5.cpu().numpy()
    for c in range(5):
        assert abs(i5[c]["iters"] - ie[c]["iters"]) <= 2
        assert np.linalg.norm(X5[:, c] - Xe[:, c]) <= 1e-3 * np.linalg.norm(Xe[:, c])
    # 13 columns under one shift: the projection runs in column groups 8 + 4 + 1
    # (streaming passes over the basis instead of GEMMs); eager and graph agree
    B13 = _cuda(B[:, 7:20].copy())
    X13, i13, s13 = P.solve_batch(B13, [0] * 13, tol=tol, check_every=4)
    X13g, i13g, s13g = P.solve_batch(B13, [0] * 13, tol=tol, check_every=4, use_graph=True)
    assert s13 == rr.RR_OK and s13g == rr.RR_OK
    assert torch.equal(X13, X13g)
    X13 = X13.cpu().numpy()
    for c in range(13):
        assert i13[c]["status"] == rr.RR_OK
        assert abs(i13[c]["iters"] - ie[7 + c]["iters"]) <= 2
        assert np.linalg.norm(X13[:, c] - Xe[:, 7 + c]) <= 1e-3 * np.linalg.norm(Xe[:, 7 + c])
        rel64 = osol.relres(op.shifted(mu), X13[:, c], B[:, 7 + c])
        assert rel64 <= tol + dA * np.linalg.norm(X13[:, c]) / np.linalg.norm(B[:, 7 + c])


def test_batched_full_size_in_the_bench_configuration():
    """The batched workload at its full size (kernel ridge n = 50,000, 256 right-hand
    sides x 4 shifts on one joint SRHT basis, tol 1e-6, the bench's call): every column
    converges with float64 relres <= tol; on 12 sampled columns the device float64
    residual agrees on 32 sampled rows with the oracle's kernel formula, and its norm
    over the whole column with the library's relres."""
    from oracle.operators import kernel_block
    prob = workloads.cfg_batched()
    n, k = prob.n, prob.B.shape[1]
    kop = rr.kernel_operator(rr.OP_RBF, _cuda(prob.pts), prob.kconst, prob.scale)
    mus_idx = [j for j in range(len(prob.mus)) for _ in range(k)]
    Bh = np.concatenate([prob.B] * len(prob.mus), axis=1)
    P = rr.build_precond(kop, prob.mus, l=prob.l, sketch="srht", seed=prob.omega_seed, prec="fp32")
    X, infos, st = P.solve_batch(_cuda(Bh), mus_idx, tol=prob.tol, certify=False, check_every=4)
    assert st == rr.RR_OK
    assert all(i["status"] == rr.RR_OK and i["relres_fp64"] <= prob.tol for i in infos)
    rng = np.random.default_rng(21)
    cols = np.sort(rng.choice(Bh.shape[1], 12, replace=False))
    rows = np.sort(rng.choice(n, 32, replace=False))
    Xp = prob.pts.T.astype(np.float64)
    Kr = prob.scale * kernel_block(rr.OP_RBF, prob.kconst, Xp[rows], Xp)
    Xc = X[:, cols.tolist()].contiguous()
    Xh = Xc.cpu().numpy()
    for q, c in enumerate(cols):
        mu = prob.mus[mus_idx[c]]
        r = (_cuda(Bh[:, c].copy()) - rr.apply_operator(kop, mu, "fp64", Xc[:, q].contiguous())).cpu().numpy()
        r_or = Bh[rows, c] - Kr @ Xh[:, q] - mu * Xh[rows, q]
        scale = np.abs(Kr) @ np.abs(Xh[:, q]) + mu * np.abs(Xh[rows, q]) + np.abs(Bh[rows, c])
        assert np.all(np.abs(r_or - r[rows]) <= 1e-13 * scale), (c, np.max(np.abs(r_or - r[rows]) / scale))
        rel = np.linalg.norm(r) / np.linalg.norm(Bh[:, c])
        assert abs(rel - infos[c]["relres_fp64"]) <= 1e-6 * rel + 1e-14, (c, rel, infos[c]["relres_fp64"])


def test_batched_dense_operator():
    prob = workloads.cfg_small_dense(n=900, d=8, l=30)
    kop = rr.kernel_operator(rr.OP_RBF, _cuda(prob.pts), prob.kconst, 1.0)
    A = rr.kernel_to_dense(kop, "fp64")
    op = Operator.from_problem(prob)
    mus = [1e-2, 1e-3]
    P = rr.build_precond(rr.dense_operator(A), mus, l=30, seed=3)
    B = np.random.default_rng(7).standard_normal((prob.n, 4))
    X, infos, st = P.solve_batch(_cuda(B), [0, 1, 0, 1], tol=1e-9)
    X = X.cpu().numpy()
    assert st == rr.RR_OK
    for c in range(4):
        assert osol.relres(op.shifted(mus[c % 2]), X[:, c], B[:, c]) <= 1e-9 * 1.0001


@pytest.fixture(scope="module")
def precision_small():
    prob = workloads.cfg_precision(n=3001, l=130)
    op = Operator.from_problem(prob)
    kop = rr.kernel_operator(rr.OP_MATERN32, _cuda(prob.pts), prob.kconst, 1.0)
    A = rr.kernel_to_dense(kop, "fp64")
    return prob, op, A


def test_dense_mixed_sketch_matches_oracle(precision_small):
    # bf16 A and bf16 Omega on MFMA, float32 accumulation: |dY| <= 2^-8 |A| |Omega| + 2^-20 |A||Omega|
    prob, op, A = precision_small
    mu, l, n = prob.mus[0], prob.l, prob.n
    Y = rr.sketch(rr.dense_operator(A), mu, l, sketch="gaussian", seed=prob.omega_seed,
                  prec="mixed").cpu().numpy()
    Om = orng.omega("gaussian", prob.omega_seed, n, l, bf16=True)
    Yo = op.dense @ Om + mu * Om
    bound = (np.abs(op.dense) @ np.abs(Om)) * 2.0 ** -8
    assert np.all(np.abs(Y - Yo) <= bound)


def test_dense_mixed_solve_with_fp64_refinement(precision_small):
    # float32 matvec inside PCG, float64 residual at every restart: the float64 relative
    # residual reaches 1e-10 (outer iterative refinement)
    prob, op, A = precision_small
    mu, tol = prob.mus[0], 1e-10
    P = rr.build_precond(rr.dense_operator(A), [mu], l=prob.l, sketch="gaussian",
                         seed=prob.omega_seed, prec="mixed")
    x, info = P.solve(_cuda(prob.b), tol=tol)
    assert info["rc"] == rr.RR_OK
    x = x.cpu().numpy()
    rel = osol.relres(op.shifted(mu), x, prob.b)
    assert rel <= tol * 1.0001
    assert abs(info["relres_fp64"] - rel) <= 1e-3 * rel
    xs = osol.direct(op.dense, mu, prob.b)
    cond = np.linalg.cond(op.dense + mu * np.eye(prob.n))
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= 10 * tol * cond
    # plain CG with the same refinement needs more iterations
    i0 = rr.build_precond(rr.dense_operator(A), [mu], l=0, prec="mixed").solve(
        _cuda(prob.b), tol=tol, maxit=20000)[1]
    assert i0["rc"] == rr.RR_OK and i0["iters"] > info["iters"]


def _serving_requests(count, seed, spacing=0.004, n_range=(600, 3000)):
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(count):
        n = int(rng.integers(*n_range))
        d = int(rng.choice([4, 8, 16]))
        pts = rng.standard_normal((d, n)).astype(np.float32)
        bw = workloads.median_pairwise_distance(pts, 500)
        m = int(rng.integers(1, 4))
        reqs.append(dict(kind=rr.OP_RBF, pts=pts, kconst=float(np.float32(1 / (2 * bw * bw))),
                         scale=1.0 / n, mu=float(10 ** rng.uniform(-5, -2)), l=int(np.ceil(n / 32)),
                         seed=100 + i, B=rng.standard_normal((n, m)), t_arrival=i * spacing))
    return reqs


def test_serving_alone_equals_mixed_and_oracle():
    from paper_2509_19747_amd import binding as rb
    reqs = _serving_requests(10, 3)
    kw = dict(build=dict(prec="fp32", sketch="gaussian"), solve=dict(tol=1e-6, certify=True))
    mixed, stats = rb.serve(reqs, max_slots=4, graph_iters=8, **kw)
    assert stats["status"] == rr.RR_OK, stats.get("first_error")
    assert stats["served"] == len(reqs) and stats["rejected"] == 0
    assert stats["ok"] == len(reqs) and stats["failed"] == 0
    # every request's PCG batches ran as replayed graphs (no invalidated capture)
    assert stats["graph_fallbacks"] == 0
    assert stats["max_active"] >= 2
    assert 0 < stats["p50_ms"] <= stats["p99_ms"]
    for i, r in enumerate(reqs):
        alone, st1 = rb.serve([dict(r, t_arrival=0.0)], max_slots=1, graph_iters=8, **kw)
        assert mixed[i]["info"]["status"] == rr.RR_OK, stats.get("first_error")
        assert mixed[i]["info"]["graph_fallbacks"] == 0
        assert alone[0]["info"]["status"] == rr.RR_OK
        assert st1["graph_fallbacks"] == 0
        assert np.array_equal(alone[0]["X"], mixed[i]["X"])      # bitwise: batch-invariant
        op = Operator(kind=rr.OP_RBF, pts=r["pts"], kconst=r["kconst"], scale=r["scale"])
        for j in range(r["B"].shape[1]):
            rel = osol.relres(op.shifted(r["mu"]), mixed[i]["X"][:, j], r["B"][:, j])
            n = r["pts"].shape[1]
            dA = n * 2.0 ** -23 * r["scale"]
            assert rel <= 1e-6 + dA * np.linalg.norm(mixed[i]["X"][:, j]) / np.linalg.norm(r["B"][:, j])


def test_serving_stream_at_the_workload_sizes():
    """The first 24 requests of the serving workload's own stream (n log-uniform up to
    32,768, l = n/32, 1-8 right-hand sides, the bench's server settings): every request
    OK with no graph fallback, each column's float64 relres <= tol, and for the three
    largest requests the residual on 24 sampled rows of every column against the
    oracle's kernel formula."""
    from oracle.operators import kernel_block
    from paper_2509_19747_amd import binding as rb
    stream = workloads.serving_stream(num=24, rate=200.0)
    reqs = []
    for r in stream:
        p = r.problem
        reqs.append(dict(kind=p.kind, pts=p.pts, kconst=p.kconst, scale=p.scale, mu=p.mus[0], l=p.l,
                         seed=p.omega_seed, B=p.B, t_arrival=r.t_arrival))
    kw = dict(build=dict(prec="fp32", sketch="gaussian"), solve=dict(tol=1e-6, certify=False))
    res, stats = rb.serve(reqs, hbm_budget=96 << 30, max_slots=16, graph_iters=8, **kw)
    assert stats["status"] == rr.RR_OK, stats.get("first_error")
    assert stats["ok"] == len(reqs) and stats["failed"] == 0 and stats["graph_fallbacks"] == 0
    for q, r in zip(res, reqs):
        assert q["info"]["status"] == rr.RR_OK and q["info"]["relres_fp64"] <= 1e-6
    rng = np.random.default_rng(9)
    for i in np.argsort([r["pts"].shape[1] for r in reqs])[-3:]:
        r, X = reqs[i], res[i]["X"]
        n = r["pts"].shape[1]
        Xp = r["pts"].T.astype(np.float64)
        rows = np.sort(rng.choice(n, 24, replace=False))
        Kr = r["scale"] * kernel_block(rr.OP_RBF, r["kconst"], Xp[rows], Xp)
        op = Operator(kind=rr.OP_RBF, pts=r["pts"], kconst=r["kconst"], scale=r["scale"])
        for j in range(r["B"].shape[1]):
            x = X[:, j]
            r_or = r["B"][rows, j] - Kr @ x - r["mu"] * x[rows]
            assert np.linalg.norm(r_or) <= 1e-6 * np.linalg.norm(r["B"][:, j]) * 1.01
        rel = osol.relres(op.shifted(r["mu"]), X[:, 0], r["B"][:, 0])
        assert rel <= 1e-6 * 1.0001, (i, n, rel)


def test_serving_grouped_equals_per_request_graphs():
    """Grouped serving (the PCG batches of all waiting requests in one replay of
    persistent kernels over the device work list) gives bitwise the results of
    per-request graphs, alone and in the mix, and meets tol against the oracle.  The
    mix covers both kernels, record lengths 4/8/16, an odd and a wide right-hand-side
    block (padded pair, projection groups of width 4, 2 and 1) and a product with
    several column blocks per work item."""
    from paper_2509_19747_amd import binding as rb
    reqs = _serving_requests(6, 21, n_range=(700, 2600))
    rng = np.random.default_rng(77)
    reqs[1]["kind"] = rr.OP_MATERN32
    reqs[1]["kconst"] = float(np.float32(np.sqrt(3.0) / workloads.median_pairwise_distance(reqs[1]["pts"], 500)))
    reqs[2]["B"] = rng.standard_normal((reqs[2]["pts"].shape[1], 7))
    n = 9000
    pts = rng.standard_normal((8, n)).astype(np.float32)
    bw = workloads.median_pairwise_distance(pts, 500)
    reqs.append(dict(kind=rr.OP_RBF, pts=pts, kconst=float(np.float32(1 / (2 * bw * bw))), scale=1.0 / n,
                     mu=1e-4, l=int(np.ceil(n / 32)), seed=901, B=rng.standard_normal((n, 5)),
                     t_arrival=reqs[-1]["t_arrival"] + 0.004))
    kw = dict(build=dict(prec="fp32", sketch="gaussian"), solve=dict(tol=1e-6, certify=True))
    grouped, sg = rb.serve(reqs, max_slots=4, graph_iters=8, grouped=1, **kw)
    assert sg["status"] == rr.RR_OK, sg.get("first_error")
    assert sg["ok"] == len(reqs) and sg["group_replays"] > 0 and sg["group_max"] >= 2
    lanes2, s2 = rb.serve(reqs, max_slots=4, graph_iters=8, grouped=2, **kw)
    assert s2["status"] == rr.RR_OK and s2["group_replays"] > 0
    single, ss = rb.serve(reqs, max_slots=4, graph_iters=8, grouped=0, **kw)
    assert ss["status"] == rr.RR_OK and ss["group_replays"] == 0
    for i, r in enumerate(reqs):
        g, p = grouped[i], single[i]
        assert g["info"]["status"] == rr.RR_OK and p["info"]["status"] == rr.RR_OK
        assert g["info"]["iters"] == p["info"]["iters"]
        assert np.array_equal(g["X"], p["X"]), i
        assert np.array_equal(lanes2[i]["X"], p["X"]), i
        alone, sa = rb.serve([dict(r, t_arrival=0.0)], max_slots=1, graph_iters=8, grouped=1, **kw)
        assert sa["group_max"] == 1
        assert np.array_equal(alone[0]["X"], g["X"]), i
        op = Operator(kind=r["kind"], pts=r["pts"], kconst=r["kconst"], scale=r["scale"])
        n = r["pts"].shape[1]
        for j in range(r["B"].shape[1]):
            rel = osol.relres(op.shifted(r["mu"]), g["X"][:, j], r["B"][:, j])
            dA = n * 2.0 ** -23 * r["scale"]
            assert rel <= 1e-6 + dA * np.linalg.norm(g["X"][:, j]) / np.linalg.norm(r["B"][:, j])


def test_serving_grouped_rejects_bad_config():
    from paper_2509_19747_amd import binding as rb
    reqs = _serving_requests(1, 3)
    with pytest.raises(rb.RRError):
        rb.serve(reqs, graph_iters=0, grouped=1)
    with pytest.raises(rb.RRError):
        rb.serve(reqs, graph_iters=8, grouped=9)


def test_serving_rejects_over_budget():
    from paper_2509_19747_amd import binding as rb
    reqs = _serving_requests(3, 5)
    res, stats = rb.serve(reqs, hbm_budget=1 << 20, max_slots=2)
    assert stats["rejected"] == 3 and stats["served"] == 0 and stats["ok"] == 0
    assert all(r["info"]["status"] == rr.RR_ENOMEM for r in res)


def test_serving_with_torch_allocator():
    """rr_serve_config.alloc: every request buffer and handle allocation goes through
    the caller's allocator (PyTorch's caching allocator here); results equal the
    library-pool run bitwise."""
    from paper_2509_19747_amd import binding as rb
    reqs = _serving_requests(4, 9)
    kw = dict(build=dict(prec="fp32", sketch="gaussian"), solve=dict(tol=1e-6, certify=False))
    ta = rb.TorchAllocator()
    a, sa = rb.serve(reqs, max_slots=2, graph_iters=8, allocator=ta, **kw)
    p, sp = rb.serve(reqs, max_slots=2, graph_iters=8, **kw)
    assert sa["status"] == rr.RR_OK and sa["ok"] == len(reqs) and sa["graph_fallbacks"] == 0
    assert not ta.live   # every block handed out was given back
    for x, y in zip(a, p):
        assert np.array_equal(x["X"], y["X"])


def test_concurrent_solves_on_one_handle():
    """Solves on one handle from several threads and streams at once use their own
    workspaces and give the same result as a solve alone."""
    import threading
    prob = workloads.cfg_small_dense(n=900, d=8, l=40)
    kop = rr.kernel_operator(rr.OP_RBF, _cuda(prob.pts), prob.kconst, prob.scale)
    P = rr.build_precond(rr.dense_operator(rr.kernel_to_dense(kop, "fp64")), prob.mus, l=prob.l,
                         seed=prob.omega_seed)
    b = _cuda(prob.b)
    x0, i0 = P.solve(b, tol=1e-10)
    torch.cuda.synchronize()
    out = [None] * 4
    def run(k):
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            x, info = P.solve(b, tol=1e-10, stream=s, use_graph=(k % 2 == 1))
            s.synchronize()
            out[k] = (x, info)
    ts = [threading.Thread(target=run, args=(k,)) for k in range(4)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    for x, info in out:
        assert info["rc"] == rr.RR_OK and info["iters"] == i0["iters"]
        assert torch.equal(x, x0)


# ------------------------------------------------- R-RandRAND, split, MINRES
from oracle import variants as ovar  # noqa: E402


def _oracle_variant(op, prob, mu, method, krylov, tol, P_or=None, Omega=None, omega_bf16=False,
                    sketch="gaussian"):
    Pr = P_or or orr.build(op, [mu], prob.l, sketch, prob.omega_seed, omega_bf16=omega_bf16)[0]
    amu = op.shifted(mu)
    if method == "c":
        return ovar.c_randrand_minres(amu, Pr.apply, prob.b, tol), Pr
    Om = Omega if Omega is not None else orng.omega(sketch, prob.omega_seed, prob.n, prob.l, bf16=omega_bf16)
    proj = ovar.Projections(Pr.Q, Pr.T, Pr.R, Om)
    if method == "r":
        return ovar.r_randrand(amu, proj, Pr.normE, prob.b, tol, krylov=krylov), Pr
    return ovar.split_r_randrand(amu, proj, prob.b, tol, krylov=krylov), Pr


@pytest.mark.parametrize("method,krylov", [("c", "minres"), ("r", "cg"), ("r", "minres"),
                                           ("split", "cg"), ("split", "minres")])
def test_variant_solvers_fp64_match_oracle(dense_small, method, krylov):
    """Algorithms RandRAND_CG, RandRAND_CG_split and the MINRES branch of RandRAND_PCG
    in float64 against the oracle: relres within 1e-8 of the oracle's (both <= tol),
    iteration counts within max(2, 3 %), the first 20 per-iteration residuals entry by
    entry, and the forward error against the direct solve."""
    prob, op, kop, A = dense_small
    mu, tol = prob.mus[0], 1e-10
    P = rr.build_precond(rr.dense_operator(A), [mu], l=prob.l, seed=prob.omega_seed)
    h = np.full(600, np.nan)
    x, info = P.solve(_cuda(prob.b), tol=tol, method=method, krylov=krylov, history=h)
    x = x.cpu().numpy()
    ref, _ = _oracle_variant(op, prob, mu, method, krylov, tol)
    assert ref.status == osol.OK
    rel = osol.relres(op.shifted(mu), x, prob.b)
    assert info["rc"] == rr.RR_OK and rel <= tol * 1.0001 and rel <= ref.relres + 1e-8
    assert abs(info["iters"] - ref.iters) <= max(2, int(0.03 * ref.iters)), (info["iters"], ref.iters)
    k = min(info["iters"], ref.iters, 20)
    np.testing.assert_allclose(h[: k + 1], np.array(ref.history)[: k + 1], rtol=1e-6, atol=0)
    xs = osol.direct(op.dense, mu, prob.b)
    cond = np.linalg.cond(op.dense + mu * np.eye(prob.n))
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= 10 * tol * cond


def test_variant_solver_graph_equals_eager(dense_small):
    prob, op, kop, A = dense_small
    P = rr.build_precond(rr.dense_operator(A), prob.mus, l=prob.l, seed=prob.omega_seed)
    b = _cuda(prob.b)
    for method, krylov in (("r", "minres"), ("split", "cg"), ("c", "minres")):
        x1, i1 = P.solve(b, tol=1e-9, method=method, krylov=krylov, use_graph=False, check_every=4)
        x2, i2 = P.solve(b, tol=1e-9, method=method, krylov=krylov, use_graph=True, check_every=4)
        assert torch.equal(x1, x2) and i1["iters"] == i2["iters"] and i2["graph_fallbacks"] == 0


@pytest.mark.parametrize("method,krylov", [("c", "minres"), ("r", "cg"), ("split", "minres")])
def test_variant_solvers_kernel_fp32_with_refinement(method, krylov):
    """Float32-class kernel operator with float64 refinement: every variant reaches
    float64 relres <= tol against the oracle operator; iteration counts near the
    oracle's float64 run of the same algorithm (the R recovery uses the bf16-sketch
    basis, so its counts may exceed the float64 ones by a few cycles)."""
    prob = workloads.cfg_kernel_ridge(n=4000, d=16, l=120)
    mu = prob.mus[0]
    op = Operator.from_problem(prob)
    kop = rr.kernel_operator(rr.OP_RBF, _cuda(prob.pts), prob.kconst, prob.scale)
    P = rr.build_precond(kop, [mu], l=prob.l, sketch="srht", seed=prob.omega_seed, prec="fp32")
    x, info = P.solve(_cuda(prob.b), tol=prob.tol, method=method, krylov=krylov, maxit=5000)
    x = x.cpu().numpy()
    rel = osol.relres(op.shifted(mu), x, prob.b)
    assert info["rc"] == rr.RR_OK and rel <= prob.tol * 1.0001
    assert abs(info["relres_fp64"] - rel) <= 1e-6 * rel + 1e-14
    ref, _ = _oracle_variant(op, prob, mu, method, krylov, prob.tol, omega_bf16=True, sketch="srht")
    assert ref.status == osol.OK
    assert info["iters"] <= 1.5 * ref.iters + 5 and info["iters"] >= 0.5 * ref.iters, (info["iters"], ref.iters)


def test_variant_solver_rejects_joint_basis_and_nys(dense_small):
    prob, op, kop, A = dense_small
    Pj = rr.build_precond(rr.dense_operator(A), [1e-2, 1e-3], l=20, seed=1)
    with pytest.raises(rr.RRError):
        Pj.solve(_cuda(prob.b), method="r")
    Pn = rr.build_precond(rr.dense_operator(A), [1e-3], l=20, seed=1, tau_rule="nys")
    with pytest.raises(rr.RRError):
        Pn.solve(_cuda(prob.b), method="r")
    x, info = Pn.solve(_cuda(prob.b), method="split", tol=1e-8)
    assert info["rc"] == rr.RR_OK


# ---------------------------------------------- q = 1, shift sweeps, adaptive l
def test_q1_build_fp64_matches_oracle(dense_small):
    """Omega = A X (eq. testmatrix, q = 1) in float64 against the oracle: Q, R, G, tau."""
    prob, op, kop, A = dense_small
    mu, l = prob.mus[0], prob.l
    P = rr.build_precond(rr.dense_operator(A), [mu], l=l, sketch="gaussian", seed=prob.omega_seed, q=1)
    g = P.export(0)
    o = orr.build(op, [mu], l, "gaussian", prob.omega_seed, q=1)[0]
    rel = lambda a, b_: np.linalg.norm(a - b_) / np.linalg.norm(b_)
    # A X entries are sums with cancellation: compare normwise (float64 product rounding)
    assert rel(P.omega(), orr.test_matrix(op, "gaussian", prob.omega_seed, l, q=1)) < 1e-13
    assert rel(g["Q"], o.Q) < 1e-9 and rel(g["R"], o.R) < 1e-9 and rel(g["G"], o.G) < 1e-8
    assert abs(g["tau"] - o.tau) < 1e-8 * o.tau
    x, info = P.solve(_cuda(prob.b), tol=1e-10)
    ref = osol.pcg(op.shifted(mu), o.apply, prob.b, 1e-10)
    assert info["rc"] == rr.RR_OK and abs(info["iters"] - ref.iters) <= max(2, int(0.03 * ref.iters))


def test_q1_kernel_fp32_solve():
    prob = workloads.cfg_kernel_ridge(n=4000, d=16, l=120)
    mu = prob.mus[0]
    op = Operator.from_problem(prob)
    kop = rr.kernel_operator(rr.OP_RBF, _cuda(prob.pts), prob.kconst, prob.scale)
    P0 = rr.build_precond(kop, [mu], l=prob.l, sketch="srht", seed=prob.omega_seed, prec="fp32")
    P1 = rr.build_precond(kop, [mu], l=prob.l, sketch="srht", seed=prob.omega_seed, prec="fp32", q=1)
    x, info = P1.solve(_cuda(prob.b), tol=prob.tol)
    rel = osol.relres(op.shifted(mu), x.cpu().numpy(), prob.b)
    assert info["rc"] == rr.RR_OK and rel <= prob.tol
    # the power iteration captures the dominant range at least as well here
    assert P1.export(0, with_q=False)["normE"] <= 1.05 * P0.export(0, with_q=False)["normE"]


def test_shifted_cholesky_sweep_matches_oracle():
    """Several shifts from one orthogonalisation at alpha = max mu (Section 5.1, shifted
    Cholesky) against the oracle: Q_mu, R, G, tau per shift; batched solves reach tol."""
    prob = workloads.cfg_small_dense(n=900, d=8, l=40)
    op = Operator.from_problem(prob)
    kop = rr.kernel_operator(rr.OP_RBF, _cuda(prob.pts), prob.kconst, prob.scale)
    A = rr.kernel_to_dense(kop, "fp64")
    mus = [1e-2, 1e-3, 1e-4]
    P = rr.build_precond(rr.dense_operator(A), mus, l=prob.l, seed=prob.omega_seed, multi="shifted_chol")
    o = orr.build(op, mus, prob.l, "gaussian", prob.omega_seed, multi="shifted_chol")
    rel = lambda a, b_: np.linalg.norm(a - b_) / np.linalg.norm(b_)
    for j in range(len(mus)):
        g = P.export(j)
        assert rel(g["Q"], o[j].Q) < 1e-8 and rel(g["R"], o[j].R) < 1e-8 and rel(g["G"], o[j].G) < 1e-7
        assert abs(g["tau"] - o[j].tau) < 1e-7 * o[j].tau
    B = np.stack([prob.b] * 3, axis=1)
    X, infos, st = P.solve_batch(_cuda(B), [0, 1, 2], tol=1e-9)
    for j, mu in enumerate(mus):
        r = osol.relres(op.shifted(mu), X[:, j].cpu().numpy(), prob.b)
        assert infos[j]["status"] == rr.RR_OK and r <= 1e-9 * 1.0001


def test_adaptive_sketch_size_matches_oracle(dense_small):
    """eq. ad_criterion: the device's doubling loop picks the oracle's l and ||E||."""
    prob, op, kop, A = dense_small
    mu = prob.mus[0]
    kw = dict(l=8, sketch="gaussian", seed=prob.omega_seed, l_max=256, ad_factor=3.0)
    P = rr.build_precond(rr.dense_operator(A), [mu], **kw)
    n, l, _ = P.shape
    Po, lo, trail = orr.build_adaptive(op, mu, 8, 256, f=3.0, seed=prob.omega_seed)
    assert l == lo and len(trail) >= 2
    assert abs(P.export(0, with_q=False)["normE"] - Po.normE) <= 1e-8 * Po.normE


# ---------------------------------------------------------------- basis-less
def test_colsample_omega_bit_exact():
    n, l = 1000, 37
    prob = workloads.cfg_small_dense(n=n, d=8, l=l)
    kop = rr.kernel_operator(rr.OP_RBF, _cuda(prob.pts), prob.kconst, prob.scale)
    P = rr.build_precond(kop, [1e-3], l=l, sketch="colsample", seed=99)
    assert np.array_equal(P.omega(), orng.colsample_omega(99, n, l))
    Pb = rr.build_precond(kop, [1e-3], l=l, sketch="colsample", seed=99, basis="less")
    assert np.array_equal(Pb.omega(), orng.colsample_omega(99, n, l))


@pytest.mark.parametrize("reorth", [False, True])
@pytest.mark.parametrize("orth", ["sketched", "cholqr"])
def test_basisless_fp64_matches_oracle(orth, reorth):
    """Algorithm BL_RandRAND_PCG in float64 against the oracle: R, T, G, tau and the
    implicit Q (formed on export), with Y streamed over several row blocks (n = 12,000,
    l = 200); PCG iterations and relres against the oracle's run."""
    prob = workloads.cfg_kernel_ridge(n=12_000, d=8, l=200)
    mu = prob.mus[0]
    op = Operator.from_problem(prob)
    kop = rr.kernel_operator(rr.OP_RBF, _cuda(prob.pts), prob.kconst, prob.scale)
    P = rr.build_precond(kop, [mu], l=prob.l, sketch="colsample", seed=prob.omega_seed, basis="less",
                         orth=orth, reorth=reorth, prec="fp64")
    g = P.export(0)
    o = orr.build_basisless(op, mu, prob.l, "colsample", prob.omega_seed, reorth=reorth)
    if orth == "cholqr":
        ex = orr.build(op, [mu], prob.l, "colsample", prob.omega_seed, orth=orr.CHOLQR, reorth=reorth)[0]
        o_R, o_G, o_T, o_tau, o_Q = ex.R, ex.G, ex.T, ex.tau, ex.Q
    else:
        o_R, o_G, o_T, o_tau, o_Q = o.R, o.G, o.T, o.tau, o.Q
    rel = lambda a, b_: np.linalg.norm(a - b_) / np.linalg.norm(b_)
    assert rel(g["R"], o_R) < 1e-9 and rel(g["G"], o_G) < 1e-8 and rel(g["Q"], o_Q) < 1e-9
    assert np.abs(g["T"] - o_T).max() < 1e-10
    assert abs(g["tau"] - o_tau) < 1e-8 * o_tau
    x, info = P.solve(_cuda(prob.b), tol=1e-9)
    Pref = o if orth == "sketched" else ex
    ref = osol.pcg(op.shifted(mu), Pref.apply, prob.b, 1e-9)
    rel64 = osol.relres(op.shifted(mu), x.cpu().numpy(), prob.b)
    assert info["rc"] == rr.RR_OK and rel64 <= 1e-9 * 1.0001 and rel64 <= ref.relres + 1e-8
    assert abs(info["iters"] - ref.iters) <= max(2, int(0.03 * ref.iters)), (info["iters"], ref.iters)


@pytest.mark.parametrize("kind,d,prec,n,l", [(rr.OP_MATERN32, 20, "fp64", 3000, 100),
                                             (rr.OP_RBF, 3, "fp64", 3000, 100),
                                             (rr.OP_RBF, 3, "fp32", 3000, 100),
                                             (rr.OP_MATERN32, 7, "fp32", 3000, 100),
                                             (rr.OP_RBF, 16, "fp64", 1001, 37)])
def test_basisless_record_lengths_and_kinds(kind, d, prec, n, l):
    """The basis-less kernel blocks at the record lengths 4, 8, 16 and 32 and for both
    kernels (n = 3,000, l = 100; and a ragged n = 1,001, l = 37, not a multiple of the
    four sampled rows per block nor of the 128-column chunks): in float64 the implicit
    Q, R and tau against the oracle's Algorithm BL_RandRAND_PCG; in both precisions the
    PCG result against the oracle operator and the explicit handle on the same column
    sample."""
    mu = 1e-3
    rng = np.random.default_rng(50 + d)
    pts = rng.standard_normal((d, n)).astype(np.float32)
    kconst, scale = (0.3 if kind == rr.OP_MATERN32 else 0.5 / d), 1.0 / n
    op = Operator(kind=kind, pts=pts, kconst=kconst, scale=scale)
    b = rng.standard_normal(n)
    kop = rr.kernel_operator(kind, _cuda(pts), kconst, scale)
    kw = dict(l=l, sketch="colsample", seed=7, prec=prec)
    Pb = rr.build_precond(kop, [mu], basis="less", **kw)
    Pe = rr.build_precond(kop, [mu], **kw)
    if prec == "fp64":
        g = Pb.export(0)
        o = orr.build_basisless(op, mu, l, "colsample", 7)
        rel = lambda a, b_: np.linalg.norm(a - b_) / np.linalg.norm(b_)
        assert rel(g["R"], o.R) < 1e-9 and rel(g["Q"], o.Q) < 1e-9
        assert abs(g["tau"] - o.tau) < 1e-8 * o.tau
    tol = 1e-8 if prec == "fp64" else 1e-6
    xb, ib = Pb.solve(_cuda(b), tol=tol)
    xe, ie = Pe.solve(_cuda(b), tol=tol)
    for x, info in ((xb, ib), (xe, ie)):
        assert info["rc"] == rr.RR_OK
        assert osol.relres(op.shifted(mu), x.cpu().numpy(), b) <= tol * 1.0001
    assert abs(ib["iters"] - ie["iters"]) <= max(3, int(0.15 * ie["iters"])), (ib["iters"], ie["iters"])


def test_basisless_fp32_kernel_ridge_solve():
    """Basis-less float32-class handle at n = 20,000, l = 500 (no n x l basis stored):
    float64 relres <= tol with refinement; C-RandRAND MINRES on it as well; iteration
    counts near the explicit-basis handle on the same column sample."""
    prob = workloads.cfg_kernel_ridge(n=20_000, d=16, l=500)
    mu = prob.mus[0]
    op = Operator.from_problem(prob)
    kop = rr.kernel_operator(rr.OP_RBF, _cuda(prob.pts), prob.kconst, prob.scale)
    kw = dict(l=prob.l, sketch="colsample", seed=prob.omega_seed, prec="fp32")
    Pb = rr.build_precond(kop, [mu], basis="less", **kw)
    Pe = rr.build_precond(kop, [mu], **kw)
    b = _cuda(prob.b)
    xb, ib = Pb.solve(b, tol=prob.tol)
    xe, ie = Pe.solve(b, tol=prob.tol)
    for x, info in ((xb, ib), (xe, ie)):
        assert info["rc"] == rr.RR_OK
        assert osol.relres(op.shifted(mu), x.cpu().numpy(), prob.b) <= prob.tol
    assert abs(ib["iters"] - ie["iters"]) <= max(3, int(0.15 * ie["iters"]))
    xm, im = Pb.solve(b, tol=prob.tol, krylov="minres")
    assert im["rc"] == rr.RR_OK and osol.relres(op.shifted(mu), xm.cpu().numpy(), prob.b) <= prob.tol
    with pytest.raises(rr.RRError):
        Pb.solve(b, method="r")
    with pytest.raises(rr.RRError):
        Pb.solve_batch(torch.stack([b, b], 1), [0, 0])


# ------------------------------------------------------------ block solvers
@pytest.mark.parametrize("method", ["minres", "cg"])
def test_block_solvers_match_oracle(method):
    """Block preconditioned MINRES / block CG in float64 against the oracle: six
    right-hand sides (one zero) under one shift, then eleven under two shifts of a
    joint-basis handle (groups per shift); solutions, block iterations and the
    per-column residuals."""
    prob = workloads.cfg_batched(n=2500, d=16, l=60, nrhs=11)
    op = Operator.from_problem(prob)
    kop = rr.kernel_operator(rr.OP_RBF, _cuda(prob.pts), prob.kconst, prob.scale)
    mus = prob.mus[1:3]
    P = rr.build_precond(kop, mus, l=prob.l, sketch="srht", seed=prob.omega_seed, prec="fp64")
    tol = 1e-9
    B = prob.B[:, :6].copy()
    B[:, 3] = 0.0
    X, infos, st = P.solve_batch(_cuda(B), [0] * 6, tol=tol, krylov="block_" + method)
    X = X.cpu().numpy()
    assert st == rr.RR_OK
    Po = orr.build(op, mus, prob.l, "srht", prob.omega_seed)
    ref = oblk.solve_block(op.shifted(mus[0]), Po[0].apply, B, tol, method=method)
    assert ref.status == osol.OK
    assert np.all(X[:, 3] == 0.0)
    for c in range(6):
        assert infos[c]["status"] == rr.RR_OK
        if c == 3:
            assert infos[c]["relres_work"] == 0.0
            continue
        rel64 = osol.relres(op.shifted(mus[0]), X[:, c], B[:, c])
        assert rel64 <= tol * 1.0001
        # two float64 evaluations of b - A x in different summation orders differ by
        # about n u (||A|| ||x|| / ||b|| + 1), ~1e-12 here
        assert abs(infos[c]["relres_fp64"] - rel64) <= 1e-12
        assert abs(infos[c]["iters"] - ref.iters[c]) <= 1, (infos[c]["iters"], ref.iters[c])
    xs = np.linalg.solve(op.to_dense() + mus[0] * np.eye(prob.n), B)
    assert np.linalg.norm(X - xs) <= 1e-6 * np.linalg.norm(xs)
    # two shifts, columns interleaved: each shift's columns form their own group
    idx = [j % 2 for j in range(11)]
    X2, inf2, st = P.solve_batch(_cuda(prob.B), idx, tol=tol, krylov="block_" + method)
    X2 = X2.cpu().numpy()
    assert st == rr.RR_OK
    for g in (0, 1):
        cols = [c for c in range(11) if idx[c] == g]
        rg = oblk.solve_block(op.shifted(mus[g]), Po[g].apply, prob.B[:, cols], tol, method=method)
        for k, c in enumerate(cols):
            assert inf2[c]["status"] == rr.RR_OK
            assert osol.relres(op.shifted(mus[g]), X2[:, c], prob.B[:, c]) <= tol * 1.0001
            # block CG to 1e-9 over ~60 steps: the rounding of the float64 entries moves
            # the last steps' residual across tol (counts within 2)
            assert abs(inf2[c]["iters"] - rg.iters[k]) <= 2
        assert len({inf2[c]["iters"] for c in cols}) == 1


def test_block_minres_groups_and_cycle_cap():
    """40 columns under one shift: groups of 32 and 8 (each group's columns share a
    count, the 8 alone give the same result), and a cycle cap of 3 block steps
    (restarts, still converging)."""
    prob = workloads.cfg_batched(n=3000, d=16, l=60, nrhs=40)
    op = Operator.from_problem(prob)
    mu = prob.mus[1]
    kop = rr.kernel_operator(rr.OP_RBF, _cuda(prob.pts), prob.kconst, prob.scale)
    P = rr.build_precond(kop, [mu], l=prob.l, sketch="srht", seed=prob.omega_seed, prec="fp64")
    tol = 1e-8
    X, infos, st = P.solve_batch(_cuda(prob.B), [0] * 40, tol=tol, krylov="block_minres")
    X = X.cpu().numpy()
    assert st == rr.RR_OK
    assert rr.BLOCK_MAX == 32
    assert len({i["iters"] for i in infos[:32]}) == 1 and len({i["iters"] for i in infos[32:]}) == 1
    X8, i8, _ = P.solve_batch(_cuda(prob.B[:, 32:]), [0] * 8, tol=tol, krylov="block_minres")
    assert np.array_equal(X8.cpu().numpy(), X[:, 32:])
    assert i8[0]["iters"] == infos[32]["iters"]
    for c in range(40):
        assert osol.relres(op.shifted(mu), X[:, c], prob.B[:, c]) <= tol * 1.0001
    Po = orr.build(op, [mu], prob.l, "srht", prob.omega_seed)[0]
    Xc, ic, st = P.solve_batch(_cuda(prob.B[:, :5]), [0] * 5, tol=tol, krylov="block_minres", block_kmax=3)
    assert st == rr.RR_OK and ic[0]["restarts"] >= 2
    ref = oblk.solve_block(op.shifted(mu), Po.apply, prob.B[:, :5], tol, kmax=3)
    assert ic[0]["iters"] == ref.iters[0] and ic[0]["restarts"] == ref.restarts[0]


def test_block_minres_fp32_ten_rhs():
    """Ten right-hand sides (the paper's block size for its 10-class problem) on a
    float32-class handle at n = 20,000: every column at tol in float64 (refinement),
    fewer block steps than the largest single-column PCG count."""
    prob = workloads.cfg_kernel_ridge(n=20_000, d=16, l=500)
    mu = prob.mus[0]
    op = Operator.from_problem(prob)
    kop = rr.kernel_operator(rr.OP_RBF, _cuda(prob.pts), prob.kconst, prob.scale)
    P = rr.build_precond(kop, [mu], l=prob.l, sketch="srht", seed=prob.omega_seed, prec="fp32")
    rng = np.random.default_rng(5)
    B = np.sign(rng.standard_normal((prob.n, 10)))
    for method in ("block_minres", "block_cg"):
        X, infos, st = P.solve_batch(_cuda(B), [0] * 10, tol=prob.tol, krylov=method)
        X = X.cpu().numpy()
        assert st == rr.RR_OK
        rows = np.random.default_rng(1).choice(prob.n, 64, replace=False)
        for c in range(10):
            assert infos[c]["relres_fp64"] <= prob.tol
        Xp, ip, _ = P.solve_batch(_cuda(B), [0] * 10, tol=prob.tol)
        assert infos[0]["iters"] <= max(i["iters"] for i in ip)
        # sampled rows of the float64 residual against the oracle's rows
        Kr = op.scale * orr_kernel_rows(op, rows)
        R = B[rows] - (Kr @ X + mu * X[rows])
        assert np.abs(R).max() <= 10 * prob.tol * np.abs(B).max() * np.sqrt(prob.n)


def orr_kernel_rows(op, rows):
    from oracle.operators import kernel_block
    return kernel_block(op.kind, op.kconst, op.X[rows], op.X)


def test_block_dependent_columns_and_guards():
    prob = workloads.cfg_batched(n=1500, d=8, l=40, nrhs=3)
    kop = rr.kernel_operator(rr.OP_RBF, _cuda(prob.pts), prob.kconst, prob.scale)
    P = rr.build_precond(kop, [prob.mus[1]], l=prob.l, sketch="srht", seed=prob.omega_seed, prec="fp64")
    B = prob.B.copy()
    B[:, 2] = 2.0 * B[:, 0]
    X, infos, st = P.solve_batch(_cuda(B), [0] * 3, tol=1e-8, krylov="block_minres",
                                 ok=(rr.RR_OK, rr.RR_EBREAKDOWN))
    assert st == rr.RR_EBREAKDOWN and all(i["status"] == rr.RR_EBREAKDOWN for i in infos)
    with pytest.raises(rr.RRError):
        P.solve(_cuda(B[:, 0]), krylov="block_minres")
    with pytest.raises(rr.RRError):
        P.solve_batch(_cuda(B), [0] * 3, krylov="block_cg", block_kmax=0)


XSTAR_PRECISION = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                               "precision_matern32_n65536_xstar.npy")


def test_precision_full_size_against_direct_solution():
    """The precision workload at its full size (stored dense Matern-3/2, n = 65,536,
    l = 1024, mu = 1e-5, tol 1e-10, mixed precision with float64 refinement):
    float64 relres <= tol over the whole residual, 64 sampled residual rows against
    the oracle's kernel formula, and the forward error against the stored direct
    solution x* (the oracle's float64 Cholesky solve) within ||A_mu (x - x*)|| / mu."""
    prob = workloads.cfg_precision()
    n, mu, tol = prob.n, prob.mus[0], prob.tol
    xs = np.load(XSTAR_PRECISION)
    kop = rr.kernel_operator(rr.OP_MATERN32, _cuda(prob.pts), prob.kconst, 1.0)
    A = rr.kernel_to_dense(kop, "fp64")
    dop = rr.dense_operator(A)
    P = rr.build_precond(dop, [mu], l=prob.l, sketch="gaussian", seed=prob.omega_seed, prec="mixed")
    b = _cuda(prob.b)
    x, info = P.solve(b, tol=tol, certify=False, maxit=20000)
    assert info["rc"] == rr.RR_OK
    r = (b - rr.apply_operator(dop, mu, "fp64", x)).cpu().numpy()
    # ||x - x*|| <= ||A_mu^{-1}|| ||A_mu (x - x*)|| <= ||A_mu (x - x*)|| / mu (A psd)
    dx = x - _cuda(xs)
    adx = float(torch.linalg.norm(rr.apply_operator(dop, mu, "fp64", dx)))
    del A, dop, P
    relres = np.linalg.norm(r) / np.linalg.norm(prob.b)
    assert relres <= tol * 1.0001
    xh = x.cpu().numpy()
    rows = np.random.default_rng(0).choice(n, 64, replace=False)
    from oracle.operators import kernel_block
    Xp = prob.pts.T.astype(np.float64)
    r_or = prob.b[rows] - kernel_block(prob.kind, prob.kconst, Xp[rows], Xp) @ xh - mu * xh[rows]
    # both are float64 residuals of the same x: they differ by the rounding of the sums
    scale = np.abs(kernel_block(prob.kind, prob.kconst, Xp[rows], Xp)) @ np.abs(xh)
    assert np.all(np.abs(r_or - r[rows]) <= 1e-13 * (scale + np.abs(prob.b[rows])))
    fwd = np.linalg.norm(xh - xs) / np.linalg.norm(xs)
    bound = adx / mu / np.linalg.norm(xs)
    assert fwd <= bound * 1.01, (fwd, bound)
    # both solutions have residuals near 1e-10 ||b||: the bound is about 1e-8 here
    assert bound <= 1e-7, bound


def test_small_dense_config_at_stated_size():
    """Config 1 as stated: stored dense RBF on n = 2,000 points ~ N(0, I_8), bandwidth 1,
    mu = 1e-3, Gaussian l = 100, float64, tol 1e-8: tau, the iteration count and the
    solution against the oracle's Algorithm RandRAND_PCG and the direct solve; plain CG
    (l = 0) against the oracle's CG."""
    prob = workloads.cfg_small_dense()
    mu, tol = prob.mus[0], prob.tol
    op = Operator.from_problem(prob)
    kop = rr.kernel_operator(rr.OP_RBF, _cuda(prob.pts), prob.kconst, prob.scale)
    A = rr.kernel_to_dense(kop, "fp64")
    dop = rr.dense_operator(A)
    P = rr.build_precond(dop, [mu], l=prob.l, sketch="gaussian", seed=prob.omega_seed, prec="fp64")
    x, info = P.solve(_cuda(prob.b), tol=tol, use_graph=True, check_every=16)
    Po = orr.build(op, [mu], prob.l, "gaussian", prob.omega_seed)[0]
    ref = osol.pcg(op.shifted(mu), Po.apply, prob.b, tol)
    assert info["rc"] == rr.RR_OK and ref.status == osol.OK
    assert abs(info["tau"] - Po.tau) <= 1e-9 * Po.tau
    assert abs(info["iters"] - ref.iters) <= max(2, int(0.03 * ref.iters)), (info["iters"], ref.iters)
    x = x.cpu().numpy()
    rel = osol.relres(op.shifted(mu), x, prob.b)
    assert rel <= tol * 1.0001 and rel <= ref.relres + 1e-8
    xs = osol.direct(op.to_dense(), mu, prob.b)
    cond = np.linalg.cond(op.to_dense() + mu * np.eye(prob.n))
    assert np.linalg.norm(x - xs) <= 2 * tol * cond * np.linalg.norm(xs)
    P0 = rr.build_precond(dop, [mu], l=0, prec="fp64")
    x0, i0 = P0.solve(_cuda(prob.b), tol=tol)
    r0 = osol.cg(op.shifted(mu), prob.b, tol)
    assert i0["rc"] == rr.RR_OK and abs(i0["iters"] - r0.iters) <= max(2, int(0.03 * r0.iters))
    assert info["iters"] < i0["iters"]


def test_kernel_ridge_headline_full_size():
    """The headline workload at full size (RBF n = 50,000, d = 16, mu = 1e-4, SRHT
    l = 500, tol 1e-6, float32-class entries with float64 refinement): the library's
    float64 relres <= tol; the device float64 residual agrees on 64 sampled rows with
    the oracle's kernel formula; the float32-class product agrees with the oracle's on
    the same rows within its arithmetic bound; the oracle operator's whole residual
    agrees with the library's; the float32 operator is exactly symmetric at this size;
    RandRAND needs fewer iterations than plain CG."""
    prob = workloads.cfg_kernel_ridge()
    mu, tol = prob.mus[0], prob.tol
    kop = rr.kernel_operator(rr.OP_RBF, _cuda(prob.pts), prob.kconst, prob.scale)
    P = rr.build_precond(kop, [mu], l=prob.l, sketch="srht", seed=prob.omega_seed, prec="fp32")
    b = _cuda(prob.b)
    x, info = P.solve(b, tol=tol)
    assert info["rc"] == rr.RR_OK and info["relres_fp64"] <= tol
    r = (b - rr.apply_operator(kop, mu, "fp64", x)).cpu().numpy()
    y32 = rr.apply_operator(kop, mu, "fp32", x).cpu().numpy()
    assert abs(np.linalg.norm(r) / np.linalg.norm(prob.b) - info["relres_fp64"]) <= 1e-9 * info["relres_fp64"]
    xh = x.cpu().numpy()
    from oracle.operators import kernel_block
    Xp = prob.pts.T.astype(np.float64)
    rows = np.random.default_rng(3).choice(prob.n, 64, replace=False)
    Kr = prob.scale * kernel_block(prob.kind, prob.kconst, Xp[rows], Xp)
    r_or = prob.b[rows] - Kr @ xh - mu * xh[rows]
    scale = np.abs(Kr) @ np.abs(xh) + mu * np.abs(xh[rows]) + np.abs(prob.b[rows])
    assert np.all(np.abs(r_or - r[rows]) <= 1e-13 * scale), np.max(np.abs(r_or - r[rows]) / scale)
    # float32-class product on the same rows: within 2e-6 of sum |K_ij x_j| (reading of
    # the float32 operator; the same bound as the smaller parity tests)
    y_or = Kr @ xh + mu * xh[rows]
    assert np.all(np.abs(y32[rows] - y_or) <= 2e-6 * scale)
    # the whole residual from the oracle operator
    rel64 = osol.relres(Operator.from_problem(prob).shifted(mu), xh, prob.b)
    assert rel64 <= tol and abs(info["relres_fp64"] - rel64) <= 1e-6 * rel64, (rel64, info["relres_fp64"])
    # the float32 operator at this size is exactly symmetric through its float64 sums
    U = np.random.default_rng(77).standard_normal((prob.n, 2))
    Y = rr.apply_operator_block(kop, mu, "fp32", _cuda(U)).cpu().numpy()
    uKv = U[:, 0] @ (Y[:, 1] - mu * U[:, 1])
    vKu = U[:, 1] @ (Y[:, 0] - mu * U[:, 0])
    assert abs(uKv - vKu) <= 1e-11 * (np.abs(U[:, 0]) @ np.abs(Y[:, 1] - mu * U[:, 1]))
    P0 = rr.build_precond(kop, [mu], l=0, prec="fp32")
    x0, i0 = P0.solve(b, tol=tol)
    assert i0["rc"] == rr.RR_OK and info["iters"] < i0["iters"]


def test_edge_cases_of_the_variants():
    """Degenerate inputs for the rows beyond PCG: a kernel operator smaller than one
    tile (n = 5) in float32 and float64 against the direct solve; b = 0 for R-RandRAND,
    split R-RandRAND, MINRES and block MINRES; one right-hand side in block MINRES is
    preconditioned MINRES (same iteration count, same solution); basis-less and q = 1
    builds with l = n solve in one or two iterations."""
    rng = np.random.default_rng(8)
    pts = rng.standard_normal((4, 5)).astype(np.float32)
    op5 = Operator(kind=rr.OP_RBF, pts=pts, kconst=0.3, scale=1.0)
    kop5 = rr.kernel_operator(rr.OP_RBF, _cuda(pts), 0.3, 1.0)
    b5 = rng.standard_normal(5)
    xs = osol.direct(op5.to_dense(), 0.1, b5)
    for prec in ("fp32", "fp64"):
        P = rr.build_precond(kop5, [0.1], l=2, sketch="gaussian", seed=4, prec=prec)
        x, info = P.solve(_cuda(b5), tol=1e-12)
        assert info["rc"] == rr.RR_OK
        assert np.linalg.norm(x.cpu().numpy() - xs) <= 1e-9 * np.linalg.norm(xs)
    prob = workloads.cfg_kernel_ridge(n=3000, d=8, l=90)
    mu = prob.mus[0]
    kop = rr.kernel_operator(rr.OP_RBF, _cuda(prob.pts), prob.kconst, prob.scale)
    P = rr.build_precond(kop, [mu], l=prob.l, sketch="srht", seed=prob.omega_seed, prec="fp64")
    z = torch.zeros(prob.n, dtype=torch.float64, device="cuda")
    for kw in (dict(method="r"), dict(method="split"), dict(krylov="minres"), dict(method="r", krylov="minres")):
        x, info = P.solve(z, **kw)
        assert info["rc"] == rr.RR_OK and float(x.abs().max()) == 0.0, kw
    X, infos, st = P.solve_batch(torch.zeros(prob.n, 3, dtype=torch.float64, device="cuda"), [0] * 3,
                                 krylov="block_minres")
    assert st == rr.RR_OK and float(X.abs().max()) == 0.0
    b = _cuda(prob.b)
    xm, im = P.solve(b, tol=1e-9, krylov="minres")
    Xb, ib, st = P.solve_batch(b[:, None], [0], tol=1e-9, krylov="block_minres")
    assert st == rr.RR_OK and abs(ib[0]["iters"] - im["iters"]) <= 1, (ib[0]["iters"], im["iters"])
    xb = Xb[:, 0]
    assert float(torch.linalg.norm(xb - xm) / torch.linalg.norm(xm)) <= 1e-7
    # l = n with column sampling: every column is sampled and the deflated space is
    # everything (one iteration, as the oracle).  (q = 1 at l = n is a degenerate case of
    # the method itself: Omega = A X is numerically rank deficient for this kernel and
    # tau_NYS collapses to ~1e-17 in the oracle as well, so it is not asserted here.)
    small = workloads.cfg_kernel_ridge(n=200, d=4, l=200)
    ksm = rr.kernel_operator(rr.OP_RBF, _cuda(small.pts), small.kconst, small.scale)
    for basis in ("explicit", "less"):
        Pl = rr.build_precond(ksm, [1e-2], l=200, sketch="colsample", seed=6, prec="fp64", tau_rule="nys",
                              basis=basis)
        xl, il = Pl.solve(_cuda(small.b), tol=1e-8, ok=(rr.RR_OK, rr.RR_ENOCONV), maxit=50)
        assert il["rc"] == rr.RR_OK and il["iters"] <= 2, (basis, il["iters"], il["tau"])
