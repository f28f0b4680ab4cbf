"""The no-allocation operator product (rr_apply_operator_noalloc) against the
allocating rr_apply_operator: the same kernels, so bitwise-equal results; two
calls in a row, the second with a smaller operator (the shared scratch keeps the
first call's contents)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
rr = pytest.importorskip("paper_2509_19747_amd")
from paper_2509_19747_amd import binding as rb  # noqa: E402

pytestmark = pytest.mark.gpu


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("kind", [rr.OP_RBF, rr.OP_MATERN32])
def test_noalloc_kernel_operator_matches_allocating_entry(kind):
    for n, d, prec in [(20_000, 16, "fp32"), (3_001, 8, "fp32"), (12_345, 16, "fp64"), (777, 4, "fp64")]:
        rng = np.random.default_rng(n + d)
        pts = rng.standard_normal((d, n)).astype(np.float32)
        kop = rr.kernel_operator(kind, _cuda(pts), 0.5 / d, 1.0 / n)
        u = _cuda(rng.standard_normal(n))
        ref = rr.apply_operator(kop, 1e-3, prec, u)
        y = torch.full_like(u, np.nan)
        rb.apply_operator_noalloc(kop, 1e-3, prec, u, y)
        torch.cuda.synchronize()
        assert torch.equal(y, ref), (n, d, prec)


def test_noalloc_dense_operator_matches_allocating_entry():
    for n, prec in [(2_000, "fp32"), (1_500, "fp64"), (901, "mixed")]:
        rng = np.random.default_rng(n)
        M = rng.standard_normal((n, n))
        A = _cuda(M @ M.T / n)
        dop = rr.dense_operator(A)
        u = _cuda(rng.standard_normal(n))
        ref = rr.apply_operator(dop, 1e-2, prec, u)
        y = torch.full_like(u, np.nan)
        rb.apply_operator_noalloc(dop, 1e-2, prec, u, y)
        torch.cuda.synchronize()
        assert torch.equal(y, ref), (n, prec)


def test_noalloc_rejects_an_operator_beyond_the_scratch():
    n = 200_000
    pts = torch.zeros((16, n), dtype=torch.float32, device="cuda")
    kop = rr.kernel_operator(rr.OP_RBF, pts, 0.1, 1.0 / n)
    u = torch.zeros(n, dtype=torch.float64, device="cuda")
    with pytest.raises(rr.RRError) as e:
        rb.apply_operator_noalloc(kop, 0.0, "fp32", u)
    assert e.value.status == rr.RR_EINVAL
