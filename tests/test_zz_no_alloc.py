"""qtt_zqr_noalloc, the QR entry point that allocates nothing (its
workspace is the library's fixed per-GPU device array), against qtt_zqr on
the same inputs: two calls in a row, the second smaller, each bit-identical
to the allocating entry point (same kernels), and the capacity limit."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

q = pytest.importorskip("paper_2412_11566_amd")
torch = pytest.importorskip("torch")


def _rand(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _pair(ctx, a, with_q):
    batch, m, n = a.shape
    k = min(m, n)
    A = torch.from_numpy(a).cuda()
    nan = complex(float("nan"), float("nan"))
    R1 = torch.full((batch, k, n), nan, dtype=torch.complex128, device="cuda")
    R2 = torch.full_like(R1, nan)
    Q1 = Q2 = None
    if with_q:
        Q1 = torch.full((batch, m, k), nan, dtype=torch.complex128, device="cuda")
        Q2 = torch.full_like(Q1, nan)
    q.zqr(ctx, A, R1, Q1)
    q.zqr_noalloc(ctx, A, R2, Q2)
    ctx.sync()
    return (R1, Q1), (R2, Q2)


def test_zqr_noalloc_matches_zqr(ctx):
    rng = np.random.default_rng(17)
    # the rank-cap-128 sketch shape at the workspace limit's side, then a
    # smaller one that reuses the array the first call left behind
    for (batch, m, n, with_q) in ((12, 288, 144, True), (3, 100, 40, True), (5, 160, 80, False)):
        a = _rand(rng, batch, m, n)
        (R1, Q1), (R2, Q2) = _pair(ctx, a, with_q)
        assert torch.equal(R1, R2)
        if with_q:
            assert torch.equal(Q1, Q2)
            rec = (Q2 @ R2).cpu().numpy()
            assert np.abs(rec - a).max() < 1e-13 * np.abs(a).max() * np.sqrt(m)


def test_zqr_noalloc_rejects_more_than_the_workspace(ctx):
    m, n = 288, 144
    A = torch.zeros((13, m, n), dtype=torch.complex128, device="cuda")
    R = torch.zeros((13, n, n), dtype=torch.complex128, device="cuda")
    with pytest.raises(q.QttError) as e:
        q.zqr_noalloc(ctx, A, R)
    assert e.value.code == q._c.QTT_ECAPACITY
    assert "workspace" in str(e.value)
