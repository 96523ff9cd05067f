"""Batched complex GEMM (the contraction under every core product and
factorisation) against numpy, on both the matrix-core and the vector path,
over all operand modes, ragged tile tails and alpha/beta."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

SHAPES = [(32, 32, 8), (64, 64, 16), (70, 45, 33), (128, 256, 96), (33, 97, 130),
          (200, 40, 9), (16, 80, 40), (80, 12, 40), (5, 7, 3), (16, 16, 4), (151, 80, 153),
          (17, 161, 21),
          # long contractions over few output tiles: the split-K path
          (160, 80, 800), (96, 40, 517), (64, 64, 2000), (16, 16, 1584)]


def _mfma_shape(M, N, K):
    return M >= 16 and N >= 16 and K >= 4


def _rand(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _op(x, o):
    return x if o == "N" else (np.swapaxes(x, 1, 2) if o == "T" else np.conj(np.swapaxes(x, 1, 2)))


@pytest.mark.parametrize("path", [0, 1, 2, 4, 5, 6, 7, 8, 9, 10])
@pytest.mark.parametrize("ops", ["NN", "TN", "CN", "NT", "NC", "CT"])
def test_zgemm(ctx, path, ops):
    """path 0 automatic, 1 vector ALU, 2 matrix cores with the tile chosen
    per shape, 4..10 matrix cores with each FP64 tile variant forced."""
    import torch
    import paper_2412_11566_amd as q
    rng = np.random.default_rng(7)
    for (M, N, K) in SHAPES:
        if path >= 2 and not _mfma_shape(M, N, K):
            continue
        batch = 3
        a = _rand(rng, batch, *((M, K) if ops[0] == "N" else (K, M)))
        b = _rand(rng, batch, *((K, N) if ops[1] == "N" else (N, K)))
        c = _rand(rng, batch, M, N)
        alpha, beta = 0.5 - 1.25j, (0.0 if M % 2 else 0.75 + 0.5j)
        ref = alpha * (_op(a, ops[0]) @ _op(b, ops[1])) + beta * c
        A = torch.from_numpy(a).cuda()
        B = torch.from_numpy(b).cuda()
        Cm = torch.from_numpy(c).cuda()
        q.zgemm(ctx, A, B, Cm, ops[0], ops[1], alpha, beta, path)
        out = Cm.cpu().numpy()
        err = np.abs(out - ref).max() / (np.abs(ref).max() + 1e-300)
        # FP64 with K-term dot products: |error| <= K u |a||b| elementwise
        assert err < 64 * K * 2.2e-16, (M, N, K, ops, path, err)


@pytest.mark.parametrize("ops", ["NN", "CN", "NT"])
def test_zgemm_fp32_matrix_cores(ctx, ops):
    """FP32 operands and accumulation (the QTT_PREC_FP32 contractions):
    error within the FP32 bound sqrt(K)-scaled, against an FP64 reference."""
    import torch
    import paper_2412_11566_amd as q
    rng = np.random.default_rng(9)
    for (M, N, K) in [(32, 32, 8), (70, 45, 33), (160, 80, 800), (128, 256, 96), (64, 64, 2000)]:
        a = _rand(rng, 2, *((M, K) if ops[0] == "N" else (K, M)))
        b = _rand(rng, 2, *((K, N) if ops[1] == "N" else (N, K)))
        ref = _op(a, ops[0]) @ _op(b, ops[1])
        A = torch.from_numpy(a).cuda()
        B = torch.from_numpy(b).cuda()
        Cm = torch.zeros((2, M, N), dtype=torch.complex128, device="cuda")
        q.zgemm(ctx, A, B, Cm, ops[0], ops[1], 1.0, 0.0, path=3)
        out = Cm.cpu().numpy()
        # entries of a and b are O(1): |error| ~ sqrt(K) * 6e-8 * |a||b| per term
        err = np.abs(out - ref).max() / np.sqrt(K)
        assert err < 5e-6, (M, N, K, ops, err)
        assert np.abs(out - ref).max() > 0.0   # really computed in FP32


@pytest.mark.parametrize("ops", ["NN", "CN", "NT", "TC"])
def test_zgemm_split_bf16(ctx, ops):
    """Split-BF16 operands with FP32 accumulation (the QTT_PREC_BF16X3
    contractions).  Each operand is hi + lo in bf16 (relative error 2^-16
    after the split) and the dropped lo*lo term is of the same order, so a
    real product carries ~3 * 2^-16 relative error at worst and the K-sum
    grows like sqrt(K) for random signs: |error| / sqrt(K) < 2e-4 for O(1)
    entries.  Beside that bound: plain bf16 (2^-8) would miss it by far, and
    the result must be less accurate than FP32 contractions (it is really
    the split-BF16 path)."""
    import torch
    import paper_2412_11566_amd as q
    rng = np.random.default_rng(11)
    for (M, N, K) in [(32, 32, 8), (70, 45, 33), (160, 80, 800), (128, 256, 96), (64, 64, 2000),
                      (17, 161, 31), (96, 40, 517)]:
        a = _rand(rng, 2, *((M, K) if ops[0] == "N" else (K, M)))
        b = _rand(rng, 2, *((K, N) if ops[1] == "N" else (N, K)))
        ref = _op(a, ops[0]) @ _op(b, ops[1])
        A = torch.from_numpy(a).cuda()
        B = torch.from_numpy(b).cuda()
        Cm = torch.full((2, M, N), 0.5 + 0.25j, dtype=torch.complex128, device="cuda")
        c0 = Cm.cpu().numpy()
        q.zgemm(ctx, A, B, Cm, ops[0], ops[1], 0.5 - 1.0j, 2.0, path=q._c.QTT_GEMM_PATH_BF16X3)
        out = Cm.cpu().numpy()
        want = (0.5 - 1.0j) * ref + 2.0 * c0
        err = np.abs(out - want).max() / np.sqrt(K)
        assert err < 2e-4, (M, N, K, ops, err)
        C32 = torch.zeros((2, M, N), dtype=torch.complex128, device="cuda")
        q.zgemm(ctx, A, B, C32, ops[0], ops[1], 1.0, 0.0, path=3)
        e32 = np.abs(C32.cpu().numpy() - ref).max()
        assert np.abs(out - want).max() > e32


@pytest.mark.parametrize("path", [2, 3, 16])
def test_zgemm_split_k_back_to_back(ctx, path):
    """Split-K products issued back to back on one stream, with no host
    synchronisation between them (different grids, batches, beta; each
    reuses workspace the previous one released), and the same product twice
    giving bit-identical results (slices summed in fixed order)."""
    import torch
    import paper_2412_11566_amd as q
    rng = np.random.default_rng(13)
    cases = [(160, 80, 800, 1), (96, 40, 517, 5), (64, 64, 2000, 2), (16, 16, 1584, 40),
             (160, 80, 800, 3), (33, 20, 1200, 7)]
    outs = []
    for (M, N, K, nb) in cases + cases[:2]:
        a = _rand(rng, nb, M, K)
        b = _rand(rng, nb, K, N)
        c = _rand(rng, nb, M, N)
        beta = 0.0 if nb % 2 else -0.5 + 0.25j
        A = torch.from_numpy(a).cuda()
        B = torch.from_numpy(b).cuda()
        Cm = torch.from_numpy(c).cuda()
        q.zgemm(ctx, A, B, Cm, "N", "N", 1.5, beta, path)
        outs.append((Cm, (a @ b) * 1.5 + beta * c, K))
    for Cm, ref, K in outs:
        d = np.abs(Cm.cpu().numpy() - ref).max()
        if path == 2:    # FP64: the K u bound of test_zgemm
            assert d / np.abs(ref).max() < 64 * K * 2.2e-16, (path, K, d)
        else:            # FP32 and split-BF16: the sqrt(K) bounds above (alpha 1.5)
            assert d / 1.5 / np.sqrt(K) < (5e-6 if path == 3 else 2e-4), (path, K, d)
    # repeat one product on the same inputs: identical bits
    a = _rand(rng, 2, 160, 4000)
    b = _rand(rng, 2, 4000, 80)
    A = torch.from_numpy(a).cuda()
    B = torch.from_numpy(b).cuda()
    C1 = torch.zeros((2, 160, 80), dtype=torch.complex128, device="cuda")
    C2 = torch.zeros_like(C1)
    q.zgemm(ctx, A, B, C1, "N", "N", 1.0, 0.0, path)
    q.zgemm(ctx, A, B, C2, "N", "N", 1.0, 0.0, path)
    assert torch.equal(C1, C2)


def test_zgemm_mfma_rejects_small(ctx):
    import torch
    import paper_2412_11566_amd as q
    A = torch.zeros((1, 15, 8), dtype=torch.complex128, device="cuda")
    B = torch.zeros((1, 8, 64), dtype=torch.complex128, device="cuda")
    Cm = torch.zeros((1, 15, 64), dtype=torch.complex128, device="cuda")
    with pytest.raises(q.QttError):
        q.zgemm(ctx, A, B, Cm, path=2)
    with pytest.raises(q.QttError):
        q.zgemm(ctx, A, B, Cm, path=11)   # no such tile variant
