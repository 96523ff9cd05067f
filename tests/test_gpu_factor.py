"""The small dense factorisations of TT-rounding (Householder QR and the
one-sided Jacobi SVD of the square factor) against the definitions and
numpy, on shapes that reach every kernel variant, ragged tails, wide and
rank-deficient matrices."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

QR_SHAPES = [(6, 6), (16, 40), (30, 20), (64, 64), (50, 64), (100, 64), (128, 33), (160, 64),
             (192, 50), (256, 64), (200, 64), (64, 100), (40, 128), (128, 80), (100, 128),
             (160, 80), (150, 128), (160, 128), (192, 80), (300, 70), (20, 300), (1, 5), (7, 1),
             (16, 16), (33, 16), (200, 16), (100, 30), (300, 30), (70, 48), (250, 40), (224, 64),
             (168, 80), (96, 96), (150, 96), (110, 112), (112, 128), (128, 128), (80, 80)]


def _rand(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _check_qr(a, R, Q, full_rank=True):
    batch, m, n = a.shape
    k = min(m, n)
    scale = np.linalg.norm(a.reshape(batch, -1), axis=1)[:, None, None]
    assert np.all(np.tril(R, -1) == 0)
    assert np.abs(np.diagonal(R, axis1=1, axis2=2).imag).max() == 0.0
    rec = Q @ R
    assert np.abs(rec - a).max() / scale.max() < 1e-13 * np.sqrt(m)
    eye = np.eye(k)[None]
    assert np.abs(np.conj(np.swapaxes(Q, 1, 2)) @ Q - eye).max() < 1e-13 * np.sqrt(m)
    if full_rank:
        _, Rn = np.linalg.qr(a)
        assert np.abs(np.abs(R) - np.abs(Rn)).max() / scale.max() < 1e-12


@pytest.mark.parametrize("shape", QR_SHAPES)
def test_zqr(ctx, shape):
    import torch
    import paper_2412_11566_amd as q
    m, n = shape
    k = min(m, n)
    rng = np.random.default_rng(m * 1000 + n)
    a = _rand(rng, 3, m, n)
    A = torch.from_numpy(a).cuda()
    R = torch.zeros((3, k, n), dtype=torch.complex128, device="cuda")
    Q = torch.zeros((3, m, k), dtype=torch.complex128, device="cuda")
    q.zqr(ctx, A, R, Q)
    _check_qr(a, R.cpu().numpy(), Q.cpu().numpy())
    # R alone must equal the R of the Q-forming call
    R2 = torch.zeros_like(R)
    q.zqr(ctx, A, R2)
    assert torch.equal(R, R2)


# shapes of the blocked matrix-core kernel (m >= n, 16 < n <= 96, m <= 192):
# full and partial last panels, padded row blocks, every column-group count
QR_BLOCKED_SHAPES = [(160, 80), (128, 80), (96, 80), (160, 64), (64, 64), (48, 48), (128, 33),
                     (17, 17), (192, 96), (100, 50), (33, 20), (150, 96), (80, 80), (191, 95),
                     (160, 40), (24, 18)]


@pytest.mark.parametrize("shape", QR_BLOCKED_SHAPES)
def test_zqr_blocked(ctx, shape):
    """Blocked Householder QR (panels of 16 columns, compact WY block
    reflectors on the matrix cores) against the definition and numpy."""
    import torch
    import paper_2412_11566_amd as q
    m, n = shape
    k = min(m, n)
    rng = np.random.default_rng(m * 7 + n)
    a = _rand(rng, 3, m, n)
    A = torch.from_numpy(a).cuda()
    R = torch.zeros((3, k, n), dtype=torch.complex128, device="cuda")
    Q = torch.zeros((3, m, k), dtype=torch.complex128, device="cuda")
    q.zqr(ctx, A, R, Q, path=2)
    _check_qr(a, R.cpu().numpy(), Q.cpu().numpy())
    R2 = torch.zeros_like(R)
    q.zqr(ctx, A, R2, path=2)
    assert torch.equal(R, R2)


# shapes of the workspace-resident blocked kernel (m >= n, m <= 320,
# n <= 160): the sketched unfoldings of rank caps up to 144 + 16, ragged
# last panels and row blocks
QR_BIG_SHAPES = [(288, 144), (272, 136), (320, 160), (256, 128), (290, 130), (200, 100),
                 (144, 144), (97, 97), (193, 17), (320, 1), (161, 160), (230, 150)]


@pytest.mark.parametrize("shape", QR_BIG_SHAPES)
def test_zqr_big(ctx, shape):
    """Blocked QR with the matrix in the workspace: against the definition
    and numpy; R alone equals the R of the Q-forming call; a rank-deficient
    matrix with a zero and a tiny column keeps Q orthonormal and finite."""
    import torch
    import paper_2412_11566_amd as q
    m, n = shape
    k = min(m, n)
    rng = np.random.default_rng(m * 31 + n)
    a = _rand(rng, 2, m, n)
    A = torch.from_numpy(a).cuda()
    # outputs start as NaN: every entry of R (zeros below the diagonal
    # included) and of Q must be written
    nan = complex(float("nan"), float("nan"))
    R = torch.full((2, k, n), nan, dtype=torch.complex128, device="cuda")
    Q = torch.full((2, m, k), nan, dtype=torch.complex128, device="cuda")
    q.zqr(ctx, A, R, Q, path=6)
    _check_qr(a, R.cpu().numpy(), Q.cpu().numpy())
    R2 = torch.full_like(R, nan)
    q.zqr(ctx, A, R2, path=6)
    assert torch.equal(R, R2)
    if n >= 8:
        d = _rand(rng, 2, m, 5) @ _rand(rng, 2, 5, n)
        d[:, :, 3] = 0.0
        d[:, :, 6] *= 1e-300
        A = torch.from_numpy(d).cuda()
        q.zqr(ctx, A, R, Q, path=6)
        Rn, Qn = R.cpu().numpy(), Q.cpu().numpy()
        assert np.all(np.isfinite(Rn)) and np.all(np.isfinite(Qn))
        _check_qr(d, Rn, Qn, full_rank=False)


def test_zqr_big_rejects_uncovered(ctx):
    import torch
    import paper_2412_11566_amd as q
    for (m, n) in [(321, 64), (200, 161), (100, 120)]:
        k = min(m, n)
        A = torch.zeros((1, m, n), dtype=torch.complex128, device="cuda")
        R = torch.zeros((1, k, n), dtype=torch.complex128, device="cuda")
        with pytest.raises(q.QttError):
            q.zqr(ctx, A, R, path=6)


QR_TWO_COL_SHAPES = [(160, 80), (128, 80), (96, 80), (160, 64), (64, 64), (48, 48), (128, 32),
                     (200, 64), (33, 20), (17, 17), (250, 40), (100, 96), (16, 90), (5, 70)]


@pytest.mark.parametrize("shape", QR_TWO_COL_SHAPES)
def test_zqr_two_columns_per_lane(ctx, shape):
    """Unblocked register kernel with two columns per lane."""
    import torch
    import paper_2412_11566_amd as q
    m, n = shape
    k = min(m, n)
    rng = np.random.default_rng(m * 13 + n)
    a = _rand(rng, 3, m, n)
    A = torch.from_numpy(a).cuda()
    R = torch.zeros((3, k, n), dtype=torch.complex128, device="cuda")
    Q = torch.zeros((3, m, k), dtype=torch.complex128, device="cuda")
    q.zqr(ctx, A, R, Q, path=4)
    _check_qr(a, R.cpu().numpy(), Q.cpu().numpy(), full_rank=m >= n)
    R2 = torch.zeros_like(R)
    q.zqr(ctx, A, R2, path=4)
    assert torch.equal(R, R2)


QR_ONE_ROWBLOCK_SHAPES = [(160, 80), (128, 80), (96, 80), (160, 64), (64, 64), (48, 48), (128, 32),
                          (33, 20), (17, 17), (100, 96), (160, 17), (150, 90)]


@pytest.mark.parametrize("shape", QR_ONE_ROWBLOCK_SHAPES)
def test_zqr_one_rowblock(ctx, shape):
    """One wave per 16-column group over all rows (one barrier per column),
    Q from the panel vectors as matrix-core block reflectors."""
    import torch
    import paper_2412_11566_amd as q
    m, n = shape
    k = min(m, n)
    rng = np.random.default_rng(m * 17 + n)
    a = _rand(rng, 3, m, n)
    A = torch.from_numpy(a).cuda()
    R = torch.zeros((3, k, n), dtype=torch.complex128, device="cuda")
    Q = torch.zeros((3, m, k), dtype=torch.complex128, device="cuda")
    q.zqr(ctx, A, R, Q, path=5)
    _check_qr(a, R.cpu().numpy(), Q.cpu().numpy())
    R2 = torch.zeros_like(R)
    q.zqr(ctx, A, R2, path=5)
    assert torch.equal(R, R2)


def test_zqr_blocked_rejects_uncovered(ctx):
    import torch
    import paper_2412_11566_amd as q
    for (m, n) in [(40, 64), (200, 64), (100, 16), (100, 100)]:
        k = min(m, n)
        A = torch.zeros((1, m, n), dtype=torch.complex128, device="cuda")
        R = torch.zeros((1, k, n), dtype=torch.complex128, device="cuda")
        with pytest.raises(q.QttError):
            q.zqr(ctx, A, R, path=2)


@pytest.mark.parametrize("shape", [(160, 80), (64, 40), (128, 128)])
def test_zqr_rank_deficient_and_generic_path(ctx, shape):
    import torch
    import paper_2412_11566_amd as q
    m, n = shape
    k = min(m, n)
    rng = np.random.default_rng(5)
    a = _rand(rng, 2, m, 5) @ _rand(rng, 2, 5, n)
    a[:, :, 3] = 0.0                       # an exactly zero column
    for path in (0, 1, 2, 3, 4, 5):
        if path == 2 and not (m >= n and 16 < n <= 96 and m <= 192):
            continue
        if path == 4 and n > 96:
            continue
        if path == 5 and not (m >= n and 16 < n <= 96 and m <= 160):
            continue
        A = torch.from_numpy(a).cuda()
        R = torch.zeros((2, k, n), dtype=torch.complex128, device="cuda")
        Q = torch.zeros((2, m, k), dtype=torch.complex128, device="cuda")
        q.zqr(ctx, A, R, Q, path=path)
        _check_qr(a, R.cpu().numpy(), Q.cpu().numpy(), full_rank=False)


@pytest.mark.parametrize("shape", [(160, 80), (64, 64), (200, 40)])
def test_zqr_tiny_columns(ctx, shape):
    """Columns with norms near the bottom of the double range (numerically
    zero directions of a sketch) must not produce inf or NaN."""
    import torch
    import paper_2412_11566_amd as q
    m, n = shape
    k = min(m, n)
    rng = np.random.default_rng(11)
    a = _rand(rng, 2, m, n)
    a[:, :, 1] *= 1e-155
    a[:, :, 5] *= 1e-300
    for path in (0, 2, 4, 5):
        if path == 2 and not (m >= n and 16 < n <= 96 and m <= 192):
            continue
        if path == 5 and not (m >= n and 16 < n <= 96 and m <= 160):
            continue
        A = torch.from_numpy(a).cuda()
        R = torch.zeros((2, k, n), dtype=torch.complex128, device="cuda")
        Q = torch.zeros((2, m, k), dtype=torch.complex128, device="cuda")
        q.zqr(ctx, A, R, Q, path=path)
        R, Q = R.cpu().numpy(), Q.cpu().numpy()
        assert np.all(np.isfinite(R)) and np.all(np.isfinite(Q))
        _check_qr(a, R, Q, full_rank=False)


@pytest.mark.parametrize("n", [1, 2, 7, 16, 33, 64, 80, 96, 97, 128, 144, 160, 161, 230, 320])
def test_zjacobi(ctx, n):
    import torch
    import paper_2412_11566_amd as q
    rng = np.random.default_rng(n)
    a = _rand(rng, 3, n, n)
    if n >= 16:   # graded singular values down to 1e-12 in the last matrix
        u, _, vh = np.linalg.svd(a[2])
        a[2] = (u * np.logspace(0, -12, n)) @ vh
    A = torch.from_numpy(a).cuda()
    U = torch.zeros_like(A)
    S = torch.zeros((3, n), dtype=torch.float64, device="cuda")
    q.zjacobi(ctx, A, U, S)
    U, S = U.cpu().numpy(), S.cpu().numpy()
    for b in range(3):
        sv = np.linalg.svd(a[b], compute_uv=False)
        assert np.all(np.diff(S[b]) <= 0)
        assert np.abs(S[b] - sv).max() < 1e-13 * sv[0] * np.sqrt(n)
        # U^H A A^H U = diag(S^2) and U has orthonormal columns
        g = np.conj(U[b].T) @ a[b]
        assert np.abs(g @ np.conj(g.T) - np.diag(S[b] ** 2)).max() < 1e-12 * sv[0] ** 2
        assert np.abs(np.conj(U[b].T) @ U[b] - np.eye(n)).max() < 1e-12 * n


def test_zjacobi_rejects_large(ctx):
    import torch
    import paper_2412_11566_amd as q
    A = torch.zeros((1, 321, 321), dtype=torch.complex128, device="cuda")
    with pytest.raises(q.QttError):
        q.zjacobi(ctx, A, torch.zeros_like(A), torch.zeros((1, 321), dtype=torch.float64, device="cuda"))
