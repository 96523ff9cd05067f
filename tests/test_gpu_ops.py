"""GPU parity of the single C-ABI operations against the CPU oracle.

Tiny seeded trains (n = 2: 4^3 voxels, L = 7 cores) so the oracle densifies
everything; comparisons are on gauge-invariant quantities (dense tensors,
norms, ranks of exact roundings).
"""
import numpy as np
import pytest

from oracle import dense as D, qtt as Q
from oracle.voigt import iso_voigt
import microstructures as M
from tests.helpers import dense, random_tt, rel

pytestmark = pytest.mark.gpu

q = pytest.importorskip("paper_2412_11566_amd")


def voigt_dims(n):
    return [6] + [2] * (3 * n)


def rand_strain(rng, n, r, batch=2):
    dims = voigt_dims(n)
    L = len(dims)
    ranks = [1] + [min(r, int(np.prod(dims[:k])), int(np.prod(dims[k:]))) for k in range(1, L)] + [1]
    return random_tt(rng, dims, ranks, batch)


def test_roundtrip_and_norm(ctx):
    rng = np.random.default_rng(1)
    cores = rand_strain(rng, 2, 5, batch=3)
    t = q.tt_from_cores(ctx, cores)
    back = t.cores()
    for a, b in zip(cores, back):
        assert np.array_equal(a, b)
    nrm = q.tt_norm(ctx, t)
    for b in range(3):
        assert abs(nrm[b] - np.linalg.norm(dense(cores, b))) <= 1e-13 * nrm[b]


def test_round_exact_and_bound(ctx):
    rng = np.random.default_rng(2)
    cores = rand_strain(rng, 2, 9, batch=2)
    ref = [dense(cores, b) for b in range(2)]
    t = q.tt_from_cores(ctx, cores)
    q.tt_round(ctx, t, 1e-14, 0)
    out = t.cores()
    for b in range(2):
        assert rel(dense(out, b), ref[b]) < 1e-12
    # truncating rounding: bound of eq. rounding_condition_tt and oracle ranks
    for delta in (1e-1, 1e-2):
        t = q.tt_from_cores(ctx, cores)
        disc = q.tt_round(ctx, t, delta, 0)
        out = t.cores()
        for b in range(2):
            e = rel(dense(out, b), ref[b])
            assert e <= delta * (1 + 1e-9)
            assert abs(e - disc[b]) <= 1e-9 + 1e-6 * e
            oc, _ = Q.tt_round([c[b] for c in cores], delta)
            # common ranks of the batch are the max over its elements
        ranks_each = [Q.ranks(Q.tt_round([c[b] for c in cores], delta)[0]) for b in range(2)]
        assert t.ranks == [max(x) for x in zip(*ranks_each)]


def test_round_cap(ctx):
    """Cap-limited rounding: error equals the discarded mass and sits
    between the best rank-cap error of the worst unfolding and sqrt(L-1)
    times it (quasi-optimality of sequential truncation)."""
    rng = np.random.default_rng(3)
    cores = rand_strain(rng, 2, 12, batch=1)
    full = dense(cores)
    t = q.tt_from_cores(ctx, cores)
    disc = q.tt_round(ctx, t, 1e-14, 4)
    assert max(t.ranks) <= 4
    e = rel(dense(t.cores()), full)
    assert abs(e - disc[0]) <= 1e-9
    L = full.ndim
    tails = []
    for k in range(1, L):
        s = np.linalg.svd(full.reshape(int(np.prod(full.shape[:k])), -1), compute_uv=False)
        tails.append(np.sqrt((s[4:] ** 2).sum()) / np.linalg.norm(full))
    lo = max(tails)
    assert lo * (1 - 1e-9) <= e <= np.sqrt(L - 1) * lo * (1 + 1e-9)


def test_axpby(ctx):
    rng = np.random.default_rng(4)
    x = rand_strain(rng, 2, 3, batch=2)
    y = rand_strain(rng, 2, 4, batch=2)
    z = q.tt_axpby(ctx, 0.7, q.tt_from_cores(ctx, x), -1.3, q.tt_from_cores(ctx, y))
    zc = z.cores()
    for b in range(2):
        assert rel(dense(zc, b), 0.7 * dense(x, b) - 1.3 * dense(y, b)) < 1e-14


def _sfft_reference(field, n):
    """S on a (6, N, N, N) field: N^{3/2} ifftn with bit-reversed output
    indices (the plain definition of the reduced QFT on each axis)."""
    N = 1 << n
    r = Q.bitrev(np.arange(N), n)
    f = N ** 1.5 * np.fft.ifftn(field, axes=(1, 2, 3))
    return f[:, r][:, :, r][:, :, :, r]


@pytest.mark.parametrize("flags", [q.QTT_NO_ROUND if hasattr(q, "QTT_NO_ROUND") else 2, 4])
def test_sfft_apply(ctx, flags):
    n = 2
    rng = np.random.default_rng(5)
    x = rand_strain(rng, n, 6, batch=2)
    S = q.sfft_build(ctx, n, 1e-14)
    y = q.sfft_apply(ctx, S, q.tt_from_cores(ctx, x), delta=1e-14, cap=0, seed=11, flags=flags)
    yc = y.cores()
    N = 1 << n
    for b in range(2):
        ref = _sfft_reference(dense(x, b).reshape(6, N, N, N), n)
        assert rel(dense(yc, b).reshape(6, N, N, N), ref) < 1e-11


def test_sfft_materialised_ranks_128(ctx):
    """Materialised SFFT product on ranks up to 128 (product bonds up to
    256, bond ranks 6, 12, 24, 48, 96 that do not divide the workgroup
    size, so threads of one workgroup span several output columns), batch
    of two, against the library FFT at bit-reversed indices; the rank-640
    product is covered at full size."""
    n = 4
    N = 1 << n
    rng = np.random.default_rng(15)
    x = rand_strain(rng, n, 128, batch=2)
    S = q.sfft_build(ctx, n, 1e-14)
    y = q.sfft_apply(ctx, S, q.tt_from_cores(ctx, x), flags=q.QTT_NO_ROUND)
    xr = [x[0].shape[1]] + [c.shape[3] for c in x]
    assert y.ranks == [a * b for a, b in zip(S.ranks, xr)]
    yc = y.cores()
    for b in range(2):
        ref = _sfft_reference(dense(x, b).reshape(6, N, N, N), n)
        assert rel(dense(yc, b).reshape(6, N, N, N), ref) < 1e-11


def test_sfft_inverse_roundtrip(ctx):
    n = 2
    rng = np.random.default_rng(6)
    x = rand_strain(rng, n, 5, batch=1)
    S = q.sfft_build(ctx, n, 1e-14)
    y = q.sfft_apply(ctx, S, q.tt_from_cores(ctx, x), delta=1e-14, seed=1)
    z = q.sfft_apply(ctx, S, y, inverse=True, delta=1e-14, seed=2)
    assert rel(dense(z.cores()), dense(x)) < 1e-11


def test_sfft_operator_cores(ctx):
    """Operator densified equals the reduced QFT on each axis (n = 3)."""
    n = 3
    S = q.sfft_build(ctx, n, 1e-14)
    cores = S.cores()
    assert np.allclose(cores[0].reshape(6, 6), np.eye(6))
    ax = cores[1:1 + n]
    assert rel(Q.tto_full(ax), Q.qn_matrix(n)) < 1e-13


def test_hadamard(ctx):
    n = 2
    N = 1 << n
    rng = np.random.default_rng(7)
    phase = M.sphere(N, 0.3)
    lame = np.array([[1.0, 0.5], [4.0, 3.0]])
    lame0 = (2.5, 1.75)
    Cd, chi = q.from_voxels(ctx, phase, lame, lame0, 1e-14)
    x = rand_strain(rng, n, 6, batch=2)
    for flags in (2, 4):
        y = q.tt_hadamard(ctx, Cd, q.tt_from_cores(ctx, x), delta=1e-14, seed=3, flags=flags)
        dC = D.stiffness_per_phase(lame) - iso_voigt(*lame0)[None]
        for b in range(2):
            ref = D.apply_local(dC, phase, dense(x, b).reshape(6, N, N, N))
            assert rel(dense(y.cores(), b).reshape(6, N, N, N), ref) < 1e-11


@pytest.mark.parametrize("n", [2, 3, 4])
def test_green_apply(ctx, n):
    """The Green operator, its four factors assembled from the direction
    train that the device TT-SVD builds, against the oracle's Green table
    (direct scheme, Nyquist rule) on every voxel."""
    N = 1 << n
    lam0, mu0 = 2.3, 1.4
    rng = np.random.default_rng(8)
    Gm = q.green_build(ctx, n, lam0, mu0, 1e-14)
    x = rand_strain(rng, n, 6, batch=2)
    y = q.green_apply(ctx, Gm, q.tt_from_cores(ctx, x), delta=1e-14, seed=4, flags=4)
    Gt = Q.green_tensor(n, lam0, mu0)
    for b in range(2):
        xd = dense(x, b).reshape(6, N, N, N)
        ref = np.einsum("vwxyz,wxyz->vxyz", Gt, xd)
        assert rel(dense(y.cores(), b).reshape(6, N, N, N), ref) < 1e-10


def test_mean_apply(ctx):
    n = 2
    N = 1 << n
    rng = np.random.default_rng(9)
    phase = M.sphere(N, 0.3)
    lame = np.array([[1.0, 0.5], [4.0, 3.0]])
    lame0 = (2.5, 1.75)
    Cd, _ = q.from_voxels(ctx, phase, lame, lame0, 1e-14)
    x = rand_strain(rng, n, 6, batch=2)
    m = q.tt_mean_apply(ctx, Cd, q.tt_from_cores(ctx, x))
    dC = D.stiffness_per_phase(lame) - iso_voigt(*lame0)[None]
    for b in range(2):
        ref = D.apply_local(dC, phase, dense(x, b).reshape(6, N, N, N)).mean(axis=(1, 2, 3))
        assert np.abs(m[b] - ref).max() < 1e-12 * max(1.0, np.abs(ref).max())


def test_error_paths(ctx):
    with pytest.raises(q.QttError):
        q.sfft_build(ctx, 0, 1e-10)
    with pytest.raises(q.QttError):
        q.green_build(ctx, 3, 1.0, -1.0, 1e-10)
