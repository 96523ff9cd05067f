"""Pins of the AMEn-adapted product in ``oracle.amen`` (App. B).

Each pin comes from a source other than the sweep it checks: the product
A x formed densely from its definition, the TT-SVD ranks of that dense
product, the Galerkin condition of eq. galerkin_condition checked on the
dense frame, and the rounding bound of Sec. 3 for truncated products.
"""
import numpy as np
import pytest

from oracle import amen as AM, qtt as Q

DIMS = [6] + [2] * 6


def _rtt(rng, ranks, dims=DIMS):
    return [rng.standard_normal((ranks[k], d, ranks[k + 1]))
            + 1j * rng.standard_normal((ranks[k], d, ranks[k + 1])) for k, d in enumerate(dims)]


def _rtto(rng, ranks, dims=DIMS):
    return [rng.standard_normal((ranks[k], d, d, ranks[k + 1]))
            + 1j * rng.standard_normal((ranks[k], d, d, ranks[k + 1])) for k, d in enumerate(dims)]


def _caps(r, dims=DIMS):
    """ranks min(r, structural) for a train of dims"""
    L = len(dims)
    return [1] + [min(r, int(np.prod(dims[:k])), int(np.prod(dims[k:]))) for k in range(1, L)] + [1]


@pytest.fixture(scope="module")
def problem():
    rng = np.random.default_rng(1)
    A = _rtto(rng, [1, 2, 3, 3, 3, 3, 2, 1])
    x = _rtt(rng, [1, 3, 4, 4, 4, 4, 2, 1])
    full = Q.tto_full(A) @ Q.tt_full(x).ravel()
    return A, x, full, rng


def _err(y, full):
    return np.linalg.norm(Q.tt_full(y).ravel() - full) / np.linalg.norm(full)


def test_exact_product_from_a_full_rank_guess(problem):
    """With an initial guess at the structural ranks one sweep gives A x to
    rounding, with the ranks of the TT-SVD of the dense product."""
    A, x, full, rng = problem
    y0 = _rtt(rng, _caps(64))
    z0 = _rtt(rng, _caps(4))
    y, m, _ = AM.amen_mv(A, x, y0, z0, 1e-14, sweeps=1)
    assert _err(y, full) < 1e-13
    assert Q.ranks(y) == Q.ranks(Q.tt_svd(full.reshape(DIMS), 1e-12))


@pytest.mark.parametrize("ry,rz,need", [(2, 4, 4), (2, 8, 3), (4, 4, 3)])
def test_enrichment_grows_the_rank_to_the_product(problem, ry, rz, need):
    """From a rank-ry guess the residual enrichment (rank rz) reaches the
    exact product within `need` sweeps; without it the rank would stay ry."""
    A, x, full, rng = problem
    y0 = _rtt(rng, _caps(ry))
    z0 = _rtt(rng, _caps(rz))
    y1, _, _ = AM.amen_mv(A, x, y0, z0, 1e-12, sweeps=1, tol=0.0)
    assert max(Q.ranks(y1)) <= ry
    y, m, ch = AM.amen_mv(A, x, y0, z0, 1e-12, sweeps=8)
    assert _err(y, full) < 1e-13
    assert m <= need + 1        # the sweep after the exact one confirms
    assert ch < 1e-12


def test_galerkin_condition_of_the_last_core(problem):
    """After a sweep the last core is the projection of A x onto the frame
    of the other cores (eq. galerkin_condition): Y^H (A x) = y_L, with Y the
    dense left frame, orthonormal."""
    A, x, full, rng = problem
    y0 = AM._right_orthonormal(_rtt(rng, _caps(3)))
    z0 = AM._right_orthonormal(_rtt(rng, _caps(4)))
    y, z, kept = AM.amen_sweep(A, x, y0, z0, 1e-12, 1 << 30)
    F = y[0].reshape(-1, y[0].shape[2])                              # left frame, open bond
    for c in y[1:-1]:
        F = (F @ c.reshape(c.shape[0], -1)).reshape(-1, c.shape[2])
    assert np.abs(F.conj().T @ F - np.eye(F.shape[1])).max() < 1e-12
    proj = F.conj().T @ full.reshape(F.shape[0], -1)
    assert np.abs(proj - y[-1][:, :, 0]).max() < 1e-12 * np.abs(full).max()
    # the compact product's last core is the projection onto the kept columns
    yc = AM.compact(y, kept)
    Fc = F[:, :kept[-2]]
    assert np.abs(Fc.conj().T @ full.reshape(F.shape[0], -1) - yc[-1][:, :, 0]).max() < 1e-12 * np.abs(full).max()


@pytest.mark.parametrize("delta", [1e-2, 1e-4])
def test_truncated_product_meets_the_rounding_bound(problem, delta):
    """Truncated at delta: ||y - A x|| <= delta ||A x|| (Sec. 3, eq.
    rounding_condition_tt, summed over the bonds) once the sweeps settle,
    with ranks no larger than the TT-SVD's at the same delta."""
    A, x, full, rng = problem
    y0 = _rtt(rng, _caps(4))
    z0 = _rtt(rng, _caps(6))
    y, m, ch = AM.amen_mv(A, x, y0, z0, delta, sweeps=10, tol=delta * 1e-3)
    assert _err(y, full) <= delta * (1 + 1e-6)
    ref = Q.ranks(Q.tt_svd(full.reshape(DIMS), delta))
    assert all(a <= b + 1 for a, b in zip(Q.ranks(y), ref))


def test_rank_cap(problem):
    A, x, full, rng = problem
    y0 = _rtt(rng, _caps(4))
    z0 = _rtt(rng, _caps(4))
    y, _, _ = AM.amen_mv(A, x, y0, z0, 1e-12, cap=5, sweeps=6)
    assert max(Q.ranks(y)) <= 5
    # the best rank-5 approximation's error bounds it from below
    assert _err(y, full) >= _err(Q.tt_svd(full.reshape(DIMS), 0.0, 5), full) * 0.999


def test_identity_operator_rounds_the_train():
    """A = I: the product is x itself, truncated at delta within the bound."""
    rng = np.random.default_rng(7)
    x = _rtt(rng, _caps(6))
    I = [np.eye(d).reshape(1, d, d, 1).astype(np.complex128) for d in DIMS]
    y0 = _rtt(rng, _caps(2))
    z0 = _rtt(rng, _caps(4))
    xf = Q.tt_full(x).ravel()
    y, _, _ = AM.amen_mv(I, x, y0, z0, 1e-14, sweeps=8)
    assert _err(y, xf) < 1e-13
    y, _, _ = AM.amen_mv(I, x, y0, z0, 0.3, sweeps=8, tol=1e-6)
    assert _err(y, xf) <= 0.3


def test_planted_conjugation_slip_is_caught(problem, monkeypatch):
    """A plausible slip, the frame core not conjugated in the left
    interface, breaks the exact-product pin (complex cores)."""
    A, x, full, rng = problem
    y0 = _rtt(rng, _caps(64))
    z0 = _rtt(rng, _caps(4))

    def slip(PL, wk, Ak, xk):
        return np.einsum("aib,apc,pijq,cjd->bqd", wk, PL, Ak, xk, optimize=True)

    monkeypatch.setattr(AM, "_left_step", slip)
    y, _, _ = AM.amen_mv(A, x, y0, z0, 1e-14, sweeps=1)
    assert _err(y, full) > 1e-2
