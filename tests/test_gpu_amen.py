"""The AMEn-adapted product (App. B) on the device against the oracle's
sweep from the same initial guesses (the seeded random trains are inputs
of both), and against the dense product A x: the SFFT operator (full
cores) and the raised stiffness operator (diagonal cores), exact and
truncated, batched, and the error paths."""
import numpy as np
import pytest

from oracle import amen as AM, qtt as Q
import microstructures as M
from tests.helpers import batch_element, dense, random_tt, rel

pytestmark = pytest.mark.gpu

q = pytest.importorskip("paper_2412_11566_amd")


def _dims(n):
    return [6] + [2] * (3 * n)


def _ranks(dims, r):
    L = len(dims)
    return [1] + [min(r, int(np.prod(dims[:k])), int(np.prod(dims[k:]))) for k in range(1, L)] + [1]


def _dense_product(A, xc):
    return Q.tto_full(A) @ Q.tt_full(xc).ravel()


@pytest.mark.parametrize("n,ry,rz", [(2, 3, 4), (2, 1, 8), (3, 4, 6)])
def test_amen_sfft_matches_oracle_and_dense(ctx, n, ry, rz):
    """SFFT x train: the device sweeps and the oracle's give the same
    product, equal to the dense A x, after the same number of sweeps."""
    rng = np.random.default_rng(30 + n + ry)
    dims = _dims(n)
    x = random_tt(rng, dims, _ranks(dims, 5), batch=1)
    y0 = random_tt(rng, dims, _ranks(dims, ry), batch=1)
    z0 = random_tt(rng, dims, _ranks(dims, rz), batch=1)
    S = q.sfft_build(ctx, n, 1e-14)
    y, m, ch = q.amen_apply(ctx, S, q.tt_from_cores(ctx, x), q.tt_from_cores(ctx, y0),
                            q.tt_from_cores(ctx, z0), 1e-12, sweeps=10)
    Sh = Q.sfft_3d(n, 1e-14)
    yo, mo, cho = AM.amen_mv(Sh, batch_element(x, 0), batch_element(y0, 0), batch_element(z0, 0),
                             1e-12, sweeps=10)
    full = _dense_product(Sh, batch_element(x, 0))
    got = dense(y.cores(), 0).ravel()
    assert rel(got, full) < 1e-10
    assert rel(got, Q.tt_full(yo).ravel()) < 1e-10
    assert m == mo
    assert y.ranks == Q.ranks(yo)


def test_amen_stiffness_diagonal_cores(ctx):
    """The raised stiffness operator (diagonal cores) of a 4^3 sphere."""
    n = 2
    rng = np.random.default_rng(41)
    phase = M.sphere(4, 0.3)
    lame = np.array([[1.0, 0.5], [4.0, 3.0]])
    lame0 = (2.5, 1.75)
    Cd, _ = q.from_voxels(ctx, phase, lame, lame0, 1e-14)
    dims = _dims(n)
    x = random_tt(rng, dims, _ranks(dims, 4), batch=2)
    y0 = random_tt(rng, dims, _ranks(dims, 2), batch=2)
    z0 = random_tt(rng, dims, _ranks(dims, 4), batch=2)
    y, m, ch = q.amen_apply(ctx, Cd, q.tt_from_cores(ctx, x), q.tt_from_cores(ctx, y0),
                            q.tt_from_cores(ctx, z0), 1e-12, sweeps=10)
    Ch = Q.stiffness_tto(phase, lame, lame0, 1e-14)
    for b in range(2):
        full = _dense_product(Ch, batch_element(x, b))
        assert rel(dense(y.cores(), b).ravel(), full) < 1e-10
    assert ch < 1e-12


@pytest.mark.parametrize("delta", [1e-3, 1e-6])
def test_amen_truncated_matches_oracle(ctx, delta):
    """Truncated at delta: the same ranks and the same product as the
    oracle's sweeps (to 1e-8), within the rounding bound of the dense
    product."""
    n = 3
    rng = np.random.default_rng(52)
    dims = _dims(n)
    # a train with a small second component: truncated at 1e-3, kept at 1e-6
    x1 = batch_element(random_tt(rng, dims, _ranks(dims, 3), batch=1), 0)
    x2 = batch_element(random_tt(rng, dims, _ranks(dims, 3), batch=1), 0)
    x = [c[None] for c in Q.tt_add(x1, Q.tt_scale(x2, 1e-4 * Q.tt_norm(x1) / Q.tt_norm(x2)))]
    y0 = random_tt(rng, dims, _ranks(dims, 3), batch=1)
    z0 = random_tt(rng, dims, _ranks(dims, 5), batch=1)
    S = q.sfft_build(ctx, n, 1e-14)
    y, m, _ = q.amen_apply(ctx, S, q.tt_from_cores(ctx, x), q.tt_from_cores(ctx, y0),
                           q.tt_from_cores(ctx, z0), delta, sweeps=8, tol=delta * 1e-3)
    Sh = Q.sfft_3d(n, 1e-14)
    yo, mo, _ = AM.amen_mv(Sh, batch_element(x, 0), batch_element(y0, 0), batch_element(z0, 0),
                           delta, sweeps=8, tol=delta * 1e-3)
    full = _dense_product(Sh, batch_element(x, 0))
    got = dense(y.cores(), 0).ravel()
    assert y.ranks == Q.ranks(yo)
    assert rel(got, Q.tt_full(yo).ravel()) < 1e-8
    assert rel(got, full) <= delta * (1 + 1e-6)


def test_amen_cap(ctx):
    n = 2
    rng = np.random.default_rng(61)
    dims = _dims(n)
    x = random_tt(rng, dims, _ranks(dims, 6), batch=1)
    y0 = random_tt(rng, dims, _ranks(dims, 2), batch=1)
    z0 = random_tt(rng, dims, _ranks(dims, 4), batch=1)
    S = q.sfft_build(ctx, n, 1e-14)
    y, _, _ = q.amen_apply(ctx, S, q.tt_from_cores(ctx, x), q.tt_from_cores(ctx, y0),
                           q.tt_from_cores(ctx, z0), 1e-12, cap=5, sweeps=6)
    assert max(y.ranks) <= 5
    Sh = Q.sfft_3d(n, 1e-14)
    yo, _, _ = AM.amen_mv(Sh, batch_element(x, 0), batch_element(y0, 0), batch_element(z0, 0),
                          1e-12, cap=5, sweeps=6)
    assert rel(dense(y.cores(), 0).ravel(), Q.tt_full(yo).ravel()) < 1e-8


def test_amen_rejects(ctx):
    n = 2
    rng = np.random.default_rng(3)
    dims = _dims(n)
    x = q.tt_from_cores(ctx, random_tt(rng, dims, _ranks(dims, 3), batch=1))
    y0 = q.tt_from_cores(ctx, random_tt(rng, dims, _ranks(dims, 3), batch=1))
    z0 = q.tt_from_cores(ctx, random_tt(rng, dims, _ranks(dims, 3), batch=1))
    G = q.green_build(ctx, n, 1.0, 1.0, 1e-12)
    with pytest.raises(q.QttError) as e:
        q.amen_apply(ctx, G, x, y0, z0, 1e-10)
    assert e.value.code == q._c.QTT_EINVAL
    S = q.sfft_build(ctx, n, 1e-12)
    zb = q.tt_from_cores(ctx, random_tt(rng, dims, _ranks(dims, 3), batch=2))
    with pytest.raises(q.QttError) as e:
        q.amen_apply(ctx, S, x, y0, zb, 1e-10)
    assert e.value.code == q._c.QTT_EINVAL
    with pytest.raises(q.QttError):
        q.amen_apply(ctx, S, x, y0, z0, 1e-10, sweeps=0)


def test_solve_with_amen_green_products(ctx):
    """Alg. 2 with the Green step's products by AMEn (App. B), warm-started
    per factor: the 16^3 sphere at delta 1e-8 with a cap that does not bind
    reaches the converged dense C_eff to 1e-5, like the sketch."""
    from oracle import dense as D
    p = M.config_c0()
    opts = q.SolveOptions(delta=1e-8, tol=1e-8, cap=128, max_iter=300, matvec=q.QTT_MV_AMEN)
    C, rep, _ = q.ls_solve(ctx, p.phase, p.lame, p.lame0, opts)
    Cref, _ = D.effective_stiffness(p.phase, p.lame, p.lame0, tol=1e-12)
    assert rep.status == 0
    assert max(rep.iterations) <= 80
    assert rel(C, Cref) < 1e-5
    assert np.abs(C - C.T).max() < 1e-5 * np.abs(C).max()


def test_solve_rejects_unknown_matvec(ctx):
    p = M.config_c0()
    with pytest.raises(q.QttError) as e:
        q.ls_solve(ctx, p.phase, p.lame, p.lame0,
                   q.SolveOptions(delta=1e-8, tol=1e-4, cap=32, max_iter=5, matvec=9))
    assert e.value.code == q._c.QTT_EINVAL


def test_solve_amen_with_staggered_and_plane(ctx):
    """The AMEn Green products with the staggered-grid factors (16^3
    sphere against the oracle's staggered golden) and with the plane-strain
    factors (64^2 circle against the plane-strain oracle), delta 1e-8."""
    import json
    import os
    from oracle import plane as P2
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "ceff_c0stag.json")))
    p = M.config_c0()
    opts = q.SolveOptions(delta=1e-8, tol=1e-8, cap=128, max_iter=300, matvec=q.QTT_MV_AMEN)
    C, rep, _ = q.ls_solve(ctx, p.phase, p.lame, p.lame0, opts, scheme="staggered")
    assert rep.status == 0
    assert rel(C, np.array(g["ceff"]).reshape(6, 6)) < 1e-5
    lame = M.suite_lame()
    l0 = M.reference_medium(lame)
    ph = M.geometry("circle", 64, 2)
    C2, rep2, _ = q.ls_solve(ctx, ph, lame, l0, opts, load_mask=0x7)
    Cref, _ = P2.effective_stiffness2(ph, lame, l0, tol=1e-12, max_iter=5000)
    assert rep2.status == 0
    assert rel(C2, Cref) < 1e-5
