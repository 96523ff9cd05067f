"""The staggered-grid Green operator (App. A, Table 3) on the device: the
four factors over the device-built train of the staggered directions
against the oracle's table (built from the discrete gradient and pinned
against the real-space difference operator), and Alg. 2 with it against
the dense basic scheme with the same operator: untruncated to rounding,
truncated at delta 1e-8 against the converged oracle C_eff, batched, and
the adjoint gradient against the oracle's energy identity."""
import json
import os

import numpy as np
import pytest

from oracle import dense as D, qtt as Q
import microstructures as M
from tests.helpers import dense, random_tt, rel

pytestmark = pytest.mark.gpu

q = pytest.importorskip("paper_2412_11566_amd")
HERE = os.path.dirname(os.path.abspath(__file__))


def _rand_strain(rng, n, r, batch=2):
    dims = [6] + [2] * (3 * n)
    L = len(dims)
    ranks = [1] + [min(r, int(np.prod(dims[:k])), int(np.prod(dims[k:]))) for k in range(1, L)] + [1]
    return random_tt(rng, dims, ranks, batch)


@pytest.mark.parametrize("n", [2, 3, 4])
def test_staggered_green_apply(ctx, n):
    """Every voxel of G x against the oracle's staggered table in the SFFT
    momentum order (exact sketch, rounding at 1e-14)."""
    N = 1 << n
    lam0, mu0 = 2.3, 1.4
    rng = np.random.default_rng(18)
    Gm = q.green_build(ctx, n, lam0, mu0, 1e-14, scheme="staggered")
    x = _rand_strain(rng, n, 6, batch=2)
    y = q.green_apply(ctx, Gm, q.tt_from_cores(ctx, x), delta=1e-14, seed=4, flags=4)
    Gt = Q.green_tensor(n, lam0, mu0, "staggered")
    for b in range(2):
        xd = dense(x, b).reshape(6, N, N, N)
        ref = np.einsum("vwxyz,wxyz->vxyz", Gt, xd)
        assert rel(dense(y.cores(), b).reshape(6, N, N, N), ref) < 1e-10
    # and the direct operator is a different one
    Gd = Q.green_tensor(n, lam0, mu0, "direct")
    xd = dense(x, 0).reshape(6, N, N, N)
    assert rel(dense(y.cores(), 0).reshape(6, N, N, N), np.einsum("vwxyz,wxyz->vxyz", Gd, xd)) > 1e-3


def test_staggered_exact_same_iterations(ctx):
    """16^3 sphere, untruncated: C_eff within 1e-10 of Alg. 1 with the
    staggered operator after the same number of updates."""
    p = M.config_c0(exact=True)
    m = 8
    opts = q.SolveOptions(delta=1e-14, tol=0.0, cap=0, max_iter=m, exact=True)
    C, rep, _ = q.ls_solve(ctx, p.phase, p.lame, p.lame0, opts, scheme="staggered")
    Cref, _ = D.effective_stiffness(p.phase, p.lame, p.lame0, tol=0.0, fixed_iters=m,
                                    scheme="staggered")
    assert rel(C, Cref) < 1e-10
    Cd, _ = D.effective_stiffness(p.phase, p.lame, p.lame0, tol=0.0, fixed_iters=m)
    assert rel(C, Cd) > 1e-4   # not the direct scheme's result


def test_staggered_c0_delta_1e8(ctx):
    """16^3 sphere at delta 1e-8 with a cap that does not bind: C_eff within
    1e-5 of the oracle's converged staggered C_eff (stored by
    tests/golden/make_golden.py c0stag); symmetric."""
    g = json.load(open(os.path.join(HERE, "golden", "ceff_c0stag.json")))
    Cref = np.array(g["ceff"]).reshape(6, 6)
    p = M.config_c0()
    opts = q.SolveOptions(delta=1e-8, tol=1e-8, cap=128, max_iter=300)
    C, rep, _ = q.ls_solve(ctx, p.phase, p.lame, p.lame0, opts, scheme="staggered")
    assert rep.status == 0
    assert rel(C, Cref) < 1e-5
    assert np.abs(C - C.T).max() < 1e-5 * np.abs(C).max()


def test_staggered_batch_matches_single(ctx):
    """Two 8^3 structures with different reference media in one batch, the
    staggered operator shared with per-structure scalars: each C_eff equals
    the oracle's staggered C_eff."""
    probs = []
    for s in range(2):
        ph = M.sphere(8, 0.25 + 0.05 * s).astype(np.uint8)
        lame = np.array([[1.0 + s, 0.5], [5.0, 3.0 + s]])
        probs.append((ph, lame, M.reference_medium(lame)))
    opts = q.SolveOptions(delta=1e-14, tol=1e-12, cap=0, max_iter=300, exact=True)
    Cb, reps = q.batch_solve(ctx, probs, opts, scheme="staggered")
    for (ph, lame, l0), Cs in zip(probs, Cb):
        Cref, _ = D.effective_stiffness(ph, lame, l0, tol=1e-13, scheme="staggered")
        assert rel(Cs, Cref) < 1e-10
    assert all(r.status == 0 for r in reps)


def test_staggered_adjoint_gradient(ctx):
    """dC_eff/d(lambda_p, mu_p) through the adjoint solve with the staggered
    operator (self-adjoint) against the oracle's energy identity on the
    converged staggered fields, 8^3 sphere, untruncated."""
    p = M.Problem("s8", 3, M.sphere(8, 0.3), [(1.0, 0.3), (6.0, 0.25)], cap=0, delta=1e-14, tol=1e-13)
    C, it, fields = D.effective_stiffness(p.phase, p.lame, p.lame0, tol=1e-13, keep_fields=True,
                                          scheme="staggered")
    ge = D.gradient_energy(p.phase, fields)
    opts = q.SolveOptions(delta=1e-14, tol=1e-12, cap=0, max_iter=400, exact=True)
    Cg, rep, eps = q.ls_solve(ctx, p.phase, p.lame, p.lame0, opts, keep_eps=True, scheme="staggered")
    assert rep.status == 0
    assert np.abs(Cg - C).max() < 1e-10 * np.abs(C).max()
    J, arep = q.ls_adjoint(ctx, p.phase, p.lame, p.lame0, opts, eps, scheme="staggered")
    assert arep.status == 0
    assert np.abs(J - ge).max() < 1e-9 * np.abs(ge).max()


def test_staggered_rejects_unknown_scheme(ctx):
    with pytest.raises(q.QttError) as e:
        q.green_build(ctx, 3, 1.0, 1.0, 1e-10, scheme=5)
    assert e.value.code == q._c.QTT_EINVAL
    p = M.config_c0()
    with pytest.raises(q.QttError) as e:
        q.ls_solve(ctx, p.phase, p.lame, p.lame0, q.SolveOptions(delta=1e-8, tol=1e-4, cap=32,
                                                                  max_iter=5), scheme=7)
    assert e.value.code == q._c.QTT_EINVAL
