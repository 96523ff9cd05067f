"""The adjoint Lippmann-Schwinger solve and the differentiable C_eff:
the GPU Jacobian dC_eff/d(lambda_p, mu_p) (C0 fixed) against the dense
oracle's energy identity, its dense adjoint, central finite differences of
GPU forward solves, and through torch.autograd."""
import numpy as np
import pytest

from oracle import dense as D
import microstructures as M

pytestmark = pytest.mark.gpu

q = pytest.importorskip("paper_2412_11566_amd")


@pytest.fixture(scope="module")
def sphere8():
    p = M.Problem("s8", 3, M.sphere(8, 0.3), [(1.0, 0.3), (6.0, 0.25)], cap=0, delta=1e-14, tol=1e-13)
    C, it, fields = D.effective_stiffness(p.phase, p.lame, p.lame0, tol=1e-13, keep_fields=True)
    ge = D.gradient_energy(p.phase, fields)
    return p, C, ge


def _exact_opts(tol=1e-12):
    return q.SolveOptions(delta=1e-14, tol=tol, cap=0, max_iter=400, exact=True)


def test_adjoint_untruncated_matches_oracle(ctx, sphere8):
    p, Cref, ge = sphere8
    opts = _exact_opts()
    prep = q.prepare(ctx, p.phase, p.lame, p.lame0, opts.delta)
    C, rep, eps = q.ls_solve_prepared(ctx, prep, opts, keep_eps=True)
    assert rep.status == 0
    assert np.abs(C - Cref).max() < 1e-10 * np.abs(Cref).max()
    J, arep = q.ls_adjoint_prepared(ctx, prep, opts, eps)
    assert arep.status == 0
    assert J.shape == (6, 6, 4)
    assert np.abs(J - ge).max() < 1e-9 * np.abs(ge).max()
    # the unprepared entry point gives the same Jacobian
    J2, _ = q.ls_adjoint(ctx, p.phase, p.lame, p.lame0, opts, eps)
    assert np.abs(J2 - J).max() < 1e-12 * np.abs(J).max()


def test_adjoint_matches_gpu_finite_differences(ctx, sphere8):
    p, _, _ = sphere8
    opts = _exact_opts()
    prep = q.prepare(ctx, p.phase, p.lame, p.lame0, opts.delta)
    _, _, eps = q.ls_solve_prepared(ctx, prep, opts, keep_eps=True)
    J, _ = q.ls_adjoint_prepared(ctx, prep, opts, eps)
    h = 1e-5
    for ph in range(2):
        for t in range(2):
            lp, lm = p.lame.copy(), p.lame.copy()
            d = h * p.lame[ph, t]
            lp[ph, t] += d
            lm[ph, t] -= d
            Cp, _, _ = q.ls_solve(ctx, p.phase, lp, p.lame0, opts)
            Cm, _, _ = q.ls_solve(ctx, p.phase, lm, p.lame0, opts)
            fd = (Cp - Cm) / (2 * d)
            assert np.abs(fd - J[:, :, 2 * ph + t]).max() < 1e-6 * np.abs(J).max()


def test_autograd_backward_is_adjoint(ctx, sphere8):
    import torch
    p, Cref, ge = sphere8
    opts = _exact_opts()
    lame = torch.tensor(p.lame, dtype=torch.float64, requires_grad=True)
    C = q.ceff(lame, p.phase, p.lame0, ctx, opts)
    assert np.abs(C.detach().numpy() - Cref).max() < 1e-10 * np.abs(Cref).max()
    W = torch.tensor(np.random.default_rng(3).standard_normal((6, 6)))
    (C * W).sum().backward()
    expect = np.einsum("kl,klt->t", W.numpy(), ge).reshape(2, 2)
    assert np.abs(lame.grad.numpy() - expect).max() < 1e-9 * np.abs(expect).max()


def test_adjoint_truncated_16(ctx):
    """16^3 sphere at delta 1e-8 with a non-binding cap: the Jacobian within
    1e-5 of the converged dense energy identity."""
    p = M.config_c0()
    C, it, fields = D.effective_stiffness(p.phase, p.lame, p.lame0, tol=1e-12, keep_fields=True)
    ge = D.gradient_energy(p.phase, fields)
    opts = q.SolveOptions(delta=1e-8, tol=1e-8, cap=128, max_iter=300)
    prep = q.prepare(ctx, p.phase, p.lame, p.lame0, opts.delta)
    Cg, rep, eps = q.ls_solve_prepared(ctx, prep, opts, keep_eps=True)
    J, arep = q.ls_adjoint_prepared(ctx, prep, opts, eps)
    assert arep.status == 0
    assert np.abs(J - ge).max() < 1e-5 * np.abs(ge).max()
    # symmetry of the Jacobian in (k, l) (energy identity)
    assert np.abs(J - np.swapaxes(J, 0, 1)).max() < 1e-5 * np.abs(J).max()


def _square(N, seed):
    rng = np.random.default_rng(seed)
    ph = (M.spheres(N, rng.uniform(0, 1, (3, 3)), np.array([0.22, 0.15, 0.1]))[:, :, 0]).astype(np.uint8)
    assert ph.max() == 1   # both phases present (the Jacobian has 4 columns)
    return ph


@pytest.mark.parametrize("scheme", ["direct", "staggered"])
def test_plane_adjoint_untruncated_matches_oracle(ctx, scheme):
    """Plane strain (Voigt 3) on a 16^2 pixel grid, untruncated: the
    Jacobian (3, 3, 4) against the plane oracle's energy identity, both
    entry points, and the cotangent form."""
    from oracle import plane as P2
    ph = _square(16, 5)
    lame = np.array([[1.0, 0.5], [6.0, 2.5]])
    l0 = M.reference_medium(lame)
    Cref, _, f = P2.effective_stiffness2(ph, lame, l0, tol=1e-13, max_iter=5000, scheme=scheme,
                                         keep_fields=True)
    ge = P2.gradient_energy2(ph, f)
    opts = _exact_opts()
    prep = q.prepare(ctx, ph, lame, l0, opts.delta, scheme=scheme)
    C, rep, eps = q.ls_solve_prepared(ctx, prep, opts, keep_eps=True)
    assert rep.status == 0 and C.shape == (3, 3)
    assert np.abs(C - Cref).max() < 1e-10 * np.abs(Cref).max()
    J, arep = q.ls_adjoint_prepared(ctx, prep, opts, eps)
    assert arep.status == 0
    assert J.shape == (3, 3, 4)
    assert np.abs(J - ge).max() < 1e-9 * np.abs(ge).max()
    J2, _ = q.ls_adjoint(ctx, ph, lame, l0, opts, eps, scheme=scheme)
    assert np.abs(J2 - J).max() < 1e-12 * np.abs(J).max()
    W = np.random.default_rng(4).standard_normal((3, 3))
    g, _ = q.ls_adjoint_prepared(ctx, prep, opts, eps, gbar=W)
    assert np.abs(g - np.einsum("kl,klt->t", W, J)).max() < 1e-12 * np.abs(J).max() * 9


def test_plane_autograd_and_mismatched_eps(ctx):
    """torch.autograd through a plane-strain C_eff (3, 3); the adjoint
    rejects strain trains of another problem (three-dimensional, or fewer
    than the three load cases)."""
    import torch
    from oracle import plane as P2
    ph = _square(16, 4)
    lame_np = np.array([[1.0, 0.5], [6.0, 2.5]])
    l0 = M.reference_medium(lame_np)
    _, _, f = P2.effective_stiffness2(ph, lame_np, l0, tol=1e-13, max_iter=5000, keep_fields=True)
    ge = P2.gradient_energy2(ph, f)
    opts = _exact_opts()
    lame = torch.tensor(lame_np, dtype=torch.float64, requires_grad=True)
    C = q.ceff(lame, ph, l0, ctx, opts)
    assert tuple(C.shape) == (3, 3)
    W = torch.tensor(np.random.default_rng(5).standard_normal((3, 3)))
    (C * W).sum().backward()
    expect = np.einsum("kl,klt->t", W.numpy(), ge).reshape(2, 2)
    assert np.abs(lame.grad.numpy() - expect).max() < 1e-9 * np.abs(expect).max()
    # strain trains of a 3D problem, and of a single load case
    p3 = M.Problem("s4", 2, M.sphere(4, 0.3), [(1.0, 0.3), (6.0, 0.25)], cap=0, delta=1e-14, tol=1e-13)
    _, _, e3 = q.ls_solve(ctx, p3.phase, p3.lame, p3.lame0, opts, keep_eps=True)
    prep = q.prepare(ctx, ph, lame_np, l0, opts.delta)
    with pytest.raises(q.QttError) as e:
        q.ls_adjoint_prepared(ctx, prep, opts, e3)
    assert e.value.code == q._c.QTT_EINVAL
    prep1 = q.prepare(ctx, ph, lame_np, l0, opts.delta, load_mask=0x1)
    _, _, e1 = q.ls_solve_prepared(ctx, prep1, opts, keep_eps=True)
    with pytest.raises(q.QttError) as e:
        q.ls_adjoint_prepared(ctx, prep, opts, e1)
    assert e.value.code == q._c.QTT_EINVAL


def test_plane_adjoint_truncated_64(ctx):
    """The 64^2 circle of the geometry suite at delta 1e-8 with a cap that
    does not bind: the Jacobian within 1e-5 of the converged plane
    oracle's energy identity, and symmetric in (k, l)."""
    from oracle import plane as P2
    lame = M.suite_lame()
    l0 = M.reference_medium(lame)
    ph = M.geometry("circle", 64, 2)
    _, _, f = P2.effective_stiffness2(ph, lame, l0, tol=1e-12, max_iter=5000, keep_fields=True)
    ge = P2.gradient_energy2(ph, f)
    opts = q.SolveOptions(delta=1e-8, tol=1e-8, cap=128, max_iter=300)
    prep = q.prepare(ctx, ph, lame, l0, opts.delta)
    _, rep, eps = q.ls_solve_prepared(ctx, prep, opts, keep_eps=True)
    J, arep = q.ls_adjoint_prepared(ctx, prep, opts, eps)
    assert rep.status == 0 and arep.status == 0
    assert np.abs(J - ge).max() < 1e-5 * np.abs(ge).max()
    assert np.abs(J - np.swapaxes(J, 0, 1)).max() < 1e-5 * np.abs(J).max()
