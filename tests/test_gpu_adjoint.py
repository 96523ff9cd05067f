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
