"""The gradient of the four-fibre workload as its configuration states it,
at 64^3 where the dense oracle is cheap: dC_eff/d(lambda, mu) of both
phases (C0 held fixed) from the GPU adjoint solve at the workload's own
rank cap 64 and rounding accuracy 1e-8, against

* the oracle's energy identity <eps^k : dC : eps^l> of the converged dense
  basic scheme,
* the oracle's central finite differences with relative step 1e-6,
* the oracle's dense adjoint fixed point,

and central finite differences of untruncated GPU forward solves (step
1e-6).  The fibres are z-invariant, so the oracle runs on the (64, 64, 1)
slice (iterates and averages unchanged, pinned in the oracle tests); on the
GPU the strain rank at 64^3 stays below 64, so the cap does not bind.
"""
import numpy as np
import pytest

from oracle import dense as D
import microstructures as M

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

q = pytest.importorskip("paper_2412_11566_amd")


@pytest.fixture(scope="module")
def fib64():
    p = M.config_c2(6)
    ph = p.phase[:, :, :1].copy()
    C, it, fields = D.effective_stiffness(ph, p.lame, p.lame0, tol=1e-13, keep_fields=True)
    ge = D.gradient_energy(ph, fields)
    gf = D.gradient_fd(ph, p.lame, p.lame0, tol=1e-13, rel_step=1e-6)
    return p, ph, C, fields, ge, gf


def _rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def test_gpu_gradient_64_fibres(ctx, fib64):
    p, ph, C, fields, ge, gf = fib64
    opts = q.SolveOptions(delta=1e-8, tol=1e-8, cap=64, max_iter=400, streams=3)
    prep = q.prepare(ctx, p.phase, p.lame, p.lame0, opts.delta)
    Cg, rep, eps = q.ls_solve_prepared(ctx, prep, opts, keep_eps=True)
    assert rep.status == 0 and rep.max_rank <= 64
    assert _rel(Cg, C) < 1e-6
    J, arep = q.ls_adjoint_prepared(ctx, prep, opts, eps)
    assert arep.status == 0
    assert J.shape == (6, 6, 4)
    assert _rel(J, ge) < 1e-5
    assert _rel(J, gf) < 1e-5
    # energy identity symmetry of the GPU Jacobian
    assert _rel(np.swapaxes(J, 0, 1), J) < 1e-5


@pytest.mark.parametrize("param", range(4), ids=["lam_matrix", "mu_matrix", "lam_fibre", "mu_fibre"])
def test_gpu_finite_differences_64_fibres(ctx, fib64, param):
    """Central differences (step 1e-6 relative) of GPU forward solves at
    rounding accuracy 1e-12 (the rank stays below the cap, so the sketch
    is exact up to rounding) against the oracle's energy-identity and
    finite-difference gradients, one modulus at a time."""
    p, ph, C, fields, ge, gf = fib64
    opts = q.SolveOptions(delta=1e-12, tol=1e-12, cap=64, max_iter=600, streams=3)
    ph_i, t = divmod(param, 2)
    lp, lm = p.lame.copy(), p.lame.copy()
    h = 1e-6 * p.lame[ph_i, t]
    lp[ph_i, t] += h
    lm[ph_i, t] -= h
    Cp, rp, _ = q.ls_solve(ctx, p.phase, lp, p.lame0, opts)
    Cm, rm, _ = q.ls_solve(ctx, p.phase, lm, p.lame0, opts)
    assert rp.status == 0 and rm.status == 0
    fd = (Cp - Cm) / (2 * h)
    scale = np.abs(ge).max()
    assert np.abs(fd - ge[:, :, param]).max() / scale < 1e-5
    assert np.abs(fd - gf[:, :, param]).max() / scale < 1e-5
