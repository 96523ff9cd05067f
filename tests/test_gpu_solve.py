"""GPU parity of ls_solve (Alg. 2) against the dense basic scheme (Alg. 1)."""
import numpy as np
import pytest

from oracle import dense as D
import microstructures as M
from tests.helpers import rel

pytestmark = pytest.mark.gpu

q = pytest.importorskip("paper_2412_11566_amd")


def test_same_iterations_untruncated_8(ctx):
    """Untruncated Alg. 2 equals Alg. 1 after the same number of updates."""
    p = M.Problem("s8", 3, M.sphere(8, 0.3), [(1.0, 0.3), (10.0, 0.3)], cap=0, delta=1e-14, tol=0)
    m = 6
    opts = q.SolveOptions(delta=1e-14, tol=0.0, cap=0, max_iter=m, exact=True)
    C, rep, _ = q.ls_solve(ctx, p.phase, p.lame, p.lame0, opts)
    Cref, _ = D.effective_stiffness(p.phase, p.lame, p.lame0, tol=0.0, fixed_iters=m)
    assert rep.iterations == [m] * 6
    assert rel(C, Cref) < 1e-10


def test_homogeneous_one_iteration(ctx):
    p = M.homogeneous(2, 3.0, 0.25)
    lame0 = (0.7, 0.9)
    opts = q.SolveOptions(delta=1e-12, tol=1e-12, cap=0, max_iter=5, exact=True)
    C, rep, _ = q.ls_solve(ctx, p.phase, p.lame, lame0, opts)
    from oracle.voigt import iso_voigt
    assert np.abs(C - iso_voigt(*p.lame[0])).max() < 1e-12 * np.abs(C).max()


def test_c0_exact_same_iterations(ctx):
    """16^3 sphere, untruncated FP64 path: 1e-10 relative to Alg. 1 after
    the same number of updates."""
    p = M.config_c0(exact=True)
    m = 8
    opts = q.SolveOptions(delta=1e-14, tol=0.0, cap=0, max_iter=m, exact=True)
    C, rep, _ = q.ls_solve(ctx, p.phase, p.lame, p.lame0, opts)
    Cref, _ = D.effective_stiffness(p.phase, p.lame, p.lame0, tol=0.0, fixed_iters=m)
    assert rel(C, Cref) < 1e-10


@pytest.mark.parametrize("orth", ["cholqr", "householder", "auto"])
def test_c0_delta_1e8(ctx, orth):
    """16^3 sphere at rounding tolerance 1e-8 with a cap that does not bind
    (128 = largest structural rank): C_eff within 1e-5 of the converged
    dense basic scheme; symmetric.  Both orthonormalisations of the range
    finder (CholeskyQR2 with Householder fallback, Householder only)."""
    p = M.config_c0()
    mode = {"cholqr": q.QTT_ORTH_CHOLQR, "householder": q.QTT_ORTH_HOUSEHOLDER, "auto": q.QTT_ORTH_AUTO}[orth]
    opts = q.SolveOptions(delta=1e-8, tol=1e-8, cap=128, max_iter=300, orth=mode)
    C, rep, _ = q.ls_solve(ctx, p.phase, p.lame, p.lame0, opts)
    Cref, it = D.effective_stiffness(p.phase, p.lame, p.lame0, tol=1e-12)
    assert rep.status == 0
    assert max(rep.iterations) <= 80
    assert rel(C, Cref) < 1e-5
    assert np.abs(C - C.T).max() < 1e-5 * np.abs(C).max()


def test_c0_split_bf16_contractions(ctx):
    """Split-BF16 contractions (hi + lo bf16 operands, FP32 accumulation;
    sketches, QR, SVD and residuals FP64) on the 16^3 sphere with a cap that
    does not bind.  A split-BF16 real product carries up to ~3 * 2^-16 =
    4.6e-5 relative error, so the relative update cannot fall much below
    1e-5 (the FP64 solve reaches 1e-8) and the solve runs to tol 1e-4; C_eff
    within 1e-4 of the converged dense scheme (about 1e-5 measured)."""
    p = M.config_c0()
    opts = q.SolveOptions(delta=1e-8, tol=1e-4, cap=128, max_iter=200, precision=q.QTT_PREC_BF16X3)
    C, rep, _ = q.ls_solve(ctx, p.phase, p.lame, p.lame0, opts)
    Cref, _ = D.effective_stiffness(p.phase, p.lame, p.lame0, tol=1e-12)
    assert rep.status == 0
    assert rel(C, Cref) < 1e-4
    assert np.abs(C - C.T).max() < 1e-4 * np.abs(C).max()


def test_c0_cap32_binding(ctx):
    """With the workload's cap 32 the cap binds (the converged strain needs
    rank ~96 for 1e-4): the loop stays bounded and C_eff is within the
    truncation level (a few 1e-3), not 1e-5."""
    p = M.config_c0()
    opts = q.SolveOptions(delta=p.delta, tol=p.tol, cap=32, max_iter=40)
    C, rep, _ = q.ls_solve(ctx, p.phase, p.lame, p.lame0, opts)
    Cref, _ = D.effective_stiffness(p.phase, p.lame, p.lame0, tol=1e-12)
    assert rep.max_rank <= 32
    assert max(rep.residual) < 0.1
    assert rel(C, Cref) < 1e-2


def test_c0_fp32_contractions(ctx):
    """FP32 contractions (FP64 sketches, QR, SVD and residuals): C_eff of the
    16^3 sphere within 1e-5 of the converged dense scheme at tol 1e-5 (the
    fixed point stalls near 1e-6 in FP32)."""
    p = M.config_c0()
    opts = q.SolveOptions(delta=1e-8, tol=1e-5, cap=128, max_iter=200, precision=q.QTT_PREC_FP32)
    C, rep, _ = q.ls_solve(ctx, p.phase, p.lame, p.lame0, opts)
    Cref, _ = D.effective_stiffness(p.phase, p.lame, p.lame0, tol=1e-12)
    assert rep.status == 0
    assert rel(C, Cref) < 1e-5


def test_concurrent_load_case_groups(ctx):
    """Load cases solved as 3 concurrent groups (own streams and pools),
    forward and adjoint: C_eff, the merged strain train (zero-padded ranks),
    the merged adjoint train and the gradient agree with the one-stream
    solve."""
    p = M.config_c0()
    prep = q.prepare(ctx, p.phase, p.lame, p.lame0, 1e-8)
    res = {}
    for ns in (1, 3):
        opts = q.SolveOptions(delta=1e-8, tol=1e-9, cap=128, max_iter=300, streams=ns, seed=3)
        C, rep, eps = q.ls_solve_prepared(ctx, prep, opts, keep_eps=True)
        assert rep.status == 0 and all(it > 0 for it in rep.iterations)
        g, arep = q.ls_adjoint_prepared(ctx, prep, q.SolveOptions(delta=1e-8, tol=1e-9, cap=128,
                                                                   max_iter=300, seed=4,
                                                                   streams=ns),
                                        eps, gbar=np.ones((6, 6)))
        assert arep.status == 0 and all(it > 0 for it in arep.iterations)
        res[ns] = (C, np.asarray(g))
    Cref, _ = D.effective_stiffness(p.phase, p.lame, p.lame0, tol=1e-12)
    assert rel(res[3][0], Cref) < 1e-5
    assert rel(res[3][0], res[1][0]) < 1e-6
    assert np.abs(res[3][1] - res[1][1]).max() < 1e-5 * np.abs(res[1][1]).max()


def test_kernel_statistics(ctx):
    """Sampled kernel statistics of a solve: every launch is counted, every
    s-th is timed (the matrix-core GEMM by its own real-time-counter span,
    also when the load cases run as concurrent groups), the durations are
    positive and below the solve's wall time, and reset clears them."""
    import time
    p = M.config_c0()
    prep = q.prepare(ctx, p.phase, p.lame, p.lame0, 1e-8)
    nfam = len(q._c.KERNEL_FAMILIES)
    mfma = q._c.QTT_K_MFMA
    for ns, stride in ((1, 1), (3, 4)):
        opts = q.SolveOptions(delta=1e-8, tol=1e-9, cap=128, max_iter=20, streams=ns, seed=3)
        q.stats_enable(ctx, stride)
        q.stats_reset(ctx)
        t = time.perf_counter()
        q.ls_solve_prepared(ctx, prep, opts)
        wall = time.perf_counter() - t
        timed = [q.stats_get(ctx, f) for f in range(nfam)]
        every = [q.stats_get_all(ctx, f) for f in range(nfam)]
        q.stats_enable(ctx, False)
        total_all = sum(a["launches"] for a in every)
        total_timed = sum(s["launches"] for s in timed)
        assert every[mfma]["launches"] > 0 and timed[mfma]["launches"] > 0
        assert timed[mfma]["seconds"] > 0.0
        if stride == 1:
            assert total_timed == total_all
        else:
            # one sampling counter per group, each starting at its group index
            assert abs(total_timed - total_all / stride) <= ns + 2
        for s, a in zip(timed, every):
            if s["launches"]:
                avg = s["seconds"] / s["launches"]
                assert 0.0 <= avg < wall, (s["family"], avg, wall)
                assert s["flops"] <= a["flops"] * (1 + 1e-12)
        q.stats_reset(ctx)
        assert q.stats_get(ctx, mfma)["launches"] == 0
        assert q.stats_get_all(ctx, mfma)["launches"] == 0
