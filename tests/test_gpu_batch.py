"""Many structures solved together (one train batch of 6 load cases per
structure, one stiffness-operator instance per structure, shared SFFT and
Green factors): against single solves and the dense oracle."""
import numpy as np
import pytest

from oracle import dense as D
import microstructures as M
from tests.helpers import rel

pytestmark = pytest.mark.gpu

q = pytest.importorskip("paper_2412_11566_amd")


def _structures8():
    lj = lambda E, nu: M.lame_from_young(E, nu)
    out = []
    for ph, mods in ((M.sphere(8, 0.3), [(1.0, 0.3), (10.0, 0.3)]),
                     (M.sphere(8, 0.2, centre=(0.3, 0.6, 0.5)), [(1.0, 0.3), (5.0, 0.2)]),
                     (M.laminate(8, 1, 0.5), [(1.0, 0.3), (20.0, 0.25)])):
        lame = np.array([lj(E, nu) for E, nu in mods])
        out.append((ph, lame, M.reference_medium(lame)))
    return out


def test_batch_exact_equals_single_and_oracle(ctx):
    m = 5
    opts = q.SolveOptions(delta=1e-14, tol=0.0, cap=0, max_iter=m, exact=True)
    probs = _structures8()
    Cb, reps = q.batch_solve(ctx, probs, opts)
    for (ph, lame, lame0), C, rep in zip(probs, Cb, reps):
        Cs, _, _ = q.ls_solve(ctx, ph, lame, lame0, opts)
        Co, _ = D.effective_stiffness(ph, lame, lame0, tol=0.0, fixed_iters=m)
        assert rep.iterations == [m] * 6
        assert rel(C, Cs) < 1e-10
        assert rel(C, Co) < 1e-10


def test_batch_truncated_16(ctx):
    """Four 16^3 structures at delta 1e-8 (non-binding cap): each C_eff
    within 1e-5 of the converged dense scheme."""
    rng = np.random.default_rng(5)
    probs = []
    p0 = M.config_c0()
    probs.append((p0.phase, p0.lame, p0.lame0))
    for i in range(3):
        cs, rad = M.random_spheres(rng, 2 + i, 0.1, 0.2)
        ph = M.spheres(16, cs, rad).astype(np.uint8)
        lame = np.array([M.lame_from_young(1.0, 0.3), M.lame_from_young(4.0 + 3 * i, 0.25)])
        probs.append((ph, lame, M.reference_medium(lame)))
    opts = q.SolveOptions(delta=1e-8, tol=1e-8, cap=128, max_iter=300)
    Cb, reps = q.batch_solve(ctx, probs, opts)
    for (ph, lame, lame0), C, rep in zip(probs, Cb, reps):
        Co, _ = D.effective_stiffness(ph, lame, lame0, tol=1e-12)
        assert rep.status == 0
        assert rel(C, Co) < 1e-5


def test_batch_mixed_sizes_and_masks(ctx):
    """Grouping by grid size and the single-solve path for partial load
    masks give the same results as individual solves."""
    opts = q.SolveOptions(delta=1e-14, tol=0.0, cap=0, max_iter=3, exact=True)
    p16 = M.config_c0()
    probs = _structures8()[:2] + [(p16.phase, p16.lame, p16.lame0)]
    Cb, reps = q.batch_solve(ctx, probs, opts)
    for (ph, lame, lame0), C in zip(probs, Cb):
        Cs, _, _ = q.ls_solve(ctx, ph, lame, lame0, opts)
        assert rel(C, Cs) < 1e-10


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batch_random_spheres_16(ctx, prec):
    """The batched workload's random-sphere recipe on 16^3 (cap = largest
    structural rank, delta 1e-7, tol 1e-5), batched with FP64 or FP32
    contractions: each C_eff within 1e-5 of the converged dense scheme."""
    ps = [M.config_c3_structure(i, grid_n=4) for i in range(4)]
    opts = q.SolveOptions(delta=1e-7, tol=1e-5, cap=ps[0].cap, max_iter=400,
                          precision=q.QTT_PREC_FP32 if prec == "fp32" else q.QTT_PREC_FP64)
    Cb, reps = q.batch_solve(ctx, [(p.phase, p.lame, p.lame0) for p in ps], opts)
    for p, C, rep in zip(ps, Cb, reps):
        Co, _ = D.effective_stiffness(p.phase, p.lame, p.lame0, tol=1e-10)
        assert rep.status == 0
        assert rel(C, Co) < 1e-5


def test_batch_rank_buckets(ctx):
    """Rank buckets (the geometry rank of Sec. 5.2) split the 16^3 and 8^3
    structures into batches of alike ranks: every C_eff equals the
    unbucketed batch's and the oracle's (exact sketch, fixed updates)."""
    m = 4
    opts = q.SolveOptions(delta=1e-14, tol=0.0, cap=0, max_iter=m, exact=True)
    probs = list(_structures8())
    p0 = M.config_c0()
    probs.append((p0.phase, p0.lame, p0.lame0))
    lam = M.laminate(16).astype(np.uint8)
    probs.append((lam, p0.lame, p0.lame0))
    Cb, _ = q.batch_solve(ctx, probs, opts)
    ob = q.SolveOptions(delta=1e-14, tol=0.0, cap=0, max_iter=m, exact=True, rank_buckets=True)
    Ck, reps = q.batch_solve(ctx, probs, ob)
    for (ph, lame, lame0), C1, C2, rep in zip(probs, Cb, Ck, reps):
        Co, _ = D.effective_stiffness(ph, lame, lame0, tol=0.0, fixed_iters=m)
        assert rep.iterations == [m] * 6
        assert rel(C2, C1) < 1e-10
        assert rel(C2, Co) < 1e-10
