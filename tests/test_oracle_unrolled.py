"""Pins of ``oracle.unrolled``: the derivative of the C_eff after exactly
M updates against central differences of the fixed-count dense solve (a
polynomial in the moduli, so the differences are accurate), its C_M
against that solve, and the converged limit (the energy identity)."""
import numpy as np
import pytest

from oracle import dense as D, plane as P2, unrolled as U
import microstructures as M


def _sphere():
    p = M.Problem("s8", 3, M.sphere(8, 0.3), [(1.0, 0.3), (6.0, 0.25)], cap=0, delta=1e-14, tol=1e-13)
    return p.phase, np.asarray(p.lame), p.lame0


def _fd(phase, lame, lame0, steps, scheme, h=1e-5):
    lame = np.asarray(lame, dtype=np.float64)
    out = []
    for p in range(lame.shape[0]):
        for t in range(2):
            d = h * lame[p, t]
            lp, lm = lame.copy(), lame.copy()
            lp[p, t] += d
            lm[p, t] -= d
            if phase.ndim == 3:
                Cp, _ = D.effective_stiffness(phase, lp, lame0, tol=0, fixed_iters=steps, scheme=scheme)
                Cm, _ = D.effective_stiffness(phase, lm, lame0, tol=0, fixed_iters=steps, scheme=scheme)
            else:
                Cp, _ = P2.effective_stiffness2(phase, lp, lame0, tol=0, fixed_iters=steps, scheme=scheme)
                Cm, _ = P2.effective_stiffness2(phase, lm, lame0, tol=0, fixed_iters=steps, scheme=scheme)
            out.append((Cp - Cm) / (2 * d))
    return np.stack(out, axis=-1)


@pytest.mark.parametrize("steps,scheme", [(1, "direct"), (4, "direct"), (3, "staggered")])
def test_unrolled_matches_finite_differences_3d(steps, scheme):
    ph, lame, l0 = _sphere()
    C, J = U.unrolled_gradient(ph, lame, l0, steps, scheme)
    Cref, _ = D.effective_stiffness(ph, lame, l0, tol=0, fixed_iters=steps, scheme=scheme)
    assert np.abs(C - Cref).max() < 1e-13 * np.abs(Cref).max()
    fd = _fd(ph, lame, l0, steps, scheme)
    assert np.abs(J - fd).max() < 1e-8 * np.abs(J).max()


def test_unrolled_matches_finite_differences_plane():
    rng = np.random.default_rng(4)
    ph = (M.spheres(16, rng.uniform(0, 1, (3, 3)), np.array([0.22, 0.15, 0.1]))[:, :, 0]).astype(np.uint8)
    lame = np.array([[1.0, 0.5], [6.0, 2.5]])
    l0 = M.reference_medium(lame)
    C, J = U.unrolled_gradient(ph, lame, l0, 5)
    Cref, _ = P2.effective_stiffness2(ph, lame, l0, tol=0, fixed_iters=5)
    assert np.abs(C - Cref).max() < 1e-13 * np.abs(Cref).max()
    assert np.abs(J - _fd(ph, lame, l0, 5, "direct")).max() < 1e-8 * np.abs(J).max()


def test_unrolled_reaches_the_converged_gradient():
    """Many updates: the unrolled derivative tends to the energy identity
    of the converged fixed point."""
    ph, lame, l0 = _sphere()
    _, _, f = D.effective_stiffness(ph, lame, l0, tol=1e-14, keep_fields=True)
    ge = D.gradient_energy(ph, f)
    _, J = U.unrolled_gradient(ph, lame, l0, 60)
    assert np.abs(J - ge).max() < 1e-10 * np.abs(ge).max()
    _, J3 = U.unrolled_gradient(ph, lame, l0, 3)
    assert np.abs(J3 - ge).max() > 1e-4 * np.abs(ge).max()   # not yet at the limit


def test_planted_missing_explicit_term_is_caught(monkeypatch):
    """A plausible slip, the last iterate's explicit term dropped, fails the
    finite-difference pin."""
    ph, lame, l0 = _sphere()
    real = U._dlocal
    calls = {"n": 0}

    def skip_first(Dt, phase, p, f):
        calls["n"] += 1
        out = real(Dt, phase, p, f)
        return out * 0 if calls["n"] <= 6 * 4 else out

    monkeypatch.setattr(U, "_dlocal", skip_first)
    _, J = U.unrolled_gradient(ph, lame, l0, 2)
    monkeypatch.undo()
    assert np.abs(J - _fd(ph, lame, l0, 2, "direct")).max() > 1e-3 * np.abs(J).max()
