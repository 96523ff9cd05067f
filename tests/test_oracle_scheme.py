"""Pins of the dense basic scheme (Alg. 1) and the effective stiffness."""
import numpy as np
import pytest

from oracle import bounds as B, dense as D
from oracle.voigt import iso_voigt
import microstructures as M


def test_homogeneous_returns_C_after_one_update():
    p = M.homogeneous(3, 2.0, 0.3)
    C, it = D.effective_stiffness(p.phase, p.lame, (0.6, 0.4), tol=1e-13)
    assert np.abs(C - iso_voigt(*p.lame[0])).max() < 1e-13
    assert it == [1] * 6


def test_laminate_closed_form_after_one_update():
    """Layers normal to x: analytic after one update (Sec. 5.2)."""
    p = M.config_c1_laminate(3)
    C, it = D.effective_stiffness(p.phase, p.lame, p.lame0, tol=1e-13)
    f = [p.volume_fraction(0), p.volume_fraction(1)]
    ref = B.laminate_x(B.iso_phases(p.lame), f)
    assert np.abs(C - ref).max() < 1e-12 * np.abs(ref).max()
    one, _ = D.effective_stiffness(p.phase, p.lame, p.lame0, tol=0, fixed_iters=1)
    assert np.abs(one - ref).max() < 1e-12 * np.abs(ref).max()


def test_laminate_formula_reduces_to_harmonic_and_arithmetic_means():
    """1D checks of the closed form: for a laminate of two isotropic phases
    C11 is the harmonic mean of (lam + 2 mu) and C44 (23 shear in the
    layer plane) the arithmetic mean of mu."""
    lame = np.array([[1.0, 0.5], [3.0, 2.0]])
    C = B.laminate_x(B.iso_phases(lame), [0.25, 0.75])
    m = lame[:, 0] + 2 * lame[:, 1]
    assert C[0, 0] == pytest.approx(1.0 / (0.25 / m[0] + 0.75 / m[1]))
    assert C[3, 3] == pytest.approx(0.25 * 0.5 + 0.75 * 2.0)
    assert C[5, 5] == pytest.approx(1.0 / (0.25 / 0.5 + 0.75 / 2.0))


@pytest.fixture(scope="module")
def sphere16():
    p = M.config_c0()
    C, it = D.effective_stiffness(p.phase, p.lame, p.lame0, tol=1e-10)
    return p, C, it


def test_sphere_symmetry_and_bounds(sphere16):
    p, C, it = sphere16
    assert np.abs(C - C.T).max() < 1e-10 * np.abs(C).max()
    f = [p.volume_fraction(0), p.volume_fraction(1)]
    Cs = B.iso_phases(p.lame)
    assert np.linalg.eigvalsh(B.voigt_bound(Cs, f) - C).min() > -1e-10
    assert np.linalg.eigvalsh(C - B.reuss_bound(Cs, f)).min() > -1e-10
    k1, m1 = B.bulk_shear(*p.lame[0])
    k2, m2 = B.bulk_shear(*p.lame[1])
    (klo, khi), _ = B.hashin_shtrikman(k1, m1, f[0], k2, m2, f[1])
    keff = (C[0, 0] + 2 * C[0, 1]) / 3
    assert klo <= keff <= khi


def test_sphere_permutation_symmetry(sphere16):
    """x, y, z permutations are symmetries of the centred sphere and of the
    Nyquist rule: C11 = C22 = C33, C12 = C13 = C23, C44 = C55 = C66."""
    _, C, _ = sphere16
    d = np.abs(C).max()
    assert max(abs(C[0, 0] - C[1, 1]), abs(C[0, 0] - C[2, 2])) < 1e-10 * d
    assert max(abs(C[0, 1] - C[0, 2]), abs(C[0, 1] - C[1, 2])) < 1e-10 * d
    assert max(abs(C[3, 3] - C[4, 4]), abs(C[3, 3] - C[5, 5])) < 1e-10 * d


def test_iterations_match_contrast(sphere16):
    """Contrast 10 at tol 1e-10: the basic scheme contracts at a rate near
    (contrast - 1)/(contrast + 1) ~ 0.82, i.e. tens of iterations."""
    _, _, it = sphere16
    assert 40 <= min(it) and max(it) <= 120


def test_hs_bounds_formula_limits():
    # equal phases collapse both bounds to the phase moduli
    (klo, khi), (mlo, mhi) = B.hashin_shtrikman(2.0, 1.0, 0.3, 2.0 + 1e-12, 1.0 + 1e-12, 0.7)
    assert klo == pytest.approx(2.0) and khi == pytest.approx(2.0)
    assert mlo == pytest.approx(1.0) and mhi == pytest.approx(1.0)


@pytest.mark.parametrize("scheme", ["direct", "staggered"])
def test_z_invariant_geometry_reduces_to_one_slice(scheme):
    """For a z-invariant microstructure only the xi_z = 0 modes carry energy,
    so Alg. 1 on the (N, N, 1) grid reproduces the (N, N, N) iterates and
    C_eff (used to compute the 256^3 fibre references)."""
    p = M.config_c2(3)
    C3, it3 = D.effective_stiffness(p.phase, p.lame, p.lame0, tol=1e-10, scheme=scheme)
    C1, it1 = D.effective_stiffness(p.phase[:, :, :1].copy(), p.lame, p.lame0, tol=1e-10,
                                    scheme=scheme)
    assert it3 == it1
    assert np.abs(C3 - C1).max() < 1e-12 * np.abs(C3).max()
