"""Pins of the Hashin-Shtrikman bounds in ``oracle.bounds`` (the bound
checks of the effective stiffness).

Each pin comes from a source other than the formula it checks:

* Walpole's form of the same bounds (Walpole 1966): with reference phase a,
  K = [sum_i f_i / (k_i + 4 mu_a / 3)]^-1 - 4 mu_a / 3 and
  G = [sum_i f_i / (mu_i + z_a)]^-1 - z_a, z_a = mu_a (9 k_a + 8 mu_a) / (6 (k_a + 2 mu_a)).
* Eshelby's dilute-sphere result written with the matrix Poisson ratio nu:
  dk/df = (k_b - k_a) / (1 + alpha (k_b - k_a) / k_a), alpha = (1 + nu) / (3 (1 - nu));
  dmu/df = (mu_b - mu_a) / (1 + beta (mu_b - mu_a) / mu_a), beta = 2 (4 - 5 nu) / (15 (1 - nu)).
  The bound whose reference phase is the matrix has exactly these slopes at f_b = 0.
* Hashin's coated-sphere assemblage, which attains the bulk bound whose
  reference phase is the coating: the radial elasticity problem of one
  coated sphere under a hydrostatic boundary displacement, solved here as a
  3x3 linear system.
* The ordering Reuss <= lower <= upper <= Voigt for well-ordered phases.
"""
import numpy as np
import pytest

from oracle import bounds as B


def _walpole(ka, ma, phases):
    """Bounds in Walpole's form for reference phase (ka, ma); phases: list
    of (k, mu, f)."""
    c = 4.0 * ma / 3.0
    z = ma * (9.0 * ka + 8.0 * ma) / (6.0 * (ka + 2.0 * ma))
    K = 1.0 / sum(f / (k + c) for k, _, f in phases) - c
    G = 1.0 / sum(f / (m + z) for _, m, f in phases) - z
    return K, G


def _phase_pairs(count=200, seed=11):
    rng = np.random.default_rng(seed)
    for _ in range(count):
        E1, E2 = np.sort(rng.uniform(0.1, 100.0, 2))
        nu1, nu2 = rng.uniform(-0.5, 0.49, 2)
        f1 = rng.uniform(0.01, 0.99)
        k1, m1 = E1 / (3 * (1 - 2 * nu1)), E1 / (2 * (1 + nu1))
        k2, m2 = E2 / (3 * (1 - 2 * nu2)), E2 / (2 * (1 + nu2))
        if not (k1 <= k2 and m1 <= m2):
            continue  # well-ordered pairs only: the bounds then bracket
        yield k1, m1, f1, k2, m2, 1.0 - f1


def test_hs_equals_walpole_form():
    """Both bounds agree with Walpole's form on random well-ordered phase
    pairs (the soft phase is the reference of the lower bound)."""
    n = 0
    for k1, m1, f1, k2, m2, f2 in _phase_pairs():
        (klo, khi), (mlo, mhi) = B.hashin_shtrikman(k1, m1, f1, k2, m2, f2)
        ph = [(k1, m1, f1), (k2, m2, f2)]
        Klo, Glo = _walpole(k1, m1, ph)
        Khi, Ghi = _walpole(k2, m2, ph)
        assert klo == pytest.approx(Klo, rel=1e-12) and khi == pytest.approx(Khi, rel=1e-12)
        assert mlo == pytest.approx(Glo, rel=1e-12) and mhi == pytest.approx(Ghi, rel=1e-12)
        # the argument order of the phases does not matter
        (a, b), (c, d) = B.hashin_shtrikman(k2, m2, f2, k1, m1, f1)
        assert (a, b, c, d) == pytest.approx((klo, khi, mlo, mhi), rel=1e-12)
        n += 1
    assert n > 40


def test_hs_dilute_slopes_are_eshelby():
    """At f_b -> 0 the bound referenced on the matrix (phase a) has
    Eshelby's dilute-sphere slopes (written with the matrix Poisson ratio)."""
    for E_a, nu_a, E_b, nu_b in ((1.0, 0.3, 10.0, 0.3), (1.0, 0.35, 20.0, 0.25),
                                 (5.0, 0.2, 0.5, 0.4), (2.0, -0.2, 30.0, 0.1)):
        ka, ma = E_a / (3 * (1 - 2 * nu_a)), E_a / (2 * (1 + nu_a))
        kb, mb = E_b / (3 * (1 - 2 * nu_b)), E_b / (2 * (1 + nu_b))
        h = 1e-7
        (klo, khi), (mlo, mhi) = B.hashin_shtrikman(ka, ma, 1.0 - h, kb, mb, h)
        # the matrix is the reference of the lower bound when it is softer
        soft_matrix = ka <= kb and ma <= mb
        kk, mm = (klo, mlo) if soft_matrix else (khi, mhi)
        alpha = (1 + nu_a) / (3 * (1 - nu_a))
        beta = 2 * (4 - 5 * nu_a) / (15 * (1 - nu_a))
        dk = (kb - ka) / (1 + alpha * (kb - ka) / ka)
        dm = (mb - ma) / (1 + beta * (mb - ma) / ma)
        assert (kk - ka) / h == pytest.approx(dk, rel=1e-5)
        assert (mm - ma) / h == pytest.approx(dm, rel=1e-5)


def _coated_sphere_bulk(k_core, m_core, k_coat, m_coat, f_core):
    """Effective bulk modulus of a coated sphere (core radius a = f^(1/3),
    coating to radius 1) under u(1) = e r: radial fields u = A r (core),
    u = B r + C / r^2 (coating), with sigma_rr = 3 k A (core) and
    3 k B - 4 mu C / r^3 (coating).  Continuity of u and sigma_rr at r = a
    and u(1) = e give A, B, C; k_eff = sigma_rr(1) / (3 e)."""
    a = f_core ** (1.0 / 3.0)
    e = 1.0
    M = np.array([[a, -a, -1.0 / a ** 2],
                  [3 * k_core, -3 * k_coat, 4 * m_coat / a ** 3],
                  [0.0, 1.0, 1.0]])
    A, Bc, Cc = np.linalg.solve(M, [0.0, 0.0, e])
    return (3 * k_coat * Bc - 4 * m_coat * Cc) / (3 * e)


def test_hs_bulk_attained_by_coated_spheres():
    for k1, m1, f1, k2, m2, f2 in _phase_pairs(60, seed=5):
        (klo, khi), _ = B.hashin_shtrikman(k1, m1, f1, k2, m2, f2)
        # soft coating around stiff cores: the lower bound; and the reverse
        assert klo == pytest.approx(_coated_sphere_bulk(k2, m2, k1, m1, f2), rel=1e-10)
        assert khi == pytest.approx(_coated_sphere_bulk(k1, m1, k2, m2, f1), rel=1e-10)


def test_hs_inside_voigt_reuss():
    for k1, m1, f1, k2, m2, f2 in _phase_pairs():
        (klo, khi), (mlo, mhi) = B.hashin_shtrikman(k1, m1, f1, k2, m2, f2)
        kV, kR = f1 * k1 + f2 * k2, 1.0 / (f1 / k1 + f2 / k2)
        mV, mR = f1 * m1 + f2 * m2, 1.0 / (f1 / m1 + f2 / m2)
        t = 1e-12
        assert kR * (1 - t) <= klo <= khi * (1 + t) and khi <= kV * (1 + t)
        assert mR * (1 - t) <= mlo <= mhi * (1 + t) and mhi <= mV * (1 + t)


def test_hs_planted_coefficient_error_is_caught():
    """A plausible slip in the shear formula (6 -> 5 in the f_a term) keeps
    the equal-phase limit but fails Walpole's form."""
    def bad_mbound(ka, ma, fa, kb, mb, fb):
        return ma + fb / (1.0 / (mb - ma) + 5.0 * fa * (ka + 2.0 * ma) / (5.0 * ma * (3.0 * ka + 4.0 * ma)))
    k1, m1, f1, k2, m2, f2 = next(iter(_phase_pairs()))
    _, G = _walpole(k1, m1, [(k1, m1, f1), (k2, m2, f2)])
    assert abs(bad_mbound(k1, m1, f1, k2, m2, f2) - G) > 1e-6 * abs(G)


def test_voigt_reuss_matrices_of_isotropic_phases():
    """The matrix bounds of oracle.bounds on isotropic phases are isotropic
    with the arithmetic (Voigt) and harmonic (Reuss) means of the bulk and
    shear moduli taken separately (the isotropic stiffness acts as 3 kappa
    and 2 mu on its two eigenspaces)."""
    from oracle.voigt import iso_voigt
    rng = np.random.default_rng(2)
    for _ in range(20):
        lam = rng.uniform(0.1, 5.0, 3)
        mu = rng.uniform(0.1, 5.0, 3)
        f = rng.dirichlet(np.ones(3))
        Cs = np.stack([iso_voigt(l, m) for l, m in zip(lam, mu)])
        k = lam + 2 * mu / 3
        kV, mV = f @ k, f @ mu
        kR, mR = 1 / (f @ (1 / k)), 1 / (f @ (1 / mu))
        assert np.allclose(B.voigt_bound(Cs, f), iso_voigt(kV - 2 * mV / 3, mV), rtol=1e-12, atol=1e-12)
        assert np.allclose(B.reuss_bound(Cs, f), iso_voigt(kR - 2 * mR / 3, mR), rtol=1e-12, atol=1e-12)
