"""Pins of the plane-strain oracle (``oracle.plane``) against the
three-dimensional one on z-invariant grids: only xi_z = 0 modes exist on an
(N, N, 1) grid, where the 3D direct Green operator's in-plane block is the
plane-strain operator, and in-plane loads leave the out-of-plane
displacement at zero for isotropic phases, so the in-plane block of the 3D
C_eff is the plane-strain C_eff."""
import numpy as np

from oracle import bounds as B, dense as D, plane as P2
from oracle.voigt import iso_voigt
import microstructures as M

IN = [0, 1, 5]   # Voigt 11, 22, 12 among (11, 22, 33, 23, 13, 12)


def test_plane_stiffness_is_the_3d_in_plane_block():
    for lam, mu in ((1.0, 0.5), (7.0, 2.0)):
        assert np.array_equal(P2.iso_voigt2(lam, mu), iso_voigt(lam, mu)[np.ix_(IN, IN)])


def test_green_table_is_the_3d_in_plane_block():
    N = 8
    G2 = P2.gamma_table2(N, 1.3, 0.7)
    G3 = D.gamma_table((N, N, 1), 1.3, 0.7)[:, :, :, :, 0]
    assert np.abs(G2 - G3[np.ix_(IN, IN)]).max() < 1e-14


def test_effective_stiffness_equals_3d_on_a_z_invariant_grid():
    rng = np.random.default_rng(3)
    ph = (M.spheres(16, rng.uniform(0, 1, (3, 3)), np.array([0.2, 0.15, 0.1]))[:, :, 0]).astype(np.uint8)
    lame = np.array([[1.0, 0.5], [6.0, 2.5]])
    l0 = M.reference_medium(lame)
    C2, it2 = P2.effective_stiffness2(ph, lame, l0, tol=1e-12)
    C3, it3 = D.effective_stiffness(ph[:, :, None].copy(), lame, l0, tol=1e-12)
    assert np.abs(C2 - C3[np.ix_(IN, IN)]).max() < 1e-11 * np.abs(C2).max()
    assert it2 == [it3[i] for i in IN]


def test_plane_laminate_closed_form_after_one_update():
    lam = M.laminate(16)[:, :, 0].astype(np.uint8)
    lame = np.array([[1.0, 0.5], [6.0, 2.5]])
    f = [np.mean(lam == 0), np.mean(lam == 1)]
    ref = B.laminate_x(B.iso_phases(lame), f)[np.ix_(IN, IN)]
    C, _ = P2.effective_stiffness2(lam, lame, M.reference_medium(lame), tol=0, fixed_iters=1)
    assert np.abs(C - ref).max() < 1e-12 * np.abs(ref).max()


def test_homogeneous_after_one_update():
    ph = np.zeros((8, 8), np.uint8)
    C, it = P2.effective_stiffness2(ph, np.array([[2.0, 1.0]]), (1.0, 0.8), tol=1e-13)
    assert np.abs(C - P2.iso_voigt2(2.0, 1.0)).max() < 1e-13 and it == [1, 1, 1]


def test_staggered_plane_is_the_3d_in_plane_block():
    """The plane staggered table and C_eff equal the 3D staggered ones'
    in-plane blocks on an (N, N, 1) grid (q_z = 0: both difference symbols
    of z vanish and u_3 decouples)."""
    N = 8
    G2 = P2.gamma_table2_staggered(N, 1.3, 0.7)
    G3 = D.gamma_table_staggered((N, N, 1), 1.3, 0.7)[:, :, :, :, 0]
    assert np.abs(G2 - G3[np.ix_(IN, IN)]).max() < 1e-14
    rng = np.random.default_rng(4)
    ph = (M.spheres(16, rng.uniform(0, 1, (2, 3)), np.array([0.2, 0.15]))[:, :, 0]).astype(np.uint8)
    lame = np.array([[1.0, 0.5], [6.0, 2.5]])
    l0 = M.reference_medium(lame)
    C2, it2 = P2.effective_stiffness2(ph, lame, l0, tol=1e-12, scheme="staggered")
    C3, it3 = D.effective_stiffness(ph[:, :, None].copy(), lame, l0, tol=1e-12, scheme="staggered")
    assert np.abs(C2 - C3[np.ix_(IN, IN)]).max() < 1e-11 * np.abs(C2).max()
    assert it2 == [it3[i] for i in IN]


def _two_phase_square(N, seed):
    rng = np.random.default_rng(seed)
    return (M.spheres(N, rng.uniform(0, 1, (3, 3)), np.array([0.22, 0.15, 0.1]))[:, :, 0]).astype(np.uint8)


def test_plane_gradient_energy_identity_matches_finite_differences():
    """The energy identity of the plane-strain C_eff against central
    differences of forward solves (both schemes)."""
    ph = _two_phase_square(16, 5)
    lame = np.array([[1.0, 0.5], [6.0, 2.5]])
    l0 = M.reference_medium(lame)
    for scheme in ("direct", "staggered"):
        C, _, f = P2.effective_stiffness2(ph, lame, l0, tol=1e-13, max_iter=5000, scheme=scheme,
                                          keep_fields=True)
        ge = P2.gradient_energy2(ph, f)
        gf = P2.gradient_fd2(ph, lame, l0, tol=1e-13, rel_step=1e-5, scheme=scheme)
        assert np.abs(ge - gf).max() < 1e-6 * np.abs(ge).max()
        # symmetric in (k, l)
        assert np.abs(ge - np.swapaxes(ge, 0, 1)).max() < 1e-12 * np.abs(ge).max()


def test_plane_gradient_is_the_3d_in_plane_block():
    """On an (N, N, 1) grid the plane gradient is the in-plane block of the
    three-dimensional energy identity."""
    ph = _two_phase_square(16, 9)
    lame = np.array([[1.0, 0.5], [6.0, 2.5]])
    l0 = M.reference_medium(lame)
    _, _, f2 = P2.effective_stiffness2(ph, lame, l0, tol=1e-13, keep_fields=True)
    _, _, f3 = D.effective_stiffness(ph[:, :, None].copy(), lame, l0, tol=1e-13, keep_fields=True)
    g2 = P2.gradient_energy2(ph, f2)
    g3 = D.gradient_energy(ph[:, :, None].copy(), f3)
    assert np.abs(g2 - g3[np.ix_(IN, IN)]).max() < 1e-11 * np.abs(g2).max()
