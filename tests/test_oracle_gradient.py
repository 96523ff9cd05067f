"""Pins of the gradient references (C0 held fixed)."""
import numpy as np
import pytest

from oracle import dense as D
import microstructures as M


@pytest.fixture(scope="module")
def prob():
    p = M.Problem("s8", 3, M.sphere(8, 0.3), [(1.0, 0.3), (6.0, 0.25)], cap=0, delta=1e-14, tol=1e-13)
    C, it, fields = D.effective_stiffness(p.phase, p.lame, p.lame0, tol=1e-13, keep_fields=True)
    return p, C, fields


def test_energy_identity_matches_central_fd(prob):
    p, C, fields = prob
    ge = D.gradient_energy(p.phase, fields)
    gf = D.gradient_fd(p.phase, p.lame, p.lame0, tol=1e-13, rel_step=1e-5)
    assert np.abs(ge - gf).max() < 1e-6 * np.abs(gf).max()


def test_dense_adjoint_matches_energy_identity(prob):
    p, C, fields = prob
    adj = D.adjoint_fields(p.phase, p.lame, p.lame0, tol=1e-13)
    ga = D.gradient_adjoint(p.phase, p.lame, p.lame0, fields, adj)
    ge = D.gradient_energy(p.phase, fields)
    assert np.abs(ga - ge).max() < 1e-9 * np.abs(ge).max()


def test_gradient_homogeneity(prob):
    """C_eff is homogeneous of degree one in the phase moduli (with C0
    scaled too); with C0 fixed, sum_theta theta dC/dtheta is C_eff's
    derivative along the scaling of the phases only -- checked against a
    finite difference along that single direction."""
    p, C, fields = prob
    ge = D.gradient_energy(p.phase, fields)
    th = p.lame.ravel()
    dir_deriv = np.einsum("klt,t->kl", ge, th)
    h = 1e-5
    Cp, _ = D.effective_stiffness(p.phase, p.lame * (1 + h), p.lame0, tol=1e-13)
    Cm, _ = D.effective_stiffness(p.phase, p.lame * (1 - h), p.lame0, tol=1e-13)
    assert np.abs(dir_deriv - (Cp - Cm) / (2 * h)).max() < 1e-6 * np.abs(C).max()


def test_euler_identity_fibres_shrinks_with_grid():
    """C is linear in each phase's (lambda, mu), so the energy-identity
    Jacobian satisfies sum_theta theta dC_eff/dtheta = <eps^k : C : eps^l>,
    which equals C_eff where Hill's lemma holds.  The Nyquist average of the
    Green table is not a projection, so on the four-fibre geometry the
    identity holds to a deviation that shrinks with the grid (3.4e-3 at 8^3,
    1.2e-3 at 16^3): the bound the full-size adjoint check builds on."""
    dev = []
    for n in (3, 4):
        p = M.config_c2(n=n)
        C, it, fields = D.effective_stiffness(p.phase, p.lame, p.lame0, tol=1e-12, keep_fields=True)
        J = D.gradient_energy(p.phase, fields)
        E = np.einsum("klt,t->kl", J, np.asarray(p.lame).ravel())
        dev.append(np.linalg.norm(E - C) / np.linalg.norm(C))
        assert np.abs(J - J.transpose(1, 0, 2)).max() < 1e-12 * np.abs(J).max()
    assert dev[0] < 5e-3 and dev[1] < 2e-3 and dev[1] < dev[0]


def test_references_agree_on_the_64_fibres():
    """The gradient references on the four-fibre workload at 64^3 (the
    (64, 64, 1) slice of the z-invariant geometry): energy identity,
    central differences with the workload's step 1e-6, dense adjoint."""
    p = M.config_c2(6)
    ph = p.phase[:, :, :1].copy()
    C, it, fields = D.effective_stiffness(ph, p.lame, p.lame0, tol=1e-13, keep_fields=True)
    ge = D.gradient_energy(ph, fields)
    gf = D.gradient_fd(ph, p.lame, p.lame0, tol=1e-13, rel_step=1e-6)
    adj = D.adjoint_fields(ph, p.lame, p.lame0, tol=1e-13)
    ga = D.gradient_adjoint(ph, p.lame, p.lame0, fields, adj)
    scale = np.abs(ge).max()
    assert np.abs(gf - ge).max() < 1e-6 * scale
    assert np.abs(ga - ge).max() < 1e-9 * scale
