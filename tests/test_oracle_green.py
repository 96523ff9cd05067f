"""Pins of the oracle's Green operator (App. A, direct scheme)."""
import numpy as np
import pytest

from oracle import dense as D
from oracle.voigt import (PAIRS, iso_tensor, iso_voigt, strain_tensor_to_voigt,
                          stress_voigt_to_tensor, strain_voigt_to_tensor)

LAM0, MU0 = 1.7, 0.9


def test_closed_form_equals_acoustic_tensor_form():
    rng = np.random.default_rng(0)
    xi = rng.normal(size=(64, 3))
    a = D.gamma_tensor(xi, LAM0, MU0)
    b = D.gamma_tensor_acoustic(xi, iso_tensor(LAM0, MU0))
    assert np.abs(a - b).max() < 1e-14


def test_zero_frequency_is_zero():
    assert np.abs(D.gamma_tensor(np.zeros((1, 3)), LAM0, MU0)).max() == 0.0


def test_projection_properties():
    """Gamma C0 Gamma = Gamma and Gamma C0 eps = eps for compatible eps =
    sym(xi (x) a) (Gamma is the C0-orthogonal projection on compatible
    fields)."""
    rng = np.random.default_rng(1)
    C0 = iso_tensor(LAM0, MU0)
    for _ in range(10):
        xi = rng.normal(size=(1, 3))
        G = D.gamma_tensor(xi, LAM0, MU0)[0]
        GCG = np.einsum("ijkl,klmn,mnpq->ijpq", G, C0, G)
        assert np.abs(GCG - G).max() < 1e-13
        a = rng.normal(size=3)
        eps = 0.5 * (np.outer(xi[0], a) + np.outer(a, xi[0]))
        back = np.einsum("ijkl,klmn,mn->ij", G, C0, eps)
        assert np.abs(back - eps).max() < 1e-13


def test_voigt_weights_map_stress_to_engineering_strain():
    rng = np.random.default_rng(2)
    xi = rng.normal(size=(5, 3))
    G = D.gamma_tensor(xi, LAM0, MU0)
    GV = D.gamma_voigt(xi, LAM0, MU0)
    tau_v = rng.normal(size=6)
    tau = stress_voigt_to_tensor(tau_v)
    for p in range(5):
        eps = np.einsum("ijkl,kl->ij", G[p], tau)
        assert np.abs(GV[p] @ tau_v - strain_tensor_to_voigt(eps)).max() < 1e-14
        assert np.abs(GV[p] - GV[p].T).max() < 1e-14


def test_table_is_hermitian_and_real():
    N = 8
    T = D.gamma_table(N, LAM0, MU0)
    neg = (-np.arange(N)) % N
    Tn = T[:, :, neg][:, :, :, neg][:, :, :, :, neg]
    assert np.abs(Tn - np.conj(T)).max() < 1e-15
    assert np.abs(T.imag).max() == 0.0
    assert np.abs(T[:, :, 0, 0, 0]).max() == 0.0


def test_table_off_nyquist_matches_formula():
    N = 8
    T = D.gamma_table(N, LAM0, MU0)
    f = D.frequencies(N)
    ix, iy, iz = 1, 3, 6
    g = D.gamma_voigt(np.array([[f[ix], f[iy], f[iz]]]), LAM0, MU0)[0]
    assert np.abs(T[:, :, ix, iy, iz] - g).max() < 1e-15


def test_nyquist_average_of_the_two_representatives():
    N = 8
    T = D.gamma_table(N, LAM0, MU0)
    # index (N/2, 1, 2): average over xi_x = -N/2 and +N/2
    a = D.gamma_voigt(np.array([[-4.0, 1.0, 2.0]]), LAM0, MU0)[0]
    b = D.gamma_voigt(np.array([[4.0, 1.0, 2.0]]), LAM0, MU0)[0]
    assert np.abs(T[:, :, 4, 1, 2] - 0.5 * (a + b)).max() < 1e-15


def test_voigt_helpers_roundtrip():
    rng = np.random.default_rng(3)
    v = rng.normal(size=6)
    assert np.allclose(strain_tensor_to_voigt(strain_voigt_to_tensor(v)), v)
    C = iso_voigt(LAM0, MU0)
    assert C[0, 0] == pytest.approx(LAM0 + 2 * MU0)
    assert C[0, 1] == pytest.approx(LAM0)
    assert C[3, 3] == pytest.approx(MU0)
    assert len(PAIRS) == 6


def test_voigt_entrywise_form_equals_tensor_form():
    rng = np.random.default_rng(5)
    xi = rng.normal(size=(40, 3))
    xi[0] = 0.0
    a = D.gamma_voigt(xi, LAM0, MU0)
    b = D.gamma_voigt_direct(xi[:, 0], xi[:, 1], xi[:, 2], LAM0, MU0)
    assert np.abs(a - b.transpose(2, 0, 1)).max() < 1e-14
