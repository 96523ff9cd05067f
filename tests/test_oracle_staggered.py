"""Pins of the staggered-grid Green operator in ``oracle.dense`` (App. A,
Table 3: forward differences k+ on the normal strains, backward differences
k- on the shears).

Each pin comes from a source other than the Fourier formula it checks:

* the real-space staggered discretisation built as a sparse difference
  matrix D (displacements to engineering-Voigt strains), with the Green
  operator D (D^T C0 D)^+ D^T applied by a dense pseudo-inverse;
* the generic symbol form with the direct scheme's k = i q, which must give
  the Moulinec-Suquet closed form (``gamma_voigt``);
* the projector identities G C0 G = G and G C0 B = B per frequency;
* the continuum limit: at small |q| the staggered operator tends to the
  direct one at the same direction;
* the laminate closed form, which the staggered scheme (pointwise C(x))
  reaches after one update like the direct one (Sec. 5.2).
"""
import numpy as np
import pytest

from oracle import bounds as B, dense as D
from oracle.voigt import PAIRS, iso_voigt
import microstructures as M


def _difference_matrix(shape, forward_normal=True):
    """Real-space staggered symmetric gradient: u (3, Nx, Ny, Nz) ->
    engineering-Voigt strain (6, Nx, Ny, Nz).  Normal strains
    eps_ii(x) = u_i(x + e_i) - u_i(x); shears
    gamma_ij(x) = u_i(x) - u_i(x - e_j) + u_j(x) - u_j(x - e_i), periodic.
    ``forward_normal=False`` swaps the two differences (a planted mistake)."""
    NN = int(np.prod(shape))
    idx = np.arange(NN).reshape(shape)
    Dm = np.zeros((6 * NN, 3 * NN))
    for I, (i, j) in enumerate(PAIRS):
        rows = I * NN + idx.ravel()
        if i == j:
            s = 1 if forward_normal else -1
            nb = np.roll(idx, -s, axis=i).ravel()   # x + s e_i
            sign = 1.0 if forward_normal else -1.0
            Dm[rows, i * NN + nb] += sign
            Dm[rows, i * NN + idx.ravel()] -= sign
        else:
            s = 1 if forward_normal else -1
            for a, b in ((i, j), (j, i)):              # u_a differenced along b
                nb = np.roll(idx, s, axis=b).ravel()   # x - s e_b
                sign = 1.0 if forward_normal else -1.0
                Dm[rows, a * NN + idx.ravel()] += sign
                Dm[rows, a * NN + nb] -= sign
    return Dm


def _real_space_gamma(shape, lam0, mu0, forward_normal=True):
    NN = int(np.prod(shape))
    Dm = _difference_matrix(shape, forward_normal)
    C0 = np.kron(iso_voigt(lam0, mu0), np.eye(NN))
    K = Dm.T @ C0 @ Dm
    return Dm @ np.linalg.pinv(K, rcond=1e-12) @ Dm.T


@pytest.mark.parametrize("shape", [(4, 4, 4), (4, 2, 8)])
def test_staggered_table_equals_real_space_operator(shape):
    """G_h applied through the FFT equals the real-space staggered Green
    operator D (D^T C0 D)^+ D^T on random polarizations."""
    lam0, mu0 = 1.7, 0.9
    Gr = _real_space_gamma(shape, lam0, mu0)
    G = D.gamma_table_staggered(shape, lam0, mu0)
    rng = np.random.default_rng(3)
    for _ in range(3):
        tau = rng.standard_normal((6,) + shape)
        got = D.apply_gamma(G, tau)
        want = (Gr @ tau.ravel()).reshape((6,) + shape)
        assert np.abs(got.imag).max() < 1e-12
        assert np.abs(got.real - want).max() < 1e-11 * np.abs(want).max()


def test_swapped_differences_are_caught():
    """Backward differences on the normal strains (the mirrored grid) give
    another operator: the real-space pin separates the two."""
    shape = (4, 4, 4)
    G = D.gamma_table_staggered(shape, 1.7, 0.9)
    Gr = _real_space_gamma(shape, 1.7, 0.9, forward_normal=False)
    tau = np.random.default_rng(4).standard_normal((6,) + shape)
    got = D.apply_gamma(G, tau).real
    want = (Gr @ tau.ravel()).reshape((6,) + shape)
    assert np.abs(got - want).max() > 1e-3 * np.abs(want).max()


def test_symbol_form_with_direct_gradient_is_closed_form():
    """B (B^H C0 B)^-1 B^H with k = i xi for both strain kinds equals the
    Moulinec-Suquet closed form in Voigt form."""
    rng = np.random.default_rng(5)
    xi = rng.standard_normal((50, 3))
    xi[0] = 0.0
    lam0, mu0 = 2.3, 1.1
    Bs = D.strain_symbol(1j * xi, 1j * xi)
    got = D.gamma_voigt_symbol(Bs, iso_voigt(lam0, mu0))
    want = D.gamma_voigt(xi, lam0, mu0)
    assert np.abs(got - want).max() < 1e-13 * np.abs(want).max()


def test_projector_identities():
    """Per frequency: G C0 G = G and G C0 B = B (the strain of a compatible
    displacement is reproduced)."""
    lam0, mu0 = 1.2, 0.8
    C0 = iso_voigt(lam0, mu0)
    rng = np.random.default_rng(6)
    q = rng.uniform(0, 2 * np.pi, (40, 3))
    kp, km = D.staggered_symbols(q)
    Bs = D.strain_symbol(kp, km)
    G = D.gamma_voigt_symbol(Bs, C0)
    assert np.abs(G @ C0[None] @ G - G).max() < 1e-12 * np.abs(G).max()
    assert np.abs(G @ C0[None] @ Bs - Bs).max() < 1e-12 * np.abs(Bs).max()
    # Hermitian per frequency (self-adjoint operator)
    assert np.abs(G - np.conj(G).transpose(0, 2, 1)).max() < 1e-13 * np.abs(G).max()


def test_continuum_limit_is_direct_scheme():
    """At q = h d with a fixed direction d the staggered operator tends to
    the direct one at d, with an error of order h."""
    lam0, mu0 = 1.2, 0.8
    d = np.array([[0.3, -0.5, 0.81]])
    want = D.gamma_voigt(d, lam0, mu0)
    errs = []
    for h in (1e-2, 1e-3):
        kp, km = D.staggered_symbols(h * d)
        G = D.gamma_voigt_symbol(D.strain_symbol(kp, km), iso_voigt(lam0, mu0))
        errs.append(np.abs(G - want).max())
    assert errs[1] < 2e-3 * np.abs(want).max()
    assert 5.0 < errs[0] / errs[1] < 20.0      # first order in h


def test_table_zero_frequency_and_hermitian():
    G = D.gamma_table_staggered((8, 4, 2), 1.0, 0.5)
    assert np.all(G[:, :, 0, 0, 0] == 0)
    idx = [(-np.arange(n)) % n for n in (8, 4, 2)]
    Gn = G[:, :, idx[0]][:, :, :, idx[1]][:, :, :, :, idx[2]]
    assert np.abs(G - np.conj(Gn)).max() < 1e-14


def test_staggered_laminate_closed_form_after_one_update():
    """Layers normal to x with the staggered Green operator: the laminate
    closed form after one update, as with the direct scheme (Sec. 5.2)."""
    p = M.config_c1_laminate(3)
    f = [p.volume_fraction(0), p.volume_fraction(1)]
    ref = B.laminate_x(B.iso_phases(p.lame), f)
    one, _ = D.effective_stiffness(p.phase, p.lame, p.lame0, tol=0, fixed_iters=1,
                                   scheme="staggered")
    assert np.abs(one - ref).max() < 1e-12 * np.abs(ref).max()


def test_staggered_sphere_differs_from_direct_and_stays_in_bounds():
    """On a sphere the two discretisations give different C_eff (a few
    percent at 8^3), both between the Voigt and Reuss bounds."""
    p = M.config_c0()
    phase = p.phase[::2, ::2, ::2].copy()
    Cd, _ = D.effective_stiffness(phase, p.lame, p.lame0, tol=1e-10)
    Cs, _ = D.effective_stiffness(phase, p.lame, p.lame0, tol=1e-10, scheme="staggered")
    assert np.abs(Cs - Cd).max() > 1e-4 * np.abs(Cd).max()
    f = np.array([np.mean(phase == q) for q in range(len(p.lame))])
    Cp = D.stiffness_per_phase(p.lame)
    V = B.voigt_bound(Cp, f)
    R = B.reuss_bound(Cp, f)
    for C in (Cd, Cs):
        assert np.linalg.eigvalsh(V - C).min() > -1e-10
        assert np.linalg.eigvalsh(C - R).min() > -1e-10
