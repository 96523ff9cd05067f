"""Pins of the dense-vector QTT oracle (Sec. 3, Sec. 4, App. C)."""
import math
import os

import numpy as np
import pytest

from oracle import dense as D, qtt as Q
import microstructures as M

HERE = os.path.dirname(os.path.abspath(__file__))


def rand_tt(rng, dims, r):
    L = len(dims)
    ranks = [1] + [min(r, int(np.prod(dims[:k])), int(np.prod(dims[k:]))) for k in range(1, L)] + [1]
    return [rng.standard_normal((ranks[k], d, ranks[k + 1])) + 1j * rng.standard_normal((ranks[k], d, ranks[k + 1]))
            for k, d in enumerate(dims)]


def test_tt_svd_roundtrip_and_bound():
    rng = np.random.default_rng(0)
    T = rng.standard_normal((6, 2, 2, 2, 2, 2, 2))
    c = Q.tt_svd(T, 1e-14)
    assert np.abs(Q.tt_full(c) - T).max() < 1e-12
    for delta in (0.3, 0.1, 0.01):
        c = Q.tt_svd(T, delta)
        assert np.linalg.norm(Q.tt_full(c) - T) <= delta * np.linalg.norm(T) * (1 + 1e-12)


def test_rounding_bound_and_rank_rules():
    """eq. rounding_condition_tt, and Table 2: r(x+y) <= r(x)+r(y),
    r(Ax) <= r(A) r(x)."""
    rng = np.random.default_rng(1)
    dims = [6, 2, 2, 2, 2, 2, 2]
    x = rand_tt(rng, dims, 5)
    y = rand_tt(rng, dims, 3)
    s = Q.tt_add(x, y)
    assert Q.ranks(s) == [a + b if 0 < k < len(dims) else 1 for k, (a, b) in
                          enumerate(zip(Q.ranks(x), Q.ranks(y)))]
    assert np.abs(Q.tt_full(s) - Q.tt_full(x) - Q.tt_full(y)).max() < 1e-12
    full = Q.tt_full(s)
    for delta in (1e-1, 1e-3):
        r, disc = Q.tt_round(s, delta)
        err = np.linalg.norm(Q.tt_full(r) - full) / np.linalg.norm(full)
        assert err <= delta * (1 + 1e-10)
        assert abs(err - disc) < 1e-10
    A = [rng.standard_normal((a, d, d, b)) for a, d, b in zip([1, 2, 2, 2, 2, 2, 2], dims, [2, 2, 2, 2, 2, 2, 1])]
    z = Q.tto_apply(A, x)
    assert Q.ranks(z) == [a * b for a, b in zip(Q.ranks(A), Q.ranks(x))]
    ref = Q.tto_full(A) @ Q.tt_full(x).ravel()
    assert np.abs(Q.tt_full(z).ravel() - ref).max() < 1e-10 * np.abs(ref).max()


def test_raise_gives_hadamard_product():
    """App. C: raising a TT to a diagonal TTO turns TTO x TT into the
    element-wise product; ranks multiply (Table 2)."""
    rng = np.random.default_rng(2)
    dims = [2] * 6
    a = rand_tt(rng, dims, 3)
    b = rand_tt(rng, dims, 4)
    z = Q.tto_apply(Q.raise_tt(a), b)
    ref = Q.tt_full(a) * Q.tt_full(b)
    assert np.abs(Q.tt_full(z) - ref).max() < 1e-13 * np.abs(ref).max()
    assert max(Q.ranks(z)) <= max(Q.ranks(a)) * max(Q.ranks(b))


def _qft_circuit(n):
    """Q_n from its gates: H on qubit b, then cP(pi/2^(a-b)) between qubit b
    and every later qubit a (Sec. 4.1); qubit 0 is the most significant."""
    N = 1 << n
    H = np.array([[1, 1], [1, -1]]) / math.sqrt(2)
    U = np.eye(N, dtype=complex)
    for b in range(n):
        U = np.kron(np.kron(np.eye(1 << b), H), np.eye(1 << (n - b - 1))) @ U
        for a in range(b + 1, n):
            d = np.ones(N, dtype=complex)
            for s in range(N):
                if (s >> (n - 1 - b)) & 1 and (s >> (n - 1 - a)) & 1:
                    d[s] = np.exp(1j * math.pi / 2 ** (a - b))
            U = d[:, None] * U
    return U


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_reduced_qft_matrix_equals_circuit(n):
    assert np.abs(Q.qn_matrix(n) - _qft_circuit(n)).max() < 1e-13


@pytest.mark.parametrize("n", [2, 3])
def test_sfft_is_bitreversed_inverse_dft(n):
    """S x = N^{3/2} ifftn(x) at bit-reversed momentum indices."""
    rng = np.random.default_rng(3)
    N = 1 << n
    x = rng.normal(size=(6, N, N, N)) + 1j * rng.normal(size=(6, N, N, N))
    S = Q.sfft_3d(n, 1e-14)
    y = Q.field_from_tt(Q.tto_apply(S, Q.tt_from_field(x, n, 1e-14)), n)
    r = Q.bitrev(np.arange(N), n)
    ref = N ** 1.5 * np.fft.ifftn(x, axes=(1, 2, 3))[:, r][:, :, r][:, :, :, r]
    assert np.abs(y - ref).max() < 1e-11 * np.abs(ref).max()


def test_sfft_ranks_match_the_paper():
    """Sec. 5.2: SFFT ranks converge to 10 for n >= 8 at delta = 1e-10."""
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "sfft_rank.txt"))
            if l.strip() and not l.startswith("#")]
    for n, r in rows:
        assert max(Q.ranks(Q.qn_tto(int(n), 1e-10))) == int(r)


def test_green_tt_densifies_to_table():
    n = 2
    lam0, mu0 = 2.3, 1.4
    G = Q.green_tto(n, lam0, mu0, 1e-14)
    dense = Q.tto_full(G)  # (6 N^3) x (6 N^3) diagonal in space
    Gt = Q.green_tensor(n, lam0, mu0)
    N3 = (1 << n) ** 3
    d = dense.reshape(6, N3, 6, N3)
    diag = np.einsum("vxwx->vwx", d).reshape(6, 6, 1 << n, 1 << n, 1 << n)
    assert np.abs(diag - Gt).max() < 1e-12
    off = d.copy()
    for i in range(N3):
        off[:, i, :, i] = 0
    assert np.abs(off).max() < 1e-12


@pytest.mark.parametrize("scheme", ["direct", "staggered"])
def test_green_momentum_convention(scheme):
    """S^H (G_TT . S x) = ifftn(G_h . fftn(x)) (the SFFT convention), for
    both discretisations of App. A."""
    n = 2
    N = 1 << n
    lam0, mu0 = 2.3, 1.4
    rng = np.random.default_rng(4)
    x = rng.normal(size=(6, N, N, N))
    S = Q.sfft_3d(n, 1e-14)
    xt = Q.tt_from_field(x.astype(complex), n, 1e-14)
    G = Q.green_tto(n, lam0, mu0, 1e-14, scheme=scheme)
    y = Q.tto_apply(Q.tto_adjoint(S), Q.tto_apply(G, Q.tto_apply(S, xt)))
    ref = D.apply_gamma(D.green_table(N, lam0, mu0, scheme), x.astype(complex))
    assert np.abs(Q.field_from_tt(y, n) - ref).max() < 1e-11 * np.abs(ref).max()
    if scheme == "staggered":
        # a real field stays real: the staggered operator is real in space
        assert np.abs(ref.imag).max() < 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("scheme", ["direct", "staggered"])
def test_untruncated_alg2_equals_alg1_same_iterations(scheme):
    p = M.Problem("s4", 2, M.sphere(4, 0.3), [(1.0, 0.3), (10.0, 0.3)], cap=0, delta=1e-14, tol=0)
    C2, _ = Q.qtt_effective_stiffness(p.phase, p.lame, p.lame0, 1e-14, 1 << 30, 0.0, fixed_iters=3,
                                      scheme=scheme)
    C1, _ = D.effective_stiffness(p.phase, p.lame, p.lame0, 0.0, fixed_iters=3, scheme=scheme)
    assert np.abs(C2 - C1).max() < 1e-11 * np.abs(C1).max()


def test_tt_entry_matches_full():
    rng = np.random.default_rng(21)
    dims = [6, 2, 2, 2, 2, 2, 2]
    x = rand_tt(rng, dims, 5)
    F = Q.tt_full(x)
    for _ in range(20):
        idx = tuple(int(rng.integers(d)) for d in dims)
        assert abs(Q.tt_entry(x, idx) - F[idx]) < 1e-12 * np.abs(F).max()


@pytest.mark.parametrize("n", [2, 3])
def test_sfft_entry_matches_library_fft(n):
    """Entrywise SFFT of a train (used on sampled outputs at full size) equals
    N^(3/2) ifftn of the dense field read at bit-reversed indices, the
    library-FFT form of the reduced QFT on each axis."""
    N = 1 << n
    rng = np.random.default_rng(22 + n)
    x = rand_tt(rng, [6] + [2] * (3 * n), 7)
    f = Q.tt_full(x).reshape(6, N, N, N)
    ref = N ** 1.5 * np.fft.ifftn(f, axes=(1, 2, 3))
    r = Q.bitrev(np.arange(N), n)
    for _ in range(40):
        v = int(rng.integers(6))
        k = [int(a) for a in rng.integers(N, size=3)]
        want = ref[v, r[k[0]], r[k[1]], r[k[2]]]
        assert abs(Q.sfft_entry(x, n, v, k) - want) < 1e-12 * np.abs(ref).max()
