"""Dense-vector quantized tensor-train reference in FP64 (oracle; test infrastructure).

Plain NumPy tensor-train arithmetic, written from the paper:

* TT format (Sec. 3, eq. tt_format) with cores (r_{k-1}, d_k, r_k);
  TTO format (Sec. 3, eq. tto_format) with cores (r_{k-1}, d_out, d_in, r_k).
* TTO x TT contraction, rank r(A) r(x) (Table 2, "z = Ax (contract)").
* Raising a TT to a diagonal TTO so that TTO x TT is the Hadamard product
  (Sec. 3, eq. tt_to_tto; App. C).
* TT-rounding: right-to-left QR orthogonalisation then left-to-right
  truncated SVDs so that ||v - v~||_F <= delta_acc ||v||_F
  (Sec. 3, eq. rounding_condition_tt).  Per-bond threshold
  delta_acc / sqrt(L - 1) * ||v||_F with L the number of cores (reading of
  the garbled delta_trunc formula; Oseledets 2011, Thm. 2.2).  The rank kept
  at a bond is the smallest one whose discarded squared singular values sum
  to at most the squared threshold, then clipped to the cap, and at least 1.
* TT-SVD of a dense tensor with the same rule (Sec. 4.3, binary
  discretisation followed by successive SVDs).
* The SFFT operator: the reduced QFT Q_n of Sec. 4.1 (QFT circuit without
  the final bit-reversal SWAPs) on each spatial axis, identity on the Voigt
  control core (Sec. 4.3, controlled QTT).  Its plain definition is the
  matrix Q_n[k, j] = N^(-1/2) exp(+2 pi i j rev_n(k) / N); the TTO is the
  TT-SVD of that matrix with the (out, in) bit pair of each qubit as one
  physical index.
* Green TT: the Nyquist-symmetrised Green table in the SFFT momentum
  convention (Sec. 4.3: indices reversed per axis, then complex conjugate),
  with a 6x6 Voigt control core.
* Alg. 2 (SFFT-based homogenization) with every product followed by
  TT-rounding.
"""
from __future__ import annotations

import math

import numpy as np

from . import dense as D
from .voigt import iso_voigt

# ---------------------------------------------------------------------------
# basic TT / TTO arithmetic
# ---------------------------------------------------------------------------


def tt_full(cores) -> np.ndarray:
    """Dense tensor of a TT, shape (d_1, ..., d_L)."""
    out = cores[0]                                   # (1, d, r)
    for c in cores[1:]:
        out = np.tensordot(out, c, axes=([out.ndim - 1], [0]))
    return out.reshape(out.shape[1:-1])


def tto_full(cores) -> np.ndarray:
    """Dense matrix of a TTO, shape (prod d_out, prod d_in)."""
    out = cores[0]                                   # (1, o, i, r)
    for c in cores[1:]:
        out = np.tensordot(out, c, axes=([out.ndim - 1], [0]))
    t = out.reshape(out.shape[1:-1])                 # (o1, i1, o2, i2, ...)
    L = t.ndim // 2
    perm = list(range(0, 2 * L, 2)) + list(range(1, 2 * L, 2))
    t = t.transpose(perm)
    dout = int(np.prod(t.shape[:L]))
    return t.reshape(dout, -1)


def ranks(cores) -> list:
    return [c.shape[0] for c in cores] + [cores[-1].shape[-1]]


def _keep(sigma: np.ndarray, thr: float, cap: int) -> int:
    """Smallest r with sum_{i>=r} sigma_i^2 <= thr^2, clipped to [1, cap]."""
    tail = np.concatenate([np.cumsum((sigma ** 2)[::-1])[::-1], [0.0]])
    r = int(np.argmax(tail <= thr * thr))
    return max(1, min(r, cap, sigma.size))


def tt_svd(T: np.ndarray, delta: float, cap: int = 1 << 30):
    """TT-SVD of a dense tensor (all axes are physical indices)."""
    dims = T.shape
    L = len(dims)
    nrm = np.linalg.norm(T)
    thr = delta / math.sqrt(max(L - 1, 1)) * nrm
    cores = []
    M = T.reshape(1, -1).astype(np.complex128)
    r = 1
    for k in range(L - 1):
        M = M.reshape(r * dims[k], -1)
        U, s, Vh = np.linalg.svd(M, full_matrices=False)
        rk = _keep(s, thr, cap)
        cores.append(U[:, :rk].reshape(r, dims[k], rk))
        M = s[:rk, None] * Vh[:rk]
        r = rk
    cores.append(M.reshape(r, dims[-1], 1))
    return cores


def tto_apply(A, x):
    """Materialised TTO x TT product; core ranks multiply (Table 2)."""
    out = []
    for a, c in zip(A, x):
        z = np.einsum("aijb,cjd->acibd", a, c)
        ra, rc, d, rb, rd = z.shape
        out.append(z.reshape(ra * rc, d, rb * rd))
    return out


def raise_tt(cores):
    """Diagonal TTO with G(i, j) = C(i) delta(i, j) (eq. tt_to_tto)."""
    out = []
    for c in cores:
        r0, d, r1 = c.shape
        g = np.zeros((r0, d, d, r1), dtype=np.complex128)
        for i in range(d):
            g[:, i, i, :] = c[:, i, :]
        out.append(g)
    return out


def tto_adjoint(A):
    """Conjugate transpose of a TTO, core by core."""
    return [np.conj(a.transpose(0, 2, 1, 3)) for a in A]


def tt_scale(x, alpha):
    return [x[0] * alpha] + [c.copy() for c in x[1:]]


def tt_add(x, y):
    """Sum of two TTs with the same physical dims; ranks add (Table 2)."""
    L = len(x)
    out = []
    for k, (a, b) in enumerate(zip(x, y)):
        if k == 0:
            out.append(np.concatenate([a, b], axis=2))
        elif k == L - 1:
            out.append(np.concatenate([a, b], axis=0))
        else:
            r0a, d, r1a = a.shape
            r0b, _, r1b = b.shape
            c = np.zeros((r0a + r0b, d, r1a + r1b), dtype=np.complex128)
            c[:r0a, :, :r1a] = a
            c[r0a:, :, r1a:] = b
            out.append(c)
    return out


def orthogonalize_right(x):
    """Right-to-left QR sweep; cores 1..L-1 become right-orthogonal."""
    x = [c.astype(np.complex128).copy() for c in x]
    for k in range(len(x) - 1, 0, -1):
        r0, d, r1 = x[k].shape
        M = x[k].reshape(r0, d * r1)
        Q, R = np.linalg.qr(M.conj().T)             # M = R^H Q^H
        x[k] = Q.conj().T.reshape(-1, d, r1)
        x[k - 1] = np.tensordot(x[k - 1], R.conj().T, axes=([2], [0]))
    return x


def tt_norm(x) -> float:
    """Frobenius norm via orthogonalisation (no Gram cancellation)."""
    y = orthogonalize_right(x)
    return float(np.linalg.norm(y[0]))


def tt_round(x, delta: float, cap: int = 1 << 30):
    """TT-rounding (Sec. 3).  Returns (cores, relative discarded mass)."""
    L = len(x)
    y = orthogonalize_right(x)
    nrm = float(np.linalg.norm(y[0]))
    if nrm == 0.0:
        return [np.zeros((1, c.shape[1], 1), np.complex128) for c in x], 0.0
    thr = delta / math.sqrt(max(L - 1, 1)) * nrm
    disc = 0.0
    for k in range(L - 1):
        r0, d, r1 = y[k].shape
        U, s, Vh = np.linalg.svd(y[k].reshape(r0 * d, r1), full_matrices=False)
        rk = _keep(s, thr, cap)
        disc += float((s[rk:] ** 2).sum())
        y[k] = U[:, :rk].reshape(r0, d, rk)
        y[k + 1] = np.tensordot(s[:rk, None] * Vh[:rk], y[k + 1], axes=([1], [0]))
    return y, math.sqrt(disc) / nrm


def tt_dot(x, y) -> complex:
    """<x, y> = sum conj(x) y, chain contraction."""
    M = np.ones((1, 1), dtype=np.complex128)
    for a, b in zip(x, y):
        M = np.einsum("ab,aic,bid->cd", M, np.conj(a), b)
    return complex(M[0, 0])


# ---------------------------------------------------------------------------
# operators of the SFFT-based scheme
# ---------------------------------------------------------------------------


def bitrev(k: np.ndarray, n: int) -> np.ndarray:
    k = np.asarray(k)
    out = np.zeros_like(k)
    for b in range(n):
        out |= ((k >> b) & 1) << (n - 1 - b)
    return out


def tt_entry(cores, idx) -> complex:
    """One entry x[i_1, ..., i_L] of a TT with cores (r_{k-1}, d_k, r_k):
    the product of the core slices at the indices (Sec. 3, eq. tt_format)."""
    v = np.ones(1, dtype=np.complex128)
    for c, i in zip(cores, idx):
        v = v @ c[:, int(i), :]
    return complex(v[0])


def sfft_entry(cores, n: int, v: int, k) -> complex:
    """Entry (v, k_x, k_y, k_z) of the SFFT applied to a controlled QTT
    strain train (Voigt core, then n bits per axis, most significant first),
    from the plain definition of the reduced QFT on each axis (Sec. 4.1):
    (S x)[v, k] = N^(-3/2) sum_j x[v, j] exp(+2 pi i j . rev_n(k) / N).
    The phase factorises over the bits of j, so each bit core is summed
    over its two values with that bit's phase; no dense field is formed."""
    N = 1 << n
    vec = np.asarray(cores[0])[0, int(v), :].astype(np.complex128)
    for a in range(3):
        m = int(bitrev(np.array([int(k[a])]), n)[0])
        for t in range(n):
            c = np.asarray(cores[1 + a * n + t])
            w = np.exp(2j * np.pi * (1 << (n - 1 - t)) * m / N)
            vec = vec @ (c[:, 0, :] + w * c[:, 1, :])
    return complex(vec[0]) / N ** 1.5


def qn_matrix(n: int) -> np.ndarray:
    """Reduced QFT Q_n[k, j] = N^-1/2 exp(2 pi i j rev(k) / N) (Sec. 4.1)."""
    N = 1 << n
    k = np.arange(N)
    ph = np.outer(bitrev(k, n), np.arange(N)) % N
    return np.exp(2j * np.pi * ph / N) / math.sqrt(N)


def qn_tto(n: int, delta: float, cap: int = 1 << 30):
    """TTO of Q_n by TT-SVD with the (out, in) bit pair per qubit."""
    N = 1 << n
    Q = qn_matrix(n).reshape([2] * n + [2] * n)
    perm = []
    for a in range(n):
        perm += [a, n + a]
    T = Q.transpose(perm).reshape([4] * n)
    cores = tt_svd(T, delta, cap)
    return [c.reshape(c.shape[0], 2, 2, c.shape[2]) for c in cores]


def identity_voigt_core() -> np.ndarray:
    return np.eye(6, dtype=np.complex128).reshape(1, 6, 6, 1)


def sfft_3d(n: int, delta: float, cap: int = 1 << 30):
    """SFFT TTO on a controlled QTT: Voigt identity, then Q_n on x, y, z."""
    q = qn_tto(n, delta, cap)
    return [identity_voigt_core()] + [c.copy() for _ in range(3) for c in q]


def green_tensor(n: int, lam0: float, mu0: float, scheme: str = "direct") -> np.ndarray:
    """Dense Green operator in the SFFT momentum order, shape (6,6,N,N,N).

    Entry at momentum index (kx, ky, kz) is G_h at DFT index
    (-rev(kx), -rev(ky), -rev(kz)) mod N, which equals conj G_h(rev(k)):
    indices reversed per axis, then conjugated (Sec. 4.3).  ``scheme``:
    the discretisation of App. A, Table 3 (``direct`` or ``staggered``).
    """
    N = 1 << n
    G = D.green_table(N, lam0, mu0, scheme)
    m = (-bitrev(np.arange(N), n)) % N
    return G[:, :, m][:, :, :, m][:, :, :, :, m]


def green_tto(n: int, lam0: float, mu0: float, delta: float, cap: int = 1 << 30,
              scheme: str = "direct"):
    """Raised Green TTO with a 6x6 Voigt control core."""
    T = green_tensor(n, lam0, mu0, scheme).reshape([36] + [2] * (3 * n))
    cores = tt_svd(T, delta, cap)
    c0 = cores[0].reshape(1, 6, 6, cores[0].shape[2])
    return [c0] + raise_tt(cores[1:])


def stiffness_tto(phase: np.ndarray, lame, lame0, delta: float, cap: int = 1 << 30,
                  include_c0: bool = False):
    """Raised TTO of C(x) - C0 (or C(x) with ``include_c0``).

    The one-hot phase tensor (P, 2, ..., 2) is compressed by TT-SVD; its
    first core (1, P, r) is contracted with the per-phase Voigt matrices.
    """
    lame = np.asarray(lame, dtype=np.float64)
    P = lame.shape[0]
    n3 = int(round(math.log2(phase.size)))
    onehot = np.stack([(phase == p).astype(np.float64) for p in range(P)])
    cores = tt_svd(onehot.reshape([P] + [2] * n3), delta, cap)
    Cp = D.stiffness_per_phase(lame)
    if not include_c0:
        Cp = Cp - iso_voigt(*lame0)[None]
    c0 = np.einsum("pvw,ipr->ivwr", Cp, cores[0])
    return [c0] + raise_tt(cores[1:])


def coarsen_majority(phase: np.ndarray, nphase: int) -> np.ndarray:
    """The geometry one discretisation order lower: the majority phase of
    every 2 x 2 x 2 block of voxels (2 x 2 block of pixels for a plane
    geometry), ties to the lowest phase id."""
    d = phase.ndim
    h = phase.shape[0] // 2
    blocks = phase.reshape((h, 2) * d).transpose(tuple(range(0, 2 * d, 2)) + tuple(range(1, 2 * d, 2)))
    blocks = blocks.reshape((h,) * d + (2 ** d,))
    counts = np.stack([(blocks == p).sum(axis=-1) for p in range(nphase)], axis=-1)
    return np.argmax(counts, axis=-1).astype(np.uint8)     # argmax: first maximum


def rank_estimate(phase: np.ndarray, nphase: int, delta: float):
    """Applicability estimate from two discretisation orders (Sec. 5.2):
    the largest bond rank of the one-hot phase train (TT-SVD at delta) of
    the coarsened geometry (order n - 1) and of the geometry (order n), and
    their ratio; 3D voxels or plane pixels (the bits of x, then y, then z,
    most significant first)."""
    def top(ph):
        oh = np.stack([(ph == p).astype(np.float64) for p in range(nphase)])
        n3 = int(round(math.log2(ph.size)))
        return max(ranks(tt_svd(oh.reshape([nphase] + [2] * n3), delta)))
    rc = top(coarsen_majority(phase, nphase))
    rf = top(phase)
    return rc, rf, rf / rc


def const_tt(E: np.ndarray, n: int):
    """Rank-1 TT of a constant Voigt field (Sec. 4.3, constant operands)."""
    c0 = np.asarray(E, dtype=np.complex128).reshape(1, 6, 1)
    one = np.ones((1, 2, 1), dtype=np.complex128)
    return [c0] + [one.copy() for _ in range(3 * n)]


def field_from_tt(x, n: int) -> np.ndarray:
    N = 1 << n
    return tt_full(x).reshape(6, N, N, N)


def tt_from_field(f: np.ndarray, n: int, delta: float, cap: int = 1 << 30):
    return tt_svd(np.asarray(f).reshape([6] + [2] * (3 * n)), delta, cap)


# ---------------------------------------------------------------------------
# Alg. 2
# ---------------------------------------------------------------------------


def qtt_ls(phase: np.ndarray, lame, lame0, E, delta: float, cap: int, tol: float,
           max_iter: int = 2000, fixed_iters: int | None = None, ops=None):
    """SFFT-based homogenization (Alg. 2) with rounding after every product.

    Returns (eps TT, iterations, residual history, max rank seen).
    """
    n = int(round(math.log2(phase.shape[0])))
    if ops is None:
        ops = build_operators(phase, lame, lame0, delta)
    S, SH, G, Cd = ops
    Et = const_tt(E, n)
    normE = float(np.linalg.norm(E)) * (1 << n) ** 1.5
    eps = [c.copy() for c in Et]
    hist = []
    rmax = 1
    m = 0
    while True:
        tau, _ = tt_round(tto_apply(Cd, eps), delta, cap)
        th, _ = tt_round(tto_apply(S, tau), delta, cap)
        eh, _ = tt_round(tto_apply(G, th), delta, cap)
        y, _ = tt_round(tto_apply(SH, eh), delta, cap)
        new, _ = tt_round(tt_add(Et, tt_scale(y, -1.0)), delta, cap)
        res = tt_norm(tt_add(new, tt_scale(eps, -1.0))) / normE
        hist.append(res)
        rmax = max(rmax, max(ranks(new)), max(ranks(tau)), max(ranks(th)),
                   max(ranks(eh)), max(ranks(y)))
        eps = new
        m += 1
        if fixed_iters is not None:
            if m >= fixed_iters:
                break
        elif res < tol or m >= max_iter:
            break
    return eps, m, hist, rmax


def build_operators(phase, lame, lame0, delta, scheme: str = "direct"):
    n = int(round(math.log2(phase.shape[0])))
    S = sfft_3d(n, delta)
    return (S, tto_adjoint(S), green_tto(n, *lame0, delta, scheme=scheme),
            stiffness_tto(phase, lame, lame0, delta))


def qtt_effective_stiffness(phase, lame, lame0, delta, cap, tol, max_iter=2000,
                            fixed_iters=None, scheme: str = "direct"):
    """C_eff from Alg. 2; the mean stress is taken on the densified strain."""
    n = int(round(math.log2(phase.shape[0])))
    ops = build_operators(phase, lame, lame0, delta, scheme)
    C = np.zeros((6, 6))
    iters = []
    for k in range(6):
        E = np.zeros(6)
        E[k] = 1.0
        eps, m, _, _ = qtt_ls(phase, lame, lame0, E, delta, cap, tol, max_iter,
                              fixed_iters, ops)
        C[:, k] = D.mean_stress(phase, lame, field_from_tt(eps, n))
        iters.append(m)
    return C, iters
