"""Dense-pixel FFT-based homogenization in two dimensions (oracle; test
infrastructure): plane strain, Voigt dimension 3, the same Alg. 1 as
``oracle.dense`` on N x N pixel grids.

* Voigt order (11, 22, 12), engineering shear for strain, plain stress.
  The isotropic plane-strain stiffness keeps lambda and mu:
  C = [[lam + 2 mu, lam, 0], [lam, lam + 2 mu, 0], [0, 0, mu]].
* Green operators from their discrete gradients (B (B^H C0 B)^-1 B^H with
  the strain symbol B): the direct scheme k = i q of App. A, Table 3, with
  the Nyquist rule of the three-dimensional oracle, and the staggered grid
  (forward differences on the normal strains, backward on the shear).
* The paper's 2D problems (Sec. 5, Figs. of the 2D geometries) use this
  Voigt dimension; a z-invariant three-dimensional problem whose load keeps
  eps_33 = gamma_13 = gamma_23 = 0 is the same plane-strain problem, which
  the pins use.
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft

from .dense import frequencies, gamma_voigt_symbol, staggered_symbols

PAIRS2 = [(0, 0), (1, 1), (0, 1)]


def iso_voigt2(lam: float, mu: float) -> np.ndarray:
    """Plane-strain isotropic Voigt stiffness (11, 22, 12)."""
    return np.array([[lam + 2 * mu, lam, 0.0], [lam, lam + 2 * mu, 0.0], [0.0, 0.0, mu]])


def strain_symbol2(k: np.ndarray, k_shear: np.ndarray | None = None) -> np.ndarray:
    """B (P, 3, 2): eps_11 = k_1 u_1, eps_22 = k_2 u_2,
    gamma_12 = s_2 u_1 + s_1 u_2 with s = k_shear (default k)."""
    k = np.asarray(k, dtype=np.complex128)
    s = k if k_shear is None else np.asarray(k_shear, dtype=np.complex128)
    B = np.zeros(k.shape[:-1] + (3, 2), dtype=np.complex128)
    B[..., 0, 0] = k[..., 0]
    B[..., 1, 1] = k[..., 1]
    B[..., 2, 0] = s[..., 1]
    B[..., 2, 1] = s[..., 0]
    return B


def gamma_table2(N, lam0: float, mu0: float) -> np.ndarray:
    """Nyquist-symmetrised plane-strain Green table (3, 3, Nx, Ny) in DFT
    order (direct scheme): G_h(idx) = (G(xi(idx)) + conj G(xi(-idx))) / 2."""
    shape = (N, N) if np.isscalar(N) else tuple(N)
    C0 = iso_voigt2(lam0, mu0)
    f = [frequencies(n) for n in shape]
    neg = [fa[(-np.arange(n)) % n] for fa, n in zip(f, shape)]

    def table(fx, fy):
        X, Y = np.meshgrid(fx, fy, indexing="ij")
        xi = np.stack([X, Y], axis=-1).reshape(-1, 2)
        return gamma_voigt_symbol(strain_symbol2(1j * xi), C0).reshape(shape + (3, 3))

    G = 0.5 * (table(*f) + np.conj(table(*neg)))
    return G.transpose(2, 3, 0, 1).copy()


def gamma_table2_staggered(N, lam0: float, mu0: float) -> np.ndarray:
    """Plane-strain staggered-grid Green table (App. A, Table 3: forward
    differences on the normal strains, backward on the shear), (3, 3, Nx,
    Ny) in DFT order; the symbols are 2 pi-periodic (no Nyquist rule)."""
    shape = (N, N) if np.isscalar(N) else tuple(N)
    C0 = iso_voigt2(lam0, mu0)
    qs = [2.0 * np.pi * np.arange(n) / n for n in shape]
    Q = np.stack(np.meshgrid(*qs, indexing="ij"), axis=-1).reshape(-1, 2)
    kp, km = staggered_symbols(Q)
    G = gamma_voigt_symbol(strain_symbol2(kp, km), C0)
    return G.reshape(shape + (3, 3)).transpose(2, 3, 0, 1).copy()


def green_table2(shape, lam0: float, mu0: float, scheme: str = "direct") -> np.ndarray:
    if scheme == "direct":
        return gamma_table2(shape, lam0, mu0)
    if scheme == "staggered":
        return gamma_table2_staggered(shape, lam0, mu0)
    raise ValueError(f"unknown scheme {scheme!r}")


def basic_scheme2(phase: np.ndarray, lame, lame0, E, tol: float, max_iter: int = 2000,
                  G: np.ndarray | None = None, fixed_iters: int | None = None):
    """Alg. 1 on an N x N pixel grid (plane strain); returns (eps (3, N, N),
    iterations, residual history)."""
    lam0, mu0 = lame0
    if G is None:
        G = gamma_table2(phase.shape, lam0, mu0)
    dC = np.stack([iso_voigt2(l, m) for l, m in np.asarray(lame)]) - iso_voigt2(lam0, mu0)[None]
    E = np.asarray(E, dtype=np.float64)
    eps = np.broadcast_to(E[:, None, None], (3,) + phase.shape).astype(np.complex128)
    normE = np.linalg.norm(E) * np.sqrt(phase.size)
    hist = []
    m = 0
    while True:
        tau = np.zeros_like(eps)
        for p in range(dC.shape[0]):
            msk = phase == p
            tau[:, msk] = dC[p] @ eps[:, msk]
        th = sfft.fft2(tau, axes=(1, 2))
        eh = np.einsum("vwxy,wxy->vxy", G, th)
        new = E[:, None, None] - sfft.ifft2(eh, axes=(1, 2))
        res = np.linalg.norm(new - eps) / normE
        hist.append(res)
        eps = new
        m += 1
        if fixed_iters is not None:
            if m >= fixed_iters:
                break
        elif res < tol or m >= max_iter:
            break
    return eps, m, hist


def effective_stiffness2(phase: np.ndarray, lame, lame0, tol: float, max_iter: int = 2000,
                         fixed_iters: int | None = None, scheme: str = "direct",
                         keep_fields: bool = False):
    """Plane-strain C_eff (3 x 3, columns = unit load cases) from Alg. 1
    with the Green operator of ``scheme``; with ``keep_fields`` also the
    three strain fields (3, N, N)."""
    G = green_table2(phase.shape, *lame0, scheme)
    Cp = np.stack([iso_voigt2(l, m) for l, m in np.asarray(lame)])
    C = np.zeros((3, 3))
    its = []
    fields = []
    for k in range(3):
        E = np.zeros(3)
        E[k] = 1.0
        eps, m, _ = basic_scheme2(phase, lame, lame0, E, tol, max_iter, G=G, fixed_iters=fixed_iters)
        if keep_fields:
            fields.append(eps)
        s = np.zeros(3, dtype=np.complex128)
        for p in range(Cp.shape[0]):
            msk = phase == p
            if msk.any():
                s += Cp[p] @ eps[:, msk].sum(axis=1)
        C[:, k] = (s / phase.size).real
        its.append(m)
    if keep_fields:
        return C, its, fields
    return C, its


# ---------------------------------------------------------------------------
# Gradients of the plane-strain C_eff with respect to the phase Lame
# parameters, C0 held fixed; theta = (lam_0, mu_0, lam_1, mu_1, ...).
# ---------------------------------------------------------------------------

def gradient_energy2(phase: np.ndarray, fields: list) -> np.ndarray:
    """dC_kl/dtheta = < eps^k : dC/dtheta : eps^l > over the pixels (the
    energy identity of the converged fixed point, C0 fixed), (3, 3,
    2 * nphase)."""
    nphase = int(phase.max()) + 1
    basis = (iso_voigt2(1.0, 0.0), iso_voigt2(0.0, 1.0))
    out = np.zeros((3, 3, 2 * nphase))
    re = [f.real for f in fields]
    for p in range(nphase):
        m = phase == p
        if not m.any():
            continue
        for t, dC in enumerate(basis):
            for k in range(3):
                for l in range(3):
                    out[k, l, 2 * p + t] = np.einsum("vx,vw,wx->", re[k][:, m], dC,
                                                     re[l][:, m]) / phase.size
    return out


def gradient_fd2(phase: np.ndarray, lame, lame0, tol: float, rel_step: float = 1e-6,
                 max_iter: int = 5000, scheme: str = "direct") -> np.ndarray:
    """Central finite differences of the plane-strain C_eff in each phase
    (lam, mu), C0 fixed."""
    lame = np.asarray(lame, dtype=np.float64)
    out = np.zeros((3, 3, 2 * lame.shape[0]))
    for p in range(lame.shape[0]):
        for t in range(2):
            h = rel_step * max(abs(lame[p, t]), 1e-3)
            lp, lm = lame.copy(), lame.copy()
            lp[p, t] += h
            lm[p, t] -= h
            Cp, _ = effective_stiffness2(phase, lp, lame0, tol, max_iter, scheme=scheme)
            Cm, _ = effective_stiffness2(phase, lm, lame0, tol, max_iter, scheme=scheme)
            out[:, :, 2 * p + t] = (Cp - Cm) / (2.0 * h)
    return out
