"""Closed forms that pin the dense oracle (test infrastructure).

* Laminate effective stiffness for layers normal to x (exact for a 1D
  microstructure: the basic scheme reaches it after one update, Sec. 5.2).
  Split Voigt indices into n = {11, 13, 12} (traction components, continuous
  across the layers: stresses constant) and t = {22, 33, 23} (in-plane
  strains, continuous: constant).  With <.> the volume average:
      C*_nn = <C_nn^-1>^-1
      C*_nt = C*_nn <C_nn^-1 C_nt>,    C*_tn = C*_nt^T
      C*_tt = <C_tt - C_tn C_nn^-1 C_nt> + <C_tn C_nn^-1> C*_nn <C_nn^-1 C_nt>
* Voigt and Reuss bounds (arithmetic / harmonic averages of the stiffness).
* Hashin-Shtrikman bounds on the bulk and shear moduli of a two-phase
  composite with isotropic phases (Hashin and Shtrikman 1963).
"""
from __future__ import annotations

import numpy as np

from .voigt import iso_voigt

N_IDX = [0, 4, 5]   # 11, 13, 12
T_IDX = [1, 2, 3]   # 22, 33, 23


def laminate_x(C_phases: np.ndarray, fractions: np.ndarray) -> np.ndarray:
    """Effective Voigt stiffness of layers normal to x."""
    f = np.asarray(fractions, dtype=np.float64)
    Cs = np.asarray(C_phases, dtype=np.float64)
    inv_nn = [np.linalg.inv(C[np.ix_(N_IDX, N_IDX)]) for C in Cs]
    Cnn = np.linalg.inv(sum(fi * a for fi, a in zip(f, inv_nn)))
    a_nt = sum(fi * a @ C[np.ix_(N_IDX, T_IDX)] for fi, a, C in zip(f, inv_nn, Cs))
    a_tn = sum(fi * C[np.ix_(T_IDX, N_IDX)] @ a for fi, a, C in zip(f, inv_nn, Cs))
    Cnt = Cnn @ a_nt
    Ctt = sum(fi * (C[np.ix_(T_IDX, T_IDX)] - C[np.ix_(T_IDX, N_IDX)] @ a
                    @ C[np.ix_(N_IDX, T_IDX)]) for fi, a, C in zip(f, inv_nn, Cs))
    Ctt = Ctt + a_tn @ Cnn @ a_nt
    out = np.zeros((6, 6))
    out[np.ix_(N_IDX, N_IDX)] = Cnn
    out[np.ix_(N_IDX, T_IDX)] = Cnt
    out[np.ix_(T_IDX, N_IDX)] = Cnt.T
    out[np.ix_(T_IDX, T_IDX)] = Ctt
    return out


def voigt_bound(C_phases, fractions) -> np.ndarray:
    return sum(f * C for f, C in zip(fractions, C_phases))


def reuss_bound(C_phases, fractions) -> np.ndarray:
    return np.linalg.inv(sum(f * np.linalg.inv(C) for f, C in zip(fractions, C_phases)))


def bulk_shear(lam: float, mu: float) -> tuple[float, float]:
    return lam + 2.0 * mu / 3.0, mu


def hashin_shtrikman(k1, m1, f1, k2, m2, f2):
    """HS (lower, upper) bounds on bulk and shear moduli; returns
    ((k_lo, k_hi), (m_lo, m_hi)).  Phase a is the reference of each formula."""
    def kbound(ka, ma, fa, kb, mb, fb):
        return ka + fb / (1.0 / (kb - ka) + 3.0 * fa / (3.0 * ka + 4.0 * ma))

    def mbound(ka, ma, fa, kb, mb, fb):
        return ma + fb / (1.0 / (mb - ma)
                          + 6.0 * fa * (ka + 2.0 * ma) / (5.0 * ma * (3.0 * ka + 4.0 * ma)))

    soft_is_1 = (k1 <= k2 and m1 <= m2)
    if not soft_is_1:
        k1, m1, f1, k2, m2, f2 = k2, m2, f2, k1, m1, f1
    klo = kbound(k1, m1, f1, k2, m2, f2)
    khi = kbound(k2, m2, f2, k1, m1, f1)
    mlo = mbound(k1, m1, f1, k2, m2, f2)
    mhi = mbound(k2, m2, f2, k1, m1, f1)
    return (klo, khi), (mlo, mhi)


def iso_phases(lame) -> np.ndarray:
    return np.stack([iso_voigt(l, m) for l, m in np.asarray(lame)])
