"""Voigt notation and isotropic stiffness (Sec. 2, Voigt notation paragraph).

Order (11, 22, 33, 23, 13, 12).  Strains carry engineering shear
(gamma_ij = 2 eps_ij), stresses are plain, so that sigma_V = C_V eps_V and
C_V[I, J] = C_ijkl for I <-> (ij), J <-> (kl).
"""
from __future__ import annotations

import numpy as np

PAIRS = [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]
# weight of a Voigt strain entry relative to the tensor entry
W = np.array([1.0, 1.0, 1.0, 2.0, 2.0, 2.0])


def lame_from_young(E: float, nu: float) -> tuple[float, float]:
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    return lam, mu


def iso_tensor(lam: float, mu: float) -> np.ndarray:
    """C_ijkl = lam d_ij d_kl + mu (d_ik d_jl + d_il d_jk)."""
    d = np.eye(3)
    return (lam * np.einsum("ij,kl->ijkl", d, d)
            + mu * (np.einsum("ik,jl->ijkl", d, d) + np.einsum("il,jk->ijkl", d, d)))


def tensor_to_voigt_stiffness(C: np.ndarray) -> np.ndarray:
    """C_V[I, J] = C_ijkl."""
    out = np.empty((6, 6))
    for I, (i, j) in enumerate(PAIRS):
        for J, (k, l) in enumerate(PAIRS):
            out[I, J] = C[i, j, k, l]
    return out


def iso_voigt(lam: float, mu: float) -> np.ndarray:
    return tensor_to_voigt_stiffness(iso_tensor(lam, mu))


def strain_tensor_to_voigt(e: np.ndarray) -> np.ndarray:
    """3x3 (...,3,3) strain -> engineering Voigt (..., 6)."""
    return np.stack([W[I] * e[..., i, j] for I, (i, j) in enumerate(PAIRS)], axis=-1)


def strain_voigt_to_tensor(v: np.ndarray) -> np.ndarray:
    e = np.zeros(v.shape[:-1] + (3, 3), dtype=v.dtype)
    for I, (i, j) in enumerate(PAIRS):
        e[..., i, j] = v[..., I] / W[I]
        e[..., j, i] = v[..., I] / W[I]
    return e


def stress_tensor_to_voigt(s: np.ndarray) -> np.ndarray:
    return np.stack([s[..., i, j] for (i, j) in PAIRS], axis=-1)


def stress_voigt_to_tensor(v: np.ndarray) -> np.ndarray:
    s = np.zeros(v.shape[:-1] + (3, 3), dtype=v.dtype)
    for I, (i, j) in enumerate(PAIRS):
        s[..., i, j] = v[..., I]
        s[..., j, i] = v[..., I]
    return s


def dC_dlam() -> np.ndarray:
    """Derivative of the isotropic Voigt stiffness with respect to lambda."""
    return iso_voigt(1.0, 0.0)


def dC_dmu() -> np.ndarray:
    """Derivative of the isotropic Voigt stiffness with respect to mu."""
    return iso_voigt(0.0, 1.0)
