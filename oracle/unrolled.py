"""Gradient of the C_eff that a fixed number of updates returns (oracle;
test infrastructure, never called by the library).

The converged-fixed-point gradient (``dense.gradient_energy``) is the
derivative of the limit of Alg. 1.  A solve stopped after M updates returns
C_M = < C eps_M > instead, with eps_0 = E and eps_{m+1} = E - G (C - C0)
eps_m (G the real-space Green operator of Sec. 2, C0 held fixed).  Its
exact derivative is the reverse mode of those M updates:

* the cotangent of eps_M for row k of C_M is the field a_M = C(x) e_k;
* going back, a_m = -(C - C0) G a_{m+1} (G self-adjoint, C symmetric);
* dC_M[k, l] / dtheta = < e_k . dC eps^l_M > - sum_{m < M} < G a^k_{m+1},
  dC eps^l_m >, with dC = dC/dtheta supported on one phase.

Both the three-dimensional problem (Voigt 6) and plane strain (Voigt 3)
are covered; the forward keeps every iterate.  theta = (lam_0, mu_0,
lam_1, mu_1, ...).
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft

from . import dense as D
from . import plane as P2


def _setup(phase, lame, lame0, scheme):
    dim = phase.ndim
    if dim == 3:
        iso, G = D.iso_voigt, D.green_table(phase.shape, *lame0, scheme)
    elif dim == 2:
        iso, G = P2.iso_voigt2, P2.green_table2(phase.shape, *lame0, scheme)
    else:
        raise ValueError("phase must be 2D or 3D")
    Cp = np.stack([iso(l, m) for l, m in np.asarray(lame, dtype=np.float64)])
    dC = Cp - iso(*lame0)[None]
    basis = (iso(1.0, 0.0), iso(0.0, 1.0))
    return dim, Cp.shape[1], G, Cp, dC, basis


def _gamma(G, f, dim):
    axes = tuple(range(1, dim + 1))
    th = sfft.fftn(f, axes=axes)
    return sfft.ifftn(np.einsum("vw...,w...->v...", G, th), axes=axes)


def _local(Cp, phase, f):
    out = np.zeros_like(f)
    for p in range(Cp.shape[0]):
        m = phase == p
        if m.any():
            out[:, m] = Cp[p] @ f[:, m]
    return out


def _dlocal(Dt, phase, p, f):
    """dC/dtheta f for theta = (phase p, modulus basis Dt)."""
    out = np.zeros_like(f)
    m = phase == p
    out[:, m] = Dt @ f[:, m]
    return out


def unrolled_gradient(phase: np.ndarray, lame, lame0, steps: int, scheme: str = "direct"):
    """(C_M (V, V), dC_M/dtheta (V, V, 2 nphase)) after exactly ``steps``
    updates of Alg. 1 for every unit load case."""
    dim, V, G, Cp, dC, basis = _setup(phase, lame, lame0, scheme)
    nphase = Cp.shape[0]
    total = phase.size
    # forward, every iterate kept
    eps = []
    for l in range(V):
        E = np.zeros(V)
        E[l] = 1.0
        e = np.broadcast_to(E.reshape((V,) + (1,) * dim), (V,) + phase.shape).astype(np.complex128)
        hist = [e]
        for _ in range(steps):
            e = E.reshape((V,) + (1,) * dim) - _gamma(G, _local(dC, phase, e), dim)
            hist.append(e)
        eps.append(hist)
    C = np.zeros((V, V))
    for l in range(V):
        C[:, l] = (_local(Cp, phase, eps[l][steps]).reshape(V, -1).sum(axis=1) / total).real
    J = np.zeros((V, V, 2 * nphase))
    thetas = [(p, t) for p in range(nphase) for t in range(2)]
    # explicit term at the last iterate
    for i, (p, t) in enumerate(thetas):
        for l in range(V):
            v = _dlocal(basis[t], phase, p, eps[l][steps])
            J[:, l, i] += (v.reshape(V, -1).sum(axis=1) / total).real
    # reverse sweep, one cotangent train per row k
    for k in range(V):
        ek = np.zeros(V)
        ek[k] = 1.0
        a = _local(Cp, phase, np.broadcast_to(ek.reshape((V,) + (1,) * dim),
                                              (V,) + phase.shape).astype(np.complex128))
        for m in range(steps - 1, -1, -1):
            g = _gamma(G, a, dim)
            for i, (p, t) in enumerate(thetas):
                for l in range(V):
                    v = _dlocal(basis[t], phase, p, eps[l][m])
                    J[k, l, i] -= (np.sum(np.conj(g) * v) / total).real
            a = -_local(dC, phase, g)
    return C, J
