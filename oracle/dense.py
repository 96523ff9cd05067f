"""Dense-voxel FFT-based homogenization in FP64 (oracle; test infrastructure).

Follows the paper:
* Lippmann-Schwinger equation eps = E - Gamma0 * [(C - C0) eps] and the
  FFT-based basic scheme, Sec. 2, Alg. 1.
* Effective stiffness column k = volume average of C eps for unit macro
  strain E = e_k, Sec. 2 (text after Alg. 1).
* Green operator in Fourier space, App. A, eq. orig_green_eshelby with the
  direct scheme k_j = i q_j (Table 3), and the Hermitian symmetrisation at
  the Nyquist frequencies given in App. A; the staggered-grid scheme of
  Table 3 from its discrete gradient (``gamma_table_staggered``).

Readings (where the paper is silent or garbled):
* Stopping test of Alg. 1: ||eps_{m+1} - eps_m||_F / ||E||_F with both
  norms taken over all voxels and the six stored Voigt components.
* Nyquist rule: G_h(idx) = (G(xi(idx)) + conj G(xi(-idx mod N))) / 2 where
  xi(idx) is the representative frequency of DFT index idx.  Off the Nyquist
  planes this is the identity; it makes G_h Hermitian in the DFT sense.
* Voigt Green operator: G_V[I, J] = w_I w_J Gamma_ijkl, w = (1,1,1,2,2,2):
  it maps a plain-Voigt polarization to an engineering-Voigt strain.
"""
from __future__ import annotations

import os

import numpy as np
import scipy.fft as sfft

from .voigt import PAIRS, W, iso_voigt

_WORKERS = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else 1


def set_workers(n: int) -> None:
    """Number of threads scipy.fft uses in this module."""
    global _WORKERS
    _WORKERS = max(1, int(n))


def frequencies(N: int) -> np.ndarray:
    """Representative integer frequency of each DFT index (Nyquist -> -N/2)."""
    idx = np.arange(N)
    return np.where(idx < (N + 1) // 2, idx, idx - N).astype(np.float64)


def gamma_tensor(xi: np.ndarray, lam0: float, mu0: float) -> np.ndarray:
    """Moulinec-Suquet closed form Gamma_ijkl(xi) for isotropic C0.

    Gamma_ijkl = [d_ki x_l x_j + d_li x_k x_j + d_kj x_l x_i + d_lj x_k x_i]
                 / (4 mu0 |x|^2)
                 - (lam0 + mu0) / (mu0 (lam0 + 2 mu0)) x_i x_j x_k x_l / |x|^4
    with Gamma(0) = 0.  ``xi`` has shape (P, 3); returns (P, 3, 3, 3, 3).
    This is App. A eq. orig_green_eshelby for the direct scheme.
    """
    xi = np.asarray(xi, dtype=np.float64)
    n2 = (xi * xi).sum(axis=1)
    safe = np.where(n2 > 0, n2, 1.0)
    d = np.eye(3)
    xx = np.einsum("pi,pj->pij", xi, xi)
    t1 = (np.einsum("ki,plj->pijkl", d, xx) + np.einsum("li,pkj->pijkl", d, xx)
          + np.einsum("kj,pli->pijkl", d, xx) + np.einsum("lj,pki->pijkl", d, xx))
    t1 /= (4.0 * mu0 * safe)[:, None, None, None, None]
    t2 = np.einsum("pij,pkl->pijkl", xx, xx)
    t2 *= ((lam0 + mu0) / (mu0 * (lam0 + 2.0 * mu0)) / (safe * safe))[:, None, None, None, None]
    g = t1 - t2
    g[n2 == 0] = 0.0
    return g


def gamma_tensor_acoustic(xi: np.ndarray, C0: np.ndarray) -> np.ndarray:
    """Gamma_ijkl = sym[ xi_i (xi_m C0_mjkn xi_n)^-1 xi_l ] evaluated numerically.

    App. A eq. orig_green_eshelby taken literally: acoustic tensor inverted
    per frequency, symmetrised over (i, j) and (k, l).  ``C0`` is a full
    3x3x3x3 stiffness tensor.  Used to pin ``gamma_tensor``.
    """
    xi = np.asarray(xi, dtype=np.float64)
    out = np.zeros((xi.shape[0], 3, 3, 3, 3))
    for p, x in enumerate(xi):
        if not np.any(x):
            continue
        K = np.einsum("m,mjkn,n->jk", x, C0, x)
        Ki = np.linalg.inv(K)
        raw = np.einsum("i,jk,l->ijkl", x, Ki, x)
        s = 0.25 * (raw + raw.transpose(1, 0, 2, 3) + raw.transpose(0, 1, 3, 2)
                    + raw.transpose(1, 0, 3, 2))
        out[p] = s
    return out


def gamma_voigt(xi: np.ndarray, lam0: float, mu0: float) -> np.ndarray:
    """Voigt form G_V[I, J] = w_I w_J Gamma_ijkl(xi); shape (P, 6, 6)."""
    g = gamma_tensor(xi, lam0, mu0)
    out = np.empty((g.shape[0], 6, 6))
    for I, (i, j) in enumerate(PAIRS):
        for J, (k, l) in enumerate(PAIRS):
            out[:, I, J] = W[I] * W[J] * g[:, i, j, k, l]
    return out


def gamma_voigt_direct(x: np.ndarray, y: np.ndarray, z: np.ndarray, lam0: float,
                       mu0: float) -> np.ndarray:
    """Same operator as ``gamma_voigt``, written entry by entry in Voigt form
    on arrays of frequency components (any common shape); returns
    (6, 6) + shape.  Used for whole grids."""
    xs = (x, y, z)
    n2 = x * x + y * y + z * z
    safe = np.where(n2 > 0, n2, 1.0)
    c = (lam0 + mu0) / (mu0 * (lam0 + 2.0 * mu0))
    d = np.eye(3)
    out = np.empty((6, 6) + np.shape(x))
    for I, (i, j) in enumerate(PAIRS):
        for J, (k, l) in enumerate(PAIRS):
            t1 = (d[k, i] * xs[l] * xs[j] + d[l, i] * xs[k] * xs[j]
                  + d[k, j] * xs[l] * xs[i] + d[l, j] * xs[k] * xs[i]) / (4.0 * mu0 * safe)
            t2 = c * xs[i] * xs[j] * xs[k] * xs[l] / (safe * safe)
            out[I, J] = np.where(n2 > 0, W[I] * W[J] * (t1 - t2), 0.0)
    return out


def gamma_table(N, lam0: float, mu0: float) -> np.ndarray:
    """Nyquist-symmetrised Voigt Green table on the DFT grid.

    ``N`` is an int (cubic grid) or a shape (Nx, Ny, Nz).  Returns a complex
    array (6, 6, Nx, Ny, Nz) indexed by DFT indices (numpy ``fftn`` order).
    For the direct scheme it is real.
    """
    shape = (N, N, N) if np.isscalar(N) else tuple(N)
    f = [frequencies(n) for n in shape]
    neg = [fa[(-np.arange(n)) % n] for fa, n in zip(f, shape)]   # xi of index -idx mod N
    out = np.empty((6, 6) + shape, dtype=np.complex128)
    fy, fz = np.meshgrid(f[1], f[2], indexing="ij")
    ny, nz = np.meshgrid(neg[1], neg[2], indexing="ij")
    for ix in range(shape[0]):
        g = gamma_voigt_direct(np.full(fy.shape, f[0][ix]), fy, fz, lam0, mu0)
        gn = gamma_voigt_direct(np.full(fy.shape, neg[0][ix]), ny, nz, lam0, mu0)
        out[:, :, ix] = 0.5 * (g + np.conj(gn))
    return out


# ---------------------------------------------------------------------------
# Discrete Green operators from a discrete gradient (App. A, Table 3)
# ---------------------------------------------------------------------------

def staggered_symbols(q: np.ndarray):
    """Fourier symbols of the staggered grid (App. A, Table 3): the forward
    difference k+ = exp(+i q) - 1 and the backward difference
    k- = 1 - exp(-i q), per axis, for q in radians (any shape)."""
    q = np.asarray(q, dtype=np.float64)
    return np.exp(1j * q) - 1.0, 1.0 - np.exp(-1j * q)


def strain_symbol(k_normal: np.ndarray, k_shear: np.ndarray) -> np.ndarray:
    """Symbol B (..., 6, 3) of a discrete symmetric gradient: the
    engineering-Voigt strain of the displacement mode u exp(i q . x) is B u,
    with normal strains eps_ii = k_normal_i u_i and shears
    gamma_ij = k_shear_j u_i + k_shear_i u_j (i != j).  Arguments (..., 3).
    The staggered grid takes k+ for the normal and k- for the shear strains
    (its Green operator in App. A pairs k+ with i = j and k- otherwise); the
    direct scheme takes k = i q for both."""
    kn = np.asarray(k_normal, dtype=np.complex128)
    ks = np.asarray(k_shear, dtype=np.complex128)
    B = np.zeros(kn.shape[:-1] + (6, 3), dtype=np.complex128)
    for I, (i, j) in enumerate(PAIRS):
        if i == j:
            B[..., I, i] = kn[..., i]
        else:
            B[..., I, i] = ks[..., j]
            B[..., I, j] = ks[..., i]
    return B


def gamma_voigt_symbol(B: np.ndarray, C0: np.ndarray) -> np.ndarray:
    """Green operator of a discrete gradient with symbol B (P, 6, 3) for the
    Voigt stiffness C0 (6, 6): the displacement solving the discrete
    equilibrium B^H (C0 B u + tau) = 0 gives the strain B u = -G tau with
    G = B (B^H C0 B)^-1 B^H (App. A eq. orig_green_eshelby with the
    acoustic tensor B^H C0 B inverted numerically per frequency; 0 where
    B = 0).  It maps a plain-Voigt polarization to an engineering-Voigt
    strain, like ``gamma_voigt``.  Returns (P, V, V) complex for a Voigt
    dimension V (6 in 3D, 3 for plane strain)."""
    B = np.asarray(B, dtype=np.complex128)
    out = np.zeros((B.shape[0], B.shape[1], B.shape[1]), dtype=np.complex128)
    live = np.abs(B).reshape(B.shape[0], -1).max(axis=1) > 0
    Bl = B[live]
    K = np.conj(Bl).transpose(0, 2, 1) @ C0[None] @ Bl
    out[live] = Bl @ np.linalg.inv(K) @ np.conj(Bl).transpose(0, 2, 1)
    return out


def gamma_table_staggered(N, lam0: float, mu0: float) -> np.ndarray:
    """Staggered-grid Voigt Green table on the DFT grid (App. A, Table 3),
    complex (6, 6, Nx, Ny, Nz) in numpy ``fftn`` order.  DFT index m of an
    axis of length N is the frequency q = 2 pi m / N; the symbols are
    2 pi-periodic, so no Nyquist representative has to be chosen and the
    table is Hermitian in the DFT sense by construction."""
    shape = (N, N, N) if np.isscalar(N) else tuple(N)
    C0 = iso_voigt(lam0, mu0)
    qs = [2.0 * np.pi * np.arange(n) / n for n in shape]
    Q = np.stack(np.meshgrid(*qs, indexing="ij"), axis=-1).reshape(-1, 3)
    kp, km = staggered_symbols(Q)
    G = gamma_voigt_symbol(strain_symbol(kp, km), C0)
    return G.reshape(shape + (6, 6)).transpose(3, 4, 0, 1, 2).copy()


SCHEMES = ("direct", "staggered")


def green_table(shape, lam0: float, mu0: float, scheme: str = "direct") -> np.ndarray:
    """Voigt Green table of a discretisation scheme (App. A, Table 3):
    ``direct`` (k = i q, Nyquist-symmetrised) or ``staggered``."""
    if scheme == "direct":
        return gamma_table(shape, lam0, mu0)
    if scheme == "staggered":
        return gamma_table_staggered(shape, lam0, mu0)
    raise ValueError(f"unknown scheme {scheme!r}")


def stiffness_per_phase(lame: np.ndarray) -> np.ndarray:
    return np.stack([iso_voigt(l, m) for l, m in np.asarray(lame)])


def apply_gamma(G: np.ndarray, field: np.ndarray) -> np.ndarray:
    """Real-space Green operator: ifftn(G_h . fftn(field)) for a (6, N,N,N) field."""
    th = sfft.fftn(field, axes=(1, 2, 3), workers=_WORKERS)
    eh = np.einsum("vwxyz,wxyz->vxyz", G, th, optimize=True)
    return sfft.ifftn(eh, axes=(1, 2, 3), workers=_WORKERS)


def apply_local(Cp: np.ndarray, phase: np.ndarray, field: np.ndarray) -> np.ndarray:
    """Pointwise Voigt product C(x) field(x) for per-phase matrices ``Cp``."""
    out = np.zeros_like(field)
    for p in range(Cp.shape[0]):
        m = phase == p
        if not m.any():
            continue
        out[:, m] = Cp[p] @ field[:, m]
    return out


def basic_scheme(phase: np.ndarray, lame: np.ndarray, lame0, E: np.ndarray,
                 tol: float, max_iter: int = 2000, G: np.ndarray | None = None,
                 fixed_iters: int | None = None):
    """Alg. 1: eps_{m+1} = E - F^-1[ G_h F[(C - C0) eps_m] ], eps_0 = E.

    Returns (eps, iterations, residual history).  ``fixed_iters`` runs exactly
    that many updates regardless of the stopping test.
    """
    shape = phase.shape
    lam0, mu0 = lame0
    if G is None:
        G = gamma_table(shape, lam0, mu0)
    dC = stiffness_per_phase(lame) - iso_voigt(lam0, mu0)[None]
    E = np.asarray(E, dtype=np.float64)
    eps = np.broadcast_to(E[:, None, None, None], (6,) + shape).astype(np.complex128)
    normE = np.linalg.norm(E) * np.sqrt(phase.size)
    hist = []
    m = 0
    while True:
        tau = apply_local(dC, phase, eps)
        new = E[:, None, None, None] - apply_gamma(G, tau)
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


def mean_stress(phase: np.ndarray, lame: np.ndarray, eps: np.ndarray) -> np.ndarray:
    """Volume average of C(x) eps(x) (plain Voigt stress), real part."""
    Cp = stiffness_per_phase(lame)
    s = np.zeros(6, dtype=np.complex128)
    total = phase.size
    for p in range(Cp.shape[0]):
        m = phase == p
        if m.any():
            s += Cp[p] @ eps[:, m].sum(axis=1)
    return (s / total).real


def effective_stiffness(phase: np.ndarray, lame: np.ndarray, lame0, tol: float,
                        max_iter: int = 2000, keep_fields: bool = False,
                        fixed_iters: int | None = None, scheme: str = "direct"):
    """C_eff (6x6, columns = unit load cases e_k) from Alg. 1 with the Green
    operator of ``scheme`` (see ``green_table``).

    Returns (C_eff, iterations per load case[, fields]).
    """
    G = green_table(phase.shape, *lame0, scheme)
    C = np.zeros((6, 6))
    iters = []
    fields = []
    for k in range(6):
        E = np.zeros(6)
        E[k] = 1.0
        eps, m, _ = basic_scheme(phase, lame, lame0, E, tol, max_iter, G=G,
                                 fixed_iters=fixed_iters)
        C[:, k] = mean_stress(phase, lame, eps)
        iters.append(m)
        if keep_fields:
            fields.append(eps)
    if keep_fields:
        return C, iters, fields
    return C, iters


# ---------------------------------------------------------------------------
# Gradients with respect to the phase Lame parameters, C0 held fixed.
# theta = (lam_0, mu_0, lam_1, mu_1, ...) over phases.
# ---------------------------------------------------------------------------

def _dC_basis():
    return iso_voigt(1.0, 0.0), iso_voigt(0.0, 1.0)


def gradient_energy(phase: np.ndarray, fields: list) -> np.ndarray:
    """dC_kl/dtheta = < eps^k : dC/dtheta : eps^l > (energy identity).

    Exact at convergence for a self-adjoint Green operator with C0 fixed.
    Returns (6, 6, 2*nphase).
    """
    nphase = int(phase.max()) + 1
    dl, dm = _dC_basis()
    total = phase.size
    out = np.zeros((6, 6, 2 * nphase))
    re = [f.real for f in fields]
    for p in range(nphase):
        m = phase == p
        if not m.any():
            continue
        for t, dC in enumerate((dl, dm)):
            for k in range(6):
                ek = re[k][:, m]
                for l in range(6):
                    out[k, l, 2 * p + t] = np.einsum("vx,vw,wx->", ek, dC, re[l][:, m]) / total
    return out


def gradient_fd(phase: np.ndarray, lame: np.ndarray, lame0, tol: float,
                rel_step: float = 1e-6, max_iter: int = 4000) -> np.ndarray:
    """Central finite differences of C_eff in each phase (lam, mu), C0 fixed."""
    lame = np.asarray(lame, dtype=np.float64)
    nphase = lame.shape[0]
    out = np.zeros((6, 6, 2 * nphase))
    for p in range(nphase):
        for t in range(2):
            h = rel_step * max(abs(lame[p, t]), 1e-3)
            lp = lame.copy()
            lm = lame.copy()
            lp[p, t] += h
            lm[p, t] -= h
            Cp, _ = effective_stiffness(phase, lp, lame0, tol, max_iter)
            Cm, _ = effective_stiffness(phase, lm, lame0, tol, max_iter)
            out[:, :, 2 * p + t] = (Cp - Cm) / (2.0 * h)
    return out


def adjoint_fields(phase: np.ndarray, lame: np.ndarray, lame0, tol: float,
                   max_iter: int = 4000):
    """Adjoint fixed points w_k = C e_k - (C - C0) G[w_k], k = 1..6.

    With G = F^-1 G_h F self-adjoint and C symmetric, w_k solves the
    transpose of the forward system (I + G dC) eps = e.
    """
    G = gamma_table(phase.shape, *lame0)
    Cp = stiffness_per_phase(lame)
    dC = Cp - iso_voigt(*lame0)[None]
    out = []
    for k in range(6):
        e = np.zeros(6)
        e[k] = 1.0
        ce = apply_local(Cp, phase, np.broadcast_to(e[:, None, None, None],
                                                      (6,) + phase.shape).astype(np.complex128))
        w = ce.copy()
        nrm = np.linalg.norm(ce)
        for _ in range(max_iter):
            new = ce - apply_local(dC, phase, apply_gamma(G, w))
            res = np.linalg.norm(new - w) / nrm
            w = new
            if res < tol:
                break
        out.append(w)
    return out


def gradient_adjoint(phase: np.ndarray, lame: np.ndarray, lame0, fields: list,
                     adj: list) -> np.ndarray:
    """dC_kl/dtheta = <e_k . dC eps^l> - <w_k, G[dC eps^l]> (dense adjoint)."""
    G = gamma_table(phase.shape, *lame0)
    nphase = np.asarray(lame).shape[0]
    dl, dm = _dC_basis()
    total = phase.size
    out = np.zeros((6, 6, 2 * nphase))
    for p in range(nphase):
        for t, dC in enumerate((dl, dm)):
            dCp = np.zeros((nphase, 6, 6))
            dCp[p] = dC
            for l in range(6):
                v = apply_local(dCp, phase, fields[l])
                gv = apply_gamma(G, v)
                first = v.sum(axis=(1, 2, 3)) / total
                for k in range(6):
                    second = np.sum(adj[k] * gv) / total
                    out[k, l, 2 * p + t] = (first[k] - second).real
    return out
