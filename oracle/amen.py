"""AMEn-adapted approximate matrix-vector product y ~ A x in TT format
(oracle; test infrastructure, never called by the library).

App. B: instead of forming A x (ranks multiply) and rounding it, the cost
||y - A x||^2 = (y, y) - 2 Re (A x, y) + const is minimised core by core.
With every core of y but the k-th orthonormal (frames Y_<k on the left,
Y_>k on the right), the local minimiser satisfies the Galerkin condition
(eq. galerkin_condition): y_k = Y_<k^H (A x) Y_>k, the projection of A x
onto the frame.  Each core update is followed by a rank adaptation: the
local solution is truncated by SVD, the residual z ~ A x - y is carried as
a low-rank train of its own (updated by the same projections in its own
frame), and its core enriches the solution's core before the QR that makes
it orthonormal for the next step (Dolgov and Savostyanov 2014, the AMEn
enrichment).  Sweeps run left to right; before each, y and z are made
right-orthonormal by a QR sweep.

Readings (the appendix gives the steps, not every detail):
* local truncation threshold: delta / sqrt(L - 1) times the norm of the
  local core (= ||y|| in the orthonormal frame), rank clipped to ``cap``;
* enrichment core: the residual A x - y projected with y's left frame and
  z's right frame;
* the approximate residual keeps its ranks (the random initial z fixes
  them, capped by the structural ranks);
* the enriched core is the QR basis of [u, e] (u the kept left singular
  vectors, e the enrichment core), whose first r columns span u; the
  result keeps only those columns on every bond (and the matching rows of
  the next core), i.e. the truncated ranks: the enrichment steers the
  frames of the next sweep but is not part of the returned product, so its
  ranks stay within ``cap`` and no extra rounding follows;
* stopping: the relative change ||y_new - y_old|| / ||y_new|| of the
  returned product between two sweeps below ``tol``, or ``sweeps`` sweeps;
  the sweeps after the first start from the enriched train;
* The random initial y and z are inputs (the caller draws them).

Cores: y, z, x (r, d, r'); A (rho, d_out, d_in, rho').
"""
from __future__ import annotations

import numpy as np

from . import qtt as Q


def _local(PL, Ak, xk, PR):
    """Projection of (A x) at core k onto a left interface PL (a, rho, c)
    and a right interface PR (b, rho', c'): (a, d_out, b)."""
    return np.einsum("apc,pijq,cjd,bqd->aib", PL, Ak, xk, PR, optimize=True)


def _left_step(PL, wk, Ak, xk):
    """Left interface through core k: sum conj(w) PL A x -> (a', rho', c')."""
    return np.einsum("aib,apc,pijq,cjd->bqd", np.conj(wk), PL, Ak, xk, optimize=True)


def _right_step(PR, wk, Ak, xk):
    """Right interface through core k: sum conj(w) A x PR -> (a, rho, c)."""
    return np.einsum("aib,pijq,cjd,bqd->apc", np.conj(wk), Ak, xk, PR, optimize=True)


def _frame_left(PL, zk, yk):
    """z-y interface through core k from the left: (rz', ry')."""
    return np.einsum("aib,ac,cid->bd", np.conj(zk), PL, yk, optimize=True)


def _frame_right(PR, zk, yk):
    """z-y interface through core k from the right: (rz, ry)."""
    return np.einsum("aib,cid,bd->ac", np.conj(zk), yk, PR, optimize=True)


def _right_orthonormal(cores):
    """QR sweep right to left: cores 1..L-1 right-orthonormal (the same
    train)."""
    out = [c.astype(np.complex128).copy() for c in cores]
    for k in range(len(out) - 1, 0, -1):
        r0, d, r1 = out[k].shape
        q, r = np.linalg.qr(out[k].reshape(r0, d * r1).T)
        kk = q.shape[1]
        out[k] = q.T.reshape(kk, d, r1)
        out[k - 1] = np.einsum("aib,cb->aic", out[k - 1], r)
    return out


def _keep(s, thr, cap):
    tail = np.sqrt(np.cumsum((s ** 2)[::-1]))[::-1]
    r = int(np.sum(tail > thr))
    return max(1, min(r, cap, len(s)))


def amen_sweep(A, x, y, z, delta, cap):
    """One left-to-right AMEn sweep (App. B); y and z right-orthonormal on
    entry (cores 1..L-1).  Returns the enriched y (left-orthonormal but the
    last core), the new z, and the kept (truncated) rank of every bond."""
    L = len(x)
    y = [c.copy() for c in y]
    z = [c.copy() for c in z]
    one = np.ones((1, 1, 1), dtype=np.complex128)
    # right interfaces of the current frames
    PyR = [None] * (L + 1)
    PzR = [None] * (L + 1)
    SR = [None] * (L + 1)
    PyR[L] = one
    PzR[L] = one
    SR[L] = np.ones((1, 1), dtype=np.complex128)
    for k in range(L - 1, 0, -1):
        PyR[k] = _right_step(PyR[k + 1], y[k], A[k], x[k])
        PzR[k] = _right_step(PzR[k + 1], z[k], A[k], x[k])
        SR[k] = _frame_right(SR[k + 1], z[k], y[k])
    PyL, PzL, SL = one, one, np.ones((1, 1), dtype=np.complex128)
    thr_scale = delta / np.sqrt(max(L - 1, 1))
    kept = [1] * (L + 1)
    for k in range(L):
        yk = _local(PyL, A[k], x[k], PyR[k + 1])       # Galerkin solution
        if k == L - 1:
            y[k] = yk
            # the residual's last core in its frame
            z[k] = (_local(PzL, A[k], x[k], PzR[k + 1])
                    - np.einsum("ab,bic->aic", SL, yk, optimize=True))
            break
        ry, d, ry2 = yk.shape
        M = yk.reshape(ry * d, ry2)
        U, s, Vh = np.linalg.svd(M, full_matrices=False)
        r = _keep(s, thr_scale * np.linalg.norm(s), cap)
        u = U[:, :r]
        kept[k + 1] = r
        yt = (u @ (s[:r, None] * Vh[:r])).reshape(ry, d, ry2)   # truncated local core
        # approximate residual in z's own frame
        zk = (_local(PzL, A[k], x[k], PzR[k + 1])
              - np.einsum("ab,bic,dc->aid", SL, yt, SR[k + 1], optimize=True))
        # enrichment: residual with y's left frame and z's right frame
        ek = _local(PyL, A[k], x[k], PzR[k + 1]) - np.einsum("bic,dc->bid", yt, SR[k + 1])
        ue = np.concatenate([u, ek.reshape(ry * d, -1)], axis=1)
        qy, _ = np.linalg.qr(ue)
        y[k] = qy.reshape(ry, d, qy.shape[1])
        rz, _, rz2 = zk.shape
        qz, _ = np.linalg.qr(zk.reshape(rz * d, rz2))
        z[k] = qz.reshape(rz, d, qz.shape[1])
        PyL = _left_step(PyL, y[k], A[k], x[k])
        PzL = _left_step(PzL, z[k], A[k], x[k])
        SL = _frame_left(SL, z[k], y[k])
    return y, z, kept


def compact(y, kept):
    """The product without its enrichment: on every bond the first kept[k]
    basis columns (which span the truncated singular vectors) and the
    matching rows of the next core."""
    return [c[:kept[k], :, :kept[k + 1]].copy() for k, c in enumerate(y)]


def amen_mv(A, x, y0, z0, delta, cap=1 << 30, sweeps=4, tol=None):
    """y ~ A x by AMEn sweeps from the initial guesses y0 and z0 (App. B).

    Returns (y, sweeps run, relative change of the last sweep).  ``tol``
    defaults to ``delta``."""
    tol = delta if tol is None else tol
    y = _right_orthonormal(y0)
    z = _right_orthonormal(z0)
    prev = None
    out = None
    change = np.inf
    m = 0
    for m in range(1, sweeps + 1):
        y, z, kept = amen_sweep(A, x, y, z, delta, cap)
        out = compact(y, kept)
        if prev is not None:
            nrm = Q.tt_norm(out)
            change = Q.tt_norm(Q.tt_add(out, Q.tt_scale(prev, -1.0))) / max(nrm, 1e-300)
            if change < tol:
                break
        prev = [c.copy() for c in out]
        if m < sweeps:
            y = _right_orthonormal(y)
            z = _right_orthonormal(z)
    return out, m, change
