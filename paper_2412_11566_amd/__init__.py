"""qtthom: SFFT-based homogenization on quantized tensor trains, MI355X-native.

Thin Python binding over the C ABI of ``include/qtthom.h`` (same names).  It
only marshals arguments: the tensor-train arithmetic, the operators and the
Lippmann-Schwinger loop run in the HIP library ``libqtthom.so``.  PyTorch
is used for the device and stream handle only (``torch.cuda`` current
stream), never for compute.

Method: Hauck, Kabel, Ali, Gauger, "SFFT-based homogenization" (arXiv
2412.11566): Sec. 2 Alg. 1 (basic scheme), Sec. 4.3 Alg. 2 (the same fixed
point on controlled QTT strain fields).
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np

from . import _capi as _c
from ._capi import (QTT_EXACT, QTT_INVERSE, QTT_NO_ROUND, QTT_OK, QTT_ENOCONV,
                    QTT_ORTH_AUTO, QTT_ORTH_CHOLQR, QTT_ORTH_HOUSEHOLDER, QTT_PREC_BF16X3, QTT_PREC_FP32,
                    QTT_PREC_FP64, QTT_SCHEME_DIRECT, QTT_SCHEME_STAGGERED, QTT_MV_SKETCH,
                    QTT_MV_AMEN)

__all__ = [
    "QttError", "Context", "Tensor", "SolveOptions", "SolveReport",
    "tt_from_cores", "const_strain", "sfft_build", "green_build", "from_voxels", "rank_estimate",
    "sfft_apply", "tt_hadamard", "green_apply", "amen_apply", "tt_round", "tt_norm", "tt_axpby",
    "tt_mean_apply", "ls_solve", "ls_adjoint", "ls_unrolled", "ls_unrolled_prepared", "batch_solve", "Prepared", "prepare",
    "ls_solve_prepared", "stats_enable", "stats_get", "stats_reset", "tensor_create",
    "tensor_wrap", "tensor_export", "NotConvergedWarning",
    "QTT_EXACT", "QTT_INVERSE", "QTT_NO_ROUND", "QTT_ORTH_AUTO", "QTT_ORTH_CHOLQR", "QTT_ORTH_HOUSEHOLDER",
    "QTT_PREC_BF16X3", "QTT_PREC_FP32", "QTT_PREC_FP64", "QTT_SCHEME_DIRECT", "QTT_SCHEME_STAGGERED",
    "SCHEMES", "QTT_MV_SKETCH", "QTT_MV_AMEN",
]


class QttError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"qtthom error {_c.ERR_NAMES.get(code, code)}: {msg}")
        self.code = code


class NotConvergedWarning(RuntimeWarning):
    """A fixed point (forward or adjoint) stopped at max_iter."""


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_int))


class Context:
    """A qtthom context on one HIP device and stream."""

    def __init__(self, device: int = 0, stream: int | None = None):
        import torch  # device/stream plumbing only
        if not torch.cuda.is_available():
            raise QttError(_c.QTT_EHIP, "no HIP device visible")
        if stream is None:
            stream = torch.cuda.current_stream(device).cuda_stream
        h = C.c_void_p()
        rc = _c.lib().qtt_create(device, C.c_void_p(stream) if stream else None, C.byref(h))
        if rc != QTT_OK:
            raise QttError(rc, "qtt_create failed")
        self.h = h

    def check(self, rc: int, allow=()):
        if rc != QTT_OK and rc not in allow:
            msg = _c.lib().qtt_last_error(self.h)
            raise QttError(rc, msg.decode() if msg else "")
        return rc

    def sync(self):
        self.check(_c.lib().qtt_sync(self.h))

    def close(self):
        if getattr(self, "h", None):
            _c.lib().qtt_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Tensor:
    """Owning handle of a qtt_tensor (train batch or operator)."""

    def __init__(self, ctx: Context, h: C.c_void_p):
        self.ctx = ctx
        self.h = h

    def __del__(self):
        # at interpreter shutdown the module globals may already be gone
        if getattr(self, "h", None) and _c is not None:
            try:
                _c.lib().qtt_tensor_destroy(self.h)
            except Exception:
                pass
            self.h = None

    def shape(self):
        kind, L, B = C.c_int(), C.c_int(), C.c_int()
        _c.lib().qtt_tensor_shape(self.h, C.byref(kind), C.byref(L), C.byref(B),
                                  None, None, None)
        dout = np.zeros(L.value, np.int32)
        din = np.zeros(L.value, np.int32)
        ranks = np.zeros(L.value + 1, np.int32)
        _c.lib().qtt_tensor_shape(self.h, None, None, None, _ip(dout), _ip(din), _ip(ranks))
        return {"kind": kind.value, "L": L.value, "batch": B.value,
                "dims_out": dout.tolist(), "dims_in": din.tolist(), "ranks": ranks.tolist()}

    @property
    def ranks(self):
        return self.shape()["ranks"]

    def nbytes(self) -> int:
        """Bytes of all cores (the qtt_tt_from_host layout)."""
        return 16 * int(_c.lib().qtt_tensor_size(self.h))

    def cores(self):
        """Host copies: trains -> list of (B, r0, d, r1); operators -> (r0, dout, din, r1)."""
        s = self.shape()
        n = _c.lib().qtt_tensor_size(self.h)
        buf = np.zeros(2 * n, np.float64)
        self.ctx.check(_c.lib().qtt_tensor_to_host(self.ctx.h, self.h, _dp(buf), n))
        z = buf.view(np.complex128)
        out, off = [], 0
        r = s["ranks"]
        for k in range(s["L"]):
            if s["kind"] == 0:
                shp = (s["batch"], r[k], s["dims_out"][k], r[k + 1])
            else:
                shp = (r[k], s["dims_out"][k], s["dims_in"][k], r[k + 1])
            cnt = int(np.prod(shp))
            out.append(z[off:off + cnt].reshape(shp).copy())
            off += cnt
        return out


def _new(ctx: Context, fn, *args) -> Tensor:
    h = C.c_void_p()
    ctx.check(fn(ctx.h, *args, C.byref(h)))
    return Tensor(ctx, h)


def tt_from_cores(ctx: Context, cores) -> Tensor:
    """Upload a batch of trains; cores[k] has shape (B, r_{k-1}, d_k, r_k)."""
    cores = [np.ascontiguousarray(c, dtype=np.complex128) for c in cores]
    B = cores[0].shape[0]
    dims = np.array([c.shape[2] for c in cores], np.int32)
    ranks = np.array([cores[0].shape[1]] + [c.shape[3] for c in cores], np.int32)
    data = np.concatenate([c.ravel() for c in cores]).view(np.float64)
    return _new(ctx, _c.lib().qtt_tt_from_host, len(cores), _ip(dims), _ip(ranks), B, _dp(data))


def _train_shape(dims, ranks):
    dims = np.ascontiguousarray(dims, dtype=np.int32)
    ranks = np.ascontiguousarray(ranks, dtype=np.int32)
    if ranks.shape[0] != dims.shape[0] + 1:
        raise ValueError("ranks must have len(dims) + 1 entries")
    return dims, ranks


def tensor_create(ctx: Context, dims, ranks, batch: int = 1) -> Tensor:
    """Zero-filled trains in library device memory (qtt_tensor_create)."""
    d, r = _train_shape(dims, ranks)
    return _new(ctx, _c.lib().qtt_tensor_create, len(d), _ip(d), _ip(r), int(batch))


def tensor_wrap(ctx: Context, buf, dims, ranks, batch: int = 1) -> Tensor:
    """Trains over a caller-owned device buffer (qtt_tensor_wrap): ``buf`` is
    a contiguous complex128 torch device tensor holding the cores one after
    another, each (batch, r_{k-1}, d_k, r_k).  No copy; the returned handle
    keeps a reference to ``buf``."""
    import torch
    if buf.dtype != torch.complex128 or not buf.is_cuda or not buf.is_contiguous():
        raise ValueError("tensor_wrap: a contiguous complex128 device tensor")
    d, r = _train_shape(dims, ranks)
    t = _new(ctx, _c.lib().qtt_tensor_wrap, len(d), _ip(d), _ip(r), int(batch),
             C.c_void_p(buf.data_ptr()), buf.numel() * 16)
    t._owner = buf
    return t


def tensor_export(ctx: Context, t: Tensor, out=None):
    """All cores of a train copied device-to-device into a complex128 torch
    tensor (qtt_tensor_export); returns that tensor (flat)."""
    import torch
    n = int(_c.lib().qtt_tensor_size(t.h))
    if out is None:
        out = torch.empty(n, dtype=torch.complex128, device="cuda")
    if out.dtype != torch.complex128 or not out.is_cuda or not out.is_contiguous():
        raise ValueError("tensor_export: a contiguous complex128 device tensor")
    ctx.check(_c.lib().qtt_tensor_export(ctx.h, t.h, C.c_void_p(out.data_ptr()), out.numel() * 16))
    return out


def const_strain(ctx: Context, n: int, E) -> Tensor:
    E = np.ascontiguousarray(np.atleast_2d(E), dtype=np.float64)
    return _new(ctx, _c.lib().qtt_const_strain, n, E.shape[0], _dp(E))


def sfft_build(ctx: Context, n: int, delta: float) -> Tensor:
    return _new(ctx, _c.lib().qtt_sfft_build, n, delta)


# Green-operator discretisations (App. A, Table 3)
SCHEMES = {"direct": 0, "staggered": 1}


def _scheme(scheme) -> int:
    if isinstance(scheme, str):
        if scheme not in SCHEMES:
            raise ValueError(f"scheme: one of {sorted(SCHEMES)}")
        return SCHEMES[scheme]
    return int(scheme)


def green_build(ctx: Context, n: int, lam0: float, mu0: float, delta: float,
                scheme="direct") -> Tensor:
    return _new(ctx, _c.lib().qtt_green_build_scheme, n, lam0, mu0, delta, _scheme(scheme))


def from_voxels(ctx: Context, phase, lame, lame0, delta: float, cap: int = 0):
    """(C - C0) raised operator and the one-hot phase train; ``phase`` is a
    host array or a torch uint8 device tensor (read in place), cubic (3D,
    Voigt 6) or square (plane strain, Voigt 3)."""
    p, keep = _problem(phase, lame, lame0, 0)
    l0 = np.ascontiguousarray(lame0, dtype=np.float64)
    h, chi = C.c_void_p(), C.c_void_p()
    ctx.check(_c.lib().qtt_from_voxels_dim(
        ctx.h, p.phase, p.phase_on_device, p.n, p.nphase, p.lame, _dp(l0), delta, cap, p.dim,
        C.byref(h), C.byref(chi)))
    del keep
    return Tensor(ctx, h), Tensor(ctx, chi)


def rank_estimate(ctx: Context, phase, nphase: int, delta: float):
    """Largest one-hot bond rank of the geometry at its order n and at
    order n - 1 (2 x 2 x 2 majority coarsening of a cubic voxel array, 2 x 2
    of a square pixel array), and their ratio; ``phase`` is a host array or
    a torch uint8 device tensor."""
    p, keep = _problem(phase, np.zeros((nphase, 2)), (1.0, 1.0), 0)
    r = (C.c_int * 2)()
    g = C.c_double(0.0)
    ctx.check(_c.lib().qtt_rank_estimate_dim(ctx.h, p.phase, p.phase_on_device, p.n, nphase, delta,
                                             p.dim, C.cast(r, C.POINTER(C.c_int)), C.byref(g)))
    del keep
    return int(r[0]), int(r[1]), g.value


def _prod(fn, ctx, A, x, flags, delta, cap, seed):
    h = C.c_void_p()
    ctx.check(fn(ctx.h, A.h, x.h, C.byref(h), flags, delta, cap, seed))
    return Tensor(ctx, h)


def sfft_apply(ctx, S, x, inverse=False, delta=1e-10, cap=0, seed=0, flags=0) -> Tensor:
    return _prod(_c.lib().sfft_apply, ctx, S, x, flags | (QTT_INVERSE if inverse else 0),
                 delta, cap, seed)


def tt_hadamard(ctx, A, x, delta=1e-10, cap=0, seed=0, flags=0) -> Tensor:
    return _prod(_c.lib().tt_hadamard, ctx, A, x, flags, delta, cap, seed)


def green_apply(ctx, G, x, delta=1e-10, cap=0, seed=0, flags=0) -> Tensor:
    return _prod(_c.lib().green_apply, ctx, G, x, flags, delta, cap, seed)


def amen_apply(ctx, A, x, y0, z0, delta: float, cap: int = 0, sweeps: int = 4, tol=None):
    """y ~ A x by the AMEn-adapted product (App. B) from the initial guesses
    y0, z0 (trains); returns (y, sweeps run, last relative change)."""
    h = C.c_void_p()
    m = C.c_int(0)
    ch = C.c_double(0.0)
    ctx.check(_c.lib().tt_amen_apply(ctx.h, A.h, x.h, y0.h, z0.h, delta, cap, sweeps,
                                     delta if tol is None else tol, C.byref(h), C.byref(m),
                                     C.byref(ch)))
    return Tensor(ctx, h), m.value, ch.value


def tt_round(ctx, x: Tensor, delta: float, cap: int = 0) -> np.ndarray:
    B = x.shape()["batch"]
    disc = np.zeros(B)
    ctx.check(_c.lib().tt_round(ctx.h, x.h, delta, cap, _dp(disc)))
    return disc


def tt_norm(ctx, x: Tensor) -> np.ndarray:
    out = np.zeros(x.shape()["batch"])
    ctx.check(_c.lib().tt_norm(ctx.h, x.h, _dp(out)))
    return out


def tt_axpby(ctx, alpha, x, beta, y) -> Tensor:
    h = C.c_void_p()
    ctx.check(_c.lib().tt_axpby(ctx.h, alpha, x.h, beta, y.h, C.byref(h)))
    return Tensor(ctx, h)


def tt_mean_apply(ctx, A, x) -> np.ndarray:
    B = x.shape()["batch"]
    out = np.zeros(2 * 6 * B)
    ctx.check(_c.lib().tt_mean_apply(ctx.h, A.h, x.h, _dp(out)))
    return out.view(np.complex128).reshape(B, 6)


@dataclass
class SolveOptions:
    delta: float = 1e-8
    tol: float = 1e-6
    cap: int = 64
    max_iter: int = 1000
    precision: int = QTT_PREC_FP64
    oversample: int = 16
    exact: bool = False
    seed: int = 0
    streams: int = 1
    # entries of the per-load-case residual history to record (0: none)
    history: int = 0
    # range-finder orthonormalisation: QTT_ORTH_AUTO (default),
    # QTT_ORTH_HOUSEHOLDER or QTT_ORTH_CHOLQR
    orth: int = 0
    # the Green step's products: QTT_MV_SKETCH (default) or QTT_MV_AMEN
    matvec: int = 0
    # batch_solve: split grid-size groups by the geometry-rank bucket
    rank_buckets: bool = False

    def c(self) -> _c.SolveOpts:
        o = _c.SolveOpts(self.delta, self.tol, self.cap, self.max_iter, self.precision,
                         self.oversample, int(self.exact), self.seed, self.streams)
        o.orth = self.orth
        o.matvec = self.matvec
        o.rank_buckets = int(self.rank_buckets)
        if self.history > 0:
            buf = np.zeros(6 * self.history)
            o.history = _dp(buf)
            o.history_len = self.history
            o._hist = buf  # kept alive with the struct
        return o


@dataclass
class SolveReport:
    iterations: list
    residual: list
    max_rank: int
    discarded: float
    status: int
    seconds_setup: float
    seconds_solve: float
    # (6, history) relative updates per load case, NaN past the last
    # update (SolveOptions.history > 0 only)
    history: np.ndarray | None = None


def _problem(phase, lame, lame0, load_mask, scheme="direct"):
    """qtt_problem from a host array or a torch uint8 device tensor (then
    the library reads the voxels from device memory)."""
    on_dev = not isinstance(phase, np.ndarray) and getattr(phase, "is_cuda", False)
    if on_dev:
        import torch
        if phase.dtype != torch.uint8 or not phase.is_contiguous():
            raise ValueError("device phase: a contiguous uint8 tensor")
        shape = tuple(phase.shape)
        ptr = C.cast(C.c_void_p(phase.data_ptr()), C.POINTER(C.c_uint8))
    else:
        phase = np.ascontiguousarray(phase, dtype=np.uint8)
        shape = phase.shape
        ptr = phase.ctypes.data_as(C.POINTER(C.c_uint8))
    n = int(round(np.log2(shape[0])))
    dim = len(shape)
    if dim not in (2, 3) or shape != (1 << n,) * dim:
        raise ValueError("phase must be a cubic (or, for plane strain, square) array with side 2**n")
    lame = np.ascontiguousarray(lame, dtype=np.float64)
    p = _c.Problem(n, ptr, lame.shape[0], _dp(lame), (C.c_double * 2)(*lame0), load_mask,
                   int(on_dev), _scheme(scheme), dim)
    return p, (phase, lame)


def _report(r: _c.Report, o: _c.SolveOpts | None = None) -> SolveReport:
    h = None
    if o is not None and getattr(o, "_hist", None) is not None:
        h = o._hist.reshape(6, -1).copy()
    return SolveReport(list(r.iterations), list(r.residual), r.max_rank, r.discarded, r.status,
                       r.seconds_setup, r.seconds_solve, h)


def ls_solve(ctx: Context, phase, lame, lame0, opts: SolveOptions, load_mask: int = 0x3F,
             keep_eps: bool = False, scheme="direct"):
    """Alg. 2 for the selected unit load cases with the Green operator of
    ``scheme`` (``SCHEMES``); returns (C_eff, report, eps).  A square
    (N, N) ``phase`` is a plane-strain problem: C_eff is then 3 x 3 (Voigt
    11, 22, 12) and load_mask bits 0..2 select its load cases."""
    p, keep = _problem(phase, lame, lame0, load_mask, scheme)
    o = opts.c()
    Ceff = np.zeros(36)
    rep = _c.Report()
    eps = C.c_void_p()
    rc = _c.lib().ls_solve(ctx.h, C.byref(p), C.byref(o), _dp(Ceff), C.byref(rep),
                           C.byref(eps) if keep_eps else None)
    ctx.check(rc, allow=(QTT_ENOCONV,))
    del keep
    C6 = Ceff.reshape(6, 6)
    return (C6[:3, :3].copy() if p.dim == 2 else C6), _report(rep, o), (Tensor(ctx, eps) if keep_eps else None)


def ls_adjoint(ctx: Context, phase, lame, lame0, opts: SolveOptions, eps: Tensor, gbar=None,
               scheme="direct"):
    """Adjoint LS solve; returns the Jacobian (V, V, 2*nphase) or the
    gradient (2*nphase,) when the cotangent ``gbar`` (V, V) is given; V = 6,
    or 3 for a plane-strain (square) phase array."""
    p, keep = _problem(phase, lame, lame0, 0x3F, scheme)
    o = opts.c()
    nt = 2 * np.asarray(lame).shape[0]
    V = 3 if p.dim == 2 else 6
    rep = _c.Report()
    if gbar is None:
        out = np.zeros(V * V * nt)
        rc = _c.lib().ls_adjoint(ctx.h, C.byref(p), C.byref(o), eps.h, None, _dp(out), C.byref(rep))
        ctx.check(rc, allow=(QTT_ENOCONV,))
        return out.reshape(V, V, nt), _report(rep)
    g = np.ascontiguousarray(gbar, dtype=np.float64).reshape(V * V)
    out = np.zeros(nt)
    rc = _c.lib().ls_adjoint(ctx.h, C.byref(p), C.byref(o), eps.h, _dp(g), _dp(out), C.byref(rep))
    ctx.check(rc, allow=(QTT_ENOCONV,))
    del keep
    return out, _report(rep)


def batch_solve(ctx: Context, problems, opts: SolveOptions, scheme="direct"):
    """Many structures: problems = [(phase, lame, lame0)]; returns (C_eff[count], reports)."""
    ps, keeps = [], []
    for phase, lame, lame0 in problems:
        p, k = _problem(phase, lame, lame0, 0x3F, scheme)
        ps.append(p)
        keeps.append(k)
    arr = (_c.Problem * len(ps))(*ps)
    reps = (_c.Report * len(ps))()
    Ceff = np.zeros(36 * len(ps))
    o = opts.c()
    rc = _c.lib().qtt_batch_solve(ctx.h, len(ps), arr, C.byref(o), _dp(Ceff), reps)
    ctx.check(rc, allow=(QTT_ENOCONV,))
    return Ceff.reshape(-1, 6, 6), [_report(r) for r in reps]


class Prepared:
    """Operators of one problem built once (qtt_prepare)."""

    def __init__(self, ctx: Context, h: C.c_void_p, keep):
        self.ctx = ctx
        self.h = h
        self._keep = keep

    def __del__(self):
        if getattr(self, "h", None) and _c is not None:
            try:
                _c.lib().qtt_prepared_destroy(self.h)
            except Exception:
                pass
            self.h = None


def prepare(ctx: Context, phase, lame, lame0, delta: float, load_mask: int = 0x3F,
            scheme="direct") -> Prepared:
    p, keep = _problem(phase, lame, lame0, load_mask, scheme)
    h = C.c_void_p()
    ctx.check(_c.lib().qtt_prepare(ctx.h, C.byref(p), delta, C.byref(h)))
    pr = Prepared(ctx, h, keep)
    pr.dim = p.dim
    return pr


def ls_solve_prepared(ctx: Context, prep: Prepared, opts: SolveOptions, keep_eps: bool = False):
    o = opts.c()
    Ceff = np.zeros(36)
    rep = _c.Report()
    eps = C.c_void_p()
    rc = _c.lib().ls_solve_prepared(ctx.h, prep.h, C.byref(o), _dp(Ceff), C.byref(rep),
                                    C.byref(eps) if keep_eps else None)
    ctx.check(rc, allow=(QTT_ENOCONV,))
    C6 = Ceff.reshape(6, 6)
    return (C6[:3, :3].copy() if getattr(prep, "dim", 3) == 2 else C6), _report(rep, o), \
        (Tensor(ctx, eps) if keep_eps else None)


def stats_enable(ctx: Context, on=True):
    """on: False/0 off, True/1 every launch timed, s > 1 every s-th launch."""
    ctx.check(_c.lib().qtt_stats_enable(ctx.h, int(on)))


def stats_reset(ctx: Context):
    ctx.check(_c.lib().qtt_stats_reset(ctx.h))


def stats_get(ctx: Context, family: int) -> dict:
    n = C.c_longlong()
    sec, fl, by = C.c_double(), C.c_double(), C.c_double()
    ctx.check(_c.lib().qtt_stats_get(ctx.h, family, C.byref(n), C.byref(sec), C.byref(fl),
                                     C.byref(by)))
    return {"family": _c.KERNEL_FAMILIES[family], "launches": n.value, "seconds": sec.value,
            "flops": fl.value, "bytes": by.value}


def stats_get_all(ctx: Context, family: int) -> dict:
    """Launch count, flops and bytes over every launch of a family (timed or
    not)."""
    n = C.c_longlong()
    fl, by = C.c_double(), C.c_double()
    ctx.check(_c.lib().qtt_stats_get_all(ctx.h, family, C.byref(n), C.byref(fl), C.byref(by)))
    return {"family": _c.KERNEL_FAMILIES[family], "launches": n.value, "flops": fl.value,
            "bytes": by.value}


_OPS = {"N": 0, "T": 1, "C": 2}


def zgemm(ctx: Context, A, B, Cm, opA: str = "N", opB: str = "N", alpha: complex = 1.0,
          beta: complex = 0.0, path: int = 0):
    """C[b] = alpha op(A[b]) op(B[b]) + beta C[b] on torch complex128 device
    tensors of shape (batch, rows, cols), contiguous.  Extents are checked
    here because the C entry point cannot see caller allocations."""
    import torch
    for t in (A, B, Cm):
        if t.dtype != torch.complex128 or t.dim() != 3 or not t.is_contiguous() or not t.is_cuda:
            raise ValueError("zgemm operands: contiguous complex128 device tensors (batch, r, c)")
    batch = Cm.shape[0]
    if A.shape[0] != batch or B.shape[0] != batch:
        raise ValueError("zgemm: batch mismatch")
    M, N = Cm.shape[1], Cm.shape[2]
    K = A.shape[2] if opA == "N" else A.shape[1]
    if (A.shape[1] if opA == "N" else A.shape[2]) != M:
        raise ValueError("zgemm: A does not match C")
    if (B.shape[1] if opB == "N" else B.shape[2]) != K or (B.shape[2] if opB == "N" else B.shape[1]) != N:
        raise ValueError("zgemm: B does not match")
    al = np.array([complex(alpha).real, complex(alpha).imag])
    be = np.array([complex(beta).real, complex(beta).imag])
    ctx.check(_c.lib().qtt_zgemm(
        ctx.h, _OPS[opA], _OPS[opB], M, N, K, _dp(al), C.c_void_p(A.data_ptr()), A.shape[2],
        C.c_void_p(B.data_ptr()), B.shape[2], _dp(be), C.c_void_p(Cm.data_ptr()), N, batch,
        A.shape[1] * A.shape[2], B.shape[1] * B.shape[2], M * N, path))


def _dev3(t, name):
    import torch
    if t.dtype != torch.complex128 or t.dim() != 3 or not t.is_contiguous() or not t.is_cuda:
        raise ValueError(f"{name}: contiguous complex128 device tensor (batch, rows, cols)")


def zqr(ctx: Context, A, R, Q=None, path: int = 0):
    """Householder QR of a batch of matrices: A (batch, m, n) -> R (batch,
    k, n) and optionally Q (batch, m, k), k = min(m, n)."""
    _dev3(A, "A")
    _dev3(R, "R")
    batch, m, n = A.shape
    k = min(m, n)
    if tuple(R.shape) != (batch, k, n):
        raise ValueError("zqr: R must be (batch, min(m, n), n)")
    qp = None
    if Q is not None:
        _dev3(Q, "Q")
        if tuple(Q.shape) != (batch, m, k):
            raise ValueError("zqr: Q must be (batch, m, min(m, n))")
        qp = C.c_void_p(Q.data_ptr())
    ctx.check(_c.lib().qtt_zqr(ctx.h, batch, m, n, C.c_void_p(A.data_ptr()),
                               C.c_void_p(R.data_ptr()), qp, path))


def zorth(ctx: Context, A, Q, path: int = 0):
    """qtt_zorth: orthonormal basis Q (batch, m, n) of the columns of A
    (batch, m, n); returns the per-matrix fallback flags (1: Householder).
    path 0: spread over the device, 1: one fused workgroup per matrix."""
    _dev3(A, "A")
    _dev3(Q, "Q")
    if tuple(Q.shape) != tuple(A.shape):
        raise ValueError("zorth: Q must have the shape of A")
    batch, m, n = A.shape
    flags = (C.c_int * batch)()
    ctx.check(_c.lib().qtt_zorth(ctx.h, batch, m, n, C.c_void_p(A.data_ptr()),
                                 C.c_void_p(Q.data_ptr()), flags, path))
    return list(flags)


def zqr_noalloc(ctx: Context, A, R, Q=None):
    """qtt_zqr_noalloc: the QR of ``zqr`` (path 0) on the library's fixed
    device workspace; asynchronous on the context's stream, allocates
    nothing."""
    _dev3(A, "A")
    _dev3(R, "R")
    batch, m, n = A.shape
    k = min(m, n)
    if tuple(R.shape) != (batch, k, n):
        raise ValueError("zqr_noalloc: R must be (batch, min(m, n), n)")
    qp = None
    if Q is not None:
        _dev3(Q, "Q")
        if tuple(Q.shape) != (batch, m, k):
            raise ValueError("zqr_noalloc: Q must be (batch, m, min(m, n))")
        qp = C.c_void_p(Q.data_ptr())
    ctx.check(_c.lib().qtt_zqr_noalloc(ctx.h, batch, m, n, C.c_void_p(A.data_ptr()),
                                       C.c_void_p(R.data_ptr()), qp))


def zjacobi(ctx: Context, A, U, S):
    """One-sided Jacobi of square matrices: A (batch, n, n) -> U (batch, n,
    n), S (batch, n) float64 descending, with A V = U diag(S)."""
    import torch
    _dev3(A, "A")
    _dev3(U, "U")
    batch, n, n2 = A.shape
    if n != n2 or tuple(U.shape) != (batch, n, n):
        raise ValueError("zjacobi: square A and U of the same shape")
    if S.dtype != torch.float64 or tuple(S.shape) != (batch, n) or not S.is_contiguous() or not S.is_cuda:
        raise ValueError("zjacobi: S must be a contiguous float64 device tensor (batch, n)")
    ctx.check(_c.lib().qtt_zjacobi(ctx.h, batch, n, C.c_void_p(A.data_ptr()),
                                   C.c_void_p(U.data_ptr()), C.c_void_p(S.data_ptr())))


def ls_adjoint_prepared(ctx: Context, prep: Prepared, opts: SolveOptions, eps: Tensor, gbar=None):
    """ls_adjoint on a prepared problem (operators not rebuilt); eps from
    ls_solve_prepared(..., keep_eps=True) of the same prepared object."""
    o = opts.c()
    nt = 2 * prep._keep[1].shape[0]
    V = 3 if getattr(prep, "dim", 3) == 2 else 6
    rep = _c.Report()
    if gbar is None:
        out = np.zeros(V * V * nt)
        rc = _c.lib().ls_adjoint_prepared(ctx.h, prep.h, C.byref(o), eps.h, None, _dp(out),
                                          C.byref(rep))
        ctx.check(rc, allow=(QTT_ENOCONV,))
        return out.reshape(V, V, nt), _report(rep)
    g = np.ascontiguousarray(gbar, dtype=np.float64).reshape(V * V)
    out = np.zeros(nt)
    rc = _c.lib().ls_adjoint_prepared(ctx.h, prep.h, C.byref(o), eps.h, _dp(g), _dp(out),
                                      C.byref(rep))
    ctx.check(rc, allow=(QTT_ENOCONV,))
    return out, _report(rep)


def _unrolled_out(rc_fn, V, nt, gbar, want_grad):
    Ceff = np.zeros(36)
    rep = _c.Report()
    if not want_grad:
        rc = rc_fn(None, _dp(Ceff), None, C.byref(rep))
        out = None
    elif gbar is None:
        J = np.zeros(V * V * nt)
        rc = rc_fn(None, _dp(Ceff), _dp(J), C.byref(rep))
        out = J.reshape(V, V, nt)
    else:
        g = np.ascontiguousarray(gbar, dtype=np.float64).reshape(V * V)
        out = np.zeros(nt)
        rc = rc_fn(_dp(g), _dp(Ceff), _dp(out), C.byref(rep))
    return rc, Ceff.reshape(6, 6)[:V, :V].copy(), out, rep


def ls_unrolled(ctx: Context, phase, lame, lame0, opts: SolveOptions, steps: int, every: int = 0,
                gbar=None, want_grad: bool = True, scheme="direct"):
    """C_eff after exactly ``steps`` updates and its derivative with respect
    to the phase Lame parameters (reverse mode of the updates, every
    ``every``-th iterate kept, 0 or 1: all); returns (C_eff (V, V), Jacobian
    (V, V, 2*nphase) or gradient (2*nphase,) for a cotangent ``gbar`` or
    None without ``want_grad``, report)."""
    p, keep = _problem(phase, lame, lame0, 0x3F, scheme)
    o = opts.c()
    V = 3 if p.dim == 2 else 6
    nt = 2 * np.asarray(lame).shape[0]
    rc, Cv, out, rep = _unrolled_out(
        lambda g, Ce, gr, r: _c.lib().ls_unrolled(ctx.h, C.byref(p), C.byref(o), int(steps),
                                                  int(every), g, Ce, gr, r), V, nt, gbar, want_grad)
    ctx.check(rc)
    del keep
    return Cv, out, _report(rep)


def ls_unrolled_prepared(ctx: Context, prep: Prepared, opts: SolveOptions, steps: int,
                         every: int = 0, gbar=None, want_grad: bool = True):
    """ls_unrolled on a prepared problem."""
    o = opts.c()
    V = 3 if getattr(prep, "dim", 3) == 2 else 6
    nt = 2 * prep._keep[1].shape[0]
    rc, Cv, out, rep = _unrolled_out(
        lambda g, Ce, gr, r: _c.lib().ls_unrolled_prepared(ctx.h, prep.h, C.byref(o), int(steps),
                                                           int(every), g, Ce, gr, r),
        V, nt, gbar, want_grad)
    ctx.check(rc)
    return Cv, out, _report(rep)


def _not_converged(what: str, rep: SolveReport, policy: str):
    if rep.status == QTT_OK or policy == "ignore":
        return
    msg = (f"{what} fixed point stopped at max_iter (status {rep.status}); "
           f"iterations {rep.iterations}, last relative updates {rep.residual}")
    if policy == "raise":
        raise QttError(rep.status, msg)
    import warnings
    warnings.warn(msg, NotConvergedWarning, stacklevel=3)


def _autograd_function():
    import torch

    class CeffFn(torch.autograd.Function):
        """C_eff as a differentiable function of the phase Lame parameters.

        forward(lame (nphase, 2) float64 tensor, phase, lame0, ctx, opts,
        policy, reports) -> C_eff (6, 6) float64, (3, 3) for a plane-strain
        (square) phase array.  The forward solve keeps
        its strain trains; backward runs the adjoint LS solve
        (ls_adjoint_prepared) with the incoming cotangent and returns
        dL/dlame.  The reference medium lame0 is held fixed (not
        differentiated).  The gradient is that of the converged fixed point
        (energy/adjoint form), so a forward or adjoint solve that stopped
        at max_iter is reported by ``policy``: "raise" (QttError),
        "warn" (NotConvergedWarning) or "ignore".  ``reports`` (a dict) receives
        the forward report under "forward" and the adjoint one under
        "adjoint".  ``unrolled`` = (steps, every) or None: then C_eff is that
        of exactly ``steps`` updates and backward its exact derivative
        (ls_unrolled_prepared)."""

        @staticmethod
        def forward(actx, lame, phase, lame0, qctx, opts, policy, reports, unrolled):
            lam = lame.detach().cpu().numpy().astype(np.float64)
            prep = prepare(qctx, phase, lam, lame0, opts.delta)
            if unrolled is not None:
                Ceff, _, rep = ls_unrolled_prepared(qctx, prep, opts, unrolled[0], unrolled[1],
                                                    want_grad=False)
                eps = None
            else:
                Ceff, rep, eps = ls_solve_prepared(qctx, prep, opts, keep_eps=True)
                _not_converged("forward", rep, policy)
            reports["forward"] = rep
            actx.saved = (qctx, prep, opts, eps, lame.shape, lame.dtype, lame.device, policy,
                          reports, unrolled)
            return torch.as_tensor(Ceff, dtype=torch.float64, device=lame.device)

        @staticmethod
        def backward(actx, gC):
            qctx, prep, opts, eps, shape, dtype, device, policy, reports, unrolled = actx.saved
            g = gC.detach().cpu().numpy().astype(np.float64)
            if unrolled is not None:
                _, grad, arep = ls_unrolled_prepared(qctx, prep, opts, unrolled[0], unrolled[1],
                                                     gbar=g)
            else:
                grad, arep = ls_adjoint_prepared(qctx, prep, opts, eps, gbar=g)
                _not_converged("adjoint", arep, policy)
            reports["adjoint"] = arep
            return (torch.as_tensor(grad.reshape(shape), dtype=dtype, device=device),
                    None, None, None, None, None, None, None)

    return CeffFn


_CeffFn = None


def ceff(lame, phase, lame0, ctx: Context, opts: SolveOptions, on_noconv: str = "raise",
         steps: int | None = None, every: int = 0):
    """Differentiable C_eff: ``ceff(lame_tensor, ...)`` returns a (6, 6)
    torch tensor ((3, 3) for plane strain) whose backward is the adjoint
    solve.  ``on_noconv``:
    "raise", "warn" or "ignore" when the forward or adjoint fixed point
    stops at max_iter.  The returned tensor carries ``qtt_reports``, a dict
    with the forward report ("forward") and, after backward, the adjoint
    report ("adjoint").  With ``steps``, C_eff is that of exactly ``steps``
    updates and backward is its exact derivative (ls_unrolled, every
    ``every``-th iterate kept); ``on_noconv`` does not apply then."""
    global _CeffFn
    if on_noconv not in ("raise", "warn", "ignore"):
        raise ValueError("on_noconv: 'raise', 'warn' or 'ignore'")
    if _CeffFn is None:
        _CeffFn = _autograd_function()
    reports = {"forward": None, "adjoint": None}
    unrolled = None if steps is None else (int(steps), int(every))
    out = _CeffFn.apply(lame, phase, lame0, ctx, opts, on_noconv, reports, unrolled)
    out.qtt_reports = reports
    return out
