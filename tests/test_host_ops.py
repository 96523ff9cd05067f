"""Host-side operator construction (no GPU): the library's SFFT, Green and
stiffness builders checked against the oracle's plain definitions."""
import ctypes as C
import os

import numpy as np
import pytest

from oracle import qtt as Q, dense as D
from oracle.voigt import iso_voigt
import microstructures as M

_capi = pytest.importorskip("paper_2412_11566_amd._capi")

if not os.path.exists(_capi.HOSTLIB_PATH):
    pytest.skip("libqtthom_host.so not built (run __graft_entry__.build())", allow_module_level=True)

hl = _capi.hostlib()
P = lambda a: a.ctypes.data_as(C.POINTER(C.c_int))
DP = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))


def dump(fn, L=64, cap=1 << 22):
    ranks = np.zeros(L + 1, np.int32)
    dout = np.zeros(L, np.int32)
    din = np.zeros(L, np.int32)
    buf = np.zeros(2 * cap)
    nc = fn(P(ranks), P(dout), P(din), DP(buf), cap)
    assert nc > 0, nc
    z = buf.view(np.complex128)
    cores, off = [], 0
    for k in range(nc):
        shp = (ranks[k], dout[k], din[k], ranks[k + 1])
        cnt = int(np.prod(shp))
        cores.append(z[off:off + cnt].reshape(shp).copy())
        off += cnt
    return cores


def per_voxel(cores, N):
    t = cores[0][0]
    for c in cores[1:]:
        t = np.tensordot(t, np.einsum("aiib->aib", c), axes=([t.ndim - 1], [0]))
    return t.reshape(cores[0].shape[1], cores[0].shape[2], N, N, N)


@pytest.mark.parametrize("n,delta,tol", [(3, 1e-14, 1e-13), (5, 1e-14, 1e-13), (8, 1e-10, 1e-9)])
def test_qn_tto_matches_reduced_qft(n, delta, tol):
    ranks = np.zeros(n + 1, np.int32)
    buf = np.zeros(2 * (1 << 20))
    nc = hl.qtt_host_qn_tto(n, delta, P(ranks), DP(buf), 1 << 20)
    assert nc == n
    z = buf.view(np.complex128)
    cores, off = [], 0
    for k in range(n):
        shp = (ranks[k], 2, 2, ranks[k + 1])
        cnt = int(np.prod(shp))
        cores.append(z[off:off + cnt].reshape(shp))
        off += cnt
    assert np.abs(Q.tto_full(cores) - Q.qn_matrix(n)).max() < tol
    if n == 8:
        assert max(ranks) == 10   # Sec. 5.2: SFFT rank 10 for n >= 8


@pytest.mark.parametrize("n", [2, 3, 4])
def test_green_bounded_chain_matches_table(n):
    N = 1 << n
    lam0, mu0 = 2.3, 1.4
    consts = np.zeros(2)
    ops = [per_voxel(dump(lambda *a, w=w: hl.qtt_host_green(n, lam0, mu0, 1e-14, w, *a, DP(consts))), N)
           for w in range(4)]
    rng = np.random.default_rng(0)
    tau = rng.standard_normal((6, N, N, N)) + 1j * rng.standard_normal((6, N, N, N))
    ap = lambda O, x: np.einsum("oixyz,ixyz->oxyz", O, x)
    u = ap(ops[0], tau)
    s = ap(ops[1], u)
    p = ap(ops[2], s)
    e = ap(ops[3], consts[0] * u - consts[1] * p)
    ref = np.einsum("vwxyz,wxyz->vxyz", Q.green_tensor(n, lam0, mu0), tau)
    assert np.linalg.norm(e - ref) < 1e-12 * np.linalg.norm(ref)


def test_stiffness_operator():
    n, N = 3, 8
    ph = M.sphere(N, 0.3)
    lame = np.array([[1.0, 0.5], [3.0, 2.0]])
    l0 = np.array([2.0, 1.25])
    ops = dump(lambda *a: hl.qtt_host_stiffness(ph.ctypes.data_as(C.POINTER(C.c_uint8)), n, 2,
                                                DP(lame), DP(l0), 1e-14, *a))
    t = per_voxel(ops, N)
    ref = np.stack([iso_voigt(*lame[q]) - iso_voigt(*l0) for q in range(2)])[ph]
    assert np.abs(t.transpose(2, 3, 4, 0, 1) - ref).max() < 1e-13
