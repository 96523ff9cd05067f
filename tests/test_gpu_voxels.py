"""Row a0 on the device: qtt_from_voxels builds the one-hot phase train by a
TT-SVD on the GPU (tall-skinny QR tree, Jacobi SVD of the R factor,
right-to-left) and the raised stiffness operator C(x) - C0 from it
(Sec. 4.3 binary discretisation; App. D: recomputed per geometry).

Checked against the per-voxel definition (C of the voxel's phase minus C0)
on every voxel at 16^3 and 64^3, against the oracle's TT-SVD ranks, on
sampled voxels at 256^3, and for device and host voxel arrays alike."""
import numpy as np
import pytest

from oracle import qtt as Q
from oracle.voigt import iso_voigt
import microstructures as M

pytestmark = pytest.mark.gpu

q = pytest.importorskip("paper_2412_11566_amd")
torch = pytest.importorskip("torch")


def _diag_train(op_cores):
    """Diagonal of a raised operator as a train: core 0 (1, 36, r), spatial
    cores (r, 2, r') from the full (r, dout, din, r') cores."""
    c0 = op_cores[0]
    out = [c0.reshape(1, 36, c0.shape[3])]
    for c in op_cores[1:]:
        out.append(np.stack([c[:, i, i, :] for i in range(c.shape[1])], axis=1))
    return out


def _exact(phase, lame, lame0):
    C0 = iso_voigt(*lame0)
    dC = np.stack([iso_voigt(*lp) - C0 for lp in lame])   # (P, 6, 6)
    return dC[phase.ravel()]                                # (N^3, 6, 6)


def _three_phase(n, seed=3):
    rng = np.random.default_rng(seed)
    N = 1 << n
    base = M.sphere(N, 0.3)
    extra = M.spheres(N, np.array([[0.2, 0.7, 0.3]]), np.array([0.15]))
    ph = base.astype(np.uint8)
    ph[extra == 1] = 2
    return ph, np.array([[0.6, 0.4], [5.0, 3.0], [12.0, 9.0]]), (6.3, 4.7)


CASES = {
    "sphere16": lambda: (M.config_c0().phase, M.config_c0().lame, M.config_c0().lame0),
    "sphere64": lambda: (M.config_c1_sphere().phase, M.config_c1_sphere().lame, M.config_c1_sphere().lame0),
    "fibres64": lambda: (M.config_c2(6).phase, M.config_c2(6).lame, M.config_c2(6).lame0),
    "three16": lambda: _three_phase(4),
}


@pytest.mark.parametrize("case", list(CASES))
def test_from_voxels_every_voxel(ctx, case):
    """At rounding accuracy 1e-14 (numerical rank only) the operator equals
    the per-voxel definition to rounding; at 1e-10 it has the oracle's
    TT-SVD ranks; at 1e-8 the one-hot train meets the TT-SVD bound
    ||chi~ - chi||_F <= delta ||chi||_F (Sec. 3, eq. rounding_condition_tt)
    with ranks no larger."""
    phase, lame, lame0 = CASES[case]()
    A, chi = q.from_voxels(ctx, phase, lame, lame0, 1e-14)
    d = Q.tt_full(_diag_train(A.cores()))                   # (36, 2, ..., 2)
    got = d.reshape(6, 6, -1).transpose(2, 0, 1)
    ref = _exact(phase, lame, lame0)
    P = len(lame)
    onehot = np.stack([(phase.ravel() == p) for p in range(P)]).astype(float)
    ch = Q.tt_full([c[0] for c in chi.cores()]).reshape(P, -1)
    # rounding level of a TT-SVD over 3n bonds: 1e-12 of ||chi||_F =
    # sqrt(N^3), on the train and (times the largest |C_p - C0| entry) on
    # the operator
    nrm = np.sqrt(phase.size)
    assert np.linalg.norm(ch - onehot) < 1e-12 * nrm
    assert np.abs(got - ref).max() < 1e-12 * nrm * np.abs(ref).max()
    # ranks at 1e-10, where the threshold (1e-10 / sqrt(L - 1) ||chi||)
    # lies far below every true singular value and far above rounding noise
    # (at 1e-14 it sits at the noise level, where either TT-SVD may keep a
    # noise value): the oracle's left-to-right TT-SVD has the same ranks
    A10, _ = q.from_voxels(ctx, phase, lame, lame0, 1e-10)
    ocores = Q.stiffness_tto(phase, lame, lame0, 1e-10)
    assert A10.ranks == [1] + [c.shape[-1] for c in ocores]
    A8, chi8 = q.from_voxels(ctx, phase, lame, lame0, 1e-8)
    ch8 = Q.tt_full([c[0] for c in chi8.cores()]).reshape(P, -1)
    nrm = np.sqrt(phase.size)
    assert np.linalg.norm(ch8 - onehot) <= 1e-8 * nrm * (1 + 1e-6)
    assert all(a <= b for a, b in zip(A8.ranks, A10.ranks))


def test_from_voxels_device_array_and_host_array_agree(ctx):
    p = M.config_c0()
    Ah, _ = q.from_voxels(ctx, p.phase, p.lame, p.lame0, 1e-10)
    dph = torch.from_numpy(np.ascontiguousarray(p.phase)).cuda()
    Ad, _ = q.from_voxels(ctx, dph, p.lame, p.lame0, 1e-10)
    assert Ad.ranks == Ah.ranks
    for a, b in zip(Ad.cores(), Ah.cores()):
        assert np.abs(a - b).max() == 0.0


def test_from_voxels_256_sampled(ctx):
    """The four-fibre workload at 256^3 (accuracy 1e-12): 2000 seeded
    voxels evaluated from the operator train against the definition."""
    import time
    p = M.config_c2()
    t = time.perf_counter()
    A, _ = q.from_voxels(ctx, p.phase, p.lame, p.lame0, 1e-12)
    dt = time.perf_counter() - t
    cores = _diag_train(A.cores())
    rng = np.random.default_rng(5)
    idx = rng.integers(0, p.phase.size, 2000)
    n3 = 3 * p.n
    ref = _exact(p.phase, p.lame, p.lame0)[idx]
    for e, v in enumerate(idx):
        bits = [(int(v) >> (n3 - 1 - k)) & 1 for k in range(n3)]
        vec = cores[0][0]                                   # (36, r)
        for k, b in enumerate(bits):
            vec = vec @ cores[k + 1][:, b, :]
        got = vec[:, 0].reshape(6, 6)
        assert np.abs(got - ref[e]).max() < 1e-10 * np.abs(ref).max()
    assert dt < 30.0, dt


def test_from_voxels_rank_cap(ctx):
    p = M.config_c0()
    with pytest.raises(q.QttError) as e:
        q.from_voxels(ctx, p.phase, p.lame, p.lame0, 1e-10, cap=1)
    assert e.value.code == q._c.QTT_ECAPACITY
    bad = p.phase.copy()
    bad[0, 0, 0] = 7
    with pytest.raises(q.QttError) as e:
        q.from_voxels(ctx, bad, p.lame, p.lame0, 1e-10)
    assert e.value.code == q._c.QTT_EINVAL


def _diag_train_plane(op_cores):
    c0 = op_cores[0]
    out = [c0.reshape(1, 9, c0.shape[3])]
    for c in op_cores[1:]:
        out.append(np.stack([c[:, i, i, :] for i in range(c.shape[1])], axis=1))
    return out


@pytest.mark.parametrize("name,N,P", [("circle", 32, 2), ("voronoi", 64, 2), ("spots", 64, 2), ("three", 32, 3)])
def test_from_voxels_plane_every_pixel(ctx, name, N, P):
    """Plane-strain geometries (2n binary cores, a 3 x 3 control core): the
    operator equals the per-pixel plane-strain stiffness minus C0's on every
    pixel to rounding at accuracy 1e-14, and the one-hot train meets the
    TT-SVD bound at 1e-8 (Sec. 3, eq. rounding_condition_tt)."""
    from oracle import plane as P2
    if name == "three":
        ph = M.geometry("circle", N, 2, seed=1).astype(np.uint8)
        ph[M.geometry("square", N, 2, seed=1) == 1] = 2
    else:
        ph = M.geometry(name, N, 2, seed=1)
    lame = np.array([[0.6, 0.4], [5.0, 3.0], [12.0, 9.0]])[:P]
    l0 = (6.3, 4.7)
    A, chi = q.from_voxels(ctx, ph, lame, l0, 1e-14)
    got = Q.tt_full(_diag_train_plane(A.cores())).reshape(3, 3, -1).transpose(2, 0, 1)
    dC = np.stack([P2.iso_voigt2(*lp) - P2.iso_voigt2(*l0) for lp in lame])
    ref = dC[ph.ravel()]
    # rounding level of a TT-SVD over 2n bonds, as for the 3D operator
    nrm = np.sqrt(ph.size)
    assert np.abs(got - ref).max() < 1e-12 * nrm * np.abs(ref).max()
    onehot = np.stack([(ph.ravel() == p) for p in range(P)]).astype(float)
    _, chi8 = q.from_voxels(ctx, ph, lame, l0, 1e-8)
    c = Q.tt_full([x[0] for x in chi8.cores()]).reshape(P, -1)
    assert np.linalg.norm(c - onehot) <= 1e-8 * nrm * (1 + 1e-6)
