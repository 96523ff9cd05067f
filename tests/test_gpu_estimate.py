"""The two-order applicability estimate (Sec. 5.2) on the device: the
majority coarsening and both device TT-SVDs give the oracle's ranks
(integers, exact) on the benchmark geometries; host and device voxel
arrays agree; bad inputs are errors."""
import numpy as np
import pytest

from oracle import qtt as Q
import microstructures as M

pytestmark = pytest.mark.gpu

q = pytest.importorskip("paper_2412_11566_amd")
torch = pytest.importorskip("torch")


def _three16():
    ph = M.sphere(16, 0.3).astype(np.uint8)
    ph[M.spheres(16, np.array([[0.2, 0.7, 0.3]]), np.array([0.15])) == 1] = 2
    return ph


CASES = {
    "sphere16": lambda: (M.config_c0().phase, 2),
    "sphere32": lambda: (M.sphere(32, 0.3).astype(np.uint8), 2),
    "fibres64": lambda: (M.config_c2(6).phase, 2),
    "three16": lambda: (_three16(), 3),
    "laminate32": lambda: (M.laminate(32).astype(np.uint8), 2),
    "c3_struct": lambda: (M.config_c3_structure(0, grid_n=5).phase, 2),
}


@pytest.mark.parametrize("case", list(CASES))
def test_rank_estimate_matches_oracle(ctx, case):
    ph, P = CASES[case]()
    # 1e-10: far below every true singular value of a one-hot train and far
    # above the rounding noise, so both TT-SVDs keep the same ranks
    got = q.rank_estimate(ctx, ph, P, 1e-10)
    want = Q.rank_estimate(ph, P, 1e-10)
    assert got[:2] == want[:2]
    assert got[2] == pytest.approx(want[2])


def test_rank_estimate_device_array(ctx):
    ph = M.config_c0().phase
    a = q.rank_estimate(ctx, ph, 2, 1e-8)
    b = q.rank_estimate(ctx, torch.from_numpy(np.ascontiguousarray(ph)).cuda(), 2, 1e-8)
    assert a == b


def test_rank_estimate_rejects(ctx):
    ph = M.config_c0().phase.copy()
    ph[0, 0, 0] = 5
    with pytest.raises(q.QttError) as e:
        q.rank_estimate(ctx, ph, 2, 1e-8)
    assert e.value.code == q._c.QTT_EINVAL
    with pytest.raises(q.QttError) as e:
        q.rank_estimate(ctx, np.zeros((2, 2, 2), np.uint8), 1, 1e-8)
    assert e.value.code == q._c.QTT_EINVAL


def test_rank_estimate_beyond_the_device_path(ctx):
    """64^3 random spheres: the one-hot bonds exceed the device TT-SVD's
    160, so the host decomposes them; the ranks equal the oracle's."""
    p = M.config_c3_structure(1)
    if p.n != 6:
        pytest.skip("structure 1 is not on the 64^3 grid")
    got = q.rank_estimate(ctx, p.phase, 2, 1e-10)
    want = Q.rank_estimate(p.phase, 2, 1e-10)
    assert got[:2] == want[:2]
    assert got[1] > 160


PLANE = ["laminate", "square", "circle", "checkerboard", "spots", "voronoi"]


@pytest.mark.parametrize("name", PLANE)
@pytest.mark.parametrize("n", [5, 7])
def test_plane_rank_estimate_matches_oracle(ctx, name, n):
    """Plane geometries of the paper's suite (2 x 2 majority coarsening,
    2n-bit one-hot trains): the oracle's ranks, exactly."""
    ph = M.geometry(name, 1 << n, 2, seed=1)
    got = q.rank_estimate(ctx, ph, 2, 1e-10)
    want = Q.rank_estimate(ph, 2, 1e-10)
    assert got[:2] == want[:2]
    assert got[2] == pytest.approx(want[2])


def test_plane_rank_estimate_device_array(ctx):
    ph = M.geometry("voronoi", 64, 2, seed=1)
    a = q.rank_estimate(ctx, ph, 2, 1e-8)
    b = q.rank_estimate(ctx, torch.from_numpy(np.ascontiguousarray(ph)).cuda(), 2, 1e-8)
    assert a == b
