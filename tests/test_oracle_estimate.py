"""Pins of the two-order applicability estimate in ``oracle.qtt`` (Sec. 5.2:
compress the geometry at two discretisation orders): the majority
coarsening against brute force, and the ranks against facts fixed by the
structure of the quantized train."""
import numpy as np

from oracle import qtt as Q
import microstructures as M


def test_majority_coarsening_brute_force():
    rng = np.random.default_rng(4)
    ph = rng.integers(0, 3, (8, 8, 8)).astype(np.uint8)
    c = Q.coarsen_majority(ph, 3)
    for x in range(4):
        for y in range(4):
            for z in range(4):
                blk = ph[2 * x:2 * x + 2, 2 * y:2 * y + 2, 2 * z:2 * z + 2].ravel()
                cnt = np.bincount(blk, minlength=3)
                assert c[x, y, z] == int(np.flatnonzero(cnt == cnt.max())[0])   # ties: lowest id


def test_upsampled_geometry_keeps_its_rank():
    """A geometry repeated 2 x 2 x 2 per voxel coarsens back to itself, and
    its one-hot train only gains rank-1 cores (the finest bit of each axis
    is irrelevant): the same largest rank at both orders."""
    rng = np.random.default_rng(5)
    base = M.spheres(16, rng.uniform(0, 1, (3, 3)), np.array([0.2, 0.15, 0.1])).astype(np.uint8)
    up = base.repeat(2, 0).repeat(2, 1).repeat(2, 2)
    assert np.array_equal(Q.coarsen_majority(up, 2), base)
    rc, rf, g = Q.rank_estimate(up, 2, 1e-10)
    assert rc == rf and g == 1.0


def test_laminate_rank_does_not_grow():
    for N in (16, 32):
        rc, rf, g = Q.rank_estimate(M.laminate(N).astype(np.uint8), 2, 1e-10)
        assert (rc, rf, g) == (2, 2, 1.0)


def test_random_phases_reach_the_structural_rank():
    """Independent random voxels: every unfolding of the one-hot train is as
    large as it can be.  With two phases chi_0 = 1 - chi_1, so after the
    phase core and k of the 3n bits the rank is min(2^k + 1, 2^(3n - k)):
    17 at order 3 (k = 4), and at most 8 at order 2."""
    rng = np.random.default_rng(6)
    ph = rng.integers(0, 2, (8, 8, 8)).astype(np.uint8)
    rc, rf, _ = Q.rank_estimate(ph, 2, 1e-12)
    assert rf == max(min(2 ** k + 1, 2 ** (9 - k)) for k in range(1, 9))
    assert rc <= max(min(2 ** k + 1, 2 ** (6 - k)) for k in range(1, 6))


def test_majority_coarsening_brute_force_plane():
    rng = np.random.default_rng(14)
    ph = rng.integers(0, 3, (16, 16)).astype(np.uint8)
    c = Q.coarsen_majority(ph, 3)
    assert c.shape == (8, 8)
    for x in range(8):
        for y in range(8):
            cnt = np.bincount(ph[2 * x:2 * x + 2, 2 * y:2 * y + 2].ravel(), minlength=3)
            assert c[x, y] == int(np.flatnonzero(cnt == cnt.max())[0])   # ties: lowest id


def test_plane_estimate_structural_facts():
    """Plane geometries: an upsampled geometry keeps its rank, a laminate
    stays at rank 2, and independent random pixels reach the structural
    rank min(2^k + 1, 2^(2n - k))."""
    rng = np.random.default_rng(15)
    base = (rng.uniform(size=(16, 16)) < 0.3).astype(np.uint8)
    up = base.repeat(2, 0).repeat(2, 1)
    assert np.array_equal(Q.coarsen_majority(up, 2), base)
    rc, rf, g = Q.rank_estimate(up, 2, 1e-10)
    assert rc == rf and g == 1.0
    lam = M.geometry("laminate", 32, 2)
    assert Q.rank_estimate(lam, 2, 1e-10) == (2, 2, 1.0)
    ph = rng.integers(0, 2, (16, 16)).astype(np.uint8)
    rc, rf, _ = Q.rank_estimate(ph, 2, 1e-12)
    assert rf == max(min(2 ** k + 1, 2 ** (8 - k)) for k in range(1, 8))
    assert rc <= max(min(2 ** k + 1, 2 ** (6 - k)) for k in range(1, 6))
