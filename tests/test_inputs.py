"""The seeded workload generators: determinism, sizes and the stated geometry."""
import numpy as np

from paper_0810_0233_amd import inputs


def test_unit_moments_are_unit_and_seeded():
    a = inputs.random_moments(1000, 5)
    b = inputs.random_moments(1000, 5)
    np.testing.assert_array_equal(a, b)
    np.testing.assert_allclose(np.linalg.norm(a, axis=1), 1.0, rtol=1e-15)
    assert abs(a.mean(axis=0)).max() < 0.1


def test_ferrofluid_hard_core_and_fraction():
    from scipy.spatial import cKDTree

    pos, box = inputs.ferrofluid(3000, 9)
    side = inputs.ferrofluid_side(3000)
    assert pos.shape == (3000, 3)
    assert np.all(pos >= 0) and np.all(pos < side)
    d, _ = cKDTree(pos).query(pos, k=2)
    assert d[:, 1].min() >= 1.0
    pos2, _ = inputs.ferrofluid(3000, 9, batch=777)  # candidate order does not depend on batching
    np.testing.assert_array_equal(pos, pos2)
    assert abs(3000 * np.pi / 6 / side ** 3 - 0.1) < 1e-12


def test_sphere_cut_counts():
    pos, box = inputs.sphere_cut(1000, 16)
    assert pos.shape == (1000, 3)
    c = np.full(3, 7.5)
    r = np.linalg.norm(pos - c, axis=1)
    # every omitted site is at least as far as every kept one
    allpos, _ = inputs.lattice(16, 16, 16)
    rall = np.sort(np.linalg.norm(allpos - c, axis=1))
    assert r.max() <= rall[1000] + 1e-12


def test_aligned_moments_fraction():
    m = inputs.aligned_moments(2000, 5, 3000)
    assert m.shape == (5, 2000, 3)
    zfrac = [(np.all(m[b] == [0, 0, 1.0], axis=1)).mean() for b in range(5)]
    assert zfrac[0] == 0.0
    assert abs(zfrac[-1] - 0.5) < 1e-9


def test_clusters_inside_box():
    pos, box = inputs.clusters(4, 500, 1)
    assert pos.shape == (2000, 3)
    assert np.all(pos >= 0) and np.all(pos < 512)


def test_film_holes():
    pos, box = inputs.film_with_holes(128, 128, 4, 3, 7, rmin=5, rmax=10)
    assert pos.shape[0] % 4 == 0
    assert pos.shape[0] < 128 * 128 * 4
    assert set(np.unique(pos[:, 2])) == {0.0, 1.0, 2.0, 3.0}
