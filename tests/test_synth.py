"""CPU checks of the seeded input generators: the workloads have the shapes, distributions and
structure they are described with, and are reproducible from their seeds."""
import numpy as np
import pytest

import synth


def distinct(coords, dims):
    keys = np.zeros(coords.shape[1], dtype=np.int64)
    for t, d in enumerate(dims):
        keys = keys * d + coords[t].astype(np.int64)
    return np.unique(keys).size == keys.size


def test_uniform_coords_distinct_in_range_and_reproducible():
    for dims, nnz in (([40, 30, 20], 5000), ([10 ** 6, 10 ** 6, 10 ** 3], 20000)):
        a = synth.uniform_coords(np.random.default_rng(3), dims, nnz)
        b = synth.uniform_coords(np.random.default_rng(3), dims, nnz)
        assert a.shape == (3, nnz) and a.dtype == np.int32
        np.testing.assert_array_equal(a, b)
        assert distinct(a, dims)
        for t, d in enumerate(dims):
            assert a[t].min() >= 0 and a[t].max() < d
    # the whole space, exactly once
    full = synth.uniform_coords(np.random.default_rng(1), [3, 4, 5], 60)
    assert distinct(full, [3, 4, 5])


def test_zipf_index_is_bounded_and_hot_first():
    rng = np.random.default_rng(0)
    idx = synth.zipf_index(rng, 1000, 1.2, 200000)
    assert idx.min() >= 0 and idx.max() < 1000
    cnt = np.bincount(idx, minlength=1000)
    # P(k) ~ k^-1.2: frequencies fall with the index; ratio of the first two is about 2^1.2
    assert cnt[0] > cnt[1] > cnt[3] > cnt[15] > cnt[255]
    assert abs(cnt[0] / cnt[1] - 2 ** 1.2) < 0.1


def test_skewed_recipe():
    w = synth.skewed(dims=(50000, 10000, 365), nnz=200000, R=10)
    assert w.nnz == 200000 and distinct(w.coords, w.dims)
    assert (w.vals > 0).all()                                  # log-normal values
    c0 = np.bincount(w.coords[0], minlength=w.dims[0])
    c2 = np.bincount(w.coords[2], minlength=w.dims[2])
    assert c0[0] == c0.max() and c0[0] > 50 * np.median(c0[c0 > 0])   # Zipf mode: hot first row
    assert c2.max() < 2 * c2.mean()                            # uniform mode
    assert [u.shape for u in w.U_init] == [(d, 10) for d in w.dims]


def test_order4_and_completion_recipes():
    w = synth.order4(dims=(500, 400, 50, 10), nnz=20000, R=4)
    assert w.order == 4 and distinct(w.coords, w.dims) and (0 <= w.vals).all() and (w.vals < 1).all()
    for u in w.U_init:   # orthonormal initial factors
        np.testing.assert_allclose(u.T @ u, np.eye(4), atol=1e-12)
    c = synth.completion(dims=(300, 200, 50), nnz=30000, R=4, noise=0.0)
    assert c.G_init.shape == (4, 4, 4) and distinct(c.coords, c.dims)


def test_planted_values_match_dense_model():
    rng = np.random.default_rng(5)
    dims, R = [7, 6, 5], (3, 2, 4)
    G = rng.standard_normal(R)
    F = [rng.standard_normal((d, r)) for d, r in zip(dims, R)]
    dense = np.einsum("abc,ia,jb,kc->ijk", G, *F)
    coords = synth.uniform_coords(rng, dims, 100)
    got = synth.planted_values(coords, G, F, batch=17)
    np.testing.assert_allclose(got, dense[coords[0], coords[1], coords[2]], rtol=1e-12, atol=1e-12)


def test_lowrank_recipe_small():
    w = synth.lowrank_f32(dims=(300, 200, 100), nnz=5000, R=4, noise=0.0)
    assert w.dtype == "f32" and distinct(w.coords, w.dims)
    assert np.isfinite(w.vals).all() and np.abs(w.vals).max() > 0


def test_streams_are_independent_of_sizes():
    """The sub-streams come from the seed alone: the initial factors do not depend on nnz."""
    a = synth.small_uniform(9, [50, 40, 30], [3, 3, 3], 100)
    b = synth.small_uniform(9, [50, 40, 30], [3, 3, 3], 900)
    for u, v in zip(a.U_init, b.U_init):
        np.testing.assert_array_equal(u, v)


def test_image_like_shape_and_determinism():
    a, b = synth.image_like(), synth.image_like()
    assert a.dims == [130, 150] and a.ranks == [30, 30] and a.sweeps == 12
    assert np.array_equal(a.coords, b.coords) and np.array_equal(a.vals, b.vals)
    assert 0.45 <= a.nnz / (130 * 150) <= 0.55
    assert a.vals.min() > 0.0 and a.vals.max() <= 1.0
    assert np.unique(a.coords[0] * 150 + a.coords[1]).size == a.nnz
