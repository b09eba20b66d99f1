"""Input generators: determinism and the documented distributions."""
import numpy as np

from paper_2009_04755_amd import synth


def test_dense_deterministic_and_normalised():
    a, ca = synth.dense_patterns(32, 500, 8, 0.05, config=0)
    b, cb = synth.dense_patterns(32, 500, 8, 0.05, config=0)
    assert synth.sha256(a, ca) == synth.sha256(b, cb)
    assert synth.sha256(a) != synth.sha256(synth.dense_patterns(32, 500, 8, 0.05, config=0, salt=1)[0])
    x = a.astype(np.float64)
    assert np.abs(x.mean(axis=1)).max() < 1e-8
    np.testing.assert_allclose(np.linalg.norm(x, axis=1), 1.0, atol=1e-6)
    assert list(ca[:10]) == [i % 8 for i in range(10)]


def test_clouds_shape_and_sizes():
    off, xy = synth.point_clouds(200, config=2)
    off2, xy2 = synth.point_clouds(200, config=2)
    assert synth.sha256(off, xy) == synth.sha256(off2, xy2)
    cnt = np.diff(off)
    assert cnt.min() >= 50 and cnt.max() <= 400
    assert xy.dtype == np.float32 and xy.size == 2 * off[-1]
    cen = synth.cloud_centroids(off, xy)
    assert cen.shape == (200, 2)
    # rotation about (0.5,0.5) and shift in [-0.5,0.5]^2 keep centroids within ~[-0.3, 1.3]
    assert np.all(cen > -0.5) and np.all(cen < 1.5)


def test_rigid_starts_ranges():
    p = synth.rigid_starts(10000)
    assert p.shape == (10000, 3)
    assert np.all(p[:, 0] >= -np.pi) and np.all(p[:, 0] < np.pi + 1e-6)
    assert np.all(np.abs(p[:, 1:]) <= 0.5)


def test_sparse_vectors_structure():
    off, keys, vals = synth.sparse_vectors(20, key_space=20 ** 4, nnz_mean=2000, nnz_min=200, nnz_max=10000)
    assert off[0] == 0 and np.all(np.diff(off) >= 200) and np.all(np.diff(off) <= 10000)
    for i in range(20):
        k = keys[off[i]:off[i + 1]]
        v = vals[off[i]:off[i + 1]].astype(np.float64)
        assert np.all(np.diff(k) > 0) and k.min() >= 0 and k.max() < 20 ** 4
        assert abs(v.sum() - 1.0) < 1e-4 and np.all(v > 0)
    o2, k2, v2 = synth.sparse_vectors(20, key_space=20 ** 4, nnz_mean=2000, nnz_min=200, nnz_max=10000)
    assert synth.sha256(off, keys, vals) == synth.sha256(o2, k2, v2)
