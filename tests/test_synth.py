"""Seeded input generators: shapes, value distributions, reproducibility."""
import numpy as np

import synth


def test_image_like_shape_and_distribution():
    X = synth.image_like(3000, 1)
    assert X.shape == (3000, 784) and X.dtype == np.float32
    assert abs((X == 0).mean() - 0.80) <= 0.02
    assert X.min() == 0 and X.max() <= 255 and np.array_equal(X, np.rint(X))
    # squared norms below 2^23 keep every pair distance exact in FP32
    assert (X.astype(np.float64) ** 2).sum(1).max() < 2 ** 23
    assert np.array_equal(X, synth.image_like(3000, 1))


def test_lowd_blobs():
    X, lab = synth.lowd_blobs(20000, 2, return_labels=True)
    assert X.shape == (20000, 3)
    assert abs((lab == -1).mean() - 0.1) < 1e-3
    assert X.min() > -0.2 and X.max() < 1.2


def test_gaussian_and_integer():
    X = synth.gaussian_mixture(500, 8, 10, 0)
    assert X.shape == (500, 8) and X.dtype == np.float32
    Y = synth.integer_points(100, 5, 7, 1)
    assert Y.min() >= 0 and Y.max() <= 7 and np.array_equal(Y, np.rint(Y))


def test_anisotropic_clusters_small():
    X = synth.anisotropic_clusters(2000, 96, 3, 10)
    assert X.shape == (2000, 96) and np.isfinite(X).all()


def test_batched_sizes():
    b = synth.batched_datasets(64, 4)
    Ns = [x.shape[0] for x, _ in b]
    ds = {x.shape[1] for x, _ in b}
    assert min(Ns) >= 500 and max(Ns) <= 20000 and ds <= {16, 64, 128}


def test_paper_gaussian_datasets():
    """Sec. 4: single variant ~ N(0, 2I); non-single variant: mean e_i/d per
    coordinate (uniform over the d basis centres), covariance 2I + the
    spread of the centres."""
    X = synth.single_gaussian(200000, 4, 1).astype(np.float64)
    assert np.allclose(X.mean(0), 0.0, atol=0.02)
    assert np.allclose(np.cov(X.T), 2.0 * np.eye(4), atol=0.03)
    d = 8
    Y = synth.synthetic_gaussian(400000, d, 2).astype(np.float64)
    assert np.allclose(Y.mean(0), 1.0 / d, atol=0.02)
    centre_cov = np.eye(d) / d - np.full((d, d), 1.0 / d**2)
    assert np.allclose(np.cov(Y.T), 2.0 * np.eye(d) + centre_cov, atol=0.03)


def test_audio_like_shape():
    """Audio-shaped stand-in: 54387 x 192 FP32, seeded, per-feature spread
    falling along the vector, consecutive frames of a sentence close."""
    X = synth.audio_like(54387, 192, 7)
    assert X.shape == (54387, 192) and X.dtype == np.float32
    assert np.array_equal(X[:100], synth.audio_like(54387, 192, 7)[:100])
    sd = X.std(0)
    assert sd[:16].mean() > 2 * sd[-16:].mean()
    step = np.linalg.norm(X[1:2000] - X[:1999], axis=1)
    rand = np.linalg.norm(X[1:2000] - X[np.random.default_rng(0).permutation(1999)], axis=1)
    assert np.median(step) < 0.6 * np.median(rand)
