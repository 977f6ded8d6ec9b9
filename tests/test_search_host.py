"""The re-grouping step of the hierarchical search (Sec 3.2: k-means on the
particle positions between rungs), host code of the library, against
scikit-learn's k-means on data whose clusters are unambiguous."""
import numpy as np
import pytest

from paper_2408_13170_amd import B

sklearn = pytest.importorskip("sklearn.cluster")
metrics = pytest.importorskip("sklearn.metrics")


def _blobs(seed=0, k=5, per=600, dim=7):
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.0, 1.0, (k, dim))
    # well separated: minimum centre distance >> spread
    while np.min([np.linalg.norm(a - b) for i, a in enumerate(centres) for b in centres[i + 1:]]) < 0.3:
        centres = rng.uniform(0.0, 1.0, (k, dim))
    x = np.concatenate([c + 0.01 * rng.standard_normal((per, dim)) for c in centres])
    return x, np.repeat(np.arange(k), per), centres


def test_kmeans_recovers_separated_clusters_like_sklearn():
    x, truth, centres = _blobs()
    labels, ctr = B.scs_kmeans(x, 5, iters=100, seed=7)
    assert ctr.shape == (5, 7)
    assert metrics.adjusted_rand_score(truth, labels) == 1.0
    ref = sklearn.KMeans(n_clusters=5, n_init=10, random_state=0).fit(x)
    assert metrics.adjusted_rand_score(ref.labels_, labels) == 1.0
    # centres: the cluster means
    for c in range(5):
        assert np.allclose(ctr[c], x[labels == c].mean(axis=0), atol=1e-12)
    # labels numbered by first appearance
    first = [labels[np.argmax(labels == c)] for c in range(5)]
    assert sorted(np.unique(labels)) == list(range(5))
    assert list(dict.fromkeys(labels)) == list(range(5)) and first == list(range(5))


def test_kmeans_deterministic_and_drops_empty_clusters():
    x, _, _ = _blobs(seed=3)
    a, _ = B.scs_kmeans(x, 5, seed=11)
    b, _ = B.scs_kmeans(x, 5, seed=11)
    assert np.array_equal(a, b)
    # three distinct points repeated: at most three clusters survive
    pts = np.repeat(np.array([[0.0] * 7, [1.0] * 7, [0.0] * 6 + [5.0]]), 4, axis=0)
    lab, ctr = B.scs_kmeans(pts, 6, seed=1)
    assert len(ctr) == 3
    for c in range(3):
        assert np.all(pts[lab == c] == pts[lab == c][0])


def test_kmeans_argument_errors():
    with pytest.raises(B.ScsError):
        B.scs_kmeans(np.zeros((4, 2)), 0)
    with pytest.raises(B.ScsError):
        B.scs_kmeans(np.zeros((4, 2)), 2, iters=0)


@pytest.mark.parametrize("seed,n,k,dim", [(0, 500, 6, 9), (1, 2000, 6, 9), (2, 37, 5, 3), (3, 8, 8, 2)])
def test_kmeans_matches_oracle(seed, n, k, dim):
    """The library's k-means against the oracle's, on overlapping clusters
    where the seeding and the Lloyd iterations decide the result: the same
    labels, centres to rounding."""
    from oracle import search as S

    rng = np.random.default_rng(seed)
    x = np.concatenate([rng.normal(rng.uniform(0, 1, dim), 0.2, (n // 3 + 1, dim)) for _ in range(3)])[:n]
    lab, ctr = B.scs_kmeans(x, k, iters=100, seed=seed + 40)
    olab, octr = S.kmeans(x, k, 100, seed=seed + 40)
    assert np.array_equal(lab, olab)
    assert ctr.shape == octr.shape and np.allclose(ctr, octr, rtol=0, atol=1e-13)
