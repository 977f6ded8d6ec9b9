"""The re-grouping's k-means on the device (scs_kmeans_device, the routine the
search runs between rungs, Sec 3.2) against the host k-means (scs_kmeans,
itself pinned to the k-means oracle and to scikit-learn in
test_search_host.py): the same labels and kept clusters, centres within
rounding, on random and clustered data at the search's size (6 x 10^4
particles, 9 features: seven dimensions, two of them periodic), on small and
degenerate inputs, and the same result on every call."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2408_13170_amd import B  # noqa: E402


def _both(x, k, iters=100, seed=0):
    dev = torch.device("cuda:0")
    xd = torch.tensor(x, dtype=torch.float64, device=dev)
    ld, cd = B.scs_kmeans_device(xd, k, iters=iters, seed=seed)
    torch.cuda.synchronize()
    lh, ch = B.scs_kmeans(x, k, iters=iters, seed=seed)
    return ld.cpu().numpy(), cd.cpu().numpy(), lh, ch


def _check(x, k, iters=100, seed=0):
    ld, cd, lh, ch = _both(x, k, iters, seed)
    print(f"n={len(x)} k={k}: device {cd.shape[0]} clusters, host {ch.shape[0]}; "
          f"labels differ at {int(np.sum(ld != lh))} points")
    assert np.array_equal(ld, lh)
    assert cd.shape == ch.shape
    scale = max(1.0, float(np.abs(ch).max()))
    assert np.abs(cd - ch).max() <= 1e-12 * scale
    return ld


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_device_kmeans_matches_host_search_size(seed):
    """Positions of a search-sized swarm set in the features the re-grouping
    uses (scaled to the box, periodic ones on the circle)."""
    rng = np.random.default_rng(seed)
    n = 60000
    u = rng.uniform(0.0, 1.0, (n, 7))
    # a few concentrations, as swarms that converged on different peaks leave them
    for c in range(4):
        idx = rng.choice(n, 6000, replace=False)
        u[idx] = np.clip(rng.uniform(0.1, 0.9, 7) + 0.02 * rng.standard_normal((6000, 7)), 0.0, 1.0)
    a = 2.0 * np.pi * u[:, 5:7]
    x = np.concatenate([u[:, :5], np.cos(a[:, :1]) / (2 * np.pi), np.sin(a[:, :1]) / (2 * np.pi),
                        np.cos(a[:, 1:]) / (2 * np.pi), np.sin(a[:, 1:]) / (2 * np.pi)], axis=1)
    _check(np.ascontiguousarray(x), 6, iters=100, seed=seed + 17)


def test_device_kmeans_separated_blobs_and_small_inputs():
    rng = np.random.default_rng(5)
    centres = np.eye(5, 9) * 3.0
    x = np.concatenate([c + 0.01 * rng.standard_normal((1500, 9)) for c in centres])
    lab = _check(x, 5, seed=3)
    assert sorted(np.bincount(lab)) == [1500] * 5
    # fewer points than clusters (k clamps to n), one point, odd sizes
    _check(rng.uniform(size=(4, 3)), 6, seed=1)
    _check(rng.uniform(size=(1, 2)), 3, seed=2)
    _check(rng.uniform(size=(1031, 16)), 7, seed=4)
    # repeated points: zero total weight in the seeding, clusters dropped
    pts = np.repeat(np.array([[0.0] * 7, [1.0] * 7, [0.0] * 6 + [5.0]]), 400, axis=0)
    lab = _check(pts, 6, seed=1)
    assert lab.max() == 2
    same = np.zeros((100, 4))
    assert _check(same, 3, seed=9).max() == 0


def test_device_kmeans_repeatable_and_errors():
    rng = np.random.default_rng(8)
    xd = torch.tensor(rng.uniform(size=(20000, 9)), device="cuda:0")
    a, ca = B.scs_kmeans_device(xd, 6, seed=5)
    b, cb = B.scs_kmeans_device(xd, 6, seed=5)
    assert torch.equal(a, b) and torch.equal(ca, cb)
    with pytest.raises(B.ScsError):
        B.scs_kmeans_device(xd, 0)
    with pytest.raises(B.ScsError):
        B.scs_kmeans_device(torch.zeros((10, 17), dtype=torch.float64, device="cuda:0"), 2)
    with pytest.raises(B.ScsError):
        B.scs_kmeans_device(xd, 2, iters=0)
