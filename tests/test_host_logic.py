"""Host-side logic without a GPU: the synthetic division rule of the
variable-population workload and the autotuner's cache handling."""
import json

import numpy as np

from paper_2105_00039_amd import workloads


def test_grow_and_divide_conserves_volume_and_places_daughters():
    pop = workloads.uniform(5000, mean_neighbors=12.0, seed=5)
    x, y, z, d = pop.arrays()
    rng = np.random.default_rng(6)
    growth, d_max = 1.05, 12.0
    x2, y2, z2, d2 = workloads.grow_and_divide(x, y, z, d, rng, growth=growth, d_max=d_max)
    grown = d * growth
    div = np.nonzero(grown > d_max)[0]
    n, k = len(x), len(div)
    assert len(x2) == n + k and k > 0
    # total volume: the growth, then each division halves a mother's volume twice over
    np.testing.assert_allclose(np.sum(d2 ** 3), np.sum(grown ** 3), rtol=1e-12)
    # agents that did not divide are only grown
    keep = np.setdiff1d(np.arange(n), div)
    assert np.array_equal(d2[keep], grown[keep]) and np.array_equal(x2[keep], x[keep])
    # daughter pairs: mother index i and appended index n + j, half a grown
    # diameter apart, centred on the mother, each with half the volume
    for j, i in enumerate(div):
        p1 = np.array([x2[i], y2[i], z2[i]])
        p2 = np.array([x2[n + j], y2[n + j], z2[n + j]])
        np.testing.assert_allclose(np.linalg.norm(p1 - p2), grown[i] / 2, rtol=1e-12)
        np.testing.assert_allclose((p1 + p2) / 2, [x[i], y[i], z[i]], atol=1e-9)
        np.testing.assert_allclose(d2[i] ** 3, grown[i] ** 3 / 2, rtol=1e-12)
        assert d2[n + j] == d2[i]
    # seeded: the same draws give the same population
    again = workloads.grow_and_divide(x, y, z, d, np.random.default_rng(6), growth=growth, d_max=d_max)
    for a, b in zip(again, (x2, y2, z2, d2)):
        assert np.array_equal(a, b)


def test_grow_and_divide_without_division_only_grows():
    x, y, z = np.zeros(3), np.zeros(3), np.arange(3.0) * 20
    d = np.array([8.0, 9.0, 10.0])
    x2, y2, z2, d2 = workloads.grow_and_divide(x, y, z, d, np.random.default_rng(0))
    assert len(x2) == 3 and np.array_equal(d2, d * 1.02) and np.array_equal(z2, z)


def test_autotune_cache_loading(tmp_path):
    # importing the tuner needs only the package (no GPU call happens here)
    from paper_2105_00039_amd import autotune
    table, path = autotune._load(None)
    assert table == {} and path is None
    d = {"k": 40}
    table, path = autotune._load(d)
    assert table is d and path is None
    p = tmp_path / "cache.json"
    table, path = autotune._load(p)
    assert table == {} and path == str(p)
    p.write_text(json.dumps({"f32|n2^21|occ2^1.5|sims1": 32}))
    table, path = autotune._load(str(p))
    assert table == {"f32|n2^21|occ2^1.5|sims1": 32}
    # the library default comes first (kept on ties): 24-entry lists, 64
    # threads, each lane walking its runs in turn; every triple appears once
    assert autotune.CHOICES[0] == (24, 64, "lanes")
    assert len(set(autotune.CHOICES)) == len(autotune.CHOICES) == 8
    assert {c[1] for c in autotune.CHOICES} == {64, 256}
    # entries of older caches (list length only, or list and block) read with
    # the default block size and walk
    assert autotune._as_choice(40) == (40, 64, "lanes")
    assert autotune._as_choice([32, 128]) == (32, 128, "lanes")
    assert autotune._as_choice([40, 128, "planes"]) == (40, 128, "planes")
