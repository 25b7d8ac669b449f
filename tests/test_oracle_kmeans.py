"""Pins of k-means shift migration (Section 3.2) and of the shared PRNG."""
import os

import numpy as np
import pytest

from oracle import kmeans, prng

HERE = os.path.dirname(__file__)


def test_splitmix64_reference_outputs():
    vals = [int(l, 16) for l in open(os.path.join(HERE, "golden", "splitmix64_seed0.txt"))
            if l.strip() and not l.startswith("#")]
    assert [prng.splitmix64(0, i) for i in range(len(vals))] == vals
    arr = prng.splitmix64_array(0, 0, len(vals))
    assert [int(v) for v in arr] == vals


def test_prng_derived_draws():
    u = prng.uniform(123, 0, 200000)
    assert u.min() >= 0.0 and u.max() < 1.0 and abs(u.mean() - 0.5) < 0.005
    r = prng.rademacher(123, 0, 200000)
    assert set(np.unique(r)) == {-1.0, 1.0} and abs(r.mean()) < 0.01
    g = prng.gauss(9, 0, 200000)
    assert abs(g.mean()) < 0.01 and abs(g.std() - 1.0) < 0.01
    # the same index gives the same draw regardless of the block it is taken in
    assert np.array_equal(prng.uniform(5, 10, 5), prng.uniform(5, 0, 15)[10:])


def test_lloyd_fixed_point():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(c, 0.05, 30) for c in (-2, -1, 0.5, 3)])
    c, lab = kmeans.lloyd(x, [-2.5, -0.5, 0.0, 2.0])
    # every point sits at its nearest centroid and every centroid is its members' mean
    assert np.array_equal(lab, kmeans.assign(x, c))
    for j in range(4):
        assert c[j] == pytest.approx(np.mean(x[lab == j]), rel=1e-15, abs=1e-15)
    assert np.allclose(np.sort(c), [-2, -1, 0.5, 3], atol=0.05)


def test_lloyd_vs_brute_force_optimum():
    rng = np.random.default_rng(1)
    for trial in range(20):
        x = np.sort(rng.uniform(0, 1, 11))
        k = 3
        best = kmeans.brute_force_1d(x, k)
        c, _ = kmeans.lloyd(x, kmeans.kmeanspp_init(x, k, seed=trial))
        assert kmeans.objective(x, c) >= best - 1e-12
    # well separated clusters: Lloyd from the previous shifts reaches the optimum
    x = np.array([0.0, 0.1, 0.2, 5.0, 5.1, 9.0, 9.3, 9.6])
    c, _ = kmeans.lloyd(x, [1.0, 4.0, 8.0])
    assert abs(kmeans.objective(x, c) - kmeans.brute_force_1d(x, 3)) < 1e-12


def test_ties_go_to_lower_centroid_and_empty_cluster_keeps_centroid():
    lab = kmeans.assign(np.array([1.0]), np.array([0.0, 2.0]))
    assert lab[0] == 0
    c, lab = kmeans.lloyd(np.array([0.0, 0.1]), [0.05, 10.0])
    assert c[1] == 10.0 and np.all(lab == 0)


def _worked_cases():
    cases, cur = [], {}
    for line in open(os.path.join(HERE, "golden", "kmeanspp_worked.txt")):
        if not line.strip() or line.startswith("#"):
            continue
        key, *vals = line.split()
        cur[key] = [float(v) for v in vals]
        if key == "centres":
            cases.append(cur)
            cur = {}
    return cases


def test_kmeanspp_hand_worked_cases():
    cases = _worked_cases()
    assert len(cases) == 4
    for c in cases:
        got = kmeans.kmeanspp_from_draws(c["points"], len(c["draws"]), c["draws"])
        assert list(got) == c["centres"]


def test_kmeanspp_seeded_draws_are_the_splitmix64_substream():
    rng = np.random.default_rng(5)
    x = rng.uniform(-3, 3, 40)
    for seed in (0, 7, 123456789):
        s = prng.derive(seed, prng.TAG_KMEANSPP)
        u = [prng.uniform(s, c, 1)[0] for c in range(6)]
        assert np.array_equal(kmeans.kmeanspp_init(x, 6, seed), kmeans.kmeanspp_from_draws(x, 6, u))


def test_kmeanspp_d2_law():
    # second centre over a fine uniform grid of draws: the share of draws that
    # pick point i is D^2_i / sum D^2 up to the grid step
    x = np.array([0.0, 1.0, 3.0, 7.0, 8.0])
    d2 = (x - 3.0) ** 2
    M = 5400
    hits = np.zeros(x.size)
    for t in range(M):
        c = kmeans.kmeanspp_from_draws(x, 2, [0.5, (t + 0.5) / M])
        hits[int(np.flatnonzero(x == c[1])[0])] += 1
    assert np.all(np.abs(hits / M - d2 / d2.sum()) <= 1.0 / M)
    # the seeded stream follows the same law: second centre given the first
    counts = np.zeros(x.size)
    for seed in range(12000):
        c = kmeans.kmeanspp_init(x, 2, seed)
        if c[0] == 3.0:
            counts[int(np.flatnonzero(x == c[1])[0])] += 1
    m = counts.sum()
    p = d2 / d2.sum()
    assert m > 1800 and counts[2] == 0
    assert np.all(np.abs(counts / m - p) <= 4.0 * np.sqrt(p * (1 - p) / m) + 1e-12)


def test_kmeanspp_reproducible_and_distinct():
    rng = np.random.default_rng(3)
    x = rng.uniform(-5, 5, 300)
    a = kmeans.kmeanspp_init(x, 16, seed=42)
    b = kmeans.kmeanspp_init(x, 16, seed=42)
    assert np.array_equal(a, b) and len(set(a)) == 16
    new, _ = kmeans.migrate(x, np.linspace(-5, 5, 16), use_kmeanspp=True, seed=42)
    assert np.all(np.diff(new) > 0)
