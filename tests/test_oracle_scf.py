"""Pins of oracle/scf.py: the worked example of Fig. clustermap, a bijective
migration, structural invariants, and the partial trace on a constructed pencil."""
import os

import numpy as np

from oracle import scf
from paper_1908_06043_amd import inputs

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "clustermap_example.txt")


def read_golden():
    d = {}
    for line in open(GOLD):
        if line.startswith("#") or not line.strip():
            continue
        k, *v = line.split()
        d[k] = [float(t) for t in v]
    return d


def test_clustermap_worked_example():
    g = read_golden()
    out = scf.migrate_probes(g["values"], np.array(g["probe_of"], dtype=int), g["prev_shifts"])
    assert np.array_equal(out["shifts"], np.array(g["new_shifts"]))
    assert 0.5 * (out["shifts"][0] + out["shifts"][1]) == g["new_tau"][0]
    assert out["deleted"] == 1 and out["inserted"] == 1 and out["merged"] == 1
    assert out["members"] == [[0, 1, 2, 3], [4, 5, 6, 7]]
    assert list(out["origin"]) == [-1, 1]   # the probe at sigma_2 keeps the red half


def test_bijective_migration_moves_shifts_to_centroids():
    rng = np.random.default_rng(0)
    a = rng.normal(-3.0, 0.1, 9)
    b = rng.normal(2.0, 0.1, 7)
    x = np.concatenate([a, b])
    probe_of = np.array([0] * 9 + [1] * 7)
    out = scf.migrate_probes(x, probe_of, [-2.5, 2.5])
    assert out["merged"] == out["deleted"] == out["inserted"] == 0
    assert list(out["origin"]) == [0, 1]
    assert out["shifts"][0] == scf._mean(x, list(range(9)))
    assert out["shifts"][1] == scf._mean(x, list(range(9, 16)))


def test_migration_invariants():
    rng = np.random.default_rng(3)
    for trial in range(20):
        n_s = int(rng.integers(2, 7))
        x = np.sort(rng.uniform(-5, 5, int(rng.integers(3 * n_s, 40))))
        prev = np.sort(rng.uniform(-6, 6, n_s))
        probe_of = rng.integers(0, n_s, x.size)
        out = scf.migrate_probes(x, probe_of, prev, use_kmeanspp=bool(trial % 2), seed=trial)
        assert out["shifts"].size == n_s
        assert np.all(np.diff(out["shifts"]) >= 0)
        allm = sorted(i for m in out["members"] for i in m)
        assert allm == list(range(x.size))
        for s, m in zip(out["shifts"], out["members"]):
            assert s == scf._mean(x, m)
        assert out["inserted"] == out["deleted"]


def test_partial_trace_is_sum_of_eigenvalues():
    P = inputs.pencil_scf(80, 8, seed=2)
    X = P.eigvecs()[:, :12]
    assert abs(scf.partial_trace(X, P.A) - np.sum(P.lam[:12])) <= 1e-12 * np.sum(np.abs(P.lam[:12]))
