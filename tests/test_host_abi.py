"""CPU checks of the C ABI: the library loads and exports every declared entry point,
and the host-only planner functions agree with the oracle."""
import os
import re

import numpy as np
import pytest

from oracle import kmeans, kpm, prng, validate as oval
from paper_1908_06043_amd import _lib, api

HERE = os.path.dirname(os.path.abspath(__file__))
HEADER = os.path.join(os.path.dirname(HERE), "include", "sislice.h")


def declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(sislice_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    names = declared()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(_lib.EXPORTED)


def test_status_strings_and_defaults():
    lib = _lib.load()
    for code in (0, -1, -2, -3, -4, 1, 2, 3):
        assert lib.sislice_status_string(code)
    o = api.default_opts()
    assert (o.block, o.max_basis, o.kpm_moments, o.kpm_vectors, o.tol) == (8, 112, 64, 20, 1e-10)


def test_splitmix64_matches_oracle():
    for seed in (0, 1, 12345, 2**63 + 7):
        for i in (0, 1, 2, 1000):
            assert api.splitmix64(seed, i) == prng.splitmix64(seed, i)


def test_kpm_cdos_and_placement_match_oracle():
    rng = np.random.default_rng(0)
    mu = np.concatenate([[1.0], rng.normal(0, 0.05, 63) / (1 + np.arange(63))])
    a, b, n = -5.2, 5.3, 4096
    g = kpm.jackson(64)
    for w in np.linspace(a, b, 17):
        assert api.kpm_cdos(mu, a, b, n, w) == pytest.approx(kpm.cdos(w, mu, g, a, b, n), abs=1e-9)
    sig, top = api.kpm_place(mu, a, b, n, 400, 16, 2.0)
    osig, _, otop = kpm.place_shifts(mu, a, b, n, 400, 16, 2.0)
    assert np.allclose(sig, osig, rtol=0, atol=1e-10) and top == pytest.approx(otop, abs=1e-10)


def test_kmeans_matches_oracle_bit_for_bit():
    rng = np.random.default_rng(1)
    x = np.sort(np.concatenate([rng.normal(c, 0.07, 40) for c in (-3, -1.2, 0.4, 2.5)]))
    prev = np.array([-3.5, -1.0, 0.0, 3.0])
    c, lab = api.kmeans_shifts(x, prev)
    oc, olab = kmeans.migrate(x, prev)
    assert np.array_equal(c, oc) and np.array_equal(lab, olab)
    c, lab = api.kmeans_shifts(x, n_s=6, use_kmeanspp=True, seed=7)
    oc, olab = kmeans.migrate(x, np.zeros(6), use_kmeanspp=True, seed=7)
    assert np.array_equal(c, oc)


def test_validation_matches_oracle():
    rng = np.random.default_rng(2)
    lam = np.sort(rng.uniform(-3, 3, 60))
    sig = np.array([-2.0, -0.7, 0.5, 1.9])
    top = 2.6
    nus = [int(np.sum(lam < s)) for s in sig]
    nut = int(np.sum(lam < top))
    th, rs = [], []
    for j, s in enumerate(sig):
        lo = sig[j - 1] if j else -np.inf
        hi = sig[j + 1] if j + 1 < len(sig) else top
        t = lam[(lam > lo) & (lam < hi)].copy()
        if j == 1:
            t = np.concatenate([t[:-2], [t[0] + 1e-3]])          # a missing value and a spurious one
        r = rng.uniform(0, 1e-12, t.size)
        th.append(t)
        rs.append(r)
    out = api.validate(sig, nus, th, rs, top, nut)
    ref = oval.validate(sig, nus, th, rs, top, nut)
    assert list(out["slice_case"]) == [s["case"] for s in ref["slices"]]
    assert list(out["slice_exact"]) == [s["n_exact"] for s in ref["slices"]]
    assert list(out["slice_cand"]) == [s["n_cand"] for s in ref["slices"]]
    flat = np.concatenate(th)
    got = np.sort(flat[out["chosen"] == 1])
    assert np.array_equal(got, np.array([v[0] for v in ref["validated"]]))


def test_gpu_entry_points_refuse_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    with pytest.raises(RuntimeError):
        api.handle()


def test_scf_migrate_matches_oracle():
    from oracle import scf as oscf
    import os
    gold = {}
    path = os.path.join(HERE, "golden", "clustermap_example.txt")
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        k, *v = line.split()
        gold[k] = [float(t) for t in v]
    out = api.scf_migrate(gold["values"], [int(v) for v in gold["probe_of"]], gold["prev_shifts"])
    assert list(out["shifts"]) == gold["new_shifts"]
    assert (out["merged"], out["deleted"], out["inserted"]) == (1, 1, 1)
    rng = np.random.default_rng(11)
    for trial in range(40):
        n_s = int(rng.integers(2, 9))
        x = rng.uniform(-5, 5, int(rng.integers(3 * n_s, 60)))
        prev = np.sort(rng.uniform(-6, 6, n_s))
        po = rng.integers(0, n_s, x.size).astype(np.int32)
        ref = oscf.migrate_probes(x, po, prev, use_kmeanspp=bool(trial % 3 == 0), seed=trial)
        got = api.scf_migrate(x, po, prev, use_kmeanspp=bool(trial % 3 == 0), seed=trial)
        assert np.array_equal(got["shifts"], ref["shifts"])         # bit-exact
        assert list(got["origin"]) == list(ref["origin"])
        for r, members in enumerate(ref["members"]):
            assert all(got["value_probe"][i] == r for i in members)
        assert (got["merged"], got["deleted"], got["inserted"]) == (
            ref["merged"], ref["deleted"], ref["inserted"])


@pytest.mark.parametrize("mode", [0, 1])
def test_dos_plan_matches_oracle(mode):
    from oracle import dos as odos
    from oracle.kpm import Operator
    from paper_1908_06043_amd import inputs
    for P, n_e, n_s, k in ((inputs.pencil_clusters4(200, 0), 40, 4, 40),
                           (inputs.pencil_scf(600, 60, seed=3), 60, 6, 60)):
        runs = odos.lanczos_runs(Operator(P.A, P.B), k, 4, seed=1)
        d = odos.LanczosDOS(runs, P.n, k)
        if mode == 0:
            ref, top = odos.plan_cdos(d, n_e, n_s)
        else:
            ritz = np.concatenate([th for th, _ in runs])
            ref, top, _ = odos.plan_cluster(d, ritz, n_e, n_s, k)
        th = np.stack([t for t, _ in runs])
        z2 = np.stack([z for _, z in runs])
        sig, top2 = api.dos_plan(th, z2, P.n, n_e, n_s, mode=mode)
        scale = np.max(np.abs(th))
        assert abs(top2 - top) <= 1e-12 * scale
        assert np.max(np.abs(sig - ref)) <= 1e-12 * scale
