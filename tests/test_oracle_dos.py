"""Pins of oracle/dos.py (the paper's Lanczos DOS planner): the closed forms of
the CDOS and of the DOS expectation against quadrature, exact Lanczos on a
diagonal operator, DOSCluster on separated clusters, and the planners' outputs."""
import numpy as np
import pytest
from scipy.integrate import quad

from oracle import dos as odos
from oracle.kpm import Operator
from paper_1908_06043_amd import inputs


def synthetic(seed=0, n=100):
    rng = np.random.default_rng(seed)
    runs = []
    for _ in range(3):
        th = np.sort(rng.uniform(-2, 2, 12))
        z2 = rng.uniform(0.1, 1.0, 12)
        runs.append((th, z2 / z2.sum()))
    return odos.LanczosDOS(runs, n, 12)


def test_cdos_and_expectation_closed_forms_against_quadrature():
    d = synthetic()
    lo, hi = -1.3, 0.7
    num = quad(lambda w: float(d.phi(w)[0]), lo, hi, limit=400, epsabs=1e-12)[0]
    assert abs(num - (d.cdos(hi)[0] - d.cdos(lo)[0])) <= 1e-9
    assert abs(d.cdos(-50.0)[0]) <= 1e-12 and abs(d.cdos(50.0)[0] - d.n) <= 1e-9
    m1 = quad(lambda w: w * float(d.phi(w)[0]), lo, hi, limit=400, epsabs=1e-12)[0]
    assert abs(m1 / num - d.expectation(lo, hi)) <= 1e-8


def test_full_lanczos_on_diagonal_operator_is_exact():
    n = 40
    a = np.sort(np.random.default_rng(1).uniform(-3, 3, n))
    P = inputs.pencil_diag(a)
    op = Operator(P.A, P.B)
    runs = odos.lanczos_runs(op, n, 1, seed=5)
    th, z2 = runs[0]
    assert np.max(np.abs(th - a)) <= 1e-10
    # zeta_j^2 = squared component of the normalised start on eigenvector j
    from oracle import prng
    v = prng.gauss(prng.derive(5, odos.TAG_DOS), 0, n)
    v = v / np.linalg.norm(v)
    assert np.max(np.abs(z2 - v ** 2)) <= 1e-10


def test_dos_cluster_separates_clusters():
    rng = np.random.default_rng(2)
    centres = [-2.0, 0.0, 2.5]
    a = np.sort(np.concatenate([rng.normal(c, 0.02, 20) for c in centres]))
    P = inputs.pencil_diag(a)
    op = Operator(P.A, P.B)
    # a short Lanczos run resolves each cluster as a few Ritz values; the coarse
    # grid n_omega = 10 k of the paper's first pass
    k = 12
    runs = odos.lanczos_runs(op, k, 2, seed=3)
    d = odos.LanczosDOS(runs, 60, k)
    ritz = np.concatenate([th for th, _ in runs])
    I = odos.dos_cluster(d, -3.0, 3.5, 10 * k, ritz)
    assert len(I) == 3
    for (l, u), c in zip(I, centres):
        inside = a[(a > l) & (a <= u)]
        assert inside.size == 20 and np.all(np.abs(inside - c) < 0.2)


def test_planners_return_n_s_ordered_shifts():
    P = inputs.pencil_clusters4(200, 0)
    for mode in ("cdos", "cluster"):
        out = odos.plan(P.A, P.B, 40, 4, k=60, nv=4, seed=0, mode=mode)
        s, top = out["sigmas"], out["omega_top"]
        assert s.size == 4 and np.all(np.diff(s) > 0) and s[-1] < top
        assert abs(out["dos"].cdos(top)[0] - (40 + 2 * 40 / 4)) <= 1e-6
    d = out["dos"]
    sig, top = odos.plan_cdos(d, 40, 4)
    a, _ = odos.window(d, 40, 4)
    # midpoints of equal-count intervals: Phi at the interval ends is equally spaced
    pa, pt = d.cdos(a)[0], d.cdos(top)[0]
    K = (pt - pa) / 4
    ends = [a] + [d.root(pa + j * K, a, top) for j in (1, 2, 3)] + [top]
    assert np.allclose(sig, [0.5 * (ends[j] + ends[j + 1]) for j in range(4)], rtol=0, atol=1e-12)


def test_small_interval_merges_into_smaller_neighbour():
    d = synthetic(seed=4)
    I = [(-2.5, -1.0), (-1.0, -0.999), (-0.999, 2.5)]
    out = odos._merge_small(d, I)
    assert len(out) == 2
    g0, g2 = odos._gamma(d, I[0]), odos._gamma(d, I[2])
    if g0 <= g2:
        assert out[0] == (-2.5, -0.999)
    else:
        assert out[1] == (-1.0, 2.5)
