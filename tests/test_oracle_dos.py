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


class PiecewiseLinearDOS:
    """A DOS given by hand: phi piecewise linear through the knots (xs, ys), Phi its
    exact integral from xs[0], so that gamma and the grid values are known by hand."""

    def __init__(self, xs, ys):
        self.xs = np.asarray(xs, dtype=np.float64)
        self.ys = np.asarray(ys, dtype=np.float64)
        seg = np.diff(self.xs) * (self.ys[1:] + self.ys[:-1]) / 2.0
        self.cum = np.concatenate([[0.0], np.cumsum(seg)])
        self.a, self.b = float(self.xs[0]), float(self.xs[-1])

    def phi(self, w):
        return np.interp(np.atleast_1d(np.asarray(w, dtype=np.float64)), self.xs, self.ys)

    def cdos(self, w):
        w = np.atleast_1d(np.asarray(w, dtype=np.float64))
        i = np.clip(np.searchsorted(self.xs, w, side="right") - 1, 0, self.xs.size - 2)
        return self.cum[i] + (w - self.xs[i]) * (self.ys[i] + self.phi(w)) / 2.0

    def root(self, target, lo, hi):
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if float(self.cdos(mid)[0]) < target:
                lo = mid
            else:
                hi = mid
        return 0.5 * (lo + hi)


def two_peak_dos():
    # [0, 8]: tent background 1 + min(w, 8 - w) / 8 plus triangles of height 27.1
    # at 3 (support [2, 4]) and at 5 (support [4, 6]): gamma(0, 8) = 10 + 2 * 27.1
    # = 64.2.  [8, 16]: tent 1 + min(w - 8, 16 - w) / 8 plus a triangle of height
    # 62.65 at 12 (support [10, 14]): gamma(8, 16) = 10 + 2 * 62.65 = 135.3.
    xs = [0, 2, 3, 4, 5, 6, 8, 10, 12, 14, 16]
    ys = [1, 1.25, 1.375 + 27.1, 1.5, 1.375 + 27.1, 1.25, 1, 1.25, 1.5 + 62.65, 1.25, 1]
    return PiecewiseLinearDOS(xs, ys)


def test_refinement_splits_the_wide_interval_on_the_doubled_grid():
    d = two_peak_dos()
    assert odos._gamma(d, (0, 8)) == pytest.approx(64.2, abs=1e-12)
    assert odos._gamma(d, (8, 16)) == pytest.approx(135.3, abs=1e-12)
    assert odos.count(d, (0, 8)) == 65 and odos.count(d, (0, 16)) == 200
    ritz = np.array([3.0, 5.0, 12.0])
    # Worked by hand.  Round 1: (0, 8) has gamma 64.2 > 50 and is searched again
    # with n' = 2 * 65 / 200 * 100 = 65 points (step 1/8); the grid maxima are
    # w = 3 and w = 5 and the least phi between them is phi(4) = 1.5, so (0, 8)
    # becomes (0, 4), (4, 8).  (8, 16) (gamma 135.3) is searched with
    # n' = 2 * 136 / 200 * 100 = 136 points and shows one maximum: it stays.
    # Round 2: gamma(0, 4) = gamma(4, 8) = 32.1 <= 50, (8, 16) stays: done.
    # (With gamma in place of C = ceil(gamma) the grid would have
    # round(2 * 64.2 / 199.5 * 100) = 64 points and no point at w = 4.)
    out = odos.refine(d, [(0.0, 8.0), (8.0, 16.0)], 0.0, 16.0, 100, ritz)
    assert out == [(0.0, 4.0), (4.0, 8.0), (8.0, 16.0)]
    # at most 50 estimated eigenvalues: not searched again
    out = odos.refine(d, [(0.0, 8.0), (8.0, 16.0)], 0.0, 16.0, 100, ritz, big=70.0)
    assert out == [(0.0, 8.0), (8.0, 16.0)]
    # a sub-interval without a Ritz value is dropped by DOSCluster's last step,
    # so a single remaining interval does not replace the searched one
    out = odos.refine(d, [(0.0, 8.0), (8.0, 16.0)], 0.0, 16.0, 100, np.array([3.0, 12.0]))
    assert out == [(0.0, 8.0), (8.0, 16.0)]


def test_safeguards_split_and_merge_worked_by_hand():
    # uniform DOS phi = 10 on [0, 10]: gamma(l, u) = 10 (u - l) and the CDOS
    # midpoint of (l, u) is (l + u) / 2
    d = PiecewiseLinearDOS([0, 10], [10, 10])
    I = odos.safeguards(d, [(0, 1), (1, 4), (4, 5)], 5)
    # gammas 10 30 10: split (1, 4) at 2.5; then 10 15 15 10: the tie goes to the
    # lower interval, (1, 2.5) splits at 1.75
    exp = [(0, 1), (1, 1.75), (1.75, 2.5), (2.5, 4), (4, 5)]
    assert len(I) == 5 and np.allclose(np.array(I, dtype=float), exp, rtol=0, atol=1e-12)
    # too many: gammas 10 30 10 20, the emptiest is (0, 1) (tie: lower); its only
    # neighbour (1, 4) is adjacent -> (0, 4).  Then 40 10 20: (4, 5) has list
    # neighbours (0, 4) (adjacent) and (6, 8) (not adjacent, though emptier):
    # it merges into (0, 4).
    assert odos.safeguards(d, [(0, 1), (1, 4), (4, 5), (6, 8)], 2) == [(0, 5), (6, 8)]
    # both neighbours adjacent: the one with fewer estimated eigenvalues
    assert odos.safeguards(d, [(0, 2), (2, 3), (3, 6)], 2) == [(0, 3), (3, 6)]
    # no adjacent neighbour: the list neighbour takes it
    assert odos.safeguards(d, [(0, 1), (2, 3), (5, 9)], 2) == [(0, 3), (5, 9)]
    # already n_s intervals: unchanged
    assert odos.safeguards(d, [(0, 1), (1, 4)], 2) == [(0, 1), (1, 4)]
