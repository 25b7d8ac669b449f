"""Pins of the oracle's Bunch-Kaufman LDL^T and Sylvester inertia (Sections 2.1, 2.2).

Every check is against something other than the oracle itself: the exact inertia of
pencils built with known eigenvalues, brute-force eigenvalue counts, LAPACK's own
?sytrf (through scipy), backward error, and special cases with closed forms.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import bk
from paper_1908_06043_amd import inputs

U = np.finfo(np.float64).eps / 2


def lapack_inertia(C):
    _, d, _ = sla.ldl(C, lower=True)           # LAPACK ?sytrf underneath
    w = np.linalg.eigvalsh(d)
    return int(np.sum(w < 0)), int(np.sum(w == 0)), int(np.sum(w > 0))


@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (7, 2), (64, 3), (157, 4)])
def test_inertia_matches_eigenvalue_count_random(n, seed):
    C = inputs.random_symmetric(n, seed)
    f = bk.bk_ldlt(C)
    w = np.linalg.eigvalsh(C)
    assert bk.inertia(f) == (int(np.sum(w < 0)), 0, int(np.sum(w > 0)))
    assert bk.inertia(f) == lapack_inertia(C)


@pytest.mark.parametrize("n,seed", [(16, 0), (97, 1), (200, 2)])
def test_backward_error(n, seed):
    C = inputs.random_symmetric(n, seed)
    f = bk.bk_ldlt(C)
    assert bk.backward_error(C, f) <= 50 * n * U
    L = f["L"]
    assert np.allclose(np.diag(L), 1.0) and np.all(np.triu(L, 1) == 0)


def test_inertia_known_spectrum_pencil():
    P = inputs.pencil_clusters4(200, 0)
    sig = inputs.safe_shifts(P.lam, np.linspace(-2.1, 2.1, 23))
    for s in sig:
        f = bk.bk_ldlt(bk.shifted(P.A, P.B, s))
        neg, zero, pos = bk.inertia(f)
        assert neg == int(np.sum(P.lam < s))
        assert zero == 0 and neg + pos == 200


def test_inertia_scf_pencil_small():
    P = inputs.pencil_scf(300, 30, seed=3)
    sig = inputs.safe_shifts(P.lam, [-5.5, -4.9, -4.5, -3.0, 0.0, 4.99, 6.0])
    for s in sig:
        f = bk.bk_ldlt(bk.shifted(P.A, P.B, s))
        assert bk.inertia(f)[0] == int(np.sum(P.lam < s))


def test_special_cases_spd_and_above_spectrum():
    P = inputs.pencil_clusters4(120, 5)
    f = bk.bk_ldlt(bk.shifted(P.A, P.B, P.lam[0] - 1.0))        # SPD: no negative pivot
    assert bk.inertia(f) == (0, 0, 120)
    f = bk.bk_ldlt(bk.shifted(P.A, P.B, P.lam[-1] + 1.0))       # negative definite
    assert bk.inertia(f) == (120, 0, 0)


def test_diagonal_pencil_is_exact():
    a = np.array([3.0, -1.0, 0.5, -2.5, 7.0, 0.25])
    sigma = 0.5
    C = np.diag(a) - sigma * np.eye(6)
    f = bk.bk_ldlt(C)
    # no off-diagonal entries: every step is a 1x1 pivot without interchange
    assert np.array_equal(f["perm"], np.arange(6))
    assert np.all(f["blk"] == 1)
    assert np.array_equal(f["d"], a - sigma)                     # bit-exact
    assert np.array_equal(f["L"], np.eye(6))
    assert bk.inertia(f) == (3, 1, 2)                            # a_2 - sigma == 0 exactly
    assert f["zero_pivots"] == 1


def test_two_by_two_blocks_have_negative_determinant():
    # with alpha = (1+sqrt 17)/8 a 2x2 pivot is taken only when |c11 c22| < alpha^2 c21^2
    total = 0
    for seed in range(6):
        C = inputs.random_symmetric(80, seed)
        f = bk.bk_ldlt(C)
        for k in np.nonzero(f["blk"] == 2)[0]:
            a, c, b = f["d"][k], f["d"][k + 1], f["e"][k]
            assert a * c - b * b < 0
            assert abs(a * c) < bk.ALPHA ** 2 * b * b * (1 + 1e-12)
            total += 1
    assert total > 20


def test_pivot_rule_forces_2x2_on_zero_diagonal():
    # [[0, 1], [1, 0]]: |a11| = 0 < alpha * 1 and |a22| = 0 < alpha * 1 -> one 2x2 block
    f = bk.bk_ldlt(np.array([[0.0, 1.0], [1.0, 0.0]]))
    assert list(f["blk"]) == [2, 0]
    assert bk.inertia(f) == (1, 0, 1)
    # [[1e-3, 1], [1, 5]]: |a22| = 5 >= alpha * 1 -> 1x1 pivot on a22 after interchange
    f = bk.bk_ldlt(np.array([[1e-3, 1.0], [1.0, 5.0]]))
    assert list(f["perm"]) == [1, 0] and list(f["blk"]) == [1, 1]
    assert f["d"][0] == 5.0


@pytest.mark.parametrize("n,seed", [(50, 0), (133, 1)])
def test_ldlt_solve_residual(n, seed):
    C = inputs.random_symmetric(n, seed)
    f = bk.bk_ldlt(C)
    rng = np.random.default_rng(seed)
    Ub = rng.standard_normal((n, 5))
    X = bk.ldlt_solve(f, Ub)
    r = np.linalg.norm(C @ X - Ub) / (np.linalg.norm(C) * np.linalg.norm(X))
    assert r < 1e3 * n * U
    x1 = bk.ldlt_solve(f, Ub[:, 0])
    assert np.allclose(x1, X[:, 0], rtol=0, atol=1e-12 * np.abs(X).max())
