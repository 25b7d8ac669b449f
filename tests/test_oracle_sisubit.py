"""Pins of CholeskyQR, Algorithm 2, Rayleigh-Ritz and residuals (Section 2.1)."""
import numpy as np
import scipy.linalg as sla

from oracle import bk, sisubit
from paper_1908_06043_amd import inputs


def test_cholesky_qr_b_orthonormal_same_span():
    P = inputs.pencil_clusters4(120, 1)
    rng = np.random.default_rng(0)
    V = rng.standard_normal((120, 9))
    Q = sisubit.cholesky_qr(V, P.B)
    assert np.max(np.abs(Q.T @ P.B @ Q - np.eye(9))) < 1e-13
    # same span: V = Q (Q^T B V)
    assert np.linalg.norm(V - Q @ (Q.T @ P.B @ V)) < 1e-12 * np.linalg.norm(V)


def test_rayleigh_ritz_full_space_is_dense_eigensolve():
    P = inputs.pencil_clusters4(60, 2)
    V = sisubit.cholesky_qr(np.eye(60), P.B)
    om, X = sisubit.rayleigh_ritz(P.A, P.B, V)
    ref = sla.eigh(P.A, P.B, eigvals_only=True)
    assert np.max(np.abs(om - ref)) < 1e-13 * np.max(np.abs(ref))
    assert np.max(np.abs(om - P.lam)) < 1e-13 * np.max(np.abs(P.lam))
    assert np.max(np.abs(X.T @ P.B @ X - np.eye(60))) < 1e-12


def test_residual_of_exact_eigenpairs_is_rounding():
    P = inputs.pencil_clusters4(100, 3)
    X = P.eigvecs()
    anorm = sisubit.norm2_sym(P.A)
    r = sisubit.residual_norms(P.A, P.B, X, P.lam, anorm)
    assert r.max() < 1e-14
    r_bad = sisubit.residual_norms(P.A, P.B, X, P.lam + 1e-6, anorm)
    assert r_bad.min() > 1e-8                       # a wrong value is visible


def test_norm2_matches_svd():
    P = inputs.pencil_clusters4(80, 4)
    assert abs(sisubit.norm2_sym(P.A) - np.linalg.norm(P.A, 2)) < 1e-12 * np.linalg.norm(P.A, 2)


def test_algorithm2_converges_to_nearest_eigenpairs():
    P = inputs.pencil_clusters4(200, 0)
    sigma = inputs.safe_shifts(P.lam, [-0.45])[0]
    k = 24
    rng = np.random.default_rng(7)
    V = rng.standard_normal((200, k))
    anorm = sisubit.norm2_sym(P.A)
    fac = bk.bk_ldlt(bk.shifted(P.A, P.B, sigma))
    for _ in range(25):
        lam, X, _ = sisubit.sisubit(P.A, P.B, V, sigma, 4, fac=fac)
        V = X
    res = sisubit.residual_norms(P.A, P.B, X, lam, anorm)
    # the 8 eigenvalues closest to sigma are converged and equal the construction's
    near = np.argsort(np.abs(P.lam - sigma))[:8]
    got = np.sort(lam[np.argsort(np.abs(lam - sigma))[:8]])
    assert np.max(np.abs(got - np.sort(P.lam[near]))) < 1e-12
    assert np.max(res[np.argsort(np.abs(lam - sigma))[:8]]) < 1e-12
    assert np.max(np.abs(X.T @ P.B @ X - np.eye(k))) < 1e-12


def test_norm2_power_iteration_branch():
    # above order 1500 the norm comes from power iteration: a symmetric matrix with
    # a known spectrum (largest |lambda| = 3, next 2.5) in a random orthogonal basis
    n = 1600
    lam = np.linspace(-2.5, 2.5, n)
    lam[n // 3] = 3.0
    Q, _ = np.linalg.qr(np.random.default_rng(11).standard_normal((n, n)))
    A = (Q * lam) @ Q.T
    A = 0.5 * (A + A.T)
    assert abs(sisubit.norm2_sym(A) - 3.0) < 1e-12
    # a largest eigenvalue of negative sign is found by its modulus
    assert abs(sisubit.norm2_sym(-A) - 3.0) < 1e-12
