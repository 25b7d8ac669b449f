"""Reverse-mode derivative of the lowest n_e eigenpairs of the pencil (A, B).

TEST INFRASTRUCTURE ONLY (see the package header).

The paper computes the lowest eigenpairs of the symmetric-definite pencil of
its problem statement (Section 1, eq. seq_gep); it does not differentiate them.
The gradient is textbook first-order perturbation theory of that problem.  For
A x_i = lam_i B x_i with x_i^T B x_i = 1 and simple eigenvalues:

  d lam_i = x_i^T (dA - lam_i dB) x_i
  d x_i   = sum_{j != i} x_j x_j^T (dA - lam_i dB) x_i / (lam_i - lam_j)
            - 1/2 x_i (x_i^T dB x_i)

For a loss with cotangents g_lam (n_e) and g_X (n x n_e), dL = sum_i g_lam_i
d lam_i + sum_i g_X_i^T d x_i.  Gradients are returned in the symmetric
convention: G_A and G_B are symmetric and dL = tr(G_A dA) + tr(G_B dB) for
symmetric dA, dB.

Two independent forms:

* ``grad_sum_over_states`` -- the definition above written out over the full
  eigendecomposition (dense ``eigh`` of the pencil, every j);
* ``grad_projected`` -- the form that needs only the lowest n_e pairs: the sum
  over the unoccupied j is the vector z_i that solves
  (A - lam_i B) z_i = -(I - B X X^T) g_X_i with X^T B z_i = 0 (a bordered dense
  solve here), and the occupied-occupied terms are an n_e x n_e matrix.

``loss_density`` is the training-style loss sum_i f(lam_i) + tr(W X X^T) with
f(lam) = lam^2, evaluated by a dense eigensolve (for finite differences).
Pins: tests/test_oracle_adjoint.py (central differences of ``loss_density``,
the Hellmann-Feynman special case, the two forms against each other).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def _sym(M):
    return 0.5 * (M + M.T)


def lowest_pairs(A, B, n_e):
    """The lowest n_e eigenpairs of (A, B), B-orthonormal (dense LAPACK solve)."""
    lam, X = sla.eigh(A, B, subset_by_index=[0, n_e - 1])
    return lam, X


def loss_density(A, B, n_e, W):
    """L = sum_i lam_i^2 + tr(W P), P = X X^T over the lowest n_e pairs."""
    lam, X = lowest_pairs(A, B, n_e)
    return float(np.sum(lam ** 2) + np.sum((W @ X) * X))


def density_cotangents(lam, X, W):
    """Cotangents of ``loss_density``: g_lam = 2 lam, g_X = (W + W^T) X."""
    return 2.0 * lam, (W + W.T) @ X


def grad_sum_over_states(A, B, n_e, g_lam, g_X, X=None):
    """(G_A, G_B) from the full eigendecomposition (the perturbation formulas).

    g_X refers to particular eigenvectors: each is fixed only up to its sign, so
    the occupied columns of the full decomposition take the signs of ``X`` (the
    vectors the cotangent was computed for; default: ``lowest_pairs``)."""
    if X is None:
        X = lowest_pairs(A, B, n_e)[1]
    lam_all, X_all = sla.eigh(A, B)
    sg = np.sign(np.sum(X_all[:, :n_e] * (B @ X), axis=0))
    X_all[:, :n_e] *= sg[None, :]
    lo = lam_all[:n_e]
    Xo = X_all[:, :n_e]
    g_lam = np.asarray(g_lam, dtype=np.float64)
    K = X_all.T @ g_X                       # K[j, i] = x_j^T g_X_i
    D = lo[None, :] - lam_all[:, None]      # D[j, i] = lam_i - lam_j
    own = np.zeros_like(D, dtype=bool)
    own[np.arange(n_e), np.arange(n_e)] = True
    F = np.where(own, 0.0, 1.0 / np.where(own, 1.0, D))
    C = K * F                               # coefficient of x_j in d x_i per unit (dA - lam_i dB)
    kii = np.diag(K[:n_e, :])
    GA = (Xo * g_lam[None, :]) @ Xo.T + _sym(X_all @ C @ Xo.T)
    GB = (-(Xo * (g_lam * lo)[None, :]) @ Xo.T
          - _sym(X_all @ (C * lo[None, :]) @ Xo.T)
          - 0.5 * (Xo * kii[None, :]) @ Xo.T)
    return _sym(GA), _sym(GB)


def projected_rhs(B, X, g_X):
    """-(I - B X X^T) g_X: the unoccupied part of the eigenvector cotangents."""
    return -(g_X - (B @ X) @ (X.T @ g_X))


def solve_projected(A, B, X, lam_i, r):
    """z with (A - lam_i B) z = r and X^T B z = 0, by the bordered system
    [[A - lam_i B, B X], [X^T B, 0]] [z; mu] = [r; 0]."""
    n, m = X.shape
    BX = B @ X
    K = np.zeros((n + m, n + m))
    K[:n, :n] = A - lam_i * B
    K[:n, n:] = BX
    K[n:, :n] = BX.T
    rhs = np.concatenate([r, np.zeros(m)])
    return np.linalg.solve(K, rhs)[:n]


def occupied_blocks(lam, g_lam, K):
    """The n_e x n_e middle matrices of the occupied-occupied part.

    With K = X^T g_X, S = (K + K^T)/2, T = (K - K^T)/2 and F_ji = 1/(lam_i - lam_j)
    (0 on the diagonal):
      M_A = diag(g_lam) + T o F
      M_B = -diag(lam g_lam) - S/2 - (lam_i + lam_j) (T o F) / 2
    so that G_A gets X M_A X^T and G_B gets X M_B X^T."""
    m = lam.size
    S = 0.5 * (K + K.T)
    T = 0.5 * (K - K.T)
    D = lam[None, :] - lam[:, None]        # D[j, i] = lam_i - lam_j
    eye = np.eye(m, dtype=bool)
    F = np.where(eye, 0.0, 1.0 / np.where(eye, 1.0, D))
    TF = T * F
    MA = np.diag(g_lam) + TF
    MB = -np.diag(lam * g_lam) - 0.5 * S - 0.5 * (lam[None, :] + lam[:, None]) * TF
    return MA, MB


def grad_projected(A, B, n_e, g_lam, g_X, lam=None, X=None):
    """(G_A, G_B) from the lowest n_e pairs and n_e projected solves:
      G_A = X M_A X^T + (Z X^T + X Z^T)/2
      G_B = X M_B X^T - (Z Lam X^T + X Lam Z^T)/2
    with column i of Z the solution of (A - lam_i B) z_i = -(I - B X X^T) g_X_i,
    X^T B z_i = 0."""
    if lam is None or X is None:
        lam, X = lowest_pairs(A, B, n_e)
    g_lam = np.asarray(g_lam, dtype=np.float64)
    R = projected_rhs(B, X, g_X)
    Z = np.column_stack([solve_projected(A, B, X, lam[i], R[:, i]) for i in range(n_e)])
    MA, MB = occupied_blocks(lam, g_lam, X.T @ g_X)
    GA = X @ MA @ X.T + 0.5 * (Z @ X.T + X @ Z.T)
    GB = X @ MB @ X.T - 0.5 * ((Z * lam[None, :]) @ X.T + X @ (Z * lam[None, :]).T)
    return _sym(GA), _sym(GB), Z
