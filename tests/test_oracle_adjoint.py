"""Pins of oracle/adjoint.py: central differences of dense eigensolves, the
eigenvalue-only closed form on constructed pencils, and the two gradient forms
against each other."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import adjoint as adj
from paper_1908_06043_amd import inputs


def _pencil(n=48, n_e=10, seed=3):
    return inputs.pencil_adjoint(n, n_e, seed)


def _tr(G, E):
    return float(np.sum(G * E))


def test_density_loss_central_differences():
    n, n_e, h = 48, 10, 1e-6
    P = _pencil(n, n_e)
    W = inputs.sym_gaussian(n, 7)
    lam, X = adj.lowest_pairs(P.A, P.B, n_e)
    gl, gx = adj.density_cotangents(lam, X, W)
    GA, GB = adj.grad_sum_over_states(P.A, P.B, n_e, gl, gx, X)
    GA2, GB2, _ = adj.grad_projected(P.A, P.B, n_e, gl, gx, lam, X)
    E = inputs.sym_directions(n, 12, 11)
    fd, an, an2 = [], [], []
    for t in range(12):
        e = E[t]
        if t % 2 == 0:  # perturb A
            fp = adj.loss_density(P.A + h * e, P.B, n_e, W)
            fm = adj.loss_density(P.A - h * e, P.B, n_e, W)
            an.append(_tr(GA, e))
            an2.append(_tr(GA2, e))
        else:           # perturb B (stays positive definite)
            fp = adj.loss_density(P.A, P.B + h * e, n_e, W)
            fm = adj.loss_density(P.A, P.B - h * e, n_e, W)
            an.append(_tr(GB, e))
            an2.append(_tr(GB2, e))
        fd.append((fp - fm) / (2 * h))
    fd, an, an2 = map(np.array, (fd, an, an2))
    assert np.linalg.norm(fd - an) <= 1e-6 * np.linalg.norm(an)
    assert np.linalg.norm(fd - an2) <= 1e-6 * np.linalg.norm(an2)
    assert np.all(np.abs(fd - an) <= 1e-6 * (np.abs(an) + 1e-3 * np.linalg.norm(an)))


def _aligned_pairs(A, B, n_e, Xref):
    lam, X = adj.lowest_pairs(A, B, n_e)
    s = np.sign(np.sum(X * (B @ Xref), axis=0))
    return lam, X * s[None, :]


def test_general_cotangent_central_differences():
    # a loss that is not invariant under the eigenvector signs: sum_i c_i lam_i +
    # sum_i u_i^T x_i, with each x_i's sign fixed continuously (aligned in B with
    # the unperturbed vector); this pins the antisymmetric occupied block and the
    # normalisation term
    n, n_e, h = 40, 8, 1e-6
    P = _pencil(n, n_e, seed=5)
    rng = np.random.default_rng(9)
    c = rng.standard_normal(n_e)
    U = rng.standard_normal((n, n_e))
    lam0, X0 = adj.lowest_pairs(P.A, P.B, n_e)

    def L(A, B):
        lam, X = _aligned_pairs(A, B, n_e, X0)
        return float(c @ lam + np.sum(U * X))

    GA, GB = adj.grad_sum_over_states(P.A, P.B, n_e, c, U, X0)
    GA2, GB2, _ = adj.grad_projected(P.A, P.B, n_e, c, U, lam0, X0)
    E = inputs.sym_directions(n, 8, 21)
    for t in range(8):
        e = E[t]
        if t % 2 == 0:
            fd = (L(P.A + h * e, P.B) - L(P.A - h * e, P.B)) / (2 * h)
            a, a2 = _tr(GA, e), _tr(GA2, e)
        else:
            fd = (L(P.A, P.B + h * e) - L(P.A, P.B - h * e)) / (2 * h)
            a, a2 = _tr(GB, e), _tr(GB2, e)
        scale = abs(a) + 1e-2 * (np.linalg.norm(GA) + np.linalg.norm(GB))
        assert abs(fd - a) <= 1e-6 * scale, (t, fd, a)
        assert abs(fd - a2) <= 1e-6 * scale, (t, fd, a2)


def test_eigenvalue_only_closed_form():
    # g_X = 0, g_lam = 1: dL = sum_i x_i^T (dA - lam_i dB) x_i, so G_A = X X^T and
    # G_B = -X Lam X^T with the constructed X = L^{-T} Q and Lam (no eigensolve)
    n, n_e = 60, 12
    P = _pencil(n, n_e, seed=8)
    Xc = P.eigvecs()[:, :n_e]
    lc = P.lam[:n_e]
    GA, GB = adj.grad_sum_over_states(P.A, P.B, n_e, np.ones(n_e), np.zeros((n, n_e)))
    GA2, GB2, Z = adj.grad_projected(P.A, P.B, n_e, np.ones(n_e), np.zeros((n, n_e)))
    ref_A = Xc @ Xc.T
    ref_B = -(Xc * lc[None, :]) @ Xc.T
    for G, R in ((GA, ref_A), (GA2, ref_A), (GB, ref_B), (GB2, ref_B)):
        assert np.max(np.abs(G - R)) <= 1e-11 * np.max(np.abs(R))
    assert np.max(np.abs(Z)) == 0.0


def test_projected_solution_properties():
    n, n_e = 50, 9
    P = _pencil(n, n_e, seed=4)
    lam, X = adj.lowest_pairs(P.A, P.B, n_e)
    W = inputs.sym_gaussian(n, 2)
    gl, gx = adj.density_cotangents(lam, X, W)
    _, _, Z = adj.grad_projected(P.A, P.B, n_e, gl, gx, lam, X)
    R = adj.projected_rhs(P.B, X, gx)
    # the right-hand sides are orthogonal to the occupied vectors
    assert np.max(np.abs(X.T @ R)) <= 1e-12 * np.max(np.abs(R))
    # Z is B-orthogonal to X and solves the shifted systems
    assert np.max(np.abs(X.T @ P.B @ Z)) <= 1e-12 * np.max(np.abs(Z))
    for i in range(n_e):
        res = P.A @ Z[:, i] - lam[i] * (P.B @ Z[:, i]) - R[:, i]
        assert np.linalg.norm(res) <= 1e-11 * np.linalg.norm(R[:, i])
    # and equals the sum over the unoccupied states
    la, Xa = sla.eigh(P.A, P.B)
    Zs = np.column_stack([Xa[:, n_e:] @ ((Xa[:, n_e:].T @ gx[:, i]) / (lam[i] - la[n_e:]))
                          for i in range(n_e)])
    assert np.max(np.abs(Z - Zs)) <= 1e-10 * np.max(np.abs(Zs))


def test_gap_of_adjoint_workload():
    P = inputs.pencil_adjoint(400, 40, 0)
    assert P.lam[40] - P.lam[39] >= 0.05 - 1e-12
