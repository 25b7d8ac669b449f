"""Pins of the KPM density of states, its closed-form CDOS and the shift placement."""
import math

import numpy as np
import pytest

from oracle import kpm
from paper_1908_06043_amd import inputs


def test_jackson_is_autocorrelation_of_sine_window():
    # the Jackson kernel is |sum_j a_j e^{i j t}|^2 with a_j = sin(pi (j+1)/(M+1)), so its
    # damping factors are the normalised autocorrelation of that window
    for M in (4, 16, 64):
        g = kpm.jackson(M)
        a = np.sin(math.pi * (np.arange(M) + 1) / (M + 1))
        ac = np.array([np.sum(a[: M - k] * a[k:]) for k in range(M)]) / np.sum(a * a)
        assert np.max(np.abs(g - ac)) < 1e-15
        assert g[0] == pytest.approx(1.0, abs=1e-15)


def test_moments_exact_for_diagonal_operator():
    # diagonal H: v^T T_k(H) v = sum_i v_i^2 T_k(h_i) = trace T_k(H) for v in {+-1}^N
    rng = np.random.default_rng(0)
    lam = np.sort(rng.uniform(-3, 2, 77))
    P = inputs.pencil_diag(lam)
    op = kpm.Operator(P.A, P.B)
    a, b = -3.5, 2.5
    mu = kpm.moments(op, a, b, 40, 5, seed=3)
    t = (lam - 0.5 * (a + b)) / (0.5 * (b - a))
    exact = np.array([np.mean(np.cos(k * np.arccos(t))) for k in range(40)])
    assert np.max(np.abs(mu - exact)) < 1e-13
    assert mu[0] == 1.0


def test_generalized_operator_is_congruent_to_pencil():
    P = inputs.pencil_clusters4(60, 1)
    op = kpm.Operator(P.A, P.B)
    H = op(np.eye(60))
    w = np.linalg.eigvalsh(0.5 * (H + H.T))
    assert np.max(np.abs(w - P.lam)) < 1e-12


def test_cdos_closed_form_matches_quadrature_of_density():
    rng = np.random.default_rng(1)
    lam = np.sort(rng.uniform(-1, 1, 50))
    P = inputs.pencil_diag(lam)
    op = kpm.Operator(P.A, P.B)
    a, b = -1.2, 1.3
    M = 32
    mu = kpm.moments(op, a, b, M, 3, seed=0)
    g = kpm.jackson(M)
    # density in theta: phi(theta) d theta = (N/pi) [g0 mu0 + 2 sum g_k mu_k cos(k theta)] d theta
    def dens(th):
        v = g[0] * mu[0] + 2 * sum(g[k] * mu[k] * np.cos(k * th) for k in range(1, M))
        return v * 50 / math.pi
    for omega in (-1.0, -0.3, 0.0, 0.77):
        tt = math.acos((omega - 0.05) / 1.25)
        x = np.linspace(tt, math.pi, 200001)
        y = dens(x)
        quad = float(np.sum(0.5 * (y[1:] + y[:-1]) * np.diff(x)))
        assert kpm.cdos(omega, mu, g, a, b, 50) == pytest.approx(quad, abs=1e-6)
    assert kpm.cdos(a, mu, g, a, b, 50) == pytest.approx(0.0, abs=1e-12)
    assert kpm.cdos(b, mu, g, a, b, 50) == pytest.approx(50.0, abs=1e-12)


def test_cdos_tracks_eigenvalue_count_within_resolution():
    rng = np.random.default_rng(2)
    lam = np.sort(rng.uniform(-1, 1, 400))
    P = inputs.pencil_diag(lam)
    op = kpm.Operator(P.A, P.B)
    a, b = -1.05, 1.05
    M = 128
    mu = kpm.moments(op, a, b, M, 1, seed=0)
    g = kpm.jackson(M)
    grid = np.linspace(-0.9, 0.9, 37)
    phi = kpm.cdos(grid, mu, g, a, b, 400)
    assert np.all(np.diff(phi) >= -1e-9)                    # Jackson damping keeps it monotone
    res = math.pi * (b - a) / M                              # kernel resolution
    for w, p in zip(grid, phi):
        lo = np.sum(lam < w - res)
        hi = np.sum(lam < w + res)
        assert lo - 1 <= p <= hi + 1


def test_bounds_enclose_spectrum():
    P = inputs.pencil_scf(300, 30, seed=1)
    op = kpm.Operator(P.A, P.B)
    a, b = kpm.lanczos_bounds(op, seed=0)
    assert a < P.lam[0] and b > P.lam[-1]
    assert b - a < 1.2 * (P.lam[-1] - P.lam[0])


def test_place_shifts_equal_counts_and_midpoints():
    P = inputs.pencil_scf(300, 60, seed=2)
    pl = kpm.plan(P.A, P.B, 60, 6, M=64, nv=10, seed=0)
    g = kpm.jackson(64)
    om = pl["omegas"]
    top_count = 60 + 2.0 * 10.0
    assert kpm.cdos(pl["omega_top"], pl["mu"], g, pl["a"], pl["b"], 300) == pytest.approx(top_count, abs=1e-6)
    for j in range(1, 7):
        assert kpm.cdos(om[j], pl["mu"], g, pl["a"], pl["b"], 300) == pytest.approx(top_count * j / 6, abs=1e-6)
    assert om[-1] == pytest.approx(pl["omega_top"], abs=1e-9)
    assert np.allclose(pl["sigmas"], 0.5 * (om[:-1] + om[1:]), rtol=0, atol=1e-15)
    assert np.all(np.diff(pl["sigmas"]) > 0)
