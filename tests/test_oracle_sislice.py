"""End-to-end pin of the oracle's per-pencil driver against the construction and LAPACK."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import kpm, sislice
from paper_1908_06043_amd import inputs


@pytest.fixture(scope="module")
def n200():
    P = inputs.pencil_clusters4(200, 0)
    pl = kpm.plan(P.A, P.B, 40, 4, M=64, nv=20, seed=0)
    sig = inputs.safe_shifts(P.lam, pl["sigmas"])
    top = inputs.safe_shifts(P.lam, [pl["omega_top"]])[0]
    return P, sig, top, sislice.solve(P.A, P.B, 40, sig, top, seed=0)


def test_lowest_eigenpairs_match_construction_and_lapack(n200):
    P, sig, top, r = n200
    assert r["status"] == sislice.STATUS_OK
    assert r["evals"].size == 40
    anorm = r["anorm"]
    assert np.max(np.abs(r["evals"] - P.lam[:40])) <= 1e-10 * anorm
    ref = sla.eigh(P.A, P.B, eigvals_only=True, subset_by_index=[0, 39])
    assert np.max(np.abs(r["evals"] - ref)) <= 1e-10 * anorm
    assert r["resid"].max() <= 1e-10
    X = r["evecs"]
    assert np.max(np.abs(X.T @ P.B @ X - np.eye(40))) <= 1e-10


def test_inertias_are_exact_counts(n200):
    P, sig, top, r = n200
    assert list(r["nus"]) == [int(np.sum(P.lam < s)) for s in sig]
    assert r["nu_top"] == int(np.sum(P.lam < top))
    assert all(s["case"] != 1 for s in r["slices"])


def test_missing_slice_is_reported():
    P = inputs.pencil_clusters4(200, 0)
    # only two shifts far below the window top: the top slice holds more eigenvalues
    # than the last probe can converge with a fixed tiny basis
    sig = inputs.safe_shifts(P.lam, [-1.6, -1.5])
    top = inputs.safe_shifts(P.lam, [0.8])[0]
    r = sislice.solve(P.A, P.B, 40, sig, top, seed=0, max_rounds=2, basis=16)
    assert r["status"] in (sislice.STATUS_MISSING, sislice.STATUS_NOT_CONVERGED)
