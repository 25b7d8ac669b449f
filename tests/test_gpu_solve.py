"""GPU parity of the shift-invert solve X = C^{-1} Y through the library's factors."""
import numpy as np
import pytest
import torch

from oracle import bk
from paper_1908_06043_amd import inputs

pytestmark = pytest.mark.gpu


def dev(M):
    return torch.from_numpy(np.ascontiguousarray(M)).cuda()


@pytest.mark.parametrize("n,nrhs,seed", [(1, 1, 0), (5, 3, 1), (64, 8, 2), (65, 8, 3), (130, 20, 4),
                                         (333, 8, 5), (777, 33, 6), (1000, 64, 7),
                                         (2500, 8, 8)])
def test_solve_matches_oracle(gpu_lib, n, nrhs, seed):
    C = inputs.random_symmetric(n, seed)
    f = gpu_lib.ldlt_factor(dev(C), dev(np.eye(n)), 0.0)
    rng = np.random.default_rng(seed)
    Y = rng.standard_normal((n, nrhs))
    X = gpu_lib.ldlt_solve(f, dev(Y)).cpu().numpy()
    ref = bk.ldlt_solve(bk.bk_ldlt(C), Y)
    kappa = np.linalg.cond(C)

    def backward(Xs):
        return np.linalg.norm(C @ Xs - Y) / (np.linalg.norm(C) * np.linalg.norm(Xs))

    # both are backward stable, so the solutions agree to cond(C) times the sum of
    # their backward errors (each at least one rounding); the oracle's own
    # Bunch-Kaufman growth sets its share at larger n
    r, r_ref = backward(X), backward(ref)
    assert r < 1e-13
    bound = 10.0 * max(kappa, 1.0) * (max(r, 1e-16) + max(r_ref, 1e-16))
    assert np.linalg.norm(X - ref) / np.linalg.norm(ref) < bound


def test_solve_pencil_shift_and_repeat(gpu_lib):
    P = inputs.pencil_scf(500, 50, seed=1)
    s = inputs.safe_shifts(P.lam, [P.lam[20] + 0.3 * (P.lam[21] - P.lam[20])])[0]
    C = bk.shifted(P.A, P.B, s)
    f = gpu_lib.ldlt_factor(dev(P.A), dev(P.B), s)
    rng = np.random.default_rng(3)
    Y = rng.standard_normal((500, 8))
    X1 = gpu_lib.ldlt_solve(f, dev(Y)).cpu().numpy()
    X2 = gpu_lib.ldlt_solve(f, dev(Y)).cpu().numpy()
    assert np.array_equal(X1, X2)                        # deterministic, epoch flags reused
    r = np.linalg.norm(C @ X1 - Y) / (np.linalg.norm(C) * np.linalg.norm(X1))
    assert r < 1e-13


def test_bounded_waits_report_an_error_and_recover(gpu_lib):
    """The hand-off waits of the sweeps are bounded.  With the bound forced to zero
    polls from the host, every wait that does not find its block at the first look
    gives up at once (the kernels still run to completion): the solve reports
    SISLICE_ERR_HIP.  With the default bound restored, the next solve is correct."""
    P = inputs.pencil_scf(1000, 100, seed=1)
    A, B = dev(P.A), dev(P.B)
    print("bounded waits: solve with a zero wait bound", flush=True)
    gpu_lib.set_wait_limit(0)
    try:
        out = gpu_lib.solve(A, B, 100, 8, check=False)
    finally:
        gpu_lib.set_wait_limit(1 << 21)
    assert out["status"] == -2
    print("bounded waits: solve with the default bound", flush=True)
    out = gpu_lib.solve(A, B, 100, 8)
    ev = out["evals"].cpu().numpy()
    assert out["status"] == 0 and np.max(np.abs(ev - P.lam[:100])) <= 1e-10 * np.max(np.abs(P.lam))
