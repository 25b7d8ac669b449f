"""A posteriori certificate of the plain path at the SCF sequence's size:
N=12288, lowest n_e=1200, 48 KPM shifts (the per-step solve of that workload).

At this order no dense eigensolve runs in test time, so correctness is certified
on the host from the returned pairs themselves (Sec. 2.2: residuals plus inertia
counts make the match one to one):
  * exactly n_e pairs, ascending;
  * every normalised residual ||A x - lambda B x|| / (||A||_2 ||x||) <= 1e-10,
    recomputed on the host with ||A||_2 computed on the host;
  * X^T B X = I to 1e-10;
  * the inertia nu(sigma_j) of every shift and of the top boundary equals the
    number of constructed eigenvalues below it (bit-exact), and the number of
    returned eigenvalues below each shift under the top returned value equals
    nu(sigma_j): no eigenvalue is missing from any slice;
  * the eigenvalues equal the construction's lowest n_e within 1e-10 ||A||_2.
"""
import numpy as np
import pytest

from gpu_helpers import host_norm2
from paper_1908_06043_amd import inputs

pytestmark = pytest.mark.gpu


def test_n12288_ne1200_48_shifts_certificate(gpu_lib):
    api = gpu_lib
    n, n_e, n_s = 12288, 1200, 48
    print(f"certificate: building the N={n} pencil on the device", flush=True)
    A, B, lam = inputs.make_pencil_device(n, lambda r, m: inputs.spectrum_scf(r, m, n_e), 0, "cuda")
    plan = api.plan_shifts_kpm(A, B, n_e, n_s)
    print("certificate: solve", flush=True)
    out = api.solve(A, B, n_e, n_s, sigmas=plan["sigmas"], omega_top=plan["omega_top"], check=False)
    assert out["status"] == 0, (out["status"], out["report"])
    ev = out["evals"].cpu().numpy()
    X = out["evecs"].cpu().numpy()
    rep = out["report"]
    print("certificate: host checks", flush=True)
    assert ev.size == n_e and np.all(np.diff(ev) >= 0)
    Ah = A.cpu().numpy()
    Bh = B.cpu().numpy()
    del A, B
    anorm = host_norm2(Ah)
    BX = Bh @ X
    R = Ah @ X - BX * ev[None, :]
    rn = np.linalg.norm(R, axis=0) / (anorm * np.linalg.norm(X, axis=0))
    assert rn.max() <= 1e-10, rn.max()
    assert np.max(np.abs(X.T @ BX - np.eye(n_e))) <= 1e-10
    sig = plan["sigmas"]
    nu = [int(x) for x in rep["nu"]]
    assert nu == [int(np.sum(lam < s)) for s in sig]
    top = out["omega_top"]
    assert int(rep["nu_top"]) == int(np.sum(lam < top)) and int(rep["nu_top"]) >= n_e
    for s, v in zip(sig, nu):
        if s <= ev[-1]:
            assert int(np.sum(ev < s)) == v
    assert np.max(np.abs(ev - lam[:n_e])) <= 1e-10 * anorm
