"""GPU parity of the eigenpair adjoint (sislice_adjoint) and its autograd Function.

Bar: G_A and G_B within 1e-6 relative (max-norm) of the oracle's dense
sum-over-states gradient, exactly symmetric; central differences of the GPU
forward solve agree with tr(G E) to 1e-6 relative; reusing the solve's
factorizations and refactoring give the same gradients.
"""
import numpy as np
import pytest
import torch

from oracle import adjoint as adj
from oracle import kpm
from paper_1908_06043_amd import inputs

pytestmark = pytest.mark.gpu


def dev(M):
    return torch.from_numpy(np.ascontiguousarray(M)).cuda()


def rel_max(G, R):
    return float(np.max(np.abs(G - R)) / np.max(np.abs(R)))


def setup(n, n_e, n_s, seed, wseed):
    P = inputs.pencil_adjoint(n, n_e, seed)
    pl = kpm.plan(P.A, P.B, n_e, n_s, M=64, nv=20, seed=0)
    sig = inputs.safe_shifts(P.lam, pl["sigmas"])
    top = inputs.safe_shifts(P.lam, [pl["omega_top"]])[0]
    W = inputs.sym_gaussian(n, wseed)
    return P, sig, top, W


@pytest.fixture(scope="module")
def small():
    return setup(240, 40, 4, 1, 5)


def forward(api, A, B, n_e, sig, top):
    out = api.solve(A, B, n_e, len(sig), sigmas=sig, omega_top=top)
    assert out["status"] == 0
    return out


def test_density_gradient_matches_oracle(gpu_lib, small):
    api = gpu_lib
    P, sig, top, W = small
    n_e = 40
    print(f"adjoint density n={P.n} n_e={n_e} shifts={len(sig)}", flush=True)
    A, B, Wd = dev(P.A), dev(P.B), dev(W)
    out = forward(api, A, B, n_e, sig, top)
    lam, X = out["evals"], out["evecs"]
    GA, GB, rep = api.adjoint(A, B, lam, X, 2.0 * lam, 2.0 * (Wd @ X), sig, out["omega_top"],
                              out["report"]["factor_id"])
    assert rep["status"] == 0 and rep["reused_factors"] == 1 and rep["breakdowns"] == 0
    assert rep["max_rel_residual"] <= 1e-10
    GA, GB = GA.cpu().numpy(), GB.cpu().numpy()
    assert np.array_equal(GA, GA.T) and np.array_equal(GB, GB.T)
    lo, Xo = adj.lowest_pairs(P.A, P.B, n_e)
    gl, gx = adj.density_cotangents(lo, Xo, W)
    RA, RB = adj.grad_sum_over_states(P.A, P.B, n_e, gl, gx, Xo)
    assert rel_max(GA, RA) <= 1e-6, rel_max(GA, RA)
    assert rel_max(GB, RB) <= 1e-6, rel_max(GB, RB)


def test_eigenvalue_only_gradient(gpu_lib, small):
    # g_X = None: G_A = X diag(g) X^T, G_B = -X diag(lam g) X^T with the constructed X
    api = gpu_lib
    P, sig, top, _ = small
    n_e = 40
    A, B = dev(P.A), dev(P.B)
    out = forward(api, A, B, n_e, sig, top)
    g = torch.linspace(-1.0, 2.0, n_e, dtype=torch.float64, device="cuda")
    GA, GB, rep = api.adjoint(A, B, out["evals"], out["evecs"], g, None, sig, out["omega_top"],
                              out["report"]["factor_id"])
    assert rep["iterations"] == 0
    Xc = P.eigvecs()[:, :n_e]
    gh = g.cpu().numpy()
    RA = (Xc * gh[None, :]) @ Xc.T
    RB = -(Xc * (gh * P.lam[:n_e])[None, :]) @ Xc.T
    assert rel_max(GA.cpu().numpy(), RA) <= 1e-8
    assert rel_max(GB.cpu().numpy(), RB) <= 1e-8


def test_zero_cotangents_give_zero(gpu_lib, small):
    api = gpu_lib
    P, sig, top, _ = small
    A, B = dev(P.A), dev(P.B)
    out = forward(api, A, B, 40, sig, top)
    GA, GB, rep = api.adjoint(A, B, out["evals"], out["evecs"], None, None, sig, out["omega_top"],
                              out["report"]["factor_id"])
    assert float(GA.abs().max()) == 0.0 and float(GB.abs().max()) == 0.0


def test_refactor_path_matches_reuse(gpu_lib, small):
    api = gpu_lib
    P, sig, top, W = small
    A, B, Wd = dev(P.A), dev(P.B), dev(W)
    out = forward(api, A, B, 40, sig, top)
    lam, X = out["evals"], out["evecs"]
    gx = 2.0 * (Wd @ X)
    GA1, GB1, r1 = api.adjoint(A, B, lam, X, 2.0 * lam, gx, sig, out["omega_top"],
                               out["report"]["factor_id"])
    GA2, GB2, r2 = api.adjoint(A, B, lam, X, 2.0 * lam, gx, sig, out["omega_top"], 0)
    assert r1["reused_factors"] == 1 and r2["reused_factors"] == 0
    assert rel_max(GA2.cpu().numpy(), GA1.cpu().numpy()) <= 1e-12
    assert rel_max(GB2.cpu().numpy(), GB1.cpu().numpy()) <= 1e-12


def test_autograd_function(gpu_lib, small):
    api = gpu_lib
    P, sig, top, W = small
    n_e = 40
    A = dev(P.A).requires_grad_(True)
    B = dev(P.B).requires_grad_(True)
    Wd = dev(W)
    lam, X = api.eigh_pencil(A, B, n_e, len(sig), sigmas=sig, omega_top=top)
    loss = (lam ** 2).sum() + (Wd * (X @ X.T)).sum()
    loss.backward()
    lo, Xo = adj.lowest_pairs(P.A, P.B, n_e)
    gl, gx = adj.density_cotangents(lo, Xo, W)
    RA, RB = adj.grad_sum_over_states(P.A, P.B, n_e, gl, gx, Xo)
    assert rel_max(A.grad.cpu().numpy(), RA) <= 1e-6
    assert rel_max(B.grad.cpu().numpy(), RB) <= 1e-6
    lv = float(loss.detach())
    assert abs(lv - adj.loss_density(P.A, P.B, n_e, W)) <= 1e-9 * abs(lv)


def test_no_usable_preconditioner_rejected(gpu_lib, small):
    # every point above lambda_{n_e+1}: no positive definite preconditioner
    api = gpu_lib
    P, sig, top, W = small
    A, B = dev(P.A), dev(P.B)
    n_e = 10
    out = forward(api, A, B, 40, sig, top)
    lam = out["evals"][:n_e].contiguous()
    X = out["evecs"][:, :n_e]
    hi = inputs.safe_shifts(P.lam, [P.lam[20], P.lam[30]])
    GA, GB, rep = api.adjoint(A, B, lam, X, 2.0 * lam, X, hi[:1], hi[1], 0, check=False)
    assert rep["status"] == -1


def _fd_directions(api, P, W, sig, top, n_e, G, nd, seed, h=1e-6):
    """Central differences of the GPU forward loss sum lam^2 + tr(W X X^T) along nd
    symmetric unit directions (even: applied to A, odd: to B) against tr(G E)."""
    A, B, Wd = dev(P.A), dev(P.B), dev(W)
    opts = api.default_opts(tol=1e-12)

    def loss(Ad, Bd):
        o = api.solve(Ad, Bd, n_e, len(sig), sigmas=sig, omega_top=top, opts=opts)
        assert o["status"] == 0
        l, x = o["evals"], o["evecs"]
        return float((l ** 2).sum() + ((Wd @ x) * x).sum())

    E = inputs.sym_directions(P.n, nd, seed)
    fd, an = [], []
    for t in range(nd):
        e = dev(E[t])
        if t % 2 == 0:
            fd.append((loss(A + h * e, B) - loss(A - h * e, B)) / (2 * h))
            an.append(float(np.sum(G[0] * E[t])))
        else:
            fd.append((loss(A, B + h * e) - loss(A, B - h * e)) / (2 * h))
            an.append(float(np.sum(G[1] * E[t])))
    return np.array(fd), np.array(an)


def test_central_differences_small(gpu_lib, small):
    # 50 directions, h = 1e-6, on the N = 240 pencil: 1e-6 relative
    api = gpu_lib
    P, sig, top, W = small
    n_e = 40
    A, B, Wd = dev(P.A), dev(P.B), dev(W)
    opts = api.default_opts(tol=1e-12)
    out = api.solve(A, B, n_e, len(sig), sigmas=sig, omega_top=top, opts=opts)
    lam, X = out["evals"], out["evecs"]
    GA, GB, rep = api.adjoint(A, B, lam, X, 2.0 * lam, 2.0 * (Wd @ X), sig, out["omega_top"],
                              out["report"]["factor_id"])
    G = (GA.cpu().numpy(), GB.cpu().numpy())
    fd, an = _fd_directions(api, P, W, sig, out["omega_top"], n_e, G, 50, 77)
    err = np.linalg.norm(fd - an) / np.linalg.norm(an)
    print(f"central differences n=240: relative error {err:.2e}", flush=True)
    assert err <= 1e-6


@pytest.fixture(scope="module")
def full():
    return setup(2048, 200, 8, 0, 1)


def test_full_size_gradient_and_central_differences(gpu_lib, full):
    # the adjoint workload (N = 2048, n_e = 200): the dense oracle gradient to 1e-6
    # relative, and central differences (h = 1e-6) of the GPU forward solve on 50
    # symmetric directions.  At this size the differences are limited by the noise of
    # the forward loss itself (its FP64 rounding and the solver's residual tolerance),
    # which the quotient divides by h.  That noise is measured: the loss at the
    # unperturbed pencil from three more Lanczos start seeds spreads by `noise`, and a
    # central difference of two such evaluations errs by at most about noise / h; the
    # bound adds 3 noise / h to the 1e-6 relative bar.
    api = gpu_lib
    P, sig, top, W = full
    n, n_e = P.n, 200
    print(f"adjoint full n={n} n_e={n_e} shifts={len(sig)}", flush=True)
    A, B, Wd = dev(P.A), dev(P.B), dev(W)
    opts = api.default_opts(tol=1e-12)
    out = api.solve(A, B, n_e, len(sig), sigmas=sig, omega_top=top, opts=opts)
    assert out["status"] == 0
    lam, X = out["evals"], out["evecs"]
    GA, GB, rep = api.adjoint(A, B, lam, X, 2.0 * lam, 2.0 * (Wd @ X), sig, out["omega_top"],
                              out["report"]["factor_id"])
    assert rep["status"] == 0 and rep["reused_factors"] == 1
    GA, GB = GA.cpu().numpy(), GB.cpu().numpy()
    lo, Xo = adj.lowest_pairs(P.A, P.B, n_e)
    gl, gx = adj.density_cotangents(lo, Xo, W)
    RA, RB = adj.grad_sum_over_states(P.A, P.B, n_e, gl, gx, Xo)
    print(f"rel max err GA {rel_max(GA, RA):.2e} GB {rel_max(GB, RB):.2e}", flush=True)
    assert rel_max(GA, RA) <= 1e-6 and rel_max(GB, RB) <= 1e-6
    h = 1e-6
    fd, an = _fd_directions(api, P, W, sig, out["omega_top"], n_e, (GA, GB), 50, 123, h)

    def loss_seed(seed):
        o = api.solve(A, B, n_e, len(sig), sigmas=sig, omega_top=out["omega_top"],
                      opts=api.default_opts(tol=1e-12, seed=seed))
        assert o["status"] == 0
        l, x = o["evals"], o["evecs"]
        return float((l ** 2).sum() + ((Wd @ x) * x).sum())

    ls = [loss_seed(sd) for sd in (0, 1, 2, 3)]
    noise = max(abs(v - ls[0]) for v in ls[1:])
    u = np.finfo(np.float64).eps / 2
    C = float(np.sum(lo ** 2) + n_e * np.linalg.norm(W, 2))
    floor = 3.0 * max(noise, u * C) / h
    err = np.abs(fd - an)
    print(f"central differences n=2048: relative error {np.linalg.norm(fd - an) / np.linalg.norm(an):.2e}, "
          f"max abs {err.max():.2e}; loss spread over seeds {noise:.2e} (u C = {u * C:.2e}), "
          f"floor {floor:.2e}", flush=True)
    assert np.all(err <= 1e-6 * np.abs(an) + floor)
