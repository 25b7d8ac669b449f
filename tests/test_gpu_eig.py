"""GPU parity of the small symmetric eigensolver used for the projected problems."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("m,batch,seed", [(1, 1, 0), (2, 3, 1), (7, 2, 2), (64, 4, 3), (111, 2, 4), (112, 3, 5)])
def test_sym_eig_matches_lapack(gpu_lib, m, batch, seed):
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((batch, m, m))
    M = 0.5 * (G + G.transpose(0, 2, 1))
    W, V = gpu_lib.sym_eig(torch.from_numpy(M).cuda())
    W = W.cpu().numpy()
    V = V.cpu().numpy()
    for b in range(batch):
        ref = np.linalg.eigvalsh(M[b])
        scale = np.abs(ref).max()
        assert np.max(np.abs(W[b] - ref)) <= 1e-13 * scale
        assert np.all(np.diff(W[b]) >= 0)
        assert np.max(np.abs(V[b].T @ V[b] - np.eye(m))) <= 1e-13
        assert np.max(np.abs(M[b] @ V[b] - V[b] * W[b][None, :])) <= 1e-13 * scale


def test_sym_eig_graded_spectrum_relative_accuracy(gpu_lib):
    # shift-invert projected matrices mix eigenvalues from 1e-3 to 1e3
    rng = np.random.default_rng(9)
    m = 96
    Q, _ = np.linalg.qr(rng.standard_normal((m, m)))
    lam = np.sort(np.concatenate([rng.uniform(-1e3, 1e3, 20), rng.uniform(-1e-2, 1e-2, 76)]))
    M = (Q * lam) @ Q.T
    M = 0.5 * (M + M.T)
    W, V = gpu_lib.sym_eig(torch.from_numpy(M).cuda())
    W = W.cpu().numpy()
    ref = np.linalg.eigvalsh(M)
    assert np.max(np.abs(W - ref)) <= 1e-12 * 1e3


def test_sym_eig_clustered_batch_over_record_chunks(gpu_lib):
    # 70 matrices of order 112 span two chunks of the rotation record; the spectra
    # repeat eigenvalues (multiplicity 4) so the eigenvectors are checked through
    # orthogonality and the residual, which do not depend on the basis chosen
    rng = np.random.default_rng(11)
    batch, m = 70, 112
    Ms = []
    for _ in range(batch):
        Q, _ = np.linalg.qr(rng.standard_normal((m, m)))
        lam = np.repeat(rng.uniform(-5.0, 5.0, m // 4), 4)
        M = (Q * lam) @ Q.T
        Ms.append(0.5 * (M + M.T))
    M = np.stack(Ms)
    W, V = gpu_lib.sym_eig(torch.from_numpy(M).cuda())
    W = W.cpu().numpy()
    V = V.cpu().numpy()
    for b in (0, 1, 63, 64, 69):
        ref = np.linalg.eigvalsh(M[b])
        scale = np.abs(ref).max()
        assert np.max(np.abs(W[b] - ref)) <= 1e-13 * scale
        assert np.max(np.abs(V[b].T @ V[b] - np.eye(m))) <= 1e-13
        assert np.max(np.abs(M[b] @ V[b] - V[b] * W[b][None, :])) <= 1e-13 * scale
