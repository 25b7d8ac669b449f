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
    # matrices per chunk of the record: 256 MiB over 40 sweeps x 111 rounds x 56 pairs
    # of (c, s) at order 112 (67), so chunk - 1 and chunk sit on either side of the seam
    chunk = (256 << 20) // (40 * 111 * 56 * 16)
    assert 1 < chunk < batch - 1
    for b in (0, 1, chunk - 1, chunk, batch - 1):
        ref = np.linalg.eigvalsh(M[b])
        scale = np.abs(ref).max()
        assert np.max(np.abs(W[b] - ref)) <= 1e-13 * scale
        assert np.max(np.abs(V[b].T @ V[b] - np.eye(m))) <= 1e-13
        assert np.max(np.abs(M[b] @ V[b] - V[b] * W[b][None, :])) <= 1e-13 * scale


def test_sym_eig_mixed_orders_in_one_batch(gpu_lib):
    # the solve path launches one batch over probes whose projected orders differ;
    # odd orders pad the round-robin with a dummy player
    from paper_1908_06043_amd import api
    rng = np.random.default_rng(13)
    orders = [1, 2, 7, 37, 64, 111, 112, 50, 3, 112, 96]
    mats = []
    for m in orders:
        G = rng.standard_normal((m, m))
        mats.append(0.5 * (G + G.T) + np.diag(rng.uniform(-3.0, 3.0, m)))
    out = api.sym_eig_var([torch.from_numpy(x).cuda() for x in mats])
    for x, (W, V) in zip(mats, out):
        m = x.shape[0]
        W = W.cpu().numpy()
        V = V.cpu().numpy()
        ref = np.linalg.eigvalsh(x)
        scale = np.abs(ref).max()
        assert np.max(np.abs(W - ref)) <= 1e-13 * scale
        assert np.max(np.abs(V.T @ V - np.eye(m))) <= 1e-13
        assert np.max(np.abs(x @ V - V * W[None, :])) <= 1e-13 * scale
