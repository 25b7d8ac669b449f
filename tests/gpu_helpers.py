"""Helpers for the GPU parity tests: decode the library's documented factor format,
and the host-side spectral norm that scales the tolerances."""
import numpy as np
import scipy.sparse.linalg as spla


def host_norm2(A):
    """||A||_2 of a symmetric host matrix, computed on the host (never taken from
    the library): exact below order 1500, else the largest-magnitude eigenvalue by
    ARPACK's Lanczos to 1e-12 relative."""
    A = np.asarray(A)
    if A.shape[0] <= 1500:
        return float(np.max(np.abs(np.linalg.eigvalsh(A))))
    v0 = np.ones(A.shape[0])
    w = spla.eigsh(A, k=1, which="LM", tol=1e-12, v0=v0, return_eigenvectors=False)
    return float(np.abs(w[0]))


def decode_factor(LD, ipiv):
    """LD (n x n, mathematical indexing) and ipiv as documented in include/sislice.h ->
    (L unit lower, D block diagonal, perm, blocks)."""
    LD = np.asarray(LD)
    ipiv = np.asarray(ipiv).astype(np.int64)
    n = LD.shape[0]
    two = ipiv < 0
    perm = np.where(two, -ipiv - 1, ipiv)
    L = np.tril(LD, -1) + np.eye(n)
    D = np.diag(np.diag(LD)).copy()
    k = 0
    blocks = []
    while k < n:
        if two[k]:
            assert k + 1 < n and two[k + 1], "unpaired 2x2 marker"
            D[k + 1, k] = D[k, k + 1] = LD[k + 1, k]
            L[k + 1, k] = 0.0
            blocks.append(2)
            k += 2
        else:
            blocks.append(1)
            k += 1
    return L, D, perm, blocks


def backward_error(C, LD, ipiv):
    L, D, perm, _ = decode_factor(LD, ipiv)
    assert sorted(perm.tolist()) == list(range(C.shape[0])), "ipiv is not a permutation"
    PCP = C[np.ix_(perm, perm)]
    return float(np.linalg.norm(PCP - L @ D @ L.T) / np.linalg.norm(C))


def inertia_of(D):
    w = np.linalg.eigvalsh(D)
    return int(np.sum(w < 0)), int(np.sum(w == 0)), int(np.sum(w > 0))
