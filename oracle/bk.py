"""Unblocked Bunch-Kaufman LDL^T and the Sylvester inertia read from D.

The paper (Section 2.1) names the Bunch-Kaufman LDL^T factorization of
A - sigma B as the major cost of a spectral probe, and (Section 2.2) reads the
exact eigenvalue count below sigma from D by Sylvester's law of inertia.  The
paper does not restate the pivoting rule; this is the textbook rule of Bunch and
Kaufman (1977) with alpha = (1 + sqrt(17)) / 8, applied column by column with no
blocking.

Conventions (shared with the library's documented output format, not its code):

* ``perm[i]`` is the original index of the row at position i, so that
  ``C[perm][:, perm] = L D L^T``;
* L is unit lower triangular; D is block diagonal with 1x1 and 2x2 blocks;
  ``d`` holds diag(D) and ``e[k] = D[k+1, k]`` for a 2x2 block at (k, k+1);
* ``blk[k]`` is 1 for a 1x1 pivot at k, 2 for the first row of a 2x2 block and
  0 for its second row.

Inertia of D (a reading: the paper says "number of negative diagonal elements",
which is exact only for 1x1 pivots): count the negative eigenvalues of each
block.  A 2x2 block with det < 0 has one negative and one positive eigenvalue;
det > 0 gives two of the sign of its trace; det == 0 gives one zero eigenvalue
and one of the sign of the trace.
"""
from __future__ import annotations

import math

import numpy as np

ALPHA = (1.0 + math.sqrt(17.0)) / 8.0


def bk_ldlt(C, max_steps=None):
    """Factor symmetric C (only symmetry is assumed; the full array is read).

    Returns dict(L, d, e, perm, blk, zero_pivots, k).  ``max_steps`` stops after
    that many pivot columns (used to time a bounded sample of a large
    factorization); ``k`` is the number of columns factored.
    """
    S = np.array(C, dtype=np.float64, copy=True)
    S = 0.5 * (S + S.T)
    n = S.shape[0]
    L = np.eye(n)
    d = np.zeros(n)
    e = np.zeros(n)
    blk = np.zeros(n, dtype=np.int64)
    perm = np.arange(n)
    zero_pivots = 0

    def swap(i, j, k):
        # symmetric interchange of rows/columns i and j of the trailing matrix,
        # and of rows i and j of the already computed columns 0..k-1 of L
        S[[i, j], :] = S[[j, i], :]
        S[:, [i, j]] = S[:, [j, i]]
        L[[i, j], :k] = L[[j, i], :k]
        perm[[i, j]] = perm[[j, i]]

    k = 0
    limit = n if max_steps is None else min(n, int(max_steps))
    while k < limit:
        absakk = abs(S[k, k])
        if k + 1 < n:
            col = np.abs(S[k + 1:, k])
            imax = k + 1 + int(np.argmax(col))
            colmax = float(col[imax - k - 1])
        else:
            imax, colmax = k, 0.0
        if max(absakk, colmax) == 0.0:
            # the whole column is zero: a zero 1x1 pivot, nothing to eliminate
            d[k] = 0.0
            blk[k] = 1
            zero_pivots += 1
            k += 1
            continue
        if absakk >= ALPHA * colmax:
            kstep, kp = 1, k
        else:
            r = np.abs(S[k:, imax]).copy()
            r[imax - k] = 0.0
            rowmax = float(np.max(r))
            if absakk * rowmax >= ALPHA * colmax * colmax:
                kstep, kp = 1, k
            elif abs(S[imax, imax]) >= ALPHA * rowmax:
                kstep, kp = 1, imax
            else:
                kstep, kp = 2, imax
        kk = k + kstep - 1
        if kp != kk:
            swap(kk, kp, k)
        if kstep == 1:
            dk = S[k, k]
            d[k] = dk
            blk[k] = 1
            if dk == 0.0:
                zero_pivots += 1
            else:
                c = S[k + 1:, k].copy()
                L[k + 1:, k] = c / dk
                S[k + 1:, k + 1:] -= np.outer(c, c) / dk
        else:
            D2 = S[k:k + 2, k:k + 2].copy()
            d[k], d[k + 1], e[k] = D2[0, 0], D2[1, 1], D2[1, 0]
            blk[k], blk[k + 1] = 2, 0
            Cc = S[k + 2:, k:k + 2].copy()
            Lb = Cc @ np.linalg.inv(D2)
            L[k + 2:, k:k + 2] = Lb
            S[k + 2:, k + 2:] -= Lb @ Cc.T
        k += kstep
    return dict(L=L, d=d, e=e, perm=perm, blk=blk, zero_pivots=zero_pivots, k=k)


def d_matrix(f):
    """Dense block-diagonal D of a factorization."""
    n = f["d"].size
    D = np.diag(f["d"])
    for k in range(n):
        if f["blk"][k] == 2:
            D[k + 1, k] = D[k, k + 1] = f["e"][k]
    return D


def inertia(f):
    """(n_negative, n_zero, n_positive) of D, block by block (see module docstring)."""
    neg = zero = pos = 0
    d, e, blk = f["d"], f["e"], f["blk"]
    n = d.size
    k = 0
    while k < n:
        if blk[k] == 1:
            if d[k] < 0:
                neg += 1
            elif d[k] == 0:
                zero += 1
            else:
                pos += 1
            k += 1
        else:
            a, c, b = d[k], d[k + 1], e[k]
            det = a * c - b * b
            tr = a + c
            if det < 0:
                neg += 1
                pos += 1
            elif det > 0:
                if tr < 0:
                    neg += 2
                else:
                    pos += 2
            else:
                zero += 1
                if tr < 0:
                    neg += 1
                elif tr > 0:
                    pos += 1
                else:
                    zero += 1
            k += 2
    return neg, zero, pos


def shifted(A, B, sigma):
    """C = A - sigma B (Algorithm 2, second step)."""
    return np.asarray(A, dtype=np.float64) - float(sigma) * np.asarray(B, dtype=np.float64)


def ldlt_solve(f, U):
    """X = C^{-1} U through the factorization: permute, L^{-1}, D^{-1}, L^{-T}, unpermute."""
    import scipy.linalg as sla
    U = np.asarray(U, dtype=np.float64)
    vec = U.ndim == 1
    if vec:
        U = U[:, None]
    perm = f["perm"]
    y = U[perm, :]
    z = sla.solve_triangular(f["L"], y, lower=True, unit_diagonal=True)
    w = np.linalg.solve(d_matrix(f), z)
    v = sla.solve_triangular(f["L"].T, w, lower=False, unit_diagonal=True)
    X = np.empty_like(v)
    X[perm, :] = v
    return X[:, 0] if vec else X


def backward_error(C, f):
    """||P C P^T - L D L^T||_F / ||C||_F."""
    p = f["perm"]
    PCP = np.asarray(C)[np.ix_(p, p)]
    R = PCP - f["L"] @ d_matrix(f) @ f["L"].T
    return float(np.linalg.norm(R) / max(np.linalg.norm(C), 1e-300))
