"""Per-pencil spectrum slicing driver (Algorithm 1 on a fixed pencil, one pass).

For a given ascending shift set sigma_1..sigma_ns and a top boundary omega_top:

1. factor A - sigma_j B for every shift and for omega_top (Bunch-Kaufman) and
   read the inertias nu(sigma_j) = #{lambda < sigma_j} (Section 2.2);
2. per probe j run Algorithm 2 (M subspace iterations, Rayleigh-Ritz) repeatedly,
   warm-started from its previous Ritz vectors exactly as the paper re-seeds
   successive SCF steps (Section 2.1), until the Ritz values inside the probe's
   window (sigma_{j-1}, sigma_{j+1}) (ends: -inf and omega_top) that meet the
   residual tolerance number nu(sigma_{j+1}) - nu(sigma_{j-1});
3. validate the slices (Section 2.2) and return the lowest n_e validated pairs.

The basis size of probe j is max(2 * need_j, 16) (the paper advises a basis
several times the wanted count, Section 2.1 / 5.4).  Start blocks are Gaussian
draws from the shared SplitMix64 stream.
"""
from __future__ import annotations

import numpy as np

from . import bk, prng, sisubit, validate

STATUS_OK, STATUS_SINGULAR, STATUS_NOT_CONVERGED, STATUS_MISSING = 0, 1, 2, 3


def probe_start_block(seed, j, n, k):
    s = prng.derive(seed, prng.TAG_LANCZOS ^ (j << 32))
    return prng.gauss(s, 0, n * k).reshape(k, n).T.copy()


def solve(A, B, n_e, sigmas, omega_top, tol=1e-10, M=4, seed=0, max_rounds=100,
          anorm=None, basis=None):
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    n = A.shape[0]
    sig = np.sort(np.asarray(sigmas, dtype=np.float64))
    ns = sig.size
    if anorm is None:
        anorm = sisubit.norm2_sym(A)
    facs = [bk.bk_ldlt(bk.shifted(A, B, s)) for s in sig]
    inert = [bk.inertia(f) for f in facs]
    top_fac = bk.bk_ldlt(bk.shifted(A, B, omega_top))
    top_inert = bk.inertia(top_fac)
    status = STATUS_OK
    if any(i[1] > 0 for i in inert) or top_inert[1] > 0:
        status = STATUS_SINGULAR
    nus = np.array([i[0] for i in inert], dtype=np.int64)
    nu_top = int(top_inert[0])
    thetas, resids, vecs, rounds = [], [], [], []
    for j in range(ns):
        lo = sig[j - 1] if j > 0 else -np.inf
        hi = sig[j + 1] if j + 1 < ns else omega_top
        nu_lo = nus[j - 1] if j > 0 else 0
        nu_hi = nus[j + 1] if j + 1 < ns else nu_top
        need = int(nu_hi - nu_lo)
        k = min(n, basis if basis is not None else max(2 * need, 16))
        V = probe_start_block(seed, j, n, k)
        lam = X = res = None
        r = 0
        for r in range(1, max_rounds + 1):
            lam, X, _ = sisubit.sisubit(A, B, V, sig[j], M, fac=facs[j])
            res = sisubit.residual_norms(A, B, X, lam, anorm)
            inwin = (lam > lo) & (lam < hi)
            if np.count_nonzero(inwin & (res <= tol)) >= need:
                break
            V = X
        thetas.append(lam)
        resids.append(res)
        vecs.append(X)
        rounds.append(r)
    val = validate.validate(sig, nus, thetas, resids, omega_top, nu_top)
    chosen = val["validated"][:n_e]
    if any(s["case"] == validate.CASE_MISSING for s in val["slices"]) or len(chosen) < n_e:
        status = status or STATUS_MISSING
    evals = np.array([c[0] for c in chosen])
    res = np.array([c[1] for c in chosen])
    evecs = np.stack([vecs[c[2]][:, c[3]] for c in chosen], axis=1) if chosen else np.zeros((n, 0))
    if status == STATUS_OK and np.any(res > tol):
        status = STATUS_NOT_CONVERGED
    return dict(evals=evals, evecs=evecs, resid=res, nus=nus, nu_top=nu_top, slices=val["slices"],
                rounds=rounds, status=status, anorm=anorm, thetas=thetas, resids=resids)
