"""Slice validation (Section 2.2).

Shifts sigma_1 < ... < sigma_ns split the region into slices.  For the interior
slice (sigma_j, sigma_{j+1}) the point tau = (sigma_j + sigma_{j+1}) / 2 splits
the candidates: Ritz values of SP(sigma_j) in [sigma_j, tau] and Ritz values of
SP(sigma_{j+1}) in (tau, sigma_{j+1}) (a value exactly at tau belongs to the
lower probe).  The exact count of the slice is the difference of the inertias
nu(sigma_{j+1}) - nu(sigma_j), nu(s) = #{lambda < s}.  Three cases: equal counts
validate all candidates; more exact than candidates flags missing eigenpairs;
fewer keeps the n_exact candidates with the smallest residual norms (ties broken
by distance to the probe's own shift, then by value).

End slices (readings): the bottom slice is (-inf, sigma_1) with nu(-inf) = 0 and
takes candidates from SP(sigma_1); the top slice is [sigma_ns, omega_top) with
omega_top a boundary point whose inertia nu_top was computed like any shift, and
takes candidates from SP(sigma_ns).
"""
from __future__ import annotations

import numpy as np

CASE_OK, CASE_MISSING, CASE_TRIMMED = 0, 1, 2


def validate(sigmas, nus, thetas, resids, omega_top, nu_top):
    """sigmas: ascending shifts; nus: inertia per shift; thetas/resids: per-probe
    arrays of Ritz values and residual norms.  Returns dict with per-slice records
    and the validated (value, residual, probe, index) list sorted by value."""
    sig = np.asarray(sigmas, dtype=np.float64)
    ns = sig.size
    nus = np.asarray(nus, dtype=np.int64)
    lo_edge = np.concatenate([[-np.inf], sig])                 # slice s = [lo_edge[s], hi_edge[s])
    hi_edge = np.concatenate([sig, [omega_top]])
    nu_lo = np.concatenate([[0], nus])
    nu_hi = np.concatenate([nus, [nu_top]])
    slices = []
    validated = []
    for s in range(ns + 1):
        a, b = lo_edge[s], hi_edge[s]
        n_exact = int(nu_hi[s] - nu_lo[s])
        cands = []
        if s == 0:
            p = 0
            th = np.asarray(thetas[p])
            for i in np.nonzero(th < b)[0]:
                cands.append((float(th[i]), float(resids[p][i]), p, int(i)))
        elif s == ns:
            p = ns - 1
            th = np.asarray(thetas[p])
            for i in np.nonzero((th >= a) & (th < b))[0]:
                cands.append((float(th[i]), float(resids[p][i]), p, int(i)))
        else:
            tau = 0.5 * (a + b)
            p = s - 1
            th = np.asarray(thetas[p])
            for i in np.nonzero((th >= a) & (th <= tau))[0]:
                cands.append((float(th[i]), float(resids[p][i]), p, int(i)))
            p = s
            th = np.asarray(thetas[p])
            for i in np.nonzero((th > tau) & (th < b))[0]:
                cands.append((float(th[i]), float(resids[p][i]), p, int(i)))
        n_cand = len(cands)
        if n_exact == n_cand:
            case = CASE_OK
            keep = cands
        elif n_exact > n_cand:
            case = CASE_MISSING
            keep = cands
        else:
            case = CASE_TRIMMED

            def key(c):
                return (c[1], abs(c[0] - sig[c[2]]), c[0])
            keep = sorted(cands, key=key)[: max(n_exact, 0)]
        slices.append(dict(lo=float(a), hi=float(b), n_exact=n_exact, n_cand=n_cand, case=case))
        validated.extend(keep)
    validated.sort(key=lambda c: c[0])
    return dict(slices=slices, validated=validated)
