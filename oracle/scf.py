"""Probe migration between SCF steps (Section 3.2) and the partial-trace monitor
(Section 3.3).

TEST INFRASTRUCTURE ONLY (see the package header).

After a solve, the validated Ritz values are clustered by k-means (``kmeans``),
seeded with the previous shifts (k-means++ after a DOS placement).  Each
cluster is mapped to the probe with which it overlaps most: the probe that
validated most of its members (reading: ties go to the probe whose previous
shift is nearest the cluster's centroid, then to the lower index).  Clusters
mapped to one probe are merged, and the probe's new shift is the mean of the
merged values.  A probe that no cluster maps to is deleted.  To keep n_s probes,
the probe holding the most values is split by 2-means (reading: Lloyd from its
smallest and largest value); the half whose centroid is nearer that probe's
previous shift stays with it, the other half seeds an inserted probe.  This
repeats until there are n_s probes again or no probe holds two values.

Means are left-to-right sums in ascending value index, so the library's C++
reproduces them bit for bit.  The partial trace eta(V, A) = tr(V^T A V) of the
previous eigenvectors under the previous and the new A is the monitor that
sends a step back to the DOS planner when the spectrum moved too much.
"""
from __future__ import annotations

import numpy as np

from . import kmeans


def _mean(x, idx):
    total = 0.0
    for i in idx:                          # left-to-right, ascending index
        total += float(x[i])
    return total / len(idx)


def _overlap_map(lab, probe_of, cent, prev, n_s):
    """Cluster -> probe of maximal overlap (-1 for an empty cluster)."""
    out = []
    for k in range(cent.size):
        members = np.nonzero(lab == k)[0]
        if members.size == 0:
            out.append(-1)
            continue
        cnt = np.bincount(np.asarray(probe_of)[members], minlength=n_s)
        best = -1
        for p in range(n_s):
            if best < 0 or cnt[p] > cnt[best] or (
                    cnt[p] == cnt[best] and abs(prev[p] - cent[k]) < abs(prev[best] - cent[k])):
                best = p
        out.append(best)
    return out


def split2(x, idx):
    """2-means of the values x[idx] from their smallest and largest value:
    (low half, high half) as ascending index lists, or None if one half is empty."""
    vals = np.asarray([x[i] for i in idx])
    c, lab = kmeans.lloyd(vals, [vals.min(), vals.max()])
    lo = [idx[t] for t in range(len(idx)) if lab[t] == 0]
    hi = [idx[t] for t in range(len(idx)) if lab[t] == 1]
    if not lo or not hi:
        return None
    return lo, hi


def migrate_probes(ritz, probe_of, prev_shifts, use_kmeanspp=False, seed=0):
    """New shifts (ascending), the values that seed each new probe, the previous
    probe each continues (-1: inserted) and the counts merged/deleted/inserted."""
    x = np.asarray(ritz, dtype=np.float64)
    prev = np.asarray(prev_shifts, dtype=np.float64)
    n_s = prev.size
    init = kmeans.kmeanspp_init(x, n_s, seed) if use_kmeanspp else prev
    cent, lab = kmeans.lloyd(x, np.sort(init))
    cmap = _overlap_map(lab, probe_of, cent, prev, n_s)
    probes = []                            # [origin, previous shift, member indices]
    merged = 0
    for p in range(n_s):
        ks = [k for k in range(cent.size) if cmap[k] == p]
        if not ks:
            continue
        merged += len(ks) - 1
        members = sorted(int(i) for k in ks for i in np.nonzero(lab == k)[0])
        probes.append([p, float(prev[p]), members])
    deleted = n_s - len(probes)
    inserted = 0
    while len(probes) < n_s:
        big = max(range(len(probes)), key=lambda q: (len(probes[q][2]), -q))
        if len(probes[big][2]) < 2:
            break
        halves = split2(x, probes[big][2])
        if halves is None:
            break
        lo, hi = halves
        ref = probes[big][1]
        keep_lo = abs(_mean(x, lo) - ref) <= abs(_mean(x, hi) - ref)
        stay, go = (lo, hi) if keep_lo else (hi, lo)
        probes[big][2] = stay
        probes.append([-1, _mean(x, go), go])
        inserted += 1
    shifts = np.array([_mean(x, pr[2]) for pr in probes])
    order = np.argsort(shifts, kind="stable")
    return dict(shifts=shifts[order], members=[probes[q][2] for q in order],
                origin=np.array([probes[q][0] for q in order], dtype=np.int64),
                merged=merged, deleted=deleted, inserted=inserted)


def partial_trace(V, A):
    """eta(V, A) = tr(V^T A V)."""
    return float(np.sum(V * (A @ V)))
