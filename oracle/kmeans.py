"""k-means shift migration (Section 3.2).

Lloyd's algorithm on the one-dimensional set of validated Ritz values: assign
every value to its nearest centroid, move every centroid to the mean of its
members, repeat.  The initial centroids are the previous shifts; after a DOS
placement the paper seeds with k-means++ (first centre uniform, later centres
drawn with probability proportional to the squared distance to the nearest
chosen centre).  Readings: assignment ties go to the lower centroid, an empty
cluster keeps its centroid, a centroid is the left-to-right sum of its members in
index order divided by their number, iteration stops when no assignment changes
or after 300 sweeps; the draws come from SplitMix64 (uniform u in [0,1) per draw, stream
index = draw number) so that every process seeding with the same value agrees.
"""
from __future__ import annotations

import numpy as np

from . import prng


def assign(x, c):
    """Index of the nearest centroid for each point (ties -> lower index)."""
    d = np.abs(np.asarray(x)[:, None] - np.asarray(c)[None, :])
    return np.argmin(d, axis=1)          # argmin returns the first (lowest) index on ties


def lloyd(x, c0, max_iter=300):
    x = np.asarray(x, dtype=np.float64)
    c = np.array(c0, dtype=np.float64, copy=True)
    lab = None
    for _ in range(max_iter):
        new = assign(x, c)
        if lab is not None and np.array_equal(new, lab):
            break
        lab = new
        for j in range(c.size):
            members = x[lab == j]
            if members.size:
                total = 0.0
                for v in members:          # left-to-right sum in index order
                    total += float(v)
                c[j] = total / members.size
    return c, lab


def kmeanspp_from_draws(x, k, u):
    """k-means++ seeding from given uniform draws u[0..k) in [0, 1): the first
    centre is point floor(u[0] n) (clamped to n - 1); centre c >= 1 is the first
    point i whose running sum of squared distances to the nearest chosen centre,
    D^2(x_0) + ... + D^2(x_i) (left to right), exceeds u[c] times their total.
    A zero total (every point is a chosen centre) repeats the last centre."""
    x = np.asarray(x, dtype=np.float64)
    n = x.size
    centres = [x[min(int(u[0] * n), n - 1)]]
    d2 = (x - centres[0]) ** 2
    for c in range(1, k):
        total = 0.0
        for v in d2:                       # left-to-right sum in index order
            total += float(v)
        if total == 0.0:
            centres.append(centres[-1])
            continue
        target = u[c] * total
        cum = 0.0
        pick = n - 1
        for i in range(n):
            cum += d2[i]
            if cum > target:
                pick = i
                break
        centres.append(x[pick])
        d2 = np.minimum(d2, (x - x[pick]) ** 2)
    return np.array(centres)


def kmeanspp_init(x, k, seed):
    """k-means++ with draw c taken from SplitMix64 output c of the k-means++
    sub-stream of `seed`."""
    s = prng.derive(seed, prng.TAG_KMEANSPP)
    return kmeanspp_from_draws(x, k, prng.uniform(s, 0, k))


def migrate(ritz, prev_shifts, use_kmeanspp=False, seed=0, max_iter=300):
    """New shifts = sorted centroids of k-means on the validated Ritz values."""
    k = len(prev_shifts)
    init = kmeanspp_init(ritz, k, seed) if use_kmeanspp else np.asarray(prev_shifts, dtype=np.float64)
    init = np.sort(init)
    c, lab = lloyd(ritz, init, max_iter)
    return np.sort(c), lab


def objective(x, c):
    x = np.asarray(x)
    lab = assign(x, c)
    return float(np.sum((x - np.asarray(c)[lab]) ** 2))


def brute_force_1d(x, k):
    """Optimal k-means objective in 1-D: clusters are contiguous in sorted order (DP)."""
    x = np.sort(np.asarray(x, dtype=np.float64))
    n = x.size
    pre = np.concatenate([[0.0], np.cumsum(x)])
    pre2 = np.concatenate([[0.0], np.cumsum(x * x)])

    def cost(i, j):  # points i..j-1
        m = j - i
        s = pre[j] - pre[i]
        return (pre2[j] - pre2[i]) - s * s / m

    INF = float("inf")
    dp = np.full((k + 1, n + 1), INF)
    dp[0, 0] = 0.0
    for c in range(1, k + 1):
        for j in range(1, n + 1):
            best = INF
            for i in range(c - 1, j):
                if dp[c - 1, i] < INF:
                    best = min(best, dp[c - 1, i] + cost(i, j))
            dp[c, j] = best
    return float(dp[k, n])
