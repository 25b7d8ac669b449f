"""Lanczos density-of-states shift selection (Section 3.1: eq. dos, eq. cdos,
eq. cdos_root, Algorithm DOSCluster, its refinement, the DOS-expectation shifts
and the safeguards).

TEST INFRASTRUCTURE ONLY (see the package header).

Estimator.  n_v runs of k-step Lanczos (full reorthogonalisation) on
H = L_B^{-1} A L_B^{-T} (the first of the two forms the paper gives), each from a
normalised Gaussian start vector; run r gives Ritz pairs (theta_j, g_j) and
zeta_j = e_1^T g_j.  Each Ritz value carries a Gaussian of width nu_j:

  phi(w) = N / sqrt(2 pi) * mean_r sum_j zeta_j^2 / nu_j exp(-kappa_j(w)^2)
  Phi(w) = N / 2 * mean_r sum_j zeta_j^2 (erf(kappa_j(w)) + 1)
  kappa_j(w) = (w - theta_j) / (nu_j sqrt 2)

(the paper's formulas for one run, averaged over the runs).  Readings where the
paper is open: d_j = max(theta_j - theta_{j-1}, theta_{j+1} - theta_j) (one-sided
at the ends), floored at 1e-3 (b - a) / k with [a, b] the range of all Ritz
values; nu_j = d_j / 3, so each Gaussian is down to exp(-4.5) at distance d_j.

Planners.
* ``plan_cdos``: equal-count roots of Phi on [a, omega_top] with omega_top the
  root of Phi = n_e + top_margin n_e / n_s, one shift at each interval midpoint
  (the same reading of eq. cdos_root as the KPM planner).
* ``plan_cluster``: DOSCluster on a grid of n_omega = 10 k points of
  [a, omega_top]; intervals with gamma = Phi(u) - Phi(l) < 2 merge into the
  adjacent interval with fewer estimated eigenvalues; intervals with gamma > 50
  are searched again with n_omega' = 2 C(l, u) / C(a, omega_top) n_omega points,
  C = ceil(gamma) (rounded half up, at least 10) and replaced when that finds two
  or more; repeated until nothing changes (at most 20 rounds); then the
  safeguards: while fewer than n_s intervals, the one with the most eigenvalues
  is split at its CDOS midpoint; while more, the one with the fewest merges into
  its adjacent neighbour with fewer (or, isolated, into the nearest); each shift
  is the DOS expectation over its interval (the psi formula).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

from . import prng
from .kpm import Operator

TAG_DOS = 0x444F53            # start vectors of the Lanczos DOS runs


def lanczos_runs(op, k, nv, seed):
    """n_v runs of k-step Lanczos: list of (theta (k,), zeta2 (k,))."""
    n = op.n
    s = prng.derive(seed, TAG_DOS)
    out = []
    for r in range(nv):
        v = prng.gauss(s, r * n, n)
        v = v / np.linalg.norm(v)
        V = np.zeros((n, k))
        alpha = np.zeros(k)
        beta = np.zeros(k)
        V[:, 0] = v
        m = k
        for j in range(k):
            w = op(V[:, j:j + 1])[:, 0]
            alpha[j] = V[:, j] @ w
            w = w - alpha[j] * V[:, j] - (beta[j - 1] * V[:, j - 1] if j > 0 else 0.0)
            for _ in range(2):                       # full reorthogonalisation, twice
                w = w - V[:, :j + 1] @ (V[:, :j + 1].T @ w)
            if j + 1 < k:
                beta[j] = np.linalg.norm(w)
                if beta[j] == 0.0:
                    m = j + 1
                    break
                V[:, j + 1] = w / beta[j]
        T = np.diag(alpha[:m]) + np.diag(beta[:m - 1], 1) + np.diag(beta[:m - 1], -1)
        th, G = np.linalg.eigh(T)
        out.append((th, G[0, :] ** 2))
    return out


class LanczosDOS:
    """phi, Phi and the DOS expectation of the estimate (eq. dos / cdos)."""

    def __init__(self, runs, n, k):
        self.n = n
        allth = np.concatenate([th for th, _ in runs])
        self.a, self.b = float(allth.min()), float(allth.max())
        floor = 1e-3 * (self.b - self.a) / k
        self.th, self.z2, self.nu = [], [], []
        for th, z2 in runs:
            d = np.empty_like(th)
            for j in range(th.size):
                left = th[j] - th[j - 1] if j > 0 else -np.inf
                right = th[j + 1] - th[j] if j + 1 < th.size else -np.inf
                d[j] = max(left, right, floor)
            self.th.append(th)
            self.z2.append(z2)
            self.nu.append(d / 3.0)
        self.nv = len(runs)

    def phi(self, w):
        w = np.atleast_1d(np.asarray(w, dtype=np.float64))
        tot = np.zeros_like(w)
        for th, z2, nu in zip(self.th, self.z2, self.nu):
            kap = (w[:, None] - th[None, :]) / (nu[None, :] * math.sqrt(2.0))
            tot += np.sum(z2[None, :] / nu[None, :] * np.exp(-kap ** 2), axis=1)
        return self.n / math.sqrt(2.0 * math.pi) * tot / self.nv

    def cdos(self, w):
        w = np.atleast_1d(np.asarray(w, dtype=np.float64))
        tot = np.zeros_like(w)
        for th, z2, nu in zip(self.th, self.z2, self.nu):
            kap = (w[:, None] - th[None, :]) / (nu[None, :] * math.sqrt(2.0))
            tot += np.sum(z2[None, :] * (erf(kap) + 1.0), axis=1)
        return self.n / 2.0 * tot / self.nv

    def expectation(self, l, u):
        """(1 / gamma(l, u)) int_l^u w phi(w) dw through psi (closed form)."""
        tot = 0.0
        for th, z2, nu in zip(self.th, self.z2, self.nu):
            def psi(w):
                kap = (w - th) / (nu * math.sqrt(2.0))
                return th / 2.0 * erf(kap) - nu / math.sqrt(2.0 * math.pi) * np.exp(-kap ** 2)
            tot += float(np.sum(z2 * (psi(u) - psi(l))))
        gam = float(self.cdos(u)[0] - self.cdos(l)[0])
        return self.n * tot / self.nv / gam

    def root(self, target, lo, hi, rel=1e-12):
        """w in [lo, hi] with Phi(w) = target (bisection; Phi is increasing)."""
        flo = float(self.cdos(lo)[0]) - target
        if flo >= 0:
            return lo
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if float(self.cdos(mid)[0]) - target < 0:
                lo = mid
            else:
                hi = mid
            if hi - lo <= rel * (self.b - self.a):
                break
        return 0.5 * (lo + hi)


def window(dos, n_e, n_s, top_margin=2.0):
    """[a, omega_top] with Phi(omega_top) = n_e + top_margin n_e / n_s."""
    span = dos.b - dos.a
    a = dos.a - 0.01 * span
    hi = dos.b + 0.01 * span
    top = dos.root(n_e + top_margin * n_e / n_s, a, hi)
    return a, top


def plan_cdos(dos, n_e, n_s, top_margin=2.0):
    """Equal-count roots and interval midpoints (eq. cdos_root)."""
    a, top = window(dos, n_e, n_s, top_margin)
    pa = float(dos.cdos(a)[0])
    K = (float(dos.cdos(top)[0]) - pa) / n_s
    pts = [a] + [dos.root(pa + j * K, a, top) for j in range(1, n_s)] + [top]
    return np.array([0.5 * (pts[j] + pts[j + 1]) for j in range(n_s)]), top


def dos_cluster(dos, lo, hi, n_omega, ritz):
    """Algorithm DOSCluster: intervals between the local minimisers that separate the
    local maximisers of phi on an n_omega-point grid of [lo, hi], keeping those
    that contain a Ritz value."""
    w = lo + (hi - lo) / (n_omega - 1) * np.arange(n_omega)
    f = dos.phi(w)
    mx = [i for i in range(n_omega)
          if (i == 0 or f[i] > f[i - 1]) and (i == n_omega - 1 or f[i] >= f[i + 1])]
    if len(mx) <= 1:
        return [(lo, hi)]
    mu = [lo]
    for j in range(len(mx) - 1):
        seg = range(mx[j] + 1, mx[j + 1])
        if len(seg) == 0:
            i = mx[j]
        else:
            i = min(seg, key=lambda t: (f[t], t))
        mu.append(float(w[i]))
    mu.append(hi)
    iv = [(mu[j], mu[j + 1]) for j in range(len(mu) - 1) if mu[j + 1] > mu[j]]
    return [(l, u) for (l, u) in iv if np.any((ritz > l) & (ritz <= u))]


def _gamma(dos, iv):
    return float(dos.cdos(iv[1])[0] - dos.cdos(iv[0])[0])


def _merge_small(dos, I, tol=2.0):
    """Merge intervals with gamma < tol into the adjacent interval with fewer
    estimated eigenvalues (adjacent: sharing an endpoint); isolated ones stay."""
    changed = True
    while changed:
        changed = False
        for j, iv in enumerate(I):
            if len(I) == 1 or _gamma(dos, iv) >= tol:
                continue
            cands = []
            if j > 0 and I[j - 1][1] == iv[0]:
                cands.append(j - 1)
            if j + 1 < len(I) and I[j + 1][0] == iv[1]:
                cands.append(j + 1)
            if not cands:
                continue
            t = min(cands, key=lambda q: (_gamma(dos, I[q]), q))
            lo, hi = min(I[t][0], iv[0]), max(I[t][1], iv[1])
            keep = [I[q] for q in range(len(I)) if q not in (j, t)]
            I = sorted(keep + [(lo, hi)])
            changed = True
            break
    return I


def count(dos, iv):
    """C(l, u) = ceil(gamma(l, u)), the approximate eigenvalue count of Sec. 3.1."""
    return math.ceil(_gamma(dos, iv))


def refine(dos, I, a, top, n_omega, ritz, big=50.0, rounds=20):
    """Refinement steps 2-4 of Sec. 3.1: merge intervals with gamma < 2 into the
    adjacent interval with fewer estimated eigenvalues; rerun DOSCluster on every
    interval with gamma > big over n_omega' = 2 C(l, u) / C(a, top) n_omega grid
    points (rounded half up; at least 10 points is this project's own floor) and
    replace it when that finds two or more intervals; repeat until nothing is
    replaced (at most `rounds` times)."""
    c_all = count(dos, (a, top))
    for _ in range(rounds):
        I = _merge_small(dos, I)
        new = []
        grew = False
        for iv in I:
            if _gamma(dos, iv) > big:
                nw = max(10, int(math.floor(2.0 * count(dos, iv) / c_all * n_omega + 0.5)))
                sub = dos_cluster(dos, iv[0], iv[1], nw, ritz)
                if len(sub) >= 2:
                    new.extend(sub)
                    grew = True
                    continue
            new.append(iv)
        I = sorted(new)
        if not grew:
            break
    return I


def safeguards(dos, I, n_s):
    """Exactly n_s intervals (Sec. 3.1 safeguards): while too few, split the
    interval with the most estimated eigenvalues at its CDOS midpoint (ties: the
    lower one); while too many, merge the one with the fewest (ties: the lower
    one) into its adjacent neighbour with fewer (ties: the lower one), or, when it
    has no adjacent neighbour, into the nearer of its list neighbours."""
    I = list(I)
    while len(I) < n_s:
        j = max(range(len(I)), key=lambda q: (_gamma(dos, I[q]), -q))
        l, u = I[j]
        mid = dos.root(0.5 * (float(dos.cdos(l)[0]) + float(dos.cdos(u)[0])), l, u)
        I = sorted(I[:j] + [(l, mid), (mid, u)] + I[j + 1:])
    while len(I) > n_s:
        j = min(range(len(I)), key=lambda q: (_gamma(dos, I[q]), q))
        cands = [q for q in (j - 1, j + 1) if 0 <= q < len(I)]
        adj = [q for q in cands if I[q][1] == I[j][0] or I[q][0] == I[j][1]]
        pool = adj if adj else cands
        t = min(pool, key=lambda q: (_gamma(dos, I[q]), q))
        lo, hi = min(I[t][0], I[j][0]), max(I[t][1], I[j][1])
        keep = [I[q] for q in range(len(I)) if q not in (j, t)]
        I = sorted(keep + [(lo, hi)])
    return I


def plan_cluster(dos, ritz, n_e, n_s, k, top_margin=2.0, big=50.0):
    """DOSCluster with refinement, safeguards and DOS-expectation shifts."""
    a, top = window(dos, n_e, n_s, top_margin)
    n_omega = 10 * k
    I = dos_cluster(dos, a, top, n_omega, ritz)
    I = refine(dos, I, a, top, n_omega, ritz, big)
    I = safeguards(dos, I, n_s)
    shifts = np.array([dos.expectation(l, u) for l, u in I])
    return np.sort(shifts), top, I


def plan(A, B, n_e, n_s, k=80, nv=8, seed=0, mode="cluster"):
    op = Operator(A, B)
    runs = lanczos_runs(op, k, nv, seed)
    dos = LanczosDOS(runs, op.n, k)
    if mode == "cdos":
        sig, top = plan_cdos(dos, n_e, n_s)
        return dict(sigmas=sig, omega_top=top, dos=dos)
    ritz = np.concatenate([th for th, _ in runs])
    sig, top, iv = plan_cluster(dos, ritz, n_e, n_s, k)
    return dict(sigmas=sig, omega_top=top, dos=dos, intervals=iv)
