"""Seeded synthetic symmetric-definite pencils with known eigenpairs.

This module only generates inputs.  It holds none of the eigensolver's
arithmetic and is shared by the oracle-based tests and by the HIP path's
tests and benchmark, so that both sides see bit-identical pencils.

Construction (the problem statement of Section 1, eq. ``seq_gep``: A symmetric,
B symmetric positive definite):

* ``L`` unit lower triangular with ``L[i, j] = z * scale * exp(-(i-j)/decay)``
  for ``i > j``, ``z ~ N(0, 1)``;
* ``Q`` Haar-orthogonal (QR of a Gaussian matrix, sign-fixed by ``diag(R)``);
* ``B = L L^T`` and ``A = L Q diag(lam) Q^T L^T``.

Then ``X = L^{-T} Q`` satisfies ``A X = B X diag(lam)`` and ``X^T B X = I``,
so the generalized eigenvalues are exactly ``lam`` (up to the rounding of
forming ``A``) and the Sylvester inertia of ``A - sigma B`` is
``#{lam_i < sigma}``.

The random draws are taken from one ``numpy.random.default_rng(seed)`` stream
in the order L, Q, spectrum.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Pencil:
    A: np.ndarray          # n x n symmetric, float64, C-contiguous (== column-major)
    B: np.ndarray          # n x n SPD
    lam: np.ndarray        # ascending generalized eigenvalues used in the construction
    L: np.ndarray          # unit lower factor with B = L L^T
    Q: np.ndarray          # orthogonal factor; X = L^{-T} Q
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.A.shape[0]

    def eigvecs(self) -> np.ndarray:
        """X = L^{-T} Q (B-orthonormal eigenvectors, columns ordered like ``lam``)."""
        import scipy.linalg as sla
        return sla.solve_triangular(self.L.T, self.Q, lower=False, unit_diagonal=True)


def _unit_lower(rng, n, scale, decay):
    z = rng.standard_normal((n, n))
    i = np.arange(n)
    dist = (i[:, None] - i[None, :]).astype(np.float64)
    L = np.tril(z * scale * np.exp(-np.abs(dist) / decay), -1)
    L[np.diag_indices(n)] = 1.0
    return L


def _haar(rng, n):
    g = rng.standard_normal((n, n))
    q, r = np.linalg.qr(g)
    q *= np.sign(np.diag(r))[None, :]
    return q


def spectrum_clusters4(rng, n, lo=-2.0, hi=2.0, std=0.1):
    """Four Gaussian clusters centred at -1.5, -0.5, 0.5, 1.5 (std 0.1), resampled into [lo, hi]."""
    centres = np.array([-1.5, -0.5, 0.5, 1.5])
    sizes = np.full(4, n // 4)
    sizes[: n - sizes.sum()] += 1
    out = []
    for c, m in zip(centres, sizes):
        v = rng.normal(c, std, m)
        bad = (v < lo) | (v > hi)
        while bad.any():
            v[bad] = rng.normal(c, std, bad.sum())
            bad = (v < lo) | (v > hi)
        out.append(v)
    return np.sort(np.concatenate(out))


def spectrum_scf(rng, n, n_e, lo=-5.0, hi=5.0, n_clusters=12, std=0.05, gap=0.1,
                 forced_gap_at=None, forced_gap=0.0):
    """Half uniform background on [lo, hi], half in ``n_clusters`` Gaussian clusters
    (centres uniform on [lo, hi], std ``std``).  Two gaps of width ``gap`` are emptied
    at the 1/3 and 2/3 points of [lam_1, lam_{n_e}] of the first draw; values falling
    in a gap (or outside [lo, hi]) are redrawn from their own component.  If
    ``forced_gap_at = i`` then additionally lam_{i+1} - lam_i >= forced_gap is enforced
    by shifting the upper part of the spectrum (used by the adjoint workload)."""
    n_bg = n // 2
    n_cl = n - n_bg
    centres = rng.uniform(lo, hi, n_clusters)
    sizes = np.full(n_clusters, n_cl // n_clusters)
    sizes[: n_cl - sizes.sum()] += 1
    comp_centre = np.concatenate([np.full(n_bg, np.nan)] + [np.full(m, c) for c, m in zip(centres, sizes)])

    def draw(mask):
        v = np.empty(mask.sum())
        cc = comp_centre[mask]
        bgm = np.isnan(cc)
        v[bgm] = rng.uniform(lo, hi, bgm.sum())
        v[~bgm] = rng.normal(cc[~bgm], std)
        return v

    vals = np.empty(n)
    allm = np.ones(n, dtype=bool)
    vals[allm] = draw(allm)
    bad = (vals < lo) | (vals > hi)
    while bad.any():
        vals[bad] = draw(bad)
        bad = (vals < lo) | (vals > hi)
    s = np.sort(vals)
    l1, lne = s[0], s[min(n_e, n) - 1]
    gaps = [l1 + (lne - l1) / 3.0, l1 + 2.0 * (lne - l1) / 3.0]

    def in_gap(v):
        m = (v < lo) | (v > hi)
        for g in gaps:
            m |= np.abs(v - g) < gap / 2.0
        return m

    bad = in_gap(vals)
    while bad.any():
        vals[bad] = draw(bad)
        bad = in_gap(vals)
    lam = np.sort(vals)
    if forced_gap_at is not None and forced_gap > 0.0:
        i = int(forced_gap_at)
        d = lam[i] - lam[i - 1]
        if d < forced_gap:
            lam[i:] += forced_gap - d
    return lam, np.array(gaps)


def make_pencil(n, lam_fn, seed, scale=0.05, decay=5.0, meta=None) -> Pencil:
    """Build the pencil for spectrum generator ``lam_fn(rng, n)`` (returns ascending lam
    or (lam, extra))."""
    rng = np.random.default_rng(seed)
    L = _unit_lower(rng, n, scale, decay)
    Q = _haar(rng, n)
    got = lam_fn(rng, n)
    extra = None
    if isinstance(got, tuple):
        got, extra = got
    lam = np.sort(np.asarray(got, dtype=np.float64))
    M = (Q * lam[None, :]) @ Q.T
    A = L @ M @ L.T
    A = 0.5 * (A + A.T)
    B = L @ L.T
    B = 0.5 * (B + B.T)
    m = dict(meta or {})
    m.update(seed=seed, n=n)
    if extra is not None:
        m["gaps"] = extra
    return Pencil(np.ascontiguousarray(A), np.ascontiguousarray(B), lam, L, Q, m)


# ---------------------------------------------------------------- workloads

def pencil_clusters4(n=200, seed=0) -> Pencil:
    """N=200 plain workload: four Gaussian clusters in [-2, 2]."""
    return make_pencil(n, lambda r, m: spectrum_clusters4(r, m), seed,
                       meta=dict(workload="clusters4"))


def pencil_scf(n=4096, n_e=400, seed=0, **kw) -> Pencil:
    """SCF-shaped workload: 12 clusters + uniform background in [-5, 5], two gaps."""
    return make_pencil(n, lambda r, m: spectrum_scf(r, m, n_e, **kw), seed,
                       meta=dict(workload="scf", n_e=n_e))


def pencil_diag(a, b=None) -> Pencil:
    """Diagonal pencil (A = diag(a), B = diag(b) or I): eigenvalues a/b."""
    a = np.asarray(a, dtype=np.float64)
    n = a.size
    bb = np.ones(n) if b is None else np.asarray(b, dtype=np.float64)
    A = np.diag(a)
    B = np.diag(bb)
    lam = np.sort(a / bb)
    return Pencil(A, B, lam, np.diag(np.sqrt(bb)), np.eye(n), dict(workload="diag"))


def random_symmetric(n, seed, scale=1.0):
    """Dense random symmetric matrix with N(0, scale^2) entries (used for factor tests)."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((n, n)) * scale
    return np.ascontiguousarray(0.5 * (g + g.T))


def safe_shifts(lam, sigmas, rel_gap=1e-6, norm=None):
    """Move each shift so that min_i |sigma - lam_i| >= rel_gap * ||A||, so that the
    Sylvester count of A - sigma B is pinned by the known spectrum on both sides."""
    lam = np.sort(np.asarray(lam, dtype=np.float64))
    nrm = float(np.max(np.abs(lam))) if norm is None else float(norm)
    tol = rel_gap * max(nrm, 1e-300)
    out = []
    for s in np.asarray(sigmas, dtype=np.float64):
        s = float(s)
        for _ in range(64):
            i = np.searchsorted(lam, s)
            near = []
            if i < lam.size:
                near.append(lam[i])
            if i > 0:
                near.append(lam[i - 1])
            d = min(abs(s - x) for x in near) if near else np.inf
            if d >= tol:
                break
            # step to the midpoint of the surrounding gap that is wide enough
            lo = lam[i - 1] if i > 0 else s - 4 * tol
            hi = lam[i] if i < lam.size else s + 4 * tol
            if hi - lo > 2 * tol:
                s = 0.5 * (lo + hi)
            else:
                s = hi + 2 * tol
        out.append(s)
    return np.array(out)


def pencil_adjoint(n=2048, n_e=200, seed=0, gap=0.05) -> Pencil:
    """Adjoint workload: the SCF-shaped spectrum with lam_{n_e+1} - lam_{n_e} >= gap, so
    that the occupied subspace (the lowest n_e) is separated from the rest."""
    return make_pencil(n, lambda r, m: spectrum_scf(r, m, n_e, forced_gap_at=n_e, forced_gap=gap),
                       seed, meta=dict(workload="adjoint", n_e=n_e, gap=gap))


def sym_gaussian(n, seed):
    """W = (G + G^T) / sqrt(2) with G ~ N(0, 1) entries (the density-matrix weight)."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((n, n))
    return np.ascontiguousarray((g + g.T) / np.sqrt(2.0))


def sym_directions(n, k, seed):
    """k symmetric perturbation directions with N(0, 1) entries, each scaled to unit
    Frobenius norm (finite-difference checks of gradients); shape (k, n, n)."""
    rng = np.random.default_rng(seed)
    out = np.empty((k, n, n))
    for t in range(k):
        g = rng.standard_normal((n, n))
        e = 0.5 * (g + g.T)
        out[t] = e / np.linalg.norm(e)
    return out


def batched_sizes(count=64, seed=7):
    """Orders of the batched workload: N_p = 512 + 256 * U{0..10}, seeded; pencil p uses
    seed 1000 + p, n_e = N_p // 10 and the SCF-shaped spectrum scaled to N_p."""
    rng = np.random.default_rng(seed)
    return [int(512 + 256 * k) for k in rng.integers(0, 11, count)]


def make_pencil_device(n, lam_fn, seed, device, scale=0.05, decay=5.0):
    """The ``make_pencil`` construction with its Gaussian draws (L, Q) taken from torch's
    generator on ``device`` and the products formed there: the same recipe, shapes
    and spectrum (``lam_fn`` draws from numpy's generator), a different random stream.
    For large benchmark inputs that the host would take minutes to build.
    Returns (A, B, lam) with A, B float64 device tensors."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    f64 = dict(dtype=torch.float64, device=device)
    z = torch.randn((n, n), generator=g, **f64)
    i = torch.arange(n, **f64)
    L = torch.tril(z * scale * torch.exp(-(i[:, None] - i[None, :]).abs() / decay), -1)
    L += torch.eye(n, **f64)
    G = torch.randn((n, n), generator=g, **f64)
    Q, R = torch.linalg.qr(G)
    Q = Q * torch.sign(torch.diagonal(R))[None, :]
    got = lam_fn(np.random.default_rng(seed), n)
    lam = np.sort(np.asarray(got[0] if isinstance(got, tuple) else got, dtype=np.float64))
    M = (Q * torch.from_numpy(lam).to(device)[None, :]) @ Q.T
    A = L @ M @ L.T
    A = 0.5 * (A + A.T)
    B = L @ L.T
    B = 0.5 * (B + B.T)
    return A.contiguous(), B.contiguous(), lam


def sym_perturbation(n, seed, norm2=1e-3):
    """E = (G + G^T)/2 with G ~ N(0, 1) entries, scaled to ||E||_2 = norm2 (the SCF
    sequence's step A_k = A_{k-1} + E_k)."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((n, n))
    e = 0.5 * (g + g.T)
    return np.ascontiguousarray(e * (norm2 / np.max(np.abs(np.linalg.eigvalsh(e)))))


def sym_perturbation_device(n, seed, norm2, device, iters=60):
    """The same construction drawn from torch's generator on ``device``; ||E||_2 by
    power iteration (for orders where a dense eigensolve on the host is slow)."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    G = torch.randn((n, n), generator=g, dtype=torch.float64, device=device)
    E = 0.5 * (G + G.T)
    v = torch.randn(n, generator=g, dtype=torch.float64, device=device)
    lam = 0.0
    for _ in range(iters):
        w = E @ v
        lam = float(torch.linalg.norm(w))
        v = w / lam
    return (E * (norm2 / lam)).contiguous()


def sym_gaussian_device(n, seed, device):
    """W = (G + G^T) / sqrt(2) with G ~ N(0, 1) drawn from torch's generator on
    ``device`` (the density-matrix weight at orders the host builds slowly)."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    G = torch.randn((n, n), generator=g, dtype=torch.float64, device=device)
    return ((G + G.T) / np.sqrt(2.0)).contiguous()
