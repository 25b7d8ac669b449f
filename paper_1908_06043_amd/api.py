"""Thin torch-facing binding of the HIP library (argument marshalling only).

Every computation happens in the library's gfx950 kernels; torch provides device
memory and the current HIP stream.  Matrices are passed as square float64 CUDA
tensors; the library reads them as column-major, i.e. it sees the transpose of
a row-major torch tensor, which for the symmetric A and B is the same matrix.
Column-major outputs are returned as views with mathematical indexing.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib
from ._lib import AdjointReport, BatchReport, Opts, Problem, Report, ScfReport, SisliceError

_handles = {}


def _require_gpu():
    if not torch.cuda.is_available():
        raise RuntimeError("paper_1908_06043_amd needs a ROCm GPU (gfx950); none is visible")


def handle(device=None):
    """Library handle for `device`, bound to torch's current stream on each call."""
    _require_gpu()
    lib = _lib.load()
    dev = torch.cuda.current_device() if device is None else int(device)
    h = _handles.get(dev)
    if h is None:
        hp = C.c_void_p()
        with torch.cuda.device(dev):
            st = lib.sislice_create(C.byref(hp), dev, C.c_void_p(torch.cuda.current_stream().cuda_stream))
        if st != 0:
            raise SisliceError(st, "sislice_create")
        h = hp.value
        _handles[dev] = h
    st = lib.sislice_set_stream(C.c_void_p(h), C.c_void_p(torch.cuda.current_stream(dev).cuda_stream))
    if st != 0:
        raise SisliceError(st, "sislice_set_stream")
    return C.c_void_p(h)


def set_wait_limit(polls, device=None):
    """Polls after which a device-side hand-off wait gives up (sislice_set_wait_limit)."""
    _check(_lib.load().sislice_set_wait_limit(handle(device), int(polls)), "sislice_set_wait_limit")


def _mat(M, name):
    if not (isinstance(M, torch.Tensor) and M.is_cuda and M.dtype == torch.float64 and M.dim() == 2
            and M.shape[0] == M.shape[1] and M.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous square float64 CUDA tensor")
    return M


def default_opts(**kw) -> Opts:
    o = Opts()
    _lib.load().sislice_default_opts(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def _check(st, where, ok=(0,)):
    if st not in ok:
        raise SisliceError(st, where)
    return st


@dataclass
class Factor:
    LDt: torch.Tensor      # (n, n): LDt[j, i] = LD(i, j) (column-major storage)
    ipiv: torch.Tensor     # int32 (n,)
    inertia: tuple
    status: int

    @property
    def LD(self):
        return self.LDt.t()


def ldlt_factor(A, B, sigma) -> Factor:
    """Bunch-Kaufman LDL^T of A - sigma B with the inertia of D."""
    return ldlt_factor_multi(A, B, [sigma])[0]


def ldlt_factor_multi(A, B, sigmas):
    A = _mat(A, "A")
    B = _mat(B, "B")
    n = A.shape[0]
    sig = np.ascontiguousarray(np.asarray(sigmas, dtype=np.float64).ravel())
    S = sig.size
    LDts = [torch.empty((n, n), dtype=torch.float64, device=A.device) for _ in range(S)]
    ipivs = [torch.empty(n, dtype=torch.int32, device=A.device) for _ in range(S)]
    ld_ptrs = (C.c_void_p * S)(*[t.data_ptr() for t in LDts])
    ip_ptrs = (C.c_void_p * S)(*[t.data_ptr() for t in ipivs])
    inert = np.zeros(3 * S, dtype=np.int64)
    lib = _lib.load()
    st = lib.sislice_ldlt_factor_multi(handle(A.device.index), n, A.data_ptr(), n, B.data_ptr(), n, S,
                                       sig.ctypes.data_as(_lib.c_double_p), ld_ptrs, n, ip_ptrs,
                                       inert.ctypes.data_as(_lib.c_int64_p))
    _check(st, "sislice_ldlt_factor_multi", ok=(0, 1))
    return [Factor(LDts[s], ipivs[s], tuple(int(x) for x in inert[3 * s:3 * s + 3]), st) for s in range(S)]


def ldlt_solve(f: Factor, X):
    """Returns C^{-1} X for X of shape (n, nrhs) (or (n,)) using the factors."""
    vec = X.dim() == 1
    Xc = (X[:, None] if vec else X).t().contiguous()   # (nrhs, n) = column-major n x nrhs
    n = f.LDt.shape[0]
    nrhs = Xc.shape[0]
    lib = _lib.load()
    st = lib.sislice_ldlt_solve(handle(X.device.index), n, f.LDt.data_ptr(), n, f.ipiv.data_ptr(),
                                nrhs, Xc.data_ptr(), n)
    _check(st, "sislice_ldlt_solve")
    out = Xc.t()
    return out[:, 0] if vec else out


def sym_eig(M):
    """Eigen-decomposition of a batch of small symmetric matrices (m <= 112)."""
    Mb = M if M.dim() == 3 else M[None]
    batch, m, _ = Mb.shape
    Ac = Mb.transpose(1, 2).contiguous()
    W = torch.empty((batch, m), dtype=torch.float64, device=M.device)
    V = torch.empty((batch, m, m), dtype=torch.float64, device=M.device)   # V[b, j, i] = vec j, comp i
    lib = _lib.load()
    st = lib.sislice_sym_eig(handle(M.device.index), m, batch, Ac.data_ptr(), m, W.data_ptr(), V.data_ptr())
    _check(st, "sislice_sym_eig")
    Vm = V.transpose(1, 2)
    return (W[0], Vm[0]) if M.dim() == 2 else (W, Vm)


def sym_eig_var(mats):
    """Eigen-decompositions of a batch of small symmetric matrices of different orders
    (a list of square tensors on one device, orders <= 112), in one launch.  Returns a
    list of (W, V) with W ascending and V[:, j] the eigenvector of W[j]."""
    orders = [int(x.shape[0]) for x in mats]
    batch, mmax = len(mats), max(orders) if mats else 0
    dev = mats[0].device
    Ap = torch.zeros((batch, mmax, mmax), dtype=torch.float64, device=dev)
    for b, x in enumerate(mats):
        Ap[b, :orders[b], :orders[b]] = x.t()   # column-major blocks: Ap[b, j, i] = A_b(i, j)
    W = torch.zeros((batch, mmax), dtype=torch.float64, device=dev)
    V = torch.zeros((batch, mmax, mmax), dtype=torch.float64, device=dev)   # V[b, j, i] = vec j, comp i
    m = np.ascontiguousarray(np.asarray(orders, dtype=np.int32))
    lib = _lib.load()
    st = lib.sislice_sym_eig_var(handle(dev.index), batch, m.ctypes.data_as(_lib.c_int32_p), mmax,
                                 Ap.data_ptr(), mmax, W.data_ptr(), V.data_ptr())
    _check(st, "sislice_sym_eig_var")
    return [(W[b, :orders[b]], V[b, :orders[b], :orders[b]].t()) for b in range(batch)]


def sisubit(A, B, sigma, V0, M):
    """The paper's Algorithm 2 from the start basis V0 (n x k): M shift-invert
    applications with CholeskyQR, then Rayleigh-Ritz.  Returns (evals, X, resid)."""
    A = _mat(A, "A")
    B = _mat(B, "B")
    n, k = V0.shape
    V0t = V0.t().contiguous()                      # column-major n x k
    ev = torch.empty(k, dtype=torch.float64, device=A.device)
    Xt = torch.empty((k, n), dtype=torch.float64, device=A.device)
    rs = torch.empty(k, dtype=torch.float64, device=A.device)
    st = _lib.load().sislice_sisubit(handle(A.device.index), n, A.data_ptr(), n, B.data_ptr(), n,
                                     float(sigma), k, V0t.data_ptr(), n, int(M), ev.data_ptr(),
                                     Xt.data_ptr(), n, rs.data_ptr())
    _check(st, "sislice_sisubit")
    return ev, Xt.t(), rs


def plan_shifts_kpm(A, B, n_e, n_s, opts=None):
    A = _mat(A, "A")
    B = _mat(B, "B")
    n = A.shape[0]
    o = opts or default_opts()
    sig = np.zeros(n_s)
    top = C.c_double()
    mom = np.zeros(o.kpm_moments)
    bnd = np.zeros(2)
    lib = _lib.load()
    st = lib.sislice_plan_shifts_kpm(handle(A.device.index), n, A.data_ptr(), n, B.data_ptr(), n,
                                     n_e, n_s, C.byref(o), sig.ctypes.data_as(_lib.c_double_p),
                                     C.byref(top), mom.ctypes.data_as(_lib.c_double_p),
                                     bnd.ctypes.data_as(_lib.c_double_p))
    _check(st, "sislice_plan_shifts_kpm")
    return dict(sigmas=sig, omega_top=top.value, mu=mom, a=bnd[0], b=bnd[1])


def plan_shifts_lanczos(A, B, n_e, n_s, mode=1, k=80, nv=8, opts=None):
    """The paper's Lanczos DOS shift selection (mode 0: equal-count roots, mode 1:
    DOSCluster with refinement and expectation shifts)."""
    A = _mat(A, "A")
    B = _mat(B, "B")
    n = A.shape[0]
    o = opts or default_opts()
    sig = np.zeros(n_s)
    top = C.c_double()
    bnd = np.zeros(2)
    st = _lib.load().sislice_plan_shifts_lanczos(handle(A.device.index), n, A.data_ptr(), n,
                                                B.data_ptr(), n, n_e, n_s, C.byref(o), mode, k, nv,
                                                sig.ctypes.data_as(_lib.c_double_p), C.byref(top),
                                                bnd.ctypes.data_as(_lib.c_double_p))
    _check(st, "sislice_plan_shifts_lanczos")
    return dict(sigmas=sig, omega_top=top.value, a=bnd[0], b=bnd[1])


def solve(A, B, n_e, n_s, sigmas=None, omega_top=None, opts=None, check=True):
    """Lowest n_e eigenpairs of (A, B).  Returns dict with evals, evecs (n x n_e view),
    resid, status and the report."""
    A = _mat(A, "A")
    B = _mat(B, "B")
    n = A.shape[0]
    o = opts or default_opts()
    ev = torch.empty(n_e, dtype=torch.float64, device=A.device)
    Xt = torch.empty((n_e, n), dtype=torch.float64, device=A.device)
    rs = torch.empty(n_e, dtype=torch.float64, device=A.device)
    rep = Report()
    nu = np.zeros(n_s, dtype=np.int64)
    sc = np.zeros(n_s + 1, dtype=np.int32)
    se = np.zeros(n_s + 1, dtype=np.int32)
    sd = np.zeros(n_s + 1, dtype=np.int32)
    rep.nu = nu.ctypes.data_as(_lib.c_int64_p)
    rep.slice_case = sc.ctypes.data_as(_lib.c_int32_p)
    rep.slice_exact = se.ctypes.data_as(_lib.c_int32_p)
    rep.slice_cand = sd.ctypes.data_as(_lib.c_int32_p)
    top = C.c_double(float(omega_top) if omega_top is not None else 0.0)
    if sigmas is not None:
        sig = np.ascontiguousarray(np.asarray(sigmas, dtype=np.float64))
        if sig.size != n_s:
            raise ValueError("len(sigmas) != n_s")
        sp = sig.ctypes.data_as(_lib.c_double_p)
        if omega_top is None:
            raise ValueError("omega_top is required with explicit shifts")
    else:
        sig = None
        sp = None
    lib = _lib.load()
    st = lib.sislice_solve(handle(A.device.index), n, A.data_ptr(), n, B.data_ptr(), n, n_e, n_s, sp,
                           C.byref(top), C.byref(o), ev.data_ptr(), Xt.data_ptr(), n, rs.data_ptr(),
                           C.byref(rep))
    if check:
        _check(st, "sislice_solve")
    skip = ("nu", "slice_case", "slice_exact", "slice_cand", "t_kern_ms", "n_kern")
    report = {f: getattr(rep, f) for f, _ in Report._fields_ if f not in skip}
    report["t_kern_ms"] = list(rep.t_kern_ms)
    report["n_kern"] = list(rep.n_kern)
    report.update(nu=nu, slice_case=sc, slice_exact=se, slice_cand=sd)
    return dict(evals=ev, evecs=Xt.t(), resid=rs, status=st, omega_top=top.value, report=report,
                sigmas=sig)


def adjoint(A, B, evals, evecs, g_evals, g_evecs, sigmas, omega_top, factor_id=0, tol=0.0,
            max_iter=0, check=True):
    """Symmetric gradients (G_A, G_B) of a loss with cotangents g_evals (n_e,) and
    g_evecs (n, n_e) of the eigenpairs (evals, evecs) returned by ``solve`` (either
    cotangent may be None).  Returns (G_A, G_B, report)."""
    A = _mat(A, "A")
    B = _mat(B, "B")
    n = A.shape[0]
    n_e = int(evals.shape[0])
    Xt = evecs.t().contiguous()                        # column-major n x n_e
    ge = g_evals.contiguous() if g_evals is not None else None
    gXt = g_evecs.t().contiguous() if g_evecs is not None else None
    sig = np.ascontiguousarray(np.asarray(sigmas, dtype=np.float64))
    GA = torch.empty((n, n), dtype=torch.float64, device=A.device)
    GB = torch.empty((n, n), dtype=torch.float64, device=A.device)
    rep = AdjointReport()
    lib = _lib.load()
    st = lib.sislice_adjoint(handle(A.device.index), n, A.data_ptr(), n, B.data_ptr(), n, n_e,
                             evals.contiguous().data_ptr(), Xt.data_ptr(), n,
                             ge.data_ptr() if ge is not None else None,
                             gXt.data_ptr() if gXt is not None else None, n, sig.size,
                             sig.ctypes.data_as(_lib.c_double_p), float(omega_top), int(factor_id),
                             float(tol), int(max_iter), GA.data_ptr(), n, GB.data_ptr(), n,
                             C.byref(rep))
    if check:
        _check(st, "sislice_adjoint")
    report = {f: getattr(rep, f) for f, _ in AdjointReport._fields_}
    report["status"] = st
    return GA, GB, report


def solve_batched(pencils, opts=None, workers=0, check=True):
    """Many independent pencils: ``pencils`` is a list of (A, B, n_e, n_s); each is
    planned and solved as by ``solve`` (shifts from KPM), several at a time on
    worker streams.  Returns (results, report): per pencil a dict with evals,
    evecs (n x n_e view), resid and status."""
    o = opts or default_opts()
    count = len(pencils)
    probs = (Problem * max(count, 1))()
    outs = []
    dev_index = None
    for i, (A, B, n_e, n_s) in enumerate(pencils):
        A = _mat(A, "A")
        B = _mat(B, "B")
        n = A.shape[0]
        dev_index = A.device.index
        ev = torch.empty(n_e, dtype=torch.float64, device=A.device)
        Xt = torch.empty((n_e, n), dtype=torch.float64, device=A.device)
        rs = torch.empty(n_e, dtype=torch.float64, device=A.device)
        probs[i] = Problem(n, A.data_ptr(), n, B.data_ptr(), n, n_e, n_s, ev.data_ptr(),
                           Xt.data_ptr(), n, rs.data_ptr())
        outs.append(dict(evals=ev, evecs=Xt.t(), resid=rs, _keep=(A, B, Xt)))
    status = np.zeros(max(count, 1), dtype=np.int32)
    rep = BatchReport()
    st = _lib.load().sislice_solve_batched(handle(dev_index), count, probs, C.byref(o), int(workers),
                                          status.ctypes.data_as(_lib.c_int32_p), C.byref(rep))
    if check:
        _check(st, "sislice_solve_batched")
    for i, d in enumerate(outs):
        d["status"] = int(status[i])
        d.pop("_keep")
    report = {f: getattr(rep, f) for f, _ in BatchReport._fields_}
    report["status"] = st
    return outs, report


class ScfSequence:
    """A sequence of pencils of order n (the SCF iteration): shifts planned by KPM
    on the first step and migrated afterwards, probes warm-started from the
    previous eigenvectors, the partial-trace monitor and the missing-eigenvalue
    fallback (sislice_scf_*)."""

    def __init__(self, n, n_e, n_s, opts=None, eta_tol=0.0, device=None):
        self.n, self.n_e, self.n_s = int(n), int(n_e), int(n_s)
        self._opts = opts or default_opts()
        self._dev = device
        p = C.c_void_p()
        _check(_lib.load().sislice_scf_create(handle(device), self.n, self.n_e, self.n_s,
                                              C.byref(self._opts), float(eta_tol), C.byref(p)),
               "sislice_scf_create")
        self._p = p

    def step(self, A, B, check=True):
        A = _mat(A, "A")
        B = _mat(B, "B")
        n, n_e = self.n, self.n_e
        ev = torch.empty(n_e, dtype=torch.float64, device=A.device)
        Xt = torch.empty((n_e, n), dtype=torch.float64, device=A.device)
        rs = torch.empty(n_e, dtype=torch.float64, device=A.device)
        sig = np.zeros(self.n_s)
        top = C.c_double()
        rep = ScfReport()
        handle(A.device.index)  # bind the current stream
        st = _lib.load().sislice_scf_step(self._p, A.data_ptr(), n, B.data_ptr(), n, ev.data_ptr(),
                                         Xt.data_ptr(), n, rs.data_ptr(),
                                         sig.ctypes.data_as(_lib.c_double_p), C.byref(top),
                                         C.byref(rep))
        if check:
            _check(st, "sislice_scf_step")
        report = {f: getattr(rep, f) for f, _ in ScfReport._fields_}
        return dict(evals=ev, evecs=Xt.t(), resid=rs, status=st, sigmas=sig, omega_top=top.value,
                    report=report)

    def close(self):
        if self._p is not None and self._p.value:
            _lib.load().sislice_scf_destroy(self._p)
        self._p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tuned_factor(n, device=None):
    """(nb, nbpiv, wide_min) the autotuner cached for order n, or None."""
    v = [C.c_int32(), C.c_int32(), C.c_int32()]
    ok = _lib.load().sislice_tuned_factor(handle(device), int(n), *[C.byref(x) for x in v])
    return tuple(int(x.value) for x in v) if ok else None


def tuned_nb(n, device=None):
    """Panel width the batch autotuner cached for order n (0: none yet)."""
    return int(_lib.load().sislice_tuned_nb(handle(device), int(n)))


class _PencilEig(torch.autograd.Function):
    """Lowest n_e eigenpairs of (A, B) with the library's adjoint as backward."""

    @staticmethod
    def forward(ctx, A, B, n_e, n_s, sigmas, omega_top, opts, adj_tol):
        out = solve(A.detach(), B.detach(), n_e, n_s, sigmas, omega_top, opts)
        evals = out["evals"]
        evecs = out["evecs"].contiguous()
        ctx.save_for_backward(A, B, evals, evecs)
        ctx.meta = (np.asarray(sigmas, dtype=np.float64), float(out["omega_top"]),
                    int(out["report"]["factor_id"]), adj_tol)
        return evals, evecs

    @staticmethod
    def backward(ctx, g_evals, g_evecs):
        A, B, evals, evecs = ctx.saved_tensors
        sig, top, fid, tol = ctx.meta
        GA, GB, rep = adjoint(A.detach(), B.detach(), evals, evecs, g_evals, g_evecs, sig, top,
                              fid, tol)
        global last_adjoint_report
        last_adjoint_report = rep
        return GA, GB, None, None, None, None, None, None


last_adjoint_report = None


def eigh_pencil(A, B, n_e, n_s, sigmas=None, omega_top=None, opts=None, adj_tol=0.0):
    """Differentiable lowest n_e eigenpairs (evals (n_e,), evecs (n, n_e)) of the
    symmetric-definite pencil (A, B).  Gradients w.r.t. A and B come back in the
    symmetric convention (dL = tr(G_A dA) + tr(G_B dB) for symmetric dA, dB).
    Shifts are planned with the KPM estimator when not given (the plan itself is
    piecewise constant and not differentiated)."""
    if sigmas is None:
        plan = plan_shifts_kpm(A.detach(), B.detach(), n_e, n_s, opts)
        sigmas, omega_top = plan["sigmas"], plan["omega_top"]
    return _PencilEig.apply(A, B, n_e, n_s, sigmas, omega_top, opts, adj_tol)


# ----------------------------------------------------------- host-only helpers

def kmeans_shifts(ritz, prev_shifts=None, n_s=None, use_kmeanspp=False, seed=0):
    x = np.ascontiguousarray(np.asarray(ritz, dtype=np.float64))
    k = len(prev_shifts) if prev_shifts is not None else int(n_s)
    prev = np.ascontiguousarray(np.asarray(prev_shifts if prev_shifts is not None else np.zeros(k), dtype=np.float64))
    out = np.zeros(k)
    lab = np.zeros(x.size, dtype=np.int32)
    st = _lib.load().sislice_kmeans_shifts(x.ctypes.data_as(_lib.c_double_p), x.size,
                                          prev.ctypes.data_as(_lib.c_double_p), k, int(use_kmeanspp),
                                          seed, out.ctypes.data_as(_lib.c_double_p),
                                          lab.ctypes.data_as(_lib.c_int32_p))
    _check(st, "sislice_kmeans_shifts")
    return out, lab


def dos_plan(theta, zeta2, n, n_e, n_s, mode=1, top_margin=2.0):
    """The paper's DOS shift selection from Lanczos Ritz data (host): theta and zeta2
    of shape (n_v, k).  mode 0: equal-count roots; mode 1: DOSCluster."""
    th = np.ascontiguousarray(np.asarray(theta, dtype=np.float64))
    z2 = np.ascontiguousarray(np.asarray(zeta2, dtype=np.float64))
    nv, k = th.shape
    sig = np.zeros(n_s)
    top = C.c_double()
    st = _lib.load().sislice_dos_plan(th.ctypes.data_as(_lib.c_double_p), z2.ctypes.data_as(_lib.c_double_p),
                                     k, nv, n, n_e, n_s, mode, top_margin,
                                     sig.ctypes.data_as(_lib.c_double_p), C.byref(top))
    _check(st, "sislice_dos_plan")
    return sig, top.value


def scf_migrate(ritz, probe_of, prev_shifts, use_kmeanspp=False, seed=0):
    """Probe migration between SCF steps (host): new shifts, the new probe each value
    seeds, the previous probe each new probe continues (-1: inserted) and the
    counts (merged, deleted, inserted)."""
    x = np.ascontiguousarray(np.asarray(ritz, dtype=np.float64))
    po = np.ascontiguousarray(np.asarray(probe_of, dtype=np.int32))
    prev = np.ascontiguousarray(np.asarray(prev_shifts, dtype=np.float64))
    k = prev.size
    sh = np.zeros(k)
    vp = np.zeros(x.size, dtype=np.int32)
    org = np.zeros(k, dtype=np.int32)
    nn = C.c_int32()
    stats = np.zeros(3, dtype=np.int32)
    st = _lib.load().sislice_scf_migrate(x.ctypes.data_as(_lib.c_double_p), po.ctypes.data_as(_lib.c_int32_p),
                                        x.size, prev.ctypes.data_as(_lib.c_double_p), k,
                                        int(use_kmeanspp), seed, sh.ctypes.data_as(_lib.c_double_p),
                                        vp.ctypes.data_as(_lib.c_int32_p), org.ctypes.data_as(_lib.c_int32_p),
                                        C.byref(nn), stats.ctypes.data_as(_lib.c_int32_p))
    _check(st, "sislice_scf_migrate")
    m = nn.value
    return dict(shifts=sh[:m], value_probe=vp, origin=org[:m], merged=int(stats[0]),
                deleted=int(stats[1]), inserted=int(stats[2]))


def validate(sigmas, nus, thetas, resids, omega_top, nu_top):
    sig = np.ascontiguousarray(np.asarray(sigmas, dtype=np.float64))
    ns = sig.size
    nu = np.ascontiguousarray(np.asarray(nus, dtype=np.int64))
    counts = np.array([len(t) for t in thetas], dtype=np.int64)
    offs = np.concatenate([[0], np.cumsum(counts)[:-1]]).astype(np.int64)
    th = np.ascontiguousarray(np.concatenate([np.asarray(t, dtype=np.float64) for t in thetas]) if counts.sum() else np.zeros(1))
    rs = np.ascontiguousarray(np.concatenate([np.asarray(r, dtype=np.float64) for r in resids]) if counts.sum() else np.zeros(1))
    sc = np.zeros(ns + 1, dtype=np.int32)
    se = np.zeros(ns + 1, dtype=np.int32)
    sd = np.zeros(ns + 1, dtype=np.int32)
    ch = np.zeros(max(int(counts.sum()), 1), dtype=np.int32)
    nv = _lib.load().sislice_validate(ns, sig.ctypes.data_as(_lib.c_double_p), nu.ctypes.data_as(_lib.c_int64_p),
                                      float(omega_top), int(nu_top), offs.ctypes.data_as(_lib.c_int64_p),
                                      counts.ctypes.data_as(_lib.c_int64_p), th.ctypes.data_as(_lib.c_double_p),
                                      rs.ctypes.data_as(_lib.c_double_p), sc.ctypes.data_as(_lib.c_int32_p),
                                      se.ctypes.data_as(_lib.c_int32_p), sd.ctypes.data_as(_lib.c_int32_p),
                                      ch.ctypes.data_as(_lib.c_int32_p))
    if nv < 0:
        raise SisliceError(int(nv), "sislice_validate")
    return dict(n_validated=int(nv), slice_case=sc, slice_exact=se, slice_cand=sd,
                chosen=ch[: int(counts.sum())], offsets=offs, counts=counts)


def kpm_cdos(mu, a, b, n, omega):
    mu = np.ascontiguousarray(np.asarray(mu, dtype=np.float64))
    return _lib.load().sislice_kpm_cdos(mu.ctypes.data_as(_lib.c_double_p), mu.size, a, b, n, omega)


def kpm_place(mu, a, b, n, n_e, n_s, top_margin=2.0):
    mu = np.ascontiguousarray(np.asarray(mu, dtype=np.float64))
    sig = np.zeros(n_s)
    top = C.c_double()
    st = _lib.load().sislice_kpm_place(mu.ctypes.data_as(_lib.c_double_p), mu.size, a, b, n, n_e, n_s,
                                       top_margin, sig.ctypes.data_as(_lib.c_double_p), C.byref(top))
    _check(st, "sislice_kpm_place")
    return sig, top.value


def splitmix64(seed, i):
    return int(_lib.load().sislice_splitmix64(seed, i))
