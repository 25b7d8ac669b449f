#!/usr/bin/env python3
"""Benchmark of the plain spectrum-slicing hot path on one MI355X.

One step = one pass of the whole per-pencil path on one synthetic SCF-shaped
pencil (N=4096, lowest n_e=400, 16 shifts, Lanczos block 8):
  KPM density-of-states shift placement (64 moments, 20 Rademacher vectors),
  shift-form + Bunch-Kaufman LDL^T + inertia of the 16 shifts and the top
  boundary, block shift-invert Lanczos, explicit Rayleigh-Ritz, residuals,
  slice validation, and k-means migration of the shifts from the validated
  eigenvalues.
The pencil is generated once (seeded) and is resident in HBM before timing.

The ``adjoint`` object reports the differentiated form on its own workload
(N=2048, n_e=200, 8 shifts): forward + backward eigenpairs/s against forward
only on the same pencil and GPU.  The ``batched`` object reports 64 pencils of
uneven order (512..3072) solved by the batch scheduler against the plain path
looping over the same pencils.

Prints one JSON line.  ``value`` = converged eigenpairs (validated, residual
<= 1e-10) per second.  ``roofline`` describes the dominant kernel class,
timed with HIP events on the library's stream over the timed steps.
``cpu_baseline`` times the CPU oracle on a bounded sample (see its ``sample``).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "converged eigenpairs/s at residual ≤1e-10 (FP64); batched & adjoint vs plain"
PEAK_FP64 = 78.6      # TFLOP/s, MI355X dense FP64 (vector and MFMA)
PEAK_HBM = 8000.0     # GB/s, MI355X HBM3E
KCLASS = ["bk_panel", "trailing_update_mfma", "triangular_solve", "gemm", "projected_eig", "other"]


def measured_traffic(kernel_class):
    """HBM bytes per launch of `kernel_class` from the committed counter summary
    (rocprofv3 FETCH_SIZE / WRITE_SIZE scaled by a copy kernel of known size), or None
    when no summary exists or the kernel's source has changed since it was taken."""
    import glob
    import hashlib
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*counters*.txt"))):
        for line in open(path):
            line = line.strip()
            if not line.startswith("{"):
                continue
            rec = json.loads(line)
            if rec.get("kernel_class") != kernel_class:
                continue
            src = os.path.join(ROOT, rec["source"])
            if not os.path.exists(src):
                return None
            sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
            return rec["traffic_bytes_per_launch"] if sha == rec.get("source_sha256") else None
    return None


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(P, sigmas, n_e, n_s, oracle_n=768, bk_steps=128):
    """The CPU oracle timed on the host cores.

    value: the oracle's whole plain path (its KPM planner, Bunch-Kaufman of every
    shift and of the top boundary, Algorithm 2 per probe until its window has
    converged, validation) measured end to end on the same pencil recipe at a size
    it finishes in about half a minute: N=768, n_e=75, 3 shifts, so 25 wanted
    values per slice as in the N=4096 workload (400 over 16 shifts).
    extras: a dense LAPACK solve of the N=4096 workload's lowest n_e pairs
    (scipy.linalg.eigh on the pencil, subset by index), and the oracle's
    Bunch-Kaufman on the first columns of one N=4096 shifted matrix extrapolated
    by flop count to the n_s + 1 factorizations of a step."""
    import numpy as np
    import scipy.linalg as sla
    from oracle import bk, kpm, sislice as osl
    from paper_1908_06043_amd import inputs
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    ne_o, ns_o = oracle_n * n_e // P.n, max(1, oracle_n * n_s // P.n)
    Po = inputs.pencil_scf(oracle_n, ne_o, seed=0)
    t0 = time.perf_counter()
    pl = kpm.plan(Po.A, Po.B, ne_o, ns_o, M=64, nv=20, seed=0)
    r = osl.solve(Po.A, Po.B, ne_o, pl["sigmas"], pl["omega_top"], seed=0)
    t_or = time.perf_counter() - t0
    ok = r["status"] == 0 and np.max(np.abs(r["evals"] - Po.lam[:ne_o])) <= 1e-10 * r["anorm"]
    conv = int(np.sum(r["resid"] <= 1e-10)) if ok else 0
    t0 = time.perf_counter()
    w = sla.eigh(P.A, P.B, subset_by_index=[0, n_e - 1], eigvals_only=False)[0]
    t_dense = time.perf_counter() - t0
    dense_err = float(np.max(np.abs(w - P.lam[:n_e])))
    n = P.n
    C = bk.shifted(P.A, P.B, float(sigmas[len(sigmas) // 2]))
    t0 = time.perf_counter()
    f = bk.bk_ldlt(C, max_steps=bk_steps)
    dt = time.perf_counter() - t0
    k = f["k"]
    frac = 1.0 - ((n - k) / n) ** 3            # share of the n^3/3 flops done by k columns
    t_bk_step = (n_s + 1) * dt / frac
    return {
        "value": conv / t_or, "unit": "eigenpairs/s", "cores": int(threads), "kind": "oracle",
        "cpu_model": cpu_model(), "logical_cpus": os.cpu_count(),
        "sample": (f"oracle plain path end to end (KPM plan, Bunch-Kaufman of {ns_o} shifts + top "
                   f"boundary, Algorithm 2 per probe, validation) on the same pencil recipe at "
                   f"N={oracle_n}, n_e={ne_o}, {ns_o} shifts (25 values per slice as at N={n}): "
                   f"{t_or:.1f} s for {conv} converged eigenpairs, Algorithm 2 rounds per probe "
                   f"{list(r['rounds'])}"),
        "extras": {
            "dense_lapack_eigh": {
                "value": n_e / t_dense, "unit": "eigenpairs/s", "seconds": t_dense,
                "max_abs_error_vs_construction": dense_err,
                "what": (f"scipy.linalg.eigh(A, B, subset_by_index=[0, {n_e - 1}]) on the N={n} "
                         f"workload pencil (LAPACK, not the oracle)")},
            "oracle_bk_extrapolated": {
                "value": n_e / t_bk_step, "unit": "eigenpairs/s",
                "what": (f"oracle Bunch-Kaufman, first {k} of {n} pivot columns of one shifted "
                         f"matrix: {dt:.1f} s = {100 * frac:.1f}% of its n^3/3 flops, extrapolated "
                         f"to {n_s + 1} factorizations ({t_bk_step:.0f} s) per {n_e} eigenpairs; "
                         f"no Algorithm 2 counted")},
        },
    }


def adjoint_leg(api, inputs, torch, steps=3, warmup=1):
    """Adjoint workload (N=2048, n_e=200, 8 KPM shifts): forward only (plan + solve)
    against forward + backward (plan + solve + the gradient of
    L = sum lam^2 + tr(W X X^T) with respect to A and B) on the same pencil."""
    import numpy as np
    n, n_e, n_s = 2048, 200, 8
    P = inputs.pencil_adjoint(n, n_e, 0)
    W = inputs.sym_gaussian(n, 1)
    A = torch.from_numpy(P.A).cuda()
    B = torch.from_numpy(P.B).cuda()
    Wd = torch.from_numpy(W).cuda()
    opts = api.default_opts()

    def fwd():
        plan = api.plan_shifts_kpm(A, B, n_e, n_s, opts)
        out = api.solve(A, B, n_e, n_s, sigmas=plan["sigmas"], omega_top=plan["omega_top"],
                        opts=opts, check=False)
        conv = int(out["report"]["n_converged"]) if out["status"] in (0, 2) else 0
        return plan, out, conv

    def fwd_bwd():
        plan, out, conv = fwd()
        lam, X = out["evals"], out["evecs"]
        GA, GB, rep = api.adjoint(A, B, lam, X, 2.0 * lam, 2.0 * (Wd @ X), plan["sigmas"],
                                  out["omega_top"], out["report"]["factor_id"], check=False)
        return rep, (conv if rep["status"] == 0 else 0)

    res = {}
    for name, fn in (("forward", fwd), ("forward_backward", fwd_bwd)):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        conv, reps = 0, []
        for _ in range(steps):
            r = fn()
            conv += r[-1]
            reps.append(r[0])
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        res[name] = (conv / dt, 1e3 * dt / steps, reps)
    reps = res["forward_backward"][2]
    outer_tf = float(np.mean([r["flops_outer"] / (r["t_outer_ms"] * 1e-3) / 1e12 for r in reps]))
    return {
        "workload": f"adjoint: pencil N={n} (SCF-shaped, gap >= 0.05 above lambda_{n_e}), lowest "
                    f"n_e={n_e}, {n_s} KPM shifts; loss sum lam^2 + tr(W X X^T), W = (G+G^T)/sqrt(2)",
        "value": res["forward_backward"][0], "plain_value": res["forward"][0],
        "unit": "eigenpairs/s", "ratio_vs_plain": res["forward_backward"][0] / res["forward"][0],
        "ms_forward": res["forward"][1], "ms_forward_backward": res["forward_backward"][1],
        "cg_iterations": int(np.mean([r["iterations"] for r in reps])),
        "reused_factors": int(min(r["reused_factors"] for r in reps)),
        "outer_product_tflops": outer_tf, "steps": steps, "warmup": warmup,
    }


def batched_leg(api, inputs, torch, workers=8, reps=2):
    """Batched workload (64 pencils, N = 512 + 256 U{0..10}, n_e = N/10, 8 KPM shifts
    each): the plain path looping over the pencils against sislice_solve_batched on
    the same pencils and GPU.  The first batched call (autotuning and worker
    workspaces) is untimed warm-up."""
    sizes = inputs.batched_sizes(64, 7)
    pens = []
    for p, n in enumerate(sizes):
        A, B, _ = inputs.make_pencil_device(
            n, lambda r, m, k=n // 10: inputs.spectrum_scf(r, m, k), 1000 + p, "cuda")
        pens.append((A, B, n // 10, 8))
    opts = api.default_opts()
    big = max(range(len(sizes)), key=lambda i: sizes[i])
    api.solve(*pens[big], opts=opts, check=False)          # plain warm-up at the largest order
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    conv_plain = 0
    for A, B, ne, ns in pens:
        o = api.solve(A, B, ne, ns, opts=opts, check=False)
        conv_plain += int(o["report"]["n_converged"]) if o["status"] in (0, 2) else 0
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    _, rep0 = api.solve_batched(pens, opts=opts, workers=workers, check=False)  # tunes, captures
    _, _ = api.solve_batched(pens, opts=api.default_opts(graphs=0), workers=workers, check=False)

    def timed(o):
        best = None
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            outs, rep = api.solve_batched(pens, opts=o, workers=workers, check=False)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            if best is None or dt < best[0]:
                best = (dt, rep)
        return best

    dt, rep = timed(opts)
    dt_ng, rep_ng = timed(api.default_opts(graphs=0))
    return {
        "workload": f"batched: {len(sizes)} pencils, N = 512 + 256 U{{0..10}} (sum N = {sum(sizes)}), "
                    f"n_e = N/10, 8 KPM shifts each, SCF-shaped spectra",
        "value": rep["n_converged"] / dt, "plain_value": conv_plain / t_plain, "unit": "eigenpairs/s",
        "ratio_vs_plain": (rep["n_converged"] / dt) / (conv_plain / t_plain),
        "ms_batched": 1e3 * dt, "ms_plain_loop": 1e3 * t_plain, "workers": rep["workers"],
        "graph_replays": rep["graph_replays"],
        "no_graphs": {"value": rep_ng["n_converged"] / dt_ng, "ms_batched": 1e3 * dt_ng},
        "pencils_ok": rep["n_ok"], "tune_ms_first_call": rep0["t_tune_ms"],
        "graphs_built_first_call": rep0["graphs_built"],
        "tuned": {str(n): api.tuned_factor(n) for n in sorted(set(sizes))},
    }


def driver_leg(api, torch, A, B, n_e, n_s, steps=2):
    """The plain workload with the paper's per-probe iteration (Algorithm 2, shift-invert
    subspace iteration, opts.driver = 1) in place of block Lanczos: same KPM shifts."""
    opts = api.default_opts(driver=1)
    plan = api.plan_shifts_kpm(A, B, n_e, n_s, opts)
    api.solve(A, B, n_e, n_s, sigmas=plan["sigmas"], omega_top=plan["omega_top"], opts=opts, check=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    conv = 0
    rep = None
    for _ in range(steps):
        plan = api.plan_shifts_kpm(A, B, n_e, n_s, opts)
        o = api.solve(A, B, n_e, n_s, sigmas=plan["sigmas"], omega_top=plan["omega_top"], opts=opts,
                      check=False)
        conv += int(o["report"]["n_converged"]) if o["status"] in (0, 2) else 0
        rep = o["report"]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"value": conv / dt, "unit": "eigenpairs/s", "ms_per_step": 1e3 * dt / steps,
            "status": o["status"], "rounds_max": int(rep["cycles_max"]),
            "applications": int(rep["block_steps"]),
            "ms_iteration": float(rep["t_lanczos_ms"]), "ms_factor": float(rep["t_factor_ms"])}


def planner_leg(api, A, B, n_e, n_s, reps=2):
    """On the plain workload: shifts from the KPM planner against the paper's Lanczos DOS
    planner (equal-count roots; DOSCluster), each followed by the solve."""
    import torch
    out = {}
    opts = api.default_opts()
    for name in ("kpm", "lanczos_cdos", "lanczos_cluster"):
        best = None
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if name == "kpm":
                pl = api.plan_shifts_kpm(A, B, n_e, n_s, opts)
            else:
                pl = api.plan_shifts_lanczos(A, B, n_e, n_s, mode=0 if name == "lanczos_cdos" else 1)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            o = api.solve(A, B, n_e, n_s, sigmas=pl["sigmas"], omega_top=pl["omega_top"], opts=opts,
                          check=False)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            conv = int(o["report"]["n_converged"]) if o["status"] in (0, 2) else 0
            rec = {"eigenpairs_per_s": conv / (t2 - t0), "plan_ms": 1e3 * (t1 - t0),
                   "solve_ms": 1e3 * (t2 - t1), "status": o["status"],
                   "block_steps": int(o["report"]["block_steps"]),
                   "cycles_max": int(o["report"]["cycles_max"])}
            if best is None or rec["eigenpairs_per_s"] > best["eigenpairs_per_s"]:
                best = rec
        out[name] = best
    return out


def factor_leg(api, inputs, torch, n=12288, n_s=48, reps=3, cache=None):
    """The lock-step Bunch-Kaufman factorization alone at the SCF size: the pencil of
    the SCF sequence (n_e = n/10.24), its n_s KPM shifts and the top boundary, i.e.
    n_s + 1 factorizations of order n per call (shift-form, LDL^T, inertia; the
    factors go to caller-owned buffers).  Rate = (n_s + 1) n^3/3 flops over the mean
    of `reps` calls after one untimed call; the inertias are compared with the
    construction's eigenvalue counts.  `cache` (a directory) keeps the pencil as .npy
    files: a run that finds them loads them instead of building the pencil (a run
    under a counter-collecting profiler then avoids the construction's library
    calls)."""
    import numpy as np
    n_e = n * 1200 // 12288
    names = [os.path.join(cache, f"pencil{n}_{x}.npy") for x in ("A", "B", "lam")] if cache else []
    if names and all(os.path.exists(f) for f in names):
        A = torch.from_numpy(np.load(names[0])).cuda()
        B = torch.from_numpy(np.load(names[1])).cuda()
        lam = np.load(names[2])
    else:
        A, B, lam = inputs.make_pencil_device(
            n, lambda r, m: inputs.spectrum_scf(r, m, n_e, forced_gap_at=n_e, forced_gap=0.05), 0, "cuda")
        if names:
            os.makedirs(cache, exist_ok=True)
            for f, x in zip(names, (A.cpu().numpy(), B.cpu().numpy(), lam)):
                np.save(f, x)
    plan = api.plan_shifts_kpm(A, B, n_e, n_s)
    pts = [float(x) for x in plan["sigmas"]] + [float(plan["omega_top"])]
    times = []
    ok = True
    for r in range(reps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fs = api.ldlt_factor_multi(A, B, pts)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        ok = ok and all(f.inertia[0] == int(np.sum(lam < p)) for f, p in zip(fs, pts))
        del fs
    ms = 1e3 * float(np.mean(times[1:]))
    flops = len(pts) * float(n) ** 3 / 3.0
    return {"workload": f"{len(pts)} factorizations of order {n} (SCF pencil, {n_s} KPM shifts + top boundary)",
            "ms": ms, "tflops": flops / (ms * 1e-3) / 1e12, "frac_fp64_peak": flops / (ms * 1e-3) / 1e12 / PEAK_FP64,
            "inertia_matches_construction": bool(ok), "reps": reps}


def scf_leg(api, inputs, torch, n=12288, n_e=1200, n_s=48, steps=10, driver=0, gradient=True):
    """SCF-shaped sequence A_k = A_{k-1} + E_k (||E_k||_2 = 1e-3, B fixed; the spectrum with
    a gap of 0.05 above lambda_{n_e} so that the density loss is defined): every step
    solved by the SCF driver (migrated shifts, warm starts) with the gradient of
    sum lam^2 + tr(W X X^T); step 0 (KPM shifts, cold starts) is the plain reference."""
    import numpy as np
    A, B, _ = inputs.make_pencil_device(
        n, lambda r, m: inputs.spectrum_scf(r, m, n_e, forced_gap_at=n_e, forced_gap=0.05), 0, "cuda")
    W = inputs.sym_gaussian_device(n, 77, "cuda")
    seq = api.ScfSequence(n, n_e, n_s, opts=api.default_opts(driver=driver))
    recs = []
    t_all = 0.0
    conv_all = 0
    for k in range(steps):
        if k:
            A = A + inputs.sym_perturbation_device(n, 1000 + k, 1e-3, "cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = seq.step(A, B, check=False)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        lam, X = out["evals"], out["evecs"]
        if gradient:
            GA, GB, rep = api.adjoint(A, B, lam, X, 2.0 * lam, 2.0 * (W @ X), out["sigmas"],
                                      out["omega_top"], out["report"]["factor_id"], check=False)
        else:
            GA = GB = None
            rep = {"status": None, "iterations": 0}
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        # pairs that meet the tolerance, as the plain metric counts them
        conv = int((out["resid"] <= 1e-10).sum().item()) if out["status"] in (0, 2) else 0
        r = out["report"]
        recs.append({"ms_solve": 1e3 * (t1 - t0), "ms_gradient": 1e3 * (t2 - t1),
                     "ms_factor": float(r["t_factor_ms"]),
                     "factor_tflops": float(r["flops_factor"]) / max(float(r["t_factor_ms"]), 1e-9) / 1e9,
                     "status": out["status"], "replanned": int(r["replanned"]),
                     "block_steps": int(r["block_steps"]), "cycles_max": int(r["cycles_max"]),
                     "merged_deleted_inserted": [int(r["merged"]), int(r["deleted"]), int(r["inserted"])],
                     "converged": conv,
                     "gradient_status": rep["status"], "cg_iterations": rep["iterations"]})
        t_all += t2 - t0
        conv_all += conv
        print(f"scf step {k}: solve {recs[-1]['ms_solve']:.0f} ms gradient {recs[-1]['ms_gradient']:.0f} ms "
              f"status {out['status']}/{rep['status']} replanned {r['replanned']}", file=sys.stderr,
              flush=True)
        del GA, GB
    seq.close()
    warm = [x["ms_solve"] for x in recs[1:] if x["replanned"] == 0]
    return {
        "workload": f"SCF sequence: {steps} pencils N={n}, n_e={n_e}, {n_s} shifts, ||E_k||_2=1e-3, "
                    f"per-step gradient of sum lam^2 + tr(W X X^T); per-probe iteration: "
                    + ("block Lanczos" if driver == 0 else "subspace iteration (Algorithm 2), M=4"),
        "value": conv_all / t_all, "unit": "eigenpairs/s" + (" (with gradients)" if gradient else ""),
        "plain_step_ms": recs[0]["ms_solve"],
        "warm_step_ms_mean": float(np.mean(warm)) if warm else None,
        "factor_tflops": (sum(x["ms_factor"] * x["factor_tflops"] for x in recs)
                          / max(sum(x["ms_factor"] for x in recs), 1e-9)),
        "steps": recs,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--ne", type=int, default=400)
    ap.add_argument("--ns", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint-vs-plain leg")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-vs-plain leg")
    ap.add_argument("--no-planners", action="store_true", help="skip the planner comparison")
    ap.add_argument("--no-scf", action="store_true", help="skip the SCF-sequence leg")
    ap.add_argument("--scf-n", type=int, default=12288)
    ap.add_argument("--factor-only", action="store_true",
                    help="time only the lock-step factorization at the SCF size (--scf-n, 48 shifts + "
                         "the top boundary) and print its own JSON line")
    ap.add_argument("--pencil-cache", default=None,
                    help="with --factor-only: directory where the pencil is saved on the first run "
                         "and loaded from on later runs")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="after the steps, fill a 2 GiB buffer and copy it with one elementwise kernel "
                         "(reads and writes 2 GiB, beyond the last-level cache): the reference that "
                         "scales the FETCH_SIZE / WRITE_SIZE counters to bytes")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(the shifts of a pencil are the unit of work on one MI355X)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_1908_06043_amd import api, inputs

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        return 2
    if args.factor_only:
        ns = max(8, 48 * args.scf_n // 12288)
        print(json.dumps({"factor": factor_leg(api, inputs, torch, n=args.scf_n, n_s=ns,
                                               cache=args.pencil_cache)}), flush=True)
        return 0
    n, n_e, n_s = args.n, args.ne, args.ns
    P = inputs.pencil_scf(n, n_e, seed=0)
    A = torch.from_numpy(P.A).cuda()
    B = torch.from_numpy(P.B).cuda()
    # The last warm-up step times every kernel class with HIP events: the per-class
    # breakdown, and the dominant class.  The timed steps time that class alone, so
    # the events cost a few per step instead of two per launch of every class.
    opts_all = api.default_opts(profile=1)
    opts_off = api.default_opts(profile=0)
    state = {"prev": None}

    def step(opts):
        plan = api.plan_shifts_kpm(A, B, n_e, n_s, opts)
        out = api.solve(A, B, n_e, n_s, sigmas=plan["sigmas"], omega_top=plan["omega_top"],
                        opts=opts, check=False)
        ev = out["evals"].cpu().numpy()
        conv = int(out["report"]["n_converged"]) if out["status"] in (0, 2) else 0
        new, _ = api.kmeans_shifts(ev, plan["sigmas"], use_kmeanspp=state["prev"] is None, seed=0)
        state["prev"] = new
        return out, conv

    brk = None
    for w in range(args.warmup):
        out, _ = step(opts_all if w == args.warmup - 1 else opts_off)
        brk = out["report"]
    if brk is not None:
        dom = int(np.argmax(np.asarray(brk["t_kern_ms"])[:5]))
        opts_t = api.default_opts(profile=0x100 | (1 << dom))
    else:
        opts_t = opts_all
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = []
    conv_total = 0
    for _ in range(args.steps):
        out, conv = step(opts_t)
        reps.append(out["report"])
        conv_total += conv
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_step = 1e3 * dt / args.steps
    value = conv_total / dt

    tk = np.sum([r["t_kern_ms"] for r in reps], axis=0)
    nk = np.sum([r["n_kern"] for r in reps], axis=0)
    fl_up = float(np.sum([r["flops_update"] for r in reps]))
    if brk is None:
        dom = int(np.argmax(tk[:5]))
    if dom == 1:
        achieved = fl_up / (tk[1] * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP64, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP64, "traffic": None}
    elif dom == 2:
        # a sweep pair reads the packed L once per direction: 8 n^2 bytes per active shift
        # (the library counts the shifts each launch really carried)
        by = float(np.sum([r["bytes_solve"] for r in reps]))
        achieved = by / (tk[2] * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM, "unit": "GB/s",
                "frac": achieved / PEAK_HBM, "traffic": None,
                "algorithmic_bytes_per_launch": by / max(nk[2], 1)}
    elif dom == 0:
        # a panel step (one timed ticket) reads and writes the (n - k0) x kb panel block
        # of every shift (the library counts the blocks from the panel starts)
        by = float(np.sum([r["bytes_panel"] for r in reps]))
        achieved = by / (tk[0] * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM, "unit": "GB/s",
                "frac": achieved / PEAK_HBM, "traffic": None,
                "algorithmic_bytes_per_launch": by / max(nk[0], 1)}
    else:
        roof = {"bound": "mfma", "achieved": None, "peak": PEAK_FP64, "unit": "TFLOP/s",
                "frac": None, "traffic": None}
    roof["kernel"] = KCLASS[dom]
    roof["traffic"] = measured_traffic(KCLASS[dom])
    # per-class figures: the fully timed warm-up step (the timed steps time one class)
    tk_all = np.asarray(brk["t_kern_ms"]) if brk is not None else tk / args.steps
    nk_all = np.asarray(brk["n_kern"]) if brk is not None else nk // args.steps
    roof["kernel_ms_per_step"] = {KCLASS[q]: round(float(tk_all[q]), 3) for q in range(6)}
    roof["launches_per_step"] = {KCLASS[q]: int(nk_all[q]) for q in range(6)}
    roof["timed_classes"] = [KCLASS[dom]] if brk is not None else list(KCLASS)
    # the other rooflines, from the fully timed warm-up step (one step, every class)
    by_class = {}
    if brk is not None:
        tb = np.asarray(brk["t_kern_ms"])
        if tb[2] > 0:
            a = float(brk["bytes_solve"]) / (tb[2] * 1e-3) / 1e9
            by_class["triangular_solve"] = {"bound": "hbm", "achieved": a, "peak": PEAK_HBM,
                                            "unit": "GB/s", "frac": a / PEAK_HBM}
        if tb[1] > 0:
            a = float(brk["flops_update"]) / (tb[1] * 1e-3) / 1e12
            by_class["trailing_update_mfma"] = {"bound": "mfma", "achieved": a, "peak": PEAK_FP64,
                                                "unit": "TFLOP/s", "frac": a / PEAK_FP64}
    roof["by_class_warmup_step"] = by_class
    factor_tf = float(np.mean([r["flops_factor"] / (r["t_factor_ms"] * 1e-3) / 1e12 for r in reps]))
    line = {
        "metric": METRIC, "value": value, "unit": "eigenpairs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"plain SISLICE, SCF-shaped pencil N={n} (12 Gaussian clusters + "
                               f"uniform background on [-5,5], two gaps), lowest n_e={n_e}, "
                               f"{n_s} KPM shifts (64 moments, 20 Rademacher), Lanczos block 8",
                   "n": n, "n_e": n_e, "n_shifts": n_s, "global_batch": 1,
                   "parallelism": "shifts concurrent on one GPU"},
        "breakdown_ms": {
            "factor": float(np.mean([r["t_factor_ms"] for r in reps])),
            "lanczos": float(np.mean([r["t_lanczos_ms"] for r in reps])),
            "rayleigh_ritz": float(np.mean([r["t_rr_ms"] for r in reps])),
            "solve_total": float(np.mean([r["t_total_ms"] for r in reps])),
        },
        "factor_tflops": factor_tf,
        "converged_per_step": conv_total / args.steps,
        "roofline": roof,
    }
    if not args.no_adjoint:
        line["adjoint"] = adjoint_leg(api, inputs, torch)
    if not args.no_batched:
        line["batched"] = batched_leg(api, inputs, torch)
    if not args.no_planners:
        line["planners"] = planner_leg(api, A, B, n_e, n_s)
        line["subspace_driver"] = driver_leg(api, torch, A, B, n_e, n_s)
    if not args.no_scf:
        ns = max(8, 48 * args.scf_n // 12288)
        line["scf"] = scf_leg(api, inputs, torch, n=args.scf_n, n_e=args.scf_n * 1200 // 12288, n_s=ns)
        line["scf_subspace"] = scf_leg(api, inputs, torch, n=args.scf_n, n_e=args.scf_n * 1200 // 12288,
                                       n_s=ns, steps=2, driver=1, gradient=False)
    if args.calibrate_copy:
        src = torch.empty(256 << 20, dtype=torch.float64, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        # the same copy timed: the read + write bandwidth that a streaming kernel gets
        t0 = time.perf_counter()
        for _ in range(5):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / 5
        line["calibration_copy_bytes"] = {"read": src.numel() * 8, "written": dst.numel() * 8,
                                          "read_plus_write_GBps": 2 * src.numel() * 8 / dt / 1e9}
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(P, state["prev"], n_e, n_s)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
