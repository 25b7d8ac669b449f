"""ctypes declarations of the C ABI in ``include/sislice.h`` (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libsislice.so")

c_double_p = C.POINTER(C.c_double)
c_int64_p = C.POINTER(C.c_int64)
c_int32_p = C.POINTER(C.c_int32)
c_void_pp = C.POINTER(C.c_void_p)

STATUS = {
    0: "ok", -1: "invalid argument", -2: "HIP runtime error", -3: "allocation failed",
    -4: "no gfx950 device", 1: "singular shift", 2: "not converged", 3: "missing eigenvalues",
}


class Opts(C.Structure):
    _fields_ = [("block", C.c_int32), ("max_basis", C.c_int32), ("max_cycles", C.c_int32),
                ("kpm_moments", C.c_int32), ("kpm_vectors", C.c_int32),
                ("bounds_steps", C.c_int32), ("nb", C.c_int32), ("profile", C.c_int32),
                ("tol", C.c_double), ("top_margin", C.c_double), ("seed", C.c_uint64),
                ("driver", C.c_int32), ("subspace_iters", C.c_int32), ("max_recovery", C.c_int32),
                ("graphs", C.c_int32)]


class Report(C.Structure):
    _fields_ = [("n_shifts", C.c_int64), ("n_validated", C.c_int64), ("n_converged", C.c_int64),
                ("nu_top", C.c_int64), ("omega_top", C.c_double), ("anorm", C.c_double),
                ("cycles_max", C.c_int32), ("block_steps", C.c_int32),
                ("t_factor_ms", C.c_double), ("t_lanczos_ms", C.c_double),
                ("t_rr_ms", C.c_double), ("t_host_ms", C.c_double), ("t_total_ms", C.c_double),
                ("flops_factor", C.c_double), ("nu", c_int64_p), ("slice_case", c_int32_p),
                ("slice_exact", c_int32_p), ("slice_cand", c_int32_p),
                ("t_kern_ms", C.c_double * 6), ("n_kern", C.c_int64 * 6), ("flops_update", C.c_double),
                ("bytes_solve", C.c_double), ("factor_id", C.c_uint64),
                ("probes_inserted", C.c_int32), ("recovery_rounds", C.c_int32),
                ("bytes_panel", C.c_double)]


class AdjointReport(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("reused_factors", C.c_int32), ("n_groups", C.c_int32),
                ("breakdowns", C.c_int32), ("max_rel_residual", C.c_double),
                ("t_factor_ms", C.c_double), ("t_solve_ms", C.c_double), ("t_total_ms", C.c_double),
                ("flops_outer", C.c_double), ("t_outer_ms", C.c_double)]


class ScfReport(C.Structure):
    _fields_ = [("step", C.c_int32), ("replanned", C.c_int32), ("merged", C.c_int32),
                ("deleted", C.c_int32), ("inserted", C.c_int32), ("status_solve", C.c_int32),
                ("eta_prev", C.c_double), ("eta_new", C.c_double), ("block_steps", C.c_int64),
                ("factor_id", C.c_uint64), ("t_solve_ms", C.c_double), ("t_total_ms", C.c_double),
                ("cycles_max", C.c_int32), ("probes_inserted", C.c_int32),
                ("t_factor_ms", C.c_double), ("flops_factor", C.c_double)]


class Problem(C.Structure):
    _fields_ = [("n", C.c_int64), ("A", C.c_void_p), ("lda", C.c_int64), ("B", C.c_void_p),
                ("ldb", C.c_int64), ("n_e", C.c_int64), ("n_s", C.c_int64), ("evals", C.c_void_p),
                ("evecs", C.c_void_p), ("ldx", C.c_int64), ("resid", C.c_void_p)]


class BatchReport(C.Structure):
    _fields_ = [("workers", C.c_int32), ("n_ok", C.c_int32), ("n_tuned", C.c_int32),
                ("n_converged", C.c_int64), ("t_total_ms", C.c_double), ("t_tune_ms", C.c_double),
                ("graph_replays", C.c_int64), ("graphs_built", C.c_int64)]


_SIGS = {
    "sislice_default_opts": (None, [C.POINTER(Opts)]),
    "sislice_status_string": (C.c_char_p, [C.c_int]),
    "sislice_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int, C.c_void_p]),
    "sislice_destroy": (C.c_int, [C.c_void_p]),
    "sislice_set_stream": (C.c_int, [C.c_void_p, C.c_void_p]),
    "sislice_set_wait_limit": (C.c_int, [C.c_void_p, C.c_int64]),
    "sislice_ldlt_factor": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p,
                                      C.c_int64, C.c_double, C.c_void_p, C.c_int64, C.c_void_p,
                                      c_int64_p]),
    "sislice_ldlt_factor_multi": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_int64,
                                            C.c_void_p, C.c_int64, C.c_int64, c_double_p,
                                            c_void_pp, C.c_int64, c_void_pp, c_int64_p]),
    "sislice_ldlt_solve": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p,
                                     C.c_int64, C.c_void_p, C.c_int64]),
    "sislice_ldlt_solve_noalloc": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_int64,
                                             C.c_void_p, C.c_int64, C.c_void_p, C.c_int64]),
    "sislice_plan_shifts_kpm": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_int64,
                                          C.c_void_p, C.c_int64, C.c_int64, C.c_int64,
                                          C.POINTER(Opts), c_double_p, c_double_p, c_double_p,
                                          c_double_p]),
    "sislice_plan_shifts_lanczos": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_int64,
                                              C.c_void_p, C.c_int64, C.c_int64, C.c_int64,
                                              C.POINTER(Opts), C.c_int32, C.c_int32, C.c_int32,
                                              c_double_p, c_double_p, c_double_p]),
    "sislice_solve": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p,
                                C.c_int64, C.c_int64, C.c_int64, c_double_p, c_double_p,
                                C.POINTER(Opts), C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p,
                                C.POINTER(Report)]),
    "sislice_sisubit": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p,
                                  C.c_int64, C.c_double, C.c_int64, C.c_void_p, C.c_int64,
                                  C.c_int32, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]),
    "sislice_adjoint": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p,
                                  C.c_int64, C.c_int64, C.c_void_p, C.c_void_p, C.c_int64,
                                  C.c_void_p, C.c_void_p, C.c_int64, C.c_int64, c_double_p,
                                  C.c_double, C.c_uint64, C.c_double, C.c_int32, C.c_void_p,
                                  C.c_int64, C.c_void_p, C.c_int64, C.POINTER(AdjointReport)]),
    "sislice_solve_batched": (C.c_int, [C.c_void_p, C.c_int64, C.POINTER(Problem), C.POINTER(Opts),
                                        C.c_int32, c_int32_p, C.POINTER(BatchReport)]),
    "sislice_tuned_nb": (C.c_int32, [C.c_void_p, C.c_int64]),
    "sislice_tuned_factor": (C.c_int32, [C.c_void_p, C.c_int64, c_int32_p, c_int32_p, c_int32_p]),
    "sislice_scf_create": (C.c_int, [C.c_void_p, C.c_int64, C.c_int64, C.c_int64, C.POINTER(Opts),
                                     C.c_double, C.POINTER(C.c_void_p)]),
    "sislice_scf_step": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_int64,
                                   C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, c_double_p,
                                   c_double_p, C.POINTER(ScfReport)]),
    "sislice_scf_destroy": (C.c_int, [C.c_void_p]),
    "sislice_kmeans_shifts": (C.c_int, [c_double_p, C.c_int64, c_double_p, C.c_int64, C.c_int32,
                                        C.c_uint64, c_double_p, c_int32_p]),
    "sislice_dos_plan": (C.c_int, [c_double_p, c_double_p, C.c_int32, C.c_int32, C.c_int64,
                                   C.c_int64, C.c_int64, C.c_int32, C.c_double, c_double_p,
                                   c_double_p]),
    "sislice_scf_migrate": (C.c_int, [c_double_p, c_int32_p, C.c_int64, c_double_p, C.c_int64,
                                      C.c_int32, C.c_uint64, c_double_p, c_int32_p, c_int32_p,
                                      c_int32_p, c_int32_p]),
    "sislice_validate": (C.c_int64, [C.c_int64, c_double_p, c_int64_p, C.c_double, C.c_int64,
                                     c_int64_p, c_int64_p, c_double_p, c_double_p, c_int32_p,
                                     c_int32_p, c_int32_p, c_int32_p]),
    "sislice_kpm_cdos": (C.c_double, [c_double_p, C.c_int32, C.c_double, C.c_double, C.c_int64,
                                      C.c_double]),
    "sislice_kpm_place": (C.c_int, [c_double_p, C.c_int32, C.c_double, C.c_double, C.c_int64,
                                    C.c_int64, C.c_int64, C.c_double, c_double_p, c_double_p]),
    "sislice_splitmix64": (C.c_uint64, [C.c_uint64, C.c_uint64]),
    "sislice_sym_eig_var": (C.c_int, [C.c_void_p, C.c_int32, c_int32_p, C.c_int32, C.c_void_p,
                                      C.c_int64, C.c_void_p, C.c_void_p]),
    "sislice_sym_eig": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_int64,
                                  C.c_void_p, C.c_void_p]),
}

EXPORTED = tuple(_SIGS)

_lib = None


def load():
    """Load the built library; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} (run python -m paper_1908_06043_amd.build)")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


class SisliceError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__(f"{where}: status {code} ({STATUS.get(code, 'unknown')})")
