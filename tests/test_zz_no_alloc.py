"""The allocation-free solve (sislice_ldlt_solve_noalloc) against the solve that
allocates its workspace (sislice_ldlt_solve), both called through the C ABI on
the same factors: the same kernels in the same order give bit-identical results.
Two calls in a row, the second with a smaller order and fewer right-hand sides,
check that the scratch array's contents from the first call do not leak into the
second; a third call above the array's maximum order is refused."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_1908_06043_amd import _lib, api, inputs

pytestmark = pytest.mark.gpu


def _call(name, f, Y):
    lib = _lib.load()
    n, nrhs = Y.shape
    Xc = torch.from_numpy(np.ascontiguousarray(Y.T)).cuda()   # column-major n x nrhs
    st = getattr(lib, name)(api.handle(0), n, f.LDt.data_ptr(), n, f.ipiv.data_ptr(), nrhs,
                            Xc.data_ptr(), n)
    torch.cuda.synchronize()
    return st, Xc.cpu().numpy().T


def _factor(n, seed):
    C_ = inputs.random_symmetric(n, seed)
    A = torch.from_numpy(C_).cuda()
    B = torch.eye(n, dtype=torch.float64, device="cuda")
    return C_, api.ldlt_factor(A, B, 0.0)


@pytest.mark.parametrize("first,second", [((4096, 40, 11), (1000, 8, 12)),
                                          ((2500, 64, 13), (333, 5, 14))])
def test_noalloc_solve_matches_allocating_solve(gpu_lib, first, second):
    for n, nrhs, seed in (first, second):
        print(f"no-alloc solve: n={n} nrhs={nrhs} seed={seed}", flush=True)
        C_, f = _factor(n, seed)
        Y = np.random.default_rng(seed).standard_normal((n, nrhs))
        st0, X0 = _call("sislice_ldlt_solve", f, Y)
        st1, X1 = _call("sislice_ldlt_solve_noalloc", f, Y)
        assert st0 == 0 and st1 == 0
        assert np.array_equal(X0, X1)
        r = np.linalg.norm(C_ @ X1 - Y) / (np.linalg.norm(C_) * np.linalg.norm(X1))
        assert r < 1e-13


def test_noalloc_solve_refuses_orders_beyond_its_array(gpu_lib):
    n = 4097
    lib = _lib.load()
    LD = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    ipiv = torch.zeros(n, dtype=torch.int32, device="cuda")
    X = torch.zeros((1, n), dtype=torch.float64, device="cuda")
    st = lib.sislice_ldlt_solve_noalloc(api.handle(0), n, LD.data_ptr(), n, ipiv.data_ptr(), 1,
                                        X.data_ptr(), n)
    assert st == -1
