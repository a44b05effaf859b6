"""The library's device workspace comes from the caller's allocator.

The Python binding hands torch's caching allocator to fh_create, so the
Krylov bases and work blocks of the shifted solves are torch memory (they show
in torch.cuda.memory_allocated and go back to torch's pool when the problem is
destroyed).  A handle made with allocator=None uses hipMalloc and computes the
same numbers."""
import gc

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
fh = pytest.importorskip("paper_1506_04463_amd")


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _csr(A):
    return fh.CSR(_cuda(A["rowptr"].astype(np.int32)), _cuda(A["colind"].astype(np.int32)), _cuda(A["val"]), A["n"])


def _solve(handle, A, z, sides, B, opts):
    prob = fh.Problem(handle, _csr(A))
    X, rep = fh.shifted_solve(prob, z, sides, B, opts)
    torch.cuda.synchronize()
    return prob, X, rep


def test_workspace_comes_from_torch_allocator():
    A = W.convdiff2d_csr(32, 20.0, 10.0)            # n = 1,024
    n, m, restart = A["n"], 16, 30
    # shifts left of the spectrum (which starts near 145): GMRES converges
    z = np.array([-100.0 + 200j, -100.0 + 200j, -50.0 - 100j, -50.0 - 100j])
    sides = [0, 0, 1, 1]
    B = _cuda(np.stack([W.subspace(n, m, 40 + s) for s in range(4)]))
    opts = fh.default_opts(m, solver=1, precond=2, inner_tol=1e-10, restart=restart, max_restarts=20)

    torch.cuda.synchronize()
    gc.collect()
    before = torch.cuda.memory_allocated()
    ht = fh.Handle(0)                                  # torch's caching allocator
    assert ht.allocator == "torch"
    prob, X, rep = _solve(ht, A, z, sides, B, opts)
    grown = torch.cuda.memory_allocated() - before - X.numel() * X.element_size()
    # the Krylov basis alone: (restart + 1) vectors of nsys x n x m complex128
    basis = (restart + 1) * 4 * n * m * 16
    assert grown >= basis, (grown, basis)
    assert rep["inner_relres"] <= 1e-10

    # hipMalloc handle: identical results, workspace outside torch's count
    hh = fh.Handle(0, allocator=None)
    mid = torch.cuda.memory_allocated()
    prob2, X2, rep2 = _solve(hh, A, z, sides, B, opts)
    assert torch.cuda.memory_allocated() - mid <= X2.numel() * X2.element_size() + (1 << 20)
    assert torch.equal(X, X2)
    assert rep["inner_steps"] == rep2["inner_steps"]

    # destroying the problem and the handle gives the workspace back to torch
    del prob, prob2, ht, hh
    gc.collect()
    torch.cuda.synchronize()
    held = torch.cuda.memory_allocated() - before - 2 * X.numel() * X.element_size()
    assert held < basis // 4, held


def test_allocator_failure_is_an_error():
    """A source that cannot allocate: the call fails with FH_HIP_ERROR and a
    message; nothing is computed."""
    import ctypes as C

    calls = []

    def no_mem(nbytes, stream, user):
        calls.append(int(nbytes))
        return None

    def free(ptr, nbytes, stream, user):
        pass

    fa, ff = fh._ALLOC_FN(no_mem), fh._FREE_FN(free)
    al = fh.fh_allocator(fa, ff, None)
    h = C.c_void_p()
    s = torch.cuda.current_stream(0)
    assert fh.lib().fh_create(C.byref(h), 0, C.c_void_p(s.cuda_stream), C.byref(al)) == 0
    # an allocator with a missing callback is an invalid argument 4
    bad = fh.fh_allocator(fa, fh._FREE_FN(), None)
    h2 = C.c_void_p()
    assert fh.lib().fh_create(C.byref(h2), 0, C.c_void_p(s.cuda_stream), C.byref(bad)) == -4
    A = W.convdiff2d_csr(8, 20.0, 10.0)
    Ac = _csr(A)
    mat = fh.fh_mat(fh.FH_CSR, fh.FH_R64, A["n"], 0, Ac.colind.numel(), Ac.val.data_ptr(), Ac.rowptr.data_ptr(),
                    Ac.colind.data_ptr())
    p = C.c_void_p()
    rc = fh.lib().fh_problem_create(h, C.byref(mat), None, C.byref(p))
    if rc == 0:
        Y = _cuda(W.subspace(A["n"], 4, 1).reshape(1, A["n"], 4))
        X = torch.empty_like(Y)
        zk = np.array([1.0 + 1j])
        sd = (C.c_int * 1)(0)
        opts = fh.default_opts(4, solver=1, precond=2)
        rc = fh.lib().fh_shifted_solve(h, p, 1, zk.ctypes.data_as(C.POINTER(C.c_double)), sd, 4, C.byref(opts),
                                       C.c_void_p(Y.data_ptr()), C.c_void_p(X.data_ptr()), None)
        fh.lib().fh_problem_destroy(p)
    assert rc == 100
    assert b"allocator returned no memory" in fh.lib().fh_last_error(h)
    assert calls
    fh.lib().fh_destroy(h)
