"""feasthip: non-Hermitian FEAST on AMD MI355X (gfx950).

Thin ctypes binding of ``libfeasthip.so`` (C ABI in ``include/feasthip.h``).
Argument marshalling only: every numerical step runs in the library's HIP
kernels.  PyTorch supplies device memory and the stream.  Importing this module
does not load the library; the first call does, and it raises if the library
has not been built (there is no fallback).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfeasthip.so")

FH_DENSE, FH_CSR = 0, 1
FH_R64, FH_C128 = 0, 1
FH_PREC_FP64, FH_PREC_MIXED = 0, 1
FH_SOLVER_LU, FH_SOLVER_BGMRES = 0, 1
FH_PC_NONE, FH_PC_JACOBI, FH_PC_ILU0, FH_PC_LEARNED = 0, 1, 2, 3
# fh_feast status codes (include/feasthip.h)
FH_OK, FH_NO_EIG_INSIDE, FH_NOT_CONVERGED, FH_M0_TOO_SMALL = 0, 1, 2, 3
NET_HIDDEN = 16
NET_FIXED_CHANNELS = 5

STATUS = {0: "ok", 1: "no eigenvalue inside", 2: "not converged", 3: "m0 too small",
          4: "singular shift", 5: "inner solve failed", 6: "non-finite", 7: "reduced eig failed",
          100: "hip error"}


class FeastError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"feasthip error {code} ({STATUS.get(code, 'invalid argument' if code < 0 else '?')}): {msg}")
        self.code = code


class fh_mat(C.Structure):
    _fields_ = [("kind", C.c_int), ("dtype", C.c_int), ("n", C.c_int), ("ld", C.c_int), ("nnz", C.c_longlong),
                ("val", C.c_void_p), ("rowptr", C.c_void_p), ("colind", C.c_void_p)]


class fh_contour(C.Structure):
    _fields_ = [("c_re", C.c_double), ("c_im", C.c_double), ("a", C.c_double), ("ratio", C.c_double),
                ("angle", C.c_double), ("ne", C.c_int), ("nv", C.c_int), ("verts", C.c_void_p)]


def _polygon(c: "fh_contour", polygon):
    """Set the polygon fields of c; returns the vertex buffer (keep it alive
    for the call)."""
    if polygon is None:
        return None
    v = np.ascontiguousarray(np.asarray(polygon, dtype=np.complex128).reshape(-1))
    c.nv = len(v)
    c.verts = v.ctypes.data_as(C.c_void_p)
    return v


class fh_opts(C.Structure):
    _fields_ = [("m0", C.c_int), ("max_iter", C.c_int), ("eps", C.c_double), ("precision", C.c_int),
                ("solver", C.c_int), ("restart", C.c_int), ("block", C.c_int), ("precond", C.c_int),
                ("inner_tol", C.c_double), ("max_restarts", C.c_int), ("mixed_inner_tol", C.c_double),
                ("max_refine", C.c_int), ("save_factors", C.c_int), ("resume", C.c_int), ("fallback", C.c_int),
                ("graph", C.c_int), ("orth", C.c_int), ("batch_nodes", C.c_int),
                ("sym", C.c_int), ("confirm", C.c_int), ("conj_pairs", C.c_int)]


class fh_report(C.Structure):
    _fields_ = [("info", C.c_int), ("m", C.c_int), ("iters", C.c_int), ("m0_final", C.c_int),
                ("bad_node", C.c_int), ("m_s", C.c_int), ("n_factor", C.c_longlong), ("n_solve", C.c_longlong),
                ("inner_steps", C.c_longlong), ("inner_relres", C.c_double), ("t_filter_ms", C.c_double),
                ("t_iter_ms", C.c_double), ("n_fallback", C.c_longlong), ("n_bq_retry", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)


class fh_allocator(C.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("user", C.c_void_p)]


# torch's caching allocator as the library's device-memory source.  The
# callbacks are module globals so that they outlive every handle; user carries
# the device index.  After interpreter shutdown has begun nothing is freed
# through them (the process is ending; torch may already be gone).
_shutting_down = False


def _on_exit():
    global _shutting_down
    _shutting_down = True


import atexit as _atexit  # noqa: E402

_atexit.register(_on_exit)


def _torch_alloc(nbytes, stream, user):
    try:
        torch = _torch()
        return torch.cuda.caching_allocator_alloc(int(nbytes), int(user or 0), int(stream or 0))
    except Exception:
        return None


def _torch_free(ptr, nbytes, stream, user):
    if _shutting_down or not ptr:
        return
    try:
        _torch().cuda.caching_allocator_delete(int(ptr))
    except Exception:
        pass


_TORCH_ALLOC = _ALLOC_FN(_torch_alloc)
_TORCH_FREE = _FREE_FN(_torch_free)

_lib = None


def lib():
    """Load libfeasthip.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1506_04463_amd.build` "
                          "(or __graft_entry__.build()); there is no fallback path")
    L = C.CDLL(LIB_PATH)
    vp, i, d, dp, ip = C.c_void_p, C.c_int, C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_int)
    sig = {
        "fh_create": (i, [C.POINTER(vp), i, vp, C.POINTER(fh_allocator)]),
        "fh_destroy": (i, [vp]),
        "fh_set_stream": (i, [vp, vp]),
        "fh_last_error": (C.c_char_p, [vp]),
        "fh_default_opts": (None, [C.POINTER(fh_opts)]),
        "fh_contour_nodes": (i, [C.POINTER(fh_contour), dp, dp]),
        "fh_rational": (i, [i, dp, dp, i, dp, dp]),
        "fh_problem_create": (i, [vp, C.POINTER(fh_mat), C.POINTER(fh_mat), C.POINTER(vp)]),
        "fh_problem_destroy": (i, [vp]),
        "fh_filter": (i, [vp, vp, i, dp, dp, i, vp, vp, vp, vp, C.POINTER(fh_opts), C.POINTER(fh_report)]),
        "fh_feast": (i, [vp, vp, C.POINTER(fh_contour), dp, dp, C.POINTER(fh_opts), vp, vp, vp, dp,
                         C.POINTER(fh_report)]),
        "fh_reduced_matrix": (i, [vp, vp, i, vp, vp, vp]),
        "fh_reduced_matrix_noalloc": (i, [vp, vp, i, vp, vp, vp]),
        "fh_biortho_factors": (i, [vp, i, vp, d, vp, vp, vp, ip]),
        "fh_count_estimate": (i, [vp, vp, i, dp, dp, i, vp, vp, dp, vp]),
        "fh_reduced_eig": (i, [vp, i, vp, vp, vp, vp, vp]),
        "fh_shifted_apply": (i, [vp, vp, i, i, dp, i, vp, vp]),
        "fh_residual_pair": (i, [vp, vp, i, i, dp, i, vp, vp, vp, vp, vp]),
        "fh_ilu0": (i, [vp, vp, d, d, vp]),
        "fh_ilu0_apply": (i, [vp, vp, d, d, i, i, vp, vp]),
        "fh_ilu0_apply_c64": (i, [vp, vp, d, d, i, i, vp, vp]),
        "fh_shifted_solve": (i, [vp, vp, i, dp, ip, i, C.POINTER(fh_opts), vp, vp, C.POINTER(fh_report)]),
        "fh_feast_batched": (i, [vp, i, C.POINTER(vp), C.POINTER(fh_contour), C.POINTER(fh_opts), C.POINTER(vp),
                                 C.POINTER(vp), C.POINTER(vp), C.POINTER(dp), C.POINTER(fh_report)]),
        "fh_net_create": (i, [vp, i, i, i, i, dp, d, d, C.c_ulonglong, C.POINTER(vp)]),
        "fh_net_destroy": (i, [vp]),
        "fh_net_param_count": (i, [vp]),
        "fh_net_get_params": (i, [vp, vp, C.POINTER(C.c_float)]),
        "fh_net_set_params": (i, [vp, vp, C.POINTER(C.c_float)]),
        "fh_net_forward": (i, [vp, vp, i, i, dp, ip, vp, vp]),
        "fh_net_set_fields": (i, [vp, vp, dp]),
        "fh_net_set_activations": (i, [vp, i]),
        "fh_net_train_step": (i, [vp, vp, vp, i, i, dp, ip, vp, vp, d, i, dp, C.POINTER(C.c_float)]),
        "fh_problem_set_net": (i, [vp, vp]),
        "fh_profile": (i, [vp, i]),
        "fh_profile_read": (i, [vp, i, C.c_char_p, i, C.POINTER(C.c_longlong), dp, dp, dp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _torch():
    import torch
    return torch


def _dptr(t):
    return C.c_void_p(t.data_ptr())


def _cbuf(arr):
    """complex128 numpy array -> (keepalive, double*)"""
    a = np.ascontiguousarray(np.asarray(arr, dtype=np.complex128))
    return a, a.ctypes.data_as(C.POINTER(C.c_double))


def _check_block(t, n, name):
    torch = _torch()
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.complex128 and t.is_contiguous()
            and t.dim() == 2 and t.shape[0] == n):
        raise ValueError(f"{name} must be a contiguous complex128 CUDA tensor of shape (n={n}, m)")


class Handle:
    """Library handle bound to one device and (by default) torch's current stream.

    allocator="torch" (default): the library's workspace comes from torch's
    caching allocator (it shows in torch.cuda.memory_allocated and is reused
    by torch after it is freed); allocator=None: the library calls hipMalloc."""

    def __init__(self, device=0, stream=None, allocator="torch"):
        torch = _torch()
        L = lib()
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        if allocator not in ("torch", None):
            raise ValueError("allocator must be 'torch' or None")
        al = None
        if allocator == "torch":
            al = fh_allocator(_TORCH_ALLOC, _TORCH_FREE, C.c_void_p(device))
        self.allocator = allocator
        h = C.c_void_p()
        rc = L.fh_create(C.byref(h), device, C.c_void_p(stream.cuda_stream), C.byref(al) if al is not None else None)
        if rc != 0:
            raise FeastError(rc, "fh_create")
        self._h = h

    def check(self, rc, what):
        if rc != 0:
            msg = lib().fh_last_error(self._h)
            raise FeastError(rc, f"{what}: {msg.decode() if msg else ''}")

    def profile(self, enable=True):
        self.check(lib().fh_profile(self._h, 1 if enable else 0), "fh_profile")

    def profile_stats(self):
        out = {}
        buf = C.create_string_buffer(256)
        cnt, ms, by, fl = C.c_longlong(), C.c_double(), C.c_double(), C.c_double()
        idx = 0
        while True:
            rc = lib().fh_profile_read(self._h, idx, buf, 256, C.byref(cnt), C.byref(ms), C.byref(by), C.byref(fl))
            if rc == 1:
                break
            self.check(rc, "fh_profile_read")
            out[buf.value.decode()] = {"count": cnt.value, "ms": ms.value, "bytes": by.value, "flops": fl.value}
            idx += 1
        return out

    def __del__(self):
        try:
            if getattr(self, "_h", None) and not _shutting_down:
                lib().fh_destroy(self._h)
        except Exception:
            pass


@dataclass
class CSR:
    rowptr: object   # int32 CUDA tensor (n+1)
    colind: object   # int32 CUDA tensor (nnz)
    val: object      # float64 or complex128 CUDA tensor (nnz)
    n: int


class Problem:
    """A (dense complex128 tensor or CSR) and optional dense B, prepared on the GPU."""

    def __init__(self, handle: Handle, A, B=None):
        torch = _torch()
        self.handle = handle
        m = fh_mat()
        if isinstance(A, CSR):
            m.kind, m.n, m.nnz = FH_CSR, A.n, A.colind.numel()
            m.dtype = FH_R64 if A.val.dtype == torch.float64 else FH_C128
            if A.val.dtype not in (torch.float64, torch.complex128):
                raise ValueError("CSR values must be float64 or complex128")
            for t in (A.rowptr, A.colind):
                if t.dtype != torch.int32 or not t.is_cuda or not t.is_contiguous():
                    raise ValueError("CSR index arrays must be contiguous int32 CUDA tensors")
            m.val, m.rowptr, m.colind = A.val.data_ptr(), A.rowptr.data_ptr(), A.colind.data_ptr()
            m.ld = 0
            self.n = A.n
        else:
            _check_block(A, A.shape[0], "A")
            m.kind, m.dtype, m.n, m.ld, m.nnz = FH_DENSE, FH_C128, A.shape[0], A.shape[1], 0
            m.val = A.data_ptr()
            self.n = A.shape[0]
        bm = None
        if B is not None:
            _check_block(B, self.n, "B")
            bm = fh_mat(FH_DENSE, FH_C128, self.n, B.shape[1], 0, B.data_ptr(), None, None)
        self._keep = (A, B)
        p = C.c_void_p()
        rc = lib().fh_problem_create(handle._h, C.byref(m), C.byref(bm) if bm is not None else None, C.byref(p))
        handle.check(rc, "fh_problem_create")
        self._p = p

    def __del__(self):
        try:
            if getattr(self, "_p", None) and not _shutting_down:
                lib().fh_problem_destroy(self._p)
        except Exception:
            pass


def default_opts(m0, **kw) -> fh_opts:
    o = fh_opts()
    lib().fh_default_opts(C.byref(o))
    o.m0 = m0
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def contour_nodes(center, a, ratio=1.0, angle=0.0, ne=8, polygon=None):
    """Nodes and weights of the ellipse, or of the polygon with the vertices
    `polygon` (ne / len(polygon) trapezoid intervals per side)."""
    c = fh_contour(complex(center).real, complex(center).imag, a, ratio, angle, ne)
    keep = _polygon(c, polygon)
    z = np.zeros(ne, np.complex128)
    w = np.zeros(ne, np.complex128)
    rc = lib().fh_contour_nodes(C.byref(c), z.ctypes.data_as(C.POINTER(C.c_double)),
                                w.ctypes.data_as(C.POINTER(C.c_double)))
    if rc != 0:
        raise FeastError(rc, "fh_contour_nodes")
    return z, w


def rational(z, w, lam):
    zk, zp = _cbuf(z)
    wk, wp = _cbuf(w)
    lk, lp = _cbuf(np.atleast_1d(lam))
    out = np.zeros(len(lk), np.complex128)
    rc = lib().fh_rational(len(zk), zp, wp, len(lk), lp, out.ctypes.data_as(C.POINTER(C.c_double)))
    if rc != 0:
        raise FeastError(rc, "fh_rational")
    return out


def contour_filter(prob: Problem, z, w, Y, Yh, opts: fh_opts | None = None):
    """Q = sum_j w_j (z_j B - A)^{-1} B Y ;  Qh = sum_j conj(w_j) (z_j B - A)^{-H} B^H Yh."""
    torch = _torch()
    n = prob.n
    _check_block(Y, n, "Y")
    _check_block(Yh, n, "Yh")
    m0 = Y.shape[1]
    Q = torch.empty_like(Y)
    Qh = torch.empty_like(Yh)
    zk, zp = _cbuf(z)
    wk, wp = _cbuf(w)
    rep = fh_report()
    rc = lib().fh_filter(prob.handle._h, prob._p, len(zk), zp, wp, m0, _dptr(Y), _dptr(Yh), _dptr(Q), _dptr(Qh),
                         C.byref(opts) if opts is not None else None, C.byref(rep))
    prob.handle.check(rc, "fh_filter")
    return Q, Qh, rep.as_dict()


def count_estimate(prob: Problem, z, w, V, opts: fh_opts | None = None):
    """Stochastic estimate of the number of eigenvalues inside the contour:
    (1/p) trace(V^H Q) with Q the filter applied to the probe block V (n x p,
    complex128 CUDA).  Returns (estimate as a complex number, report)."""
    n = prob.n
    _check_block(V, n, "V")
    zk, zp = _cbuf(z)
    wk, wp = _cbuf(w)
    est = np.zeros(2)
    rep = fh_report()
    rc = lib().fh_count_estimate(prob.handle._h, prob._p, len(zk), zp, wp, V.shape[1], _dptr(V),
                                 C.byref(opts) if opts is not None else None,
                                 est.ctypes.data_as(C.POINTER(C.c_double)), C.byref(rep))
    prob.handle.check(rc, "fh_count_estimate")
    return complex(est[0], est[1]), rep.as_dict()


def feast(prob: Problem, center, a, ratio=1.0, angle=0.0, ne=8, Y0=None, Yh0=None, opts: fh_opts | None = None,
          z=None, w=None, ritz0=None, polygon=None):
    """Non-Hermitian FEAST; returns dict(info, lam, X, Xh, res, report, and the
    whole final subspace Y, Yh, ritz, ritz_res).  ritz0 (with opts.resume = 1):
    Ritz values of the start columns.  polygon: complex vertices of a polygon
    contour (then center .. angle are unused)."""
    torch = _torch()
    n = prob.n
    _check_block(Y0, n, "Y0")
    _check_block(Yh0, n, "Yh0")
    m0 = Y0.shape[1]
    if opts is None:
        opts = default_opts(m0)
    Y = Y0.clone()
    Yh = Yh0.clone()
    lam = torch.zeros(m0, dtype=torch.complex128, device=Y.device)
    if ritz0 is not None:
        lam.copy_(ritz0.reshape(-1)[:m0] if isinstance(ritz0, torch.Tensor) else torch.from_numpy(np.asarray(ritz0)))
    res = np.zeros(m0)
    c = fh_contour(complex(center).real, complex(center).imag, a, ratio, angle, ne)
    keep = _polygon(c, polygon)
    zp = wp = None
    if z is not None:
        zk, zp = _cbuf(z)
        wk, wp = _cbuf(w)
    rep = fh_report()
    rc = lib().fh_feast(prob.handle._h, prob._p, C.byref(c), zp, wp, C.byref(opts), _dptr(Y), _dptr(Yh),
                        _dptr(lam), res.ctypes.data_as(C.POINTER(C.c_double)), C.byref(rep))
    if rc < 0 or rc >= 4:
        prob.handle.check(rc, "fh_feast")
    m, mt = rep.m, rep.m0_final
    return {"info": rc, "lam": lam[:m].cpu().numpy(), "X": Y[:, :m], "Xh": Yh[:, :m], "res": res[:m],
            "report": rep.as_dict(), "Y": Y[:, :mt], "Yh": Yh[:, :mt], "ritz": lam[:mt], "ritz_res": res[:mt]}


def feast_batched(probs, contours, Y0s, Yh0s, opts: fh_opts):
    """FEAST on many dense problems at once (fh_feast_batched).

    contours: list of (center, a, ratio, angle, ne[, polygon vertices]) (the
    same problem may appear with several contours); Y0s, Yh0s: lists of
    complex128 CUDA tensors (n_i, m0).  Returns (status, list of dicts as
    feast())."""
    torch = _torch()
    k = len(probs)
    m0 = opts.m0
    Ys = [Y.clone() for Y in Y0s]
    Yhs = [Y.clone() for Y in Yh0s]
    for i in range(k):
        _check_block(Ys[i], probs[i].n, "Y0")
        _check_block(Yhs[i], probs[i].n, "Yh0")
    lams = [torch.zeros(m0, dtype=torch.complex128, device=Ys[i].device) for i in range(k)]
    res = [np.zeros(m0) for _ in range(k)]
    cs = (fh_contour * k)(*[fh_contour(complex(c[0]).real, complex(c[0]).imag, c[1], c[2], c[3], c[4])
                            for c in contours])
    keep = [_polygon(cs[i], c[5] if len(c) > 5 else None) for i, c in enumerate(contours)]
    vp = C.c_void_p
    pa = (vp * k)(*[p._p.value for p in probs])
    ya = (vp * k)(*[Y.data_ptr() for Y in Ys])
    yha = (vp * k)(*[Y.data_ptr() for Y in Yhs])
    la = (vp * k)(*[l.data_ptr() for l in lams])
    ra = (C.POINTER(C.c_double) * k)(*[r.ctypes.data_as(C.POINTER(C.c_double)) for r in res])
    reps = (fh_report * k)()
    h = probs[0].handle
    rc = lib().fh_feast_batched(h._h, k, pa, cs, C.byref(opts), ya, yha, la, ra, reps)
    if rc < 0 or rc >= 4:
        h.check(rc, "fh_feast_batched")
    out = []
    for i in range(k):
        m, mt = reps[i].m, reps[i].m0_final
        out.append({"info": reps[i].info, "lam": lams[i][:m].cpu().numpy(), "X": Ys[i][:, :m], "Xh": Yhs[i][:, :m],
                    "res": res[i][:m], "report": reps[i].as_dict(), "Y": Ys[i][:, :mt], "Yh": Yhs[i][:, :mt],
                    "ritz": lams[i][:mt], "ritz_res": res[i][:mt]})
    return rc, out


def reduced_matrix(prob: Problem, Qh, Q):
    torch = _torch()
    m = Q.shape[1]
    BQ = torch.empty((m, m), dtype=torch.complex128, device=Q.device)
    prob.handle.check(lib().fh_reduced_matrix(prob.handle._h, prob._p, m, _dptr(Qh), _dptr(Q), _dptr(BQ)),
                      "fh_reduced_matrix")
    return BQ


def reduced_matrix_noalloc(prob: Problem, Qh, Q, BQ):
    """fh_reduced_matrix_noalloc: BQ (m x m complex128, caller's) = Qh^H B Q
    with the library's static device scratch (no allocation in the call)."""
    m = Q.shape[1]
    if BQ.shape != (m, m) or not BQ.is_contiguous():
        raise ValueError("BQ must be a contiguous (m, m) tensor")
    prob.handle.check(lib().fh_reduced_matrix_noalloc(prob.handle._h, prob._p, m, _dptr(Qh), _dptr(Q), _dptr(BQ)),
                      "fh_reduced_matrix_noalloc")
    return BQ


def biortho_factors(handle: Handle, BQ, eta=1e-16):
    torch = _torch()
    m = BQ.shape[0]
    gam = torch.empty(m, dtype=torch.complex128, device=BQ.device)
    S = torch.empty((m, m), dtype=torch.complex128, device=BQ.device)
    Sh = torch.empty_like(S)
    mt = C.c_int()
    handle.check(lib().fh_biortho_factors(handle._h, m, _dptr(BQ), eta, _dptr(gam), _dptr(S), _dptr(Sh),
                                          C.byref(mt)), "fh_biortho_factors")
    return gam, S, Sh, mt.value


def reduced_eig(handle: Handle, AU, BU):
    torch = _torch()
    m = AU.shape[0]
    lam = torch.empty(m, dtype=torch.complex128, device=AU.device)
    W = torch.empty((m, m), dtype=torch.complex128, device=AU.device)
    Wh = torch.empty_like(W)
    handle.check(lib().fh_reduced_eig(handle._h, m, _dptr(AU), _dptr(BU), _dptr(lam), _dptr(W), _dptr(Wh)),
                 "fh_reduced_eig")
    return lam, W, Wh


def shifted_apply(prob: Problem, side, shifts, X):
    """Out_s = shift_s X_s - op(A) X_s for a (nsys, n, m) complex128 tensor X (op = A or A^H)."""
    torch = _torch()
    nsys, n, m = X.shape
    Out = torch.empty_like(X)
    sk, sp = _cbuf(shifts)
    prob.handle.check(lib().fh_shifted_apply(prob.handle._h, prob._p, side, nsys, sp, m, _dptr(X), _dptr(Out)),
                      "fh_shifted_apply")
    return Out


def residual_pair(prob: Problem, side, shifts, B, X, Xt):
    """(R, E) with R_s = B_s - M_s X_s and E_s = Xt_s - X_s, M_s = shift_s - op(A)
    (op = A or A^H), for (nsys, n, m) complex128 tensors (CSR problems)."""
    torch = _torch()
    nsys, n, m = X.shape
    R = torch.empty_like(X)
    E = torch.empty_like(X)
    sk, sp = _cbuf(shifts)
    prob.handle.check(lib().fh_residual_pair(prob.handle._h, prob._p, side, nsys, sp, m, _dptr(B), _dptr(X), _dptr(Xt),
                                             _dptr(R), _dptr(E)), "fh_residual_pair")
    return R, E


def ilu0(prob: Problem, z):
    torch = _torch()
    nnz = prob._keep[0].colind.numel()
    lu = torch.empty(nnz, dtype=torch.complex128, device="cuda")
    prob.handle.check(lib().fh_ilu0(prob.handle._h, prob._p, complex(z).real, complex(z).imag, _dptr(lu)), "fh_ilu0")
    return lu


def ilu0_apply(prob: Problem, z, side, X):
    """(LU)^{-1} X (side 0) or (LU)^{-H} X (side 1) with the ILU(0) of (z - A);
    X: complex128 (n, m) CUDA tensor, or complex64 for the complex-FP32 apply."""
    torch = _torch()
    Out = torch.empty_like(X)
    if X.dtype == torch.complex64:
        if not (X.is_cuda and X.is_contiguous() and X.dim() == 2 and X.shape[0] == prob.n):
            raise ValueError(f"X must be a contiguous ({prob.n}, m) complex64 CUDA tensor")
        prob.handle.check(lib().fh_ilu0_apply_c64(prob.handle._h, prob._p, complex(z).real, complex(z).imag, side,
                                                  X.shape[1], C.c_void_p(X.data_ptr()), C.c_void_p(Out.data_ptr())),
                          "fh_ilu0_apply_c64")
        return Out
    prob.handle.check(lib().fh_ilu0_apply(prob.handle._h, prob._p, complex(z).real, complex(z).imag, side,
                                          X.shape[1], _dptr(X), _dptr(Out)), "fh_ilu0_apply")
    return Out


def _sides(sides, nsys):
    a = np.ascontiguousarray(np.broadcast_to(np.asarray(sides, dtype=np.int32), (nsys,)))
    return a, a.ctypes.data_as(C.POINTER(C.c_int))


def _check_batch(t, n, name):
    torch = _torch()
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.complex128 and t.is_contiguous()
            and t.dim() == 3 and t.shape[1] == n):
        raise ValueError(f"{name} must be a contiguous complex128 CUDA tensor of shape (nsys, n={n}, m)")


def shifted_solve(prob: Problem, z, sides, B, opts: fh_opts | None = None):
    """X_s = (z_s - A)^{-1} B_s (side 0) or (z_s - A)^{-H} B_s (side 1); B: (nsys, n, m) complex128.

    Right systems must come before left ones.  Returns (X, report dict)."""
    torch = _torch()
    _check_batch(B, prob.n, "B")
    nsys, n, m = B.shape
    if opts is None:
        opts = default_opts(m)
    zk, zp = _cbuf(np.broadcast_to(np.asarray(z, dtype=np.complex128), (nsys,)))
    sk, sp = _sides(sides, nsys)
    X = torch.empty_like(B)
    rep = fh_report()
    prob.handle.check(lib().fh_shifted_solve(prob.handle._h, prob._p, nsys, zp, sp, m, C.byref(opts), _dptr(B),
                                             _dptr(X), C.byref(rep)), "fh_shifted_solve")
    return X, rep.as_dict()


class Net:
    """Learned preconditioner network (3x3 or 3x3x3 conv, cin -> 16 -> 16 -> 2) on an
    (nz x) ny x nx grid."""

    def __init__(self, handle: Handle, ny, nx, fields=None, alpha=1.0, out_scale=1.0, seed=0, nz=1):
        self.handle = handle
        self.nz, self.ny, self.nx = nz, ny, nx
        self.npix = nz * ny * nx
        f = None if fields is None else np.ascontiguousarray(np.asarray(fields, dtype=np.float64).reshape(-1, self.npix))
        self.nfields = 0 if f is None else f.shape[0]
        self._fields = f
        fp = None if f is None else f.ctypes.data_as(C.POINTER(C.c_double))
        p = C.c_void_p()
        handle.check(lib().fh_net_create(handle._h, nz, ny, nx, self.nfields, fp, float(alpha), float(out_scale),
                                         C.c_ulonglong(seed), C.byref(p)), "fh_net_create")
        self.out_scale = float(out_scale)
        self._n = p
        self.n_params = lib().fh_net_param_count(p)
        self.cin = NET_FIXED_CHANNELS + self.nfields

    def get_params(self):
        a = np.zeros(self.n_params, np.float32)
        self.handle.check(lib().fh_net_get_params(self.handle._h, self._n, a.ctypes.data_as(C.POINTER(C.c_float))),
                          "fh_net_get_params")
        return a

    def set_params(self, params):
        a = np.ascontiguousarray(np.asarray(params, dtype=np.float32))
        if a.size != self.n_params:
            raise ValueError(f"expected {self.n_params} parameters")
        self.handle.check(lib().fh_net_set_params(self.handle._h, self._n, a.ctypes.data_as(C.POINTER(C.c_float))),
                          "fh_net_set_params")

    def unpack(self, params):
        """flat vector -> [(w1, b1), (w2, b2), (w3, b3)] with w [cout, cin, 3, 3(, 3)]"""
        H, cin = NET_HIDDEN, self.cin
        k = (3, 3) if self.nz == 1 else (3, 3, 3)
        T = int(np.prod(k))
        shapes = [(H, cin), (H, H), (2, H)]
        out, off = [], 0
        for co, ci in shapes:
            w = np.asarray(params[off:off + co * ci * T]).reshape((co, ci) + k)
            off += co * ci * T
            b = np.asarray(params[off:off + co])
            off += co
            out.append((w, b))
        return out

    def set_fields(self, fields):
        """Replace the constant input fields ([nfields, n] or [nfields, *grid])."""
        f = np.ascontiguousarray(np.asarray(fields, dtype=np.float64).reshape(-1, self.npix))
        if f.shape[0] != self.nfields:
            raise ValueError(f"expected {self.nfields} fields")
        self._fields = f
        self.handle.check(lib().fh_net_set_fields(self.handle._h, self._n, f.ctypes.data_as(C.POINTER(C.c_double))),
                          "fh_net_set_fields")

    def set_activations(self, bf16: bool):
        """BF16 (True) or FP32 (False, the default) activations in inference passes."""
        rc = lib().fh_net_set_activations(self._n, 1 if bf16 else 0)
        if rc != 0:
            raise FeastError(rc, "fh_net_set_activations")

    def forward(self, z, sides, V):
        """V: (nsys, n, m) complex128 -> network output of the same shape."""
        torch = _torch()
        _check_batch(V, self.npix, "V")
        nsys, n, m = V.shape
        zk, zp = _cbuf(np.broadcast_to(np.asarray(z, dtype=np.complex128), (nsys,)))
        sk, sp = _sides(sides, nsys)
        Out = torch.empty_like(V)
        self.handle.check(lib().fh_net_forward(self.handle._h, self._n, nsys, m, zp, sp, _dptr(V), _dptr(Out)),
                          "fh_net_forward")
        return Out

    def train_step(self, z, sides, R, E, lr=1e-3, update=True, want_grad=False, problem: "Problem | None" = None):
        """One loss/gradient evaluation on (residual, error) pairs; Adam step if update.

        With a CSR problem the loss is measured in the residual norm of its
        shifted operators, else in the error norm."""
        _check_batch(R, self.npix, "R")
        _check_batch(E, self.npix, "E")
        nsys, n, m = R.shape
        zk, zp = _cbuf(np.broadcast_to(np.asarray(z, dtype=np.complex128), (nsys,)))
        sk, sp = _sides(sides, nsys)
        loss = C.c_double()
        g = np.zeros(self.n_params, np.float32) if want_grad else None
        gp = g.ctypes.data_as(C.POINTER(C.c_float)) if want_grad else None
        pp = problem._p if problem is not None else None
        self.handle.check(lib().fh_net_train_step(self.handle._h, self._n, pp, nsys, m, zp, sp, _dptr(R), _dptr(E),
                                                  float(lr), int(bool(update)), C.byref(loss), gp),
                          "fh_net_train_step")
        return (loss.value, g) if want_grad else loss.value

    def __del__(self):
        try:
            if getattr(self, "_n", None) and not _shutting_down:
                lib().fh_net_destroy(self._n)
        except Exception:
            pass


def set_net(prob: Problem, net: "Net | None"):
    """Attach (or detach with None) the learned preconditioner of a CSR problem."""
    rc = lib().fh_problem_set_net(prob._p, net._n if net is not None else None)
    if rc != 0:
        raise FeastError(rc, "fh_problem_set_net: grid size does not match the problem")
    prob._net = net   # keep the network alive while attached
