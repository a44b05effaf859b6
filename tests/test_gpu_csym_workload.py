"""The headline workload's construction on a reduced grid (the complex-
symmetric operator -Lap + V - 5i W on a 64 x 64 grid of (0, 40)^2, 50 wells,
ellipse centred in the lower half-plane around its lowest eigenvalues, Ne =
24): FEAST in the headline's launch configuration (complex-FP32 GMRES(30) x 2
+ ILU(0), DCGS2, residual form; right solves only with the left block
conj(Y) D, or explicit left solves) against the oracle's FEAST with direct
solves and against ARPACK's eigenvalues, element by element."""
import numpy as np
import pytest

import workloads as W
from oracle import feast as F
from oracle import linsolve as L
from oracle import reference as R

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
fh = pytest.importorskip("paper_1506_04463_amd")


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _csr(A):
    return fh.CSR(_cuda(A["rowptr"].astype(np.int32)), _cuda(A["colind"].astype(np.int32)), _cuda(A["val"]), A["n"])


@pytest.fixture(scope="module")
def case():
    from threadpoolctl import threadpool_limits
    N = 64
    A = W.schrodinger2d_csr(N)
    eigs = R.nearest_eigenvalues(A, 60, -45.0)
    p = W.schrodinger2d(N=N, eigs=eigs, m_target=30, m0=40, ne=24)
    c = p.contour
    cont = F.Contour(c.center, c.a, c.ratio, 0.0, 24)
    with threadpool_limits(limits=2):
        ref = F.feast(L.csr_matrix(A), None, cont, p.Y0, p.Yh0, eps=1e-12, max_iter=40)
    assert ref.info == 0 and len(ref.lam) == p.info["m_in"] > 10
    return p, cont, ref, eigs


@pytest.mark.parametrize("sym", [1, 0])
def test_headline_configuration_reduced_grid(case, sym):
    p, cont, ref, eigs = case
    c = p.contour
    alpha = cont.alpha()
    h = fh.Handle(0)
    prob = fh.Problem(h, _csr(p.A))
    # confirmed exit (opts.confirm): with the inexact inner solves a true pair
    # can still be flagged spurious when the paper's test first passes (22 of
    # the 23 here), which the oracle's exact solves do not see
    o = fh.default_opts(p.m0, solver=1, precond=fh.FH_PC_ILU0, restart=30, max_restarts=2, inner_tol=1e-3,
                        precision=fh.FH_PREC_MIXED, mixed_inner_tol=1e-3, max_refine=1, max_iter=40, eps=1e-9, orth=2,
                        sym=sym, confirm=1)
    out = fh.feast(prob, c.center, c.a, c.ratio, 0.0, 24, _cuda(p.Y0), _cuda(p.Yh0), o)
    assert out["info"] == 0, out["report"]
    lam = out["lam"]
    m = len(lam)
    assert m == len(ref.lam)
    # element by element: the oracle's eigenvalues and ARPACK's (both sorted by
    # (Re, Im); the eigenvalues here are distinct in their real parts)
    assert np.max(np.abs(lam - ref.lam)) < 1e-10 * alpha
    u = eigs - c.center
    truth = np.sort_complex(eigs[(u.real / c.a) ** 2 + (u.imag / (c.ratio * c.a)) ** 2 < 1])
    assert np.max(np.abs(np.sort_complex(lam) - truth)) < 1e-10 * alpha
    X, Xh = out["X"].cpu().numpy(), out["Xh"].cpu().numpy()
    assert np.max(np.abs(Xh.conj().T @ X - np.eye(m))) < 1e-10
    # complex symmetric: Xh parallel to conj(X)
    cosang = np.abs(np.sum(X * Xh, axis=0)) / (np.linalg.norm(X, axis=0) * np.linalg.norm(Xh, axis=0))
    assert cosang.min() > 1 - 1e-10
    Ad = L.csr_matrix(p.A)
    nA = np.abs(Ad).sum(axis=0).max()
    rr = np.abs(Ad @ X - X * lam).sum(axis=0) / (nA * np.abs(X).sum(axis=0))
    rl = np.abs(Ad.conj().T @ Xh - Xh * np.conj(lam)).sum(axis=0) / (nA * np.abs(Xh).sum(axis=0))
    assert rr.max() <= 1e-10 and rl.max() <= 1e-10
    assert out["report"]["n_solve"] == out["report"]["iters"] * 24 * (1 if sym else 2)


def test_headline_configuration_learned_preconditioner(case):
    """The headline configuration's solver with the learned preconditioner:
    the 3x3 network (inputs: the block, the shift, the side and the fields V
    and W of the operator) trained on the GPU on (residual, error) pairs
    harvested from plain GMRES solves of the operator's own shifted systems at
    the 24 nodes, then FGMRES(30) x 2 in complex FP32 with the
    network as its flexible preconditioner and ILU(0) as the fallback, right
    solves only (sym = 1).  The eigenpairs equal the oracle's; ILU(0) runs the
    same FEAST for the comparison of iterations (printed)."""
    from paper_1506_04463_amd import learned
    p, cont, ref, eigs = case
    c = p.contour
    alpha = cont.alpha()
    N = p.info["N"]
    h = fh.Handle(0)
    prob = fh.Problem(h, _csr(p.A))
    hh = 40.0 / (N + 1)
    fields = np.stack([p.A["V"].ravel() / 20.0, p.A["W"].ravel()])
    # output scale: 1/max|a_ii| (h^2/4) over the grid side, since the network's
    # output per grid point is O(1) for an input of unit 2-norm
    net = fh.Net(h, N, N, fields=fields, alpha=float(c.a), out_scale=hh * hh / (4.0 * N), seed=5)
    z, _ = fh.contour_nodes(c.center, c.a, c.ratio, 0.0, 24)
    data = learned.harvest(prob, z, m=8, seed=11, steps=(0, 2, 5, 10))
    hist = learned.train(net, data, epochs=100, lr=2e-3, batch_systems=8, seed=0, problem=prob)
    assert hist[-1] < 0.7 * hist[0], hist
    fh.set_net(prob, net)
    runs, outs = {}, {}
    for name, pc in (("learned", fh.FH_PC_LEARNED), ("ilu0", fh.FH_PC_ILU0)):
        # eq:res <= 1e-10 so that the returned pairs also meet
        # ||A x - lam x||_1 / (||A||_1 ||x||_1) <= 1e-10
        o = fh.default_opts(p.m0, solver=1, precond=pc, restart=30, max_restarts=2, inner_tol=1e-3,
                            precision=fh.FH_PREC_MIXED, mixed_inner_tol=1e-3, max_refine=1, max_iter=60, eps=1e-10,
                            orth=2, sym=1, fallback=fh.FH_PC_ILU0, confirm=1)
        out = fh.feast(prob, c.center, c.a, c.ratio, 0.0, 24, _cuda(p.Y0), _cuda(p.Yh0), o)
        runs[name] = (out["info"], out["report"]["iters"], len(out["lam"]), out["report"]["n_fallback"])
        outs[name] = out
    print("training loss", hist[0], "->", hist[-1])
    print("FEAST (info, iterations, m, fallback solves) per preconditioner:", runs)
    out = outs["learned"]
    assert out["info"] == 0, out["report"]
    lam = out["lam"]
    m = len(lam)
    assert m == len(ref.lam)
    assert np.max(np.abs(lam - ref.lam)) < 1e-10 * alpha
    X, Xh = out["X"].cpu().numpy(), out["Xh"].cpu().numpy()
    assert np.max(np.abs(Xh.conj().T @ X - np.eye(m))) < 1e-10
    Ad = L.csr_matrix(p.A)
    nA = np.abs(Ad).sum(axis=0).max()
    rr = np.abs(Ad @ X - X * lam).sum(axis=0) / (nA * np.abs(X).sum(axis=0))
    assert rr.max() <= 1e-10
    assert out["report"]["n_solve"] == out["report"]["iters"] * 24
    # the network alone carried part of the solves (the rest fell back to ILU(0))
    assert out["report"]["n_fallback"] < out["report"]["n_solve"]
