"""Benchmark: non-Hermitian FEAST iterations per second on one MI355X.

Headline workload (default, the largest configuration): the complex-symmetric
2D operator A = -Lap_h + V - 5i W on a 1024 x 1024 grid (n = 1,048,576;
50 Gaussian wells of depth 20, absorbing ramp on the outer 10 %, B = I),
ellipse centred in the lower half-plane around its 116 lowest eigenvalues,
Ne = 24 trapezoidal nodes, m0 = 160.  Shifted systems: column-batched
GMRES(30) x 2 cycles + ILU(0) with delayed reorthogonalization on the
24 x 160 right-hand sides of a filter (the left block is conj(Y) D: complex
symmetric), residual form of the filter from the second iteration on.

A "step" is one full FEAST iteration (contour filter, B_Q, resize and
B-bi-orthonormalization, Rayleigh-Ritz, residuals).  The fast path (complex
FP32 Krylov solves, FP64 residual form and Rayleigh-Ritz) is timed over
exactly K steps after W warm-up steps, then continued to eq:res <= 1e-9 and
its eigenpairs checked against reference eigenvalues; the plain FP64 path
(the same solver in complex128) is timed for the comparison.  The 2D
convection-diffusion workload (256 x 256) and the others stay available with
--workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
# FEAST stopping threshold on eq:res for the iterative path: with GMRES inner
# solves at 0.02-0.2 relative accuracy eq:res levels off between 2e-10 and
# 2e-9 (FP64 and complex FP32 alike); 1e-9 is a residual
# ||Ax - lam x|| / (||A|| ||x||) of about 1.4e-12
EPS_ITER = 1e-9
EPS_DENSE = 1e-10   # dense batch: the residual level the throughput metric is stated at
ORTH = 2            # GMRES orthogonalization (fh_opts.orth), set by --orth
BATCH_NODES = 0     # headline workload: nodes per filter chunk (0: as many as fit), set by --batch-nodes


def _problem():
    import workloads as W
    return W.convdiff2d(N=256, bx=20.0, by=10.0, m_in=41, ne=16, m0=64, ratio=0.3, seed=2)


def _opts(fh, m0, precision, max_iter, eps, resume=0, conj_pairs=1):
    # GMRES(30), two cycles per solve, residual-form filter; the mixed path runs
    # one complex-FP32 solve per filter followed by its FP64 residual check.
    # orth = 2 (delayed reorthogonalization, two passes over the basis per
    # Krylov step) applies to the complex-FP32 and the FP64 solves alike.
    # conj_pairs = 2: real start blocks, conjugate Ritz pairs, n_e solves per
    # iteration instead of 2 n_e (real matrix, ellipse centred on the real axis).
    return fh.default_opts(m0, solver=fh.FH_SOLVER_BGMRES, precond=fh.FH_PC_ILU0, restart=30, max_restarts=2,
                           inner_tol=1e-3, precision=precision, mixed_inner_tol=1e-3, max_refine=1,
                           max_iter=max_iter, eps=eps, resume=resume, orth=ORTH, conj_pairs=conj_pairs)


def _traffic(kernel, workload="convdiff256"):
    """HBM bytes per launch of `kernel` measured with rocprofv3 counters
    (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy of known size) on the
    given workload, from profiles/hbm_traffic_<workload>.json; None when not
    measured for this kernel.  The counters are taken in their own runs; a
    kernel changed since then needs them taken again."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    k = t.get("kernels", {}).get(kernel)
    return None if k is None else k.get("bytes_per_launch")


def _start(torch, p, conj_pairs):
    """Seeded start blocks on the device (their real parts with conj_pairs = 2)."""
    Y0, Yh0 = (p.Y0.real.astype(np.complex128), p.Yh0.real.astype(np.complex128)) if conj_pairs == 2 else (p.Y0, p.Yh0)
    return torch.from_numpy(Y0).cuda(), torch.from_numpy(Yh0).cuda()


def run_path(fh, torch, handle, prob, p, precision, steps, warmup, profile=False, conj_pairs=1):
    """W warm-up iterations from the seeded start, then exactly K timed ones."""
    c = p.contour
    Y0, Yh0 = _start(torch, p, conj_pairs)
    ritz = None
    resume = 0
    if warmup > 0:
        out = fh.feast(prob, c.center, c.a, c.ratio, c.angle, c.ne, Y0, Yh0,
                       _opts(fh, p.m0, precision, warmup, 1e-300, conj_pairs=conj_pairs))
        Y0, Yh0, ritz, resume = out["Y"].contiguous(), out["Yh"].contiguous(), out["ritz"], 1
    if profile:
        handle.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = fh.feast(prob, c.center, c.a, c.ratio, c.angle, c.ne, Y0, Yh0,
                   _opts(fh, Y0.shape[1], precision, steps, 1e-300, resume, conj_pairs), ritz0=ritz)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    stats = handle.profile_stats() if profile else None
    if profile:
        handle.profile(False)
    return dt, out, stats


def solve_to_convergence(fh, torch, prob, p, precision, conj_pairs=1):
    """Untimed for the metric: a fresh solve from the seeded start to eq:res <= EPS_ITER
    (time-to-solution), then the returned eigenpairs are checked."""
    c = p.contour
    Y0, Yh0 = _start(torch, p, conj_pairs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fin = fh.feast(prob, c.center, c.a, c.ratio, c.angle, c.ne, Y0, Yh0,
                   _opts(fh, p.m0, precision, 60, EPS_ITER, conj_pairs=conj_pairs))
    torch.cuda.synchronize()
    tts = time.perf_counter() - t0
    alpha = abs(c.center) + max(c.a, c.ratio * c.a)
    exact = p.info["lam_sorted"][: p.info["m_in"]]
    lam = np.sort(fin["lam"].real)
    dl = float(np.max(np.abs(lam - exact))) / alpha if len(lam) == len(exact) else None
    A = p.A
    normA = float(np.max(np.bincount(A["colind"], weights=np.abs(A["val"]), minlength=A["n"])))
    max_res = float(np.max(fin["res"])) if len(fin["res"]) else None
    return {"converged": fin["info"] == 0, "m": int(len(fin["lam"])), "m_expected": int(len(exact)),
            "solves": int(fin["report"]["n_solve"]), "factorizations": int(fin["report"]["n_factor"]),
            "max_eq_res": max_res,
            # ||Ax - lam x||_1 / (||A||_1 ||x||_1) = eq:res * alpha / ||A||_1 for B = I
            "max_rel_residual": None if max_res is None else max_res * alpha / normA,
            "max_dlam_over_alpha": dl, "iterations": int(fin["report"]["iters"]), "time_to_solution_s": tts}


def cpu_baseline(p):
    """The oracle (SuperLU direct solves, complex128) on a bounded sample: the
    filter work of 2 of the 16 nodes (one factorization + right and left solves
    of 64 columns each), scaled to a FEAST iteration of 16 nodes."""
    from threadpoolctl import threadpool_limits
    from oracle import contour as ct
    from oracle import linsolve as L
    A = L.csr_matrix(p.A)
    z, w = ct.ellipse_nodes(p.contour.center, p.contour.a, p.contour.ratio, 0.0, 16)
    sample = 2
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        for j in range(sample):
            F = L.DirectFactor(L.shifted(A, None, z[j]))
            F.solve(p.Y0, "N")
            F.solve(p.Yh0, "H")
        dt = time.perf_counter() - t0
    t_iter = dt * 16 / sample
    return {"value": 1.0 / t_iter, "unit": "FEAST iterations/s", "cores": 1, "kind": "oracle",
            "sample": f"filter of {sample} of 16 nodes (SuperLU factorization + right and left solves of 64 "
                      f"columns, complex128, 1 thread), {dt:.1f} s, scaled x{16 // sample} to one iteration"}


PEAK_FP32_MFMA_TFLOPS = 157.3


def dense_batch(args):
    """Dense batch: 64 dense generalized problems (A = G/sqrt(n),
    B = I + 0.1 G'/sqrt(n)), n_i uniform in [256, 2048], Ne = 8, m0 = 32,
    circles whose radius is scaled with 1/sqrt(n_i) (about 23 eigenvalues
    inside each).  Fast path: one batched FEAST run (grouped complex-FP32 LU on
    MFMA + FP64 refinement to 1e-10, HIP-graph replay, steps 2-5 of all
    instances in lockstep); plain path: FP64 FEAST one instance at a time with
    direct solves.  Both to eq:res <= 1e-10 from the seeded starts."""
    import torch
    import workloads as W
    import paper_1506_04463_amd as fh

    count = args.count
    ps = W.gen_dense_batch(count=count, nmin=256, nmax=2048, ne=8, m0=32, seed=3, scaled_radius=True)
    handle = fh.Handle(0)
    probs = [fh.Problem(handle, torch.from_numpy(p.A).cuda(), torch.from_numpy(p.B).cuda()) for p in ps]
    Y0 = [torch.from_numpy(p.Y0).cuda() for p in ps]
    Yh0 = [torch.from_numpy(p.Yh0).cuda() for p in ps]
    conts = [(p.contour.center, p.contour.a, 1.0, 0.0, 8) for p in ps]
    ns = [p.n for p in ps]
    print(f"[bench] dense batch: {count} problems, n in [{min(ns)}, {max(ns)}], Ne=8, m0=32", file=sys.stderr,
          flush=True)
    # FP64 refinement of each complex-FP32 solve to the outer target (the same
    # iterations and eigenvalues as refining to 1e-12, measured); confirmed
    # exit on both paths, so that every problem returns all of its pairs
    # (the literal exit can stop while spurious flags hide some of them)
    o = fh.default_opts(32, eps=EPS_DENSE, max_iter=60, precision=fh.FH_PREC_MIXED, inner_tol=EPS_DENSE, max_refine=6,
                        graph=1, confirm=1)
    # warm-up on a small batch (autotuner, code objects)
    fh.feast_batched(probs[:2], conts[:2], Y0[:2], Yh0[:2], o)
    handle.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, outs = fh.feast_batched(probs, conts, Y0, Yh0, o)
    torch.cuda.synchronize()
    t_fast = time.perf_counter() - t0
    stats = handle.profile_stats()
    handle.profile(False)
    iters = [q["report"]["iters"] for q in outs]
    ms = [len(q["lam"]) for q in outs]
    print(f"[bench] batched c64+refinement: {t_fast:.2f} s, status {rc}, iterations {min(iters)}-{max(iters)}, "
          f"eigenpairs {sum(ms)}", file=sys.stderr, flush=True)
    rhs = sum(2 * 8 * 32 * it for it in iters)
    plain = None
    if not args.no_fp64:
        o64 = fh.default_opts(32, eps=EPS_DENSE, max_iter=60, confirm=1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lam64 = []
        for i in range(count):
            c = conts[i]
            r = fh.feast(probs[i], c[0], c[1], 1.0, 0.0, 8, Y0[i], Yh0[i], o64)
            lam64.append(r["lam"])
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - t0
        same = [len(a["lam"]) == len(b) and len(b) > 0 for a, b in zip(outs, lam64)]
        dl = max([float(np.max(np.abs(np.sort_complex(a["lam"]) - np.sort_complex(b)) / np.abs(np.sort_complex(b))))
                  for a, b, ok in zip(outs, lam64, same) if ok] or [float("inf")])
        plain = {"seconds": t_plain, "max_rel_dlam_vs_fast": dl, "instances_same_count": int(sum(same))}
        print(f"[bench] plain FP64 one at a time: {t_plain:.2f} s, max |dlam|/|lam| {dl:.2e}", file=sys.stderr,
              flush=True)
    mf = {k: v for k, v in stats.items() if k.startswith("ggemm_c64")}
    roof = None
    if mf:
        name, st = max(mf.items(), key=lambda kv: kv[1]["ms"])
        tf = st["flops"] / (st["ms"] * 1e-3) / 1e12
        roof = {"bound": "mfma", "kernel": name, "achieved": tf, "peak": PEAK_FP32_MFMA_TFLOPS, "unit": "TFLOP/s",
                "frac": tf / PEAK_FP32_MFMA_TFLOPS, "traffic": None, "avg_ms": st["ms"] / st["count"],
                "launches": st["count"], "flops_per_launch": st["flops"] / st["count"]}
    kernels = {k: {"ms_total": v["ms"], "count": v["count"],
                   "TFLOPs": (v["flops"] / (v["ms"] * 1e-3) / 1e12) if v.get("flops") else None}
               for k, v in sorted(stats.items(), key=lambda kv: -kv[1]["ms"])[:8]}
    line = {"metric": "dense batch: time to solution and shifted-solve RHS/s at eq:res <= 1e-10",
            "value": rhs / t_fast, "unit": "RHS/s", "n_gpus": 1, "steps": 1, "warmup": 1,
            "ms_per_step": 1000.0 * t_fast, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "c64 LU/solves + c128 refinement/Rayleigh-Ritz", "data": "synthetic",
            "config": {"workload": f"{count} dense generalized problems n in [256,2048], Ne=8, m0=32"},
            "seconds_fast": t_fast, "status": rc, "iterations": [min(iters), max(iters)], "eigenpairs": sum(ms),
            "plain_fp64": plain, "speedup_vs_fp64": None if plain is None else plain["seconds"] / t_fast,
            "roofline": roof, "kernels": kernels}
    print(json.dumps(line))


def learned3d(args):
    """Fourth configuration's operator (64^3 convection-diffusion-reaction,
    seeded smooth convection field |v| <= 30, reaction 5): cost of one
    application of the 3x3x3 network (8 input channels: residual, shift,
    side, the three field components) to a block of columns, against one
    ILU(0) apply and one SpMM of the same block, complex FP32, kernel times
    from the library's HIP-event profiler."""
    import torch
    import workloads as W
    import paper_1506_04463_amd as fh
    N, m = 64, args.columns
    v = W.smooth_field3d(N, 1)
    A = W.convdiff3d_csr(N, v)
    h = fh.Handle(0)
    prob = fh.Problem(h, fh.CSR(torch.from_numpy(A["rowptr"]).cuda(), torch.from_numpy(A["colind"]).cuda(),
                                torch.from_numpy(A["val"]).cuda(), A["n"]))
    hh = 1.0 / (N + 1)
    net = fh.Net(h, N, N, fields=v.reshape(3, -1) / 30.0, alpha=300.0, out_scale=hh * hh / 6.0, seed=1, nz=N)
    fh.set_net(prob, net)
    z = np.array([80.0 + 40.0j, 80.0 + 40.0j])
    B = torch.randn((2, A["n"], m), dtype=torch.complex128, device="cuda")
    res = {}
    for name, pc in (("learned", fh.FH_PC_LEARNED), ("learned_bf16", fh.FH_PC_LEARNED), ("ilu0", fh.FH_PC_ILU0)):
        net.set_activations(name == "learned_bf16")
        o = fh.default_opts(m, precond=pc, restart=4, max_restarts=1, inner_tol=1e-300, precision=fh.FH_PREC_MIXED,
                            mixed_inner_tol=1e-300, max_refine=1, fallback=fh.FH_PC_NONE, save_factors=1)
        fh.shifted_solve(prob, z, [0, 1], B, o)          # warm-up (factors, code objects)
        h.profile(True)
        fh.shifted_solve(prob, z, [0, 1], B, o)
        st = h.profile_stats()
        h.profile(False)
        res[name] = {k: {"ms_avg": v_["ms"] / v_["count"], "count": v_["count"],
                         "TFLOPs": v_["flops"] / (v_["ms"] * 1e-3) / 1e12 if v_["flops"] else None}
                     for k, v_ in st.items() if k.startswith(("net_", "ilu_apply", "spmm"))}
    cols = 2 * m
    fw = res["learned"].get("net_forward")
    line = {"metric": "learned preconditioner apply cost, 64^3 grid", "columns_per_apply": cols,
            "gflop_per_column": None if fw is None else fw["TFLOPs"] * fw["ms_avg"] * 1e-3 * 1e12 / cols / 1e9,
            "net_forward": fw, "net_forward_bf16_activations": res["learned_bf16"].get("net_forward"),
            "ilu_apply": res["ilu0"].get("ilu_apply_c64"), "spmm": res["ilu0"].get("spmm_c64"),
            "peak_bf16_mfma_tflops": 2500.0}
    print(json.dumps(line))


def csym(args):
    """Complex-symmetric 2D operator A = -Lap_h + V - i eta W (256 x 256 grid,
    n = 65,536, A = A^T; 50 Gaussian wells, absorbing ramp), circle around the
    40 lowest eigenvalues (well-bound states, located once on the CPU with
    scipy's shift-invert ARPACK), Ne = 16, m0 = 64, mixed path.  FEAST with
    the left subspace taken as the conjugate of the right one (opts.sym = 1:
    Ne solves per iteration) against the general algorithm (2 Ne solves):
    both solved to eq:res <= 1e-9 from the same seeded start (eigenvalues
    compared), and iterations 2..K+1 (K <= 2) of that start timed.""" 
    import scipy.sparse as sps
    import scipy.sparse.linalg as spla
    import torch
    import workloads as W
    import paper_1506_04463_amd as fh
    A = W.schrodinger2d_csr(256)
    n = A["n"]
    Asp = sps.csr_matrix((A["val"], A["colind"], A["rowptr"]), shape=(n, n))
    # the 48 lowest eigenvalues (nearest a point below the spectrum); the circle
    # spans the 40 lowest, where the shifted systems are nearly definite
    ev = spla.eigs(Asp, k=48, sigma=-60.0, return_eigenvectors=False, tol=1e-10)
    ev = ev[np.argsort(ev.real)]
    c = 0.5 * (ev[0].real + ev[39].real)
    r = 0.5 * (abs(ev[39] - c) + abs(ev[40] - c))
    target = complex(c)
    h = fh.Handle(0)
    prob = fh.Problem(h, fh.CSR(torch.from_numpy(A["rowptr"]).cuda(), torch.from_numpy(A["colind"]).cuda(),
                                torch.from_numpy(A["val"]).cuda(), n))
    m0, ne = 64, 16
    Y0 = torch.from_numpy(W.subspace(n, m0, 7)).cuda()
    Yh0 = torch.conj(Y0).resolve_conj().contiguous()
    print(f"[bench] csym: n={n} circle {target:.4f} r={r:.4g}, {int(np.sum(np.abs(ev - target) < r))} of the 48 "
          f"lowest eigenvalues inside", 
          file=sys.stderr, flush=True)

    def opts(sym, max_iter, eps, resume=0):
        o = _opts(fh, m0, fh.FH_PREC_MIXED, max_iter, eps, resume)
        o.sym = sym
        return o

    # time to solution from the seeded start first; then iterations 2..K+1 of
    # the same start timed (the general path's eigendecomposition of B_Q fails
    # from its 4th-5th iteration on this problem, an open issue: it is
    # reported, and the timed iterations stay before it)
    K = max(1, min(args.steps, 2))
    res = {}
    for sym in (1, 0):
        r_ = {"solves_per_iteration": ne * (1 if sym else 2)}
        try:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fin = fh.feast(prob, target, r, 1.0, 0.0, ne, Y0, Yh0, opts(sym, 60, EPS_ITER))
            torch.cuda.synchronize()
            r_.update({"converged": fin["info"] == 0, "iterations": int(fin["report"]["iters"]),
                       "m": int(len(fin["lam"])), "time_to_solution_s": time.perf_counter() - t0,
                       "lam": np.sort_complex(fin["lam"])})
        except fh.FeastError as e:
            r_.update({"converged": False, "error": str(e), "lam": np.zeros(0, complex)})
        out = fh.feast(prob, target, r, 1.0, 0.0, ne, Y0, Yh0, opts(sym, 1, 1e-300))
        Y, Yh, ritz = out["Y"].contiguous(), out["Yh"].contiguous(), out["ritz"]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fh.feast(prob, target, r, 1.0, 0.0, ne, Y, Yh, opts(sym, K, 1e-300, 1), ritz0=ritz)
        torch.cuda.synchronize()
        r_["ms_per_iteration"] = 1000.0 * (time.perf_counter() - t0) / K
        res[sym] = r_
        print(f"[bench] csym sym={sym}: {r_['ms_per_iteration']:.1f} ms/iteration; to eq:res <= {EPS_ITER:g}: "
              + (f"{r_['time_to_solution_s']:.2f} s, {r_['iterations']} iterations, m = {r_['m']}"
                 if "error" not in r_ else r_["error"]), file=sys.stderr, flush=True)
    # eigenvalue-count estimate: 64 Rademacher probes, right solves only
    zc, wc = fh.contour_nodes(target, r, 1.0, 0.0, ne)
    V = torch.from_numpy(np.random.default_rng(13).choice([-1.0, 1.0], size=(n, m0)).astype(np.complex128)).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    est, _ = fh.count_estimate(prob, zc, wc, V, opts(0, 1, EPS_ITER))
    torch.cuda.synchronize()
    count = {"estimate": est.real, "estimate_imag": est.imag, "probes": m0, "seconds": time.perf_counter() - t0,
             "eigenvalues_found": res[1].get("m")}
    print(f"[bench] csym count estimate: {est.real:.2f} (found {count['eigenvalues_found']}), "
          f"{count['seconds']:.2f} s", file=sys.stderr, flush=True)
    la, lb = res[1].pop("lam"), res[0].pop("lam")
    same = len(la) == len(lb) and len(la) > 0
    dl = float(np.max(np.abs(la - lb)) / (abs(target) + r)) if same else None
    line = {"metric": "FEAST iterations/s, complex symmetric (left subspace = conj(right)) vs general",
            "value": 1000.0 / res[1]["ms_per_iteration"], "unit": "FEAST iterations/s", "n_gpus": 1,
            "steps": K, "warmup": 1, "ms_per_step": res[1]["ms_per_iteration"],
            "higher_is_better": True, "dtype": "c64 inner solves + c128 refinement/Rayleigh-Ritz",
            "data": "synthetic",
            "config": {"workload": "complex-symmetric Schroedinger-type 256x256 (n=65536), Ne=16, m0=64, "
                                   "GMRES(30)x2 + ILU(0), c64 solves + FP64 residual form"},
            "sym": res[1], "general": res[0],
            "speedup_per_iteration": res[0]["ms_per_iteration"] / res[1]["ms_per_iteration"],
            "same_eigenvalue_count": same, "max_dlam_over_alpha": dl, "count_estimate": count}
    print(json.dumps(line))


def contour_grid(args):
    """The paper's multi-contour experiment on synthetic data: a 4000 x 4000
    dense matrix with its eigenvalues area-uniform in the unit disk, six
    squares (16 nodes, 4 trapezoid intervals per side) and six circles
    (16 nodes) at the same six centres, m0 = 200.  Three FEAST iterations of
    all twelve contours in one batched call (complex-FP32 grouped LU on MFMA
    + FP64 refinement, factorizations kept) against three iterations of FP64
    FEAST with direct solves one contour at a time; the Ritz values are
    matched against the prescribed eigenvalues.  The work per iteration is
    timed rather than the time to convergence: with nodes this close to the
    eigenvalues of a non-normal matrix the complex-FP32 factors are too
    ill-conditioned for the refinement to take eq:res of every inside pair
    below 1e-7 (the batched run stops at its iteration limit on all twelve
    contours, also with the solves refined to 1e-10), while FP64 FEAST meets
    eps = 1e-7 on nine of the twelve within 4-8 iterations.
    Sizes: half-side 0.13 / radius 0.17 (about 85 / 115 eigenvalues), each
    moved within +-10 % into the widest gap of the eigenvalue distances so
    that no eigenvalue sits on a contour."""
    import torch
    import workloads as W
    import paper_1506_04463_amd as fh
    n, m0, ne = 4000, 200, 16
    t0 = time.perf_counter()
    A, lam = W.dense_unit_disk(n, 12)
    print(f"[bench] contour grid: n={n} matrix built in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)

    def gap(d, nominal):
        d = np.sort(d)
        best = None
        for a, b in zip(d[:-1], d[1:]):
            if 0.9 * nominal <= a and b <= 1.1 * nominal and (best is None or b / a > best[0]):
                best = (b / a, np.sqrt(a * b))
        return nominal if best is None else best[1]

    centres = [x + 1j * y for y in (0.3, -0.3) for x in (-0.5, 0.0, 0.5)]
    conts, truth, names = [], [], []
    for c in centres:
        h = gap(np.maximum(np.abs((lam - c).real), np.abs((lam - c).imag)), 0.13)
        sq = np.array([c - h - 1j * h, c + h - 1j * h, c + h + 1j * h, c - h + 1j * h])
        x, y = (lam - c).real, (lam - c).imag
        conts.append((0.0, 1.0, 1.0, 0.0, ne, sq))
        truth.append(lam[(np.abs(x) < h) & (np.abs(y) < h)])
        names.append(f"square {c:.2f} h={h:.4f}")
    for c in centres:
        r = gap(np.abs(lam - c), 0.17)
        conts.append((c, r, 1.0, 0.0, ne))
        truth.append(lam[np.abs(lam - c) < r])
        names.append(f"circle {c:.2f} r={r:.4f}")
    h = fh.Handle(0)
    prob = fh.Problem(h, torch.from_numpy(A).cuda())
    k = len(conts)
    Y0s = [torch.from_numpy(W.subspace(n, m0, 900 + i)).cuda() for i in range(k)]
    Yh0s = [torch.from_numpy(W.subspace(n, m0, 950 + i)).cuda() for i in range(k)]
    K = 3        # timed iterations (the mixed path does not reach eps here: see above)
    o = fh.default_opts(m0, precision=fh.FH_PREC_MIXED, eps=1e-300, max_iter=K, inner_tol=EPS_DENSE,
                        max_refine=6, graph=1)
    # warm-up: one iteration of one contour (autotuner, code objects)
    o1 = fh.default_opts(m0, precision=fh.FH_PREC_MIXED, eps=1e-300, max_iter=1, inner_tol=EPS_DENSE,
                         max_refine=6, graph=1)
    fh.feast_batched([prob], conts[:1], Y0s[:1], Yh0s[:1], o1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, outs = fh.feast_batched([prob] * k, conts, Y0s, Yh0s, o)
    torch.cuda.synchronize()
    t_fast = time.perf_counter() - t0
    per = []
    for name, out, t in zip(names, outs, truth):
        rr = out["ritz"].cpu().numpy()
        rs = out["ritz_res"]
        # inside Ritz values within 1e-8 of a prescribed eigenvalue of the contour
        close = [np.min(np.abs(t - x)) < 1e-8 for x in rr] if len(t) else []
        per.append({"contour": name, "m_true": int(len(t)), "ritz_matching_true_1e-8": int(np.sum(close)),
                    "median_res": float(np.median(rs)) if len(rs) else None})
    print(f"[bench] contour grid batched c64+refinement: {K} iterations of all {k} contours in {t_fast:.2f} s "
          f"({t_fast / K:.2f} s per iteration); Ritz values matching a prescribed eigenvalue to 1e-8: "
          f"{sum(p_['ritz_matching_true_1e-8'] for p_ in per)} of {sum(len(t) for t in truth)}",
          file=sys.stderr, flush=True)
    plain = None
    if not args.no_fp64:
        o64 = fh.default_opts(m0, precision=fh.FH_PREC_FP64, eps=1e-300, max_iter=K)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        errors = 0
        for i, c in enumerate(conts):
            try:
                fh.feast(prob, c[0], c[1], c[2], c[3], c[4], Y0s[i], Yh0s[i], o64,
                         polygon=c[5] if len(c) > 5 else None)
            except fh.FeastError:
                errors += 1
        torch.cuda.synchronize()
        plain = {"seconds": time.perf_counter() - t0, "iterations_per_contour": K, "errors": errors}
        print(f"[bench] contour grid FP64 one contour at a time: {K} iterations each in {plain['seconds']:.2f} s"
              + (f" ({errors} contours failed)" if errors else ""), file=sys.stderr, flush=True)
    tts = None
    if args.tts:
        # to eq:res <= 1e-7, the batched complex-FP32 path: systems whose FP32
        # refinement stalls are solved with FP64 factors.  Exit: --confirm 1
        # (confirmed by a second passing iteration) or 2 (the paper's exit
        # iteration, every converged inside pair returned)
        ot = fh.default_opts(m0, precision=fh.FH_PREC_MIXED, eps=1e-7, max_iter=40, inner_tol=EPS_DENSE,
                             max_refine=6, graph=1, confirm=args.confirm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc2, outs2 = fh.feast_batched([prob] * k, conts, Y0s, Yh0s, ot)
        torch.cuda.synchronize()
        tts = {"seconds": time.perf_counter() - t0, "status": rc2, "confirm": args.confirm, "contours": []}
        for name, out, t in zip(names, outs2, truth):
            lamv = out["lam"]
            d = np.abs(lamv[:, None] - t[None, :]) if len(lamv) and len(t) else np.zeros((0, 0))
            tts["contours"].append({"contour": name, "info": int(out["info"]),
                                    "iterations": int(out["report"]["iters"]), "m": int(len(lamv)),
                                    "m_true": int(len(t)),
                                    "max_dlam": float(d.min(axis=1).max()) if d.size else None,
                                    "fp64_fallback_systems": int(out["report"]["n_fallback"])})
        nconv = sum(1 for c_ in tts["contours"] if c_["info"] == 0 and c_["m"] == c_["m_true"])
        print(f"[bench] contour grid to eq:res <= 1e-7 (batched c64 + FP64 fallback, confirm={args.confirm}): "
              f"{tts['seconds']:.1f} s, "
              f"{nconv} of {k} contours converged with all their eigenvalues", file=sys.stderr, flush=True)
    line = {"metric": "multi-contour FEAST (12 contours, one matrix): FEAST iterations of all contours per second",
            "value": K / t_fast, "unit": "batched iterations/s", "n_gpus": 1, "steps": K, "warmup": 1,
            "ms_per_step": 1000.0 * t_fast / K, "higher_is_better": True, "dtype": "c64 LU/solves + c128 refinement/Rayleigh-Ritz",
            "data": "synthetic",
            "config": {"workload": "4000x4000 dense, eigenvalues uniform in the unit disk, 6 squares + 6 circles, "
                                   "Ne=16, m0=200"},
            "status": rc, "contours": per, "plain_fp64": plain, "time_to_solution": tts,
            "speedup_vs_fp64": None if plain is None else plain["seconds"] / t_fast}
    print(json.dumps(line))


def copy_calibration():
    """A plain device copy of a known size (1 GiB read, 1 GiB written), run
    three times: the reference for scaling the FETCH_SIZE / WRITE_SIZE
    counters of rocprofv3 into HBM bytes.  Then the bandwidth a plain copy
    reaches (4 GiB blocks, timed with events, read + written bytes): the
    practical ceiling beside the 8 TB/s peak."""
    import torch
    nbytes = 1 << 30
    x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    big = 4 << 30
    a = torch.ones(big // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 10
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "launches": 3,
                      "copy_4gib_ms": ms, "copy_GBps_read_plus_write": 2 * big / (ms * 1e-3) / 1e9,
                      "frac_of_8TBps": 2 * big / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS}))


# --------------------------------------------------------------------------
# headline workload: the complex-symmetric 2D operator on the 1024 x 1024 grid
# --------------------------------------------------------------------------
C5_GOLDEN = os.path.join(ROOT, "tests", "golden", "schrodinger2d_N1024_lowest.json")


def _c5_eigs(path):
    if path.endswith(".npy"):
        return np.load(path)
    with open(path) as f:
        d = json.load(f)
    return np.array([complex(a, b) for a, b in d["eigenvalues"]])


def _c5_opts(fh, m0, precision, max_iter, eps, resume=0, precond=None):
    # GMRES(30), two cycles per solve, residual-form filter (the FP64
    # eigen-residual R = A Y - Y Lambda is the right-hand side of every filter
    # from the second FEAST iteration on, so the outer FEAST iteration refines
    # the complex-FP32 solves in FP64); one FP64 residual check per solve
    # (max_refine = 1: no inner correction step); delayed reorthogonalization
    # (DCGS2) on both precisions; right solves only with the left block
    # conj(Y) D (complex symmetric, opts.sym = 1) on both precisions
    return fh.default_opts(m0, solver=fh.FH_SOLVER_BGMRES, precond=fh.FH_PC_ILU0 if precond is None else precond,
                           restart=30, max_restarts=2, inner_tol=1e-3, precision=precision, mixed_inner_tol=1e-3,
                           max_refine=1, max_iter=max_iter, eps=eps, resume=resume, orth=2, sym=1,
                           batch_nodes=BATCH_NODES)


def _c5_cpu_baseline(p, sample_cols=8):
    """The oracle on the host cores: one worker process per quadrature node
    (as many as there are cores, at most Ne), each factorizing (z_j - A) with
    SuperLU and solving a sample of right-hand-side columns with the oracle's
    direct solve; scaled to a FEAST iteration's filter (Ne nodes, m0 right
    solves each -- the same right-solves-only work as the GPU path)."""
    import concurrent.futures as cf
    import multiprocessing as mp
    ne, m0 = p.contour.ne, p.m0
    cores = min(ne, max(1, len(os.sched_getaffinity(0))), int(os.environ.get("OMP_NUM_THREADS", "64")))
    z = _c5_nodes(p)
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with cf.ProcessPoolExecutor(max_workers=cores, mp_context=ctx) as ex:
        futs = [ex.submit(_c5_cpu_node, p.info["N"], complex(z[j]), sample_cols) for j in range(cores)]
        res = [f.result() for f in futs]
    wall = time.perf_counter() - t0
    t_fact = max(r[0] for r in res)
    t_col = max(r[1] for r in res) / sample_cols
    per_node = t_fact + t_col * m0
    rounds = -(-ne // cores)
    t_iter = rounds * per_node
    return {"value": 1.0 / t_iter, "unit": "FEAST iterations/s", "cores": cores, "kind": "oracle",
            "sample": f"{cores} nodes in parallel processes (one per core): SuperLU factorization of z_j - A "
                      f"({t_fact:.1f} s) and {sample_cols} right-hand-side columns ({t_col:.2f} s each), "
                      f"{wall:.1f} s wall; scaled to {ne} nodes x {m0} columns ({rounds} rounds of "
                      f"{per_node:.1f} s), the filter only"}


def _c5_nodes(p):
    from oracle import contour as ct
    c = p.contour
    z, _ = ct.ellipse_nodes(c.center, c.a, c.ratio, c.angle, c.ne)
    return z


def _c5_cpu_node(N, zj, cols):
    import workloads as W
    from threadpoolctl import threadpool_limits
    from oracle import linsolve as L
    with threadpool_limits(limits=1):
        A = L.csr_matrix(W.schrodinger2d_csr(N))
        t0 = time.perf_counter()
        F = L.DirectFactor(L.shifted(A, None, zj))
        t1 = time.perf_counter()
        F.solve(W.subspace(A.shape[0], cols, 77), "N")
        t2 = time.perf_counter()
    return t1 - t0, t2 - t1


def schrodinger(args):
    """Headline workload: A = -Lap_h + V - 5i W on the 1024 x 1024 grid
    (n = 1,048,576, complex symmetric), ellipse centred in the lower
    half-plane around its 116 lowest eigenvalues, Ne = 24, m0 = 160.  The fast
    path (complex-FP32 GMRES(30) x 2 + ILU(0), FP64 residual form) and the
    plain FP64 path (the same solver in complex128) are timed per FEAST
    iteration; the fast run then continues to eq:res <= 1e-9 and its
    eigenpairs are checked against the reference eigenvalues (ARPACK
    shift-invert, tests/golden) and for X^H X = I, Xh = conj(X) and the
    1-norm residual of the eigenpair gate."""
    import torch
    import workloads as W
    import paper_1506_04463_amd as fh

    N = args.grid
    eigs = _c5_eigs(args.eigs or C5_GOLDEN)
    p = W.schrodinger2d(N=N, eigs=eigs, m0=160, ne=24)
    c = p.contour
    A = p.A
    handle = fh.Handle(0)
    prob = fh.Problem(handle, fh.CSR(torch.from_numpy(A["rowptr"]).cuda(), torch.from_numpy(A["colind"]).cuda(),
                                     torch.from_numpy(A["val"]).cuda(), p.n))
    alpha = abs(c.center) + max(c.a, c.ratio * c.a)
    print(f"[bench] {p.name}: n={p.n} nnz={len(A['colind'])} ellipse c={c.center:.4f} a={c.a:.4f} ratio={c.ratio} "
          f"({p.info['m_in']} reference eigenvalues inside) Ne={c.ne} m0={p.m0}", file=sys.stderr, flush=True)
    ne = c.ne

    def feast(Y, Yh, o, ritz=None):
        return fh.feast(prob, c.center, c.a, c.ratio, c.angle, ne, Y, Yh, o, ritz0=ritz)

    Y0 = torch.from_numpy(p.Y0).cuda()
    Yh0 = torch.from_numpy(p.Yh0).cuda()
    # fast path: warm-up iterations, K timed ones, then on to convergence
    t_all = time.perf_counter()
    done_it, resume = 0, 0
    Y, Yh, ritz = Y0, Yh0, None
    if args.warmup > 0:
        out = feast(Y0, Yh0, _c5_opts(fh, p.m0, fh.FH_PREC_MIXED, args.warmup, 1e-300))
        done_it = out["report"]["iters"]
        print(f"[bench] fast path: {done_it} warm-up iteration(s), {time.perf_counter() - t_all:.1f} s",
              file=sys.stderr, flush=True)
        Y, Yh, ritz, resume = out["Y"].contiguous(), out["Yh"].contiguous(), out["ritz"], 1
    handle.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = feast(Y, Yh, _c5_opts(fh, Y.shape[1], fh.FH_PREC_MIXED, args.steps, 1e-300, resume), ritz)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    stats = handle.profile_stats()
    handle.profile(False)
    ms_mx = 1000.0 * dt / args.steps
    rep_mx = out["report"]
    done_it += rep_mx["iters"]
    print(f"[bench] fast path: {ms_mx:.1f} ms per FEAST iteration ({args.steps} timed)", file=sys.stderr, flush=True)
    valid = None
    if not args.no_validate:
        Y, Yh, ritz = out["Y"].contiguous(), out["Yh"].contiguous(), out["ritz"]
        t1 = time.perf_counter()
        fin = feast(Y, Yh, _c5_opts(fh, Y.shape[1], fh.FH_PREC_MIXED, args.max_iter, EPS_ITER, 1), ritz)
        torch.cuda.synchronize()
        valid = _c5_validate(fh, torch, prob, p, fin, eigs, alpha)
        valid["iterations"] = done_it + fin["report"]["iters"]
        valid["time_to_solution_s"] = time.perf_counter() - t_all
        print(f"[bench] validation: {json.dumps(valid)}", file=sys.stderr, flush=True)
    del Y, Yh, out
    if valid is not None:
        del fin
    plain = None
    if not args.no_fp64:
        torch.cuda.empty_cache()
        # the same iterations as the fast path: W warm-up, then K timed
        K64 = args.steps if args.fp64_steps is None else max(1, args.fp64_steps)
        Y6, Yh6, r6, res6 = Y0, Yh0, None, 0
        if args.warmup > 0:
            o64 = feast(Y0, Yh0, _c5_opts(fh, p.m0, fh.FH_PREC_FP64, args.warmup, 1e-300))
            Y6, Yh6, r6, res6 = o64["Y"].contiguous(), o64["Yh"].contiguous(), o64["ritz"], 1
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        o64 = feast(Y6, Yh6, _c5_opts(fh, Y6.shape[1], fh.FH_PREC_FP64, K64, 1e-300, res6), r6)
        torch.cuda.synchronize()
        dt64 = time.perf_counter() - t0
        del Y6, Yh6
        ms64 = 1000.0 * dt64 / K64
        plain = {"ms_per_step": ms64, "steps": K64, "warmup": args.warmup, "value": 1000.0 / ms64,
                 "inner_steps_last": o64["report"]["inner_steps"]}
        print(f"[bench] plain FP64: {ms64:.1f} ms per FEAST iteration ({K64} timed after {args.warmup} warm-up)",
              file=sys.stderr, flush=True)
    dom = max(stats.items(), key=lambda kv: kv[1]["ms"])
    name, st = dom
    achieved = st["bytes"] / (st["ms"] * 1e-3) / 1e9
    roof = {"bound": "hbm", "kernel": name, "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS,
            "traffic": _traffic(name, f"schrodinger{N}") if N == 1024 else None,
            "avg_ms": st["ms"] / st["count"],
            "launches": st["count"], "bytes_per_launch": st["bytes"] / st["count"],
            "share_of_step": st["ms"] / (args.steps * ms_mx)}
    kernels = {k: {"ms_total": v["ms"], "count": v["count"], "share": v["ms"] / (args.steps * ms_mx),
                   "GBps": v["bytes"] / (v["ms"] * 1e-3) / 1e9 if v["bytes"] else None,
                   "frac_hbm": (v["bytes"] / (v["ms"] * 1e-3) / 1e9 / PEAK_HBM_GBS) if v["bytes"] else None}
               for k, v in sorted(stats.items(), key=lambda kv: -kv[1]["ms"])[:10]}
    cpu = None if args.no_cpu else _c5_cpu_baseline(p)
    rhs = ne * p.m0
    line = {
        "metric": "FEAST iterations/sec & shifted-solve RHS/s at residual <=1e-10 vs plain FP64",
        "value": 1000.0 / ms_mx, "unit": "FEAST iterations/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_mx, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "c64 (Krylov solves) + f64/c128 (residual form, Rayleigh-Ritz)",
        "data": "synthetic",
        "config": {"workload": f"complex-symmetric -Lap+V-5iW {N}x{N} (n={p.n}, nnz={len(A['colind'])}), "
                               f"50 wells, ellipse in the lower half-plane around {p.info['m_in']} eigenvalues, "
                               f"Ne={ne}, m0={p.m0}",
                   "solver": "GMRES(30) x 2 cycles + ILU(0), DCGS2, right solves only (sym), residual form",
                   "rhs_per_iteration": rhs},
        # the filter's solves run a fixed Krylov budget, not to a tolerance:
        # this rate counts right-hand sides processed, not solved to 1e-10
        "rhs_per_s_fixed_budget": rhs * 1000.0 / ms_mx,
        "rhs_solve": f"{ne} x {p.m0} right-hand sides per iteration, each a fixed budget of 2 GMRES(30) cycles "
                     f"(no per-solve tolerance); worst relative residual of the last timed filter "
                     f"{rep_mx['inner_relres']:.2e}, relative to the residual-form right-hand side.  The "
                     f"eigenpairs are held to the FEAST exit, eq:res <= {EPS_ITER:g} (see validity)",
        "plain_fp64": plain,
        "speedup_vs_fp64": None if plain is None else plain["ms_per_step"] / ms_mx,
        "validity": valid, "roofline": roof, "kernels": kernels,
        "hbm_target_0_6": _hbm_target(kernels), "cpu_baseline": cpu}
    print(json.dumps(line))


def _hbm_target(kernels, target=0.6):
    """The Krylov kernels (Gram-Schmidt passes, sparse products, ILU(0)
    sweeps and layout moves) among the listed ones, split by whether their
    algorithmic bytes reach `target` of the 8 TB/s HBM peak."""
    out = {"target": target, "met": {}, "below": {}}
    for k, v in kernels.items():
        if v.get("frac_hbm") is None or not k.startswith(("dcgs_", "spmm", "ilu_", "blk_perm", "cgs_")):
            continue
        out["met" if v["frac_hbm"] >= target else "below"][k] = round(v["frac_hbm"], 3)
    return out


def _c5_validate(fh, torch, prob, p, fin, eigs, alpha):
    """Returned eigenpairs against the reference eigenvalues inside the
    contour (count and complex distance), X^H X = I, Xh parallel to conj(X)
    and the 1-norm residual ||A x - lam x||_1 / (||A||_1 ||x||_1) of both
    sides, with A x from the library's sparse product."""
    c = p.contour
    u = (eigs - c.center) * np.exp(-1j * c.angle)
    ref_in = eigs[(u.real / c.a) ** 2 + (u.imag / (c.ratio * c.a)) ** 2 < 1.0]
    lam = fin["lam"]
    m = len(lam)
    out = {"converged": fin["info"] == 0, "m": m, "m_reference_inside": int(len(ref_in)),
           "m_s": fin["report"]["m_s"]}
    if m == 0:
        return out
    d = np.abs(lam[:, None] - ref_in[None, :]).min(axis=1)
    out["max_dlam_over_alpha"] = float(d.max() / alpha)
    X, Xh = fin["X"], fin["Xh"]
    G = (Xh.conj().T @ X).cpu().numpy()
    out["max_abs_XhX_minus_I"] = float(np.max(np.abs(G - np.eye(m))))
    cosang = (torch.abs((torch.conj(X) * torch.conj(Xh)).sum(0)) /
              (torch.linalg.vector_norm(X, dim=0) * torch.linalg.vector_norm(Xh, dim=0))).cpu().numpy()
    out["min_cos_Xh_conjX"] = float(cosang.min())
    A = p.A
    normA = float(np.max(np.bincount(A["colind"], weights=np.abs(A["val"]), minlength=A["n"])))
    worst = 0.0
    for side, V, lv in ((0, X, lam), (1, Xh, np.conj(lam))):
        for k0 in range(0, m, 32):
            k1 = min(m, k0 + 32)
            blk = V[:, k0:k1].contiguous()
            AX = -fh.shifted_apply(prob, side, np.zeros(1), blk.unsqueeze(0))[0]        # A x (or A^H x)
            lt = torch.from_numpy(np.ascontiguousarray(lv[k0:k1])).to(blk.device)
            r = torch.abs(AX - blk * lt[None, :]).sum(0) / (normA * torch.abs(blk).sum(0))
            worst = max(worst, float(r.max()))
    out["max_rel_residual"] = worst
    out["max_eq_res"] = float(np.max(fin["res"]))
    return out


# --------------------------------------------------------------------------
# fourth configuration: 3D convection-diffusion-reaction with the learned
# preconditioner inside FEAST
# --------------------------------------------------------------------------
C4_TRAIN_FIELDS = range(4001, 4033)


def convdiff3d_learned(args):
    """-Lap u + v.grad u + 5u on the 64^3 grid (n = 262,144) with the
    held-out convection field (seed 4000), ellipse around its lowest ~64
    eigenvalues, Ne = 16, m0 = 96.  A 3x3x3 network (8 inputs: residual,
    shift, side, the field v/30; 16 / 16 / 2 channels) is trained on the GPU on
    (residual, error) pairs harvested from plain GMRES on the operators of 32
    other seeded fields (4001-4032), then used as the flexible preconditioner
    of FGMRES(30) x 2 inside FEAST (ILU(0) fallback).  FEAST is run to
    eq:res <= 1e-9 with each preconditioner -- learned, ILU(0), Jacobi, none --
    and the iterations, time per iteration, time to solution and eigenvalues
    (against the reference, tests/golden) are reported; the unpreconditioned
    FP64 solve of fresh systems with known solutions judges the network's
    error."""
    import torch
    import workloads as W
    import paper_1506_04463_amd as fh
    from paper_1506_04463_amd import learned

    N = args.grid3d
    eigs = _c5_eigs(args.eigs or os.path.join(ROOT, "tests", "golden", f"convdiff3d_N{N}_lowest.json"))
    p = W.convdiff3d(N=N, field_seed=4000, eigs=eigs, m_target=64, ne=16, m0=96)
    c = p.contour
    h = fh.Handle(0)

    def csr(A):
        return fh.CSR(torch.from_numpy(A["rowptr"]).cuda(), torch.from_numpy(A["colind"]).cuda(),
                      torch.from_numpy(A["val"]).cuda(), A["n"])

    prob = fh.Problem(h, csr(p.A))
    alpha = abs(c.center) + max(c.a, c.ratio * c.a)
    hh = 1.0 / (N + 1)
    z, _ = fh.contour_nodes(c.center, c.a, c.ratio, 0.0, c.ne)
    print(f"[bench] {p.name}: n={p.n} ellipse c={c.center:.3f} a={c.a:.3f} ratio={c.ratio:.3f} "
          f"({p.info['m_in']} reference eigenvalues inside) Ne={c.ne} m0={p.m0}", file=sys.stderr, flush=True)
    want = [x.strip() for x in args.preconds.split(",") if x.strip()]
    # --- training on the other fields
    t0 = time.perf_counter()
    if "learned" not in want:
        args.train_fields = 0
    # output scale 1/max|a_ii| = h^2/6, divided by sqrt(n) with --net-scale rootn
    # (the network's output per grid point is O(1) for an input of unit 2-norm)
    osc = hh * hh / 6.0 / (np.sqrt(p.n) if args.net_scale == "rootn" else 1.0)
    net = fh.Net(h, N, N, fields=p.info["field"].reshape(3, -1) / 30.0, alpha=float(c.a), out_scale=osc,
                 seed=5, nz=N)
    nfields = args.train_fields
    sets = []
    for k, seed in enumerate(list(C4_TRAIN_FIELDS)[:nfields]):
        v = W.smooth_field3d(N, seed)
        pk = fh.Problem(h, csr(W.convdiff3d_csr(N, v)))
        # four nodes per field (rotating), two columns, iterates after 0, 2, 5 steps
        zk = z[[(k + 4 * q) % c.ne for q in range(4)]]
        sets.append((v.reshape(3, -1) / 30.0, pk, learned.harvest(pk, zk, m=2, seed=seed, steps=(0, 2, 5))))
        print(f"[bench] harvested field {seed} ({time.perf_counter() - t0:.1f} s)", file=sys.stderr, flush=True)
    t_h = time.perf_counter() - t0
    hist = [float("nan")]
    for ep in range(args.epochs if nfields else 0):
        hist += learned.train_fields(net, sets, epochs=1, lr=2e-3, batch_systems=8, seed=ep)
        print(f"[bench] epoch {ep + 1}: loss {hist[-1]:.4f} ({time.perf_counter() - t0:.1f} s)", file=sys.stderr,
              flush=True)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    del sets
    net.set_fields(p.info["field"].reshape(3, -1) / 30.0)
    fh.set_net(prob, net)
    print(f"[bench] network trained on {nfields} fields: harvest {t_h:.1f} s, total {t_train:.1f} s, loss "
          f"{hist[1] if len(hist) > 1 else float('nan'):.3f} -> {hist[-1]:.3f}", file=sys.stderr, flush=True)
    judge = None if not nfields else learned.evaluate(prob, z[:4], m=4, seed=98, tol=1e-8, restart=30,
                                                      max_restarts=4, fallback=fh.FH_PC_ILU0)
    print(f"[bench] fixed Krylov budget on fresh systems (unpreconditioned FP64 as the judge): {judge}",
          file=sys.stderr, flush=True)
    # --- FEAST with each preconditioner
    Y0 = torch.from_numpy(p.Y0).cuda()
    Yh0 = torch.from_numpy(p.Yh0).cuda()
    runs = {}
    u = (eigs - c.center)
    ref_in = eigs[(u.real / c.a) ** 2 + (u.imag / (c.ratio * c.a)) ** 2 < 1.0]
    # ilu0-conj: ILU(0) with n_e solves per iteration instead of 2 n_e (real
    # start blocks, conjugate Ritz pairs; the matrix is real and the ellipse
    # centred on the real axis)
    for name, pc, cpairs in (("learned", fh.FH_PC_LEARNED, 1), ("ilu0", fh.FH_PC_ILU0, 1),
                             ("ilu0-conj", fh.FH_PC_ILU0, 2), ("jacobi", fh.FH_PC_JACOBI, 1),
                             ("none", fh.FH_PC_NONE, 1)):
        if name not in want:
            continue
        o = fh.default_opts(p.m0, solver=fh.FH_SOLVER_BGMRES, precond=pc, restart=30, max_restarts=2,
                            inner_tol=1e-3, precision=fh.FH_PREC_MIXED, mixed_inner_tol=1e-3, max_refine=1,
                            max_iter=args.max_iter, eps=EPS_ITER, orth=2, fallback=fh.FH_PC_ILU0, confirm=1,
                            conj_pairs=cpairs)
        y0, yh0 = (Y0, Yh0) if cpairs == 1 else (Y0.real.to(Y0.dtype), Yh0.real.to(Yh0.dtype))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        try:
            out = fh.feast(prob, c.center, c.a, c.ratio, 0.0, c.ne, y0, yh0, o)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t1
            lam = out["lam"]
            d = float(np.abs(lam[:, None] - ref_in[None, :]).min(axis=1).max() / alpha) if len(lam) else None
            r = {"info": out["info"], "iterations": out["report"]["iters"], "seconds": dt,
                 "s_per_iteration": dt / max(1, out["report"]["iters"]), "m": int(len(lam)),
                 "m_reference_inside": int(len(ref_in)), "max_dlam_over_alpha": d,
                 "fallback_solves": out["report"]["n_fallback"], "last_inner_relres": out["report"]["inner_relres"],
                 "solves": out["report"]["n_solve"], "factorizations": out["report"]["n_factor"]}
        except fh.FeastError as e:
            r = {"error": str(e), "seconds": time.perf_counter() - t1}
        runs[name] = r
        print(f"[bench] FEAST with {name}: {json.dumps(r)}", file=sys.stderr, flush=True)
    line = {"metric": "FEAST time to solution (eq:res <= 1e-9) with the learned preconditioner vs ILU(0), "
                      "Jacobi, none", "unit": "s", "higher_is_better": False, "n_gpus": 1,
            "value": runs.get("learned", {}).get("seconds"), "dtype": "c64 Krylov solves, BF16 network weights",
            "data": "synthetic",
            "config": {"workload": f"3D convection-diffusion-reaction {N}^3 (n={p.n}), held-out field, "
                                   f"{p.info['m_in']} eigenvalues, Ne=16, m0=96, FGMRES(30) x 2"},
            "training": {"fields": nfields, "epochs": args.epochs, "seconds": t_train, "loss_first": hist[1] if len(hist) > 1 else None,
                         "out_scale": osc,
                         "loss_last": hist[-1]},
            "fixed_budget_judge": judge, "feast": runs}
    print(json.dumps(line))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed FEAST iterations (default: 2 on the headline "
                                                              "workload, 16 on convdiff)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed warm-up iterations (default 1 / 4)")
    ap.add_argument("--fp64-steps", type=int, default=None, help="headline workload: timed plain FP64 iterations "
                                                                  "(default: --steps)")
    ap.add_argument("--max-iter", type=int, default=30, help="headline workload: iteration limit of the "
                                                             "validation run")
    ap.add_argument("--grid", type=int, default=1024, help="headline workload: grid points per side")
    ap.add_argument("--grid3d", type=int, default=64, help="convdiff3d: grid points per side")
    ap.add_argument("--train-fields", type=int, default=32, help="convdiff3d: training convection fields")
    ap.add_argument("--epochs", type=int, default=20, help="convdiff3d: training epochs")
    ap.add_argument("--preconds", default="learned,ilu0,ilu0-conj,jacobi,none", help="convdiff3d: preconditioners to run")
    ap.add_argument("--net-scale", default="one", choices=["one", "rootn"],
                    help="convdiff3d: network output scale h^2/6 (one) or h^2/(6 sqrt(n)) (rootn)")
    ap.add_argument("--eigs", default=None, help="headline workload: reference eigenvalues (.npy or the golden "
                                                 "JSON; default the 1024 x 1024 one)")
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 comparison run")
    ap.add_argument("--batch-nodes", type=int, default=0, help="headline workload: quadrature nodes solved "
                                                               "together (fh_opts.batch_nodes; 0 = as many as fit)")
    ap.add_argument("--tts", action="store_true", help="contour-grid: also run the batched path to eq:res <= 1e-7")
    ap.add_argument("--confirm", type=int, default=1, choices=[0, 1, 2],
                    help="contour-grid --tts: exit rule (fh_opts.confirm)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-validate", action="store_true")
    ap.add_argument("--columns", type=int, default=128, help="learned3d: columns per system")
    ap.add_argument("--workload", default="schrodinger",
                    choices=["schrodinger", "convdiff", "dense-batch", "copy-calibration", "learned3d", "csym",
                             "contour-grid", "convdiff3d"],
                    help="schrodinger: the headline workload, complex-symmetric 1024 x 1024 (default); convdiff: "
                         "2D convection-diffusion 256 x 256; dense-batch: 64 dense problems; copy-calibration: a "
                         "1 GiB device copy (reference for the HBM byte counters)")
    ap.add_argument("--count", type=int, default=64, help="dense-batch: number of problems")
    ap.add_argument("--orth", type=int, default=2, choices=[0, 1, 2],
                    help="GMRES orthogonalization: 0 CGS2, 1 one projection, 2 delayed reorthogonalization "
                         "(both precisions)")
    args = ap.parse_args()
    global ORTH, BATCH_NODES
    ORTH = args.orth
    BATCH_NODES = args.batch_nodes
    if args.steps is None:
        args.steps = 2 if args.workload == "schrodinger" else 16
    if args.warmup is None:
        args.warmup = 1 if args.workload == "schrodinger" else 4
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU sharding of the "
              "contour filter (one node group per GPU) is a design only and not built", file=sys.stderr)
        sys.exit(2)
    if args.workload == "dense-batch":
        dense_batch(args)
        return
    if args.workload == "copy-calibration":
        copy_calibration()
        return
    if args.workload == "learned3d":
        learned3d(args)
        return
    if args.workload == "csym":
        csym(args)
        return
    if args.workload == "contour-grid":
        contour_grid(args)
        return
    if args.workload == "schrodinger":
        schrodinger(args)
        return
    if args.workload == "convdiff3d":
        convdiff3d_learned(args)
        return
    import torch
    import paper_1506_04463_amd as fh

    p = _problem()
    handle = fh.Handle(0)
    A = p.A
    prob = fh.Problem(handle, fh.CSR(torch.from_numpy(A["rowptr"]).cuda(), torch.from_numpy(A["colind"]).cuda(),
                                     torch.from_numpy(A["val"]).cuda(), A["n"]))
    print(f"[bench] {p.name}: n={p.n} nnz={len(A['colind'])} Ne=16 m0={p.m0}", file=sys.stderr, flush=True)

    dt_mx, out_mx, stats = run_path(fh, torch, handle, prob, p, fh.FH_PREC_MIXED, args.steps, args.warmup,
                                    profile=True)
    ms_mx = 1000.0 * dt_mx / args.steps
    print(f"[bench] mixed: {ms_mx:.1f} ms/iteration", file=sys.stderr, flush=True)
    plain = None
    if not args.no_fp64:
        dt_64, out_64, _ = run_path(fh, torch, handle, prob, p, fh.FH_PREC_FP64, args.steps, args.warmup)
        ms_64 = 1000.0 * dt_64 / args.steps
        plain = {"value": 1000.0 / ms_64, "ms_per_step": ms_64}
        print(f"[bench] fp64: {ms_64:.1f} ms/iteration", file=sys.stderr, flush=True)
    # the same mixed path with n_e solves per iteration instead of 2 n_e
    dt_h, _, _ = run_path(fh, torch, handle, prob, p, fh.FH_PREC_MIXED, args.steps, args.warmup, conj_pairs=2)
    half = {"ms_per_step": 1000.0 * dt_h / args.steps, "solves_per_iteration": 16,
            "speedup_vs_2ne_solves": dt_mx / dt_h}
    print(f"[bench] mixed, conj_pairs=2 (n_e solves): {half['ms_per_step']:.1f} ms/iteration", file=sys.stderr,
          flush=True)
    valid = None
    if not args.no_validate:
        valid = solve_to_convergence(fh, torch, prob, p, fh.FH_PREC_MIXED)
        print(f"[bench] validation: {valid}", file=sys.stderr, flush=True)
        half["time_to_solution"] = solve_to_convergence(fh, torch, prob, p, fh.FH_PREC_MIXED, conj_pairs=2)
        print(f"[bench] validation, conj_pairs=2: {half['time_to_solution']}", file=sys.stderr, flush=True)
        if plain is not None:
            v64 = solve_to_convergence(fh, torch, prob, p, fh.FH_PREC_FP64)
            plain["time_to_solution"] = v64
            print(f"[bench] fp64 validation: {v64}", file=sys.stderr, flush=True)

    # dominant kernel (largest total time) -> achieved algorithmic bandwidth
    dom = max(stats.items(), key=lambda kv: kv[1]["ms"])
    name, st = dom
    avg_ms = st["ms"] / st["count"]
    achieved = st["bytes"] / (st["ms"] * 1e-3) / 1e9
    roof = {"bound": "hbm", "kernel": name, "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS, "traffic": _traffic(name), "avg_ms": avg_ms, "launches": st["count"],
            "bytes_per_launch": st["bytes"] / st["count"],
            "share_of_step": st["ms"] / (args.steps * ms_mx)}
    kernels = {k: {"ms_total": v["ms"], "count": v["count"], "GBps": v["bytes"] / (v["ms"] * 1e-3) / 1e9,
                   "frac_hbm": (v["bytes"] / (v["ms"] * 1e-3) / 1e9 / PEAK_HBM_GBS) if v["bytes"] else None}
               for k, v in sorted(stats.items(), key=lambda kv: -kv[1]["ms"])[:8]}
    cpu = None if args.no_cpu else cpu_baseline(p)
    rhs = 2 * 16 * p.m0
    line = {
        "metric": "FEAST iterations/sec & shifted-solve RHS/s at residual <=1e-10 vs plain FP64",
        "stop_eq_res": EPS_ITER,
        "value": 1000.0 / ms_mx,
        "unit": "FEAST iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_mx,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64 inner solves + c128 residual check, residual form and Rayleigh-Ritz",
        "data": "synthetic",
        "config": {"workload": "convdiff2d 256x256 (n=65536, nnz=326656), Pe 20 along (1,0.5), ellipse around 41 "
                               "eigenvalues, Ne=16, m0=64, GMRES(30)x2 + ILU(0), c64 solves + FP64 residual form",
                   "rhs_per_iteration": rhs,
                   "orthogonalization": {0: "CGS2", 1: "CGS", 2: "DCGS2"}[ORTH]},
        # fixed Krylov budget per right-hand side (2 GMRES(30) cycles), not a tolerance
        "rhs_per_s_fixed_budget": rhs * 1000.0 / ms_mx,
        "plain_fp64": plain,
        # real matrix and an ellipse centred on the real axis: real start blocks,
        # conjugate Ritz pairs, 16 solves per iteration instead of 32 (Table tab:solve)
        "conj_subspace": half,
        "speedup_vs_fp64": None if plain is None else plain["ms_per_step"] / ms_mx,
        "time_to_solution_speedup_vs_fp64": (None if plain is None or valid is None or "time_to_solution" not in plain
                                             else plain["time_to_solution"]["time_to_solution_s"] /
                                             valid["time_to_solution_s"]),
        "validity": valid,
        "roofline": roof,
        "kernels": kernels,
        "hbm_target_0_6": _hbm_target(kernels),
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
