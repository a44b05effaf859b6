"""Training glue for the learned preconditioner (library calls only).

The network (``Net``) is trained on pairs (r_k, e_k) harvested from the
library's own shifted solves: for a block of exact solutions x* (random) and
b = M x*, x_k is the iterate of plain (unpreconditioned) GMRES after k steps,
r_k = b - M x_k its residual and e_k = x* - x_k its error, so that
M e_k = r_k holds to rounding with M = z - A (right systems) or (z - A)^H
(left systems); no accurate solve is needed.
Every product, solve, forward and backward pass runs in the library; torch
only holds the device buffers and draws the random right-hand sides.
"""
from __future__ import annotations

import numpy as np

from . import (FH_PC_ILU0, FH_PC_LEARNED, FH_PC_NONE, FH_PREC_FP64, Net, Problem, default_opts, residual_pair,
               shifted_apply, shifted_solve)


def _torch():
    import torch
    return torch


def _systems(z):
    """every node twice: right systems first, then the left ones"""
    z = np.asarray(z, dtype=np.complex128)
    return np.concatenate([z, z]), np.array([0] * len(z) + [1] * len(z), dtype=np.int32)


def _randn_blocks(nsys, n, m, seed, device="cuda"):
    torch = _torch()
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    re = torch.randn((nsys, n, m), generator=g, device=device, dtype=torch.float64)
    im = torch.randn((nsys, n, m), generator=g, device=device, dtype=torch.float64)
    return torch.complex(re, im).contiguous()


def apply_op(prob: Problem, zs, sides, X):
    """M_s X_s for every system (right systems first)."""
    torch = _torch()
    sides = np.asarray(sides)
    nr = int(np.count_nonzero(sides == 0))
    out = torch.empty_like(X)
    if nr:
        out[:nr] = shifted_apply(prob, 0, zs[:nr], X[:nr].contiguous())
    if nr < len(sides):
        out[nr:] = shifted_apply(prob, 1, np.conj(zs[nr:]), X[nr:].contiguous())
    return out


def pairs(prob: Problem, zs, sides, B, X, Xt):
    """(B_s - M_s X_s, Xt_s - X_s) for every system (right systems first), by the library."""
    torch = _torch()
    sides = np.asarray(sides)
    nr = int(np.count_nonzero(sides == 0))
    R = torch.empty_like(X)
    E = torch.empty_like(X)
    for lo, hi, side, sh in ((0, nr, 0, zs[:nr]), (nr, len(sides), 1, np.conj(zs[nr:]))):
        if hi > lo:
            R[lo:hi], E[lo:hi] = residual_pair(prob, side, sh, B[lo:hi].contiguous(), X[lo:hi].contiguous(),
                                               Xt[lo:hi].contiguous())
    return R, E


def harvest(prob: Problem, z, m=8, seed=0, steps=(0, 2, 5, 10)):
    """Pairs from plain GMRES: for each k in steps, (r_k, e_k) for all 2 ne systems.

    Returns dict(z=[P] complex, sides=[P] int, R=[P, n, m], E=[P, n, m]) with
    P = 2 ne len(steps) systems (device tensors)."""
    torch = _torch()
    zs, sides = _systems(z)
    xs = _randn_blocks(len(zs), prob.n, m, seed)
    B = apply_op(prob, zs, sides, xs)
    Rs, Es, Z, S = [], [], [], []
    for k in steps:
        if k == 0:                       # x_0 = 0: the right-hand side and the solution
            Rs.append(B.clone())
            Es.append(xs.clone())
        else:
            o = default_opts(m, precision=FH_PREC_FP64, precond=FH_PC_NONE, restart=int(k), max_restarts=1,
                             inner_tol=1e-300)
            xk, _ = shifted_solve(prob, zs, sides, B, o)
            r, e = pairs(prob, zs, sides, B, xk, xs)
            Rs.append(r)
            Es.append(e)
        Z.append(zs)
        S.append(sides)
    return dict(z=np.concatenate(Z), sides=np.concatenate(S), R=torch.cat(Rs).contiguous(),
                E=torch.cat(Es).contiguous())


def train(net: Net, data, epochs=50, lr=1e-3, batch_systems=8, seed=0, problem: Problem | None = None):
    """Adam over shuffled batches of systems; returns the mean loss of each epoch.

    With ``problem`` (the CSR problem the pairs come from) the loss is the
    residual-norm one, ||M (net(r) - e)||^2 / ||r||^2, else the error-norm one."""
    rng = np.random.default_rng(seed)
    P = data["R"].shape[0]
    hist = []
    for _ in range(epochs):
        perm = rng.permutation(P)
        tot, cnt = 0.0, 0
        for i in range(0, P, batch_systems):
            idx = np.sort(perm[i:i + batch_systems])
            it = _torch().as_tensor(idx, device=data["R"].device)
            R = data["R"].index_select(0, it).contiguous()
            E = data["E"].index_select(0, it).contiguous()
            loss = net.train_step(data["z"][idx], data["sides"][idx], R, E, lr=lr, problem=problem)
            tot += loss * len(idx)
            cnt += len(idx)
        hist.append(tot / cnt)
    return hist


def train_fields(net: Net, sets, epochs=50, lr=1e-3, batch_systems=8, seed=0):
    """Train one network on several operators that differ by a coefficient
    field: sets is a list of (fields, problem, data); every epoch visits the
    sets in turn, switching the network's input fields.  Returns the mean
    loss of each epoch (residual-norm loss of each set's operator)."""
    rng = np.random.default_rng(seed)
    hist = []
    for ep in range(epochs):
        tot, cnt = 0.0, 0
        for k in rng.permutation(len(sets)):
            fields, prob, data = sets[k]
            net.set_fields(fields)
            h = train(net, data, epochs=1, lr=lr, batch_systems=batch_systems, seed=seed * 1000 + ep, problem=prob)
            tot += h[0] * data["R"].shape[0]
            cnt += data["R"].shape[0]
        hist.append(tot / cnt)
    return hist


def evaluate(prob: Problem, z, m=4, seed=1, tol=1e-8, restart=30, max_restarts=10, precision=FH_PREC_FP64,
             fallback=FH_PC_NONE, sides=None):
    """Each preconditioner (none, the attached network in FGMRES, ILU(0)) on
    fresh systems with a known solution x* (random, b = M x*) and the same
    Krylov budget (restart x max_restarts steps, stopping early at tol):
    steps taken, worst final relative residual, largest column error
    ||x - x*|| / ||x*||.  The unpreconditioned FP64 solve ("none") is the
    reference the others are judged against."""
    torch = _torch()
    if sides is None:
        zs, sides = _systems(z)
    else:
        zs, sides = np.asarray(z, dtype=np.complex128), np.asarray(sides, dtype=np.int32)
    xs = _randn_blocks(len(zs), prob.n, m, seed)
    B = apply_op(prob, zs, sides, xs)
    out = {}
    for name, pc in (("none", FH_PC_NONE), ("learned", FH_PC_LEARNED), ("ilu0", FH_PC_ILU0)):
        o = default_opts(m, precision=FH_PREC_FP64 if name == "none" else precision, precond=pc, restart=restart,
                         max_restarts=max_restarts, inner_tol=tol, mixed_inner_tol=1e-4, max_refine=20,
                         save_factors=0, fallback=fallback)
        X, rep = shifted_solve(prob, zs, sides, B, o)
        err = (torch.linalg.vector_norm(X - xs, dim=1) / torch.linalg.vector_norm(xs, dim=1)).max().item()
        out[name] = dict(steps=int(rep["inner_steps"]), relres=float(rep["inner_relres"]), err=err,
                         fallback=int(rep["n_fallback"]))
    return out
