"""Reference (oracle) of the learned preconditioner network, NumPy float64.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).  The paper has no learned
component; this network is the one the build uses as a flexible preconditioner
inside FGMRES: three 3x3 convolutions with zero padding on the solution grid,
Cin -> H -> H -> 2 channels, bias, ReLU after the first two.  The input
channels are (Re r, Im r)/||r||_2 followed by optional constant fields; the
output (Re e, Im e) is scaled back by ||r||_2.

Layouts follow the HIP kernels: an activation is an array [ny, nx, C, m]
(grid row, grid column, channel, batch column) on a 2D grid, or
[nz, ny, nx, C, m] on a 3D grid; weights are [Cout, Cin, 3, 3] or
[Cout, Cin, 3, 3, 3] (offsets -1, 0, 1 in each axis, slowest axis first).
The same functions serve both: the number of spatial axes is x.ndim - 2.

Two losses over the columns c of a batch, with o_c = out[:, :, 0, c] + i
out[:, :, 1, c] and t_c the (scaled) error target:
* plain: mean_c ||o_c - t_c||^2 / ||t_c||^2;
* operator-weighted: mean_c ||M_c (o_c - t_c)||^2 / ||M_c t_c||^2, where M_c
  is the shifted operator of the column's system, so that M_c t_c is the
  (scaled) residual; this measures how close M_c net(r) is to r.

Parity status: pinned by central finite differences of both losses in
tests/test_oracle_convnet.py (gradients), and by a direct sum for the forward
convolution; the HIP kernels are checked against these functions.
"""
from __future__ import annotations

import itertools

import numpy as np


def _offsets(d):
    return itertools.product(range(3), repeat=d)


def conv3x3(x, w, b):
    """x [*S, Cin, m], w [Cout, Cin, 3 (x d)], b [Cout] -> [*S, Cout, m]; zero padding."""
    d = x.ndim - 2
    S = x.shape[:d]
    cout = w.shape[0]
    xp = np.pad(x, [(1, 1)] * d + [(0, 0), (0, 0)])
    out = np.zeros(S + (cout, x.shape[-1])) + b[(None,) * d + (slice(None), None)]
    for off in _offsets(d):
        patch = xp[tuple(slice(o, o + n) for o, n in zip(off, S))]    # input at (s + off - 1)
        out += np.einsum("oc,...cm->...om", w[(slice(None), slice(None)) + off], patch)
    return out


def conv3x3_backward(x, w, gout):
    """Gradients of sum(gout * conv3x3(x, w, b)) w.r.t. x, w, b."""
    d = x.ndim - 2
    S = x.shape[:d]
    xp = np.pad(x, [(1, 1)] * d + [(0, 0), (0, 0)])
    gw = np.zeros_like(w)
    gxp = np.zeros_like(xp)
    for off in _offsets(d):
        sl = tuple(slice(o, o + n) for o, n in zip(off, S))
        patch = xp[sl]
        gw[(slice(None), slice(None)) + off] = np.einsum("pom,pcm->oc", gout.reshape(-1, *gout.shape[-2:]),
                                                         patch.reshape(-1, *patch.shape[-2:]))
        gxp[sl] += np.einsum("oc,...om->...cm", w[(slice(None), slice(None)) + off], gout)
    gb = gout.sum(axis=tuple(range(d)) + (d + 1,))
    return gxp[tuple(slice(1, -1) for _ in range(d))], gw, gb


def bf16_round(a):
    """Nearest bfloat16 value (8 significant bits, float32's exponent range,
    ties to even) of the float32 rounding of a, returned as float64."""
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def forward(params, x, act_round=None):
    """params: list of (w, b) for the 3 layers; returns output and cache.

    act_round (optional): a rounding applied to the inputs of the first two
    layers (x and a1), for an inference mode that stores those activations
    in a narrower format."""
    (w1, b1), (w2, b2), (w3, b3) = params
    r = act_round if act_round is not None else (lambda v: v)
    z1 = conv3x3(r(x), w1, b1)
    a1 = np.maximum(z1, 0.0)
    z2 = conv3x3(r(a1), w2, b2)
    a2 = np.maximum(z2, 0.0)
    out = conv3x3(a2, w3, b3)
    return out, (x, z1, a1, z2, a2)


def backward(params, cache, gout):
    (w1, b1), (w2, b2), (w3, b3) = params
    x, z1, a1, z2, a2 = cache
    ga2, gw3, gb3 = conv3x3_backward(a2, w3, gout)
    gz2 = ga2 * (z2 > 0)
    ga1, gw2, gb2 = conv3x3_backward(a1, w2, gz2)
    gz1 = ga1 * (z1 > 0)
    _, gw1, gb1 = conv3x3_backward(x, w1, gz1)
    return [(gw1, gb1), (gw2, gb2), (gw3, gb3)]


def encode(r, ny, nx, fields=None, nz=None):
    """r [n, m] complex -> input [(nz,) ny, nx, 2 + F, m] and the column norms."""
    n, m = r.shape
    S = (ny, nx) if nz is None else (nz, ny, nx)
    nr = np.linalg.norm(r, axis=0)
    s = np.where(nr > 0, 1.0 / np.where(nr > 0, nr, 1.0), 0.0)
    rr = (r * s[None, :]).reshape(S + (m,))
    chans = [rr.real, rr.imag]
    if fields is not None:
        for f in fields:                                  # S or S + (m,)
            f = np.asarray(f, dtype=np.float64)
            chans.append(np.broadcast_to(f[..., None] if f.ndim == len(S) else f, S + (m,)))
    return np.stack(chans, axis=len(S)), nr


def loss_and_grad(params, x, target):
    """Mean over columns of ||net(x) - t||^2 / ||t||^2 with t = target [*S, 2, m]."""
    out, cache = forward(params, x)
    diff = out - target
    ax = tuple(range(x.ndim - 1))
    tn = (target ** 2).sum(axis=ax)
    tn = np.where(tn > 0, tn, 1.0)
    m = x.shape[-1]
    loss = float(((diff ** 2).sum(axis=ax) / tn).mean())
    gout = 2.0 * diff / tn / m
    return loss, backward(params, cache, gout)


def loss_and_grad_op(params, x, target, ops):
    """Operator-weighted loss; ops[c] is the dense complex operator of column c."""
    out, cache = forward(params, x)
    S = out.shape[:-2]
    m = out.shape[-1]
    gout = np.zeros_like(out)
    total = 0.0
    for c in range(m):
        d = (out[..., 0, c] + 1j * out[..., 1, c] - target[..., 0, c] - 1j * target[..., 1, c]).ravel()
        t = (target[..., 0, c] + 1j * target[..., 1, c]).ravel()
        Md = ops[c] @ d
        den = np.vdot(ops[c] @ t, ops[c] @ t).real
        den = den if den > 0 else 1.0
        total += np.vdot(Md, Md).real / den
        g = 2.0 * (ops[c].conj().T @ Md) / den / m
        gout[..., 0, c] = g.real.reshape(S)
        gout[..., 1, c] = g.imag.reshape(S)
    return total / m, backward(params, cache, gout)
