"""Pins of the oracle's conv-net reference (the learned preconditioner has no
counterpart in the paper): a direct summation of the convolution, kernels with
known action (identity, shift), and central finite differences of the loss."""
import numpy as np

from oracle import convnet as N


def _params(rng, cin, h):
    shapes = [(h, cin), (h, h), (2, h)]
    return [(0.3 * rng.standard_normal((o, i, 3, 3)), 0.1 * rng.standard_normal(o)) for o, i in shapes]


def test_conv_direct_sum_and_known_kernels():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((5, 6, 3, 2))
    w = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    y = N.conv3x3(x, w, b)
    for (yy, xx, o, m) in [(0, 0, 1, 0), (2, 3, 3, 1), (4, 5, 0, 1)]:
        s = b[o]
        for dy in range(3):
            for dx in range(3):
                py, px = yy + dy - 1, xx + dx - 1
                if 0 <= py < 5 and 0 <= px < 6:
                    s += sum(w[o, c, dy, dx] * x[py, px, c, m] for c in range(3))
        assert abs(y[yy, xx, o, m] - s) < 1e-12
    wid = np.zeros((3, 3, 3, 3)); wid[np.arange(3), np.arange(3), 1, 1] = 1.0
    np.testing.assert_allclose(N.conv3x3(x, wid, np.zeros(3)), x)
    wsh = np.zeros((1, 1, 3, 3)); wsh[0, 0, 1, 2] = 1.0        # picks the right neighbour
    xs = x[:, :, :1]
    ys = N.conv3x3(xs, wsh, np.zeros(1))
    np.testing.assert_allclose(ys[:, :-1], xs[:, 1:])
    np.testing.assert_allclose(ys[:, -1], 0.0)


def test_gradients_finite_differences():
    rng = np.random.default_rng(1)
    params = _params(rng, 4, 5)
    x = rng.standard_normal((6, 5, 4, 3))
    t = rng.standard_normal((6, 5, 2, 3))
    loss, grads = N.loss_and_grad(params, x, t)
    h = 1e-6
    for layer, idx in [(0, (2, 1, 0, 2)), (1, (4, 3, 1, 1)), (2, (1, 4, 2, 0)), (0, (0, 0, 1, 1))]:
        w, b = params[layer]
        wp = [(p[0].copy(), p[1].copy()) for p in params]
        wm = [(p[0].copy(), p[1].copy()) for p in params]
        wp[layer][0][idx] += h
        wm[layer][0][idx] -= h
        fd = (N.loss_and_grad(wp, x, t)[0] - N.loss_and_grad(wm, x, t)[0]) / (2 * h)
        assert abs(fd - grads[layer][0][idx]) < 1e-6 * max(1.0, abs(fd))
    for layer, o in [(0, 3), (2, 1)]:
        wp = [(p[0].copy(), p[1].copy()) for p in params]
        wm = [(p[0].copy(), p[1].copy()) for p in params]
        wp[layer][1][o] += h
        wm[layer][1][o] -= h
        fd = (N.loss_and_grad(wp, x, t)[0] - N.loss_and_grad(wm, x, t)[0]) / (2 * h)
        assert abs(fd - grads[layer][1][o]) < 1e-6 * max(1.0, abs(fd))


def test_encode_normalizes_columns():
    rng = np.random.default_rng(2)
    r = rng.standard_normal((12, 3)) + 1j * rng.standard_normal((12, 3))
    x, nr = N.encode(r, 3, 4, fields=[np.ones((3, 4))])
    assert x.shape == (3, 4, 3, 3)
    np.testing.assert_allclose(np.sqrt((x[:, :, :2] ** 2).sum(axis=(0, 1, 2))), 1.0)
    np.testing.assert_allclose(nr, np.linalg.norm(r, axis=0))


def test_operator_loss_gradients_finite_differences_and_special_cases():
    rng = np.random.default_rng(3)
    ny, nx, m = 4, 3, 3
    n = ny * nx
    params = _params(rng, 4, 5)
    x = rng.standard_normal((ny, nx, 4, m))
    t = rng.standard_normal((ny, nx, 2, m))
    ops = [rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)) for _ in range(m)]
    loss, grads = N.loss_and_grad_op(params, x, t, ops)
    h = 1e-6
    for layer, idx in [(0, (2, 1, 0, 2)), (1, (4, 3, 1, 1)), (2, (1, 4, 2, 0))]:
        wp = [(p[0].copy(), p[1].copy()) for p in params]
        wm = [(p[0].copy(), p[1].copy()) for p in params]
        wp[layer][0][idx] += h
        wm[layer][0][idx] -= h
        fd = (N.loss_and_grad_op(wp, x, t, ops)[0] - N.loss_and_grad_op(wm, x, t, ops)[0]) / (2 * h)
        assert abs(fd - grads[layer][0][idx]) < 1e-6 * max(1.0, abs(fd))
    for layer, o in [(0, 2), (2, 0)]:
        wp = [(p[0].copy(), p[1].copy()) for p in params]
        wm = [(p[0].copy(), p[1].copy()) for p in params]
        wp[layer][1][o] += h
        wm[layer][1][o] -= h
        fd = (N.loss_and_grad_op(wp, x, t, ops)[0] - N.loss_and_grad_op(wm, x, t, ops)[0]) / (2 * h)
        assert abs(fd - grads[layer][1][o]) < 1e-6 * max(1.0, abs(fd))
    # identity operators reduce it to the plain loss; a scaled operator changes nothing
    eye = [np.eye(n, dtype=complex)] * m
    l1, g1 = N.loss_and_grad_op(params, x, t, eye)
    l0, g0 = N.loss_and_grad(params, x, t)
    assert abs(l1 - l0) < 1e-12 * l0
    np.testing.assert_allclose(g1[1][0], g0[1][0], rtol=1e-10, atol=1e-14)
    l2, _ = N.loss_and_grad_op(params, x, t, [3j * M for M in ops])
    assert abs(l2 - loss) < 1e-12 * loss


def test_conv3d_direct_sum_and_gradients():
    """The 3D case of the same functions: a direct sum of the 27 taps and
    central finite differences of the loss."""
    rng = np.random.default_rng(5)
    x = rng.standard_normal((3, 4, 5, 2, 2))
    w = rng.standard_normal((3, 2, 3, 3, 3))
    b = rng.standard_normal(3)
    y = N.conv3x3(x, w, b)
    for (zz, yy, xx, o, m) in [(0, 0, 0, 1, 0), (1, 2, 3, 2, 1), (2, 3, 4, 0, 1)]:
        s = b[o]
        for dz in range(3):
            for dy in range(3):
                for dx in range(3):
                    pz, py, px = zz + dz - 1, yy + dy - 1, xx + dx - 1
                    if 0 <= pz < 3 and 0 <= py < 4 and 0 <= px < 5:
                        s += sum(w[o, c, dz, dy, dx] * x[pz, py, px, c, m] for c in range(2))
        assert abs(y[zz, yy, xx, o, m] - s) < 1e-12
    # 2D functions are the 3D ones on a single plane with only the middle taps
    w2 = rng.standard_normal((3, 2, 3, 3))
    w3 = np.zeros((3, 2, 3, 3, 3)); w3[:, :, 1] = w2
    x2 = rng.standard_normal((4, 5, 2, 2))
    np.testing.assert_allclose(N.conv3x3(x2[None], w3, b)[0], N.conv3x3(x2, w2, b), atol=1e-12)
    shapes = [(4, 3), (4, 4), (2, 4)]
    params = [(0.3 * rng.standard_normal((o, i, 3, 3, 3)), 0.1 * rng.standard_normal(o)) for o, i in shapes]
    x = rng.standard_normal((3, 3, 4, 3, 2))
    t = rng.standard_normal((3, 3, 4, 2, 2))
    loss, grads = N.loss_and_grad(params, x, t)
    h = 1e-6
    for layer, idx in [(0, (1, 2, 0, 1, 2)), (1, (3, 0, 2, 2, 1)), (2, (1, 3, 1, 0, 0))]:
        wp = [(p[0].copy(), p[1].copy()) for p in params]
        wm = [(p[0].copy(), p[1].copy()) for p in params]
        wp[layer][0][idx] += h
        wm[layer][0][idx] -= h
        fd = (N.loss_and_grad(wp, x, t)[0] - N.loss_and_grad(wm, x, t)[0]) / (2 * h)
        assert abs(fd - grads[layer][0][idx]) < 1e-6 * max(1.0, abs(fd))


def test_bf16_round_definition():
    """bfloat16 rounding against values fixed by the format: representable
    values are unchanged, halfway cases go to the even neighbour, the nearest
    neighbour otherwise, and the float32 exponent range is kept."""
    ulp = 2.0 ** -7                                  # spacing of bfloat16 in [1, 2)
    exact = np.array([0.0, 1.0, -1.5, 1.0 + ulp, 3.0 * 2.0 ** 100, 2.0 ** -126, 255.0])
    np.testing.assert_array_equal(N.bf16_round(exact), exact)
    # halfway: 1 + ulp/2 lies between 1 (even) and 1 + ulp (odd) -> 1
    assert N.bf16_round(1.0 + ulp / 2) == 1.0
    # halfway between 1 + ulp (odd) and 1 + 2 ulp (even) -> 1 + 2 ulp
    assert N.bf16_round(1.0 + 1.5 * ulp) == 1.0 + 2 * ulp
    # nearest otherwise, both signs
    assert N.bf16_round(1.0 + 0.6 * ulp) == 1.0 + ulp
    assert N.bf16_round(-(1.0 + 0.4 * ulp)) == -1.0
    # at most half a bfloat16 ulp from the float32 value: 2^-8 relative (the
    # ulp of [2^e, 2^(e+1)) is 2^(e-7)), and a bfloat16 value (low 16 bits zero)
    v = np.random.default_rng(3).standard_normal(10000) * 10.0 ** np.random.default_rng(4).uniform(-20, 20, 10000)
    r = N.bf16_round(v)
    f = np.float32(v).astype(np.float64)
    assert np.all(np.abs(r - f) <= 2.0 ** -8 * np.abs(f))
    assert np.all(np.float32(r).view(np.uint32) & 0xFFFF == 0)
    # and the nearest one: the neighbour on the other side is farther
    step = 2.0 ** (np.floor(np.log2(np.abs(r))) - 7)
    other = r + np.sign(f - r) * step
    assert np.all(np.abs(other - f) >= np.abs(r - f))


def test_forward_with_activation_rounding():
    """forward(..., act_round) equals the layer-by-layer composition with the
    rounding applied to the first two layers' inputs (and not the third's)."""
    rng = np.random.default_rng(8)
    params = [(rng.standard_normal((4, 3, 3, 3)), rng.standard_normal(4)),
              (rng.standard_normal((4, 4, 3, 3)), rng.standard_normal(4)),
              (rng.standard_normal((2, 4, 3, 3)), rng.standard_normal(2))]
    x = rng.standard_normal((5, 6, 3, 2))
    got, _ = N.forward(params, x, act_round=N.bf16_round)
    (w1, b1), (w2, b2), (w3, b3) = params
    a1 = np.maximum(N.conv3x3(N.bf16_round(x), w1, b1), 0.0)
    a2 = np.maximum(N.conv3x3(N.bf16_round(a1), w2, b2), 0.0)
    np.testing.assert_array_equal(got, N.conv3x3(a2, w3, b3))
    plain, _ = N.forward(params, x)
    assert np.abs(got - plain).max() > 0                      # the rounding is not a no-op
    assert np.abs(got - plain).max() < 0.05 * np.abs(plain).max()
