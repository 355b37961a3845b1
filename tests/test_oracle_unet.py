"""Pins of the warm-start network's FP64 oracle (oracle/unet.py).

Each convolution is checked against closed forms (identity and shift taps,
neighbour counts), a pure-Python loop over the definition on a tiny input, and
the adjoint identities that tie its backward to its forward; the whole
network's backward is checked against central finite differences and Adam's
first step against its closed form.
"""
import itertools

import numpy as np
import pytest

from oracle import unet as U


def _center(ci, co):
    w = np.zeros((27, ci, co))
    w[13] = np.eye(ci, co)
    return w


def test_identity_tap_stride1_and_2():
    g = np.random.default_rng(0)
    x = g.standard_normal((2, 5, 6, 7, 3))
    y = U.conv3d(x, _center(3, 3), np.zeros(3))
    np.testing.assert_array_equal(y, x)
    y2 = U.conv3d(x, _center(3, 3), np.zeros(3), stride=2)
    assert y2.shape == (2, 3, 3, 4, 3)
    np.testing.assert_array_equal(y2, x[:, ::2, ::2, ::2])


@pytest.mark.parametrize("d", [(0, 0, 1), (0, 1, 0), (1, 0, 0), (-1, 0, 0), (0, -1, 1)])
def test_shift_tap(d):
    # a single tap at offset d reads x[p + d] (zero outside the grid)
    dz, dy, dx = d
    t = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)
    w = np.zeros((27, 1, 1))
    w[t] = 1.0
    g = np.random.default_rng(1)
    x = g.standard_normal((1, 4, 5, 6, 1))
    y = U.conv3d(x, w, np.zeros(1))
    D, H, W = 4, 5, 6
    for z, yy, xx in itertools.product(range(D), range(H), range(W)):
        q = (z + dz, yy + dy, xx + dx)
        inside = 0 <= q[0] < D and 0 <= q[1] < H and 0 <= q[2] < W
        want = x[0, q[0], q[1], q[2], 0] if inside else 0.0
        assert y[0, z, yy, xx, 0] == want


def test_all_ones_counts_neighbours():
    x = np.ones((1, 4, 5, 3, 1))
    w = np.ones((27, 1, 1))
    y = U.conv3d(x, w, np.full(1, 0.5))[0, ..., 0]

    def cnt(i, n):
        return 3 - (i == 0) - (i == n - 1)
    for z, yy, xx in itertools.product(range(4), range(5), range(3)):
        assert y[z, yy, xx] == cnt(z, 4) * cnt(yy, 5) * cnt(xx, 3) + 0.5


@pytest.mark.parametrize("stride", [1, 2])
def test_conv_matches_loops(stride):
    g = np.random.default_rng(2)
    x = g.standard_normal((1, 3, 4, 5, 2))
    w = g.standard_normal((27, 2, 3))
    b = g.standard_normal(3)
    y = U.conv3d(x, w, b, stride)
    D, H, W = 3, 4, 5
    Do, Ho, Wo = [(n - 1) // stride + 1 for n in (D, H, W)]
    assert y.shape == (1, Do, Ho, Wo, 3)
    for z, yy, xx, co in itertools.product(range(Do), range(Ho), range(Wo), range(3)):
        acc = b[co]
        for dz, dy, dx in itertools.product((-1, 0, 1), repeat=3):
            qz, qy, qx = stride * z + dz, stride * yy + dy, stride * xx + dx
            if 0 <= qz < D and 0 <= qy < H and 0 <= qx < W:
                t = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)
                for ci in range(2):
                    acc += x[0, qz, qy, qx, ci] * w[t, ci, co]
        assert abs(y[0, z, yy, xx, co] - acc) < 1e-12


@pytest.mark.parametrize("stride,shape", [(1, (2, 5, 4, 6)), (2, (1, 7, 6, 5)), (2, (2, 4, 4, 4))])
def test_conv_backward_adjoint(stride, shape):
    # <conv(x, w), dy> = <x, dx> = <w, dw> (bias 0) and db = sum dy
    g = np.random.default_rng(3)
    x = g.standard_normal(shape + (3,))
    w = g.standard_normal((27, 3, 4))
    y = U.conv3d(x, w, np.zeros(4), stride)
    dy = g.standard_normal(y.shape)
    dx, dw, db = U.conv3d_backward(x, w, dy, stride)
    lhs = np.sum(y * dy)
    assert abs(np.sum(x * dx) - lhs) < 1e-10 * abs(lhs) + 1e-10
    assert abs(np.sum(w * dw) - lhs) < 1e-10 * abs(lhs) + 1e-10
    # dw is the gradient for every direction V, not just w: linearity in w
    V = g.standard_normal(w.shape)
    yv = U.conv3d(x, V, np.zeros(4), stride)
    assert abs(np.sum(yv * dy) - np.sum(V * dw)) < 1e-10 * np.abs(yv * dy).sum()
    np.testing.assert_allclose(db, dy.sum(axis=(0, 1, 2, 3)), rtol=1e-12)


@pytest.mark.parametrize("f,fine", [(2, (4, 4, 4)), (2, (5, 6, 7)), (4, (9, 6, 13)), (4, (4, 4, 4))])
def test_upsample_adjoint(f, fine):
    g = np.random.default_rng(4)
    coarse = tuple((n - 1) // f + 1 for n in fine)
    a = g.standard_normal((2,) + coarse + (3,))
    u = U.upsample(a, fine, f)
    assert u.shape == (2,) + fine + (3,)
    # nearest neighbour: u[z, y, x] = a[z // f, y // f, x // f]
    for z, y, x in ((fine[0] - 1, 1, fine[2] - 1), (0, fine[1] - 1, 2)):
        np.testing.assert_array_equal(u[1, z, y, x], a[1, z // f, y // f, x // f])
    d = g.standard_normal(u.shape)
    assert abs(np.sum(u * d) - np.sum(a * U.upsample_backward(d, coarse, f))) < 1e-11


def test_two_halvings_match_a_quarter():
    # the level-2 grid of two stride-2 convolutions is the up4 coarse grid
    for n in range(1, 40):
        assert U.out_size(U.out_size(n, 2), 2) == (n - 1) // 4 + 1


def test_net_backward_finite_differences():
    g = np.random.default_rng(5)
    P = U.init_params(7)
    for k in P:
        if k.endswith(".b"):
            P[k] = 0.1 * g.standard_normal(P[k].shape)
    x = np.zeros((2, 6, 5, 4, 8))
    x[..., :2] = g.standard_normal((2, 6, 5, 4, 2))
    tgt = g.standard_normal((2, 6, 5, 4))

    def loss(PP):
        y, _ = U.forward(PP, x)
        return U.mse(y, tgt)[0]

    y, c = U.forward(P, x)
    assert y.shape == (2, 6, 5, 4)
    L, dy = U.mse(y, tgt)
    G = U.backward(P, c, dy)
    assert sorted(G) == sorted(P)
    # Directional derivatives along a random direction in each parameter
    # block.  The network is piecewise linear in each weight (ReLU): a step
    # that moves a pre-activation across zero spoils one difference, so the
    # check takes the best of a few step sizes; a wrong gradient misses at all.
    for name in sorted(P):
        V = g.standard_normal(P[name].shape)
        an = float(np.sum(G[name] * V))
        errs = []
        for eps in (1e-6, 3e-7, 1e-7):
            Pp, Pm = dict(P), dict(P)
            Pp[name] = P[name] + eps * V
            Pm[name] = P[name] - eps * V
            errs.append(abs((loss(Pp) - loss(Pm)) / (2 * eps) - an))
        assert min(errs) <= 1e-6 * max(abs(an), 1e-2), (name, errs, an)


def test_mse_gradient():
    g = np.random.default_rng(6)
    y, t = g.standard_normal(50), g.standard_normal(50)
    L, d = U.mse(y, t)
    assert abs(L - np.mean((y - t) ** 2)) < 1e-14
    e = 1e-6
    for i in (0, 17, 49):
        yp, ym = y.copy(), y.copy()
        yp[i] += e
        ym[i] -= e
        assert abs((U.mse(yp, t)[0] - U.mse(ym, t)[0]) / (2 * e) - d[i]) < 1e-8


def test_h1_loss_sine_mode_and_gradient():
    # a Dirichlet sine mode is an eigenvector of the 7-point Laplacian with
    # eigenvalue sum_d (2 - 2 cos(pi k_d h_d)), h_d = 1 / (n_d + 1)
    D, H, W = 7, 6, 9
    kz, ky, kx = 2, 1, 3
    z = np.arange(1, D + 1)[:, None, None] / (D + 1)
    y = np.arange(1, H + 1)[None, :, None] / (H + 1)
    x = np.arange(1, W + 1)[None, None, :] / (W + 1)
    v = np.sin(np.pi * kz * z) * np.sin(np.pi * ky * y) * np.sin(np.pi * kx * x)
    lam = sum(2 - 2 * np.cos(np.pi * k / (n + 1)) for k, n in ((kz, D), (ky, H), (kx, W)))
    e = v[None]
    np.testing.assert_allclose(U.laplacian7(e), lam * e, atol=1e-12)
    L, _ = U.h1_loss(e, np.zeros_like(e), 0.25)
    assert abs(L - (lam + 0.25) * np.sum(v * v) / v.size) < 1e-12
    g = np.random.default_rng(8)
    yy, tt = g.standard_normal((2, 4, 5, 3)), g.standard_normal((2, 4, 5, 3))
    L, d = U.h1_loss(yy, tt, 0.1)
    assert L > 0
    h = 1e-6
    for idx in ((0, 0, 0, 0), (1, 2, 3, 1), (0, 3, 4, 2)):
        yp, ym = yy.copy(), yy.copy()
        yp[idx] += h
        ym[idx] -= h
        fd = (U.h1_loss(yp, tt, 0.1)[0] - U.h1_loss(ym, tt, 0.1)[0]) / (2 * h)
        assert abs(fd - d[idx]) < 1e-7


def test_adam_first_step_is_signed_lr():
    # after one step from zero moments, m_hat = g and v_hat = g^2 exactly
    g = np.random.default_rng(7)
    P = {"a": g.standard_normal(20)}
    G = {"a": g.standard_normal(20)}
    M = {"a": np.zeros(20)}
    V = {"a": np.zeros(20)}
    P0 = P["a"].copy()
    U.adam(P, G, M, V, 1, lr=0.01, eps=0.0)
    np.testing.assert_allclose(P["a"], P0 - 0.01 * np.sign(G["a"]), rtol=0, atol=1e-15)


def test_adam_constant_gradient_steps_are_signed_lr():
    # with the same gradient g at steps 1..t from zero moments,
    # m_t = (1 - b1^t) g and v_t = (1 - b2^t) g^2, so the bias-corrected
    # moments are g and g^2 at EVERY step and each step moves by lr sign(g)
    # (eps = 0); a bias correction of 1 - b1*t instead of 1 - b1^t fails at t = 2
    g = np.random.default_rng(8)
    G = {"a": g.standard_normal(16)}
    P = {"a": g.standard_normal(16)}
    M = {"a": np.zeros(16)}
    V = {"a": np.zeros(16)}
    for t in (1, 2, 3):
        P0 = P["a"].copy()
        U.adam(P, G, M, V, t, lr=0.01, eps=0.0)
        np.testing.assert_allclose(P["a"] - P0, -0.01 * np.sign(G["a"]), rtol=1e-12, atol=0)


def test_adam_two_steps_by_hand():
    # scalar gradients 1 then -2, b1 = 0.9, b2 = 0.999, lr = 1, eps = 0:
    # m2 = 0.9*0.1 - 0.2 = -0.11, v2 = 0.999*0.001 + 0.004 = 0.004999,
    # m_hat = -0.11/0.19 = -11/19, v_hat = 0.004999/0.001999 = 4999/1999,
    # second step = -m_hat/sqrt(v_hat) = (11/19) sqrt(1999/4999)
    P = {"a": np.zeros(1)}
    M = {"a": np.zeros(1)}
    V = {"a": np.zeros(1)}
    U.adam(P, {"a": np.array([1.0])}, M, V, 1, lr=1.0, eps=0.0)
    np.testing.assert_allclose(P["a"], [-1.0], rtol=1e-15)
    U.adam(P, {"a": np.array([-2.0])}, M, V, 2, lr=1.0, eps=0.0)
    step2 = (11.0 / 19.0) * (1999.0 / 4999.0) ** 0.5
    np.testing.assert_allclose(P["a"], [-1.0 + step2], rtol=1e-13)


def test_param_count():
    P = U.init_params(0)
    n = sum(v.size for v in P.values())
    assert 150_000 <= n <= 300_000
