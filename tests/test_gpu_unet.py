"""The warm-start network's HIP kernels against its FP64 oracle (oracle/unet.py).

Single convolutions (forward, input gradient, weight and bias gradients) are
fed BF16-exact operands, so the only differences are FP32 summation order:
the bound is 1e-5 of the sum of absolute terms.  The whole network runs with
BF16 activations, BF16 GEMM weights and BF16 output gradients (unit roundoff
2^-9 per rounding, about a dozen roundings deep, and ReLU masks that flip
where a pre-activation is within rounding of zero).  A numpy emulation of
those roundings on this case gives a relative L2 error of 6e-3 in the output
and up to 6e-2 in a layer's weight gradient; the bounds are 2e-2 and 0.15.
"""
import numpy as np
import pytest

from oracle import unet as U

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    from paper_2501_03743_amd import sstep
    with sstep.Handle(0) as h:
        yield h


def _bf16(a):
    return torch.from_numpy(np.asarray(a, dtype=np.float32)).bfloat16().float()


def flat_params(P):
    """Oracle parameters in the library's order: per layer W[27][Ci][Co], b[Co];
    then the head's w[16], b[1]."""
    parts = []
    for name, _, _, _ in U.LAYERS:
        parts += [P[name + ".w"].ravel(), P[name + ".b"].ravel()]
    parts += [P["head.w"].ravel(), P["head.b"].ravel()]
    return np.concatenate(parts)


def unflat(v):
    out, o = {}, 0
    for name, ci, co, _ in U.LAYERS:
        n = 27 * ci * co
        out[name + ".w"] = v[o:o + n].reshape(27, ci, co)
        o += n
        out[name + ".b"] = v[o:o + co]
        o += co
    out["head.w"] = v[o:o + U.HEAD_C]
    out["head.b"] = v[o + U.HEAD_C:o + U.HEAD_C + 1]
    assert o + U.HEAD_C + 1 == v.size
    return out


def test_mfma_operand_layout(H):
    # small integers: every product and sum is exact in BF16 x BF16 -> FP32
    g = np.random.default_rng(0)
    A = g.integers(-8, 9, (16, 32)).astype(np.float32)
    B = g.integers(-8, 9, (32, 16)).astype(np.float32)
    D = H.mfma_selftest(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda())
    np.testing.assert_array_equal(D.cpu().numpy(), A.astype(np.float64) @ B)


LAYER_SHAPES = [(ci, co, st) for _, ci, co, st in U.LAYERS]


@pytest.mark.parametrize("ci,co,stride", LAYER_SHAPES)
def test_conv_forward(H, ci, co, stride):
    g = np.random.default_rng(ci * 100 + co + stride)
    x = _bf16(g.standard_normal((2, 7, 6, 5, ci)))
    w = _bf16(g.standard_normal((27, ci, co)) * 0.2)
    y = H.conv3d(x.cuda(), w.cuda(), stride).cpu().numpy()
    xd, wd = x.double().numpy(), w.double().numpy()
    ref = U.conv3d(xd, wd, np.zeros(co), stride)
    bound = U.conv3d(np.abs(xd), np.abs(wd), np.zeros(co), stride)
    assert y.shape == ref.shape
    assert np.all(np.abs(y - ref) <= 1e-5 * bound + 1e-30)


@pytest.mark.parametrize("ci,co,stride", [s for s in LAYER_SHAPES if s[0] % 16 == 0])
def test_conv_input_grad(H, ci, co, stride):
    g = np.random.default_rng(ci * 7 + co + stride)
    shape = (2, 7, 6, 5)
    oshape = (2,) + tuple((n - 1) // stride + 1 for n in shape[1:])
    dy = _bf16(g.standard_normal(oshape + (co,)))
    w = _bf16(g.standard_normal((27, ci, co)) * 0.2)
    dx = H.conv3d_input_grad(dy.cuda(), w.cuda(), shape[1:], stride).cpu().numpy()
    x0 = np.zeros(shape + (ci,))
    ref, _, _ = U.conv3d_backward(x0, w.double().numpy(), dy.double().numpy(), stride)
    bound, _, _ = U.conv3d_backward(x0, np.abs(w.double().numpy()), np.abs(dy.double().numpy()),
                                    stride)
    assert dx.shape == ref.shape
    assert np.all(np.abs(dx - ref) <= 1e-5 * bound + 1e-30)


@pytest.mark.parametrize("ci,co,stride", LAYER_SHAPES)
def test_conv_weight_grad(H, ci, co, stride):
    g = np.random.default_rng(ci * 3 + co * 5 + stride)
    shape = (2, 9, 7, 6)
    oshape = (2,) + tuple((n - 1) // stride + 1 for n in shape[1:])
    x = _bf16(g.standard_normal(shape + (ci,)))
    dy = _bf16(g.standard_normal(oshape + (co,)))
    dw, db = H.conv3d_wgrad(x.cuda(), dy.cuda(), stride)
    xd, dyd = x.double().numpy(), dy.double().numpy()
    w0 = np.zeros((27, ci, co))
    _, ref_w, ref_b = U.conv3d_backward(xd, w0, dyd, stride)
    _, bw, _ = U.conv3d_backward(np.abs(xd), w0, np.abs(dyd), stride)
    assert np.all(np.abs(dw.cpu().numpy() - ref_w) <= 1e-5 * bw + 1e-30)
    bb = np.abs(dyd).sum(axis=(0, 1, 2, 3))
    assert np.all(np.abs(db.cpu().numpy() - ref_b) <= 1e-5 * bb)


def _case(seed, shape=(2, 12, 10, 9)):
    g = np.random.default_rng(seed)
    inp = np.zeros(shape + (2,), dtype=np.float32)
    inp[..., 0] = g.standard_normal(shape) * 0.5
    inp[..., 1] = g.standard_normal(shape)
    tgt = (0.3 * inp[..., 1] + 0.1 * g.standard_normal(shape)).astype(np.float32)
    return inp, tgt


def _oracle_input(inp):
    x = np.zeros(inp.shape[:-1] + (8,))
    x[..., :2] = inp
    return x


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def test_net_forward_backward_against_oracle(H):
    _net_parity(H, _case(1), backward=True)


def test_net_backward_midsize_ragged(H):
    """Forward and backward on a ragged 50 x 44 x 39 grid (many tiles per
    layer, odd sizes at every downsampling), to the same bars."""
    _net_parity(H, _case(6, (1, 50, 44, 39)), backward=True)


def test_net_forward_96cubed(H):
    """The forward pass at the warm-start benchmark's grid (96^3), to the
    same output bar (the rounding depth per output does not grow with the
    grid; the FP64 backward oracle at this size takes about a minute, so the
    gradients are checked on the ragged mid-size grid above)."""
    _net_parity(H, _case(7, (1, 96, 96, 96)), backward=False)


def _net_parity(H, case, backward):
    inp, tgt = case
    B = inp.shape[0]
    P = U.init_params(3)
    g = np.random.default_rng(4)
    for k in P:
        if k.endswith(".b"):
            P[k] = 0.05 * g.standard_normal(P[k].shape)
    net = H.net(inp.shape[1:4], max_batch=B, seed=0)
    net.set_state(flat_params(P).astype(np.float32))
    inp_d, tgt_d = torch.from_numpy(inp).cuda(), torch.from_numpy(tgt).cuda()
    y = net.forward(inp_d)
    loss, dy = net.loss(y, tgt_d)
    net.zero_grad()
    net.backward(dy)
    torch.cuda.synchronize()
    # oracle with the same (FP32) parameters
    P32 = unflat(flat_params(P).astype(np.float32).astype(np.float64))
    yo, cache = U.forward(P32, _oracle_input(inp.astype(np.float64)))
    lo, dyo = U.mse(yo, tgt.astype(np.float64))
    e_y = _rel(y.cpu().numpy(), yo)
    print("grid %s: output rel err %.2e" % (inp.shape[1:4], e_y), flush=True)
    assert e_y < 2e-2, e_y
    assert abs(loss - lo) <= 2e-2 * lo
    if not backward:
        net.close()
        return
    Go = U.backward(P32, cache, dyo)
    # the loss gradient is formed from the library's own output
    np.testing.assert_allclose(dy.cpu().numpy(), 2 * (y.cpu().numpy() - tgt) / tgt.size,
                               rtol=1e-6, atol=1e-12)
    _, grads = net.params()
    G = unflat(grads.cpu().numpy().astype(np.float64))
    errs = {k: _rel(G[k], Go[k]) for k in Go}
    print("output rel err %.2e; gradient rel errs %s" % (e_y, errs))
    bad = {k: v for k, v in errs.items() if v > 0.15}
    assert not bad, errs
    net.close()


def test_h1_loss_kernel(H):
    inp, tgt = _case(5, (2, 9, 7, 6))
    net = H.net(inp.shape[1:4], max_batch=2, seed=3)
    y = net.forward(torch.from_numpy(inp).cuda())
    loss, dy = net.loss_h1(y, torch.from_numpy(tgt).cuda(), 0.05)
    lo, dyo = U.h1_loss(y.cpu().numpy().astype(np.float64), tgt.astype(np.float64), 0.05)
    assert abs(loss - lo) <= 1e-5 * abs(lo)
    np.testing.assert_allclose(dy.cpu().numpy(), dyo, rtol=1e-4, atol=1e-6 * np.abs(dyo).max())
    net.close()


def test_net_deterministic_and_state_roundtrip(H):
    inp, tgt = _case(2, (1, 9, 8, 11))
    inp_d, tgt_d = torch.from_numpy(inp).cuda(), torch.from_numpy(tgt).cuda()
    n1 = H.net(inp.shape[1:4], max_batch=1, seed=11)
    n2 = H.net(inp.shape[1:4], max_batch=1, seed=12)
    outs, grads = [], []
    for _ in range(2):
        y = n1.forward(inp_d)
        _, dy = n1.loss(y, tgt_d)
        n1.zero_grad()
        n1.backward(dy)
        outs.append(y.clone())
        grads.append(n1.params()[1].clone())
    assert torch.equal(outs[0], outs[1])
    assert torch.equal(grads[0], grads[1])
    n1.adam_step(1e-3)
    n2.set_state(n1.get_state())
    assert torch.equal(n1.forward(inp_d), n2.forward(inp_d))
    np.testing.assert_array_equal(n1.get_state(), n2.get_state())
    n1.close()
    n2.close()


def test_adam_kernel(H):
    net = H.net((4, 4, 4), max_batch=1, seed=5)
    p, gr = net.params()
    n = net.count
    g = np.random.default_rng(9)
    p0 = g.standard_normal(n).astype(np.float32)
    g1 = g.standard_normal(n).astype(np.float32)
    g2 = g.standard_normal(n).astype(np.float32)
    state = np.zeros((3, n), dtype=np.float32)
    state[0] = p0
    net.set_state(state)
    P, M, V = {"a": p0.astype(np.float64)}, {"a": np.zeros(n)}, {"a": np.zeros(n)}
    for step, gg in ((1, g1), (2, g2)):
        gr.copy_(torch.from_numpy(gg).cuda())
        net.adam_step(lr=1e-2, b1=0.9, b2=0.999, eps=1e-8)
        U.adam(P, {"a": gg.astype(np.float64)}, M, V, step, lr=1e-2)
    torch.cuda.synchronize()
    st = net.get_state()
    np.testing.assert_allclose(st[0], P["a"], rtol=0, atol=2e-6)
    np.testing.assert_allclose(st[1], M["a"], rtol=1e-5, atol=1e-7)
    # beta2 = 0.999 rounds to FP32 with a relative error of 1.3e-5 in 1 - beta2
    np.testing.assert_allclose(st[2], V["a"], rtol=3e-5, atol=1e-9)
    net.close()


def test_training_reduces_loss(H):
    inp, tgt = _case(3, (2, 16, 16, 16))
    inp_d, tgt_d = torch.from_numpy(inp).cuda(), torch.from_numpy(tgt).cuda()
    net = H.net(inp.shape[1:4], max_batch=2, seed=1)
    losses = []
    for _ in range(60):
        y = net.forward(inp_d)
        loss, dy = net.loss(y, tgt_d)
        losses.append(loss)
        net.zero_grad()
        net.backward(dy)
        net.adam_step(2e-3)
    print("losses", losses[0], losses[-1])
    assert np.all(np.isfinite(losses))
    assert losses[-1] < 0.5 * losses[0], (losses[0], losses[-1])
    net.close()


def test_net_rejects_bad_shapes(H):
    from paper_2501_03743_amd import sstep
    with pytest.raises(sstep.SspError):
        H.net((2, 8, 8))
    net = H.net((8, 8, 8), max_batch=1)
    with pytest.raises(ValueError):
        net.forward(torch.zeros((1, 8, 8, 9, 2), device="cuda"))
    with pytest.raises(sstep.SspError):
        net.forward(torch.zeros((2, 8, 8, 8, 2), device="cuda"))
    net.close()


def _fields(shape, seed):
    """log k ~ N(0, 0.25) and a source f whose mean square is exactly 4
    (values 0, +-2, +-4 in the proportions 3/8, 1/2, 1/8), so rms(f) = 2 and
    f / rms(f) are exact in any summation order."""
    g = np.random.default_rng(seed)
    n = int(np.prod(shape))
    assert n % 8 == 0
    mag = np.concatenate([np.zeros(3 * n // 8), np.full(n // 2, 2.0), np.full(n // 8, 4.0)])
    f = g.permutation(mag) * g.choice([-1.0, 1.0], n)
    logk = 0.5 * g.standard_normal(n)
    return logk, f


@pytest.mark.parametrize("shape", [(40, 30, 26), (96, 96, 96)])
def test_predict_matches_forward(H, shape):
    """ssp_net_predict (features, forward with the decoder's concatenations
    read in place, FP64 scaling) equals the composition of the FP32 input
    pair, ssp_net_forward (which builds the concatenated buffers) and
    y * rms(f) * out_scale, bit for bit."""
    from paper_2501_03743_amd import sstep
    P = U.init_params(3)
    g = np.random.default_rng(8)
    for k in P:
        if k.endswith(".b"):
            P[k] = 0.05 * g.standard_normal(P[k].shape)
    net = H.net(shape, max_batch=1, seed=0)
    net.set_state(flat_params(P).astype(np.float32))
    out_scale = 0.37
    for seed, zero_f in ((0, False), (1, True)):
        logk, f = _fields(shape, seed)
        if zero_f:
            f[:] = 0.0
        fs = float(np.sqrt(np.sum(f * f) / f.size)) or 1.0
        inp = np.stack([logk, f / fs], axis=-1).astype(np.float32).reshape((1,) + shape + (2,))
        y = net.forward(torch.from_numpy(inp).cuda())
        ref = y.reshape(-1).double() * (fs * out_scale)
        x = net.predict(torch.from_numpy(logk).cuda(), torch.from_numpy(f).cuda(), out_scale)
        torch.cuda.synchronize()
        assert torch.equal(x, ref), (seed, float((x - ref).abs().max()))
        assert float(ref.abs().max()) > 0.0
    # its activations are not a training forward's
    with pytest.raises(sstep.SspError):
        net.backward(torch.zeros(int(np.prod(shape)), device="cuda"))
    net.close()
