"""GPU checks of the warm-start network kernels against the FP64 oracle.

The oracle rounds the operands to bfloat16 exactly as the kernels do and
accumulates in FP64; the kernels accumulate in FP32 on the matrix cores, so
layer outputs and gradients agree to FP32 accumulation error (norm-relative
1e-5), at 16^3, at the training size 64^3, at the smallest grid 8^3 and at
56^3 (a last weight-gradient block with fewer tiles).  A chained forward pass can
differ by one bfloat16 rounding of an intermediate activation, so it is
compared at 2e-2 (the inference forward against the same network run layer
by layer on the GPU at 2e-3), and so are the losses of chained training
steps; the loss
kernel alone is compared on the GPU's own network output (1e-6), and two
Adam steps against the oracle's to 2% of the learning rate on the weights
whose gradients stand far above Adam's epsilon.
"""
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

L = 16


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def nrel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-30))


@pytest.fixture(scope="module")
def net():
    from paper_1102_2193_amd import nn
    say("case: network on a 16^3 grid")
    return nn.Net(L, seed=3)


def rand_layer(rng, l):
    from paper_1102_2193_amd import nn
    W = rng.normal(size=(nn.COUT[l], nn.CIN[l], 27)).astype(np.float32) * 0.1
    b = rng.normal(size=nn.COUT[l]).astype(np.float32) * 0.1
    return W, b


@pytest.mark.parametrize("l", [0, 1, 2, 3])
def test_layer_forward_matches_oracle(net, l):
    from oracle import cnn
    from paper_1102_2193_amd import nn
    say("case: layer %d forward" % l)
    rng = np.random.default_rng(10 + l)
    W, b = rand_layer(rng, l)
    net.set_layer(l, W, b)
    x = rng.normal(size=(nn.CIN[l], L, L, L)).astype(np.float32)
    z = net.layer_forward(l, x)
    ref = cnn.conv3d(cnn.bf16_round(x), cnn.bf16_round(W), b.astype(np.float64))
    e = nrel(z, ref)
    say("   rel err %.3e" % e)
    assert e < 1e-5


@pytest.mark.parametrize("l", [0, 1, 2, 3])
def test_layer_backward_matches_oracle(net, l):
    from oracle import cnn
    from paper_1102_2193_amd import nn
    say("case: layer %d backward" % l)
    rng = np.random.default_rng(20 + l)
    W, b = rand_layer(rng, l)
    net.set_layer(l, W, b)
    x = rng.normal(size=(nn.CIN[l], L, L, L)).astype(np.float32)
    dz = rng.normal(size=(nn.COUT[l], L, L, L)).astype(np.float32)
    dW, db, dx = net.layer_backward(l, x, dz)
    rdx, rdW, rdb = cnn.conv3d_backward(cnn.bf16_round(x), cnn.bf16_round(W), cnn.bf16_round(dz))
    e = (nrel(dW, rdW), nrel(db, rdb), nrel(dx, rdx))
    say("   rel err dW %.3e db %.3e dx %.3e" % e)
    assert max(e) < 1e-5


def test_features_match_oracle(net):
    from oracle import cnn
    from paper_1102_2193_amd import inputs, nn
    say("case: features")
    pitch = 16.0
    c = nn.make_case((7.3, 8.0, 8.6), 4.5, pitch, "planar", 0.495, 0.5)
    f = net.features(c)
    qh = inputs.helix_q(L, L, L, 2 * math.pi / pitch, 1.0)
    ref = cnn.features(L, (7.3, 8.0, 8.6), 4.5, pitch, -1.0, qh)
    np.testing.assert_allclose(f, ref, atol=2e-7)


def test_chained_forward_and_warm_start(net):
    from oracle import cnn
    from paper_1102_2193_amd import inputs, lc, nn
    say("case: chained forward, warm start into a context")
    rng = np.random.default_rng(5)
    params = cnn.init_params(11)
    for l, (W, b) in enumerate(params):
        net.set_layer(l, W.astype(np.float32), (rng.normal(size=b.shape) * 0.05).astype(np.float32))
    params = [(net.get_layer(l)[0].astype(np.float64), net.get_layer(l)[1].astype(np.float64)) for l in range(4)]
    pitch = 16.0
    c = nn.make_case((8.0, 8.0, 8.0), 3.5, pitch, "normal", 0.495, 0.5)
    dq = net.predict(c)
    qh = inputs.helix_q(L, L, L, 2 * math.pi / pitch, 1.0)
    x = cnn.features(L, (8.0, 8.0, 8.0), 3.5, pitch, 1.0, qh)
    ref, _ = cnn.forward(params, x, bf16=True)
    e = nrel(dq, ref)
    say("   chained rel err %.3e" % e)
    assert e < 2e-2
    ctx = lc.Context([dict(nx=L, precision="fp64", **inputs.NEMATIC)])
    net.warm_start(c, ctx, 0)
    Q = ctx.get_Q(0)
    np.testing.assert_allclose(Q, 0.495 * qh + 0.5 * dq, atol=1e-6)


def test_predict_matches_the_layer_chain(net):
    """The inference forward (first layer computing its features in the
    halo staging, 16-byte output rows) against the same network run layer
    by layer through the single-layer calls (features read from the FP64
    feature kernel, activations packed to BF16 from FP32 SiLU on the host):
    they differ only where an FP32 versus FP64 feature or SiLU value falls
    on the other side of a BF16 rounding."""
    from paper_1102_2193_amd import nn
    say("case: predict against the layer chain")
    rng = np.random.default_rng(12)
    for l in range(4):
        W, b = rand_layer(rng, l)
        net.set_layer(l, W * 0.5, b * 0.5)
    c = nn.make_case((6.2, 9.0, 7.7), 4.0, 12.0, "planar", 0.495, 0.5)
    dq = net.predict(c)
    x = net.features(c)
    for l in range(4):
        z = net.layer_forward(l, x)
        if l < 3:
            zd = z.astype(np.float64)
            x = (zd / (1.0 + np.exp(-zd))).astype(np.float32)
    e = nrel(dq, z)
    say("   predict vs layer chain rel err %.3e" % e)
    assert e < 2e-3   # measured 3.1e-4


def test_training_step_follows_gradient(net):
    from oracle import cnn
    from paper_1102_2193_amd import inputs, nn
    say("case: one training step")
    rng = np.random.default_rng(6)
    params = cnn.init_params(12)
    for l, (W, b) in enumerate(params):
        net.set_layer(l, W.astype(np.float32), b.astype(np.float32))
    params = [(net.get_layer(l)[0].astype(np.float64), net.get_layer(l)[1].astype(np.float64)) for l in range(4)]
    pitch = 16.0
    c = nn.make_case((8.0, 8.0, 8.0), 3.5, pitch, "normal", 0.495, 0.5)
    qh = inputs.helix_q(L, L, L, 2 * math.pi / pitch, 1.0)
    target = 0.495 * qh + 0.05 * rng.normal(size=(5, L, L, L))
    fluid = rng.uniform(size=(L, L, L)) > 0.1
    x = cnn.features(L, (8.0, 8.0, 8.0), 3.5, pitch, 1.0, qh)
    out, cache = cnn.forward(params, x, bf16=True)
    loss_ref, g = cnn.loss_and_grad(out, 0.495 * qh, target, fluid, 0.5)
    grads = cnn.backward(params, cache, g, bf16=True)
    lr = 1e-3
    loss = net.train_step(c, target, fluid, lr)
    say("   loss %.6e vs oracle %.6e" % (loss, loss_ref))
    assert loss == pytest.approx(loss_ref, rel=1e-2)
    for l in range(4):
        W1, _ = net.get_layer(l)
        step = params[l][0] - W1.astype(np.float64)
        gW = grads[l][0]
        big = np.abs(gW) > 0.05 * np.abs(gW).max()
        # first Adam step moves each weight by lr against the sign of its gradient
        agree = np.mean(np.sign(step[big]) == np.sign(gW[big]))
        say("   layer %d: sign agreement %.4f, |step| %.3e" % (l, agree, np.abs(step[big]).mean()))
        assert agree > 0.97
        np.testing.assert_allclose(np.abs(step[big]), lr, rtol=1e-2)


@pytest.fixture(scope="module")
def net64():
    from paper_1102_2193_amd import nn
    say("case: network on a 64^3 grid (the training size)")
    return nn.Net(64, seed=4)


@pytest.mark.parametrize("l", [0, 1, 2, 3])
def test_layer_forward_backward_64cubed(net64, l):
    """Layer parity at the training size: 262,144 sites per layer, the
    weight gradient summed by 256 blocks and then across blocks."""
    from oracle import cnn
    from paper_1102_2193_amd import nn
    say("case: layer %d forward and backward at 64^3" % l)
    n = 64
    rng = np.random.default_rng(40 + l)
    W, b = rand_layer(rng, l)
    net64.set_layer(l, W, b)
    x = rng.normal(size=(nn.CIN[l], n, n, n)).astype(np.float32)
    z = net64.layer_forward(l, x)
    xr, Wr = cnn.bf16_round(x), cnn.bf16_round(W)
    ez = nrel(z, cnn.conv3d(xr, Wr, b.astype(np.float64)))
    dz = rng.normal(size=(nn.COUT[l], n, n, n)).astype(np.float32)
    dW, db, dx = net64.layer_backward(l, x, dz)
    rdx, rdW, rdb = cnn.conv3d_backward(xr, Wr, cnn.bf16_round(dz))
    e = (ez, nrel(dW, rdW), nrel(db, rdb), nrel(dx, rdx))
    say("   rel err z %.3e dW %.3e db %.3e dx %.3e" % e)
    assert max(e) < 1e-5


@pytest.mark.parametrize("n", [8, 56])
def test_layer_forward_backward_smallest_and_ragged_grids(n):
    """8^3, the smallest grid the network takes: two convolution blocks,
    every halo wrapping onto the block's own tile, two weight-gradient
    blocks.  56^3: 686 weight-gradient tiles over 229 blocks of three, the
    last block with two.  Every layer forward and backward, as at 64^3."""
    from oracle import cnn
    from paper_1102_2193_amd import nn
    net = nn.Net(n, seed=9)
    for l in range(4):
        say("case: layer %d forward and backward at %d^3" % (l, n))
        rng = np.random.default_rng(60 + l)
        W, b = rand_layer(rng, l)
        net.set_layer(l, W, b)
        x = rng.normal(size=(nn.CIN[l], n, n, n)).astype(np.float32)
        z = net.layer_forward(l, x)
        xr, Wr = cnn.bf16_round(x), cnn.bf16_round(W)
        ez = nrel(z, cnn.conv3d(xr, Wr, b.astype(np.float64)))
        dz = rng.normal(size=(nn.COUT[l], n, n, n)).astype(np.float32)
        dW, db, dx = net.layer_backward(l, x, dz)
        rdx, rdW, rdb = cnn.conv3d_backward(xr, Wr, cnn.bf16_round(dz))
        e = (ez, nrel(dW, rdW), nrel(db, rdb), nrel(dx, rdx))
        say("   rel err z %.3e dW %.3e db %.3e dx %.3e" % e)
        assert max(e) < 1e-5
    net.close()


def _two_step_case(L, seed):
    from oracle import cnn
    from paper_1102_2193_amd import inputs, nn
    rng = np.random.default_rng(seed)
    pitch = 16.0
    pos = (L / 2, L / 2 - 0.3, L / 2 + 0.2)
    c = nn.make_case(pos, 3.5, pitch, "normal", 0.495, 0.5)
    qh = inputs.helix_q(L, L, L, 2 * math.pi / pitch, 1.0)
    target = 0.495 * qh + 0.05 * rng.normal(size=(5, L, L, L))
    fluid = rng.uniform(size=(L, L, L)) > 0.1
    x = cnn.features(L, pos, 3.5, pitch, 1.0, qh)
    return c, qh, target, fluid, x


def test_loss_of_the_gpu_output():
    """k_loss alone: the loss the training step reports equals the FP64 loss
    of the network output the GPU itself produced (lr = 0: no update)."""
    from oracle import cnn
    from paper_1102_2193_amd import nn
    say("case: loss kernel on the GPU's own output")
    net = nn.Net(L, seed=5)
    params = cnn.init_params(13)
    for l, (W, b) in enumerate(params):
        net.set_layer(l, W.astype(np.float32), b.astype(np.float32))
    c, qh, target, fluid, _ = _two_step_case(L, 7)
    dq = net.predict(c)
    ref, _ = cnn.loss_and_grad(dq, 0.495 * qh, target, fluid, 0.5)
    loss = net.train_step(c, target, fluid, 0.0)
    say("   loss %.9e vs FP64 of the same output %.9e" % (loss, ref))
    # FP32 residuals, FP64 sums: a few FP32 roundings of each term
    assert loss == pytest.approx(ref, rel=1e-6)
    net.close()


def test_two_adam_steps_match_oracle():
    """Two training steps on one case against the oracle's forward, backward
    and Adam in FP64 (bfloat16 operands as on the GPU).  The second Adam step
    mixes both gradients through the moments and the bias corrections
    (t = 2), so the weights after it test k_adam's arithmetic, not only the
    signs of a first step."""
    from oracle import cnn
    from paper_1102_2193_amd import nn
    say("case: two training steps against the oracle's Adam")
    net = nn.Net(L, seed=6)   # fresh Adam state (t = 0, zero moments)
    params = cnn.init_params(14)
    for l, (W, b) in enumerate(params):
        net.set_layer(l, W.astype(np.float32), (np.full(b.shape, 0.01)).astype(np.float32))
    p0 = [(net.get_layer(l)[0].astype(np.float64), net.get_layer(l)[1].astype(np.float64)) for l in range(4)]
    c, qh, target, fluid, x = _two_step_case(L, 8)
    lr = 1e-3
    losses = [net.train_step(c, target, fluid, lr) for _ in range(2)]
    p, state, ref_losses, grads_all = p0, cnn.adam_init(p0), [], []
    for _ in range(2):
        out, cache = cnn.forward(p, x, bf16=True)
        loss, g = cnn.loss_and_grad(out, 0.495 * qh, target, fluid, 0.5)
        grads = cnn.backward(p, cache, g, bf16=True)
        ref_losses.append(loss)
        grads_all.append(grads)
        p, state = cnn.adam_step(p, grads, state, lr)
    say("   losses %s vs oracle %s" % (losses, ref_losses))
    for a, r in zip(losses, ref_losses):
        assert a == pytest.approx(r, rel=1e-2)
    for l in range(4):
        W2, b2 = (v.astype(np.float64) for v in net.get_layer(l))
        for name, got, ref, start, k in (("W", W2, p[l][0], p0[l][0], 0), ("b", b2, p[l][1], p0[l][1], 1)):
            g1, g2 = grads_all[0][l][k], grads_all[1][l][k]
            # elements whose gradients are far above Adam's epsilon in both steps
            big = (np.abs(g1) > 1e-3 * np.abs(g1).max()) & (np.abs(g2) > 1e-3 * np.abs(g2).max())
            d = np.abs((got - start) - (ref - start))[big]
            say("   layer %d %s: %d elements, max |step - oracle step| / lr %.3e" % (l, name, big.sum(), d.max() / lr))
            assert big.sum() > 0.5 * big.size
            assert d.max() < 0.02 * lr
    net.close()
