"""Parity of the learned-null kernels (features, network forward/backward, Adam) with the
FP64 CPU oracle (needs an MI355X)."""
import os
import tempfile

import numpy as np
import pytest

import workloads
from oracle import mlp
from oracle.features import column_moments, step_features
from tests.gpu_util import dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(lib):
    c = lib.Context(0)
    yield c
    c.close()


def _net(lib, ctx, seed=3):
    g = workloads.rng(seed)
    p = workloads.mlp_init(seed)
    p[1024:1088] = g.standard_normal(64).astype(np.float32) * 0.1
    net = lib.ThresholdNet(ctx, p)
    mu = g.standard_normal(16).astype(np.float32)
    sd = (0.5 + g.random(16)).astype(np.float32)
    net.set_norm(mu, sd)
    return net, p, mu, sd


def _std(feats, mu, sd):
    # the device standardises in FP32; the oracle takes those FP32 inputs exactly
    return ((feats - mu) / sd).astype(np.float32).astype(np.float64)


def test_params_are_bf16_rounded(lib, ctx):
    net, p, _, _ = _net(lib, ctx)
    assert np.array_equal(net.params(bf16=False), p)
    assert np.array_equal(net.params(bf16=True), mlp.bf16_round(p))


def test_forward_matches_oracle(lib, ctx):
    net, p, mu, sd = _net(lib, ctx)
    feats = workloads.rng(4).standard_normal((1000, 16)).astype(np.float32) * 3
    out = net.forward(dev(feats)).cpu().numpy()
    ref, _ = mlp.forward(mlp.bf16_round(p).astype(np.float64), _std(feats, mu, sd))
    scale = np.abs(ref).max()
    assert np.max(np.abs(out - ref)) <= 1e-5 * scale


def test_gradient_matches_oracle(lib, ctx):
    net, p, mu, sd = _net(lib, ctx, seed=5)
    g = workloads.rng(6)
    for B in (1, 31, 64, 1000):
        feats = g.standard_normal((B, 16)).astype(np.float32)
        targ = g.standard_normal((B, 2)).astype(np.float32)
        grad, loss = net.grad(dev(feats), dev(targ))
        grad = grad.cpu().numpy()
        w = mlp.bf16_round(p).astype(np.float64)
        x = _std(feats, mu, sd)
        ref = mlp.backward(w, x, targ)
        assert np.max(np.abs(grad - ref)) <= 1e-4 * np.abs(ref).max(), B
        assert abs(float(loss.cpu()[0]) - mlp.loss(w, x, targ)) <= 1e-5 * mlp.loss(w, x, targ)


def test_adam_step_matches_oracle(lib, ctx):
    net, p, mu, sd = _net(lib, ctx, seed=7)
    g = workloads.rng(8)
    B = 256
    feats = g.standard_normal((B, 16)).astype(np.float32)
    targ = g.standard_normal((B, 2)).astype(np.float32)
    lr = 1e-3
    net.train(dev(feats), dev(targ), epochs=1, batch=B, lr=lr)
    got = net.params(bf16=False)
    w = mlp.bf16_round(p).astype(np.float64)
    grad = mlp.backward(w, _std(feats, mu, sd), targ)
    ref, _, _ = mlp.adam_step(p.astype(np.float64), grad, np.zeros_like(grad), np.zeros_like(grad), 1, lr)
    # the first Adam step moves every weight by ~lr * sign(g); compare the moves
    mv, rmv = got - p, ref - p
    big = np.abs(grad) > 1e-3 * np.abs(grad).max()
    assert np.allclose(mv[big], rmv[big], rtol=1e-3, atol=1e-6 * lr)
    assert np.array_equal(net.params(bf16=True), mlp.bf16_round(got))


def test_training_reduces_loss_and_roundtrips(lib, ctx):
    g = workloads.rng(9)
    B = 4096
    feats = g.standard_normal((B, 16)).astype(np.float32)
    targ = np.stack([np.sin(feats[:, 0]) + 0.5 * feats[:, 1], feats[:, 2] * feats[:, 3]], 1).astype(np.float32)
    net = lib.ThresholdNet(ctx, workloads.mlp_init(10))
    hist = net.train(dev(feats), dev(targ), epochs=40, batch=256, lr=3e-3)
    assert hist[-1] < 0.3 * hist[0]
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "net.bin")
        net.save(path)
        net2 = lib.ThresholdNet.load(ctx, path)
        a = net.forward(dev(feats[:100])).cpu().numpy()
        b = net2.forward(dev(feats[:100])).cpu().numpy()
        assert np.array_equal(a, b)


def test_step_features_match_oracle(lib, ctx):
    net = workloads.ar2_network(seed=1, T=2005)
    from oracle.stats import embed
    cand, y = embed(net.data, target=0, max_lag=5)
    g = workloads.rng(11)
    cm = g.standard_normal(9) * 0.01
    idx = [0, 3, 4, 7, 9, 12, 20, 21, 24]
    f = ctx.step_features(dev(cm), dev(y), dev(cand), idx, 1, 1, 3, 4, 200).cpu().numpy()
    ref = step_features(y.size, 1, 1, 3, 4, 200, cm, column_moments(y), [column_moments(cand[i]) for i in idx])
    assert np.allclose(f, ref.astype(np.float32), rtol=2e-6, atol=1e-6)
