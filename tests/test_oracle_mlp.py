"""Pins of the MLP and feature oracles (CPU only)."""
import numpy as np
import pytest
import torch
from scipy import stats

import workloads
from oracle import mlp
from oracle.features import column_moments, step_features


def test_param_count():
    assert mlp.N_PARAMS == 5378


def test_bf16_round_matches_library():
    g = workloads.rng(1)
    a = np.concatenate([g.standard_normal(20000).astype(np.float32) * 10.0 ** g.integers(-5, 5, 20000),
                        np.array([0.0, -0.0, 1.0, 1.00390625, 1.01171875, 3.0e38], np.float32)])
    a = a.astype(np.float32)
    ref = torch.from_numpy(a).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(mlp.bf16_round(a), ref)
    # ties to even: 1 + 2^-8 is halfway between 1 and 1 + 2^-7 -> rounds to 1
    assert mlp.bf16_round(np.float32(1.00390625)) == 1.0


def _torch_mlp(flat, feats):
    p = {k: torch.from_numpy(np.array(v)) for k, v in mlp.unpack(flat).items()}
    f = torch.from_numpy(np.asarray(feats, np.float64))
    h1 = torch.relu(torch.nn.functional.linear(f, p["W1"], p["b1"]))
    h2 = torch.relu(torch.nn.functional.linear(h1, p["W2"], p["b2"]))
    return torch.nn.functional.linear(h2, p["W3"], p["b3"])


def test_forward_matches_library():
    flat = mlp.bf16_round(workloads.mlp_init(3)).astype(np.float64)
    feats = workloads.rng(2).standard_normal((37, 16))
    out, _ = mlp.forward(flat, feats)
    assert np.allclose(out, _torch_mlp(flat, feats).numpy(), rtol=1e-13, atol=1e-13)


def test_backward_finite_differences():
    g = workloads.rng(3)
    flat = workloads.mlp_init(4).astype(np.float64)
    flat[1024:1088] = g.standard_normal(64) * 0.1  # nonzero biases
    feats = g.standard_normal((9, 16))
    targ = g.standard_normal((9, 2))
    grad = mlp.backward(flat, feats, targ)
    idx = np.concatenate([g.choice(mlp.N_PARAMS, 200, replace=False), [5376, 5377, 1087, 5183]])
    h = 1e-6
    for i in idx:
        e = np.zeros_like(flat)
        e[i] = h
        fd = (mlp.loss(flat + e, feats, targ) - mlp.loss(flat - e, feats, targ)) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-7 + 1e-5 * abs(grad[i]), i


def test_backward_matches_autograd():
    g = workloads.rng(5)
    flat = workloads.mlp_init(6).astype(np.float64)
    feats = g.standard_normal((33, 16))
    targ = g.standard_normal((33, 2))
    t = torch.from_numpy(flat.copy()).requires_grad_(True)
    offs, parts = 0, {}
    for name, shape in mlp.SIZES:
        n = int(np.prod(shape))
        parts[name] = t[offs:offs + n].reshape(shape)
        offs += n
    f = torch.from_numpy(feats)
    h1 = torch.relu(f @ parts["W1"].T + parts["b1"])
    h2 = torch.relu(h1 @ parts["W2"].T + parts["b2"])
    out = h2 @ parts["W3"].T + parts["b3"]
    L = 0.5 * ((out - torch.from_numpy(targ)) ** 2).sum() / 33
    L.backward()
    assert np.allclose(mlp.backward(flat, feats, targ), t.grad.numpy(), rtol=1e-12, atol=1e-14)


def test_adam_matches_library():
    g = workloads.rng(7)
    w0 = g.standard_normal(50)
    wt = torch.tensor(w0.copy(), requires_grad=True)
    opt = torch.optim.Adam([wt], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    w, m, v = w0.copy(), np.zeros(50), np.zeros(50)
    for step in range(1, 6):
        grad = g.standard_normal(50)
        wt.grad = torch.tensor(grad)
        opt.step()
        w, m, v = mlp.adam_step(w, grad, m, v, step, 1e-2)
    assert np.allclose(w, wt.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_column_moments_match_library():
    g = workloads.rng(8)
    col = (g.standard_normal(5000) ** 3 + 0.5 * np.arange(5000) / 5000).astype(np.float32)
    sk, ku, ac = column_moments(col)
    a = col.astype(np.float64)
    assert abs(sk - stats.skew(a, bias=True)) < 1e-10
    assert abs(ku - stats.kurtosis(a, fisher=True, bias=True)) < 1e-10
    d = a - a.mean()
    assert abs(ac - np.dot(d[:-1], d[1:]) / np.dot(d, d)) < 1e-12


def test_step_features_layout():
    cm = np.array([0.1, 0.3, 0.2, 0.3])
    f = step_features(10000, 1, 1, 3, 4, 200, cm, (0.5, 1.0, 0.2), [(1, 2, 0.5), (3, 4, -0.5)] * 2)
    assert f.shape == (16,)
    assert f[0] == pytest.approx(np.log(10000)) and f[3] == 3 and f[4] == 4
    assert f[5] == pytest.approx(np.log(4)) and f[6] == pytest.approx(np.log(200))
    assert f[7] == pytest.approx(30.0) and f[8] == pytest.approx(30.0)
    assert f[9] == pytest.approx(100 * 0.225) and f[10] == pytest.approx(100 * np.std(cm))
    assert f[13] == pytest.approx(2.0) and f[14] == pytest.approx(3.0) and f[15] == pytest.approx(0.5)
