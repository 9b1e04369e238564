"""The learned null: training examples, standardisation and calibration against the CPU
oracle, and the gate inside select_parents (needs an MI355X)."""
import numpy as np
import pytest

import workloads
from oracle import mlp
from oracle.features import column_moments, step_features
from oracle.ksg import ksg_cmi
from oracle.stats import embed, max_statistic, order_statistic_threshold
from tests.gpu_util import dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(lib):
    c = lib.Context(0)
    yield c
    c.close()


def _net_data(seed, T):
    return workloads.ar2_network(seed=seed, T=T, burn=200).data


def test_null_examples_match_oracle(lib, ctx):
    data = _net_data(70, 305)  # N = 300
    cand, y = embed(data, target=0, max_lag=5)
    P = 39
    perms = workloads.permutations(y.size, P, seed=71)
    cond = [0, 7]
    pool = [c for c in range(cand.shape[0]) if c not in cond][:9]
    table, _ = ctx.greedy_step(dev(cand), dev(y), pool, cond, dev(perms), k=4)
    g = workloads.rng(72)
    subsets = [[0], list(range(9)), [1, 4, 8], sorted(g.choice(9, 5, replace=False).tolist())]
    feats, targ, obs = ctx.null_examples(table, pool, subsets, dev(cand), dev(y), dz=2, k=4)
    feats, targ, obs = feats.cpu().numpy(), targ.cpu().numpy(), obs.cpu().numpy()
    # oracle table of the same step
    z = np.stack([cand[c] for c in cond], 1)
    ref = np.empty((len(pool), P + 1))
    for ci, c in enumerate(pool):
        ref[ci, 0] = ksg_cmi(cand[c], y, z, 4)
        for p in range(P):
            ref[ci, p + 1] = ksg_cmi(cand[c][perms[p]], y, z, 4)
    ymom = column_moments(y)
    n = y.size
    for si, sub in enumerate(subsets):
        ms = max_statistic(ref[sub], 0.05)
        f = step_features(n, 1, 1, 2, 4, P, ref[sub, 0], ymom, [column_moments(cand[pool[r]]) for r in sub])
        assert np.allclose(feats[si], f.astype(np.float32), rtol=2e-6, atol=2e-6), si
        assert abs(targ[si, 0] - np.sqrt(n) * ms.tau05) <= 1e-5 * max(1, abs(np.sqrt(n) * ms.tau05))
        assert abs(targ[si, 1] - np.sqrt(n) * ms.tau01) <= 1e-5 * max(1, abs(np.sqrt(n) * ms.tau01))
        assert abs(obs[si, 0] - np.sqrt(n) * ms.t_obs) <= 1e-11
        assert obs[si, 1] == float(ms.significant)


def test_fit_norm_matches_numpy(lib, ctx):
    g = workloads.rng(73)
    feats = (g.standard_normal((3001, 16)) * np.arange(1, 17) + np.arange(16)).astype(np.float32)
    feats[:, 5] = 2.5  # constant feature -> sd 1
    net = lib.ThresholdNet(ctx, workloads.mlp_init(1))
    net.fit_norm(dev(feats))
    # the standardisation in use equals numpy's mean/std: check through the forward pass
    p = workloads.mlp_init(1)
    out = net.forward(dev(feats[:50])).cpu().numpy()
    f64 = feats.astype(np.float64)
    mu = f64.mean(0)
    sd = f64.std(0)
    sd[5] = 1.0
    x = ((feats[:50] - mu.astype(np.float32)) / sd.astype(np.float32)).astype(np.float32).astype(np.float64)
    ref, _ = mlp.forward(mlp.bf16_round(p).astype(np.float64), x)
    assert np.max(np.abs(out - ref)) <= 1e-4 * max(1.0, np.abs(ref).max())


def _calib_ref(pred, obs, rate, include_rate=None):
    s = np.maximum(np.abs(pred[:, 1] - pred[:, 0]), 1e-30)
    u = (obs[:, 0] - pred[:, 0]) / s
    sig = obs[:, 1] > 0.5
    allow_lo = int(np.floor(rate / 2 * len(u)))
    allow_hi = allow_lo if include_rate is None else int(np.floor(include_rate * len(u)))
    un = np.sort(u[~sig])[::-1]
    up = np.sort(u[sig])
    hi = max(0.0, un[allow_hi]) if un.size > allow_hi else 0.0
    lo = max(0.0, -up[allow_lo]) if up.size > allow_lo else 0.0
    return lo, hi


def test_calibration_matches_reference(lib, ctx):
    g = workloads.rng(74)
    B = 4000
    p = workloads.mlp_init(5)
    net = lib.ThresholdNet(ctx, p)
    feats = g.standard_normal((B, 16)).astype(np.float32)
    w = mlp.bf16_round(p).astype(np.float64)
    pred, _ = mlp.forward(w, feats.astype(np.float64))
    obs = np.stack([pred[:, 0] + g.standard_normal(B) * np.abs(pred[:, 1] - pred[:, 0]),
                    (g.random(B) < 0.5).astype(np.float64)], 1)
    r = net.calibrate(dev(feats), dev(obs), rate=0.01)
    lo, hi = _calib_ref(pred, obs, 0.01)
    assert abs(r["margin_lo"] - lo) <= 1e-4 * max(1, lo) and abs(r["margin_hi"] - hi) <= 1e-4 * max(1, hi)
    assert r["wrong"] <= 2 * int(0.005 * B) + 2


@pytest.mark.parametrize("include_rate", [0.0, 0.001, 0.02])
def test_calibration_per_side_matches_reference(lib, ctx, include_rate):
    g = workloads.rng(75)
    B = 3000
    p = workloads.mlp_init(6)
    net = lib.ThresholdNet(ctx, p)
    feats = g.standard_normal((B, 16)).astype(np.float32)
    w = mlp.bf16_round(p).astype(np.float64)
    pred, _ = mlp.forward(w, feats.astype(np.float64))
    obs = np.stack([pred[:, 0] + g.standard_normal(B) * np.abs(pred[:, 1] - pred[:, 0]),
                    (g.random(B) < 0.4).astype(np.float64)], 1)
    r = net.calibrate(dev(feats), dev(obs), rate=0.01, include_rate=include_rate)
    lo, hi = _calib_ref(pred, obs, 0.01, include_rate)
    assert abs(r["margin_lo"] - lo) <= 1e-4 * max(1, lo) and abs(r["margin_hi"] - hi) <= 1e-4 * max(1, hi)
    # wrong inclusions are bounded by the include allowance (ties at the margin aside)
    s_ = np.maximum(np.abs(pred[:, 1] - pred[:, 0]), 1e-30)
    u = (obs[:, 0] - pred[:, 0]) / s_
    assert int(np.sum((u > r["margin_hi"] + 1e-4 * max(1, hi)) & (obs[:, 1] < 0.5))) <= int(include_rate * B)
    # the symmetric form equals rate/2 on both sides
    r2 = net.calibrate(dev(feats), dev(obs), rate=0.01, include_rate=0.005)
    r3 = net.calibrate(dev(feats), dev(obs), rate=0.01)
    assert r2["margin_lo"] == r3["margin_lo"] and r2["margin_hi"] == r3["margin_hi"]


def _dataset(lib, ctx, seeds, P=500, n_sub=64, m_max=4, steps=3):
    """Examples from greedy steps of seeded 20-node logistic-map networks (one trial,
    N = 2995, 100 candidates; targets, conditioning sets and subsets seeded)."""
    from paper_1807_10459_amd.learned_null import StepSpec, build_dataset
    specs = []
    for s in seeds:
        net = workloads.logistic_network(seed=s, n_trials=1, T=3000)
        g = workloads.rng(s + 5000)
        target = int(g.integers(0, 20))
        dcand, dy = ctx.embed(dev(net.data), target=target, max_lag=5)
        perms = dev(workloads.permutations(dy.shape[0], P, seed=s + 6000))
        true = [src * 5 + lag - 1 for (src, tgt, lag) in net.edges if tgt == target]
        true += [target * 5, target * 5 + 1]
        for _ in range(steps):
            m = int(g.integers(0, m_max + 1))
            if g.random() < 0.5:  # conditioning on (a prefix of) the true parents and own past
                rest = [c for c in range(100) if c not in true]
                cond = sorted((true + [rest[i] for i in g.permutation(len(rest))])[:m])
            else:
                cond = sorted(g.choice(100, m, replace=False).tolist())
            pool = [c for c in range(100) if c not in cond]
            subs = [list(range(len(pool)))]
            for _ in range(n_sub - 1):
                size = int(np.exp(g.uniform(0, np.log(len(pool)))))
                subs.append(sorted(g.choice(len(pool), max(1, size), replace=False).tolist()))
            specs.append(StepSpec(dcand, dy, pool, cond, perms, subs))
    return build_dataset(ctx, specs)


def test_learned_gate_gain_over_table_and_select_parents(lib, ctx):
    """Train on steps of seeded networks, calibrate on held-out networks, then (a) compare the
    fraction of held-out steps left to the surrogate test with that of a bucket-mean threshold
    table calibrated the same way (the ablation: what the network gains), and (b) run
    select_parents with the gate, judged by the plain test."""
    import torch
    from paper_1807_10459_amd.learned_null import calibrate, train_threshold_net
    feats, targ, obs, _ = _dataset(lib, ctx, range(100, 132))
    hf, ht, ho, _ = _dataset(lib, ctx, range(300, 310))
    order = torch.from_numpy(workloads.permutations(feats.shape[0], 1, seed=7)[0].astype(np.int64)).cuda()
    net, hist = train_threshold_net(ctx, feats[order].contiguous(), targ[order].contiguous(),
                                    workloads.mlp_init(11), epochs=60, batch=512, lr=2e-3)
    assert hist[-1] < 0.25 * hist[0]
    rate = 0.01
    cal = calibrate(net, hf, ho, rate=rate)
    # baseline: mean thresholds per (log N, log c, d_z) bucket of the training set
    F, Tg = feats.cpu().numpy(), targ.cpu().numpy()
    HF, HO = hf.cpu().numpy(), ho.cpu().numpy()

    def key(f):
        return (round(float(f[0]), 1), int(np.floor(float(f[5]) / 0.5)), int(f[3]))
    table = {}
    for f, t in zip(F, Tg):
        table.setdefault(key(f), []).append(t)
    glob = Tg.mean(0)
    pred_tab = np.array([np.mean(table[key(f)], 0) if key(f) in table else glob for f in HF])
    lo, hi = _calib_ref(pred_tab, HO, rate)
    s = np.maximum(np.abs(pred_tab[:, 1] - pred_tab[:, 0]), 1e-30)
    u = (HO[:, 0] - pred_tab[:, 0]) / s
    fallback_tab = float(np.mean((u <= hi) & (u >= -lo)))
    mse_net = float(((net.forward(hf).cpu().numpy() - ht.cpu().numpy()) ** 2).sum(1).mean())
    mse_tab = float(((pred_tab - ht.cpu().numpy()) ** 2).sum(1).mean())
    print(f"held-out: network fallback {cal['fallback']:.3f} mse {mse_net:.4f}; "
          f"bucket table fallback {fallback_tab:.3f} mse {mse_tab:.4f}")
    assert cal["fallback"] < fallback_tab
    assert cal["wrong"] <= int(rate * HF.shape[0]) + 1
    # the gate in select_parents, judged by the plain test on every step
    data = workloads.logistic_network(seed=999, n_trials=1, T=3000).data
    perms = dev(workloads.permutations(2995, 500, seed=998))
    plain = ctx.select_parents(dev(data), 4, perms, k=4, max_lag=5)
    judged = ctx.select_parents(dev(data), 4, perms, k=4, max_lag=5, learned=net,
                                margin_lo=cal["margin_lo"], margin_hi=cal["margin_hi"], judge=True)
    for st in judged["steps"]:
        print("judged step", st)
    assert judged["parents"] == plain["parents"]
    assert all(st["plain"] in (0, 1) and st["verdict"] in (-1, 0, 1) for st in judged["steps"])
    assert judged["n_disagree"] <= 1
    learned = ctx.select_parents(dev(data), 4, perms, k=4, max_lag=5, learned=net,
                                 margin_lo=cal["margin_lo"], margin_hi=cal["margin_hi"])
    assert learned["n_fallback"] + learned["n_gate_decided"] == learned["n_steps"]
    assert learned["n_gate_decided"] >= 1 and learned["n_cmi"] < plain["n_cmi"]
    if judged["n_disagree"] == 0:
        assert learned["parents"] == plain["parents"]


def test_verify_stop_confirms_every_predicted_stop(lib, ctx):
    """A gate that never includes (margin_hi huge) and stops whenever u < 0: with verify_stop
    every predicted stop runs the plain test, so the selection is the plain one step for step
    and no step is decided by the gate alone; without it the first predicted stop ends the
    selection there."""
    net = lib.ThresholdNet(ctx, workloads.mlp_init(21))
    data = workloads.logistic_network(seed=998, n_trials=1, T=3000).data
    perms = dev(workloads.permutations(2995, 200, seed=997))
    kw = dict(k=4, max_lag=5, prune=False)
    plain = ctx.select_parents(dev(data), 6, perms, **kw)
    ver = ctx.select_parents(dev(data), 6, perms, learned=net, margin_lo=0.0, margin_hi=1e30, verify_stop=True, **kw)
    assert ver["parents"] == plain["parents"] and ver["n_steps"] == plain["n_steps"]
    assert ver["n_gate_decided"] == 0 and ver["n_fallback"] == ver["n_steps"]
    verdicts = [st["verdict"] for st in ver["steps"]]
    assert all(v in (-1, 0) for v in verdicts)
    assert all(st["plain"] == pst["plain"] for st, pst in zip(ver["steps"], plain["steps"]))
    raw = ctx.select_parents(dev(data), 6, perms, learned=net, margin_lo=0.0, margin_hi=1e30, **kw)
    if -1 in verdicts:
        first = verdicts.index(-1)
        assert raw["n_steps"] == first + 1 and raw["n_gate_decided"] == 1
        assert raw["parents"] == plain["parents"][:first]
    else:
        assert raw["parents"] == plain["parents"]


def test_deep_step_margins(lib, ctx):
    """With deep_dz = 1 the first step (no conditioning) uses margin_lo/margin_hi and every later
    step the deep pair: huge shallow margins leave step 0 to the surrogates, zero deep margins let
    the gate decide every later step; negative deep_dz is rejected."""
    net = lib.ThresholdNet(ctx, workloads.mlp_init(22))
    data = workloads.logistic_network(seed=996, n_trials=1, T=3000).data
    perms = dev(workloads.permutations(2995, 99, seed=995))
    r = ctx.select_parents(dev(data), 5, perms, k=4, max_lag=5, learned=net, margin_lo=1e30, margin_hi=1e30,
                           deep_margins=(1, 0.0, 0.0), max_steps=6)
    v = [st["verdict"] for st in r["steps"]]
    assert v[0] == 0 and r["n_fallback"] >= 1
    assert all(x in (-1, 1) for x in v[1:]), v
    assert r["n_gate_decided"] == r["n_steps"] - 1
    with pytest.raises(lib.KsgError):
        ctx.select_parents(dev(data), 5, perms, k=4, max_lag=5, learned=net, deep_margins=(-1, 0.0, 0.0))
