"""Benchmark: KSG CMI estimates per second, surrogates included, on one MI355X.

Workload (default): greedy parent selection for node 0 of the seeded 5-node linear AR(2)
network, N = 10,000 embedded points, 25 lagged candidates (5 variables x lags 1..5), k = 4,
200 permutation surrogates per candidate, conditioning sets of 1..8 dimensions (the
"forced path": Z = the first m candidates of a fixed seeded order, true parents first).
One step = the whole hot path over that input: lagged embedding, then for m = 1..8 one
batched launch over all (25 - m) x 201 CMI problems (surrogate gathers, k-NN radius,
strict range counts, FP64 digamma sums) and the max-statistic test.  That is 32,964 CMI
estimates per step.  Inputs are resident in HBM before timing starts.

Prints one JSON line.  The roofline object is for the dominant search kernel (the one with
the most device time in the timed steps; each launch is timed by its own HIP events):
algorithmic operations executed (as counted by the library: distances, maxima and compares
of the pairs it visits) over its time, against the FP32 VALU peak for operations that are
not fused multiply-adds: the 157.3 TFLOP/s FP32 vector figure counts an FMA as two
operations, so 78.6 T lane-operations per second (256 CUs x 4 SIMDs x 32 lanes per clock x
2.4 GHz).  "kernels" lists every search kernel the same way.  cpu_baseline times the CPU
oracle on a sample of the same CMIs.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# VALU lane-instructions per second of the part: 256 CUs x 4 SIMDs x 32 lanes x 2.4 GHz (the
# 157.3 TFLOP/s FP32 vector figure counts an FMA as two operations)
PEAK_VALU = 157.3e12 / 2
N_PERM = 200
MAX_LAG = 5
K = 4
FORCED_M = range(1, 9)


def forced_order(net, n_vars=5, L=MAX_LAG, seed=1):
    """Candidate order of the forced path: true parents first, then a seeded shuffle."""
    import workloads
    tgt = net.params["target"]
    first = [tgt * L + 0, tgt * L + 1] + [src * L + (lag - 1) for (src, _, lag) in net.edges]
    rest = [c for c in range(n_vars * L) if c not in first]
    rest = [rest[i] for i in workloads.rng(seed + 7).permutation(len(rest))]
    return first + rest


def _cpu_task(args):
    cand_c, y, z, k, alg = args
    from oracle.ksg import ksg_cmi
    from oracle.ksg2 import ksg2_cmi
    t0 = time.perf_counter()
    v = (ksg2_cmi if alg == 2 else ksg_cmi)(cand_c, y, z, k)
    return v, time.perf_counter() - t0


def cpu_baseline(cand, y, perms, order, sample_per_m=2, workers=None, alg=1):
    """The oracle on a bounded sample of the step's CMIs: (CMI/s, cores, description, values)."""
    import multiprocessing as mp
    tasks, keys = [], []
    for m in FORCED_M:
        z = np.stack([cand[c] for c in order[:m]], axis=1)
        pool = [c for c in range(cand.shape[0]) if c not in order[:m]]
        for s in range(sample_per_m):
            ci = (3 * s + m) % len(pool)
            p = s  # round s (0 = original)
            x = cand[pool[ci]] if p == 0 else cand[pool[ci]][perms[p - 1]]
            tasks.append((x, y, z, K, alg))
            keys.append((m, ci, p))
    workers = workers or (os.cpu_count() or 1)
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(workers) as pool_:
        res = pool_.map(_cpu_task, tasks)
    wall = time.perf_counter() - t0
    vals = {k: r[0] for k, r in zip(keys, res)}
    desc = (f"{len(tasks)} of the step's CMIs ({sample_per_m} per conditioning size m=1..8, N=10000, "
            f"k=4) with the NumPy oracle in {workers} processes: {wall:.1f} s wall, "
            f"{sum(r[1] for r in res):.1f} s CPU")
    return len(tasks) / wall, workers, desc, vals


def kdtree_context(cand, y, perms, order, per_m=2):
    """Context only (not the oracle, not parity): KSG with SciPy's k-d tree in FP64 on all host
    threads, on the same sample of the step's CMIs as the oracle baseline: (CMI/s, threads)."""
    from scipy.spatial import cKDTree
    from oracle.harmonic import harmonic_table
    h = harmonic_table(cand.shape[1])

    def ksg_tree(x, z):
        n = x.shape[0]
        xz = np.concatenate([x[:, None], z], 1).astype(np.float64)
        yz = np.concatenate([y[:, None], z], 1).astype(np.float64)
        joint = np.concatenate([x[:, None], y[:, None], z], 1).astype(np.float64)
        d, _ = cKDTree(joint).query(joint, k=K + 1, p=np.inf, workers=-1)
        r = np.nextafter(d[:, K], 0)
        cnt = [cKDTree(c).query_ball_point(c, r=r, p=np.inf, return_length=True, workers=-1) - 1
               for c in (xz, yz, z.astype(np.float64))]
        return h[K - 1] - (h[cnt[0]] + h[cnt[1]] - h[cnt[2]]).mean()

    n_done = 0
    t0 = time.perf_counter()
    for m in FORCED_M:
        z = np.stack([cand[c] for c in order[:m]], axis=1)
        pool = [c for c in range(cand.shape[0]) if c not in order[:m]]
        for s_ in range(per_m):
            ci = (3 * s_ + m) % len(pool)
            x = cand[pool[ci]] if s_ == 0 else cand[pool[ci]][perms[s_ - 1]]
            ksg_tree(x, z)
            n_done += 1
    return n_done / (time.perf_counter() - t0), os.cpu_count()


# ---------------------------------------------------------------------------------------------
# Learned null: training set from seeded networks (seeds disjoint from the evaluation network)


# (kind, seed, size): ar2 -> N; logistic -> trials of 3000 samples.  Seeds are disjoint from
# the evaluation network (logistic seed 3).
AR2_PLAN = [("ar2", 1000 + i, n) for i, n in enumerate([2000] * 30 + [5000] * 16 + [10000] * 8)]
TRAIN_PLAN = AR2_PLAN + [("logistic", 2000 + i, t) for i, t in enumerate([1] * 40 + [2] * 12 + [5] * 8 + [10] * 6)]
# more paths of the evaluation's size class (10 trials, N = 29,950), whose selections run deepest
DEEP_PLAN = [("logistic", 2066 + i, 10) for i in range(6)]


def _subsets_for(g):
    def f(n_pool, step):
        subs = [list(range(n_pool))]
        for _ in range(127):
            size = int(np.exp(g.uniform(0, np.log(n_pool))))
            subs.append(sorted(g.choice(n_pool, max(1, size), replace=False).tolist()))
        return subs
    return f


def c4_dataset(ctx, plan, log=print):
    """Training examples from the plain greedy paths of seeded networks (one target each)."""
    import torch
    import workloads
    from paper_1807_10459_amd.learned_null import greedy_path_examples
    parts = []
    t0 = time.perf_counter()
    for i, (kind, seed, size) in enumerate(plan):
        g = workloads.rng(seed + 50_000)
        if kind == "ar2":
            net = workloads.ar2_network(seed=seed, T=size + MAX_LAG, burn=500)
            P, target = 200, 0
        else:
            net = workloads.logistic_network(seed=seed, n_trials=size, T=3000)
            P, target = 500, int(g.integers(0, 20))
        data = torch.from_numpy(net.data).cuda()
        cand, y = ctx.embed(data, target=target, max_lag=MAX_LAG)
        perms = torch.from_numpy(workloads.permutations(y.shape[0], P, seed=seed + 60_000)).cuda()
        f, t, o, steps, _, _ = greedy_path_examples(ctx, cand, y, perms, _subsets_for(g), k=K)
        parts.append((f, t, o))
        log(f"dataset: {i + 1}/{len(plan)} paths, {sum(p[0].shape[0] for p in parts)} examples, "
            f"{time.perf_counter() - t0:.1f} s")
    feats = torch.cat([p[0] for p in parts])
    targ = torch.cat([p[1] for p in parts])
    obs = torch.cat([p[2] for p in parts])
    net_id = torch.cat([torch.full((p[0].shape[0],), i, dtype=torch.int32, device=p[0].device)
                        for i, p in enumerate(parts)])
    return feats, targ, obs, net_id


def _margins(pred, obs, rate):
    """Gate margins by the rule of ksg_gate_calibrate: u = (obs - p05) / |p01 - p05|; each margin
    the smallest value >= 0 leaving at most floor(rate/2 * B) examples decided wrongly on its side."""
    s = np.maximum(np.abs(pred[:, 1] - pred[:, 0]), 1e-30)
    u = (obs[:, 0] - pred[:, 0]) / s
    sig = obs[:, 1] > 0.5
    allow = int(np.floor(rate / 2 * len(u)))
    un = np.sort(u[~sig])[::-1]
    up = np.sort(u[sig])
    hi = max(0.0, float(un[allow])) if un.size > allow else 0.0
    lo = max(0.0, float(-up[allow])) if up.size > allow else 0.0
    return lo, hi, u


def bucket_table_ablation(F, Tg, HF, HO, rate, eval_steps):
    """The gate driven by a mean-threshold table instead of the network: the training targets
    averaged per (log N to 0.1, log c in steps of 0.5) bucket (the global mean for an empty
    bucket), calibrated on the same held-out examples at the same rate.  Reports its held-out
    fallback fraction and, on the evaluation run's judged steps (N, c, t_obs, plain decision),
    the steps it would decide, leave to the surrogates, and decide wrongly."""
    def key(logn, logc):
        return (round(float(logn), 1), int(np.floor(float(logc) / 0.5)))
    table = {}
    for f, t in zip(F, Tg):
        table.setdefault(key(f[0], f[5]), []).append(t)
    means = {kk: np.mean(v, axis=0) for kk, v in table.items()}
    glob = Tg.mean(axis=0)

    def predict(logn, logc):
        return means.get(key(logn, logc), glob)
    pred = np.array([predict(f[0], f[5]) for f in HF])
    lo, hi, u = _margins(pred, HO, rate)
    band = (u <= hi) & (u >= -lo)
    decided, fallback, wrong = 0, 0, 0
    for (n, c, t_obs, plain) in eval_steps:
        p05, p01 = predict(np.log(n), np.log(c))
        uu = (np.sqrt(n) * t_obs - p05) / max(abs(p01 - p05), 1e-30)
        if uu > hi or uu < -lo:
            decided += 1
            wrong += int((uu > hi) != (plain == 1))
        else:
            fallback += 1
    return {"margin_lo": round(lo, 4), "margin_hi": round(hi, 4), "buckets": len(means),
            "held_out_fallback": round(float(band.mean()), 4),
            "eval_steps_decided": decided, "eval_steps_fallback": fallback, "eval_steps_wrong": wrong}


def selection_bench(ctx, log):
    """Parents/s of the learned null against the plain permutation test on the AR(2) network
    (N = 10,000, 25 candidates, k = 4, 200 surrogates), every node as target.  The threshold
    network is trained in this run on the plain greedy paths of the 54 seeded AR(2) training
    networks (seeds disjoint from the evaluation network), margins calibrated on the held-out
    ones at 0.25 % wrong decisions; that one-time cost is reported apart from the timed runs."""
    import torch
    import workloads
    from paper_1807_10459_amd.learned_null import calibrate, train_threshold_net
    t0 = time.perf_counter()
    feats, targ, obs, net_id = c4_dataset(ctx, AR2_PLAN, log=lambda m: None)
    t_data = time.perf_counter() - t0
    held = (net_id % 7) == 3
    tr = torch.nonzero(~held).flatten()
    order = torch.from_numpy(workloads.permutations(tr.numel(), 1, seed=4242)[0].astype(np.int64)).cuda()
    tr = tr[order]
    t1 = time.perf_counter()
    net, hist = train_threshold_net(ctx, feats[tr].contiguous(), targ[tr].contiguous(), workloads.mlp_init(4243),
                                    epochs=60, batch=512, lr=2e-3)
    hi = torch.nonzero(held).flatten()
    cal = calibrate(net, feats[hi].contiguous(), obs[hi].contiguous(), rate=0.0025)
    t_train = time.perf_counter() - t1
    ev = workloads.ar2_network(seed=1)
    data = torch.from_numpy(ev.data).cuda()
    perms = torch.from_numpy(workloads.permutations(ev.data.shape[2] - MAX_LAG, N_PERM, seed=11)).cuda()
    n_vars = ev.data.shape[1]
    res = {}
    for mode in ("plain", "learned"):
        kw = dict(k=K, max_lag=MAX_LAG, alpha=0.05)
        if mode == "learned":
            kw.update(learned=net, margin_lo=cal["margin_lo"], margin_hi=cal["margin_hi"])
        ctx.select_parents(data, 0, perms, max_steps=1, **kw)  # warm-up
        torch.cuda.synchronize()
        tm = time.perf_counter()
        out = {t: ctx.select_parents(data, t, perms, **kw) for t in range(n_vars)}
        torch.cuda.synchronize()
        res[mode] = (out, time.perf_counter() - tm)
        log(f"selection {mode}: " + "; ".join(f"{t}: {r['parents']}" for t, r in out.items()))
    (plain, t_p), (learned, t_l) = res["plain"], res["learned"]
    n_p = sum(len(r["parents"]) for r in plain.values())
    n_l = sum(len(r["parents"]) for r in learned.values())
    agree = sum(1 for t in range(n_vars) for v in range(n_vars)
                if (v in {a for a, _ in plain[t]["parents"]}) == (v in {a for a, _ in learned[t]["parents"]}))
    return {"workload": "AR(2) 5-node network, every node as target, N=10000, 25 candidates, k=4, 200 surrogates",
            "learned_parents_per_s": round(n_l / t_l, 3), "plain_parents_per_s": round(n_p / t_p, 3),
            "speedup": round((n_l / t_l) / max(n_p / t_p, 1e-12), 2),
            "plain_seconds": round(t_p, 3), "learned_seconds": round(t_l, 3),
            "parents_plain": n_p, "parents_learned": n_l,
            "pair_agreement": agree / (n_vars * n_vars),
            "exact_parent_sets": sum(int(plain[t]["parents"] == learned[t]["parents"]) for t in range(n_vars)),
            "candidate_decisions": {"learned_gate_steps": sum(r["n_gate_decided"] for r in learned.values()),
                                    "learned_fallback_steps": sum(r["n_fallback"] for r in learned.values()),
                                    "plain_steps": sum(r["n_steps"] for r in plain.values())},
            "cmi_estimates": {"plain": sum(r["n_cmi"] for r in plain.values()),
                              "learned": sum(r["n_cmi"] for r in learned.values())},
            "training": {"examples": int(feats.shape[0]), "held_out": int(hi.numel()), "dataset_s": round(t_data, 1),
                         "train_and_calibrate_s": round(t_train, 1), "loss_first": round(hist[0], 5),
                         "loss_last": round(hist[-1], 5), "margins": [round(cal["margin_lo"], 4),
                                                                      round(cal["margin_hi"], 4)]}}


def c4_evaluate(ctx, args, log):
    """Learned-null vs plain greedy selection on the 20-node logistic network (seed 3)."""
    import torch
    import workloads
    from paper_1807_10459_amd.learned_null import calibrate, train_threshold_net
    t0 = time.perf_counter()
    if args.dataset:  # training sets written earlier by --dump-dataset (same recipes), concatenated
        parts, off = [], 0
        for path in args.dataset:
            d = np.load(path)
            parts.append([d["feats"], d["targ"], d["obs"], d["net_id"] + off])
            off = int(parts[-1][3].max()) + 1  # network ids stay distinct across the files
        feats, targ, obs, net_id = (torch.from_numpy(np.concatenate([q[i] for q in parts])).cuda() for i in range(4))
    else:
        feats, targ, obs, net_id = c4_dataset(ctx, TRAIN_PLAN, log=log)
    t_data = time.perf_counter() - t0
    held = (net_id % 7) == 3
    tr = torch.nonzero(~held).flatten()
    if args.real_weight > 1:
        # the full-pool example of every step (the first of its step's examples: the steps of a
        # path come in order, each with the full pool and 127 subsets) repeated real_weight times
        nid = net_id.cpu().numpy()
        first_row = np.r_[0, np.nonzero(np.diff(nid))[0] + 1]
        row_in_path = np.arange(nid.size) - np.repeat(first_row, np.diff(np.r_[first_row, nid.size]))
        real = torch.from_numpy(row_in_path % 128 == 0).cuda()
        tr = torch.cat([tr] + [tr[real[tr]]] * (args.real_weight - 1))
    order = torch.from_numpy(workloads.permutations(tr.numel(), 1, seed=4242)[0].astype(np.int64)).cuda()
    tr = tr[order]
    t1 = time.perf_counter()
    net, hist = train_threshold_net(ctx, feats[tr].contiguous(), targ[tr].contiguous(),
                                    workloads.mlp_init(4243), epochs=60, batch=512, lr=2e-3)
    t_train = time.perf_counter() - t1
    # margins from the held-out networks of the evaluation's size class (N >= 14,000: 5 and 10
    # trials; feature 0 is log N): the gate's errors grow with N and with the step's depth
    hi_idx = torch.nonzero(held & (feats[:, 0] >= float(np.log(14000.0)))).flatten()
    cal = calibrate(net, feats[hi_idx].contiguous(), obs[hi_idx].contiguous(), rate=0.0025,
                    include_rate=args.include_rate)
    deep = None
    if args.deep_dz > 0:  # margins of their own for the deep steps (feature 3 is d_z)
        dp_idx = torch.nonzero(held & (feats[:, 0] >= float(np.log(14000.0))) & (feats[:, 3] >= args.deep_dz)).flatten()
        cal_d = calibrate(net, feats[dp_idx].contiguous(), obs[dp_idx].contiguous(), rate=0.0025,
                          include_rate=args.include_rate)
        deep = (args.deep_dz, cal_d["margin_lo"], cal_d["margin_hi"])
        log(f"deep-step calibration (d_z >= {args.deep_dz}, {dp_idx.numel()} examples): {cal_d}")
    log(f"dataset {feats.shape[0]} examples in {t_data:.1f} s; training {t_train:.1f} s "
        f"(loss {hist[0]:.4f} -> {hist[-1]:.4f}); calibration {cal}")

    net3 = workloads.logistic_network(seed=3)
    data = torch.from_numpy(net3.data).cuda()
    N = net3.data.shape[0] * (net3.data.shape[2] - MAX_LAG)
    perms = torch.from_numpy(workloads.permutations(N, 500, seed=33)).cuda()
    targets = [int(t) for t in args.targets.split(",")] if args.targets else list(range(20))
    res = {}
    # plain: the permutation test on every step, no network; learned: the gate first, the
    # surrogates only for borderline steps; judged (--judge): the gate and the plain test on every
    # step, the plain decision taken (per-step agreement of the gate, not timed against)
    modes = (() if args.plain_json else ("plain",)) + ("learned",) + (("judged",) if args.judge else ())
    if args.plain_json:
        # plain results of earlier runs of this workload (the plain path is deterministic: same
        # network, permutations and options); their targets together must be the requested ones
        recs = [json.loads(open(f).read().strip().splitlines()[-1]) for f in args.plain_json]
        got = sorted(t for r in recs for t in r["targets"])
        if got != sorted(targets):
            raise SystemExit(f"--plain-json covers targets {got}, not the requested {sorted(targets)}")
        plain_rec = {int(t): {"parents": [tuple(p) for p in ps]} for r in recs for t, ps in r["parents_plain"].items()}
        res["plain"] = (plain_rec, sum(r["plain_seconds"] for r in recs))
    for mode in modes:
        torch.cuda.synchronize()
        tm = time.perf_counter()
        out = {}
        for t in targets:
            kw = dict(k=K, max_lag=MAX_LAG, alpha=0.05, omnibus=True)
            if mode != "plain":
                kw.update(learned=net, margin_lo=cal["margin_lo"], margin_hi=cal["margin_hi"], judge=mode == "judged",
                          verify_stop=True, deep_margins=deep)
            out[t] = ctx.select_parents(data, t, perms, **kw)
            log(f"{mode} target {t}: parents {out[t]['parents']} steps {out[t]['n_steps']} "
                f"truncated {out[t]['truncated']} fallback {out[t]['n_fallback']} disagree {out[t]['n_disagree']} "
                f"{time.perf_counter() - tm:.1f} s")
        torch.cuda.synchronize()
        res[mode] = (out, time.perf_counter() - tm)
    plain, t_plain = res["plain"]
    learned, t_learned = res["learned"]

    def sources(r, t):  # final parent variables (omnibus-gated sources + target past)
        vs = {v for (v, _) in r["parents"] if v == t}
        # a plain record read from an earlier line holds the final parent list only (the
        # omnibus test, which both runs apply to their own parent sets, gated it there)
        if "omnibus_tested" not in r or (r["omnibus_tested"] and r["omnibus_significant"]):
            vs |= {v for (v, _) in r["parents"] if v != t}
        return vs
    n_vars = 20
    agree_pairs = sum(1 for t in targets for v in range(n_vars)
                      if (v in sources(plain[t], t)) == (v in sources(learned[t], t)))
    exact = sum(1 for t in targets if plain[t]["parents"] == learned[t]["parents"])
    n_par_plain = sum(len(r["parents"]) for r in plain.values())
    n_par_learned = sum(len(r["parents"]) for r in learned.values())
    # per-step agreement without a judge run: along each target's common path (steps whose
    # conditioning sets agree), the learned run's decision (the gate's, or the surrogates' on a
    # borderline step) against the plain run's
    steps_compared, steps_agree = 0, 0
    for t in (targets if not args.plain_json else ()):
        pp, ll = plain[t], learned[t]
        for i in range(min(len(pp["steps"]), len(ll["steps"]))):
            if pp["candidates"][:i] != ll["candidates"][:i]:
                break
            st_l = ll["steps"][i]
            dec_l = (st_l["verdict"] > 0) if st_l["verdict"] in (-1, 1) else (st_l["plain"] == 1)
            steps_compared += 1
            steps_agree += int(dec_l == (pp["steps"][i]["plain"] == 1))
    if "judged" in res:
        steps_judged = sum(r["n_steps"] for r in res["judged"][0].values())
        disagree = sum(r["n_disagree"] for r in res["judged"][0].values())
    true_edges = {(s_, t_) for (s_, t_, _) in net3.edges}
    # ablation: the same gate driven by a per-(N, c) bucket mean-threshold table, evaluated on
    # the plain run's judged steps (pool size c = 100 - step in the multivariate-TE pool)
    eval_steps = [(N, n_vars * MAX_LAG - i, st["t_obs"], st["plain"])
                  for r in plain.values() for i, st in enumerate(r.get("steps", ())) if st["plain"] in (0, 1)]
    ablation = bucket_table_ablation(feats[tr].cpu().numpy(), targ[tr].cpu().numpy(),
                                     feats[hi_idx].cpu().numpy(), obs[hi_idx].cpu().numpy(), 0.0025, eval_steps)
    ablation["network_held_out_fallback"] = round(cal["fallback"], 4)
    ablation["network_eval_steps_decided"] = sum(1 for r in learned.values() for st in r["steps"]
                                                 if st["verdict"] in (-1, 1))
    log(f"ablation: {ablation}")
    return {
        "metric": "parents/sec learned vs plain null (20-node logistic network, N=29950, 500 surrogates)",
        "value": round(n_par_learned / t_learned, 4),
        "unit": "parents/s",
        "plain_parents_per_s": round(n_par_plain / t_plain, 4),
        "speedup": round((n_par_learned / t_learned) / max(n_par_plain / t_plain, 1e-12), 2),
        "targets": targets,
        "plain_seconds": round(t_plain, 2),
        "learned_seconds": round(t_learned, 2),
        "pair_agreement": agree_pairs / (len(targets) * n_vars),
        "exact_parent_set_rate": exact / len(targets),
        "step_agreement_common_path": steps_agree / steps_compared if steps_compared else None,
        "steps_compared": steps_compared,
        "judged_step_agreement": (1.0 - disagree / max(steps_judged, 1)) if "judged" in res else None,
        "truncated_targets_plain": (sum(int(r["truncated"]) for r in plain.values()) if not args.plain_json
                                    else sum(r["truncated_targets_plain"] for r in recs)),
        "plain_from": args.plain_json,
        "include_rate": args.include_rate,
        "deep_margins": deep,
        "real_weight": args.real_weight,
        "omnibus": {str(t): [r["omnibus_tested"], r["omnibus_significant"]] for t, r in learned.items()},
        "truncated_targets_learned": sum(int(r["truncated"]) for r in learned.values()),
        "parents_plain": {str(t): r["parents"] for t, r in plain.items()},
        "parents_learned": {str(t): r["parents"] for t, r in learned.items()},
        "learned_fallback_steps": sum(r["n_fallback"] for r in learned.values()),
        "learned_gate_steps": sum(r["n_gate_decided"] for r in learned.values()),
        "learned_cmi": sum(r["n_cmi"] for r in learned.values()),
        "plain_cmi": (sum(r["n_cmi"] for r in plain.values()) if not args.plain_json
                      else sum(r["plain_cmi"] for r in recs)),
        "calibration": cal,
        "training": {"examples": int(feats.shape[0]), "held_out": int(hi_idx.numel()),
                     "dataset_s": round(t_data, 1), "train_s": round(t_train, 1),
                     "loss_first": hist[0], "loss_last": hist[-1]},
        "ablation_bucket_table": ablation,
        "true_source_edges_found_plain": sum(1 for t in targets for v in sources(plain[t], t)
                                             if v != t and (v, t) in true_edges),
        "true_source_edges": sum(1 for t in targets for (s_, t_) in true_edges if t_ == t),
    }


# Parent set that the plain greedy selection returns for target 0 of the 20-node logistic
# network (seed 3, 500 surrogates, k = 4): (variable, lag) pairs in inclusion order.
OMNIBUS_PARENTS = [(0, 1), (2, 2), (15, 1), (15, 2), (0, 2), (2, 3), (2, 1), (0, 3), (2, 4), (15, 3),
                   (2, 5), (0, 5), (6, 1), (0, 4), (9, 2)]


def omnibus_bench(ksg, args):
    """The omnibus test of that parent set: I(10 source columns ; Y | 5 target-past columns) and
    500 surrogates permuting the source block's rows jointly (501 problems of 16 columns at
    N = 29,950), one batched launch per step."""
    import torch
    import workloads
    net = workloads.logistic_network(seed=3)
    data = torch.from_numpy(net.data).cuda()
    ctx = ksg.Context(0)
    ctx.set_option(ctx.OPT_WINDOWS, 0 if args.no_windows else 1)
    ctx.set_option(ctx.OPT_ALGORITHM, args.algorithm)
    cand, y = ctx.embed(data, target=0, max_lag=MAX_LAG)
    N = y.shape[0]
    idx = [v * MAX_LAG + lag - 1 for (v, lag) in OMNIBUS_PARENTS]
    src = [c for c in idx if c // MAX_LAG != 0]
    tgt = [c for c in idx if c // MAX_LAG == 0]
    xs = cand[src].contiguous()
    zs = cand[tgt].contiguous()
    y1 = y.reshape(1, -1).contiguous()
    P = 500
    perms = torch.from_numpy(workloads.permutations(N, P, seed=33)).cuda()
    probs = [ksg.Problem(xs, y1, zs, K)] + [ksg.Problem(xs, y1, zs, K, perm_x=perms[p]) for p in range(P)]
    for _ in range(args.warmup):
        ctx.cmi_batch(probs)
    torch.cuda.synchronize()
    ctx.set_option(ctx.OPT_TIMING, 1)
    ctx.take_timing()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = ctx.cmi_batch(probs)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.take_timing()
    kern = ctx.last_kernels()
    ctx.set_option(ctx.OPT_TIMING, 0)
    ms, ops, nl = kern["single"]
    D = len(src) + 1 + len(tgt)
    # VALU lane-instructions per launch from the committed counter record of this launch (the
    # window search at D = 16 under algorithm 1), over this run's mean launch time
    rec_key = ("alg2" if args.algorithm == 2 else "single") if args.no_windows else \
        ("window_alg2" if args.algorithm == 2 else "window")
    valu_instr = _counter_record("valu_wave_instructions_per_launch", rec_key, OMNIBUS_RECORD, OMNIBUS_SOURCES)
    t_launch = ms / nl * 1e-3
    achieved = None if valu_instr is None else valu_instr * 64 / t_launch
    pairs = N * (N - 1)
    brute = (P + 1) * pairs * (4 * D + 2)
    res = out.cpu().numpy()
    line = {
        "metric": "CMI estimates/sec incl. surrogates (omnibus test, N=29950, k=4)"
                  + (", KSG algorithm 2" if args.algorithm == 2 else ""),
        "value": round((P + 1) * args.steps / wall, 1),
        "unit": "CMI/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1000.0 * wall / args.steps, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "dtype_note": "FP32 differences, maxima and compares; FP64 only in the digamma sums",
        "data": "synthetic",
        "config": {"workload": f"omnibus test of target 0's parent set, 20-node logistic network, "
                               f"N={N}, {len(src)} source + 1 target + {len(tgt)} target-past columns "
                               f"(D={D}), k=4, {P} surrogates"},
        "roofline": {"bound": "alu", "achieved": None if achieved is None else round(achieved / 1e12, 3),
                     "peak": round(PEAK_VALU / 1e12, 3), "unit": "T VALU lane-instructions/s",
                     "frac": None if achieved is None else round(achieved / PEAK_VALU, 4), "traffic": None,
                     "kernel": KERNEL_NAMES[rec_key],
                     "kernel_ms_per_launch": round(ms / nl, 3), "launches": nl,
                     "valu_wave_instructions_per_launch": valu_instr,
                     "how": "achieved = SQ_INSTS_VALU per launch (committed rocprofv3 counter record) x 64 "
                            "lanes / this run's mean launch time (HIP events)",
                     # the kernel's own count of the operations over the pairs it visits, and the
                     # method's brute-force count (N(N-1)(4D+2) per problem), each over the launch time
                     "executed_ops_per_launch": ops / nl,
                     "executed_ops_rate": round(ops / (ms * 1e-3) / 1e12, 3),
                     "effective_ops_rate": round(brute / t_launch / 1e12, 3)},
        "omnibus_cmi": float(res[0]),
        "omnibus_pval": float(np.mean(res[1:] >= res[0])),
    }
    if not args.no_cpu_baseline:
        from oracle.ksg import ksg_cmi
        from oracle.ksg2 import ksg2_cmi
        xs_np, y_np, zs_np = xs.cpu().numpy().T, y.cpu().numpy(), zs.cpu().numpy().T
        t1 = time.perf_counter()
        ref = (ksg2_cmi if args.algorithm == 2 else ksg_cmi)(xs_np, y_np, zs_np, K)
        dt = time.perf_counter() - t1
        line["cpu_baseline"] = {"value": round(1.0 / dt, 5), "unit": "CMI/s", "cores": 1, "kind": "oracle",
                                "cpu_model": _cpu_model(),
                                "sample": "the original (unpermuted) omnibus CMI, one process"}
        line["parity_spot_check_abs_err"] = abs(float(res[0]) - ref)
    ctx.close()
    return line


TRAFFIC_SOURCES = ("ksg_group.inc.h", "ksg_search.inc.h", "ksg_yzcount.hip")
OMNIBUS_RECORD = "omnibus_window_kernel_counters.json"
OMNIBUS_SOURCES = ("ksg_window.inc.h", "ksg_search.inc.h", "ksg_window.hip")
KERNEL_NAMES = {"radius": "ksg_group_radius_kernel (k-NN radius of each problem of a group, "
                          "Y/Z distances shared, key-ordered windows)",
                "yz_count": "ksg_yzcount_kernel (n_YZ and n_Z of every problem of a step at once: "
                            "rank histogram over the sorted radii)",
                "x_count": "ksg_group_xcount_kernel (n_XZ of each problem of a group, digamma partial sums)",
                "single": "ksg_batch_kernel (brute-force radius, counts and digamma partial sums)",
                "window": "ksg_window_kernel (rows in key order, radius and counts within each tile's "
                          "key window; operations counted over the pairs visited)",
                "alg2": "ksg_alg2_kernel (KSG algorithm 2: indexed top-k, neighbour rectangles, "
                        "rectangle counts and partial sums)",
                "window_alg2": "ksg_window_kernel<D, 5, 2> (KSG algorithm 2 in key order: k-th neighbour "
                               "distance, rectangle sides, <= counts; operations counted over the pairs visited)"}


def _host_cpu():
    """lscpu's model, sockets, physical cores and hardware threads of the host (Linux)."""
    import subprocess
    info = {}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for ln in out.splitlines():
            if ":" in ln:
                key, val = ln.split(":", 1)
                info[key.strip()] = val.strip()
    except (OSError, subprocess.SubprocessError):
        pass

    def num(key):
        try:
            return int(info.get(key, ""))
        except ValueError:
            return None
    sockets, cores_per, threads = num("Socket(s)"), num("Core(s) per socket"), num("CPU(s)")
    return {"model": info.get("Model name", _cpu_model()), "sockets": sockets,
            "family_model_stepping": [info.get("CPU family"), info.get("Model"), info.get("Stepping")],
            "physical_cores": sockets * cores_per if sockets and cores_per else None,
            "hardware_threads": threads, "threads_usable": os.cpu_count()}


def _cpu_model():
    """The host CPU's model name (Linux), for the CPU baseline's record."""
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def uneven_bench(ksg, args):
    """64 independent problems of uneven size and shape (N log-uniform in [2000, 50000], d_x and
    d_y in 1..2, d_z in 0..10, k in {4, 8}; Gaussian with random correlations): one batched
    launch set per step.  Problems with k <= 4, a Z column and N at or above the window
    threshold of their column count run the key-ordered window search, the rest the
    brute-force kernels compiled per shape or width.  The batch is timed on an autotuned
    context (group sizes, brute-force tile heights, window thresholds per column count) and on
    one with the fixed defaults (tile height 256, windows from N = 2048)."""
    import torch
    import workloads

    def soa(pts):  # row-major [N][d] -> device [d][N] (None for d == 0)
        return torch.from_numpy(np.ascontiguousarray(pts.T)).cuda() if pts.shape[1] else None

    probs, _ = workloads.uneven_batch(seed=2)
    cols = [(soa(p.x), soa(p.y), soa(p.z)) for p in probs]
    batch = [ksg.Problem(x, y, z, p.k) for (x, y, z), p in zip(cols, probs)]

    def run(tuned):
        ctx = ksg.Context(0)
        t_tune = time.perf_counter()
        choices = ctx.autotune(8192) if tuned else None
        t_tune = time.perf_counter() - t_tune
        ctx.set_option(ctx.OPT_WINDOWS, 0 if args.no_windows else 1)
        for _ in range(args.warmup):
            ctx.cmi_batch(batch)
        torch.cuda.synchronize()
        ctx.set_option(ctx.OPT_TIMING, 1)
        ctx.take_timing()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            out = ctx.cmi_batch(batch)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        # the search span of each step (first launch to last, the launches running side by side
        # on several streams) and the per-launch durations summed
        span_ms, _, ops = ctx.take_timing()
        kern = ctx.last_kernels()
        ctx.set_option(ctx.OPT_TIMING, 0)
        ctx.close()
        return dict(wall=wall, span_ms=span_ms, ops=ops, kern=kern, out=out.cpu().numpy(), choices=choices,
                    tune_s=t_tune)

    fixed = run(False)
    tuned = run(True)
    best = tuned if tuned["wall"] <= fixed["wall"] else fixed
    ms, _, nl = best["kern"]["single"]
    res = best["out"]
    brute = [p.n * (p.n - 1) * (4 * sum(p.dims) + 2) for p in probs]
    win_n = (tuned["choices"] or {}).get("window_min_n", {})
    n_win = sum(1 for p in probs if p.k <= 4 and p.dims[2] >= 1 and sum(p.dims) <= 16 and
                win_n.get(str(sum(p.dims)), 2048) is not None and p.n >= (win_n.get(str(sum(p.dims))) or 2048))
    line = {
        "metric": "CMI estimates/sec (64-problem uneven batch, N in [2000, 50000], k in {4, 8})",
        "value": round(len(probs) * args.steps / best["wall"], 2),
        "unit": "CMI/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1000.0 * best["wall"] / args.steps, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "dtype_note": "FP32 differences, maxima and compares; FP64 only in the digamma sums",
        "data": "synthetic",
        "config": {"workload": f"64 Gaussian problems, N log-uniform in [2000, 50000] (sum {sum(p.n for p in probs)}), "
                               f"d_x, d_y in 1..2, d_z in 0..10, k in {{4, 8}}; {n_win} searched with key-ordered "
                               f"windows under the tuned thresholds" + (" (windows off)" if args.no_windows else "")},
        "autotune": {"choices": tuned["choices"], "seconds": round(tuned["tune_s"], 3),
                     "tuned_ms_per_step": round(1000.0 * tuned["wall"] / args.steps, 2),
                     "fixed_ms_per_step": round(1000.0 * fixed["wall"] / args.steps, 2),
                     "tuned_search_span_ms": round(tuned["span_ms"] / args.steps, 3),
                     "fixed_search_span_ms": round(fixed["span_ms"] / args.steps, 3),
                     "headline": "tuned" if best is tuned else "fixed"},
        "roofline": {"bound": "alu", "achieved": None, "peak": round(PEAK_VALU / 1e12, 3),
                     "unit": "T VALU lane-instructions/s", "frac": None, "traffic": None,
                     "kernel": "single-problem search kernels (brute force per shape or width, and "
                               "the key-ordered window search), one launch per column count, run side by side",
                     "search_span_ms_per_step": round(best["span_ms"] / args.steps, 3),
                     "kernel_ms_sum_per_step": round(ms / args.steps, 3),
                     "launches_per_step": nl / args.steps,
                     "executed_ops_per_step": best["ops"] / args.steps,
                     "effective_ops_rate": round(float(sum(brute)) / (best["span_ms"] / args.steps * 1e-3) / 1e12, 3),
                     "brute_force_ops_per_step": float(sum(brute))},
    }
    if not args.no_cpu_baseline:
        from oracle.ksg import ksg_cmi
        order = sorted(range(len(probs)), key=lambda i: probs[i].n)
        done, sample_ops, worst = [], 0.0, 0.0
        t1 = time.perf_counter()
        for i in order:  # smallest problems first, until about 15 s of oracle time
            p = probs[i]
            ref = ksg_cmi(p.x, p.y, p.z, p.k)
            worst = max(worst, abs(float(res[i]) - ref) / max(1.0, abs(ref)),
                        abs(float(fixed["out"][i]) - ref) / max(1.0, abs(ref)))
            done.append(i)
            sample_ops += brute[i]
            if time.perf_counter() - t1 > 15.0:
                break
        dt = time.perf_counter() - t1
        # the sample's brute-force operation rate, priced at the batch's mean work per CMI
        cps = (sample_ops / dt) / (sum(brute) / len(probs))
        line["cpu_baseline"] = {"value": round(cps, 4), "unit": "CMI/s", "cores": 1, "kind": "oracle",
                                "cpu_model": _cpu_model(), "host": _host_cpu(),
                                "sample": f"the {len(done)} smallest problems (N {probs[done[0]].n}.."
                                          f"{probs[done[-1]].n}), one process, {dt:.1f} s; rate scaled by "
                                          f"the batch's mean brute-force operations per CMI"}
        line["parity_spot_check_max_rel_err"] = worst
    return line


def _kernel_source_hash(sources=None):
    import hashlib
    return hashlib.sha256(b"".join(open(os.path.join(ROOT, "paper_1807_10459_amd", "csrc", f), "rb").read()
                                   for f in (sources or TRAFFIC_SOURCES))).hexdigest()


def _counter_record(field, kernel, record="ksg_group_kernels_traffic.json", sources=None):
    """A per-launch figure of a kernel from a committed counter record under profiles/ (HBM
    bytes, VALU wave-instructions), or None when the kernel sources changed since the counters
    were taken."""
    path = os.path.join(ROOT, "profiles", record)
    try:
        rec = json.load(open(path))
        if _kernel_source_hash(sources) == rec["kernel_source_sha256"]:
            return rec[field].get(kernel)
    except (OSError, KeyError, ValueError, AttributeError):
        pass
    return None


def _traffic_record(kernel):
    return _counter_record("traffic_bytes_per_launch", kernel)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--algorithm", type=int, default=1, choices=[1, 2],
                    help="KSG algorithm of the estimates (2: neighbour rectangles, searched one by one)")
    ap.add_argument("--no-windows", action="store_true",
                    help="search ungrouped problems by brute force over all rows (no key-ordered windows)")
    ap.add_argument("--group-size", type=int, default=-1,
                    help="problems searched together (-1 tuned, 0 off, 8, 16)")
    ap.add_argument("--workload", default="ar2", choices=["ar2", "c4", "modes", "omnibus", "uneven"],
                    help="ar2: CMI/s on the AR(2) forced path (default); c4: learned vs plain null")
    ap.add_argument("--targets", default=None, help="c4: comma-separated targets (default all 20)")
    ap.add_argument("--dataset", nargs="+", default=None,
                    help="c4: load the training set from these npz files (concatenated)")
    ap.add_argument("--plan", default="train", choices=["train", "deep"],
                    help="--dump-dataset: the training networks (train), or six more of the evaluation's "
                         "size class (deep)")
    ap.add_argument("--deep-dz", type=int, default=0,
                    help="c4: steps conditioning on at least this many columns use margins calibrated on "
                         "the held-out examples of that depth")
    ap.add_argument("--real-weight", type=int, default=1,
                    help="c4: repeat each step's full-pool training example this many times")
    ap.add_argument("--include-rate", type=float, default=None,
                    help="c4: calibrate the gate with this allowance of wrong inclusions (and rate/2 of wrong "
                         "stops) instead of rate/2 on both sides")
    ap.add_argument("--plain-json", nargs="+", default=None,
                    help="c4: skip the plain run and compare with the plain results of earlier c4 lines "
                         "(their targets together must be the requested ones)")
    ap.add_argument("--judge", action="store_true",
                    help="c4: also run the judged selection (gate and plain test on every step)")
    ap.add_argument("--dump-dataset", default=None,
                    help="build the learned-null training set and save it (npz) instead of benchmarking")
    ap.add_argument("--no-selection", action="store_true",
                    help="skip the learned-vs-plain parent selection on the AR(2) network")
    ap.add_argument("--no-graph", action="store_true",
                    help="skip the pass that replays the steps from HIP graphs")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 1 GiB device-to-device copy (a known-size kernel for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py times one GPU: the library runs on one device and has no collectives, so "
              f"--gpus {args.gpus} is not supported (the path would shard by targets or by work items)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1807_10459_amd as ksg
    import workloads

    if args.workload == "c4":
        ctx = ksg.Context(0)
        line = c4_evaluate(ctx, args, log=lambda m: print(m, file=sys.stderr, flush=True))
        print(json.dumps(line))
        return

    if args.workload == "modes":  # the selection variants on the AR(2) network, target 0
        ctx = ksg.Context(0)
        net = workloads.ar2_network(seed=1)
        N = net.data.shape[2] - MAX_LAG
        data = torch.from_numpy(net.data).cuda()
        perms = torch.from_numpy(workloads.permutations(N, N_PERM, seed=11)).cuda()
        ctx.autotune(8192)
        ctx.select_parents(data, 0, perms, k=K, max_lag=MAX_LAG, max_steps=1)  # warm-up
        true_src = sorted({s_ for (s_, t_, _) in net.edges if t_ == 0})
        out = {}
        runs = (("mte", False, False, 1), ("mte", True, False, 1), ("mte", True, True, 1),
                ("bte", False, False, 1), ("mmi", False, False, 1), ("mte", False, False, 2))
        for mode, prune, seq, alg in runs:
            ctx.set_option(ctx.OPT_ALGORITHM, alg)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = ctx.select_parents(data, 0, perms, k=K, max_lag=MAX_LAG, mode=mode, prune=prune, omnibus=True,
                                   sequential=seq)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            srcs = sorted({v for (v, _) in r["parents"] if v != 0})
            name = mode + ("+prune" if prune else "") + ("+seq" if seq else "") + (" (KSG 2)" if alg == 2 else "")
            out[name] = {
                "seconds": round(dt, 3), "cmi_per_s": round(r["n_cmi"] / dt, 1), "n_cmi": r["n_cmi"],
                "steps": r["n_steps"], "parents": r["parents"], "pruned": r["pruned"],
                "seq_removed": r["seq_removed"], "seq_pval": [round(v, 4) for v in r["seq_pval"]],
                "source_vars": srcs, "omnibus_pval": r["omnibus_pval"]}
            print(f"{name}: {dt:.2f} s, {r['n_cmi']} CMIs, parents {r['parents']}", file=sys.stderr, flush=True)
        ctx.set_option(ctx.OPT_ALGORITHM, 1)
        print(json.dumps({"workload": "selection variants, AR(2) 5-node network, target 0, N=10000, "
                                      "k=4, 200 surrogates", "true_source_vars": true_src, "runs": out}))
        return

    if args.workload == "omnibus":
        line = omnibus_bench(ksg, args)
        print(json.dumps(line))
        return

    if args.workload == "uneven":
        line = uneven_bench(ksg, args)
        print(json.dumps(line))
        return

    if args.dump_dataset:
        ctx = ksg.Context(0)
        f, t, o, nid = c4_dataset(ctx, TRAIN_PLAN if args.plan == "train" else DEEP_PLAN,
                                  log=lambda m: print(m, file=sys.stderr, flush=True))
        np.savez_compressed(args.dump_dataset, feats=f.cpu().numpy(), targ=t.cpu().numpy(),
                            obs=o.cpu().numpy(), net_id=nid.cpu().numpy())
        print(json.dumps({"dataset": args.dump_dataset, "examples": int(f.shape[0])}))
        return

    net = workloads.ar2_network(seed=1)
    order = forced_order(net)
    N = net.data.shape[2] - MAX_LAG
    perms_np = workloads.permutations(N, N_PERM, seed=11)
    data = torch.from_numpy(net.data).cuda()
    perms = torch.from_numpy(perms_np).cuda()
    ctx = ksg.Context(0)
    t_tune = time.perf_counter()
    tuned = ctx.autotune(8192) if (args.group_size == -1 and args.algorithm == 1) else None
    t_tune = time.perf_counter() - t_tune
    ctx.set_option(ctx.OPT_GROUP_SIZE, args.group_size)
    ctx.set_option(ctx.OPT_ALGORITHM, args.algorithm)
    ctx.set_option(ctx.OPT_WINDOWS, 0 if args.no_windows else 1)
    tables = {m: torch.empty((25 - m, N_PERM + 1), dtype=torch.float64, device="cuda") for m in FORCED_M}
    # every step embeds again, into the same buffers (so a captured graph finds the same addresses)
    emb = ctx.embed(data, target=0, max_lag=MAX_LAG)

    def step():
        cand, y = ctx.embed(data, target=0, max_lag=MAX_LAG, out=emb)
        results = {}
        for m in FORCED_M:
            cond = order[:m]
            pool = [c for c in range(25) if c not in cond]
            _, r = ctx.greedy_step(cand, y, pool, cond, perms, k=K, out=tables[m])
            results[m] = r
        return cand, y, results

    # The inputs are checked for non-finite values and permutation range once, before timing
    # (as select_parents does); the timed steps trust them.
    for _ in range(args.warmup):
        step()
    ctx.set_option(ctx.OPT_CHECK_FINITE, 0)
    step()

    def timed(use_graph, timing):
        ctx.set_option(ctx.OPT_USE_GRAPH, int(use_graph))
        if use_graph:
            step()  # capture
        ctx.set_option(ctx.OPT_TIMING, int(timing))
        ctx.take_timing()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            res = step()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        k = ctx.take_timing()
        kern = ctx.last_kernels()
        ctx.set_option(ctx.OPT_TIMING, 0)
        ctx.set_option(ctx.OPT_USE_GRAPH, 0)
        return wall, k, kern, res

    # (1) direct launches, every search launch timed by its own HIP events on its stream
    wall, (k_ms, k_launches, k_ops), kern, (cand, y, results) = timed(False, True)
    # (2) the same steps replayed from HIP graphs (one graph per greedy step)
    g_wall, _, _, _ = timed(True, False) if args.algorithm == 1 and not args.no_graph else (None, None, None, None)
    graph_stats = ctx.graph_stats()
    head_wall = min(wall, g_wall) if g_wall else wall

    n_cmi = sum((25 - m) * (N_PERM + 1) for m in FORCED_M)
    value = n_cmi * args.steps / head_wall
    kernels = {}
    for name, (ms, ops, nl) in kern.items():
        if nl:
            kernels[name] = {"ms_per_launch": round(ms / nl, 3), "launches": nl,
                             "executed_ops_per_launch": ops / nl,
                             "executed_ops_rate": round(ops / (ms * 1e-3) / 1e12, 3)}
    dom = max(kernels, key=lambda kname: kern[kname][0])
    d_ms, d_ops, d_n = kern[dom]
    t_launch = d_ms / d_n * 1e-3
    # Algorithmic operations of the method (brute force over ordered pairs):
    # radius 2D per pair, counts 2D + 2 per pair, for every problem of the step.
    pairs = N * (N - 1)
    brute_radius = sum((25 - m) * (N_PERM + 1) * pairs * 2 * (m + 2) for m in FORCED_M) * args.steps
    brute_counts = sum((25 - m) * (N_PERM + 1) * pairs * (2 * (m + 2) + 2) for m in FORCED_M) * args.steps
    brute_of = {"radius": brute_radius, "x_count": brute_counts, "yz_count": brute_counts,
                "single": brute_radius + brute_counts}
    for name, rec in kernels.items():
        ms_total = kern[name][0]
        rec["effective_ops_rate"] = round(brute_of.get(name, 0.0) / (ms_total * 1e-3) / 1e12, 3)
        vi = _counter_record("valu_wave_instructions_per_launch", name)
        if vi is not None:
            rec["valu_lane_instr_rate"] = round(vi * 64 / (ms_total / kern[name][2] * 1e-3) / 1e12, 3)
            rec["frac"] = round(vi * 64 / (ms_total / kern[name][2] * 1e-3) / PEAK_VALU, 4)
    valu_instr = _counter_record("valu_wave_instructions_per_launch", dom)
    achieved = None if valu_instr is None else valu_instr * 64 / t_launch
    roofline = {
        "bound": "alu",
        "achieved": None if achieved is None else round(achieved / 1e12, 3),
        "peak": round(PEAK_VALU / 1e12, 3),
        "unit": "T VALU lane-instructions/s",
        "frac": None if achieved is None else round(achieved / PEAK_VALU, 4),
        "traffic": _traffic_record(dom),
        "kernel": KERNEL_NAMES[("alg2" if args.no_windows else "window_alg2") if args.algorithm == 2 else
                               ("window" if dom == "single" and not args.no_windows else dom)],
        "kernel_ms_per_launch": round(d_ms / d_n, 3),
        "launches": d_n,
        "valu_wave_instructions_per_launch": valu_instr,
        "how": "achieved = SQ_INSTS_VALU per launch (committed rocprofv3 counter record) x 64 lanes / this "
               "run's mean launch time (HIP events); peak = 256 CUs x 4 SIMDs x 32 lanes x 2.4 GHz",
        # the method's brute-force operation count for the launch's problems over its time: above the
        # peak because the key windows, exact skips and shared Y/Z distances do not execute most of it
        "effective_ops_rate": kernels[dom]["effective_ops_rate"],
        "algorithmic_ops_per_launch": brute_of.get(dom, 0.0) / d_n,
    }
    search = {"ms_per_step": round(k_ms / args.steps, 3), "kernels": kernels}

    line = {
        "metric": "CMI estimates/sec incl. surrogates (N=10k, k=4)",
        "value": round(value, 1),
        "unit": "CMI/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1000.0 * head_wall / args.steps, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "dtype_note": "FP32 differences, maxima and compares; FP64 only in the digamma sums",
        "data": "synthetic",
        "config": {"workload": "AR(2) 5-node greedy selection, target 0, N=10000, 25 candidates, "
                               "k=4, 200 surrogates, conditioning dims m=1..8 (forced path), "
                               f"{n_cmi} CMIs per step" + (", KSG algorithm 2" if args.algorithm == 2 else ""),
                   "n_cmi_per_step": n_cmi},
        "launch_modes": {"direct_ms_per_step": round(1000.0 * wall / args.steps, 2),
                         "graph_ms_per_step": None if g_wall is None else round(1000.0 * g_wall / args.steps, 2),
                         "headline": "graph" if g_wall and g_wall < wall else "direct",
                         "graph_captures": graph_stats["captures"], "graph_replays": graph_stats["replays"]},
        "roofline": roofline,
        "search": search,
        "autotune": {"choices": tuned, "seconds": round(t_tune, 3)} if tuned else None,
        "device": {k_: v_ for k_, v_ in ksg.device_props(0).items()
                   if k_ in ("name", "arch", "cus", "clock_khz", "mem_clock_khz", "mem_bus_bits",
                             "total_mem", "l2_bytes", "lds_per_cu")},
    }

    if args.copy_calibration:
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        line["copy_calibration_bytes"] = {"read": src.numel() * 4, "write": dst.numel() * 4}
        del src, dst

    if not args.no_cpu_baseline:
        cand_np = cand.cpu().numpy()
        y_np = y.cpu().numpy()
        workers = os.cpu_count() or 1
        per_m = max(2, -(-workers // 8))  # at least one task per worker
        cps, cores, desc, vals = cpu_baseline(cand_np, y_np, perms_np, order, sample_per_m=per_m,
                                              workers=workers, alg=args.algorithm)
        # The sampled oracle values double as a parity spot check of the timed run.
        worst = 0.0
        for (m, ci, p), v in vals.items():
            g = float(tables[m][ci, p].cpu())
            worst = max(worst, abs(g - v) / max(1.0, abs(v)))
        line["cpu_baseline"] = {"value": round(cps, 3), "unit": "CMI/s", "cores": cores, "kind": "oracle",
                                "cpu_model": _cpu_model(), "host": _host_cpu(), "sample": desc}
        line["parity_spot_check_max_rel_err"] = worst
        kps, threads = kdtree_context(cand_np, y_np, perms_np, order)
        line["cpu_context"] = {"value": round(kps, 3), "unit": "CMI/s", "threads": threads,
                               "kind": "SciPy cKDTree KSG in FP64 (context only: a tree search, not the "
                                       "oracle and not FP32-exact)",
                               "sample": "16 of the step's CMIs (2 per m)"}
    line["steps_detail"] = {str(m): {"c_star_candidate": [c for c in range(25) if c not in order[:m]][r["c_star"]],
                                     "t_obs": round(r["t_obs"], 6), "pval": r["pval"]}
                            for m, r in results.items()}
    if not args.no_selection and args.algorithm == 1:
        # the metric's second half: parents/s with the learned null against the plain test
        line["selection"] = selection_bench(ctx, log=lambda m: print(m, file=sys.stderr, flush=True))
    print(json.dumps(line))
    ctx.close()


if __name__ == "__main__":
    main()
