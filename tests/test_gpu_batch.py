"""The batch engine's launch options against the direct path and the oracle (needs an MI355X):
HIP graph capture and replay of a batch (KSG_OPT_USE_GRAPH) and grouped launches split into
many chunks (KSG_OPT_GROUP_CHUNK)."""
import numpy as np
import pytest

import workloads
from oracle.ksg import ksg_cmi
from tests.gpu_util import dev, soa, tol

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(lib):
    c = lib.Context(0)
    yield c
    c.close()


def _step_batch(lib, n=1500, n_cand=6, n_perm=11, m=3, k=4, seed=0):
    """The candidates x surrogates of one greedy step (grouped), host copies for the oracle."""
    g = workloads.rng(1200 + seed)
    p = workloads.random_problem(1300 + seed, n, 1, 1, m, k)
    cands = g.standard_normal((n_cand, n)).astype(np.float32)
    cands[2] = (cands[2] + p.y[:, 0]).astype(np.float32)
    perms = workloads.permutations(n, n_perm, seed=1400 + seed)
    y, z, dc, dp = soa(p.y), soa(p.z), dev(cands), dev(perms)
    probs = [lib.Problem(dc[c], y, z, k, perm_x=None if q == 0 else dp[q - 1])
             for c in range(n_cand) for q in range(n_perm + 1)]
    host = (p, cands, perms)
    return probs, host, (y, z, dc, dp)


def _mixed_batch(lib):
    """Window, wide and brute-force problems in one batch (launches on the auxiliary streams)."""
    pw = workloads.random_problem(1501, 2300, 1, 1, 3, 4)   # key-ordered windows
    pd = workloads.random_problem(1502, 900, 3, 2, 14, 4)   # 19 columns: the wide kernel
    pb = workloads.random_problem(1503, 800, 1, 2, 2, 8)    # brute force (k = 8)
    cols = [(soa(p.x), soa(p.y), soa(p.z)) for p in (pw, pd, pb)]
    probs = [lib.Problem(*cols[0], 4), lib.Problem(*cols[1], 4), lib.Problem(*cols[2], 8)]
    return probs, (pw, pd, pb), cols


def _run(ctx, probs, out):
    import torch
    ctx.cmi_batch(probs, out=out)
    torch.cuda.synchronize()
    return out.cpu().numpy().copy()


@pytest.mark.parametrize("which", ["step", "mixed", "step_alg2"])
def test_graph_replay_matches_direct_and_oracle(lib, ctx, which):
    """Captured once, replayed three times with eager work and synchronisations in between:
    every replay equals the direct launches bit for bit (same kernels, same summation order)
    and the oracle to 1e-12 (KSG algorithm 2: its own oracle)."""
    import torch
    if which.startswith("step"):
        probs, (p, cands, perms), keep = _step_batch(lib)
    else:
        probs, host, keep = _mixed_batch(lib)
    out = torch.empty(len(probs), dtype=torch.float64, device="cuda")
    ctx.set_option(ctx.OPT_CHECK_FINITE, 0)
    ctx.set_option(ctx.OPT_ALGORITHM, 2 if which == "step_alg2" else 1)
    try:
        ctx.set_option(ctx.OPT_USE_GRAPH, 0)
        direct = _run(ctx, probs, out)
        ctx.set_option(ctx.OPT_USE_GRAPH, 1)
        s0 = ctx.graph_stats()
        first = _run(ctx, probs, out)  # captured and launched
        assert np.array_equal(first, direct)
        for rep in range(3):
            out.fill_(-1.0)
            # eager work of the program between the replays
            other = workloads.random_problem(1600 + rep, 400, 1, 1, 1, 4)
            ctx.cmi(soa(other.x), soa(other.y), soa(other.z), 4)
            torch.cuda.synchronize()
            got = _run(ctx, probs, out)
            assert np.array_equal(got, direct), rep
        s1 = ctx.graph_stats()
        assert s1["replays"] - s0["replays"] >= 3 and s1["captures"] > s0["captures"]
    finally:
        ctx.set_option(ctx.OPT_USE_GRAPH, 0)
        ctx.set_option(ctx.OPT_CHECK_FINITE, 1)
        ctx.set_option(ctx.OPT_ALGORITHM, 1)
    if which.startswith("step"):
        from oracle.ksg2 import ksg2_cmi
        est = ksg2_cmi if which == "step_alg2" else ksg_cmi
        n_perm = perms.shape[0]
        for idx in (0, 1, 2 * (n_perm + 1), len(probs) - 1):
            c, q = divmod(idx, n_perm + 1)
            x = cands[c] if q == 0 else cands[c][perms[q - 1]]
            ref = est(x, p.y, p.z, 4)
            assert abs(direct[idx] - ref) <= tol(ref), idx
    else:
        for i, (hp, k) in enumerate(zip(host, (4, 4, 8))):
            ref = ksg_cmi(hp.x, hp.y, hp.z, k)
            assert abs(direct[i] - ref) <= tol(ref), i


def test_graph_retired_when_work_buffers_grow(lib, ctx):
    """A larger batch reallocates the work buffers a captured graph writes; the graph is not
    replayed with stale addresses: the next call captures again and still matches."""
    import torch
    probs, _, keep = _step_batch(lib, n=700, n_cand=3, n_perm=5, seed=1)
    big, _, keep2 = _step_batch(lib, n=6000, n_cand=8, n_perm=15, m=5, seed=2)
    out = torch.empty(len(probs), dtype=torch.float64, device="cuda")
    out_big = torch.empty(len(big), dtype=torch.float64, device="cuda")
    ctx.set_option(ctx.OPT_CHECK_FINITE, 0)
    try:
        ctx.set_option(ctx.OPT_USE_GRAPH, 0)
        direct = _run(ctx, probs, out)
        direct_big = _run(ctx, big, out_big)
        ctx.set_option(ctx.OPT_USE_GRAPH, 1)
        assert np.array_equal(_run(ctx, probs, out), direct)
        assert np.array_equal(_run(ctx, big, out_big), direct_big)
        c0 = ctx.graph_stats()["captures"]
        assert np.array_equal(_run(ctx, probs, out), direct)
        assert np.array_equal(_run(ctx, big, out_big), direct_big)
        assert ctx.graph_stats()["held"] >= 1 and ctx.graph_stats()["captures"] >= c0
    finally:
        ctx.set_option(ctx.OPT_USE_GRAPH, 0)
        ctx.set_option(ctx.OPT_CHECK_FINITE, 1)
    assert ctx.graph_stats()["held"] == 0  # switching the option off drops the graphs


def test_stale_graphs_are_freed(lib):
    """On a fresh context: a small batch is captured, then a larger one grows the work buffers
    (retiring the first graph, which is freed at once); the small batch then captures again,
    and every result equals the direct launches."""
    import torch
    c = lib.Context(0)
    try:
        probs, _, keep = _step_batch(lib, n=700, n_cand=3, n_perm=5, seed=3)
        big, _, keep2 = _step_batch(lib, n=6000, n_cand=8, n_perm=15, m=5, seed=4)
        out = torch.empty(len(probs), dtype=torch.float64, device="cuda")
        out_big = torch.empty(len(big), dtype=torch.float64, device="cuda")
        c.set_option(c.OPT_CHECK_FINITE, 0)
        c.set_option(c.OPT_USE_GRAPH, 1)
        first = _run(c, probs, out)
        assert c.graph_stats()["held"] == 1
        got_big = _run(c, big, out_big)
        assert c.graph_stats()["held"] == 1  # the small batch's graph was retired and freed
        again = _run(c, probs, out)
        st = c.graph_stats()
        assert st["held"] == 2 and st["captures"] == 3 and st["replays"] == 0
        c.set_option(c.OPT_USE_GRAPH, 0)
        assert np.array_equal(first, _run(c, probs, out)) and np.array_equal(again, first)
        assert np.array_equal(got_big, _run(c, big, out_big))
    finally:
        c.close()


def test_select_parents_with_graphs(lib, ctx):
    """select_parents under KSG_OPT_USE_GRAPH gives the selection of the direct path."""
    net = workloads.ar2_network(seed=1, T=1205, burn=300)
    perms = workloads.permutations(1200, 19, seed=71)
    data, dperm = dev(net.data), dev(perms)
    ref = ctx.select_parents(data, 0, dperm, k=4, max_lag=5)
    ctx.set_option(ctx.OPT_USE_GRAPH, 1)
    try:
        got = ctx.select_parents(data, 0, dperm, k=4, max_lag=5)
        again = ctx.select_parents(data, 0, dperm, k=4, max_lag=5)
    finally:
        ctx.set_option(ctx.OPT_USE_GRAPH, 0)
    for r in (got, again):
        assert r["parents"] == ref["parents"] and r["pval"] == ref["pval"] and r["cmi"] == ref["cmi"]


def test_grouped_batch_in_many_chunks(lib, ctx):
    """Grouped launches split into five chunks of two groups (the Y/Z set crossing every chunk
    boundary) give the estimates of one chunk bit for bit, and the oracle's in every chunk."""
    import torch
    n, n_cand, n_perm = 700, 6, 11  # 72 problems: 9 groups of 8
    probs, (p, cands, perms), keep = _step_batch(lib, n=n, n_cand=n_cand, n_perm=n_perm, m=2, seed=3)
    out = torch.empty(len(probs), dtype=torch.float64, device="cuda")
    ctx.set_option(ctx.OPT_GROUP_SIZE, 8)
    try:
        whole = _run(ctx, probs, out)
        ctx.set_option(ctx.OPT_GROUP_CHUNK, 2 * 8 * 704)  # two groups of 8 x 704 padded rows
        split = _run(ctx, probs, out)
    finally:
        ctx.set_option(ctx.OPT_GROUP_CHUNK, 0)
        ctx.set_option(ctx.OPT_GROUP_SIZE, -1)
    assert np.array_equal(whole, split)
    for chunk in range(5):  # one problem from every chunk of 16 consecutive problems
        idx = min(16 * chunk + 5, len(probs) - 1)
        c, q = divmod(idx, n_perm + 1)
        x = cands[c] if q == 0 else cands[c][perms[q - 1]]
        ref = ksg_cmi(x, p.y, p.z, 4)
        assert abs(split[idx] - ref) <= tol(ref), idx
    with pytest.raises(lib.KsgError):
        ctx.set_option(ctx.OPT_GROUP_CHUNK, -1)


def test_workspace_limit_reports_enomem(lib):
    """KSG_OPT_MEM_LIMIT caps the workspace: a batch that needs more fails with KSG_ENOMEM before
    any launch, the context stays usable, and a larger limit runs the same batch to the
    oracle's estimates (an out-of-memory path forced from the host)."""
    import torch
    probs, (p, cands, perms), keep = _step_batch(lib, n=3000, n_cand=4, n_perm=7, seed=5)
    c = lib.Context(0)
    try:
        c.set_option(c.OPT_MEM_LIMIT, 1 << 20)  # 1 MiB: less than the packed columns
        with pytest.raises(lib.KsgError) as e:
            c.cmi_batch(probs)
        assert e.value.status == 4 and "limit" in e.value.message
        c.set_option(c.OPT_MEM_LIMIT, 1 << 30)
        got = c.cmi_batch(probs).cpu().numpy()
        with pytest.raises(lib.KsgError):
            c.set_option(c.OPT_MEM_LIMIT, -1)
    finally:
        c.close()
    torch.cuda.synchronize()
    for idx in (0, 9, len(probs) - 1):
        ci, q = divmod(idx, perms.shape[0] + 1)
        x = cands[ci] if q == 0 else cands[ci][perms[q - 1]]
        ref = ksg_cmi(x, p.y, p.z, 4)
        assert abs(got[idx] - ref) <= tol(ref), idx

