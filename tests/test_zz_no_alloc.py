"""cmi_ksg_noalloc (the estimate without allocation, for callers that cannot allocate) against
the allocating entry point cmi_ksg and the oracle, through the C ABI (needs an MI355X)."""
import numpy as np
import pytest

import workloads
from oracle.ksg import ksg_cmi
from tests.gpu_util import soa, tol

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(lib):
    c = lib.Context(0)
    yield c
    c.close()


def _both(ctx, p, k):
    import torch
    x, y, z = soa(p.x), soa(p.y), soa(p.z)
    out = torch.full((1,), -7.0, dtype=torch.float64, device="cuda")
    ctx.cmi_noalloc(x, y, z, k, out=out)
    torch.cuda.synchronize()
    return float(out.cpu()[0]), ctx.cmi(x, y, z, k)


def test_noalloc_matches_cmi_ksg_two_calls(lib, ctx):
    """Two calls in a row, the second smaller (fewer rows, other shape and k), each equal to the
    allocating entry point's estimate and to the oracle's; then the first again."""
    big = workloads.random_problem(501, 3001, 1, 1, 2, 4)    # 12 tiles, ragged; windows in cmi_ksg
    small = workloads.random_problem(502, 777, 2, 1, 3, 8)   # 4 tiles, X/Y swapped, generic shape
    for p, k in ((big, 4), (small, 8), (big, 4)):
        got, ref_api = _both(ctx, p, k)
        ref = ksg_cmi(p.x, p.y, p.z, k)
        assert abs(got - ref_api) <= tol(ref_api), (p.n, got, ref_api)
        assert abs(got - ref) <= tol(ref), (p.n, got, ref)


def test_noalloc_limits_and_nonfinite(lib, ctx):
    import torch
    n = lib.KSG_NOALLOC_MAX_N + 1
    col = torch.zeros((1, n), dtype=torch.float32, device="cuda")
    with pytest.raises(lib.KsgError) as e:
        ctx.cmi_noalloc(col, col, None, 4)
    assert e.value.status == 1
    wide = torch.zeros((16, 100), dtype=torch.float32, device="cuda")
    one = torch.zeros((1, 100), dtype=torch.float32, device="cuda")
    with pytest.raises(lib.KsgError) as e:
        ctx.cmi_noalloc(one, one, wide, 4)  # 18 columns
    assert e.value.status == 1
    with pytest.raises(lib.KsgError) as e:
        ctx.cmi_noalloc(one[:, :4], one[:, :4], None, 4)  # N <= k
    assert e.value.status == 2
    p = workloads.random_problem(503, 300, 1, 1, 1, 4)
    x = p.x.copy()
    x[17, 0] = np.inf
    out = ctx.cmi_noalloc(soa(x), soa(p.y), soa(p.z), 4)
    torch.cuda.synchronize()
    assert np.isnan(float(out.cpu()[0]))
    # the flag is cleared by the next call
    got, ref_api = _both(ctx, p, 4)
    assert abs(got - ref_api) <= tol(ref_api)


def test_noalloc_at_the_size_limit(lib, ctx):
    """N = KSG_NOALLOC_MAX_N rows and 16 columns (the largest call the static array holds),
    then a small call: both equal the allocating entry point's estimate."""
    big = workloads.random_problem(504, lib.KSG_NOALLOC_MAX_N, 1, 1, 14, 4)
    small = workloads.random_problem(505, 500, 1, 2, 0, 4)
    for p in (big, small):
        got, ref_api = _both(ctx, p, 4)
        assert abs(got - ref_api) <= tol(ref_api), (p.n, got, ref_api)
