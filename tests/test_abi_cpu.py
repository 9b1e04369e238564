"""C-ABI boundary checks that need no GPU: the library loads, exports every declared entry
point, its host-side harmonic table matches the oracle's, and argument errors are reported
without touching a device."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ksgcmi.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*([a-z_0-9]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = _declared()
    for fn in ("cmi_ksg", "cmi_ksg_batch", "select_parents", "ksg_maxstat", "ksg_embed",
               "ksg_mlp_train", "ksg_mlp_forward", "ksg_mlp_grad"):
        assert fn in names


def test_library_exports_every_declared_symbol():
    import paper_1807_10459_amd as ksg
    out = subprocess.run(["nm", "-D", "--defined-only", ksg.lib_path], capture_output=True, text=True,
                         check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing
    for n in _declared():
        assert hasattr(ksg.lib, n)


def test_harmonic_table_matches_oracle():
    import paper_1807_10459_amd as ksg
    from oracle.harmonic import harmonic_table
    h = ksg.harmonic_table(60000)
    ref = harmonic_table(60000)
    assert np.array_equal(h, ref)


def test_status_strings_and_null_context():
    import paper_1807_10459_amd as ksg
    L = ksg.lib
    assert ksg.status_string(0) == "ok"
    assert ksg.status_string(2).startswith("too few")
    assert L.ksg_version() >= 10000
    # every entry point rejects a null context before any device work
    d = C.c_double()
    dims = (C.c_int32 * 3)(1, 1, 0)
    assert L.cmi_ksg(None, None, None, None, 10, dims, 4, C.byref(d)) == 1
    assert L.cmi_ksg_batch(None, None, 0, None) == 1
    assert L.ksg_maxstat(None, None, 1, 1, 0.05, None) == 1
    assert L.ksg_embed(None, None, 1, 10, 1, 0, 1, None, None) == 1
    assert L.select_parents(None, None, 1, 10, 1, 0, None, None) == 1
    assert L.ksg_ctx_set_option(None, 1, 0) == 1
    assert L.ksg_harmonic_table(-1, None) == 1
    assert L.ksg_last_error(None) == b"null context"
    L.ksg_ctx_destroy(None)  # no-op


def test_no_device_reported_without_gpu():
    import torch
    import paper_1807_10459_amd as ksg
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = C.c_void_p()
    assert ksg.lib.ksg_device_count() == 0
    assert ksg.lib.ksg_ctx_create(C.byref(h), 0, None) == 6  # KSG_ENODEV
    assert ksg.lib.ksg_ctx_create(None, 0, None) == 1


def test_product_never_imports_the_oracle():
    pkg = os.path.join(ROOT, "paper_1807_10459_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in txt.replace("the oracle", ""), f
                assert "import workloads" not in txt, f


def test_fdr_bh_matches_oracle():
    """The library's Benjamini-Hochberg (host code) against the oracle's."""
    import paper_1807_10459_amd as ksg
    import workloads
    from oracle.stats import fdr_bh
    g = workloads.rng(15)
    for _ in range(200):
        m = int(g.integers(0, 25))
        p = np.where(g.random(m) < 0.3, g.random(m) * 0.01, g.random(m))
        p[g.random(m) < 0.2] = 0.02  # ties
        alpha = float(g.choice([0.01, 0.05, 0.2]))
        assert np.array_equal(ksg.fdr_bh(p, alpha), fdr_bh(p, alpha))
    with pytest.raises(ksg.KsgError):
        ksg.fdr_bh([0.1], 1.5)


def test_maxstat_sequential_matches_oracle():
    """The library's sequential max-statistic test (host code) against the oracle's."""
    import paper_1807_10459_amd as ksg
    import workloads
    from oracle.stats import max_statistic_sequential
    g = workloads.rng(16)
    for _ in range(300):
        c = int(g.integers(0, 8))
        P = int(g.integers(1, 40))
        t = np.round(g.standard_normal((c, P + 1)), 1)  # coarse values: ties
        t[:, 0] += g.random() * 2.0 * (g.random(c) < 0.5)  # some clearly significant rows
        alpha = float(g.choice([0.05, 0.2, 0.5]))
        sig, p = ksg.maxstat_sequential(t.reshape(c, P + 1), alpha)
        rs, rp = max_statistic_sequential(t.reshape(c, P + 1), alpha)
        assert np.array_equal(sig, rs) and np.array_equal(p, rp)
    with pytest.raises(ksg.KsgError):
        ksg.maxstat_sequential(np.zeros((2, 3)), 0.0)
