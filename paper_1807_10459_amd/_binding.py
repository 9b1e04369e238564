"""ctypes binding of ``libksgcmi.so``: argument marshalling only."""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
lib_path = os.path.join(_HERE, "libksgcmi.so")

KSG_MAX_DIMS = 32
KSG_MAX_K = 16
KSG_NOALLOC_MAX_N = 65536
MLP_NPARAMS = 5378
MLP_NFEAT = 16

_STATUS = {0: "KSG_OK", 1: "KSG_EINVAL", 2: "KSG_ETOOFEW", 3: "KSG_ENONFINITE", 4: "KSG_ENOMEM",
           5: "KSG_EDEVICE", 6: "KSG_ENODEV", 7: "KSG_EBUFSMALL"}


class KsgError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_STATUS.get(status, status)}: {message}")
        self.status = status
        self.message = message


class _Problem(C.Structure):
    _fields_ = [("n", C.c_int64), ("dx", C.c_int32), ("dy", C.c_int32), ("dz", C.c_int32),
                ("k", C.c_int32), ("x", C.c_void_p), ("y", C.c_void_p), ("z", C.c_void_p),
                ("perm_x", C.c_void_p), ("eps_out", C.c_void_p), ("counts_out", C.c_void_p),
                ("local_out", C.c_void_p)]


class _MaxStat(C.Structure):
    _fields_ = [("c_star", C.c_int32), ("count", C.c_int32), ("significant", C.c_int32),
                ("n_perm", C.c_int32), ("t_obs", C.c_double), ("pval", C.c_double),
                ("tau05", C.c_double), ("tau01", C.c_double)]


class _DeviceProps(C.Structure):
    _fields_ = [("name", C.c_char * 128), ("arch", C.c_char * 64), ("cus", C.c_int32), ("clock_khz", C.c_int32),
                ("mem_clock_khz", C.c_int32), ("mem_bus_bits", C.c_int32), ("total_mem", C.c_int64),
                ("l2_bytes", C.c_int32), ("lds_per_cu", C.c_int32), ("lds_per_block", C.c_int32),
                ("wave_size", C.c_int32)]


class _SelectOpts(C.Structure):
    _fields_ = [("k", C.c_int32), ("max_lag", C.c_int32), ("n_perm", C.c_int32),
                ("omnibus", C.c_int32), ("alpha", C.c_double), ("perms", C.c_void_p),
                ("learned", C.c_void_p), ("margin_lo", C.c_double), ("margin_hi", C.c_double),
                ("judge", C.c_int32), ("max_steps", C.c_int32), ("mode", C.c_int32), ("prune", C.c_int32),
                ("sequential", C.c_int32), ("max_cond", C.c_int32), ("resume", C.c_void_p),
                ("n_resume", C.c_int32), ("verify_stop", C.c_int32), ("deep_dz", C.c_int32),
                ("margin_lo_deep", C.c_double), ("margin_hi_deep", C.c_double)]


class _ParentSet(C.Structure):
    _fields_ = [("capacity", C.c_int32), ("n", C.c_int32), ("var", C.c_void_p), ("lag", C.c_void_p),
                ("cmi", C.c_void_p), ("pval", C.c_void_p), ("n_steps", C.c_int32),
                ("n_fallback", C.c_int32), ("n_disagree", C.c_int32), ("n_gate_decided", C.c_int32),
                ("omnibus_tested", C.c_int32), ("omnibus_significant", C.c_int32),
                ("omnibus_cmi", C.c_double), ("omnibus_pval", C.c_double), ("n_cmi", C.c_int64),
                ("step_capacity", C.c_int32), ("step_tobs", C.c_void_p), ("step_pred", C.c_void_p),
                ("step_verdict", C.c_void_p), ("step_plain", C.c_void_p), ("n_pruned", C.c_int32),
                ("pruned", C.c_void_p), ("n_seq_removed", C.c_int32), ("seq_removed", C.c_void_p),
                ("seq_pval", C.c_void_p), ("truncated", C.c_int32)]


def _load():
    # The HIP runtime is process-wide: load PyTorch's first so that the library and the
    # tensors it is handed share one runtime instance.
    import torch  # noqa: F401
    if not os.path.exists(lib_path):
        raise ImportError(f"{lib_path} is missing: build it with __graft_entry__.build() "
                          "(hipcc --offload-arch=gfx950)")
    L = C.CDLL(lib_path)
    vp, i32, i64, d, f = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_float
    sig = {
        "ksg_version": ([], i32),
        "ksg_status_string": ([i32], C.c_char_p),
        "ksg_device_count": ([], i32),
        "ksg_harmonic_table": ([i64, vp], i32),
        "ksg_device_props_get": ([i32, C.POINTER(_DeviceProps)], i32),
        "ksg_ctx_create": ([C.POINTER(vp), i32, vp], i32),
        "ksg_ctx_destroy": ([vp], None),
        "ksg_last_error": ([vp], C.c_char_p),
        "ksg_ctx_set_option": ([vp, i32, i64], i32),
        "ksg_autotune": ([vp, i64, C.c_char_p, vp], i32),
        "ksg_last_work": ([vp, vp], i32),
        "ksg_graph_stats": ([vp, C.POINTER(i64), C.POINTER(i64), C.POINTER(i64)], i32),
        "ksg_last_kernels": ([vp, vp, vp, vp], i32),
        "ksg_take_timing": ([vp, C.POINTER(d), C.POINTER(i64), C.POINTER(d)], i32),
        "cmi_ksg": ([vp, vp, vp, vp, i64, vp, i32, C.POINTER(d)], i32),
        "cmi_ksg_batch": ([vp, C.POINTER(_Problem), i32, vp], i32),
        "cmi_ksg_noalloc": ([vp, vp, vp, vp, i64, vp, i32, vp], i32),
        "ksg_maxstat": ([vp, vp, i32, i32, d, C.POINTER(_MaxStat)], i32),
        "ksg_embed": ([vp, vp, i32, i64, i32, i32, i32, vp, vp], i32),
        "ksg_greedy_step": ([vp, vp, vp, i64, vp, i32, vp, i32, vp, i32, i32, d, vp, C.POINTER(_MaxStat)], i32),
        "select_parents": ([vp, vp, i32, i64, i32, i32, C.POINTER(_SelectOpts), C.POINTER(_ParentSet)], i32),
        "ksg_mlp_create": ([vp, C.POINTER(vp), vp], i32),
        "ksg_mlp_destroy": ([vp], None),
        "ksg_mlp_set_norm": ([vp, vp, vp], i32),
        "ksg_mlp_get_params": ([vp, vp, i32], i32),
        "ksg_mlp_set_params": ([vp, vp], i32),
        "ksg_mlp_forward": ([vp, vp, vp, i64, vp], i32),
        "ksg_mlp_grad": ([vp, vp, vp, vp, i64, vp, vp], i32),
        "ksg_mlp_train": ([vp, vp, vp, vp, i64, i32, i32, f, vp], i32),
        "ksg_mlp_save": ([vp, C.c_char_p], i32),
        "ksg_mlp_load": ([vp, C.POINTER(vp), C.c_char_p], i32),
        "ksg_null_examples": ([vp, vp, i32, i32, vp, vp, vp, i32, vp, i32, vp, i64, i32, i32, vp, vp, vp], i32),
        "ksg_mlp_fit_norm": ([vp, vp, vp, i64], i32),
        "ksg_gate_calibrate": ([vp, vp, vp, vp, i64, d, C.POINTER(d), C.POINTER(d), C.POINTER(d),
                                C.POINTER(i64)], i32),
        "ksg_gate_calibrate_sides": ([vp, vp, vp, vp, i64, d, d, C.POINTER(d), C.POINTER(d), C.POINTER(d),
                                      C.POINTER(i64)], i32),
        "ksg_step_features": ([vp, vp, i32, vp, vp, i64, vp, i32, i32, i32, i32, i32, vp], i32),
        "ksg_fdr_bh": ([vp, i32, d, vp], i32),
        "ksg_maxstat_sequential": ([vp, i32, i32, d, vp, vp], i32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    return L


lib = _load()


def status_string(st: int) -> str:
    return lib.ksg_status_string(st).decode()


def harmonic_table(nmax: int) -> np.ndarray:
    out = np.empty(nmax + 1, dtype=np.float64)
    st = lib.ksg_harmonic_table(nmax, out.ctypes.data)
    if st:
        raise KsgError(st, "ksg_harmonic_table")
    return out


def device_props(device: int = 0) -> dict:
    """What the HIP runtime reports for a device (see ksg_device_props_get)."""
    p = _DeviceProps()
    st = lib.ksg_device_props_get(int(device), C.byref(p))
    if st:
        raise KsgError(st, "ksg_device_props_get")
    out = {f: getattr(p, f) for f, _ in _DeviceProps._fields_}
    out["name"] = p.name.decode(errors="replace")
    out["arch"] = p.arch.decode(errors="replace")
    return out


def fdr_bh(pvals, alpha: float = 0.05) -> np.ndarray:
    """Benjamini-Hochberg decisions across targets (see ksg_fdr_bh)."""
    p = np.ascontiguousarray(np.asarray(pvals, dtype=np.float64))
    out = np.zeros(p.size, np.int32)
    st = lib.ksg_fdr_bh(p.ctypes.data, p.size, float(alpha), out.ctypes.data)
    if st:
        raise KsgError(st, "ksg_fdr_bh")
    return out.astype(bool)


def maxstat_sequential(table, alpha: float = 0.05):
    """Sequential max-statistic test of a host table [rows][P+1] (see ksg_maxstat_sequential);
    returns (significant bool [rows], pval [rows])."""
    t = np.ascontiguousarray(np.asarray(table, dtype=np.float64))
    if t.ndim != 2 or t.shape[1] < 2:
        raise ValueError("table must be [rows][n_perm + 1] with n_perm >= 1")
    sig = np.zeros(t.shape[0], np.int32)
    pv = np.zeros(t.shape[0], np.float64)
    st = lib.ksg_maxstat_sequential(t.ctypes.data, t.shape[0], t.shape[1] - 1, float(alpha),
                                    sig.ctypes.data, pv.ctypes.data)
    if st:
        raise KsgError(st, "ksg_maxstat_sequential")
    return sig.astype(bool), pv


MODES = {"mte": 0, "bte": 1, "mmi": 2}


def _ptr(t) -> Optional[int]:
    """Device address of a CUDA tensor (None passes NULL)."""
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a torch tensor on a HIP device")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return t.data_ptr()


def _check_dtype(t, dtype, name):
    if t is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")


@dataclasses.dataclass
class Problem:
    """One I(X;Y|Z) problem over device tensors in SoA layout: x [dx][n], y [dy][n], z [dz][n]."""

    x: object
    y: object
    z: object = None
    k: int = 4
    perm_x: object = None
    eps_out: object = None
    counts_out: object = None
    local_out: object = None

    def _c(self) -> _Problem:
        import torch
        x, y, z = self.x, self.y, self.z
        for t, nm in ((x, "x"), (y, "y"), (z, "z")):
            _check_dtype(t, torch.float32, nm)
        _check_dtype(self.perm_x, torch.int32, "perm_x")
        _check_dtype(self.eps_out, torch.float32, "eps_out")
        _check_dtype(self.counts_out, torch.int32, "counts_out")
        _check_dtype(self.local_out, torch.float64, "local_out")
        x2 = x if x.dim() == 2 else x.view(1, -1)
        y2 = y if y.dim() == 2 else y.view(1, -1)
        z2 = None if z is None else (z if z.dim() == 2 else z.view(1, -1))
        n = x2.shape[1]
        dz = 0 if z2 is None else z2.shape[0]
        return _Problem(n, x2.shape[0], y2.shape[0], dz, int(self.k), _ptr(x2), _ptr(y2),
                        _ptr(z2) if dz > 0 else None, _ptr(self.perm_x), _ptr(self.eps_out),
                        _ptr(self.counts_out), _ptr(self.local_out))


class Context:
    """A library context on one device, issuing work on the current torch stream."""

    OPT_CHECK_FINITE = 1
    OPT_GROUP_SIZE = 2
    OPT_USE_GRAPH = 3
    OPT_TIMING = 4
    OPT_ALGORITHM = 5
    OPT_WINDOWS = 6
    OPT_GROUP_CHUNK = 7
    OPT_TILE_Q = 8
    OPT_MEM_LIMIT = 9

    def __init__(self, device: int = 0, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(device).cuda_stream
        h = C.c_void_p()
        st = lib.ksg_ctx_create(C.byref(h), int(device), C.c_void_p(stream))
        if st:
            raise KsgError(st, f"ksg_ctx_create(device={device})")
        self._h = h
        self.device = device

    def close(self):
        if getattr(self, "_h", None):
            lib.ksg_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _check(self, st: int, what: str):
        if st:
            raise KsgError(st, f"{what}: {lib.ksg_last_error(self._h).decode()}")

    def set_option(self, option: int, value: int):
        self._check(lib.ksg_ctx_set_option(self._h, option, int(value)), "ksg_ctx_set_option")

    def autotune(self, n: int = 8192, cache_path: Optional[str] = None):
        """Tune the launch shapes by timing (see ksg_autotune); returns the choices: group size per
        conditioning dimension m = 0..14 (k <= 4, k <= 8), brute-force tile height for launches of
        few / many work-groups, smallest N searched with key-ordered windows per column count D
        (None: never)."""
        out = np.zeros(46, np.int32)
        self._check(lib.ksg_autotune(self._h, int(n), cache_path.encode() if cache_path else None,
                                     out.ctypes.data), "ksg_autotune")
        big = np.iinfo(np.int32).max
        return {"k<=4": out[:15].tolist(), "k<=8": out[15:30].tolist(),
                "tile_q": {"few_groups": int(out[30]), "many_groups": int(out[31])},
                "window_min_n": {str(D): (None if int(v) == big else int(v))
                                 for D, v in zip(range(3, 17), out[32:46])}}

    def graph_stats(self) -> dict:
        """Batches captured into graphs, graph replays and graphs held (KSG_OPT_USE_GRAPH)."""
        a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
        self._check(lib.ksg_graph_stats(self._h, C.byref(a), C.byref(b), C.byref(c)), "ksg_graph_stats")
        return dict(captures=a.value, replays=b.value, held=c.value)

    def take_timing(self):
        """(search-kernel milliseconds, launches, algorithmic FP32 ops) since the last call."""
        ms, n, ops = C.c_double(), C.c_int64(), C.c_double()
        self._check(lib.ksg_take_timing(self._h, C.byref(ms), C.byref(n), C.byref(ops)), "ksg_take_timing")
        return ms.value, n.value, ops.value

    def last_work(self):
        """Grouped-kernel work counters behind the last take_timing: (radius problem-steps,
        X-count problem-steps, radius shared operations / 256, Y/Z count operations, X-count
        shared operations / 256); a step is 4 references x 64 lanes."""
        w = (C.c_uint64 * 5)()
        self._check(lib.ksg_last_work(self._h, w), "ksg_last_work")
        return tuple(int(v) for v in w)

    KERNELS = ("radius", "yz_count", "x_count", "single")

    def last_kernels(self):
        """Per-kernel {name: (ms, ops, launches)} of the last take_timing."""
        ms, ops, n = (C.c_double * 4)(), (C.c_double * 4)(), (C.c_int64 * 4)()
        self._check(lib.ksg_last_kernels(self._h, ms, ops, n), "ksg_last_kernels")
        return {k: (ms[i], ops[i], int(n[i])) for i, k in enumerate(self.KERNELS)}

    # ---------------------------------------------------------------- estimator
    def cmi(self, x, y, z=None, k: int = 4) -> float:
        p = Problem(x, y, z, k)._c()
        dims = (C.c_int32 * 3)(p.dx, p.dy, p.dz)
        out = C.c_double()
        self._check(lib.cmi_ksg(self._h, p.x, p.y, p.z, p.n, dims, int(k), C.byref(out)), "cmi_ksg")
        return out.value

    def cmi_noalloc(self, x, y, z=None, k: int = 4, out=None):
        """cmi_ksg_noalloc: the estimate into the device FP64 tensor out[0] (a new one-element
        tensor when out is None), queued on the stream without allocating in the library."""
        import torch
        p = Problem(x, y, z, k)._c()
        if out is None:
            out = torch.empty(1, dtype=torch.float64, device=x.device)
        _check_dtype(out, torch.float64, "out")
        dims = (C.c_int32 * 3)(p.dx, p.dy, p.dz)
        self._check(lib.cmi_ksg_noalloc(self._h, p.x, p.y, p.z, p.n, dims, int(k), _ptr(out)), "cmi_ksg_noalloc")
        return out

    def cmi_batch(self, problems: Sequence[Problem], out=None):
        import torch
        n = len(problems)
        if out is None:
            out = torch.empty(n, dtype=torch.float64, device=f"cuda:{self.device}")
        _check_dtype(out, torch.float64, "out")
        arr = (_Problem * max(n, 1))(*[p._c() for p in problems])
        self._check(lib.cmi_ksg_batch(self._h, arr, n, _ptr(out) if n else None), "cmi_ksg_batch")
        return out

    def maxstat(self, table, alpha: float = 0.05) -> dict:
        import torch
        _check_dtype(table, torch.float64, "table")
        c, p1 = table.shape
        r = _MaxStat()
        self._check(lib.ksg_maxstat(self._h, _ptr(table), c, p1 - 1, float(alpha), C.byref(r)), "ksg_maxstat")
        return dict(c_star=r.c_star, count=r.count, significant=bool(r.significant), n_perm=r.n_perm,
                    t_obs=r.t_obs, pval=r.pval, tau05=r.tau05, tau01=r.tau01)

    def embed(self, data, target: int, max_lag: int, out=None):
        """Candidate columns [n_vars*max_lag][N] and target column [N]; out = (cand, y) to write
        into caller-owned buffers (fixed addresses, e.g. for graph replay of later steps)."""
        import torch
        _check_dtype(data, torch.float32, "data")
        n_trials, n_vars, T = data.shape
        N = n_trials * (T - max_lag)
        if out is None:
            cand = torch.empty((n_vars * max_lag, N), dtype=torch.float32, device=data.device)
            y = torch.empty(N, dtype=torch.float32, device=data.device)
        else:
            cand, y = out
            _check_dtype(cand, torch.float32, "cand")
            _check_dtype(y, torch.float32, "y")
            if tuple(cand.shape) != (n_vars * max_lag, N) or tuple(y.shape) != (N,) or not (
                    cand.is_contiguous() and y.is_contiguous()):
                raise ValueError(f"embed: out must be contiguous [{n_vars * max_lag}][{N}] and [{N}]")
        self._check(lib.ksg_embed(self._h, _ptr(data), n_vars, T, n_trials, int(target), int(max_lag),
                                  _ptr(cand), _ptr(y)), "ksg_embed")
        return cand, y

    def greedy_step(self, cand, y, pool, cond, perms, k: int = 4, alpha: float = 0.05, out=None):
        """One greedy step: CMI table [len(pool)][P+1] (device FP64) and the max-statistic result."""
        import torch
        _check_dtype(cand, torch.float32, "cand")
        _check_dtype(y, torch.float32, "y")
        _check_dtype(perms, torch.int32, "perms")
        pool = np.ascontiguousarray(np.asarray(pool, np.int32))
        cond = np.ascontiguousarray(np.asarray(cond, np.int32).reshape(-1))
        P = perms.shape[0]
        if out is None:
            out = torch.empty((len(pool), P + 1), dtype=torch.float64, device=cand.device)
        r = _MaxStat()
        self._check(lib.ksg_greedy_step(self._h, _ptr(cand), _ptr(y), y.shape[0], pool.ctypes.data, len(pool),
                                        cond.ctypes.data if cond.size else None, cond.size, _ptr(perms), P,
                                        int(k), float(alpha), _ptr(out), C.byref(r)), "ksg_greedy_step")
        return out, dict(c_star=r.c_star, count=r.count, significant=bool(r.significant), n_perm=r.n_perm,
                         t_obs=r.t_obs, pval=r.pval, tau05=r.tau05, tau01=r.tau01)

    def select_parents(self, data, target: int, perms, k: int = 4, max_lag: int = 5,
                       alpha: float = 0.05, omnibus: bool = False, learned: "ThresholdNet" = None,
                       margin_lo: float = 1.0, margin_hi: float = 1.0, judge: bool = False,
                       max_steps: int = 0, capacity: int = 64, mode: str = "mte",
                       prune: bool = False, sequential: bool = False, max_cond: int = 0,
                       resume: Sequence[int] = (), verify_stop: bool = False,
                       deep_margins: tuple | None = None) -> dict:
        """Parents of one target.  mode: "mte" (multivariate TE), "bte" (bivariate TE) or "mmi"
        (multivariate MI); prune: min-statistic pruning of the selected sources; sequential:
        sequential max-statistic test of the kept sources; max_cond: conditioning columns allowed
        (0 = the library's limit); "truncated" in the result reports a selection that ended at it;
        resume: candidate indices an earlier run included (in order), to continue from them;
        verify_stop: with a learned null, a step the gate would stop on runs the plain test;
        deep_margins: (deep_dz, margin_lo, margin_hi) for the steps that condition on at least
        deep_dz columns."""
        import torch
        _check_dtype(data, torch.float32, "data")
        _check_dtype(perms, torch.int32, "perms")
        n_trials, n_vars, T = data.shape
        opts = _SelectOpts(int(k), int(max_lag), int(perms.shape[0]), int(bool(omnibus)), float(alpha),
                           _ptr(perms), learned._h if learned is not None else None, float(margin_lo),
                           float(margin_hi), int(bool(judge)), int(max_steps), MODES[mode], int(bool(prune)),
                           int(bool(sequential)), int(max_cond))
        opts.verify_stop = int(bool(verify_stop))
        if deep_margins is not None:
            opts.deep_dz, opts.margin_lo_deep, opts.margin_hi_deep = (int(deep_margins[0]), float(deep_margins[1]),
                                                                      float(deep_margins[2]))
        res_arr = np.ascontiguousarray(np.asarray(list(resume), dtype=np.int32))
        if res_arr.size:
            opts.resume, opts.n_resume = res_arr.ctypes.data, int(res_arr.size)
        var = np.zeros(capacity, np.int32)
        lag = np.zeros(capacity, np.int32)
        cmi = np.zeros(capacity, np.float64)
        pv = np.zeros(capacity, np.float64)
        scap = capacity + 1
        s_t = np.zeros(scap, np.float64)
        s_p = np.zeros((scap, 2), np.float32)
        s_v = np.zeros(scap, np.int32)
        s_pl = np.zeros(scap, np.int32)
        ps = _ParentSet(capacity, 0, var.ctypes.data, lag.ctypes.data, cmi.ctypes.data, pv.ctypes.data)
        ps.step_capacity = scap
        ps.step_tobs, ps.step_pred = s_t.ctypes.data, s_p.ctypes.data
        ps.step_verdict, ps.step_plain = s_v.ctypes.data, s_pl.ctypes.data
        prn = np.zeros(capacity, np.int32)
        ps.pruned = prn.ctypes.data
        srm = np.zeros(capacity, np.int32)
        spv = np.zeros(capacity, np.float64)
        ps.seq_removed, ps.seq_pval = srm.ctypes.data, spv.ctypes.data
        self._check(lib.select_parents(self._h, _ptr(data), n_vars, T, n_trials, int(target),
                                       C.byref(opts), C.byref(ps)), "select_parents")
        n = ps.n
        return dict(parents=[(int(var[i]), int(lag[i])) for i in range(n)],
                    candidates=[int(var[i]) * max_lag + int(lag[i]) - 1 for i in range(n)],
                    cmi=cmi[:n].tolist(), pval=pv[:n].tolist(), n_steps=ps.n_steps,
                    n_fallback=ps.n_fallback, n_disagree=ps.n_disagree,
                    n_gate_decided=ps.n_gate_decided, omnibus_tested=bool(ps.omnibus_tested),
                    omnibus_significant=bool(ps.omnibus_significant), omnibus_cmi=ps.omnibus_cmi,
                    omnibus_pval=ps.omnibus_pval, n_cmi=ps.n_cmi,
                    pruned=[int(v) for v in prn[:min(ps.n_pruned, capacity)]],
                    seq_removed=[int(v) for v in srm[:min(ps.n_seq_removed, capacity)]],
                    seq_pval=spv[:n].tolist(), truncated=bool(ps.truncated),
                    steps=[dict(t_obs=float(s_t[i]), pred=[float(s_p[i, 0]), float(s_p[i, 1])],
                                verdict=int(s_v[i]), plain=int(s_pl[i]))
                           for i in range(min(ps.n_steps, scap))])

    def null_examples(self, table, row_cand, subsets, cand, y, dz: int, k: int = 4):
        """Training examples from one step's surrogate table (see ksg_null_examples)."""
        import torch
        _check_dtype(table, torch.float64, "table")
        rows, p1 = table.shape
        rc = np.ascontiguousarray(np.asarray(row_cand, np.int32))
        off, sr = _csr(subsets)
        n_sub = len(subsets)
        feats = torch.empty((n_sub, MLP_NFEAT), dtype=torch.float32, device=table.device)
        targ = torch.empty((n_sub, 2), dtype=torch.float32, device=table.device)
        obs = torch.empty((n_sub, 2), dtype=torch.float64, device=table.device)
        self._check(lib.ksg_null_examples(self._h, _ptr(table), rows, p1 - 1, rc.ctypes.data, off.ctypes.data,
                                          sr.ctypes.data, n_sub, _ptr(cand), cand.shape[0], _ptr(y), y.shape[0],
                                          int(dz), int(k), _ptr(feats), _ptr(targ), _ptr(obs)),
                    "ksg_null_examples")
        return feats, targ, obs

    def step_features(self, orig_cmi, y, cand, cand_idx, dx, dy, dz, k, n_perm):
        import torch
        _check_dtype(orig_cmi, torch.float64, "orig_cmi")
        idx = np.ascontiguousarray(np.asarray(cand_idx, dtype=np.int32))
        out = torch.empty(MLP_NFEAT, dtype=torch.float32, device=orig_cmi.device)
        self._check(lib.ksg_step_features(self._h, _ptr(orig_cmi), len(idx), _ptr(y), _ptr(cand),
                                          y.shape[0], idx.ctypes.data, dx, dy, dz, k, n_perm, _ptr(out)),
                    "ksg_step_features")
        return out


def _csr(subsets):
    off = np.zeros(len(subsets) + 1, np.int32)
    off[1:] = np.cumsum([len(s) for s in subsets])
    rows = np.ascontiguousarray(np.concatenate([np.asarray(s, np.int32) for s in subsets]))
    return off, rows


class ThresholdNet:
    """The learned-null 16-64-64-2 network (BF16 parameters, FP32 accumulation) on one device."""

    def __init__(self, ctx: Context, init_params=None, _handle=None):
        self.ctx = ctx
        if _handle is not None:
            self._h = _handle
            return
        p = np.ascontiguousarray(np.asarray(init_params, dtype=np.float32))
        if p.size != MLP_NPARAMS:
            raise ValueError(f"expected {MLP_NPARAMS} parameters")
        h = C.c_void_p()
        ctx._check(lib.ksg_mlp_create(ctx._h, C.byref(h), p.ctypes.data), "ksg_mlp_create")
        self._h = h

    @classmethod
    def load(cls, ctx: Context, path: str) -> "ThresholdNet":
        h = C.c_void_p()
        ctx._check(lib.ksg_mlp_load(ctx._h, C.byref(h), path.encode()), "ksg_mlp_load")
        return cls(ctx, _handle=h)

    def close(self):
        if getattr(self, "_h", None):
            lib.ksg_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def save(self, path: str):
        st = lib.ksg_mlp_save(self._h, path.encode())
        if st:
            raise KsgError(st, f"ksg_mlp_save({path})")

    def set_norm(self, mu, sd):
        mu = np.ascontiguousarray(np.asarray(mu, np.float32))
        sd = np.ascontiguousarray(np.asarray(sd, np.float32))
        st = lib.ksg_mlp_set_norm(self._h, mu.ctypes.data, sd.ctypes.data)
        if st:
            raise KsgError(st, "ksg_mlp_set_norm")

    def params(self, bf16: bool = False) -> np.ndarray:
        out = np.empty(MLP_NPARAMS, np.float32)
        st = lib.ksg_mlp_get_params(self._h, out.ctypes.data, int(bf16))
        if st:
            raise KsgError(st, "ksg_mlp_get_params")
        return out

    def set_params(self, p):
        p = np.ascontiguousarray(np.asarray(p, np.float32))
        st = lib.ksg_mlp_set_params(self._h, p.ctypes.data)
        if st:
            raise KsgError(st, "ksg_mlp_set_params")

    def fit_norm(self, feats):
        self.ctx._check(lib.ksg_mlp_fit_norm(self.ctx._h, self._h, _ptr(feats), feats.shape[0]), "ksg_mlp_fit_norm")

    def calibrate(self, feats, obs, rate: float = 0.0025, include_rate: float | None = None) -> dict:
        """Gate margins (ksg_gate_calibrate); with include_rate, ksg_gate_calibrate_sides with
        rate/2 for wrong stops and include_rate for wrong inclusions."""
        lo, hi, fb, wrong = C.c_double(), C.c_double(), C.c_double(), C.c_int64()
        if include_rate is None:
            self.ctx._check(lib.ksg_gate_calibrate(self.ctx._h, self._h, _ptr(feats), _ptr(obs), feats.shape[0],
                                                   float(rate), C.byref(lo), C.byref(hi), C.byref(fb),
                                                   C.byref(wrong)), "ksg_gate_calibrate")
        else:
            self.ctx._check(lib.ksg_gate_calibrate_sides(self.ctx._h, self._h, _ptr(feats), _ptr(obs),
                                                         feats.shape[0], float(rate) / 2, float(include_rate),
                                                         C.byref(lo), C.byref(hi), C.byref(fb), C.byref(wrong)),
                            "ksg_gate_calibrate_sides")
        return dict(margin_lo=lo.value, margin_hi=hi.value, fallback=fb.value, wrong=wrong.value)

    def forward(self, feats):
        import torch
        _check_dtype(feats, torch.float32, "feats")
        out = torch.empty((feats.shape[0], 2), dtype=torch.float32, device=feats.device)
        self.ctx._check(lib.ksg_mlp_forward(self.ctx._h, self._h, _ptr(feats), feats.shape[0], _ptr(out)),
                        "ksg_mlp_forward")
        return out

    def grad(self, feats, targets):
        import torch
        g = torch.empty(MLP_NPARAMS, dtype=torch.float32, device=feats.device)
        loss = torch.empty(1, dtype=torch.float32, device=feats.device)
        self.ctx._check(lib.ksg_mlp_grad(self.ctx._h, self._h, _ptr(feats), _ptr(targets), feats.shape[0],
                                         _ptr(g), _ptr(loss)), "ksg_mlp_grad")
        return g, loss

    def train(self, feats, targets, epochs: int, batch: int, lr: float) -> np.ndarray:
        hist = np.zeros(max(epochs, 1), np.float32)
        self.ctx._check(lib.ksg_mlp_train(self.ctx._h, self._h, _ptr(feats), _ptr(targets), feats.shape[0],
                                          int(epochs), int(batch), float(lr), hist.ctypes.data),
                        "ksg_mlp_train")
        return hist[:epochs]
