"""MI355X (gfx950) nearest-neighbour conditional mutual information for greedy TE inference.

Thin Python binding over the C ABI of ``libksgcmi.so`` (declared in ``include/ksgcmi.h``).
It only marshals arguments: every step of the estimator, the surrogate test, the greedy
selection and the threshold network runs in the library's HIP kernels.  PyTorch provides
device memory and the stream; the library is loaded from this directory and the package
fails loudly when it is missing.
"""
from ._binding import (  # noqa: F401
    KSG_MAX_DIMS,
    KSG_MAX_K,
    KSG_NOALLOC_MAX_N,
    MLP_NFEAT,
    MLP_NPARAMS,
    Context,
    KsgError,
    Problem,
    ThresholdNet,
    device_props,
    fdr_bh,
    maxstat_sequential,
    harmonic_table,
    lib,
    lib_path,
    status_string,
)
