"""Helpers shared by the GPU tests: moving seeded numpy inputs to device tensors."""
import numpy as np


def dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def soa(points):
    """Row-major [N][d] float32 points -> device SoA [d][N] float32 (None for d == 0)."""
    import torch
    if points is None:
        return None
    p = np.asarray(points, dtype=np.float32)
    if p.ndim == 1:
        p = p[:, None]
    if p.shape[1] == 0:
        return None
    return torch.from_numpy(np.ascontiguousarray(p.T)).cuda()


def tol(ref):
    """Floating-point acceptance bound for a CMI value: 1e-12 relative, 1e-12 nats absolute floor."""
    return 1e-12 * max(abs(ref), 1.0)
