"""Shared helpers for the test suite (no method arithmetic here)."""
import numpy as np


def rel_err(got, want) -> float:
    got = np.asarray(got)
    want = np.asarray(want)
    den = np.linalg.norm(want.ravel())
    return float(np.linalg.norm((got - want).ravel()) / (den if den > 0 else 1.0))


def gpu_available() -> bool:
    try:
        import torch

        return torch.cuda.is_available()
    except Exception:
        return False


def to_dev(a, dtype=None):
    import torch

    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def to_host(t):
    return t.detach().cpu().numpy()
