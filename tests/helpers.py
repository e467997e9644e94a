"""Shared test helpers: GPU availability, oracle/HIP comparisons."""
import numpy as np
import pytest


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def require_gpu():
    if not gpu_available():
        pytest.skip("no HIP device")


def perturbed(nstar, seed=0, scale=0.3):
    rng = np.random.default_rng(seed)
    return nstar * np.exp(scale * rng.standard_normal(nstar.shape))


def to_dev(x, device="cuda"):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=device)


def to_np(t):
    return t.detach().cpu().numpy()


def maxrel(a, b, floor=0.0):
    a = np.asarray(a)
    b = np.asarray(b)
    den = np.maximum(np.abs(b), floor)
    with np.errstate(divide="ignore", invalid="ignore"):
        r = np.where(den > 0, np.abs(a - b) / den, np.abs(a - b))
    return float(np.max(r))
