"""Helpers shared by the GPU tests (comparison metrics, skip logic)."""
import numpy as np
import pytest


def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def rel_maxnorm(a, b):
    """max|a - b| / max|b| in float64."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def announce(msg):
    print(f"[case] {msg}", flush=True)
