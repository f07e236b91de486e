"""Helpers shared by the GPU tests (device selection, skips, tolerances)."""
import pytest


def require_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch
