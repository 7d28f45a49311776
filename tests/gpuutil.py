"""Helpers shared by the GPU tests (no arithmetic of the method here)."""
import numpy as np
import pytest


def need_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1206_3215_amd import binding  # noqa: F401  (fails loudly if libpst.so is missing)
    return torch


def to_dev(a, torch, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def to_host(t):
    return t.detach().cpu().numpy()


def rel_err(a, ref):
    """max |a - ref| / max |ref| (complex modulus)."""
    return float(np.max(np.abs(np.asarray(a) - ref)) / np.max(np.abs(ref)))
