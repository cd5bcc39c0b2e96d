"""Shared helpers of the GPU tests (device transfer, tolerances)."""
import numpy as np
import pytest


def need_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1510_03298_amd import glam  # raises if the library is missing
    return torch, glam


def rel_inf(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    den = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / (den if den > 0 else 1.0))


def dev(glam, a, dt):
    return glam.to_device_colmajor(a, dt)


def rounded(glam, torch, a, dt):
    """The values the device sees after conversion to dtype dt (as float64 numpy, same shape)."""
    t = torch.from_numpy(np.asarray(a, dtype=np.float64)).to(glam.torch_dtype(dt)).to(torch.float64)
    return t.numpy()
