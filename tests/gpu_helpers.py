"""Shared plumbing of the GPU tests: device tensors <-> numpy, ragged batches."""
import numpy as np
import torch

DEV = torch.device("cuda", 0)


def c2d(arr) -> torch.Tensor:
    """complex128 numpy -> interleaved float64 device tensor."""
    a = np.ascontiguousarray(np.asarray(arr, dtype=np.complex128))
    return torch.from_numpy(a.view(np.float64).copy()).to(DEV)


def c64d(arr) -> torch.Tensor:
    a = np.ascontiguousarray(np.asarray(arr, dtype=np.complex64))
    return torch.from_numpy(a.view(np.float32).copy()).to(DEV)


def d2c(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy().astype(np.float64).view(np.complex128)


def f64d(arr) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(np.asarray(arr, np.float64))).to(DEV)


def zeros_c(n):
    return torch.zeros(2 * int(n), dtype=torch.float64, device=DEV)


def ragged(ns):
    n = np.asarray(ns, np.int64)
    off = np.concatenate([[0], np.cumsum(n)[:-1]]).astype(np.int64)
    return n, off


def relerr(a, b):
    a, b = np.asarray(a), np.asarray(b)
    den = np.max(np.abs(b)) if b.size else 1.0
    return float(np.max(np.abs(a - b)) / (den if den > 0 else 1.0)) if a.size else 0.0
