"""Test helpers: population-order mapping between the oracle and the C ABI,
and GPU availability."""
import os

import numpy as np

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def abi_index(dim):
    """abi_index(dim)[k] = library population index of oracle direction k."""
    c, _, _ = oracle.lattice(dim)
    return np.array([(c[k, 0] + 1) + 3 * (c[k, 1] + 1) + (9 * (c[k, 2] + 1) if dim == 3 else 0)
                     for k in range(c.shape[0])])


def to_abi(dim, arr):
    out = np.empty_like(arr)
    out[abi_index(dim)] = arr
    return out


def from_abi(dim, arr):
    return np.asarray(arr)[abi_index(dim)]


def gpu_available():
    try:
        import torch

        return torch.cuda.is_available()
    except Exception:
        return False


def rel_err(got, want):
    return float(np.abs(np.asarray(got) - np.asarray(want)).max() /
                 max(float(np.abs(want).max()), 1e-300))
