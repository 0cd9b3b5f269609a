"""Helpers shared by the GPU parity tests (data movement and error norms only)."""
from __future__ import annotations

import numpy as np
import torch


def dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a)).to("cuda").to(dtype).contiguous()


def host(t):
    return t.detach().cpu().numpy()


def counts_np(t, K, M):
    """GPU counts tensor (int64 bits) -> numpy uint64 [K, Mz, My, Mx]."""
    return host(t).view(np.uint64).reshape(K, M[2], M[1], M[0])


def rel_max(a, b):
    """max |a - b| / max |b| (relative max-norm)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    scale = np.abs(b).max() if b.size else 0.0
    if scale == 0.0:
        return float(np.abs(a - b).max()) if a.size else 0.0
    return float(np.abs(a - b).max() / scale)


def by_tag(arr, tag, N):
    out = np.zeros((N,) + arr.shape[1:], dtype=arr.dtype)
    out[tag] = arr
    return out


def box_delta(a, b, L):
    """Minimum-image difference of positions a - b in a box L."""
    d = np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64)
    Lv = np.asarray(L, dtype=np.float64)
    return d - Lv * np.rint(d / Lv)
