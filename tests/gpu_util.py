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


def drifted(R, L, sigma_cells, h_cell, seed):
    """Positions R [N, 4] moved by Gaussian steps of sigma_cells cells, wrapped into the box."""
    rng = np.random.default_rng(seed)
    out = R.copy()
    xyz = R[:, :3].astype(np.float64) + rng.standard_normal((len(R), 3)) * sigma_cells * h_cell
    Lf = np.broadcast_to(np.asarray(L, dtype=np.float32), (3,))
    out[:, :3] = np.mod(xyz, Lf.astype(np.float64)).astype(np.float32)
    out[:, :3] = np.where(out[:, :3] >= Lf, np.float32(0), out[:, :3])
    return out


def field_of(st):
    """Counts (any-order scatter), potential and gradient of the current positions."""
    from paper_1310_2041_amd import hpf
    hpf.hpf_density_scatter(st.R, st.T, st.mesh, st.K, st.counts)
    hpf.hpf_field_potential(st.counts, st.mesh, st.field, st.V, None)
    hpf.hpf_field_gradient(st.V, st.mesh, st.K, st.G)
