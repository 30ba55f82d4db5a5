"""Helpers of the GPU parity tests: layout conversion and oracle replay."""

import numpy as np


def to_oracle(t, ndim):
    """Library layout (n2, n1, n0) tensor -> numpy float64 indexed [x, y(, z)]."""
    a = t.detach().cpu().double().numpy()
    if ndim == 2:
        return np.ascontiguousarray(a[0].T)
    return np.ascontiguousarray(a.transpose(2, 1, 0))


def plane_to_oracle(t, ndim):
    a = t.detach().cpu().double().numpy()
    return np.ascontiguousarray(a[0]) if ndim == 2 else np.ascontiguousarray(a.T)


def to_device(a, ndim, torch, dtype, device="cuda"):
    """numpy [x, y(, z)] -> library layout tensor (n2, n1, n0)."""
    if ndim == 2:
        a = a.T[None, :, :]
    else:
        a = a.transpose(2, 1, 0)
    return torch.from_numpy(np.ascontiguousarray(a)).to(device=device, dtype=dtype)


def rel_l2(a, b, mask=None):
    if mask is not None:
        a, b = a[mask], b[mask]
    den = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (den if den > 0 else 1.0)


def mean_free(p, active):
    q = np.where(active, p, 0.0)
    return np.where(active, q - q[active].mean(), 0.0)
