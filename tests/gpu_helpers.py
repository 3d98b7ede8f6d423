"""Shared helpers of the GPU parity tests (host-side only)."""
import numpy as np
import torch

from paper_2601_10557_amd import colmajor


def to_dev(x, dtype=torch.complex128):
    t = torch.from_numpy(np.ascontiguousarray(x)).to(dtype)
    t = colmajor(t).cuda()
    if t.stride(0) != 1:
        t = colmajor(t)
    return t


def to_host(t):
    return t.detach().cpu().numpy()


def dev_blocks(p):
    """A, B as C-contiguous device tensors (the binding's convention)."""
    return (torch.from_numpy(np.ascontiguousarray(p.A)).cuda(),
            torch.from_numpy(np.ascontiguousarray(p.B)).cuda())


def align_columns(V, Vref):
    """Scale each column of V by the unit complex number that best matches
    Vref (eigenvectors are unique up to phase)."""
    out = V.copy()
    for j in range(V.shape[1]):
        c = np.vdot(V[:, j], Vref[:, j])
        out[:, j] = V[:, j] * (c / abs(c) if abs(c) > 0 else 1.0)
    return out


def print_case(name, **kw):
    print(f"[gpu case] {name} " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)
