"""Device-side seeded generator for the large synthetic problems.

Same structure as ``synth.problems`` (Hermitian A = Q diag(d) Q^H with Q
Haar-unitary, complex symmetric B with ||B||_2 = c min d, raw Gaussian
initial block and Lanczos starts), drawn with torch on the GPU so that the
m = 16000 and m = 30000 workloads can be built in seconds.  The draws come
from a ``torch.Generator`` on the device seeded with ``seed``; d comes from
``numpy.random.default_rng(seed)`` with the same rules as the host
generator.  The spectral norm of B is estimated by power iteration on
B^H B (it underestimates ||B||_2 by well under 1%, which keeps SH definite
with the same margin).  Input construction only: none of the eigensolver's
arithmetic is here.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import torch

from .problems import CONFIGS


@dataclasses.dataclass
class DeviceProblem:
    name: str
    m: int
    A: torch.Tensor        # (m, m) complex128, C-contiguous, Hermitian
    B: torch.Tensor        # (m, m) complex128, C-contiguous, symmetric
    d: np.ndarray
    coupling: float
    nev: int
    nex: int
    deg: int
    tol: float
    deg_min: int
    deg_max: int
    w0_raw: torch.Tensor   # (n, nevex) complex128
    lanczos_raw: torch.Tensor  # (n, 4) complex128
    seed: int

    @property
    def n(self) -> int:
        return 2 * self.m

    @property
    def nevex(self) -> int:
        return self.nev + self.nex


def _cnormal(shape, gen, device):
    re = torch.randn(shape, dtype=torch.float64, device=device, generator=gen)
    im = torch.randn(shape, dtype=torch.float64, device=device, generator=gen)
    return torch.complex(re, im)


def _spectral_norm(B: torch.Tensor, gen, iters: int = 300) -> float:
    x = _cnormal((B.shape[0], 1), gen, B.device)
    x = x / torch.linalg.vector_norm(x)
    Bh = B.conj().T.contiguous()
    s = 0.0
    for _ in range(iters):
        y = Bh @ (B @ x)
        s = float(torch.linalg.vector_norm(y))
        x = y / s
    return math.sqrt(s)


def config_problem_device(i: int, seed: int = 0, device="cuda", m=None, nev=None, nex=None) -> DeviceProblem:
    c = dict(CONFIGS[i])
    name = c.pop("name")
    m = c["m"] if m is None else m
    nev = c["nev"] if nev is None else nev
    nex = c["nex"] if nex is None else nex
    rng = np.random.default_rng(seed)
    d = np.asarray(c["d_draw"](rng, m), dtype=np.float64)
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    z = _cnormal((m, m), gen, device) / math.sqrt(2.0)
    q, r = torch.linalg.qr(z)
    del z
    ph = torch.diagonal(r)
    ph = ph / ph.abs()
    del r
    q = q * ph[None, :]
    dt = torch.from_numpy(d).to(device=device, dtype=torch.complex128)
    A = (q * dt[None, :]) @ q.conj().T.contiguous()
    del q
    A = 0.5 * (A + A.conj().T.contiguous())
    g = _cnormal((m, m), gen, device)
    B = 0.5 * (g + g.T.contiguous())
    del g
    B = B * (c["coupling"] * float(d.min()) / _spectral_norm(B, gen))
    B = 0.5 * (B + B.T.contiguous())
    n = 2 * m
    w0 = _cnormal((n, nev + nex), gen, device)
    lz = _cnormal((n, 4), gen, device)
    deg = c["deg"]
    return DeviceProblem(name=name, m=m, A=A.contiguous(), B=B.contiguous(), d=d, coupling=c["coupling"],
                         nev=nev, nex=nex, deg=deg, tol=c["tol"], deg_min=c.get("deg_min", deg),
                         deg_max=c.get("deg_max", deg), w0_raw=w0, lanczos_raw=lz, seed=seed)
