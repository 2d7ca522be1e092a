"""Scaled factorization residual evaluated with torch, for large matrices that
already sit on the device (test infrastructure).

``factor_residual(A0, LU, ipiv)`` computes ||P A - L U||_F / (||A||_F n eps),
eps = 2**-53, the same quantity as ``oracle.r_factor``, with torch's FP64
products in column slabs so that only one n x slab product is alive at a
time.  It runs on whatever device the tensors live on; its value is pinned
on the CPU against a hand-worked example in ``test_residual_pins.py``.
"""
from __future__ import annotations

import numpy as np

import oracle


def factor_residual(A0, LU, ipiv: np.ndarray, slab: int = 4096) -> float:
    import torch
    n = A0.shape[0]
    if n == 0:
        return 0.0
    perm = torch.tensor(oracle.perm_from_ipiv(ipiv), device=A0.device)
    L = torch.tril(LU, -1)
    L.diagonal().fill_(1.0)
    acc = 0.0
    for c0 in range(0, n, slab):
        c1 = min(n, c0 + slab)
        U = torch.triu(LU[:, c0:c1], diagonal=-c0)[:c1, :]      # rows < c1 of U's columns c0..c1
        R = A0[perm, c0:c1] - L[:, :c1] @ U
        acc += float((R * R).sum().item())
        del U, R
    del L
    return acc ** 0.5 / (torch.linalg.norm(A0).item() * n * 2.0 ** -53)
