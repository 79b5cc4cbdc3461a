"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds input generation only -- none of the method's arithmetic.
Both the CPU oracle and the GPU library consume what it produces; neither is
imported here.

Workloads:

* H-equation (eq. (3.2) of Kelley, "Newton's Method in Three Precisions"):
  the problem is fully described by (N, c); the initial iterate is ones.
* Dense tanh system F(x) = A x + 0.1 tanh(x) - b (not from the paper; it is
  the pivoting workload): A = U diag(s) V^T, U and V the orthogonal factors
  of the QR factorisations of seeded N(0,1) matrices with the signs fixed so
  that R has a positive diagonal, s log-spaced from 1 to cond
  (s_k = cond^(k/(N-1))), b = A 1 + 0.1 tanh(1) so that x* = 1 exactly,
  x_0 = 0.
* Serving stream: seeded Poisson arrivals of H-equation requests with N drawn
  uniformly from {128, 256, 512, 1024, 2048} and c uniformly from
  [0.5, 0.999].
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np


@dataclasses.dataclass(frozen=True)
class HeqCase:
    n: int
    c: float

    def x0(self) -> np.ndarray:
        return np.ones(self.n)


def _orthogonal(n: int, seed: int) -> np.ndarray:
    g = np.random.default_rng(seed).standard_normal((n, n))
    q, r = np.linalg.qr(g)
    return q * np.sign(np.diag(r))[None, :]


def dense_tanh_system(n: int, cond: float, seed_u: int = 1, seed_v: int = 2):
    """(A, b, x0) for the dense tanh workload, FP64, A in Fortran order (CPU, numpy)."""
    U = _orthogonal(n, seed_u)
    V = _orthogonal(n, seed_v)
    s = cond ** (np.arange(n) / max(n - 1, 1))
    A = np.asfortranarray((U * s[None, :]) @ V.T)
    b = A @ np.ones(n) + 0.1 * np.tanh(1.0)
    return A, b, np.zeros(n)


def dense_tanh_system_torch(n: int, cond: float, device, seed_u: int = 1, seed_v: int = 2):
    """Same recipe generated with torch on ``device`` (for sizes numpy is too slow at).

    Returns (A, b, x0) as FP64 torch tensors; A is column-major (A.T contiguous).
    The random streams are torch's, so A differs from the numpy recipe's matrix
    of the same seed; x* = 1 holds exactly for both.
    """
    import torch

    def orth(seed):
        g = torch.Generator(device=device)
        g.manual_seed(seed)
        m = torch.randn(n, n, generator=g, device=device, dtype=torch.float64)
        q, r = torch.linalg.qr(m)
        return q * torch.sign(torch.diagonal(r))[None, :]

    U = orth(seed_u)
    V = orth(seed_v)
    s = cond ** (torch.arange(n, device=device, dtype=torch.float64) / max(n - 1, 1))
    A = (U * s[None, :]) @ V.T
    del U, V
    ones = torch.ones(n, device=device, dtype=torch.float64)
    b = A @ ones + 0.1 * float(np.tanh(1.0))
    A_cm = A.T.contiguous().T  # column-major storage
    return A_cm, b, torch.zeros(n, device=device, dtype=torch.float64)


@dataclasses.dataclass(frozen=True)
class Request:
    rid: int
    arrival_s: float
    n: int
    c: float


def serving_stream(count: int = 2000, rate_per_s: float = 200.0, seed: int = 7,
                   sizes=(128, 256, 512, 1024, 2048), c_range=(0.5, 0.999)) -> List[Request]:
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, size=count)
    t = np.cumsum(gaps)
    ns = rng.choice(np.asarray(sizes), size=count)
    cs = rng.uniform(c_range[0], c_range[1], size=count)
    return [Request(i, float(t[i]), int(ns[i]), float(cs[i])) for i in range(count)]


def random_matrix(n: int, seed: int, dist: str = "normal", diag_shift: Optional[float] = None):
    """Seeded dense test matrix (FP64, Fortran order) for factorisation tests."""
    rng = np.random.default_rng(seed)
    if dist == "normal":
        A = rng.standard_normal((n, n))
    elif dist == "uniform":
        A = rng.uniform(-1.0, 1.0, (n, n))
    else:
        raise ValueError(dist)
    if diag_shift is not None:
        A = A + diag_shift * np.eye(n)
    return np.asfortranarray(A)
