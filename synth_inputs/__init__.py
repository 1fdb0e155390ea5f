"""Seeded synthetic inputs for the rank-1 SVD update.

This module is shared by the CPU oracle, the tests and the benchmark. It holds
no arithmetic of the update method itself: it only draws random factors and
vectors with the shapes and value distributions of the workloads below.

Workloads (the method itself is the symmetric rank-one update route of the
paper's Section 6; the paper's own experiments used unseeded random matrices):

* ``uniform``    sigma_i ~ U[lo, hi], sorted descending.
* ``geometric``  sigma_i = 10**(-6 i / m), i = 0..m-1.
* ``clustered``  geometric, plus 32 pairs whose second member sits at relative
                 distance 1e-11 below the first, plus 5 % of the projected
                 update components p = U^T a set to zero (optionally q = V^T b
                 zeroed at the same indices as well).

Orthogonal factors are Haar distributed: Q = qr(G) diag(sign(diag R)) with G a
seeded standard Gaussian matrix. The update vectors have i.i.d. N(0, 1/n)
entries.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np


@dataclass
class Problem:
    """One rank-1 update problem A = U diag(sigma) V^T (m <= n), plus a and b."""

    U: np.ndarray          # m x m, orthogonal
    sigma: np.ndarray      # m, descending, >= 0
    V: np.ndarray          # n x n, orthogonal
    a: np.ndarray          # m
    b: np.ndarray          # n
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return self.U.shape[0]

    @property
    def n(self) -> int:
        return self.V.shape[0]


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def haar(n: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-distributed orthogonal n x n matrix from a Gaussian QR."""
    if n == 0:
        return np.zeros((0, 0))
    G = rng.standard_normal((n, n))
    Q, R = np.linalg.qr(G)
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return Q * s[None, :]


def haar_torch(n: int, seed: int, device: str = "cuda"):
    """Haar orthogonal matrix built on a torch device (for sizes where a host QR is slow).

    The Gaussian is drawn on the host from a seeded torch generator and the QR
    runs on ``device``; the result stays on ``device``.
    """
    import torch

    g = torch.Generator(device="cpu")
    g.manual_seed(seed)
    G = torch.randn((n, n), generator=g, dtype=torch.float64).to(device)
    Q, R = torch.linalg.qr(G)
    s = torch.sign(torch.diagonal(R))
    s[s == 0] = 1.0
    return (Q * s[None, :]).contiguous()


def sigma_uniform(m: int, lo: float, hi: float, rng: np.random.Generator) -> np.ndarray:
    return np.sort(rng.uniform(lo, hi, size=m))[::-1].copy()


def sigma_geometric(m: int) -> np.ndarray:
    return 10.0 ** (-6.0 * np.arange(m) / max(m, 1))


def cluster_indices(m: int, pairs: int = 32) -> np.ndarray:
    """Indices i_k = floor((k + 1/2) m / pairs); sigma_{i_k + 1} is moved next to sigma_{i_k}."""
    idx = np.floor((np.arange(pairs) + 0.5) * m / pairs).astype(np.int64)
    return idx[idx + 1 < m]


def sigma_clustered(m: int, pairs: int = 32, rel: float = 1e-11) -> np.ndarray:
    s = sigma_geometric(m)
    for i in cluster_indices(m, pairs):
        s[i + 1] = s[i] * (1.0 - rel)
    return s


def make_problem(m: int, n: int, sigma: str = "uniform", seed: int = 0,
                 lo: float = 0.1, hi: float = 10.0, zero_frac: float = 0.0,
                 zero_q: bool = False, U: Optional[np.ndarray] = None,
                 V: Optional[np.ndarray] = None) -> Problem:
    """Build a seeded problem on the host (numpy, float64)."""
    if not (1 <= m <= n):
        raise ValueError("need 1 <= m <= n")
    rng = rng_for(seed)
    if U is None:
        U = haar(m, rng)
    if V is None:
        V = haar(n, rng)
    if sigma == "uniform":
        s = sigma_uniform(m, lo, hi, rng)
    elif sigma == "geometric":
        s = sigma_geometric(m)
    elif sigma == "clustered":
        s = sigma_clustered(m)
    elif sigma == "zero":
        s = np.zeros(m)
    else:
        raise ValueError(sigma)
    scale = 1.0 / np.sqrt(n)
    a = rng.standard_normal(m) * scale
    b = rng.standard_normal(n) * scale
    zeroed = np.zeros(0, dtype=np.int64)
    if zero_frac > 0.0:
        # Zero a fraction of the projected components p = U^T a (and q = V^T b).
        k = int(round(zero_frac * m))
        zeroed = np.sort(rng.choice(m, size=k, replace=False))
        p = rng.standard_normal(m) * scale
        p[zeroed] = 0.0
        a = U @ p
        if zero_q:
            q = rng.standard_normal(n) * scale
            q[zeroed] = 0.0
            b = V @ q
    meta = dict(m=m, n=n, sigma=sigma, seed=seed, zeroed=zeroed, zero_q=zero_q)
    return Problem(U=U, sigma=s, V=V, a=a, b=b, meta=meta)


def paper_random_square(n: int, lo: float, hi: float, seed: int):
    """A square matrix with i.i.d. U[lo, hi] entries and update vectors of the same law.

    Shape and value range follow the paper's numerical experiments (square
    random matrices with entries in a fixed interval); the factors are those of
    numpy's LAPACK SVD of that matrix.
    """
    rng = rng_for(seed)
    A = rng.uniform(lo, hi, size=(n, n))
    a = rng.uniform(lo, hi, size=n)
    b = rng.uniform(lo, hi, size=n)
    U, s, Vt = np.linalg.svd(A)
    return Problem(U=U, sigma=s, V=Vt.T.copy(), a=a, b=b, meta=dict(kind="paper_random", n=n, seed=seed)), A


def batched_sizes(count: int = 512, seed: int = 4, lo: int = 64, hi: int = 1024):
    """Sizes of the batched workload: m log-uniform in [lo, hi], n = m + U{0..m}."""
    rng = rng_for(seed)
    m = np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi), size=count))).astype(np.int64)
    n = m + rng.integers(0, m + 1)
    return m, n


def serving_sizes(count: int = 64, seed: int = 5, choices=(256, 1024, 2048, 4096, 8192)):
    rng = rng_for(seed)
    return rng.choice(np.asarray(choices), size=count)
