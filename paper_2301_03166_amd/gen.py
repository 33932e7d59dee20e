"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds random-matrix construction only; none of the factorization,
checksum or refinement arithmetic lives here.  Host generators use numpy's
PCG64 and return Fortran-ordered float64 arrays; the ``*_torch`` variants build
the same distributions directly in device memory for sizes where host
generation would take minutes (their random streams differ from the host
ones, so a test always hands one and the same buffer to both sides).

Distributions (one per workload of the evaluation):
  * SPD:      A = G G^T / n + n I, G_ij ~ N(0,1)
  * general:  A_ij ~ U(-1, 1)
  * MP solve: A = H_1 ... H_8 diag(s) H_8 ... H_1, s_i = kappa^(-i/(n-1)),
              H_j = I - 2 v v^T / (v^T v), v ~ N(0,1)^n; b ~ U(-1, 1)
  * batched:  integer sizes uniform on [lo, hi], one seed per matrix
"""
from __future__ import annotations

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def spd(n: int, seed: int) -> np.ndarray:
    g = rng(seed).standard_normal((n, n))
    a = g @ g.T
    a /= n
    a[np.diag_indices(n)] += n
    return np.asfortranarray(a)


def general(n: int, seed: int) -> np.ndarray:
    return np.asfortranarray(rng(seed).uniform(-1.0, 1.0, (n, n)))


def rhs(n: int, seed: int) -> np.ndarray:
    return rng(seed).uniform(-1.0, 1.0, n)


def reflectors(n: int, seed: int, count: int = 8) -> np.ndarray:
    return rng(seed).standard_normal((count, n))


def mp_matrix(n: int, kappa: float, seed: int) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """A = Q diag(s) Q^T with Q = H_1 ... H_8; returns (A, s, V) with V the reflector vectors."""
    s = kappa ** (-np.arange(n) / max(n - 1, 1))
    V = reflectors(n, seed)
    a = np.diag(s)
    for v in V[::-1]:
        t = 2.0 / (v @ v)
        av = a @ v
        vav = v @ av
        # H a H = a - t v (v^T a) - t (a v) v^T + t^2 (v^T a v) v v^T   (a symmetric)
        a = a - t * np.outer(v, av) - t * np.outer(av, v) + (t * t * vav) * np.outer(v, v)
    return np.asfortranarray(a), s, V


def mp_exact_solution(b: np.ndarray, s: np.ndarray, V: np.ndarray) -> np.ndarray:
    """x* = Q diag(1/s) Q^T b applied reflector by reflector (closed form of the MP generator)."""
    y = np.array(b, dtype=np.float64)
    for v in V:        # Q^T = H_8 ... H_1, so H_1 acts first
        y = y - (2.0 / (v @ v)) * v * (v @ y)
    y = y / s
    for v in V[::-1]:  # Q = H_1 ... H_8, so H_8 acts first
        y = y - (2.0 / (v @ v)) * v * (v @ y)
    return y


def chol_exact(n: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """A = L0 L0^T with L0 lower, diagonal in {1,2,4}, off-diagonal integers in [-2, 2]."""
    r = rng(seed)
    L = np.tril(r.integers(-2, 3, (n, n)).astype(np.float64), -1)
    L[np.diag_indices(n)] = r.choice([1.0, 2.0, 4.0], n)
    return np.asfortranarray(L @ L.T), np.asfortranarray(L)


def lu_exact(n: int, seed: int) -> tuple[np.ndarray, np.ndarray, np.ndarray, np.ndarray]:
    """A = P0 L0 U0 with small dyadic entries (|l| < 1, so pivots are unique)."""
    r = rng(seed)
    L = np.tril(r.choice([0.0, 0.25, -0.25, 0.5, -0.5], (n, n)), -1)
    L[np.diag_indices(n)] = 1.0
    U = np.triu(r.integers(-3, 4, (n, n)).astype(np.float64), 1)
    U[np.diag_indices(n)] = r.choice([1.0, -1.0, 2.0, -2.0, 4.0, -4.0], n)
    perm = r.permutation(n)
    P = np.eye(n)[perm]
    return np.asfortranarray(P @ L @ U), P, L, U


def lu_tie(n: int, seed: int) -> np.ndarray:
    """A = L0 U0 with L0 entries in {-1, 0, 1}: every column has ties for the pivot."""
    r = rng(seed)
    L = np.tril(r.choice([-1.0, 0.0, 1.0], (n, n)), -1)
    L[np.diag_indices(n)] = 1.0
    U = np.triu(r.integers(-3, 4, (n, n)).astype(np.float64), 1)
    U[np.diag_indices(n)] = r.choice([1.0, -1.0, 2.0, -2.0], n)
    return np.asfortranarray(L @ U)


def batch_sizes(count: int, lo: int, hi: int, seed: int) -> np.ndarray:
    return rng(seed).integers(lo, hi + 1, count).astype(np.int32)


def batch_seeds(count: int, base: int) -> list[int]:
    ss = np.random.SeedSequence(base).spawn(count)
    return [int(s.generate_state(1)[0]) for s in ss]


def fault_plan(kind: str, n: int, nb: int, seed: int, iters: int | None = None) -> dict:
    """One single-bit flip after the trailing update of a uniformly drawn iteration,
    at a uniformly drawn stored element of the trailing matrix it produced."""
    r = rng(seed)
    N = -(-n // nb)
    if N < 2:
        raise ValueError("no trailing matrix")
    k = int(r.integers(0, N - 1)) if iters is None else int(iters)
    c1 = (k + 1) * nb
    r0 = k * nb if kind == "qr" else c1
    while True:
        i = int(r.integers(r0, n))
        j = int(r.integers(c1, n))
        if kind != "chol" or i >= j:
            break
    return {"iter": k, "row": i, "col": j, "bit": int(r.integers(0, 64)), "target": 0}


# ---------------------------------------------------------------- device --
def spd_torch(n: int, seed: int, device, chunk: int = 4096):
    import torch
    g = torch.Generator(device=device).manual_seed(seed)
    G = torch.randn((n, n), generator=g, dtype=torch.float64, device=device)
    a = torch.empty((n, n), dtype=torch.float64, device=device)
    for c in range(0, n, chunk):
        a[:, c:c + chunk] = G @ G[c:c + chunk].T
    del G
    a /= n
    a.diagonal().add_(n)
    return a  # symmetric, so row- and column-major storage coincide


def general_torch(n: int, seed: int, device):
    import torch
    g = torch.Generator(device=device).manual_seed(seed)
    return torch.rand((n, n), generator=g, dtype=torch.float64, device=device).mul_(2.0).sub_(1.0)


def mp_torch(n: int, kappa: float, seed: int, device):
    """The mixed-precision test matrix of ``mp_matrix`` built in device memory
    (same s and reflectors, so the closed-form solution of ``mp_exact_solution``
    applies); returns (A, s, V) with A a torch tensor and s, V numpy arrays."""
    import torch
    s = kappa ** (-np.arange(n) / max(n - 1, 1))
    V = reflectors(n, seed)
    a = torch.diag(torch.from_numpy(s).to(device))
    for v in V[::-1]:
        vt = torch.from_numpy(v).to(device)
        t = 2.0 / float(v @ v)
        av = a @ vt
        vav = float(vt @ av)
        a.addr_(vt, av, alpha=-t)
        a.addr_(av, vt, alpha=-t)
        a.addr_(vt, vt, alpha=t * t * vav)
    return a, s, V  # symmetric: row- and column-major storage coincide


def batch_torch(sizes, seeds, kind: str, device, dtype=None):
    """Matrices of the given orders packed one after another in one flat
    device buffer (column-major each); SPD for kind == "chol" (G G^T/n + n I),
    U(-1, 1) otherwise.  Returns (flat, views)."""
    import torch
    dtype = dtype or torch.float64
    offs = np.concatenate([[0], np.cumsum(np.asarray(sizes, dtype=np.int64) ** 2)])
    flat = torch.empty(int(offs[-1]), dtype=dtype, device=device)
    views = []
    for q, (n, sd) in enumerate(zip(sizes, seeds)):
        n = int(n)
        g = torch.Generator(device=device).manual_seed(int(sd))
        if kind == "chol":
            G = torch.randn((n, n), generator=g, dtype=torch.float64, device=device)
            m = G @ G.T / n
            m.diagonal().add_(n)
        else:
            m = torch.rand((n, n), generator=g, dtype=torch.float64, device=device).mul_(2.0).sub_(1.0)
        v = torch.as_strided(flat, (n, n), (1, n), int(offs[q]))
        v.copy_(m.t())
        views.append(v)
    return flat, views
