"""The backward-error check of the benchmark and the full-size tests (CPU,
with LAPACK factors from scipy): it equals the dense residual formed with
numpy, sees a planted error of known size, and the orthogonality probe of
the QR factors reports rounding level (and a planted loss of orthogonality
within the probe estimator's spread, a factor of about 2 with 8 probes)."""
import numpy as np
import pytest
import scipy.linalg as sl
import torch

import bench
from paper_2301_03166_amd import gen


def col(a):
    return torch.from_numpy(np.asfortranarray(a))


def qr_q(F, tau):
    n = F.shape[0]
    Q = np.eye(n)
    for j in range(n - 1, -1, -1):
        v = np.zeros(n)
        v[j] = 1.0
        v[j + 1:] = F[j + 1:, j]
        Q -= tau[j] * np.outer(v, v @ Q)
    return Q


def dense_error(kind, A, F, aux):
    n = A.shape[0]
    if kind == "chol":
        L = np.tril(F)
        E = A - L @ L.T
    elif kind == "lu":
        p = bench.ipiv_perm(aux)
        E = A[p] - (np.tril(F, -1) + np.eye(n)) @ np.triu(F)
    else:
        E = qr_q(F, aux).T @ A - np.triu(F)
    return np.linalg.norm(E) / np.linalg.norm(A)


@pytest.mark.parametrize("kind", ["chol", "lu", "qr"])
def test_backward_error_matches_dense_residual(kind):
    n = 300
    A = gen.spd(n, 1) if kind == "chol" else gen.general(n, 2)
    if kind == "chol":
        F, aux = np.tril(sl.cholesky(A, lower=True)), None
    elif kind == "lu":
        F, piv = sl.lu_factor(A)
        aux = (piv + 1).astype(np.int32)
    else:
        F, aux, _, _ = sl.lapack.dgeqrf(A)
    for planted in (0.0, 1e-7):
        F2 = np.array(F, order="F")
        F2[200, 100 if kind != "qr" else 250] += planted * np.linalg.norm(A)
        be, orth = bench.backward_error(kind, col(A), col(F2), None if aux is None else torch.from_numpy(aux))
        ref = dense_error(kind, A, F2, aux)
        if planted:  # the planted error dominates: the two evaluations agree
            assert abs(be - ref) <= 0.05 * ref and be > 0.5e-7
        else:  # rounding level either way (the orders of evaluation differ)
            assert be < 3e-15 and ref < 3e-15
        if kind == "qr":
            Q = qr_q(F2, aux)
            exact = np.linalg.norm(np.eye(n) - Q.T @ Q) / np.sqrt(n)
            assert orth < 2.5 * exact + 1e-15 and orth > exact / 2.5


def test_ipiv_perm_matches_sequential_swaps():
    ipiv = np.array([3, 3, 4, 4], dtype=np.int32)
    A = np.arange(16.0).reshape(4, 4)
    B = A.copy()
    for j, q in enumerate(ipiv - 1):
        B[[j, q]] = B[[q, j]]
    assert np.array_equal(A[bench.ipiv_perm(ipiv)], B)
