"""The side-stream schedule (panel checks, checksum carries and LU's left
interchanges beside the trailing-update product) against the one-stream
schedule of the same library (profiled calls keep one stream).  Each
element is computed by the same kernels in the same order either way, so
the factors must agree bitwise; a sampled residual of the LU factors at a
size above the small parity cases pins them to PA = LU as well."""
import numpy as np
import pytest

from paper_2301_03166_amd import gen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h():
    import torch
    from paper_2301_03166_amd import abft
    assert torch.cuda.is_available()
    with abft.Handle() as hh:
        yield hh


def dev(a):
    import torch
    return torch.from_numpy(np.asfortranarray(a)).cuda()


def clean(rep):
    return rep.status == 0 and rep.flagged_tiles == 0 and rep.panel_flags == 0


def test_getrf_side_stream_matches_one_stream(h):
    n, nb = 9472, 512
    A = gen.general(n, seed=9472)
    d1, d2 = dev(A), dev(A)
    ipiv1, info1, rep1 = h.getrf(d1, nb)
    ipiv2, info2, rep2 = h.getrf(d2, nb, profile=True)
    assert info1 == info2 == 0
    assert clean(rep1) and clean(rep2)
    F1, F2 = d1.cpu().numpy(), d2.cpu().numpy()
    assert np.array_equal(np.asarray(ipiv1.cpu()), np.asarray(ipiv2.cpu()))
    assert np.array_equal(F1, F2)
    # sampled columns of P A - L U
    piv = np.asarray(ipiv1.cpu()).astype(np.int64)
    p = np.arange(n)
    for j, q in enumerate(piv):
        q -= 1
        p[j], p[q] = p[q], p[j]
    L = np.tril(F1, -1) + np.eye(n)
    rng = np.random.default_rng(1)
    for j in rng.choice(n, 4, replace=False):
        u = np.triu(F1[:, j:j + 1], -j)[:, 0]  # column j of U: rows 0..j
        u[j + 1:] = 0.0
        r = A[p, j] - L @ u
        # componentwise scale: |PA - LU| <= gamma_n |L| |U| (gamma_n ~ 1e-12 here)
        assert np.linalg.norm(r) / np.linalg.norm(np.abs(L) @ np.abs(u)) < 1e-13


@pytest.mark.parametrize("kind", ["chol", "qr"])
def test_side_stream_matches_one_stream(h, kind):
    n, nb = 2600, 256
    A = gen.spd(n, seed=n) if kind == "chol" else gen.general(n, seed=n)
    d1, d2 = dev(A), dev(A)
    if kind == "chol":
        i1, r1 = h.potrf(d1, nb)
        i2, r2 = h.potrf(d2, nb, profile=True)
    else:
        t1, i1, r1 = h.geqrf(d1, nb)
        t2, i2, r2 = h.geqrf(d2, nb, profile=True)
        assert np.array_equal(t1.cpu().numpy(), t2.cpu().numpy())
    assert i1 == i2 == 0
    assert clean(r1) and clean(r2)
    assert r1.max_ratio == r2.max_ratio
    assert np.array_equal(d1.cpu().numpy(), d2.cpu().numpy())
