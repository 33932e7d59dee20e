"""abft_potrf_noalloc (built-in scratch, no workspace) against abft_potrf on
the same inputs: bitwise-equal factors and reports (the same kernels in the
same order), over two calls in a row with the second smaller than the first,
plus the size limit and the rejected profiling flag."""
import ctypes as C

import numpy as np
import pytest

import oracle
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


def test_noalloc_matches_potrf_two_calls(h):
    for n, nb, f in ((3000, 256, {"iter": 2, "row": 1700, "col": 900, "bit": 60}), (700, 128, None)):
        A = gen.spd(n, n)
        d1, d2 = dev(A), dev(A)
        faults = [f] if f else None
        i1, r1 = h.potrf(d1, nb, faults=faults)
        i2, r2 = h.potrf_noalloc(d2, nb, faults=faults)
        assert i1 == i2 == 0
        assert np.array_equal(np.tril(d1.cpu().numpy()), np.tril(d2.cpu().numpy()))
        assert np.array_equal(np.triu(d2.cpu().numpy(), 1), np.triu(A, 1))
        assert r1.status == r2.status and r1.events() == r2.events()
        assert r1.max_ratio == r2.max_ratio
        if f:
            assert r2.corrected == 1 and r2.events() == [(2, 1, 1700, 900)]
        else:
            assert r2.status == 0 and r2.flagged_tiles == 0
        # and the oracle agrees with both
        Ao = A.copy(order="F")
        oracle.potrf(Ao, nb, faults=faults)
        Lo = np.tril(Ao)
        assert np.linalg.norm(np.tril(d2.cpu().numpy()) - Lo) / np.linalg.norm(Lo) < 1e-14


def test_noalloc_limits(h):
    import torch
    from paper_2301_03166_amd import abft
    # beyond the built-in scratch: rejected before any work is enqueued
    A = torch.zeros((1, 1), dtype=torch.float64, device="cuda")
    opts, _ = abft.make_opts(512)
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    rc = abft.lib().abft_potrf_noalloc(h._h, 40000, A.data_ptr(), 40000, C.byref(opts), info.data_ptr(), None)
    assert rc == -101
    # profiling would create events: rejected
    opts, _ = abft.make_opts(64, profile=True)
    d = dev(gen.spd(64, 1))
    rc = abft.lib().abft_potrf_noalloc(h._h, 64, d.data_ptr(), 64, C.byref(opts), info.data_ptr(), None)
    assert rc == -102
