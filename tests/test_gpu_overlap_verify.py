"""Verification beside the next panel (ABFT_FLAG_OVERLAP_VERIFY) against the
serial schedule.  The same tiles are verified with the same sums and the
same kernels factor every panel, so the factors, the pivots / tau, the
report's counts, max_ratio and events must be equal bitwise; a planted flip
in either part of the trailing matrix (the next panel's block column, which
is verified first, or the tiles verified beside the panel) must be corrected
the same way.  The larger case is also held to the oracle."""
import numpy as np
import pytest

import oracle
from paper_2301_03166_amd import abft, gen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h():
    import torch
    assert torch.cuda.is_available()
    with abft.Handle() as hh:
        yield hh


def dev(a):
    import torch
    return torch.from_numpy(np.asfortranarray(a)).cuda()


def run(h, kind, A, nb, **kw):
    d = dev(A)
    if kind == "chol":
        info, rep = h.potrf(d, nb, **kw)
        aux = None
    elif kind == "lu":
        aux, info, rep = h.getrf(d, nb, **kw)
        aux = aux.cpu().numpy()
    else:
        aux, info, rep = h.geqrf(d, nb, **kw)
        aux = aux.cpu().numpy()
    F = d.cpu().numpy()
    return (np.tril(F) if kind == "chol" else F), aux, info, rep


def matrix(kind, n, seed):
    return gen.spd(n, seed) if kind == "chol" else gen.general(n, seed)


def same(a, b):
    Fa, xa, ia, ra = a
    Fb, xb, ib, rb = b
    assert ia == ib
    assert (ra.status, ra.flagged_tiles, ra.corrected, ra.checksum_repaired, ra.uncorrectable, ra.panel_flags,
            ra.first_flag_iter) == (rb.status, rb.flagged_tiles, rb.corrected, rb.checksum_repaired,
                                    rb.uncorrectable, rb.panel_flags, rb.first_flag_iter)
    assert ra.max_ratio == rb.max_ratio
    assert ra.events() == rb.events()
    if xa is not None:
        assert np.array_equal(xa, xb)
    assert np.array_equal(Fa, Fb)


@pytest.mark.parametrize("kind", ["chol", "lu", "qr"])
@pytest.mark.parametrize("n,nb", [(3000, 256), (2600, 384), (1000, 128), (700, 512), (1537, 512)])
def test_overlap_matches_serial(h, kind, n, nb):
    A = matrix(kind, n, n + nb)
    a = run(h, kind, A, nb, overlap=True)
    b = run(h, kind, A, nb, overlap=False)
    assert a[2] == 0 and a[3].status == 0 and a[3].flagged_tiles == 0
    same(a, b)


@pytest.mark.parametrize("kind", ["chol", "lu", "qr"])
@pytest.mark.parametrize("where", ["next_panel", "beside"])
def test_overlap_flip_corrected_like_serial(h, kind, where):
    """One flip after the update of iteration 1: in the next panel's block
    column (verified first on the caller's stream) or three tile-columns to
    its right (verified on the restricted stream beside the panel)."""
    n, nb = 2048, 256
    A = matrix(kind, n, 5)
    col = 2 * nb + 17 if where == "next_panel" else 5 * nb + 40
    f = {"iter": 1, "target": 0, "row": 6 * nb + 3, "col": col, "bit": 55}
    a = run(h, kind, A, nb, faults=[f], overlap=True)
    b = run(h, kind, A, nb, faults=[f], overlap=False)
    c = run(h, kind, A, nb, overlap=False)
    same(a, b)
    assert a[3].corrected == 1 and a[3].uncorrectable == 0
    # the corrected element is recomputed from its checksum: equal to the
    # clean run's up to rounding, and so is everything computed from it
    assert np.linalg.norm(a[0] - c[0]) / np.linalg.norm(c[0]) < 1e-12


def test_overlap_levels_match_serial(h):
    """Per-iteration levels rising mid-factorization: the encode pass of a
    newly protected stretch waits for the tiles verified beside the panel."""
    n, nb = 2048, 256
    levels = [abft.PROTECT_NONE, abft.PROTECT_SINGLE, abft.PROTECT_SINGLE, abft.PROTECT_FULL, abft.PROTECT_FULL,
              abft.PROTECT_NONE, abft.PROTECT_FULL, abft.PROTECT_FULL]
    for kind in ("chol", "lu", "qr"):
        A = matrix(kind, n, 9)
        same(run(h, kind, A, nb, levels=levels, overlap=True), run(h, kind, A, nb, levels=levels, overlap=False))


@pytest.mark.timeout(600)
@pytest.mark.parametrize("kind", ["chol", "lu", "qr"])
def test_overlap_large_vs_oracle(h, kind):
    """n = 6144, nb = 512: cooperative leaves of many workgroups beside the
    restricted stream's verification; bitwise equal to the serial schedule
    and within rounding of the oracle."""
    n, nb = 6144, 512
    A = matrix(kind, n, 31)
    a = run(h, kind, A, nb, overlap=True)
    same(a, run(h, kind, A, nb, overlap=False))
    F, aux, info, rep = a
    assert info == 0 and rep.status == 0
    O = A.copy(order="F")
    if kind == "chol":
        oracle.potrf(O, nb)
        O = np.tril(O)
        assert np.linalg.norm(F - O) / np.linalg.norm(O) < 1e-13
    elif kind == "lu":
        oaux, _, _ = oracle.getrf(O, nb)
        assert np.array_equal(aux, oaux)
        assert np.linalg.norm(F - O) / np.linalg.norm(O) < 1e-12
    else:
        oaux, _ = oracle.geqrf(O, nb)
        assert np.max(np.abs(aux - oaux)) < 1e-12
        assert np.linalg.norm(np.triu(F) - np.triu(O)) / np.linalg.norm(np.triu(O)) < 1e-12


@pytest.mark.parametrize("kind", ["chol", "lu", "qr"])
def test_overlap_on_a_caller_stream(h, kind):
    """A call made on a non-default stream (no detour through the handle's
    own stream) orders the restricted stream's work after and before that
    stream: same results as the serial schedule on the default stream."""
    import torch
    n, nb = 2600, 256
    A = matrix(kind, n, 41)
    ref = run(h, kind, A, nb, overlap=False)
    st = torch.cuda.Stream()
    d = dev(A)
    st.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(st):
        if kind == "chol":
            info, rep = h.potrf(d, nb, overlap=True)
            aux = None
        elif kind == "lu":
            aux, info, rep = h.getrf(d, nb, overlap=True)
        else:
            aux, info, rep = h.geqrf(d, nb, overlap=True)
    torch.cuda.current_stream().wait_stream(st)
    torch.cuda.synchronize()
    F = d.cpu().numpy()
    got = ((np.tril(F) if kind == "chol" else F), None if aux is None else aux.cpu().numpy(), info, rep)
    same(got, ref)
