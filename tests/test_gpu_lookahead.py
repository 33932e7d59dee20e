"""The look-ahead schedule (the next panel factored on a panel stream with
its own compute units while the rest of the trailing matrix is updated and
verified on the update stream) against the one-stream schedule and the
oracle.  Where both schedules give the cooperative leaves the same shape
(the panel fits the workgroups each stream may use), every element is
computed by the same kernels in the same order, so the factors agree
bitwise; beyond that the panel stream's narrower leaves change rounding
only, checked against the oracle."""
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


def clean(rep):
    return rep.status == 0 and rep.flagged_tiles == 0 and rep.panel_flags == 0


def run(h, kind, A, nb, **kw):
    d = dev(A)
    if kind == "chol":
        info, rep = h.potrf(d, nb, **kw)
        return np.tril(d.cpu().numpy()), None, info, rep
    if kind == "lu":
        aux, info, rep = h.getrf(d, nb, **kw)
    else:
        aux, info, rep = h.geqrf(d, nb, **kw)
    return d.cpu().numpy(), aux.cpu().numpy(), info, rep


@pytest.mark.parametrize("kind", ["chol", "lu", "qr"])
@pytest.mark.parametrize("n,nb,la", [(3000, 256, 32), (2600, 384, 16), (1000, 128, 8), (700, 512, 32)])
def test_lookahead_matches_one_stream(h, kind, n, nb, la):
    A = gen.spd(n, n + nb) if kind == "chol" else gen.general(n, seed=n + nb)
    F1, a1, i1, r1 = run(h, kind, A, nb, lookahead=la)
    F2, a2, i2, r2 = run(h, kind, A, nb)
    assert i1 == i2 == 0 and clean(r1) and clean(r2)
    assert r1.max_ratio == r2.max_ratio
    assert r1.events() == r2.events()
    if a1 is not None:
        assert np.array_equal(a1, a2)
    assert np.array_equal(F1, F2)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("kind", ["chol", "lu", "qr"])
def test_lookahead_large_vs_oracle(h, kind):
    """n = 9472, nb = 512 with a 64-unit panel stream: the first LU / QR
    panels need 32-wide leaves spread over the panel stream's workgroups
    (the Cholesky panel has no cooperative leaf and keeps its shape)."""
    n, nb = 9472, 512
    A = gen.spd(n, 77) if kind == "chol" else gen.general(n, seed=77)
    F, aux, info, rep = run(h, kind, A, nb, lookahead=64)
    assert info == 0 and clean(rep)
    O = A.copy(order="F")
    if kind == "chol":
        oracle.potrf(O, nb)
        O = np.tril(O)
        assert np.linalg.norm(F - O) / np.linalg.norm(O) < 1e-13
        assert np.array_equal(F, run(h, kind, A, nb)[0])
    elif kind == "lu":
        oaux, _, orep = oracle.getrf(O, nb)
        assert np.array_equal(aux, oaux)
        assert np.linalg.norm(F - O) / np.linalg.norm(O) < 1e-12
    else:
        oaux, orep = oracle.geqrf(O, nb)
        assert np.max(np.abs(aux - oaux)) < 1e-12
        assert np.linalg.norm(np.triu(F) - np.triu(O)) / np.linalg.norm(np.triu(O)) < 1e-12


@pytest.mark.parametrize("chol", [False, True])
def test_lookahead_mixed_precision_matches_one_stream(h, chol):
    import torch
    n, nb = 2048, 256
    A, s, V = gen.mp_matrix(n, 1e2, seed=21)
    b = gen.rhs(n, seed=24)
    x1, ir1, rep1 = h.gesv_mp(dev(A), torch.from_numpy(b).cuda(), 3, nb=nb, chol=chol, lookahead=32)
    x2, ir2, rep2 = h.gesv_mp(dev(A), torch.from_numpy(b).cuda(), 3, nb=nb, chol=chol)
    assert ir1.converged and ir2.converged and ir1.iters == ir2.iters
    assert torch.equal(x1, x2)
    assert rep1.status == rep2.status == 0


@pytest.mark.parametrize("kind", ["chol", "lu", "qr"])
def test_product_tile_depth_bitwise(h, kind):
    """The trailing-update product with 32-deep K tiles against the default
    16-deep ones: the same MFMA products in the same K order, so the factors
    and reports are equal bitwise."""
    n, nb = 1800, 256
    A = gen.spd(n, 5) if kind == "chol" else gen.general(n, seed=5)
    outs = []
    for bk in (0, 32):
        d = dev(A)
        if kind == "chol":
            info, rep = h.potrf(d, nb, tmu_bk=bk)
            aux = None
        elif kind == "lu":
            aux, info, rep = h.getrf(d, nb, tmu_bk=bk)
        else:
            aux, info, rep = h.geqrf(d, nb, tmu_bk=bk)
        assert info == 0 and clean(rep)
        outs.append((d.cpu().numpy(), None if aux is None else aux.cpu().numpy(), rep.max_ratio))
    assert np.array_equal(outs[0][0], outs[1][0])
    if kind != "chol":
        assert np.array_equal(outs[0][1], outs[1][1])
    assert outs[0][2] == outs[1][2]
