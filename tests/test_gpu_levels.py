"""GPU parity of the per-iteration protection levels (single-side and full
checksums, adaptive switching) and of the 1D correction (a whole row or
column of a tile rebuilt from the other side's checksums after a fault in an
operand of the trailing update), against the oracle on the same inputs and
fault plans."""
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


def gpu(h, kind, A, nb, **kw):
    dA = dev(A)
    if kind == "chol":
        info, rep = h.potrf(dA, nb, **kw)
    elif kind == "lu":
        ipiv, info, rep = h.getrf(dA, nb, **kw)
    else:
        tau, info, rep = h.geqrf(dA, nb, **kw)
    F = dA.cpu().numpy()
    return (np.tril(F) if kind == "chol" else F), rep


def orc(kind, A, nb, **kw):
    Ao = A.copy(order="F")
    if kind == "chol":
        info, rep = oracle.potrf(Ao, nb, **kw)
    elif kind == "lu":
        ipiv, info, rep = oracle.getrf(Ao, nb, **kw)
    else:
        tau, rep = oracle.geqrf(Ao, nb, **kw)
    return (np.tril(Ao) if kind == "chol" else Ao), rep


def matrix(kind, n, seed):
    return gen.spd(n, seed) if kind == "chol" else gen.general(n, seed)


@pytest.mark.parametrize("kind", ["chol", "lu", "qr"])
def test_uniform_levels(h, kind):
    n, nb = 700, 128
    N = -(-n // nb)
    A = matrix(kind, n, 3)
    full, rf = gpu(h, kind, A, nb)
    lfull, rlf = gpu(h, kind, A, nb, levels=[2] * N)
    none, rn = gpu(h, kind, A, nb, protect=False)
    lnone, rln = gpu(h, kind, A, nb, levels=[0] * N)
    single, rs = gpu(h, kind, A, nb, protect=1)
    assert np.array_equal(full, lfull) and rf.max_ratio == rlf.max_ratio and rf.status == rlf.status == 0
    assert np.array_equal(none, lnone) and rn.status == rln.status == 0 and rln.max_ratio == 0.0
    assert np.array_equal(single, full) and rs.status == 0 and rs.flagged_tiles == 0 and rs.max_ratio < 0.5
    O, ro = orc(kind, A, nb, protect=oracle.SINGLE)
    assert ro.status == 0
    assert np.linalg.norm(single - O) / np.linalg.norm(O) < 1e-12


@pytest.mark.parametrize("kind", ["chol", "lu"])
def test_adaptive_levels_exact(h, kind):
    n, nb = 192, 32
    levels = [0, 0, 1, 1, 2, 2]
    if kind == "chol":
        A, L0 = gen.chol_exact(n, seed=8)
        F, rep = gpu(h, kind, A, nb, levels=levels)
        assert np.array_equal(F, L0)
    else:
        A, P, L0, U0 = gen.lu_exact(n, seed=8)
        F, rep = gpu(h, kind, A, nb, levels=levels)
        assert np.array_equal(np.tril(F, -1) + np.eye(n), L0) and np.array_equal(np.triu(F), U0)
    assert rep.status == 0 and rep.max_ratio == 0.0


@pytest.mark.parametrize("kind", ["chol", "lu", "qr"])
@pytest.mark.parametrize("lev", [0, 1, 2])
def test_adaptive_levels_flip_matches_oracle(h, kind, lev):
    n, nb = 192, 32
    A = matrix(kind, n, 4)
    f = gen.fault_plan(kind, n, nb, seed=41, iters=2)
    f["bit"] = 61
    levels = [2, 2, lev, 2, 2, 2]
    G, rep = gpu(h, kind, A, nb, levels=levels, faults=[f])
    O, orep = orc(kind, A, nb, levels=levels, faults=[f])
    assert rep.status == orep.status and rep.events() == sorted(orep.events())
    if lev:
        assert rep.events() == [(2, 1, f["row"], f["col"])]
        assert np.linalg.norm(G - O) / np.linalg.norm(O) < 1e-12
    else:
        assert rep.status == 0 and rep.flagged_tiles == 0


def lu_exact_operand(side):
    n, nb = 160, 32
    A, P, L0, U0 = gen.lu_exact(n, seed=5)
    if side == "L":
        i, j = next((i, j) for i in range(64, n) for j in range(32, 64) if abs(L0[i, j]) > 0)
    else:
        i, j = next((i, j) for i in range(32, 64) for j in range(64, n) if abs(U0[i, j]) > 0)
    return A, L0, U0, {"iter": 1, "target": 3 if side == "L" else 4, "row": i, "col": j, "bit": 52}, n, nb


@pytest.mark.parametrize("side", ["L", "U"])
def test_lu_operand_fault_rebuilt_exactly(h, side):
    A, L0, U0, f, n, nb = lu_exact_operand(side)
    F, rep = gpu(h, "lu", A, nb, faults=[f])
    O, orep = orc("lu", A, nb, faults=[f])
    assert np.array_equal(np.tril(F, -1) + np.eye(n), L0) and np.array_equal(np.triu(F), U0)
    assert rep.status == orep.status == 1 and rep.corrected == orep.corrected == 3
    assert rep.events() == sorted(orep.events())
    assert {e[1] for e in rep.events()} == {5 if side == "L" else 6}


@pytest.mark.parametrize("side", ["L", "U"])
def test_lu_operand_fault_single_side(h, side):
    A, L0, U0, f, n, nb = lu_exact_operand(side)
    F, rep = gpu(h, "lu", A, nb, faults=[f], protect=1)
    O, orep = orc("lu", A, nb, faults=[f], protect=oracle.SINGLE)
    assert rep.status == orep.status and rep.status & 4
    assert rep.events() == sorted(orep.events())


@pytest.mark.parametrize("target,row,col", [(3, 100, 40), (3, 40, 35), (4, 5, 100)])
def test_qr_operand_fault_matches_oracle(h, target, row, col):
    n, nb = 160, 32
    A = gen.general(n, 7)
    clean, _ = gpu(h, "qr", A, nb)
    f = {"iter": 1, "target": target, "row": row, "col": col, "bit": 60}
    G, rep = gpu(h, "qr", A, nb, faults=[f])
    O, orep = orc("qr", A, nb, faults=[f])
    assert rep.status == orep.status == 1
    assert rep.events() == sorted(orep.events())
    assert np.max(np.abs(G - clean)) <= 1e-12 * np.max(np.abs(clean))


def test_chol_operand_fault_cross_matches_oracle(h):
    n, nb = 160, 32
    S, L0 = gen.chol_exact(n, seed=3)
    f = {"iter": 1, "target": 3, "row": 100, "col": 40, "bit": 62}
    dS = dev(S)
    info, rep = h.potrf(dS, nb, faults=[f])
    Ao = S.copy(order="F")
    oinfo, orep = oracle.potrf(Ao, nb, faults=[f])
    # the cross through the diagonal tile cannot be rebuilt (a wrong row and a
    # wrong column in one tile), the tile stays wrong and the factorization
    # breaks down in the panel that holds it; the oracle stops there, the GPU
    # completes the factorization on NaN data, so the reports are compared up
    # to the breakdown: corrections, the uncorrectable tile and their events
    assert info == oinfo == 101
    last = (oinfo - 1) // nb
    assert rep.status & 5 == orep.status & 5 == 5
    assert [e for e in rep.events() if e[0] < last] == sorted(e for e in orep.events() if e[0] < last)


@pytest.mark.parametrize("kind,target", [("lu", 3), ("lu", 4), ("qr", 3), ("qr", 4)])
def test_operand_fault_random_larger(h, kind, target):
    """A 1D error across several 128-wide tiles of a random matrix: the same
    rebuilt lines as the oracle, and the clean factors back to rounding."""
    n, nb = 1000, 128
    A = gen.general(n, 11)
    k = 2
    c0, c1 = k * nb, (k + 1) * nb
    if target == 3:
        f = {"iter": k, "target": 3, "row": 700, "col": c0 + 17, "bit": 60}
    elif kind == "lu":
        f = {"iter": k, "target": 4, "row": c0 + 9, "col": 777, "bit": 60}
    else:
        f = {"iter": k, "target": 4, "row": 9, "col": 777, "bit": 60}
    clean, _ = gpu(h, kind, A, nb)
    G, rep = gpu(h, kind, A, nb, faults=[f])
    O, orep = orc(kind, A, nb, faults=[f])
    assert rep.status == orep.status == 1
    assert rep.events() == sorted(orep.events())
    assert len(rep.events()) >= 4
    assert np.max(np.abs(G - clean)) <= 1e-11 * np.max(np.abs(clean))
