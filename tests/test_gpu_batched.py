"""GPU parity of the batched protected factorizations (one persistent
kernel, block and tile size 32) against the oracle, matrix by matrix."""
import numpy as np
import pytest

import oracle
from paper_2301_03166_amd import gen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h():
    from paper_2301_03166_amd import abft
    with abft.Handle() as hh:
        yield hh


def dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.asfortranarray(a)).cuda()
    return t if dtype is None else t.to(dtype)


SIZES = [1, 5, 31, 32, 33, 64, 100, 129, 200, 255, 300, 512]


@pytest.mark.parametrize("chol", [True, False])
def test_batched_fp64_matches_oracle(h, chol):
    mats0 = [gen.spd(n, 100 + n) if chol else gen.general(n, 100 + n) for n in SIZES]
    mats = [dev(a) for a in mats0]
    infos, ipivs, reps = h.batched(mats, chol)
    for q, (n, a0) in enumerate(zip(SIZES, mats0)):
        g = mats[q].cpu().numpy()
        o = a0.copy(order="F")
        if chol:
            oinfo, orep = oracle.potrf(o, 32)
            g, o = np.tril(g), np.tril(o)
        else:
            opiv, oinfo, orep = oracle.getrf(o, 32)
            assert np.array_equal(ipivs[q].cpu().numpy()[:n], opiv), n
        assert infos[q] == oinfo == 0, n
        assert np.linalg.norm(g - o) <= 1e-12 * np.linalg.norm(o), n
        assert reps[q].status == 0 and reps[q].flagged_tiles == 0, n
        assert reps[q].max_ratio < 0.5


@pytest.mark.parametrize("chol", [True, False])
def test_batched_exact_integer_cases(h, chol):
    sizes = [7, 32, 70, 160]
    made = [gen.chol_exact(n, n) if chol else gen.lu_exact(n, n) for n in sizes]
    mats = [dev(m[0]) for m in made]
    infos, ipivs, reps = h.batched(mats, chol)
    for q, n in enumerate(sizes):
        g = mats[q].cpu().numpy()
        if chol:
            assert np.array_equal(np.tril(g), made[q][1])
        else:
            assert np.array_equal(np.tril(g, -1) + np.eye(n), made[q][2])
            assert np.array_equal(np.triu(g), made[q][3])
        assert reps[q].max_ratio == 0.0 and reps[q].status == 0


def test_batched_fp32(h):
    import torch
    sizes = [40, 96, 257]
    mats0 = [gen.general(n, 7 + n) for n in sizes]
    mats = [dev(a, torch.float32) for a in mats0]
    infos, ipivs, reps = h.batched(mats, chol=False)
    for q, n in enumerate(sizes):
        g = mats[q].cpu().numpy().astype(np.float64)
        P = np.arange(n)
        for j, p in enumerate(ipivs[q].cpu().numpy()[:n]):
            P[j], P[p - 1] = P[p - 1], P[j]
        L, U = np.tril(g, -1) + np.eye(n), np.triu(g)
        assert np.linalg.norm(mats0[q][P] - L @ U) / np.linalg.norm(mats0[q]) < 1e-5
        assert reps[q].status == 0


@pytest.mark.parametrize("chol", [True, False])
def test_batched_faults_corrected(h, chol):
    sizes = [128, 200, 256, 96]
    mats0 = [gen.spd(n, 3 + n) if chol else gen.general(n, 3 + n) for n in sizes]
    faults = []
    for q, n in enumerate(sizes):
        f = gen.fault_plan("chol" if chol else "lu", n, 32, seed=77 + q)
        f["bit"] = 60 - q
        f["matrix"] = q
        faults.append(f)
    clean = [dev(a) for a in mats0]
    h.batched(clean, chol)
    mats = [dev(a) for a in mats0]
    infos, ipivs, reps = h.batched(mats, chol, faults=faults)
    for q, n in enumerate(sizes):
        f = faults[q]
        assert reps[q].corrected == 1, (q, reps[q].status)
        assert reps[q].events()[0] == (f["iter"], 1, f["row"], f["col"])
        o = mats0[q].copy(order="F")
        ff = dict(f)
        if chol:
            _, orep = oracle.potrf(o, 32, faults=[ff])
        else:
            _, _, orep = oracle.getrf(o, 32, faults=[ff])
        assert orep.corrected == 1 and orep.events()[0] == reps[q].events()[0]
        g, c = mats[q].cpu().numpy(), clean[q].cpu().numpy()
        if chol:
            g, c = np.tril(g), np.tril(c)
        assert np.max(np.abs(g - c)) <= 1e-12 * np.max(np.abs(c))


def test_batched_chol_diagonal_tile_flips(h):
    """Flips inside Cholesky diagonal tiles, one per matrix, including the far
    corner (nb-1, 0) of a tile; each is corrected as the oracle corrects it."""
    n = 128
    pos = [(95, 64), (87, 64), (70, 70), (63, 32)]
    mats0 = [gen.spd(n, 0) for _ in pos]
    faults = [{"iter": (p[1] // 32) - 1, "row": p[0], "col": p[1], "bit": 57, "matrix": q} for q, p in enumerate(pos)]
    clean = [dev(a) for a in mats0]
    h.batched(clean, True)
    mats = [dev(a) for a in mats0]
    infos, ipivs, reps = h.batched(mats, True, faults=faults)
    for q, f in enumerate(faults):
        o = mats0[q].copy(order="F")
        _, orep = oracle.potrf(o, 32, faults=[{k: v for k, v in f.items() if k != "matrix"}])
        assert orep.status == 1 and reps[q].status == 1, (q, orep.status, reps[q].status)
        assert reps[q].events()[0] == orep.events()[0] == (f["iter"], 1, f["row"], f["col"])
        g, c = np.tril(mats[q].cpu().numpy()), np.tril(clean[q].cpu().numpy())
        assert np.max(np.abs(g - c)) <= 1e-12 * np.max(np.abs(c))


@pytest.mark.parametrize("chol", [True, False])
def test_batched_graph_replay_matches_eager(h, chol):
    """Graph capture on first use, replays afterwards: every replay (with
    eager work and synchronizations between them) equals the eager call."""
    import torch
    sizes = [200, 37, 512, 96, 33, 260]
    mats0 = [gen.spd(n, 90 + n) if chol else gen.general(n, 90 + n) for n in sizes]
    ref = [dev(a) for a in mats0]
    infos0, ipivs0, reps0 = h.batched(ref, chol)
    work = [dev(a) for a in mats0]
    state = h.batched_args(work, chol)
    for rep in range(4):
        for q, a in enumerate(mats0):
            work[q].copy_(torch.from_numpy(np.asfortranarray(a)))
        infos, ipivs, reps = h.batched(work, chol, state=state, graph=True)
        torch.cuda.synchronize()
        scratch = torch.randn(256, 256, dtype=torch.float64, device="cuda") @ torch.randn(256, 256, dtype=torch.float64,
                                                                                            device="cuda")
        torch.cuda.synchronize()
        del scratch
        for q in range(len(sizes)):
            assert torch.equal(work[q], ref[q]), (rep, q)
            assert reps[q].status == 0
            if not chol:
                assert torch.equal(ipivs[q], ipivs0[q])
        assert np.array_equal(infos, infos0)


@pytest.mark.parametrize("chol", [True, False])
def test_batched_fp32_matches_oracle(h, chol):
    """Binary32 batched factors against the oracle's binary32 emulation
    (every operation rounded to binary32) on the same binary32 inputs:
    the same pivots, factors within binary32 rounding of each other, and a
    backward error within 2x of the oracle's."""
    import torch
    sizes = [1, 31, 33, 100, 200, 333, 512]
    mats0 = [(gen.spd(n, 200 + n) if chol else gen.general(n, 200 + n)).astype(np.float32).astype(np.float64)
             for n in sizes]
    mats = [dev(a, torch.float32) for a in mats0]
    infos, ipivs, reps = h.batched(mats, chol)
    u32 = 2.0 ** -24
    for q, (n, a0) in enumerate(zip(sizes, mats0)):
        g = mats[q].cpu().numpy().astype(np.float64)
        o = a0.copy(order="F")
        if chol:
            oinfo, orep = oracle.potrf(o, 32, prec=oracle.PR32)
            g, o = np.tril(g), np.tril(o)
            berr = lambda F: np.linalg.norm(a0 - F @ F.T) / np.linalg.norm(a0)
        else:
            opiv, oinfo, orep = oracle.getrf(o, 32, prec=oracle.PR32)
            gp = ipivs[q].cpu().numpy()[:n]
            assert np.array_equal(gp, opiv), n
            P = np.arange(n)
            for j, p in enumerate(gp):
                P[j], P[p - 1] = P[p - 1], P[j]
            berr = lambda F: np.linalg.norm(a0[P] - (np.tril(F, -1) + np.eye(n)) @ np.triu(F)) / np.linalg.norm(a0)
        assert infos[q] == oinfo == 0, n
        assert np.linalg.norm(g - o) <= 8 * n * u32 * np.linalg.norm(o), n
        assert berr(g) <= 2.0 * berr(o) + u32, (n, berr(g), berr(o))
        assert reps[q].status == 0 and orep.status == 0, n
