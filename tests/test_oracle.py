"""Pins for the CPU oracle: every check compares it with something other than
itself -- exact integer/dyadic constructions, brute-force unblocked versions,
closed forms, LAPACK (scipy) as a third-party cross-check, and the ABFT
invariants.  None of these tests needs a GPU."""
import numpy as np
import pytest
import scipy.linalg as sla
from scipy.linalg import lapack

import oracle
from paper_2301_03166_amd import gen

U64 = 2.0 ** -53


def lower(a):
    return np.tril(a)


def unit_lower(a):
    return np.tril(a, -1) + np.eye(a.shape[0])


def perm_from_ipiv(ipiv, n):
    p = np.arange(n)
    for j, q in enumerate(ipiv):
        q -= 1
        p[j], p[q] = p[q], p[j]
    return p


# ------------------------------------------------------------------ Cholesky
@pytest.mark.parametrize("n,nb", [(1, 1), (7, 3), (16, 4), (33, 8), (50, 16), (64, 64), (40, 128)])
def test_potrf_exact_integer(n, nb):
    """A = L0 L0^T with small integers: every intermediate is an exact integer,
    so the blocked factor must equal L0 bit for bit, and every carried checksum
    must equal the recomputed one exactly (d = 0 at every verify)."""
    A, L0 = gen.chol_exact(n, seed=n * 31 + nb)
    info, rep = oracle.potrf(A, nb)
    assert info == 0
    assert np.array_equal(lower(A), L0)
    assert rep.flagged_tiles == 0 and rep.panel_flags == 0 and rep.status == 0
    assert rep.max_ratio == 0.0


def test_potrf_diag_perfect_squares():
    d = np.array([1.0, 4.0, 9.0, 16.0, 25.0, 36.0])
    A = np.asfortranarray(np.diag(d))
    info, _ = oracle.potrf(A, 4)
    assert info == 0 and np.array_equal(np.diag(A), np.sqrt(d))


@pytest.mark.parametrize("n,nb", [(17, 5), (48, 16), (64, 7)])
def test_potrf_blocked_vs_unblocked(n, nb):
    A0 = gen.spd(n, seed=n + nb)
    A1, A2 = A0.copy(order="F"), A0.copy(order="F")
    assert oracle.potrf(A1, nb)[0] == 0
    assert oracle.potrf_unb(A2) == 0
    assert np.max(np.abs(lower(A1) - lower(A2))) <= 64 * n * U64 * np.max(np.abs(lower(A2)))


def test_potrf_vs_lapack_and_backward_error():
    n, nb = 96, 32
    A0 = gen.spd(n, seed=5)
    A = A0.copy(order="F")
    assert oracle.potrf(A, nb)[0] == 0
    L = lower(A)
    ref, info = lapack.dpotrf(A0, lower=1)
    assert info == 0
    assert np.linalg.norm(L - np.tril(ref)) <= 16 * n * U64 * np.linalg.norm(np.tril(ref))
    assert np.linalg.norm(A0 - L @ L.T) / np.linalg.norm(A0) < 1e-15


def test_potrf_not_spd_info():
    A, _ = gen.chol_exact(12, seed=3)
    A[7, 7] = -1.0  # leading minor of order 8 is no longer positive definite
    A = np.asfortranarray(A)
    info, _ = oracle.potrf(A, 4)
    assert info == 8


# ------------------------------------------------------------------------ LU
@pytest.mark.parametrize("n,nb", [(1, 1), (9, 4), (24, 8), (37, 10), (64, 16), (30, 64)])
def test_getrf_exact_dyadic(n, nb):
    """A = P0 L0 U0 with |l| < 1 and dyadic values: partial pivoting must
    recover P0, L0 and U0 exactly, for any summation order."""
    A, P, L0, U0 = gen.lu_exact(n, seed=7 * n + nb)
    ipiv, info, rep = oracle.getrf(A, nb)
    assert info == 0
    assert np.array_equal(unit_lower(A), L0)
    assert np.array_equal(np.triu(A), U0)
    perm = perm_from_ipiv(ipiv, n)
    assert np.array_equal(np.eye(n)[perm] @ P, np.eye(n))  # P A = L U  with  P = P0^T
    assert rep.flagged_tiles == 0 and rep.panel_flags == 0 and rep.max_ratio == 0.0


def test_getrf_first_index_tie_break():
    """L0 entries in {-1,0,1}: each pivot column has ties; only a first-index
    rule keeps the identity permutation."""
    n = 20
    A = gen.lu_tie(n, seed=11)
    ipiv, info, _ = oracle.getrf(A, 8)
    assert info == 0
    assert np.array_equal(ipiv, np.arange(1, n + 1))


def test_getrf_singular_column():
    n = 10
    A = gen.general(n, seed=2)
    A[:, 4] = 0.0
    A = np.asfortranarray(A)
    _, info, _ = oracle.getrf(A, 3, protect=False)
    assert info == 5


@pytest.mark.parametrize("n,nb", [(33, 8), (64, 16)])
def test_getrf_vs_lapack(n, nb):
    A0 = gen.general(n, seed=n)
    A = A0.copy(order="F")
    ipiv, info, _ = oracle.getrf(A, nb)
    lu, piv, linfo = lapack.dgetrf(A0)
    assert info == 0 and linfo == 0
    assert np.array_equal(ipiv, piv + 1)
    assert np.max(np.abs(A - lu)) <= 1e3 * U64 * np.max(np.abs(lu))
    B = A0.copy(order="F")
    ipiv2, _ = oracle.getrf_unb(B)
    assert np.array_equal(ipiv2, ipiv)
    perm = perm_from_ipiv(ipiv, n)
    L, U = unit_lower(A), np.triu(A)
    assert np.linalg.norm(A0[perm] - L @ U) / np.linalg.norm(A0) < 1e-15


# ------------------------------------------------------------------------ QR
def qr_q(A, tau):
    n = A.shape[0]
    Q = np.eye(n)
    for j in range(n - 1, -1, -1):
        v = np.zeros(n)
        v[j] = 1.0
        v[j + 1:] = A[j + 1:, j]
        Q -= tau[j] * np.outer(v, v @ Q)
    return Q


def test_geqrf_upper_triangular_is_fixed_point():
    n = 21
    A0 = np.asfortranarray(np.triu(gen.general(n, seed=4)))
    A = A0.copy(order="F")
    tau, rep = oracle.geqrf(A, 8)
    assert np.all(tau == 0.0)
    assert np.array_equal(A, A0)
    assert rep.flagged_tiles == 0 and rep.panel_flags == 0


def test_geqrf_orthogonal_input_closed_form():
    """A = Q from the reflector generator: R must be diagonal with |R_ii| = 1."""
    n = 40
    _, _, V = gen.mp_matrix(n, 1.0, seed=9)
    Q = np.eye(n)
    for v in V:
        Q = Q - (2.0 / (v @ v)) * np.outer(Q @ v, v)
    A = np.asfortranarray(Q)
    oracle.geqrf(A, 16)
    R = np.triu(A)
    assert np.allclose(np.abs(np.diag(R)), 1.0, atol=1e-13)
    assert np.max(np.abs(R - np.diag(np.diag(R)))) < 1e-13


@pytest.mark.parametrize("n,nb", [(30, 8), (64, 16), (45, 45)])
def test_geqrf_vs_lapack_and_invariants(n, nb):
    A0 = gen.general(n, seed=3 * n + nb)
    A = A0.copy(order="F")
    tau, rep = oracle.geqrf(A, nb)
    qr, ltau, _, info = lapack.dgeqrf(A0)
    assert info == 0
    assert np.max(np.abs(tau - ltau)) < 1e-13
    assert np.max(np.abs(np.triu(A) - np.triu(qr))) < 1e-12 * np.max(np.abs(qr))
    Q = qr_q(A, tau)
    R = np.triu(A)
    assert np.linalg.norm(A0 - Q @ R) / np.linalg.norm(A0) < 1e-14
    assert np.linalg.norm(np.eye(n) - Q.T @ Q) / np.sqrt(n) < 1e-14
    assert rep.flagged_tiles == 0 and rep.panel_flags == 0


def test_geqrf_blocked_vs_unblocked():
    n = 50
    A0 = gen.general(n, seed=8)
    A1, A2 = A0.copy(order="F"), A0.copy(order="F")
    t1, _ = oracle.geqrf(A1, 12)
    t2 = oracle.geqrf_unb(A2)
    assert np.max(np.abs(t1 - t2)) < 1e-13
    assert np.max(np.abs(A1 - A2)) < 1e-12


# ---------------------------------------------------------------- ABFT layer
def test_encode_closed_form():
    """Column side [e, w] per tile-row and row side [e, w] per tile-column."""
    m, n, nb = 5, 4, 2
    A = np.asfortranarray(np.arange(1.0, m * n + 1).reshape(n, m).T)
    colchk, rowchk = oracle.encode(A, nb)
    for I in range(3):
        rows = A[I * nb:(I + 1) * nb]
        w = np.arange(1, rows.shape[0] + 1)
        assert np.array_equal(colchk[2 * I], rows.sum(0))
        assert np.array_equal(colchk[2 * I + 1], w @ rows)
    for J in range(2):
        cols = A[:, J * nb:(J + 1) * nb]
        w = np.arange(1, cols.shape[1] + 1)
        assert np.array_equal(rowchk[:, 2 * J], cols.sum(1))
        assert np.array_equal(rowchk[:, 2 * J + 1], cols @ w)
    nfl, flags, mr = oracle.verify(A, nb, colchk, rowchk)
    assert nfl == 0 and mr == 0.0
    B = A.copy(order="F")
    B[3, 2] += 1.0
    nfl, flags, _ = oracle.verify(B, nb, colchk, rowchk)
    assert nfl == 1 and flags[1, 1] == 1


@pytest.mark.parametrize("kind", ["chol", "lu", "qr"])
def test_no_false_alarms_random(kind):
    n, nb = 96, 16
    for seed in range(4):
        A = gen.spd(n, seed) if kind == "chol" else gen.general(n, seed)
        if kind == "chol":
            info, rep = oracle.potrf(A, nb)
        elif kind == "lu":
            _, info, rep = oracle.getrf(A, nb)
        else:
            _, rep = oracle.geqrf(A, nb)
        assert rep.flagged_tiles == 0 and rep.panel_flags == 0 and rep.status == 0
        assert 0.0 < rep.max_ratio < 0.35


def _run(kind, A, nb, faults=None, tau_scale=2.0):
    if kind == "chol":
        info, rep = oracle.potrf(A, nb, faults=faults, tau_scale=tau_scale)
        return rep, {}
    if kind == "lu":
        ipiv, info, rep = oracle.getrf(A, nb, faults=faults, tau_scale=tau_scale)
        return rep, {"ipiv": ipiv}
    tau, rep = oracle.geqrf(A, nb, faults=faults, tau_scale=tau_scale)
    return rep, {"tau": tau}


def _make(kind, n, seed):
    return gen.spd(n, seed) if kind == "chol" else gen.general(n, seed)


@pytest.mark.parametrize("kind", ["chol", "lu", "qr"])
@pytest.mark.parametrize("bit", [62, 60, 55, 52, 45])
def test_single_flip_detected_and_corrected(kind, bit):
    """A significant single-bit flip in the trailing matrix is located at the
    injected element and corrected; the factors then match the clean run."""
    n, nb = 80, 16
    A0 = _make(kind, n, seed=bit)
    clean = A0.copy(order="F")
    rep0, aux0 = _run(kind, clean, nb)
    f = gen.fault_plan(kind, n, nb, seed=1000 + bit)
    f["bit"] = bit
    A = A0.copy(order="F")
    rep, aux = _run(kind, A, nb, faults=[f])
    assert rep.status & oracle.ST_CORRECTED and not rep.status & oracle.ST_UNCORRECTABLE
    assert rep.corrected == 1 and rep.first_flag_iter == f["iter"]
    ev = rep.events()
    assert ev[0] == (f["iter"], 1, f["row"], f["col"])
    scale = np.max(np.abs(clean))
    assert np.max(np.abs(A - clean)) <= 1e-12 * scale
    for k in aux0:
        assert np.allclose(aux[k], aux0[k], rtol=0, atol=1e-12)


@pytest.mark.parametrize("pos", [(87, 64), (95, 64), (70, 70), (95, 95), (80, 79)])
@pytest.mark.parametrize("bit", [57, 55, 62])
def test_chol_diagonal_tile_flip_corrected(pos, bit):
    """Cholesky keeps one triangle of a diagonal tile; a flip anywhere in it
    shows in two columns (the element and its mirror) and is corrected.  The
    rebuilt element carries the column checksum's rounding, which the
    recheck sees multiplied by the element's row weight (up to nb): the far
    corner (nb-1, 0) of the tile is the case that exercises that allowance.
    Bit 62 turns an off-diagonal entry (|a| ~ 0.1) into ~1e307, whose
    weighted column sum overflows: the pattern of two flagged columns alone
    names the element and its mirror."""
    n, nb = 128, 32
    A0 = gen.spd(n, 0)
    clean = A0.copy(order="F")
    oracle.potrf(clean, nb)
    f = {"iter": 1, "row": pos[0], "col": pos[1], "bit": bit}
    A = A0.copy(order="F")
    info, rep = oracle.potrf(A, nb, faults=[f])
    assert info == 0
    assert rep.status & oracle.ST_CORRECTED and not rep.status & oracle.ST_UNCORRECTABLE
    assert rep.events()[0] == (1, 1, pos[0], pos[1])
    L, L0 = np.tril(A), np.tril(clean)
    assert np.max(np.abs(L - L0)) <= 1e-12 * np.max(np.abs(L0))


@pytest.mark.parametrize("kind", ["chol", "lu", "qr"])
def test_low_bit_flip_harmless(kind):
    """Bit 0 changes an element by one ulp: undetectable by any floating-point
    checksum and harmless for the backward error."""
    n, nb = 64, 16
    A0 = _make(kind, n, seed=2)
    f = gen.fault_plan(kind, n, nb, seed=77)
    f["bit"] = 0
    A = A0.copy(order="F")
    rep, _ = _run(kind, A, nb, faults=[f])
    assert not rep.status & oracle.ST_UNCORRECTABLE
    clean = A0.copy(order="F")
    _run(kind, clean, nb)
    assert np.max(np.abs(A - clean)) <= 1e-12 * np.max(np.abs(clean))


@pytest.mark.parametrize("kind", ["lu", "qr"])
def test_two_flips_same_tile_uncorrectable(kind):
    n, nb = 64, 16
    A = _make(kind, n, seed=5)
    k = 1
    base = (k + 1) * nb
    f1 = {"iter": k, "row": base + 2, "col": base + 3, "bit": 61}
    f2 = {"iter": k, "row": base + 5, "col": base + 9, "bit": 61}
    rep, _ = _run(kind, A, nb, faults=[f1, f2])
    assert rep.status & oracle.ST_UNCORRECTABLE


def test_nan_and_inf_flips_corrected():
    n, nb = 64, 16
    A0 = gen.general(n, seed=6)
    clean = A0.copy(order="F")
    _run("lu", clean, nb)
    # bit 62 on an entry of magnitude in [1,2) turns it into +-Inf/NaN territory
    A = A0.copy(order="F")
    f = {"iter": 0, "row": 40, "col": 50, "bit": 62}
    rep, _ = _run("lu", A, nb, faults=[f])
    assert rep.corrected == 1 and not rep.status & oracle.ST_UNCORRECTABLE
    assert np.max(np.abs(A - clean)) <= 1e-12 * np.max(np.abs(clean))


@pytest.mark.parametrize("target", [1, 2])
def test_checksum_flip_repaired(target):
    n, nb = 64, 16
    A0 = gen.general(n, seed=9)
    clean = A0.copy(order="F")
    _run("lu", clean, nb)
    A = A0.copy(order="F")
    # column checksums: row 2I (+1) of tile-row I; row checksums: column 2J (+1)
    f = {"iter": 1, "target": target, "row": 2 * 3 if target == 1 else 50, "col": 45 if target == 1 else 2 * 3,
         "bit": 58}
    rep, _ = _run("lu", A, nb, faults=[f])
    assert rep.status & oracle.ST_REPAIRED and rep.checksum_repaired == 1
    assert not rep.status & (oracle.ST_CORRECTED | oracle.ST_UNCORRECTABLE)
    assert np.array_equal(A, clean)


def _one_line_case(flag_side):
    """A 64 x 64 matrix whose tile (1, 0) (nb = 32) has one line of large
    entries: row i0 = 40 (flag_side "col": a perturbation of element (40, 5)
    only exceeds the column's threshold) or column j0 = 5 (flag_side "row":
    only the row's).  Returns (A, i0, j0)."""
    A = np.asfortranarray(gen.rng(31).uniform(-1, 1, (64, 64)))
    i0, j0 = 40, 5
    if flag_side == "col":
        A[i0, 0:32] = 1e6
        A[i0, j0] = 0.375
    else:
        A[32:64, j0] = 1e6
        A[i0, j0] = 0.375
    return A, i0, j0


@pytest.mark.parametrize("flag_side", ["col", "row"])
def test_single_line_flag_located_by_ratio(flag_side):
    """Off-diagonal tile where only one side flags: the weighted / plain
    difference ratio of the flagged line is the element's position (1-based)
    inside the tile, so the located element is the perturbed one, and it is
    rebuilt from its column checksum to within that checksum's tolerance."""
    A, i0, j0 = _one_line_case(flag_side)
    colchk, rowchk = oracle.encode(A, 32)
    orig = A[i0, j0]
    A[i0, j0] += 1e-10
    _, flags, _ = oracle.verify(A, 32, colchk, rowchk)
    assert flags[1, 0] == 1 and flags.sum() == 1
    rep = oracle.verify_correct(A, 32, colchk, rowchk)
    assert rep.flagged_tiles == 1 and rep.corrected == 1 and rep.status == oracle.ST_CORRECTED
    assert rep.events() == [(0, 1, i0, j0)]
    # the rebuilt value: the column sum minus the other entries, exact up to
    # the rounding of that column's sums (tolerance 16 u sum |column|)
    tol = 16 * U64 * np.abs(A[32:64, j0]).sum()
    assert abs(A[i0, j0] - orig) <= tol
    if flag_side == "col":
        assert abs(A[i0, j0] - orig) < 1e-13  # the column is O(1): far below the perturbation
    # and the refreshed checksums now pass
    _, flags, _ = oracle.verify(A, 32, colchk, rowchk)
    assert flags.sum() == 0


def test_chol_diagonal_tile_checksum_repair():
    """A flipped row-checksum entry of a diagonal tile in the symmetric view:
    no column of the tile flags, so no data element is suspect; the tile's
    checksums are re-encoded from its data, and the factor is bitwise the
    clean one (the data never changed)."""
    n, nb = 96, 32
    A0 = gen.spd(n, seed=12)
    clean = A0.copy(order="F")
    oracle.potrf(clean, nb)
    A = A0.copy(order="F")
    f = {"iter": 0, "target": 2, "row": 45, "col": 2 * 1, "bit": 56}
    info, rep = oracle.potrf(A, nb, faults=[f])
    assert info == 0
    assert rep.status == oracle.ST_REPAIRED and rep.checksum_repaired == 1 and rep.corrected == 0
    assert rep.events() == [(0, 2, 32, 32)]
    assert np.array_equal(np.tril(A), np.tril(clean))


@pytest.mark.parametrize("k,i,j,bit", [(2, 246, 219, 18), (0, 79, 78, 17), (0, 252, 241, 21), (2, 224, 205, 18),
                                        (2, 213, 205, 20), (1, 172, 133, 19), (2, 254, 192, 20)])
def test_chol_diagonal_tile_near_threshold_flip_located_by_pattern(k, i, j, bit):
    """Mid-mantissa flips (a few thresholds in size) inside diagonal tiles:
    both columns of the element and its mirror flag, while the weighted /
    plain ratios carry rounding noise of the weighted sums that can move them
    off an integer by more than the 0.25 acceptance.  Under the one fault per
    tile model the two flagged columns alone name the element; it is rebuilt,
    and the factor is the clean one to rounding."""
    n, nb = 256, 64
    A0 = gen.spd(n, 21)
    clean = A0.copy(order="F")
    oracle.potrf(clean, nb)
    f = {"iter": k, "row": i, "col": j, "bit": bit}
    A = A0.copy(order="F")
    info, rep = oracle.potrf(A, nb, faults=[f])
    assert info == 0 and rep.status == oracle.ST_CORRECTED
    assert rep.events() == [(k, 1, i, j)]
    assert np.max(np.abs(np.tril(A) - np.tril(clean))) <= 1e-14 * np.max(np.abs(clean))


def test_chol_diagonal_tile_column_checksum_entry_repaired():
    """A flipped plain (e) entry of a diagonal tile's column checksums: one
    column's plain difference flags, its weighted one and every row agree, so
    no data element is suspect; the checksums are re-encoded and the factor
    is bitwise the clean one."""
    n, nb = 96, 32
    A0 = gen.spd(n, seed=12)
    clean = A0.copy(order="F")
    oracle.potrf(clean, nb)
    A = A0.copy(order="F")
    f = {"iter": 0, "target": 1, "row": 2 * 1, "col": 45, "bit": 56}
    info, rep = oracle.potrf(A, nb, faults=[f])
    assert info == 0
    assert rep.status == oracle.ST_REPAIRED and rep.checksum_repaired == 1 and rep.corrected == 0
    assert rep.events() == [(0, 2, 32, 32)]
    assert np.array_equal(np.tril(A), np.tril(clean))


def _huge_offdiag_plan(n, nb, k, seed):
    """An element of an off-diagonal tile of the Cholesky trailing matrix after
    iteration k whose bit-62 flip gives a finite value near 1e307 (|a| in
    [1/16, 1/2)) placed at least 20 rows into its tile, so that its weighted
    column sum (row weight >= 21) overflows; the trailing matrix is the
    Schur complement formed from the clean factor."""
    A0 = gen.spd(n, seed)
    L = A0.copy(order="F")
    oracle.potrf(L, nb)
    L = np.tril(L)
    c1 = (k + 1) * nb
    S = L[c1:, c1:] @ L[c1:, c1:].T
    for i in range(c1 + nb, n):
        for j in range(c1, i - nb + 1):
            if (i // nb) != (j // nb) and (i % nb) >= 20 and 1 / 16 <= abs(S[i - c1, j - c1]) < 0.5:
                return A0, np.tril(L), {"iter": k, "row": i, "col": j, "bit": 62}
    raise AssertionError("no candidate")


def test_huge_flip_full_corrected_single_side_not_repaired():
    """A flip to ~1e307 in an off-diagonal tile: with full checksums the
    flagged row and column intersect at the element, which is rebuilt; with
    the column side alone the weighted / plain ratio overflows and the row
    cannot be named, and the tile is reported uncorrectable (a data error is
    never taken for a checksum error: its weighted sum is flagged too)."""
    n, nb = 128, 32
    A0, Lc, f = _huge_offdiag_plan(n, nb, 0, seed=4)
    A = A0.copy(order="F")
    info, rep = oracle.potrf(A, nb, faults=[f])
    assert info == 0 and rep.status == oracle.ST_CORRECTED
    assert rep.events() == [(0, 1, f["row"], f["col"])]
    assert np.max(np.abs(np.tril(A) - Lc)) <= 1e-12 * np.max(np.abs(Lc))
    A = A0.copy(order="F")
    info, rep = oracle.potrf(A, nb, faults=[f], protect=oracle.SINGLE)
    assert rep.status & oracle.ST_UNCORRECTABLE and not rep.status & oracle.ST_REPAIRED
    assert rep.checksum_repaired == 0


# ------------------------------------------------------------ MP + refinement
def test_bf16_fp16_rounding_vs_libraries():
    import torch
    x = gen.rng(1).standard_normal(4000) * np.exp(gen.rng(2).uniform(-30, 30, 4000))
    x = x.astype(np.float32).astype(np.float64)
    bf = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(oracle.round_bf16(x), bf)
    h = x.astype(np.float16).astype(np.float64)
    assert np.array_equal(oracle.round_fp16(x), h)


def test_mp_generator_closed_form_and_reference_solve():
    n, kappa = 200, 1e6
    A, s, V = gen.mp_matrix(n, kappa, seed=21)
    sv = np.linalg.svd(A, compute_uv=False)
    assert abs(sv[0] / sv[-1] / kappa - 1) < 1e-6
    b = gen.rhs(n, seed=24)
    xs = gen.mp_exact_solution(b, s, V)
    xr = oracle.solve_ref(A, b)
    assert np.linalg.norm(xr - xs, np.inf) / np.linalg.norm(xs, np.inf) < 50 * kappa * U64


@pytest.mark.parametrize("prec,kappa,expect", [(oracle.PR32, 1e2, True), (oracle.PR32, 1e6, True),
                                                (oracle.PRBF16, 1e2, True), (oracle.PRBF16, 1e10, False),
                                                (oracle.PRF16, 1e2, True)])
def test_mp_refinement_outcomes(prec, kappa, expect):
    n = 128
    A, s, V = gen.mp_matrix(n, kappa, seed=21)
    b = gen.rhs(n, seed=24)
    x, info, ir = oracle.gesv_mp(A, b, prec, nb=32)
    assert info == 0
    assert bool(ir.converged) == expect
    if expect:
        xr = oracle.solve_ref(A, b)
        err = np.linalg.norm(x - xr, np.inf) / np.linalg.norm(xr, np.inf)
        assert err < max(1e-12, 20 * kappa * U64)


def test_mp_cholesky_refinement():
    n = 96
    A, s, V = gen.mp_matrix(n, 1e2, seed=22)
    b = gen.rhs(n, seed=24)
    x, info, ir = oracle.gesv_mp(A, b, oracle.PRBF16, nb=32, chol=True)
    assert info == 0 and ir.converged
    xs = gen.mp_exact_solution(b, s, V)
    assert np.linalg.norm(x - xs, np.inf) / np.linalg.norm(xs, np.inf) < 1e-12


@pytest.mark.parametrize("ta,tb,unit,lower", [(0, 0, 0, 0), (0, 1, 0, 1), (1, 0, 1, 0), (0, 0, 1, 0), (0, 1, 0, 0)])
def test_gemm_definition_brute_force(ta, tb, unit, lower):
    """The oracle's update product against explicit triple loops on small
    integer operands (every sum exact)."""
    rng = np.random.default_rng(4)
    m, n, k = 5, 4, 6
    A = rng.integers(-5, 6, size=(k, m) if ta else (m, k)).astype(float)
    B = rng.integers(-5, 6, size=(n, k) if tb else (k, n)).astype(float)
    C = rng.integers(-5, 6, size=(m, n)).astype(float)
    alpha, beta = -2.0, 3.0
    out = oracle.gemm(A, B, C, ta, tb, alpha, beta, lower=bool(lower), unit_lower_a=bool(unit))
    for i in range(m):
        for j in range(n):
            if lower and i < j:
                assert out[i, j] == C[i, j]
                continue
            s = 0.0
            for p in range(k):
                r, c = (p, i) if ta else (i, p)
                a = A[r, c]
                if unit:
                    a = 0.0 if r < c else (1.0 if r == c else a)
                b = B[j, p] if tb else B[p, j]
                s += a * b
            assert out[i, j] == beta * C[i, j] + alpha * s


# ------------------------------------------------------------- threading
@pytest.mark.parametrize("kind", ["chol", "lu", "qr"])
def test_threads_do_not_change_results(kind):
    """The oracle's parallel loops give every element to one thread with the
    serial order of operations: one thread and several threads must agree bit
    for bit, on the factors, the reports and with a planned flip."""
    n, nb = 700, 128
    A = gen.spd(n, 7) if kind == "chol" else gen.general(n, 7)
    f = gen.fault_plan(kind, n, nb, seed=3)
    f["bit"] = 60
    outs = []
    saved = oracle.get_threads()
    try:
        for t in (1, 5):
            oracle.set_threads(t)
            B = A.copy(order="F")
            if kind == "chol":
                aux, rep = oracle.potrf(B, nb, faults=[f])
            elif kind == "lu":
                aux, _, rep = oracle.getrf(B, nb, faults=[f])
            else:
                aux, rep = oracle.geqrf(B, nb, faults=[f])
            outs.append((B, np.asarray(aux), rep.status, rep.corrected, rep.max_ratio, rep.events()))
    finally:
        oracle.set_threads(saved)
    (B1, a1, *r1), (B2, a2, *r2) = outs
    assert np.array_equal(B1, B2) and np.array_equal(a1, a2) and r1 == r2
    assert r1[1] == 1  # the flip was found and corrected


# ------------------------------------------- protection levels (Alg. 1 ABFT half)
def _fact(kind, A, nb, **kw):
    if kind == "chol":
        info, rep = oracle.potrf(A, nb, **kw)
        return rep
    if kind == "lu":
        ipiv, info, rep = oracle.getrf(A, nb, **kw)
        return rep
    tau, rep = oracle.geqrf(A, nb, **kw)
    return rep


def _same_report(a, b):
    return (a.status, a.flagged_tiles, a.corrected, a.uncorrectable, a.panel_flags, a.max_ratio, a.events()) == \
        (b.status, b.flagged_tiles, b.corrected, b.uncorrectable, b.panel_flags, b.max_ratio, b.events())


@pytest.mark.parametrize("kind", ["chol", "lu", "qr"])
def test_levels_reduce_to_the_uniform_levels(kind):
    """levels all FULL is protect=True, all NONE is protect=False (bitwise
    factors, identical reports), and single-side protection leaves the clean
    factorization's data untouched (the checks only read)."""
    n, nb = 200, 32
    N = -(-n // nb)
    A0 = gen.spd(n, 3) if kind == "chol" else gen.general(n, 3)
    runs = {}
    for name, kw in (("full", {}), ("levels_full", {"levels": [2] * N}), ("none", {"protect": False}),
                     ("levels_none", {"levels": [0] * N}), ("single", {"protect": oracle.SINGLE})):
        A = A0.copy(order="F")
        runs[name] = (A, _fact(kind, A, nb, **kw))
    assert np.array_equal(runs["full"][0], runs["levels_full"][0])
    assert _same_report(runs["full"][1], runs["levels_full"][1])
    assert np.array_equal(runs["none"][0], runs["levels_none"][0])
    assert runs["none"][1].status == 0 and runs["none"][1].flagged_tiles == 0 and runs["none"][1].max_ratio == 0.0
    assert np.array_equal(runs["single"][0], runs["full"][0])
    assert runs["single"][1].status == 0 and 0.0 < runs["single"][1].max_ratio < 0.5


@pytest.mark.parametrize("kind", ["chol", "lu"])
def test_adaptive_levels_exact_carries(kind):
    """Integer / dyadic inputs: with the level switching none -> single ->
    full the carried checksums still equal the recomputed sums exactly
    (max_ratio 0 after every re-encode) and the factors are the exact ones."""
    n, nb = 192, 32
    levels = [0, 0, 1, 1, 2, 2]
    if kind == "chol":
        A, L0 = gen.chol_exact(n, seed=8)
        rep = _fact(kind, A, nb, levels=levels)
        assert np.array_equal(np.tril(A), L0)
    else:
        A, P, L0, U0 = gen.lu_exact(n, seed=8)
        rep = _fact(kind, A, nb, levels=levels)
        assert np.array_equal(np.tril(A, -1) + np.eye(n), L0) and np.array_equal(np.triu(A), U0)
    assert rep.status == 0 and rep.max_ratio == 0.0


@pytest.mark.parametrize("kind", ["chol", "lu", "qr"])
def test_adaptive_levels_flip_outcomes(kind):
    """A flip in an unprotected iteration goes unseen (and changes the
    result); the same flip in a single-side or full iteration is located at
    the planted element and corrected back to the clean result."""
    n, nb = 192, 32
    A0 = gen.spd(n, 4) if kind == "chol" else gen.general(n, 4)
    clean = A0.copy(order="F")
    _fact(kind, clean, nb)
    f = gen.fault_plan(kind, n, nb, seed=41, iters=2)
    f["bit"] = 61
    for lev, expect in ((0, "unseen"), (1, "corrected"), (2, "corrected")):
        levels = [2, 2, lev, 2, 2, 2]
        A = A0.copy(order="F")
        rep = _fact(kind, A, nb, levels=levels, faults=[f])
        diff = np.max(np.abs(np.tril(A - clean) if kind == "chol" else A - clean))
        if expect == "unseen":
            assert rep.status == 0 and rep.flagged_tiles == 0
            assert diff > 1e-6
        else:
            assert rep.status == oracle.ST_CORRECTED
            assert rep.events() == [(2, oracle.EV_CORRECTED, f["row"], f["col"])]
            assert diff <= 1e-12 * np.max(np.abs(clean))


# ------------------------------------------------- 1D errors: operand faults
def _lu_exact_operand(side):
    """LU of an exact dyadic matrix with one operand of iteration 1's update
    flipped in bit 52 (the exponent's lowest bit: the value doubles or
    halves): side "L" an element of L21 (a row of the update goes wrong),
    side "U" one of U12 (a column)."""
    n, nb = 160, 32
    A, P, L0, U0 = gen.lu_exact(n, seed=5)
    if side == "L":
        i, j = next((i, j) for i in range(64, n) for j in range(32, 64) if abs(L0[i, j]) > 0)
    else:
        i, j = next((i, j) for i in range(32, 64) for j in range(64, n) if abs(U0[i, j]) > 0)
    f = {"iter": 1, "target": 3 if side == "L" else 4, "row": i, "col": j, "bit": 52}
    return A, L0, U0, f, n, nb


@pytest.mark.parametrize("side", ["L", "U"])
def test_operand_fault_rebuilt_exactly(side):
    """Full checksums: a wrong row (column) of each tile it crosses is
    rebuilt from the column (row) checksums; with dyadic data every rebuilt
    element is exact, so the factors are bitwise L0, U0 and the events name
    the row (column) in every tile of the update it crossed."""
    A, L0, U0, f, n, nb = _lu_exact_operand(side)
    ipiv, info, rep = oracle.getrf(A, nb, faults=[f])
    assert np.array_equal(np.tril(A, -1) + np.eye(n), L0) and np.array_equal(np.triu(A), U0)
    assert rep.status == oracle.ST_CORRECTED and rep.corrected == 3 and rep.flagged_tiles == 3
    if side == "L":
        assert rep.events() == [(1, oracle.EV_ROW_REBUILT, f["row"], c) for c in (64, 96, 128)]
    else:
        r0 = 64
        assert rep.events() == [(1, oracle.EV_COL_REBUILT, r, f["col"]) for r in (r0, 96, 128)]


@pytest.mark.parametrize("side", ["L", "U"])
def test_operand_fault_single_side_uncorrectable(side):
    """Single-side (column) checksums detect the 1D error but cannot locate
    it: every tile it crossed is reported uncorrectable."""
    A, L0, U0, f, n, nb = _lu_exact_operand(side)
    ipiv, info, rep = oracle.getrf(A, nb, faults=[f], protect=oracle.SINGLE)
    assert rep.status & oracle.ST_UNCORRECTABLE and rep.flagged_tiles >= 1
    assert not np.array_equal(np.triu(A), U0)


@pytest.mark.parametrize("target,row,col", [(3, 100, 40), (3, 40, 35), (4, 5, 100)])
def test_qr_operand_fault_rebuilt(target, row, col):
    """QR: a flipped element of V (inside the panel's unit triangle or below
    it) or of W2 = T^T V^T C spreads along a row / column of C; it is rebuilt
    and the factors match the clean ones to rounding."""
    n, nb = 160, 32
    A0 = gen.general(n, 7)
    clean = A0.copy(order="F")
    tc, _ = oracle.geqrf(clean, nb)
    A = A0.copy(order="F")
    tau, rep = oracle.geqrf(A, nb, faults=[{"iter": 1, "target": target, "row": row, "col": col, "bit": 60}])
    assert rep.status == oracle.ST_CORRECTED and rep.uncorrectable == 0
    kinds = {e[1] for e in rep.events()}
    assert kinds == {oracle.EV_ROW_REBUILT if target == 3 else oracle.EV_COL_REBUILT}
    assert np.max(np.abs(A - clean)) <= 1e-12 * np.max(np.abs(clean))
    assert np.max(np.abs(tau - tc)) <= 1e-12


def test_chol_operand_fault_cross_detected():
    """Cholesky's update reads L21 twice (L21 L21^T): one flipped element
    corrupts a row and a column of the symmetric trailing matrix.  The tiles
    off the diagonal see a 1D error and are rebuilt; the diagonal tile sees
    the row and the column crossing (beyond the per-tile model) and is
    reported uncorrectable."""
    n, nb = 160, 32
    S, L0 = gen.chol_exact(n, seed=3)
    info, rep = oracle.potrf(S, nb, faults=[{"iter": 1, "target": 3, "row": 100, "col": 40, "bit": 62}])
    ev = rep.events()
    assert (1, oracle.EV_ROW_REBUILT, 100, 64) in ev and (1, oracle.EV_COL_REBUILT, 128, 100) in ev
    assert (1, oracle.EV_UNCORRECTABLE, 96, 96) in ev
    assert rep.status & oracle.ST_UNCORRECTABLE
