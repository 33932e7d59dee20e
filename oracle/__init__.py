"""Python loader for the plain CPU oracle (``oracle/oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark are the only callers.  The product library never imports
this package.  All arrays are numpy float64 / int32, column-major (Fortran
order), and are modified in place where the C routine factors in place.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

PR64, PR32, PRBF16, PRF16 = 0, 1, 2, 3

# status bits shared by the report structs
ST_CORRECTED, ST_REPAIRED, ST_UNCORRECTABLE, ST_PANEL = 1, 2, 4, 8
# protection levels: none, column checksums only (single side), both sides (full)
NONE, SINGLE, FULL = 0, 1, 2
# event kinds
EV_CORRECTED, EV_REPAIRED, EV_UNCORRECTABLE, EV_PANEL, EV_ROW_REBUILT, EV_COL_REBUILT = 1, 2, 3, 4, 5, 6


class Fault(C.Structure):
    _fields_ = [("iter", C.c_int32), ("target", C.c_int32), ("row", C.c_int64), ("col", C.c_int64),
                ("bit", C.c_int32), ("pad", C.c_int32)]


class Event(C.Structure):
    _fields_ = [("iter", C.c_int32), ("kind", C.c_int32), ("row", C.c_int64), ("col", C.c_int64)]


class Report(C.Structure):
    _fields_ = [("flagged_tiles", C.c_int64), ("corrected", C.c_int64), ("checksum_repaired", C.c_int64),
                ("uncorrectable", C.c_int64), ("panel_flags", C.c_int64), ("first_flag_iter", C.c_int32),
                ("status", C.c_int32), ("max_ratio", C.c_double), ("nev", C.c_int32), ("pad", C.c_int32),
                ("ev", Event * 16)]

    def events(self):
        return [(self.ev[i].iter, self.ev[i].kind, self.ev[i].row, self.ev[i].col) for i in range(min(self.nev, 16))]


class IRReport(C.Structure):
    _fields_ = [("iters", C.c_int32), ("converged", C.c_int32), ("failed_reason", C.c_int32), ("pad", C.c_int32),
                ("resid_norm", C.c_double), ("x_norm", C.c_double), ("a_norm", C.c_double),
                ("last_dx", C.c_double)]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain IEEE arithmetic, no FP contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        # -ffp-contract=off: no fused multiply-add behind the code's back;
        # AVX2 + FMA3 at most, so the library built here also runs on other x86
        # hosts (fma() is then one instruction; the sums stay as written)
        subprocess.check_call(["gcc", "-O3", "-mavx2", "-mfma", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
                               "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        d, i, i64 = C.c_double, C.c_int, C.c_int64
        P = C.c_void_p
        _lib.orc_potrf_unb.argtypes = [i, P, i]
        _lib.orc_getrf_unb.argtypes = [i, P, i, P]
        _lib.orc_geqrf_unb.argtypes = [i, P, i, P]
        _lib.orc_abft_potrf.argtypes = [i, i, P, i, i, i, d, P, i, P, P]
        _lib.orc_abft_getrf.argtypes = [i, i, P, i, P, i, i, d, P, i, P, P]
        _lib.orc_abft_geqrf.argtypes = [i, i, P, i, P, i, d, P, i, P, P]
        _lib.orc_encode.argtypes = [i, i, P, i, i, P, i, P, i]
        _lib.orc_verify.argtypes = [i, i, P, i, i, P, i, P, i, d, P, P]
        _lib.orc_verify_correct.argtypes = [i, i, P, i, P, P, d, P]
        _lib.orc_getrs.argtypes = [i, P, i, P, P]
        _lib.orc_potrs.argtypes = [i, P, i, P]
        _lib.orc_gesv_mp.argtypes = [i, i, P, i, P, P, i, i, i, P]
        _lib.orc_solve_ref.argtypes = [i, P, i, P, P, i]
        _lib.orc_round_bf16.argtypes = [d]
        _lib.orc_round_bf16.restype = d
        _lib.orc_round_fp16.argtypes = [d]
        _lib.orc_round_fp16.restype = d
        _lib.orc_set_threads.argtypes = [i]
        del i64
    return _lib


def set_threads(t):
    """Threads of the oracle's parallel loops (results do not depend on it)."""
    lib().orc_set_threads(int(t))


def get_threads():
    return int(lib().orc_get_threads())


def _f64(a):
    assert a.dtype == np.float64 and a.flags.f_contiguous, "expected a Fortran-ordered float64 array"
    return a.ctypes.data


def _faults(faults):
    if not faults:
        return None, 0, None
    arr = (Fault * len(faults))()
    for q, f in enumerate(faults):
        arr[q].iter, arr[q].target, arr[q].row, arr[q].col, arr[q].bit = (
            int(f["iter"]), int(f.get("target", 0)), int(f["row"]), int(f["col"]), int(f["bit"]))
    return C.cast(arr, C.c_void_p), len(faults), arr


def potrf_unb(A):
    return lib().orc_potrf_unb(A.shape[0], _f64(A), A.shape[0] if A.ndim == 2 else 1)


def getrf_unb(A):
    n = A.shape[0]
    ipiv = np.zeros(n, dtype=np.int32)
    info = lib().orc_getrf_unb(n, _f64(A), n, ipiv.ctypes.data)
    return ipiv, info


def geqrf_unb(A):
    n = A.shape[0]
    tau = np.zeros(n)
    lib().orc_geqrf_unb(n, _f64(A), n, tau.ctypes.data)
    return tau


def _level(protect):
    """True -> full checksums, False -> none, or a level 0 / 1 / 2"""
    if protect is True:
        return FULL
    if protect is False or protect is None:
        return NONE
    return int(protect)


def _levels(levels, n, nb):
    """per-iteration protection levels as an int8 array (or None)"""
    if levels is None:
        return None, None
    arr = np.ascontiguousarray(levels, dtype=np.int8)
    assert arr.shape == (-(-n // nb),), "one level per iteration"
    return arr.ctypes.data, arr


def potrf(A, nb, prec=PR64, protect=True, tau_scale=4.0, faults=None, levels=None):
    """Blocked right-looking Cholesky (lower) with optional ABFT; returns (info, Report).
    protect: True / False or a level (NONE, SINGLE, FULL); levels: one level per iteration."""
    n = A.shape[0]
    rep = Report()
    fp, nf, keep = _faults(faults)
    lp, lkeep = _levels(levels, n, nb)
    info = lib().orc_abft_potrf(n, nb, _f64(A), A.shape[0], prec, _level(protect), tau_scale, fp, nf, lp,
                                C.byref(rep))
    del keep, lkeep
    return info, rep


def getrf(A, nb, prec=PR64, protect=True, tau_scale=4.0, faults=None, levels=None):
    n = A.shape[0]
    ipiv = np.zeros(n, dtype=np.int32)
    rep = Report()
    fp, nf, keep = _faults(faults)
    lp, lkeep = _levels(levels, n, nb)
    info = lib().orc_abft_getrf(n, nb, _f64(A), A.shape[0], ipiv.ctypes.data, prec, _level(protect), tau_scale,
                                fp, nf, lp, C.byref(rep))
    del keep, lkeep
    return ipiv, info, rep


def geqrf(A, nb, protect=True, tau_scale=4.0, faults=None, levels=None):
    n = A.shape[0]
    tau = np.zeros(n)
    rep = Report()
    fp, nf, keep = _faults(faults)
    lp, lkeep = _levels(levels, n, nb)
    lib().orc_abft_geqrf(n, nb, _f64(A), A.shape[0], tau.ctypes.data, _level(protect), tau_scale, fp, nf, lp,
                         C.byref(rep))
    del keep, lkeep
    return tau, rep


def encode(A, nb):
    m, n = A.shape
    Tr, Tc = -(-m // nb), -(-n // nb)
    colchk = np.zeros((2 * Tr, n), order="F")
    rowchk = np.zeros((m, 2 * Tc), order="F")
    lib().orc_encode(m, n, _f64(A), m, nb, _f64(colchk), 2 * Tr, _f64(rowchk), m)
    return colchk, rowchk


def verify(A, nb, colchk, rowchk, tau_scale=4.0):
    m, n = A.shape
    Tr, Tc = -(-m // nb), -(-n // nb)
    flags = np.zeros((Tr, Tc), dtype=np.int32, order="F")
    mr = C.c_double(0.0)
    nfl = lib().orc_verify(m, n, _f64(A), m, nb, _f64(colchk), colchk.shape[0], _f64(rowchk), rowchk.shape[0],
                           tau_scale, flags.ctypes.data, C.byref(mr))
    return nfl, flags, mr.value


def verify_correct(A, nb, colchk, rowchk, tau_scale=4.0):
    """Verify square A (in place) against its checksums with the
    factorizations' locate / correct rules; returns the Report.  colchk and
    rowchk (from encode) are refreshed in place."""
    n = A.shape[0]
    assert A.shape == (n, n) and colchk.shape == (2 * -(-n // nb), n) and rowchk.shape == (n, 2 * -(-n // nb))
    rep = Report()
    lib().orc_verify_correct(n, nb, _f64(A), n, _f64(colchk), _f64(rowchk), tau_scale, C.byref(rep))
    return rep


def getrs(LU, ipiv, b):
    x = np.array(b, dtype=np.float64, copy=True)
    lib().orc_getrs(LU.shape[0], _f64(LU), LU.shape[0], ipiv.ctypes.data, x.ctypes.data)
    return x


def potrs(L, b):
    x = np.array(b, dtype=np.float64, copy=True)
    lib().orc_potrs(L.shape[0], _f64(L), L.shape[0], x.ctypes.data)
    return x


def gesv_mp(A, b, prec, nb=64, chol=False, max_iter=30):
    n = A.shape[0]
    x = np.zeros(n)
    ir = IRReport()
    info = lib().orc_gesv_mp(n, nb, _f64(A), n, np.ascontiguousarray(b, dtype=np.float64).ctypes.data,
                             x.ctypes.data, prec, int(chol), max_iter, C.byref(ir))
    return x, info, ir


def solve_ref(A, b, iters=3):
    n = A.shape[0]
    x = np.zeros(n)
    bb = np.ascontiguousarray(b, dtype=np.float64)
    lib().orc_solve_ref(n, _f64(A), n, bb.ctypes.data, x.ctypes.data, iters)
    return x


def round_bf16(x):
    return np.vectorize(lib().orc_round_bf16)(np.asarray(x, dtype=np.float64))


def round_fp16(x):
    return np.vectorize(lib().orc_round_fp16)(np.asarray(x, dtype=np.float64))


def gemm(A, B, C, transa=False, transb=False, alpha=1.0, beta=0.0, lower=False, unit_lower_a=False):
    """The update product of each iteration of the blocked decompositions
    (the trailing-matrix update, Sec. 2): returns beta*C + alpha*op(A) op(B)
    in float64, with the stored A read as unit lower triangular when asked
    (Householder vectors) and, for symmetric updates, only entries i >= j
    written (the others keep C's values).  beta == 0 ignores C's values."""
    A = np.array(A, dtype=np.float64)
    if unit_lower_a:
        A = np.tril(A, -1) + np.eye(*A.shape)
    opA = A.T if transa else A
    opB = np.asarray(B, dtype=np.float64).T if transb else np.asarray(B, dtype=np.float64)
    prod = alpha * (opA @ opB)
    C = np.array(C, dtype=np.float64)
    out = prod if beta == 0.0 else beta * C + prod
    if lower:
        keep = np.tril(np.ones(C.shape, dtype=bool))
        out = np.where(keep, out, C)
    return out
