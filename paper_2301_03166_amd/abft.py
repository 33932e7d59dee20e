"""Python binding of the C ABI in include/abft.h (argument marshalling only).

Every computation runs in the HIP library ``libabft.so`` built in-tree by
``paper_2301_03166_amd._build``; there is no fallback path.  PyTorch provides
device memory and the stream: matrices are CUDA (HIP) tensors in column-major
layout, i.e. ``A.stride(0) == 1`` and ``lda = A.stride(1)`` -- a
Fortran-ordered numpy array passed through ``torch.from_numpy(...).cuda()``
keeps that layout, and ``colmajor(t)`` makes one from any tensor.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# the in-tree build; ABFT_LIB names another build of the same library
LIB_PATH = os.environ.get("ABFT_LIB") or os.path.join(HERE, "libabft.so")

F64, F32, BF16, F16 = 0, 1, 2, 3
PROTECT_NONE, PROTECT_SINGLE, PROTECT_FULL = 0, 1, 2
OP_POTRF, OP_GETRF, OP_GEQRF, OP_GESV_MP, OP_POSV_MP, OP_POTRF_BATCHED, OP_GETRF_BATCHED = 1, 2, 3, 4, 5, 6, 7
ERR_HIP, ERR_WORKSPACE, ERR_UNSUPPORTED = -100, -101, -102
ST_CORRECTED, ST_REPAIRED, ST_UNCORRECTABLE, ST_PANEL, ST_INTERNAL = 1, 2, 4, 8, 16


class Fault(C.Structure):
    _fields_ = [("iter", C.c_int32), ("target", C.c_int32), ("row", C.c_int64), ("col", C.c_int64),
                ("bit", C.c_int32), ("matrix", C.c_int32)]


class Event(C.Structure):
    _fields_ = [("iter", C.c_int32), ("kind", C.c_int32), ("row", C.c_int64), ("col", C.c_int64)]


class Report(C.Structure):
    _fields_ = [("flagged_tiles", C.c_int64), ("corrected", C.c_int64), ("checksum_repaired", C.c_int64),
                ("uncorrectable", C.c_int64), ("panel_flags", C.c_int64), ("first_flag_iter", C.c_int32),
                ("status", C.c_int32), ("max_ratio", C.c_double), ("nev", C.c_int32), ("pad", C.c_int32),
                ("ev", Event * 16), ("fault_delta", C.c_double), ("fault_d", C.c_double),
                ("fault_tau", C.c_double)]

    def events(self):
        return sorted((self.ev[i].iter, self.ev[i].kind, self.ev[i].row, self.ev[i].col)
                      for i in range(min(self.nev, 16)))


class IRReport(C.Structure):
    _fields_ = [("iters", C.c_int32), ("converged", C.c_int32), ("failed_reason", C.c_int32), ("info", C.c_int32),
                ("resid_norm", C.c_double), ("x_norm", C.c_double), ("a_norm", C.c_double), ("last_dx", C.c_double)]


class Profile(C.Structure):
    _fields_ = [("ms_total", C.c_double), ("ms_panel", C.c_double), ("ms_tmu", C.c_double),
                ("ms_carry", C.c_double), ("ms_verify", C.c_double), ("tmu_flops", C.c_double),
                ("verify_bytes", C.c_double), ("tmu_launches", C.c_int32), ("iters", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Opts(C.Structure):
    _fields_ = [("nb", C.c_int32), ("protect", C.c_int32), ("tau_scale", C.c_double),
                ("faults", C.POINTER(Fault)), ("nfaults", C.c_int32), ("flags", C.c_int32),
                ("wgs_per_cu", C.c_int32), ("nlevels", C.c_int32), ("levels", C.POINTER(C.c_int8)),
                ("lookahead", C.c_int32), ("tmu_bk", C.c_int32)]


class AbftError(RuntimeError):
    pass


_lib = None


def lib():
    """Load libabft.so; raise if it has not been built (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise AbftError(f"{LIB_PATH} is missing: build it with paper_2301_03166_amd._build.build()")
        L = C.CDLL(LIB_PATH)
        P, i64, i32, d, sz = C.c_void_p, C.c_int64, C.c_int32, C.c_double, C.c_size_t
        L.abft_create.argtypes = [C.POINTER(P), P]
        L.abft_destroy.argtypes = [P]
        L.abft_set_stream.argtypes = [P, P]
        L.abft_get_profile.argtypes = [P, C.POINTER(Profile)]
        L.abft_workspace_size.argtypes = [P, C.c_int, i64, i32, C.POINTER(Opts), C.POINTER(sz)]
        L.abft_set_workspace.argtypes = [P, P, sz]
        L.abft_get_iter_profile.argtypes = [P, i32, P, C.POINTER(i32)]
        L.abft_report_fetch.argtypes = [P, P, C.POINTER(Report)]
        L.abft_potrf.argtypes = [P, i64, P, i64, P, sz, C.POINTER(Opts), P, P]
        L.abft_potrf_noalloc.argtypes = [P, i64, P, i64, C.POINTER(Opts), P, P]
        L.abft_getrf.argtypes = [P, i64, P, i64, P, P, sz, C.POINTER(Opts), P, P]
        L.abft_geqrf.argtypes = [P, i64, P, i64, P, P, sz, C.POINTER(Opts), P, P]
        L.abft_gemm.argtypes = [P, i32, i32, i32, i64, i64, i64, d, P, i64, P, i64, d, P, i64, P, sz]
        L.abft_encode.argtypes = [P, i64, i64, P, i64, i32, P, i64, P, i64]
        L.abft_verify.argtypes = [P, i64, i64, P, i64, i32, P, i64, P, i64, d, i32, P, P]
        L.abft_gesv_mp.argtypes = [P, i64, P, i64, P, P, i32, i32, P, sz, C.POINTER(Opts), P, P]
        L.abft_posv_mp.argtypes = [P, i64, P, i64, P, P, i32, i32, P, sz, C.POINTER(Opts), P, P]
        L.abft_potrf_batched.argtypes = [P, i32, i32, P, P, P, i32, P, sz, C.POINTER(Opts), P, P]
        L.abft_getrf_batched.argtypes = [P, i32, i32, P, P, P, P, i32, P, sz, C.POINTER(Opts), P, P]
        _lib = L
    return _lib


def _check(rc, what):
    if rc != 0:
        raise AbftError(f"{what} returned {rc}")


def colmajor(t):
    """A column-major copy (stride(0) == 1) of a 2-D tensor with the same values."""
    return t.t().contiguous().t()


def _ld(A):
    """Leading dimension of a column-major 2-D tensor (size-1 dimensions carry no stride)."""
    if A.dim() != 2:
        raise AbftError("matrices must be 2-D tensors")
    m, n = A.shape
    if m > 1 and A.stride(0) != 1:
        raise AbftError("matrices must be column-major (stride(0) == 1)")
    lda = A.stride(1) if n > 1 else m
    if lda < max(m, 1):
        raise AbftError("column stride smaller than the number of rows")
    return max(lda, 1)


FLAG_PROFILE, FLAG_GRAPH, FLAG_OVERLAP_VERIFY = 1, 2, 4
GEMM_LOWER, GEMM_UNIT_LOWER_A = 1, 2


def protect_level(protect):
    """True -> PROTECT_FULL, False / None -> PROTECT_NONE, or a level 0 / 1 / 2 as given"""
    if protect is True:
        return PROTECT_FULL
    if protect is False or protect is None:
        return PROTECT_NONE
    return int(protect)


def make_opts(nb, protect=True, tau_scale=4.0, faults=None, profile=False, graph=False, wgs_per_cu=0, levels=None,
              lookahead=0, tmu_bk=0, overlap=False):
    """abft_opts plus the host arrays it points to (keep them alive for the call);
    lookahead: CUs of the look-ahead panel stream (<= 0: off); tmu_bk: K depth
    of the trailing-update product tiles (0 / 16 / 32); overlap: verify the
    trailing tiles beside the next panel (ABFT_FLAG_OVERLAP_VERIFY)"""
    o = Opts()
    o.wgs_per_cu = int(wgs_per_cu)
    o.lookahead = int(lookahead)
    o.tmu_bk = int(tmu_bk)
    o.nb, o.protect, o.tau_scale = int(nb), protect_level(protect), float(tau_scale)
    o.flags = (FLAG_PROFILE if profile else 0) | (FLAG_GRAPH if graph else 0) | (FLAG_OVERLAP_VERIFY if overlap else 0)
    keep = []
    if faults:
        fa = (Fault * len(faults))()
        for q, f in enumerate(faults):
            fa[q].iter, fa[q].target = int(f["iter"]), int(f.get("target", 0))
            fa[q].row, fa[q].col, fa[q].bit = int(f["row"]), int(f["col"]), int(f["bit"])
            fa[q].matrix = int(f.get("matrix", 0))
        o.faults, o.nfaults = C.cast(fa, C.POINTER(Fault)), len(faults)
        keep.append(fa)
    if levels is not None:
        la = (C.c_int8 * len(levels))(*[int(v) for v in levels])
        o.levels, o.nlevels = C.cast(la, C.POINTER(C.c_int8)), len(levels)
        keep.append(la)
    return o, keep


class Handle:
    """Owns an abft_handle bound to torch's current stream and cached workspaces."""

    def __init__(self, device=None):
        import torch
        self.torch = torch
        self.device = torch.device(device or "cuda")
        self._h = C.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib().abft_create(C.byref(self._h), C.c_void_p(torch.cuda.current_stream().cuda_stream)),
                   "abft_create")
        self._ws = {}

    def close(self):
        """Finish the handle's work and destroy it (abft_destroy synchronizes
        its streams first).  Call it before the process exits: a handle left to
        the interpreter's teardown may be destroyed after the HIP runtime."""
        h, self._h = self._h, None
        if h:
            self.torch.cuda.synchronize(self.device)
            self._ws.clear()
            _check(lib().abft_destroy(h), "abft_destroy")

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _sync_stream(self):
        lib().abft_set_stream(self._h, C.c_void_p(self.torch.cuda.current_stream(self.device).cuda_stream))

    def workspace(self, op, n, opts, batch=0):
        size = C.c_size_t()
        _check(lib().abft_workspace_size(self._h, op, int(n), int(batch), C.byref(opts), C.byref(size)),
               "abft_workspace_size")
        buf = self._ws.get(op)
        if buf is None or buf.numel() < size.value:
            self._ws[op] = buf = self.torch.empty(max(size.value, 1), dtype=self.torch.uint8, device=self.device)
        return buf, size.value

    def new_report(self):
        return self.torch.zeros(C.sizeof(Report), dtype=self.torch.uint8, device=self.device)

    @staticmethod
    def read_report(buf):
        raw = bytes(buf.cpu().numpy().tobytes())
        return Report.from_buffer_copy(raw)

    def report_fetch(self, buf):
        """abft_report_fetch: the report in device buffer `buf` after the work
        enqueued on the current stream (synchronizes that stream)."""
        out = Report()
        self._sync_stream()
        _check(lib().abft_report_fetch(self._h, buf.data_ptr(), C.byref(out)), "abft_report_fetch")
        return out

    def set_workspace(self, buf):
        """abft_set_workspace: register a uint8 device tensor as the handle's
        workspace (None unregisters); calls made with dwork == NULL use it."""
        if buf is None:
            _check(lib().abft_set_workspace(self._h, None, 0), "abft_set_workspace")
        else:
            _check(lib().abft_set_workspace(self._h, buf.data_ptr(), buf.numel() * buf.element_size()),
                   "abft_set_workspace")
        self._registered_ws = buf

    # ------------------------------------------------------------ factorizations
    def potrf(self, A, nb, protect=True, tau_scale=4.0, faults=None, report=None, info=None, sync=True,
              profile=False, levels=None, lookahead=0, tmu_bk=0, overlap=True):
        """In-place Cholesky (lower) of column-major A; returns (info, Report) when sync.
        protect: True / False or a PROTECT_* level; levels: one PROTECT_* level per iteration;
        lookahead: compute units of the look-ahead panel stream (<= 0: one stream);
        tmu_bk: K depth of the trailing-update product tiles (0 = 16, or 32);
        overlap: verify the trailing tiles beside the next panel (the default;
        False: everything on the handle's stream)."""
        return self._factor(OP_POTRF, A, nb, protect, tau_scale, faults, report, info, sync, profile=profile,
                            levels=levels, lookahead=lookahead, tmu_bk=tmu_bk, overlap=overlap)

    def potrf_noalloc(self, A, nb, protect=True, tau_scale=4.0, faults=None, report=None, info=None, sync=True):
        """abft_potrf_noalloc: the Cholesky of potrf with the library's built-in
        scratch (no workspace).  report / info may be caller tensors (nothing is
        allocated by the call itself); returns (info, Report) when sync."""
        torch = self.torch
        n = A.shape[0]
        if A.shape[1] != n or A.dtype != torch.float64 or not A.is_cuda:
            raise AbftError("expected a square float64 device matrix")
        opts, keep = make_opts(nb, protect, tau_scale, faults)
        rep = report if report is not None else self.new_report()
        inf = info if info is not None else torch.zeros(1, dtype=torch.int32, device=self.device)
        self._sync_stream()
        rc = lib().abft_potrf_noalloc(self._h, n, A.data_ptr(), _ld(A), C.byref(opts), inf.data_ptr(), rep.data_ptr())
        del keep
        _check(rc, "abft_potrf_noalloc")
        if not sync:
            return ()
        torch.cuda.synchronize(self.device)
        return int(inf.item()), self.read_report(rep)

    def getrf(self, A, nb, protect=True, tau_scale=4.0, faults=None, ipiv=None, report=None, info=None, sync=True,
              profile=False, levels=None, lookahead=0, tmu_bk=0, overlap=True):
        torch = self.torch
        if ipiv is None:
            ipiv = torch.zeros(A.shape[0], dtype=torch.int32, device=self.device)
        out = self._factor(OP_GETRF, A, nb, protect, tau_scale, faults, report, info, sync, aux=ipiv, profile=profile,
                           levels=levels, lookahead=lookahead, tmu_bk=tmu_bk, overlap=overlap)
        return (ipiv,) + out if sync else ipiv

    def geqrf(self, A, nb, protect=True, tau_scale=4.0, faults=None, tau=None, report=None, info=None, sync=True,
              profile=False, levels=None, lookahead=0, tmu_bk=0, overlap=True):
        torch = self.torch
        if tau is None:
            tau = torch.zeros(A.shape[0], dtype=torch.float64, device=self.device)
        out = self._factor(OP_GEQRF, A, nb, protect, tau_scale, faults, report, info, sync, aux=tau, profile=profile,
                           levels=levels, lookahead=lookahead, tmu_bk=tmu_bk, overlap=overlap)
        return (tau,) + out if sync else tau

    def profile(self):
        """Phase profile of the last call made with profile=True."""
        p = Profile()
        _check(lib().abft_get_profile(self._h, C.byref(p)), "abft_get_profile")
        return p.as_dict()

    ITER_PHASES = ("pd", "pu", "tmu", "carry", "verify")

    def iter_profile(self):
        """Per-iteration phase times (ms) of the last call made with
        profile=True: a dict phase -> list over iterations."""
        n = C.c_int32()
        _check(lib().abft_get_iter_profile(self._h, 0, None, C.byref(n)), "abft_get_iter_profile")
        cap = n.value
        buf = (C.c_double * max(1, 5 * cap))()
        _check(lib().abft_get_iter_profile(self._h, cap, buf, C.byref(n)), "abft_get_iter_profile")
        return {ph: [buf[q * cap + k] for k in range(cap)] for q, ph in enumerate(self.ITER_PHASES)}

    def _factor(self, op, A, nb, protect, tau_scale, faults, report, info, sync, aux=None, profile=False, levels=None,
                lookahead=0, tmu_bk=0, overlap=True):
        torch = self.torch
        n = A.shape[0]
        if A.shape[1] != n or A.dtype != torch.float64 or not A.is_cuda:
            raise AbftError("expected a square float64 device matrix")
        lda = _ld(A)
        if nb is None or nb == "auto":  # the autotuned block size and product tile for this operation and size class
            from . import autotune
            name = {OP_POTRF: "potrf", OP_GETRF: "getrf"}.get(op, "geqrf")
            nb = autotune.lookup_nb(name, n)
            if tmu_bk == 0:
                tmu_bk = autotune.lookup_tmu_bk(name, n)
        opts, keep = make_opts(nb, protect, tau_scale, faults, profile, levels=levels, lookahead=lookahead,
                               tmu_bk=tmu_bk, overlap=overlap)
        ws, wbytes = self.workspace(op, n, opts)
        rep = report if report is not None else self.new_report()
        inf = info if info is not None else torch.zeros(1, dtype=torch.int32, device=self.device)
        self._sync_stream()
        L = lib()
        if op == OP_POTRF:
            rc = L.abft_potrf(self._h, n, A.data_ptr(), lda, ws.data_ptr(), wbytes, C.byref(opts), inf.data_ptr(),
                              rep.data_ptr())
        elif op == OP_GETRF:
            rc = L.abft_getrf(self._h, n, A.data_ptr(), lda, aux.data_ptr(), ws.data_ptr(), wbytes, C.byref(opts),
                              inf.data_ptr(), rep.data_ptr())
        else:
            rc = L.abft_geqrf(self._h, n, A.data_ptr(), lda, aux.data_ptr(), ws.data_ptr(), wbytes, C.byref(opts),
                              inf.data_ptr(), rep.data_ptr())
        del keep
        _check(rc, f"op {op}")
        if not sync:
            return ()
        torch.cuda.synchronize(self.device)
        return int(inf.item()), self.read_report(rep)

    # ------------------------------------------------------------ mixed precision
    def gesv_mp(self, A, b, prec, nb=256, max_iter=30, chol=False, protect=True, tau_scale=4.0, faults=None,
                x=None, report=None, ir=None, sync=True, profile=False, lookahead=0, overlap=False):
        """Solve A x = b: binary32 factorization (trailing update in `prec`) + FP64 refinement,
        or the FP64 factorization and direct solve when prec == F64.  Returns (x, IRReport, Report).
        overlap: the factorization verifies the trailing tiles beside the next panel (off by
        default: at n = 16384 the restricted stream's creation per call costs what it saves)."""
        torch = self.torch
        n = A.shape[0]
        if A.shape[1] != n or A.dtype != torch.float64 or not A.is_cuda:
            raise AbftError("expected a square float64 device matrix")
        lda = _ld(A)
        bb = b.contiguous()
        if x is None:
            x = torch.zeros(n, dtype=torch.float64, device=self.device)
        op = OP_POSV_MP if chol else OP_GESV_MP
        opts, keep = make_opts(nb, protect, tau_scale, faults, profile, lookahead=lookahead, overlap=overlap)
        ws, wbytes = self.workspace(op, n, opts)
        rep = report if report is not None else self.new_report()
        irb = ir if ir is not None else torch.zeros(C.sizeof(IRReport), dtype=torch.uint8, device=self.device)
        self._sync_stream()
        fn = lib().abft_posv_mp if chol else lib().abft_gesv_mp
        rc = fn(self._h, n, A.data_ptr(), lda, bb.data_ptr(), x.data_ptr(), int(prec), int(max_iter), ws.data_ptr(),
                wbytes, C.byref(opts), irb.data_ptr(), rep.data_ptr())
        del keep
        _check(rc, "abft_gesv_mp")
        if not sync:
            return x
        torch.cuda.synchronize(self.device)
        return x, IRReport.from_buffer_copy(bytes(irb.cpu().numpy().tobytes())), self.read_report(rep)

    # ------------------------------------------------------------ batched
    def batched(self, mats, chol, protect=True, tau_scale=4.0, faults=None, nmax=None, sync=True, state=None,
                graph=False, wgs_per_cu=None):
        """Factor a list of column-major square matrices (all float64 or all float32) in place with one
        batched call (block / tile size 32).  Returns (infos, ipivs, reports) when sync; `state` keeps the
        device argument arrays alive so that graph=True calls replay the library's captured graph."""
        torch = self.torch
        batch = len(mats)
        prec = F64 if mats[0].dtype == torch.float64 else F32
        if state is None:
            state = self.batched_args(mats, chol)
        ns, ptrs, ldas, ipivs, piv_ptrs, infos, reps = state
        if wgs_per_cu is None:  # the autotuned choice for this operation and precision
            from . import autotune
            wgs_per_cu = autotune.lookup_wgs("potrf" if chol else "getrf", "f64" if prec == F64 else "f32")
        opts, keep = make_opts(32, protect, tau_scale, faults, graph=graph, wgs_per_cu=wgs_per_cu)
        op = OP_POTRF_BATCHED if chol else OP_GETRF_BATCHED
        ws, wbytes = self.workspace(op, 0, opts, batch=batch)
        nm = int(nmax if nmax is not None else max(m.shape[0] for m in mats))
        self._sync_stream()
        if chol:
            rc = lib().abft_potrf_batched(self._h, batch, nm, ns.data_ptr(), ptrs.data_ptr(), ldas.data_ptr(), prec,
                                          ws.data_ptr(), wbytes, C.byref(opts), infos.data_ptr(), reps.data_ptr())
        else:
            rc = lib().abft_getrf_batched(self._h, batch, nm, ns.data_ptr(), ptrs.data_ptr(), ldas.data_ptr(),
                                          piv_ptrs.data_ptr(), prec, ws.data_ptr(), wbytes, C.byref(opts),
                                          infos.data_ptr(), reps.data_ptr())
        del keep
        _check(rc, "abft_batched")
        if not sync:
            return state
        torch.cuda.synchronize(self.device)
        rsz = C.sizeof(Report)
        raw = reps.cpu().numpy().tobytes()
        reports = [Report.from_buffer_copy(raw[i * rsz:(i + 1) * rsz]) for i in range(batch)]
        return infos.cpu().numpy(), ipivs, reports

    def batched_args(self, mats, chol):
        torch = self.torch
        dev = self.device
        ns = torch.tensor([m.shape[0] for m in mats], dtype=torch.int32, device=dev)
        ptrs = torch.tensor([m.data_ptr() for m in mats], dtype=torch.int64, device=dev)
        ldas = torch.tensor([_ld(m) for m in mats], dtype=torch.int32, device=dev)
        ipivs = None if chol else [torch.zeros(max(m.shape[0], 1), dtype=torch.int32, device=dev) for m in mats]
        piv_ptrs = None if chol else torch.tensor([p.data_ptr() for p in ipivs], dtype=torch.int64, device=dev)
        infos = torch.zeros(len(mats), dtype=torch.int32, device=dev)
        reps = torch.zeros(len(mats) * C.sizeof(Report), dtype=torch.uint8, device=dev)
        return ns, ptrs, ldas, ipivs, piv_ptrs, infos, reps

    # ------------------------------------------------------------ update primitive
    def gemm(self, A, B, C, transa=False, transb=False, alpha=1.0, beta=0.0, lower=False, unit_lower_a=False,
             work=None):
        """C = beta*C + alpha*op(A)*op(B) on column-major FP64 tensors (abft_gemm)."""
        m, n = C.shape
        k = A.shape[0] if transa else A.shape[1]
        flags = (GEMM_LOWER if lower else 0) | (GEMM_UNIT_LOWER_A if unit_lower_a else 0)
        self._sync_stream()
        _check(lib().abft_gemm(self._h, int(bool(transa)), int(bool(transb)), flags, m, n, k, float(alpha),
                               A.data_ptr(), _ld(A), B.data_ptr(), _ld(B), float(beta), C.data_ptr(), _ld(C),
                               work.data_ptr() if work is not None else None,
                               work.numel() * work.element_size() if work is not None else 0), "abft_gemm")
        return C

    # ------------------------------------------------------------ checksums
    def encode(self, A, nb):
        torch = self.torch
        m, n = A.shape
        Tr, Tc = -(-m // nb), -(-n // nb)
        colchk = colmajor(torch.zeros((2 * Tr, n), dtype=torch.float64, device=self.device))
        rowchk = colmajor(torch.zeros((m, 2 * Tc), dtype=torch.float64, device=self.device))
        self._sync_stream()
        _check(lib().abft_encode(self._h, m, n, A.data_ptr(), _ld(A), nb, colchk.data_ptr(), _ld(colchk),
                                 rowchk.data_ptr(), _ld(rowchk)), "abft_encode")
        return colchk, rowchk

    def verify(self, A, nb, colchk, rowchk, tau_scale=4.0, correct=False):
        torch = self.torch
        m, n = A.shape
        Tr, Tc = -(-m // nb), -(-n // nb)
        flags = colmajor(torch.zeros((Tr, Tc), dtype=torch.int32, device=self.device))
        rep = self.new_report()
        self._sync_stream()
        _check(lib().abft_verify(self._h, m, n, A.data_ptr(), _ld(A), nb, colchk.data_ptr(), _ld(colchk),
                                 rowchk.data_ptr(), _ld(rowchk), tau_scale, int(bool(correct)), flags.data_ptr(),
                                 rep.data_ptr()), "abft_verify")
        torch.cuda.synchronize(self.device)
        return flags, self.read_report(rep)
