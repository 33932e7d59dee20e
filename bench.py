#!/usr/bin/env python3
"""Benchmark of the ABFT-protected one-sided decompositions on one MI355X.

One step = one pass of the hot path over synthetic inputs resident in HBM:

* FP64 legs (the headline): ABFT-protected Cholesky, LU (partial pivoting)
  and Householder QR of an n x n matrix (default n = 32768, nb = 512; SPD
  A = G G^T/n + n I for Cholesky, U(-1,1) entries for LU and QR), full
  row + column checksums verified every iteration.  Each factorization works
  in place, so it first restores its matrix from a pristine device copy (a
  device-to-device copy outside the leg's timed events).
* Mixed-precision leg: A x = b at n = 16384 (A = Q diag(s) Q^T, kappa 1e2),
  FP64 direct solve against binary32 / bf16 / fp16 trailing updates with FP64
  iterative refinement, LU and Cholesky; speedup at forward error <= 1e-12
  against the closed-form solution.
* Batched leg: 4096 matrices of orders uniform on [32, 512], ABFT Cholesky
  and LU in FP64 and FP32, one library call each, replayed from the HIP graph
  the library captured on first use.

Prints ONE JSON line.  `value` is the useful FP64 TFLOP/s of the three
FP64 legs (n^3/3 + 2n^3/3 + 4n^3/3 per step over their timed duration);
`roofline` is the FP64 trailing-update product (flops per launch / average
launch time, both measured by the library with HIP events on its stream);
`cpu_baseline` is the plain CPU oracle on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(n=8192, nb=512):
    """The plain CPU oracle (as it stands, OpenMP over independent elements
    on every host core) on a bounded sample of the workload: the three ABFT
    decompositions of an n x n matrix, useful TFLOP/s; the time of the
    full-size (n = 32768) step is extrapolated from it by n^3 and labelled
    as such."""
    import platform
    import oracle
    from paper_2301_03166_amd import gen
    A = gen.spd(n, 11)
    B = gen.general(n, 12)
    Cm = gen.general(n, 13)
    threads = oracle.get_threads()
    t = time.perf_counter()
    oracle.potrf(A, nb)
    oracle.getrf(B, nb)
    oracle.geqrf(Cm, nb)
    dt = time.perf_counter() - t
    flops = 7.0 * n ** 3 / 3.0
    return {"value": flops / dt / 1e12, "unit": "TFLOP/s", "cores": threads, "kind": "oracle",
            "sample": f"ABFT Cholesky+LU+QR, n={n}, nb={nb}, one run each ({dt:.1f} s on {threads} threads, "
                      f"{platform.processor() or platform.machine()})",
            "extrapolated_step_s_n32768": dt * (32768.0 / n) ** 3}


def ipiv_perm(ipiv):
    """Row order p with (P A) = A[p] for LAPACK 1-based interchanges."""
    import numpy as np
    piv = np.asarray(ipiv, dtype=np.int64) - 1
    p = np.arange(len(piv))
    for j, q in enumerate(piv):
        p[j], p[q] = p[q], p[j]
    return p


def _qr_blocks(F, tau, Y, transpose, block=512):
    """Y := Q^T Y (transpose) or Q Y with Q = H_0 ... H_{n-1} from the geqrf
    storage F / tau, one compact-WY block at a time.  The block's T comes from
    T^{-1} = strict_upper(V^T V) + diag(1 / tau) (valid for nonzero tau)."""
    import torch
    n = F.shape[0]
    starts = list(range(0, n, block))
    for c0 in (starts if transpose else starts[::-1]):
        c1 = min(n, c0 + block)
        V = torch.tril(F[c0:, c0:c1], diagonal=-1)
        V.diagonal().fill_(1.0)
        t = tau[c0:c1]
        Tinv = torch.triu(V.T @ V, diagonal=1)
        Tinv.diagonal().copy_(1.0 / t)
        Z = V.T @ Y[c0:]
        if transpose:  # T^T Z: solve Tinv^T W = Z
            Wv = torch.linalg.solve_triangular(Tinv.T.contiguous(), Z, upper=False)
        else:
            Wv = torch.linalg.solve_triangular(Tinv, Z, upper=True)
        Y[c0:] -= V @ Wv
    return Y


def backward_error(kind, A0, F, aux=None, probes=8, seed=0):
    """Normwise relative backward error ||E||_F / ||A||_F of a factorization,
    with E = A - L L^T (chol), P A - L U (lu) or Q^T A - R (qr) formed densely
    by FP64 products on the device (the evaluation LAPACK's test drivers use).
    A0 and F are n x n column-major FP64 tensors (the input and the factored
    matrix); aux is ipiv (lu) or tau (qr).  For qr the second value estimates
    ||I - Q^T Q||_F / sqrt(n) with Gaussian probes x ~ N(0, I) (E ||M x||^2 =
    ||M||_F^2, averaged over `probes` columns)."""
    import torch
    n = A0.shape[0]
    orth = None
    if kind == "chol":
        L = torch.tril(F)
        E = A0.clone()
        E.addmm_(L, L.T, alpha=-1.0)
        del L
    elif kind == "lu":
        p = torch.from_numpy(ipiv_perm(aux.cpu().numpy())).to(A0.device)
        L = torch.tril(F, diagonal=-1)
        L.diagonal().fill_(1.0)
        U = torch.triu(F)
        E = A0[p]
        E.addmm_(L, U, alpha=-1.0)
        del L, U
    else:
        tau = aux
        E = _qr_blocks(F, tau, A0.clone(), transpose=True)
        E -= torch.triu(F)
        g = torch.Generator(device=A0.device).manual_seed(seed)
        X = torch.randn((n, probes), generator=g, dtype=torch.float64, device=A0.device)
        Q = _qr_blocks(F, tau, _qr_blocks(F, tau, X.clone(), transpose=False), transpose=True)
        orth = float(torch.linalg.norm(Q - X) / probes ** 0.5 / n ** 0.5)
    be = float(torch.linalg.norm(E) / torch.linalg.norm(A0))
    del E
    return be, orth


def fp64_legs(h, torch, dev, args, legs):
    from paper_2301_03166_amd import gen
    n, nb = args.n, args.nb
    log(f"generating FP64 inputs n={n}")
    pristine = {}
    if "chol" in legs:
        pristine["chol"] = gen.spd_torch(n, 11, dev)
    if "lu" in legs:
        pristine["lu"] = gen.general_torch(n, 12, dev)
    if "qr" in legs:
        pristine["qr"] = gen.general_torch(n, 13, dev)
    work = torch.empty((n, n), dtype=torch.float64, device=dev)
    ipiv = torch.zeros(n, dtype=torch.int32, device=dev)
    tau = torch.zeros(n, dtype=torch.float64, device=dev)
    reports = {k: h.new_report() for k in legs}
    infos = {k: torch.zeros(1, dtype=torch.int32, device=dev) for k in legs}
    flops = {"chol": n ** 3 / 3.0, "lu": 2.0 * n ** 3 / 3.0, "qr": 4.0 * n ** 3 / 3.0}
    ev = {k: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for k in legs}
    leg_ms = {k: [] for k in legs}
    prof_acc = {}
    profile = not args.no_profile

    def run(k, protect=True, prof=False):
        A = work.t()  # column-major view of the row-major buffer
        A.copy_(pristine[k].t())
        e0, e1 = ev[k]
        e0.record()
        kw = dict(protect=protect, report=reports[k], info=infos[k], sync=False, profile=prof,
                  overlap=bool(args.overlap))
        if k == "chol":
            h.potrf(A, nb, **kw)
        elif k == "lu":
            h.getrf(A, nb, ipiv=ipiv, **kw)
        else:
            h.geqrf(A, nb, tau=tau, **kw)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    log(f"FP64 warmup x{args.warmup}")
    for _ in range(args.warmup):
        for k in legs:
            run(k)
    status = {k: None for k in legs}
    for s in range(args.steps):
        for k in legs:
            leg_ms[k].append(run(k))
            rep = h.read_report(reports[k])
            st = {"info": int(infos[k].item()), "abft_status": rep.status, "flagged_tiles": rep.flagged_tiles,
                  "max_ratio": rep.max_ratio}
            if status[k] is None or st["abft_status"] or st["info"]:
                status[k] = st
        log(f"FP64 step {s}: " + ", ".join(f"{k} {leg_ms[k][-1]:.1f} ms" for k in legs))
    # backward error of each leg's factors (one more untimed run per leg,
    # residual formed densely on the device, see backward_error)
    if not args.no_check:
        for k in legs:
            run(k)
            be, orth = backward_error(k, pristine[k].t(), work.t(),
                                      ipiv if k == "lu" else (tau if k == "qr" else None))
            status[k]["backward_error"] = be
            status[k]["backward_error_over_nu"] = be / (n * 2.0 ** -53)
            if orth is not None:
                status[k]["orthogonality"] = orth
            log(f"{k}: backward error {be:.2e}" + (f", orthogonality {orth:.2e}" if orth is not None else ""))
    # phase profile (separate run per leg: the profiled call waits on its own events)
    if profile:
        for k in legs:
            run(k, prof=True)
            p = h.profile()
            prof_acc[k] = {f: p[f] for f in ("ms_total", "ms_panel", "ms_tmu", "ms_carry", "ms_verify", "tmu_flops",
                                             "tmu_launches", "verify_bytes")}
            from paper_2301_03166_amd import timemodel
            prof_acc[k]["time_model"] = timemodel.validate(h.iter_profile(), k, n, nb)
    unprot = {}
    if not args.no_overhead:
        for k in legs:
            unprot[k] = run(k, protect=False)
        log("unprotected: " + ", ".join(f"{k} {unprot[k]:.1f} ms" for k in legs))
    del work, pristine
    torch.cuda.empty_cache()
    per_leg = {}
    for k in legs:
        ms = sum(leg_ms[k]) / len(leg_ms[k])
        d = {"ms": ms, "tflops": flops[k] / ms / 1e9, "frac_fp64_peak": flops[k] / ms / 1e9 / FP64_PEAK_TFLOPS}
        if k in unprot:
            d["ms_unprotected"] = unprot[k]
            d["checksum_overhead_pct"] = 100.0 * (ms - unprot[k]) / unprot[k]
        if k in prof_acc:
            a = prof_acc[k]
            d.update({"ms_panel": a["ms_panel"], "ms_tmu": a["ms_tmu"], "ms_carry": a["ms_carry"],
                      "ms_verify": a["ms_verify"],
                      "tmu_tflops": a["tmu_flops"] / a["ms_tmu"] / 1e9 if a["ms_tmu"] > 0 else None,
                      "verify_gbs": a["verify_bytes"] / a["ms_verify"] / 1e6 if a["ms_verify"] > 0 else None,
                      "time_model_prediction_error": a["time_model"]})
        per_leg[k] = d
    total_ms = sum(sum(leg_ms[k]) for k in legs)
    value = sum(flops[k] for k in legs) * args.steps / total_ms / 1e9
    roof = None
    if prof_acc:
        ms = sum(a["ms_tmu"] for a in prof_acc.values())
        fl = sum(a["tmu_flops"] for a in prof_acc.values())
        launches = sum(a["tmu_launches"] for a in prof_acc.values())
        achieved = fl / ms / 1e9 if ms > 0 else None
        roof = {"bound": "mfma", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / FP64_PEAK_TFLOPS if achieved else None, "traffic": measured_traffic(),
                "kernel": "k_dgemm (FP64 trailing-matrix update products)", "launches": launches,
                "avg_launch_ms": ms / launches if launches else None,
                "flops_per_launch": fl / launches if launches else None}
    return value, total_ms / args.steps, per_leg, status, roof


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_dgemm_tmu_traffic_n32768_nb512.md")
DGEMM_SRC = os.path.join(ROOT, "paper_2301_03166_amd", "csrc", "dgemm.hip")


def measured_traffic():
    """HBM bytes per trailing-update launch from the committed counter
    summary (FETCH_SIZE + WRITE_SIZE, calibrated), or None when the product
    kernel's source has changed since the counters were taken."""
    import hashlib
    try:
        kv = {}
        with open(TRAFFIC_FILE) as f:
            for line in f:
                if "=" in line and line.strip().startswith(("source_sha256", "traffic_bytes_per_launch")):
                    k, v = line.split("=", 1)
                    kv[k.strip()] = v.strip().strip("`")
        with open(DGEMM_SRC, "rb") as f:
            cur = hashlib.sha256(f.read()).hexdigest()
        if kv.get("source_sha256") != cur:
            return None
        return float(kv["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def mp_leg(h, torch, dev, args):
    """Mixed-precision solves at each condition number: the FP64 direct solve
    and binary32 / bf16 / fp16 trailing updates with FP64 refinement, LU and
    Cholesky, forward error against the generator's closed-form solution.
    The speedup is quoted at kappa = 1e2 (the forward-error target 1e-12 is
    reachable there; at larger kappa FP64 itself ends near kappa u, so a
    refined solve counts as accurate when it is within 2x of the FP64 solve's
    error, and a failure to converge is reported as such)."""
    import numpy as np
    from paper_2301_03166_amd import abft, gen
    n, nb = args.mp_n, args.mp_nb
    precs = [("f64", abft.F64), ("f32", abft.F32), ("bf16", abft.BF16), ("f16", abft.F16)]
    kappas = [float(k) for k in args.mp_kappas.split(",")]
    per_kappa = {}
    for kappa in kappas:
        log(f"generating MP input n={n} kappa={kappa:g}")
        A, s, V = gen.mp_torch(n, kappa, 21, dev)
        A = A.t()  # symmetric: the same values, column-major view
        b_h = gen.rhs(n, 24)
        b = torch.from_numpy(b_h).to(dev)
        xs = gen.mp_exact_solution(b_h, s, V)
        out = {}
        reps = max(1, min(args.steps, 5))
        for chol in (False, True):
            kind = "chol" if chol else "lu"
            res = {}
            for name, p in precs:
                x = torch.zeros(n, dtype=torch.float64, device=dev)
                h.gesv_mp(A, b, p, nb=nb, chol=chol, x=x)  # warmup
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                times = []
                for _ in range(reps):
                    e0.record()
                    x, ir, rep = h.gesv_mp(A, b, p, nb=nb, chol=chol, x=x)
                    e1.record()
                    torch.cuda.synchronize()
                    times.append(e0.elapsed_time(e1))
                err = float(np.linalg.norm(x.cpu().numpy() - xs, np.inf) / np.linalg.norm(xs, np.inf))
                res[name] = {"ms": sum(times) / len(times), "forward_error": err, "ir_iters": int(ir.iters),
                             "converged": bool(ir.converged) if p != abft.F64 else True,
                             "failed_reason": int(ir.failed_reason), "factor_info": int(ir.info),
                             "abft_status": rep.status}
            base = res["f64"]["ms"]
            target = 1e-12 if kappa <= 1e2 else 2.0 * res["f64"]["forward_error"]
            for k in ("f32", "bf16", "f16"):
                res[k]["accurate"] = bool(res[k]["converged"] and res[k]["forward_error"] <= target)
            ok = [k for k in ("f32", "bf16", "f16") if res[k]["accurate"]]
            best = min(ok, key=lambda k: res[k]["ms"]) if ok else None
            out[kind] = {"solves": res, "target_forward_error": target, "best": best,
                         "speedup_vs_fp64": base / res[best]["ms"] if best else None}
            log(f"MP {kind} kappa {kappa:g}: " + ", ".join(
                f"{k} {v['ms']:.1f} ms err {v['forward_error']:.1e}" + ("" if v["converged"] else " (no conv.)")
                for k, v in res.items()))
        del A, b
        torch.cuda.empty_cache()
        per_kappa[f"{kappa:g}"] = out
    head = per_kappa.get("100", next(iter(per_kappa.values())))
    sp = [v["speedup_vs_fp64"] for v in head.values() if v["speedup_vs_fp64"]]
    return {"n": n, "nb": nb, "kappa_headline": 1e2, "target_forward_error": 1e-12,
            "speedup_vs_fp64": min(sp) if len(sp) == 2 else None, "lu": head["lu"], "chol": head["chol"],
            "by_kappa": per_kappa}


def batched_leg(h, torch, dev, args):
    import numpy as np
    from paper_2301_03166_amd import gen
    cnt = args.batch
    sizes = gen.batch_sizes(cnt, 32, 512, 31)
    seeds = gen.batch_seeds(cnt, 31)
    out = {}
    for kind in ("chol", "lu"):
        chol = kind == "chol"
        for dname, dt in (("f64", torch.float64), ("f32", torch.float32)):
            log(f"generating batched {kind} {dname}")
            pristine, _ = gen.batch_torch(sizes, seeds, kind, dev, dtype=dt)
            flat = torch.empty_like(pristine)
            offs = np.concatenate([[0], np.cumsum(sizes.astype(np.int64) ** 2)])
            views = [torch.as_strided(flat, (int(nn), int(nn)), (1, int(nn)), int(offs[q]))
                     for q, nn in enumerate(sizes)]
            state = h.batched_args(views, chol)
            flat.copy_(pristine)
            h.batched(views, chol, state=state, graph=True, sync=False)  # capture + first replay
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            times = []
            for _ in range(max(3, args.steps)):
                flat.copy_(pristine)
                e0.record()
                h.batched(views, chol, state=state, graph=True, sync=False)
                e1.record()
                torch.cuda.synchronize()
                times.append(e0.elapsed_time(e1))
            infos = state[5].cpu().numpy()
            raw = state[6].cpu().numpy().tobytes()
            from paper_2301_03166_amd.abft import Report
            import ctypes
            rsz = ctypes.sizeof(Report)
            flagged = sum(1 for q in range(cnt) if Report.from_buffer_copy(raw[q * rsz:(q + 1) * rsz]).status)
            fl = float(np.sum(sizes.astype(np.float64) ** 3)) * (1.0 / 3.0 if chol else 2.0 / 3.0)
            ms = float(np.median(times))
            out[f"{kind}_{dname}"] = {"ms": ms, "tflops": fl / ms / 1e9, "min_ms": min(times),
                                      "info_nonzero": int(np.count_nonzero(infos)), "abft_flagged": flagged}
            log(f"batched {kind} {dname}: {ms:.2f} ms {fl / ms / 1e9:.2f} TFLOP/s")
            if args.batch_faults:
                out[f"{kind}_{dname}"]["faults"] = batched_faults(h, torch, gen, kind, dname, sizes, flat, pristine,
                                                                  views, state)
            del pristine, flat, views, state
            torch.cuda.empty_cache()
    return {"matrices": cnt, "orders": "uniform on [32, 512]", "graph": True, "legs": out}


def batched_faults(h, torch, gen, kind, dname, sizes, flat, pristine, views, state):
    """One untimed batched call with one seeded single-bit flip in each of
    len(sizes) / 64 matrices (chosen without replacement among those with a
    trailing matrix, n > 32): outcomes against the clean factors of the
    timed calls (equal to the precision's rounding, or, where pivots moved,
    a backward error within 2x of the clean factors'), and every other
    matrix must come out bitwise unchanged."""
    import numpy as np
    from paper_2301_03166_amd.abft import Report
    import ctypes
    chol = kind == "chol"
    clean = flat.clone()
    clean_piv = None if chol else [p.clone() for p in state[3]]
    r = gen.rng(64 + (0 if chol else 1) + (0 if dname == "f64" else 2))
    cand = np.flatnonzero(np.asarray(sizes) > 32)
    pick = np.sort(r.choice(cand, size=len(sizes) // 64, replace=False))
    faults = []
    for q in pick:
        f = gen.fault_plan(kind, int(sizes[q]), 32, seed=int(r.integers(0, 2 ** 31)))
        if dname == "f32":
            f["bit"] = int(f["bit"]) % 32
        f["matrix"] = int(q)
        faults.append(f)
    flat.copy_(pristine)
    h.batched(views, chol, state=state, faults=faults, sync=True)
    raw = state[6].cpu().numpy().tobytes()
    rsz = ctypes.sizeof(Report)
    tol = 1e-12 if dname == "f64" else 1e-5
    tally = {"flips": len(faults), "corrected": 0, "checksum_repaired": 0, "uncorrectable": 0,
             "undetected_harmless": 0, "undetected_corrupting": 0, "corrected_but_wrong": 0,
             "other_matrices_changed": 0, "results_within_backward_error": 0,
             "significant_flips": 0, "significant_detected": 0, "subthreshold_flips": 0, "subthreshold_detected": 0,
             "unverified_flips": 0, "max_undetected_delta_over_tau": 0.0}
    fset = {f["matrix"]: f for f in faults}
    for q, v in enumerate(views):
        rep = Report.from_buffer_copy(raw[q * rsz:(q + 1) * rsz])
        cv = torch.as_strided(clean, v.shape, v.stride(), v.storage_offset())
        g, c = (torch.tril(v), torch.tril(cv)) if chol else (v, cv)
        if q not in fset:
            tally["other_matrices_changed"] += int(rep.status != 0 or not torch.equal(g, c))
            continue
        same = float((g - c).abs().max()) <= tol * float(c.abs().max())
        if not same:
            # partial pivoting may pick the other of two near-equal pivots after
            # a flip or a rebuild known to rounding: then the factors differ but
            # are as good, judged by the backward error against the clean run's
            A0 = torch.as_strided(pristine, v.shape, v.stride(), v.storage_offset()).double()
            bf, _ = backward_error(kind, A0, v.double(), None if chol else state[3][q])
            bc, _ = backward_error(kind, A0, cv.double(), None if chol else clean_piv[q])
            same = bf <= 2.0 * bc
            tally["results_within_backward_error"] += int(same)
        if rep.status & 4:
            tally["uncorrectable"] += 1
        elif rep.status & 1:
            tally["corrected"] += 1
            tally["corrected_but_wrong"] += int(not same)
        elif rep.status & 2:
            tally["checksum_repaired"] += 1
        else:
            tally["undetected_harmless" if same else "undetected_corrupting"] += 1
        # |delta| / tau of the flip against its column checksum's threshold
        # (tau < 0: the flip was not verified), as in the fault campaign
        detected = bool(rep.status & 7)
        ratio = rep.fault_delta / rep.fault_tau if rep.fault_tau > 0 else (math.inf if rep.fault_tau == 0 else None)
        if ratio is None:
            tally["unverified_flips"] += 1
        else:
            sig = ratio > 1.0
            tally["significant_flips" if sig else "subthreshold_flips"] += 1
            tally["significant_detected" if sig else "subthreshold_detected"] += int(detected)
            if not detected:
                tally["max_undetected_delta_over_tau"] = max(tally["max_undetected_delta_over_tau"], ratio)
    tally["significant_detected_pct"] = (100.0 * tally["significant_detected"] / tally["significant_flips"]
                                         if tally["significant_flips"] else None)
    del clean
    log(f"batched {kind} {dname} faults: {tally}")
    return tally


class PowerSampler:
    """Board power sampled in a thread through the amdsmi library (socket
    power, W).  Any failure leaves the sampler disabled (energy: null)."""

    def __init__(self, period=0.02):
        self.period, self.samples, self.ok, self._stop = period, [], False, None
        try:
            import amdsmi
            amdsmi.amdsmi_init()
            self._smi = amdsmi
            self._h = amdsmi.amdsmi_get_processor_handles()[0]
            self.read()
            self.ok = True
        except Exception as e:  # no library, no permission, no device
            log(f"power sampling unavailable: {e}")

    def read(self):
        info = self._smi.amdsmi_get_power_info(self._h)
        for key in ("current_socket_power", "socket_power", "average_socket_power"):
            v = info.get(key) if isinstance(info, dict) else None
            if isinstance(v, (int, float)) and v > 0:
                return float(v)
        raise RuntimeError(f"no socket power in {info}")

    def start(self):
        import threading
        self.samples = []
        self._stop = threading.Event()

        def loop():
            while not self._stop.is_set():
                try:
                    self.samples.append((time.perf_counter(), self.read()))
                except Exception:
                    pass
                time.sleep(self.period)
        self._t = threading.Thread(target=loop, daemon=True)
        self._t.start()

    def stop(self):
        self._stop.set()
        self._t.join(timeout=2)
        return list(self.samples)


def energy_leg(h, torch, dev, args):
    """Energy per factorization: repeated ABFT LU factorizations for >= 2 s
    with board power sampled meanwhile; gross and above the idle level."""
    from paper_2301_03166_amd import gen
    ps = PowerSampler()
    if not ps.ok:
        return None
    n, nb = args.energy_n, args.nb
    A0 = gen.general_torch(n, 12, dev)
    W = torch.empty_like(A0)
    ipiv = torch.zeros(n, dtype=torch.int32, device=dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    rep = h.new_report()
    # idle level: let the board settle after the previous legs (the reported
    # power trails the load), then take the median of two seconds of samples
    torch.cuda.synchronize()
    time.sleep(4.0)
    ps.start()
    time.sleep(2.0)
    idle = ps.stop()
    reps, t0 = 0, time.perf_counter()
    ps.start()
    while time.perf_counter() - t0 < 2.5 or reps < 3:
        W.copy_(A0)
        h.getrf(W.t(), nb, ipiv=ipiv, report=rep, info=info, sync=False)
        torch.cuda.synchronize()
        reps += 1
    t1 = time.perf_counter()
    busy = ps.stop()
    del A0, W
    torch.cuda.empty_cache()
    if len(busy) < 10 or not idle:
        return None
    p_idle = sorted(p for _, p in idle)[len(idle) // 2]
    joules = 0.0
    for (ta, pa), (tb, pb) in zip(busy[:-1], busy[1:]):
        joules += 0.5 * (pa + pb) * (tb - ta)
    span = busy[-1][0] - busy[0][0]
    per = joules / reps * (t1 - t0) / span if span > 0 else None
    return {"workload": f"ABFT LU n={n} nb={nb} (includes the device copy that restores A)", "repetitions": reps,
            "seconds": t1 - t0, "sample_period_s": ps.period, "samples": len(busy), "avg_power_w":
            sum(p for _, p in busy) / len(busy), "idle_power_w": p_idle, "joules_per_factorization": per,
            "joules_above_idle_per_factorization": (per - p_idle * (t1 - t0) / reps) if per else None}


def campaign_leg(h, torch, dev, args):
    """Seeded single-bit fault campaign.  For each decomposition, pairs
    r = 0 .. R/2 - 1 of runs on their own seeded matrix: a clean run (false
    alarms are counted over these distinct matrices) and a run with one flip
    (uniform iteration, stored trailing element and bit 0..63, seeded per
    pair).

    Each flip is classified by the size of the change it made, |delta| (the
    library records it when it plants the flip), against tau, the threshold
    of the column checksum that covers the element at the verification right
    after the flip (also recorded).  A flip with |delta| > tau must be
    detected; below tau it is at the level of the checksums' rounding and may
    pass, which is harmless when the result stays as accurate as the clean
    one.  A faulted run's result is correct when its factors equal the clean
    run's to 1e-12 (relative, max norm) or, failing that (a rebuilt element
    is only known to its column's rounding, and partial pivoting can then
    pick a different one of two near-equal pivots), when its backward error
    is within 2x of the clean run's.  The campaign stops at the first call
    that reports a cooperative-kernel wait expiry."""
    import math
    from paper_2301_03166_amd import gen
    n, nb, R = args.campaign_n, args.campaign_nb, args.campaign
    classes = (("sign_exponent_52_63", 52, 64), ("mantissa_40_51", 40, 52), ("mantissa_20_39", 20, 40),
               ("mantissa_0_19", 0, 20))
    out = {}
    for d, kind in enumerate(("chol", "lu", "qr")):
        ref = torch.empty((n, n), dtype=torch.float64, device=dev)
        W = torch.empty_like(ref)
        adt = torch.float64 if kind == "qr" else torch.int32
        aux_ref, aux_f = torch.zeros(n, dtype=adt, device=dev), torch.zeros(n, dtype=adt, device=dev)

        def run(A0, dst, faults, aux):
            dst.copy_(A0)
            A = dst.t()
            if kind == "chol":
                info, rep = h.potrf(A, nb, faults=faults)
            elif kind == "lu":
                _, info, rep = h.getrf(A, nb, faults=faults, ipiv=aux)
            else:
                _, info, rep = h.geqrf(A, nb, faults=faults, tau=aux)
            return rep

        tally = {"clean_runs": 0, "false_alarms": 0, "faulted_runs": 0, "corrected": 0, "checksum_repaired": 0,
                 "uncorrectable": 0, "undetected": 0, "results_equal_clean": 0, "results_within_backward_error": 0,
                 "results_wrong": 0, "internal_errors": 0, "significant_flips": 0, "significant_detected": 0,
                 "subthreshold_flips": 0, "subthreshold_detected": 0, "unverified_flips": 0}
        by_class = {c[0]: {"flips": 0, "detected": 0, "significant": 0, "significant_detected": 0}
                    for c in classes}
        undetected, uncorrectable = [], []
        min_detected_ratio, max_undetected_ratio = math.inf, 0.0
        for r in range(max(1, R // 2)):
            seed = 100000 * (d + 1) + r
            A0 = gen.spd_torch(n, seed, dev) if kind == "chol" else gen.general_torch(n, seed, dev)
            rep = run(A0, ref, None, aux_ref)
            tally["clean_runs"] += 1
            tally["false_alarms"] += int(rep.status != 0)
            if rep.status & 16:
                tally["internal_errors"] += 1
                break
            f = gen.fault_plan(kind, n, nb, seed=10 ** 6 * (d + 1) + r)
            rep = run(A0, W, [f], aux_f)
            if rep.status & 16:
                tally["internal_errors"] += 1
                break
            ref_t, Wt = ref.t(), W.t()
            scale = float(ref_t.abs().max())
            diff = float((torch.tril(Wt - ref_t) if kind == "chol" else (Wt - ref_t)).abs().max())
            tally["faulted_runs"] += 1
            if diff <= 1e-12 * scale:
                tally["results_equal_clean"] += 1
            else:
                bf, _ = backward_error(kind, A0.t(), Wt, None if kind == "chol" else aux_f)
                bc, _ = backward_error(kind, A0.t(), ref_t, None if kind == "chol" else aux_ref)
                tally["results_within_backward_error" if bf <= 2.0 * bc else "results_wrong"] += 1
            detected = bool(rep.status & 7)
            if rep.status & 4:
                tally["uncorrectable"] += 1
            elif rep.status & 1:
                tally["corrected"] += 1
            elif rep.status & 2:
                tally["checksum_repaired"] += 1
            else:
                tally["undetected"] += 1
            # |delta| / tau of this flip (tau < 0: the flip was not verified)
            ratio = rep.fault_delta / rep.fault_tau if rep.fault_tau > 0 else (math.inf if rep.fault_tau == 0 else None)
            if ratio is None:
                tally["unverified_flips"] += 1
            else:
                sig = ratio > 1.0
                tally["significant_flips" if sig else "subthreshold_flips"] += 1
                tally["significant_detected" if sig else "subthreshold_detected"] += int(detected)
                if detected:
                    min_detected_ratio = min(min_detected_ratio, ratio)
                else:
                    max_undetected_ratio = max(max_undetected_ratio, ratio)
            if not detected:
                undetected.append({"bit": int(f["bit"]), "delta_over_tau": ratio})
            if rep.status & 4:
                uncorrectable.append({"pair": r, "plan": {k: int(v) for k, v in f.items()}, "delta_over_tau": ratio})
            for name, lo, hi in classes:
                if lo <= f["bit"] < hi:
                    c = by_class[name]
                    c["flips"] += 1
                    c["detected"] += int(detected)
                    if ratio is not None and ratio > 1.0:
                        c["significant"] += 1
                        c["significant_detected"] += int(detected)
            del A0
            if r % 100 == 99:
                log(f"campaign {kind}: {r + 1} pairs")
        fr = max(1, tally["faulted_runs"])
        tally["detected_pct"] = 100.0 * (fr - tally["undetected"]) / fr
        tally["significant_detected_pct"] = (100.0 * tally["significant_detected"] / tally["significant_flips"]
                                             if tally["significant_flips"] else None)
        tally["correct_result_pct"] = 100.0 * (tally["results_equal_clean"] +
                                               tally["results_within_backward_error"]) / fr
        tally["min_detected_delta_over_tau"] = min_detected_ratio if min_detected_ratio < math.inf else None
        tally["max_undetected_delta_over_tau"] = max_undetected_ratio
        for c in by_class.values():
            c["detected_pct"] = 100.0 * c["detected"] / c["flips"] if c["flips"] else None
        tally["by_bit_class"] = by_class
        tally["undetected_flips"] = sorted(undetected, key=lambda e: e["bit"])
        tally["uncorrectable_flips"] = uncorrectable
        out[kind] = tally
        log(f"campaign {kind}: " + json.dumps({k: v for k, v in tally.items()
                                               if k not in ("by_bit_class", "undetected_flips", "uncorrectable_flips")}))
        del ref, W
        torch.cuda.empty_cache()
    return {"n": n, "nb": nb, "runs_per_decomposition": 2 * max(1, R // 2),
            "plan": "pairs of runs on one seeded matrix each: clean, then one flip (iteration, stored trailing "
                    "element and bit 0..63 uniform, seeded per pair) compared with the clean factors",
            "significant": "|delta| > tau of the element's column checksum at the verification after the flip",
            "outcomes": out}


def gemm_leg(h, torch, dev, args):
    """The trailing-update product alone on its first-iteration shapes
    (m' = n - nb, K = nb): LU's C -= L21 U12 (NN), Cholesky's lower
    C -= L21 L21^T (NT, lower tiles only) and QR's W = V^T C (TN, K = n) and
    C -= V W2 (NN), each timed over `reps` launches with HIP events."""
    n, nb = args.n, args.nb
    m = n - nb
    g = torch.Generator(device=dev).manual_seed(5)
    A = torch.randn((n, nb), dtype=torch.float64, device=dev, generator=g).t().contiguous().t()  # n x nb col-major
    B = torch.randn((nb, n), dtype=torch.float64, device=dev, generator=g).t().contiguous().t()  # nb x n col-major
    Cm = torch.randn((n, n), dtype=torch.float64, device=dev, generator=g).t()  # col-major n x n
    W = torch.zeros((nb, m), dtype=torch.float64, device=dev).t().contiguous().t()
    out = {}
    cases = {
        "lu_nn": (lambda: h.gemm(A[:m], B[:, :m], Cm[:m, :m], alpha=-1.0, beta=1.0), 2.0 * m * m * nb),
        "chol_nt_lower": (lambda: h.gemm(A[:m], A[:m], Cm[:m, :m], transb=True, alpha=-1.0, beta=1.0, lower=True),
                          1.0 * m * (m + 1) * nb),
        "qr_tn": (lambda: h.gemm(A, Cm[:, :m], W, transa=True, alpha=1.0, beta=0.0), 2.0 * nb * m * n),
        "qr_nn": (lambda: h.gemm(A, W, Cm[:, :m], alpha=-1.0, beta=1.0), 2.0 * n * m * nb),
    }
    # a plain device copy of known size (n x n FP64 read and written once):
    # the reference for scaling the HBM traffic counters of the products
    Cc = torch.empty_like(Cm)
    cases["copy_ref"] = (lambda: Cc.copy_(Cm), 0.0)
    for name, (fn, fl) in cases.items():
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.gemm_reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.gemm_reps
        if name == "copy_ref":
            out[name] = {"ms": ms, "bytes": 16.0 * n * n, "gbs": 16.0 * n * n / ms / 1e6}
            log(f"copy {ms:.3f} ms {16.0 * n * n / ms / 1e6:.0f} GB/s")
            continue
        out[name] = {"ms": ms, "tflops": fl / ms / 1e9, "frac_fp64_peak": fl / ms / 1e9 / FP64_PEAK_TFLOPS,
                     "m": m, "k": nb if name != "qr_tn" else n}
        log(f"gemm {name}: {ms:.3f} ms {fl / ms / 1e9:.1f} TFLOP/s")
    return out


def trace_summary(path):
    """Compact summary of a rocprofv3 CSV (the raw traces are too large to
    keep): for a kernel trace, per kernel (template arguments kept) and
    stream the launch count, total and average duration, and the durations
    of each trailing-update product launch (ROLE = 1 instances); for a
    counter collection, per kernel and counter the dispatch count and the
    summed value."""
    import collections
    import csv
    import re
    import statistics

    def short(name):
        m = re.search(r"(k_\w+)(<[^()]*?>)?", name)
        return (m.group(1) + (m.group(2) or "")) if m else name[:60]

    with open(path) as f:
        rd = csv.DictReader(f)
        if "Counter_Name" in (rd.fieldnames or []):
            agg = collections.defaultdict(lambda: [0, 0.0])
            for r in rd:
                a = agg[(short(r["Kernel_Name"]), r["Counter_Name"])]
                a[0] += 1
                a[1] += float(r["Counter_Value"])
            return {"counters": [{"kernel": k[0], "counter": k[1], "dispatches": v[0], "sum": v[1]}
                                 for k, v in sorted(agg.items())]}
        agg = collections.defaultdict(list)
        first, last = None, 0
        for r in rd:
            a, b = int(r["Start_Timestamp"]), int(r["End_Timestamp"])
            first = a if first is None else min(first, a)
            last = max(last, b)
            agg[(short(r["Kernel_Name"]), r["Stream_Id"])].append((b - a) / 1e6)
    kern = sorted(({"kernel": k[0], "stream": k[1], "calls": len(v), "total_ms": sum(v), "avg_ms": statistics.mean(v)}
                   for k, v in agg.items()), key=lambda x: -x["total_ms"])
    tmu = {f"{k[0]} stream {k[1]}": v for k, v in agg.items()
           if k[0].startswith("k_dgemm<") and re.search(r", 1, (16|32)>$", k[0])}
    return {"span_ms": (last - first) / 1e6 if first is not None else 0.0, "kernels": kern, "tmu_launch_ms": tmu}


def main():
    if len(sys.argv) == 3 and sys.argv[1] == "--trace-summary":
        print(json.dumps(trace_summary(sys.argv[2])), flush=True)
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=32768)
    ap.add_argument("--nb", type=int, default=512)
    ap.add_argument("--legs", default="chol,lu,qr")
    ap.add_argument("--overlap", type=int, default=1,
                    help="1: verify the trailing tiles beside the next panel (ABFT_FLAG_OVERLAP_VERIFY); 0: serially")
    ap.add_argument("--mp-n", type=int, default=16384)
    ap.add_argument("--mp-nb", type=int, default=512)
    ap.add_argument("--mp-kappas", default="1e2,1e6,1e10")
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--campaign", type=int, default=400, help="fault-campaign runs per decomposition (0: skip)")
    ap.add_argument("--campaign-n", type=int, default=8192)
    ap.add_argument("--campaign-nb", type=int, default=256)
    ap.add_argument("--energy-n", type=int, default=16384)
    ap.add_argument("--no-energy", action="store_true")
    ap.add_argument("--no-mp", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batch-faults", type=int, default=1, help="untimed batched call with one flip per 64 matrices")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--no-overhead", action="store_true")
    ap.add_argument("--no-check", action="store_true", help="skip the backward-error check of each leg")
    ap.add_argument("--gemm-only", action="store_true",
                    help="time only the trailing-update products on their first-iteration shapes")
    ap.add_argument("--gemm-reps", type=int, default=10)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; the factorization is not sharded "
                                   "across GPUs (run with --gpus 1)"}), flush=True)
        sys.exit(2)

    import torch
    from paper_2301_03166_amd import abft

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    h = abft.Handle(dev)
    if args.gemm_only:
        res = gemm_leg(h, torch, dev, args)
        h.close()
        print(json.dumps({"gemm": res, "n": args.n, "nb": args.nb}), flush=True)
        return
    legs = [x for x in args.legs.split(",") if x]
    t0 = time.perf_counter()
    value, ms_step, per_leg, status, roof = fp64_legs(h, torch, dev, args, legs) if legs else (None, None, {}, {},
                                                                                              None)
    mp = None if args.no_mp else mp_leg(h, torch, dev, args)
    batched = None if args.no_batched else batched_leg(h, torch, dev, args)
    campaign = campaign_leg(h, torch, dev, args) if args.campaign > 0 else None
    energy = None if args.no_energy else energy_leg(h, torch, dev, args)
    wall = time.perf_counter() - t0
    h.close()
    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        cpu = cpu_baseline()

    out = {
        "metric": "FP64 TFLOP/s ABFT LU/Cholesky/QR n=32768; MP+IR speedup vs FP64 @1e-12 error",
        "value": value, "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "ABFT-protected FP64 " + "+".join(legs) + f", n={args.n}, nb={args.nb}, one "
                               "matrix each, full row+column checksums verified every iteration",
                   "n": args.n, "nb": args.nb, "legs": legs},
        "legs": per_leg, "status": status,
        "roofline": roof,
        "mp": mp, "batched": batched, "fault_campaign": campaign, "energy": energy,
        "wall_s": wall,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
