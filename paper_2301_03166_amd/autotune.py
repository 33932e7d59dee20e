"""Autotuner of the library's launch shapes, measured on the device.

Three choices are tuned, all by timing the library's own calls on synthetic
inputs of the requested shape (HIP events on the handle's stream, best of a
few repetitions) and keeping the fastest:

* the block size nb of the large factorizations (it is also the checksum
  tile: it sets the panel width, the K extent of the trailing-update product
  and the verify granularity) jointly with the trailing-update product's
  tile shape (128 x 128 output tiles with K steps of 16, two workgroups per
  CU, or of 32, one workgroup per CU), per operation and size class (the
  next power of two of n);
* the number of persistent workgroups per compute unit of the batched
  factorizations, per operation and precision (binary32 panels take half the
  LDS, so two workgroups can share a CU).

Results live in a JSON table beside this file (``tuned.json``); lookups fall
back to fixed defaults for size classes that were never tuned.

    python -m paper_2301_03166_amd.autotune --ops potrf,getrf,geqrf --sizes 8192,16384,32768 --batched

The table committed beside this file was measured on one MI355X with that
command; its entries record every candidate's time.
"""
from __future__ import annotations

import argparse
import json
import os
import time

TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned.json")
NB_CANDIDATES = (128, 256, 384, 512)
BK_CANDIDATES = (16, 32)
WGS_CANDIDATES = (1, 2)


def size_class(n: int) -> int:
    return 1 << max(0, (int(n) - 1).bit_length())


def load(path: str = TABLE) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save(table: dict, path: str = TABLE) -> None:
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def default_nb(op: str, n: int) -> int:
    if n <= 2048:
        return 128
    if n <= 12288:
        return 256
    return 512


def lookup_nb(op: str, n: int, table: dict | None = None) -> int:
    t = load() if table is None else table
    e = t.get("nb", {}).get(f"{op}:{size_class(n)}")
    nb = int(e["best"]) if e else default_nb(op, n)
    return max(1, min(nb, max(1, int(n))))


def lookup_tmu_bk(op: str, n: int, table: dict | None = None) -> int:
    """K depth of the trailing-update product tiles (16 when untuned)."""
    t = load() if table is None else table
    e = t.get("nb", {}).get(f"{op}:{size_class(n)}")
    return int(e.get("tmu_bk", 16)) if e else 16


def lookup_wgs(op: str, prec: str, table: dict | None = None) -> int:
    t = load() if table is None else table
    e = t.get("batched", {}).get(f"{op}:{prec}")
    return int(e["best"]) if e else 1


def _time(fn, reps):
    import torch
    best = None
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    return best


def tune_nb(h, op: str, n: int, candidates=NB_CANDIDATES, reps: int = 2, bks=BK_CANDIDATES) -> dict:
    """Time the ABFT factorization `op` of an order-n synthetic matrix for
    every candidate block size and product tile depth; returns {"best": nb,
    "tmu_bk": bk, "ms": {"nb/bk": ms}}."""
    import torch
    from . import gen
    dev = h.device
    A0 = gen.spd_torch(n, 11, dev) if op == "potrf" else gen.general_torch(n, 12, dev)
    W = torch.empty_like(A0)
    ipiv = torch.zeros(n, dtype=torch.int32, device=dev)
    tau = torch.zeros(n, dtype=torch.float64, device=dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    rep = h.new_report()
    res = {}
    for nb in candidates:
        if nb > n:
            continue
        for bk in bks:
            def run():
                W.copy_(A0)
                A = W.t()
                if op == "potrf":
                    h.potrf(A, nb, report=rep, info=info, sync=False, tmu_bk=bk)
                elif op == "getrf":
                    h.getrf(A, nb, ipiv=ipiv, report=rep, info=info, sync=False, tmu_bk=bk)
                else:
                    h.geqrf(A, nb, tau=tau, report=rep, info=info, sync=False, tmu_bk=bk)
            run()
            torch.cuda.synchronize()
            res[(nb, bk)] = _time(run, reps)
    del A0, W
    torch.cuda.empty_cache()
    best = min(res, key=res.get)
    return {"best": int(best[0]), "tmu_bk": int(best[1]), "ms": {f"{k[0]}/{k[1]}": v for k, v in res.items()}}


def tune_batched(h, op: str, prec: str, count: int = 2048, candidates=WGS_CANDIDATES, reps: int = 3) -> dict:
    """Time the batched factorization of `count` matrices with orders uniform
    on [32, 512] for each persistent-workgroups-per-CU candidate."""
    import numpy as np
    import torch
    from . import gen
    dev = h.device
    chol = op == "potrf"
    dt = torch.float64 if prec == "f64" else torch.float32
    sizes = gen.batch_sizes(count, 32, 512, 31)
    seeds = gen.batch_seeds(count, 31)
    pristine, _ = gen.batch_torch(sizes, seeds, "chol" if chol else "lu", dev, dtype=dt)
    flat = torch.empty_like(pristine)
    offs = np.concatenate([[0], np.cumsum(sizes.astype(np.int64) ** 2)])
    views = [torch.as_strided(flat, (int(s), int(s)), (1, int(s)), int(offs[q])) for q, s in enumerate(sizes)]
    state = h.batched_args(views, chol)
    res = {}
    for g in candidates:
        def run():
            h.batched(views, chol, state=state, sync=False, wgs_per_cu=g)
        flat.copy_(pristine)
        run()
        torch.cuda.synchronize()
        best = None
        for _ in range(reps):
            flat.copy_(pristine)
            ms = _time(run, 1)
            best = ms if best is None else min(best, ms)
        res[g] = best
    del pristine, flat, views, state
    torch.cuda.empty_cache()
    b = min(res, key=res.get)
    return {"best": int(b), "ms": {str(k): v for k, v in res.items()}, "count": count}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--ops", default="potrf,getrf,geqrf")
    ap.add_argument("--sizes", default="4096,8192,16384")
    ap.add_argument("--candidates", default=",".join(map(str, NB_CANDIDATES)))
    ap.add_argument("--batched", action="store_true")
    ap.add_argument("--batch-count", type=int, default=2048)
    ap.add_argument("--out", default=TABLE)
    args = ap.parse_args(argv)
    from . import abft
    h = abft.Handle()
    table = load(args.out)
    cands = tuple(int(x) for x in args.candidates.split(","))
    t0 = time.time()
    for op in [x for x in args.ops.split(",") if x]:
        for n in [int(x) for x in args.sizes.split(",") if x]:
            r = tune_nb(h, op, n, cands)
            table.setdefault("nb", {})[f"{op}:{size_class(n)}"] = dict(r, n=n)
            print(f"[autotune] {op} n={n}: best nb={r['best']} tmu_bk={r['tmu_bk']}  {r['ms']}", flush=True)
            save(table, args.out)
    if args.batched:
        for op in ("potrf", "getrf"):
            for prec in ("f64", "f32"):
                r = tune_batched(h, op, prec, args.batch_count)
                table.setdefault("batched", {})[f"{op}:{prec}"] = r
                print(f"[autotune] batched {op} {prec}: best wgs_per_cu={r['best']}  {r['ms']}", flush=True)
                save(table, args.out)
    h.close()
    print(f"[autotune] done in {time.time() - t0:.1f} s -> {args.out}", flush=True)


if __name__ == "__main__":
    main()
