"""Per-iteration time model of the blocked one-sided decompositions.

The paper predicts the execution time of every task of iteration k from
the measured times of earlier iterations and the ratio of the tasks'
theoretical time complexity between iterations (section "Bi-directional
slack reclamation", subsection on slack prediction, Tab. 2).  Its enhanced
predictor weights the p last neighbours:

    T'_k = sum_{i=1..p} w_i r_{k-i,k} T_{k-i},   p = 4, w = (1/2, 1/4, 1/8, 1/8)

where r_{j,k} = W(k) / W(j) is the ratio of the task's theoretical work in
iterations k and j; the earlier state of the art profiles the first
iteration only, T'_k = r_{0,k} T_0.  With ABFT the slack of iteration k is
the predicted time of the update side (TMU and PU with their checksum
update and verification) minus that of the panel side (PD with its
checksum work and the CPU-GPU transfer).

Readings (the paper gives Tab. 2's ratios without their derivation, and
some entries are garbled):

* The work W(k) of each task is derived here from the operation shapes of
  iteration k (0-based; panel columns [k b, k b + w), w = min(b, n - k b),
  m = n - k b panel rows, t = m - w trailing order) with the standard flop
  counts: Cholesky PD (panel factor and L21 solve) w^3/3 + t w^2, TMU t^2 w;
  LU PD (m x w panel with pivoting) m w^2 - w^3/3, PU (U12 solve) w^2 t,
  TMU 2 t^2 w; QR PD (m x w Householder panel) 2 m w^2 - 2 w^3/3, TMU
  (V^T C, T^T W, C - V W2) 4 m t w + 2 w^2 t.  Checksum carries are GEMMs of
  the checksum rows (2 rows per tile-row) with the update's right operand:
  4 (t / b) t w for the column side of LU (QR: 4 (m / b) t w, its tile-rows
  start at the panel) and half that for Cholesky's lower part, plus the
  same again for the row side; verification
  streams the trailing matrix: 8 t^2 bytes (LU), 8 m t (QR, rows from the
  panel down), 8 b^2 T(T+1)/2 with T = t / b tiles (Cholesky's lower tiles).
* Tab. 2's entries for TMU-LU, PU-LU and TMU-QR agree with these ratios to
  first order in b / (n - k b) (the printed forms differ by the choice of
  1- or 0-based iteration index, a second-order difference); the entries
  for Cholesky's TMU (a factor (1 + k)) and for PD-LU / PD-QR (coefficients
  6 b and b / 6) do not follow from any flop count of those operations and
  are taken as garbled.
* The predictor's second term is printed with T_{k-21}; read T_{k-2}.  For
  k < p only the k available neighbours are used, their weights rescaled
  to sum to 1; iteration 0 has no prediction (it is the profiled one).
* The CPU-GPU transfer term is zero: panel and update both run on the GPU.
"""
from __future__ import annotations

WEIGHTS = (0.5, 0.25, 0.125, 0.125)
OPS = ("pd", "pu", "tmu", "carry", "verify")


def shape(n: int, b: int, k: int):
    """(w, m, t): panel width, panel rows and trailing order of iteration k"""
    c0 = k * b
    w = min(b, n - c0)
    m = n - c0
    return w, m, m - w


def work(kind: str, op: str, n: int, b: int, k: int) -> float:
    """Theoretical work of task `op` in iteration k of decomposition `kind`
    ('chol', 'lu', 'qr'): flops for pd / pu / tmu / carry, bytes for verify."""
    w, m, t = shape(n, b, k)
    if w <= 0:
        return 0.0
    T = t / b
    if kind == "chol":
        return {"pd": w ** 3 / 3.0 + t * w * w, "pu": 0.0, "tmu": float(t) * t * w,
                "carry": 2.0 * T * t * w + 2.0 * t * T * w, "verify": 8.0 * b * b * T * (T + 1) / 2.0}[op]
    if kind == "lu":
        return {"pd": m * w * w - w ** 3 / 3.0, "pu": float(w) * w * t, "tmu": 2.0 * t * t * w,
                "carry": 4.0 * T * t * w + 4.0 * t * T * w, "verify": 8.0 * t * t}[op]
    if kind == "qr":
        return {"pd": 2.0 * m * w * w - 2.0 * w ** 3 / 3.0, "pu": 0.0, "tmu": 4.0 * m * t * w + 2.0 * w * w * t,
                "carry": 4.0 * (m / b) * t * w + 4.0 * m * T * w, "verify": 8.0 * m * t}[op]
    raise ValueError(kind)


def iterations(n: int, b: int) -> int:
    return -(-n // b)


def ratio(kind: str, op: str, n: int, b: int, j: int, k: int) -> float:
    """r_{j,k} = W(k) / W(j): the ratio of the task's theoretical work
    between iterations j and k (0 when iteration j has none)."""
    wj = work(kind, op, n, b, j)
    return work(kind, op, n, b, k) / wj if wj > 0 else 0.0


def table2_ratio(kind: str, op: str, n: int, b: int, k: int) -> float | None:
    """Tab. 2's printed ratio of the task between iterations k and k + 1 for
    the entries that follow from a flop count (TMU-LU, PU-LU, TMU-QR), in
    the paper's form; None for the others (garbled or omitted)."""
    if kind == "lu" and op == "tmu":
        return 1.0 - 2.0 * b / (n - k * b)
    if kind == "lu" and op == "pu":
        return 1.0 - b / (n - k * b - b)
    if kind == "qr" and op == "tmu":
        x, y = n - k * b - b, n - k * b + b
        return 1.0 - b / x - b / y + b * b / (x * y)
    return None


def predict_neighbours(times, kind: str, op: str, n: int, b: int, k: int, weights=WEIGHTS) -> float | None:
    """T'_k from the measured times of the p = len(weights) last iterations
    (the paper's enhanced prediction); None for k = 0."""
    p = min(len(weights), k)
    if p == 0:
        return None
    wsum = sum(weights[:p])
    return sum(weights[i - 1] / wsum * ratio(kind, op, n, b, k - i, k) * times[k - i] for i in range(1, p + 1))


def predict_first(times, kind: str, op: str, n: int, b: int, k: int) -> float | None:
    """T'_k from the first iteration alone (the earlier state of the art)."""
    if k == 0:
        return None
    return ratio(kind, op, n, b, 0, k) * times[0]


def slack(pred: dict, k: int) -> float:
    """Predicted slack of iteration k: the update side (TMU, PU and their
    checksum carries and verification) minus the panel side (PD); the
    transfer term is zero in an all-GPU design."""
    return pred["tmu"][k] + pred["pu"][k] + pred["carry"][k] + pred["verify"][k] - pred["pd"][k]


def prediction_error(times, kind: str, op: str, n: int, b: int, predictor, k0: int = 1,
                     floor: float = 0.0) -> float | None:
    """Mean |T'_k - T_k| / T_k over the iterations k >= k0 whose measured
    time exceeds `floor` (ms)."""
    errs = []
    for k in range(k0, len(times)):
        if times[k] <= floor or work(kind, op, n, b, k) <= 0:
            continue
        p = predictor(times, kind, op, n, b, k)
        if p is not None:
            errs.append(abs(p - times[k]) / times[k])
    return sum(errs) / len(errs) if errs else None


def validate(iter_ms: dict, kind: str, n: int, b: int, floor: float = 0.05) -> dict:
    """Both predictors against one factorization's measured per-iteration
    phase times (dict op -> list of ms, as Handle.iter_profile returns)."""
    out = {}
    for op in OPS:
        ts = iter_ms.get(op)
        if not ts or max(ts) <= floor or all(work(kind, op, n, b, k) <= 0 for k in range(len(ts))):
            continue
        out[op] = {"neighbours_p4": prediction_error(ts, kind, op, n, b, predict_neighbours, floor=floor),
                   "first_iteration": prediction_error(ts, kind, op, n, b, predict_first, floor=floor),
                   "iterations": len(ts), "total_ms": sum(ts)}
    return out
