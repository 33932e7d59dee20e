// Host drivers and the C ABI (include/abft.h).
//
// Every factorization is a sequence of kernel launches on the handle's
// stream with no host synchronisation inside the loop: per iteration the
// panel (recursive, leaves of 32 columns), the interchanges (LU), the panel
// update, the trailing update on FP64 MFMA, the checksum carry (four thin
// GEMMs: values and magnitudes for the column and the row side), an optional
// planned bit flip, and the verify / correct pass over the trailing tiles.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>

#include "common.hpp"
#include "kernels.hpp"

using namespace abft;

// A captured batched call: the arguments it was captured with and its
// executable graph (replayed when a later call passes the same arguments).
struct BatchGraph {
  int chol, prec, batch, protect, wgs;
  double ts;
  const void *dn, *dA, *dlda, *dipiv, *dwork, *dinfo, *dreps;
  hipGraphExec_t exec;
};
constexpr int MAX_GRAPHS = 8;

struct abft_handle_s {
  hipStream_t stream;
  int device;
  int cus;
  abft_profile prof;
  hipEvent_t* ev;  // event pool for profiled calls
  int nev;
  hipStream_t cap;  // side stream used only for graph capture (created on first use)
  hipStream_t side;  // checksum carries beside the trailing update (created on first use)
  hipEvent_t fork_ev, join_ev;
  BatchGraph graphs[MAX_GRAPHS];
  int ngraphs, next_graph;
  void* ws;  // workspace registered with abft_set_workspace (used by calls passing dwork == NULL)
  size_t ws_bytes;
  double* iter_ms;  // per-iteration phase times of the last profiled call (host, phase-major)
  int iter_n;
  // look-ahead schedule: an update stream and a panel stream on disjoint
  // sets of compute units (created on first use; la_pcus units for the panel)
  hipStream_t la_main, la_panel;
  int la_pcus;
  hipEvent_t la_ev[4];
  // verification beside the next panel: a stream restricted to part of the
  // compute units (created on first use)
  hipStream_t vb;
  hipEvent_t vb_ev[2];
  // non-blocking stream for overlapped calls made on the null stream
  hipStream_t own;
  hipEvent_t own_ev[2];
};

// a call's workspace: its own, else the one registered with the handle
static inline void use_ws(abft_handle h, void*& dwork, size_t& bytes) {
  if (!dwork) {
    dwork = h->ws;
    bytes = h->ws_bytes;
  }
}

namespace {

constexpr int LEAFW = 32;   // leaf width of the Cholesky panel and the triangular solves
constexpr int CLEAFW = 64;  // widest cooperative LU / QR leaf (narrower where it cannot cover the rows)
constexpr int MAXNB = 512;
constexpr double U64 = 1.1102230246251565e-16;  // 2^-53
constexpr double U32 = 5.9604644775390625e-08;  // 2^-24

#define TRY(x)                 \
  do {                         \
    int _e = (x);              \
    if (_e) return _e;         \
  } while (0)

inline size_t al(size_t b) { return (b + 255) & ~(size_t)255; }
// split-K partials: at least 128 MB (a split that fills about 512
// workgroups of 128 x 128 tiles keeps S m n near 512 * 128^2), and room for
// four partial copies of QR's nb x n product W = V^T C (its split evens out
// the last round of workgroups)
inline size_t splitk_elems(int64_t n, int nb) {
  return std::max<size_t>((size_t)1 << 24, (size_t)4 * nb * n);
}
// cooperative-leaf exchange records (SLOT_WORDS 8-byte words), two columns
// alternating: per column 4G (3 + 2w) + 2w words (LU) or G 2w + 2w (QR);
// G <= 256, w <= 64
constexpr size_t CTR_BYTES = 4096;  // grid-barrier counters: top + 16 groups, 128 bytes apart

// Phase timer of profiled calls: event pairs recorded on the stream, summed
// per phase after one synchronisation at the end of the call.
// phases of a profiled call; the per-iteration record keeps them apart in this order
enum { PH_PANEL = 0, PH_PU = 1, PH_TMU = 2, PH_CARRY = 3, PH_VERIFY = 4, PH_N = 5 };
struct Prof {
  abft_handle h;
  bool on;
  int used;
  int tags[8192];
  int iter_of[8192];
  double tmu_flops = 0, verify_bytes = 0;
  int tmu_launches = 0, iters = 0;
  explicit Prof(abft_handle hh, const abft_opts* o) : h(hh), on(o && (o->flags & ABFT_FLAG_PROFILE)), used(0) {
    if (!on) return;
    if (!h->ev) {
      h->nev = 8192;
      h->ev = (hipEvent_t*)calloc(h->nev, sizeof(hipEvent_t));
      for (int i = 0; i < h->nev; ++i) (void)hipEventCreate(&h->ev[i]);
    }
  }
  int begin(int tag) {
    if (!on || used + 2 > h->nev) return -1;
    int i = used;
    used += 2;
    tags[i / 2] = tag;
    iter_of[i / 2] = iters > 0 ? iters - 1 : 0;
    (void)hipEventRecord(h->ev[i], h->stream);
    return i;
  }
  void end(int i) {
    if (i >= 0) (void)hipEventRecord(h->ev[i + 1], h->stream);
  }
  void finish() {
    if (!on) return;
    abft_profile p;
    memset(&p, 0, sizeof(p));
    const int ni = iters > 0 ? iters : 1;
    double* im = (double*)realloc(h->iter_ms, sizeof(double) * PH_N * ni);
    if (im) {
      h->iter_ms = im;
      h->iter_n = ni;
      memset(im, 0, sizeof(double) * PH_N * ni);
    } else {
      h->iter_n = 0;
    }
    if (used) {
      (void)hipEventSynchronize(h->ev[used - 1]);
      float ms;
      double ph[PH_N] = {0, 0, 0, 0, 0};
      for (int i = 0; i < used; i += 2)
        if (hipEventElapsedTime(&ms, h->ev[i], h->ev[i + 1]) == hipSuccess) {
          ph[tags[i / 2]] += ms;
          if (h->iter_n) h->iter_ms[tags[i / 2] * h->iter_n + std::min(iter_of[i / 2], h->iter_n - 1)] += ms;
        }
      if (hipEventElapsedTime(&ms, h->ev[0], h->ev[used - 1]) == hipSuccess) p.ms_total = ms;
      p.ms_panel = ph[PH_PANEL] + ph[PH_PU];
      p.ms_tmu = ph[PH_TMU];
      p.ms_carry = ph[PH_CARRY];
      p.ms_verify = ph[PH_VERIFY];
    }
    p.tmu_flops = tmu_flops;
    p.verify_bytes = verify_bytes;
    p.tmu_launches = tmu_launches;
    p.iters = iters;
    h->prof = p;
  }
};

// The side stream of an iteration runs what the trailing-matrix update's
// product neither reads nor writes: the checksum carry (it reads the panel
// operands L21, U12 or V, W2 and the checksum rows, and writes the checksum
// arrays), the panel checks (they read the panel and write the report and
// the panel flags) and, for LU, the interchanges of the already factored
// columns left of the panel and of the row checksums.  It runs concurrently
// with the update's product, and the main stream waits for it before the
// verification.  Profiled calls keep one stream so that each phase's
// events time that phase alone.
struct Side {
  hipStream_t main, s;
  bool on;
  Side(abft_handle h, bool want) : main(h->stream), s(h->stream), on(false) {
    if (!want) return;
    if (!h->side) {
      if (hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking) != hipSuccess) { h->side = nullptr; return; }
      if (hipEventCreateWithFlags(&h->fork_ev, hipEventDisableTiming) != hipSuccess ||
          hipEventCreateWithFlags(&h->join_ev, hipEventDisableTiming) != hipSuccess) {
        (void)hipStreamDestroy(h->side);
        h->side = nullptr;
        return;
      }
    }
    s = h->side;
    on = true;
    fe = h->fork_ev;
    je = h->join_ev;
  }
  // side stream starts after everything enqueued on the main stream so far
  int fork() {
    if (!on) return 0;
    pending = true;
    if (hipEventRecord(fe, main) != hipSuccess || hipStreamWaitEvent(s, fe, 0) != hipSuccess) return ABFT_ERR_HIP;
    return 0;
  }
  // main stream continues after everything enqueued on the side stream
  int join() {
    if (!on) return 0;
    pending = false;
    if (hipEventRecord(je, s) != hipSuccess || hipStreamWaitEvent(main, je, 0) != hipSuccess) return ABFT_ERR_HIP;
    return 0;
  }
  // a call that returns early (an error between fork and join) still leaves
  // the caller's stream ordered after the side stream's work
  ~Side() {
    if (pending) (void)join();
  }
  bool pending = false;
  hipEvent_t fe = nullptr, je = nullptr;
};

// Look-ahead schedule of a blocked factorization.  The call's work moves
// from the caller's stream to the handle's update stream (compute units
// [0, cus - P)); the next panel is factored on the panel stream (units
// [cus - P, cus)) while the update stream finishes the current iteration,
// and the update stream waits for it before the next iteration.  The
// caller's stream is ordered before (entry) and after (exit) both.  Off for
// profiled calls (one stream), fault plans and per-iteration levels.
int la_streams(abft_handle h, int pcus) {
  if (h->la_pcus == pcus && h->la_main) return 0;
  if (h->la_main) {
    if (hipStreamSynchronize(h->la_main) != hipSuccess || hipStreamSynchronize(h->la_panel) != hipSuccess)
      return ABFT_ERR_HIP;
    (void)hipStreamDestroy(h->la_main);
    (void)hipStreamDestroy(h->la_panel);
    h->la_main = h->la_panel = nullptr;
    h->la_pcus = 0;
  }
  if (!h->la_ev[0])
    for (int i = 0; i < 4; ++i)
      if (hipEventCreateWithFlags(&h->la_ev[i], hipEventDisableTiming) != hipSuccess) return ABFT_ERR_HIP;
  const int words = (h->cus + 31) / 32;
  uint32_t mm[16] = {0}, pm[16] = {0};
  if (words > 16) return ABFT_ERR_UNSUPPORTED;
  for (int c = 0; c < h->cus; ++c) (c < h->cus - pcus ? mm : pm)[c / 32] |= 1u << (c % 32);
  if (hipExtStreamCreateWithCUMask(&h->la_main, words, mm) != hipSuccess) {
    h->la_main = nullptr;
    return ABFT_ERR_HIP;
  }
  if (hipExtStreamCreateWithCUMask(&h->la_panel, words, pm) != hipSuccess) {
    (void)hipStreamDestroy(h->la_main);
    h->la_main = h->la_panel = nullptr;
    return ABFT_ERR_HIP;
  }
  h->la_pcus = pcus;
  return 0;
}

struct Look {
  abft_handle h;
  bool on = false;
  hipStream_t caller = nullptr, ms = nullptr, ps = nullptr;
  int pmaxg = 0, mmaxg = 0;  // workgroup bounds of the cooperative panel leaves on each stream
  // rows_per_cu: panel rows one compute unit's LDS holds in the narrowest
  // cooperative leaf; the panel share is raised to cover the first panel
  Look(abft_handle hh, const abft_opts* o, bool allowed, int64_t n, int nb, int rows_per_cu) : h(hh) {
    if (!allowed || o->lookahead <= 0 || (o->flags & ABFT_FLAG_PROFILE) || (o->faults && o->nfaults > 0) ||
        o->levels || n <= nb)
      return;
    // the panel stream must hold the first panel's leaf rows in its units' LDS
    const int need = (int)std::min<int64_t>(h->cus, (n + rows_per_cu - 1) / rows_per_cu);
    const int pc = std::max(need, std::min(o->lookahead, h->cus / 2));
    if (pc >= h->cus) return;
    if (la_streams(h, pc)) return;  // (no masked streams: the one-stream schedule)
    caller = h->stream;
    if (hipEventRecord(h->la_ev[0], caller) != hipSuccess || hipStreamWaitEvent(h->la_main, h->la_ev[0], 0) != hipSuccess)
      return;
    ms = h->la_main;
    ps = h->la_panel;
    pmaxg = std::min(pc, 256);
    mmaxg = std::min(h->cus - pc, 256);
    h->stream = ms;
    on = true;
  }
  // the panel stream starts after everything enqueued on the update stream so far
  int fork_panel() {
    if (hipEventRecord(h->la_ev[1], ms) != hipSuccess || hipStreamWaitEvent(ps, h->la_ev[1], 0) != hipSuccess)
      return ABFT_ERR_HIP;
    return 0;
  }
  // the update stream continues after everything enqueued on the panel stream
  int join_panel() {
    if (hipEventRecord(h->la_ev[2], ps) != hipSuccess || hipStreamWaitEvent(ms, h->la_ev[2], 0) != hipSuccess)
      return ABFT_ERR_HIP;
    return 0;
  }
  // (the restricted streams live for one call, as the verification stream
  // beside the panel does: their existence slows other work on the device)
  int finish() {
    if (!on) return 0;
    on = false;
    h->stream = caller;
    if (join_panel()) return ABFT_ERR_HIP;
    if (hipEventRecord(h->la_ev[3], ms) != hipSuccess || hipStreamWaitEvent(caller, h->la_ev[3], 0) != hipSuccess)
      return ABFT_ERR_HIP;
    (void)hipStreamDestroy(h->la_main);
    (void)hipStreamDestroy(h->la_panel);
    h->la_main = h->la_panel = nullptr;
    h->la_pcus = 0;
    return 0;
  }
  ~Look() { (void)finish(); }
};

// Verification beside the next panel (ABFT_FLAG_OVERLAP_VERIFY).  After the
// trailing update of iteration k, the tiles of the next panel's block column
// are verified and corrected on the caller's stream; the other trailing
// tiles are verified and corrected on a stream restricted to half of the
// compute units, while the next panel is factored on the caller's stream
// (the panel reads and writes only its own block column, and its
// cooperative leaves find the other half free).  join() comes before
// anything else touches the trailing matrix or its checksums.  The
// restricted stream is created for each call and destroyed at its end.
int vb_stream(abft_handle h) {
  if (h->vb) return 0;
  const int words = (h->cus + 31) / 32;
  uint32_t mm[16] = {0};
  if (words > 16 || h->cus < 2) return ABFT_ERR_UNSUPPORTED;
  for (int c = 0; c < h->cus / 2; ++c) mm[c / 32] |= 1u << (c % 32);
  for (int i = 0; i < 2; ++i)
    if (!h->vb_ev[i] && hipEventCreateWithFlags(&h->vb_ev[i], hipEventDisableTiming) != hipSuccess) {
      h->vb_ev[i] = nullptr;
      return ABFT_ERR_HIP;
    }
  if (hipExtStreamCreateWithCUMask(&h->vb, words, mm) != hipSuccess) {
    h->vb = nullptr;
    return ABFT_ERR_HIP;
  }
  return 0;
}

// A call that overlaps work on the restricted stream runs off the null
// stream: the restricted stream is a blocking stream, so every launch on
// the null stream would wait for its work.  When the handle's stream is the
// null stream, the call's work goes to a non-blocking stream of the handle,
// ordered after the null stream's earlier work on entry, and the null
// stream waits for it on exit.
struct OffNull {
  abft_handle h;
  bool on = false;
  OffNull(abft_handle hh, const abft_opts* o, bool allowed = true) : h(hh) {
    if (!allowed || h->stream || !(o->flags & ABFT_FLAG_OVERLAP_VERIFY) || (o->flags & ABFT_FLAG_PROFILE) || o->lookahead > 0)
      return;
    if (!h->own) {  // (the stream and both events, or nothing: the call then stays on the null stream)
      hipStream_t st = nullptr;
      hipEvent_t e0 = nullptr, e1 = nullptr;
      if (hipEventCreateWithFlags(&e0, hipEventDisableTiming) != hipSuccess ||
          hipEventCreateWithFlags(&e1, hipEventDisableTiming) != hipSuccess ||
          hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        return;
      }
      h->own = st;
      h->own_ev[0] = e0;
      h->own_ev[1] = e1;
    }
    if (hipEventRecord(h->own_ev[0], nullptr) != hipSuccess || hipStreamWaitEvent(h->own, h->own_ev[0], 0) != hipSuccess)
      return;
    h->stream = h->own;
    on = true;
  }
  ~OffNull() {
    if (!on) return;
    h->stream = nullptr;
    if (hipEventRecord(h->own_ev[1], h->own) != hipSuccess || hipStreamWaitEvent(nullptr, h->own_ev[1], 0) != hipSuccess)
      (void)hipStreamSynchronize(h->own);  // (the caller must still find the work done after its stream)
  }
};

struct Beside {
  abft_handle h;
  hipStream_t main, s = nullptr;
  hipEvent_t fe = nullptr, je = nullptr;
  bool want = false, pending = false;
  Beside(abft_handle hh, const abft_opts* o, bool allowed) : h(hh), main(hh->stream) {
    want = allowed && (o->flags & ABFT_FLAG_OVERLAP_VERIFY) && !(o->flags & ABFT_FLAG_PROFILE) && o->lookahead <= 0;
  }
  // true when the rest of the trailing matrix can go to the restricted
  // stream (created on the first such use in the call; without it the
  // call verifies everything on the caller's stream)
  bool ready() {
    if (!want) return false;
    if (!s) {
      if (vb_stream(h)) {
        want = false;
        return false;
      }
      s = h->vb;
      fe = h->vb_ev[0];
      je = h->vb_ev[1];
    }
    return true;
  }
  // the restricted stream starts after everything enqueued on the main stream so far
  int fork() {
    pending = true;
    if (hipEventRecord(fe, main) != hipSuccess || hipStreamWaitEvent(s, fe, 0) != hipSuccess) return ABFT_ERR_HIP;
    return 0;
  }
  // the main stream continues after the restricted stream's work
  int join() {
    if (!pending) return 0;
    pending = false;
    if (hipEventRecord(je, s) != hipSuccess || hipStreamWaitEvent(main, je, 0) != hipSuccess) return ABFT_ERR_HIP;
    return 0;
  }
  // the restricted stream lives for one call: while a stream restricted to
  // part of the device exists, other work on the device was measured to run
  // slower (LU at n = 32768: 880 -> 990 ms)
  ~Beside() {
    (void)join();
    if (s) {
      (void)hipStreamDestroy(h->vb);
      h->vb = nullptr;
    }
  }
};

// Workspace carve-up shared by the three factorizations.
struct Ws {
  double *colchk, *rowchk, *gc, *gr, *S, *Sa, *Tm, *Ta;
  double *Tfac, *W, *W2, *Wp, *Wp2, *Xq, *Yq, *Z, *Zabs, *E, *bt, *scr;
  double *porig, *stage, *slots, *splitk;
  size_t splitk_n;  // elements of splitk
  int *tflags, *moves, *pflags;
  unsigned* ctr;
  size_t bytes;
};

Ws carve(char* base, int64_t n, int nb, int op, int elem) {
  Ws w;
  memset(&w, 0, sizeof(w));
  const int64_t N = (n + nb - 1) / nb;
  size_t off = 0;
  auto take = [&](size_t b) -> char* {
    char* p = base ? base + off : nullptr;
    off += al(b);
    return p;
  };
  const size_t chk = (size_t)2 * N * n * sizeof(double);
  w.colchk = (double*)take(chk);
  w.rowchk = (double*)take(chk);
  w.gc = (double*)take(chk);
  w.gr = (double*)take(chk);
  w.S = (double*)take((size_t)2 * N * nb * sizeof(double));
  w.Sa = (double*)take((size_t)2 * N * nb * sizeof(double));
  w.Tm = (double*)take((size_t)2 * N * nb * sizeof(double));
  w.Ta = (double*)take((size_t)2 * N * nb * sizeof(double));
  w.tflags = (int*)take((size_t)N * N * sizeof(int));
  w.pflags = (int*)take((size_t)N * sizeof(int));
  w.ctr = (unsigned*)take(CTR_BYTES);
  w.slots = (double*)take(SLOT_WORDS * sizeof(double));
  if (op == ABFT_OP_GETRF || op == ABFT_OP_GESV_MP) {
    w.porig = (double*)take((size_t)n * nb * elem);
    w.stage = (double*)take((size_t)2 * nb * n * elem);
    w.moves = (int*)take((size_t)(4 * nb + 4) * sizeof(int));
  }
  if (op == ABFT_OP_GEQRF) {
    w.splitk_n = splitk_elems(n, nb);
    w.splitk = (double*)take(w.splitk_n * sizeof(double));
    w.Tfac = (double*)take((size_t)nb * nb * sizeof(double));
    w.W = (double*)take((size_t)nb * n * sizeof(double));
    w.W2 = (double*)take((size_t)nb * n * sizeof(double));
    w.Wp = (double*)take((size_t)nb * nb * sizeof(double));
    w.Wp2 = (double*)take((size_t)nb * nb * sizeof(double));
    w.Xq = (double*)take((size_t)nb * nb * sizeof(double));
    w.Yq = (double*)take((size_t)nb * nb * sizeof(double));
    w.Z = (double*)take((size_t)nb * nb * sizeof(double));
    w.Zabs = (double*)take((size_t)nb * nb * sizeof(double));
    w.scr = (double*)take((size_t)5 * nb * nb * sizeof(double));
    w.E = (double*)take((size_t)4 * nb * sizeof(double));
    w.bt = (double*)take((size_t)nb * sizeof(double));
  }
  w.bytes = off;
  return w;
}

int check_opts(const abft_opts* o, int64_t n, int& nb, int& protect, double& ts) {
  if (!o) return -7;
  nb = o->nb;
  protect = o->protect;
  ts = o->tau_scale > 0 ? o->tau_scale : 4.0;
  if (nb < 1 || nb > MAXNB) return -7;
  if (protect < ABFT_PROTECT_NONE || protect > ABFT_PROTECT_FULL) return -7;
  if (o->tmu_bk != 0 && o->tmu_bk != 16 && o->tmu_bk != 32) return -7;
  if (o->levels) {
    const int64_t N = (n + nb - 1) / nb;
    if (o->nlevels < N) return -7;
    for (int64_t k = 0; k < N; ++k)
      if (o->levels[k] < ABFT_PROTECT_NONE || o->levels[k] > ABFT_PROTECT_FULL) return -7;
  }
  return 0;
}

// protection level of iteration k (the caller's per-iteration levels, or
// the call's level), and whether any iteration is protected
inline int level_at(const abft_opts* o, int k, int protect) { return o->levels ? o->levels[k] : protect; }
inline bool any_protected(const abft_opts* o, int N, int protect) {
  if (!o->levels) return protect != ABFT_PROTECT_NONE;
  for (int k = 0; k < N; ++k)
    if (o->levels[k]) return true;
  return false;
}
// role of the trailing-update product launches: 1 = 128 x 128 x 16 tiles
// (two workgroups per CU), 2 = 128 x 128 x 32 tiles (one per CU)
inline int tmu_role(const abft_opts* o) { return o->tmu_bk == 32 ? 2 : 1; }
inline bool has_operand_faults(const abft_opts* o) {
  for (int q = 0; q < (o->faults ? o->nfaults : 0); ++q)
    if (o->faults[q].target == 3 || o->faults[q].target == 4) return true;
  return false;
}

inline int split(int w, int leaf = LEAFW) { return ((w / 2 + leaf - 1) / leaf) * leaf; }

// ----------------------------------------------------------------- faults
// A flip of a matrix element records its size in the report, and its position
// (frow, fcol; -1 when none) lets that iteration's verification record the
// difference and threshold of the column checksum that covers it.
template <typename T>
int apply_faults(hipStream_t s, const abft_opts* o, int iter, T* A, int64_t lda, const Ws& w, int64_t n, int N,
                 abft_report* rep, int64_t& frow, int64_t& fcol) {
  frow = fcol = -1;
  for (int q = 0; q < o->nfaults; ++q) {
    const abft_fault& f = o->faults[q];
    if (f.iter != iter) continue;
    if (f.target == 0) {
      if (f.row < 0 || f.row >= n || f.col < 0 || f.col >= n) continue;
      TRY(inject(s, A + f.row + f.col * lda, sizeof(T) == 4, f.bit, rep));
      frow = f.row;
      fcol = f.col;
    } else if (f.target == 1 && w.colchk) {
      if (f.row < 0 || f.row >= 2 * N || f.col < 0 || f.col >= n) continue;
      TRY(inject(s, w.colchk + f.row + f.col * 2 * N, 0, f.bit));
    } else if (f.target == 2 && w.rowchk) {
      if (f.row < 0 || f.row >= n || f.col < 0 || f.col >= 2 * N) continue;
      TRY(inject(s, w.rowchk + f.row + f.col * n, 0, f.bit));
    }
  }
  return 0;
}

// Operand faults of iteration `iter` (targets 3 / 4): XOR the bit of the
// stored operand element; called before the trailing-update product and
// again after it, which restores the element.  W2 (QR's right operand, nb x
// columns [c1, n)) is addressed by (p, matrix column).
template <typename T>
int apply_operand_faults(hipStream_t s, const abft_opts* o, int iter, T* A, int64_t lda, int64_t n, const double* W2,
                         int ldw2, int64_t c1) {
  for (int q = 0; q < (o->faults ? o->nfaults : 0); ++q) {
    const abft_fault& f = o->faults[q];
    if (f.iter != iter || (f.target != 3 && f.target != 4)) continue;
    if (f.target == 4 && W2) {
      if (f.row < 0 || f.row >= ldw2 || f.col < c1 || f.col >= n) continue;
      TRY(inject(s, (void*)(W2 + f.row + (f.col - c1) * ldw2), 0, f.bit));
    } else {
      if (f.row < 0 || f.row >= n || f.col < 0 || f.col >= n) continue;
      TRY(inject(s, A + f.row + f.col * lda, sizeof(T) == 4, f.bit));
    }
  }
  return 0;
}

// ----------------------------------------------------------------- panels
// GEMM on the data type of the factorization: FP64 MFMA for double data;
// for binary32 data FP32 MFMA, or bf16 / fp16 products with FP32
// accumulation when prec asks for them (trailing update only).
// role 1 marks the trailing-matrix update (its own kernel instance in profiles)
inline int gemmT(hipStream_t s, int prec, int ta, int tb, int lower, int m, int n, int k, double alpha,
                 const double* A, int64_t lda, const double* B, int64_t ldb, double beta, double* C, int64_t ldc,
                 int64_t doff, int role = 0) {
  (void)prec;
  return gemm64(s, ta, tb, 0, 0, lower, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, doff, 0, 0, 0, nullptr, 0,
                role);
}
inline int gemmT(hipStream_t s, int prec, int ta, int tb, int lower, int m, int n, int k, double alpha,
                 const float* A, int64_t lda, const float* B, int64_t ldb, double beta, float* C, int64_t ldc,
                 int64_t doff, int role = 0) {
  (void)role;
  return gemm32(s, prec, ta, tb, lower, m, n, k, (float)alpha, A, lda, B, ldb, (float)beta, C, ldc, doff);
}
template <typename T>
constexpr int panel_prec() {
  return sizeof(T) == 8 ? ABFT_F64 : ABFT_F32;
}

// Cholesky panel, columns [c0, c1), rows [c0, n): recursive halves; the
// right half is updated by the left half's columns with the lower-masked
// MFMA GEMM.
template <typename T>
int chol_panel(hipStream_t s, T* A, int64_t lda, int64_t n, int64_t c0, int64_t c1, int32_t* info) {
  const int w = (int)(c1 - c0);
  if (w <= LEAFW) {
    TRY(potrf_leaf(s, A, lda, c0, w, info));
    return trsm_rlt_leaf(s, A, lda, c0 + w, n, c0, w);
  }
  const int h = split(w);
  TRY(chol_panel(s, A, lda, n, c0, c0 + h, info));
  const int64_t r = c0 + h;
  TRY(gemmT(s, panel_prec<T>(), 0, 1, 1, (int)(n - r), (int)(c1 - r), h, -1.0, A + r + c0 * lda, lda,
            A + r + c0 * lda, lda, 1.0, A + r + r * lda, lda, 0));
  return chol_panel(s, A, lda, n, r, c1, info);
}

// X = L^{-1} B: L unit lower at (c0, c0) of order w, B = rows [c0, c0+w) of
// columns [j0, j1).  One blocked launch (strips of B in LDS) up to the
// largest block size for few columns; recursive halves with a product in
// between beyond it, and for many columns down to TRSM_REC_W rows (each
// strip's substitution is a chain of w/32 dependent block steps, while the
// products in between run at MFMA rate over all columns at once).
constexpr int TRSM_REC_W = 256;
constexpr int64_t TRSM_REC_COLS = 4096;
template <typename T>
int trsm_llu(hipStream_t s, T* A, int64_t lda, int64_t c0, int w, int64_t j0, int64_t j1) {
  if (j1 <= j0) return 0;
  if (w <= LEAFW) return trsm_llu_leaf(s, A, lda, c0, w, j0, j1);
  if (w <= 512 && (w <= TRSM_REC_W || j1 - j0 < TRSM_REC_COLS)) return trsm_llu_blk(s, A, lda, c0, w, j0, j1);
  const int h = split(w);
  TRY(trsm_llu(s, A, lda, c0, h, j0, j1));
  TRY(gemmT(s, panel_prec<T>(), 0, 0, 0, w - h, (int)(j1 - j0), h, -1.0, A + (c0 + h) + c0 * lda, lda,
            A + c0 + j0 * lda, lda, 1.0, A + (c0 + h) + j0 * lda, lda, 0));
  return trsm_llu(s, A, lda, c0 + h, w - h, j0, j1);
}

template <typename T>
struct LuCtx {
  hipStream_t s;
  T* A;
  int64_t lda, n;
  int32_t *ipiv, *info;
  const Ws* w;
  unsigned ctr_base;
  abft_report* rep;
  int maxg;
};

// LU panel, columns [c0, c1), rows [c0, n) (recursive, LAPACK getrf2 order)
template <typename T>
int lu_panel(LuCtx<T>& c, int64_t c0, int64_t c1) {
  const int w = (int)(c1 - c0);
  if (w <= CLEAFW) {
    const int rc =
        getrf_leaf(c.s, c.A, c.lda, c.n, c0, w, c.ipiv, c.info, c.w->slots, c.w->ctr, &c.ctr_base, c.rep, c.maxg);
    if (rc != ABFT_ERR_UNSUPPORTED || w <= LEAFW) return rc;  // else too many rows for one wide leaf: split
  }
  const int h = w <= CLEAFW ? split(w) : split(w, CLEAFW);
  TRY(lu_panel(c, c0, c0 + h));
  TRY(perm_build(c.s, c.ipiv, c0, h, c.n, c.w->moves));
  TRY(laswp(c.s, c.A, c.lda, c0 + h, c1, c.w->moves, (T*)c.w->stage, (double*)nullptr, 0, 1));
  TRY(trsm_llu(c.s, c.A, c.lda, c0, h, c0 + h, c1));
  const int64_t r = c0 + h;
  TRY(gemmT(c.s, panel_prec<T>(), 0, 0, 0, (int)(c.n - r), (int)(c1 - r), h, -1.0, c.A + r + c0 * c.lda, c.lda,
            c.A + c0 + r * c.lda, c.lda, 1.0, c.A + r + r * c.lda, c.lda, 0));
  TRY(lu_panel(c, r, c1));
  TRY(perm_build(c.s, c.ipiv, r, w - h, c.n, c.w->moves));
  return laswp(c.s, c.A, c.lda, c0, r, c.w->moves, (T*)c.w->stage, (double*)nullptr, 0, 1);
}

struct QrCtx {
  hipStream_t s;
  double* A;
  int64_t lda, n;
  double* tau;
  const Ws* w;
  int nb;
  int64_t cb;  // first column of the current block panel
  unsigned ctr_base;
  abft_report* rep;
  int maxg;
};

// Householder panel, columns [c0, c1), rows [c0, n), with its T factor at
// Tfac[(c0-cb) + (c0-cb)*nb] (recursive; T merged as T12 = -T1 V1^T V2 T2)
int qr_panel(QrCtx& c, int64_t c0, int64_t c1) {
  const int w = (int)(c1 - c0);
  const int toff = (int)(c0 - c.cb);
  const int nb = c.nb;
  double* A = c.A;
  const int64_t lda = c.lda, n = c.n;
  if (w <= CLEAFW) {
    const int rc = geqrf_leaf(c.s, A, lda, n, c0, w, c.tau, c.w->Tfac, nb, toff, c.w->slots, c.w->ctr, &c.ctr_base,
                              c.rep, c.maxg);
    if (rc != ABFT_ERR_UNSUPPORTED || w <= LEAFW) return rc;  // else too many rows for one wide leaf: split
  }
  const int h = w <= CLEAFW ? split(w) : split(w, CLEAFW);
  TRY(qr_panel(c, c0, c0 + h));
  const int64_t r = c0 + h;
  double* V1 = A + c0 + c0 * lda;
  double* T1 = c.w->Tfac + toff + (int64_t)toff * nb;
  // apply H1^T = I - V1 T1^T V1^T to the right half
  TRY(gemm64(c.s, 1, 0, 1, 0, 0, h, (int)(c1 - r), (int)(n - c0), 1.0, V1, lda, A + c0 + r * lda, lda, 0.0, c.w->Wp,
             nb, 0, 0, 0, 0, c.w->splitk, c.w->splitk_n));
  TRY(gemm64(c.s, 1, 0, 0, 0, 0, h, (int)(c1 - r), h, 1.0, T1, nb, c.w->Wp, nb, 0.0, c.w->Wp2, nb, 0));
  TRY(gemm64(c.s, 0, 0, 1, 0, 0, (int)(n - c0), (int)(c1 - r), h, -1.0, V1, lda, c.w->Wp2, nb, 1.0, A + c0 + r * lda,
             lda, 0));
  TRY(qr_panel(c, r, c1));
  // T12 = -T1 (V1^T V2) T2 ; rows of V2 above r are zero
  double* T2 = c.w->Tfac + (toff + h) + (int64_t)(toff + h) * nb;
  TRY(gemm64(c.s, 1, 0, 0, 1, 0, h, w - h, (int)(n - r), 1.0, A + r + c0 * lda, lda, A + r + r * lda, lda, 0.0,
             c.w->Xq, nb, 0, 0, 0, 0, c.w->splitk, c.w->splitk_n));
  TRY(gemm64(c.s, 0, 0, 0, 0, 0, h, w - h, h, 1.0, T1, nb, c.w->Xq, nb, 0.0, c.w->Yq, nb, 0));
  return gemm64(c.s, 0, 0, 0, 0, 0, h, w - h, w - h, -1.0, c.w->Yq, nb, T2, nb, 0.0,
                c.w->Tfac + toff + (int64_t)(toff + h) * nb, nb, 0);
}

// Column- and row-side checksum carry of an update C -= X Y over tile-rows
// [I0, N) and tile-columns [J0, N):
//   colchk(2I.., j) -= S(2I.., :) Y(:, j)      gc = Sa |Y|
//   rowchk(i, 2J..) -= X(i, :) Tm(:, 2J..)      gr = |X| Ta
// X(i,p) = Xp[i + p*ldx] for rows [xr0, n) (fx: operand mode of X),
// Y(p,j) = Yp[p + j*ldy] (ty = 0) or Yp[j + p*ldy] (ty = 1) for columns
// [yc0, n); the row-side matrices are Tm / Ta (nb x 2N) or, with tS = 1,
// the transposes of S / Sa (symmetric update, Y = X^T).
template <typename T>
int carry(hipStream_t s, const Ws& w, int64_t n, int nb, int I0, int J0, int kw, const T* Xp, int64_t ldx,
          int64_t xr0, int fx, const T* Yp, int64_t ldy, int ty, int64_t yc0, int tS, int rnd = 0, int rowside = 1) {
  const int N = (int)((n + nb - 1) / nb);
  const int ldS = 2 * N;
  const int isf = sizeof(T) == 4;
  const int mr = 2 * (N - I0), ncol = (int)(n - yc0);
  // column side
  TRY(gemm64(s, 0, ty, 0, 0, 0, mr, ncol, kw, -1.0, w.S + 2 * I0, ldS, Yp, ldy, 1.0, w.colchk + 2 * I0 + yc0 * ldS,
             ldS, 0, 0, isf, rnd));
  TRY(gemm64(s, 0, ty, 0, 2, 0, mr, ncol, kw, 1.0, w.Sa + 2 * I0, ldS, Yp, ldy, 0.0, w.gc + 2 * I0 + yc0 * ldS, ldS,
             0, 0, isf, rnd));
  if (!rowside) return 0;  // single-side checksums: the row side is neither carried nor compared
  // row side
  const int nr = (int)(n - xr0), mc = 2 * (N - J0);
  const double* Bm = tS ? w.S + 2 * J0 : w.Tm + (int64_t)2 * J0 * nb;
  const double* Ba = tS ? w.Sa + 2 * J0 : w.Ta + (int64_t)2 * J0 * nb;
  const int64_t ldb = tS ? ldS : nb;
  TRY(gemm64(s, 0, tS, fx, 0, 0, nr, mc, kw, -1.0, Xp, ldx, Bm, ldb, 1.0, w.rowchk + xr0 + (int64_t)2 * J0 * n, n, 0,
             isf, 0, rnd));
  return gemm64(s, 0, tS, fx == 1 ? 3 : 2, 0, 0, nr, mc, kw, 1.0, Xp, ldx, Ba, ldb, 0.0,
                w.gr + xr0 + (int64_t)2 * J0 * n, n, 0, isf, 0, rnd);
}


inline int op_rnd(int prec) { return prec == ABFT_BF16 ? 1 : (prec == ABFT_F16 ? 2 : 0); }

// Blocked right-looking Cholesky (lower) with per-tile full checksums.
// T = double (prec ABFT_F64) or float (ABFT_F32 / ABFT_BF16 / ABFT_F16).
template <typename T>
int potrf_impl(abft_handle h, int64_t n, T* dA, int64_t lda, const Ws& w, const abft_opts* opts, int nb, int protect,
               double ts, int prec, int32_t* dinfo, abft_report* drep, bool one_stream = false) {
  OffNull off(h, opts, !one_stream);
  // (the look-ahead moves the work to the update stream when on; the
  // Cholesky panel has no cooperative leaf, so any panel share holds it)
  Look la(h, opts, !one_stream && !has_operand_faults(opts), n, nb, 1 << 30);
  hipStream_t s = h->stream;
  TRY(report_init(s, drep, dinfo));
  if (n == 0) return report_fini(s, drep);
  TRY(fill_zero(s, w.pflags, (size_t)((n + nb - 1) / nb) * sizeof(int)));
  const int N = (int)((n + nb - 1) / nb);
  const int ldc = 2 * N;
  const double u = sizeof(T) == 8 ? U64 : U32;
  const double tsu = ts * u, tsu_p = 2.0 * ts * u * sqrt((double)nb);
  const int rnd = op_rnd(prec);
  const bool opf = has_operand_faults(opts);
  const int trole = tmu_role(opts);  // the trailing-update product's launches (and their tile depth)
  Prof pf(h, opts);
  // (nothing to overlap without checksums; operand faults need the update
  // product and the carry in order)
  Side side(h, any_protected(opts, N, protect) && !pf.on && !one_stream && !opf);
  Beside vb(h, opts, !pf.on && !one_stream && !opf && !la.on);
  int t, prev = ABFT_PROTECT_NONE;
  for (int k = 0; k < N; ++k) {
    const int64_t c0 = (int64_t)k * nb;
    const int kw = (int)std::min<int64_t>(nb, n - c0);
    const int64_t c1 = c0 + kw;
    const int lev = level_at(opts, k, protect);
    pf.iters++;
    if (lev > prev) {  // a protected stretch starts from checksums of the data
      TRY(vb.join());
      t = pf.begin(PH_VERIFY);
      TRY(verify_tiles<T>(s, dA, lda, n, n, nb, k, k, 1, 0, w.colchk, ldc, w.rowchk, n, nullptr, nullptr, tsu, nullptr,
                          nullptr, -1));
      pf.end(t);
    }
    prev = lev;
    t = pf.begin(PH_PANEL);
    // (with look-ahead, panel k was factored during iteration k - 1)
    if (!(la.on && k > 0)) TRY(chol_panel(s, dA, lda, n, c0, c1, dinfo));
    TRY(vb.join());  // (the rest of the trailing matrix verified beside the panel)
    // the panel check only reads (the panel, its checksum rows, colchk of the
    // panel's columns): it goes to the side stream with the carry
    const bool fork = side.on && lev && c1 < n;
    auto check_k = [&](hipStream_t cs) -> int {
      // e^T A_Ik = (e^T L_I) L_kk^T:  M(p, j) = L(c0 + j, c0 + p), p <= j
      return panel_check<T>(cs, w.S, w.Sa, ldc, k, N, kw, dA + c0 + c0 * lda, lda, 1, 1, 0, 1.0, nullptr, nullptr,
                            nullptr, -1, w.colchk, ldc, c0, kw, tsu_p, drep, k, nb, w.pflags);
    };
    if (lev) {
      TRY(xsums<T>(s, dA, lda, n, nb, k, c0, kw, k, 1, w.S, w.Sa, ldc, 0));
      if (!fork) TRY(check_k(s));
    }
    pf.end(t);
    if (c1 >= n) break;
    const int64_t m = n - c1;
    T* L21 = dA + c1 + c0 * lda;
    auto carry_k = [&](hipStream_t cs) -> int {
      if (rnd) TRY(xsums<T>(cs, dA, lda, n, nb, k + 1, c0, kw, k, 1, w.S, w.Sa, ldc, rnd));
      return carry<T>(cs, w, n, nb, k + 1, k + 1, kw, L21, lda, c1, 0, L21, lda, 1, c1, 1, rnd,
                      lev == ABFT_PROTECT_FULL);
    };
    if (fork) {
      TRY(side.fork());
      TRY(check_k(side.s));
      TRY(carry_k(side.s));
    }
    if (opf) TRY(apply_operand_faults<T>(s, opts, k, dA, lda, n, nullptr, 0, c1));
    if (la.on) {
      // the next panel's block column first (its lower tiles), the carry
      // joined, that column verified; then panel k + 1 on the panel stream
      // beside the rest of the update and its verification
      const int64_t c2 = std::min<int64_t>(n, c1 + nb);
      const int kw2 = (int)(c2 - c1);
      TRY(gemmT(s, prec, 0, 1, 1, (int)m, kw2, kw, -1.0, L21, lda, L21, lda, 1.0, dA + c1 + c1 * lda, lda, 0, trole));
      if (fork) {
        TRY(side.join());
      } else if (lev) {
        TRY(carry_k(s));
      }
      if (lev) {
        TRY(verify_tiles<T>(s, dA, lda, n, c2, nb, k + 1, k + 1, 1, 1, w.colchk, ldc, w.rowchk, n, w.gc, w.gr, tsu,
                            w.tflags, drep, k, lev));
        TRY(correct_tiles<T>(s, dA, lda, n, c2, nb, k + 1, k + 1, 1, w.colchk, ldc, w.rowchk, n, w.gc, w.gr, tsu,
                             w.tflags, drep, k, lev));
      }
      TRY(la.fork_panel());
      TRY(chol_panel(la.ps, dA, lda, n, c1, c2, dinfo));
      if (c2 < n) {
        const int64_t m2 = n - c2;
        TRY(gemmT(s, prec, 0, 1, 1, (int)m2, (int)m2, kw, -1.0, L21 + kw2, lda, L21 + kw2, lda, 1.0,
                  dA + c2 + c2 * lda, lda, 0, trole));
        if (lev) {
          TRY(verify_tiles<T>(s, dA, lda, n, n, nb, k + 2, k + 2, 1, 1, w.colchk, ldc, w.rowchk, n, w.gc, w.gr, tsu,
                              w.tflags, drep, k, lev));
          TRY(correct_tiles<T>(s, dA, lda, n, n, nb, k + 2, k + 2, 1, w.colchk, ldc, w.rowchk, n, w.gc, w.gr, tsu,
                               w.tflags, drep, k, lev));
        }
      }
      TRY(la.join_panel());
      continue;
    }
    t = pf.begin(PH_TMU);
    TRY(gemmT(s, prec, 0, 1, 1, (int)m, (int)m, kw, -1.0, L21, lda, L21, lda, 1.0, dA + c1 + c1 * lda, lda, 0, trole));
    pf.end(t);
    if (opf) TRY(apply_operand_faults<T>(s, opts, k, dA, lda, n, nullptr, 0, c1));
    pf.tmu_flops += (double)m * (double)(m + 1) * kw;
    pf.tmu_launches++;
    if (fork) {
      TRY(side.join());
    } else if (lev) {
      t = pf.begin(PH_CARRY);
      TRY(carry_k(s));
      pf.end(t);
    }
    int64_t frow = -1, fcol = -1;
    if (opts->faults) TRY(apply_faults<T>(s, opts, k, dA, lda, w, n, N, drep, frow, fcol));
    if (lev) {
      t = pf.begin(PH_VERIFY);
      // with verification beside the next panel: that panel's block column
      // here, the tiles right of it on the restricted stream
      const int64_t c2 = std::min<int64_t>(n, c1 + nb);
      const bool beside = c2 < n && vb.ready();
      const int64_t ncv = beside ? c2 : n;
      TRY(verify_tiles<T>(s, dA, lda, n, ncv, nb, k + 1, k + 1, 1, 1, w.colchk, ldc, w.rowchk, n, w.gc, w.gr, tsu,
                          w.tflags, drep, k, lev, frow, fcol));
      TRY(correct_tiles<T>(s, dA, lda, n, ncv, nb, k + 1, k + 1, 1, w.colchk, ldc, w.rowchk, n, w.gc, w.gr, tsu,
                           w.tflags, drep, k, lev));
      if (beside) {
        TRY(vb.fork());
        TRY(verify_tiles<T>(vb.s, dA, lda, n, n, nb, k + 2, k + 2, 1, 1, w.colchk, ldc, w.rowchk, n, w.gc, w.gr, tsu,
                            w.tflags, drep, k, lev, frow, fcol));
        TRY(correct_tiles<T>(vb.s, dA, lda, n, n, nb, k + 2, k + 2, 1, w.colchk, ldc, w.rowchk, n, w.gc, w.gr, tsu,
                             w.tflags, drep, k, lev));
      }
      pf.end(t);
      const double mt = (double)m / nb;
      pf.verify_bytes += (double)sizeof(T) * nb * nb * (mt * (mt + 1) / 2);
    }
  }
  TRY(report_fini(s, drep));
  pf.finish();
  return 0;
}

// Blocked right-looking LU with partial pivoting and per-tile full checksums.
template <typename T>
int getrf_impl(abft_handle h, int64_t n, T* dA, int64_t lda, int32_t* dipiv, const Ws& w, const abft_opts* opts,
               int nb, int protect, double ts, int prec, int32_t* dinfo, abft_report* drep) {
  OffNull off(h, opts);
  TRY(report_init(h->stream, drep, dinfo));
  if (n == 0) return report_fini(h->stream, drep);
  TRY(fill_zero(h->stream, w.pflags, (size_t)((n + nb - 1) / nb) * sizeof(int)));
  TRY(fill_zero(h->stream, w.ctr, CTR_BYTES));
  TRY(fill_zero(h->stream, w.slots, SLOT_WORDS * sizeof(double)));  // leaf records: sequence numbers restart
  const int N = (int)((n + nb - 1) / nb);
  const int ldc = 2 * N;
  const double u = sizeof(T) == 8 ? U64 : U32;
  const double tsu = ts * u, tsu_p = 2.0 * ts * u * sqrt((double)nb);
  const int rnd = op_rnd(prec);
  const bool opf = has_operand_faults(opts);
  const int trole = tmu_role(opts);  // the trailing-update product's launches (and their tile depth)
  // (the look-ahead moves the work to the update stream when on)
  Look la(h, opts, !opf, n, nb, (int)((144 * 1024) / ((LEAFW + 1) * sizeof(T))));
  hipStream_t s = h->stream;
  Prof pf(h, opts);
  Side side(h, !pf.on && !opf);
  Beside vb(h, opts, !pf.on && !opf && !la.on);
  int t, prev = ABFT_PROTECT_NONE;
  LuCtx<T> c{s, dA, lda, n, dipiv, dinfo, &w, 0u, drep, la.on ? la.mmaxg : std::min(h->cus, 256)};
  T* porig = (T*)w.porig;
  T* stage = (T*)w.stage;
  for (int k = 0; k < N; ++k) {
    const int64_t c0 = (int64_t)k * nb;
    const int kw = (int)std::min<int64_t>(nb, n - c0);
    const int64_t c1 = c0 + kw;
    const int lev = level_at(opts, k, protect);
    pf.iters++;
    if (lev > prev) {  // a protected stretch starts from checksums of the data
      TRY(vb.join());
      t = pf.begin(PH_VERIFY);
      TRY(verify_tiles<T>(s, dA, lda, n, n, nb, k, k, 0, 0, w.colchk, ldc, w.rowchk, n, nullptr, nullptr, tsu, nullptr,
                          nullptr, -1));
      pf.end(t);
    }
    prev = lev;
    t = pf.begin(PH_PANEL);
    if (!(la.on && k > 0)) {  // (with look-ahead, panel k was factored during iteration k - 1)
      if (lev)
        if (hipMemcpy2DAsync(porig, n * sizeof(T), dA + c0 + c0 * lda, lda * sizeof(T), (n - c0) * sizeof(T), kw,
                             hipMemcpyDeviceToDevice, s) != hipSuccess)
          return ABFT_ERR_HIP;
      TRY(lu_panel(c, c0, c1));
    }
    TRY(vb.join());  // (the rest of the trailing matrix verified beside the panel; the interchanges move its rows)
    TRY(perm_build(s, dipiv, c0, kw, n, w.moves));
    // the interchanges of the factored columns to the left and of the row
    // checksums go to the side stream with the carry (nothing before the
    // carry reads them), except after the last panel
    const bool defer = side.on && c1 < n;
    // the panel checks only read (panel, U12, checksum rows, colchk of
    // tile-row k and of the panel's columns): deferred likewise
    auto check_pd = [&](hipStream_t cs) -> int {  // e^T (P A)_I = (e^T L_I) U_kk
      return panel_check<T>(cs, w.S, w.Sa, ldc, k, N, kw, dA + c0 + c0 * lda, 1, lda, 1, 0, 1.0, nullptr, nullptr,
                            nullptr, -1, w.colchk, ldc, c0, kw, tsu_p, drep, k, nb, w.pflags);
    };
    auto check_pu = [&](hipStream_t cs) -> int {  // (e^T L_kk) U12 = e^T A12 on tile-row k
      return panel_check<T>(cs, w.S, w.Sa, ldc, k, k + 1, kw, dA + c0 + c1 * lda, 1, lda, 0, 0, 1.0, nullptr, nullptr,
                            nullptr, -1, w.colchk, ldc, c1, (int)(n - c1), tsu_p, drep, k, nb, w.pflags);
    };
    if (!defer) TRY(laswp(s, dA, lda, 0, c0, w.moves, stage, (double*)nullptr, 0, nb));
    TRY(laswp(s, dA, lda, c1, n, w.moves, stage, lev ? w.colchk : (double*)nullptr, ldc, nb));
    if (lev) {
      // column checksums of the panel follow the interchanges of the original panel values
      TRY(laswp(s, porig - c0, n, 0, kw, w.moves, stage, w.colchk + c0 * ldc, ldc, nb));
      if (!defer) TRY(laswp(s, w.rowchk, n, 0, 2 * N, w.moves, (double*)w.stage, (double*)nullptr, 0, nb));
      TRY(xsums<T>(s, dA, lda, n, nb, k, c0, kw, k, 2, w.S, w.Sa, ldc, 0));
      if (!defer) TRY(check_pd(s));
    }
    if (c1 >= n) {
      pf.end(t);
      break;
    }
    pf.end(t);
    t = pf.begin(PH_PU);
    TRY(trsm_llu(s, dA, lda, c0, kw, c1, n));
    if (lev && !defer) TRY(check_pu(s));
    pf.end(t);
    const int64_t m = n - c1;
    T* L21 = dA + c1 + c0 * lda;
    T* U12 = dA + c0 + c1 * lda;
    auto carry_k = [&](hipStream_t cs) -> int {
      if (rnd) TRY(xsums<T>(cs, dA, lda, n, nb, k + 1, c0, kw, k, 2, w.S, w.Sa, ldc, rnd));
      if (lev == ABFT_PROTECT_FULL) TRY(ysums<T>(cs, dA + c0, lda, n, nb, k + 1, kw, w.Tm, w.Ta, nb, rnd));
      return carry<T>(cs, w, n, nb, k + 1, k + 1, kw, L21, lda, c1, 0, U12, lda, 0, c1, 0, rnd,
                      lev == ABFT_PROTECT_FULL);
    };
    if (side.on) {  // (w.moves, w.stage and porig stay unchanged until the join)
      TRY(side.fork());
      TRY(laswp(side.s, dA, lda, 0, c0, w.moves, stage, (double*)nullptr, 0, nb));
      if (lev) {
        TRY(check_pd(side.s));
        TRY(check_pu(side.s));
        TRY(laswp(side.s, w.rowchk, n, 0, 2 * N, w.moves, (double*)w.stage, (double*)nullptr, 0, nb));
        TRY(carry_k(side.s));
      }
    }
    if (opf) TRY(apply_operand_faults<T>(s, opts, k, dA, lda, n, nullptr, 0, c1));
    if (la.on) {
      // the next panel's block column first: update, carry (joined), verify
      const int64_t c2 = std::min<int64_t>(n, c1 + nb);
      const int kw2 = (int)(c2 - c1);
      TRY(gemmT(s, prec, 0, 0, 0, (int)m, kw2, kw, -1.0, L21, lda, U12, lda, 1.0, dA + c1 + c1 * lda, lda, 0, trole));
      TRY(side.join());
      if (lev) {
        TRY(verify_tiles<T>(s, dA, lda, n, c2, nb, k + 1, k + 1, 0, 1, w.colchk, ldc, w.rowchk, n, w.gc, w.gr, tsu,
                            w.tflags, drep, k, lev));
        TRY(correct_tiles<T>(s, dA, lda, n, c2, nb, k + 1, k + 1, 0, w.colchk, ldc, w.rowchk, n, w.gc, w.gr, tsu,
                             w.tflags, drep, k, lev));
      }
      // panel k + 1 on the panel stream, beside the rest of the update
      TRY(la.fork_panel());
      if (lev)
        if (hipMemcpy2DAsync(porig, n * sizeof(T), dA + c1 + c1 * lda, lda * sizeof(T), (n - c1) * sizeof(T), kw2,
                             hipMemcpyDeviceToDevice, la.ps) != hipSuccess)
          return ABFT_ERR_HIP;
      c.s = la.ps;
      c.maxg = la.pmaxg;
      const int prc = lu_panel(c, c1, c2);
      c.s = s;
      c.maxg = la.mmaxg;
      TRY(prc);
      if (c2 < n) {
        TRY(gemmT(s, prec, 0, 0, 0, (int)m, (int)(n - c2), kw, -1.0, L21, lda, U12 + (int64_t)kw2 * lda, lda, 1.0,
                  dA + c1 + c2 * lda, lda, 0, trole));
        if (lev) {
          TRY(verify_tiles<T>(s, dA, lda, n, n, nb, k + 1, k + 2, 0, 1, w.colchk, ldc, w.rowchk, n, w.gc, w.gr, tsu,
                              w.tflags, drep, k, lev));
          TRY(correct_tiles<T>(s, dA, lda, n, n, nb, k + 1, k + 2, 0, w.colchk, ldc, w.rowchk, n, w.gc, w.gr, tsu,
                               w.tflags, drep, k, lev));
        }
      }
      TRY(la.join_panel());
      continue;
    }
    t = pf.begin(PH_TMU);
    TRY(gemmT(s, prec, 0, 0, 0, (int)m, (int)m, kw, -1.0, L21, lda, U12, lda, 1.0, dA + c1 + c1 * lda, lda, 0, trole));
    pf.end(t);
    if (opf) TRY(apply_operand_faults<T>(s, opts, k, dA, lda, n, nullptr, 0, c1));
    pf.tmu_flops += 2.0 * (double)m * (double)m * kw;
    pf.tmu_launches++;
    if (side.on) {
      TRY(side.join());
    } else if (lev) {
      t = pf.begin(PH_CARRY);
      TRY(carry_k(s));
      pf.end(t);
    }
    int64_t frow = -1, fcol = -1;
    if (opts->faults) TRY(apply_faults<T>(s, opts, k, dA, lda, w, n, N, drep, frow, fcol));
    if (lev) {
      t = pf.begin(PH_VERIFY);
      const int64_t c2 = std::min<int64_t>(n, c1 + nb);
      const bool beside = c2 < n && vb.ready();
      const int64_t ncv = beside ? c2 : n;
      TRY(verify_tiles<T>(s, dA, lda, n, ncv, nb, k + 1, k + 1, 0, 1, w.colchk, ldc, w.rowchk, n, w.gc, w.gr, tsu,
                          w.tflags, drep, k, lev, frow, fcol));
      TRY(correct_tiles<T>(s, dA, lda, n, ncv, nb, k + 1, k + 1, 0, w.colchk, ldc, w.rowchk, n, w.gc, w.gr, tsu,
                           w.tflags, drep, k, lev));
      if (beside) {
        TRY(vb.fork());
        TRY(verify_tiles<T>(vb.s, dA, lda, n, n, nb, k + 1, k + 2, 0, 1, w.colchk, ldc, w.rowchk, n, w.gc, w.gr, tsu,
                            w.tflags, drep, k, lev, frow, fcol));
        TRY(correct_tiles<T>(vb.s, dA, lda, n, n, nb, k + 1, k + 2, 0, w.colchk, ldc, w.rowchk, n, w.gc, w.gr, tsu,
                             w.tflags, drep, k, lev));
      }
      pf.end(t);
      pf.verify_bytes += (double)sizeof(T) * (double)m * (double)m;
    }
  }
  TRY(report_fini(s, drep));
  pf.finish();
  return la.finish();
}


// ------------------------------------------------------------ mixed precision
// Extra workspace of the mixed-precision solve, after the factorization's.
struct MpWs {
  void* F;          // factor copy (float, or double for the FP64 reference)
  int32_t *ipiv, *perm, *info;
  uint64_t* xw;  // solution words of the triangular solves (2n)
  unsigned* counter;
  double *r, *xd, *part, *norms;
  float* d32;
  size_t bytes;
};
constexpr int NSPLIT = 32;

MpWs carve_mp(char* base, size_t off, int64_t n, int elem) {
  MpWs m;
  memset(&m, 0, sizeof(m));
  auto take = [&](size_t b) -> char* {
    char* p = base ? base + off : nullptr;
    off += al(b);
    return p;
  };
  m.F = take((size_t)n * n * elem);
  m.ipiv = (int32_t*)take((size_t)n * 4);
  m.perm = (int32_t*)take((size_t)n * 4);
  m.info = (int32_t*)take(256);
  m.counter = (unsigned*)take(256);
  m.xw = (uint64_t*)take((size_t)n * 16);
  m.r = (double*)take((size_t)n * 8);
  m.xd = (double*)take((size_t)n * 8);
  m.part = (double*)take((size_t)NSPLIT * n * 8);
  m.norms = (double*)take(256);
  m.d32 = (float*)take((size_t)n * 4);
  m.bytes = off;
  return m;
}

int read_norms(hipStream_t s, const double* dn, double* hn, int cnt) {
  if (hipMemcpyAsync(hn, dn, cnt * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess) return ABFT_ERR_HIP;
  return hipStreamSynchronize(s) == hipSuccess ? 0 : ABFT_ERR_HIP;
}

// x := M^{-1} P x for the factor of the solve (float or double data)
template <typename T>
int solve_factor(hipStream_t s, const T* F, int64_t n, const int* perm, int chol, T* x, const MpWs& m,
                 uint32_t& seq, abft_report* rep) {
  (void)perm;
  TRY(trsv<T>(s, F, n, (int)n, chol ? 2 : 0, x, m.counter, m.xw, ++seq, rep));
  return trsv<T>(s, F, n, (int)n, chol ? 3 : 1, x, m.counter, m.xw, ++seq, rep);
}

int gesv_mp_impl(abft_handle h, int64_t n, const double* dA, int64_t lda, const double* db, double* dx, int prec,
                 int max_iter, void* dwork, size_t work_bytes, const abft_opts* opts, abft_ir_report* dir,
                 abft_report* drep, int chol) {
  if (!h) return -1;
  if (n < 0) return -2;
  if (!dA && n > 0) return -3;
  if (lda < std::max<int64_t>(1, n)) return -4;
  if (!db && n > 0) return -5;
  if (!dx && n > 0) return -6;
  if (prec < ABFT_F64 || prec > ABFT_F16) return -7;
  if (max_iter < 0) return -8;
  int nb, protect;
  double ts;
  TRY(check_opts(opts, n, nb, protect, ts));
  if (n > 40000) return ABFT_ERR_UNSUPPORTED;
  hipStream_t s = h->stream;
  const int elem = prec == ABFT_F64 ? 8 : 4;
  use_ws(h, dwork, work_bytes);
  Ws w = carve((char*)dwork, n, nb, chol ? ABFT_OP_POTRF : ABFT_OP_GETRF, elem);
  MpWs m = carve_mp((char*)dwork, w.bytes, n, elem);
  if (!dwork || work_bytes < m.bytes) return ABFT_ERR_WORKSPACE;
  abft_ir_report ir;
  memset(&ir, 0, sizeof(ir));
  auto finish = [&]() -> int {
    if (dir && hipMemcpyAsync(dir, &ir, sizeof(ir), hipMemcpyHostToDevice, s) != hipSuccess) return ABFT_ERR_HIP;
    return hipStreamSynchronize(s) == hipSuccess ? 0 : ABFT_ERR_HIP;
  };
  if (n == 0) {
    TRY(report_init(s, drep, m.info));
    TRY(report_fini(s, drep));
    ir.converged = 1;
    return finish();
  }
  const int ni = (int)n;
  double hn[8];
  uint32_t seq = 0;  // sequence numbers of the triangular solves (their words start cleared)
  TRY(fill_zero(s, m.xw, (size_t)n * 16));
  // factorization of a working copy
  if (prec == ABFT_F64) {
    if (hipMemcpy2DAsync(m.F, n * 8, dA, lda * 8, n * 8, n, hipMemcpyDeviceToDevice, s) != hipSuccess)
      return ABFT_ERR_HIP;
    if (chol) TRY(potrf_impl<double>(h, n, (double*)m.F, n, w, opts, nb, protect, ts, prec, m.info, drep));
    else TRY(getrf_impl<double>(h, n, (double*)m.F, n, m.ipiv, w, opts, nb, protect, ts, prec, m.info, drep));
  } else {
    TRY(convert_f64_f32(s, dA, lda, (float*)m.F, n, n, n));
    if (chol) TRY(potrf_impl<float>(h, n, (float*)m.F, n, w, opts, nb, protect, ts, prec, m.info, drep));
    else TRY(getrf_impl<float>(h, n, (float*)m.F, n, m.ipiv, w, opts, nb, protect, ts, prec, m.info, drep));
  }
  TRY(fill_zero(s, m.norms, 64));
  TRY(anorm(s, dA, lda, ni, m.part, NSPLIT, m.norms));
  if (hipMemcpyAsync(&ir.info, m.info, 4, hipMemcpyDeviceToHost, s) != hipSuccess) return ABFT_ERR_HIP;
  TRY(read_norms(s, m.norms, hn, 8));
  ir.a_norm = hn[4];
  if (ir.info != 0) {
    ir.failed_reason = 4;
    return finish();
  }
  const int* perm = nullptr;
  if (!chol) {
    TRY(perm_vector(s, m.ipiv, ni, m.perm));
    perm = m.perm;
  }
  const double u = U64;
  if (prec == ABFT_F64) {
    // direct FP64 solve (reference method)
    TRY(gather64(s, db, perm, m.xd, ni));
    TRY(solve_factor<double>(s, (const double*)m.F, n, perm, chol, m.xd, m, seq, drep));
    TRY(copy_f64(s, m.xd, dx, ni));
    TRY(fill_zero(s, m.norms, 32));
    TRY(residual(s, dA, lda, ni, dx, db, m.r, m.part, NSPLIT, m.norms));
    TRY(read_norms(s, m.norms, hn, 2));
    ir.resid_norm = hn[0];
    ir.x_norm = hn[1];
    ir.converged = 1;
    return finish();
  }
  // x0 from the low-precision factors
  TRY(gather_scale(s, db, perm, 1.0, m.d32, ni));
  TRY(solve_factor<float>(s, (const float*)m.F, n, perm, chol, m.d32, m, seq, drep));
  TRY(f32_to_f64(s, m.d32, dx, ni));
  double prev = INFINITY;
  for (int it = 1; it <= max_iter; ++it) {
    TRY(fill_zero(s, m.norms, 32));
    TRY(residual(s, dA, lda, ni, dx, db, m.r, m.part, NSPLIT, m.norms));
    TRY(read_norms(s, m.norms, hn, 2));
    const double rn = hn[0], xn = hn[1];
    ir.resid_norm = rn;
    ir.x_norm = xn;
    if (!(rn <= 1.79e308) || !(xn <= 1.79e308)) { ir.failed_reason = 2; break; }
    if (rn <= u * ir.a_norm * xn) { ir.converged = 1; break; }
    const double sc = rn > 0 ? rn : 1.0;
    TRY(gather_scale(s, m.r, perm, 1.0 / sc, m.d32, ni));
    TRY(solve_factor<float>(s, (const float*)m.F, n, perm, chol, m.d32, m, seq, drep));
    TRY(update_x(s, dx, m.d32, sc, ni, m.norms));
    TRY(read_norms(s, m.norms, hn, 4));
    const double dn = hn[2], xn2 = hn[3];
    ir.last_dx = dn;
    ir.iters = it;
    if (!(dn <= 1.79e308)) { ir.failed_reason = 2; break; }
    if (dn <= u * xn2) { ir.converged = 1; break; }
    if (it >= 2 && dn > 0.5 * prev && dn > 1e3 * u * xn2) { ir.failed_reason = 1; break; }
    prev = dn;
  }
  if (!ir.converged && !ir.failed_reason) ir.failed_reason = 3;
  return finish();
}

}  // namespace

// ------------------------------------------------------ no-allocation scratch
// Scratch of abft_potrf_noalloc: a device array in the library's code object,
// so that entry point needs no workspace argument and allocates nothing.  Each
// GPU holds its own copy (at its own address) until the process ends.  Host
// code never uses the array's name as an address (it is a host-side stand-in);
// the device address of each GPU's copy is looked up once, with that device
// current, and kept in g_scratch.
constexpr size_t NOALLOC_BYTES = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];
constexpr int MAX_DEVICES = 64;
static void* g_scratch[MAX_DEVICES];
static std::mutex g_scratch_mu;

static int scratch_ptr(int device, void** out) {
  if (device < 0 || device >= MAX_DEVICES) return ABFT_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[device]) {
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return ABFT_ERR_HIP;
    if (cur != device && hipSetDevice(device) != hipSuccess) return ABFT_ERR_HIP;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess || !p) return ABFT_ERR_HIP;
    g_scratch[device] = p;
  }
  *out = g_scratch[device];
  return 0;
}

// ===================================================================== ABI
extern "C" {

int abft_create(abft_handle* h, void* stream) {
  if (!h) return -1;
  abft_handle p = (abft_handle)calloc(1, sizeof(abft_handle_s));
  if (!p) return ABFT_ERR_HIP;
  p->stream = (hipStream_t)stream;
  if (hipGetDevice(&p->device) != hipSuccess) { free(p); return ABFT_ERR_HIP; }
  if (hipDeviceGetAttribute(&p->cus, hipDeviceAttributeMultiprocessorCount, p->device) != hipSuccess) {
    free(p);
    return ABFT_ERR_HIP;
  }
  // the no-allocation scratch of this device (abft_potrf_noalloc retries the
  // lookup, and fails loudly, if it did not succeed here)
  void* sp = nullptr;
  (void)scratch_ptr(p->device, &sp);
  *h = p;
  return 0;
}

int abft_destroy(abft_handle h) {
  if (!h) return 0;
  // finish every call still in flight on the handle's streams before their
  // streams, events and graphs go away
  int rc = 0;
  if (hipStreamSynchronize(h->stream) != hipSuccess) rc = ABFT_ERR_HIP;
  if (h->side && hipStreamSynchronize(h->side) != hipSuccess) rc = ABFT_ERR_HIP;
  if (h->cap && hipStreamSynchronize(h->cap) != hipSuccess) rc = ABFT_ERR_HIP;
  if (h->ev) {
    for (int i = 0; i < h->nev; ++i) (void)hipEventDestroy(h->ev[i]);
    free(h->ev);
  }
  for (int i = 0; i < h->ngraphs; ++i) (void)hipGraphExecDestroy(h->graphs[i].exec);
  if (h->cap) (void)hipStreamDestroy(h->cap);
  if (h->side) {
    (void)hipStreamDestroy(h->side);
    (void)hipEventDestroy(h->fork_ev);
    (void)hipEventDestroy(h->join_ev);
  }
  if (h->la_main) {
    if (hipStreamSynchronize(h->la_main) != hipSuccess) rc = ABFT_ERR_HIP;
    if (hipStreamSynchronize(h->la_panel) != hipSuccess) rc = ABFT_ERR_HIP;
    (void)hipStreamDestroy(h->la_main);
    (void)hipStreamDestroy(h->la_panel);
  }
  for (int i = 0; i < 4; ++i)
    if (h->la_ev[i]) (void)hipEventDestroy(h->la_ev[i]);
  if (h->vb) {
    if (hipStreamSynchronize(h->vb) != hipSuccess) rc = ABFT_ERR_HIP;
    (void)hipStreamDestroy(h->vb);
  }
  if (h->own) {
    if (hipStreamSynchronize(h->own) != hipSuccess) rc = ABFT_ERR_HIP;
    (void)hipStreamDestroy(h->own);
  }
  for (int i = 0; i < 2; ++i)
    if (h->own_ev[i]) (void)hipEventDestroy(h->own_ev[i]);
  for (int i = 0; i < 2; ++i)
    if (h->vb_ev[i]) (void)hipEventDestroy(h->vb_ev[i]);
  free(h->iter_ms);
  free(h);
  return rc;
}

int abft_set_stream(abft_handle h, void* stream) {
  if (!h) return -1;
  h->stream = (hipStream_t)stream;
  return 0;
}

int abft_set_workspace(abft_handle h, void* dwork, size_t bytes) {
  if (!h) return -1;
  if (!dwork && bytes) return -2;
  h->ws = dwork;
  h->ws_bytes = dwork ? bytes : 0;
  return 0;
}

int abft_report_fetch(abft_handle h, const abft_report* drep, abft_report* out) {
  if (!h) return -1;
  if (!drep) return -2;
  if (!out) return -3;
  if (hipMemcpyAsync(out, drep, sizeof(abft_report), hipMemcpyDeviceToHost, h->stream) != hipSuccess)
    return ABFT_ERR_HIP;
  return hipStreamSynchronize(h->stream) == hipSuccess ? 0 : ABFT_ERR_HIP;
}

int abft_get_profile(abft_handle h, abft_profile* out) {
  if (!h) return -1;
  if (!out) return -2;
  *out = h->prof;
  return 0;
}

int abft_get_iter_profile(abft_handle h, int32_t cap, double* ms, int32_t* iters) {
  if (!h) return -1;
  if (cap < 0) return -2;
  if (!ms && cap > 0) return -3;
  if (!iters) return -4;
  const int n = std::min<int>(cap, h->iter_n);
  for (int ph = 0; ph < PH_N; ++ph)
    for (int k = 0; k < n; ++k) ms[ph * cap + k] = h->iter_ms[ph * h->iter_n + k];
  *iters = h->iter_n;
  return 0;
}

int abft_workspace_size(abft_handle h, int op, int64_t n, int32_t batch, const abft_opts* opts, size_t* bytes) {
  (void)h;
  (void)batch;
  if (!bytes) return -6;
  if (n < 0) return -3;
  int nb, protect;
  double ts;
  TRY(check_opts(opts, n, nb, protect, ts));
  if (op == ABFT_OP_POTRF_BATCHED || op == ABFT_OP_GETRF_BATCHED) {
    if (batch < 0) return -4;
    *bytes = batched_ws_bytes(batch);
    return 0;
  }
  if (op == ABFT_OP_GESV_MP || op == ABFT_OP_POSV_MP) {
    // sized for the largest precision (the FP64 reference solve)
    Ws w = carve(nullptr, n, nb, op == ABFT_OP_POSV_MP ? ABFT_OP_POTRF : ABFT_OP_GETRF, sizeof(double));
    *bytes = carve_mp(nullptr, w.bytes, n, sizeof(double)).bytes;
    return 0;
  }
  if (op < ABFT_OP_POTRF || op > ABFT_OP_GEQRF) return ABFT_ERR_UNSUPPORTED;
  Ws w = carve(nullptr, n, nb, op, sizeof(double));
  *bytes = w.bytes;
  return 0;
}

int abft_potrf(abft_handle h, int64_t n, double* dA, int64_t lda, void* dwork, size_t work_bytes,
               const abft_opts* opts, int32_t* dinfo, abft_report* drep) {
  if (!h) return -1;
  if (n < 0) return -2;
  if (!dA && n > 0) return -3;
  if (lda < std::max<int64_t>(1, n)) return -4;
  int nb, protect;
  double ts;
  TRY(check_opts(opts, n, nb, protect, ts));
  if (!dinfo) return -8;
  use_ws(h, dwork, work_bytes);
  Ws w = carve((char*)dwork, n, nb, ABFT_OP_POTRF, sizeof(double));
  if (!dwork || work_bytes < w.bytes) return ABFT_ERR_WORKSPACE;
  return potrf_impl<double>(h, n, dA, lda, w, opts, nb, protect, ts, ABFT_F64, dinfo, drep);
}

int abft_potrf_noalloc(abft_handle h, int64_t n, double* dA, int64_t lda, const abft_opts* opts, int32_t* dinfo,
                       abft_report* drep) {
  if (!h) return -1;
  if (n < 0) return -2;
  if (!dA && n > 0) return -3;
  if (lda < std::max<int64_t>(1, n)) return -4;
  int nb, protect;
  double ts;
  TRY(check_opts(opts, n, nb, protect, ts));
  if (opts->flags & ABFT_FLAG_PROFILE) return ABFT_ERR_UNSUPPORTED;  // (profiling creates events)
  if (!dinfo) return -6;
  const size_t need = carve(nullptr, n, nb, ABFT_OP_POTRF, sizeof(double)).bytes;
  if (need > NOALLOC_BYTES) return ABFT_ERR_WORKSPACE;
  void* base = nullptr;
  TRY(scratch_ptr(h->device, &base));
  Ws w = carve((char*)base, n, nb, ABFT_OP_POTRF, sizeof(double));
  return potrf_impl<double>(h, n, dA, lda, w, opts, nb, protect, ts, ABFT_F64, dinfo, drep, true);
}

int abft_getrf(abft_handle h, int64_t n, double* dA, int64_t lda, int32_t* dipiv, void* dwork, size_t work_bytes,
               const abft_opts* opts, int32_t* dinfo, abft_report* drep) {
  if (!h) return -1;
  if (n < 0) return -2;
  if (!dA && n > 0) return -3;
  if (lda < std::max<int64_t>(1, n)) return -4;
  if (!dipiv && n > 0) return -5;
  int nb, protect;
  double ts;
  TRY(check_opts(opts, n, nb, protect, ts));
  if (!dinfo) return -9;
  use_ws(h, dwork, work_bytes);
  Ws w = carve((char*)dwork, n, nb, ABFT_OP_GETRF, sizeof(double));
  if (!dwork || work_bytes < w.bytes) return ABFT_ERR_WORKSPACE;
  return getrf_impl<double>(h, n, dA, lda, dipiv, w, opts, nb, protect, ts, ABFT_F64, dinfo, drep);
}

int abft_geqrf(abft_handle h, int64_t n, double* dA, int64_t lda, double* dtau, void* dwork, size_t work_bytes,
               const abft_opts* opts, int32_t* dinfo, abft_report* drep) {
  if (!h) return -1;
  if (n < 0) return -2;
  if (!dA && n > 0) return -3;
  if (lda < std::max<int64_t>(1, n)) return -4;
  if (!dtau && n > 0) return -5;
  int nb, protect;
  double ts;
  TRY(check_opts(opts, n, nb, protect, ts));
  if (!dinfo) return -9;
  use_ws(h, dwork, work_bytes);
  Ws w = carve((char*)dwork, n, nb, ABFT_OP_GEQRF, sizeof(double));
  if (!dwork || work_bytes < w.bytes) return ABFT_ERR_WORKSPACE;
  OffNull off(h, opts);
  TRY(report_init(h->stream, drep, dinfo));
  if (n == 0) return report_fini(h->stream, drep);
  TRY(fill_zero(h->stream, w.pflags, (size_t)((n + nb - 1) / nb) * sizeof(int)));
  TRY(fill_zero(h->stream, w.ctr, CTR_BYTES));
  TRY(fill_zero(h->stream, w.slots, SLOT_WORDS * sizeof(double)));  // leaf records: sequence numbers restart
  const int N = (int)((n + nb - 1) / nb);
  const int ldc = 2 * N;
  const double tsu = ts * U64, tsu_p = 2.0 * ts * U64 * sqrt((double)nb);
  const bool opf = has_operand_faults(opts);
  const int trole = tmu_role(opts);  // the trailing-update product's launches (and their tile depth)
  // (the look-ahead moves the work to the update stream when on)
  Look la(h, opts, !opf, n, nb, (int)((140 * 1024) / ((LEAFW + 1) * sizeof(double))));
  hipStream_t s = h->stream;
  QrCtx c{s, dA, lda, n, dtau, &w, nb, 0, 0u, drep, la.on ? la.mmaxg : std::min(h->cus, 256)};
  Prof pf(h, opts);
  Side side(h, any_protected(opts, N, protect) && !pf.on && !opf);
  Beside vb(h, opts, !pf.on && !opf && !la.on);
  int t, prev = ABFT_PROTECT_NONE;
  for (int k = 0; k < N; ++k) {
    const int64_t c0 = (int64_t)k * nb;
    const int kw = (int)std::min<int64_t>(nb, n - c0);
    const int64_t c1 = c0 + kw;
    const int lev = level_at(opts, k, protect);
    c.cb = c0;
    pf.iters++;
    if (lev > prev) {  // a protected stretch starts from checksums of the data
      TRY(vb.join());
      TRY(verify_tiles<double>(s, dA, lda, n, n, nb, k, k, 0, 0, w.colchk, ldc, w.rowchk, n, nullptr, nullptr, tsu,
                               nullptr, nullptr, -1));
    }
    prev = lev;
    t = pf.begin(PH_PANEL);
    if (!(la.on && k > 0)) {  // (with look-ahead, panel k was factored during iteration k - 1)
      TRY(fill_zero(s, w.Tfac, (size_t)nb * nb * sizeof(double)));
      TRY(qr_panel(c, c0, c1));
    }
    TRY(vb.join());  // (the rest of the trailing matrix verified beside the panel)
    // the panel check reads the panel, T and colchk of the panel's columns
    // only: on the side stream it runs beside the trailing update
    auto check_k = [&](hipStream_t cs) -> int {
      TRY(qr_check_prep(cs, dA, lda, c0, kw, n - c0, w.Tfac, nb, w.scr, w.Z, w.Zabs, w.E, w.bt));
      // e^T A_I = [I==k] e^T R - (e^T V_I) T V1^T R
      return panel_check(cs, w.S, w.Sa, ldc, k, N, kw, w.Z, 1, kw, 0, 0, -1.0, w.Zabs, w.E, w.bt, k, w.colchk, ldc,
                         c0, kw, tsu_p, drep, k, nb, w.pflags);
    };
    const bool fork = side.on && lev && c1 < n;
    if (lev) {
      TRY(xsums<double>(s, dA, lda, n, nb, k, c0, kw, k, 2, w.S, w.Sa, ldc, 0));
      if (fork) {
        TRY(side.fork());
        TRY(check_k(side.s));
      } else {
        TRY(check_k(s));
      }
    }
    pf.end(t);
    if (c1 >= n) break;
    const int64_t m = n - c1;
    double* V = dA + c0 + c0 * lda;
    double* C = dA + c0 + c1 * lda;
    // C -= V T^T V^T C: the two products with the full panel height are the
    // trailing update proper (timed per launch); W2 = T^T W is a small product
    int S = 0;
    t = pf.begin(PH_TMU);
    TRY(gemm64(s, 1, 0, 1, 0, 0, kw, (int)m, (int)(n - c0), 1.0, V, lda, C, lda, 0.0, w.W, nb, 0, 0, 0, 0, w.splitk,
               w.splitk_n, trole, &S));
    pf.end(t);
    if (S > 1) TRY(splitk_reduce(s, w.splitk, S, kw, (int)m, 0.0, w.W, nb));
    TRY(gemm64(s, 1, 0, 0, 0, 0, kw, (int)m, kw, 1.0, w.Tfac, nb, w.W, nb, 0.0, w.W2, nb, 0));
    auto carry_k = [&](hipStream_t cs) -> int {
      if (lev == ABFT_PROTECT_FULL) TRY(ysums<double>(cs, w.W2 - c1 * nb, nb, n, nb, k + 1, kw, w.Tm, w.Ta, nb, 0));
      return carry(cs, w, n, nb, k, k + 1, kw, V, lda, c0, 1, w.W2, nb, 0, c1, 0, 0, lev == ABFT_PROTECT_FULL);
    };
    if (fork) {  // (W2 is final here; the second product only reads it)
      TRY(side.fork());
      TRY(carry_k(side.s));
    }
    if (opf) TRY(apply_operand_faults<double>(s, opts, k, dA, lda, n, w.W2, nb, c1));
    if (la.on) {
      // the next panel's block column first: update, carry and panel check
      // (joined: the next panel overwrites T), verify
      const int64_t c2 = std::min<int64_t>(n, c1 + nb);
      const int kw2 = (int)(c2 - c1);
      TRY(gemm64(s, 0, 0, 1, 0, 0, (int)(n - c0), kw2, kw, -1.0, V, lda, w.W2, nb, 1.0, C, lda, 0, 0, 0, 0, nullptr, 0,
                 trole));
      if (fork) {
        TRY(side.join());
      } else if (lev) {
        TRY(carry_k(s));
      }
      if (lev) {
        TRY(verify_tiles<double>(s, dA, lda, n, c2, nb, k, k + 1, 0, 1, w.colchk, ldc, w.rowchk, n, w.gc, w.gr, tsu,
                                 w.tflags, drep, k, lev));
        TRY(correct_tiles<double>(s, dA, lda, n, c2, nb, k, k + 1, 0, w.colchk, ldc, w.rowchk, n, w.gc, w.gr, tsu,
                                  w.tflags, drep, k, lev));
      }
      // panel k + 1 on the panel stream, beside the rest of the update
      TRY(la.fork_panel());
      c.s = la.ps;
      c.maxg = la.pmaxg;
      c.cb = c1;
      int prc = fill_zero(la.ps, w.Tfac, (size_t)nb * nb * sizeof(double));
      if (!prc) prc = qr_panel(c, c1, c2);
      c.s = s;
      c.maxg = la.mmaxg;
      TRY(prc);
      if (c2 < n) {
        TRY(gemm64(s, 0, 0, 1, 0, 0, (int)(n - c0), (int)(n - c2), kw, -1.0, V, lda, w.W2 + (int64_t)kw2 * nb, nb, 1.0,
                   C + (int64_t)kw2 * lda, lda, 0, 0, 0, 0, nullptr, 0, trole));
        if (lev) {
          TRY(verify_tiles<double>(s, dA, lda, n, n, nb, k, k + 2, 0, 1, w.colchk, ldc, w.rowchk, n, w.gc, w.gr, tsu,
                                   w.tflags, drep, k, lev));
          TRY(correct_tiles<double>(s, dA, lda, n, n, nb, k, k + 2, 0, w.colchk, ldc, w.rowchk, n, w.gc, w.gr, tsu,
                                    w.tflags, drep, k, lev));
        }
      }
      TRY(la.join_panel());
      continue;
    }
    t = pf.begin(PH_TMU);
    TRY(gemm64(s, 0, 0, 1, 0, 0, (int)(n - c0), (int)m, kw, -1.0, V, lda, w.W2, nb, 1.0, C, lda, 0, 0, 0, 0, nullptr,
               0, trole));
    pf.end(t);
    if (opf) TRY(apply_operand_faults<double>(s, opts, k, dA, lda, n, w.W2, nb, c1));
    pf.tmu_flops += 4.0 * (double)(n - c0) * (double)m * kw;
    pf.tmu_launches += 2;
    if (fork) {
      TRY(side.join());
    } else if (lev) {
      t = pf.begin(PH_CARRY);
      TRY(carry_k(s));
      pf.end(t);
    }
    int64_t frow = -1, fcol = -1;
    if (opts->faults) TRY(apply_faults<double>(s, opts, k, dA, lda, w, n, N, drep, frow, fcol));
    if (lev) {
      t = pf.begin(PH_VERIFY);
      const int64_t c2 = std::min<int64_t>(n, c1 + nb);
      const bool beside = c2 < n && vb.ready();
      const int64_t ncv = beside ? c2 : n;
      TRY(verify_tiles<double>(s, dA, lda, n, ncv, nb, k, k + 1, 0, 1, w.colchk, ldc, w.rowchk, n, w.gc, w.gr, tsu,
                               w.tflags, drep, k, lev, frow, fcol));
      TRY(correct_tiles<double>(s, dA, lda, n, ncv, nb, k, k + 1, 0, w.colchk, ldc, w.rowchk, n, w.gc, w.gr, tsu,
                                w.tflags, drep, k, lev));
      if (beside) {
        TRY(vb.fork());
        TRY(verify_tiles<double>(vb.s, dA, lda, n, n, nb, k, k + 2, 0, 1, w.colchk, ldc, w.rowchk, n, w.gc, w.gr,
                                 tsu, w.tflags, drep, k, lev, frow, fcol));
        TRY(correct_tiles<double>(vb.s, dA, lda, n, n, nb, k, k + 2, 0, w.colchk, ldc, w.rowchk, n, w.gc, w.gr, tsu,
                                  w.tflags, drep, k, lev));
      }
      pf.end(t);
      pf.verify_bytes += 8.0 * (double)(n - c0) * (double)m;
    }
  }
  TRY(report_fini(s, drep));
  pf.finish();
  return la.finish();
}

int abft_gemm(abft_handle h, int32_t transa, int32_t transb, int32_t flags, int64_t m, int64_t n, int64_t k,
              double alpha, const double* dA, int64_t lda, const double* dB, int64_t ldb, double beta, double* dC,
              int64_t ldc, void* dwork, size_t work_bytes) {
  if (!h) return -1;
  if (transa != 0 && transa != 1) return -2;
  if (transb != 0 && transb != 1) return -3;
  if (flags & ~(ABFT_GEMM_LOWER | ABFT_GEMM_UNIT_LOWER_A)) return -4;
  const int64_t lim = 0x7fffffff;
  if (m < 0 || m > lim) return -5;
  if (n < 0 || n > lim) return -6;
  if (k < 0 || k > lim) return -7;
  if (lda < std::max<int64_t>(1, transa ? k : m)) return -10;
  if (ldb < std::max<int64_t>(1, transb ? n : k)) return -12;
  if (ldc < std::max<int64_t>(1, m)) return -15;
  if (m == 0 || n == 0) return 0;
  const int lower = (flags & ABFT_GEMM_LOWER) ? 1 : 0, fa = (flags & ABFT_GEMM_UNIT_LOWER_A) ? 1 : 0;
  if (transa && transb) return ABFT_ERR_UNSUPPORTED;
  if (lower && !(transa == 0 && transb == 1)) return ABFT_ERR_UNSUPPORTED;
  if (fa && transb) return ABFT_ERR_UNSUPPORTED;
  double* ws = (dwork && work_bytes >= sizeof(double)) ? (double*)dwork : nullptr;
  return gemm64(h->stream, transa, transb, fa, 0, lower, (int)m, (int)n, (int)k, alpha, dA, lda, dB, ldb, beta, dC,
                ldc, 0, 0, 0, 0, ws, ws ? work_bytes / sizeof(double) : 0);
}

int abft_encode(abft_handle h, int64_t m, int64_t n, const double* dA, int64_t lda, int32_t nb, double* dcolchk,
                int64_t ldc, double* drowchk, int64_t ldr) {
  if (!h) return -1;
  if (m < 0) return -2;
  if (n < 0) return -3;
  if (lda < std::max<int64_t>(1, m)) return -5;
  if (nb < 1 || nb > MAXNB) return -6;
  const int64_t Tr = (m + nb - 1) / nb;
  if (ldc < std::max<int64_t>(1, 2 * Tr)) return -8;
  if (ldr < std::max<int64_t>(1, m)) return -10;
  if (m == 0 || n == 0) return 0;
  return verify_tiles<double>(h->stream, dA, lda, m, n, nb, 0, 0, 0, 0, dcolchk, ldc, drowchk, ldr, nullptr, nullptr,
                              0.0, nullptr, nullptr, -1);
}

int abft_verify(abft_handle h, int64_t m, int64_t n, double* dA, int64_t lda, int32_t nb, double* dcolchk,
                int64_t ldc, double* drowchk, int64_t ldr, double tau_scale, int32_t correct, int32_t* dflags,
                abft_report* drep) {
  if (!h) return -1;
  if (m < 0) return -2;
  if (n < 0) return -3;
  if (lda < std::max<int64_t>(1, m)) return -5;
  if (nb < 1 || nb > MAXNB) return -6;
  const int64_t Tr = (m + nb - 1) / nb;
  if (ldc < std::max<int64_t>(1, 2 * Tr)) return -8;
  if (ldr < std::max<int64_t>(1, m)) return -10;
  if (correct && !dflags) return -13;
  hipStream_t s = h->stream;
  TRY(report_init(s, drep, nullptr));
  if (m == 0 || n == 0) return report_fini(s, drep);
  const double tsu = (tau_scale > 0 ? tau_scale : 4.0) * U64;
  TRY(verify_tiles<double>(s, dA, lda, m, n, nb, 0, 0, 0, correct ? 1 : 2, dcolchk, ldc, drowchk, ldr, nullptr,
                           nullptr, tsu, dflags, drep, 0));
  if (correct)
    TRY(correct_tiles<double>(s, dA, lda, m, n, nb, 0, 0, 0, dcolchk, ldc, drowchk, ldr, nullptr, nullptr, tsu, dflags,
                              drep, 0));
  return report_fini(s, drep);
}

int abft_gesv_mp(abft_handle h, int64_t n, const double* dA, int64_t lda, const double* db, double* dx, int32_t prec,
                 int32_t max_iter, void* dwork, size_t work_bytes, const abft_opts* opts, abft_ir_report* dir,
                 abft_report* drep) {
  return gesv_mp_impl(h, n, dA, lda, db, dx, prec, max_iter, dwork, work_bytes, opts, dir, drep, 0);
}
int abft_posv_mp(abft_handle h, int64_t n, const double* dA, int64_t lda, const double* db, double* dx, int32_t prec,
                 int32_t max_iter, void* dwork, size_t work_bytes, const abft_opts* opts, abft_ir_report* dir,
                 abft_report* drep) {
  return gesv_mp_impl(h, n, dA, lda, db, dx, prec, max_iter, dwork, work_bytes, opts, dir, drep, 1);
}
static int batched_common(abft_handle h, int chol, int32_t batch, int32_t nmax, const int32_t* dn, void* const* dA,
                          const int32_t* dlda, int32_t* const* dipiv, int32_t prec, void* dwork, size_t work_bytes,
                          const abft_opts* opts, int32_t* dinfo, abft_report* dreps) {
  if (!h) return -1;
  if (batch < 0) return -2;
  if (nmax < 0 || nmax > 512) return -3;
  if (batch > 0 && (!dn || !dA || !dlda)) return -4;
  if (!chol && batch > 0 && !dipiv) return -7;
  if (prec != ABFT_F64 && prec != ABFT_F32) return ABFT_ERR_UNSUPPORTED;
  int nb, protect;
  double ts;
  TRY(check_opts(opts, nmax, nb, protect, ts));
  if (nb != 32) return ABFT_ERR_UNSUPPORTED;  // the batched kernels use 32-wide blocks and tiles
  if (protect == ABFT_PROTECT_SINGLE || opts->levels) return ABFT_ERR_UNSUPPORTED;  // full checksums or none
  if (batch == 0) return 0;
  if (!dinfo || !dreps) return -11;
  use_ws(h, dwork, work_bytes);
  if (!dwork || work_bytes < batched_ws_bytes(batch)) return ABFT_ERR_WORKSPACE;
  const int nf = opts->faults ? opts->nfaults : 0;
  if (opts->wgs_per_cu < 0 || opts->wgs_per_cu > 4) return -10;
  const int wgs = std::max(1, (int)opts->wgs_per_cu) * h->cus;
  if (!(opts->flags & ABFT_FLAG_GRAPH) || nf > 0)
    return batched_factor(h->stream, chol, prec, batch, dn, dA, dlda, dipiv, dwork, protect, ts, opts->faults, nf,
                          dinfo, dreps, wgs);
  // graph path: replay the graph captured for these arguments, or capture it
  for (int i = 0; i < h->ngraphs; ++i) {
    const BatchGraph& g = h->graphs[i];
    if (g.chol == chol && g.prec == prec && g.batch == batch && g.protect == protect && g.ts == ts && g.wgs == wgs &&
        g.dn == dn &&
        g.dA == dA && g.dlda == dlda && g.dipiv == dipiv && g.dwork == dwork && g.dinfo == dinfo && g.dreps == dreps)
      return hipGraphLaunch(g.exec, h->stream) == hipSuccess ? 0 : ABFT_ERR_HIP;
  }
  if (!h->cap && hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking) != hipSuccess) return ABFT_ERR_HIP;
  if (hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) return ABFT_ERR_HIP;
  const int rc = batched_factor(h->cap, chol, prec, batch, dn, dA, dlda, dipiv, dwork, protect, ts, nullptr, 0, dinfo,
                                dreps, wgs);
  hipGraph_t graph = nullptr;
  const hipError_t ec = hipStreamEndCapture(h->cap, &graph);
  if (rc || ec != hipSuccess || !graph) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc ? rc : ABFT_ERR_HIP;
  }
  hipGraphExec_t exec = nullptr;
  const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ei != hipSuccess) return ABFT_ERR_HIP;
  int slot;
  if (h->ngraphs < MAX_GRAPHS) {
    slot = h->ngraphs++;
  } else {  // evict round-robin, after the stream has finished any replay of it
    slot = h->next_graph++ % MAX_GRAPHS;
    if (hipStreamSynchronize(h->stream) != hipSuccess) return ABFT_ERR_HIP;
    (void)hipGraphExecDestroy(h->graphs[slot].exec);
  }
  h->graphs[slot] = BatchGraph{chol, prec, batch, protect, wgs, ts, dn, dA, dlda, dipiv, dwork, dinfo, dreps, exec};
  return hipGraphLaunch(exec, h->stream) == hipSuccess ? 0 : ABFT_ERR_HIP;
}

int abft_potrf_batched(abft_handle h, int32_t batch, int32_t nmax, const int32_t* dn, void* const* dA,
                       const int32_t* dlda, int32_t prec, void* dwork, size_t work_bytes, const abft_opts* opts,
                       int32_t* dinfo, abft_report* dreps) {
  return batched_common(h, 1, batch, nmax, dn, dA, dlda, nullptr, prec, dwork, work_bytes, opts, dinfo, dreps);
}
int abft_getrf_batched(abft_handle h, int32_t batch, int32_t nmax, const int32_t* dn, void* const* dA,
                       const int32_t* dlda, int32_t* const* dipiv, int32_t prec, void* dwork, size_t work_bytes,
                       const abft_opts* opts, int32_t* dinfo, abft_report* dreps) {
  return batched_common(h, 0, batch, nmax, dn, dA, dlda, dipiv, prec, dwork, work_bytes, opts, dinfo, dreps);
}

}  // extern "C"
