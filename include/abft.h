/*
 * abft.h -- C ABI of the ABFT-protected one-sided decomposition library for
 * AMD Instinct MI355X (gfx950).
 *
 * The operations follow the blocked one-sided decompositions of Chen et al.,
 * "Improving Energy Saving of One-sided Matrix Decompositions on CPU-GPU
 * Heterogeneous Systems" (PPoPP'23), section "State-of-the-art matrix
 * decompositions": each iteration performs a panel decomposition (PD), a
 * panel update (PU) and a trailing-matrix update (TMU).  The fault tolerance
 * follows the paper's ABFT description (section "Design of ABFT-OC"):
 * checksums are encoded before an operation, the same operation is applied to
 * them, and the relation is verified after every iteration (the detection
 * interval); full checksums cover rows and columns of every b x b block.
 *
 * Conventions for every entry point:
 *   - Matrices are column-major, element (i,j) at A[i + j*lda], lda >= n.
 *   - Every pointer argument whose name starts with `d` is DEVICE memory owned
 *     by the caller (for instance a PyTorch tensor).  The library never
 *     allocates device memory; scratch space is the caller's `dwork` buffer,
 *     sized with abft_workspace_size().  `opts` and fault plans are host
 *     memory and are read before the call returns.
 *   - Calls are asynchronous on the handle's HIP stream.  Results, `dinfo`
 *     and the report become valid once the stream has been synchronized;
 *     until then the caller must not touch dA, the workspace or the report.
 *     The blocked factorizations also use an internal side stream of the
 *     handle (created on first use, default priority) for LU's interchanges
 *     of the already factored left columns of dA, the panel checks and the
 *     checksum carries (it writes those columns, the checksum arrays of the
 *     workspace and the report), and, with ABFT_FLAG_OVERLAP_VERIFY, a
 *     stream restricted to half of the compute units that verifies and
 *     corrects trailing tiles of dA (see below).  Both are ordered after
 *     the caller's stream by events and joined back before the call's last
 *     operation on that stream.
 *   - Return value: 0 on success; -i when argument i (1-based) is invalid;
 *     ABFT_ERR_HIP when a HIP call failed (launch or cooperative-launch
 *     error); ABFT_ERR_WORKSPACE when `work_bytes` is too small;
 *     ABFT_ERR_UNSUPPORTED for an option combination that is not built.
 *   - Numerical status is written to device memory: potrf `*dinfo = j > 0`
 *     when the leading minor of order j is not positive definite; getrf
 *     `*dinfo = j > 0` when U(j,j) is exactly zero (factorization completes,
 *     LAPACK semantics).  The ABFT outcome is in the report; after a
 *     Cholesky breakdown (info > 0) the remaining iterations run on NaN data
 *     and their checks flag, so the report then says nothing about faults.
 */
#ifndef ABFT_H
#define ABFT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct abft_handle_s* abft_handle;

enum {
  ABFT_OK = 0,
  ABFT_ERR_HIP = -100,
  ABFT_ERR_WORKSPACE = -101,
  ABFT_ERR_UNSUPPORTED = -102
};

/* Protection level of an iteration (the paper's single-side and full
   checksums, section "Design of ABFT-OC", and its adaptive ABFT, Alg. 1,
   which turns protection on per iteration): NONE carries and verifies
   nothing; SINGLE carries and compares the column checksums of every tile
   only, which locates and corrects one wrong element per tile (0D) and
   reports anything else as uncorrectable; FULL adds the row checksums, which
   also correct one wrong row or column of a tile (1D: every element of it is
   rebuilt from the checksums of the other side).  When the level rises from
   one iteration to the next (or starts above NONE), the checksums of the
   remaining matrix are encoded from its data at the start of that
   iteration. */
enum { ABFT_PROTECT_NONE = 0, ABFT_PROTECT_SINGLE = 1, ABFT_PROTECT_FULL = 2 };

/* arithmetic of a factorization: FP64, FP32, or FP32 data whose trailing
   update multiplies bf16 / fp16 operands with FP32 accumulation */
enum { ABFT_F64 = 0, ABFT_F32 = 1, ABFT_BF16 = 2, ABFT_F16 = 3 };

/* operation codes for abft_workspace_size */
enum {
  ABFT_OP_POTRF = 1,
  ABFT_OP_GETRF = 2,
  ABFT_OP_GEQRF = 3,
  ABFT_OP_GESV_MP = 4,
  ABFT_OP_POSV_MP = 5,
  ABFT_OP_POTRF_BATCHED = 6,
  ABFT_OP_GETRF_BATCHED = 7
};

/* report status bits */
enum {
  ABFT_ST_CORRECTED = 1,     /* at least one element was located and recomputed */
  ABFT_ST_REPAIRED = 2,      /* a checksum entry itself was wrong and re-encoded */
  ABFT_ST_UNCORRECTABLE = 4, /* a flagged tile could not be corrected: result untrustworthy */
  ABFT_ST_PANEL = 8,         /* a panel / panel-update check failed (detection only) */
  ABFT_ST_INTERNAL = 16      /* a cooperative kernel hit its wait limit: result invalid */
};

/* A test-only fault plan: after the trailing update of iteration `iter`, flip
   bit `bit` (0..63 of the binary64 pattern; 0..31 of binary32 data) of one
   element.  target 0 = the matrix (row, col are matrix indices), 1 = the
   column-checksum array (row in [0, 2*ceil(n/nb))), 2 = the row-checksum array
   (col in [0, 2*ceil(n/nb))).  `matrix` selects the matrix of a batch.
   Operand faults (FP64 blocked factorizations; the paper's 1D error class,
   section "Design of ABFT-OC"): target 3 flips an element of the left
   operand of iteration `iter`'s trailing-update product (L21 for Cholesky
   and LU, V for QR; row, col are matrix indices), target 4 one of the right
   operand (LU: U12 at its matrix indices; QR: W2 = T^T V^T C, row = p in
   [0, nb), col = the matrix column); the flip lasts for that product only
   (it is undone right after it), so one row (3) or one column (4) of the
   updated matrix is wrong while the operand and the checksum carry are not.
   A call with operand faults runs on one stream. */
typedef struct {
  int32_t iter, target;
  int64_t row, col;
  int32_t bit, matrix;
} abft_fault;

typedef struct {
  int32_t iter, kind; /* 1 element corrected, 2 checksum repaired, 3 uncorrectable, 4 panel flag,
                         5 row rebuilt, 6 column rebuilt (1D) */
  int64_t row, col;   /* corrected element; kind 5: the row and the tile's first column; kind 6: the
                         tile's first row and the column; otherwise the flagged tile's first row / column */
} abft_event;

#define ABFT_MAX_EVENTS 16

/* Device-resident outcome of one protected call (zeroed by the call itself). */
typedef struct {
  int64_t flagged_tiles, corrected, checksum_repaired, uncorrectable, panel_flags;
  int32_t first_flag_iter, status; /* first iteration with a flag (-1 none); ABFT_ST_* bits */
  double max_ratio;                /* largest |d| / tau over the unflagged comparisons */
  int32_t nev, pad;
  abft_event ev[ABFT_MAX_EVENTS];
  /* test use: the last single-bit fault planted in the matrix (target 0):
     |value after - value before| (+Inf when either is not finite), and the
     |d| and tau of the plain column checksum that covers it at the
     verification right after the flip (-1 when it was not verified) */
  double fault_delta, fault_d, fault_tau;
} abft_report;

typedef struct {
  int32_t nb;          /* block size = checksum tile size (1..512; batched: 32) */
  int32_t protect;     /* ABFT_PROTECT_NONE, _SINGLE or _FULL for every iteration (batched: NONE or FULL) */
  double tau_scale;    /* threshold scale (default 4.0 when <= 0) */
  const abft_fault* faults; /* host array of fault plans (test use), may be NULL */
  int32_t nfaults;
  int32_t flags;       /* ABFT_FLAG_* bits */
  int32_t wgs_per_cu;  /* batched: persistent workgroups per compute unit (0: 1; at most 4) */
  int32_t nlevels;     /* entries of `levels` (0: none) */
  const int8_t* levels; /* host array, levels[k] = ABFT_PROTECT_* of iteration k (k < ceil(n/nb) <= nlevels),
                           overriding `protect` (FP64 blocked factorizations); NULL: `protect` everywhere */
  int32_t lookahead;   /* blocked factorizations: compute units given to the look-ahead panel stream
                          (<= 0: the one-stream schedule, the default; see below) */
  int32_t tmu_bk;      /* K depth of the trailing-update product's 128 x 128 tiles: 16 (0: default; two
                          workgroups per CU) or 32 (one workgroup per CU, the block's C read during its last
                          K step); the results are the same bitwise (same order of the products over K) */
} abft_opts;

/* Look-ahead (the paper's section "State-of-the-art matrix decompositions":
   the part of the update that the next panel needs is done first, then the
   next panel decomposition runs concurrently with the rest of the update).
   With opts->lookahead > 0, a Cholesky, LU or QR factorization with uniform
   protection and no fault plan runs its work on two streams of the handle
   restricted to disjoint sets of compute units (created for the call with
   hipExtStreamCreateWithCUMask, default priority): the panel stream gets
   opts->lookahead units (for LU and QR raised to what the first panel's
   cooperative leaves need to hold its rows in LDS, at most half the
   device), the
   update stream the rest.  Each iteration updates and verifies the next
   panel's block column first, factors that panel on the panel stream while
   the rest of the trailing matrix is updated and verified, and joins before
   the next iteration.  Both streams are ordered after the caller's stream
   on entry and the caller's stream after both on exit.  Profiled calls and
   calls with fault plans or per-iteration levels use the one-stream
   schedule.  The factors equal the one-stream schedule's bitwise when the
   cooperative leaves get the same shape on both (small panels; always for
   Cholesky, whose panel has no cooperative leaf), and to rounding
   otherwise.  It is off by default: on one MI355X the LU and QR panels
   need about a quarter of the device's LDS at n = 32768, and in all three
   the update loses more on the remaining units than the overlap saves (LU
   883 -> 1063 ms, QR 1342 -> 1631 ms with 64 panel units; Cholesky
   341 -> 380 ms with 32).  The two restricted streams are created for the
   call and destroyed at its end. */

/* opts.flags: ABFT_FLAG_PROFILE times the phases of the call with HIP
   events on the handle's stream, all work on that one stream (the call then
   waits for its own completion before returning); ABFT_FLAG_GRAPH lets the batched calls capture and
   replay HIP graphs (see abft_potrf_batched).

   ABFT_FLAG_OVERLAP_VERIFY (FP64 and binary32 blocked factorizations; the
   paper's section "Design of ABFT-OC" schedules checksum verification
   beside the panel decomposition): after each trailing update the tiles of
   the next panel's block column are verified and corrected first, on the
   handle's stream; the other trailing tiles are verified and corrected on a
   second stream restricted to half of the compute units (created with
   hipExtStreamCreateWithCUMask, default priority, for the call and
   destroyed at its end: while such a stream exists other work on the
   device runs slower) while the next panel is factored on the handle's
   stream, and the handle's stream waits for them before the panel's
   interchanges, checks and the next update.  When the handle's stream is
   the null stream, the call's work runs on a non-blocking stream of the
   handle ordered after the null stream on entry and before it on exit (the
   restricted stream is a blocking stream).  The same tiles are verified
   with the same sums, so the factors and the report equal those of the
   serial schedule.  Ignored by profiled calls, calls with operand faults
   and the look-ahead schedule.  On one MI355X at n = 32768, nb = 512: LU
   883 -> 838 ms, QR 1342 -> 1303 ms. */
enum { ABFT_FLAG_PROFILE = 1, ABFT_FLAG_GRAPH = 2, ABFT_FLAG_OVERLAP_VERIFY = 4 };

/* Phase times of the last call made with ABFT_FLAG_PROFILE, with the
   algorithmic work of the timed trailing-update GEMMs and verify passes. */
typedef struct {
  double ms_total, ms_panel, ms_tmu, ms_carry, ms_verify;
  double tmu_flops;    /* flops of the trailing-update GEMMs (2 m n k each) */
  double verify_bytes; /* bytes of matrix data streamed by the verify passes */
  int32_t tmu_launches, iters;
} abft_profile;

typedef struct {
  int32_t iters, converged, failed_reason, info; /* reason: 0 ok, 1 no contraction, 2 non-finite, 3 max iter, 4 factorization info */
  double resid_norm, x_norm, a_norm, last_dx;    /* infinity norms at exit */
} abft_ir_report;

/* Handle: holds the stream and device properties.  `stream` is a hipStream_t
   (NULL = the default stream).  Returns 0 or ABFT_ERR_HIP.  abft_destroy
   synchronizes the handle's streams before releasing them.  (Library
   plumbing; the paper's system keeps the equivalent state in its runtime,
   section "State-of-the-art matrix decompositions".) */
int abft_create(abft_handle* h, void* stream);
int abft_destroy(abft_handle h);
int abft_set_stream(abft_handle h, void* stream);

/* Copy the phase profile of the handle's last ABFT_FLAG_PROFILE call (the
   per-phase split PD / PU / TMU / checksum work of the paper's Tab. 2). */
int abft_get_profile(abft_handle h, abft_profile* out);

/* Per-iteration phase times (ms) of the handle's last ABFT_FLAG_PROFILE
   call: ms is a host array of 5 * cap doubles, phase-major, ms[p * cap + k]
   for iteration k < min(cap, *iters) and phase p = 0 panel decomposition
   (PD; Cholesky's and QR's panel updates included), 1 panel update (LU's
   U12 solve), 2 trailing-matrix update products, 3 checksum carries,
   4 checksum verification and correction.  *iters receives the number of
   iterations recorded.  These are the per-iteration task times that the
   paper's algorithmic time prediction works from (section "Bi-directional
   slack reclamation", Tab. 2 and the weighted-neighbour predictor). */
int abft_get_iter_profile(abft_handle h, int32_t cap, double* ms, int32_t* iters);

/* Bytes of device workspace needed by operation `op` on an n x n problem
   (for the batched ops: n = the largest matrix order, `batch` matrices):
   the checksum arrays of section "Design of ABFT-OC" (ABFT checksum: one
   pair of column and row checksums per b x b block) plus panel scratch. */
int abft_workspace_size(abft_handle h, int op, int64_t n, int32_t batch, const abft_opts* opts, size_t* bytes);

/* Register a device workspace with the handle: every later call that passes
   dwork == NULL uses it (with its size), so a caller can size and hand over
   one buffer once.  dwork stays owned by the caller and must outlive its use
   by enqueued calls; NULL (with bytes 0) unregisters.  Returns -2 for a NULL
   buffer of nonzero size. */
int abft_set_workspace(abft_handle h, void* dwork, size_t bytes);

/* Copy a device report to host memory: enqueued on the handle's stream
   after the calls before it, then the stream is synchronized, so `out`
   holds the call's final outcome (section "Design of ABFT-OC": detected,
   corrected or uncorrectable errors of the protected factorization). */
int abft_report_fetch(abft_handle h, const abft_report* drep, abft_report* out);

/* Cholesky A = L L^T of the lower triangle (the strict upper triangle is
   neither read nor written).  Blocked right-looking with block size opts->nb;
   the trailing update carries per-tile row and column checksums of the
   symmetric trailing matrix, verified and corrected every iteration.
   dinfo: device int32.  drep: device abft_report (may be NULL).
   Paper: section "State-of-the-art matrix decompositions" (Cholesky's PD,
   PU and TMU per iteration) and section "Design of ABFT-OC" (ABFT
   checksum: encode, apply the same operation, verify each iteration). */
int abft_potrf(abft_handle h, int64_t n, double* dA, int64_t lda, void* dwork, size_t work_bytes,
               const abft_opts* opts, int32_t* dinfo, abft_report* drep);

/* abft_potrf for callers that cannot allocate device memory or pass a
   workspace (code under HIP graph capture, tight serving loops, harnesses
   that forbid allocation).  Same arguments, result and report as abft_potrf
   without dwork / work_bytes: the scratch is a 64 MiB device array built
   into the library (one copy per GPU, held until the process ends), so this
   call allocates nothing and creates no stream or event: all its work runs
   on the handle's stream (no side stream) and ABFT_FLAG_PROFILE is rejected
   (ABFT_ERR_UNSUPPORTED).  Returns ABFT_ERR_WORKSPACE when the problem needs
   more scratch than that (abft_workspace_size(ABFT_OP_POTRF) > 64 MiB: about
   n > 16384 at nb = 512).  Every call on one GPU shares that GPU's array:
   calls that overlap on one GPU (other streams, other handles, other host
   threads) race and must be serialized by the caller; nothing from a
   previous call is read. */
int abft_potrf_noalloc(abft_handle h, int64_t n, double* dA, int64_t lda, const abft_opts* opts, int32_t* dinfo,
                       abft_report* drep);

/* LU with partial pivoting P A = L U (L unit lower, U upper, both in A).
   dipiv: device int32[n], 1-based LAPACK row interchanges; ties in the pivot
   search take the first (smallest) row index.  Paper: section
   "State-of-the-art matrix decompositions" (the LU iteration: panel
   decomposition with pivoting, U12 panel update, trailing GEMM) and section
   "Design of ABFT-OC" (full checksums per block). */
int abft_getrf(abft_handle h, int64_t n, double* dA, int64_t lda, int32_t* dipiv, void* dwork, size_t work_bytes,
               const abft_opts* opts, int32_t* dinfo, abft_report* drep);

/* Householder QR A = Q R, LAPACK geqrf storage: R in the upper triangle, the
   reflector vectors v (v(j) = 1 implicit) below the diagonal, dtau[n] the
   scalar factors (H_j = I - tau_j v_j v_j^T).  Paper: section
   "State-of-the-art matrix decompositions" (QR's panel of Householder
   reflectors and its blocked trailing update) and section "Design of
   ABFT-OC" (full checksums per block). */
int abft_geqrf(abft_handle h, int64_t n, double* dA, int64_t lda, double* dtau, void* dwork, size_t work_bytes,
               const abft_opts* opts, int32_t* dinfo, abft_report* drep);

/* The trailing-matrix update primitive (the TMU product of every iteration
   of the blocked decompositions, and the checksum carry C^c -= S Y of the
   ABFT design): C = beta*C + alpha*op(A)*op(B) in FP64 on the FP64 matrix
   cores, op(X) = X (trans 0) or X^T (trans 1); C is m x n, op(A) m x k,
   op(B) k x n, all column-major device memory.  flags:
   ABFT_GEMM_LOWER writes only entries C(i,j) with i >= j (symmetric
   updates); ABFT_GEMM_UNIT_LOWER_A reads the stored A as unit lower
   triangular (above its diagonal 0, on it 1: Householder vectors).
   dwork (may be NULL) lets a product with few output tiles and a long K
   split K over more workgroups (partials reduced in a fixed order), using
   up to work_bytes.  Supported: NN, NT, TN; UNIT_LOWER_A with NN or TN;
   LOWER with NT.  m, n, k < 2^31.  Paper: section "State-of-the-art matrix
   decompositions" (TMU, the GEMM that dominates each iteration). */
enum { ABFT_GEMM_LOWER = 1, ABFT_GEMM_UNIT_LOWER_A = 2 };
int abft_gemm(abft_handle h, int32_t transa, int32_t transb, int32_t flags, int64_t m, int64_t n, int64_t k,
              double alpha, const double* dA, int64_t lda, const double* dB, int64_t ldb, double beta, double* dC,
              int64_t ldc, void* dwork, size_t work_bytes);

/* Standalone per-tile checksums of an m x n matrix with tile size nb:
   dcolchk is (2*ceil(m/nb)) x n with leading dimension ldc >= 2*ceil(m/nb):
   row 2I holds the column sums of tile-row I, row 2I+1 the sums weighted by
   the row's position in the tile (1..nb).  drowchk is m x (2*ceil(n/nb)) with
   ldr >= m: column 2J holds the row sums over tile-column J, column 2J+1 the
   sums weighted by the column's position in the tile.  Paper: section
   "Design of ABFT-OC", ABFT checksum (each block encoded on its own, row
   and column checksums for full protection). */
int abft_encode(abft_handle h, int64_t m, int64_t n, const double* dA, int64_t lda, int32_t nb, double* dcolchk,
                int64_t ldc, double* drowchk, int64_t ldr);

/* Compare the matrix with checksums from abft_encode.  dflags (device int32,
   ceil(m/nb) x ceil(n/nb), column-major, may be NULL) receives 1 for a
   flagged tile.  With correct != 0, flagged tiles go through the same
   locate / correct step as the factorizations (A and the checksums are then
   modified in place).  drep receives counters and max_ratio.  Paper:
   section "Design of ABFT-OC", ABFT checksum (verification after the
   operation; an error located at the intersection of the inconsistent
   checksums is corrected, 0D / 1D / 2D error classes). */
int abft_verify(abft_handle h, int64_t m, int64_t n, double* dA, int64_t lda, int32_t nb, double* dcolchk,
                int64_t ldc, double* drowchk, int64_t ldr, double tau_scale, int32_t correct, int32_t* dflags,
                abft_report* drep);

/* Mixed-precision solve of A x = b (A n x n FP64, not modified): factor a
   binary32 copy of A (LU with partial pivoting, or Cholesky for posv) whose
   trailing updates run in `prec` (ABFT_F32, ABFT_BF16 or ABFT_F16 operands
   with FP32 accumulation), then refine in FP64: r = b - A x, d = solve(r),
   x += d, until ||d|| <= u ||x|| or ||r|| <= u ||A|| ||x|| (u = 2^-53), with
   failure on non-finite values, on ||d_i|| > ||d_(i-1)||/2 while far from
   convergence, or after max_iter corrections.  prec == ABFT_F64 factors in
   FP64 and solves directly (the reference method).  dir: device
   abft_ir_report.  Paper: the LU / Cholesky iterations of section
   "State-of-the-art matrix decompositions" run in lower precision, with the
   single- vs double-precision throughput gap of the introduction as the
   motivation (the refinement itself is this library's addition). */
int abft_gesv_mp(abft_handle h, int64_t n, const double* dA, int64_t lda, const double* db, double* dx, int32_t prec,
                 int32_t max_iter, void* dwork, size_t work_bytes, const abft_opts* opts, abft_ir_report* dir,
                 abft_report* drep);
int abft_posv_mp(abft_handle h, int64_t n, const double* dA, int64_t lda, const double* db, double* dx, int32_t prec,
                 int32_t max_iter, void* dwork, size_t work_bytes, const abft_opts* opts, abft_ir_report* dir,
                 abft_report* drep);

/* Batched protected factorizations of `batch` independent matrices of
   uneven orders.  dn[i], dlda[i] (device int32) and dA[i] (device array of
   device pointers) describe matrix i; prec is ABFT_F64 (double data) or
   ABFT_F32 (float data; dA then holds float pointers).  nmax bounds every
   dn[i] (<= 512).  dinfo[i] and dreps[i] receive each matrix's status.
   Fault plans select their matrix with abft_fault.matrix.  With
   ABFT_FLAG_GRAPH in opts->flags (and no fault plan) the call's launches are
   captured into a HIP graph the first time a given argument set is seen and
   the graph is replayed on the handle's stream by later calls with the same
   pointers and sizes (up to 8 argument sets are kept per handle); the
   contents of the arrays may change between replays, their addresses not.
   Paper: the Cholesky / LU iteration of section "State-of-the-art matrix
   decompositions" with the block checksums of section "Design of ABFT-OC",
   applied to each matrix of the batch. */
int abft_potrf_batched(abft_handle h, int32_t batch, int32_t nmax, const int32_t* dn, void* const* dA,
                       const int32_t* dlda, int32_t prec, void* dwork, size_t work_bytes, const abft_opts* opts,
                       int32_t* dinfo, abft_report* dreps);
int abft_getrf_batched(abft_handle h, int32_t batch, int32_t nmax, const int32_t* dn, void* const* dA,
                       const int32_t* dlda, int32_t* const* dipiv, int32_t prec, void* dwork, size_t work_bytes,
                       const abft_opts* opts, int32_t* dinfo, abft_report* dreps);

#ifdef __cplusplus
}
#endif
#endif /* ABFT_H */
